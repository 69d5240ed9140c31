"""The tile table (no GPU needed): rt_tuning_set / rt_tuning_plan on the host,
the precision guard of the planner, and the committed table's well-formedness."""
import os

import pytest

from paper_1905_07311_amd import rtucker


@pytest.fixture
def restore_table():
    yield
    if os.path.exists(rtucker.TUNING_FILE):
        rtucker.set_tuning(rtucker.read_tuning(rtucker.TUNING_FILE))
    else:
        rtucker.set_tuning([])


def _entry(**kw):
    e = {"op": 0, "dtype": rtucker.RT_F32, "prec": rtucker.PREC["f32"], "stride": 0, "j_lo": 256, "j_hi": 1023,
         "k_lo": 1, "k_hi": 1 << 40, "ell_lo": 1, "ell_hi": 64, "kind": 1, "rb": 2, "rw": 1, "wgs": 512}
    e.update(kw)
    return e


def test_plan_follows_the_table(restore_table):
    rtucker.set_tuning([])
    p = rtucker.tuning_plan("f32", "f32", (512, 512, 512), 0, 35)
    assert not p["from_table"] and p["kind"] == 3            # built-in: split-bfloat16 float32 sketch
    rtucker.set_tuning([_entry()])
    p = rtucker.tuning_plan("f32", "f32", (512, 512, 512), 0, 35)
    assert p["from_table"] and (p["kind"], p["rb"], p["rw"]) == (1, 2, 1)
    assert 0 < p["wgs"] <= 512 and p["j_lo"] == p["j_hi"] == 512 and p["k_lo"] == 512 * 512
    # outside the entry's bucket (another stride class, J, ell): built-in again
    assert not rtucker.tuning_plan("f32", "f32", (512, 512, 512), 1, 35)["from_table"]
    assert not rtucker.tuning_plan("f32", "f32", (100, 512, 512), 0, 35)["from_table"]
    # first matching entry wins
    rtucker.set_tuning([_entry(kind=0, wgs=4096), _entry()])
    p = rtucker.tuning_plan("f32", "f32", (512, 512, 512), 0, 35)
    assert p["from_table"] and p["kind"] == 0


def test_precision_guard(restore_table):
    # the bfloat16 sketch never serves a float32 request, the float32-accurate
    # kernel never a float64 one: such entries are skipped
    rtucker.set_tuning([_entry(kind=4, rb=2, rw=0)])
    p = rtucker.tuning_plan("f32", "f32", (512, 512, 512), 0, 35)
    assert not p["from_table"] and p["kind"] == 3
    rtucker.set_tuning([_entry(dtype=rtucker.RT_F64, prec=rtucker.PREC["f64"], kind=3, rb=2, rw=0)])
    assert not rtucker.tuning_plan("f64", "f64", (512, 512, 512), 0, 35)["from_table"]
    # a variant that cannot serve the shape (x8 columns needed) is skipped too
    rtucker.set_tuning([_entry(stride=2, kind=3, rb=2, rw=0)])
    assert not rtucker.tuning_plan("f32", "f32", (512, 512, 512), 2, 35)["from_table"]


def test_malformed_entries_are_rejected(restore_table):
    for bad in (_entry(kind=2), _entry(j_lo=9, j_hi=3), _entry(op=7), _entry(stride=5), _entry(wgs=-1)):
        with pytest.raises(rtucker.RtError):
            rtucker.set_tuning([bad])


def test_committed_table_is_well_formed():
    if not os.path.exists(rtucker.TUNING_FILE):
        pytest.skip("no tile table committed")
    import json
    doc = json.load(open(rtucker.TUNING_FILE))
    assert doc["arch"] == "gfx950" and doc["entries"]
    for e in doc["entries"]:
        prec = e["prec"]
        assert (e["dtype"] == rtucker.RT_F64) == (prec == rtucker.PREC["f64"])
        allowed = {rtucker.PREC["f64"]: {0}, rtucker.PREC["f32"]: {0, 1, 3}, rtucker.PREC["bf16"]: {0, 1, 4}}[prec]
        assert e["kind"] in allowed
        m = e["measured"]
        J = m["dims"][m["mode"]]
        assert e["j_lo"] <= J <= e["j_hi"] and e["ell_lo"] <= m["ell"] <= e["ell_hi"]
        assert m["best_ms"] <= m["builtin_ms"] * 1.0001
    # the installed table gives each tuned problem the choice of the first entry
    # whose bucket holds it
    for e in doc["entries"]:
        m = e["measured"]
        J, K = m["dims"][m["mode"]], 1
        for i, v in enumerate(m["dims"]):
            K *= v if i != m["mode"] else 1
        first = next(f for f in doc["entries"]
                     if f["dtype"] == e["dtype"] and f["prec"] == e["prec"] and f["stride"] == e["stride"]
                     and f["j_lo"] <= J <= f["j_hi"] and f["k_lo"] <= K <= f["k_hi"]
                     and f["ell_lo"] <= m["ell"] <= f["ell_hi"])
        p = rtucker.tuning_plan(e["dtype"], e["prec"], m["dims"], m["mode"], m["ell"])
        assert p["from_table"] and p["kind"] == first["kind"]
