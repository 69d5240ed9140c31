"""Pins of the oracle's Omega stream (oracle/philox.py).

* the Philox4x32-10 block function agrees bit for bit with rocRAND's own
  engine (an independent implementation, compiled from its headers on the host);
* the Box-Muller normals have the moments and distribution of N(0, 1) and the
  columns are uncorrelated;
* the column map: column k of Omega is word k mod 4 of block floor(k/4).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_kat(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_kernel.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = str(tmp_path_factory.mktemp("kat") / "kat")
    subprocess.run([hipcc, "-O1", os.path.join(HERE, "rocrand_philox_kat.cpp"), "-o", exe],
                   check=True, capture_output=True, timeout=600)
    return exe


def _tuples():
    rng = np.random.default_rng(7)
    tup = [(0, 0, 0, 0), (2**64 - 1, 2**62 - 1, 2**32 - 1, 2**32 - 1), (1, 0, 0, 0), (0, 1, 0, 0),
           (0, 0, 1, 0), (0, 0, 0, 1), (0x123456789ABCDEF, 2**32, 5, 2), (42, 2**32 - 1, 8, 4)]
    for _ in range(200):
        tup.append((int(rng.integers(0, 2**63)), int(rng.integers(0, 2**40)),
                    int(rng.integers(0, 2**20)), int(rng.integers(0, 8))))
    return tup


def test_philox_block_matches_rocrand(rocrand_kat):
    tup = _tuples()
    inp = "\n".join(" ".join(str(v) for v in t) for t in tup) + "\n"
    out = subprocess.run([rocrand_kat], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(w) for w in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    ctr = np.array([[c & 0xFFFFFFFF, c >> 32, q, m] for (_, c, q, m) in tup], dtype=np.uint64)
    key = np.array([[s & 0xFFFFFFFF, s >> 32] for (s, _, _, _) in tup], dtype=np.uint64)
    got = oracle.philox4x32_10(ctr, key).astype(np.uint64)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


def test_normals_moments_and_ks():
    from scipy import stats
    Om = oracle.omega(seed=3, mode=1, nrows=50000, cols=8)
    z = Om.ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    kurt = np.mean(z ** 4) / np.mean(z ** 2) ** 2
    assert abs(kurt - 3.0) < 0.1
    assert stats.kstest(z, "norm").pvalue > 1e-4
    C = np.corrcoef(Om.T)
    off = C[~np.eye(C.shape[0], dtype=bool)]
    assert np.max(np.abs(off)) < 5 / np.sqrt(Om.shape[0])


def test_column_map_and_streams():
    rows = np.arange(100)
    full = oracle.omega(seed=11, mode=2, nrows=100, cols=12)
    for q in range(3):
        blk = oracle.omega_block(11, 2, rows, q)
        assert np.array_equal(full[:, 4 * q:4 * q + 4], blk)
    # a column subset equals the same columns of the full matrix (adaptive blocks)
    sub = oracle.omega(seed=11, mode=2, nrows=100, cols=range(5, 11))
    assert np.array_equal(sub, full[:, 5:11])
    # different mode or seed -> different stream
    assert not np.allclose(oracle.omega(11, 3, 100, 4), full[:, :4])
    assert not np.allclose(oracle.omega(12, 2, 100, 4), full[:, :4])


def test_box_muller_pairs_closed_form():
    # z0^2 + z1^2 = -2 ln u0 for the first pair (Box-Muller radius), so the
    # transform used the right words in the right order
    rows = np.arange(1000, dtype=np.uint64)
    ctr = np.stack([rows, np.zeros_like(rows), np.zeros_like(rows), np.zeros_like(rows)], axis=1)
    w = oracle.philox4x32_10(ctr, np.array([5, 0], dtype=np.uint64))
    z = oracle.omega_block(5, 0, rows, 0)
    u0 = (w[:, 0].astype(np.float64) + 0.5) * 2.0 ** -32
    u2 = (w[:, 2].astype(np.float64) + 0.5) * 2.0 ** -32
    u1 = (w[:, 1].astype(np.float64) + 0.5) * 2.0 ** -32
    np.testing.assert_allclose(z[:, 0] ** 2 + z[:, 1] ** 2, -2 * np.log(u0), rtol=1e-12)
    np.testing.assert_allclose(z[:, 2] ** 2 + z[:, 3] ** 2, -2 * np.log(u2), rtol=1e-12)
    ang = np.mod(np.arctan2(z[:, 1], z[:, 0]) / (2 * np.pi), 1.0)
    d = np.abs(ang - u1)
    assert np.max(np.minimum(d, 1 - d)) < 1e-12
