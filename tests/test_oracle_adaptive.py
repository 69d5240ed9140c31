"""Pins of the adaptive path (§4, Alg. 4 and Alg. 5) in the oracle."""
import collections
import os

import numpy as np
import pytest

import oracle
from paper_1905_07311_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))


def load_hilbert_table():
    rows = []
    with open(os.path.join(HERE, "golden", "hilbert_adapt.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            I, eps, r1, r2, r3 = line.split()
            rows.append((int(I), float(eps), (int(r1), int(r2), int(r3))))
    return rows


@pytest.mark.parametrize("I,eps,ranks", load_hilbert_table())
def test_table_hilbert_adapt(I, eps, ranks):
    X = inputs.hilbert((I, I, I))
    got = collections.Counter()
    for seed in range(5):
        res = oracle.adaptive_rsthosvd(X, eps, 1, seed=seed, order=[0, 1, 2])
        assert res.rel_err(X) <= eps
        got[tuple(res.ranks)] += 1
    modal = got.most_common(1)[0][0]
    assert modal == ranks, (modal, got)


@pytest.mark.parametrize("b", [1, 3, 8])
@pytest.mark.parametrize("eps", [1e-1, 1e-2, 1e-4])
def test_guarantee(b, eps):
    rng = np.random.default_rng(int(1000 * eps) + b)
    X = inputs.lowrank_tensor(rng, (18, 15, 12), (10, 9, 8), noise=1e-5,
                              core_scale=inputs.graded_scale((10, 9, 8), 0.7))
    for seed in range(3):
        for res in (oracle.adaptive_rsthosvd(X, eps, b, seed=seed),
                    oracle.adaptive_rhosvd(X, eps, b, seed=seed)):
            assert res.rel_err(X) <= eps
            for A in res.factors:
                assert np.allclose(A.T @ A, np.eye(A.shape[1]), atol=1e-12)
            direct = oracle.fro2(X - res.reconstruct())
            assert abs(direct - (oracle.fro2(X) - oracle.fro2(res.core))) <= 1e-11 * oracle.fro2(X)


def _closed_form(lam, eps, d):
    """Ranks and error of adaptive R-STHOSVD on an orthogonally decomposable
    tensor with mode spectra lam, assuming each range finder captures the exact
    dominant subspace: mode 1 needs sum_{k>=r} lam_k^2 <= tau^2, later modes only
    see the terms kept so far."""
    lam2 = lam ** 2
    tau2 = eps ** 2 * lam2.sum() / d
    ranks, margins = [], []
    keep = len(lam)
    for _ in range(d):
        tails = np.array([lam2[r:keep].sum() for r in range(keep + 1)])
        r = int(np.argmax(tails <= tau2))
        margins.append((tau2 / max(tails[r], 1e-300), tails[r - 1] / tau2 if r > 0 else np.inf))
        ranks.append(r)
        keep = min(keep, r)
    err = np.sqrt(lam2[keep:].sum() / lam2.sum())
    return ranks, err, margins


def test_odeco_closed_form():
    d, n, decay, eps = 3, 20, 0.5, 2e-2
    lam = decay ** np.arange(n)
    ranks, err, margins = _closed_form(lam, eps, d)
    for lo, hi in margins:
        assert lo > 1.3 and hi > 1.3          # thresholds not borderline
    rng = np.random.default_rng(11)
    X = inputs.odeco(rng, (n,) * d, decay)
    tally = collections.Counter()
    for b in (1, 2, 4, 8):
        for seed in range(5):
            res = oracle.adaptive_rsthosvd(X, eps, b, seed=seed, order=[0, 1, 2])
            tally[tuple(res.ranks)] += 1
            # the closed form is the optimum: a randomized subspace can only need
            # the same rank or one more, and the error stays within tolerance
            assert all(r <= g <= r + 1 for r, g in zip(ranks, res.ranks))
            e = res.rel_err(X)
            assert err * (1 - 1e-9) <= e <= eps
            if res.ranks == ranks and res.info[0]["qb_cols"] >= ranks[0] + 8:
                # well-oversampled range: the subspaces are the exact dominant ones
                assert abs(e - err) <= 1e-3 * err
    assert tally.most_common(1)[0][0] == tuple(ranks)


def test_per_mode_tolerance_zero_means_uncompressed():
    rng = np.random.default_rng(12)
    X = inputs.lowrank_tensor(rng, (12, 10, 9), (5, 5, 5), noise=1e-4)
    eps = 1e-2
    res = oracle.adaptive_rsthosvd(X, eps, 2, seed=1, eps_per_mode=[eps / np.sqrt(2), 0.0, eps / np.sqrt(2)])
    assert res.factors[1] is None and res.ranks[1] == 10
    assert res.rel_err(X) <= eps


def test_zero_tensor_gives_rank_zero():
    X = np.zeros((6, 7, 8))
    res = oracle.adaptive_rsthosvd(X, 1e-3, 2, seed=0)
    assert res.ranks == [0, 0, 0]
    assert res.core.size == 0


def test_range_exhaustion_inside_a_block():
    # exact multilinear rank (3, 2, 4) and block 8 > rank: the rank-revealing drop
    # must stop the range finder without driving the indicator E negative
    rng = np.random.default_rng(13)
    X = inputs.lowrank_tensor(rng, (15, 14, 13), (3, 2, 4))
    res = oracle.adaptive_rsthosvd(X, 1e-8, 8, seed=2)
    assert res.ranks == [3, 2, 4]
    assert res.rel_err(X) < 1e-12
    for inf in res.info:
        assert inf["E"] > -1e-12 * oracle.fro2(X)
