"""Pins of the oracle's bfloat16 rounding and of the reduced-precision sketch
variant of Alg. 1."""
import numpy as np
import torch

import oracle


def test_round_bf16_hand_values():
    # bfloat16 keeps 8 significant bits: spacing 2^-7 on [1, 2), 2^-6 on [2, 4)
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 0.75 * 2.0 ** -7, 1 + 1.25 * 2.0 ** -7,
                  -2.0 - 2.0 ** -7, -2.0 - 3 * 2.0 ** -7, 0.0, 3.4e38, 1e-40])
    want = np.array([1.0, 1.0,                 # tie to the even neighbour 1
                     1 + 2.0 ** -6,            # tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
                     1 + 2.0 ** -7, 1 + 2.0 ** -7,
                     -2.0,                     # tie to the even neighbour
                     -2.0 - 2.0 ** -5,         # tie between -2 - 2^-6 (odd) and -2 - 2^-5 (even)
                     0.0, np.inf,              # above the largest finite value + half a step
                     2.0 ** -133])             # subnormal: spacing 2^-133
    assert np.array_equal(oracle.round_bf16(x), want)


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(100000), rng.standard_normal(1000) * 1e30,
                        rng.standard_normal(1000) * 1e-30]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oracle.round_bf16(x), ref)


def test_rounded_sketch_variant():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((30, 200))
    Om = oracle.omega(5, 0, 200, 9)
    # operands already bfloat16 values: the variant is the plain algorithm
    Xb, Ob = oracle.round_bf16(X), oracle.round_bf16(Om)
    U1, S1, V1, Q1 = oracle.randsvd(Xb, 6, 3, Ob, sketch_round=oracle.round_bf16)
    U2, S2, V2, Q2 = oracle.randsvd(Xb, 6, 3, Ob)
    assert np.array_equal(Q1, Q2) and np.array_equal(U1, U2)
    # general operands: the sketch differs from the exact one by about 2^-8
    _, _, _, Qr = oracle.randsvd(X, 6, 3, Om, sketch_round=oracle.round_bf16)
    _, _, _, Qe = oracle.randsvd(X, 6, 3, Om)
    d = np.linalg.norm(Qr @ Qr.T - Qe @ Qe.T, 2)
    assert 1e-5 < d < 0.5
