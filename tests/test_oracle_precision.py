"""Pins of the oracle's bfloat16 two-piece split and of the bfloat16-sketch
variant of Alg. 1 (the product h h' + h m' + m h')."""
import numpy as np
import torch

import oracle


def _is_bf16(v):
    v = np.asarray(v, dtype=np.float32)
    return np.array_equal(torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy(), v)


def test_split_bf16_hand_values():
    # bfloat16 keeps 8 significant bits: spacing 2^-7 on [1, 2), 2^-6 on [2, 4)
    x = np.array([1.5, 1 + 2.0 ** -7 + 2.0 ** -9, -(3 + 2.0 ** -10), 1 + 2.0 ** -8 + 2.0 ** -17, 0.0,
                  1 + 2.0 ** -7 - 2.0 ** -20])
    h, m = oracle.split_bf16(x)
    assert np.array_equal(h, [1.5, 1 + 2.0 ** -7, -3.0, 1.0, 0.0, 1.0])
    # 1 + 2^-7 - 2^-20 = 1 + (2^-8 + ... + 2^-19) + 2^-20 ... truncated: m keeps 2^-8 .. 2^-15
    assert np.array_equal(m, [0.0, 2.0 ** -9, -(2.0 ** -10), 2.0 ** -8, 0.0, 2.0 ** -7 - 2.0 ** -15])
    rem = x - h - m
    assert np.array_equal(rem, [0.0, 0.0, 0.0, 2.0 ** -17, 0.0, 2.0 ** -15 - 2.0 ** -20])


def test_split_bf16_properties():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(100000), rng.standard_normal(1000) * 1e30,
                        rng.standard_normal(1000) * 1e-30]).astype(np.float32).astype(np.float64)
    h, m = oracle.split_bf16(x)
    rem = x - h - m                                   # exact in float64
    assert _is_bf16(h) and _is_bf16(m)
    # the remainder has at most 8 significant bits (checked where it is a normal float32)
    big = np.abs(x) > 2.0 ** -100
    assert _is_bf16(rem[big])
    # truncation: each piece is the bfloat16 next to its argument towards zero
    assert np.all(np.abs(h) <= np.abs(x)) and np.all(np.sign(h) * np.sign(x) >= 0)
    assert np.all(np.abs(m) <= np.abs(x - h))
    # the next bfloat16 away from zero (magnitude bits + 2^16) lies beyond |x|
    mag = np.abs(h).astype(np.float32).view(np.int32).astype(np.int64)
    nxt = (mag + 0x10000).astype(np.int32).view(np.float32).astype(np.float64)
    assert np.all(nxt > np.abs(x))
    # two pieces leave less than 2^-15 of every normal value
    assert np.all(np.abs(rem) < 2.0 ** -15 * np.abs(x))


def test_sketch_bf16x3_expansion_and_bound():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 200))
    B = oracle.omega(5, 0, 200, 9)
    Y = oracle.sketch_bf16x3(A, B)
    hA, mA = oracle.split_bf16(A)
    hB, mB = oracle.split_bf16(B)
    # operands that are exactly h + m: the sketch is the product less the m m' term
    A2, B2 = hA + mA, hB + mB
    assert np.allclose(oracle.sketch_bf16x3(A2, B2), A2 @ B2 - mA @ mB, rtol=0, atol=1e-13)
    # each product within 2^-13 |x| |y| of the exact one (2 x 2^-15 from the
    # remainders, m m' below 2^-14), plus float64 rounding
    A32, B32 = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    err = np.abs(Y - A32 @ B32)
    assert np.all(err <= 2.0 ** -13 * (np.abs(A32) @ np.abs(B32)) + 1e-12)
    rel = np.linalg.norm(Y - A32 @ B32) / np.linalg.norm(A32 @ B32)
    assert 1e-8 < rel < 1e-4


def test_bf16x3_sketch_variant():
    rng = np.random.default_rng(1)
    X = rng.standard_normal((30, 200))
    Om = oracle.omega(5, 0, 200, 9)
    # operands already bfloat16 values: the variant is the plain algorithm
    Xb, Ob = oracle.split_bf16(X)[0], oracle.split_bf16(Om)[0]
    U1, S1, V1, Q1 = oracle.randsvd(Xb, 6, 3, Ob, sketch=oracle.sketch_bf16x3)
    U2, S2, V2, Q2 = oracle.randsvd(Xb, 6, 3, Ob)
    assert np.array_equal(Q1, Q2) and np.array_equal(U1, U2)
    # general operands: the basis moves by about the sketch's 2^-15 rounding
    _, _, _, Qr = oracle.randsvd(X, 6, 3, Om, sketch=oracle.sketch_bf16x3)
    _, _, _, Qe = oracle.randsvd(X, 6, 3, Om)
    d = np.linalg.norm(Qr @ Qr.T - Qe @ Qe.T, 2)
    assert 1e-9 < d < 1e-3
