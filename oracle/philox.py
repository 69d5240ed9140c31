"""Gaussian test matrices Omega drawn from a counter-based stream (oracle side).

The paper draws every Omega with i.i.d. N(0,1) entries (Alg. 1 input, §2.4;
Alg. 2 and Alg. 3, §3.1) and notes that Omega never has to be stored: its
entries can be produced on the fly, column-wise or in blocks (§3.1, remark
after Alg. 2).  It fixes no generator.  One is fixed here so that the HIP
path and this oracle see the same Omega:

* Philox4x32-10, the counter-based generator of Salmon, Moraes, Dror and
  Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).  Ten rounds of
  the 4x32 Philox S-box; each round multiplies words 0 and 2 by the constants
  M0 and M1 (full 64-bit products split into high and low halves), mixes the
  high halves with words 1 and 3 and the round key, and then bumps the key by
  the Weyl constants W0 and W1.
* key     = (seed mod 2^32, seed >> 32)
* counter = (c mod 2^32, c >> 32, floor(k/4), mode)
  where c is the column index of the mode-`mode` unfolding (row-major order over
  the remaining modes, i.e. the row index of Omega) and k the column of Omega.
* each 32-bit output word w becomes u = (w + 1/2) 2^-32 in (0, 1), and the
  Box-Muller transform (1958) turns (u0, u1) and (u2, u3) into the four
  normals for columns 4 floor(k/4) + t, t = 0..3:
      z0 = sqrt(-2 ln u0) cos(2 pi u1),  z1 = sqrt(-2 ln u0) sin(2 pi u1),
      z2 = sqrt(-2 ln u2) cos(2 pi u3),  z3 = sqrt(-2 ln u2) sin(2 pi u3).

Pins (tests/test_oracle_philox.py): the raw 32-bit block function is compared
bit for bit with rocRAND's independent Philox4x32-10 engine (built from its
headers on the host); the normals are checked by moments and a KS test.
"""
import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(counter, key):
    """Philox4x32 with 10 rounds (Salmon et al. 2011).

    counter: (N, 4) array of uint32 words (x0, x1, x2, x3)
    key:     (N, 2) or (2,) array of uint32 words (k0, k1)
    returns  (N, 4) uint32 output words.
    """
    ctr = np.asarray(counter, dtype=np.uint64).reshape(-1, 4)
    key = np.asarray(key, dtype=np.uint64)
    if key.ndim == 1:
        key = np.broadcast_to(key, (ctr.shape[0], 2))
    x0, x1, x2, x3 = (ctr[:, i].copy() for i in range(4))
    k0 = key[:, 0].copy()
    k1 = key[:, 1].copy()
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    w0 = np.uint64(PHILOX_W0)
    w1 = np.uint64(PHILOX_W1)
    for _ in range(10):
        p0 = m0 * x0          # < 2^64, exact in uint64
        p1 = m1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
        k0 = (k0 + w0) & _MASK
        k1 = (k1 + w1) & _MASK
    return np.stack([x0, x1, x2, x3], axis=1).astype(np.uint32)


def _uniform(words):
    """(w + 1/2) 2^-32, exact in float64; strictly inside (0, 1)."""
    return (words.astype(np.float64) + 0.5) * 2.0 ** -32


def box_muller(words):
    """Four normals from four 32-bit words (two Box-Muller pairs), float64."""
    u = _uniform(words)
    r01 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r23 = np.sqrt(-2.0 * np.log(u[:, 2]))
    a1 = 2.0 * np.pi * u[:, 1]
    a3 = 2.0 * np.pi * u[:, 3]
    return np.stack([r01 * np.cos(a1), r01 * np.sin(a1),
                     r23 * np.cos(a3), r23 * np.sin(a3)], axis=1)


def omega_block(seed, mode, rows, q):
    """Normals Omega[c, 4q + t], t = 0..3, for every c in `rows` (1-D int array).

    Returns a (len(rows), 4) float64 array.
    """
    rows = np.asarray(rows, dtype=np.uint64)
    n = rows.shape[0]
    ctr = np.empty((n, 4), dtype=np.uint64)
    ctr[:, 0] = rows & _MASK
    ctr[:, 1] = rows >> np.uint64(32)
    ctr[:, 2] = np.uint64(q)
    ctr[:, 3] = np.uint64(mode)
    seed = int(seed)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    return box_muller(philox4x32_10(ctr, key))


def omega(seed, mode, nrows, cols):
    """Explicit Omega restricted to columns `cols` (an int, meaning range(cols),
    or an iterable of column indices), for rows c = 0..nrows-1.

    This is the matrix Omega_j of Alg. 1-3 (explicitly materialised here; the
    HIP path never stores it)."""
    if isinstance(cols, (int, np.integer)):
        cols = np.arange(int(cols))
    cols = np.asarray(list(cols), dtype=np.int64)
    out = np.empty((nrows, cols.shape[0]), dtype=np.float64)
    rows = np.arange(nrows, dtype=np.uint64)
    cache = {}
    for j, k in enumerate(cols):
        q = int(k) // 4
        if q not in cache:
            cache[q] = omega_block(seed, mode, rows, q)
        out[:, j] = cache[q][:, int(k) % 4]
    return out
