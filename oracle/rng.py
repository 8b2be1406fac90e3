"""Bit-specified Gaussian test matrix Omega for the oracle (test infrastructure).

The paper only says that Omega is a standard Gaussian matrix (randn(n, b) in
Algorithm 2, randn(n, l~) in Algorithm 4).  To compare a GPU run with this oracle
entry by entry both sides must draw the *same* Omega, so the draw is pinned to a
published counter-based generator and a published Gaussian transform, and each
side implements it on its own:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as
  1, 2, 3", SC'11): 10 rounds of the 4x32 Philox S-box with multipliers
  0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 / 0xBB67AE85.
* Entry Omega(i, 2p+q), q in {0,1}, uses counter (i, p, stream, batch) and key
  (seed mod 2^32, seed div 2^32).  The four output words w0..w3 give two
  uniforms with 52 random bits each:
      u1 = (((w0 << 32 | w1) >> 12) + 1/2) * 2^-52,   u2 likewise from (w2, w3),
  so u1, u2 lie strictly inside (0, 1).
* Box-Muller (Box & Muller 1958): r = sqrt(-2 ln u1), q = 0 takes r cos(2 pi u2),
  q = 1 takes r sin(2 pi u2).
* ln, sqrt, sin and cos are written here from their Taylor / Newton definitions
  with IEEE-754 binary64 +, -, *, / only, in a fixed order (NumPy never fuses a
  multiply and an add), so that any implementation that performs the same
  operation sequence without contraction reproduces the bits:
    - ln x: x = m 2^e with m in [sqrt(1/2), sqrt(2)); s = (m-1)/(m+1);
      ln m = 2 s (1 + s^2/3 + ... + s^22/23) in Horner form; ln x = e ln2 + ln m.
    - sqrt y: initial guess from halving the biased exponent bits, then six
      Newton steps g <- (g + y/g)/2.
    - sin, cos of 2 pi u: quadrant from trunc(4u), fold the remaining fraction
      f to [0, 1/2] by f -> 1 - f (swapping sin and cos), x = f pi/2 in
      [0, pi/4]; sin x = x + x z (S1 + z (S2 + ... + z S8)),
      cos x = 1 + z (C1 + ... + z C8), z = x^2, with S_k = (-1)^k/(2k+1)! and
      C_k = (-1)^k/(2k)!.
"""
from __future__ import annotations

import numpy as np

_MASK32 = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)

LN2 = float.fromhex("0x1.62e42fefa39efp-1")        # nearest binary64 to ln 2
SQRT_HALF = float.fromhex("0x1.6a09e667f3bcdp-1")  # nearest binary64 to sqrt(1/2)
PIO2 = float.fromhex("0x1.921fb54442d18p+0")       # nearest binary64 to pi/2

# 1/(2k+1) for the atanh series, k = 11 .. 1 (Horner order, highest first)
_ATANH_COEF = [1.0 / float(2 * k + 1) for k in range(11, 0, -1)]
# Taylor coefficients, highest order first
_SIN_COEF = [(-1.0) ** k / float(np.prod(np.arange(1, 2 * k + 2, dtype=np.float64)))
             for k in range(8, 0, -1)]
_COS_COEF = [(-1.0) ** k / float(np.prod(np.arange(1, 2 * k + 1, dtype=np.float64)))
             for k in range(8, 0, -1)]


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 bijection; all arguments are uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(v, dtype=np.uint64) & _MASK32 for v in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK32
    for r in range(10):
        if r > 0:
            k0 = (k0 + _W0) & _MASK32
            k1 = (k1 + _W1) & _MASK32
        p0 = c0 * _M0            # 32x32 -> 64-bit product, exact in uint64
        p1 = c2 * _M1
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform52(w_hi, w_lo):
    """Two 32-bit words -> a binary64 strictly inside (0, 1) with 52 random bits."""
    x = ((w_hi << np.uint64(32)) | w_lo) >> np.uint64(12)
    return (x.astype(np.float64) + 0.5) * 2.0 ** -52


def own_log(x):
    """ln x for normal positive binary64 x, from the atanh series (see module doc)."""
    x = np.asarray(x, dtype=np.float64)
    bits = x.view(np.uint64)
    e = ((bits >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1022
    m = ((bits & np.uint64(0x000FFFFFFFFFFFFF)) | np.uint64(1022 << 52)).view(np.float64)
    low = m < SQRT_HALF
    m = np.where(low, m + m, m)
    e = np.where(low, e - 1, e)
    s = (m - 1.0) / (m + 1.0)
    z = s * s
    p = np.full_like(s, _ATANH_COEF[0])
    for c in _ATANH_COEF[1:]:
        p = p * z + c
    p = p * z + 1.0
    lnm = (s + s) * p
    return e.astype(np.float64) * LN2 + lnm


def own_sqrt(y):
    """sqrt y for normal positive binary64 y: exponent-halving guess + 6 Newton steps."""
    y = np.asarray(y, dtype=np.float64)
    g = ((y.view(np.uint64) >> np.uint64(1)) + np.uint64(0x1FF8000000000000)).view(np.float64)
    for _ in range(6):
        g = 0.5 * (g + y / g)
    return g


def own_sincos_2pi(u):
    """(sin 2 pi u, cos 2 pi u) for u in (0, 1), see module doc."""
    u = np.asarray(u, dtype=np.float64)
    v = u * 4.0
    q = v.astype(np.int64)               # truncation; v > 0
    f = v - q.astype(np.float64)         # exact
    swap = f > 0.5
    g = np.where(swap, 1.0 - f, f)       # exact (Sterbenz)
    x = g * PIO2
    z = x * x
    ps = np.full_like(x, _SIN_COEF[0])
    for c in _SIN_COEF[1:]:
        ps = ps * z + c
    sx = x + x * (z * ps)
    pc = np.full_like(x, _COS_COEF[0])
    for c in _COS_COEF[1:]:
        pc = pc * z + c
    cx = 1.0 + z * pc
    sf = np.where(swap, cx, sx)
    cf = np.where(swap, sx, cx)
    sin_t = np.select([q == 0, q == 1, q == 2], [sf, cf, -sf], -cf)
    cos_t = np.select([q == 0, q == 1, q == 2], [cf, -sf, -cf], sf)
    return sin_t, cos_t


def gaussian_pairs(seed: int, stream: int, batch: int, rows, pairs):
    """Box-Muller pair (z0, z1) for every (row, pair) index; arrays broadcast."""
    rows = np.asarray(rows, dtype=np.uint64)
    pairs = np.asarray(pairs, dtype=np.uint64)
    rows, pairs = np.broadcast_arrays(rows, pairs)
    k0 = np.uint64(seed & 0xFFFFFFFF)
    k1 = np.uint64((seed >> 32) & 0xFFFFFFFF)
    w0, w1, w2, w3 = philox4x32_10(rows, pairs, np.uint64(stream), np.uint64(batch), k0, k1)
    u1 = uniform52(w0, w1)
    u2 = uniform52(w2, w3)
    r = own_sqrt(-2.0 * own_log(u1))
    s, c = own_sincos_2pi(u2)
    return r * c, r * s


def gaussian_matrix(seed: int, rows: int, cols: int, row0: int = 0, col0: int = 0,
                    stream: int = 0, batch: int = 0, chunk_rows: int = 4096) -> np.ndarray:
    """Omega[row0:row0+rows, col0:col0+cols] as a C-contiguous float64 array."""
    out = np.empty((rows, cols), dtype=np.float64)
    if rows == 0 or cols == 0:
        return out
    p_lo = col0 // 2
    p_hi = (col0 + cols + 1) // 2
    pidx = np.arange(p_lo, p_hi, dtype=np.uint64)
    for r0 in range(0, rows, chunk_rows):
        r1 = min(rows, r0 + chunk_rows)
        ridx = np.arange(row0 + r0, row0 + r1, dtype=np.uint64)[:, None]
        z0, z1 = gaussian_pairs(seed, stream, batch, ridx, pidx[None, :])
        inter = np.empty((r1 - r0, 2 * (p_hi - p_lo)), dtype=np.float64)
        inter[:, 0::2] = z0
        inter[:, 1::2] = z1
        off = col0 - 2 * p_lo
        out[r0:r1] = inter[:, off:off + cols]
    return out
