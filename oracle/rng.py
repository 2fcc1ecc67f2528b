"""Wiener increments for the oracle (test infrastructure, see package doc).

The paper draws, per Monte-Carlo sample and time step, one normal Wiener
increment with mean 0 and variance dt per space dimension, shared by every
node of every element of that sample (Sec. 5.2 after eq. def_dx; the
Conclusions add that per-node or per-element increments are unstable).  It
names no generator, so the increments come from a counter-based generator:

* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): 10 rounds of the 4x32 Philox S-box with multipliers
  0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9, 0xBB67AE85.
  Counter = (step n, sample s, attempt a, stream id), key = (seed low 32
  bits, seed high 32 bits).
* Uniform pair: k = (r0 >> 6) * 2**26 + (r1 >> 6) (a 52-bit integer) and
  v = (2k + 1) * 2**-52 - 1, exactly representable, in (-1, 1), never 0;
  the second coordinate from (r2, r3) the same way.
* Marsaglia polar method: s = va*va + vb*vb (each product and the sum rounded
  once, no fused multiply-add); accept when s < 1, otherwise retry with the
  attempt counter + 1 (at most 64 attempts; if all fail, both normals are 0).
  Then r = sqrt((-2 * log(s)) / s), za = va * r, zb = vb * r.  One dimension
  uses za; two dimensions use (za, zb) for (x, y).
* log(s) is computed by the method below, not by the C library, so that an
  independent implementation doing the same IEEE operations in the same order
  gets the same bits: write s = m * 2**e with m in [sqrt(1/2), sqrt(2)) (exact),
  t = (m - 1) / (m + 1), log m = 2 atanh t = 2 (t + t * (t^2 * P(t^2))) with
  P(x) = sum_{k=1}^{11} x^(k-1) / (2k+1) in Horner form, and
  log s = e * LN2_HI + (e * LN2_LO + log m) with LN2_HI equal to ln 2 rounded
  to 33 significant bits (so e * LN2_HI is exact) and LN2_LO = ln 2 - LN2_HI
  rounded to float64 (Cody-Waite argument reduction).
"""
import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF
MAX_ATTEMPTS = 64

LN2_HI = float.fromhex("0x1.62e42fef00000p-1")
LN2_LO = float.fromhex("0x1.473de6af278edp-34")
SQRT_HALF = float.fromhex("0x1.6a09e667f3bcdp-1")
# 1/(2k+1), k = 1..11, each the correctly rounded float64 quotient
ATANH_COEF = [np.float64(1.0) / np.float64(2 * k + 1) for k in range(1, 12)]


def _u32(x):
    return np.asarray(x, dtype=np.uint64) & np.uint64(MASK32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 block function; arguments broadcast, returns 4 uint64 arrays of 32-bit words."""
    c0, c1, c2, c3 = (_u32(c) for c in (c0, c1, c2, c3))
    k0, k1 = _u32(k0), _u32(k1)
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    c0, c1, c2, c3, k0, k1 = (a.copy() for a in (c0, c1, c2, c3, k0, k1))
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & np.uint64(MASK32)
            k1 = (k1 + np.uint64(PHILOX_W1)) & np.uint64(MASK32)
        p0 = m0 * c0                      # < 2^64, exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK32)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def own_log(s):
    """Natural log of s > 0 (normal float64) by the fixed recipe in the module doc."""
    s = np.asarray(s, dtype=np.float64)
    m0, e0 = np.frexp(s)                  # s = m0 * 2**e0, m0 in [0.5, 1)
    small = m0 < SQRT_HALF
    m = np.where(small, m0 * 2.0, m0)
    e = np.where(small, e0 - 1, e0).astype(np.float64)
    f = m - 1.0
    den = m + 1.0
    t = f / den
    t2 = t * t
    p = np.full_like(t, ATANH_COEF[10])
    for k in range(9, -1, -1):
        p = ATANH_COEF[k] + t2 * p
    a = t2 * p
    b = t * a
    c = t + b
    lm = 2.0 * c
    a1 = e * LN2_LO
    a2 = a1 + lm
    a3 = e * LN2_HI
    return a3 + a2


def uniform_pair_v(r0, r1, r2, r3):
    """Map four 32-bit words to (va, vb) in (-1, 1), exactly."""
    ka = ((r0 >> np.uint64(6)) << np.uint64(26)) + (r1 >> np.uint64(6))
    kb = ((r2 >> np.uint64(6)) << np.uint64(26)) + (r3 >> np.uint64(6))
    two52 = np.int64(1) << np.int64(52)
    va = ((2 * ka.astype(np.int64) + 1) - two52).astype(np.float64) * 2.0 ** -52
    vb = ((2 * kb.astype(np.int64) + 1) - two52).astype(np.float64) * 2.0 ** -52
    return va, vb


def normal_pair(seed, step, sample, stream=0):
    """Standard normal pair (za, zb) for each sample index (array) at one step."""
    sample = np.atleast_1d(np.asarray(sample, dtype=np.uint64))
    seed = int(seed)
    k0, k1 = seed & MASK32, (seed >> 32) & MASK32
    za = np.zeros(sample.shape, dtype=np.float64)
    zb = np.zeros(sample.shape, dtype=np.float64)
    todo = np.ones(sample.shape, dtype=bool)
    for attempt in range(MAX_ATTEMPTS):
        idx = np.nonzero(todo)[0]
        if idx.size == 0:
            break
        r0, r1, r2, r3 = philox4x32_10(step, sample[idx], attempt, stream, k0, k1)
        va, vb = uniform_pair_v(r0, r1, r2, r3)
        s = va * va + vb * vb
        ok = s < 1.0
        acc = idx[ok]
        s_ok = s[ok]
        lg = own_log(s_ok)
        q = (-2.0 * lg) / s_ok
        r = np.sqrt(q)
        za[acc] = va[ok] * r
        zb[acc] = vb[ok] * r
        todo[acc] = False
    return za, zb
