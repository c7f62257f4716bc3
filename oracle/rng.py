"""Random-number contract of the method, oracle side (test infrastructure).

The paper draws random samples (Section 4.1, "shaking"; Algorithm 1: the
sample S_w of size s_w), random sample sizes (Algorithm 1: s_w uniform in
[s_min, s_max]) and K-means++ candidates (Section 3; Section 5: three
candidate points), but fixes no generator.  The reading taken here, which the
GPU library implements independently from the same published definitions:

* Generator: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random
  numbers: as easy as 1, 2, 3", SC'11).  Block function B(ctr, key) maps a
  256-bit counter and a 128-bit key to four 64-bit words.
* Key of a stream: (seed, (worker << 8) | purpose) with the purposes below.
* u(w)      = (w >> 11) * 2**-53, a double in [0, 1).
* mulhi(w,N) = floor(w * N / 2**64), an integer in [0, N).
* Sampling without replacement: a 4-round balanced Feistel network on
  2h-bit integers, h = max(1, ceil(ceil(log2 m) / 2)), with cycle walking
  into [0, m).  Round r uses the key word K_r = B((g, 0, 0, 0), key)[r] and
  the round function F(R) = mix64(R xor K_r) & (2**h - 1), where mix64 is the
  SplitMix64 output finaliser (Steele, Lea, Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014).  Sample element i is
  pi(i) walked into [0, m); the sample is therefore a set of distinct rows.
"""

import numpy as np

MASK64 = (1 << 64) - 1

# Philox4x64 constants (multipliers and Weyl key increments) from the SC'11 paper.
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B
PHILOX_ROUNDS = 10

# SplitMix64 finaliser constants (Steele, Lea, Flood 2014).
MIX_C1 = 0xBF58476D1CE4E5B9
MIX_C2 = 0x94D049BB133111EB

# Purposes: which draw a stream serves.
PURPOSE_SIZE = 1     # sample-size draw, once per worker and round
PURPOSE_SAMPLE = 2   # the sample S_w of one pass
PURPOSE_KMPP = 3     # K-means++ candidates
PURPOSE_RECALC = 4   # sample used to re-evaluate an incumbent after a size change
PURPOSE_FINAL = 5    # the shared sample of size s_opt used for the final choice
FINAL_WORKER = 0xFFFFFF


def stream_key(seed, worker, purpose):
    """Two 64-bit key words of the stream (seed, worker, purpose)."""
    return (int(seed) & MASK64, ((int(worker) << 8) | int(purpose)) & MASK64)


# --------------------------------------------------------------------------
# Philox4x64-10, scalar form with Python integers (exact, easy to read).
# --------------------------------------------------------------------------
def philox_block_scalar(ctr, key):
    """B(ctr, key): ten Philox4x64 rounds; ctr is 4 ints, key is 2 ints."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(PHILOX_ROUNDS):
        if r > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * x0          # 128-bit products
        p1 = PHILOX_M1 * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0, p1 & MASK64,
                          (p0 >> 64) ^ x3 ^ k1, p0 & MASK64)
    return (x0, x1, x2, x3)


# --------------------------------------------------------------------------
# Philox4x64-10, vectorised over arrays of counters (numpy uint64).
# --------------------------------------------------------------------------
_U32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """(hi, lo) 64-bit halves of the 128-bit product a*b, elementwise (uint64)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.uint64(b)
    a_lo, a_hi = a & _U32, a >> _S32
    b_lo, b_hi = b & _U32, b >> _S32
    p_ll = a_lo * b_lo
    p_lh = a_lo * b_hi
    p_hl = a_hi * b_lo
    p_hh = a_hi * b_hi
    mid = (p_ll >> _S32) + (p_lh & _U32) + (p_hl & _U32)
    hi = p_hh + (p_lh >> _S32) + (p_hl >> _S32) + (mid >> _S32)
    lo = a * b
    return hi, lo


def philox_block(c0, c1, c2, c3, key):
    """Vectorised B(ctr, key): counter words are broadcastable uint64 arrays."""
    shape = np.broadcast_shapes(np.shape(c0), np.shape(c1), np.shape(c2), np.shape(c3))
    x0, x1, x2, x3 = (np.broadcast_to(np.asarray(c, dtype=np.uint64), shape).copy()
                      for c in (c0, c1, c2, c3))
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    with np.errstate(over="ignore"):
        for r in range(PHILOX_ROUNDS):
            if r > 0:
                k0 = (k0 + PHILOX_W0) & MASK64
                k1 = (k1 + PHILOX_W1) & MASK64
            hi0, lo0 = _mulhilo(x0, PHILOX_M0)
            hi1, lo1 = _mulhilo(x2, PHILOX_M1)
            x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1,
                              hi0 ^ x3 ^ np.uint64(k1), lo0)
    return x0, x1, x2, x3


# --------------------------------------------------------------------------
# Conversions of one 64-bit word.
# --------------------------------------------------------------------------
def u01(w):
    """u(w) = (w >> 11) * 2**-53, exactly representable double in [0, 1)."""
    return float(int(w) >> 11) * (2.0 ** -53)


def mulhi(w, n):
    """floor(w * n / 2**64): an unbiased-enough integer in [0, n) for n < 2**63."""
    return (int(w) * int(n)) >> 64


# --------------------------------------------------------------------------
# Feistel sampler.
# --------------------------------------------------------------------------
def mix64(z):
    """SplitMix64 finaliser, elementwise on uint64 arrays."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX_C1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX_C2)
        z = z ^ (z >> np.uint64(31))
    return z


def feistel_half_bits(m):
    """h = max(1, ceil(ceil(log2 m) / 2)); the permuted domain is [0, 4**h) >= [0, m)."""
    m = int(m)
    if m < 1:
        raise ValueError("m must be >= 1")
    lg = (m - 1).bit_length()          # ceil(log2 m) for m >= 1
    return max(1, (lg + 1) // 2)


def feistel_round_keys(key, g):
    """K_0..K_3 = B((g, 0, 0, 0), key)."""
    return philox_block_scalar((g, 0, 0, 0), key)


def feistel_permute(x, h, round_keys):
    """One application of the 4-round Feistel bijection on [0, 4**h), elementwise."""
    mask = np.uint64((1 << h) - 1)
    x = np.asarray(x, dtype=np.uint64)
    left = x >> np.uint64(h)
    right = x & mask
    for r in range(4):
        f = mix64(right ^ np.uint64(round_keys[r])) & mask
        left, right = right, left ^ f
    return (left << np.uint64(h)) | right


def sample_indices(m, s, seed, worker, purpose, g):
    """Indices of a sample of s distinct rows out of m (the 'random sample of size s').

    Element i of the sample is the first value < m on the cycle of the Feistel
    permutation started at i (cycle walking), for i = 0..s-1, in that order.
    """
    m, s = int(m), int(s)
    if not (0 <= s <= m):
        raise ValueError("need 0 <= s <= m")
    h = feistel_half_bits(m)
    rk = feistel_round_keys(stream_key(seed, worker, purpose), g)
    y = feistel_permute(np.arange(s, dtype=np.uint64), h, rk)
    pending = y >= np.uint64(m)
    while pending.any():
        y[pending] = feistel_permute(y[pending], h, rk)
        pending = y >= np.uint64(m)
    return y.astype(np.int64)
