"""Stochastic rounding of stored populations to BF16 or FP16: a storage option
of the library (the paper computes in double precision and has no such step).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Definition (the contract the library documents for its BF16 storage):

* random bits, counter-based: for node n (linear index, x fastest), the step t
  being computed, the direction pair k (directions 2k and 2k+1 in the library's
  direction order) and the seed,
  h = fmix32(n*0x9E3779B1 + t*0x85EBCA77 + k*0xC2B2AE3D + seed) modulo 2^32;
  direction 2k takes the low 16 bits of h, direction 2k+1 the high 16 bits.
  fmix32 is the 32-bit finalizer of Austin Appleby's MurmurHash3 (SMHasher,
  public domain).
* BF16: a finite FP32 value with bit pattern b and random r in [0, 2^16)
  is stored as the BF16 pattern (b + r) >> 16.  The magnitude therefore rounds
  up with probability equal to its distance above the BF16 value below it, in
  units of the BF16 spacing, so the stored value is unbiased.  Inf stays Inf
  and NaN stays NaN.
* FP16, |v| >= 2^-14 (its normal range): the FP32 bits of |v| plus r >> 3,
  with the 13 fraction bits FP16 lacks cleared, then an exact conversion (Inf
  on overflow).  |v| < 2^-14 (subnormal, spacing 2^-24): the same on
  s = |v| + 2^-14 rounded to FP32 (whose grid in [2^-14, 2^-13] is 2^-37, 13
  bits below the subnormal spacing), then the 2^-14 taken back off exactly.
  Unbiased up to that FP32 rounding of s (at most 2^-38).

Pins (tests/test_oracle_rounding.py): MurmurHash3_x86_32 published test
vectors, whose last step is fmix32 (``murmur3_x86_32`` below exists only to
reach them); exhaustive unbiasedness over all 2^16 random values; bracketing
by the neighbours numpy's float16 gives, sign symmetry and the special
values.
"""
import numpy as np

M32 = 0xFFFFFFFF


def fmix32(h):
    """MurmurHash3's 32-bit finalizer; h a Python int or an integer array."""
    if isinstance(h, (int, np.integer)):
        h = int(h) & M32
        h ^= h >> 16
        h = (h * 0x85EBCA6B) & M32
        h ^= h >> 13
        h = (h * 0xC2B2AE35) & M32
        h ^= h >> 16
        return h
    h = np.asarray(h).astype(np.uint64) & M32
    h ^= h >> np.uint64(16)
    h = (h * np.uint64(0x85EBCA6B)) & np.uint64(M32)
    h ^= h >> np.uint64(13)
    h = (h * np.uint64(0xC2B2AE35)) & np.uint64(M32)
    h ^= h >> np.uint64(16)
    return h.astype(np.uint32)


def _rotl32(x, r):
    return ((x << r) | (x >> (32 - r))) & M32


def murmur3_x86_32(key: bytes, seed: int) -> int:
    """MurmurHash3_x86_32 of a byte string (little-endian blocks), plain Python."""
    c1, c2 = 0xCC9E2D51, 0x1B873593
    h = seed & M32
    nblocks = len(key) // 4
    for i in range(nblocks):
        k = int.from_bytes(key[4 * i:4 * i + 4], "little")
        k = _rotl32((k * c1) & M32, 15)
        h ^= (k * c2) & M32
        h = _rotl32(h, 13)
        h = (h * 5 + 0xE6546B64) & M32
    tail = key[4 * nblocks:]
    if tail:
        k = int.from_bytes(tail, "little")
        k = _rotl32((k * c1) & M32, 15)
        h ^= (k * c2) & M32
    h ^= len(key)
    return fmix32(h)


def random_bits(n_nodes, q, step, seed):
    """The 16-bit random values r[a, n] (a in the library's direction order)."""
    return random_bits_at(np.arange(n_nodes), q, step, seed)


def random_bits_at(nodes, q, step, seed):
    """random_bits at the given linear node indices only: r[a, i] for nodes[i]."""
    n = np.asarray(nodes).astype(np.uint64)
    base = (n * np.uint64(0x9E3779B1) + np.uint64((step * 0x85EBCA77) & M32)
            + np.uint64(seed & M32)) & np.uint64(M32)
    r = np.empty((q, n.size), dtype=np.uint32)
    for k in range((q + 1) // 2):
        h = fmix32((base + np.uint64((k * 0xC2B2AE3D) & M32)) & np.uint64(M32))
        r[2 * k] = h & np.uint32(0xFFFF)
        if 2 * k + 1 < q:
            r[2 * k + 1] = h >> np.uint32(16)
    return r


def stochastic_bf16(v32, r16):
    """BF16 values (as float64) of FP32 values v32 rounded with random r16."""
    v32 = np.asarray(v32, dtype=np.float32)
    b = v32.view(np.uint32).astype(np.uint64)
    finite = (b & 0x7F800000) != 0x7F800000
    out = np.where(finite, b + np.asarray(r16, dtype=np.uint64), b)
    out = (out >> np.uint64(16)) << np.uint64(16)
    res = out.astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(v32), np.nan, res)


def stochastic_f16(v32, r16):
    """FP16 values (as float64) of FP32 values v32 rounded with random r16."""
    v32 = np.asarray(v32, dtype=np.float32)
    r = np.broadcast_to(np.asarray(r16, dtype=np.uint64), v32.shape)
    b = v32.view(np.uint32).astype(np.uint64)
    a = b & np.uint64(0x7FFFFFFF)
    finite = a < 0x7F800000
    sub = a < 0x38800000                         # below FP16's smallest normal, 2^-14
    mag32 = a.astype(np.uint32).view(np.float32)
    with np.errstate(invalid="ignore"):         # Inf / NaN lanes are replaced below
        # FP16 subnormals: offset by 2^-14 (an FP32 addition, rounded to nearest)
        s = np.where(sub, mag32 + np.float32(2.0 ** -14), mag32).astype(np.float32)
        sb = s.view(np.uint32).astype(np.uint64)
        y = ((sb + (r >> np.uint64(3))) & np.uint64(0xFFFFE000)).astype(np.uint32).view(np.float32)
        mag = np.where(sub, y.astype(np.float64) - 2.0 ** -14, y.astype(np.float64))
    with np.errstate(over="ignore"):
        out = np.where(b >> np.uint64(31) != 0, -mag, mag).astype(np.float16).astype(np.float64)
        special = v32.astype(np.float16).astype(np.float64)
    return np.where(finite, out, special)
