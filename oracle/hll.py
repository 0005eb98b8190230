"""Reference HyperLogLog distinct-value estimator (numpy, exact integer hashing).

TEST INFRASTRUCTURE ONLY: used by tests to check the GPU sketch kernels.

The sketch is HyperLogLog as stated by Flajolet, Fusy, Gandouet and Meunier
("HyperLogLog: the analysis of a near-optimal cardinality estimation
algorithm", AofA 2007), with the corrections of that paper's practical
version:
  * m = 2^p registers (p = 12 here), all starting at 0;
  * a value x is hashed to 64 bits; the first p bits of the hash (its top
    bits) choose register j, and the register keeps the maximum of rho(w),
    the position of the leftmost 1 in the remaining 64 - p bits (1-based;
    64 - p + 1 when they are all zero);
  * the raw estimate is E = alpha_m m^2 / sum_j 2^-M[j] with
    alpha_m = 0.7213 / (1 + 1.079 / m) (m >= 128);
  * small-range correction: if E <= 5m/2 and V > 0 registers are zero, the
    estimate is linear counting, m ln(m / V).
A 64-bit hash needs no large-range correction.

The hash of a uint32 value v is MurmurHash3's 64-bit finalizer ("fmix64",
Austin Appleby's MurmurHash3, public domain) applied to v + 0x9E3779B97F4A7C15
(floor(2^64 / golden ratio), the increment of SplitMix64), written out here
from that definition.  The standard error of the estimate is about
1.04 / sqrt(m) (1.6% for p = 12).
"""
import numpy as np

P = 12
M = 1 << P
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)


def fmix64(k):
    """MurmurHash3's 64-bit finalizer on a uint64 array (wrapping arithmetic)."""
    k = np.asarray(k, np.uint64).copy()
    with np.errstate(over="ignore"):
        k ^= k >> np.uint64(33)
        k *= np.uint64(0xFF51AFD7ED558CCD)
        k ^= k >> np.uint64(33)
        k *= np.uint64(0xC4CEB9FE1A85EC53)
        k ^= k >> np.uint64(33)
    return k


def hash_values(values):
    v = np.asarray(values, np.uint32).astype(np.uint64)
    with np.errstate(over="ignore"):
        return fmix64(v + _GOLDEN)


def registers(values):
    """The m registers of the sketch of `values` (uint32 array)."""
    h = hash_values(values)
    idx = (h >> np.uint64(64 - P)).astype(np.int64)
    rest = h << np.uint64(P)          # the other 64 - P bits, left-aligned
    # rho: 1 + leading zeros of the remaining bits (64 - P + 1 if all zero)
    rho = np.full(len(h), 64 - P + 1, np.int64)
    nz = rest != 0
    r = rest[nz]
    lz = np.zeros(len(r), np.int64)
    for shift in (32, 16, 8, 4, 2, 1):   # count leading zeros by halving
        s = np.uint64(64 - shift)
        top_clear = (r >> s) == 0
        lz += np.where(top_clear, shift, 0)
        r = np.where(top_clear, r << np.uint64(shift), r)
    rho[nz] = lz + 1
    reg = np.zeros(M, np.int64)
    np.maximum.at(reg, idx, rho)
    return reg


def estimate_from(reg):
    reg = np.asarray(reg, np.int64)
    m = float(M)
    alpha = 0.7213 / (1.0 + 1.079 / m)
    e = alpha * m * m / float(np.sum(np.ldexp(1.0, -reg)))
    zeros = int(np.count_nonzero(reg == 0))
    if e <= 2.5 * m and zeros > 0:
        e = m * np.log(m / zeros)
    return e


def estimate(values):
    """Distinct-value estimate of a uint32 column."""
    return estimate_from(registers(values))


def exact_ndv(values):
    """The exact number of distinct values (sort + unique)."""
    return int(len(np.unique(np.asarray(values, np.uint32))))
