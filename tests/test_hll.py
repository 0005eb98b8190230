"""HyperLogLog: the CPU reference pinned by what the estimator's analysis
fixes (Flajolet et al. 2007: relative standard error 1.04 / sqrt(m), linear
counting for small cardinalities, registers that ignore repeats and merge
by maximum), and the GPU sketch kernels checked against it."""
import numpy as np
import pytest

from oracle import hll

SIGMA = 1.04 / np.sqrt(hll.M)          # 1.6% for 2^12 registers


def _values(ndv, rows, zipf_s, seed):
    """rows values over ndv distinct ids (every id present), uniform or
    Zipf(s)-weighted repeats, ids scattered over the uint32 range."""
    rng = np.random.default_rng(seed)
    ids = rng.choice(np.uint64(0xFFFFFFFE), size=ndv, replace=False).astype(np.uint32)
    if zipf_s == 0:
        extra = rng.integers(0, ndv, size=rows - ndv)
    else:
        w = 1.0 / np.arange(1, ndv + 1) ** zipf_s
        extra = rng.choice(ndv, size=rows - ndv, p=w / w.sum())
    v = np.concatenate([ids, ids[extra]])
    rng.shuffle(v)
    return v


@pytest.mark.parametrize("zipf_s", [0.0, 1.0, 1.5])
@pytest.mark.parametrize("ndv", [20_000, 200_000, 1_000_000])
def test_estimate_within_the_standard_error(ndv, zipf_s):
    errs = []
    for seed in range(6):
        v = _values(ndv, 2 * ndv, zipf_s, seed)
        assert hll.exact_ndv(v) == ndv
        errs.append(hll.estimate(v) / ndv - 1)
    errs = np.array(errs)
    # every sketch within 3 standard errors, and their mean unbiased within
    # 3 standard errors of a mean of six
    assert np.all(np.abs(errs) <= 3 * SIGMA), errs
    assert abs(errs.mean()) <= 3 * SIGMA / np.sqrt(len(errs)), errs


@pytest.mark.parametrize("ndv", [1, 10, 100, 2000])
def test_small_cardinalities_use_linear_counting(ndv):
    v = _values(ndv, 3 * ndv, 0.0, 7)
    # m ln(m / V): with no two values in one register this is m ln(m / (m - n)),
    # within n^2 / m of n; with collisions linear counting is still within a
    # few standard errors
    e = hll.estimate(v)
    assert abs(e - ndv) <= max(1.0, 3 * SIGMA * ndv), (e, ndv)


def test_registers_ignore_repeats_and_merge_by_maximum():
    rng = np.random.default_rng(3)
    a = rng.integers(0, 1 << 31, 50_000).astype(np.uint32)
    b = rng.integers(0, 1 << 31, 70_000).astype(np.uint32)
    ra, rb = hll.registers(a), hll.registers(b)
    assert np.array_equal(hll.registers(np.concatenate([a, a, a[::-1]])), ra)
    assert np.array_equal(hll.registers(np.concatenate([a, b])), np.maximum(ra, rb))
    # every register value lies in 0 .. 64 - p + 1
    assert ra.min() >= 0 and ra.max() <= 64 - hll.P + 1


def test_rho_counts_leading_zeros_from_one():
    # registers from the definition, value by value, on a small sample
    v = np.arange(1000, dtype=np.uint32) * 7919
    h = hll.hash_values(v)
    reg = np.zeros(hll.M, np.int64)
    for x in h.tolist():
        j = x >> (64 - hll.P)
        w = (x << hll.P) & ((1 << 64) - 1)
        rho = 64 - hll.P + 1 if w == 0 else 64 - w.bit_length() + 1
        reg[j] = max(reg[j], rho)
    assert np.array_equal(hll.registers(v), reg)


@pytest.mark.gpu
@pytest.mark.parametrize("zipf_s", [0.0, 1.0])
def test_gpu_sketches_match_the_reference(zipf_s):
    from paper_2501_13051_amd import fv
    import torch
    cols = [_values(ndv, 3 * ndv, zipf_s, 11 + i) for i, ndv in enumerate([50, 3000, 40_000, 250_000, 2_000_000])]
    n = min(len(c) for c in cols)
    cols = [c[:n] for c in cols]
    got_host = fv.hll_ndv(cols)
    got_dev = fv.hll_ndv([torch.from_numpy(c.view(np.int32)).cuda() for c in cols])
    for c, g, d in zip(cols, got_host, got_dev):
        ref = hll.estimate(c)
        exact = hll.exact_ndv(c)
        print(f"ndv {exact}: reference {ref:.3f}, gpu {g:.3f}", flush=True)
        # the same registers give the same estimate up to summation order
        assert abs(g - ref) <= 1e-9 * ref and abs(d - ref) <= 1e-9 * ref
        assert abs(g - exact) <= max(1.0, 3 * SIGMA * exact)


@pytest.mark.gpu
def test_gpu_sketch_batches_and_empty_input():
    from paper_2501_13051_amd import fv
    rng = np.random.default_rng(5)
    cols = [rng.integers(0, k, 100_000).astype(np.uint32) for k in (10, 100, 1000, 10_000, 5, 50, 500, 5000, 7, 70)]
    got = fv.hll_ndv(cols)          # 10 columns: two batches of sketches
    for c, g in zip(cols, got):
        assert abs(g - hll.estimate(c)) <= 1e-9 * max(1.0, g)
    assert np.all(fv.hll_ndv([np.zeros(0, np.uint32)]) == 0)
