"""fv_hll_ndv_noalloc, the sketch entry point that allocates nothing, against
fv_hll_ndv (the allocating entry point with the same kernels): identical
estimates on two calls in a row (the second smaller), under HIP graph capture
with replays, and a clear error past the scratch array's limit."""
import ctypes

import numpy as np
import pytest

from paper_2501_13051_amd import fv

pytestmark = pytest.mark.gpu


def _cols(seed, n_cols, n_rows):
    rng = np.random.default_rng(seed)
    out = []
    for c in range(n_cols):
        hi = int(10 ** (1 + c % 7))
        out.append(rng.integers(0, hi, n_rows).astype(np.uint32))
    return out


def _dev(cols):
    import torch
    return [torch.from_numpy(c.view(np.int32)).cuda() for c in cols]


def _noalloc(cols_dev):
    import torch
    out = torch.full((len(cols_dev),), -1.0, dtype=torch.float64, device="cuda")
    fv.hll_ndv_noalloc(cols_dev, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def test_noalloc_matches_the_allocating_entry_point_twice():
    big = _cols(1, 8, 300_000)
    small = _cols(2, 3, 20_000)          # second call: fewer columns and rows
    for cols in (big, small):
        got = _noalloc(_dev(cols))
        ref = fv.hll_ndv(_dev(cols))
        assert got.shape == ref.shape
        assert np.array_equal(got, ref), (got, ref)
    # and once more at the larger size: nothing of the smaller call is left over
    assert np.array_equal(_noalloc(_dev(big)), fv.hll_ndv(_dev(big)))


def test_noalloc_in_a_captured_graph():
    import torch
    cols = _dev(_cols(3, 5, 100_000))
    ref = fv.hll_ndv(cols)
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    fv.hll_ndv_noalloc(cols, out)        # first call outside the capture (device set-up)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            fv.hll_ndv_noalloc(cols, out, stream=s)
    for rep in range(3):
        out.fill_(-1.0)
        other = fv.hll_ndv(_dev(_cols(10 + rep, 2, 5000)))   # eager work between replays
        assert other.shape == (2,)
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep


def test_noalloc_rejects_too_many_columns_and_empty_input():
    import torch
    cols = _dev(_cols(4, 9, 1000))
    out = torch.zeros(9, dtype=torch.float64, device="cuda")
    with pytest.raises(fv.FvError) as ei:
        fv.hll_ndv_noalloc(cols, out)
    assert ei.value.status == "FV_EINVAL"
    assert "at most" in fv.lib().fv_global_error().decode()
    empty = [torch.zeros(0, dtype=torch.int32, device="cuda")]
    assert np.array_equal(_noalloc(empty), np.zeros(1))
