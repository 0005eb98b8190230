"""The join-cardinality MLP: CPU reference pinned by finite differences,
GPU gradients and BF16 inference checked against it."""
import numpy as np
import pytest

from oracle import mlp


def _data(seed, n=300):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 30, size=(n, 8))
    y = np.log2(1 + np.exp2(X[:, 0] * 0.7 + X[:, 1] * 0.3 - X[:, 3] * 0.2)) / 16
    p = rng.normal(0, 0.3, size=mlp.N_PARAMS)
    return X, y, p


def test_reference_gradient_matches_finite_differences():
    X, y, p = _data(1, n=40)
    _, g = mlp.loss_and_grad(X, y, p)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    eps = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = eps
        fd = (mlp.loss(X, y, p + e) - mlp.loss(X, y, p - e)) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def _f32(bits):
    return np.array([bits], np.uint32).view(np.float32)


# (float32 bits in, BF16 bits out) derived by hand from round-to-nearest-even
# on the 16 dropped bits: below half rounds down, above half up, exactly half
# to the neighbour whose last kept bit is 0.
RNE_CASES = [
    (0x3F800000, 0x3F800000),   # 1.0 is exact
    (0x3F807FFF, 0x3F800000),   # just below the half-way point
    (0x3F808000, 0x3F800000),   # tie, kept last bit 0 (even): stays (round-half-up would go up)
    (0x3F808001, 0x3F810000),   # just above the tie: up (truncation would stay)
    (0x3F818000, 0x3F820000),   # tie, kept last bit 1 (odd): up to even (truncation stays)
    (0xBF818000, 0xBF820000),   # the same tie negative: magnitude rounds up
    (0xBF808000, 0xBF800000),   # negative tie to even: magnitude stays
    (0xBF80FFFF, 0xBF810000),   # negative, above half: magnitude up
    (0x7F7E8000, 0x7F7E0000),   # tie just under the largest BF16: even, stays
    (0x7F7F7FFF, 0x7F7F0000),   # rounds to the largest finite BF16
    (0x7F7F8000, 0x7F800000),   # tie at the largest BF16 (odd): overflows to +inf
    (0x00008000, 0x00000000),   # subnormal tie to even zero
    (0x00018000, 0x00020000),   # subnormal tie, odd: up
    (0x80000000, 0x80000000),   # -0.0 stays
]


@pytest.mark.parametrize("bits_in,bits_out", RNE_CASES, ids=[f"{a:08x}" for a, _ in RNE_CASES])
def test_bf16_rounds_to_nearest_even(bits_in, bits_out):
    got = mlp.bf16(_f32(bits_in)).view(np.uint32)[0]
    assert got == bits_out, f"{bits_in:08x} -> {got:08x}, expected {bits_out:08x}"


def test_bf16_reference_within_rounding_bound():
    X, y, p = _data(3)
    exact = mlp.forward(X, p)[-1]
    approx = mlp.forward_bf16(X, p)
    # every BF16 rounding is a relative error of at most 2^-9; the bound adds
    # them along the absolute-value forward pass (inputs, weights, two layers)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    x = np.abs(X * mlp.IN_SCALE)
    a1 = x @ np.abs(W1).T + np.abs(b1)
    a2 = a1 @ np.abs(W2).T + np.abs(b2)
    a3 = (a2 @ np.abs(W3).T + np.abs(b3))[:, 0]
    bound = 8 * 2.0 ** -9 * a3 + 1e-6
    assert np.all(np.abs(approx - exact) <= bound)


@pytest.mark.gpu
def test_gpu_gradient_matches_reference():
    from paper_2501_13051_amd import fv
    for seed in (4, 5):
        X, y, p = _data(seed, n=500)
        loss, g = fv.mlp_grad(X.astype(np.float32), y.astype(np.float32), p.astype(np.float32))
        ref_loss, ref_g = mlp.loss_and_grad(X.astype(np.float32), y.astype(np.float32), p.astype(np.float32))
        assert abs(loss - ref_loss) <= 1e-4 * max(1.0, ref_loss)
        W = mlp.unpack(ref_g)
        G = mlp.unpack(g)
        for a, b in zip(G, W):   # per-tensor max-norm relative error
            assert np.max(np.abs(a - b)) <= 1e-4 * max(1e-6, np.max(np.abs(b))), (np.max(np.abs(a - b)), np.max(np.abs(b)))


@pytest.mark.gpu
def test_gpu_bf16_inference_matches_reference():
    from paper_2501_13051_amd import fv
    X, y, p = _data(6, n=700)
    got = fv.mlp_predict(X.astype(np.float32), p.astype(np.float32))
    ref = mlp.forward_bf16(X.astype(np.float32), p.astype(np.float32))
    assert np.allclose(got, ref, rtol=1e-4, atol=1e-5)


@pytest.mark.gpu
def test_gpu_training_fits_a_size_law():
    from paper_2501_13051_amd import fv
    X, y, _ = _data(7, n=2000)
    untrained = np.mean((y - np.mean(y)) ** 2)
    params, loss = fv.mlp_train(X.astype(np.float32), y.astype(np.float32), steps=1500, lr=3e-3, seed=11)
    assert loss < 0.05 * untrained, (loss, untrained)
    assert abs(mlp.loss(X, y, params) - loss) <= 1e-3 * max(1.0, loss) + 1e-6
