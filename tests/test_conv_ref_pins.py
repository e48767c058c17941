"""Pins of the FP64 convolution reference used to check the network kernels."""
import numpy as np
import pytest
import scipy.signal as ss

from oracle import conv_ref as C


@pytest.mark.parametrize("dil", [1, 2, 3, 10, 27])
def test_forward_equals_scipy_correlation(dil):
    """Dilations up to and beyond the image size (taps that fall wholly in
    the zero padding contribute nothing)."""
    rng = np.random.default_rng(dil)
    B, H, W, Ci, Co = 2, 9, 11, 3, 4
    x = rng.normal(size=(B, H, W, Ci))
    w = rng.normal(size=(Co, 9, Ci))
    b = rng.normal(size=Co)
    _, y = C.conv3x3_fwd(x, w, b, dil, relu=False)
    for bi in range(B):
        for co in range(Co):
            ref = np.full((H, W), b[co])
            for ci in range(Ci):
                k = np.zeros((2 * dil + 1, 2 * dil + 1))
                k[::dil, ::dil] = w[co, :, ci].reshape(3, 3)
                ref += ss.correlate2d(x[bi, :, :, ci], k, mode="same", boundary="fill")
            np.testing.assert_allclose(y[bi, :, :, co], ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("relu", [False, True])
def test_backward_matches_finite_differences(relu):
    rng = np.random.default_rng(5)
    B, H, W, Ci, Co, dil = 1, 6, 7, 2, 3, 2
    x = rng.normal(size=(B, H, W, Ci))
    w = rng.normal(size=(Co, 9, Ci))
    b = rng.normal(size=Co)
    g = rng.normal(size=(B, H, W, Co))

    def loss(x_, w_, b_):
        return float((C.conv3x3_fwd(x_, w_, b_, dil, relu)[1] * g).sum())

    z, _ = C.conv3x3_fwd(x, w, b, dil, relu)
    dx, dw, db = C.conv3x3_bwd(x, z, g, w, dil, relu)
    h = 1e-6
    for (arr, grad) in ((x, dx), (w, dw), (b, db)):
        it = np.nditer(arr, flags=["multi_index"])
        idxs = [it.multi_index for _ in it][:: max(1, arr.size // 25)]
        for ix in idxs:
            a1 = arr.copy(); a1[ix] += h
            a2 = arr.copy(); a2[ix] -= h
            args1 = [a1 if arr is x else x, a1 if arr is w else w, a1 if arr is b else b]
            args2 = [a2 if arr is x else x, a2 if arr is w else w, a2 if arr is b else b]
            fd = (loss(*args1) - loss(*args2)) / (2 * h)
            assert abs(fd - grad[ix]) <= 1e-5 * (1 + abs(fd)), (ix, fd, grad[ix])


def test_adam_first_step_moves_by_lr():
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    w1, m, v = C.adam(w, g, np.zeros(3), np.zeros(3), 0.01, 0.9, 0.999, 1e-12, 1)
    # bias-corrected first step is lr * sign(g)
    np.testing.assert_allclose(w1, w - 0.01 * np.sign(g), rtol=1e-8)


def test_adam_constant_gradient_bias_corrected_steps():
    """Under a constant gradient g the moments are m_t = (1 - b1^t) g and
    v_t = (1 - b2^t) g^2, so the bias-corrected estimates are exactly g and
    g^2 at every step and each step moves w by lr * g / (|g| + eps): with a
    negligible eps, lr * sign(g) at steps 1 to 5 (a wrong power in either
    correction, or no correction, fails from step 2 on)."""
    w0 = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -4.0, 1e-3, -0.02])
    w, m, v = w0.copy(), np.zeros(4), np.zeros(4)
    for step in range(1, 6):
        w, m, v = C.adam(w, g, m, v, 0.01, 0.9, 0.999, 1e-12, step)
        np.testing.assert_allclose(w, w0 - 0.01 * step * np.sign(g), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(m, (1 - 0.9 ** step) * g, rtol=1e-12)
        np.testing.assert_allclose(v, (1 - 0.999 ** step) * g * g, rtol=1e-12)
