"""Pins of the FP64 network reference (oracle/unet.py) against things it does not
compute itself: finite differences, adjoint identities, a library correlation,
closed forms of Adam and of special kernels."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import unet as U


def rnd(shape, seed):
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(shape)


def test_conv_identity_and_shift_kernels():
    x = rnd((2, 5, 6, 3), 0)
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, 1, 1, c] = 1.0
    assert np.array_equal(U.conv3x3(x, w), x)
    # a kernel that reads offset (dy, dx) = (-1, +1) is a periodic shift of the input
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, 0, 2, c] = 1.0
    ref = np.roll(x, shift=(1, -1), axis=(1, 2))
    assert np.array_equal(U.conv3x3(x, w), ref)
    # all-ones kernel on a constant field: 9 C_in times the constant, plus the bias
    xc = np.full((1, 4, 4, 5), 0.25)
    y = U.conv3x3(xc, np.ones((2, 3, 3, 5)), np.array([1.0, -1.0]))
    assert np.allclose(y[..., 0], 9 * 5 * 0.25 + 1) and np.allclose(y[..., 1], 9 * 5 * 0.25 - 1)


def test_conv_matches_library_correlation_with_wrap():
    """Each (out, in) channel pair is scipy's 2-D correlation with periodic boundaries."""
    x = rnd((2, 7, 9, 3), 1)
    w = rnd((4, 3, 3, 3), 2)
    b = rnd(4, 3)
    y = U.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(ndimage.correlate(x[n, :, :, i], w[o, :, :, i], mode="wrap") for i in range(3))
            assert np.allclose(y[n, :, :, o], ref, rtol=0, atol=1e-12)


def test_conv_gradients_against_finite_differences():
    """L = sum(conv(x, w, b) * R) is linear in each of x, w, b, so central differences
    are exact up to rounding."""
    x, w, b, R = rnd((1, 5, 4, 3), 4), rnd((2, 3, 3, 3), 5), rnd(2, 6), rnd((1, 5, 4, 2), 7)
    L = lambda x_, w_, b_: float(np.sum(U.conv3x3(x_, w_, b_) * R))
    gx = U.conv3x3_grad_input(R, w)
    gw, gb = U.conv3x3_grad_weight(x, R)
    h = 1e-3
    for idx in [(0, 0, 0, 0), (0, 4, 3, 2), (0, 2, 1, 1), (0, 0, 3, 0)]:
        e = np.zeros_like(x); e[idx] = h
        assert abs((L(x + e, w, b) - L(x - e, w, b)) / (2 * h) - gx[idx]) < 1e-10
    for idx in [(0, 0, 0, 0), (1, 2, 2, 2), (0, 1, 0, 1), (1, 0, 2, 0)]:
        e = np.zeros_like(w); e[idx] = h
        assert abs((L(x, w + e, b) - L(x, w - e, b)) / (2 * h) - gw[idx]) < 1e-10
    for o in range(2):
        e = np.zeros(2); e[o] = h
        assert abs((L(x, w, b + e) - L(x, w, b - e)) / (2 * h) - gb[o]) < 1e-10


def test_conv_adjoint_identity():
    x, w, g = rnd((2, 6, 8, 4), 8), rnd((5, 3, 3, 4), 9), rnd((2, 6, 8, 5), 10)
    lhs = np.sum(U.conv3x3(x, w) * g)
    rhs = np.sum(x * U.conv3x3_grad_input(g, w))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs) + 1e-12


def test_pool_and_upsample():
    x = rnd((2, 6, 4, 3), 11)
    m = U.maxpool2(x)
    assert m.shape == (2, 3, 2, 3)
    assert m[1, 2, 1, 2] == max(x[1, 4, 2, 2], x[1, 4, 3, 2], x[1, 5, 2, 2], x[1, 5, 3, 2])
    g = rnd(m.shape, 12)
    gx = U.maxpool2_grad(x, g)
    # generic inputs have no ties: finite differences of sum(maxpool(x) g)
    h = 1e-6
    for idx in [(0, 0, 0, 0), (1, 5, 3, 2), (0, 3, 2, 1), (1, 1, 0, 0)]:
        e = np.zeros_like(x); e[idx] = h
        fd = (np.sum(U.maxpool2(x + e) * g) - np.sum(U.maxpool2(x - e) * g)) / (2 * h)
        assert abs(fd - gx[idx]) < 1e-8
    # exact ties go to the first maximum in row-major window order
    t = np.zeros((1, 2, 2, 1))
    gt = U.maxpool2_grad(t, np.ones((1, 1, 1, 1)))
    assert gt[0, 0, 0, 0] == 1 and gt.sum() == 1
    # a tie between (0, 1) and (1, 0) goes to (0, 1), which comes first row by row
    t = np.array([[0.0, 2.0], [2.0, 1.0]]).reshape(1, 2, 2, 1)
    gt = U.maxpool2_grad(t, np.ones((1, 1, 1, 1)))
    assert gt[0, 0, 1, 0] == 1 and gt.sum() == 1
    # upsample: repetition, and its gradient is the adjoint
    u = U.upsample2(m)
    assert u.shape == x.shape and u[0, 3, 1, 2] == m[0, 1, 0, 2]
    gu = rnd(u.shape, 13)
    assert abs(np.sum(u * gu) - np.sum(m * U.upsample2_grad(gu))) < 1e-12


def test_mse_gradient_and_adam_closed_forms():
    p, t = rnd((2, 3, 4), 14), rnd((2, 3, 4), 15)
    loss, g = U.mse(p, t)
    assert loss == pytest.approx(np.mean((p - t) ** 2), rel=1e-15)
    h = 1e-6
    e = np.zeros_like(p); e[1, 2, 3] = h
    fd = (U.mse(p + e, t)[0] - U.mse(p - e, t)[0]) / (2 * h)
    assert abs(fd - g[1, 2, 3]) < 1e-8
    # constant gradient: bias correction makes every step lr * g / (|g| + eps)
    w0 = rnd(5, 16)
    gconst = np.array([0.3, -2.0, 1e-3, -1e-5, 7.0])
    w, m, v = w0.copy(), np.zeros(5), np.zeros(5)
    for t_ in range(1, 6):
        w, m, v = U.adam(w, gconst, m, v, t_, lr=0.01, eps=1e-8)
    ref = w0 - 5 * 0.01 * gconst / (np.abs(gconst) + 1e-8)
    assert np.allclose(w, ref, rtol=0, atol=1e-12)


def test_bf16_rounding():
    assert U.bf16_round(np.array([1.0]))[0] == 1.0
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even gives 1
    assert U.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0
    assert U.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    assert U.bf16_round(np.array([1 + 2 ** -7]))[0] == 1 + 2 ** -7
    assert U.bf16_round(np.array([-3.0e38]))[0] < -3.0e38 * 0.99


def test_unet_gradients_against_finite_differences():
    """Whole network (three levels, small widths) on an 8 x 8 periodic field: analytic
    gradients of the MSE loss against central differences on sampled entries."""
    arch = U.Arch(widths=(3, 4, 5), in_channels=3, used_inputs=3, outputs=2)
    p = U.init_params(arch, seed=3)
    for k in p:
        if k.endswith(".b"):
            p[k] = rnd(p[k].shape, sum(map(ord, k))) * 0.1
    x = rnd((2, 8, 8, 3), 17)
    t = rnd((2, 8, 8, 2), 18)

    def loss(pp, xx):
        return U.mse(U.forward(arch, pp, xx)[0], t)[0]

    out, cache = U.forward(arch, p, x)
    _, dout = U.mse(out, t)
    gr, gx = U.backward(arch, p, cache, dout)
    assert set(gr) == set(p)
    h = 1e-6
    rng = np.random.Generator(np.random.PCG64(19))
    checked = 0
    for k in sorted(p):
        for _ in range(2):
            idx = tuple(int(rng.integers(0, s)) for s in p[k].shape)
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pp[k][idx] += h
            lp = loss(pp, x)
            pp[k][idx] -= 2 * h
            lm = loss(pp, x)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - gr[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, gr[k][idx])
            checked += 1
    for idx in [(0, 0, 0, 0), (1, 7, 3, 1), (0, 4, 5, 0), (1, 2, 6, 2)]:
        e = np.zeros_like(x); e[idx] = h
        fd = (loss(p, x + e) - loss(p, x - e)) / (2 * h)
        assert abs(fd - gx[idx]) <= 1e-6 * max(1.0, abs(fd))
    assert checked == 2 * len(p)


def test_unet_mutations_are_caught():
    """Plausible slips in the reference (a dropped skip gradient, a transposed tap)
    change its gradients by far more than the finite-difference agreement above."""
    arch = U.Arch(widths=(3, 4), in_channels=2, used_inputs=2)
    p = U.init_params(arch, seed=5)
    x, t = rnd((1, 4, 4, 2), 20), rnd((1, 4, 4, 1), 21)
    out, cache = U.forward(arch, p, x)
    _, dout = U.mse(out, t)
    gr, _ = U.backward(arch, p, cache, dout)
    w = p["e0a.w"]
    g = rnd((1, 4, 4, 3), 22)
    good = U.conv3x3_grad_input(g, w)
    bad = U.conv3x3_grad_input(g, w[:, ::-1, ::-1, :])  # taps flipped
    assert np.abs(good - bad).max() > 1e-3


def test_init_scales_are_he_normal():
    """He et al. (2015) normal initialisation: std sqrt(2 / fan_in) with fan_in = 9 C_in for a
    3x3 convolution, zero biases; the head's std is 1/sqrt(C).  Sample std within 3 % on
    the widest layers (tens of thousands of draws each)."""
    arch = U.Arch()
    p = U.init_params(arch, 5)
    for name, ci, co in arch.convs():
        w = p[name + ".w"]
        if w.size >= 20000:
            assert abs(w.std() / np.sqrt(2.0 / (9 * ci)) - 1) < 0.03, name
        assert not p[name + ".b"].any()
    arch1 = U.Arch(widths=(256, 512), outputs=1)
    hw = U.init_params(arch1, 6)["head.w"]
    assert hw.shape == (1, 256) and abs(hw.std() * np.sqrt(256) - 1) < 0.15


def test_head_adds_the_density_and_temperature_channels():
    """The input layout: channel 0 the normalised density, channel 1 the conditioning value
    (the run's reduced temperature), channel 2 the normalised temperature deviation; a
    one-output head is a residual on the density, a two-output head on density and
    temperature, never on the conditioning channel.  With the head's weights and bias
    zero the outputs are those input channels."""
    for outputs, want in ((1, [10.0]), (2, [10.0, 30.0])):
        arch = U.Arch(widths=(8, 16), outputs=outputs)
        p = U.init_params(arch, 7)
        p["head.w"][:] = 0
        x = np.zeros((1, 4, 4, arch.in_channels))
        x[..., 0], x[..., 1], x[..., 2] = 10.0, 20.0, 30.0
        out, _ = U.forward(arch, p, x)
        assert np.array_equal(out[0, 1, 2], np.array(want))
