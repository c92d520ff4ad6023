"""GPU parity of the warm-start network kernels (include/unet.h) against the FP64
reference (oracle/unet.py), through the C ABI.

Inputs are bfloat16-representable, so every product on the matrix cores is exact
and the only error is the FP32 accumulation: for a sum of K products the bound
is gamma_K * sum |terms| with gamma_K = K u / (1 - K u), u = 2^-24.  Results
stored as bfloat16 are compared with the reference rounded to bfloat16, allowing
one bfloat16 step where the FP32 result sits at a rounding boundary.

The whole network is checked layer by layer: every tensor one training step
stores is compared with the reference applied to the GPU's own stored inputs of
that step (teacher forcing), to one bfloat16 step plus the accumulation bound.
End to end, the reference runs with bfloat16 rounding at every point where the GPU
stores bfloat16, so only FP32 accumulation order and the rare value that lands on
the other side of a rounding boundary or ReLU gate remain; against the exact FP64
reference (no storage rounding) the difference is reported, not a parity bar.
"""
import numpy as np
import pytest

from oracle import unet as U
from tests.parity_helpers import say

pytestmark = pytest.mark.gpu

U_F32 = 2.0 ** -24


def gamma(k):
    return k * U_F32 / (1 - k * U_F32)


def bf(shape, seed, scale=1.0):
    """bfloat16-representable FP64 values."""
    r = np.random.Generator(np.random.PCG64(seed)).standard_normal(shape) * scale
    return U.bf16_round(r)


def dev_bf16(a):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    assert np.array_equal(t.float().numpy(), np.asarray(a, dtype=np.float32))  # exact: values are bf16
    return t.cuda()


def dev_f32(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def lib():
    from paper_2106_01557_amd import unet
    return unet


def ck(code):
    u = lib()
    assert code == 0, u.library().unet_last_error().decode()


CONV_CASES = [  # N, H, W, Cin, Cout
    (3, 4, 8, 8, 16),      # generic reduction path (C_in = 8), ragged pixel tail, partial channel tile
    (2, 8, 16, 32, 32),    # LDS-staged form, 256 x 32 tiles
    (1, 16, 8, 40, 64),    # C_in not a multiple of 32: chunks straddle taps
    (2, 8, 8, 96, 96),     # C_out = 96: three 32-wide tiles (pixel count below the LDS tile)
    (1, 32, 32, 64, 128),  # LDS-staged form, 128 x 128 tiles
    (1, 16, 16, 64, 64),   # LDS-staged form, 256 x 64 tiles
    (1, 16, 16, 32, 96),   # LDS-staged form, three 32-wide column tiles
    (1, 16, 16, 128, 256), # LDS-staged form, four channel blocks per tap, two column tiles
    (1, 16, 32, 8, 64),    # C_in = 8 halo-tile form (first layer), two column tiles
]


@pytest.mark.parametrize("case", CONV_CASES, ids=lambda c: "x".join(map(str, c)))
def test_conv3x3_forward_fp32_output(case):
    import torch
    N, H, W, ci, co = case
    say(f"case: conv3x3 forward {case}")
    u = lib()
    x, w, b = bf((N, H, W, ci), 1), bf((co, 3, 3, ci), 2, 0.3), bf(co, 3)
    ref = U.conv3x3(x, w, b)
    bound = gamma(9 * ci + 1) * (U.conv3x3(np.abs(x), np.abs(w)) + np.abs(b))
    y = torch.zeros((N, H, W, co), dtype=torch.float32, device="cuda")
    xd, wd, bd = dev_bf16(x), dev_bf16(w), dev_f32(b)  # keep the operands alive until the kernel ran
    ck(u.library().unet_conv3x3_fwd(u.ptr(xd), ci, 0, u.ptr(wd), u.ptr(bd), u.ptr(y), co, 0, None, 0, 0, N, H, W, ci,
                                    co, u.OUT_F32, None))
    err = np.abs(host(y) - ref)
    assert (err <= bound + 1e-30).all(), float((err / (bound + 1e-30)).max())


@pytest.mark.parametrize("N,H,W,ci,co", [(2, 8, 16, 32, 32), (1, 16, 16, 64, 64)], ids=["32to32", "64to64"])
def test_conv3x3_relu_mask_bf16_and_strided_output(N, H, W, ci, co):
    """ReLU and a mask in the epilogue, bfloat16 output written into channels 16 .. 16 +
    C_out - 1 of a buffer whose other channels must stay untouched (one 32-channel block
    with 32 outputs per workgroup; two blocks with 64 outputs per workgroup)."""
    import torch
    say(f"case: conv3x3 relu + mask + strided bf16 output, {ci} -> {co}")
    u = lib()
    ld_in, ld_out = ci + 16, co + 32
    x = bf((N, H, W, ld_in), 4)      # input read from channels 8 .. 8 + C_in - 1
    w, b = bf((co, 3, 3, ci), 5, 0.3), bf(co, 6)
    m = bf((N, H, W, co), 7)
    ref = U.conv3x3(x[..., 8:8 + ci], w, b)
    ref = np.where(m > 0, np.maximum(ref, 0), 0.0)
    y = torch.full((N, H, W, ld_out), 7.0, dtype=torch.bfloat16, device="cuda")
    xd, wd, bd, md = dev_bf16(x), dev_bf16(w), dev_f32(b), dev_bf16(m)
    ck(u.library().unet_conv3x3_fwd(u.ptr(xd), ld_in, 8, u.ptr(wd), u.ptr(bd), u.ptr(y), ld_out, 16, u.ptr(md), co, 0,
                                    N, H, W, ci, co, u.RELU, None))
    got = host(y)
    assert (got[..., :16] == 7.0).all() and (got[..., 16 + co:] == 7.0).all()
    want = U.bf16_round(ref)
    step = np.abs(want) * 2.0 ** -7 + 1e-30
    assert (np.abs(got[..., 16:16 + co] - want) <= step).all()
    assert (got[..., 16:16 + co][ref == 0] == 0).all()


@pytest.mark.parametrize("case", [(2, 8, 16, 32, 32), (1, 16, 16, 96, 32), (2, 8, 8, 64, 128), (2, 16, 16, 64, 128)],
                         ids=lambda c: "x".join(map(str, c)))
def test_conv3x3_input_gradient_by_flipped_weights(case):
    import torch
    N, H, W, ci, co = case
    say(f"case: conv3x3 input gradient {case}")
    u = lib()
    g, w = bf((N, H, W, co), 8), bf((co, 3, 3, ci), 9, 0.3)
    ref = U.conv3x3_grad_input(g, w)
    bound = gamma(9 * co) * U.conv3x3_grad_input(np.abs(g), np.abs(w))
    wd = dev_bf16(w)
    wf = torch.empty_like(wd)
    ck(u.library().unet_flip_weights(u.ptr(wd), u.ptr(wf), co, ci, None))
    dx = torch.zeros((N, H, W, ci), dtype=torch.float32, device="cuda")
    gd = dev_bf16(g)
    ck(u.library().unet_conv3x3_fwd(u.ptr(gd), co, 0, u.ptr(wf), None, u.ptr(dx), ci, 0, None, 0, 0, N, H, W, co, ci,
                                    u.OUT_F32, None))
    err = np.abs(host(dx) - ref)
    assert (err <= bound + 1e-30).all(), float((err / (bound + 1e-30)).max())


@pytest.mark.parametrize("case", [(3, 4, 8, 8, 16), (2, 64, 64, 32, 32), (1, 16, 32, 96, 64), (2, 8, 8, 40, 128),
                                  (2, 64, 64, 8, 32),    # C_in = 8 halo-tile form, 32 output channels, 32 slabs
                                  (1, 16, 32, 8, 64)],   # C_in = 8 halo-tile form, 64 output channels
                         ids=lambda c: "x".join(map(str, c)))
def test_conv3x3_weight_gradient(case):
    """Weight and bias gradients; the 64 x 64 case splits the pixel sum over many slabs."""
    import torch
    N, H, W, ci, co = case
    say(f"case: conv3x3 weight gradient {case}")
    u = lib()
    x, g = bf((N, H, W, ci), 10), bf((N, H, W, co), 11)
    dw_ref, db_ref = U.conv3x3_grad_weight(x, g)
    bw, bb = U.conv3x3_grad_weight(np.abs(x), np.abs(g))
    P = N * H * W
    import ctypes
    nb = ctypes.c_size_t()
    ck(u.library().unet_wgrad_partial_bytes(N, H, W, ci, co, ctypes.byref(nb)))
    part = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dw = torch.zeros(co * 9 * ci, dtype=torch.float32, device="cuda")
    db = torch.zeros(co, dtype=torch.float32, device="cuda")
    xd, gd = dev_bf16(x), dev_bf16(g)
    ck(u.library().unet_conv3x3_wgrad(u.ptr(xd), ci, 0, u.ptr(gd), co, 0, u.ptr(dw), u.ptr(db), u.ptr(part), nb.value,
                                      N, H, W, ci, co, None))
    got_w = host(dw).reshape(co, 3, 3, ci)
    assert (np.abs(got_w - dw_ref) <= gamma(P) * bw + 1e-30).all()
    assert (np.abs(host(db) - db_ref) <= gamma(P) * bb + 1e-30).all()


CAT_CASES = [  # N, H, W, C_x (upsampled from half size), C_skip, C_out
    (2, 32, 32, 64, 32, 32),    # halo-tile form, 32 output channels, three channel blocks
    (1, 32, 32, 128, 64, 64),   # halo-tile form, 64 output channels
    (2, 16, 8, 64, 32, 32),     # LDS-staged form (rows of 8 pixels: no 16 x 16 tiles)
    (3, 8, 8, 32, 16, 16),      # generic form: C_in = 48 (chunks straddle taps), 16 output channels
    (1, 16, 16, 48, 32, 48),    # generic form: C_in = 80
]


def _upcat(low, skip):
    """[upsample2(low) | skip], stored whole (the reference input of the two-tensor calls)."""
    import torch
    up = low.repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)
    return torch.cat([up, skip], dim=3).contiguous()


@pytest.mark.parametrize("case", CAT_CASES, ids=lambda c: "x".join(map(str, c)))
def test_conv_of_upsampled_concatenation_equals_the_stored_concatenation(case):
    """unet_conv3x3_fwd_cat with the input [upsample2(low) | skip] read from the two
    tensors (low at half size) equals unet_conv3x3_fwd on that concatenation stored
    whole, bitwise; and that result against the FP64 reference.  Then the input-gradient
    form: the output split between two tensors equals the whole output, bitwise."""
    import torch
    N, H, W, cx, cs, co = case
    ci = cx + cs
    say(f"case: two-tensor convolution {case}")
    u = lib()
    low, skip = bf((N, H // 2, W // 2, cx), 30), bf((N, H, W, cs), 31)
    w, bias = bf((co, 3, 3, ci), 32, 0.2), bf((co,), 33, 0.1)
    lowd, skipd, wd = dev_bf16(low), dev_bf16(skip), dev_bf16(w)
    biasd = dev_f32(bias)
    cat = _upcat(lowd, skipd)
    y_ref = torch.empty((N, H, W, co), dtype=torch.bfloat16, device="cuda")
    y_cat = torch.full((N, H, W, co), 7.0, dtype=torch.bfloat16, device="cuda")
    ck(u.library().unet_conv3x3_fwd(u.ptr(cat), ci, 0, u.ptr(wd), u.ptr(biasd), u.ptr(y_ref), co, 0, None, 0, 0, N, H,
                                    W, ci, co, u.RELU, None))
    ck(u.library().unet_conv3x3_fwd_cat(u.ptr(lowd), cx, 0, cx, 1, u.ptr(skipd), cs, 0, u.ptr(wd), u.ptr(biasd),
                                        u.ptr(y_cat), co, 0, co, None, 0, 0, None, 0, 0, N, H, W, ci, co, u.RELU,
                                        None))
    torch.cuda.synchronize()
    assert torch.equal(y_cat.view(torch.int16), y_ref.view(torch.int16))
    xin = np.concatenate([np.repeat(np.repeat(low, 2, axis=1), 2, axis=2), skip], axis=3)
    want = U.relu(U.conv3x3(xin, w, bias))
    bound = gamma(9 * ci + 1) * (U.conv3x3(np.abs(xin), np.abs(w)) + np.abs(bias))
    tol = 2.0 ** -7 * np.abs(want) + 2 * bound + 1e-38
    assert (np.abs(host(y_cat) - want) <= tol).all()
    # split output: the gradient convolution from co channels back to the ci of the two branches
    g = dev_bf16(bf((N, H, W, co), 34))
    wf = dev_bf16(bf((ci, 3, 3, co), 35, 0.2))
    whole = torch.empty((N, H, W, ci), dtype=torch.bfloat16, device="cuda")
    ya = torch.full((N, H, W, cx), 3.0, dtype=torch.bfloat16, device="cuda")
    yb = torch.full((N, H, W, cs + 8), 3.0, dtype=torch.bfloat16, device="cuda")  # ld above its channels
    ck(u.library().unet_conv3x3_fwd(u.ptr(g), co, 0, u.ptr(wf), None, u.ptr(whole), ci, 0, None, 0, 0, N, H, W, co, ci,
                                    0, None))
    ck(u.library().unet_conv3x3_fwd_cat(u.ptr(g), co, 0, co, 0, None, 0, 0, u.ptr(wf), None, u.ptr(ya), cx, 0, cx,
                                        u.ptr(yb), cs + 8, 8, None, 0, 0, N, H, W, co, ci, 0, None))
    torch.cuda.synchronize()
    assert torch.equal(ya.view(torch.int16), whole[..., :cx].contiguous().view(torch.int16))
    assert torch.equal(yb[..., 8:].contiguous().view(torch.int16), whole[..., cx:].contiguous().view(torch.int16))
    assert bool((yb[..., :8] == 3.0).all())  # channels below the offset untouched


@pytest.mark.parametrize("case", CAT_CASES + [(2, 16, 8, 64, 32, 64)], ids=lambda c: "x".join(map(str, c)))
def test_weight_gradient_of_upsampled_concatenation_equals_the_stored_concatenation(case):
    """unet_conv3x3_wgrad_cat with the layer input [upsample2(low) | skip] read from the
    two tensors equals unet_conv3x3_wgrad on the concatenation stored whole, bitwise
    (halo-tile, transposing-read and generic forms), and the FP64 reference."""
    import ctypes
    import torch
    N, H, W, cx, cs, co = case
    ci = cx + cs
    say(f"case: two-tensor weight gradient {case}")
    u = lib()
    low, skip, g = bf((N, H // 2, W // 2, cx), 40), bf((N, H, W, cs), 41), bf((N, H, W, co), 42)
    lowd, skipd, gd = dev_bf16(low), dev_bf16(skip), dev_bf16(g)
    cat = _upcat(lowd, skipd)
    nb = ctypes.c_size_t()
    ck(u.library().unet_wgrad_partial_bytes(N, H, W, ci, co, ctypes.byref(nb)))
    out = []
    for two in (False, True):
        part = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        dw = torch.full((co * 9 * ci,), 5.0, dtype=torch.float32, device="cuda")
        db = torch.full((co,), 5.0, dtype=torch.float32, device="cuda")
        if two:
            ck(u.library().unet_conv3x3_wgrad_cat(u.ptr(lowd), cx, 0, cx, 1, u.ptr(skipd), cs, 0, u.ptr(gd), co, 0,
                                                  u.ptr(dw), u.ptr(db), u.ptr(part), nb.value, N, H, W, ci, co, None))
        else:
            ck(u.library().unet_conv3x3_wgrad(u.ptr(cat), ci, 0, u.ptr(gd), co, 0, u.ptr(dw), u.ptr(db), u.ptr(part),
                                              nb.value, N, H, W, ci, co, None))
        torch.cuda.synchronize()
        out.append((dw.clone(), db.clone()))
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    xin = np.concatenate([np.repeat(np.repeat(low, 2, axis=1), 2, axis=2), skip], axis=3)
    dw_ref, db_ref = U.conv3x3_grad_weight(xin, g)
    bw, bb = U.conv3x3_grad_weight(np.abs(xin), np.abs(g))
    P = N * H * W
    assert (np.abs(host(out[1][0]).reshape(co, 3, 3, ci) - dw_ref) <= gamma(P) * bw + 1e-30).all()
    assert (np.abs(host(out[1][1]) - db_ref) <= gamma(P) * bb + 1e-30).all()


@pytest.mark.parametrize("C", [8, 16, 24, 64])
def test_pool_upsample_and_their_gradients(C):
    """Channel counts from one 16-byte group per pixel to eight, including an odd group
    count; ties inside a window in each row and across its rows."""
    import torch
    say(f"case: maxpool / upsample forward and backward, C = {C}")
    u = lib()
    L = u.library()
    N, H, W = 2, 8, 16
    x = bf((N, H, W, C), 12)
    x[0, 0, 0, :] = x[0, 0, 1, :] = 5.0  # an exact tie: the first maximum takes the gradient
    x[1, 2, 3, :] = x[1, 3, 2, :] = 6.0  # top right against bottom left: top right wins
    x[1, 5, 4, :] = x[1, 5, 5, :] = 7.0  # bottom left against bottom right: bottom left wins
    dy = bf((N, H // 2, W // 2, C), 13)
    add = bf((N, H, W, C), 14)
    xd = dev_bf16(x)
    y = torch.empty((N, H // 2, W // 2, C), dtype=torch.bfloat16, device="cuda")
    ck(L.unet_maxpool2_fwd(u.ptr(xd), C, 0, u.ptr(y), C, 0, N, H, W, C, None))
    assert np.array_equal(host(y), U.maxpool2(x))
    dx = torch.empty_like(xd)
    dyd, addd = dev_bf16(dy), dev_bf16(add)
    ck(L.unet_maxpool2_bwd(u.ptr(xd), C, 0, u.ptr(dyd), C, 0, u.ptr(addd), C, 0, u.ptr(dx), C, 0, 1, N, H, W, C, None))
    ref = (U.maxpool2_grad(x, dy) + add) * (x > 0)
    want = U.bf16_round(ref)
    assert (np.abs(host(dx) - want) <= np.abs(want) * 2.0 ** -7 + 1e-30).all()
    for (n, yy, xx) in ((0, 0, 1), (1, 3, 2), (1, 5, 5)):  # tie losers get only `add`
        assert (host(dx)[n, yy, xx] == U.bf16_round(add[n, yy, xx])).all()
    # upsample forward into channels 16..31 of a 32-channel buffer, and back
    s = bf((N, H // 2, W // 2, C), 15)
    big = torch.zeros((N, H, W, 2 * C), dtype=torch.bfloat16, device="cuda")
    sd = dev_bf16(s)
    ck(L.unet_upsample2_fwd(u.ptr(sd), C, 0, u.ptr(big), 2 * C, C, N, H // 2, W // 2, C, None))
    gb = host(big)
    assert np.array_equal(gb[..., C:], U.upsample2(s)) and (gb[..., :C] == 0).all()
    gy = bf((N, H, W, 2 * C), 16)
    gate = bf((N, H // 2, W // 2, C), 17)
    dsm = torch.empty((N, H // 2, W // 2, C), dtype=torch.bfloat16, device="cuda")
    gyd, gated = dev_bf16(gy), dev_bf16(gate)
    ck(L.unet_upsample2_bwd(u.ptr(gyd), 2 * C, C, u.ptr(gated), C, 0, u.ptr(dsm), C, 0, N, H // 2, W // 2, C, None))
    ref = U.upsample2_grad(gy[..., C:]) * (gate > 0)
    want = U.bf16_round(ref)
    assert (np.abs(host(dsm) - want) <= np.abs(want) * 2.0 ** -7 + 1e-30).all()


def test_head_loss_adam_and_conversions():
    import ctypes
    import torch
    say("case: head forward/backward (two outputs), loss, Adam, bf16 conversions")
    u = lib()
    L = u.library()
    N, H, W, C, K = 2, 16, 16, 32, 2
    d = np.maximum(bf((N, H, W, C), 18), 0)
    hw, hb = bf((K, C), 19), np.array([0.125, -0.25])
    rin, tgt = bf((N, H, W, K), 20), bf((N, H, W, K), 21)
    planes = lambda a: np.ascontiguousarray(np.moveaxis(a, 3, 0))  # noqa: E731  [N,H,W,K] -> [K][N,H,W]
    out_ref = U.head(d, hw, hb, rin)
    loss_ref, dout_ref = U.mse(out_ref, tgt)
    nb = ctypes.c_size_t()
    ck(L.unet_head_partial_bytes(N, H, W, C, K, ctypes.byref(nb)))
    part = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dd, hwd, hbd = dev_bf16(d), dev_f32(hw), dev_f32(hb)
    out = torch.empty((K, N, H, W), dtype=torch.float32, device="cuda")
    dout = torch.empty_like(out)
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    rind, tgtd = dev_f32(planes(rin)), dev_f32(planes(tgt))
    ck(L.unet_head_fwd(u.ptr(dd), C, u.ptr(hwd), u.ptr(hbd), u.ptr(rind), u.ptr(tgtd), u.ptr(out), u.ptr(dout),
                       u.ptr(loss), u.ptr(part), nb.value, N, H, W, C, K, None))
    bound = gamma(C + 2) * (np.abs(d) @ np.abs(hw).T + np.abs(hb) + np.abs(rin))
    assert (np.abs(planes(out_ref) - host(out)) <= planes(bound)).all()
    assert host(loss)[0] == pytest.approx(loss_ref, rel=1e-5)
    assert np.allclose(host(dout), planes(dout_ref), rtol=1e-5, atol=1e-9)
    g = torch.empty((N, H, W, C), dtype=torch.bfloat16, device="cuda")
    dhw = torch.empty(K * C, dtype=torch.float32, device="cuda")
    dhb = torch.empty(K, dtype=torch.float32, device="cuda")
    doutd = dev_f32(host(dout))
    ck(L.unet_head_bwd(u.ptr(dd), C, u.ptr(hwd), u.ptr(doutd), u.ptr(g), u.ptr(dhw), u.ptr(dhb), u.ptr(part),
                       nb.value, N, H, W, C, K, None))
    dh = np.moveaxis(host(doutd), 0, 3)  # [N,H,W,K]
    assert np.allclose(host(dhw).reshape(K, C), dh.reshape(-1, K).T @ d.reshape(-1, C), rtol=1e-4, atol=1e-7)
    assert np.allclose(host(dhb), dh.reshape(-1, K).sum(axis=0), rtol=1e-4, atol=1e-7)
    want = U.bf16_round((dh @ hw) * (d > 0))
    acc = gamma(K) * (np.abs(dh) @ np.abs(hw))
    assert (np.abs(host(g) - want) <= np.abs(want) * 2.0 ** -7 + 2 * acc + 1e-30).all()
    # Adam: three steps against the reference
    rng = np.random.Generator(np.random.PCG64(22))
    p0, gs = rng.standard_normal(1000), [rng.standard_normal(1000) for _ in range(3)]
    pd, md, vd = dev_f32(p0), dev_f32(np.zeros(1000)), dev_f32(np.zeros(1000))
    p16 = torch.empty(1000, dtype=torch.bfloat16, device="cuda")
    pr, mr, vr = p0.astype(np.float32).astype(np.float64), np.zeros(1000), np.zeros(1000)
    for t in range(1, 4):
        gd = dev_f32(gs[t - 1])
        ck(L.unet_adam(u.ptr(pd), u.ptr(gd), u.ptr(md), u.ptr(vd), u.ptr(p16), 1000, 1e-2, 0.9, 0.999, 1e-8, t, None))
        pr, mr, vr = U.adam(pr, gs[t - 1].astype(np.float32).astype(np.float64), mr, vr, t, 1e-2)
    assert np.allclose(host(pd), pr, rtol=0, atol=1e-6)
    assert np.array_equal(host(p16), U.bf16_round(host(pd)))
    # conversions
    v = dev_f32(rng.standard_normal(777) * 1e3)
    vb = torch.empty(777, dtype=torch.bfloat16, device="cuda")
    vf = torch.empty(777, dtype=torch.float32, device="cuda")
    ck(L.unet_to_bf16(u.ptr(v), u.ptr(vb), 777, None))
    ck(L.unet_to_f32(u.ptr(vb), u.ptr(vf), 777, None))
    assert np.array_equal(host(vf), U.bf16_round(host(v)))


@pytest.mark.parametrize("case", [(2, 16, 16, 32, 2), (3, 32, 64, 16, 1), (16, 256, 256, 32, 2), (1, 8, 8, 64, 2)],
                         ids=lambda c: "x".join(map(str, c)))
def test_head_train_against_the_reference_and_the_two_passes(case):
    """unet_head_train (forward and backward of the head in one pass) against the FP64
    reference (outputs within the FP32 bound of their sums, loss, dout, the gated
    gradient within a bfloat16 step, weight and bias gradients) and against
    unet_head_fwd + unet_head_bwd, which sum each output in another order: agreement to
    FP32 rounding.  The 16 x 256^2 case is the training batch (several pixels per thread,
    2048 workgroups); the others leave threads without pixels."""
    import ctypes
    import torch
    N, H, W, C, K = case
    say(f"case: fused head {case}")
    u = lib()
    L = u.library()
    d = bf((N, H, W, C), 50)                        # both signs: the ReLU gate is exercised
    hw, hb = bf((K, C), 51), bf((K,), 52, 0.5)
    rin, tgt = bf((N, H, W, K), 53), bf((N, H, W, K), 54)
    planes = lambda a: np.ascontiguousarray(np.moveaxis(a, 3, 0))  # noqa: E731
    nb = ctypes.c_size_t()
    ck(L.unet_head_partial_bytes(N, H, W, C, K, ctypes.byref(nb)))
    dd, hwd, hbd = dev_bf16(d), dev_f32(hw), dev_f32(hb)
    rind, tgtd = dev_f32(planes(rin)), dev_f32(planes(tgt))
    res = []
    for fused in (False, True):
        part = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        out = torch.empty((K, N, H, W), dtype=torch.float32, device="cuda")
        dout = torch.empty_like(out)
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        g = torch.empty((N, H, W, C), dtype=torch.bfloat16, device="cuda")
        dhw = torch.empty(K * C, dtype=torch.float32, device="cuda")
        dhb = torch.empty(K, dtype=torch.float32, device="cuda")
        if fused:
            ck(L.unet_head_train(u.ptr(dd), C, u.ptr(hwd), u.ptr(hbd), u.ptr(rind), u.ptr(tgtd), u.ptr(out),
                                 u.ptr(dout), u.ptr(loss), u.ptr(g), u.ptr(dhw), u.ptr(dhb), u.ptr(part), nb.value,
                                 N, H, W, C, K, None))
        else:
            ck(L.unet_head_fwd(u.ptr(dd), C, u.ptr(hwd), u.ptr(hbd), u.ptr(rind), u.ptr(tgtd), u.ptr(out),
                               u.ptr(dout), u.ptr(loss), u.ptr(part), nb.value, N, H, W, C, K, None))
            ck(L.unet_head_bwd(u.ptr(dd), C, u.ptr(hwd), u.ptr(dout), u.ptr(g), u.ptr(dhw), u.ptr(dhb), u.ptr(part),
                               nb.value, N, H, W, C, K, None))
        res.append({k: host(v) for k, v in dict(out=out, dout=dout, loss=loss, g=g, dhw=dhw, dhb=dhb).items()})
    two, one = res
    out_ref = U.head(d, hw, hb, rin)
    loss_ref, dout_ref = U.mse(out_ref, tgt)
    P = N * H * W
    bound = planes(gamma(C + 2) * (np.abs(d) @ np.abs(hw).T + np.abs(hb) + np.abs(rin)))
    assert (np.abs(planes(out_ref) - one["out"]) <= bound).all()
    assert one["loss"][0] == pytest.approx(loss_ref, rel=1e-5)
    # dout = 2 (out - target) / (K P): the output's error carries over, scaled
    dtol = 2.0 / (K * P) * bound * 1.001 + 4 * 2.0 ** -24 * np.abs(planes(dout_ref)) + 1e-30
    assert (np.abs(one["dout"] - planes(dout_ref)) <= dtol).all()
    dh = np.moveaxis(one["dout"], 0, 3)
    want = U.bf16_round((dh @ hw) * (d > 0))
    acc = gamma(K) * (np.abs(dh) @ np.abs(hw))
    assert (np.abs(one["g"] - want) <= np.abs(want) * 2.0 ** -7 + 2 * acc + 1e-30).all()
    wref = dh.reshape(-1, K).T @ d.reshape(-1, C)
    wbound = gamma(P) * (np.abs(dh).reshape(-1, K).T @ np.abs(d).reshape(-1, C))
    assert (np.abs(one["dhw"].reshape(K, C) - wref) <= wbound + 1e-30).all()
    bbound = gamma(P) * np.abs(dh).reshape(-1, K).sum(axis=0)
    assert (np.abs(one["dhb"] - dh.reshape(-1, K).sum(axis=0)) <= bbound + 1e-30).all()
    # against the two separate passes: each within its bound of the exact values, and
    # what follows from dout within the effect of the two douts' difference
    assert (np.abs(one["out"] - two["out"]) <= 2 * bound).all()
    assert (np.abs(one["dout"] - two["dout"]) <= 2 * dtol).all()
    assert one["loss"][0] == pytest.approx(two["loss"][0], rel=1e-5)
    ddiff = np.abs(np.moveaxis(one["dout"] - two["dout"], 0, 3)).reshape(-1, K)
    assert (np.abs(one["dhw"] - two["dhw"]).reshape(K, C) <= 2 * wbound + ddiff.T @ np.abs(d).reshape(-1, C)
            + 1e-30).all()
    assert (np.abs(one["dhb"] - two["dhb"]) <= 2 * bbound + ddiff.sum(axis=0) + 1e-30).all()
    gdiff = (ddiff @ np.abs(hw)).reshape(N, H, W, C)
    step = np.maximum(np.abs(two["g"]), np.abs(one["g"])) * 2.0 ** -7
    assert (np.abs(one["g"] - two["g"]) <= step + 2 * acc + gdiff + 1e-30).all()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _cos(a, b):
    a, b = a.ravel(), b.ravel()
    return float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30))


TS = 0.1  # temperature normalisation of the network (theta = (T / T0 - 1) / TS)


def _net_case(widths, hw, fuse_2x2=True):
    import torch
    from paper_2106_01557_amd import unet
    net = unet.UNet(widths=widths, seed=1, fuse_2x2=fuse_2x2)
    arch = U.Arch(widths=widths, in_channels=8, used_inputs=3, outputs=2)
    p = U.init_params(arch, seed=2)
    p = {k: U.bf16_round(v) for k, v in p.items()}
    for k in p:
        if k.endswith(".b"):
            p[k] = U.bf16_round(np.random.Generator(np.random.PCG64(len(k))).standard_normal(p[k].shape) * 0.05)
    net.load_params(p)
    N = 2
    rng = np.random.Generator(np.random.PCG64(3))
    yy, xx = np.meshgrid(np.arange(hw), np.arange(hw), indexing="ij")
    rho = np.stack([0.3 + 0.2 * np.sin(2 * np.pi * (xx + 3 * n) / hw) * np.cos(2 * np.pi * yy / hw) for n in range(N)])
    rho += 0.01 * rng.standard_normal(rho.shape)
    T0 = np.array([0.07, 0.08])
    Tf = T0[:, None, None] * (1 + 0.02 * np.cos(2 * np.pi * (yy + xx) / hw) + 0.002 * rng.standard_normal(rho.shape))
    tgt = rho + 0.05 * rng.standard_normal(rho.shape)
    tgtT = Tf * (1 + 0.01 * rng.standard_normal(rho.shape))
    rv, rl, cond = np.array([0.02, 0.03]), np.array([0.31, 0.29]), np.array([0.05, -0.1])
    T = lambda a: torch.as_tensor(a, dtype=torch.float64).cuda()  # noqa: E731
    args = [T(a) for a in (rho, Tf, rv, rl, T0, cond, tgt, tgtT)]
    out, loss = net.forward(*args)
    grads = net.backward()
    nu = lambda r: (r - rv[:, None, None]) / (rl - rv)[:, None, None]  # noqa: E731
    th = lambda t: (t / T0[:, None, None] - 1) / TS  # noqa: E731
    x = np.zeros((N, hw, hw, 8))
    x[..., 0] = U.bf16_round(nu(rho))
    x[..., 1] = U.bf16_round(np.broadcast_to(cond[:, None, None], (N, hw, hw)))
    x[..., 2] = U.bf16_round(th(Tf))
    f32 = lambda a: a.astype(np.float32).astype(np.float64)  # noqa: E731
    rin = np.stack([f32(nu(rho)), f32(th(Tf))], axis=3)
    tn = np.stack([f32(nu(tgt)), f32(th(tgtT))], axis=3)
    return net, arch, p, x, rin, tn, out, loss, grads


def _within_bf16(got, want, acc_bound, name):
    """got (bfloat16 from FP32) against the FP64 value: one bfloat16 step of either plus
    twice the FP32 accumulation bound (for values near a rounding boundary or zero)."""
    tol = 2.0 ** -7 * np.maximum(np.abs(want), np.abs(got)) + 2 * acc_bound + 1e-38
    bad = np.abs(got - want) > tol
    assert not bad.any(), (name, int(bad.sum()), float(np.abs(got - want).max()))


@pytest.mark.parametrize("widths,hw", [((16, 32, 48), 16), ((32, 64, 128, 256), 32)], ids=["small", "full"])
def test_unet_every_layer_teacher_forced(widths, hw):
    """Each stored GPU tensor of one training step against the reference applied to the
    GPU's own stored inputs of that step (forward activations, the head, every
    activation gradient and every parameter gradient), with the strides and channel
    offsets the network really uses."""
    say(f"case: U-Net widths {widths} on {hw}x{hw}, every layer teacher-forced")
    # the separate 2x2 passes, so that every intermediate tensor is stored (the fused
    # forms are bitwise the same: test_fused_2x2_passes_equal_the_separate_passes)
    net, arch, p, x, rin, tn, out, loss, grads = _net_case(widths, hw, fuse_2x2=False)
    b = {k: host(v) for k, v in net.buf.items() if k not in ("wpart", "hpart")}
    L, wd = len(widths), widths
    ab = lambda a: np.abs(a)

    def conv_check(name, xin, w, bias, got, gate=None, relu_=True):
        k = 9 * xin.shape[3] + 1
        want = U.conv3x3(xin, w, bias)
        bound = gamma(k) * (U.conv3x3(ab(xin), ab(w)) + (ab(bias) if bias is not None else 0))
        if relu_:
            want = U.relu(want)
        if gate is not None:
            want = want * (gate > 0)
        _within_bf16(got, want, bound, name)

    def dgrad_check(name, g, w, got, gate=None):
        want = U.conv3x3_grad_input(g, w)
        bound = gamma(9 * g.shape[3]) * U.conv3x3_grad_input(ab(g), ab(w))
        if gate is not None:
            want = want * (gate > 0)
        _within_bf16(got, want, bound, name)

    def wgrad_check(name, xin, g):
        dw, db = U.conv3x3_grad_weight(xin, g)
        bw, bb = U.conv3x3_grad_weight(ab(xin), ab(g))
        P = g.shape[0] * g.shape[1] * g.shape[2]
        gw = host(grads[name + ".w"]).reshape(dw.shape)
        assert (np.abs(gw - dw) <= gamma(P) * bw + 1e-38).all(), name
        assert (np.abs(host(grads[name + ".b"]) - db) <= gamma(P) * bb + 1e-38).all(), name

    # forward
    assert np.array_equal(b["x0"], x)
    inp = b["x0"]
    for lvl in range(L):
        conv_check(f"e{lvl}a", inp, p[f"e{lvl}a.w"], p[f"e{lvl}a.b"], b[f"e{lvl}a"])
        conv_check(f"e{lvl}b", b[f"e{lvl}a"], p[f"e{lvl}b.w"], p[f"e{lvl}b.b"], b[f"e{lvl}b"])
        if lvl < L - 1:
            assert np.array_equal(b[f"pool{lvl}"], U.maxpool2(b[f"e{lvl}b"]))
            inp = b[f"pool{lvl}"]
    low = b[f"e{L - 1}b"]
    cats = {}
    for lvl in reversed(range(L - 1)):
        # the decoder input [upsample2(lower level) | skip], never stored on the GPU
        cat = cats[lvl] = np.concatenate([U.upsample2(low), b[f"e{lvl}b"]], axis=3)
        conv_check(f"d{lvl}a", cat, p[f"d{lvl}a.w"], p[f"d{lvl}a.b"], b[f"d{lvl}a"])
        conv_check(f"d{lvl}b", b[f"d{lvl}a"], p[f"d{lvl}b.w"], p[f"d{lvl}b.b"], b[f"d{lvl}b"])
        low = b[f"d{lvl}b"]
    gout = np.moveaxis(b["out"], 0, 3)
    assert np.array_equal(np.moveaxis(b["rin"], 0, 3), rin)
    assert np.array_equal(np.moveaxis(b["target"], 0, 3), tn)
    want = U.head(low, p["head.w"], p["head.b"], rin)
    bound = gamma(wd[0] + 2) * (ab(low) @ ab(p["head.w"]).T + ab(p["head.b"]) + ab(rin))
    assert (np.abs(gout - want) <= bound + 1e-38).all()
    assert host(loss)[0] == pytest.approx(np.mean((gout - tn) ** 2), rel=1e-5)
    # backward
    dout = np.moveaxis(b["dout"], 0, 3)
    assert np.allclose(dout, 2 * (gout - tn) / dout.size, rtol=1e-5, atol=1e-12)
    want = U.relu_grad(dout @ p["head.w"], b["d0b"])
    _within_bf16(b["gd0b"], want, gamma(2) * (ab(dout) @ ab(p["head.w"])), "head gradient")
    assert np.allclose(host(grads["head.w"]).reshape(2, -1), dout.reshape(-1, 2).T @ b["d0b"].reshape(-1, wd[0]),
                       rtol=1e-4, atol=1e-9)
    for lvl in range(L - 1):
        cu, c = wd[lvl + 1], wd[lvl]
        wgrad_check(f"d{lvl}b", b[f"d{lvl}a"], b[f"gd{lvl}b"])
        dgrad_check(f"dgrad d{lvl}b", b[f"gd{lvl}b"], p[f"d{lvl}b.w"], b[f"gd{lvl}a"], gate=b[f"d{lvl}a"])
        wgrad_check(f"d{lvl}a", cats[lvl], b[f"gd{lvl}a"])
        dcat = np.concatenate([b[f"dup{lvl}"], b[f"dskip{lvl}"]], axis=3)
        dgrad_check(f"dgrad d{lvl}a", b[f"gd{lvl}a"], p[f"d{lvl}a.w"], dcat)
        lowv, dlow = (b[f"d{lvl + 1}b"], b[f"gd{lvl + 1}b"]) if lvl + 1 < L - 1 else (b[f"e{L - 1}b"], b[f"ge{L - 1}b"])
        want = U.relu_grad(U.upsample2_grad(b[f"dup{lvl}"]), lowv)
        _within_bf16(dlow, want, gamma(4) * U.upsample2_grad(ab(b[f"dup{lvl}"])), f"upsample grad {lvl}")
    for lvl in reversed(range(L)):
        c = wd[lvl]
        if lvl < L - 1:
            eb = b[f"e{lvl}b"]
            want = U.relu_grad(U.maxpool2_grad(eb, b[f"dpool{lvl}"]) + b[f"dskip{lvl}"], eb)
            _within_bf16(b[f"ge{lvl}b"], want, gamma(2) * ab(want), f"pool grad {lvl}")
        wgrad_check(f"e{lvl}b", b[f"e{lvl}a"], b[f"ge{lvl}b"])
        dgrad_check(f"dgrad e{lvl}b", b[f"ge{lvl}b"], p[f"e{lvl}b.w"], b[f"ge{lvl}a"], gate=b[f"e{lvl}a"])
        if lvl > 0:
            wgrad_check(f"e{lvl}a", b[f"pool{lvl - 1}"], b[f"ge{lvl}a"])
            dgrad_check(f"dgrad e{lvl}a", b[f"ge{lvl}a"], p[f"e{lvl}a.w"], b[f"dpool{lvl - 1}"])
        else:
            wgrad_check("e0a", b["x0"], b["ge0a"])


@pytest.mark.parametrize("widths,hw,bars,exact_bars",
                         [((16, 32, 48), 16, (2e-3, 1e-2, 0.9999), (1.2e-2, 6e-2, 0.998)),
                          ((32, 64, 128, 256), 32, (3e-2, 1.5e-1, 0.99), (1.2e-2, 6e-2, 0.998))],
                         ids=["small", "full"])
def test_unet_end_to_end_against_reference(widths, hw, bars, exact_bars):
    """One training step end to end, first against the plain FP64 reference (no storage
    rounding anywhere): the GPU stores activations and their gradients in bfloat16, so the
    outputs may differ by a few bfloat16 steps relative (measured 4e-3 to 6e-3 relative L2
    on the outputs and 2e-2 to 3e-2 on the gradients of the full network), held at twice
    that.  Then against the reference with the GPU's bfloat16 storage points: the
    per-layer test above is the parity check; here the small network must agree to
    accumulation level, while in the deep one the rare values that fall on the other side
    of a bfloat16 rounding boundary or of a ReLU gate propagate through eighteen layers
    (measured: outputs 7e-3, gradients up to about 5e-2 relative L2), hence the wider bars."""
    out_bar, grad_bar, cos_bar = bars
    say(f"case: U-Net widths {widths} on {hw}x{hw}, end to end")
    net, arch, p, x, rin, tn, out, loss, grads = _net_case(widths, hw)
    o = np.moveaxis(host(out), 0, 3)
    got = {k: host(gv) for k, gv in grads.items()}
    gl = host(loss)[0]
    ro, cache = U.forward(arch, p, x, rin=rin)
    lref, dref = U.mse(ro, tn)
    gref, _ = U.backward(arch, p, cache, dref)
    r_exact = _rel(o - rin, ro - rin)
    worst_exact = max(_rel(got[k].reshape(gref[k].shape), gref[k]) for k in gref)
    say(f"  vs exact FP64: out rel {r_exact:.2e}, worst gradient rel {worst_exact:.2e}")
    eo, eg, ec = exact_bars
    assert r_exact < eo
    for k in gref:
        gg = got[k].reshape(gref[k].shape)
        assert _rel(gg, gref[k]) < eg and _cos(gg, gref[k]) > ec, (k, _rel(gg, gref[k]))
    ro, cache = U.forward(arch, p, x, store=U.bf16_round, rin=rin)
    lref, dref = U.mse(ro, tn)
    gref, _ = U.backward(arch, p, cache, dref, store=U.bf16_round)
    r_out = _rel(o - rin, ro - rin)
    worst = max(_rel(got[k].reshape(gref[k].shape), gref[k]) for k in gref)
    say(f"  vs bf16-storage reference: out rel {r_out:.2e}, worst gradient rel {worst:.2e}, "
        f"loss {gl:.6e} vs {lref:.6e}")
    assert r_out < out_bar
    assert gl == pytest.approx(lref, rel=out_bar)
    for k in gref:
        gg = got[k].reshape(gref[k].shape)
        assert _rel(gg, gref[k]) < grad_bar and _cos(gg, gref[k]) > cos_bar, (k, _rel(gg, gref[k]))


def test_weight_gradients_on_their_own_streams_equal_one_stream():
    """The weight gradients and their reductions run on streams of their own (one or two,
    layer by layer in turn) beside the input gradients.  Over three training steps
    (forward, backward, Adam) of the full network on four 64 x 64 problems, every loss,
    gradient and updated parameter is bitwise the same as with every kernel on one
    stream: the kernels' sums are in a fixed order, so any difference would be a missing
    dependency between the streams."""
    import torch
    from paper_2106_01557_amd import unet
    say("case: U-Net widths (32, 64, 128, 256), 4 x 64 x 64, weight gradients on 0, 1 and 2 streams of their own")
    N, hw = 4, 64
    nets = [unet.UNet(widths=(32, 64, 128, 256), seed=5, wgrad_streams=k) for k in (0, 1, 2)]
    assert nets[0].wstreams == [nets[0].stream] and len(nets[2].wstreams) == 2
    assert all(st is not nets[2].stream for st in nets[2].wstreams)
    rng = np.random.Generator(np.random.PCG64(8))
    yy, xx = np.meshgrid(np.arange(hw), np.arange(hw), indexing="ij")
    rho = np.stack([0.3 + 0.25 * np.tanh((12 + n - np.hypot(xx - 32, yy - 32)) / 2) for n in range(N)])
    rho += 0.01 * rng.standard_normal(rho.shape)
    T0 = np.array([0.07, 0.075, 0.08, 0.085])
    Tf = T0[:, None, None] * (1 + 0.002 * rng.standard_normal(rho.shape))
    tgt = rho + 0.02 * rng.standard_normal(rho.shape)
    rv, rl, cond = np.full(N, 0.02), np.full(N, 0.55), np.linspace(-0.1, 0.1, N)
    T = lambda a: torch.as_tensor(a, dtype=torch.float64).cuda()  # noqa: E731
    args = [T(a) for a in (rho, Tf, tgt, Tf, rv, rl, T0, cond)]
    for step in range(3):
        losses = [host(net.train_step(*args)).copy() for net in nets]
        torch.cuda.synchronize()
        for i, other in enumerate(nets[1:], 1):
            assert np.array_equal(losses[0], losses[i]), step
            assert torch.equal(nets[0].gflat, other.gflat), step
            assert torch.equal(nets[0].flat, other.flat), step
            assert torch.equal(nets[0].w16flat, other.w16flat), step
    assert float(nets[2].gflat.abs().max()) > 0


def test_fused_2x2_passes_equal_the_separate_passes():
    """The encoder's 2x2 pooling in the epilogue of the convolution before it, and the
    upsampling's gradient in the epilogue of the decoder's input gradient: three
    training steps of the full network on four 64 x 64 problems (fused at the 64, 32 and
    16 levels) are bitwise those of the separate passes."""
    import torch
    from paper_2106_01557_amd import unet
    say("case: U-Net widths (32, 64, 128, 256), 4 x 64 x 64, fused against separate 2x2 passes")
    N, hw = 4, 64
    nets = [unet.UNet(widths=(32, 64, 128, 256), seed=6, fuse_2x2=f) for f in (False, True)]
    rng = np.random.Generator(np.random.PCG64(9))
    yy, xx = np.meshgrid(np.arange(hw), np.arange(hw), indexing="ij")
    rho = np.stack([0.3 + 0.25 * np.tanh((10 + 2 * n - np.hypot(xx - 30, yy - 34)) / 2) for n in range(N)])
    rho += 0.01 * rng.standard_normal(rho.shape)
    T0 = np.array([0.07, 0.075, 0.08, 0.085])
    Tf = T0[:, None, None] * (1 + 0.002 * rng.standard_normal(rho.shape))
    tgt = rho + 0.02 * rng.standard_normal(rho.shape)
    rv, rl, cond = np.full(N, 0.02), np.full(N, 0.55), np.linspace(-0.1, 0.1, N)
    T = lambda a: torch.as_tensor(a, dtype=torch.float64).cuda()  # noqa: E731
    args = [T(a) for a in (rho, Tf, tgt, Tf, rv, rl, T0, cond)]
    for step in range(3):
        losses = [host(net.train_step(*args)).copy() for net in nets]
        torch.cuda.synchronize()
        assert np.array_equal(losses[0], losses[1]), step
        for k in ("pool0", "pool1", "pool2", "ge1b", "gd1b", "ge3b", "dskip0"):
            assert torch.equal(nets[0].buf[k], nets[1].buf[k]), (step, k)
        assert torch.equal(nets[0].gflat, nets[1].gflat), step
        assert torch.equal(nets[0].flat, nets[1].flat), step
    assert "dup0" in nets[0].buf and "dup0" not in nets[1].buf  # the fused form never stores it


@pytest.mark.parametrize("case", [(2, 32, 32, 32, 32), (1, 32, 64, 64, 64), (1, 16, 16, 128, 128)],
                         ids=lambda c: "x".join(map(str, c)))
def test_conv_with_pooling_equals_conv_then_pooling(case):
    """unet_conv3x3_fwd_pool: the output and its 2x2 max pooling bitwise those of
    unet_conv3x3_fwd followed by unet_maxpool2_fwd (32- and 64-wide workgroups)."""
    import torch
    N, H, W, ci, co = case
    say(f"case: convolution with pooling {case}")
    u = lib()
    L = u.library()
    x, w, b = dev_bf16(bf((N, H, W, ci), 60)), dev_bf16(bf((co, 3, 3, ci), 61, 0.2)), dev_f32(bf((co,), 62, 0.1))
    y1, y2 = (torch.empty((N, H, W, co), dtype=torch.bfloat16, device="cuda") for _ in range(2))
    p1, p2 = (torch.full((N, H // 2, W // 2, co), 9.0, dtype=torch.bfloat16, device="cuda") for _ in range(2))
    ck(L.unet_conv3x3_fwd(u.ptr(x), ci, 0, u.ptr(w), u.ptr(b), u.ptr(y1), co, 0, None, 0, 0, N, H, W, ci, co, u.RELU,
                          None))
    ck(L.unet_maxpool2_fwd(u.ptr(y1), co, 0, u.ptr(p1), co, 0, N, H, W, co, None))
    ck(L.unet_conv3x3_fwd_pool(u.ptr(x), ci, 0, u.ptr(w), u.ptr(b), u.ptr(y2), co, 0, u.ptr(p2), co, 0, N, H, W, ci, co,
                               u.RELU, None))
    torch.cuda.synchronize()
    assert torch.equal(y1.view(torch.int16), y2.view(torch.int16))
    assert torch.equal(p1.view(torch.int16), p2.view(torch.int16))
    # shapes the tiled kernel does not cover: UNET_ESHAPE, nothing written
    p3 = torch.full((N, 4, 4, co), 9.0, dtype=torch.bfloat16, device="cuda")
    y3 = torch.full((N, 8, 8, co), 9.0, dtype=torch.bfloat16, device="cuda")
    x3 = dev_bf16(bf((N, 8, 8, ci), 63))
    assert L.unet_conv3x3_fwd_pool(u.ptr(x3), ci, 0, u.ptr(w), u.ptr(b), u.ptr(y3), co, 0, u.ptr(p3), co, 0, N, 8, 8,
                                   ci, co, u.RELU, None) == u.ESHAPE
    torch.cuda.synchronize()
    assert bool((y3 == 9.0).all()) and bool((p3 == 9.0).all())


@pytest.mark.parametrize("case", [(2, 32, 32, 32, 64, 32), (1, 32, 32, 64, 128, 64), (1, 16, 32, 128, 256, 128)],
                         ids=lambda c: "x".join(map(str, c)))
def test_decoder_input_gradient_through_upsampling_equals_the_separate_calls(case):
    """unet_conv3x3_bwd_upcat: the skip branch's gradient and the lower level's gradient
    (2x2 sums of the upsampled branch's gradient, gated by the lower level's ReLU) bitwise
    those of unet_conv3x3_fwd_cat with the output split, then unet_upsample2_bwd."""
    import torch
    N, H, W, cg, clow, cs = case
    cin = clow + cs
    say(f"case: decoder input gradient through the upsampling {case}")
    u = lib()
    L = u.library()
    g, wf = dev_bf16(bf((N, H, W, cg), 70)), dev_bf16(bf((cin, 3, 3, cg), 71, 0.2))
    low = dev_bf16(bf((N, H // 2, W // 2, clow), 72))        # both signs: the gate is exercised
    dup = torch.empty((N, H, W, clow), dtype=torch.bfloat16, device="cuda")
    ds1, ds2 = (torch.empty((N, H, W, cs), dtype=torch.bfloat16, device="cuda") for _ in range(2))
    dl1, dl2 = (torch.full((N, H // 2, W // 2, clow), 9.0, dtype=torch.bfloat16, device="cuda") for _ in range(2))
    ck(L.unet_conv3x3_fwd_cat(u.ptr(g), cg, 0, cg, 0, None, 0, 0, u.ptr(wf), None, u.ptr(dup), clow, 0, clow,
                              u.ptr(ds1), cs, 0, None, 0, 0, N, H, W, cg, cin, 0, None))
    ck(L.unet_upsample2_bwd(u.ptr(dup), clow, 0, u.ptr(low), clow, 0, u.ptr(dl1), clow, 0, N, H // 2, W // 2, clow,
                            None))
    ck(L.unet_conv3x3_bwd_upcat(u.ptr(g), cg, 0, u.ptr(wf), u.ptr(dl2), clow, 0, u.ptr(low), clow, 0, clow, u.ptr(ds2),
                                cs, 0, N, H, W, cg, cin, None))
    torch.cuda.synchronize()
    assert torch.equal(ds1.view(torch.int16), ds2.view(torch.int16))
    assert torch.equal(dl1.view(torch.int16), dl2.view(torch.int16))
    assert bool((dl2 == 0).any()) and bool((dl2 != 0).any())
    # a split that is not a multiple of the workgroup's output width: UNET_ESHAPE
    if cin % 64 == 0 and cg != 32:
        ds3 = torch.empty((N, H, W, cs + 32), dtype=torch.bfloat16, device="cuda")  # sized as the call says
        assert L.unet_conv3x3_bwd_upcat(u.ptr(g), cg, 0, u.ptr(wf), u.ptr(dl2), clow, 0, u.ptr(low), clow, 0, clow - 32,
                                        u.ptr(ds3), cs + 32, 0, N, H, W, cg, cin, None) == u.ESHAPE


LARGE_CONV = [  # N, H, W, Cin, Cout: thousands of pixels, every LDS tile shape, XCD-ordered grids
    (2, 64, 64, 32, 32),     # halo-tile form (C_in = 32), four image rows per tile
    (1, 64, 64, 64, 64),
    (1, 32, 64, 128, 128),
    (1, 64, 64, 32, 96),     # halo-tile form, three column tiles
    (1, 16, 256, 32, 32),    # halo-tile form at the network's widest rows (one row per tile)
    (2, 32, 128, 32, 64),    # halo-tile form, two rows per tile, two column tiles
    (2, 2, 64, 32, 32),      # 128-pixel images: a 256-pixel tile would cross images, LDS-staged form instead
    (2, 32, 64, 8, 32),      # C_in = 8 halo-tile form (the network's first layer)
]


@pytest.mark.parametrize("case", LARGE_CONV, ids=lambda c: "x".join(map(str, c)))
def test_conv3x3_large_bf16_epilogue(case):
    """bfloat16 output with bias, ReLU and a mask at thousands of pixels: the staged
    epilogue's 16-byte stores against the reference rounded to bfloat16."""
    import torch
    N, H, W, ci, co = case
    say(f"case: conv3x3 large bf16 {case}")
    u = lib()
    x, w, b = bf((N, H, W, ci), 21), bf((co, 3, 3, ci), 22, 0.2), bf(co, 23)
    m = bf((N, H, W, co), 24)
    pre = U.conv3x3(x, w, b)
    ref = np.where(m > 0, np.maximum(pre, 0), 0.0)
    bound = gamma(9 * ci + 1) * (U.conv3x3(np.abs(x), np.abs(w)) + np.abs(b))
    y = torch.zeros((N, H, W, co), dtype=torch.bfloat16, device="cuda")
    xd, wd, bd, md = dev_bf16(x), dev_bf16(w), dev_f32(b), dev_bf16(m)
    ck(u.library().unet_conv3x3_fwd(u.ptr(xd), ci, 0, u.ptr(wd), u.ptr(bd), u.ptr(y), co, 0, u.ptr(md), co, 0, N, H,
                                    W, ci, co, u.RELU, None))
    got = host(y)
    want = U.bf16_round(ref)
    # one bfloat16 step, plus the accumulation bound where the FP32 sum may sit on the
    # other side of a rounding boundary or of the ReLU
    tol = np.abs(want) * 2.0 ** -7 + bound * (1 + 2.0 ** -7) + 1e-30
    assert (np.abs(got - want) <= tol).all(), float((np.abs(got - want) / tol).max())
    assert (got[m <= 0] == 0).all()


@pytest.mark.parametrize("case", [(1, 64, 64, 96, 32), (1, 64, 64, 64, 64), (2, 32, 32, 128, 128), (1, 16, 256, 32, 32),
                                  (1, 32, 32, 192, 64),
                                  (5, 64, 256, 32, 32)],  # 320 slabs: the wide reduction, full passes and a tail
                         ids=lambda c: "x".join(map(str, c)))
def test_conv3x3_large_input_and_weight_gradients(case):
    """Input gradient (flipped weights) and weight gradient at thousands of pixels: the
    weight gradient then spans several 128-column tiles and many pixel slabs."""
    import ctypes
    import torch
    N, H, W, ci, co = case
    say(f"case: conv3x3 large gradients {case}")
    u = lib()
    x, g, w = bf((N, H, W, ci), 25), bf((N, H, W, co), 26), bf((co, 3, 3, ci), 27, 0.2)
    gi_ref = U.conv3x3_grad_input(g, w)
    gi_bound = gamma(9 * co) * U.conv3x3_grad_input(np.abs(g), np.abs(w))
    wd = dev_bf16(w)
    wf = torch.empty_like(wd)
    ck(u.library().unet_flip_weights(u.ptr(wd), u.ptr(wf), co, ci, None))
    dx = torch.zeros((N, H, W, ci), dtype=torch.float32, device="cuda")
    gd, xd = dev_bf16(g), dev_bf16(x)
    ck(u.library().unet_conv3x3_fwd(u.ptr(gd), co, 0, u.ptr(wf), None, u.ptr(dx), ci, 0, None, 0, 0, N, H, W, co, ci,
                                    u.OUT_F32, None))
    err = np.abs(host(dx) - gi_ref)
    assert (err <= gi_bound + 1e-30).all(), float((err / (gi_bound + 1e-30)).max())
    dw_ref, db_ref = U.conv3x3_grad_weight(x, g)
    bw, bb = U.conv3x3_grad_weight(np.abs(x), np.abs(g))
    P = N * H * W
    nb = ctypes.c_size_t()
    ck(u.library().unet_wgrad_partial_bytes(N, H, W, ci, co, ctypes.byref(nb)))
    part = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    dw = torch.zeros(co * 9 * ci, dtype=torch.float32, device="cuda")
    db = torch.zeros(co, dtype=torch.float32, device="cuda")
    ck(u.library().unet_conv3x3_wgrad(u.ptr(xd), ci, 0, u.ptr(gd), co, 0, u.ptr(dw), u.ptr(db), u.ptr(part), nb.value,
                                      N, H, W, ci, co, None))
    got_w = host(dw).reshape(co, 3, 3, ci)
    assert (np.abs(got_w - dw_ref) <= gamma(P) * bw + 1e-30).all()
    assert (np.abs(host(db) - db_ref) <= gamma(P) * bb + 1e-30).all()


def test_flip_many_equals_per_layer_flips():
    """The one-launch flip of several layers (workgroup ranges per layer) is bitwise the
    per-layer flip."""
    import ctypes
    import torch
    say("case: flip many")
    u = lib()
    shapes = [(32, 8), (32, 32), (64, 96), (16, 40), (128, 64)]  # (C_out, C_in)
    ws = [dev_bf16(bf((co, 3, 3, ci), 40 + i)) for i, (co, ci) in enumerate(shapes)]
    one = [torch.empty_like(w) for w in ws]
    many = [torch.zeros_like(w) for w in ws]
    for w, o, (co, ci) in zip(ws, one, shapes):
        ck(u.library().unet_flip_weights(u.ptr(w), u.ptr(o), co, ci, None))
    n = len(shapes)
    V, I = ctypes.c_void_p, ctypes.c_int32
    ck(u.library().unet_flip_weights_many((V * n)(*[u.ptr(w) for w in ws]), (V * n)(*[u.ptr(m) for m in many]),
                                          (I * n)(*[co for co, _ in shapes]), (I * n)(*[ci for _, ci in shapes]), n,
                                          None))
    torch.cuda.synchronize()
    for o, m in zip(one, many):
        assert torch.equal(o, m)
