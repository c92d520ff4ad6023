"""The weight-gradient entry point that allocates nothing (unet_conv3x3_wgrad_noalloc):
its partial sums live in the library's static device array.  Its results must be
bitwise those of unet_conv3x3_wgrad with a caller-supplied partials buffer, on two calls
in a row (the second smaller, so it runs on what the first left in the array), and
within the FP32 accumulation bound of the FP64 reference; shapes whose partials exceed
the array are refused before any launch.
"""
import ctypes

import numpy as np
import pytest

from oracle import unet as U
from tests.parity_helpers import say

pytestmark = pytest.mark.gpu

U_F32 = 2.0 ** -24
SCRATCH_BYTES = 48 << 20          # UNET_WGRAD_SCRATCH_BYTES of include/unet.h


def _bf(shape, seed):
    r = np.random.Generator(np.random.PCG64(seed)).standard_normal(shape)
    return U.bf16_round(r)


def _dev_bf16(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.float().cpu().numpy().astype(np.float64)


def _check(code, L):
    assert code == 0, (code, L.unet_last_error())


def _both(case, seed):
    """(dw, db) from the workspace entry point and from the no-allocation one."""
    import torch
    from paper_2106_01557_amd import unet as u
    L = u.library()
    N, H, W, ci, co = case
    x, g = _bf((N, H, W, ci), seed), _bf((N, H, W, co), seed + 1)
    xd, gd = _dev_bf16(x), _dev_bf16(g)
    nb = ctypes.c_size_t()
    _check(L.unet_wgrad_partial_bytes(N, H, W, ci, co, ctypes.byref(nb)), L)
    assert nb.value <= SCRATCH_BYTES
    part = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    outs = []
    for noalloc in (False, True):
        dw = torch.full((co * 9 * ci,), float("nan"), dtype=torch.float32, device="cuda")
        db = torch.full((co,), float("nan"), dtype=torch.float32, device="cuda")
        if noalloc:
            _check(L.unet_conv3x3_wgrad_noalloc(u.ptr(xd), ci, 0, u.ptr(gd), co, 0, u.ptr(dw), u.ptr(db),
                                                N, H, W, ci, co, None), L)
        else:
            _check(L.unet_conv3x3_wgrad(u.ptr(xd), ci, 0, u.ptr(gd), co, 0, u.ptr(dw), u.ptr(db), u.ptr(part),
                                        nb.value, N, H, W, ci, co, None), L)
        outs.append((_host(dw), _host(db)))
    return x, g, outs


def test_noalloc_weight_gradient_matches_workspace_entry_point():
    # the first call fills 40 MiB of the array (512 slabs x 64 x 320 floats); the second,
    # smaller one reads a shorter prefix, written over by its own slabs.  Both must equal
    # the workspace entry point bitwise; the second is also held to the FP64 reference.
    for case, seed, ref in (((16, 128, 128, 32, 64), 30, False), ((2, 32, 32, 64, 32), 40, True)):
        say(f"case: wgrad no-alloc vs workspace entry point {case}")
        x, g, ((dw0, db0), (dw1, db1)) = _both(case, seed)
        assert np.isfinite(dw1).all() and np.isfinite(db1).all()
        assert np.array_equal(dw0, dw1) and np.array_equal(db0, db1)
        if not ref:
            continue
        N, H, W, ci, co = case
        ref_w, ref_b = U.conv3x3_grad_weight(x, g)
        bw, bb = U.conv3x3_grad_weight(np.abs(x), np.abs(g))
        P = N * H * W
        gam = P * U_F32 / (1 - P * U_F32)
        assert (np.abs(dw1.reshape(co, 3, 3, ci) - ref_w) <= gam * bw + 1e-30).all()
        assert (np.abs(db1 - ref_b) <= gam * bb + 1e-30).all()


def test_noalloc_weight_gradient_refuses_shapes_beyond_the_array():
    """A layer whose partial sums exceed the array is refused with UNET_EINVAL before any
    launch (2048 -> 1024 channels on one 16 x 16 image: 1024 x 18464 floats, 72 MiB)."""
    import torch
    from paper_2106_01557_amd import unet as u
    L = u.library()
    N, H, W, ci, co = 1, 16, 16, 2048, 1024
    nb = ctypes.c_size_t()
    _check(L.unet_wgrad_partial_bytes(N, H, W, ci, co, ctypes.byref(nb)), L)
    assert nb.value > SCRATCH_BYTES
    x = torch.zeros(N * H * W * ci, dtype=torch.bfloat16, device="cuda")
    g = torch.zeros(N * H * W * co, dtype=torch.bfloat16, device="cuda")
    dw = torch.zeros(co * 9 * ci, dtype=torch.float32, device="cuda")
    db = torch.zeros(co, dtype=torch.float32, device="cuda")
    code = L.unet_conv3x3_wgrad_noalloc(u.ptr(x), ci, 0, u.ptr(g), co, 0, u.ptr(dw), u.ptr(db), N, H, W, ci, co, None)
    assert code == -1
    assert b"static scratch" in L.unet_last_error()
    torch.cuda.synchronize()
    assert float(dw.abs().max()) == 0.0
