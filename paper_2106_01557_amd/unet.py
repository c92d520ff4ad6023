"""Learned warm start: a U-Net that maps an initial density field to a later one,
built on the network kernels of include/unet.h (bfloat16 activations, FP32
accumulation on the matrix cores, FP32 master weights and Adam).

Marshalling only: every arithmetic step of the forward pass, the backward pass and
the optimizer runs in the library's kernels; torch provides device memory and the
stream.  The architecture: encoder levels of widths (32, 64, 128, 256), each two
3x3 convolutions with ReLU followed by 2x2 max pooling (none after the last, the
bottleneck); decoder levels upsample 2x, concatenate the encoder level's output
and apply two 3x3 convolutions with ReLU; a 1x1 head with one output per predicted
field (the density and, by default, the temperature) adds its outputs to the
corresponding input fields.  Convolutions wrap around (the lattice is periodic).

Normalisation: density nu = (rho - rho_v) / (rho_l - rho_v) with the coexistence
densities at the run's T0; temperature theta = (T / T0 - 1) / theta_scale; a
conditioning channel carries the run's reduced temperature.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import lbm as _lbm

_lib = _lbm.library()
_P, _I, _F, _V, _S = ctypes.POINTER, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t

EXPORTED = ["unet_conv3x3_fwd", "unet_conv3x3_fwd_cat", "unet_conv3x3_fwd_pool", "unet_conv3x3_bwd_upcat",
            "unet_flip_weights", "unet_flip_weights_many",
            "unet_wgrad_partial_bytes", "unet_conv3x3_wgrad", "unet_conv3x3_wgrad_cat", "unet_conv3x3_wgrad_noalloc",
            "unet_maxpool2_fwd", "unet_maxpool2_bwd", "unet_upsample2_fwd", "unet_upsample2_bwd",
            "unet_prepare_input", "unet_output_fields", "unet_head_partial_bytes", "unet_head_fwd", "unet_head_bwd",
            "unet_head_train", "unet_adam",
            "unet_to_bf16", "unet_to_f32", "unet_last_error"]

RELU, OUT_F32 = 1, 2
ESHAPE = -2  # a fused call that does not cover the shape: the separate calls do

_lib.unet_conv3x3_fwd.argtypes = [_V, _I, _I, _V, _V, _V, _I, _I, _V, _I, _I, _I, _I, _I, _I, _I, _I, _V]
_lib.unet_conv3x3_fwd_cat.argtypes = [_V, _I, _I, _I, _I, _V, _I, _I, _V, _V, _V, _I, _I, _I, _V, _I, _I, _V, _I, _I,
                                      _I, _I, _I, _I, _I, _I, _V]
_lib.unet_conv3x3_fwd_pool.argtypes = [_V, _I, _I, _V, _V, _V, _I, _I, _V, _I, _I, _I, _I, _I, _I, _I, _I, _V]
_lib.unet_conv3x3_bwd_upcat.argtypes = [_V, _I, _I, _V, _V, _I, _I, _V, _I, _I, _I, _V, _I, _I, _I, _I, _I, _I, _I, _V]
_lib.unet_flip_weights.argtypes = [_V, _V, _I, _I, _V]
_lib.unet_flip_weights_many.argtypes = [ctypes.POINTER(_V), ctypes.POINTER(_V), ctypes.POINTER(_I),
                                        ctypes.POINTER(_I), _I, _V]
_lib.unet_wgrad_partial_bytes.argtypes = [_I, _I, _I, _I, _I, _P(_S)]
_lib.unet_conv3x3_wgrad.argtypes = [_V, _I, _I, _V, _I, _I, _V, _V, _V, _S, _I, _I, _I, _I, _I, _V]
_lib.unet_conv3x3_wgrad_cat.argtypes = [_V, _I, _I, _I, _I, _V, _I, _I, _V, _I, _I, _V, _V, _V, _S, _I, _I, _I, _I, _I,
                                        _V]
_lib.unet_conv3x3_wgrad_noalloc.argtypes = [_V, _I, _I, _V, _I, _I, _V, _V, _I, _I, _I, _I, _I, _V]
_lib.unet_maxpool2_fwd.argtypes = [_V, _I, _I, _V, _I, _I, _I, _I, _I, _I, _V]
_lib.unet_maxpool2_bwd.argtypes = [_V, _I, _I, _V, _I, _I, _V, _I, _I, _V, _I, _I, _I, _I, _I, _I, _I, _V]
_lib.unet_upsample2_fwd.argtypes = [_V, _I, _I, _V, _I, _I, _I, _I, _I, _I, _V]
_lib.unet_upsample2_bwd.argtypes = [_V, _I, _I, _V, _I, _I, _V, _I, _I, _I, _I, _I, _I, _V]
_D = ctypes.c_double
_lib.unet_prepare_input.argtypes = [_V, _V, _V, _V, _V, _V, _D, _V, _V, _I, _I, _I, _V]
_lib.unet_output_fields.argtypes = [_V, _I, _V, _V, _V, _D, _V, _V, _I, _I, _I, _V]
_lib.unet_head_partial_bytes.argtypes = [_I, _I, _I, _I, _I, _P(_S)]
_lib.unet_head_fwd.argtypes = [_V, _I, _V, _V, _V, _V, _V, _V, _V, _V, _S, _I, _I, _I, _I, _I, _V]
_lib.unet_head_bwd.argtypes = [_V, _I, _V, _V, _V, _V, _V, _V, _S, _I, _I, _I, _I, _I, _V]
_lib.unet_head_train.argtypes = [_V, _I, _V, _V, _V, _V, _V, _V, _V, _V, _V, _V, _V, _S, _I, _I, _I, _I, _I, _V]
_lib.unet_adam.argtypes = [_V, _V, _V, _V, _V, _S, _F, _F, _F, _F, _I, _V]
_lib.unet_to_bf16.argtypes = [_V, _V, _S, _V]
_lib.unet_to_f32.argtypes = [_V, _V, _S, _V]
_lib.unet_last_error.argtypes = []
_lib.unet_last_error.restype = ctypes.c_char_p
for _n in EXPORTED:
    if _n != "unet_last_error":
        getattr(_lib, _n).restype = ctypes.c_int


class UnetError(RuntimeError):
    pass


def _ck(code):
    if code != 0:
        raise UnetError(f"{code}: {_lib.unet_last_error().decode()}")


def ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def library():
    return _lib


def conv_layers(widths, in_channels):
    """(name, C_in, C_out) of the 3x3 convolutions: two per encoder level, then two per
    decoder level from the bottom up (the first reads the concatenation of the
    upsampled lower level and the encoder level's output)."""
    layers, cin = [], in_channels
    for lvl, c in enumerate(widths):
        layers.append((f"e{lvl}a", cin, c))
        layers.append((f"e{lvl}b", c, c))
        cin = c
    for lvl in reversed(range(len(widths) - 1)):
        layers.append((f"d{lvl}a", widths[lvl + 1] + widths[lvl], widths[lvl]))
        layers.append((f"d{lvl}b", widths[lvl], widths[lvl]))
    return layers


class UNet:
    """Parameters (FP32 masters, bfloat16 copies and flipped copies for the input
    gradient) and per-batch-shape activation buffers on one device."""

    def __init__(self, widths=(32, 64, 128, 256), in_channels=8, outputs=2, theta_scale=0.1, seed=0, device=None,
                 stream=None, wgrad_streams=2, fuse_2x2=True):
        import torch
        self.torch = torch
        self.widths = tuple(int(w) for w in widths)
        self.in_channels = int(in_channels)
        self.K = int(outputs)
        self.theta_scale = float(theta_scale)
        self.layers = conv_layers(self.widths, self.in_channels)
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.s = ctypes.c_void_p(self.stream.cuda_stream)
        # weight gradients (and their reductions) run on wgrad_streams streams of their
        # own, layer by layer in turn, beside the input gradients: a layer's two gradients
        # only read the same activations and output gradient.  0: everything on `stream`.
        if int(wgrad_streams) < 0:
            raise UnetError("wgrad_streams must be >= 0")
        self.wgrad_streams = int(wgrad_streams)
        self.wstreams = [torch.cuda.Stream(self.device) for _ in range(self.wgrad_streams)] or [self.stream]
        self.ws = [ctypes.c_void_p(st.cuda_stream) for st in self.wstreams]
        # the 2x2 max pooling in the epilogue of the convolution before it, and the
        # upsampling's gradient in the epilogue of the decoder's input gradient, where the
        # tiled kernel covers the shape (else, and with fuse_2x2=False, separate passes)
        self.fuse_2x2 = bool(fuse_2x2)
        self.t = 0
        rng = np.random.Generator(np.random.PCG64(seed))
        p = {}
        for name, ci, co in self.layers:  # He-normal weights, zero biases
            p[name + ".w"] = rng.standard_normal((co, 3, 3, ci)) * np.sqrt(2.0 / (9 * ci))
            p[name + ".b"] = np.zeros(co)
        c0 = self.widths[0]
        p["head.w"] = rng.standard_normal((self.K, c0)) / np.sqrt(c0)
        p["head.b"] = np.zeros(self.K)
        self.load_params(p)
        self._shape = None
        self._head_done = False

    # -- parameters ------------------------------------------------------------------
    def _f32(self, a):
        return self.torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device)

    def load_params(self, p: dict):
        """Parameters, Adam moments, gradients and bfloat16 copies are views into flat
        buffers (each tensor starts at a multiple of 16 elements, so every view stays
        16-byte aligned and the padding stays zero), so that one Adam launch updates
        them all."""
        torch = self.torch
        offs, total = {}, 0
        for k, v in p.items():
            n = int(np.asarray(v).size)
            offs[k] = (total, n)
            total += (n + 15) // 16 * 16
        self._offs, self._total = offs, total
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            z = lambda dt: torch.zeros(total, dtype=dt, device=self.device)  # noqa: E731
            self.flat, self.mflat, self.vflat, self.gflat = (z(torch.float32) for _ in range(4))
            self.w16flat = z(torch.bfloat16)
            view = lambda buf: {k: buf[o:o + n] for k, (o, n) in offs.items()}  # noqa: E731
            self.p, self.m, self.v, self.g = view(self.flat), view(self.mflat), view(self.vflat), view(self.gflat)
            for k, v in p.items():
                self.p[k].copy_(self._f32(v).reshape(-1))
            w16 = view(self.w16flat)
            self.w16, self.wf16 = {}, {}
            for name, ci, co in self.layers:
                self.w16[name] = w16[name + ".w"]
                self.wf16[name] = torch.empty(self.w16[name].numel(), dtype=torch.bfloat16, device=self.device)
            # descriptors of every layer for the one-launch flip after each Adam step
            n = len(self.layers)
            self._flip = ((_V * n)(*[ptr(self.w16[nm]) for nm, _, _ in self.layers]),
                          (_V * n)(*[ptr(self.wf16[nm]) for nm, _, _ in self.layers]),
                          (_I * n)(*[co for _, _, co in self.layers]), (_I * n)(*[ci for _, ci, _ in self.layers]), n)
            self._refresh_copies()
        self.t = 0

    def _refresh_copies(self):
        for name, ci, co in self.layers:
            w = self.p[name + ".w"]
            _ck(_lib.unet_to_bf16(ptr(w), ptr(self.w16[name]), w.numel(), self.s))
            _ck(_lib.unet_flip_weights(ptr(self.w16[name]), ptr(self.wf16[name]), co, ci, self.s))

    def params_numpy(self) -> dict:
        self.stream.synchronize()
        out = {}
        for k, v in self.p.items():
            a = v.cpu().numpy().astype(np.float64)
            if k.endswith(".w") and not k.startswith("head"):
                name = k[:-2]
                ci, co = next((c, o) for n, c, o in self.layers if n == name)
                a = a.reshape(co, 3, 3, ci)
            elif k == "head.w":
                a = a.reshape(self.K, -1)
            out[k] = a
        return out

    # -- buffers -----------------------------------------------------------------------
    def _alloc(self, N, H, W):
        if self._shape == (N, H, W):
            return
        torch = self.torch
        L = len(self.widths)
        if H % (1 << (L - 1)) or W % (1 << (L - 1)):
            raise UnetError(f"H and W must be multiples of {1 << (L - 1)}")
        bf = lambda *s: torch.empty(s, dtype=torch.bfloat16, device=self.device)
        f32 = lambda *s: torch.empty(s, dtype=torch.float32, device=self.device)
        b = {}
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            # rin and target hold both normalised fields ([2][N,H,W]); the head uses the first K
            b["x0"], b["rin"], b["target"] = bf(N, H, W, self.in_channels), f32(2, N, H, W), f32(2, N, H, W)
            b["out"], b["dout"] = f32(self.K, N, H, W), f32(self.K, N, H, W)
            for lvl, c in enumerate(self.widths):
                h, w = H >> lvl, W >> lvl
                b[f"e{lvl}a"], b[f"e{lvl}b"] = bf(N, h, w, c), bf(N, h, w, c)
                b[f"ge{lvl}a"] = bf(N, h, w, c)
                b[f"ge{lvl}b"] = bf(N, h, w, c)
                if lvl < L - 1:
                    cu = self.widths[lvl + 1]
                    # the decoder's input [upsample2(lower level) | e{lvl}b] is never stored:
                    # its convolution reads the two tensors; its input gradient goes to the
                    # upsampled branch (dup, full size) and the skip branch (dskip)
                    b[f"dskip{lvl}"] = bf(N, h, w, c)
                    b[f"pool{lvl}"] = bf(N, h // 2, w // 2, c)
                    b[f"dpool{lvl}"] = bf(N, h // 2, w // 2, c)
                    b[f"d{lvl}a"], b[f"d{lvl}b"] = bf(N, h, w, c), bf(N, h, w, c)
                    b[f"gd{lvl}a"], b[f"gd{lvl}b"] = bf(N, h, w, c), bf(N, h, w, c)
            need = 0
            for name, ci, co in self.layers:
                lvl = int(name[1])
                nb = _S()
                _ck(_lib.unet_wgrad_partial_bytes(N, H >> lvl, W >> lvl, ci, co, ctypes.byref(nb)))
                need = max(need, nb.value)
            nb = _S()
            _ck(_lib.unet_head_partial_bytes(N, H, W, self.widths[0], self.K, ctypes.byref(nb)))
            # one partial-sum buffer per weight-gradient stream
            b["wpart"] = [torch.empty(need, dtype=torch.uint8, device=self.device) for _ in self.wstreams]
            b["hpart"] = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
            b["loss"] = f32(1)
        self.buf = b
        self._shape = (N, H, W)

    # -- passes --------------------------------------------------------------------------
    def _conv(self, name, x, ldx, offx, y, ldy, offy, N, h, w, flags=RELU, mask=None, ldm=0, offm=0):
        ci, co = next((c, o) for n, c, o in self.layers if n == name)
        _ck(_lib.unet_conv3x3_fwd(ptr(x), ldx, offx, ptr(self.w16[name]), ptr(self.p[name + ".b"]), ptr(y), ldy,
                                  offy, ptr(mask), ldm, offm, N, h, w, ci, co, flags, self.s))

    def forward(self, rho, T, rho_v, rho_l, T0, cond, target_rho=None, target_T=None, train=False):
        """rho, T: FP64 [N, H, W] device fields (T may be None: T = T0); rho_v, rho_l, T0,
        cond: FP64 [N] device tensors (normalisation and the conditioning channel);
        target_rho, target_T: FP64 [N, H, W] device fields or None.  Returns the
        normalised prediction (FP32 [K, N, H, W], a view into the model's buffer) and,
        with a target, the loss tensor.  train (with a target): the head's backward pass
        runs here too, in the same pass over the last activation, and backward() then
        starts below the head."""
        torch = self.torch
        N, H, W = rho.shape
        self._alloc(N, H, W)
        b, L, wd = self.buf, len(self.widths), self.widths
        ts = self.theta_scale
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            _ck(_lib.unet_prepare_input(ptr(rho), ptr(T), ptr(rho_v), ptr(rho_l), ptr(T0), ptr(cond), ts, ptr(b["x0"]),
                                        ptr(b["rin"]), N, H, W, self.s))
            if target_rho is not None:
                # the targets go through the same normalisation
                _ck(_lib.unet_prepare_input(ptr(target_rho), ptr(target_T), ptr(rho_v), ptr(rho_l), ptr(T0), ptr(cond),
                                            ts, None, ptr(b["target"]), N, H, W, self.s))
            x, ldx, offx = b["x0"], self.in_channels, 0
            for lvl in range(L):
                h, w, c = H >> lvl, W >> lvl, wd[lvl]
                self._conv(f"e{lvl}a", x, ldx, offx, b[f"e{lvl}a"], c, 0, N, h, w)
                if lvl < L - 1:
                    rc = ESHAPE
                    if self.fuse_2x2:
                        rc = _lib.unet_conv3x3_fwd_pool(ptr(b[f"e{lvl}a"]), c, 0, ptr(self.w16[f"e{lvl}b"]),
                                                        ptr(self.p[f"e{lvl}b.b"]), ptr(b[f"e{lvl}b"]), c, 0,
                                                        ptr(b[f"pool{lvl}"]), c, 0, N, h, w, c, c, RELU, self.s)
                    if rc == ESHAPE:
                        self._conv(f"e{lvl}b", b[f"e{lvl}a"], c, 0, b[f"e{lvl}b"], c, 0, N, h, w)
                        rc = _lib.unet_maxpool2_fwd(ptr(b[f"e{lvl}b"]), c, 0, ptr(b[f"pool{lvl}"]), c, 0, N, h, w, c,
                                                    self.s)
                    _ck(rc)
                    x, ldx, offx = b[f"pool{lvl}"], c, 0
                else:
                    self._conv(f"e{lvl}b", b[f"e{lvl}a"], c, 0, b[f"e{lvl}b"], c, 0, N, h, w)
            low = b[f"e{L - 1}b"]
            for lvl in reversed(range(L - 1)):
                h, w, c, cu = H >> lvl, W >> lvl, wd[lvl], wd[lvl + 1]
                # input [upsample2(low) | e{lvl}b], read from the two tensors
                _ck(_lib.unet_conv3x3_fwd_cat(ptr(low), cu, 0, cu, 1, ptr(b[f"e{lvl}b"]), c, 0,
                                              ptr(self.w16[f"d{lvl}a"]), ptr(self.p[f"d{lvl}a.b"]),
                                              ptr(b[f"d{lvl}a"]), c, 0, c, None, 0, 0, None, 0, 0,
                                              N, h, w, cu + c, c, RELU, self.s))
                self._conv(f"d{lvl}b", b[f"d{lvl}a"], c, 0, b[f"d{lvl}b"], c, 0, N, h, w)
                low = b[f"d{lvl}b"]
            tgt = b["target"] if target_rho is not None else None
            self._head_done = bool(train and tgt is not None)
            if self._head_done:
                g = self.g
                _ck(_lib.unet_head_train(ptr(low), wd[0], ptr(self.p["head.w"]), ptr(self.p["head.b"]), ptr(b["rin"]),
                                         ptr(tgt), ptr(b["out"]), ptr(b["dout"]), ptr(b["loss"]), ptr(b["gd0b"]),
                                         ptr(g["head.w"]), ptr(g["head.b"]), ptr(b["hpart"]), b["hpart"].numel(),
                                         N, H, W, wd[0], self.K, self.s))
            else:
                _ck(_lib.unet_head_fwd(ptr(low), wd[0], ptr(self.p["head.w"]), ptr(self.p["head.b"]), ptr(b["rin"]),
                                       ptr(tgt), ptr(b["out"]), ptr(b["dout"]), ptr(b["loss"]), ptr(b["hpart"]),
                                       b["hpart"].numel(), N, H, W, wd[0], self.K, self.s))
        return (b["out"], b["loss"]) if target_rho is not None else b["out"]

    def backward(self):
        """Gradients (FP32, in self.g) of the loss of the last forward call with a target."""
        torch = self.torch
        N, H, W = self._shape
        b, g, L, wd = self.buf, self.g, len(self.widths), self.widths
        turn = [0]

        def wgrad(name, x, ldx, offx, gy, ldg, h, w, skip=None):
            """skip: the layer input is [upsample2(x) | skip] (x at half size, ldx channels)."""
            ci, co = next((c_, o_) for n_, c_, o_ in self.layers if n_ == name)
            k = turn[0] % len(self.wstreams)
            turn[0] += 1
            wp = b["wpart"][k]
            if self.wgrad_streams:
                # gy (and every earlier write) is complete on the main stream before the
                # weight-gradient stream reads it
                self.wstreams[k].wait_stream(self.stream)
            if skip is None:
                _ck(_lib.unet_conv3x3_wgrad(ptr(x), ldx, offx, ptr(gy), ldg, 0, ptr(g[name + ".w"]),
                                            ptr(g[name + ".b"]), ptr(wp), wp.numel(), N, h, w, ci, co, self.ws[k]))
            else:
                _ck(_lib.unet_conv3x3_wgrad_cat(ptr(x), ldx, offx, ldx, 1, ptr(skip), ci - ldx, 0, ptr(gy), ldg, 0,
                                                ptr(g[name + ".w"]), ptr(g[name + ".b"]), ptr(wp), wp.numel(), N, h, w,
                                                ci, co, self.ws[k]))

        def dgrad(name, gy, ldg, dx, lddx, h, w, mask=None, ldm=0, offm=0):
            ci, co = next((c_, o_) for n_, c_, o_ in self.layers if n_ == name)
            # input gradient = forward convolution of gy with the flipped weights
            _ck(_lib.unet_conv3x3_fwd(ptr(gy), ldg, 0, ptr(self.wf16[name]), None, ptr(dx), lddx, 0, ptr(mask), ldm,
                                      offm, N, h, w, co, ci, 0, self.s))

        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            top = b["d0b"]
            if not self._head_done:
                _ck(_lib.unet_head_bwd(ptr(top), wd[0], ptr(self.p["head.w"]), ptr(b["dout"]), ptr(b["gd0b"]),
                                       ptr(g["head.w"]), ptr(g["head.b"]), ptr(b["hpart"]), b["hpart"].numel(), N, H,
                                       W, wd[0], self.K, self.s))
            self._head_done = False
            # decoder, top level first
            for lvl in range(L - 1):
                h, w, c, cu = H >> lvl, W >> lvl, wd[lvl], wd[lvl + 1]
                wgrad(f"d{lvl}b", b[f"d{lvl}a"], c, 0, b[f"gd{lvl}b"], c, h, w)
                dgrad(f"d{lvl}b", b[f"gd{lvl}b"], c, b[f"gd{lvl}a"], c, h, w, mask=b[f"d{lvl}a"], ldm=c)
                if lvl + 1 < L - 1:
                    low, dlow = b[f"d{lvl + 1}b"], b[f"gd{lvl + 1}b"]
                else:
                    low, dlow = b[f"e{lvl + 1}b"], b[f"ge{lvl + 1}b"]
                wgrad(f"d{lvl}a", low, cu, 0, b[f"gd{lvl}a"], c, h, w, skip=b[f"e{lvl}b"])
                # input gradient, split between the upsampled branch (through the
                # upsampling's gradient and the lower level's ReLU) and the skip branch
                rc = ESHAPE
                if self.fuse_2x2:
                    rc = _lib.unet_conv3x3_bwd_upcat(ptr(b[f"gd{lvl}a"]), c, 0, ptr(self.wf16[f"d{lvl}a"]), ptr(dlow),
                                                     cu, 0, ptr(low), cu, 0, cu, ptr(b[f"dskip{lvl}"]), c, 0, N, h, w,
                                                     c, cu + c, self.s)
                if rc == ESHAPE:
                    if f"dup{lvl}" not in b:
                        b[f"dup{lvl}"] = torch.empty((N, h, w, cu), dtype=torch.bfloat16, device=self.device)
                    _ck(_lib.unet_conv3x3_fwd_cat(ptr(b[f"gd{lvl}a"]), c, 0, c, 0, None, 0, 0,
                                                  ptr(self.wf16[f"d{lvl}a"]), None, ptr(b[f"dup{lvl}"]), cu, 0, cu,
                                                  ptr(b[f"dskip{lvl}"]), c, 0, None, 0, 0, N, h, w, c, cu + c, 0,
                                                  self.s))
                    rc = _lib.unet_upsample2_bwd(ptr(b[f"dup{lvl}"]), cu, 0, ptr(low), cu, 0, ptr(dlow), cu, 0, N,
                                                 h // 2, w // 2, cu, self.s)
                _ck(rc)
            # encoder, bottleneck first
            for lvl in reversed(range(L)):
                h, w, c = H >> lvl, W >> lvl, wd[lvl]
                if lvl < L - 1:
                    # pooled-path gradient plus the skip-connection gradient, gated by e{lvl}b > 0
                    _ck(_lib.unet_maxpool2_bwd(ptr(b[f"e{lvl}b"]), c, 0, ptr(b[f"dpool{lvl}"]), c, 0,
                                               ptr(b[f"dskip{lvl}"]), c, 0, ptr(b[f"ge{lvl}b"]), c, 0, 1, N, h, w, c,
                                               self.s))
                wgrad(f"e{lvl}b", b[f"e{lvl}a"], c, 0, b[f"ge{lvl}b"], c, h, w)
                dgrad(f"e{lvl}b", b[f"ge{lvl}b"], c, b[f"ge{lvl}a"], c, h, w, mask=b[f"e{lvl}a"], ldm=c)
                if lvl > 0:
                    cp = wd[lvl - 1]
                    wgrad(f"e{lvl}a", b[f"pool{lvl - 1}"], cp, 0, b[f"ge{lvl}a"], c, h, w)
                    dgrad(f"e{lvl}a", b[f"ge{lvl}a"], c, b[f"dpool{lvl - 1}"], cp, h, w)
                else:
                    wgrad("e0a", b["x0"], self.in_channels, 0, b["ge0a"], c, h, w)
            if self.wgrad_streams:
                # every weight gradient is in place before anything later on the main
                # stream (the optimizer, the next step's passes) runs
                for st in self.wstreams:
                    self.stream.wait_stream(st)
        return g

    def adam_step(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        torch = self.torch
        self.t += 1
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            # one launch over the flat buffers; it also refreshes every bfloat16 copy
            _ck(_lib.unet_adam(ptr(self.flat), ptr(self.gflat), ptr(self.mflat), ptr(self.vflat), ptr(self.w16flat),
                               self._total, lr, b1, b2, eps, self.t, self.s))
            _ck(_lib.unet_flip_weights_many(*self._flip, self.s))

    def train_step(self, rho0, T0f, rhoT, TT, rho_v, rho_l, T0, cond, lr=1e-3):
        _, loss = self.forward(rho0, T0f, rho_v, rho_l, T0, cond, rhoT, TT, train=True)
        self.backward()
        self.adam_step(lr)
        return loss

    def predict_fields(self, rho0, T0f, rho_v, rho_l, T0, cond):
        """Predicted density and temperature (FP64 [N, H, W] device tensors; T = T0 when
        the network has one output)."""
        torch = self.torch
        out = self.forward(rho0, T0f, rho_v, rho_l, T0, cond)
        N, H, W = rho0.shape
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            rho = torch.empty((N, H, W), dtype=torch.float64, device=self.device)
            T = torch.empty_like(rho)
            _ck(_lib.unet_output_fields(ptr(out), self.K, ptr(rho_v), ptr(rho_l), ptr(T0), self.theta_scale, ptr(rho),
                                        ptr(T), N, H, W, self.s))
        return rho, T
