"""Python binding of liblbm.so (include/lbm.h): argument marshalling only.

Every step of the update runs in the HIP library.  PyTorch provides the device
memory (workspace and field tensors) and the stream.  If the library has not
been built this module raises on import: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field, fields as dc_fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

LBM_OK, LBM_EINVAL, LBM_ESPACE, LBM_EHIP, LBM_ENONFINITE, LBM_ESTATE, LBM_EIO = 0, -1, -2, -3, -4, -5, -6
EOS_KINDS = {"cs": 0, "vdw": 1}
BOUNDARIES = {"periodic": 0, "heated_outflow": 1}
PRECISIONS = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
SCHEMES = {"ab": 0, "aa": 1}
ROUNDINGS = {"nearest": 0, "stochastic": 1}
DERIVED_NAMES = ["Tc", "pc", "T0", "rho_v", "rho_l", "p_s", "cs", "c", "dt", "G2", "a_mf", "kappa", "cv",
                 "C_ref", "beta", "k", "h", "bS", "s_p", "s_q", "s_e", "omega_e", "omega_p", "tau_j_v",
                 "tau_j_l", "h_lv", "rho_wall"]
INVARIANT_NAMES = ["mass", "mom_x", "mom_y", "sum_g", "dt_sum_q", "E_p", "E_kin", "bad_nodes"]


class LbmError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"[{code}] {message}")
        self.code = code


class _Lattice(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("dx", ctypes.c_double), ("bc_x", ctypes.c_int32)]


class _Eos(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("a_t", ctypes.c_double), ("b_t", ctypes.c_double),
                ("R", ctypes.c_double), ("K_eos", ctypes.c_double)]


_PARAM_DOUBLES = ["Tr0", "K_int", "varpi", "gamma1", "gamma2", "tau_p", "s_eps", "sigma_e", "sigma_eps",
                  "sigma_q", "sigma_p", "tau_j_v", "lambda_ratio", "cv", "ste", "dTr_ste", "C_ref", "accel_x",
                  "accel_y", "cs_override", "rho_ref", "T_ref", "Tr_wall", "Tr_far", "p_out"]
_PARAM_INTS = ["precision", "scheme", "rows_per_wave", "waves_per_block", "columns_per_lane", "rounding",
               "check_every"]


class _Params(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in _PARAM_DOUBLES] + [(n, ctypes.c_int32) for n in _PARAM_INTS]


EXPORTED = ["lbm_default_params", "lbm_default_eos", "lbm_workspace_bytes", "lbm_init", "lbm_set_fields",
            "lbm_step", "lbm_moments", "lbm_invariants", "lbm_derived", "lbm_launch_shape", "lbm_step_count",
            "lbm_state_bytes",
            "lbm_save_state", "lbm_load_state", "lbm_save", "lbm_load", "lbm_destroy", "lbm_strerror", "lbm_last_error",
            "lbm_maxwell", "lbm_interface_constants", "lbm_batch_workspace_bytes", "lbm_batch_create", "lbm_batch_set_shape",
            "lbm_batch_get_shape", "lbm_batch_set_graph", "lbm_batch_step", "lbm_batch_autotune", "lbm_batch_size",
            "lbm_batch_destroy", "lbm_batch_last_error"]


class _BatchShape(ctypes.Structure):
    _fields_ = [("rows_per_wave", ctypes.c_int32), ("waves_per_block", ctypes.c_int32),
                ("queue", ctypes.c_int32), ("blocks", ctypes.c_int32)]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2106_01557_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, I, D, V, S = ctypes.POINTER, ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    lib.lbm_default_params.argtypes = [P(_Params)]
    lib.lbm_default_eos.argtypes = [P(_Eos)]
    lib.lbm_workspace_bytes.argtypes = [P(_Lattice), P(_Params), P(S)]
    lib.lbm_init.argtypes = [P(V), P(_Lattice), P(_Eos), P(_Params), V, S, V]
    lib.lbm_set_fields.argtypes = [V, V, V, V, V]
    lib.lbm_step.argtypes = [V, ctypes.c_int64]
    lib.lbm_moments.argtypes = [V, V, V, V, V]
    lib.lbm_invariants.argtypes = [V, P(D), I]
    lib.lbm_derived.argtypes = [V, P(D), I]
    lib.lbm_launch_shape.argtypes = [V, P(ctypes.c_int32), P(ctypes.c_int32), P(ctypes.c_int32)]
    lib.lbm_step_count.argtypes = [V, P(ctypes.c_int64)]
    lib.lbm_state_bytes.argtypes = [V, P(S)]
    lib.lbm_save_state.argtypes = [V, V, P(ctypes.c_int64)]
    lib.lbm_load_state.argtypes = [V, V, ctypes.c_int64]
    lib.lbm_save.argtypes = [V, ctypes.c_char_p]
    lib.lbm_load.argtypes = [V, ctypes.c_char_p]
    lib.lbm_destroy.argtypes = [V]
    lib.lbm_strerror.argtypes = [I]
    lib.lbm_strerror.restype = ctypes.c_char_p
    lib.lbm_last_error.argtypes = [V]
    lib.lbm_last_error.restype = ctypes.c_char_p
    lib.lbm_maxwell.argtypes = [P(_Eos), D, P(D)]
    lib.lbm_interface_constants.argtypes = [P(_Eos), D, D, D, D, P(D)]
    lib.lbm_batch_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, P(S)]
    lib.lbm_batch_create.argtypes = [P(V), P(V), ctypes.c_int32, V, S]
    lib.lbm_batch_set_shape.argtypes = [V, P(_BatchShape)]
    lib.lbm_batch_get_shape.argtypes = [V, P(_BatchShape)]
    lib.lbm_batch_set_graph.argtypes = [V, ctypes.c_int32]
    lib.lbm_batch_step.argtypes = [V, ctypes.c_int64]
    lib.lbm_batch_autotune.argtypes = [V, ctypes.c_int32, P(_BatchShape), P(D)]
    lib.lbm_batch_size.argtypes = [V, P(ctypes.c_int64), P(ctypes.c_int64)]
    lib.lbm_batch_destroy.argtypes = [V]
    lib.lbm_batch_last_error.argtypes = [V]
    lib.lbm_batch_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("lbm_strerror", "lbm_last_error", "lbm_batch_last_error"):
            getattr(lib, name).restype = I
    return lib


# The process must hold exactly one HIP runtime.  PyTorch ships its own
# libamdhip64.so; loading it before liblbm.so lets the library's dependency on
# libamdhip64.so.7 resolve to that same runtime.  Loading liblbm.so first would map
# a second runtime, whose device enumeration conflicts with torch's.
import torch  # noqa: E402,F401  (load order matters, see above)

_lib = load_library()


def library() -> ctypes.CDLL:
    return _lib


@dataclass
class Eos:
    kind: str = "cs"
    a_t: float = 1.0
    b_t: float = 4.0
    R: float = 1.0
    K_eos: float = 0.479820

    def _c(self) -> _Eos:
        if self.kind not in EOS_KINDS:
            raise LbmError(LBM_EINVAL, f"unknown EOS kind {self.kind!r}")
        return _Eos(EOS_KINDS[self.kind], self.a_t, self.b_t, self.R, self.K_eos)


def vdw_eos() -> Eos:
    return Eos("vdw", 9.0 / 49.0, 2.0 / 21.0, 1.0, 1.0)


def default_params() -> dict:
    p = _Params()
    _lib.lbm_default_params(ctypes.byref(p))
    return {n: getattr(p, n) for n, _ in _Params._fields_}


def _params_c(overrides: dict | None) -> _Params:
    p = _Params()
    _lib.lbm_default_params(ctypes.byref(p))
    for k, v in (overrides or {}).items():
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "scheme" and isinstance(v, str):
            v = SCHEMES[v]
        if k == "rounding" and isinstance(v, str):
            v = ROUNDINGS[v]
        if k not in _PARAM_DOUBLES and k not in _PARAM_INTS:
            raise LbmError(LBM_EINVAL, f"unknown parameter {k!r}")
        setattr(p, k, v)
    return p


def _bc(v) -> int:
    """Boundary kind in x: 'periodic' | 'heated_outflow' or the LBM_BC_* value."""
    return BOUNDARIES[v] if isinstance(v, str) else int(v)


def maxwell(Tr: float, eos: Eos | None = None) -> dict:
    """Coexistence of the EOS alone at T/Tc = Tr (host thermodynamics of the library)."""
    out = (ctypes.c_double * 4)()
    e = (eos or Eos())._c()
    code = _lib.lbm_maxwell(ctypes.byref(e), float(Tr), out)
    if code != LBM_OK:
        raise LbmError(code, f"no coexistence at Tr = {Tr}")
    return {"rho_v": out[0], "rho_l": out[1], "p_s": out[2], "Tc": out[3]}


def interface_constants(Tr: float, sigma: float = 0.01, W: float = 10.0, eos: Eos | None = None,
                        dx: float = 1.0) -> dict:
    """K_EOS and K_INT for which the flat interface at T/Tc = Tr has surface tension sigma
    and 5 %-95 % width W (the paper's procedure; its 0.01 and 10 at Tr = 0.8 give
    0.479820 and 2.294922).  Host thermodynamics of the library."""
    out = (ctypes.c_double * 2)()
    e = (eos or Eos())._c()
    code = _lib.lbm_interface_constants(ctypes.byref(e), float(Tr), float(sigma), float(W), float(dx), out)
    if code != LBM_OK:
        raise LbmError(code, _lib.lbm_last_error(None).decode())
    return {"K_eos": out[0], "K_int": out[1]}


def _check(code: int, ctx=None):
    if code != LBM_OK:
        msg = _lib.lbm_last_error(ctx).decode() or _lib.lbm_strerror(code).decode()
        raise LbmError(code, msg)


def derived_constants(nx: int, ny: int, eos: Eos | None = None, params: dict | None = None) -> dict:
    """Per-run constants from a host-only context (no GPU needed)."""
    s = Solver(nx, ny, eos=eos, params=params, host_only=True)
    try:
        return s.derived()
    finally:
        s.close()


def workspace_bytes(nx: int, ny: int, params: dict | None = None) -> int:
    lat = _Lattice(nx, ny, float((params or {}).get("dx", 1.0)), _bc((params or {}).get("bc_x", 0)))
    p = _params_c({k: v for k, v in (params or {}).items() if k not in ("dx", "bc_x")})
    out = ctypes.c_size_t()
    _check(_lib.lbm_workspace_bytes(ctypes.byref(lat), ctypes.byref(p), ctypes.byref(out)))
    return out.value


class Solver:
    """One periodic D2Q9 domain bound to a device workspace and a stream.

    params: overrides of the lbm_params fields (see include/lbm.h); 'dx' sets the
    lattice spacing and 'bc_x' the boundaries in x ('periodic' or 'heated_outflow').  precision: 'f64' | 'f32' | 'f16' | 'bf16'; scheme: 'ab' | 'aa';
    rounding (16-bit storage): 'nearest' | 'stochastic'.
    """

    def __init__(self, nx: int, ny: int, *, eos: Eos | None = None, params: dict | None = None,
                 precision: str | None = None, scheme: str | None = None, device=None, stream=None,
                 host_only: bool = False):
        params = dict(params or {})
        dx = float(params.pop("dx", 1.0))
        bc = _bc(params.pop("bc_x", 0))
        if precision is not None:
            params["precision"] = precision
        if scheme is not None:
            params["scheme"] = scheme
        self.nx, self.ny = int(nx), int(ny)
        self._lat = _Lattice(self.nx, self.ny, dx, bc)
        self._eos = (eos or Eos())._c()
        self._p = _params_c(params)
        self._ctx = ctypes.c_void_p()
        self._keep = []
        self.workspace = None
        self.stream = None
        if host_only:
            _check(_lib.lbm_init(ctypes.byref(self._ctx), ctypes.byref(self._lat), ctypes.byref(self._eos),
                                 ctypes.byref(self._p), None, 0, None))
            return
        import torch
        self.device = torch.device(device if device is not None else "cuda", )
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        nbytes = ctypes.c_size_t()
        _check(_lib.lbm_workspace_bytes(ctypes.byref(self._lat), ctypes.byref(self._p), ctypes.byref(nbytes)))
        # allocated on the stream the library uses it on: torch's caching allocator then
        # reuses the memory after this Solver is gone only in that stream's order, after
        # the work still queued on it
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self.workspace = raw[off:off + nbytes.value]
        self._raw = raw
        with torch.cuda.device(self.device):
            _check(_lib.lbm_init(ctypes.byref(self._ctx), ctypes.byref(self._lat), ctypes.byref(self._eos),
                                 ctypes.byref(self._p), ctypes.c_void_p(self.workspace.data_ptr()),
                                 nbytes.value, ctypes.c_void_p(self.stream.cuda_stream)))

    # -- helpers ---------------------------------------------------------------------
    def _dev_f64(self, a):
        import torch
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        a = a.to(device=self.device, dtype=torch.float64).contiguous()
        if tuple(a.shape) != (self.ny, self.nx):
            raise LbmError(LBM_EINVAL, f"field shape {tuple(a.shape)} != {(self.ny, self.nx)}")
        return a

    def _ptr(self, t):
        return ctypes.c_void_p(t.data_ptr()) if t is not None else None

    # -- API -------------------------------------------------------------------------
    def set_fields(self, rho, ux, uy, T):
        import torch
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            ts = [self._dev_f64(a) for a in (rho, ux, uy, T)]
            self._keep = ts
            _check(_lib.lbm_set_fields(self._ctx, *[self._ptr(t) for t in ts]), self._ctx)

    def step(self, n: int = 1):
        _check(_lib.lbm_step(self._ctx, int(n)), self._ctx)

    def moments(self, want=("rho", "ux", "uy", "T")):
        import torch
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
                   for k in ("rho", "ux", "uy", "T")}
            _check(_lib.lbm_moments(self._ctx, self._ptr(out["rho"]),
                                    self._ptr(out["ux"]) if "ux" in want else None,
                                    self._ptr(out["uy"]) if "uy" in want else None,
                                    self._ptr(out["T"]) if "T" in want else None), self._ctx)
        return {k: v for k, v in out.items() if k in want or k == "rho"}

    def moments_numpy(self):
        out = self.moments()
        self.stream.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}

    def invariants(self, raise_on_bad: bool = True) -> dict:
        buf = (ctypes.c_double * 8)()
        code = _lib.lbm_invariants(self._ctx, buf, 8)
        if code != LBM_OK and (raise_on_bad or code != LBM_ENONFINITE):
            _check(code, self._ctx)
        return dict(zip(INVARIANT_NAMES, list(buf)))

    def derived(self) -> dict:
        buf = (ctypes.c_double * 27)()
        _check(_lib.lbm_derived(self._ctx, buf, 27))
        return dict(zip(DERIVED_NAMES, list(buf)))

    def launch_shape(self) -> tuple:
        """(rows per wavefront, wavefronts per workgroup, columns per lane)."""
        r, w, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.lbm_launch_shape(self._ctx, ctypes.byref(r), ctypes.byref(w), ctypes.byref(c)))
        return r.value, w.value, c.value

    @property
    def steps(self) -> int:
        n = ctypes.c_int64()
        _check(_lib.lbm_step_count(self._ctx, ctypes.byref(n)))
        return n.value

    def save_state(self):
        import torch
        nbytes = ctypes.c_size_t()
        _check(_lib.lbm_state_bytes(self._ctx, ctypes.byref(nbytes)))
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            dst = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
            steps = ctypes.c_int64()
            _check(_lib.lbm_save_state(self._ctx, self._ptr(dst), ctypes.byref(steps)), self._ctx)
        return dst, steps.value

    def load_state(self, src, steps: int):
        _check(_lib.lbm_load_state(self._ctx, self._ptr(src), int(steps)), self._ctx)
        self._keep = [src]

    def save(self, path: str):
        """Checkpoint to a file (header + raw state; synchronising)."""
        _check(_lib.lbm_save(self._ctx, os.fsencode(path)), self._ctx)

    def load(self, path: str):
        """Restart from a checkpoint file written for the same configuration."""
        _check(_lib.lbm_load(self._ctx, os.fsencode(path)), self._ctx)

    def close(self):
        if self._ctx:
            _lib.lbm_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent Solvers (two-buffer scheme, one precision, one stream) advanced
    together by one launch per step.  The member Solvers stay usable on their own."""

    def __init__(self, members):
        import torch
        self.members = list(members)
        if not self.members:
            raise LbmError(LBM_EINVAL, "a batch needs at least one member")
        m0 = self.members[0]
        self.stream, self.device = m0.stream, m0.device
        nbytes = ctypes.c_size_t()
        p = int(m0._p.precision)
        code = _lib.lbm_batch_workspace_bytes(len(self.members), p, ctypes.byref(nbytes))
        if code != LBM_OK:
            raise LbmError(code, _lib.lbm_batch_last_error(None).decode())
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):  # see Solver
            raw = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self.workspace = raw[off:off + nbytes.value]
        arr = (ctypes.c_void_p * len(self.members))(*[m._ctx.value for m in self.members])
        self._b = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            code = _lib.lbm_batch_create(ctypes.byref(self._b), arr, len(self.members),
                                         ctypes.c_void_p(self.workspace.data_ptr()), nbytes.value)
        if code != LBM_OK:
            raise LbmError(code, _lib.lbm_batch_last_error(None).decode() or _lib.lbm_strerror(code).decode())

    def _check(self, code):
        if code != LBM_OK:
            raise LbmError(code, _lib.lbm_batch_last_error(self._b).decode() or _lib.lbm_strerror(code).decode())

    def step(self, n: int = 1):
        self._check(_lib.lbm_batch_step(self._b, int(n)))

    def set_shape(self, rows_per_wave: int = 32, waves_per_block: int = 4, queue: bool = False, blocks: int = 0):
        s = _BatchShape(int(rows_per_wave), int(waves_per_block), int(bool(queue)), int(blocks))
        self._check(_lib.lbm_batch_set_shape(self._b, ctypes.byref(s)))

    def shape(self) -> dict:
        s = _BatchShape()
        self._check(_lib.lbm_batch_get_shape(self._b, ctypes.byref(s)))
        return {"rows_per_wave": s.rows_per_wave, "waves_per_block": s.waves_per_block,
                "queue": bool(s.queue), "blocks": s.blocks}

    def set_graph(self, steps_per_graph: int):
        self._check(_lib.lbm_batch_set_graph(self._b, int(steps_per_graph)))

    def autotune(self, steps_per_candidate: int = 10) -> tuple:
        s, ms = _BatchShape(), ctypes.c_double()
        self._check(_lib.lbm_batch_autotune(self._b, int(steps_per_candidate), ctypes.byref(s), ctypes.byref(ms)))
        return ({"rows_per_wave": s.rows_per_wave, "waves_per_block": s.waves_per_block,
                 "queue": bool(s.queue), "blocks": s.blocks}, ms.value)

    def size(self) -> tuple:
        items, nodes = ctypes.c_int64(), ctypes.c_int64()
        self._check(_lib.lbm_batch_size(self._b, ctypes.byref(items), ctypes.byref(nodes)))
        return items.value, nodes.value

    def close(self):
        if self._b:
            _lib.lbm_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
