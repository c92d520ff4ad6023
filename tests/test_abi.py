"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
function include/lbm.h declares, validates its inputs before touching the device,
and derives the same per-run constants as the oracle."""
import ctypes
import dataclasses
import os
import re

import pytest

from oracle import thermo

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header="lbm.h", prefix="lbm_"):
    src = open(os.path.join(ROOT, "include", header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lbm():
    from paper_2106_01557_amd import lbm as mod
    return mod


def test_library_exports_every_declared_function(lbm):
    names = _declared()
    assert len(names) >= 15
    lib = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(lbm.EXPORTED) == names


def test_library_exports_every_network_function(lbm):
    from paper_2106_01557_amd import unet
    names = _declared("unet.h", "unet_")
    assert len(names) >= 15
    lib = ctypes.CDLL(lbm.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(unet.EXPORTED) == names


def test_network_calls_validate_before_launching(lbm):
    from paper_2106_01557_amd import unet
    lib = unet.library()
    V = ctypes.c_void_p
    buf = V(1 << 20)
    # H not a power of two, C_out not a multiple of 16, misaligned tensor, bad ld/off
    assert lib.unet_conv3x3_fwd(buf, 8, 0, buf, None, buf, 16, 0, None, 0, 0, 1, 6, 8, 8, 16, 0, None) == -1
    assert lib.unet_conv3x3_fwd(buf, 8, 0, buf, None, buf, 24, 0, None, 0, 0, 1, 8, 8, 8, 24, 0, None) == -1
    assert lib.unet_conv3x3_fwd(V((1 << 20) + 2), 8, 0, buf, None, buf, 16, 0, None, 0, 0, 1, 8, 8, 8, 16, 0,
                                None) == -1
    assert lib.unet_conv3x3_fwd(buf, 12, 0, buf, None, buf, 16, 0, None, 0, 0, 1, 8, 8, 8, 16, 0, None) == -1
    assert lib.unet_conv3x3_fwd(buf, 8, 0, buf, None, buf, 16, 0, None, 0, 0, 1, 8, 8, 8, 16, 8, None) == -1
    assert "flags" in lib.unet_last_error().decode()
    # two-tensor input and split output: channel ranges and the second tensors checked first
    cat = lib.unet_conv3x3_fwd_cat
    # arguments: x ld off C_x half, x2 ld off, w bias, y ld off C_y, y2 ld off, mask ld off, N H W C_in C_out flags
    assert cat(buf, 64, 0, 104, 1, buf, 32, 0, buf, None, buf, 32, 0, 32, None, 0, 0, None, 0, 0, 1, 8, 8, 96, 32, 0,
               None) == -1
    assert "C_x" in lib.unet_last_error().decode()
    assert cat(buf, 64, 0, 48, 1, buf, 48, 0, buf, None, buf, 32, 0, 32, None, 0, 0, None, 0, 0, 1, 8, 8, 96, 32, 0,
               None) == -1
    assert "of 32" in lib.unet_last_error().decode()
    assert cat(buf, 64, 0, 64, 1, None, 32, 0, buf, None, buf, 32, 0, 32, None, 0, 0, None, 0, 0, 1, 8, 8, 96, 32, 0,
               None) == -1
    assert "x2" in lib.unet_last_error().decode()
    assert cat(buf, 96, 0, 96, 0, buf, 32, 0, buf, None, buf, 32, 0, 32, None, 0, 0, None, 0, 0, 1, 8, 8, 96, 32, 0,
               None) == -1
    assert "x2 must be NULL" in lib.unet_last_error().decode()
    assert cat(buf, 32, 0, 32, 0, None, 0, 0, buf, None, buf, 64, 0, 64, None, 0, 0, None, 0, 0, 1, 8, 8, 32, 96, 0,
               None) == -1
    assert "y2" in lib.unet_last_error().decode()
    assert cat(buf, 32, 0, 32, 0, None, 0, 0, buf, None, buf, 64, 0, 64, buf, 16, 0, None, 0, 0, 1, 8, 8, 32, 96, 0,
               None) == -1  # y2's ld below the 32 channels it receives
    # fused 2x2 forms: bfloat16 only, and UNET_ESHAPE (-2) before any launch for shapes the
    # tiled kernel does not cover
    assert lib.unet_conv3x3_fwd_pool(buf, 32, 0, buf, None, buf, 32, 0, buf, 32, 0, 1, 32, 32, 32, 32, 2, None) == -1
    assert lib.unet_conv3x3_fwd_pool(buf, 32, 0, buf, None, buf, 32, 0, buf, 32, 0, 1, 8, 8, 32, 32, 1, None) == -2
    assert lib.unet_conv3x3_fwd_pool(buf, 16, 0, buf, None, buf, 32, 0, buf, 32, 0, 1, 32, 32, 16, 32, 1, None) == -2
    up = lib.unet_conv3x3_bwd_upcat
    # arguments: g ld off, wf, dlow ld off, low ld off, C_low, dskip ld off, N H W C_g C_in
    assert up(buf, 32, 0, buf, buf, 96, 0, buf, 96, 0, 96, buf, 32, 0, 1, 32, 32, 32, 96, None) == -1
    assert "C_low" in lib.unet_last_error().decode()
    assert up(buf, 32, 0, buf, buf, 64, 0, buf, 64, 0, 64, buf, 32, 0, 1, 8, 8, 32, 96, None) == -2
    assert up(buf, 64, 0, buf, buf, 96, 0, buf, 96, 0, 96, buf, 96, 0, 1, 32, 32, 64, 192, None) == -2  # 96 % 64
    assert up(buf, 32, 0, buf, buf, 64, 0, None, 64, 0, 64, buf, 32, 0, 1, 32, 32, 32, 96, None) == -1  # no gate
    wcat = lib.unet_conv3x3_wgrad_cat
    assert wcat(buf, 64, 0, 60, 1, buf, 36, 0, buf, 32, 0, buf, buf, buf, 1 << 30, 2, 64, 64, 96, 32, None) == -1
    assert "C_x" in lib.unet_last_error().decode()
    assert wcat(buf, 64, 0, 64, 1, None, 32, 0, buf, 32, 0, buf, buf, buf, 1 << 30, 2, 64, 64, 96, 32, None) == -1
    assert "x2" in lib.unet_last_error().decode()
    nb = ctypes.c_size_t()
    assert lib.unet_wgrad_partial_bytes(2, 64, 64, 32, 32, ctypes.byref(nb)) == 0 and nb.value > 0
    assert lib.unet_conv3x3_wgrad(buf, 32, 0, buf, 32, 0, buf, buf, buf, nb.value - 1, 2, 64, 64, 32, 32, None) == -1
    assert lib.unet_adam(buf, buf, buf, buf, None, 10, ctypes.c_float(1e-3), ctypes.c_float(0.9),
                         ctypes.c_float(0.999), ctypes.c_float(1e-8), 0, None) == -1
    # the one-launch flip: n outside [1, 64], a NULL entry, a bad channel count
    ptrs, outs = (V * 65)(*([buf] * 65)), (V * 65)(*([buf] * 65))
    co, ci = (ctypes.c_int32 * 65)(*([16] * 65)), (ctypes.c_int32 * 65)(*([8] * 65))
    assert lib.unet_flip_weights_many(ptrs, outs, co, ci, 0, None) == -1
    assert lib.unet_flip_weights_many(ptrs, outs, co, ci, 65, None) == -1
    holes = (V * 2)(buf, None)
    assert lib.unet_flip_weights_many(holes, outs, co, ci, 2, None) == -1
    assert "entry 1" in lib.unet_last_error().decode()
    co[0] = 0
    assert lib.unet_flip_weights_many(ptrs, outs, co, ci, 1, None) == -1
    # head gradient: C / 8 must divide the 256-thread workgroup
    assert lib.unet_head_bwd(buf, 24, buf, buf, buf, buf, buf, buf, 1 << 30, 1, 8, 8, 24, 2, None) == -1
    assert "C / 8" in lib.unet_last_error().decode()
    # 2x2 calls: one thread per 8 channels of a full-size pixel must fit an int index
    # (N H W = 2^30 passes the geometry check; with C = 16 there are 2^31 threads)
    assert lib.unet_maxpool2_fwd(buf, 16, 0, buf, 16, 0, 1, 1 << 15, 1 << 15, 16, None) == -1
    assert "2^31" in lib.unet_last_error().decode()
    assert lib.unet_maxpool2_bwd(buf, 16, 0, buf, 16, 0, None, 0, 0, buf, 16, 0, 1, 1, 1 << 15, 1 << 15, 16,
                                 None) == -1
    assert lib.unet_upsample2_fwd(buf, 16, 0, buf, 16, 0, 1, 1 << 14, 1 << 14, 16, None) == -1
    assert lib.unet_upsample2_bwd(buf, 16, 0, None, 0, 0, buf, 16, 0, 1, 1 << 14, 1 << 14, 16, None) == -1
    assert "2^31" in lib.unet_last_error().decode()


@pytest.mark.parametrize("eos_kind", ["cs", "vdw"])
@pytest.mark.parametrize("overrides", [{}, {"K_int": 1.0, "Tr0": 0.75}, {"tau_p": 0.8, "varpi": 0.1, "cv": 3.0}])
def test_host_constants_match_oracle(lbm, eos_kind, overrides):
    eos = lbm.Eos() if eos_kind == "cs" else lbm.vdw_eos()
    got = lbm.derived_constants(8, 8, eos=eos, params=overrides)
    oe = thermo.paper_cs_eos() if eos_kind == "cs" else thermo.vdw_eos()
    want = dataclasses.asdict(thermo.derive(oe, thermo.Params(**overrides)))
    assert got.pop("rho_wall") == 0.0  # periodic lattice: no heated wall
    for k, v in got.items():
        assert abs(v - want[k]) <= 1e-14 * max(abs(want[k]), 1e-300), (k, v, want[k])


@pytest.mark.parametrize("Tr_wall,p_out", [(0.85, 0.0), (0.9, 0.0), (0.82, 5e-4), (1.1, 0.0)])
def test_heated_wall_density_matches_oracle(lbm, Tr_wall, p_out):
    """The boundary density of the heated side (vapour root of p_EOS(rho, T_wall) = p_out,
    p_out defaulting to the saturation pressure at T0) from the library's long-double host
    thermodynamics against the 40-digit oracle, also above the critical temperature."""
    from oracle import lbm as olbm
    from oracle import stefan
    params = {"bc_x": "heated_outflow", "Tr_wall": Tr_wall, "p_out": p_out}
    got = lbm.derived_constants(1024, 4, params=params)
    model = olbm.Model.build(thermo.paper_cs_eos(), thermo.Params())
    if Tr_wall >= 1.0:
        pytest.skip("the oracle's wall density stops at the critical temperature")
    w = stefan.walls(model, Tr_wall, p_out=p_out if p_out > 0 else None)
    assert got["rho_wall"] == pytest.approx(w.rho_wall, rel=1e-13)
    assert got["rho_wall"] < got["rho_v"] if p_out == 0.0 else got["rho_wall"] > 0


@pytest.mark.parametrize("params,msg", [
    ({"bc_x": 5}, "bc_x"), ({"bc_x": "heated_outflow", "Tr_wall": 0.0}, "Tr_wall"),
    ({"bc_x": "heated_outflow", "Tr_wall": 0.85, "scheme": "aa"}, "SCHEME_AB"),
    ({"bc_x": "heated_outflow", "Tr_wall": 0.85, "precision": "f16"}, "SCHEME_AB"),
    ({"bc_x": "heated_outflow", "Tr_wall": 0.85, "p_out": 1.0}, "vapour branch"),
])
def test_bounded_lattice_validation(lbm, params, msg):
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Solver(1024, 4, params=params, host_only=True)
    assert ei.value.code == lbm.LBM_EINVAL and msg in str(ei.value), str(ei.value)
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Solver(8192, 2, params={"bc_x": "heated_outflow", "Tr_wall": 0.85}, host_only=True)
    assert "8192" in str(ei.value)


@pytest.mark.parametrize("bad,msg", [
    ({"Tr0": 1.0}, "Tr0"), ({"Tr0": -0.1}, "Tr0"), ({"K_int": 0.0}, "K_int"), ({"varpi": 0.4}, "varpi"),
    ({"tau_p": 0.0}, "tau_p"), ({"sigma_q": 2.0}, "sigma_q"), ({"s_eps": 0.0}, "s_eps"),
    ({"tau_j_v": -1.0}, "tau_j_v"), ({"lambda_ratio": 0.0}, "lambda_ratio"), ({"precision": 7}, "precision"),
    ({"scheme": 3}, "scheme"), ({"waves_per_block": 3}, "waves_per_block"), ({"columns_per_lane": 3}, "columns_per_lane"), ({"cs_override": -1.0}, "cs_override"),
    ({"cv": 0.0, "ste": 0.0}, "cv"), ({"accel_x": float("nan")}, "acceleration"),
    ({"rounding": 2}, "rounding"), ({"rounding": "stochastic"}, "stochastic"),
    ({"rounding": "stochastic", "precision": "f32"}, "stochastic"),
    ({"rounding": "stochastic", "precision": "f16", "scheme": "aa"}, "stochastic"),
    ({"check_every": -1}, "check_every"),
])
def test_invalid_parameters_are_rejected_before_any_device_call(lbm, bad, msg):
    """(stochastic rounding applies to the 16-bit formats of the two-buffer update only)"""
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Solver(16, 16, params=bad, host_only=True)
    assert ei.value.code == lbm.LBM_EINVAL
    assert msg in str(ei.value)


@pytest.mark.parametrize("nx,ny", [(0, 4), (4, 0), (-1, 3), (70000, 40000)])
def test_invalid_shapes_are_rejected(lbm, nx, ny):
    with pytest.raises(lbm.LbmError) as ei:
        lbm.Solver(nx, ny, host_only=True)
    assert ei.value.code == lbm.LBM_EINVAL


def test_invalid_eos_is_rejected(lbm):
    with pytest.raises(lbm.LbmError):
        lbm.Solver(8, 8, eos=lbm.Eos("cs", 1.0, -4.0, 1.0, 1.0), host_only=True)
    with pytest.raises(lbm.LbmError):
        lbm.Solver(8, 8, eos=lbm.Eos("redlich", 1.0, 4.0, 1.0, 1.0), host_only=True)


def test_host_only_context_refuses_device_calls(lbm, tmp_path):
    s = lbm.Solver(8, 8, host_only=True)
    with pytest.raises(lbm.LbmError) as ei:
        s.step(1)
    assert ei.value.code == lbm.LBM_ESTATE
    # checkpoint files: no state to save, none to load into (refused before the file is opened)
    for call in (s.save, s.load):
        with pytest.raises(lbm.LbmError) as ei:
            call(str(tmp_path / "state.lbm"))
        assert ei.value.code == lbm.LBM_ESTATE
    assert not os.path.exists(tmp_path / "state.lbm")
    lib = lbm.library()
    assert lib.lbm_save(None, b"x") == lbm.LBM_EINVAL and lib.lbm_load(None, b"x") == lbm.LBM_EINVAL
    s.close()


def test_check_every_is_a_parameter_with_default_zero(lbm):
    assert lbm.default_params()["check_every"] == 0
    s = lbm.Solver(8, 8, params={"check_every": 100}, host_only=True)
    s.close()


def test_workspace_size_accounts_for_scheme_and_precision(lbm):
    nx, ny = 100, 50
    ab64 = lbm.workspace_bytes(nx, ny, {"precision": "f64"})
    ab32 = lbm.workspace_bytes(nx, ny, {"precision": "f32"})
    aa32 = lbm.workspace_bytes(nx, ny, {"precision": "f32", "scheme": "aa"})
    ab16 = lbm.workspace_bytes(nx, ny, {"precision": "f16"})
    N = nx * ny
    assert ab64 >= 2 * 18 * N * 8
    assert ab32 >= 2 * 18 * N * 4
    assert aa32 < ab32 and aa32 >= 18 * N * 4
    assert ab16 >= 2 * 18 * N * 2 and ab16 < ab32


def test_strerror_covers_codes(lbm):
    lib = lbm.library()
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.lbm_strerror(code).decode() not in ("", "unknown error")
    assert lib.lbm_strerror(-99).decode() == "unknown error"


@pytest.mark.parametrize("eos_kind", ["cs", "vdw"])
@pytest.mark.parametrize("Tr", [0.6, 0.75, 0.8, 0.95])
def test_maxwell_query_matches_oracle(lbm, eos_kind, Tr):
    """lbm_maxwell (long-double host thermodynamics) against the 40-digit oracle."""
    eos = lbm.Eos() if eos_kind == "cs" else lbm.vdw_eos()
    e = thermo.paper_cs_eos() if eos_kind == "cs" else thermo.vdw_eos()
    got = lbm.maxwell(Tr, eos)
    Tc = float(thermo.critical_point(e)[0])
    rv, rl = (float(v) for v in thermo.maxwell(e, Tr * thermo.critical_point(e)[0])[:2])
    assert got["Tc"] == pytest.approx(Tc, rel=1e-14)
    assert got["rho_v"] == pytest.approx(rv, rel=1e-12)
    assert got["rho_l"] == pytest.approx(rl, rel=1e-12)


def test_maxwell_query_rejects_bad_input(lbm):
    for Tr in (0.0, 1.0, 1.2, -0.5, float("nan")):
        with pytest.raises(lbm.LbmError):
            lbm.maxwell(Tr)


def test_batch_validation_before_any_device_call(lbm):
    lib = lbm.library()
    out = ctypes.c_void_p()
    nbytes = ctypes.c_size_t()
    assert lib.lbm_batch_workspace_bytes(0, 1, ctypes.byref(nbytes)) == lbm.LBM_EINVAL
    assert lib.lbm_batch_workspace_bytes(4, 9, ctypes.byref(nbytes)) == lbm.LBM_EINVAL
    assert lib.lbm_batch_workspace_bytes(64, 1, ctypes.byref(nbytes)) == lbm.LBM_OK
    small = nbytes.value
    assert lib.lbm_batch_workspace_bytes(64, 0, ctypes.byref(nbytes)) == lbm.LBM_OK
    assert nbytes.value > small  # FP64 descriptors hold FP64 constants
    s = lbm.Solver(8, 8, host_only=True)
    arr = (ctypes.c_void_p * 1)(s._ctx.value)
    code = lib.lbm_batch_create(ctypes.byref(out), arr, 1, ctypes.c_void_p(1 << 20), 1 << 20)
    assert code == lbm.LBM_ESTATE and not out.value
    assert "host-only" in lib.lbm_batch_last_error(None).decode()
    assert lib.lbm_batch_create(ctypes.byref(out), arr, 0, ctypes.c_void_p(1 << 20), 1 << 20) == lbm.LBM_EINVAL
    null = (ctypes.c_void_p * 1)(None)
    assert lib.lbm_batch_create(ctypes.byref(out), null, 1, ctypes.c_void_p(1 << 20), 1 << 20) == lbm.LBM_EINVAL
    assert lib.lbm_batch_destroy(None) == lbm.LBM_OK
    s.close()


def test_header_is_plain_c_and_the_library_links_from_c(lbm, tmp_path):
    """include/lbm.h compiles as C99 (-Wall -Werror) and a C program linked against
    liblbm.so makes host-only calls (defaults, Maxwell query, a host-only context, error
    strings) with no Python in between."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    src = tmp_path / "abi_check.c"
    src.write_text(r'''
#include <stdio.h>
#include <string.h>
#include "lbm.h"
int main(void) {
    lbm_params p; lbm_eos e; lbm_lattice lat = {32, 16, 1.0, LBM_BC_PERIODIC};
    if (lbm_default_params(&p) != LBM_OK || lbm_default_eos(&e) != LBM_OK) return 1;
    double mx[4];
    if (lbm_maxwell(&e, p.Tr0, mx) != LBM_OK) return 2;
    lbm_ctx* c = NULL;
    if (lbm_init(&c, &lat, &e, &p, NULL, 0, NULL) != LBM_OK || c == NULL) return 3;
    double d[26];
    if (lbm_derived(c, d, 26) != LBM_OK) return 4;
    if (lbm_step(c, 1) != LBM_ESTATE) return 5;
    p.rounding = LBM_ROUND_STOCHASTIC;
    lbm_ctx* bad = NULL;
    if (lbm_init(&bad, &lat, &e, &p, NULL, 0, NULL) != LBM_EINVAL || bad != NULL) return 6;
    if (strlen(lbm_last_error(NULL)) == 0) return 7;
    printf("%.17g %.17g %.17g %.17g %s\n", mx[0], mx[1], d[3], d[8], lbm_strerror(LBM_ESTATE));
    return lbm_destroy(c);
}
''')
    lib_dir = os.path.dirname(lbm.LIB_PATH)
    exe = tmp_path / "abi_check"
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-I", os.path.join(ROOT, "include"), str(src),
           "-o", str(exe), "-L", lib_dir, "-llbm", "-Wl,-rpath," + lib_dir, "-Wl,--allow-shlib-undefined"]
    subprocess.run(cmd, check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert out.returncode == 0, (out.returncode, out.stderr)
    rv, rl, rv_d, dt, msg = out.stdout.split(maxsplit=4)
    want = thermo.maxwell(thermo.paper_cs_eos(), 0.8 * thermo.critical_point(thermo.paper_cs_eos())[0])
    assert float(rv) == pytest.approx(float(want[0]), rel=1e-12)
    assert float(rl) == pytest.approx(float(want[1]), rel=1e-12)
    assert float(rv_d) == float(rv)
    assert float(dt) == pytest.approx(0.401407522, rel=1e-8)
    assert "order" in msg


def test_interface_constants_reproduce_the_paper(lbm, golden):
    """The paper's procedure (sigma and W of the flat interface at T_r0 fix K_EOS and K_INT)
    in the library's host thermodynamics gives the printed pair for sigma = 0.01, W = 10."""
    g = golden["sigma_W_scaling"]
    got = lbm.interface_constants(0.8, g["sigma"], g["W"])
    assert got["K_eos"] == pytest.approx(g["K_eos"], abs=5e-7)
    assert got["K_int"] == pytest.approx(g["K_int"], abs=5e-7)


@pytest.mark.parametrize("eos_kind", ["cs", "vdw"])
@pytest.mark.parametrize("Tr", [0.6, 0.7, 0.9])
def test_interface_constants_match_oracle(lbm, eos_kind, Tr):
    """The constants, fed back into the 40-digit oracle, give the requested tension and
    width (the oracle integrates the same square-gradient definitions with mpmath)."""
    eos = lbm.Eos() if eos_kind == "cs" else lbm.vdw_eos()
    got = lbm.interface_constants(Tr, 0.01, 10.0, eos=eos)
    oe = thermo.paper_cs_eos() if eos_kind == "cs" else thermo.vdw_eos()
    oe = thermo.Eos(oe.kind, oe.a_t, oe.b_t, oe.R, got["K_eos"])
    d = thermo.derive(oe, thermo.Params(Tr0=Tr, K_int=got["K_int"]))
    assert float(thermo.surface_tension(oe, d.T0, d.kappa)) == pytest.approx(0.01, rel=1e-11)
    assert float(thermo.interface_width(oe, d.T0, d.kappa)) == pytest.approx(10.0, rel=1e-11)


def test_interface_constants_reject_bad_input(lbm):
    for args in ((1.0, 0.01, 10.0), (0.8, 0.0, 10.0), (0.8, 0.01, -1.0), (float("nan"), 0.01, 10.0)):
        with pytest.raises(lbm.LbmError):
            lbm.interface_constants(*args)
