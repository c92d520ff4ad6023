"""GPU parity of the HIP library against the FP64 CPU oracle, through the C ABI.

Bars (stated with the workloads): FP64 storage and arithmetic within 1e-12 of the
oracle after 1000 steps; FP32 within 1e-5; norms in parity_helpers.errors.
Every case prints its name before touching the GPU.
"""
import numpy as np
import pytest

from paper_2106_01557_amd import inputs
from tests.parity_helpers import (assert_close, errors, gpu_moments, gpu_solver, oracle_model,
                                  oracle_moments, patch, say)

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def cs_model():
    return oracle_model("cs")


def c1_fields(d, nx=64, ny=64):
    """Flat slab workload: rows 16-47 liquid, rest vapour (Maxwell densities at T_r0 = 0.8),
    +-1% uniform noise on rho (PCG64 seed 0), fluid at rest, T = T0."""
    return inputs.slab(nx, ny, d.rho_l, d.rho_v, d.T0, 16, 47, eps=0.01, seed=0)


def test_fp64_flat_slab_1000_steps(cs_model):
    d = cs_model.d
    say("case: FP64 AB 64x64 slab, 1000 steps")
    f = c1_fields(d)
    g, s = gpu_moments(64, 64, f, 1000, params={"precision": "f64"})
    o, ost = oracle_moments(cs_model, f, 1000)
    assert_close(g, o, d, TOL64, "fp64 slab")
    # invariants from the device reductions agree with the oracle's
    inv = s.invariants()
    from oracle import lbm as olbm
    oinv = olbm.invariants(cs_model, ost)
    for k in ("mass", "sum_g", "E_p", "E_kin"):
        assert abs(inv[k] - oinv[k]) <= 1e-12 * abs(oinv[k]), (k, inv[k], oinv[k])
    assert abs(inv["dt_sum_q"] - oinv["dt_sum_q"]) <= 1e-12 * abs(oinv["sum_g"])


def test_fp32_droplet_1000_steps():
    model = oracle_model("cs", {"Tr0": 0.75})
    d = model.d
    say("case: FP32 AB 96x80 droplet R=20 W=4, 1000 steps")
    f = inputs.droplet(96, 80, d.rho_l, d.rho_v, d.T0, 20, 4, eps=0.005, seed=1)
    g, _ = gpu_moments(96, 80, f, 1000, params={"precision": "f32", "Tr0": 0.75})
    o, _ = oracle_moments(model, f, 1000)
    assert_close(g, o, d, TOL32, "fp32 droplet")


@pytest.mark.parametrize("shape", [(32, 4), (1, 1), (7, 2), (5, 8), (200, 4), (4, 2), (2, 2)])
def test_fp64_ragged_tiles_and_launch_shapes(cs_model, shape):
    """70 x 45 spans two strips (62 + 8 columns) and, for most shapes, several row chunks
    with a ragged tail; every launch shape gives the same numbers as the oracle."""
    d = cs_model.d
    rows, wpb = shape
    say(f"case: FP64 AB 70x45 random smooth, 60 steps, rows_per_wave={rows} waves_per_block={wpb}")
    f = inputs.random_smooth(70, 45, 0.5 * (d.rho_l + d.rho_v), d.T0, 0.4, 0.05 * d.cs, 0.05, seed=21)
    g, _ = gpu_moments(70, 45, f, 60, params={"precision": "f64", "rows_per_wave": rows, "waves_per_block": wpb})
    o, _ = oracle_moments(cs_model, f, 60)
    assert_close(g, o, d, TOL64, f"shape {shape}")


def test_launch_shapes_are_bitwise_identical(cs_model):
    d = cs_model.d
    say("case: FP64/FP32 AB 130x67 launch-shape bitwise identity")
    f = inputs.droplet(130, 67, d.rho_l, d.rho_v, d.T0, 20, 5, eps=0.01, seed=4)
    for prec in ("f64", "f32"):
        ref = None
        for rows, wpb in [(32, 4), (1, 8), (9, 1), (67, 2), (2, 2), (3, 2), (4, 2)]:
            g, _ = gpu_moments(130, 67, f, 25, params={"precision": prec, "rows_per_wave": rows,
                                                       "waves_per_block": wpb})
            if ref is None:
                ref = g
            else:
                for k in g:
                    assert np.array_equal(g[k], ref[k]), (prec, rows, wpb, k)


@pytest.mark.parametrize("nx,ny", [(70, 45), (130, 67), (200, 96), (2, 5), (256, 3), (4, 130)])
def test_two_column_form_is_bitwise_identical(cs_model, nx, ny):
    """The two-columns-per-lane kernel (even nx, 4- and 2-byte storage) against the
    one-column kernel: same gather slots, halo columns and summation order, so the
    states agree bitwise.  Covers a strip whose only lane is both first and last
    (130 = 128 + 2), nx = 2 (both halo columns wrap onto the strip itself) and
    ragged row chunks."""
    d = cs_model.d
    say(f"case: two-column vs one-column form, {nx}x{ny}, f32/f16/bf16, 25 steps")
    f = inputs.random_smooth(nx, ny, 0.5 * (d.rho_l + d.rho_v), d.T0, 0.4, 0.04 * d.cs, 0.04, seed=nx + ny)
    for prec in ("f32", "f16", "bf16"):
        out = []
        for cols in (1, 2):
            s = gpu_solver(nx, ny, params={"precision": prec, "columns_per_lane": cols, "rows_per_wave": 16})
            assert s.launch_shape()[2] == cols
            g, _ = gpu_moments(nx, ny, f, 25, solver=s)
            out.append(g)
        for k in out[0]:
            assert np.array_equal(out[0][k], out[1][k]), (prec, k, float(np.abs(out[0][k] - out[1][k]).max()))


def test_generic_addressing_path_matches_oracle(cs_model, monkeypatch):
    """Lattices whose state exceeds the 32-bit buffer-offset range take the 64-bit
    addressing path; LBM_GENERIC_ADDRESSING=1 forces it on a small ragged lattice (two
    strips of 64 + 6 columns), which must meet the same bars against the oracle.  The
    two paths are separately compiled, so they agree to rounding, not bitwise."""
    d = cs_model.d
    say("case: FP64/FP32 AB 70x45, generic (64-bit) addressing, 60 steps")
    f = inputs.random_smooth(70, 45, 0.5 * (d.rho_l + d.rho_v), d.T0, 0.4, 0.05 * d.cs, 0.05, seed=22)
    o, _ = oracle_moments(cs_model, f, 60)
    for prec, tol in (("f64", TOL64), ("f32", TOL32)):
        params = {"precision": prec, "rows_per_wave": 16, "waves_per_block": 2}
        monkeypatch.delenv("LBM_GENERIC_ADDRESSING", raising=False)
        a, _ = gpu_moments(70, 45, f, 60, params=params)
        monkeypatch.setenv("LBM_GENERIC_ADDRESSING", "1")
        b, _ = gpu_moments(70, 45, f, 60, params=params)
        monkeypatch.delenv("LBM_GENERIC_ADDRESSING")
        say(f"  {prec}: paths differ by {errors(a, b, d)}")
        assert_close(b, o, d, tol, f"generic addressing {prec}")


@pytest.mark.parametrize("nx,ny", [(1, 64), (64, 1), (2, 2), (3, 5), (62, 3), (63, 2), (124, 7), (1, 1)])
def test_fp64_edge_shapes(cs_model, nx, ny):
    d = cs_model.d
    say(f"case: FP64 AB edge shape {nx}x{ny}, 40 steps")
    f = inputs.random_smooth(nx, ny, 0.5 * (d.rho_l + d.rho_v), d.T0, 0.5, 0.03 * d.cs, 0.03, seed=nx * 100 + ny)
    g, _ = gpu_moments(nx, ny, f, 40, params={"precision": "f64", "rows_per_wave": 4})
    o, _ = oracle_moments(cs_model, f, 40)
    assert_close(g, o, d, TOL64, f"{nx}x{ny}")


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_vdw_droplet(prec, tol):
    model = oracle_model("vdw", {"K_int": 1.0})
    d = model.d
    say(f"case: {prec} AB vdW 48x48 droplet, 300 steps")
    f = inputs.droplet(48, 48, d.rho_l, d.rho_v, d.T0, 12, 4, eps=0.01, seed=5)
    g, _ = gpu_moments(48, 48, f, 300, eos_kind="vdw", params={"precision": prec, "K_int": 1.0})
    o, _ = oracle_moments(model, f, 300)
    assert_close(g, o, d, tol, f"{prec} vdw")


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_external_acceleration(cs_model, prec, tol):
    p = {"accel_x": 2e-4, "accel_y": -1e-4}
    model = oracle_model("cs", p)
    d = model.d
    say(f"case: {prec} AB 40x36 droplet with acceleration, 200 steps")
    f = inputs.droplet(40, 36, d.rho_l, d.rho_v, d.T0, 10, 4, eps=0.01, seed=6)
    g, _ = gpu_moments(40, 36, f, 200, params=dict(p, precision=prec))
    o, _ = oracle_moments(model, f, 200)
    assert_close(g, o, d, tol, f"{prec} accel")


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_aa_scheme_matches_oracle_and_ab(cs_model, prec, tol):
    d = cs_model.d
    say(f"case: {prec} AA vs AB vs oracle 64x48 droplet, 101 steps")
    f = inputs.droplet(64, 48, d.rho_l, d.rho_v, d.T0, 14, 5, eps=0.01, seed=7)
    a, _ = gpu_moments(64, 48, f, 101, params={"precision": prec, "scheme": "aa"})
    b, _ = gpu_moments(64, 48, f, 101, params={"precision": prec, "scheme": "ab"})
    o, _ = oracle_moments(cs_model, f, 101)
    assert_close(a, o, d, tol, f"{prec} aa")
    e = errors(a, b, d)
    say(f"  aa vs ab {e}")
    assert max(e.values()) <= (1e-14 if prec == "f64" else 1e-6)


def test_run_twice_and_checkpoint_are_bitwise(cs_model):
    d = cs_model.d
    say("case: FP32 AB determinism + save/load, 80x60")
    f = inputs.droplet(80, 60, d.rho_l, d.rho_v, d.T0, 15, 4, eps=0.01, seed=8)
    a, _ = gpu_moments(80, 60, f, 57, params={"precision": "f32"})
    b, _ = gpu_moments(80, 60, f, 57, params={"precision": "f32"})
    for k in a:
        assert np.array_equal(a[k], b[k])
    for scheme in ("ab", "aa"):
        s = gpu_solver(80, 60, params={"precision": "f32", "scheme": scheme})
        s.set_fields(*f.as_tuple())
        s.step(31)
        blob, steps = s.save_state()
        s.step(26)
        want = s.moments_numpy()
        s2 = gpu_solver(80, 60, params={"precision": "f32", "scheme": scheme})
        s2.load_state(blob, steps)
        s2.step(26)
        got = s2.moments_numpy()
        for k in got:
            assert np.array_equal(got[k], want[k]), (scheme, k)


def test_gpu_conservation_over_many_steps(cs_model):
    d = cs_model.d
    say("case: FP64 AB conservation 96x96 droplet, 500 steps")
    f = inputs.droplet(96, 96, d.rho_l, d.rho_v, d.T0, 24, 5, eps=0.01, seed=9)
    s = gpu_solver(96, 96, params={"precision": "f64"})
    s.set_fields(*f.as_tuple())
    i0 = s.invariants()
    for _ in range(5):
        before = s.invariants()
        s.step(1)
        after = s.invariants()
        assert abs(after["sum_g"] - before["sum_g"] - before["dt_sum_q"]) <= 1e-13 * abs(before["sum_g"])
        s.step(99)
    i1 = s.invariants()
    assert abs(i1["mass"] / i0["mass"] - 1) < 1e-13
    scale = d.c * i0["mass"]
    assert abs(i1["mom_x"]) < 1e-13 * scale and abs(i1["mom_y"]) < 1e-13 * scale


def test_state_check_flags_bad_state(cs_model):
    from paper_2106_01557_amd import lbm
    d = cs_model.d
    say("case: state check on a negative-temperature node")
    f = inputs.uniform(16, 16, d.rho_v, d.T0)
    f.T[3, 4] = -d.T0
    s = gpu_solver(16, 16, params={"precision": "f64"})
    s.set_fields(*f.as_tuple())
    with pytest.raises(lbm.LbmError) as ei:
        s.invariants()
    assert ei.value.code == lbm.LBM_ENONFINITE
    inv = s.invariants(raise_on_bad=False)
    assert inv["bad_nodes"] == 1.0


def test_call_order_and_workspace_errors():
    import ctypes
    import torch
    from paper_2106_01557_amd import lbm
    say("case: ABI call-order and workspace errors on the device")
    s = gpu_solver(16, 16)
    with pytest.raises(lbm.LbmError) as ei:
        s.step(1)
    assert ei.value.code == lbm.LBM_ESTATE
    lib = lbm.library()
    lat = lbm._Lattice(16, 16, 1.0)
    eos = lbm.Eos()._c()
    p = lbm._params_c({})
    need = lbm.workspace_bytes(16, 16)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    ctx = ctypes.c_void_p()
    code = lib.lbm_init(ctypes.byref(ctx), ctypes.byref(lat), ctypes.byref(eos), ctypes.byref(p),
                        ctypes.c_void_p(ws.data_ptr()), need - 1, None)
    assert code == lbm.LBM_ESPACE and not ctx.value
    assert b"workspace" in lib.lbm_last_error(None)


@pytest.mark.parametrize("scheme", ["ab", "aa"])
def test_zero_steps_is_a_no_op_and_negative_count_is_rejected(cs_model, scheme):
    """lbm_step with n = 0 launches nothing: the moments are bitwise the same before and
    after it, and match the oracle's at t = 0. n < 0 is LBM_EINVAL and leaves the state
    and the step count untouched; stepping afterwards still follows the oracle."""
    from paper_2106_01557_amd import lbm
    d = cs_model.d
    say(f"case: {scheme} FP64 40x24, step(0) and step(-1)")
    f = inputs.random_smooth(40, 24, 0.5 * (d.rho_l + d.rho_v), d.T0, 0.5, 0.03 * d.cs, 0.03, seed=5)
    s = gpu_solver(40, 24, params={"precision": "f64", "scheme": scheme})
    s.set_fields(*f.as_tuple())
    m0 = s.moments_numpy()
    s.step(0)
    m1 = s.moments_numpy()
    with pytest.raises(lbm.LbmError) as ei:
        s.step(-1)
    assert ei.value.code == lbm.LBM_EINVAL
    assert s.steps == 0
    m2 = s.moments_numpy()
    for k in m0:
        assert np.array_equal(m0[k], m1[k]) and np.array_equal(m0[k], m2[k]), k
    o, _ = oracle_moments(cs_model, f, 0)
    assert_close(m0, o, d, TOL64, "t = 0")
    s.step(3)
    o3, _ = oracle_moments(cs_model, f, 3)
    assert_close(s.moments_numpy(), o3, d, TOL64, "3 steps after step(0)")


# ---- full size, in the launch configuration the benchmark times ---------------------------

def _sampled_full_size(prec, tol, steps=8, n=4096):
    """Droplet workload at full size (n x n, R = 512, W = 4, T_r 0.75, +-0.5% noise, seed 1):
    the GPU runs `steps` steps over the whole domain; the oracle runs the same steps on
    periodic patches of the same initial fields around sampled nodes (the update has a
    dependency radius of 2 nodes per step, so a patch's centre is exact)."""
    import torch
    model = oracle_model("cs", {"Tr0": 0.75})
    d = model.d
    say(f"case: {prec} AB full size {n}x{n} droplet, {steps} steps, sampled patches")
    f = inputs.droplet(n, n, d.rho_l, d.rho_v, d.T0, 512, 4, eps=0.005, seed=1)
    s = gpu_solver(n, n, params={"precision": prec, "Tr0": 0.75})
    s.set_fields(*f.as_tuple())
    s.step(steps)
    mom = s.moments()
    s.stream.synchronize()
    half = 2 * steps + 8
    margin = 2 * steps + 2
    c = n // 2
    centres = [(c, c), (c + 512, c), (c, c - 512), (c + 362, c + 362), (0, 0), (n - 1, 5), (17, n - 3),
               (c - 400, c + 300), (1234, 3001), (c + 511, c + 3)]
    worst = {}
    for cy, cx in centres:
        sub = inputs.Fields(*[np.ascontiguousarray(patch(a, cy, cx, half)) for a in f.as_tuple()])
        o, _ = oracle_moments(model, sub, steps)
        ys = (torch.arange(cy - half, cy + half) % n).to(mom["rho"].device)
        xs = (torch.arange(cx - half, cx + half) % n).to(mom["rho"].device)
        g = {k: v[ys][:, xs].cpu().numpy() for k, v in mom.items()}
        inner = (slice(margin, 2 * half - margin), slice(margin, 2 * half - margin))
        e = errors({k: v[inner] for k, v in g.items()}, {k: v[inner] for k, v in o.items()}, d)
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
    say(f"  worst sampled errors {worst}")
    assert max(worst.values()) <= tol
    inv = s.invariants()
    assert inv["bad_nodes"] == 0


def test_fp32_full_size_sampled():
    _sampled_full_size("f32", TOL32)


def test_fp64_full_size_sampled():
    _sampled_full_size("f64", TOL64)


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_near_critical_temperature_matches_oracle(prec, tol):
    """T/Tc = 0.95, a liquid around its coexistence density (linearly stable, so rounding
    differences are not amplified): the equation of state is evaluated in the arithmetic
    precision (FP32 for the FP32 form), where p_EOS cancels by a factor of about 14 but
    p_BE, which enters the collision, does not cancel."""
    model = oracle_model("cs", {"Tr0": 0.95})
    d = model.d
    say(f"case: {prec} AB 64x48 near-critical liquid (T/Tc 0.95) random smooth, 300 steps")
    f = inputs.random_smooth(64, 48, d.rho_l, d.T0, 0.05, 0.03 * d.cs, 0.02, seed=31)
    o, _ = oracle_moments(model, f, 300)
    g, s = gpu_moments(64, 48, f, 300, params={"precision": prec, "Tr0": 0.95})
    assert s.invariants()["bad_nodes"] == 0
    assert_close(g, o, d, tol, f"{prec} near critical")


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_low_temperature_slab_matches_oracle(prec, tol):
    """T/Tc = 0.70, density ratio 39, a sharp (step) slab: the steepest interfaces the
    stable range allows (at 0.65 a sharp step blows up in the oracle and on the GPU
    alike).  FP32 stays within its bar: measured 1.8e-6 (T)."""
    model = oracle_model("cs", {"Tr0": 0.7})
    d = model.d
    say(f"case: {prec} AB 64x48 sharp slab at T/Tc 0.70, 300 steps")
    f = inputs.slab(64, 48, d.rho_l, d.rho_v, d.T0, 12, 35, eps=0.01, seed=7)
    o, _ = oracle_moments(model, f, 300)
    g, s = gpu_moments(64, 48, f, 300, params={"precision": prec, "Tr0": 0.7})
    assert s.invariants()["bad_nodes"] == 0
    assert_close(g, o, d, tol, f"{prec} low-T slab")


# every model parameter away from its default and from the others, so that a swapped or
# dropped constant in the kernel (several rates equal 1 by default) changes the result
# (sigma_q above 1 together with tau_j_v = 0.15 is unstable in the oracle and on the GPU alike)
GENERAL_PARAMS = {"tau_p": 0.7, "varpi": 0.12, "gamma1": -1.5, "gamma2": 1.7, "s_eps": 1.3, "sigma_e": 1.15,
                  "sigma_eps": 0.9, "sigma_q": 0.85, "sigma_p": 0.8, "tau_j_v": 0.15, "lambda_ratio": 6.0,
                  "cv": 5.0, "C_ref": 0.07, "Tr0": 0.78}


@pytest.mark.parametrize("prec,tol", [("f64", TOL64), ("f32", TOL32)])
def test_general_model_parameters_match_oracle(prec, tol):
    """Moving droplet (u = 0.05 c_s) with every relaxation rate, model coefficient and
    heat-capacity constant distinct: all S, L and Y couplings of the collision are active
    and weighted differently (force and velocity both non-zero, so the velocity-dependent
    rows of F_m, q_m, S and Y all act), 1000 steps against the oracle."""
    model = oracle_model("cs", GENERAL_PARAMS)
    d = model.d
    say(f"case: {prec} AB 56x40 moving droplet, general parameters, 1000 steps")
    f = inputs.droplet(56, 40, d.rho_l, d.rho_v, d.T0, 11, 4, eps=0.01, seed=12)
    f = inputs.Fields(f.rho, f.ux + 0.05 * d.cs, f.uy - 0.03 * d.cs, f.T)
    o, ost = oracle_moments(model, f, 1000)
    g, s = gpu_moments(56, 40, f, 1000, params=dict(GENERAL_PARAMS, precision=prec))
    inv = s.invariants()
    assert inv["bad_nodes"] == 0
    assert_close(g, o, d, tol, f"{prec} general parameters")
    # momentum stays what the oracle conserves: the inverse transform reproduces the
    # momentum moments up to unbiased rounding (a rounded 1/6 there grew the FP32 momentum
    # by 3e-8 of itself per step: 8e-7 M c after 1000 steps, and 8e-5 in the density)
    from oracle import lbm as olbm
    oinv = olbm.invariants(model, ost)
    scale = inv["mass"] * d.c
    mtol = 1e-13 if prec == "f64" else 1e-7
    for k in ("mom_x", "mom_y"):
        assert abs(inv[k] - oinv[k]) <= mtol * scale, (k, (inv[k] - oinv[k]) / scale)
