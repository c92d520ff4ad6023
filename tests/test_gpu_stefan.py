"""The update on a domain bounded in x (the one-dimensional Stefan problem of Eqs.
(20)-(21): heated wall with vapour outflow at x = 0, wall at rest at x = nx - 1, y
periodic) on the GPU, through the C ABI, against oracle/stefan.py.

Parity: FP64 within 1e-12 and FP32 within 1e-5 of the FP64 oracle after 1000 steps (norms
of parity_helpers), on the paper's 1024 x 4 domain with a vapour layer next to the heated
wall, and on a small moving two-phase field with an odd number of rows.  Boundary columns
report the imposed boundary state on both sides.  Launch chunking and file checkpoints
leave the state bitwise unchanged.
"""
import numpy as np
import pytest

from paper_2106_01557_amd import inputs
from tests.parity_helpers import assert_close, oracle_model, say

pytestmark = pytest.mark.gpu

WALL = {"bc_x": "heated_outflow", "Tr_wall": 0.85}


def stefan_fields(d, nx=1024, ny=4, X0=20.0):
    """Vapour next to the heated wall, liquid beyond x = X0 (equilibrium flat profile at T0),
    at rest, T = T0."""
    from oracle import thermo
    eos = thermo.paper_cs_eos()
    z, r = thermo.flat_profile_table(eos, d.T0, d.kappa, 200)
    x = np.arange(nx, dtype=float)
    rho = np.repeat(np.interp(-(x - X0), z, r)[None, :], ny, axis=0)
    return inputs.Fields(rho, 0 * rho, 0 * rho, 0 * rho + d.T0)


def _oracle(model, f, steps, **walls):
    from oracle import stefan
    w = stefan.walls(model, walls.get("Tr_wall", 0.85), walls.get("Tr_far"))
    st = stefan.run(model, w, stefan.init_state(model, *f.as_tuple()), steps)
    return dict(zip(("rho", "ux", "uy", "T"), stefan.moments(model, w, st)))


def _gpu(nx, ny, f, steps, params):
    from paper_2106_01557_amd import lbm
    s = lbm.Solver(nx, ny, params=params)
    s.set_fields(*f.as_tuple())
    s.step(steps)
    return s.moments_numpy(), s


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_stefan_domain_matches_oracle(prec, tol):
    model = oracle_model("cs")
    d = model.d
    say(f"case: {prec} bounded 1024x4 Stefan start (vapour layer 20 nodes), 1000 steps")
    f = stefan_fields(d)
    o = _oracle(model, f, 1000)
    g, s = _gpu(1024, 4, f, 1000, dict(WALL, precision=prec))
    assert s.invariants()["bad_nodes"] == 0
    assert_close(g, o, d, tol, f"{prec} stefan 1024x4")


@pytest.mark.parametrize("prec,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_moving_two_phase_field_between_walls_matches_oracle(prec, tol):
    """Liquid blob in vapour with a velocity field, 37 x 5 (odd rows), far wall at
    T_r 0.82: every boundary path (outflow velocity copied from column 1, density and
    temperature of both walls, the y wrap) with motion through the boundary columns."""
    model = oracle_model("cs")
    d = model.d
    say(f"case: {prec} bounded 37x5 moving two-phase field, 1000 steps")
    f = inputs.random_smooth(37, 5, 0.5 * (d.rho_l + d.rho_v), d.T0, 0.6, 0.05 * d.cs, 0.03, seed=41)
    o = _oracle(model, f, 1000, Tr_wall=0.85, Tr_far=0.82)
    g, s = _gpu(37, 5, f, 1000, dict(WALL, Tr_far=0.82, precision=prec))
    assert s.invariants()["bad_nodes"] == 0
    assert_close(g, o, d, tol, f"{prec} bounded 37x5")


def test_largest_bounded_lattice_matches_oracle():
    """The largest lattice the bounded update takes, 8192 nodes (512 x 16: eight nodes per
    thread of its one workgroup), a moving two-phase field between the walls, FP64 within
    1e-12 of the oracle after 200 steps."""
    model = oracle_model("cs")
    d = model.d
    say("case: f64 bounded 512x16 (8192 nodes, the maximum) moving two-phase field, 200 steps")
    f = inputs.random_smooth(512, 16, 0.5 * (d.rho_l + d.rho_v), d.T0, 0.6, 0.05 * d.cs, 0.03, seed=43)
    o = _oracle(model, f, 200, Tr_wall=0.85, Tr_far=0.82)
    g, s = _gpu(512, 16, f, 200, dict(WALL, Tr_far=0.82, precision="f64"))
    assert s.invariants()["bad_nodes"] == 0
    assert_close(g, o, d, 1e-12, "f64 bounded 512x16")


def test_bounded_stepping_is_chunk_and_restart_invariant(tmp_path):
    say("case: bounded 1024x4 FP32, 5000 steps at once vs in pieces vs through a checkpoint file")
    model = oracle_model("cs")
    f = stefan_fields(model.d)
    a, _ = _gpu(1024, 4, f, 5000, dict(WALL, precision="f32"))
    from paper_2106_01557_amd import lbm
    b = lbm.Solver(1024, 4, params=dict(WALL, precision="f32", check_every=999))
    b.set_fields(*f.as_tuple())
    for n in (1, 2046, 3, 950):
        b.step(n)
    path = str(tmp_path / "bounded.lbm")
    b.save(path)
    c = lbm.Solver(1024, 4, params=dict(WALL, precision="f32", check_every=999))
    c.load(path)
    c.step(5000 - 3000)
    got = c.moments_numpy()
    assert c.steps == 5000
    for k in a:
        assert np.array_equal(a[k], got[k]), k


def test_one_row_equals_every_row_of_a_y_uniform_domain():
    """The Stefan problem is one-dimensional: with a y-uniform state every row of the
    1024 x 4 domain evolves bitwise as the 1024 x 1 domain (whose y neighbours are the row
    itself), so long runs can use one row."""
    model = oracle_model("cs")
    f4 = stefan_fields(model.d, ny=4)
    f1 = stefan_fields(model.d, ny=1)
    say("case: bounded 1024x4 vs 1024x1, y-uniform start, FP64, 3000 steps")
    a, _ = _gpu(1024, 4, f4, 3000, dict(WALL, precision="f64"))
    b, _ = _gpu(1024, 1, f1, 3000, dict(WALL, precision="f64"))
    for k in a:
        for row in range(4):
            assert np.array_equal(a[k][row], b[k][0]), (k, row)


def test_interface_approaches_the_neumann_solution():
    """Eq. (20) holds in the sharp-interface limit: once the vapour layer is much thicker
    than the interface (W = 10 nodes), X_i^2 grows at the rate 4 k^2 alpha_v with k from
    Eq. (21) (Ste = 0.005) and alpha_v = c^2 dt tau_j,v / 3.  From a 20-node layer, 4e6
    FP64 steps (t = 1.6e6, X_i 20 -> 44) on one row: X_i rises monotonically, the rate of
    X_i^2 over successive 1e6-step windows falls toward 4 k^2 alpha_v and ends within 10 %
    of it, and X_i at the end is within 8 % of Eq. (20) with t_0 set by the start
    (X_i(0) = 20).  The paper's own run (its Fig. 1) is ten times longer; the benchmark's
    Stefan workload runs that length."""
    from oracle import stefan, thermo
    model = oracle_model("cs")
    d = model.d
    k = float(thermo.stefan_root(0.005))
    alpha = d.c ** 2 * d.dt * d.tau_j_v / 3.0
    rate = 4 * k * k * alpha
    f = stefan_fields(d, ny=1)
    say("case: bounded 1024x1 FP64, 4e6 steps, interface position against Eq. (20)")
    from paper_2106_01557_amd import lbm
    s = lbm.Solver(1024, 1, params=dict(WALL, precision="f64"))
    s.set_fields(*f.as_tuple())
    ts, xs = [0.0], [stefan.interface_position(f.rho[0], d.rho_v, d.rho_l)]
    for _ in range(16):
        s.step(250_000)
        rho = s.moments_numpy()["rho"][0]
        ts.append(s.steps * d.dt)
        xs.append(stefan.interface_position(rho, d.rho_v, d.rho_l))
    assert s.invariants()["bad_nodes"] == 0
    ts, xs = np.array(ts), np.array(xs)
    rates = [np.polyfit(ts[a:a + 5], xs[a:a + 5] ** 2, 1)[0] / rate for a in (0, 4, 8, 12)]
    x_eq20 = np.sqrt(xs[0] ** 2 + rate * ts[-1])
    say(f"  X_i {xs[0]:.2f} -> {xs[-1]:.3f} (Eq. (20): {x_eq20:.3f}); rate of X_i^2 / 4k^2 alpha_v per window: "
        + ", ".join(f"{r:.4f}" for r in rates))
    assert np.all(np.diff(xs) > 0)
    assert all(b < a for a, b in zip(rates, rates[1:]))
    assert 1.0 - 0.1 < rates[-1] < 1.0 + 0.1
    assert abs(xs[-1] / x_eq20 - 1) < 0.08
