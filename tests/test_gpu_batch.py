"""Batched form on the GPU: heterogeneous lattices (sizes, EOS kinds, temperatures,
precisions) advanced by one launch per step.

Bars: a batch member is bitwise identical to the same lattice stepped alone (the
batched kernel runs the same per-strip code on the member's own constants), under
every launch shape, with graph replays and after members are stepped alone; FP64
members stay within 1e-12 of the FP64 oracle.  Every case prints its name first.
"""
import numpy as np
import pytest

from paper_2106_01557_amd import inputs
from tests.parity_helpers import assert_close, oracle_model, oracle_moments, say

pytestmark = pytest.mark.gpu

# (nx, ny, eos, Tr0, kind): ragged strips (70, 200), row tails for every shape,
# one single-strip member and temperatures across the C4 range
MEMBERS = [
    (70, 45, "cs", 0.75, "droplet"),
    (128, 64, "cs", 0.6, "slab"),
    (64, 130, "vdw", 0.9, "slab"),
    (200, 96, "cs", 0.95, "droplet"),
    (40, 36, "vdw", 0.7, "droplet"),
]


def _fields(nx, ny, d, kind, seed):
    if kind == "slab":
        return inputs.slab(nx, ny, d["rho_l"], d["rho_v"], d["T0"], ny // 4, ny - ny // 4 - 1, eps=0.01,
                           seed=seed, width=4)
    r = min(nx, ny) / 4
    return inputs.droplet(nx, ny, d["rho_l"], d["rho_v"], d["T0"], r, 4, eps=0.01, seed=seed)


def _make(precision, members=MEMBERS, stream=None, extra=None):
    from paper_2106_01557_amd import lbm
    out = []
    for k, (nx, ny, eos, tr, kind) in enumerate(members):
        e = lbm.Eos() if eos == "cs" else lbm.vdw_eos()
        s = lbm.Solver(nx, ny, eos=e, params={"Tr0": tr, "precision": precision, **(extra or {})}, stream=stream)
        f = _fields(nx, ny, s.derived(), kind, seed=10 + k)
        s.set_fields(*f.as_tuple())
        out.append((s, f))
    return out


def _twins(precision, members=MEMBERS, stream=None, extra=None):
    """Two identical sets of solvers: one for the batch, one stepped alone."""
    a = _make(precision, members, stream, extra)
    b = _make(precision, members, stream, extra)
    return [s for s, _ in a], [s for s, _ in b]


def _state(s):
    import torch
    m = s.moments()
    s.stream.synchronize()
    return {k: v.clone() for k, v in m.items()}


def _assert_bitwise(batch_members, alone, label):
    import torch
    for i, (x, y) in enumerate(zip(batch_members, alone)):
        assert x.steps == y.steps, (label, i, x.steps, y.steps)
        a, b = _state(x), _state(y)
        for k in a:
            assert torch.equal(a[k], b[k]), f"{label}: member {i} field {k} differs " \
                f"(max {float((a[k] - b[k]).abs().max())})"


SHAPES = [
    dict(rows_per_wave=32, waves_per_block=4, queue=False),
    dict(rows_per_wave=16, waves_per_block=1, queue=False),
    dict(rows_per_wave=7, waves_per_block=2, queue=False),
    dict(rows_per_wave=64, waves_per_block=4, queue=True),
    dict(rows_per_wave=5, waves_per_block=1, queue=True, blocks=3),
    dict(rows_per_wave=16, waves_per_block=2, queue=True, blocks=8),
    dict(rows_per_wave=128, waves_per_block=4, queue=True, blocks=0),
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "r{rows_per_wave}w{waves_per_block}q{}".format(
    int(s["queue"]), **s) + (f"b{s['blocks']}" if "blocks" in s else ""))
def test_batch_bitwise_equals_alone_fp32(shape):
    from paper_2106_01557_amd import lbm
    say(f"case: FP32 batch of {len(MEMBERS)} heterogeneous members, shape {shape}, 37 steps")
    mine, alone = _twins("f32")
    b = lbm.Batch(mine)
    b.set_shape(**shape)
    b.step(37)
    for s in alone:
        s.step(37)
    _assert_bitwise(mine, alone, f"shape {shape}")
    for s in mine:
        assert s.invariants()["bad_nodes"] == 0


@pytest.mark.parametrize("precision", ["f64", "f16", "bf16"])
def test_batch_bitwise_other_precisions(precision):
    from paper_2106_01557_amd import lbm
    say(f"case: {precision} batch bitwise vs alone, queue mode, 21 steps")
    mine, alone = _twins(precision)
    b = lbm.Batch(mine)
    b.set_shape(rows_per_wave=16, waves_per_block=2, queue=True)
    b.step(21)
    for s in alone:
        s.step(21)
    _assert_bitwise(mine, alone, precision)


@pytest.mark.parametrize("precision", ["f16", "bf16"])
def test_batch_stochastic_rounding_bitwise(precision):
    """Stochastic rounding draws its random bits from each member's step count, which a
    batch keeps in device counters (two per member, by launch parity).  Batched members
    stay bitwise equal to the lattices stepped alone through graph replays in queue mode,
    an odd start parity, and a member stepped alone by an even count (same buffers,
    different step count) between batched steps."""
    import torch
    from paper_2106_01557_amd import lbm
    say(f"case: {precision} stochastic rounding, batch bitwise vs alone, graphs + queue")
    stream = torch.cuda.Stream()
    mine, alone = _twins(precision, stream=stream, extra={"rounding": "stochastic"})
    b = lbm.Batch(mine)
    b.set_shape(rows_per_wave=16, waves_per_block=2, queue=True)
    b.set_graph(8)
    for n in (1, 19, 8):
        b.step(n)
        for s in alone:
            s.step(n)
        _assert_bitwise(mine, alone, f"{precision} sr after {n}")
    mine[1].step(2)
    alone[1].step(2)
    b.step(9)
    for s in alone:
        s.step(9)
    _assert_bitwise(mine, alone, f"{precision} sr after a member stepped alone")


@pytest.mark.parametrize("precision,extra", [("f32", None), ("f16", {"rounding": "stochastic"})])
def test_batch_with_odd_width_members_bitwise(precision, extra):
    """Members of odd width take the one-column form inside the batched kernel (the
    others the two-column form); the mixed batch stays bitwise equal to the lattices
    stepped alone, at the precision's default shape and in queue mode."""
    from paper_2106_01557_amd import lbm
    members = MEMBERS[:2] + [(71, 33, "cs", 0.8, "droplet"), (33, 70, "vdw", 0.75, "slab"), (1, 9, "cs", 0.8, "slab")]
    say(f"case: {precision} batch with odd-width members {extra or ''}, bitwise vs alone")
    mine, alone = _twins(precision, members=members, extra=extra)
    b = lbm.Batch(mine)
    for shape in (None, dict(rows_per_wave=3, waves_per_block=2, queue=True)):
        if shape:
            b.set_shape(**shape)
        b.step(23)
        for s in alone:
            s.step(23)
        _assert_bitwise(mine, alone, f"{precision} odd widths {shape}")


def test_batch_fp64_against_oracle():
    """Two FP64 members (CS droplet at Tr 0.8, vdW slab at Tr 0.7) after 300 batched
    steps match the FP64 oracle run on each alone."""
    from paper_2106_01557_amd import lbm
    say("case: FP64 batch vs oracle, 2 members, 300 steps")
    spec = [(40, 36, "cs", 0.8, "droplet"), (48, 32, "vdw", 0.7, "slab")]
    sols = _make("f64", spec)
    b = lbm.Batch([s for s, _ in sols])
    b.set_shape(rows_per_wave=8, waves_per_block=2, queue=True)
    b.step(300)
    for (s, f), (nx, ny, eos, tr, kind) in zip(sols, spec):
        model = oracle_model(eos, {"Tr0": tr})
        o, _ = oracle_moments(model, f, 300)
        g = s.moments_numpy()
        assert_close(g, o, model.d, 1e-12, f"fp64 batch {eos} {kind} {nx}x{ny}")


def test_batch_graph_replays_match_eager():
    """Graph replays (8 launches each) against eager twins, checked after every call with
    eager work (moments, invariants) between the replays; an odd start parity forces
    one eager launch before the first replay."""
    from paper_2106_01557_amd import lbm
    import torch
    say("case: FP32 batch hipGraph replays vs eager, queue and grid modes")
    stream = torch.cuda.Stream()
    for queue in (True, False):
        mine, alone = _twins("f32", stream=stream)
        b = lbm.Batch(mine)
        b.set_shape(rows_per_wave=16, waves_per_block=2, queue=queue)
        b.set_graph(8)
        b.step(1)
        for s in alone:
            s.step(1)
        for n in (17, 8, 24, 3):
            b.step(n)
            for s in alone:
                s.step(n)
            _assert_bitwise(mine, alone, f"graph queue={queue} after {n}")
            for s in mine:
                s.invariants()


def test_batch_member_stepped_alone_in_between():
    from paper_2106_01557_amd import lbm
    say("case: batch with a member stepped alone between batched steps, and a reset member")
    mine, alone = _twins("f32")
    b = lbm.Batch(mine)
    b.set_shape(rows_per_wave=32, waves_per_block=4, queue=True)
    b.step(5)
    mine[1].step(3)          # parity of member 1 now differs from the others
    b.step(6)
    for s in alone:
        s.step(11)
    alone[1].step(3)
    _assert_bitwise(mine, alone, "after alone-step")
    # reset a member to new fields: the batch re-reads its buffers
    d = mine[2].derived()
    f = _fields(mine[2].nx, mine[2].ny, d, "droplet", seed=99)
    mine[2].set_fields(*f.as_tuple())
    alone[2].set_fields(*f.as_tuple())
    b.step(4)
    for s in alone:
        s.step(4)
    _assert_bitwise(mine, alone, "after reset")


def test_batch_autotune_advances_exactly():
    from paper_2106_01557_amd import lbm
    say("case: batch autotune (2 steps per candidate) keeps states bitwise")
    mine, alone = _twins("f32")
    b = lbm.Batch(mine)
    shape, ms = b.autotune(2)
    say(f"  chosen {shape} at {ms:.4f} ms/step")
    assert shape["rows_per_wave"] in (2, 4, 8, 16, 32, 64, 128) and shape["waves_per_block"] in (1, 2, 4)
    assert ms > 0
    n = mine[0].steps
    assert n == 42 * 4  # 7 row counts x 3 block sizes x 2 modes, 2 warm-up + 2 timed steps each
    for s in alone:
        s.step(n)
    _assert_bitwise(mine, alone, "after autotune")
    assert b.shape()["rows_per_wave"] == shape["rows_per_wave"]


def test_batch_errors():
    from paper_2106_01557_amd import lbm
    say("case: batch argument errors")
    a = lbm.Solver(64, 64, params={"precision": "f32"})
    c = lbm.Solver(64, 64, params={"precision": "f64"})
    d = lbm.Solver(64, 64, params={"precision": "f32", "scheme": "aa"})
    with pytest.raises(lbm.LbmError, match="precision"):
        lbm.Batch([a, c])
    with pytest.raises(lbm.LbmError, match="SCHEME_AB"):
        lbm.Batch([a, d])
    with pytest.raises(lbm.LbmError, match="twice"):
        lbm.Batch([a, a])
    b = lbm.Batch([a])
    with pytest.raises(lbm.LbmError, match="no fields"):
        b.step(1)
    with pytest.raises(lbm.LbmError, match="even"):
        b.set_graph(3)
    with pytest.raises(lbm.LbmError, match="null stream"):
        b.set_graph(4)  # members on the null stream cannot be captured
    with pytest.raises(lbm.LbmError, match="shape"):
        b.set_shape(rows_per_wave=0)
    with pytest.raises(lbm.LbmError, match="shape"):
        b.set_shape(waves_per_block=8)
    with pytest.raises(lbm.LbmError, match=">= 0"):
        b.step(-1)
