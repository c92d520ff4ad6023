"""Checkpoint files and in-step failure detection on the GPU, through the C ABI.

* lbm_save / lbm_load: save -> load into a fresh context -> step is bitwise identical to
  the uninterrupted run, for both schemes (the AA scheme restarted at an odd step, where
  its slots are shifted), FP64, FP32 and 16-bit storage with stochastic rounding (whose
  random stream follows the restored step count).  A file for another configuration is
  refused with LBM_EINVAL, a corrupted or truncated one with LBM_EIO, and the context is
  left as it was.
* lbm_params.check_every: lbm_step stops at the first check that finds a bad node and
  returns LBM_ENONFINITE with the step count in the message; a healthy run with checks
  is bitwise the run without them.
"""
import os

import numpy as np
import pytest

from paper_2106_01557_amd import inputs, lbm
from tests.parity_helpers import gpu_solver, oracle_model, say

pytestmark = pytest.mark.gpu


def _fields(nx, ny, seed=3):
    d = oracle_model("cs").d
    return inputs.droplet(nx, ny, d.rho_l, d.rho_v, d.T0, 9, 4, eps=0.01, seed=seed)


@pytest.mark.parametrize("prec,scheme,rounding,split", [("f64", "ab", "nearest", 37), ("f32", "ab", "nearest", 40),
                                                        ("f32", "aa", "nearest", 33),
                                                        ("f16", "ab", "stochastic", 41),
                                                        ("bf16", "ab", "stochastic", 18)])
def test_file_checkpoint_restart_is_bitwise(tmp_path, prec, scheme, rounding, split):
    say(f"case: checkpoint file {prec}/{scheme}/{rounding}, 66x40 droplet, save after {split} of 80 steps")
    params = {"precision": prec, "scheme": scheme, "rounding": rounding}
    f = _fields(66, 40)
    ref = gpu_solver(66, 40, params=params)
    ref.set_fields(*f.as_tuple())
    ref.step(80)
    want = ref.moments_numpy()
    a = gpu_solver(66, 40, params=params)
    a.set_fields(*f.as_tuple())
    a.step(split)
    path = str(tmp_path / "state.lbm")
    a.save(path)
    assert os.path.getsize(path) == 512 + a.save_state()[0].numel()
    a.close()
    b = gpu_solver(66, 40, params=dict(params, rows_per_wave=8))  # another launch shape is allowed
    b.load(path)
    assert b.steps == split
    b.step(80 - split)
    got = b.moments_numpy()
    for k in want:
        assert np.array_equal(got[k], want[k]), (k, float(np.abs(got[k] - want[k]).max()))


def test_file_checkpoint_refuses_other_configurations_and_damaged_files(tmp_path):
    say("case: checkpoint file validation (configuration, checksum, truncation, missing file)")
    f = _fields(32, 24)
    a = gpu_solver(32, 24, params={"precision": "f32"})
    a.set_fields(*f.as_tuple())
    a.step(5)
    path = str(tmp_path / "state.lbm")
    a.save(path)
    before = a.moments_numpy()
    for other, what in (({"precision": "f64"}, "precision"), ({"precision": "f32", "Tr0": 0.75}, "Tr0"),
                        ({"precision": "f32", "scheme": "aa"}, "scheme")):
        b = gpu_solver(32, 24, params=other)
        with pytest.raises(lbm.LbmError) as ei:
            b.load(path)
        assert ei.value.code == lbm.LBM_EINVAL and what in str(ei.value), str(ei.value)
        b.close()
    c = gpu_solver(40, 24, params={"precision": "f32"})
    with pytest.raises(lbm.LbmError) as ei:
        c.load(path)
    assert ei.value.code == lbm.LBM_EINVAL and "lattice size" in str(ei.value)
    c.close()
    raw = bytearray(open(path, "rb").read())
    bad = str(tmp_path / "bad.lbm")
    raw[600] ^= 0x10                      # a payload byte
    open(bad, "wb").write(bytes(raw))
    for damaged in (bad, str(tmp_path / "short.lbm"), str(tmp_path / "missing.lbm")):
        if damaged.endswith("short.lbm"):
            open(damaged, "wb").write(bytes(raw[:1000]))
        with pytest.raises(lbm.LbmError) as ei:
            a.load(damaged)
        assert ei.value.code == lbm.LBM_EIO, str(ei.value)
    # the context kept its own state through the refused loads
    after = a.moments_numpy()
    assert a.steps == 5 and all(np.array_equal(before[k], after[k]) for k in before)


def test_check_every_stops_at_the_first_failing_check():
    say("case: check_every = 25 with one NaN temperature, 200 steps")
    f = _fields(48, 32)
    T = f.T.copy()
    T[10, 7] = np.nan                     # spreads by streaming and never leaves: every check fails
    s = gpu_solver(48, 32, params={"precision": "f32", "check_every": 25})
    s.set_fields(f.rho, f.ux, f.uy, T)
    with pytest.raises(lbm.LbmError) as ei:
        s.step(200)
    assert ei.value.code == lbm.LBM_ENONFINITE
    assert "after 25 steps" in str(ei.value), str(ei.value)
    assert s.steps == 25


def test_check_every_leaves_a_healthy_run_unchanged():
    say("case: check_every = 7 on a healthy droplet, 60 steps, against no checks")
    f = _fields(48, 32)
    out = []
    for every in (0, 7):
        s = gpu_solver(48, 32, params={"precision": "f32", "check_every": every})
        s.set_fields(*f.as_tuple())
        s.step(60)
        assert s.steps == 60
        out.append(s.moments_numpy())
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k])
