"""The guard between a predicted state and the solver (host logic, CPU tensors)."""
import numpy as np
import torch

from paper_2106_01557_amd.warmstart import guard_prediction


def test_guard_keeps_densities_and_temperatures_in_range():
    rv = torch.tensor([0.01, 0.03], dtype=torch.float64)
    rl = torch.tensor([0.35, 0.28], dtype=torch.float64)
    t0 = torch.tensor([0.07, 0.08], dtype=torch.float64)
    rho = torch.tensor([[[-0.01, 0.002, 0.2, 0.4]], [[0.02, 0.01, 0.3, 0.29]]], dtype=torch.float64)
    T = torch.tensor([[[0.05, 0.07, 0.09, 0.07]], [[0.08, 0.1, 0.06, 0.08]]], dtype=torch.float64)
    r, t = guard_prediction(rho, T, rv, rl, t0)
    want_r = [[[0.005, 0.005, 0.2, 0.35 + 0.05 * 0.34]], [[0.02, 0.015, 0.28 + 0.05 * 0.25, 0.29]]]
    want_t = [[[0.85 * 0.07, 0.07, 1.15 * 0.07, 0.07]], [[0.08, 1.15 * 0.08, 0.85 * 0.08, 0.08]]]
    assert np.allclose(r.numpy(), want_r, rtol=0, atol=1e-15)
    assert np.allclose(t.numpy(), want_t, rtol=0, atol=1e-15)
    # values inside the range pass through unchanged
    inside = (r > 0.5 * rv[:, None, None]) & (r < (rl + 0.05 * (rl - rv))[:, None, None])
    assert torch.equal(r[inside], rho[inside])
