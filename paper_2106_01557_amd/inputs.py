"""Seeded synthetic initial fields (density, velocity, temperature) for the workloads.

This module only shapes arrays: it holds none of the model's arithmetic.  The
coexistence densities and the temperature are arguments, so callers obtain them
from wherever they trust (the library's derived constants for products, the
oracle for tests).  Both the HIP path and the CPU oracle are fed the arrays made
here, so they always start from bit-identical inputs.

Conventions: arrays are float64, C-ordered, indexed [y, x]; node (x, y) sits at
integer coordinates; noise is rho <- rho * (1 + eps * U[-1, 1]) drawn from
numpy's PCG64 with the given seed.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Fields:
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray

    def as_tuple(self):
        return self.rho, self.ux, self.uy, self.T


def _noise(rho: np.ndarray, eps: float, seed: int | None) -> np.ndarray:
    if eps <= 0 or seed is None:
        return rho
    rng = np.random.Generator(np.random.PCG64(seed))
    return rho * (1.0 + eps * rng.uniform(-1.0, 1.0, size=rho.shape))


def _finish(rho, T0, ux=None, uy=None) -> Fields:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    z = np.zeros_like(rho)
    return Fields(rho,
                  z.copy() if ux is None else np.ascontiguousarray(ux, np.float64),
                  z.copy() if uy is None else np.ascontiguousarray(uy, np.float64),
                  np.full_like(rho, T0))


def tanh_blend(r_signed: np.ndarray, rho_in: float, rho_out: float, width: float) -> np.ndarray:
    """rho_in where r_signed << 0, rho_out where r_signed >> 0, tanh of 2 r / width in between."""
    return 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh(2.0 * r_signed / width)


def uniform(nx, ny, rho0, T0, ux0=0.0, uy0=0.0, eps=0.0, seed=None) -> Fields:
    rho = _noise(np.full((ny, nx), float(rho0)), eps, seed)
    return _finish(rho, T0, np.full((ny, nx), float(ux0)), np.full((ny, nx), float(uy0)))


def slab(nx, ny, rho_l, rho_v, T0, y0, y1, width=0.0, eps=0.0, seed=None) -> Fields:
    """Liquid for rows y0 <= y <= y1, vapour elsewhere.  width = 0 gives a sharp step;
    width > 0 a tanh profile whose mid-density points sit half a node outside the
    liquid rows, at y0 - 1/2 and y1 + 1/2."""
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    if width <= 0:
        rho = np.where((y >= y0) & (y <= y1), float(rho_l), float(rho_v))
    else:
        centre = 0.5 * (y0 + y1)
        half = 0.5 * (y1 - y0 + 1)
        rho = tanh_blend(np.abs(y - centre) - half, rho_l, rho_v, width)
    return _finish(_noise(rho, eps, seed), T0)


def heated_layer(nx, ny, rho_l, rho_v, T0, X0, width) -> Fields:
    """Vapour for x < X0 and liquid beyond (the start of the one-dimensional Stefan
    problem: a vapour layer against the heated side x = 0), tanh interface of the given
    width centred at x = X0, uniform in y, at rest, T = T0."""
    x = np.arange(nx, dtype=np.float64)[None, :] * np.ones((ny, 1))
    return _finish(tanh_blend(X0 - x, rho_l, rho_v, width), T0)


def droplet(nx, ny, rho_l, rho_v, T0, radius, width, cx=None, cy=None, eps=0.0, seed=None) -> Fields:
    """A circular liquid droplet (tanh interface of the given width) centred at (nx/2, ny/2)
    unless (cx, cy) are given; distances are not wrapped."""
    cx = nx / 2.0 if cx is None else cx
    cy = ny / 2.0 if cy is None else cy
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return _finish(_noise(tanh_blend(r - radius, rho_l, rho_v, width), eps, seed), T0)


def droplets(nx, ny, rho_l, rho_v, T0, centres, radii, width, eps=0.0, seed=None) -> Fields:
    """Several droplets on a periodic domain: the liquid fraction of each node is the
    largest over droplets of the periodic-image tanh profile."""
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    frac = np.zeros((ny, nx))
    for (cx, cy), rad in zip(centres, radii):
        dx = np.abs(x - cx)
        dx = np.minimum(dx, nx - dx)
        dy = np.abs(y - cy)
        dy = np.minimum(dy, ny - dy)
        r = np.sqrt(dx * dx + dy * dy)
        frac = np.maximum(frac, 0.5 - 0.5 * np.tanh(2.0 * (r - rad) / width))
    rho = rho_v + (rho_l - rho_v) * frac
    return _finish(_noise(rho, eps, seed), T0)


def shear_wave(nx, ny, rho0, T0, amp, mode=1) -> Fields:
    """ux = amp sin(2 pi mode y / ny) at uniform density and temperature."""
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    ux = amp * np.sin(2 * np.pi * mode * y / ny)
    return _finish(np.full((ny, nx), float(rho0)), T0, ux, np.zeros((ny, nx)))


def random_smooth(nx, ny, rho0, T0, amp_rho, amp_u, amp_T, seed, modes=3) -> Fields:
    """Smooth random periodic fields (a few low Fourier modes) for parity tests."""
    rng = np.random.Generator(np.random.PCG64(seed))
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")

    def field():
        out = np.zeros((ny, nx))
        for kx in range(-modes, modes + 1):
            for ky in range(-modes, modes + 1):
                a, ph = rng.uniform(-1, 1), rng.uniform(0, 2 * np.pi)
                out += a * np.cos(2 * np.pi * (kx * x / nx + ky * y / ny) + ph)
        return out / (2 * modes + 1)

    rho = rho0 * (1 + amp_rho * field())
    ux, uy = amp_u * field(), amp_u * field()
    T = T0 * (1 + amp_T * field())
    return Fields(np.ascontiguousarray(rho), np.ascontiguousarray(ux), np.ascontiguousarray(uy),
                  np.ascontiguousarray(T))
