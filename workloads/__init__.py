"""Seeded synthetic inputs for the Saint-Venant--Exner test cases.

This module is shared by the oracle, the GPU path's tests and the benchmark.
It builds initial data only (bed, depth, discharge, parameter fields and
ensemble draws) and contains none of the finite-volume scheme's arithmetic.

Every array is row-major with shape (ny, nx) (1D: shape (nx,)), index
k = j*nx + i, cell centres x_i = (i + 1/2) dx, y_j = (j + 1/2) dy: initial
data are point values at cell centres.

Test cases (paper, section "Numerical test cases"):
  * 1D dune: subsection "1D dune evolution" (bump on [300, 500] m,
    h = 10 - z_b, q0 = 10 m^2/s).
  * 1D antidune: subsection "1D antidune evolution" (parabolic bump on
    [8, 12] m, q0 = 1.7, supercritical Bernoulli depth, h0 = 0.5).
  * 2D dune: subsection "2D dune evolution cases" (bump on
    [300, 500] x [400, 600], h = 10 - z_b, u = q0/h, v = 0).
The benchmark variants (periodic 1D dune with A_g = 1e-3, periodic 2D dune
without the 0.1 m offset, the supercritical Meyer-Peter & Mueller channel,
the Grass ensemble and the adjoint set-up) are parameterised below.
"""
from __future__ import annotations

import dataclasses

import numpy as np

G = 9.81


def cell_centres(n: int, length: float) -> np.ndarray:
    dx = length / n
    return (np.arange(n, dtype=np.float64) + 0.5) * dx


# ----------------------------------------------------------------------------
# 1D dune (subsection "1D dune evolution")
# ----------------------------------------------------------------------------
def dune1d(nx: int = 1000, length: float = 1000.0, q0: float = 10.0,
           base: float = 0.1):
    """Bed 0.1 + sin^2(pi (x-300)/200) on [300, 500], 0.1 elsewhere;
    h = 10 - z_b; hu = q0.  Returns (h, hu, zb, dx)."""
    x = cell_centres(nx, length)
    inside = (x >= 300.0) & (x <= 500.0)
    zb = np.full(nx, base)
    zb[inside] = base + np.sin(np.pi * (x[inside] - 300.0) / 200.0) ** 2
    h = 10.0 - zb
    hu = np.full(nx, q0)
    return h, hu, zb, length / nx


# ----------------------------------------------------------------------------
# 2D dune (subsection "2D dune evolution cases")
# ----------------------------------------------------------------------------
def dune2d(nx: int, ny: int, lx: float = 1000.0, ly: float = 1000.0,
           q0: float = 10.0, base: float = 0.0, amplitude: float = 1.0):
    """Bed base + A sin^2(pi (x-300)/200) sin^2(pi (y-400)/200) on
    [300, 500] x [400, 600], base elsewhere; h = 10 - z_b; hu = q0; hv = 0.
    The paper uses base = 0.1, A = 1; the periodic benchmark uses base = 0.
    Returns (h, hu, hv, zb, dx, dy) with arrays of shape (ny, nx)."""
    x = cell_centres(nx, lx)[None, :]
    y = cell_centres(ny, ly)[:, None]
    inside = (x >= 300.0) & (x <= 500.0) & (y >= 400.0) & (y <= 600.0)
    bump = (np.sin(np.pi * (x - 300.0) / 200.0) ** 2
            * np.sin(np.pi * (y - 400.0) / 200.0) ** 2)
    zb = np.where(inside, base + amplitude * bump, base)
    zb = np.ascontiguousarray(np.broadcast_to(zb, (ny, nx)), dtype=np.float64)
    h = 10.0 - zb
    hu = np.full((ny, nx), q0)
    hv = np.zeros((ny, nx))
    return h, hu, hv, zb, lx / nx, ly / ny


# ----------------------------------------------------------------------------
# Supercritical Bernoulli depth (subsection "1D antidune evolution")
# ----------------------------------------------------------------------------
def bernoulli_supercritical(q0: float, head: float, zb: np.ndarray,
                            h_start: float, g: float = G,
                            iters: int = 60) -> np.ndarray:
    """Solve q0^2/(2 g h^2) + h + z_b = head for h on the supercritical
    branch (h below the critical depth (q0^2/g)^(1/3)) by Newton's method
    started from a supercritical depth."""
    hc = (q0 * q0 / g) ** (1.0 / 3.0)
    if not h_start < hc:
        raise ValueError("start depth must be supercritical")
    h = np.full(zb.shape, h_start, dtype=np.float64)
    for _ in range(iters):
        f = q0 * q0 / (2.0 * g * h * h) + h + zb - head
        df = 1.0 - q0 * q0 / (g * h * h * h)
        h_new = h - f / df
        # stay on the supercritical branch
        h_new = np.minimum(np.maximum(h_new, 0.5 * h), 0.999 * hc)
        if np.max(np.abs(h_new - h)) < 1e-15 * np.max(h):
            h = h_new
            break
        h = h_new
    return h


def antidune1d(nx: int = 2400, length: float = 24.0, q0: float = 1.7,
               h0: float = 0.5, g: float = G):
    """Parabolic bump 0.2 - 0.05 (x-10)^2 on [8, 12], 0 elsewhere; uniform
    discharge q0 and the supercritical Bernoulli depth with the head taken at
    the inflow (h0, z_b(0) = 0).  Returns (h, hu, zb, dx)."""
    x = cell_centres(nx, length)
    zb = np.where((x >= 8.0) & (x <= 12.0), 0.2 - 0.05 * (x - 10.0) ** 2, 0.0)
    head = q0 * q0 / (2.0 * g * h0 * h0) + h0 + 0.0
    h = bernoulli_supercritical(q0, head, zb, h0, g)
    hu = np.full(nx, q0)
    return h, hu, zb, length / nx


# ----------------------------------------------------------------------------
# Meyer-Peter & Mueller channel with Strickler friction
# ----------------------------------------------------------------------------
def mpm_channel(nx: int = 8192, ny: int = 2048, lx: float = 4000.0,
                ly: float = 1000.0, q0: float = 2.0, h0: float = 0.5,
                amp: float = 0.01, wavelength: float = 100.0,
                noise_std: float = 1e-4, seed: int = 0, g: float = G):
    """Bed 0.01 sin(2 pi x / 100) + N(0, 1e-4^2) noise (numpy default_rng
    (seed), drawn as one (ny, nx) array); discharge hu = q0, hv = 0; depth
    from the supercritical Bernoulli relation with the inflow head
    q0^2/(2 g h0^2) + h0 (bed level 0 at the inflow).
    Returns (h, hu, hv, zb, dx, dy)."""
    rng = np.random.default_rng(seed)
    x = cell_centres(nx, lx)[None, :]
    noise = rng.standard_normal((ny, nx))
    zb = amp * np.sin(2.0 * np.pi * x / wavelength) + noise_std * noise
    head = q0 * q0 / (2.0 * g * h0 * h0) + h0
    h = bernoulli_supercritical(q0, head, zb, h0, g)
    hu = np.full((ny, nx), q0)
    hv = np.zeros((ny, nx))
    return h, hu, hv, np.ascontiguousarray(zb), lx / nx, ly / ny


# ----------------------------------------------------------------------------
# Ensemble of Grass runs
# ----------------------------------------------------------------------------
ENSEMBLE_SIZES = (256, 384, 512, 768, 1024)


@dataclasses.dataclass
class Member:
    n: int            # n x n cells on [0, 1000]^2
    Ag: float         # Grass interaction constant
    mg: float         # Grass exponent
    amplitude: float  # bump amplitude


def ensemble_draw(n_members: int = 256, seed: int = 1,
                  sizes=ENSEMBLE_SIZES) -> list:
    """Grid side uniform on `sizes`, A_g log-uniform on [1e-4, 1e-2], m_g
    uniform on [1, 4], bump amplitude uniform on [0.5, 1.0]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_members):
        n = int(sizes[rng.integers(0, len(sizes))])
        ag = float(10.0 ** rng.uniform(-4.0, -2.0))
        mg = float(rng.uniform(1.0, 4.0))
        amp = float(rng.uniform(0.5, 1.0))
        out.append(Member(n, ag, mg, amp))
    return out


def ensemble_member_state(m: Member):
    """Periodic 2D dune of side m.n on [0, 1000]^2 with bump amplitude
    m.amplitude (no base offset), h = 10 - z_b, hu = 10, hv = 0."""
    return dune2d(m.n, m.n, amplitude=m.amplitude)


# ----------------------------------------------------------------------------
# Adjoint set-up: smooth random A_g field
# ----------------------------------------------------------------------------
def smooth_field(nx: int, ny: int, lx: float, ly: float, length_scale: float,
                 seed: int) -> np.ndarray:
    """White noise (default_rng(seed)) filtered by a periodic Gaussian of
    standard deviation `length_scale` (metres) in Fourier space, then scaled
    to max |G| = 1."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((ny, nx))
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=lx / nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=ly / ny)
    filt = np.exp(-0.5 * length_scale ** 2 * (ky[:, None] ** 2 + kx[None, :] ** 2))
    gfield = np.real(np.fft.ifft2(np.fft.fft2(w) * filt))
    return gfield / np.max(np.abs(gfield))


def adjoint_ag_field(nx: int = 1024, ny: int = 1024, lx: float = 1000.0,
                     ly: float = 1000.0, base: float = 1e-3, rel: float = 0.3,
                     length_scale: float = 50.0, seed: int = 2) -> np.ndarray:
    """A_g(x, y) = base (1 + rel G) with G the smooth field above."""
    return base * (1.0 + rel * smooth_field(nx, ny, lx, ly, length_scale, seed))


def smooth_periodic1d(nx: int = 256, length: float = 1000.0, amp: float = 0.05):
    """Small smooth periodic bed for grid-convergence studies:
    z_b = amp (1 + sin(2 pi x / L)), h = 2 - z_b, uniform discharge hu = 1.
    Returns (h, hu, zb, dx)."""
    x = cell_centres(nx, length)
    zb = amp * (1.0 + np.sin(2.0 * np.pi * x / length))
    h = 2.0 - zb
    hu = np.ones(nx)
    return h, hu, zb, length / nx


__all__ = [
    "G", "cell_centres", "dune1d", "dune2d", "bernoulli_supercritical",
    "antidune1d", "mpm_channel", "ENSEMBLE_SIZES", "Member", "ensemble_draw",
    "ensemble_member_state", "smooth_field", "adjoint_ag_field",
    "smooth_periodic1d",
]
