"""FP64 PyTorch (CPU) version of the collisionless periodic window, for an independent
gradient by autograd.

TEST INFRASTRUCTURE ONLY.  The forward is the same discrete method as the C oracle's
steps for one periodic species on a fixed neutralising background with B = 0: cloud-in-cell
deposit (index_add), background removal, the periodic three-point Poisson solve (done here
with the discrete Fourier eigenvalues 2 - 2 cos(2 pi m / N) of the same stencil, a library
primitive), centred-difference node field, linear gather, leapfrog push, periodic wrap.
The objective is the field energy 1/2 eps0 dx sum_j E_j^2 at the final positions.
"""
from __future__ import annotations

import math

import torch


def _field(x, e, dtype=torch.float64):
    N, dx, eps0 = e["ncells"], e["dx"], e["eps0"]
    sp = e["species"][0]
    g = x / dx
    j = torch.floor(g).detach()
    f = g - j
    j = j.long().clamp_(0, N - 1)
    j1 = torch.where(j + 1 == N, torch.zeros_like(j), j + 1)
    Q = torch.zeros(N, dtype=dtype).index_add(0, j, 1.0 - f).index_add(0, j1, f)
    rho = sp["q"] * sp["w"] * Q / dx
    rho = rho - rho.mean()
    m = torch.arange(N, dtype=dtype)
    lam = (2.0 - 2.0 * torch.cos(2.0 * math.pi * m / N)) / (dx * dx)
    lam[0] = 1.0
    rk = torch.fft.fft(rho.to(torch.complex128))
    pk = rk / (lam * eps0)
    pk[0] = 0.0
    phi = torch.fft.ifft(pk).real
    E = (torch.roll(phi, 1) - torch.roll(phi, -1)) / (2.0 * dx)
    return E, j, j1, f


def window_energy(e, x0, vx0, E_ext, nsteps):
    """W after nsteps; x0, vx0 are float64 tensors by particle, E_ext a 0-dim tensor."""
    N, dx, dt = e["ncells"], e["dx"], e["dt"]
    L = N * dx
    sp = e["species"][0]
    qm = sp["q"] / sp["m"]
    x, v = x0, vx0
    for _ in range(nsteps):
        E, j, j1, f = _field(x, e)
        Ep = (1.0 - f) * E[j] + f * E[j1] + E_ext
        v = v + qm * dt * Ep
        x = x + dt * v
        x = x - L * torch.floor(x / L).detach()
    E, _, _, _ = _field(x, e)
    return 0.5 * e["eps0"] * dx * (E * E).sum()
