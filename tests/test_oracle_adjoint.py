"""Pins of the FP64 autograd oracle of the collisionless window (CPU only): its forward is
the C oracle's forward, and its gradient matches central finite differences of the C
oracle; the gradient has the symmetries the physics fixes."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import adjoint_torch


def _c_oracle_W(e, st, vx, nsteps, E_ext=None):
    ee = dict(e)
    if E_ext is not None:
        ee["E_ext"] = E_ext
    o = oracle.Oracle(ee, init=False)
    o.set_particles(0, st["x"], vx, st["vy"], st["vz"], st["id"], st["next_id"])
    o.deposit()
    o.step(nsteps)
    o.solve()
    return o.diag()["field_energy"]


@pytest.fixture(scope="module")
def small():
    w = synth.c4_langmuir(ncells=128, ppc=10)
    e = w["ensembles"][0]
    st = synth.quiet_start_state(e)[0]
    return e, st


def test_autograd_forward_equals_c_oracle(small):
    e, st = small
    n = 40
    W_c = _c_oracle_W(e, st, st["vx"], n)
    W_t = adjoint_torch.window_energy(e, torch.tensor(st["x"]), torch.tensor(st["vx"]),
                                      torch.tensor(0.0, dtype=torch.float64), n).item()
    assert abs(W_t - W_c) <= 1e-10 * W_c


def test_autograd_gradient_matches_finite_differences(small):
    e, st = small
    n = 40
    v0 = torch.tensor(st["vx"], requires_grad=True)
    Eext = torch.tensor(0.0, dtype=torch.float64, requires_grad=True)
    W = adjoint_torch.window_energy(e, torch.tensor(st["x"]), v0, Eext, n)
    gv, gE = torch.autograd.grad(W, (v0, Eext))
    gv = gv.numpy()
    d = synth.rademacher(len(st["vx"]), seed=4)
    ad = float(np.dot(gv, d))
    # W is piecewise smooth (cloud-in-cell weights have kinks at nodes): a central
    # difference converges to the gradient once no particle crosses a node within +-h;
    # h = 1e-6 with the FP64 forward keeps rounding noise near 1e-10
    h = 1e-6
    fd = (_c_oracle_W(e, st, st["vx"] + h * d, n) - _c_oracle_W(e, st, st["vx"] - h * d, n)) / (2 * h)
    assert abs(ad - fd) <= 1e-4 * max(abs(fd), 1e-300), (ad, fd)
    # the coarse step of the specification averages over kinks: agreement to a few 1e-3
    h = 1e-3
    fd3 = (_c_oracle_W(e, st, st["vx"] + h * d, n) - _c_oracle_W(e, st, st["vx"] - h * d, n)) / (2 * h)
    assert abs(ad - fd3) <= 2e-2 * abs(fd3)
    # a uniform velocity shift is a change of frame: W is invariant to first order
    assert abs(gv.sum()) <= 1e-3 * np.abs(gv).sum()
    # and so, by the same symmetry, is a uniform external field (up to grid aliasing)
    hE = 1e-4
    fdE = (_c_oracle_W(e, st, st["vx"], n, E_ext=hE) - _c_oracle_W(e, st, st["vx"], n, E_ext=-hE)) / (2 * hE)
    scale = np.abs(gv).sum() * e["dt"] * n
    assert abs(gE.item() - fdE) <= 1e-3 * scale
    assert abs(fdE) <= 1e-2 * scale
