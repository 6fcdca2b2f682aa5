"""GPU parity at cell widths other than the workloads' dx = 0.5: a width that is not a power
of two (the FP64 cell index is then a true division, and x / dx can round up to N for x
just below L) and another power of two (where the FP64 pass multiplies by 1 / dx, which
gives the same result)."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import TOL_FIELD, compare_particles, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_28534_amd as P

    P.load_library()
    return P


def work_of(e, precision):
    return {"name": "t", "steps": 1, "precision": precision, "ensembles": [e]}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("dx", [0.35, 0.25])
def test_cell_width_steps_match_oracle(pic, prec, dx):
    """Five collisionless fused steps from the load: counts and wall tallies exact,
    particles within the precision's tolerance, fields within TOL_FIELD."""
    e = synth.ensemble(1500, 20, collisions=False, seed=int(dx * 100) + (1 if prec == "fp64" else 0))
    e["dx"] = dx
    sim = pic.Sim(work_of(e, prec), fused=True)
    o = oracle.Oracle(e)
    sim.step(5)
    o.step(5)
    gd, od = sim.diag(), o.diag()
    assert gd["count"] == od["count"]
    assert gd["wall_count"] == od["wall_count"]
    tol = 1e-10 if prec == "fp64" else 1e-4
    for s in range(2):
        compare_particles(sim.particles(0, s), o.particles(s), dx, prec == "fp64", vtol=tol, xtol=tol)
    g, r = sim.grid(), o.grid()
    for k in ("rho", "phi", "E"):
        assert rel(g[k], r[k]) <= TOL_FIELD, (k, rel(g[k], r[k]))
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_position_just_below_L_stays_in_the_last_cell(pic, prec):
    """x = nextafter(L, 0) with dx = 0.35, where x / dx rounds up to N: the particle
    deposits all of its charge on the wall node, as the oracle does, and the push gathers
    the wall node's field there."""
    N = 10
    e = synth.ensemble(N, 1, collisions=False, seed=3, nspecies=1)
    e["dx"] = 0.35
    e["species"][0]["capacity"] = 64
    L = N * e["dx"]
    x = np.nextafter(L, 0.0)
    assert x < L and x / e["dx"] == N
    xs = np.array([x, 0.45, 2.0])
    zeros = np.zeros(3)
    ids = np.arange(3, dtype=np.uint32)
    sim = pic.Sim(work_of(e, prec), fused=False)
    sim.set_particles(0, 0, xs, zeros, zeros, zeros, ids, 3)
    o = oracle.Oracle(e, init=False)
    o.set_particles(0, list(xs), [0.0] * 3, [0.0] * 3, [0.0] * 3, [0, 1, 2], 3)
    sim.deposit()
    o.deposit()
    Q, Qo = sim.grid()["Q"][0], o.grid()["Q"][0]
    assert Q.sum() == pytest.approx(3.0, abs=1e-6)
    assert Q[N] == pytest.approx(1.0, abs=1e-6)
    assert np.max(np.abs(Q - Qo)) <= 2.0 ** -22
    E = np.arange(N + 1, dtype=np.float64)
    sim.set_fields(E)
    sim.push()
    p = sim.particles(0, 0)
    h = e["species"][0]["q"] / e["species"][0]["m"] * e["dt"]
    k = int(np.where(p["id"] == 0)[0][0])
    assert p["vx"][k] == pytest.approx(h * E[N], rel=1e-6)
    sim.close()
