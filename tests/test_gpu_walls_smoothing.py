"""GPU parity of the floating-wall solve (R22) and the density smoothing (R23) against the
FP64 oracle, on identical seeded inputs from the synth module.

Sizes span several 1024-node solve chunks with a ragged tail, and smoothing stencils that
cross chunk boundaries and fold at the walls (or wrap when periodic).
"""
import numpy as np
import pytest

import oracle
import synth
from parity_util import TOL_FIELD, TOL_MOMENT, by_id, compare_particles, rel

pytestmark = pytest.mark.gpu

PRECISIONS = ["fp32", "fp64"]
BOUNDARIES = ["grounded", "floating", "periodic"]


@pytest.fixture(scope="module")
def pic():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_28534_amd as P

    P.load_library()
    return P


def work_of(e, precision="fp32"):
    return {"name": "t", "steps": 1, "precision": precision, "ensembles": [e]}


def ens(ncells, ppc, boundary, smooth, collisions=False, capacity=None, seed=3, B=None):
    e = synth.ensemble(ncells, ppc, collisions=collisions, periodic=(boundary == "periodic"),
                       floating=(boundary == "floating"), smooth=smooth, seed=seed, B=B)
    if capacity is not None:
        for sp in e["species"]:
            sp["capacity"] = int(capacity)
    return e


def field_tol(prec):
    return TOL_FIELD if prec == "fp32" else 1e-10


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("boundary", BOUNDARIES)
@pytest.mark.parametrize("smooth", [0, 1, 4])
def test_solve_from_injected_state(pic, prec, boundary, smooth):
    N = 4099
    e = ens(N, 3, boundary, smooth, capacity=40000)
    st = synth.random_state(e, [30011, 28999], seed=5 + smooth)
    sim = pic.Sim(work_of(e, prec), fused=False)
    sim.set_state(st)
    o = oracle.Oracle(e, init=False)
    o.set_state(st)
    sim.deposit()
    o.deposit()
    sim.solve()
    o.solve()
    g, r = sim.grid(), o.grid()
    for k in ("rho", "phi", "E"):
        assert rel(g[k], r[k]) <= field_tol(prec), (k, rel(g[k], r[k]))
    if prec == "fp32":
        # the gather table the push reads follows the same node field
        t = sim.gather_table()
        E = g["E"]
        E0 = E[:N]
        assert np.array_equal(t[:, 0], E0.astype(np.float32))


@pytest.mark.parametrize("prec", PRECISIONS)
@pytest.mark.parametrize("smooth", [0, 2])
def test_floating_solve_after_left_wall_absorption(pic, prec, smooth):
    """Particles leave through the left wall in a push in zero field; the next solve puts
    their charge on the wall (E_0 = sigma_L / eps0) and both sides agree on phi and E."""
    N = 2500
    e = ens(N, 5, "floating", smooth, capacity=20000)
    st = synth.random_state(e, [5 * N, 5 * N], seed=29, vscale=[1.0, 0.3])
    for s, k in ((0, 300), (1, 120)):
        st[s]["x"][:k] = np.linspace(1e-3, 0.08, k)
        st[s]["vx"][:k] = -1.0
    sim = pic.Sim(work_of(e, prec), fused=False)
    sim.set_state(st)
    o = oracle.Oracle(e, init=False)
    o.set_state(st)
    sim.set_fields(np.zeros(N + 1))
    o.set_fields(np.zeros(N + 1))
    sim.push()
    o.push()
    o.walls()
    gd, od = sim.diag(), o.diag()
    assert gd["wall_count"] == od["wall_count"]
    assert od["wall_count"][0][0] >= 300 and od["wall_count"][0][1] >= 120
    sim.deposit()
    o.deposit()
    sim.solve()
    o.solve()
    g, r = sim.grid(), o.grid()
    for k in ("rho", "phi", "E"):
        assert rel(g[k], r[k]) <= field_tol(prec), (k, rel(g[k], r[k]))
    sigL = sum(sp["q"] * sp["w"] * gd["wall_count"][0][s] for s, sp in enumerate(e["species"]))
    assert abs(g["E"][0] * e["eps0"] - sigL) <= 1e-12 * abs(sigL)


@pytest.mark.parametrize("prec", PRECISIONS)
def test_floating_smoothed_window_20_steps(pic, prec):
    """Twenty collisionless steps of a magnetised bounded plasma with floating walls and two
    smoothing passes: counts, wall tallies, particles and field against the oracle."""
    w = synth.scaled(synth.c2_sheath(), ncells=1500, ppc=40)
    e = w["ensembles"][0]
    e["collisions"] = False
    e["floating"] = True
    e["smooth"] = 2
    sim = pic.Sim(work_of(e, prec), fused=(prec == "fp32"))
    o = oracle.Oracle(e)
    sim.step(20)
    o.step(20)
    gd, od = sim.diag(), o.diag()
    assert gd["count"] == od["count"]
    assert gd["wall_count"] == od["wall_count"]
    for s in range(2):
        vt = 1e-9 if prec == "fp64" else 1e-4
        compare_particles(sim.particles(0, s), o.particles(s), e["dx"], prec == "fp64", vtol=vt,
                          xtol=(1e-8 if prec == "fp64" else 1e-4))
    g, r = sim.grid(), o.grid()
    assert rel(g["E"], r["E"]) <= (1e-8 if prec == "fp64" else TOL_FIELD), rel(g["E"], r["E"])
    assert rel(g["phi"], r["phi"]) <= (1e-8 if prec == "fp64" else TOL_FIELD), rel(g["phi"], r["phi"])
    for s in range(2):
        assert abs(gd["ke"][s] - od["ke"][s]) <= TOL_MOMENT * abs(od["ke"][s])


def test_floating_smoothed_collisions_fused_graph_equals_separate(pic):
    """With collisions, floating walls and smoothing, the fused graph, fused eager and
    separate-stage runs give the same state bit for bit."""
    w = synth.scaled(synth.c2_sheath(), ncells=1200, ppc=30)
    e = w["ensembles"][0]
    e["ngs_el"], e["ngs_iz"] = 0.1, 0.2
    e["floating"] = True
    e["smooth"] = 1
    for sp in e["species"]:
        sp["capacity"] *= 2
    a = pic.Sim(work_of(e), fused=True)
    b = pic.Sim(work_of(e), fused=True)
    c = pic.Sim(work_of(e), fused=False)
    a.step(25)
    for _ in range(25):
        b.step(1)
    c.step(25)
    sa, sb, sc = ([by_id(x.particles(0, s)) for s in range(2)] for x in (a, b, c))
    for s in range(2):
        for k in ("id", "x", "vx", "vy", "vz"):
            assert np.array_equal(sa[s][k], sb[s][k]), (s, k)
            assert np.array_equal(sa[s][k], sc[s][k]), (s, k)
    assert np.array_equal(a.grid()["E"], c.grid()["E"])


def test_floating_walls_gauss_at_full_size(pic):
    """The 1e5-cell, 200 ppc sheath workload with floating walls and smoothing, 40 fused
    steps: the plasma plus wall charge stays neutral, so eps0 E_0 is the left wall's charge
    and eps0 E_N minus the right wall's (properties that hold at any size)."""
    w = synth.c2_sheath()
    e = w["ensembles"][0]
    e["floating"] = True
    e["smooth"] = 1
    sim = pic.Sim(w, fused=True)
    sim.step(40)
    sim.solve()
    d = sim.diag()
    g = sim.grid()
    sig = [sum(sp["q"] * sp["w"] * d["wall_count"][wall][s] for s, sp in enumerate(e["species"]))
           for wall in range(2)]
    assert d["wall_count"][0][0] > 0 and d["wall_count"][1][0] > 0
    scale = sum(abs(sp["q"] * sp["w"]) * sp["ppc"] * e["ncells"] for sp in e["species"])
    assert abs(e["eps0"] * g["E"][0] - sig[0]) <= 1e-9 * scale
    # FP32 deposit: each particle's shares are rounded to 2^-24
    assert abs(e["eps0"] * g["E"][-1] + sig[1]) <= 1e-9 * scale + 2.0 ** -24 * scale
    assert np.all(np.isfinite(g["phi"]))
