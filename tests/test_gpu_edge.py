"""GPU edge cases of the hot path: empty species, one-cell domains, every particle absorbed
in one step, zero and near-certain collision probability, capacity overflow reported as an
error, and bad injected states rejected on the host."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import by_id, compare_particles, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_28534_amd as P

    P.load_library()
    return P


def work_of(e, precision="fp32"):
    return {"name": "edge", "steps": 1, "precision": precision, "ensembles": [e]}


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_empty_species(pic, prec):
    """No ions at all (ppc 0): the electrons alone match the oracle; with both species empty
    every count and the field stay zero."""
    e = synth.ensemble(96, 20, collisions=False, seed=9)
    e["species"][1]["ppc"] = 0
    e["species"][1]["capacity"] = 1
    sim = pic.Sim(work_of(e, prec), fused=True)
    o = oracle.Oracle(e)
    sim.step(6)
    o.step(6)
    d, od = sim.diag(), o.diag()
    assert d["count"] == od["count"] and d["count"][1] == 0
    assert d["wall_count"] == od["wall_count"]
    compare_particles(sim.particles(0, 0), o.particles(0), e["dx"], prec == "fp64", vtol=1e-4, xtol=1e-4)
    sim.close()
    e2 = synth.ensemble(50, 0, collisions=True, seed=2)
    for sp in e2["species"]:
        sp["capacity"] = 1
    sim2 = pic.Sim(work_of(e2, prec), fused=True)
    sim2.step(3)
    d2 = sim2.diag()
    assert d2["count"] == [0, 0] and d2["pushes"] == 0 and d2["coll"] == [0, 0, 0]
    assert np.all(sim2.grid()["E"] == 0.0)
    sim2.close()


def test_one_cell_domain_rejected(pic):
    """The library needs N >= 2 cells (it states so in its header): one cell is refused."""
    e = synth.ensemble(1, 300, collisions=False, seed=4)
    with pytest.raises(pic.PicError) as ei:
        pic.Sim(work_of(e), fused=True)
    assert ei.value.code == pic.PIC_EINVAL


@pytest.mark.parametrize("ncells", [2, 3])
def test_tiny_domain(pic, ncells):
    """Two and three cells between the walls: steps match the oracle (walls exact)."""
    e = synth.ensemble(ncells, 300, collisions=False, seed=4, B=synth.oblique_B())
    sim = pic.Sim(work_of(e), fused=True)
    o = oracle.Oracle(e)
    for _ in range(3):
        sim.step(1)
        o.step(1)
        d, od = sim.diag(), o.diag()
        assert d["wall_count"] == od["wall_count"]
        assert d["count"] == od["count"]
    for s in range(2):
        compare_particles(sim.particles(0, s), o.particles(s), e["dx"], False, vtol=1e-4, xtol=1e-4)


def test_everything_absorbed(pic):
    """Electrons far faster than the domain is long all leave in the first step; the walls
    tally every one, the next sort compacts them away and later steps run on what is left."""
    e = synth.ensemble(8, 50, collisions=False, seed=6, T_e=1e8, sort_every=1)
    sim = pic.Sim(work_of(e), fused=True)
    o = oracle.Oracle(e)
    sim.step(1)
    o.step(1)
    d, od = sim.diag(), o.diag()
    assert d["wall_count"] == od["wall_count"]
    assert d["count"][0] == od["count"][0]
    n = e["species"][0]["ppc"] * e["ncells"]
    assert d["wall_count"][0][0] + d["wall_count"][1][0] >= 0.98 * n
    sim.step(3)
    o.step(3)
    assert sim.diag()["count"] == o.diag()["count"]
    assert len(sim.particles(0, 0)["id"]) == o.diag()["count"][0]


def test_zero_collision_rate_is_collisionless(pic):
    """With every n_g sigma zero the null-collision bound is zero and no particle is a
    candidate: the run is bit-identical to the collisionless one."""
    e = synth.ensemble(300, 30, collisions=True, seed=12, B=synth.oblique_B())
    e["ngs_el"] = e["ngs_iz"] = e["ngs_cx"] = 0.0
    e2 = dict(e, collisions=False)
    a, b = pic.Sim(work_of(e), fused=True), pic.Sim(work_of(e2), fused=True)
    a.step(12)
    b.step(12)
    assert a.diag()["coll"] == [0, 0, 0]
    for s in range(2):
        pa, pb = by_id(a.particles(0, s)), by_id(b.particles(0, s))
        for k in ("id", "x", "vx", "vy", "vz"):
            assert np.array_equal(pa[k], pb[k]), (s, k)


def test_near_certain_collisions(pic):
    """n_g sigma so large that P_null is close to one: nearly every particle is a candidate,
    so the candidate list is full in every tile.  Decisions and channels match the oracle."""
    N = 40
    e = synth.ensemble(N, 1, seed=21)
    e["ngs_el"], e["ngs_iz"], e["ngs_cx"] = 30.0, 20.0, 5000.0
    n = 40000
    for sp in e["species"]:
        sp["capacity"] = 3 * n
    st = synth.random_state(e, [n, n], seed=31, vscale=[2.0, 3e-2])
    sim = pic.Sim(work_of(e), fused=False)
    sim.set_state(st)
    sim.set_fields(np.zeros(sim.nnodes()))
    sim.set_step(3)
    o = oracle.Oracle(e, init=False)
    o.set_state(st)
    o.set_fields(np.zeros(o.nnodes))
    o.set_step(3)
    sim.collide()
    o.collide()
    gd, od = sim.diag(), o.diag()
    assert gd["coll"] == od["coll"]
    assert gd["created"] == od["created"]
    assert sum(gd["coll"]) > 0.2 * 2 * n
    for s in range(2):
        compare_particles(sim.particles(0, s), o.particles(s), e["dx"], False, vtol=1e-5)


def test_capacity_overflow_is_reported(pic):
    """Ionisation that creates more pairs than the capacity holds: the step reports
    PIC_ECAPACITY (the kernels drop what does not fit) instead of writing out of bounds."""
    e = synth.ensemble(64, 50, seed=5)
    e["ngs_iz"], e["eps_iz"] = 50.0, 0.01
    for sp in e["species"]:
        sp["capacity"] = sp["ppc"] * e["ncells"] + 8
    sim = pic.Sim(work_of(e), fused=True)
    with pytest.raises(pic.PicError) as ei:
        sim.step(3)
    assert ei.value.code == pic.PIC_ECAPACITY
    sim.close()


def test_bad_injected_state_rejected(pic):
    e = synth.ensemble(32, 4, collisions=False, seed=1)
    sim = pic.Sim(work_of(e), fused=False)
    st = synth.random_state(e, [100, 100], seed=2)[0]
    L = e["ncells"] * e["dx"]
    bad = [dict(st, vx=np.where(np.arange(100) == 7, np.nan, st["vx"])),
           dict(st, x=np.where(np.arange(100) == 3, L, st["x"])),
           dict(st, x=np.where(np.arange(100) == 3, -0.1, st["x"])),
           dict(st, id=np.where(np.arange(100) == 5, 2 ** 31, st["id"]).astype(np.uint32))]
    for b in bad:
        with pytest.raises(pic.PicError) as ei:
            sim.set_particles(0, 0, b["x"], b["vx"], b["vy"], b["vz"], b["id"], b["next_id"])
        assert ei.value.code == pic.PIC_EINVAL
    # a good state still goes in afterwards
    sim.set_particles(0, 0, st["x"], st["vx"], st["vy"], st["vz"], st["id"], st["next_id"])
    assert len(sim.particles(0, 0)["id"]) == 100


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("periodic", [False, True])
def test_nonfinite_field_is_reported(pic, prec, periodic):
    """A NaN node field (put in through the test hook) reaches the particles of the cells
    beside that node.  The push drops them (the FP32 pass replaces a non-finite offset
    before it becomes a cell shift; the FP64 push clamps the cell of a non-finite x and
    kills the particle) and sets the sticky flag, which the next call that reads the flags
    reports as PIC_ENONFINITE.  Particles away from the node are pushed as usual."""
    N = 64
    e = synth.ensemble(N, 20, collisions=False, periodic=periodic, seed=9)
    sim = pic.Sim(work_of(e, prec), fused=False)
    E = np.zeros(sim.nnodes())
    E[10] = np.nan
    sim.set_fields(E)
    n0 = len(sim.particles(0, 0)["id"])
    sim.push()
    with pytest.raises(pic.PicError) as ei:
        sim.diag()
    assert ei.value.code == pic.PIC_ENONFINITE
    # the particles of cells 9 and 10 (the two that interpolate from node 10) are gone,
    # the others are still there (nothing else moves them out in one step at E = 0)
    p = sim.particles(0, 0)
    left = n0 - len(p["id"])
    assert 2 * 20 <= left <= 2 * 20 + 12, left
    assert np.all(np.isfinite(p["x"])) and np.all(np.isfinite(p["vx"]))
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_nonfinite_step_is_reported(pic, prec):
    """A charge weight so large that the field overflows (q w = 1e306 at 20 particles per
    cell: the prefix sums reach infinity) makes the solve's field non-finite; pic_step
    reports PIC_ENONFINITE after the step (the push drops every particle the field
    reaches, as above)."""
    e = synth.ensemble(64, 20, collisions=False, nspecies=1, seed=4, sort_every=5)
    e["species"][0]["w"] = 1e306
    sim = pic.Sim(work_of(e, prec), fused=(prec == "fp32"))
    with pytest.raises(pic.PicError) as ei:
        sim.step(1)
    assert ei.value.code == pic.PIC_ENONFINITE
    sim.close()


@pytest.mark.parametrize("fused", [False, True])
def test_fp64_grid_sizes_leave_results_unchanged(pic, fused):
    """The persistent FP64 pass at 16 and 64 blocks (its push and collide stages at half of
    that, so a few blocks steal almost every tile, and one tile can hold shares of cells
    beyond its LDS window) against the default grid: counts exact, particles and field to
    the rounding of the FP64 deposit atomics, whose order follows the schedule."""
    e = synth.ensemble(3000, 30, collisions=True, seed=77, sort_every=5)
    e["ngs_el"], e["ngs_iz"] = 0.1, 0.2
    for sp in e["species"]:
        sp["capacity"] *= 2
    ref = pic.Sim(work_of(e, "fp64"), fused=fused)
    ref.step(12)
    for grid in (16, 64):
        sim = pic.Sim(work_of(e, "fp64"), fused=fused, grid=grid)
        sim.step(12)
        a, b = sim.diag(), ref.diag()
        for key in ("count", "coll", "created", "wall_count", "pushes"):
            assert a[key] == b[key], (grid, key, a[key], b[key])
        for s in range(2):
            compare_particles(sim.particles(0, s), ref.particles(0, s), e["dx"], True, vtol=1e-9, xtol=1e-9)
        E, Er = sim.grid()["E"], ref.grid()["E"]
        assert np.max(np.abs(E - Er)) <= 1e-9 * np.max(np.abs(Er)), grid
        sim.close()
    ref.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_electrons_only_with_ionisation(pic, prec):
    """One species (no ion segment) with collisions: an ionisation creates only the new
    electron, and three steps (the births of each step placed before the next) match the
    oracle: collision and creation counts exact in FP64 and within a few threshold flips in
    FP32, particles by id (FP64), the charge of every particle accounted for."""
    e = synth.ensemble(400, 50, collisions=True, nspecies=1, seed=5)
    e["ngs_el"], e["ngs_iz"] = 0.1, 0.4
    e["species"][0]["capacity"] *= 3
    sim = pic.Sim(work_of(e, prec), fused=(prec == "fp32"))
    o = oracle.Oracle(e)
    sim.step(3)
    o.step(3)
    gd, od = sim.diag(), o.diag()
    slack = 0 if prec == "fp64" else 4
    for k in range(3):
        assert abs(gd["coll"][k] - od["coll"][k]) <= slack, (k, gd["coll"], od["coll"])
    assert abs(gd["created"][0] - od["created"][0]) <= slack
    assert gd["created"][0] > 0 and gd["coll"][1] > 0
    assert gd["wall_count"] == od["wall_count"]
    n0 = 400 * 50
    absorbed = gd["wall_count"][0][0] + gd["wall_count"][1][0]
    assert gd["count"][0] + absorbed == n0 + gd["created"][0]
    if prec == "fp64":
        compare_particles(sim.particles(0, 0), o.particles(0), e["dx"], True, vtol=1e-11, xtol=1e-10)
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_periodic_collisional_steps_match_oracle(pic, prec):
    """A periodic slab over several solve chunks with collisions, births and two sorts:
    eight fused steps against the oracle (wrap at both ends in the push, background charge
    and zero-mean potential in the solve)."""
    e = synth.ensemble(4500, 12, collisions=True, periodic=True, seed=21, sort_every=4)
    e["ngs_el"], e["ngs_iz"] = 0.1, 0.2
    for sp in e["species"]:
        sp["capacity"] *= 2
    sim = pic.Sim(work_of(e, prec), fused=True)
    o = oracle.Oracle(e)
    sim.step(8)
    o.step(8)
    gd, od = sim.diag(), o.diag()
    slack = 0 if prec == "fp64" else 6
    for k in range(3):
        assert abs(gd["coll"][k] - od["coll"][k]) <= slack, (k, gd["coll"], od["coll"])
    for s in range(2):
        assert abs(gd["created"][s] - od["created"][s]) <= slack
        assert abs(gd["count"][s] - od["count"][s]) <= slack
    assert gd["wall_count"] == [[0, 0], [0, 0]]
    g, r = sim.grid(), o.grid()
    # FP32: a collision decision within binary32 rounding of its threshold can flip and move
    # one particle's charge, so the collisional window is held to 1e-4 (the collisionless
    # windows of the parity tests to 1e-5)
    tol = 1e-10 if prec == "fp64" else 1e-4
    for k in ("rho", "phi", "E"):
        assert rel(g[k], r[k]) <= tol, (k, rel(g[k], r[k]))
    if prec == "fp64":
        for s in range(2):
            compare_particles(sim.particles(0, s), o.particles(s), e["dx"], True, vtol=1e-10, xtol=1e-10)
    sim.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_external_field_in_collisional_steps(pic, prec):
    """A uniform external field E_ext in a bounded collisional run: the push adds it at the
    gather and the null-collision bound (R11) adds |q/m| dt |E_ext| to the speed bound; four
    fused steps against the oracle (bound, counts, particles in FP64)."""
    e = synth.ensemble(900, 30, collisions=True, seed=31, E_ext=0.3)
    e["ngs_el"], e["ngs_iz"] = 0.1, 0.2
    for sp in e["species"]:
        sp["capacity"] *= 2
    sim = pic.Sim(work_of(e, prec), fused=True)
    o = oracle.Oracle(e)
    sim.step(4)
    o.step(4)
    gd, od = sim.diag(), o.diag()
    nu_o, _ = o.last_numax()
    assert np.allclose(gd["numax"], nu_o, rtol=(1e-12 if prec == "fp64" else 1e-5), atol=0)
    slack = 0 if prec == "fp64" else 4
    for k in range(3):
        assert abs(gd["coll"][k] - od["coll"][k]) <= slack, (k, gd["coll"], od["coll"])
    assert gd["wall_count"] == od["wall_count"]
    for s in range(2):
        assert abs(gd["count"][s] - od["count"][s]) <= slack
    if prec == "fp64":
        for s in range(2):
            compare_particles(sim.particles(0, s), o.particles(s), e["dx"], True, vtol=1e-10, xtol=1e-10)
    sim.close()
