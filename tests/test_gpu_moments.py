"""GPU parity of the node moments (reading R27: per-species density, mean velocity and
temperature from the cloud-in-cell shares) against the FP64 oracle, through pic_diag's
moments output.  Tolerance: rel 1e-4 (moments), tighter where the inputs are identical."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import TOL_MOMENT, rel

pytestmark = pytest.mark.gpu

KEYS = ("n", "ux", "uy", "uz", "T")


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


def _compare(gm, om, tol, label):
    for k in KEYS:
        r = rel(gm[k], om[k])
        assert r <= tol, (label, k, r)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("periodic", [False, True])
def test_moments_from_injected_state(pic, prec, periodic):
    """Identical injected particles (sorted and unsorted slots, so both the LDS window and
    the direct HBM path run; several tiles and a ragged tail)."""
    N = 2311
    e = synth.ensemble(N, 6, periodic=periodic, collisions=False, cap_factor=1.0, extra=40000)
    for sort_by_cell in (False, True):
        st = synth.random_state(e, [13007, 9001], seed=51, vscale=[1.4, 0.02], sort_by_cell=sort_by_cell)
        sim = pic.Sim(work_of(e, prec), fused=False)
        sim.set_state(st)
        o = oracle.Oracle(e, init=False)
        o.set_state(st)
        gms = sim.moments()
        for s in range(2):
            tol = 1e-11 if prec == "fp64" else 1e-6
            _compare(gms[s], o.moments(s), tol, (prec, periodic, sort_by_cell, s))
        sim.close()


def test_moments_empty_species_and_single_particle(pic):
    """An empty species gives zeros everywhere; one particle gives its two shares."""
    N = 40
    e = synth.ensemble(N, 1, collisions=False)
    sim = pic.Sim(work_of(e), fused=False)
    x = np.array([(7 + 0.25) * e["dx"]])
    sim.set_particles(0, 0, x, [0.5], [-0.25], [2.0], [3], 10)
    sim.set_particles(0, 1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0, np.uint32), 0)
    o = oracle.Oracle(e, init=False)
    o.set_particles(0, x, [0.5], [-0.25], [2.0], [3], 10)
    o.set_particles(1, np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0, np.uint32), 0)
    gm = sim.moments()
    _compare(gm[0], o.moments(0), 1e-12, "single")
    for k in KEYS:
        assert np.all(gm[1][k] == 0.0)
    assert np.count_nonzero(gm[0]["n"]) == 2


@pytest.mark.parametrize("floating", [False, True])
def test_moments_after_a_fused_window(pic, floating):
    """Twenty fused collisionless steps of the magnetised sheath slab (the graph path):
    moments of both species against the oracle's run, within the moments tolerance."""
    w = synth.scaled(synth.c2_sheath(), ncells=1500, ppc=40)
    e = w["ensembles"][0]
    e["collisions"] = False
    e["floating"] = floating
    sim = pic.Sim(work_of(e), fused=True)
    o = oracle.Oracle(e)
    sim.step(20)
    o.step(20)
    assert sim.diag()["count"] == o.diag()["count"]
    gms = sim.moments()
    for s in range(2):
        _compare(gms[s], o.moments(s), TOL_MOMENT, ("window", floating, s))


def test_moments_of_the_full_size_load(pic):
    """The 4.0e7-particle benchmark workload as loaded: density, flow and temperature of
    both species at all 100,001 nodes against the oracle's load."""
    work = synth.c2_sheath(seed=1)
    e = work["ensembles"][0]
    sim = pic.Sim(work, fused=True)
    gms = sim.moments()
    o = oracle.Oracle(e)
    for s in range(2):
        om = o.moments(s)
        _compare(gms[s], om, 1e-6, ("full", s))
        # and the load's physics: n ~ 1, T ~ T_s
        assert abs(np.mean(gms[s]["n"]) - 1.0) < 1e-2
        assert abs(np.mean(gms[s]["T"]) / e["species"][s]["T"] - 1.0) < 2e-2
    sim.close()
