"""GPU parity of the fused step on grids that span several solve chunks (1024 nodes each),
with ragged tails, smoothing halos across chunk boundaries and both wall kinds, and of
the births the step's solve launches place."""
import numpy as np
import pytest

import oracle
import synth
from parity_util import TOL_FIELD, by_id, compare_particles, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_28534_amd as P

    P.load_library()
    return P


def work_of(e):
    return {"name": "t", "steps": 1, "precision": "fp32", "ensembles": [e]}


# one node short of a chunk, exactly one chunk of cells (the wall node alone in a second
# chunk), one past, and ragged multi-chunk grids
SIZES = [1023, 1024, 1025, 4097, 6661]


@pytest.mark.parametrize("N", SIZES)
@pytest.mark.parametrize("smooth", [0, 3])
@pytest.mark.parametrize("floating", [False, True])
def test_fused_steps_match_oracle_across_chunks(pic, N, smooth, floating):
    """Three collisionless fused steps: counts and wall tallies exact, particles within the
    FP32 tolerance, rho / phi / E within TOL_FIELD, max |E| of the step's solve equal to
    that of the field read back, the field energy against the oracle's, and the deposit
    left by the last pass summing exactly to the particles alive (a node the solve failed
    to clear would add charge twice)."""
    e = synth.ensemble(N, 20, collisions=False, seed=N + 7 * smooth + (3 if floating else 0),
                       floating=floating, smooth=smooth)
    sim = pic.Sim(work_of(e), fused=True)
    o = oracle.Oracle(e)
    sim.step(3)
    o.step(3)
    gd, od = sim.diag(), o.diag()
    assert gd["count"] == od["count"]
    assert gd["wall_count"] == od["wall_count"]
    for s in range(2):
        compare_particles(sim.particles(0, s), o.particles(s), e["dx"], False, vtol=1e-4, xtol=1e-4)
    g, r = sim.grid(), o.grid()
    for k in ("rho", "phi", "E"):
        assert rel(g[k], r[k]) <= TOL_FIELD, (k, rel(g[k], r[k]))
    if not floating:
        assert g["phi"][0] == 0.0 and g["phi"][N] == 0.0
    assert gd["emax"] == np.max(np.abs(g["E"]))
    assert gd["field_energy"] == pytest.approx(od["field_energy"], rel=2 * TOL_FIELD)
    for s in range(2):
        assert g["Q"][s].sum() == pytest.approx(gd["count"][s], rel=0, abs=1e-6)
    sim.close()


def test_collisional_steps_with_births_in_the_solve(pic):
    """With collisions the graph-replayed fused step ranks and places the previous step's
    births in extra blocks of its two solve kernels: 30 steps on a 5-chunk grid agree with
    the separate-stage run (births placed by kernels of their own) bit for bit, and every
    particle is accounted for."""
    e = synth.ensemble(4500, 25, collisions=True, seed=41, sort_every=20)
    e["ngs_el"], e["ngs_iz"] = 0.1, 0.2
    for sp in e["species"]:
        sp["capacity"] *= 2
    a = pic.Sim(work_of(e), fused=True)
    b = pic.Sim(work_of(e), fused=False)
    a.step(30)
    b.step(30)
    for s in range(2):
        sa, sb = by_id(a.particles(0, s)), by_id(b.particles(0, s))
        for k in ("id", "x", "vx", "vy", "vz"):
            assert np.array_equal(sa[k], sb[k]), (s, k)
    da, db = a.diag(), b.diag()
    assert da["created"] == db["created"] and sum(da["created"]) > 0
    assert np.array_equal(a.grid()["E"], b.grid()["E"])
    n0 = 25 * 4500
    for s in range(2):
        absorbed = da["wall_count"][0][s] + da["wall_count"][1][s]
        assert da["count"][s] + absorbed == n0 + da["created"][s]
    a.close()
    b.close()
