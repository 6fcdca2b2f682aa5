"""GPU parity for the batched form (many uneven ensembles in one launch per stage) and for
the benchmark workload at its full size, in the launch configuration bench.py times."""
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


def _single(work, k):
    return dict(work, ensembles=[work["ensembles"][k]])


def test_batched_equals_each_ensemble_alone(pic):
    """64 ensembles of uneven size (cells log-uniform, ppc uniform, own seeds) advanced in one
    launch per stage give bit-identical states to each ensemble advanced alone."""
    work = synth.c3_batched(scale=0.04)
    for e in work["ensembles"]:
        e["ngs_el"], e["ngs_iz"] = 0.05, 0.1  # more events in a short run
        for sp in e["species"]:
            sp["capacity"] *= 2
    batch = pic.Sim(work, fused=True)
    batch.step(25)
    for k in (0, 7, 31, 63):
        alone = pic.Sim(_single(work, k), fused=True)
        alone.step(25)
        for s in range(2):
            a, b = by_id(batch.particles(k, s)), by_id(alone.particles(0, s))
            for key in ("id", "x", "vx", "vy", "vz"):
                assert np.array_equal(a[key], b[key]), (k, s, key)
        da, db = batch.diag(k), alone.diag(0)
        for key in ("count", "coll", "created", "wall_count", "pushes"):
            assert da[key] == db[key], (k, key)
        assert np.array_equal(batch.grid(k)["E"], alone.grid(0)["E"])
        alone.close()


@pytest.mark.parametrize("fused", [False, True])
def test_batched_fp64_queues_equal_each_ensemble_alone(pic, fused):
    """The FP64 form's persistent pass takes its tiles from per-XCD queues and steals from
    the others (load balancing inside the GPU).  Twelve uneven ensembles (a 64x spread of
    cells, own seeds, collisions with births) advanced together give each ensemble's own
    run: counts exactly, particles and fields to the rounding of the FP64 deposit atomics,
    whose order follows the schedule.  Several steps, so the queues are reused after
    their reset."""
    work = synth.c3_batched(n_ens=12, seed=11, scale=0.02)
    work["precision"] = "fp64"
    for e in work["ensembles"]:
        e["ngs_el"], e["ngs_iz"] = 0.05, 0.1
        for sp in e["species"]:
            sp["capacity"] *= 2
    batch = pic.Sim(work, fused=fused)
    batch.step(8)
    for k in (0, 5, 11):
        alone = pic.Sim(_single(work, k), fused=fused)
        alone.step(8)
        da, db = batch.diag(k), alone.diag(0)
        for key in ("count", "coll", "created", "wall_count", "pushes"):
            assert da[key] == db[key], (k, key, da[key], db[key])
        for s in range(2):
            compare_particles(batch.particles(k, s), alone.particles(0, s), work["ensembles"][k]["dx"], True,
                              vtol=1e-9, xtol=1e-9)
        assert rel(batch.grid(k)["E"], alone.grid(0)["E"]) <= 1e-9
        alone.close()
    batch.close()


def test_batched_collisionless_window_matches_oracle(pic):
    work = synth.c3_batched(n_ens=12, seed=7, scale=0.03)
    for e in work["ensembles"]:
        e["collisions"] = False
    batch = pic.Sim(work, fused=True)
    batch.step(10)
    for k, e in enumerate(work["ensembles"]):
        o = oracle.Oracle(e)
        o.step(10)
        gd, od = batch.diag(k), o.diag()
        assert gd["count"] == od["count"], k
        assert gd["wall_count"] == od["wall_count"], k
        for s in range(2):
            compare_particles(batch.particles(k, s), o.particles(s), e["dx"], False, vtol=1e-4, xtol=1e-4)
        assert rel(batch.grid(k)["E"], o.grid()["E"]) <= TOL_FIELD, (k, rel(batch.grid(k)["E"], o.grid()["E"]))


def test_bench_workload_full_size_one_step(pic):
    """The 1e5-cell x 200-ppc x 2-species workload (4.0e7 particles) at full size: the load
    matches the oracle bit for bit in position, and one fused step matches the oracle's step
    (fields within 1e-5, counts exact up to threshold-flipped collision decisions)."""
    import bench

    work = synth.c2_sheath(seed=1)
    e = work["ensembles"][0]
    shape = bench.tuned_shape(pic, work, 2)   # the launch shape bench.py times
    sim = pic.Sim(work, fused=True, **shape)
    o = oracle.Oracle(e)
    g0 = sim.grid()
    r0 = o.grid()
    n = e["species"][0]["ppc"] * e["ncells"]
    for s in range(2):
        assert g0["Q"][s].sum() == n
        # sampled load, particle by particle
        idx = np.random.default_rng(s).integers(0, n, size=20000)
        raw = sim.slots(0, s, 0, n)
        op = o.particles(s)
        assert np.array_equal(raw["id"], np.arange(n, dtype=np.uint32))
        assert np.array_equal(raw["x"], op["x"])
        assert np.max(np.abs(raw["vx"][idx] - op["vx"][idx])) <= 2**-23 * np.max(np.abs(op["vx"]))
    sim.solve()
    o.solve()
    assert rel(sim.grid()["E"], o.grid()["E"]) <= TOL_FIELD
    del g0, r0
    # one full step from the load (the step re-solves, which is idempotent)
    sim.close()
    sim2 = pic.Sim(work, fused=True, **shape)
    o2 = oracle.Oracle(e)
    sim2.step(1)
    o2.step(1)
    gd, od = sim2.diag(), o2.diag()
    assert gd["wall_count"] == od["wall_count"]
    for k in range(3):
        assert abs(gd["coll"][k] - od["coll"][k]) <= 5, (k, gd["coll"], od["coll"])
    for s in range(2):
        assert abs(gd["count"][s] - od["count"][s]) <= 5
        assert abs(gd["ke"][s] - od["ke"][s]) <= 1e-4 * od["ke"][s]
    # particle-wise after one step: all particles whose collision decision agrees
    for s in range(2):
        G, R = by_id(sim2.particles(0, s)), by_id(o2.particles(s))
        common = np.intersect1d(G["id"], R["id"])
        gi = np.isin(G["id"], common)
        ri = np.isin(R["id"], common)
        dv = np.abs(G["vx"][gi] - R["vx"][ri])
        vmax = np.max(np.abs(R["vx"]))
        bad = dv > 1e-5 * vmax                      # collided on one side only (rare)
        assert bad.sum() <= 10, bad.sum()
        dx = np.abs(G["x"][gi] - R["x"][ri])[~bad] / e["dx"]
        assert np.max(dx) <= 1e-5


def test_large_share_properties(pic):
    """1e6 cells x 500 ppc x 2 species (1.0e9 particles, about 60 GB of device memory): the
    load is exact on sampled particles, the deposit holds exactly P shares, and after one
    fused step alive + absorbed = loaded + created for each species."""
    import torch

    free, total = torch.cuda.mem_get_info()
    work = synth.c5_large(seed=1)
    e = work["ensembles"][0]
    import ctypes as C

    cfg, keep = pic.make_config(work)
    nb = C.c_size_t(0)
    pic.load_library().pic_query_workspace(C.byref(cfg), C.byref(nb))
    if nb.value > 0.9 * free:
        pytest.skip("not enough device memory")
    sim = pic.Sim(work, fused=True)
    n = e["species"][0]["ppc"] * e["ncells"]
    rng = np.random.default_rng(5)
    for s in range(2):
        ps = np.sort(rng.integers(0, n, size=2000))
        ref = oracle.init_particles(e, s, ps)
        lo = 0
        # read back in a few windows around the samples
        for chunk in np.array_split(ps, 4):
            first, last = int(chunk[0]), int(chunk[-1]) + 1
            raw = sim.slots(0, s, first, last - first)
            sel = chunk - first
            assert np.array_equal(raw["id"][sel], chunk.astype(np.uint32))
            r = {k: ref[k][lo:lo + len(chunk)] for k in ("x", "vx")}
            assert np.array_equal(raw["x"][sel], r["x"])
            assert np.max(np.abs(raw["vx"][sel] - r["vx"])) <= 2**-23 * max(np.max(np.abs(r["vx"])), 1e-30)
            lo += len(chunk)
    g = sim.grid()
    for s in range(2):
        assert g["Q"][s].sum() == n
    sim.step(1)
    d = sim.diag()
    for s in range(2):
        absorbed = d["wall_count"][0][s] + d["wall_count"][1][s]
        assert d["count"][s] + absorbed == n + d["created"][s]
    assert d["pushes"] == 2 * n
    sim.close()
    del sim
    torch.cuda.empty_cache()


def test_large_share_one_percent_slice_matches_oracle(pic):
    """A 1% slice of the 1e9-particle workload at its own density (1e4 cells x 500 ppc x 2
    species, sort every 10): three fused steps against the oracle's."""
    work = synth.c5_large(seed=1, ncells=10_000, ppc=500)
    e = work["ensembles"][0]
    sim = pic.Sim(work, fused=True)
    o = oracle.Oracle(e)
    sim.step(3)
    o.step(3)
    gd, od = sim.diag(), o.diag()
    assert gd["wall_count"] == od["wall_count"]
    assert gd["pushes"] == od["pushes"]
    for s in range(2):
        # FP32 velocities can flip a collision decision that sits within rounding of its
        # threshold; each flip can change a count by one
        assert abs(gd["count"][s] - od["count"][s]) <= 5, (s, gd["count"], od["count"])
        assert abs(gd["ke"][s] - od["ke"][s]) <= 1e-4 * abs(od["ke"][s])
    for k in range(3):
        assert abs(gd["coll"][k] - od["coll"][k]) <= 5, (k, gd["coll"], od["coll"])
    g, r = sim.grid(), o.grid()
    assert rel(g["E"], r["E"]) <= 1e-5


def test_maximum_ensemble_count_equals_each_ensemble_alone(pic):
    """PIC_MAX_ENSEMBLES (256) small uneven ensembles with collisions in one run (every
    staged table of the births placement and the candidate kernel at its largest): twelve
    fused steps, then a few ensembles checked bit for bit against each run alone."""
    work = synth.c3_batched(n_ens=256, seed=5, scale=0.004)
    for e in work["ensembles"]:
        e["ngs_el"], e["ngs_iz"] = 0.05, 0.1
        for sp in e["species"]:
            sp["capacity"] *= 2
    batch = pic.Sim(work, fused=True)
    batch.step(12)
    for k in (0, 101, 255):
        alone = pic.Sim(_single(work, k), fused=True)
        alone.step(12)
        for s in range(2):
            a, b = by_id(batch.particles(k, s)), by_id(alone.particles(0, s))
            for key in ("id", "x", "vx", "vy", "vz"):
                assert np.array_equal(a[key], b[key]), (k, s, key)
        da, db = batch.diag(k), alone.diag(0)
        for key in ("count", "coll", "created", "wall_count", "pushes"):
            assert da[key] == db[key], (k, key)
        alone.close()
    assert sum(sum(batch.diag(k)["created"]) for k in range(0, 256, 15)) > 0
    batch.close()
