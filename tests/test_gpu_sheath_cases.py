"""GPU parity of the paper's two sheath cases against the FP64 oracle: ions recycled into
neutrals at the walls (R24) and the volumetric pair source of the initially empty slab
(R25), with floating walls.  Inputs come from the synth module (seeded, synthetic)."""
import math

import numpy as np
import pytest

import oracle
import synth
from parity_util import TOL_FIELD, TOL_V32, TOL_X32, by_id, compare_particles, rel

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


def light_ions(e):
    """Hot light ions reach the walls within a short window."""
    e["species"][1]["m"] = e["m_n"] = 100.0
    e["species"][1]["T"] = e["T_n"] = 1.0
    return e


def compare_neutrals(g, o, dx, xtol=TOL_X32 + 1e-7):
    """Neutrals by id; positions to `xtol` cells (binary32 offsets gain about 2^-23 of a
    cell of rounding per step)."""
    G, O = by_id(g), by_id(o)
    assert np.array_equal(G["id"], O["id"]), (len(G["id"]), len(O["id"]))
    if len(G["id"]) == 0:
        return
    vmax = max(np.max(np.abs(O[k])) for k in ("vx", "vy", "vz"))
    for k in ("vx", "vy", "vz"):
        assert np.max(np.abs(G[k] - O[k])) <= TOL_V32 * vmax, k
    assert np.max(np.abs(G["x"] - O["x"])) / dx <= xtol


def test_recycling_one_push_from_injected_state(pic):
    """Ions next to both walls leave in one push in zero field: every one comes back as a
    neutral with its id, speed, direction and depth drawn as the oracle draws them."""
    N, n = 300, 20000
    e = synth.ensemble(N, 1, collisions=False, recycle=True, neutral_capacity=4 * n, floating=True)
    for sp in e["species"]:
        sp["capacity"] = 4 * n
    rng = np.random.default_rng(5)
    L, dx = N * e["dx"], e["dx"]
    side = rng.random(n) < 0.5
    x = np.where(side, rng.random(n) * 0.5 * dx, L - rng.random(n) * 0.5 * dx)
    st = [synth.random_state(e, [500, 500], seed=3)[0],
          {"x": x, "vx": np.where(side, -1.0, 1.0) * dx / e["dt"], "vy": rng.standard_normal(n),
           "vz": rng.standard_normal(n), "id": rng.permutation(n).astype(np.uint32) + 11,
           "next_id": n + 11}]
    sim = pic.Sim(work_of(e), fused=False)
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
    assert gd["recycled"] == od["recycled"] == n
    assert gd["neutral_count"] == od["neutral_count"] == n
    compare_neutrals(sim.particles(0, 2), o.particles(2), dx)


def test_neutrals_stream_and_leave(pic):
    """Forty pushes of a neutral set in a random field (which only the charged species
    feel): exits per wall exact, survivors' positions by id."""
    N = 500
    e = synth.ensemble(N, 4, collisions=False, recycle=True, neutral_capacity=50000)
    st = synth.random_state(e, [2000, 2000], seed=4, vscale=[1.0, 0.01])
    rng = np.random.default_rng(9)
    L = N * e["dx"]
    m = 30000
    neu = {"x": rng.random(m) * L, "vx": rng.standard_normal(m) * 2.0, "vy": rng.standard_normal(m),
           "vz": rng.standard_normal(m), "id": rng.permutation(m).astype(np.uint32), "next_id": 0}
    sim = pic.Sim(work_of(e), fused=False)
    o = oracle.Oracle(e, init=False)
    for x in (sim, o):
        x.set_state(st + [neu])
    E = synth.random_field(e, seed=6)
    sim.set_fields(E)
    o.set_fields(E)
    for _ in range(40):
        sim.push()
        o.push()
        o.walls()
    gd, od = sim.diag(), o.diag()
    assert gd["neutral_wall"] == od["neutral_wall"]
    assert gd["neutral_count"] == od["neutral_count"]
    compare_neutrals(sim.particles(0, 2), o.particles(2), e["dx"], xtol=40 * 2.0 ** -22)


def test_source_pairs_from_empty_domain(pic):
    """One creation stage in an empty domain: the source's pairs, ids, positions and
    velocities as the oracle draws them, and their deposited charge."""
    N, S = 3000, 50000
    e = synth.ensemble(N, 0, collisions=False, src_pairs=S, src_frac=0.5, floating=True)
    for sp in e["species"]:
        sp["w"] = e["dx"] / 100
        sp["capacity"] = 3 * S
    sim = pic.Sim(work_of(e), fused=False)
    o = oracle.Oracle(e)
    sim.collide()
    o.collide()
    gd, od = sim.diag(), o.diag()
    assert gd["sourced"] == od["sourced"] == S
    assert gd["count"] == od["count"] == [S, S]
    for s in range(2):
        compare_particles(sim.particles(0, s), o.particles(s), e["dx"], False)
    sim.deposit()
    o.deposit()
    g, r = sim.grid(), o.grid()
    for s in range(2):
        assert g["Q"][s].sum() == S
        assert np.max(np.abs(g["Q"][s] - r["Q"][s])) <= 2.0 ** -24 * 60 + 1e-9


def _sheath_small(collisions):
    e = synth.ensemble(1200, 30, collisions=collisions, B=synth.oblique_B(), sort_every=20,
                       floating=True, recycle=True, neutral_capacity=40000, src_pairs=300,
                       src_frac=0.5, seed=23)
    light_ions(e)
    if collisions:
        e["ngs_el"], e["ngs_iz"] = 0.1, 0.2
    for sp in e["species"]:
        sp["capacity"] = 120000
    return e


def test_sheath_case_window_vs_oracle(pic):
    """Twenty fused (graph) steps with floating recycling walls and the source, no
    collisions: every count exact, particles and neutrals by id, and the field."""
    e = _sheath_small(False)
    sim = pic.Sim(work_of(e), fused=True)
    o = oracle.Oracle(e)
    sim.step(20)
    o.step(20)
    gd, od = sim.diag(), o.diag()
    for k in ("count", "wall_count", "sourced", "recycled", "neutral_count", "neutral_wall", "pushes"):
        assert gd[k] == od[k], (k, gd[k], od[k])
    assert od["recycled"] > 0
    for s in range(2):
        compare_particles(sim.particles(0, s), o.particles(s), e["dx"], False, vtol=1e-4, xtol=1e-4)
    G, O = by_id(sim.particles(0, 2)), by_id(o.particles(2))
    assert np.array_equal(G["id"], O["id"])
    assert np.max(np.abs(G["x"] - O["x"])) / e["dx"] <= 1e-4
    assert rel(sim.grid()["E"], o.grid()["E"]) <= TOL_FIELD, rel(sim.grid()["E"], o.grid()["E"])


def test_sheath_case_collisional_paths_agree(pic):
    """With collisions as well, the fused graph, fused eager and separate-stage runs give
    the same particles and neutrals bit for bit."""
    e = _sheath_small(True)
    a = pic.Sim(work_of(e), fused=True)
    b = pic.Sim(work_of(e), fused=True)
    c = pic.Sim(work_of(e), fused=False)
    a.step(25)
    for _ in range(25):
        b.step(1)
    c.step(25)
    for s in range(3):
        sa, sb, sc = (by_id(x.particles(0, s)) for x in (a, b, c))
        for k in ("id", "x", "vx", "vy", "vz"):
            assert np.array_equal(sa[k], sb[k]), (s, k)
            assert np.array_equal(sa[k], sc[k]), (s, k)
    da, dc = a.diag(), c.diag()
    for k in ("coll", "created", "sourced", "recycled", "neutral_wall", "wall_count"):
        assert da[k] == dc[k], k
    assert da["recycled"] > 0 and da["created"][0] > 0


def test_sheath_case_restart_with_neutrals(pic):
    """A recycling, sourced, collisional run saved mid-cycle and continued in a fresh
    context matches the uninterrupted run, neutrals included."""
    e = _sheath_small(True)
    a = pic.Sim(work_of(e), fused=True)
    a.step(13)
    buf = a.save()
    a.step(9)
    b = pic.Sim(work_of(e), fused=True)
    b.load(buf)
    b.step(9)
    da, db = a.diag(), b.diag()
    for k in ("count", "coll", "created", "sourced", "recycled", "neutral_count", "neutral_wall",
              "wall_count", "step"):
        assert da[k] == db[k], k
    for s in range(3):
        pa, pb = by_id(a.particles(0, s)), by_id(b.particles(0, s))
        for k in ("id", "x", "vx", "vy", "vz"):
            assert np.array_equal(pa[k], pb[k]), (s, k)


@pytest.mark.parametrize("case", ["recycling", "source"])
def test_sheath_cases_bookkeeping_at_full_size(pic, case):
    """The 1e5-cell workloads (uniform load with recycling, 4.0e7 particles; empty slab
    with a 2e4-pair-per-step source): every particle count closes exactly after 60 fused
    steps, and the plasma plus wall charge stays zero."""
    w = synth.c6_sheath_recycling() if case == "recycling" else synth.c7_sheath_source()
    e = w["ensembles"][0]
    light_ions(e)
    sim = pic.Sim(w, fused=True)
    n0 = [sp["ppc"] * e["ncells"] for sp in e["species"]]
    sim.step(60)
    d = sim.diag()
    for s in range(2):
        absorbed = d["wall_count"][0][s] + d["wall_count"][1][s]
        assert d["count"][s] == n0[s] + d["created"][s] + d["sourced"] - absorbed, s
    assert d["recycled"] == d["wall_count"][0][1] + d["wall_count"][1][1]
    assert d["neutral_count"] + sum(d["neutral_wall"]) == d["recycled"]
    assert d["recycled"] > 0
    if case == "source":
        assert d["sourced"] == 60 * e["src_pairs"]
    wallq = sum(d["wall_charge"][wl][s] for wl in range(2) for s in range(2))
    scale = e["species"][0]["w"] * (n0[0] + d["sourced"] + d["created"][0])
    assert abs(d["charge"] + wallq) <= 1e-9 * scale
    sim.solve()
    g = sim.grid()
    sig = [sum(sp["q"] * sp["w"] * d["wall_count"][wl][s] for s, sp in enumerate(e["species"]))
           for wl in range(2)]
    assert abs(g["E"][0] - sig[0]) <= 1e-9 * scale
    assert abs(g["E"][-1] + sig[1]) <= 1e-9 * scale


def test_batched_mixed_sheath_features(pic):
    """Four ensembles in one run, with recycling and the source switched on in different
    combinations (and different sizes): each one against its own oracle over 20 fused
    steps, so per-ensemble neutral sets, source ranges and counters stay apart."""
    ens = []
    for k, (rec, src, n) in enumerate(((True, 200, 700), (False, 0, 900), (False, 150, 500), (True, 0, 1100))):
        e = synth.ensemble(n, 20, collisions=False, B=synth.oblique_B(), sort_every=20, floating=True,
                           recycle=rec, neutral_capacity=30000 if rec else 0, src_pairs=src,
                           src_frac=0.5, seed=31 + k)
        light_ions(e)
        for sp in e["species"]:
            sp["capacity"] = 80000
        ens.append(e)
    work = {"name": "mixed", "steps": 20, "precision": "fp32", "ensembles": ens}
    sim = pic.Sim(work, fused=True)
    sim.step(20)
    for k, e in enumerate(ens):
        o = oracle.Oracle(e)
        o.step(20)
        gd, od = sim.diag(k), o.diag()
        for key in ("count", "wall_count", "sourced", "recycled", "neutral_count", "neutral_wall"):
            assert gd[key] == od[key], (k, key, gd[key], od[key])
        for s in range(2):
            compare_particles(sim.particles(k, s), o.particles(s), e["dx"], False, vtol=1e-4, xtol=1e-4)
        if e["recycle"]:
            G, O = by_id(sim.particles(k, 2)), by_id(o.particles(2))
            assert np.array_equal(G["id"], O["id"])
        assert rel(sim.grid(k)["E"], o.grid()["E"]) <= TOL_FIELD, (k, rel(sim.grid(k)["E"], o.grid()["E"]))
