"""Device-state checkpoint and restart: a run saved at a step boundary and continued in a
fresh context (same configuration) gives the uninterrupted run's particles (bit for bit in
the FP32 form, whose deposit is integer; to rounding in the FP64 form, whose deposit uses
FP64 atomics), with collisions, births, absorbing walls and sorts on both sides."""
import numpy as np
import pytest

import synth
from parity_util import by_id

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_28534_amd as P

    P.load_library()
    return P


def _work(prec):
    e = synth.ensemble(700, 60, seed=17, B=synth.oblique_B(), sort_every=5)
    e["ngs_el"], e["ngs_iz"] = 0.05, 0.05   # births within a few steps
    for sp in e["species"]:
        sp["capacity"] *= 2
    return {"name": "ckpt", "steps": 1, "precision": prec, "ensembles": [e]}


@pytest.mark.parametrize("prec,fused,at", [("fp32", True, 13), ("fp32", True, 14), ("fp32", False, 13),
                                           ("fp64", False, 13)])
def test_restart_is_bit_identical(pic, prec, fused, at):
    """Save between sorts (K = 5) and continue in another context.  At step 14 the saving
    context has counted and scanned its cells for the sort that the fused FP32 pass of the
    next step performs; the restored context sorts that step in kernels of its own, with
    the same result by particle id."""
    work = _work(prec)
    a = pic.Sim(work, fused=fused)
    a.step(at)
    buf = a.save()
    a.step(9)
    b = pic.Sim(work, fused=fused)
    b.step(3)                       # a context with a history of its own is overwritten
    b.load(buf)
    b.step(9)
    da, db = a.diag(), b.diag()
    for key in ("count", "coll", "created", "wall_count", "pushes", "step"):
        assert da[key] == db[key], key
    # nu_max follows max |E|, which in the FP64 form carries the deposit's atomic order
    if prec == "fp32":
        assert da["numax"] == db["numax"]
    else:
        assert np.allclose(da["numax"], db["numax"], rtol=1e-12, atol=0)
    # the order of particles inside a cell after a sort is not fixed (atomic slot
    # reservations), so sums over slots may differ in their last bits; the fused FP32 step
    # tallies |v|^2 in binary32 over each thread's slots (which particles share a thread
    # follows that order), so its energies agree to binary32 rounding
    assert np.allclose(da["ke"], db["ke"], rtol=(1e-6 if (prec == "fp32" and fused) else 1e-13), atol=0)
    for s in range(2):
        pa, pb = by_id(a.particles(0, s)), by_id(b.particles(0, s))
        assert np.array_equal(pa["id"], pb["id"]), s
        for k in ("x", "vx", "vy", "vz"):
            if prec == "fp32":
                assert np.array_equal(pa[k], pb[k]), (s, k)
            else:  # the FP64 form deposits with FP64 atomics, whose order is not fixed
                assert np.allclose(pa[k], pb[k], rtol=1e-9, atol=1e-9 * np.max(np.abs(pa[k]))), (s, k)
    ga, gb = a.grid(), b.grid()
    if prec == "fp32":   # integer deposit: independent of order
        assert np.array_equal(ga["Q"][0], gb["Q"][0])
        assert np.array_equal(ga["E"], gb["E"])
    else:                # FP64 atomics: order shows in the last bits
        assert np.allclose(ga["E"], gb["E"], rtol=1e-12, atol=1e-12 * np.max(np.abs(ga["E"])))
    a.close()
    b.close()


def test_load_rejects_other_configuration(pic):
    a = pic.Sim(_work("fp32"), fused=True)
    buf = a.save()
    other = _work("fp32")
    other["ensembles"][0]["ncells"] = 701
    b = pic.Sim(other, fused=True)
    with pytest.raises(pic.PicError) as ei:
        b.load(buf)
    assert ei.value.code == pic.PIC_EINVAL
    with pytest.raises(pic.PicError):
        b.load(buf[:100])


@pytest.mark.parametrize("prec,collisions", [("fp32", False), ("fp64", False), ("fp64", True)])
def test_restart_matches_the_oracle_window(pic, prec, collisions):
    """Save at step 13, load into a fresh context, run on to step 20 and compare with the
    FP64 oracle's uninterrupted 20-step window by particle id (the window tolerances of the
    parity tests: fields rel 1e-5 in the FP32 form; counts exact, collisions included in
    the FP64 form, whose decisions are taken on FP64 velocities like the oracle's)."""
    import oracle
    from parity_util import TOL_FIELD, TOL_MOMENT, compare_particles, rel

    w = synth.scaled(synth.c2_sheath(), ncells=1500, ppc=40)
    e = w["ensembles"][0]
    e["collisions"] = collisions
    if collisions:
        e["ngs_el"], e["ngs_iz"] = 0.05, 0.05
        for sp in e["species"]:
            sp["capacity"] *= 2
    work = {"name": "ckpt-oracle", "steps": 1, "precision": prec, "ensembles": [e]}
    fused = prec == "fp32"
    a = pic.Sim(work, fused=fused)
    a.step(13)
    buf = a.save()
    a.close()
    b = pic.Sim(work, fused=fused)
    b.load(buf)
    b.step(7)
    o = oracle.Oracle(e)
    o.step(20)
    gd, od = b.diag(), o.diag()
    assert gd["step"] == od["step"] == 20
    for key in ("count", "wall_count", "pushes", "coll", "created"):
        assert gd[key] == od[key], (key, gd[key], od[key])
    if collisions:
        assert sum(od["coll"]) > 0 and sum(od["created"]) > 0
    for s in range(2):
        vt, xt = (1e-9, 1e-8) if prec == "fp64" else (1e-4, 1e-4)
        compare_particles(b.particles(0, s), o.particles(s), e["dx"], prec == "fp64", vtol=vt, xtol=xt)
        assert abs(gd["ke"][s] - od["ke"][s]) <= TOL_MOMENT * abs(od["ke"][s])
    g, r = b.grid(), o.grid()
    for k in ("rho", "phi", "E"):
        assert rel(g[k], r[k]) <= (1e-8 if prec == "fp64" else TOL_FIELD), (k, rel(g[k], r[k]))
    b.close()
