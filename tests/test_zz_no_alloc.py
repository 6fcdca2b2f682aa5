"""GPU check of pic_adjoint_window_noalloc, the adjoint window on the library's static device
scratch, against pic_adjoint_window on a caller buffer: the same objective and gradients on
the same state, on two calls in a row (the second with fewer particles and cells, so it runs
on what the first left in the array), and a window larger than the array is refused."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pic():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_28534_amd as P

    P.load_library()
    return P


def _sim(pic, e, st, nsteps):
    sim = pic.Sim({"name": "w", "steps": nsteps, "precision": "fp32", "ensembles": [e]}, fused=True)
    sim.set_particles(0, 0, st["x"], st["vx"], st["vy"], st["vz"], st["id"], st["next_id"])
    sim.set_step(0)
    return sim


def _both(pic, e, nsteps, ckpt):
    """Objective and gradients of the window from the caller-buffer and the static-scratch
    entry points on identical state, and the final particles of each."""
    st = synth.quiet_start_state(e)[0]
    a = _sim(pic, e, st, nsteps)
    ra = a.adjoint_window(nsteps, ckpt)
    pa = a.particles(0, 0)
    b = _sim(pic, e, st, nsteps)
    rb = b.adjoint_window_noalloc(nsteps, ckpt)
    pb = b.particles(0, 0)
    a.close()
    b.close()
    return len(st["x"]), ra, rb, pa, pb


def _check(n, ra, rb, pa, pb):
    (Wa, ga, gEa), (Wb, gb, gEb) = ra, rb
    # the two calls run the same kernels in the same order; the gradient's FP64 atomics
    # (deposit-shaped scatters) may add in another order, so agreement is to FP64 rounding
    # of those sums, far inside the adjoint's 1e-4 parity bar
    assert Wb == pytest.approx(Wa, rel=1e-12, abs=0.0)
    scale = np.max(np.abs(ga[:n]))
    assert scale > 0.0
    assert np.max(np.abs(gb[:n] - ga[:n])) <= 1e-9 * scale
    assert np.all(gb[n:] == 0.0) and np.all(ga[n:] == 0.0)
    assert abs(gEb - gEa) <= 1e-9 * scale * n
    for k in ("id", "x", "vx"):
        assert np.array_equal(pa[k], pb[k]), k


def test_noalloc_window_matches_caller_buffer_twice(pic):
    # first call: 1024 periodic cells x 100 cold electrons, 60 steps, checkpoint every 20
    e1 = synth.c4_langmuir(ncells=1024, ppc=100)["ensembles"][0]
    _check(*_both(pic, e1, 60, 20))
    # second call on the same array, smaller: 300 cells x 40, 45 steps, checkpoint every 10
    e2 = synth.c4_langmuir(ncells=300, ppc=40)["ensembles"][0]
    _check(*_both(pic, e2, 45, 10))


def test_noalloc_window_refuses_more_than_the_array(pic):
    # the full 2048-cell window with a checkpoint every step needs ~1 GB of scratch
    e = synth.c4_langmuir()["ensembles"][0]
    st = synth.quiet_start_state(e)[0]
    sim = _sim(pic, e, st, 200)
    with pytest.raises(pic.PicError) as ei:
        sim.adjoint_window_noalloc(200, 1)
    assert ei.value.code == pic.PIC_EINVAL
    assert "static array" in str(ei.value)
    sim.close()
