"""CPU checks of the C-ABI library: it loads and exports every symbol include/pic.h
declares; workspace queries and configuration validation need no GPU."""
import ctypes as C
import os
import re

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "pic.h")).read()
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2606_28534_amd as P

    return P, P.load_library()


def test_exports_every_declared_symbol(lib):
    P, L = lib
    names = declared_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
    assert set(P.EXPORTS) <= set(names)


def test_workspace_query_sizes(lib):
    P, L = lib
    for work, lo, hi in ((synth.c2_sheath(), 1.5e9, 5e9), (synth.c1_plain_small(), 1e6, 2e8)):
        cfg, keep = P.make_config(work)
        n = C.c_size_t(0)
        assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == 0
        assert lo < n.value < hi, n.value
    # the large single-GPU share fits a 288 GB device
    cfg, keep = P.make_config(synth.c5_large())
    n = C.c_size_t(0)
    assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == 0
    assert n.value < 150e9  # fits one 288 GB MI355X with room to spare


def test_bad_configs_rejected(lib):
    P, L = lib
    work = synth.c1_plain_small()
    e = work["ensembles"][0]
    n = C.c_size_t(0)
    bad = dict(e, ncells=1)
    cfg, keep = P.make_config(dict(work, ensembles=[bad]))
    assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == P.PIC_EINVAL
    bad = synth.ensemble(100, 10)
    bad["species"][0]["capacity"] = 10
    cfg, keep = P.make_config(dict(work, ensembles=[bad]))
    assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == P.PIC_EINVAL
    cfg, keep = P.make_config(work)
    cfg.precision = 7
    assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == P.PIC_EINVAL
    cfg, keep = P.make_config(work)
    cfg.n_ensembles = 0
    assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == P.PIC_EINVAL
    # launch-shape fields out of range: LDS window span and FP64 block size
    for field, value in (("window", 8), ("window", 8192), ("block", 512), ("block", 96),
                         ("sort_every", -1), ("sort_every", 5000)):
        cfg, keep = P.make_config(work)
        setattr(cfg, field, value)
        assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == P.PIC_EINVAL, (field, value)
    for field, value in (("window", 16), ("window", 4096), ("block", 128)):
        cfg, keep = P.make_config(work)
        setattr(cfg, field, value)
        assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == 0, (field, value)
    # init refuses a workspace that is too small before touching the GPU
    cfg, keep = P.make_config(work)
    h = C.c_void_p()
    assert L.pic_init(C.byref(cfg), C.c_void_p(0), 16, None, C.byref(h)) == P.PIC_EINVAL


def test_null_context_calls_fail_cleanly(lib):
    P, L = lib
    for n in ("pic_deposit", "pic_solve", "pic_push", "pic_collide", "pic_sort"):
        assert getattr(L, n)(None, None) == P.PIC_EINVAL
    assert L.pic_step(None, 1, None) == P.PIC_EINVAL
    assert L.pic_adjoint_window_noalloc(None, 1, 1, None, None, 0, None, None) == P.PIC_EINVAL
    assert L.pic_last_error(None) == b"null context"


def _c_layout(tmp_path, struct, fields):
    """sizeof and offsetof of a struct in include/pic.h, from a C program built with gcc."""
    src = tmp_path / "layout.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pic.h"', "int main(void) {",
             f'  printf("%zu\\n", sizeof({struct}));']
    lines += [f'  printf("%zu\\n", offsetof({struct}, {f}));' for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    import subprocess

    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.parametrize("struct,cls", [("pic_species_desc", "SpeciesDesc"),
                                        ("pic_ensemble_desc", "EnsembleDesc"),
                                        ("pic_config", "Config"), ("pic_diag_out", "DiagOut")])
def test_binding_structs_match_the_header(lib, tmp_path, struct, cls):
    P, L = lib
    ct = getattr(P, cls)
    names = [f[0] for f in ct._fields_]
    size, offs = _c_layout(tmp_path, struct, names)
    assert C.sizeof(ct) == size, (struct, C.sizeof(ct), size)
    assert [getattr(ct, n).offset for n in names] == offs, struct


def test_sheath_case_configs_validated(lib):
    """Recycling and the source need the FP32 form and two species; recycling needs
    bounded walls and room for neutrals; the source region is a fraction in (0, 1]."""
    P, L = lib
    n = C.c_size_t(0)
    ok = synth.c7_sheath_source(ncells=2000, capacity=200_000)
    cfg, keep = P.make_config(ok)
    assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == 0
    cfg, keep = P.make_config(synth.c6_sheath_recycling(ncells=2000, ppc=20))
    assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == 0
    cfg, keep = P.make_config(ok, precision="fp64")
    assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == P.PIC_EINVAL
    for change in ({"src_frac": 0.0}, {"src_frac": 1.5}, {"src_pairs": -1},
                   {"neutral_capacity": 0}):
        e = dict(ok["ensembles"][0], **change)
        cfg, keep = P.make_config(dict(ok, ensembles=[e]))
        assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == P.PIC_EINVAL, change
    e = dict(ok["ensembles"][0], periodic=True, floating=False)
    cfg, keep = P.make_config(dict(ok, ensembles=[e]))
    assert L.pic_query_workspace(C.byref(cfg), C.byref(n)) == P.PIC_EINVAL
