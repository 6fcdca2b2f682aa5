"""MI355X-native electrostatic 1D3V PIC Monte Carlo hot path: Python binding.

A thin ctypes layer over the C ABI of libpic.so (declared in include/pic.h).  It only
marshals arguments: torch provides the device workspace and the stream, and every stage
of the step runs in the library's HIP kernels.  If the library is missing, importing the
binding raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpic.so")

PIC_OK, PIC_EINVAL, PIC_ECAPACITY, PIC_ENONFINITE, PIC_EHIP, PIC_ESTATE = 0, -1, -2, -3, -4, -5
PIC_FP64_PLAIN, PIC_FP32_CELLOFF = 0, 1
PIC_ABSORBING, PIC_PERIODIC, PIC_FLOATING = 0, 1, 2

EXPORTS = ("pic_query_workspace", "pic_init", "pic_deposit", "pic_solve", "pic_push",
           "pic_collide", "pic_sort", "pic_step", "pic_diag", "pic_get_particles",
           "pic_get_slots", "pic_set_particles", "pic_get_grid", "pic_get_gather_table",
           "pic_set_fields", "pic_set_step",
           "pic_nnodes", "pic_set_external_field", "pic_adjoint_query",
           "pic_adjoint_window", "pic_adjoint_window_noalloc", "pic_autotune", "pic_checkpoint_size", "pic_save", "pic_load",
           "pic_timing", "pic_timing_read", "pic_stream_copy", "pic_graph_prepare", "pic_graph_launches",
           "pic_free", "pic_last_error")


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pic error {code}: {msg}")
        self.code = code


class SpeciesDesc(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("w", C.c_double), ("T", C.c_double),
                ("ppc", C.c_int64), ("capacity", C.c_int64)]


class EnsembleDesc(C.Structure):
    _fields_ = [("ncells", C.c_int64), ("dx", C.c_double), ("dt", C.c_double),
                ("eps0", C.c_double), ("B", C.c_double * 3), ("E_ext", C.c_double),
                ("seed", C.c_uint32), ("init_mode", C.c_int32), ("sp", SpeciesDesc * 2),
                ("ngs_el", C.c_double), ("ngs_iz", C.c_double), ("ngs_cx", C.c_double),
                ("eps_iz", C.c_double), ("T_n", C.c_double), ("m_n", C.c_double),
                ("perturb_amp", C.c_double), ("perturb_mode", C.c_int32),
                ("recycle", C.c_int32), ("neutral_capacity", C.c_int64), ("src_pairs", C.c_int64),
                ("src_frac", C.c_double), ("cx_relative", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("n_ensembles", C.c_int32), ("precision", C.c_int32), ("boundary", C.c_int32),
                ("nspecies", C.c_int32), ("collisions", C.c_int32), ("sort_every", C.c_int32),
                ("fused", C.c_int32), ("block", C.c_int32), ("grid", C.c_int32),
                ("window", C.c_int32), ("ppt", C.c_int32), ("sort_ppt", C.c_int32),
                ("nontemporal", C.c_int32), ("smooth", C.c_int32),
                ("ens", C.POINTER(EnsembleDesc))]


class DiagOut(C.Structure):
    _fields_ = [("count", C.c_int64 * 2), ("charge", C.c_double), ("ke", C.c_double * 2),
                ("field_energy", C.c_double), ("wall_count", (C.c_int64 * 2) * 2),
                ("wall_charge", (C.c_double * 2) * 2), ("wall_ke", (C.c_double * 2) * 2),
                ("coll", C.c_int64 * 3), ("created", C.c_int64 * 2), ("pushes", C.c_int64),
                ("step", C.c_int64), ("numax", C.c_double * 2), ("emax", C.c_double),
                ("neutral_count", C.c_int64), ("neutral_wall", C.c_int64 * 2),
                ("recycled", C.c_int64), ("sourced", C.c_int64)]

    def as_dict(self):
        return {
            "count": list(self.count), "charge": self.charge, "ke": list(self.ke),
            "field_energy": self.field_energy,
            "wall_count": [list(r) for r in self.wall_count],
            "wall_charge": [list(r) for r in self.wall_charge],
            "wall_ke": [list(r) for r in self.wall_ke],
            "coll": list(self.coll), "created": list(self.created), "pushes": self.pushes,
            "step": self.step, "numax": list(self.numax), "emax": self.emax,
            "neutral_count": self.neutral_count, "neutral_wall": list(self.neutral_wall),
            "recycled": self.recycled, "sourced": self.sourced,
        }


class Particles(C.Structure):
    _fields_ = [("x", C.POINTER(C.c_double)), ("vx", C.POINTER(C.c_double)),
                ("vy", C.POINTER(C.c_double)), ("vz", C.POINTER(C.c_double)),
                ("id", C.POINTER(C.c_uint32))]


_lib = None


def load_library():
    """Load libpic.so (after torch, so both share one HIP runtime); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; build it with python -m paper_2606_28534_amd.build (no CPU fallback)")
    import torch  # noqa: F401  (loads the HIP runtime the library binds to)
    L = C.CDLL(LIB_PATH)
    P = C.c_void_p
    L.pic_query_workspace.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
    L.pic_init.argtypes = [C.POINTER(Config), P, C.c_size_t, P, C.POINTER(P)]
    for n in ("pic_deposit", "pic_solve", "pic_push", "pic_collide", "pic_sort"):
        getattr(L, n).argtypes = [P, P]
    L.pic_step.argtypes = [P, C.c_int32, P]
    L.pic_diag.argtypes = [P, C.c_int32, C.POINTER(DiagOut), P, P]
    L.pic_get_particles.argtypes = [P, C.c_int32, C.c_int32, Particles, C.c_int64,
                                    C.POINTER(C.c_int64), P]
    L.pic_set_particles.argtypes = [P, C.c_int32, C.c_int32, Particles, C.c_int64, C.c_uint32, P]
    L.pic_get_slots.argtypes = [P, C.c_int32, C.c_int32, C.c_int64, C.c_int64, Particles, P]
    L.pic_get_grid.argtypes = [P, C.c_int32, P, P, P, P, P, P]
    L.pic_get_gather_table.argtypes = [P, C.c_int32, P, P]
    L.pic_set_fields.argtypes = [P, C.c_int32, P, P]
    L.pic_set_step.argtypes = [P, C.c_int64]
    L.pic_nnodes.argtypes = [P, C.c_int32]
    L.pic_nnodes.restype = C.c_int64
    L.pic_set_external_field.argtypes = [P, C.c_int32, C.c_double]
    L.pic_adjoint_query.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]
    L.pic_adjoint_window.argtypes = [P, C.c_int32, C.c_int32, P, C.c_size_t, C.POINTER(C.c_double),
                                     P, C.c_int64, C.POINTER(C.c_double), P]
    L.pic_adjoint_window_noalloc.argtypes = [P, C.c_int32, C.c_int32, C.POINTER(C.c_double), P, C.c_int64,
                                             C.POINTER(C.c_double), P]
    L.pic_autotune.argtypes = [P, C.c_int32, P, P]
    L.pic_checkpoint_size.argtypes = [P, C.POINTER(C.c_size_t), P]
    L.pic_save.argtypes = [P, P, C.c_size_t, P]
    L.pic_load.argtypes = [P, P, C.c_size_t, P]
    L.pic_timing.argtypes = [P, C.c_int32]
    L.pic_graph_prepare.argtypes = [P, C.c_int32]
    L.pic_graph_launches.argtypes = [P, C.POINTER(C.c_int64)]
    L.pic_timing_read.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64), P]
    L.pic_stream_copy.argtypes = [P, P, C.c_size_t, C.c_int32, P]
    L.pic_free.argtypes = [P]
    L.pic_free.restype = None
    L.pic_last_error.argtypes = [P]
    L.pic_last_error.restype = C.c_char_p
    _lib = L
    return L


def stream_copy(src, dst, nontemporal=True, stream=None):
    """Copy device tensor `src` into `dst` (same byte size, a multiple of 16) with the
    particle pass's access pattern (the library's measurement hook)."""
    import torch

    L = load_library()
    nb = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nb
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = L.pic_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nb,
                           1 if nontemporal else 0, C.c_void_p(st.cuda_stream))
    if rc != PIC_OK:
        raise PicError(rc, "pic_stream_copy")


def make_config(work, fused=True, precision=None, block=0, grid=0, window=0, ppt=0, sort_ppt=0,
                nontemporal=0):
    """Translate a workload dict ({"ensembles": [...], "precision": "fp32"|"fp64"}) into
    the C configuration.  Returns (Config, keep-alive array)."""
    ens = work["ensembles"]
    arr = (EnsembleDesc * len(ens))()
    for i, e in enumerate(ens):
        d = arr[i]
        d.ncells, d.dx, d.dt, d.eps0 = e["ncells"], e["dx"], e["dt"], e["eps0"]
        for k in range(3):
            d.B[k] = e["B"][k]
        d.E_ext, d.seed, d.init_mode = e["E_ext"], e["seed"], e["init_mode"]
        for s, sp in enumerate(e["species"]):
            d.sp[s].q, d.sp[s].m, d.sp[s].w, d.sp[s].T = sp["q"], sp["m"], sp["w"], sp["T"]
            d.sp[s].ppc, d.sp[s].capacity = sp["ppc"], sp["capacity"]
        d.ngs_el, d.ngs_iz, d.ngs_cx = e["ngs_el"], e["ngs_iz"], e["ngs_cx"]
        d.eps_iz, d.T_n, d.m_n = e["eps_iz"], e["T_n"], e["m_n"]
        d.perturb_amp, d.perturb_mode = e["perturb_amp"], e["perturb_mode"]
        d.recycle = int(e.get("recycle", False))
        d.neutral_capacity = int(e.get("neutral_capacity", 0))
        d.src_pairs = int(e.get("src_pairs", 0))
        d.src_frac = float(e.get("src_frac", 0.5))
        d.cx_relative = int(e.get("cx_relative", False))
    e0 = ens[0]
    prec = precision or work.get("precision", "fp32")
    cfg = Config()
    cfg.n_ensembles = len(ens)
    cfg.precision = PIC_FP64_PLAIN if prec == "fp64" else PIC_FP32_CELLOFF
    if e0["periodic"]:
        cfg.boundary = PIC_PERIODIC
    else:
        cfg.boundary = PIC_FLOATING if e0.get("floating", False) else PIC_ABSORBING
    cfg.smooth = int(e0.get("smooth", 0))
    cfg.nspecies = e0["nspecies"]
    cfg.collisions = int(e0["collisions"])
    cfg.sort_every = e0["sort_every"]
    cfg.fused = int(fused)
    cfg.block, cfg.grid, cfg.window, cfg.ppt, cfg.sort_ppt = block, grid, window, ppt, sort_ppt
    cfg.nontemporal = int(nontemporal)
    cfg.ens = arr
    return cfg, arr


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


class Sim:
    """One run of the PIC MC hot path on the current GPU (torch provides the memory)."""

    def __init__(self, work, fused=True, precision=None, block=0, grid=0, window=0, ppt=0,
                 sort_ppt=0, nontemporal=0, stream=None):
        import torch

        self.L = load_library()
        self.work = work
        self.cfg, self._arr = make_config(work, fused, precision, block, grid, window, ppt, sort_ppt,
                                          nontemporal)
        nbytes = C.c_size_t(0)
        self._check(self.L.pic_query_workspace(C.byref(self.cfg), C.byref(nbytes)), None)
        self.ws_bytes = nbytes.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = C.c_void_p()
        self._check(self.L.pic_init(C.byref(self.cfg), C.c_void_p(self.ws.data_ptr()),
                                    self.ws_bytes, self._s(), C.byref(self.h)), None)
        self.nens = len(work["ensembles"])
        self.nspecies = work["ensembles"][0]["nspecies"]

    def _s(self):
        return C.c_void_p(self.stream.cuda_stream)

    def _check(self, rc, h="self"):
        if rc != PIC_OK:
            hh = self.h if h == "self" else None
            msg = self.L.pic_last_error(hh).decode() if hh else "see stderr"
            raise PicError(rc, msg)

    def close(self):
        if getattr(self, "h", None):
            self.L.pic_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- stages -------------------------------------------------------------------------
    def deposit(self):
        self._check(self.L.pic_deposit(self.h, self._s()))

    def solve(self):
        self._check(self.L.pic_solve(self.h, self._s()))

    def push(self):
        self._check(self.L.pic_push(self.h, self._s()))

    def collide(self):
        self._check(self.L.pic_collide(self.h, self._s()))

    def sort(self):
        self._check(self.L.pic_sort(self.h, self._s()))

    def step(self, n=1):
        self._check(self.L.pic_step(self.h, int(n), self._s()))

    def prepare(self, n):
        """Instantiate the HIP graphs that step(n) would replay from here (no steps run)."""
        self._check(self.L.pic_graph_prepare(self.h, int(n)))

    def graph_launches(self):
        """Graph replays made by step() so far."""
        n = C.c_int64(0)
        self._check(self.L.pic_graph_launches(self.h, C.byref(n)))
        return n.value

    def set_external_field(self, E_ext, ens=0):
        self._check(self.L.pic_set_external_field(self.h, int(ens), float(E_ext)))

    def adjoint_window(self, nsteps, ckpt_every=20):
        """Run the collisionless window with its hand-written adjoint.  Returns
        (W, dW/dv_x0 indexed by particle id, dW/dE_ext)."""
        import torch

        nb = C.c_size_t(0)
        self._check(self.L.pic_adjoint_query(self.h, int(nsteps), int(ckpt_every), C.byref(nb)))
        scratch = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
        cap = int(self.work["ensembles"][0]["species"][0]["capacity"])
        g = np.zeros(cap)
        W, gE = C.c_double(0), C.c_double(0)
        self._check(self.L.pic_adjoint_window(self.h, int(nsteps), int(ckpt_every),
                                              C.c_void_p(scratch.data_ptr()), nb.value, C.byref(W),
                                              _ptr(g), cap, C.byref(gE), self._s()))
        del scratch
        return W.value, g, gE.value

    def adjoint_window_noalloc(self, nsteps, ckpt_every=20):
        """adjoint_window on the library's static device scratch (no device allocation in
        the call).  Returns (W, dW/dv_x0 indexed by particle id, dW/dE_ext)."""
        cap = int(self.work["ensembles"][0]["species"][0]["capacity"])
        g = np.zeros(cap)
        W, gE = C.c_double(0), C.c_double(0)
        self._check(self.L.pic_adjoint_window_noalloc(self.h, int(nsteps), int(ckpt_every), C.byref(W),
                                                      _ptr(g), cap, C.byref(gE), self._s()))
        return W.value, g, gE.value

    def autotune(self, trial_steps=10):
        """Let the library time its launch shapes and keep the fastest; returns the shape."""
        shape = np.zeros(5, dtype=np.int32)
        self._check(self.L.pic_autotune(self.h, int(trial_steps), _ptr(shape), self._s()))
        return {"ppt": int(shape[0]), "window": int(shape[1]), "sort_ppt": int(shape[2]),
                "nontemporal": int(shape[3]) | (int(shape[4]) << 1)}

    def save(self):
        """Checkpoint of the run at the current step boundary (a host uint8 array)."""
        nb = C.c_size_t(0)
        self._check(self.L.pic_checkpoint_size(self.h, C.byref(nb), self._s()))
        buf = np.empty(nb.value, dtype=np.uint8)
        self._check(self.L.pic_save(self.h, _ptr(buf), buf.nbytes, self._s()))
        return buf

    def load(self, buf):
        """Continue from a checkpoint written by save() of a run with the same configuration."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.L.pic_load(self.h, _ptr(buf), buf.nbytes, self._s()))

    def timing(self, enable=True):
        self._check(self.L.pic_timing(self.h, int(bool(enable))))

    def timing_read(self):
        ms, n = C.c_double(0), C.c_int64(0)
        self._check(self.L.pic_timing_read(self.h, C.byref(ms), C.byref(n), self._s()))
        return ms.value, n.value

    def set_step(self, n):
        self._check(self.L.pic_set_step(self.h, int(n)))

    # ---- data exchange ------------------------------------------------------------------
    def diag(self, ens=0):
        d = DiagOut()
        self._check(self.L.pic_diag(self.h, int(ens), C.byref(d), None, self._s()))
        return d.as_dict()

    def moments(self, ens=0):
        """Node moments (reading R27) of each species of ensemble `ens`: a list of dicts
        with n, ux, uy, uz, T per node (host arrays), computed by the library's kernels
        into a device buffer through pic_diag."""
        import torch

        nn = self.nnodes(ens)
        buf = torch.empty(self.nspecies * 5 * nn, dtype=torch.float64, device="cuda")
        d = DiagOut()
        self._check(self.L.pic_diag(self.h, int(ens), C.byref(d), C.c_void_p(buf.data_ptr()), self._s()))
        m = buf.cpu().numpy().reshape(self.nspecies, 5, nn)
        return [{k: m[s, q].copy() for q, k in enumerate(("n", "ux", "uy", "uz", "T"))}
                for s in range(self.nspecies)]

    def nnodes(self, ens=0):
        return int(self.L.pic_nnodes(self.h, int(ens)))

    def particles(self, ens=0, s=0):
        """Alive particles of species s (2: the recycled neutrals) as host arrays."""
        e = self.work["ensembles"][ens]
        cap = int(e["species"][s]["capacity"]) if s < 2 else int(e.get("neutral_capacity", 0))
        cap = max(cap, 1)
        x, vx, vy, vz = (np.empty(cap) for _ in range(4))
        ids = np.empty(cap, dtype=np.uint32)
        p = Particles(x.ctypes.data_as(C.POINTER(C.c_double)), vx.ctypes.data_as(C.POINTER(C.c_double)),
                      vy.ctypes.data_as(C.POINTER(C.c_double)), vz.ctypes.data_as(C.POINTER(C.c_double)),
                      ids.ctypes.data_as(C.POINTER(C.c_uint32)))
        n = C.c_int64(0)
        self._check(self.L.pic_get_particles(self.h, int(ens), int(s), p, cap, C.byref(n), self._s()))
        k = n.value
        return {"x": x[:k].copy(), "vx": vx[:k].copy(), "vy": vy[:k].copy(), "vz": vz[:k].copy(),
                "id": ids[:k].copy()}

    def slots(self, ens, s, first, count):
        """Raw slots [first, first + count) (absorbed slots have x = -1)."""
        x, vx, vy, vz = (np.empty(count) for _ in range(4))
        ids = np.empty(count, dtype=np.uint32)
        p = Particles(x.ctypes.data_as(C.POINTER(C.c_double)), vx.ctypes.data_as(C.POINTER(C.c_double)),
                      vy.ctypes.data_as(C.POINTER(C.c_double)), vz.ctypes.data_as(C.POINTER(C.c_double)),
                      ids.ctypes.data_as(C.POINTER(C.c_uint32)))
        self._check(self.L.pic_get_slots(self.h, int(ens), int(s), int(first), int(count), p, self._s()))
        return {"x": x, "vx": vx, "vy": vy, "vz": vz, "id": ids}

    def set_particles(self, ens, s, x, vx, vy, vz, ids, next_id):
        x, vx, vy, vz = (np.ascontiguousarray(a, dtype=np.float64) for a in (x, vx, vy, vz))
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        p = Particles(x.ctypes.data_as(C.POINTER(C.c_double)), vx.ctypes.data_as(C.POINTER(C.c_double)),
                      vy.ctypes.data_as(C.POINTER(C.c_double)), vz.ctypes.data_as(C.POINTER(C.c_double)),
                      ids.ctypes.data_as(C.POINTER(C.c_uint32)))
        self._check(self.L.pic_set_particles(self.h, int(ens), int(s), p, len(x), int(next_id), self._s()))

    def set_state(self, state, ens=0):
        for s, st in enumerate(state):
            self.set_particles(ens, s, st["x"], st["vx"], st["vy"], st["vz"], st["id"], st["next_id"])

    def grid(self, ens=0):
        nn = self.nnodes(ens)
        Q0, Q1, rho, phi, E = (np.zeros(nn) for _ in range(5))
        self._check(self.L.pic_get_grid(self.h, int(ens), _ptr(Q0), _ptr(Q1), _ptr(rho), _ptr(phi),
                                        _ptr(E), self._s()))
        return {"Q": [Q0, Q1][: self.nspecies], "rho": rho, "phi": phi, "E": E}

    def gather_table(self, ens=0):
        """The FP32 form's per-cell (E_j, E_{j+1} - E_j) table, shape (ncells, 2), float32."""
        nn = self.nnodes(ens)
        ncells = nn if self.work["ensembles"][ens]["periodic"] else nn - 1
        out = np.zeros((ncells, 2), dtype=np.float32)
        self._check(self.L.pic_get_gather_table(self.h, int(ens), _ptr(out), self._s()))
        return out

    def set_fields(self, E, ens=0):
        E = np.ascontiguousarray(E, dtype=np.float64)
        assert len(E) == self.nnodes(ens)
        self._check(self.L.pic_set_fields(self.h, int(ens), _ptr(E), self._s()))


def _picwindow():
    import torch

    class PicWindow(torch.autograd.Function):
        """Field energy W after `nsteps` collisionless steps as a function of the initial
        x velocities (indexed by particle id) and the uniform external field, with the
        gradient from the library's hand-written discrete adjoint."""

        @staticmethod
        def forward(ctx, vx0, E_ext, sim, state, nsteps, ckpt_every):
            v = vx0.detach().to("cpu", torch.float64).numpy()
            ids = state["id"]
            sim.set_external_field(float(E_ext))
            sim.set_particles(0, 0, state["x"], v[ids], state["vy"], state["vz"], ids, state["next_id"])
            sim.set_step(0)
            W, g, gE = sim.adjoint_window(int(nsteps), int(ckpt_every))
            n = vx0.shape[0]
            ctx.save_for_backward(torch.as_tensor(g[:n], dtype=vx0.dtype, device=vx0.device),
                                  torch.as_tensor(gE, dtype=E_ext.dtype, device=E_ext.device))
            return torch.as_tensor(W, dtype=vx0.dtype, device=vx0.device)

        @staticmethod
        def backward(ctx, gW):
            g, gE = ctx.saved_tensors
            return gW * g, gW * gE, None, None, None, None

    return PicWindow


def __getattr__(name):
    if name == "PicWindow":
        return _picwindow()
    raise AttributeError(name)
