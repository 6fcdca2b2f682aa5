"""CPU oracle of the electrostatic 1D3V PIC Monte Carlo step (FP64, single-threaded).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of the
benchmark may use it; the product path never imports it.  The arithmetic lives in
pic_oracle.c (plain C, one loop per stage); this module compiles it with gcc and exposes
it through ctypes.  Nothing here imports the GPU package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
HDR = os.path.join(HERE, "pic_oracle.h")
LIB = os.path.join(HERE, "liboracle.so")
# The same source built with OpenMP on its particle loops: used only to time the oracle on
# all host cores (its deposit sums per-thread partials, so it is not the parity reference).
LIB_OMP = os.path.join(HERE, "liboracle_omp.so")


def _stale(lib):
    return not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(SRC), os.path.getmtime(HDR))


def build(force=True, omp=None):
    """Compile liboracle.so (gcc, -O2, no fused multiply-add, single-threaded) and
    liboracle_omp.so (the same with -fopenmp, for timing only).  `omp` None builds both."""
    for want, lib_path, extra in ((False, LIB, []), (True, LIB_OMP, ["-fopenmp"])):
        if omp is not None and omp != want:
            continue
        if not force and not _stale(lib_path):
            continue
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wno-unknown-pragmas", "-ffp-contract=off", "-fPIC",
               "-shared", *extra, "-o", lib_path + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(lib_path + ".tmp", lib_path)
    return LIB


class _Species(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("w", C.c_double), ("T", C.c_double),
                ("ppc", C.c_int64), ("capacity", C.c_int64)]


class _Config(C.Structure):
    _fields_ = [("ncells", C.c_int64), ("periodic", C.c_int32), ("nspecies", C.c_int32),
                ("collisions", C.c_int32), ("init_mode", C.c_int32),
                ("dx", C.c_double), ("dt", C.c_double), ("eps0", C.c_double),
                ("B", C.c_double * 3), ("E_ext", C.c_double), ("seed", C.c_uint32),
                ("sort_every", C.c_int32), ("sp", _Species * 2),
                ("ngs_el", C.c_double), ("ngs_iz", C.c_double), ("ngs_cx", C.c_double),
                ("eps_iz", C.c_double), ("T_n", C.c_double), ("m_n", C.c_double),
                ("perturb_amp", C.c_double), ("perturb_mode", C.c_int32),
                ("floating", C.c_int32), ("smooth", C.c_int32), ("recycle", C.c_int32),
                ("neutral_capacity", C.c_int64), ("src_pairs", C.c_int64), ("src_frac", C.c_double),
                ("cx_relative", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("count", C.c_int64 * 2), ("charge", C.c_double), ("ke", C.c_double * 2),
                ("field_energy", C.c_double), ("wall_count", (C.c_int64 * 2) * 2),
                ("wall_charge", (C.c_double * 2) * 2), ("wall_ke", (C.c_double * 2) * 2),
                ("coll", C.c_int64 * 3), ("created", C.c_int64 * 2), ("pushes", C.c_int64),
                ("step", C.c_int64), ("neutral_count", C.c_int64), ("neutral_wall", C.c_int64 * 2),
                ("recycled", C.c_int64), ("sourced", C.c_int64)]

    def as_dict(self):
        return {
            "count": list(self.count), "charge": self.charge, "ke": list(self.ke),
            "field_energy": self.field_energy,
            "wall_count": [list(r) for r in self.wall_count],
            "wall_charge": [list(r) for r in self.wall_charge],
            "wall_ke": [list(r) for r in self.wall_ke],
            "coll": list(self.coll), "created": list(self.created), "pushes": self.pushes,
            "step": self.step, "neutral_count": self.neutral_count,
            "neutral_wall": list(self.neutral_wall), "recycled": self.recycled,
            "sourced": self.sourced,
        }


_libs = {}


def lib(omp=False):
    """The oracle's C library: the single-threaded build, or (omp=True) the OpenMP timing
    build."""
    if omp not in _libs:
        path = LIB_OMP if omp else LIB
        if not os.path.exists(path):
            build(force=True, omp=omp)
        L = C.CDLL(path)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.POINTER(_Config)]
        for name in ("orc_free", "orc_init", "orc_deposit", "orc_solve", "orc_push",
                     "orc_walls", "orc_collide", "orc_sort"):
            getattr(L, name).argtypes = [P]
            getattr(L, name).restype = None
        L.orc_error.argtypes = [P]
        L.orc_error.restype = C.c_int
        L.orc_step.argtypes = [P, C.c_int64]
        L.orc_set_particles.argtypes = [P, C.c_int, C.c_int64, P, P, P, P, P, C.c_uint32]
        L.orc_set_particles.restype = C.c_int
        L.orc_get_particles.argtypes = [P, C.c_int, P, P, P, P, P]
        L.orc_get_particles.restype = C.c_int64
        L.orc_next_id.argtypes = [P, C.c_int]
        L.orc_next_id.restype = C.c_uint32
        L.orc_nnodes.argtypes = [P]
        L.orc_nnodes.restype = C.c_int64
        L.orc_get_grid.argtypes = [P, P, P, P, P, P]
        L.orc_set_fields.argtypes = [P, P]
        L.orc_get_diag.argtypes = [P, C.POINTER(Diag)]
        L.orc_last_channels.argtypes = [P, C.c_int, P, P]
        L.orc_last_channels.restype = C.c_int64
        L.orc_last_numax.argtypes = [P, P, P]
        L.orc_moments.argtypes = [P, C.c_int, P, P, P, P, P]
        L.orc_moments.restype = None
        L.orc_set_step.argtypes = [P, C.c_int64]
        L.orc_init_particle.argtypes = [C.POINTER(_Config), C.c_int, C.c_int64, P, P, P, P]
        L.orc_philox4x32.argtypes = [P, P, P]
        L.orc_philox_batch.argtypes = [C.c_int64, P, P, P]
        L.orc_uniform.argtypes = [C.c_uint32]
        L.orc_uniform.restype = C.c_double
        L.orc_boxmuller.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double)]
        L.orc_thomas.argtypes = [C.c_int64, P, P, P, P, P]
        L.orc_smooth_nodes.argtypes = [C.c_int64, C.c_int32, C.c_int32, P]
        L.orc_smooth_nodes.restype = None
        L.orc_threads.argtypes = []
        L.orc_threads.restype = C.c_int
        _libs[omp] = L
    return _libs[omp]


def threads(omp=False):
    """Threads the oracle's particle loops use in that build."""
    return int(lib(omp).orc_threads())


def _ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else None


def make_config(e):
    """Translate an ensemble dict (see the synth module) into the oracle's C config."""
    c = _Config()
    c.ncells = e["ncells"]
    c.periodic = int(e["periodic"])
    c.nspecies = e["nspecies"]
    c.collisions = int(e["collisions"])
    c.init_mode = e["init_mode"]
    c.dx, c.dt, c.eps0 = e["dx"], e["dt"], e["eps0"]
    for i in range(3):
        c.B[i] = e["B"][i]
    c.E_ext = e["E_ext"]
    c.seed = e["seed"]
    c.sort_every = e["sort_every"]
    for s, sp in enumerate(e["species"]):
        c.sp[s].q, c.sp[s].m, c.sp[s].w, c.sp[s].T = sp["q"], sp["m"], sp["w"], sp["T"]
        c.sp[s].ppc, c.sp[s].capacity = sp["ppc"], sp["capacity"]
    c.ngs_el, c.ngs_iz, c.ngs_cx = e["ngs_el"], e["ngs_iz"], e["ngs_cx"]
    c.eps_iz, c.T_n, c.m_n = e["eps_iz"], e["T_n"], e["m_n"]
    c.perturb_amp, c.perturb_mode = e["perturb_amp"], e["perturb_mode"]
    c.floating = int(e.get("floating", False))
    c.smooth = int(e.get("smooth", 0))
    c.recycle = int(e.get("recycle", False))
    c.neutral_capacity = int(e.get("neutral_capacity", 0))
    c.src_pairs = int(e.get("src_pairs", 0))
    c.src_frac = float(e.get("src_frac", 0.5))
    c.cx_relative = int(e.get("cx_relative", False))
    return c


class Oracle:
    """One ensemble of the oracle.  Stage methods mirror the C functions."""

    def __init__(self, e, init=True, omp=False):
        self.e = e
        self._cfg = make_config(e)
        self.L = lib(omp)
        self.h = C.c_void_p(self.L.orc_create(C.byref(self._cfg)))
        self.nspecies = e["nspecies"]
        self.nnodes = int(self.L.orc_nnodes(self.h))
        if init:
            self.init()

    def __del__(self):
        try:
            if self.h:
                self.L.orc_free(self.h)
                self.h = None
        except Exception:
            pass

    @property
    def error(self):
        return int(self.L.orc_error(self.h))

    def init(self):
        self.L.orc_init(self.h)

    def deposit(self):
        self.L.orc_deposit(self.h)

    def solve(self):
        self.L.orc_solve(self.h)

    def push(self):
        self.L.orc_push(self.h)

    def walls(self):
        self.L.orc_walls(self.h)

    def collide(self):
        self.L.orc_collide(self.h)

    def sort(self):
        self.L.orc_sort(self.h)

    def step(self, n=1):
        self.L.orc_step(self.h, int(n))

    def set_step(self, n):
        self.L.orc_set_step(self.h, int(n))

    def set_particles(self, s, x, vx, vy, vz, ids, next_id):
        x = np.ascontiguousarray(x, dtype=np.float64)
        vx = np.ascontiguousarray(vx, dtype=np.float64)
        vy = np.ascontiguousarray(vy, dtype=np.float64)
        vz = np.ascontiguousarray(vz, dtype=np.float64)
        ids = np.ascontiguousarray(ids, dtype=np.uint32)
        rc = self.L.orc_set_particles(self.h, s, len(x), _ptr(x), _ptr(vx), _ptr(vy), _ptr(vz),
                                      _ptr(ids), int(next_id))
        if rc != 0:
            raise ValueError("orc_set_particles failed")

    def set_state(self, state):
        for s, st in enumerate(state):
            self.set_particles(s, st["x"], st["vx"], st["vy"], st["vz"], st["id"], st["next_id"])

    def particles(self, s):
        cap = self.e["species"][s]["capacity"] if s < 2 else int(self.e.get("neutral_capacity", 0))
        x = np.empty(cap + 1)
        vx, vy, vz = np.empty(cap + 1), np.empty(cap + 1), np.empty(cap + 1)
        ids = np.empty(cap + 1, dtype=np.uint32)
        n = int(self.L.orc_get_particles(self.h, s, _ptr(x), _ptr(vx), _ptr(vy), _ptr(vz), _ptr(ids)))
        return {"x": x[:n].copy(), "vx": vx[:n].copy(), "vy": vy[:n].copy(), "vz": vz[:n].copy(),
                "id": ids[:n].copy(), "next_id": int(self.L.orc_next_id(self.h, s))}

    def grid(self):
        nn = self.nnodes
        Q0, Q1, rho, phi, E = (np.zeros(nn) for _ in range(5))
        self.L.orc_get_grid(self.h, _ptr(Q0), _ptr(Q1), _ptr(rho), _ptr(phi), _ptr(E))
        return {"Q": [Q0, Q1][: self.nspecies], "rho": rho, "phi": phi, "E": E}

    def set_fields(self, E):
        E = np.ascontiguousarray(E, dtype=np.float64)
        assert len(E) == self.nnodes
        self.L.orc_set_fields(self.h, _ptr(E))

    def diag(self):
        d = Diag()
        self.L.orc_get_diag(self.h, C.byref(d))
        return d.as_dict()

    def moments(self, s):
        """Node moments of species s (reading R27): dict of n, ux, uy, uz, T per node."""
        out = {k: np.zeros(self.nnodes) for k in ("n", "ux", "uy", "uz", "T")}
        self.L.orc_moments(self.h, int(s), *(_ptr(out[k]) for k in ("n", "ux", "uy", "uz", "T")))
        return out

    def last_channels(self, s):
        cap = self.e["species"][s]["capacity"]
        ch = np.empty(cap + 1, dtype=np.int32)
        ids = np.empty(cap + 1, dtype=np.uint32)
        n = int(self.L.orc_last_channels(self.h, s, _ptr(ch), _ptr(ids)))
        return ch[:n].copy(), ids[:n].copy()

    def last_numax(self):
        nu = np.zeros(2)
        pn = np.zeros(2)
        self.L.orc_last_numax(self.h, _ptr(nu), _ptr(pn))
        return nu, pn


def init_particles(e, s, ps):
    """The load of particles `ps` (indices) of species s of ensemble dict e, one by one."""
    cfg = make_config(e)
    ps = np.asarray(ps, dtype=np.int64)
    out = {k: np.empty(len(ps)) for k in ("x", "vx", "vy", "vz")}
    L = lib()
    x, vx, vy, vz = (C.c_double() for _ in range(4))
    for i, p in enumerate(ps):
        L.orc_init_particle(C.byref(cfg), int(s), int(p), C.byref(x), C.byref(vx), C.byref(vy),
                            C.byref(vz))
        out["x"][i], out["vx"][i], out["vy"][i], out["vz"][i] = x.value, vx.value, vy.value, vz.value
    out["id"] = ps.astype(np.uint32)
    return out


def philox(ctr, key):
    """Philox4x32 (seven rounds, reading R17) of counter (4 words) and key (2 words) -> 4 words."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_batch(ctr, key):
    """Row-wise Philox4x32 (seven rounds): ctr (n, 4), key (n, 2) -> (n, 4)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros((len(c), 4), dtype=np.uint32)
    lib().orc_philox_batch(len(c), _ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(r):
    return float(lib().orc_uniform(int(r)))


def boxmuller(u1, u2):
    z0, z1 = C.c_double(), C.c_double()
    lib().orc_boxmuller(float(u1), float(u2), C.byref(z0), C.byref(z1))
    return z0.value, z1.value


def thomas(a, b, c, d):
    a, b, c, d = (np.ascontiguousarray(v, dtype=np.float64) for v in (a, b, c, d))
    x = np.zeros(len(b))
    lib().orc_thomas(len(b), _ptr(a), _ptr(b), _ptr(c), _ptr(d), _ptr(x))
    return x


def smooth_nodes(rho, periodic, passes):
    """`passes` of the oracle's 1-2-1 density filter (R23) on a copy of rho."""
    r = np.array(rho, dtype=np.float64, copy=True)
    lib().orc_smooth_nodes(len(r), int(bool(periodic)), int(passes), _ptr(r))
    return r
