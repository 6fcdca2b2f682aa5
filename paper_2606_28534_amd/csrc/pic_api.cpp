// pic_api.cpp -- C ABI, context and workspace management, step scheduling and HIP graph
// capture of the gfx950 PIC MC library.  See include/pic.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pic.h"
#include "pic_device.h"
#include "pic_kernels.h"

using namespace pic;

// Device scratch of pic_adjoint_window_noalloc, the adjoint window for callers that cannot
// allocate: one copy of this array on every GPU the library runs on, held until the process
// ends.  Host code never passes the array's name to a kernel or copy (on the host it is a
// stand-in, not a device address): pic_init looks up its address on the current device once
// (hipGetSymbolAddress) and every use goes through that pointer.
constexpr size_t kStaticScratchBytes = (size_t)160 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr size_t kAlign = 256;
constexpr int kCompactEvery = 20;  // sort cadence used for compaction when K = 0
constexpr int kDiagGrid = 256;


size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Sizes derived from a configuration; shared by the query and the carving.
struct Plan {
    int nens = 0, nseg = 0, nspecies = 0;
    bool f64 = false;
    std::vector<SegC> seg;
    std::vector<EnsC> ens;
    int64_t cap_tot = 0, nodes_tot = 0, cells_tot = 0, chunks_tot = 0;
    int64_t birth_stripe_cap = 0, bm_words = 0, g_tot = 0;
    int64_t scanpart = 0;
    int64_t ncap_tot = 0, rec_cap = 0, src_tot = 0;  // neutrals (R24), source (R25)
    size_t bytes = 0;
};

int build_plan(const pic_config *cfg, Plan &P, std::string &msg)
{
    if (!cfg || !cfg->ens) {
        msg = "null config";
        return PIC_EINVAL;
    }
    if (cfg->n_ensembles < 1 || cfg->n_ensembles > 256) {
        msg = "n_ensembles must be in [1, 256]";
        return PIC_EINVAL;
    }
    if (cfg->nspecies < 1 || cfg->nspecies > 2) {
        msg = "nspecies must be 1 or 2";
        return PIC_EINVAL;
    }
    if (cfg->precision != PIC_FP64_PLAIN && cfg->precision != PIC_FP32_CELLOFF) {
        msg = "bad precision";
        return PIC_EINVAL;
    }
    if (cfg->boundary != PIC_ABSORBING && cfg->boundary != PIC_PERIODIC &&
        cfg->boundary != PIC_FLOATING) {
        msg = "bad boundary";
        return PIC_EINVAL;
    }
    if (cfg->smooth < 0 || cfg->smooth > kMaxSmooth) {
        msg = "smooth must be in [0, " + std::to_string(kMaxSmooth) + "]";
        return PIC_EINVAL;
    }
    if (cfg->window != 0 && (cfg->window < 16 || cfg->window > 4096)) {
        msg = "window must be 0 (default) or in [16, 4096]";
        return PIC_EINVAL;
    }
    if (cfg->sort_every < 0 || cfg->sort_every > 4096) {
        msg = "sort_every must be in [0, 4096] (a fused run captures one sort cycle as a graph)";
        return PIC_EINVAL;
    }
    if (cfg->block != 0 && cfg->block != 64 && cfg->block != 128 && cfg->block != 256) {
        msg = "block must be 0 (default), 64, 128 or 256";
        return PIC_EINVAL;
    }
    P.nens = cfg->n_ensembles;
    P.nspecies = cfg->nspecies;
    P.nseg = P.nens * P.nspecies;
    P.f64 = cfg->precision == PIC_FP64_PLAIN;
    const bool periodic = cfg->boundary == PIC_PERIODIC;
    int64_t base = 0, gbase = 0, cbase = 0, chunk0 = 0, bm = 0, grp = 0, ecap = 0;
    int64_t nbase = 0, src_base = 0, icap = 0;
    for (int e = 0; e < P.nens; ++e) {
        const pic_ensemble_desc &D = cfg->ens[e];
        if (D.ncells < 2 || D.ncells > (int64_t)1 << 30 || !(D.dx > 0) || !(D.dt > 0) || !(D.eps0 > 0)) {
            msg = "ensemble " + std::to_string(e) + ": bad ncells/dx/dt/eps0";
            return PIC_EINVAL;
        }
        EnsC E{};
        E.ncells = D.ncells;
        E.nnodes = periodic ? D.ncells : D.ncells + 1;
        E.gbase = gbase;
        E.chunk0 = chunk0;
        E.nchunks = (E.nnodes + kChunk - 1) / kChunk;
        E.dx = D.dx;
        E.dt = D.dt;
        E.eps0 = D.eps0;
        E.E_ext = D.E_ext;
        E.L = (double)D.ncells * D.dx;
        E.ngs_el = D.ngs_el;
        E.ngs_iz = D.ngs_iz;
        E.ngs_cx = D.ngs_cx;
        E.eps_iz = D.eps_iz;
        E.vn = (D.m_n > 0) ? std::sqrt(D.T_n / D.m_n) : 0.0;
        // reading R26: a Box-Muller radius is at most sqrt(48 ln 2) (uniforms >= 2^-24) and two
        // of a neutral's three normals share one radius: |v_n| <= sqrt(96 ln 2) v_tn
        E.cx_rel = D.cx_relative ? 1 : 0;
        E.vn_max = D.cx_relative ? std::sqrt(96.0 * std::log(2.0)) * E.vn : 0.0;
        E.m_e = D.sp[0].m;
        E.m_n = D.m_n;
        E.seed = D.seed;
        E.periodic = periodic ? 1 : 0;
        E.floating = cfg->boundary == PIC_FLOATING ? 1 : 0;
        E.smooth = cfg->smooth;
        E.nspecies = P.nspecies;
        // the sheath cases' recycling walls (R24) and volumetric source (R25)
        if (D.recycle || D.src_pairs) {
            if (P.f64 || P.nspecies != 2) {
                msg = "ensemble " + std::to_string(e) + ": recycling and the source need the FP32 form and two species";
                return PIC_EINVAL;
            }
            if (D.recycle && (periodic || D.neutral_capacity < 1 || !(D.m_n > 0))) {
                msg = "ensemble " + std::to_string(e) + ": recycling needs bounded walls, neutral_capacity >= 1 and m_n > 0";
                return PIC_EINVAL;
            }
            if (D.src_pairs < 0 || D.src_pairs > ((int64_t)1 << 24) || !(D.src_frac > 0.0 && D.src_frac <= 1.0)) {
                msg = "ensemble " + std::to_string(e) + ": src_pairs must be in [0, 2^24] and src_frac in (0, 1]";
                return PIC_EINVAL;
            }
        }
        E.recycle = D.recycle ? 1 : 0;
        E.nbase = nbase;
        E.ncap = D.recycle ? (D.neutral_capacity + 255) / 256 * 256 : 0;
        nbase += E.ncap;
        E.src_pairs = D.src_pairs;
        E.src_base = src_base;
        src_base += D.src_pairs;
        E.src_x = D.src_frac * ((double)D.ncells * D.dx);
        // ids (loaded and born) stay below 2 x electron capacity, rounded to 1024
        int64_t idcap = (2 * D.sp[0].capacity + 2048) / 1024 * 1024;
        idcap = std::min<int64_t>(idcap, ((int64_t)1 << 32) - 1024);
        E.idcap = idcap;
        // birth ranking: a bit per id (whole 128-byte groups) and a count per kGroupIds ids
        E.bm_base = bm;
        E.grp_base = grp;
        const int64_t ngrp = (idcap + kGroupIds - 1) / kGroupIds;
        bm += ngrp * kGroupWords;
        grp += ngrp;
        for (int s = 0; s < P.nspecies; ++s) {
            const pic_species_desc &sp = D.sp[s];
            if (sp.capacity < sp.ppc * D.ncells || sp.capacity < 1 || sp.ppc < 0 || !(sp.m > 0)) {
                msg = "ensemble " + std::to_string(e) + " species " + std::to_string(s) +
                      ": capacity < ppc * ncells or bad mass";
                return PIC_EINVAL;
            }
            if (sp.capacity > ((int64_t)1 << 32) - 1) {
                msg = "capacity above 2^32 - 1 per species";
                return PIC_EINVAL;
            }
            E.qw[s] = sp.q * sp.w;
            SegC S{};
            S.base = base;
            // at least one aligned slot range, so an empty species still has a tile
            S.cap = std::max<int64_t>((sp.capacity + kSlotAlign - 1) / kSlotAlign, 1) * kSlotAlign;
            S.cbase = cbase;
            S.gbase = gbase;
            S.ens = e;
            S.species = s;
            S.ncells = (int32_t)D.ncells;
            S.periodic = E.periodic;
            S.h = sp.q / sp.m * 0.5 * D.dt;
            for (int k = 0; k < 3; ++k) S.t[k] = S.h * D.B[k];
            const double tt = S.t[0] * S.t[0] + S.t[1] * S.t[1] + S.t[2] * S.t[2];
            for (int k = 0; k < 3; ++k) S.s[k] = 2.0 / (1.0 + tt) * S.t[k];
            S.dt = D.dt;
            S.dx = D.dx;
            S.dtdx = D.dt / D.dx;
            S.qw = sp.q * sp.w;
            S.halfmw = 0.5 * sp.m * sp.w;
            S.m = sp.m;
            S.ngsT = cfg->collisions ? ((s == 0) ? D.ngs_el + D.ngs_iz : D.ngs_cx) : 0.0;
            S.qm_abs = std::fabs(sp.q / sp.m);
            S.seed = D.seed;
            S.other = (s == 0 && P.nspecies > 1) ? (int32_t)(P.seg.size() + 1) : -1;
            S.recycle = (s == 1 && D.recycle) ? 1 : 0;
            S.vth = std::sqrt(sp.T / sp.m);
            S.w = sp.w;
            if (s == 1) icap += sp.capacity;
            E.seg[s] = (int32_t)P.seg.size();
            P.seg.push_back(S);
            base += S.cap;
            cbase += D.ncells;
            if (s == 0) ecap += sp.capacity;
        }
        if (P.nspecies == 1) E.seg[1] = -1;
        P.ens.push_back(E);
        gbase += E.nnodes;
        chunk0 += E.nchunks;
    }
    P.cap_tot = base;
    P.ncap_tot = nbase;
    P.src_tot = src_base;
    // absorbed ions listed per step: generous against the ions within v dt of a wall
    P.rec_cap = nbase ? std::max<int64_t>(65536, icap / 256) : 0;
    P.bm_words = bm;
    P.g_tot = (grp + 1 + 4095) / 4096 * 4096;  // room for the total; whole scan tiles
    if (P.cap_tot >= ((int64_t)1 << 32)) {
        msg = "total particle capacity above 2^32 slots";
        return PIC_EINVAL;
    }
    P.nodes_tot = gbase;
    P.cells_tot = cbase;
    P.chunks_tot = chunk0;
    // births per step are ~5e-4 of the electrons; each stripe holds up to 1.5e-4 of them
    P.birth_stripe_cap = std::max<int64_t>(8192, (int64_t)std::ceil(1.5e-4 * (double)ecap));
    P.scanpart = std::max(scan_blocks(P.g_tot), scan_blocks(P.cells_tot)) + 1;
    return PIC_OK;
}

struct Carver {
    char *base;
    size_t off = 0;
    template <typename T>
    T *take(int64_t n)
    {
        T *p = base ? (T *)(base + off) : nullptr;
        off += align_up((size_t)std::max<int64_t>(n, 1) * sizeof(T));
        return p;
    }
};

// Carve the workspace (base == nullptr only measures).
size_t carve(const Plan &P, char *base, Dev &d)
{
    Carver c{base};
    memset(&d, 0, sizeof(d));
    d.nseg = P.nseg;
    d.nens = P.nens;
    d.nspecies = P.nspecies;
    d.seg = c.take<SegC>(P.nseg);
    d.ens = c.take<EnsC>(P.nens);
    for (int b = 0; b < 2; ++b) {
        d.id[b] = c.take<uint32_t>(P.cap_tot);
        if (P.f64) {
            d.x[b] = c.take<double>(P.cap_tot);
            d.dvx[b] = c.take<double>(P.cap_tot);
            d.dvy[b] = c.take<double>(P.cap_tot);
            d.dvz[b] = c.take<double>(P.cap_tot);
        } else {
            d.cell[b] = c.take<int32_t>(P.cap_tot);
            d.off[b] = c.take<float>(P.cap_tot);
            d.fvx[b] = c.take<float>(P.cap_tot);
            d.fvy[b] = c.take<float>(P.cap_tot);
            d.fvz[b] = c.take<float>(P.cap_tot);
        }
    }
    d.cap_tot = P.cap_tot;
    d.cur = c.take<int32_t>(1);
    d.n_slots = c.take<int64_t>(P.nseg);
    d.next_id = c.take<uint32_t>(P.nseg);
    d.step = c.take<int64_t>(1);
    d.nodes_tot = P.nodes_tot;
    d.cells_tot = P.cells_tot;
    d.Qi = c.take<unsigned long long>(2 * P.nodes_tot);
    d.Qd = (double *)d.Qi;
    d.rho = c.take<double>(P.nodes_tot);
    d.phi = c.take<double>(P.nodes_tot);
    d.E = c.take<double>(P.nodes_tot);
    d.Ecell = c.take<float2>(P.nodes_tot);
    d.agg = c.take<double>(P.chunks_tot * A_NAGG);
    d.part = c.take<double>(P.chunks_tot * P_NPART);
    d.emax = c.take<double>(P.nens);
    d.fe = c.take<double>(P.nens);
    d.numax = c.take<double>(P.nseg);
    d.pnull = c.take<double>(P.nseg);
    d.vmred = c.take<double>(P.nseg);
    d.vmax2 = c.take<unsigned long long>(2 * kCntStripes * P.nseg);
    d.vcur = c.take<int32_t>(1);
    d.cnt = c.take<unsigned long long>((int64_t)kCntStripes * P.nseg * C_NCNT);
    d.sums = c.take<double>((int64_t)kCntStripes * P.nseg * S_NSUM);
    d.ssum = c.take<double>((int64_t)2 * kCntStripes * P.nseg * T_NSTEP);
    d.birth_stripe_cap = P.birth_stripe_cap;
    d.births = c.take<Birth>(2 * kStripes * P.birth_stripe_cap);
    d.nbirth = c.take<uint32_t>(2 * kStripes);
    d.crec = c.take<uint4>(2 * P.cap_tot);
    d.bitmap = c.take<uint32_t>(2 * P.bm_words);
    d.bm_words = P.bm_words;
    d.gcnt = c.take<uint32_t>(2 * P.g_tot);
    d.gpre = c.take<uint32_t>(P.g_tot);
    d.g_tot = P.g_tot;
    d.ngt = P.g_tot / kGroupTile <= kMaxGroupTiles ? (int32_t)(P.g_tot / kGroupTile) : 0;
    d.gtile = c.take<uint32_t>(std::max<int64_t>(d.ngt, 1));
    d.ctile = c.take<uint32_t>(P.cap_tot / 1024 + 1);
    d.cellcnt = c.take<uint32_t>(P.cells_tot);
    d.cursor = c.take<uint32_t>(P.cells_tot);
    d.segstart = c.take<int64_t>(P.nseg);
    d.scanpart = c.take<uint32_t>(P.scanpart);
    for (int b = 0; b < 2; ++b) {
        d.ncell[b] = c.take<int32_t>(P.ncap_tot);
        d.noff[b] = c.take<float>(P.ncap_tot);
        d.nvx[b] = c.take<float>(P.ncap_tot);
        d.nvy[b] = c.take<float>(P.ncap_tot);
        d.nvz[b] = c.take<float>(P.ncap_tot);
        d.nid[b] = c.take<uint32_t>(P.ncap_tot);
    }
    d.ncap_tot = P.ncap_tot;
    d.ncur = c.take<int32_t>(1);
    d.nneu = c.take<unsigned long long>(2 * P.nens);
    d.recs = c.take<uint2>(P.rec_cap);
    d.rec_cap = P.rec_cap;
    d.nrec = c.take<uint32_t>(1);
    d.src_tot = P.src_tot;
    d.ticket = c.take<uint32_t>(8);
    d.tq = c.take<uint32_t>(16);
    d.err = c.take<int32_t>(1);
    c.take<double>(2 * kDiagGrid);  // diag scratch (last region)
    return c.off;
}

}  // namespace

struct pic_ctx {
    pic_config cfg{};
    std::vector<pic_ensemble_desc> ens;
    Plan P;
    Dev d{};
    char *ws = nullptr;
    size_t ws_bytes = 0;
    double *diag_scratch = nullptr;
    Launch L{};
    int64_t host_step = 0;
    int sort_every = 0;  // effective cadence (>= 1)
    // The histogram of the current cells has been scanned into the sort cursors, so the
    // next fused FP32 step can sort inside its particle pass.  Any call that moves, adds or
    // removes particles between steps clears it (that step then sorts the usual way).
    bool sort_ready = false;
    // The last pic_step ran the fused FP32 step with collisions, whose kernels tallied the
    // scalar diagnostics of its last step (count and sum |v|^2 per species, field energy
    // per solve chunk): pic_diag reads those instead of a pass over the particles.  Any
    // call that changes particles or fields between steps clears it.
    bool insitu = false;
    hipStream_t cap_stream = nullptr;
    // device address of the static scratch array on the context's GPU
    void *static_scratch = nullptr;
    // captured windows of the fused step, keyed by (first step's phase in the sort cycle,
    // number of steps); each replays from that phase with the prepared-sort state the
    // phase implies
    std::map<int64_t, hipGraphExec_t> graphs;
    int64_t graph_launches = 0;
    std::string msg;
    // measurement hook
    bool timing = false;
    std::vector<hipEvent_t> ev;  // pairs
    int64_t ev_used = 0;
};

namespace {

// The static scratch array's device address per GPU, looked up once per device with that
// device current (each GPU holds its own copy of the array at its own address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

hipError_t static_scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

int fail(pic_ctx *c, int code, const std::string &m)
{
    if (c) c->msg = m;
    return code;
}

int hipfail(pic_ctx *c, hipError_t e, const char *where)
{
    return fail(c, PIC_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPC(ctx, expr)                                   \
    do {                                                  \
        hipError_t _e = (expr);                           \
        if (_e != hipSuccess) return hipfail(ctx, _e, #expr); \
    } while (0)

int check_err(pic_ctx *c, hipStream_t s)
{
    int32_t err = 0;
    HIPC(c, hipMemcpyAsync(&err, c->d.err, sizeof(err), hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    if (err & (E_CAP_PART | E_CAP_BIRTH | E_CAP_ID))
        return fail(c, PIC_ECAPACITY, "capacity exceeded (flags " + std::to_string(err) + ")");
    if (err & E_NONFINITE) return fail(c, PIC_ENONFINITE, "non-finite field");
    return PIC_OK;
}

// The fused step's work after its particle pass: collision candidates (with collisions),
// recycled neutrals and the volumetric source; one launch in the FP32 form.
hipError_t launch_after_pass(pic_ctx *c, hipStream_t s, int hist)
{
    const Dev &d = c->d;
    const bool coll = c->cfg.collisions != 0;
    if (!c->P.f64) return launch_after(d, c->L.ppt, s, hist, d.cap_tot, coll);
    hipError_t e;
    if (coll && (e = launch_candidates(d, c->L, s, true, hist)) != hipSuccess) return e;
    if ((e = launch_neutrals(d, s)) != hipSuccess) return e;
    return launch_source(d, hist, s);
}

// Enqueue one full step from step count n; the step sorts when n + 1 is a multiple of K
// (never with `no_sort`).  The fused FP32 step pipelines the sort (K >= 2): the step before
// a sort step counts the cells after its push and scans the counts, and the sort step's
// particle pass writes every particle at its place in cell order (`ready` carries that
// state between the two steps).  Otherwise the sort step counts and then sorts in kernels
// of its own.
hipError_t enqueue_step(pic_ctx *c, hipStream_t s, int64_t n, bool &ready, bool no_sort)
{
    const Dev &d = c->d;
    const bool f64 = c->P.f64;
    const bool coll = c->cfg.collisions != 0;
    const int K = c->sort_every;
    const bool sort_now = !no_sort && (n + 1) % K == 0;
    hipError_t e;
    bool tm = c->timing && c->ev_used + 2 <= (int64_t)c->ev.size();
    if (c->cfg.fused) {
        const bool piped = !f64 && K >= 2 && !no_sort;
        const bool sorting = piped && sort_now && ready;
        tm = tm && !sorting;  // the measurement hook times the plain pass only
        const bool prep = piped && (n + 2) % K == 0;
        const int hist = (prep || (sort_now && !sorting)) ? 1 : 0;
        // the solve's last block computes the collision bound, so the measurement hook
        // times the particle pass alone
        if ((e = launch_solve(d, f64, c->P.chunks_tot, true, s, false, coll)) != hipSuccess) return e;
        const int stages = coll ? (SB_PUSH | SB_COLLIDE | SB_DEPOSIT) : (SB_PUSH | SB_DEPOSIT);
        if (tm && (e = hipEventRecord(c->ev[c->ev_used], s)) != hipSuccess) return e;
        if (sorting)
            e = launch_pass32_sort(d, c->L.ppt, c->L.window, s, coll, d.cap_tot, c->L.nt != 0);
        else
            e = launch_particles(d, c->L, s, f64, stages, hist, false);
        if (e != hipSuccess) return e;
        if (tm) {
            if ((e = hipEventRecord(c->ev[c->ev_used + 1], s)) != hipSuccess) return e;
            c->ev_used += 2;
        }
        if ((e = launch_after_pass(c, s, hist)) != hipSuccess) return e;
        if (coll) {
            if ((e = launch_births(d, f64, true, true, s)) != hipSuccess) return e;
        } else if ((e = launch_advance(d, s)) != hipSuccess) {
            return e;
        }
        if (sort_now && !sorting && (e = launch_sort(d, f64, c->L, s)) != hipSuccess) return e;
        if (prep && !sort_now) {
            if ((e = launch_sort_prepare(d, s)) != hipSuccess) return e;
            ready = true;
        } else {
            ready = false;
        }
        return hipSuccess;
    }
    ready = false;
    if ((e = launch_solve(d, f64, c->P.chunks_tot, false, s)) != hipSuccess) return e;
    if (tm && (e = hipEventRecord(c->ev[c->ev_used], s)) != hipSuccess) return e;
    if ((e = launch_particles(d, c->L, s, f64, SB_PUSH, 0)) != hipSuccess) return e;
    if (tm) {
        if ((e = hipEventRecord(c->ev[c->ev_used + 1], s)) != hipSuccess) return e;
        c->ev_used += 2;
    }
    if ((e = launch_neutrals(d, s)) != hipSuccess) return e;
    if (coll) {
        if ((e = launch_particles(d, c->L, s, f64, SB_COLLIDE, 0)) != hipSuccess) return e;
        if ((e = launch_candidates(d, c->L, s, f64, 0)) != hipSuccess) return e;
    }
    if ((e = launch_source(d, 0, s)) != hipSuccess) return e;
    if (coll && (e = launch_births(d, f64, true, false, s)) != hipSuccess) return e;
    if ((e = launch_zero_q(d, f64, s)) != hipSuccess) return e;
    if ((e = launch_particles(d, c->L, s, f64, SB_DEPOSIT, 0)) != hipSuccess) return e;
    if ((e = launch_advance(d, s)) != hipSuccess) return e;
    if (sort_now) {
        if ((e = launch_particles(d, c->L, s, f64, SB_HIST, 0)) != hipSuccess) return e;
        if ((e = launch_sort(d, f64, c->L, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// A window of `len` steps of the fused step, starting at step count n0, for graph capture.
// With collisions (and births small enough for the solve's extra blocks) the births of
// step i - 1 are ranked and placed by extra blocks of step i's two solve kernels instead
// of kernels of their own: the placement touches new particle slots, the slot and id
// counters, the birth lists and bitmaps, the speed-maximum halves and the step counter,
// the solve only the grid, so they run side by side, and the collision parameters and the
// particle pass after them see both.  A step that sorts in kernels of its own (FP64, K = 1,
// or no prepared counts) places its births in line before its sort, and so does the last
// step of the window.  The FP32 form pipelines the sort as enqueue_step does: the step
// before a sort step counts and scans, the sort step's pass sorts.  `ready` is the
// prepared-sort state on entry and on exit.  The state after the window is the same as
// after `len` calls of enqueue_step.
hipError_t enqueue_window(pic_ctx *c, hipStream_t s, int64_t n0, int len, bool &ready)
{
    const Dev &d = c->d;
    const bool f64 = c->P.f64;
    const bool coll = c->cfg.collisions != 0;
    hipError_t e;
    if (!coll || !births_fit_solve(d)) {
        for (int i = 0; i < len; ++i)
            if ((e = enqueue_step(c, s, n0 + i, ready, false)) != hipSuccess) return e;
        return hipSuccess;
    }
    const int K = c->sort_every;
    const int stages = SB_PUSH | SB_COLLIDE | SB_DEPOSIT;
    const bool piped = !f64 && K >= 2;
    bool pending = false;  // births of the previous step not placed yet
    for (int i = 0; i < len; ++i) {
        const int64_t n = n0 + i;
        const bool sort_now = (n + 1) % K == 0;
        const bool sorting = piped && sort_now && ready;
        const bool prep = piped && (n + 2) % K == 0;
        const int hist = (prep || (sort_now && !sorting)) ? 1 : 0;
        if ((e = launch_solve(d, f64, c->P.chunks_tot, true, s, pending, true)) != hipSuccess) return e;
        if (sorting)
            e = launch_pass32_sort(d, c->L.ppt, c->L.window, s, true, d.cap_tot, c->L.nt != 0);
        else
            e = launch_particles(d, c->L, s, f64, stages, hist, false);
        if (e != hipSuccess) return e;
        if ((e = launch_after_pass(c, s, hist)) != hipSuccess) return e;
        if (sort_now && !sorting) {
            if ((e = launch_births(d, f64, true, true, s)) != hipSuccess) return e;
            if ((e = launch_sort(d, f64, c->L, s)) != hipSuccess) return e;
            pending = false;
        } else {
            pending = true;
        }
        if (prep && !sort_now) {
            if ((e = launch_sort_prepare(d, s)) != hipSuccess) return e;
            ready = true;
        } else {
            ready = false;
        }
    }
    if (pending && (e = launch_births(d, f64, true, true, s)) != hipSuccess) return e;
    return hipSuccess;
}

// The prepared-sort state a window starting at step count n needs: in steady state the
// step before a sort step has prepared it (FP32 form, K >= 2).
bool ready_expected(const pic_ctx *c, int64_t n)
{
    const int K = c->sort_every;
    return !c->P.f64 && K >= 2 && (n + 1) % K == 0;
}

// The prepared-sort state after step n (the same after an eager step and a window).
bool ready_after(const pic_ctx *c, int64_t n)
{
    const int K = c->sort_every;
    return !c->P.f64 && K >= 2 && (n + 2) % K == 0;
}

int64_t window_key(const pic_ctx *c, int64_t n, int len)
{
    return (n % c->sort_every) * (int64_t)(c->sort_every + 1) + len;
}

void drop_graphs(pic_ctx *c)
{
    for (auto &kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

// Capture and instantiate the window of `len` steps starting at step count n (if absent).
int build_window_graph(pic_ctx *c, int64_t n, int len, hipGraphExec_t *out)
{
    const int64_t key = window_key(c, n, len);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return PIC_OK;
    }
    if (!c->cap_stream) HIPC(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPC(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    bool ready = ready_expected(c, n);
    hipError_t e = enqueue_window(c, c->cap_stream, n, len, ready);
    hipError_t e2 = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hipfail(c, e, "graph capture");
    }
    if (e2 != hipSuccess) return hipfail(c, e2, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hipfail(c, e, "hipGraphInstantiate");
    c->graphs[key] = x;
    *out = x;
    return PIC_OK;
}

// The windows pic_step(nsteps) replays from the current state: whole sort cycles, then a
// shorter tail that replays only if it was prepared (graph_tail).  A window is used only
// when the prepared-sort state is the one its first phase expects.
template <typename F>
int plan_windows(pic_ctx *c, int64_t nsteps, bool graph_tail, F &&visit)
{
    int64_t n = c->host_step;
    bool ready = c->sort_ready;
    const int K = c->sort_every;
    while (nsteps > 0) {
        const int len = (int)std::min<int64_t>(nsteps, K);
        const bool ok = c->cfg.fused && !c->timing && ready == ready_expected(c, n) &&
                        (len == K || graph_tail || c->graphs.count(window_key(c, n, len)));
        int rc = visit(n, ok ? len : 1, ok);
        if (rc) return rc;
        const int adv = ok ? len : 1;
        // the prepared-sort state after the window or the eager step, whatever it was on
        // entry: set by a step before a sort step (FP32, K >= 2)
        ready = ready_after(c, n + adv - 1);
        n += adv;
        nsteps -= adv;
    }
    return PIC_OK;
}

Launch default_launch(const pic_config *cfg, const Plan &P)
{
    Launch L;
    L.block = cfg->block > 0 ? cfg->block : 256;
    L.ppt = 4;  // particles per thread of the FP32 pass (4 or 8; the autotuner may change it)
    if (cfg->precision == PIC_FP32_CELLOFF && (cfg->ppt == 4 || cfg->ppt == 8)) L.ppt = cfg->ppt;
    L.sort_ppt = (cfg->sort_ppt == 4 || cfg->sort_ppt == 8) ? cfg->sort_ppt : 4;
    L.nt = (cfg->nontemporal & 1) ? 1 : 0;
    L.sort_nt = (cfg->nontemporal & 2) ? 1 : 0;
    int64_t tiles = 0;
    for (const SegC &S : P.seg) tiles += (S.cap + (int64_t)L.block * L.ppt - 1) / ((int64_t)L.block * L.ppt);
    int g = cfg->grid > 0 ? cfg->grid : 1024;
    g = (int)std::min<int64_t>(g, std::max<int64_t>(8, (tiles + 7) / 8 * 8));
    L.grid = std::max(8, g / 8 * 8);
    L.window = cfg->window > 0 ? cfg->window : 2048;
    return L;
}

}  // namespace

// =======================================================================================
extern "C" {

int pic_query_workspace(const pic_config *cfg, size_t *bytes)
{
    Plan P;
    std::string m;
    int rc = build_plan(cfg, P, m);
    if (rc) return rc;
    Dev d;
    *bytes = carve(P, nullptr, d);
    return PIC_OK;
}

int pic_init(const pic_config *cfg, void *workspace, size_t bytes, void *stream, pic_ctx **out)
{
    if (!out) return PIC_EINVAL;
    *out = nullptr;
    pic_ctx *c = new pic_ctx();
    int rc = build_plan(cfg, c->P, c->msg);
    if (rc) {
        fprintf(stderr, "pic_init: %s\n", c->msg.c_str());
        delete c;
        return rc;
    }
    c->cfg = *cfg;
    c->ens.assign(cfg->ens, cfg->ens + cfg->n_ensembles);
    c->cfg.ens = c->ens.data();
    const size_t need = carve(c->P, nullptr, c->d);
    if (!workspace || bytes < need) {
        fprintf(stderr, "pic_init: workspace too small (%zu < %zu)\n", bytes, need);
        delete c;
        return PIC_EINVAL;
    }
    c->ws = (char *)workspace;
    c->ws_bytes = bytes;
    carve(c->P, c->ws, c->d);
    c->d.periodic = cfg->boundary == PIC_PERIODIC;
    c->d.collisions = cfg->collisions;
    for (int e = 0; e < cfg->n_ensembles; ++e)
        if (cfg->ens[e].cx_relative) c->d.any_cx_rel = 1;
    c->diag_scratch = (double *)(c->ws + need - align_up(2 * kDiagGrid * sizeof(double)));
    c->L = default_launch(cfg, c->P);
    c->sort_every = cfg->sort_every > 0 ? cfg->sort_every : kCompactEvery;
    hipStream_t s = (hipStream_t)stream;
    Dev &d = c->d;
    auto done = [&](int code) {
        if (code != PIC_OK) {
            fprintf(stderr, "pic_init: %s\n", c->msg.c_str());
            delete c;
            return code;
        }
        *out = c;
        return PIC_OK;
    };
    hipError_t e;
#define IHIP(expr)                                              \
    if ((e = (expr)) != hipSuccess) return done(hipfail(c, e, #expr));
    IHIP(static_scratch_address(&c->static_scratch));
    IHIP(hipMemsetAsync(c->ws, 0, need, s));
    IHIP(hipMemcpyAsync((void *)d.seg, c->P.seg.data(), c->P.seg.size() * sizeof(SegC), hipMemcpyHostToDevice, s));
    IHIP(hipMemcpyAsync((void *)d.ens, c->P.ens.data(), c->P.ens.size() * sizeof(EnsC), hipMemcpyHostToDevice, s));
    std::vector<int64_t> nslots(c->P.nseg);
    std::vector<uint32_t> nid(c->P.nseg);
    for (int sg = 0; sg < c->P.nseg; ++sg) {
        const SegC &S = c->P.seg[sg];
        const pic_ensemble_desc &D = cfg->ens[S.ens];
        const pic_species_desc &sp = D.sp[S.species];
        const int64_t n = sp.ppc * D.ncells;
        nslots[sg] = n;
        nid[sg] = (uint32_t)n;
        const double vth = std::sqrt(sp.T / sp.m);
        IHIP(launch_init(d, c->P.f64, sg, n, sp.ppc, D.init_mode, vth, D.perturb_amp, D.perturb_mode, s));
    }
    IHIP(hipMemcpyAsync(d.n_slots, nslots.data(), nslots.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
    IHIP(hipMemcpyAsync(d.next_id, nid.data(), nid.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    IHIP(launch_vmax(d, c->P.f64, s));
    IHIP(launch_zero_q(d, c->P.f64, s));
    IHIP(launch_particles(d, c->L, s, c->P.f64, SB_DEPOSIT, 0));
    IHIP(hipStreamSynchronize(s));
#undef IHIP
    return done(PIC_OK);
}

int pic_deposit(pic_ctx *c, void *stream)
{
    if (!c) return PIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIPC(c, launch_zero_q(c->d, c->P.f64, s));
    HIPC(c, launch_particles(c->d, c->L, s, c->P.f64, SB_DEPOSIT, 0));
    return PIC_OK;
}

int pic_solve(pic_ctx *c, void *stream)
{
    if (!c) return PIC_EINVAL;
    HIPC(c, launch_solve(c->d, c->P.f64, c->P.chunks_tot, false, (hipStream_t)stream));
    return PIC_OK;
}

int pic_push(pic_ctx *c, void *stream)
{
    if (!c) return PIC_EINVAL;
    c->insitu = false;
    c->sort_ready = false;  // particles or the step count change: no prepared sort
    HIPC(c, launch_particles(c->d, c->L, (hipStream_t)stream, c->P.f64, SB_PUSH, 0));
    HIPC(c, launch_neutrals(c->d, (hipStream_t)stream));
    return PIC_OK;
}

int pic_collide(pic_ctx *c, void *stream)
{
    if (!c) return PIC_EINVAL;
    c->insitu = false;
    c->sort_ready = false;  // particles or the step count change: no prepared sort
    hipStream_t s = (hipStream_t)stream;
    if (c->cfg.collisions) {
        HIPC(c, launch_particles(c->d, c->L, s, c->P.f64, SB_COLLIDE, 0));
        HIPC(c, launch_candidates(c->d, c->L, s, c->P.f64, 0));
    }
    HIPC(c, launch_source(c->d, 0, s));
    if (c->cfg.collisions) HIPC(c, launch_births(c->d, c->P.f64, false, false, s));
    return PIC_OK;
}

int pic_sort(pic_ctx *c, void *stream)
{
    if (!c) return PIC_EINVAL;
    c->insitu = false;
    c->sort_ready = false;  // particles or the step count change: no prepared sort
    hipStream_t s = (hipStream_t)stream;
    HIPC(c, launch_particles(c->d, c->L, s, c->P.f64, SB_HIST, 0));
    HIPC(c, launch_sort(c->d, c->P.f64, c->L, s));
    return PIC_OK;
}

int pic_step(pic_ctx *c, int32_t nsteps, void *stream)
{
    if (!c || nsteps < 0) return PIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = plan_windows(c, nsteps, false, [&](int64_t n, int len, bool graph) -> int {
        if (graph) {
            hipGraphExec_t x = nullptr;
            int r = build_window_graph(c, n, len, &x);
            if (r) return r;
            HIPC(c, hipGraphLaunch(x, s));
            c->graph_launches += 1;
            c->sort_ready = ready_after(c, n + len - 1);
        } else {
            HIPC(c, enqueue_step(c, s, n, c->sort_ready, false));
        }
        c->host_step = n + len;
        return PIC_OK;
    });
    if (rc) return rc;
    if (nsteps > 0) c->insitu = c->cfg.fused && !c->P.f64 && c->cfg.collisions;
    return check_err(c, s);
}

int pic_graph_prepare(pic_ctx *c, int32_t nsteps)
{
    if (!c || nsteps < 0) return PIC_EINVAL;
    if (!c->cfg.fused) return PIC_OK;
    return plan_windows(c, nsteps, true, [&](int64_t n, int len, bool graph) -> int {
        if (!graph) return PIC_OK;
        hipGraphExec_t x = nullptr;
        return build_window_graph(c, n, len, &x);
    });
}

int pic_graph_launches(const pic_ctx *c, int64_t *launches)
{
    if (!c || !launches) return PIC_EINVAL;
    *launches = c->graph_launches;
    return PIC_OK;
}

int pic_set_step(pic_ctx *c, int64_t step)
{
    if (!c || step < 0) return PIC_EINVAL;
    c->sort_ready = false;  // particles or the step count change: no prepared sort
    // both birth halves clean, whatever parity the new step has
    HIPC(c, launch_births_clear_all(c->d, nullptr));
    HIPC(c, hipDeviceSynchronize());
    HIPC(c, hipMemcpy(c->d.step, &step, sizeof(step), hipMemcpyHostToDevice));
    c->host_step = step;
    return PIC_OK;
}

int64_t pic_nnodes(const pic_ctx *c, int32_t ens)
{
    if (!c || ens < 0 || ens >= c->P.nens) return PIC_EINVAL;
    return c->P.ens[ens].nnodes;
}

int pic_diag(pic_ctx *c, int32_t ens, pic_diag_out *out, double *moments_dev, void *stream)
{
    if (!c || !out || ens < 0 || ens >= c->P.nens) return PIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    if (moments_dev) {
        const EnsC &Em = c->P.ens[ens];
        for (int sp = 0; sp < c->P.nspecies; ++sp)
            HIPC(c, launch_moments(c->d, c->P.f64, Em.seg[sp], Em.nnodes, moments_dev + (int64_t)sp * 5 * Em.nnodes, s));
    }
    const int nseg = c->P.nseg;
    std::vector<unsigned long long> cnt((size_t)kCntStripes * nseg * C_NCNT);
    std::vector<double> sums((size_t)kCntStripes * nseg * S_NSUM);
    HIPC(c, hipMemcpyAsync(cnt.data(), c->d.cnt, cnt.size() * 8, hipMemcpyDeviceToHost, s));
    HIPC(c, hipMemcpyAsync(sums.data(), c->d.sums, sums.size() * 8, hipMemcpyDeviceToHost, s));
    double emax = 0, fe = 0;
    std::vector<double> numax(nseg);
    int64_t step = 0;
    if (!c->insitu) {
        HIPC(c, launch_field_energy(c->d, s));
        HIPC(c, hipMemcpyAsync(&fe, c->d.fe + ens, 8, hipMemcpyDeviceToHost, s));
    }
    HIPC(c, hipMemcpyAsync(&emax, c->d.emax + ens, 8, hipMemcpyDeviceToHost, s));
    HIPC(c, hipMemcpyAsync(numax.data(), c->d.numax, nseg * 8, hipMemcpyDeviceToHost, s));
    HIPC(c, hipMemcpyAsync(&step, c->d.step, 8, hipMemcpyDeviceToHost, s));
    memset(out, 0, sizeof(*out));
    const EnsC &E = c->P.ens[ens];
    std::vector<double> part(2 * kDiagGrid);
    // the fused step's own tallies of its last step (count, sum |v|^2 and the solve's field
    // energy), when no call has changed particles or fields since
    std::vector<double> tal;
    if (c->insitu) {
        int32_t vc = 0;
        HIPC(c, hipMemcpyAsync(&vc, c->d.vcur, 4, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
        const size_t per = (size_t)kCntStripes * nseg * T_NSTEP;
        tal.resize(per);
        HIPC(c, hipMemcpyAsync(tal.data(), c->d.ssum + (size_t)vc * per, per * 8, hipMemcpyDeviceToHost, s));
        std::vector<double> pp((size_t)E.nchunks * P_NPART);
        HIPC(c, hipMemcpyAsync(pp.data(), c->d.part + E.chunk0 * P_NPART, pp.size() * 8, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
        double f = 0.0;
        for (int64_t k = 0; k < E.nchunks; ++k) f += pp[(size_t)k * P_NPART + P_FE];
        fe = f;
    }
    for (int sp = 0; sp < c->P.nspecies; ++sp) {
        const int sg = E.seg[sp];
        double n = 0, v2 = 0;
        if (c->insitu) {
            for (int st = 0; st < kCntStripes; ++st) {
                n += tal[((size_t)st * nseg + sg) * T_NSTEP + T_N];
                v2 += tal[((size_t)st * nseg + sg) * T_NSTEP + T_V2];
            }
        } else {
            HIPC(c, launch_diag(c->d, c->P.f64, sg, c->diag_scratch, kDiagGrid, s));
            HIPC(c, hipMemcpyAsync(part.data(), c->diag_scratch, part.size() * 8, hipMemcpyDeviceToHost, s));
            HIPC(c, hipStreamSynchronize(s));
            for (int i = 0; i < kDiagGrid; ++i) {
                n += part[2 * i];
                v2 += part[2 * i + 1];
            }
        }
        const pic_species_desc &D = c->ens[ens].sp[sp];
        out->count[sp] = (int64_t)n;
        out->ke[sp] = 0.5 * D.m * D.w * v2;
        out->charge += D.q * D.w * n;
        unsigned long long a[C_NCNT] = {0};
        double kl = 0, kr = 0;
        for (int st = 0; st < kCntStripes; ++st) {
            for (int k = 0; k < C_NCNT; ++k) a[k] += cnt[((size_t)st * nseg + sg) * C_NCNT + k];
            kl += sums[((size_t)st * nseg + sg) * S_NSUM + S_KE_L];
            kr += sums[((size_t)st * nseg + sg) * S_NSUM + S_KE_R];
        }
        out->wall_count[0][sp] = (int64_t)a[C_WALL_L];
        out->wall_count[1][sp] = (int64_t)a[C_WALL_R];
        out->wall_charge[0][sp] = D.q * D.w * (double)a[C_WALL_L];
        out->wall_charge[1][sp] = D.q * D.w * (double)a[C_WALL_R];
        out->wall_ke[0][sp] = kl;
        out->wall_ke[1][sp] = kr;
        out->created[sp] = (int64_t)a[C_CREATED];
        out->pushes += (int64_t)a[C_PUSH];
        if (sp == 0) {
            out->coll[0] = (int64_t)a[C_EL];
            out->coll[1] = (int64_t)a[C_IZ];
            out->sourced = (int64_t)a[C_SOURCED];
        } else {
            out->coll[2] = (int64_t)a[C_CX];
            out->recycled = (int64_t)a[C_RECYCLED];
            out->neutral_wall[0] = (int64_t)a[C_NWALL_L];
            out->neutral_wall[1] = (int64_t)a[C_NWALL_R];
        }
        out->numax[sp] = numax[sg];
    }
    if (E.recycle) {
        int32_t nc = 0;
        unsigned long long nn = 0;
        HIPC(c, hipMemcpyAsync(&nc, c->d.ncur, 4, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
        HIPC(c, hipMemcpyAsync(&nn, c->d.nneu + (int64_t)nc * c->P.nens + ens, 8, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
        out->neutral_count = std::min<int64_t>((int64_t)nn, E.ncap);
    }
    out->field_energy = fe;
    out->emax = emax;
    out->step = step;
    return check_err(c, s);
}

namespace {
// The recycled neutral set of an ensemble (species index 2): current buffer and count.
int neutral_state(pic_ctx *c, int32_t ens, hipStream_t s, int32_t &b, int64_t &n)
{
    unsigned long long nn = 0;
    HIPC(c, hipMemcpyAsync(&b, c->d.ncur, 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    HIPC(c, hipMemcpyAsync(&nn, c->d.nneu + (int64_t)b * c->P.nens + ens, 8, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    n = std::min<int64_t>((int64_t)nn, c->P.ens[ens].ncap);
    return PIC_OK;
}

int get_neutrals(pic_ctx *c, int32_t ens, pic_particles out, int64_t cap, int64_t *count, hipStream_t s)
{
    const EnsC &E = c->P.ens[ens];
    int32_t b = 0;
    int64_t n = 0;
    int rc = neutral_state(c, ens, s, b, n);
    if (rc) return rc;
    if (n > cap) return fail(c, PIC_EINVAL, "output capacity too small");
    std::vector<int32_t> cell(n);
    std::vector<float> off(n), vx(n), vy(n), vz(n);
    const Dev &d = c->d;
    if (n) {
        HIPC(c, hipMemcpy(cell.data(), d.ncell[b] + E.nbase, n * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(off.data(), d.noff[b] + E.nbase, n * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vx.data(), d.nvx[b] + E.nbase, n * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vy.data(), d.nvy[b] + E.nbase, n * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vz.data(), d.nvz[b] + E.nbase, n * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(out.id, d.nid[b] + E.nbase, n * 4, hipMemcpyDeviceToHost));
    }
    for (int64_t i = 0; i < n; ++i) {
        out.x[i] = ((double)cell[i] + (double)off[i]) * E.dx;
        out.vx[i] = vx[i];
        out.vy[i] = vy[i];
        out.vz[i] = vz[i];
    }
    *count = n;
    return PIC_OK;
}

int set_neutrals(pic_ctx *c, int32_t ens, pic_particles in, int64_t count, hipStream_t s)
{
    const EnsC &E = c->P.ens[ens];
    if (count < 0 || count > E.ncap) return fail(c, PIC_EINVAL, "count above the neutral capacity");
    std::vector<int32_t> cell(count);
    std::vector<float> off(count), vx(count), vy(count), vz(count);
    for (int64_t i = 0; i < count; ++i) {
        if (!(in.x[i] >= 0.0 && in.x[i] < E.L)) return fail(c, PIC_EINVAL, "x outside [0, L)");
        const double g = in.x[i] / E.dx;
        const double jf = std::floor(g);
        int cl = (int)jf;
        float o = (float)(g - jf);
        if (o >= 1.0f) {
            o = 0.0f;
            cl += 1;
        }
        if (cl >= E.ncells) {  // x / dx rounded up to N: the last cell, as the device converts
            cl = (int)E.ncells - 1;
            o = 0x1.fffffep-1f;
        }
        cell[i] = cl;
        off[i] = o;
        vx[i] = (float)in.vx[i];
        vy[i] = (float)in.vy[i];
        vz[i] = (float)in.vz[i];
    }
    int32_t b = 0;
    int64_t n = 0;
    int rc = neutral_state(c, ens, s, b, n);
    if (rc) return rc;
    const Dev &d = c->d;
    if (count) {
        HIPC(c, hipMemcpy(d.ncell[b] + E.nbase, cell.data(), count * 4, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(d.noff[b] + E.nbase, off.data(), count * 4, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(d.nvx[b] + E.nbase, vx.data(), count * 4, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(d.nvy[b] + E.nbase, vy.data(), count * 4, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(d.nvz[b] + E.nbase, vz.data(), count * 4, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(d.nid[b] + E.nbase, in.id, count * 4, hipMemcpyHostToDevice));
    }
    const unsigned long long nn = (unsigned long long)count;
    HIPC(c, hipMemcpy(d.nneu + (int64_t)b * c->P.nens + ens, &nn, 8, hipMemcpyHostToDevice));
    return PIC_OK;
}
}  // namespace

int pic_get_particles(pic_ctx *c, int32_t ens, int32_t species, pic_particles out, int64_t cap,
                      int64_t *count, void *stream)
{
    if (c && count && ens >= 0 && ens < c->P.nens && species == 2 && c->P.ens[ens].recycle)
        return get_neutrals(c, ens, out, cap, count, (hipStream_t)stream);
    if (!c || !count || ens < 0 || ens >= c->P.nens || species < 0 || species >= c->P.nspecies)
        return fail(c, PIC_EINVAL, "bad ensemble/species");
    hipStream_t s = (hipStream_t)stream;
    const int sg = c->P.ens[ens].seg[species];
    const SegC &S = c->P.seg[sg];
    int64_t n = 0;
    int32_t b = 0;
    HIPC(c, hipMemcpyAsync(&n, c->d.n_slots + sg, 8, hipMemcpyDeviceToHost, s));
    HIPC(c, hipMemcpyAsync(&b, c->d.cur, 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    std::vector<uint32_t> id(n);
    HIPC(c, hipMemcpy(id.data(), c->d.id[b] + S.base, n * 4, hipMemcpyDeviceToHost));
    int64_t k = 0;
    if (c->P.f64) {
        std::vector<double> x(n), vx(n), vy(n), vz(n);
        HIPC(c, hipMemcpy(x.data(), c->d.x[b] + S.base, n * 8, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vx.data(), c->d.dvx[b] + S.base, n * 8, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vy.data(), c->d.dvy[b] + S.base, n * 8, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vz.data(), c->d.dvz[b] + S.base, n * 8, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            if (!(x[i] >= 0.0)) continue;
            if (k >= cap) return fail(c, PIC_EINVAL, "output capacity too small");
            out.x[k] = x[i];
            out.vx[k] = vx[i];
            out.vy[k] = vy[i];
            out.vz[k] = vz[i];
            out.id[k] = id[i];
            ++k;
        }
    } else {
        std::vector<int32_t> cell(n);
        std::vector<float> off(n), vx(n), vy(n), vz(n);
        HIPC(c, hipMemcpy(cell.data(), c->d.cell[b] + S.base, n * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(off.data(), c->d.off[b] + S.base, n * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vx.data(), c->d.fvx[b] + S.base, n * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vy.data(), c->d.fvy[b] + S.base, n * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vz.data(), c->d.fvz[b] + S.base, n * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            if (cell[i] == kDead) continue;
            if (k >= cap) return fail(c, PIC_EINVAL, "output capacity too small");
            out.x[k] = ((double)cell[i] + (double)off[i]) * S.dx;
            out.vx[k] = vx[i];
            out.vy[k] = vy[i];
            out.vz[k] = vz[i];
            out.id[k] = id[i];
            ++k;
        }
    }
    *count = k;
    return PIC_OK;
}

int pic_get_slots(pic_ctx *c, int32_t ens, int32_t species, int64_t first, int64_t count,
                  pic_particles out, void *stream)
{
    if (!c || ens < 0 || ens >= c->P.nens || species < 0 || species >= c->P.nspecies || first < 0 ||
        count < 0)
        return fail(c, PIC_EINVAL, "bad ensemble/species/range");
    const int sg = c->P.ens[ens].seg[species];
    const SegC &S = c->P.seg[sg];
    if (first + count > S.cap) return fail(c, PIC_EINVAL, "slot range beyond capacity");
    hipStream_t s = (hipStream_t)stream;
    int32_t b = 0;
    HIPC(c, hipMemcpyAsync(&b, c->d.cur, 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    const int64_t i0 = S.base + first;
    HIPC(c, hipMemcpy(out.id, c->d.id[b] + i0, count * 4, hipMemcpyDeviceToHost));
    if (c->P.f64) {
        HIPC(c, hipMemcpy(out.x, c->d.x[b] + i0, count * 8, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(out.vx, c->d.dvx[b] + i0, count * 8, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(out.vy, c->d.dvy[b] + i0, count * 8, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(out.vz, c->d.dvz[b] + i0, count * 8, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < count; ++i)
            if (!(out.x[i] >= 0.0)) out.x[i] = -1.0;
    } else {
        std::vector<int32_t> cell(count);
        std::vector<float> off(count), vx(count), vy(count), vz(count);
        HIPC(c, hipMemcpy(cell.data(), c->d.cell[b] + i0, count * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(off.data(), c->d.off[b] + i0, count * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vx.data(), c->d.fvx[b] + i0, count * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vy.data(), c->d.fvy[b] + i0, count * 4, hipMemcpyDeviceToHost));
        HIPC(c, hipMemcpy(vz.data(), c->d.fvz[b] + i0, count * 4, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < count; ++i) {
            out.x[i] = (cell[i] == kDead) ? -1.0 : ((double)cell[i] + (double)off[i]) * S.dx;
            out.vx[i] = vx[i];
            out.vy[i] = vy[i];
            out.vz[i] = vz[i];
        }
    }
    return PIC_OK;
}

int pic_set_particles(pic_ctx *c, int32_t ens, int32_t species, pic_particles in, int64_t count,
                      uint32_t next_id, void *stream)
{
    if (c && ens >= 0 && ens < c->P.nens && species == 2 && c->P.ens[ens].recycle)
        return set_neutrals(c, ens, in, count, (hipStream_t)stream);
    if (!c || ens < 0 || ens >= c->P.nens || species < 0 || species >= c->P.nspecies || count < 0)
        return fail(c, PIC_EINVAL, "bad ensemble/species/count");
    c->sort_ready = false;  // particles or the step count change: no prepared sort
    c->insitu = false;
    const int sg = c->P.ens[ens].seg[species];
    const SegC &S = c->P.seg[sg];
    if (count > S.cap) return fail(c, PIC_EINVAL, "count above capacity");
    const double L = c->P.ens[ens].L;
    const int64_t idcap = c->P.ens[ens].idcap;
    if ((int64_t)next_id > idcap) return fail(c, PIC_EINVAL, "next_id above the id capacity");
    for (int64_t i = 0; i < count; ++i) {
        if (!(in.x[i] >= 0.0 && in.x[i] < L)) return fail(c, PIC_EINVAL, "x outside [0, L)");
        if ((int64_t)in.id[i] >= idcap) return fail(c, PIC_EINVAL, "id above the id capacity");
        if (!std::isfinite(in.vx[i]) || !std::isfinite(in.vy[i]) || !std::isfinite(in.vz[i]))
            return fail(c, PIC_EINVAL, "non-finite velocity");
    }
    hipStream_t s = (hipStream_t)stream;
    int32_t b = 0;
    HIPC(c, hipMemcpyAsync(&b, c->d.cur, 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    HIPC(c, hipMemcpy(c->d.id[b] + S.base, in.id, count * 4, hipMemcpyHostToDevice));
    if (c->P.f64) {
        HIPC(c, hipMemcpy(c->d.x[b] + S.base, in.x, count * 8, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(c->d.dvx[b] + S.base, in.vx, count * 8, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(c->d.dvy[b] + S.base, in.vy, count * 8, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(c->d.dvz[b] + S.base, in.vz, count * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<int32_t> cell(count);
        std::vector<float> off(count), vx(count), vy(count), vz(count);
        for (int64_t i = 0; i < count; ++i) {
            const double g = in.x[i] / S.dx;
            const double jf = std::floor(g);
            int cl = (int)jf;
            float o = (float)(g - jf);
            if (o >= 1.0f) {
                o = 0.0f;
                cl += 1;
            }
            if (cl >= S.ncells) {  // x / dx rounded up to N: the last cell, as the device converts
                cl = S.ncells - 1;
                o = 0x1.fffffep-1f;
            }
            cell[i] = cl;
            off[i] = o;
            vx[i] = (float)in.vx[i];
            vy[i] = (float)in.vy[i];
            vz[i] = (float)in.vz[i];
        }
        HIPC(c, hipMemcpy(c->d.cell[b] + S.base, cell.data(), count * 4, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(c->d.off[b] + S.base, off.data(), count * 4, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(c->d.fvx[b] + S.base, vx.data(), count * 4, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(c->d.fvy[b] + S.base, vy.data(), count * 4, hipMemcpyHostToDevice));
        HIPC(c, hipMemcpy(c->d.fvz[b] + S.base, vz.data(), count * 4, hipMemcpyHostToDevice));
    }
    HIPC(c, hipMemcpy(c->d.n_slots + sg, &count, 8, hipMemcpyHostToDevice));
    HIPC(c, hipMemcpy(c->d.next_id + sg, &next_id, 4, hipMemcpyHostToDevice));
    // the speed maxima of the current half are recomputed for every segment
    int32_t vc = 0;
    HIPC(c, hipMemcpy(&vc, c->d.vcur, 4, hipMemcpyDeviceToHost));
    HIPC(c, hipMemset(c->d.vmax2 + (size_t)vc * kCntStripes * c->P.nseg, 0, (size_t)kCntStripes * c->P.nseg * 8));
    HIPC(c, launch_vmax(c->d, c->P.f64, s));
    HIPC(c, hipStreamSynchronize(s));
    return PIC_OK;
}

int pic_get_grid(pic_ctx *c, int32_t ens, double *Q0, double *Q1, double *rho, double *phi,
                 double *E, void *stream)
{
    if (!c || ens < 0 || ens >= c->P.nens) return PIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    HIPC(c, hipStreamSynchronize(s));
    const EnsC &En = c->P.ens[ens];
    const int64_t nn = En.nnodes;
    double *Qs[2] = {Q0, Q1};
    for (int sp = 0; sp < 2; ++sp) {
        if (!Qs[sp]) continue;
        if (sp >= c->P.nspecies) {
            std::fill(Qs[sp], Qs[sp] + nn, 0.0);
            continue;
        }
        if (c->P.f64) {
            HIPC(c, hipMemcpy(Qs[sp], c->d.Qd + sp * c->P.nodes_tot + En.gbase, nn * 8, hipMemcpyDeviceToHost));
        } else {
            std::vector<long long> q(nn);
            HIPC(c, hipMemcpy(q.data(), c->d.Qi + sp * c->P.nodes_tot + En.gbase, nn * 8, hipMemcpyDeviceToHost));
            for (int64_t j = 0; j < nn; ++j) Qs[sp][j] = (double)q[j] / kFix;
        }
    }
    if (rho) HIPC(c, hipMemcpy(rho, c->d.rho + En.gbase, nn * 8, hipMemcpyDeviceToHost));
    if (phi) HIPC(c, hipMemcpy(phi, c->d.phi + En.gbase, nn * 8, hipMemcpyDeviceToHost));
    if (E) HIPC(c, hipMemcpy(E, c->d.E + En.gbase, nn * 8, hipMemcpyDeviceToHost));
    return PIC_OK;
}

int pic_get_gather_table(pic_ctx *c, int32_t ens, float *out, void *stream)
{
    if (!c || !out || ens < 0 || ens >= c->P.nens) return PIC_EINVAL;
    if (c->P.f64) return fail(c, PIC_EINVAL, "the FP64 form has no gather table");
    hipStream_t s = (hipStream_t)stream;
    HIPC(c, hipStreamSynchronize(s));
    const EnsC &En = c->P.ens[ens];
    HIPC(c, hipMemcpy(out, c->d.Ecell + En.gbase, En.ncells * sizeof(float2), hipMemcpyDeviceToHost));
    return PIC_OK;
}

int pic_set_fields(pic_ctx *c, int32_t ens, const double *E, void *stream)
{
    if (!c || !E || ens < 0 || ens >= c->P.nens) return PIC_EINVAL;
    c->insitu = false;
    hipStream_t s = (hipStream_t)stream;
    HIPC(c, hipStreamSynchronize(s));
    const EnsC &En = c->P.ens[ens];
    HIPC(c, hipMemcpy(c->d.E + En.gbase, E, En.nnodes * 8, hipMemcpyHostToDevice));
    HIPC(c, launch_field_stats(c->d, c->P.f64, c->P.chunks_tot, s));
    HIPC(c, hipStreamSynchronize(s));
    return PIC_OK;
}

int pic_set_external_field(pic_ctx *c, int32_t ens, double E_ext)
{
    if (!c || ens < 0 || ens >= c->P.nens || !std::isfinite(E_ext)) return PIC_EINVAL;
    c->P.ens[ens].E_ext = E_ext;
    c->ens[ens].E_ext = E_ext;
    HIPC(c, hipMemcpy((void *)(c->d.ens + ens), &c->P.ens[ens], sizeof(EnsC), hipMemcpyHostToDevice));
    return PIC_OK;
}

namespace {

struct AdjLayout {
    int64_t n, nn, nseg_ck, K;
    size_t off_ck_cell, off_ck_off, off_ck_vx, off_xc, off_xo, off_E, off_lx, off_lv, off_lE, off_lQ,
        off_tmp, off_ext, off_fin, bytes;
};

// PIC_OK when the run is one the adjoint is defined for; otherwise *why says what is not.
int adj_check(pic_ctx *c, const char **why)
{
    if (c->P.nens != 1 || c->P.nspecies != 1) *why = "adjoint needs one ensemble and one species";
    else if (!c->d.periodic) *why = "adjoint needs a periodic domain";
    else if (c->cfg.collisions) *why = "adjoint needs a collisionless run";
    else if (c->cfg.smooth) *why = "adjoint is defined without density smoothing";
    else if (c->P.f64) *why = "adjoint is defined on the FP32 form";
    else {
        const SegC &S = c->P.seg[0];
        if (S.t[0] != 0.0 || S.t[1] != 0.0 || S.t[2] != 0.0) *why = "adjoint needs B = 0";
        else return PIC_OK;
    }
    return PIC_EINVAL;
}

AdjLayout adj_layout(pic_ctx *c, int nsteps, int K)
{
    AdjLayout A{};
    A.n = c->P.seg[0].cap;
    A.nn = c->P.ens[0].nnodes;
    A.K = K;
    A.nseg_ck = (nsteps + K - 1) / K;
    size_t o = 0;
    auto take = [&](size_t b) {
        size_t r = o;
        o += align_up(std::max<size_t>(b, 1));
        return r;
    };
    A.off_ck_cell = take((size_t)A.nseg_ck * A.n * 4);
    A.off_ck_off = take((size_t)A.nseg_ck * A.n * 4);
    A.off_ck_vx = take((size_t)A.nseg_ck * A.n * 4);
    A.off_xc = take((size_t)K * A.n * 4);
    A.off_xo = take((size_t)K * A.n * 4);
    A.off_E = take((size_t)K * A.nn * 8);
    A.off_lx = take((size_t)A.n * 8);
    A.off_lv = take((size_t)A.n * 8);
    A.off_lE = take((size_t)A.nn * 8);
    A.off_lQ = take((size_t)A.nn * 8);
    A.off_tmp = take((size_t)A.nn * 8);
    A.off_ext = take(64);
    A.off_fin = take((size_t)A.n * 4 * 5);  // final state: cell, off, vx, vy, vz
    A.bytes = o;
    return A;
}

// One forward step of the window (no sort, no collisions); optionally records x^n and E^n.
hipError_t adj_forward_step(pic_ctx *c, hipStream_t s, int32_t *xc, float *xo, double *E)
{
    const Dev &d = c->d;
    const int64_t n = c->P.seg[0].cap;
    hipError_t e;
    if (xc) {
        if ((e = hipMemcpyAsync(xc, d.cell[0], n * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(xo, d.off[0], n * 4, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    }
    if ((e = launch_solve(d, false, c->P.chunks_tot, true, s)) != hipSuccess) return e;
    if (E && (e = hipMemcpyAsync(E, d.E, c->P.ens[0].nnodes * 8, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return e;
    if ((e = launch_particles(d, c->L, s, false, SB_PUSH | SB_DEPOSIT, 0)) != hipSuccess) return e;
    return launch_advance(d, s);
}

}  // namespace

int pic_adjoint_query(pic_ctx *c, int32_t nsteps, int32_t ckpt_every, size_t *bytes)
{
    if (!c || !bytes || nsteps < 1 || ckpt_every < 1) return PIC_EINVAL;
    const char *why = "";
    if (adj_check(c, &why)) return fail(c, PIC_EINVAL, why);
    *bytes = adj_layout(c, nsteps, ckpt_every).bytes;
    return PIC_OK;
}

namespace {
// The adjoint window on scratch `base` (>= the layout's bytes).  With `gid` (device memory
// of dvx_len doubles) the gradient is scattered by id on the device into gid, which first
// receives the caller's dW_dvx so that entries of ids absent from the run stay as they
// were, and is copied back whole; without it the host scatters (host staging vectors).
int adjoint_window_impl(pic_ctx *c, int32_t nsteps, int32_t ckpt_every, char *base, size_t bytes,
                        double *W, double *dW_dvx, int64_t dvx_len, double *dW_dEext, double *gid,
                        void *stream)
{
    c->sort_ready = false;  // particles or the step count change: no prepared sort
    c->insitu = false;
    const char *why = "";
    if (adj_check(c, &why)) return fail(c, PIC_EINVAL, why);
    const AdjLayout A = adj_layout(c, nsteps, ckpt_every);
    if (bytes < A.bytes) return fail(c, PIC_EINVAL, "adjoint scratch too small");
    hipStream_t s = (hipStream_t)stream;
    Dev &d = c->d;
    int32_t *ck_cell = (int32_t *)(base + A.off_ck_cell);
    float *ck_off = (float *)(base + A.off_ck_off);
    float *ck_vx = (float *)(base + A.off_ck_vx);
    int32_t *xc = (int32_t *)(base + A.off_xc);
    float *xo = (float *)(base + A.off_xo);
    double *Eb = (double *)(base + A.off_E);
    double *lx = (double *)(base + A.off_lx);
    double *lv = (double *)(base + A.off_lv);
    double *lE = (double *)(base + A.off_lE);
    double *lQ = (double *)(base + A.off_lQ);
    double *tmp = (double *)(base + A.off_tmp);
    double *lext = (double *)(base + A.off_ext);
    char *fin = base + A.off_fin;
    const int64_t n = A.n, nn = A.nn;
    const int N = (int)c->P.ens[0].ncells;
    const SegC &S = c->P.seg[0];
    const EnsC &En = c->P.ens[0];
    const double qm = S.h * 2.0 / En.dt;  // q/m
    // the particle buffer must be buffer 0 and hold no absorbed slots (periodic, no sort here)
    int32_t b = 0;
    int64_t nslots = 0;
    HIPC(c, hipMemcpyAsync(&b, d.cur, 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipMemcpyAsync(&nslots, d.n_slots, 8, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    if (b != 0) {
        // move the live buffer to buffer 0 so the recorded pointers stay valid
        for (int k = 0; k < 5; ++k) {
            void *dst = k == 0 ? (void *)d.cell[0] : k == 1 ? (void *)d.off[0] : k == 2 ? (void *)d.fvx[0] : k == 3 ? (void *)d.fvy[0] : (void *)d.fvz[0];
            void *src = k == 0 ? (void *)d.cell[1] : k == 1 ? (void *)d.off[1] : k == 2 ? (void *)d.fvx[1] : k == 3 ? (void *)d.fvy[1] : (void *)d.fvz[1];
            HIPC(c, hipMemcpyAsync(dst, src, n * 4, hipMemcpyDeviceToDevice, s));
        }
        HIPC(c, hipMemcpyAsync(d.id[0], d.id[1], n * 4, hipMemcpyDeviceToDevice, s));
        const int32_t zero = 0;
        HIPC(c, hipMemcpyAsync(d.cur, &zero, 4, hipMemcpyHostToDevice, s));
        HIPC(c, hipStreamSynchronize(s));
    }
    if (dvx_len < nslots) return fail(c, PIC_EINVAL, "dW_dvx too short");
    int64_t step0 = 0;
    HIPC(c, hipMemcpy(&step0, d.step, 8, hipMemcpyDeviceToHost));
    // Q^0 from the current positions (they may have been injected)
    HIPC(c, launch_zero_q(d, false, s));
    HIPC(c, launch_particles(d, c->L, s, false, SB_DEPOSIT, 0));
    // forward with checkpoints
    for (int t = 0; t < nsteps; ++t) {
        if (t % ckpt_every == 0) {
            const int64_t k = t / ckpt_every;
            HIPC(c, hipMemcpyAsync(ck_cell + k * n, d.cell[0], n * 4, hipMemcpyDeviceToDevice, s));
            HIPC(c, hipMemcpyAsync(ck_off + k * n, d.off[0], n * 4, hipMemcpyDeviceToDevice, s));
            HIPC(c, hipMemcpyAsync(ck_vx + k * n, d.fvx[0], n * 4, hipMemcpyDeviceToDevice, s));
        }
        HIPC(c, adj_forward_step(c, s, nullptr, nullptr, nullptr));
    }
    // objective at the final positions
    HIPC(c, launch_solve(d, false, c->P.chunks_tot, false, s));
    HIPC(c, launch_field_energy(d, s));
    double fe = 0.0;
    HIPC(c, hipMemcpyAsync(&fe, d.fe, 8, hipMemcpyDeviceToHost, s));
    // keep the final state
    HIPC(c, hipMemcpyAsync(fin, d.cell[0], n * 4, hipMemcpyDeviceToDevice, s));
    HIPC(c, hipMemcpyAsync(fin + n * 4, d.off[0], n * 4, hipMemcpyDeviceToDevice, s));
    HIPC(c, hipMemcpyAsync(fin + n * 8, d.fvx[0], n * 4, hipMemcpyDeviceToDevice, s));
    HIPC(c, hipMemcpyAsync(fin + n * 12, d.fvy[0], n * 4, hipMemcpyDeviceToDevice, s));
    HIPC(c, hipMemcpyAsync(fin + n * 16, d.fvz[0], n * 4, hipMemcpyDeviceToDevice, s));
    // seed: lE = eps0 dx E^N -> lQ -> lx; lv = 0
    HIPC(c, hipMemsetAsync(lx, 0, n * 8, s));
    HIPC(c, hipMemsetAsync(lv, 0, n * 8, s));
    HIPC(c, hipMemsetAsync(lE, 0, nn * 8, s));
    HIPC(c, hipMemsetAsync(lext, 0, 8, s));
    HIPC(c, launch_adj_seed(d.E, lE, N, En.eps0, En.dx, s));
    HIPC(c, launch_adj_grid(lE, lQ, tmp, N, En.dx, En.eps0, S.qw, s));
    HIPC(c, launch_adj_b(d.cell[0], lQ, lx, nslots, En.dx, N, s));
    // reverse sweep, one checkpoint segment at a time
    for (int64_t k = A.nseg_ck - 1; k >= 0; --k) {
        const int t0 = (int)(k * ckpt_every), t1 = std::min(nsteps, t0 + ckpt_every);
        HIPC(c, hipMemcpyAsync(d.cell[0], ck_cell + k * n, n * 4, hipMemcpyDeviceToDevice, s));
        HIPC(c, hipMemcpyAsync(d.off[0], ck_off + k * n, n * 4, hipMemcpyDeviceToDevice, s));
        HIPC(c, hipMemcpyAsync(d.fvx[0], ck_vx + k * n, n * 4, hipMemcpyDeviceToDevice, s));
        const int64_t st = step0 + t0;
        HIPC(c, hipMemcpyAsync(d.step, &st, 8, hipMemcpyHostToDevice, s));
        HIPC(c, launch_zero_q(d, false, s));
        HIPC(c, launch_particles(d, c->L, s, false, SB_DEPOSIT, 0));
        for (int t = t0; t < t1; ++t)
            HIPC(c, adj_forward_step(c, s, xc + (int64_t)(t - t0) * n, xo + (int64_t)(t - t0) * n,
                                     Eb + (int64_t)(t - t0) * nn));
        for (int t = t1 - 1; t >= t0; --t) {
            const int32_t *cx = xc + (int64_t)(t - t0) * n;
            const float *ox = xo + (int64_t)(t - t0) * n;
            HIPC(c, launch_adj_a(d, cx, ox, Eb + (int64_t)(t - t0) * nn, lx, lv, lE, lext, nslots, En.dt,
                                 qm, En.dx, N, s));
            HIPC(c, launch_adj_grid(lE, lQ, tmp, N, En.dx, En.eps0, S.qw, s));
            HIPC(c, launch_adj_b(cx, lQ, lx, nslots, En.dx, N, s));
        }
        HIPC(c, hipStreamSynchronize(s));
    }
    // restore the final state and step count
    HIPC(c, hipMemcpyAsync(d.cell[0], fin, n * 4, hipMemcpyDeviceToDevice, s));
    HIPC(c, hipMemcpyAsync(d.off[0], fin + n * 4, n * 4, hipMemcpyDeviceToDevice, s));
    HIPC(c, hipMemcpyAsync(d.fvx[0], fin + n * 8, n * 4, hipMemcpyDeviceToDevice, s));
    HIPC(c, hipMemcpyAsync(d.fvy[0], fin + n * 12, n * 4, hipMemcpyDeviceToDevice, s));
    HIPC(c, hipMemcpyAsync(d.fvz[0], fin + n * 16, n * 4, hipMemcpyDeviceToDevice, s));
    const int64_t stN = step0 + nsteps;
    HIPC(c, hipMemcpyAsync(d.step, &stN, 8, hipMemcpyHostToDevice, s));
    c->host_step = stN;
    HIPC(c, launch_zero_q(d, false, s));
    HIPC(c, launch_particles(d, c->L, s, false, SB_DEPOSIT, 0));
    // gradients by id
    double gext = 0.0;
    if (gid) {
        int32_t *bad = (int32_t *)lext + 2;  // a flag beside lext (its 64-byte slot)
        HIPC(c, hipMemsetAsync(bad, 0, 4, s));
        HIPC(c, hipMemcpyAsync(gid, dW_dvx, (size_t)dvx_len * 8, hipMemcpyHostToDevice, s));
        HIPC(c, launch_adj_by_id(lv, d.id[0], gid, nslots, dvx_len, bad, s));
        int32_t badh = 0;
        HIPC(c, hipMemcpyAsync(&badh, bad, 4, hipMemcpyDeviceToHost, s));
        HIPC(c, hipMemcpyAsync(&gext, lext, 8, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
        if (badh) return fail(c, PIC_EINVAL, "particle id beyond dW_dvx");
        HIPC(c, hipMemcpyAsync(dW_dvx, gid, (size_t)dvx_len * 8, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
    } else {
        std::vector<double> glv(nslots);
        std::vector<uint32_t> ids(nslots);
        HIPC(c, hipMemcpyAsync(glv.data(), lv, nslots * 8, hipMemcpyDeviceToHost, s));
        HIPC(c, hipMemcpyAsync(ids.data(), d.id[0], nslots * 4, hipMemcpyDeviceToHost, s));
        HIPC(c, hipMemcpyAsync(&gext, lext, 8, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
        for (int64_t i = 0; i < nslots; ++i) {
            if ((int64_t)ids[i] >= dvx_len) return fail(c, PIC_EINVAL, "particle id beyond dW_dvx");
            dW_dvx[ids[i]] = glv[i];
        }
    }
    *W = fe;
    *dW_dEext = gext;
    return check_err(c, s);
}
}  // namespace

int pic_adjoint_window(pic_ctx *c, int32_t nsteps, int32_t ckpt_every, void *scratch_dev, size_t bytes,
                       double *W, double *dW_dvx, int64_t dvx_len, double *dW_dEext, void *stream)
{
    if (!c || !scratch_dev || nsteps < 1 || ckpt_every < 1 || !W || !dW_dvx || !dW_dEext) return PIC_EINVAL;
    return adjoint_window_impl(c, nsteps, ckpt_every, (char *)scratch_dev, bytes, W, dW_dvx, dvx_len, dW_dEext,
                               nullptr, stream);
}

int pic_adjoint_window_noalloc(pic_ctx *c, int32_t nsteps, int32_t ckpt_every, double *W, double *dW_dvx,
                               int64_t dvx_len, double *dW_dEext, void *stream)
{
    if (!c || nsteps < 1 || ckpt_every < 1 || !W || !dW_dvx || dvx_len < 0 || !dW_dEext) return PIC_EINVAL;
    if (!c->static_scratch) return fail(c, PIC_EHIP, "static scratch address not looked up");
    const char *why = "";
    if (adj_check(c, &why)) return fail(c, PIC_EINVAL, why);
    // the window's layout, then the by-id gradient (dvx_len doubles) after it
    const size_t lay = adj_layout(c, nsteps, ckpt_every).bytes;
    const size_t need = lay + align_up((size_t)std::max<int64_t>(dvx_len, 1) * 8);
    if (need > kStaticScratchBytes)
        return fail(c, PIC_EINVAL, "adjoint window needs " + std::to_string(need) +
                                       " bytes of scratch, more than the static array's " +
                                       std::to_string(kStaticScratchBytes) +
                                       " (fewer particles, steps or a longer checkpoint interval fit; "
                                       "pic_adjoint_window takes a caller buffer of any size)");
    char *base = (char *)c->static_scratch;
    return adjoint_window_impl(c, nsteps, ckpt_every, base, lay, W, dW_dvx, dvx_len, dW_dEext,
                               (double *)(base + lay), stream);
}

int pic_autotune(pic_ctx *c, int32_t trial_steps, int32_t *shape, void *stream)
{
    if (!c || trial_steps < 1) return PIC_EINVAL;
    c->insitu = false;
    hipStream_t s = (hipStream_t)stream;
    if (!c->P.f64) {
        const int ppts[2] = {4, 8};
        const int wins[3] = {1024, 2048, 4096};
        const bool verbose = std::getenv("PIC_AUTOTUNE_VERBOSE") != nullptr;
        // candidates: particles per thread x LDS window x (fused pass only) non-temporal
        // streaming; two rounds in opposite orders; a candidate's score is the sum of its
        // two median per-launch pass times, so drift of the run's state between trials
        // cancels
        const int ncand = c->cfg.fused ? 12 : 6;
        double score[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int round = 0; round < 2; ++round) {
            for (int q = 0; q < ncand; ++q) {
                const int ci = round == 0 ? q : ncand - 1 - q;
                c->L.ppt = ppts[(ci % 6) / 3];
                c->L.window = wins[ci % 3];
                c->L.nt = ci / 6;
                // every candidate starts from freshly sorted particles
                HIPC(c, launch_particles(c->d, c->L, s, false, SB_HIST, 0));
                HIPC(c, launch_sort(c->d, false, c->L, s));
                c->sort_ready = false;
                int rc = pic_timing(c, 1);
                if (rc) return rc;
                for (int t = 0; t < trial_steps; ++t) {
                    HIPC(c, enqueue_step(c, s, c->host_step, c->sort_ready, false));
                    c->host_step += 1;
                }
                HIPC(c, hipStreamSynchronize(s));
                std::vector<double> v;
                for (int64_t i = 0; i + 1 < c->ev_used; i += 2) {
                    float ms = 0.f;
                    HIPC(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
                    v.push_back(ms);
                }
                double med = 1e300;
                if (!v.empty()) {
                    std::sort(v.begin(), v.end());
                    med = v[v.size() / 2];
                }
                score[ci] += med;
                if (verbose)
                    std::fprintf(stderr, "pic_autotune: ppt %d window %d nt %d round %d median pass %.4f ms\n",
                                 c->L.ppt, c->L.window, c->L.nt, round, med);
            }
        }
        Launch bestL = c->L;
        double best = 1e300;
        for (int ci = 0; ci < ncand; ++ci) {
            if (score[ci] < best) {
                best = score[ci];
                bestL.ppt = ppts[(ci % 6) / 3];
                bestL.window = wins[ci % 3];
                bestL.nt = ci / 6;
            }
        }
        c->L = bestL;
        pic_timing(c, 0);
        // sort scatter: particles per thread x non-temporal streaming, each timed on one
        // histogram + sort after a few steps of motion since the last sort
        hipEvent_t e0, e1;
        HIPC(c, hipEventCreate(&e0));
        HIPC(c, hipEventCreate(&e1));
        double bests = 1e300;
        int bestp = c->L.sort_ppt, bestnt = c->L.sort_nt;
        for (int ci = 0; ci < 4; ++ci) {
            c->L.sort_ppt = ppts[ci % 2];
            c->L.sort_nt = ci / 2;
            for (int t = 0; t < std::max(trial_steps / 2, 2); ++t) {
                HIPC(c, enqueue_step(c, s, c->host_step, c->sort_ready, true));
                c->host_step += 1;
            }
            HIPC(c, hipEventRecord(e0, s));
            HIPC(c, launch_particles(c->d, c->L, s, false, SB_HIST, 0));
            HIPC(c, launch_sort(c->d, false, c->L, s));
            c->sort_ready = false;
            HIPC(c, hipEventRecord(e1, s));
            HIPC(c, hipEventSynchronize(e1));
            float ms = 0.f;
            HIPC(c, hipEventElapsedTime(&ms, e0, e1));
            if (verbose)
                std::fprintf(stderr, "pic_autotune: sort ppt %d nt %d %.4f ms\n", c->L.sort_ppt, c->L.sort_nt, ms);
            if (ms < bests) {
                bests = ms;
                bestp = c->L.sort_ppt;
                bestnt = c->L.sort_nt;
            }
        }
        c->L.sort_nt = bestnt;
        c->L.sort_ppt = bestp;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        drop_graphs(c);
    }
    if (shape) {
        shape[0] = c->L.ppt;
        shape[1] = c->L.window;
        shape[2] = c->L.sort_ppt;
        shape[3] = c->L.nt;
        shape[4] = c->L.sort_nt;
    }
    return check_err(c, s);
}

// ---------------------------------------------------------------------------------------
// Checkpoint / restart.  Layout: header, per-segment {n_slots, next_id}, then per segment
// its particle arrays over the slots in use, then Q, the current speed-maxima half and the
// counters and sums.
namespace {
struct CkptHeader {
    uint64_t magic;
    int64_t nseg, nens, nodes_tot, cap_tot, f64, step, bytes, ncap_tot;
};
constexpr uint64_t kCkptMagic = 0x32544b5043494d50ull;  // "PMICPKT2"

// ns: slots in use per segment, then neutrals per ensemble (recycling runs)
size_t ckpt_bytes(const pic_ctx *c, const std::vector<int64_t> &ns)
{
    const int64_t per = c->P.f64 ? 36 : 24;
    size_t b = sizeof(CkptHeader) + (size_t)c->P.nseg * 16 + (size_t)c->P.nens * 8;
    for (size_t i = 0; i < ns.size(); ++i) b += (size_t)ns[i] * (i < (size_t)c->P.nseg ? per : 24);
    b += (size_t)2 * c->P.nodes_tot * 8;
    b += (size_t)kCntStripes * c->P.nseg * 8;
    b += (size_t)kCntStripes * c->P.nseg * (C_NCNT + S_NSUM) * 8;
    return b;
}

int ckpt_counts(pic_ctx *c, hipStream_t s, std::vector<int64_t> &ns, std::vector<uint32_t> &ids)
{
    ns.assign(c->P.nseg + c->P.nens, 0);
    ids.resize(c->P.nseg);
    HIPC(c, hipMemcpyAsync(ns.data(), c->d.n_slots, (size_t)c->P.nseg * 8, hipMemcpyDeviceToHost, s));
    HIPC(c, hipMemcpyAsync(ids.data(), c->d.next_id, ids.size() * 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    for (int en = 0; en < c->P.nens; ++en) {
        if (!c->P.ens[en].recycle) continue;
        int32_t b = 0;
        int64_t n = 0;
        int rc = neutral_state(c, en, s, b, n);
        if (rc) return rc;
        ns[c->P.nseg + en] = n;
    }
    return PIC_OK;
}
}  // namespace

int pic_checkpoint_size(pic_ctx *c, size_t *bytes, void *stream)
{
    if (!c || !bytes) return PIC_EINVAL;
    std::vector<int64_t> ns;
    std::vector<uint32_t> ids;
    int rc = ckpt_counts(c, (hipStream_t)stream, ns, ids);
    if (rc) return rc;
    *bytes = ckpt_bytes(c, ns);
    return PIC_OK;
}

int pic_save(pic_ctx *c, void *host_buf, size_t bytes, void *stream)
{
    if (!c || !host_buf) return PIC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int64_t> ns;
    std::vector<uint32_t> ids;
    int rc = ckpt_counts(c, s, ns, ids);
    if (rc) return rc;
    const size_t need = ckpt_bytes(c, ns);
    if (bytes < need) return fail(c, PIC_EINVAL, "checkpoint buffer too small");
    const Dev &d = c->d;
    int32_t cur = 0;
    int64_t step = 0;
    HIPC(c, hipMemcpyAsync(&cur, d.cur, 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipMemcpyAsync(&step, d.step, 8, hipMemcpyDeviceToHost, s));
    int32_t vcur = 0;
    HIPC(c, hipMemcpyAsync(&vcur, d.vcur, 4, hipMemcpyDeviceToHost, s));
    HIPC(c, hipStreamSynchronize(s));
    char *o = (char *)host_buf;
    int32_t ncur = 0;
    if (c->P.ncap_tot) {
        HIPC(c, hipMemcpyAsync(&ncur, d.ncur, 4, hipMemcpyDeviceToHost, s));
        HIPC(c, hipStreamSynchronize(s));
    }
    CkptHeader h{kCkptMagic, c->P.nseg, c->P.nens, c->P.nodes_tot, c->P.cap_tot, c->P.f64 ? 1 : 0, step,
                 (int64_t)need, c->P.ncap_tot};
    std::memcpy(o, &h, sizeof(h));
    o += sizeof(h);
    for (int sg = 0; sg < c->P.nseg; ++sg) {
        const int64_t v[2] = {ns[sg], (int64_t)ids[sg]};
        std::memcpy(o, v, 16);
        o += 16;
    }
    std::memcpy(o, ns.data() + c->P.nseg, (size_t)c->P.nens * 8);
    o += (size_t)c->P.nens * 8;
    auto d2h = [&](const void *src, size_t n) -> hipError_t {
        hipError_t e = n ? hipMemcpyAsync(o, src, n, hipMemcpyDeviceToHost, s) : hipSuccess;
        o += n;
        return e;
    };
    for (int sg = 0; sg < c->P.nseg; ++sg) {
        const int64_t base = c->P.seg[sg].base, n = ns[sg];
        if (c->P.f64) {
            HIPC(c, d2h(d.x[cur] + base, n * 8));
            HIPC(c, d2h(d.dvx[cur] + base, n * 8));
            HIPC(c, d2h(d.dvy[cur] + base, n * 8));
            HIPC(c, d2h(d.dvz[cur] + base, n * 8));
        } else {
            HIPC(c, d2h(d.cell[cur] + base, n * 4));
            HIPC(c, d2h(d.off[cur] + base, n * 4));
            HIPC(c, d2h(d.fvx[cur] + base, n * 4));
            HIPC(c, d2h(d.fvy[cur] + base, n * 4));
            HIPC(c, d2h(d.fvz[cur] + base, n * 4));
        }
        HIPC(c, d2h(d.id[cur] + base, n * 4));
    }
    for (int en = 0; en < c->P.nens; ++en) {
        const int64_t base = c->P.ens[en].nbase, n = ns[c->P.nseg + en];
        HIPC(c, d2h(d.ncell[ncur] + base, n * 4));
        HIPC(c, d2h(d.noff[ncur] + base, n * 4));
        HIPC(c, d2h(d.nvx[ncur] + base, n * 4));
        HIPC(c, d2h(d.nvy[ncur] + base, n * 4));
        HIPC(c, d2h(d.nvz[ncur] + base, n * 4));
        HIPC(c, d2h(d.nid[ncur] + base, n * 4));
    }
    HIPC(c, d2h(c->P.f64 ? (const void *)d.Qd : (const void *)d.Qi, (size_t)2 * c->P.nodes_tot * 8));
    HIPC(c, d2h(d.vmax2 + (size_t)vcur * kCntStripes * c->P.nseg, (size_t)kCntStripes * c->P.nseg * 8));
    HIPC(c, d2h(d.cnt, (size_t)kCntStripes * c->P.nseg * C_NCNT * 8));
    HIPC(c, d2h(d.sums, (size_t)kCntStripes * c->P.nseg * S_NSUM * 8));
    HIPC(c, hipStreamSynchronize(s));
    return PIC_OK;
}

int pic_load(pic_ctx *c, const void *host_buf, size_t bytes, void *stream)
{
    if (!c || !host_buf || bytes < sizeof(CkptHeader)) return PIC_EINVAL;
    c->sort_ready = false;  // particles or the step count change: no prepared sort
    c->insitu = false;
    hipStream_t s = (hipStream_t)stream;
    CkptHeader h;
    std::memcpy(&h, host_buf, sizeof(h));
    if (h.magic != kCkptMagic || h.nseg != c->P.nseg || h.nens != c->P.nens || h.nodes_tot != c->P.nodes_tot ||
        h.cap_tot != c->P.cap_tot || h.f64 != (c->P.f64 ? 1 : 0) || (size_t)h.bytes > bytes ||
        h.ncap_tot != c->P.ncap_tot)
        return fail(c, PIC_EINVAL, "checkpoint from a different configuration");
    const char *o = (const char *)host_buf + sizeof(h);
    std::vector<int64_t> ns(c->P.nseg + c->P.nens);
    std::vector<uint32_t> ids(c->P.nseg);
    for (int sg = 0; sg < c->P.nseg; ++sg) {
        int64_t v[2];
        std::memcpy(v, o, 16);
        o += 16;
        if (v[0] < 0 || v[0] > c->P.seg[sg].cap) return fail(c, PIC_EINVAL, "checkpoint slot count");
        ns[sg] = v[0];
        ids[sg] = (uint32_t)v[1];
    }
    std::memcpy(ns.data() + c->P.nseg, o, (size_t)c->P.nens * 8);
    o += (size_t)c->P.nens * 8;
    for (int en = 0; en < c->P.nens; ++en)
        if (ns[c->P.nseg + en] < 0 || ns[c->P.nseg + en] > c->P.ens[en].ncap)
            return fail(c, PIC_EINVAL, "checkpoint neutral count");
    if (ckpt_bytes(c, ns) != (size_t)h.bytes) return fail(c, PIC_EINVAL, "checkpoint size");
    const Dev &d = c->d;
    HIPC(c, hipStreamSynchronize(s));
    // the run continues from buffer 0, both birth halves clean, speed maxima in half 0
    HIPC(c, launch_births_clear_all(d, s));
    auto h2d = [&](void *dst, size_t n) -> hipError_t {
        hipError_t e = n ? hipMemcpyAsync(dst, o, n, hipMemcpyHostToDevice, s) : hipSuccess;
        o += n;
        return e;
    };
    for (int sg = 0; sg < c->P.nseg; ++sg) {
        const int64_t base = c->P.seg[sg].base, n = ns[sg];
        if (c->P.f64) {
            HIPC(c, h2d(d.x[0] + base, n * 8));
            HIPC(c, h2d(d.dvx[0] + base, n * 8));
            HIPC(c, h2d(d.dvy[0] + base, n * 8));
            HIPC(c, h2d(d.dvz[0] + base, n * 8));
        } else {
            HIPC(c, h2d(d.cell[0] + base, n * 4));
            HIPC(c, h2d(d.off[0] + base, n * 4));
            HIPC(c, h2d(d.fvx[0] + base, n * 4));
            HIPC(c, h2d(d.fvy[0] + base, n * 4));
            HIPC(c, h2d(d.fvz[0] + base, n * 4));
        }
        HIPC(c, h2d(d.id[0] + base, n * 4));
    }
    // neutrals continue from buffer 0, with the other buffer and the absorbed-ion list empty
    std::vector<unsigned long long> nn(2 * (size_t)c->P.nens, 0ull);
    for (int en = 0; en < c->P.nens; ++en) {
        const int64_t base = c->P.ens[en].nbase, n = ns[c->P.nseg + en];
        nn[en] = (unsigned long long)n;
        HIPC(c, h2d(d.ncell[0] + base, n * 4));
        HIPC(c, h2d(d.noff[0] + base, n * 4));
        HIPC(c, h2d(d.nvx[0] + base, n * 4));
        HIPC(c, h2d(d.nvy[0] + base, n * 4));
        HIPC(c, h2d(d.nvz[0] + base, n * 4));
        HIPC(c, h2d(d.nid[0] + base, n * 4));
    }
    HIPC(c, hipMemcpyAsync(d.nneu, nn.data(), nn.size() * 8, hipMemcpyHostToDevice, s));
    {
        const int32_t z = 0;
        const uint32_t zu = 0;
        HIPC(c, hipMemcpyAsync(d.ncur, &z, 4, hipMemcpyHostToDevice, s));
        HIPC(c, hipMemcpyAsync(d.nrec, &zu, 4, hipMemcpyHostToDevice, s));
        HIPC(c, hipStreamSynchronize(s));
    }
    HIPC(c, h2d(c->P.f64 ? (void *)d.Qd : (void *)d.Qi, (size_t)2 * c->P.nodes_tot * 8));
    HIPC(c, h2d(d.vmax2, (size_t)kCntStripes * c->P.nseg * 8));
    HIPC(c, hipMemsetAsync(d.vmax2 + (size_t)kCntStripes * c->P.nseg, 0, (size_t)kCntStripes * c->P.nseg * 8, s));
    HIPC(c, h2d(d.cnt, (size_t)kCntStripes * c->P.nseg * C_NCNT * 8));
    HIPC(c, h2d(d.sums, (size_t)kCntStripes * c->P.nseg * S_NSUM * 8));
    HIPC(c, hipMemsetAsync(d.ssum, 0, (size_t)2 * kCntStripes * c->P.nseg * T_NSTEP * 8, s));
    const int32_t zero = 0;
    HIPC(c, hipMemcpyAsync(d.n_slots, ns.data(), ns.size() * 8, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(d.next_id, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(d.cur, &zero, 4, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(d.vcur, &zero, 4, hipMemcpyHostToDevice, s));
    HIPC(c, hipMemcpyAsync(d.step, &h.step, 8, hipMemcpyHostToDevice, s));
    HIPC(c, hipStreamSynchronize(s));
    c->host_step = h.step;
    drop_graphs(c);
    return check_err(c, s);
}

int pic_timing(pic_ctx *c, int32_t enable)
{
    if (!c) return PIC_EINVAL;
    c->timing = enable != 0;
    c->ev_used = 0;
    if (c->timing && c->ev.empty()) {
        c->ev.resize(2 * 65536);
        for (auto &e : c->ev) HIPC(c, hipEventCreate(&e));
    }
    return PIC_OK;
}

int pic_timing_read(pic_ctx *c, double *ms_total, int64_t *launches, void *stream)
{
    if (!c || !ms_total || !launches) return PIC_EINVAL;
    HIPC(c, hipStreamSynchronize((hipStream_t)stream));
    double tot = 0.0;
    for (int64_t i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.f;
        HIPC(c, hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        tot += ms;
    }
    *ms_total = tot;
    *launches = c->ev_used / 2;
    return PIC_OK;
}

int pic_stream_copy(const void *src, void *dst, size_t bytes, int32_t nontemporal, void *stream)
{
    if (!src || !dst || bytes % 16 != 0 || bytes / 16 > ((size_t)1 << 31) * 64) return PIC_EINVAL;
    const hipError_t e = launch_stream_copy(src, dst, (int64_t)(bytes / 4), nontemporal != 0, (hipStream_t)stream);
    return e == hipSuccess ? PIC_OK : PIC_EHIP;
}

void pic_free(pic_ctx *c)
{
    if (!c) return;
    for (auto &e : c->ev) (void)hipEventDestroy(e);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
}

const char *pic_last_error(const pic_ctx *c) { return c ? c->msg.c_str() : "null context"; }

}  // extern "C"
