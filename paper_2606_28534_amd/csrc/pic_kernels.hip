// pic_kernels.hip -- gfx950 kernels of the electrostatic 1D3V PIC Monte Carlo step.
//
// This file holds the field solve, the birth ranking and placement, particle loading,
// diagnostics, the scans of the sort, and the FP64 (plain x, v) particle pass and sort
// scatter; the FP32 cell+offset pass, candidates and sort are in pic_pass32.hip.  The FP64
// pass covers every particle stage with one template: gather + Boris push + walls,
// null-collision MC, cloud-in-cell deposit and the sort histogram are compile-time stage
// bits, so its separate-stage verbs and its fused step run the same per-particle code.  It
// streams each segment's slots once, coalesced, with persistent blocks that take tiles from
// per-XCD queues and steal from the others when theirs is empty (load balancing inside the
// GPU), and deposits with FP64 atomics, each tile's shares merged first in an LDS window.
#include <type_traits>

#include "pic.h"
#include "pic_device.h"
#include "pic_kernels.h"
#include "pic_particle.h"

namespace pic {

// =======================================================================================
// Tile scheduling of the persistent FP64 kernels: live tiles are enumerated over all
// segments.  The particle pass takes them from queues (tq_grab); the sort scatter gives
// block b a contiguous run of them.  Blocks are dispatched round-robin over the 8 XCDs, so block b is mapped
// to run (b % 8) * (G / 8) + b / 8: each XCD gets one contiguous eighth of the particles
// (and of the cells, once sorted), which keeps its L2 working set to its own part of the
// grid.
// =======================================================================================
constexpr int kMaxSeg = 512;

__device__ __forceinline__ void sched_prefix(const Dev &d, int64_t tile, int64_t *s_tpre,
                                             int64_t *s_lim = nullptr)
{
    // s_tpre[i] = sum over segments < i of ceil(n_slots / tile); nseg <= kMaxSeg.  With
    // s_lim, also each segment's first slot and end of its slots in use, [2 i] and [2 i + 1].
    __shared__ int64_t s_tmp[kMaxSeg];
    for (int i = threadIdx.x; i < d.nseg; i += blockDim.x) {
        int64_t n = d.n_slots[i];
        s_tmp[i] = (n + tile - 1) / tile;
        if (s_lim) {
            const int64_t base = d.seg[i].base;
            s_lim[2 * i] = base;
            s_lim[2 * i + 1] = base + n;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t acc = 0;
        for (int i = 0; i < d.nseg; ++i) {
            s_tpre[i] = acc;
            acc += s_tmp[i];
        }
        s_tpre[d.nseg] = acc;
    }
    __syncthreads();
}

__device__ __forceinline__ int seg_of_tile(const int64_t *s_tpre, int nseg, int64_t t)
{
    int lo = 0, hi = nseg;  // s_tpre[lo] <= t < s_tpre[hi]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (s_tpre[mid] <= t)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Single-GPU load balancing of the persistent FP64 pass (the analogue, inside one GPU, of
// the paper's particle load balancing between ranks): the live tiles are split into eight
// contiguous queues, one per XCD (queue x holds tiles [x T / 8, (x + 1) T / 8)), and a
// block takes kGrabTiles tiles at a time from the queue of its own XCD (blocks are
// dispatched round-robin over the XCDs), with the next grab in flight while it works; when
// that queue is empty it takes from the others in turn.  Blocks that draw slow tiles (many
// cell changes, births spread over the domain, atomics on shared nodes) simply take fewer,
// so the launch ends when the work does, not when the slowest static share does.  A queue
// counter is the number of tiles handed out; the last block to finish resets them.
constexpr int kGrabTiles = 4;
constexpr int kTileQueues = 8;

// First tile of the next grab from queue x (a value >= the queue's end means empty).
__device__ __forceinline__ int64_t tq_grab(const Dev &d, int x, int64_t T)
{
    return (int64_t)x * T / kTileQueues + (int64_t)atomicAdd(d.tq + x, (uint32_t)kGrabTiles);
}

__device__ __forceinline__ void block_run(int64_t T, int64_t &t0, int64_t &t1)
{
    const int64_t G = gridDim.x;
    int64_t vb = blockIdx.x;
    if ((G & 7) == 0) vb = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
    t0 = vb * T / G;
    t1 = (vb + 1) * T / G;
}

// =======================================================================================
// Block reductions of a few per-thread tallies, flushed to the striped counters.
// =======================================================================================
struct Tally {
    uint32_t push, wl, wr, el, iz, cx;
    double kel, ker, v2max;
    __device__ void zero()
    {
        push = wl = wr = el = iz = cx = 0;
        kel = ker = 0.0;
        v2max = 0.0;
    }
};

__device__ void flush_tally(const Dev &d, int seg, Tally &t, bool want_vmax)
{
    __shared__ double s_red[16][9];
    const int lane = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    double v[9] = {(double)t.push, (double)t.wl, (double)t.wr, (double)t.el, (double)t.iz,
                   (double)t.cx, t.kel, t.ker, t.v2max};
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = wave_sum_f64(v[k]);
    v[8] = wave_max_f64(v[8]);
    if (lane == 0)
        for (int k = 0; k < 9; ++k) s_red[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        double a[9];
        for (int k = 0; k < 9; ++k) a[k] = s_red[0][k];
        for (int i = 1; i < nw; ++i) {
            for (int k = 0; k < 8; ++k) a[k] += s_red[i][k];
            a[8] = fmax(a[8], s_red[i][8]);
        }
        const int st = stripe_of_block();
        unsigned long long *c = d.cnt + ((int64_t)st * d.nseg + seg) * C_NCNT;
        if (a[0] != 0.0) atomicAdd(c + C_PUSH, (unsigned long long)a[0]);
        if (a[1] != 0.0) atomicAdd(c + C_WALL_L, (unsigned long long)a[1]);
        if (a[2] != 0.0) atomicAdd(c + C_WALL_R, (unsigned long long)a[2]);
        if (a[3] != 0.0) atomicAdd(c + C_EL, (unsigned long long)a[3]);
        if (a[4] != 0.0) atomicAdd(c + C_IZ, (unsigned long long)a[4]);
        if (a[5] != 0.0) atomicAdd(c + C_CX, (unsigned long long)a[5]);
        double *sm = d.sums + ((int64_t)st * d.nseg + seg) * S_NSUM;
        if (a[6] != 0.0) unsafeAtomicAdd(sm + S_KE_L, a[6]);
        if (a[7] != 0.0) unsafeAtomicAdd(sm + S_KE_R, a[7]);
        if (want_vmax && a[8] > 0.0) {
            const int half = 1 - *d.vcur;
            atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + seg, dbits(a[8]));
        }
    }
    __syncthreads();
    t.zero();
}

// =======================================================================================
// The FP64 particle pass (the FP32 form runs in k_pass32).  A persistent grid walks the
// tiles of all segments; each stage is optional, so the same kernel serves the fused pass
// and the separate stages.  The deposit adds each tile's shares into an LDS window of FP64
// nodes, then each touched node into the FP64 node array with one atomic.
// =======================================================================================
enum Stage : int { ST_PUSH = 1, ST_COLLIDE = 2, ST_DEPOSIT = 4, ST_HIST = 8 };

template <int STAGES, int PPT>
__global__ void __launch_bounds__(256) k_particles(Dev d, int hist_rt)
{
    constexpr bool PUSH = STAGES & ST_PUSH;
    constexpr bool COLL = STAGES & ST_COLLIDE;
    constexpr bool DEPO = STAGES & ST_DEPOSIT;
    constexpr bool HISTC = STAGES & ST_HIST;  // histogram-only pass
    const bool hist = HISTC || (hist_rt != 0);
    constexpr bool NEED_V = PUSH || COLL;
    constexpr bool NEED_ID = COLL;

    __shared__ int64_t s_tpre[kMaxSeg + 1];
    __shared__ int64_t s_lim[2 * kMaxSeg];       // each segment's slots in use, from LDS
    __shared__ double s_win[(DEPO || HISTC) ? kWin64 : 1];  // the tile's deposit (or count) window
    __shared__ int s_mm[8];

    const int BLOCK = blockDim.x;
    const int64_t TILE = (int64_t)BLOCK * PPT;
    sched_prefix(d, TILE, s_tpre, s_lim);
    const int64_t T = s_tpre[d.nseg];
    const int b = *d.cur;
    const int64_t step = *d.step;
    const uint32_t tag = (uint32_t)step;
    const int st = stripe_of_block();

    Tally tal;
    tal.zero();
    int tseg = -1;
    // tile queues: own XCD's first, then the others in turn (see tq_grab)
    __shared__ int64_t s_grab;
    __shared__ bool s_last;
    const int xq = (int)(blockIdx.x % kTileQueues);
    int qi = 0;
    if (threadIdx.x == 0) s_grab = tq_grab(d, xq, T);
    __syncthreads();
    int64_t g0 = s_grab;

    for (;;) {
        const int x = (xq + qi) % kTileQueues;
        const int64_t qend = (int64_t)(x + 1) * T / kTileQueues;
        if (g0 >= qend) {
            // this queue is empty: try the next one, or stop after the last
            if (++qi == kTileQueues) break;
            __syncthreads();
            if (threadIdx.x == 0) s_grab = tq_grab(d, (xq + qi) % kTileQueues, T);
            __syncthreads();
            g0 = s_grab;
            continue;
        }
        // the next grab from the same queue, in flight while these tiles are processed
        __syncthreads();
        if (threadIdx.x == 0) s_grab = tq_grab(d, x, T);
        const int64_t g1 = min(g0 + kGrabTiles, qend);
    for (int64_t t = g0; t < g1; ++t) {
        const int sg = __builtin_amdgcn_readfirstlane(seg_of_tile(s_tpre, d.nseg, t));
        const SegC &S = d.seg[sg];
        const EnsC &e = d.ens[S.ens];
        const Seg64 G = seg64(S, e);  // gather, push and deposit constants in registers
        const int s = S.species;
        if (sg != tseg) {
            if (tseg >= 0 && (PUSH || COLL)) flush_tally(d, tseg, tal, COLL);
            tseg = sg;
        }
        // the tile's slots from LDS, so its loads wait on nothing in global memory
        const int64_t lt = t - s_tpre[sg];
        const int64_t first = s_lim[2 * sg] + lt * TILE;
        const int64_t last = min(first + TILE, s_lim[2 * sg + 1]);

        // every particle's loads are issued before any is tested, so the tile waits for
        // memory once
        PS<true> p[PPT];
        bool live[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int64_t i = first + (int64_t)k * BLOCK + threadIdx.x;
            p[k].x = -1.0;
            if (i < last) p_load<true>(d, b, i, p[k], NEED_V, NEED_ID);
        }
#pragma unroll
        for (int k = 0; k < PPT; ++k) live[k] = p_alive<true>(p[k]);
        const double numax = COLL ? d.numax[sg] : 0.0;
        const double pnull = COLL ? d.pnull[sg] : 0.0;
        // The tile in phases, each over all its particles: push (every gather issued before
        // any particle is pushed), collide, write back.  A particle still goes through push
        // then collide, and the push constants are dead once the pushes are done.
        if constexpr (PUSH) {
            double Eg[PPT];
            gather64<PPT>(d, G, p, Eg);
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (!live[k]) continue;
                const int64_t i = first + (int64_t)k * BLOCK + threadIdx.x;
                ++tal.push;
                const int wall = p_push64(d, G, p[k], Eg[k]);
                if (wall == 3) {
                    p_kill<true>(p[k]);
                    live[k] = false;
                    d.x[b][i] = -1.0;
                } else if (wall) {
                    const double v2 = speed2_rn((double)p[k].vx, (double)p[k].vy, (double)p[k].vz);
                    if (wall == 1) {
                        ++tal.wl;
                        tal.kel += S.halfmw * v2;
                    } else {
                        ++tal.wr;
                        tal.ker += S.halfmw * v2;
                    }
                    p_kill<true>(p[k]);
                    live[k] = false;
                    d.x[b][i] = -1.0;
                }
            }
        }
        int ch[PPT];  // collision channel (-1: none)
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            ch[k] = -1;
            if (COLL && live[k]) {
                double ve[3], vi[3];
                ch[k] = p_collide<true>(e, S, s, numax, pnull, tag, p[k], ve, vi);
                if (ch[k] == 0)
                    ++tal.el;
                else if (ch[k] == 2)
                    ++tal.cx;
                else if (ch[k] == 1) {
                    ++tal.iz;
                    // birth record: slot in this block's stripe, or in the next ones when
                    // it is full
                    const BirthBuf bb = birth_buf(d, (int)(tag & 1u));
                    int bst = st & (kStripes - 1);
                    uint32_t slot = atomicAdd(bb.nbirth + bst, 1u);
                    for (int a = 1; a < kStripes && (int64_t)slot >= d.birth_stripe_cap; ++a) {
                        bst = (bst + 1) & (kStripes - 1);
                        slot = atomicAdd(bb.nbirth + bst, 1u);
                    }
                    if ((int64_t)slot < d.birth_stripe_cap) {
                        Birth &B = bb.births[(int64_t)bst * d.birth_stripe_cap + slot];
                        B.pid = p[k].id;
                        B.ens = S.ens;
                        B.cell = 0;
                        B.off = 0.f;
                        B.x = p[k].x;
                        for (int q = 0; q < 3; ++q) {
                            B.ve[q] = ve[q];
                            B.vi[q] = vi[q];
                        }
                        birth_mark(bb, e, p[k].id);
                    } else {
                        atomicOr(d.err, (int)E_CAP_BIRTH);
                    }
                    const double ve2 = speed2_rn(ve[0], ve[1], ve[2]);
                    tal.v2max = fmax(tal.v2max, ve2);
                    if (S.other >= 0) {
                        const double vi2 = speed2_rn(vi[0], vi[1], vi[2]);
                        const int half = 1 - *d.vcur;
                        atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + S.other,
                                  dbits(vi2));
                    }
                    if (DEPO) {
                        // the new pair sits at the parent's position
                        global_deposit64(d, S, s, p[k].x, hist);
                        if (S.other >= 0) global_deposit64(d, d.seg[S.other], 1, p[k].x, hist);
                    }
                }
                tal.v2max = fmax(tal.v2max, speed2_rn((double)p[k].vx, (double)p[k].vy, (double)p[k].vz));
            }
        }
        // write back (the collide stage alone only the velocities it changed)
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (!(live[k] && (PUSH || ch[k] >= 0))) continue;
            const int64_t i = first + (int64_t)k * BLOCK + threadIdx.x;
            if (PUSH) d.x[b][i] = p[k].x;
            d.dvx[b][i] = p[k].vx;
            d.dvy[b][i] = p[k].vy;
            d.dvz[b][i] = p[k].vz;
        }
        // deposit through the tile's LDS window (and sort histogram), by runs of equal cell
        // across the wave's lanes
        if constexpr (DEPO) {
            tile_deposit64<PPT>(d, G, s, live, p, hist, s_win, s_mm);
        } else if (HISTC) {
            tile_deposit64<PPT, true>(d, G, s, live, p, true, s_win, s_mm);
        }
    }
        __syncthreads();
        g0 = s_grab;
    }
    if ((PUSH || COLL) && tseg >= 0) flush_tally(d, tseg, tal, COLL);
    // the last block to finish resets the queues (every block has stopped taking tiles)
    __syncthreads();
    if (threadIdx.x == 0) s_last = atomicAdd(d.tq + kTileQueues, 1u) == gridDim.x - 1;
    __syncthreads();
    if (s_last && threadIdx.x <= kTileQueues) d.tq[threadIdx.x] = 0u;
}

// =======================================================================================
// Particle load.
// =======================================================================================
template <bool F64>
__global__ void k_init(Dev d, int sg, int64_t n, int64_t ppc, int init_mode, double vth,
                       double amp, int mode)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const SegC &S = d.seg[sg];
    const EnsC &e = d.ens[S.ens];
    const int s = S.species;
    const int64_t i = S.base + p;
    double x;
    int cell = 0;
    float off = 0.f;
    if (init_mode == 0) {
        cell = (int)(p / ppc);
        const uint4 w = draw(S.seed, s, (uint32_t)p, kInitTag, 0u);
        off = u01f(w.x);
        x = ((double)cell + (double)off) * S.dx;
    } else {
        const double L = e.L;
        const double k = 6.283185307179586476925286766559 * (double)mode / L;
        const double x0 = ((double)p + 0.5) * L / (double)n;
        x = x0 + (amp / k) * sin(k * x0);
        if (x < 0.0) x += L;
        if (x >= L) x -= L;
        if (!(x >= 0.0 && x < L)) x = 0.0;
        const double g = x / S.dx;
        double jf = floor(g);
        cell = (int)jf;
        off = (float)(g - jf);
        if (off >= 1.0f) {
            off = 0.0f;
            cell += 1;
            if (cell >= S.ncells) cell = 0;
        }
    }
    double z[3];
    three_normals<double>(draw(S.seed, s, (uint32_t)p, kInitTag, 1u), z);
    if constexpr (!F64) {
        d.cell[0][i] = cell;
        d.off[0][i] = off;
        d.fvx[0][i] = (float)(vth * z[0]);
        d.fvy[0][i] = (float)(vth * z[1]);
        d.fvz[0][i] = (float)(vth * z[2]);
    } else {
        d.x[0][i] = x;
        d.dvx[0][i] = vth * z[0];
        d.dvy[0][i] = vth * z[1];
        d.dvz[0][i] = vth * z[2];
    }
    d.id[0][i] = (uint32_t)p;
}

// Max |v|^2 of every segment into the current half of vmax2 (after a load or injection).
template <bool F64>
__global__ void k_vmax(Dev d)
{
    __shared__ double s_m[16];
    const int sg = blockIdx.y;
    const SegC &S = d.seg[sg];
    const int b = *d.cur;
    const int64_t n = d.n_slots[sg];
    double m = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = S.base + p;
        if constexpr (!F64) {
            if (d.cell[b][i] == kDead) continue;
            m = fmax(m, speed2_rn(d.fvx[b][i], d.fvy[b][i], d.fvz[b][i]));
        } else {
            if (!(d.x[b][i] >= 0.0)) continue;
            m = fmax(m, speed2_rn(d.dvx[b][i], d.dvy[b][i], d.dvz[b][i]));
        }
    }
    m = wave_max_f64(m);
    if (lane_id() == 0) s_m[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)(blockDim.x / kWave); ++i) m = fmax(m, s_m[i]);
        const int half = *d.vcur;
        if (m > 0.0)
            atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + stripe_of_block()) * d.nseg + sg, dbits(m));
    }
}

// =======================================================================================
// Field solve.  With constant coefficients the three-point Poisson system on the interior
// nodes (phi_0 = phi_N = 0) factors into two prefix sums:
//   C_m = sum_{i=1..m} rho_i,  E_{m+1/2} = E_{1/2} + (dx/eps0) C_m,
//   phi_j = -dx (j E_{1/2} + (dx/eps0) sum_{m<j} C_m),
//   E_{1/2} = -(dx/eps0) sum_{m=0}^{N-1} C_m / N      (from phi_N = 0).
// This is the exact solution of the same tridiagonal system the Thomas algorithm solves,
// computed in two passes over the nodes: pass 1 reduces per-chunk aggregates, pass 2 has
// each chunk scan the aggregates of its ensemble and then its own nodes.  Node E is the
// centred difference, i.e. the mean of the two face fields, with the half-cell Gauss rule
// at bounded walls.  Periodic runs add the uniform background that cancels the deposited
// charge and shift phi to zero mean afterwards.
// =======================================================================================
__device__ __forceinline__ double node_vol(const EnsC &e, int64_t j)
{
    if (!e.periodic && (j == 0 || j == e.ncells)) return 0.5 * e.dx;
    return e.dx;
}

// Reading R23: p passes of the 1-2-1 filter equal one binomial stencil of width 2p + 1
// (weights C(2p, p + i) / 4^p) applied to the periodic extension of rho, or on a bounded
// grid to its even extension across both walls (a pass maps an even extension to an even
// extension, with rho_{-1} = rho_1 at the wall, so the passes compose into the stencil).
// Each node therefore reads its 2p + 1 neighbours once instead of p sweeps over the grid.
// smooth_fold maps a node index in [-p, nn - 1 + p] onto the grid (p <= 4 and N >= 2, so a
// couple of wraps or reflections at most).
__device__ __forceinline__ int64_t smooth_fold(const EnsC &e, int64_t m)
{
    const int64_t n = e.ncells;
    if (e.periodic) {
        while (m < 0) m += n;
        while (m >= n) m -= n;
        return m;
    }
    for (int it = 0; it < 8; ++it) {
        if (m < 0)
            m = -m;
        else if (m > n)
            m = 2 * n - m;
        else
            break;
    }
    return m;
}

// One species' deposited charge at NQ nodes (offsets into the node arrays), all loads
// issued before the first is used.
template <bool F64, int NQ>
__device__ __forceinline__ void node_q_row(const Dev &d, int64_t row, const int64_t (&at)[NQ],
                                           double (&Q)[NQ])
{
    if constexpr (!F64) {
        unsigned long long raw[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) raw[q] = d.Qi[row + at[q]];
#pragma unroll
        for (int q = 0; q < NQ; ++q) Q[q] = (double)(long long)raw[q] * (1.0 / kFix);
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) Q[q] = d.Qd[row + at[q]];
    }
}

// Charge density sum_s q_s w_s Q_s(j) / vol(j) at NQ nodes per thread (entries with ok[q]
// false give 0).  The loads are unconditional (node 0 stands in for unused entries), so the
// thread waits for memory once instead of once per node and species.
template <bool F64, int NQ>
__device__ __forceinline__ void node_rho_raw(const Dev &d, const EnsC &e, const int64_t (&j)[NQ],
                                             const bool (&ok)[NQ], double (&r)[NQ])
{
    static_assert(sizeof(e.qw) / sizeof(e.qw[0]) == 2, "at most two charged species");
    int64_t at[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) at[q] = e.gbase + (ok[q] ? j[q] : 0);
    double Q0[NQ], Q1[NQ];
    node_q_row<F64, NQ>(d, 0, at, Q0);
    const bool two = e.nspecies > 1;
    if (two) node_q_row<F64, NQ>(d, d.nodes_tot, at, Q1);
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double c = 0.0;
        c += e.qw[0] * Q0[q];
        if (two) c += e.qw[1] * Q1[q];
        r[q] = ok[q] ? c / node_vol(e, j[q]) : 0.0;
    }
}

// Block-wide inclusive scan of one double per thread (256 threads).
__device__ double block_incl_scan(double v, double *s_buf)
{
    const int lane = lane_id(), w = threadIdx.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double n = __shfl_up(v, o);
        if (lane >= o) v += n;
    }
    if (lane == kWave - 1) s_buf[w] = v;
    __syncthreads();
    double add = 0.0;
    for (int i = 0; i < w; ++i) add += s_buf[i];
    __syncthreads();
    return v + add;
}

__device__ double block_sum(double v, double *s_buf)
{
    v = wave_sum_f64(v);
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    if (lane_id() == 0) s_buf[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i) r += s_buf[i];
    __syncthreads();
    return r;
}

// N block-wide sums at once (one LDS round); same summation order as block_sum.
template <int N>
__device__ void block_sums(double (&v)[N], double *s /* N * 16 doubles */)
{
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum_f64(v[i]);
    if (lane_id() == 0) {
#pragma unroll
        for (int i = 0; i < N; ++i) s[i * 16 + w] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < N; ++i) {
        double r = 0.0;
        for (int k = 0; k < nw; ++k) r += s[i * 16 + k];
        v[i] = r;
    }
    __syncthreads();
}

__device__ __forceinline__ int chunk_ens(const Dev &d, int64_t k)
{
    int lo = 0, hi = d.nens;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (d.ens[mid].chunk0 <= k)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

constexpr int kNodesPerThread = kChunk / kSolveThreads;
// Blocks that place a step's births: the births grow with the particles (about 4.5e-4 of
// the electrons per step), so the block count does too, from 64 (enough for the 4e7-particle
// slab's ten thousand, under one per thread) to 256 from 5e8 slots on (64 batched
// ensembles: their solve kernel 61 -> 49 us; on the slab 256 blocks cost 1 us more).
__host__ __forceinline__ int place_blocks(const Dev &d)
{
    return (int)std::min<int64_t>(256, std::max<int64_t>(64, d.cap_tot >> 21));
}

// Birth ranking and placement, callable by a block of a kernel of their own or by extra
// blocks of the two solve kernels (defined with the births below).
__device__ void group_tile_scan_body(const Dev &d, int t);
template <bool F64>
__device__ void birth_place_body(const Dev &d, int deferred, int advance, int bid, int nblk);

// For the null-collision bound (R11) that the second solve kernel's last block computes: the
// largest |v|^2 of each segment over the stripes of the half the bound uses, one wave per
// segment (a block of kSolveThreads covers kSolveThreads / kWave segments), so that block
// reads one value per segment.  That half holds the previous step's maxima: the current
// one, or with the previous step's births still to be placed (`pending`), the other one,
// which their placement makes current.
__device__ void vmax_reduce_body(const Dev &d, int pending, int bid)
{
    const int half = pending ? 1 - *d.vcur : *d.vcur;
    const int sg = bid * (kSolveThreads / kWave) + (int)threadIdx.x / kWave;
    if (sg >= d.nseg) return;
    const double m2 = seg_vmax2(d, sg, half);
    if (lane_id() == 0) d.vmred[sg] = m2;
}

// Blocks [0, nchunks) solve; with `nscan` > 0, that many more blocks scan the group counts
// of the previous step's births (independent data; one tile each), so that scan costs no
// launch of its own; `nred` more blocks reduce the speed maxima for the null-collision bound
// (vmax_reduce_body).
template <bool F64>
__global__ void __launch_bounds__(kSolveThreads) k_solve1(Dev d, int nchunks, int nscan, int nred)
{
    if ((int)blockIdx.x >= nchunks) {
        const int r = (int)blockIdx.x - nchunks;
        if (r < nscan)
            group_tile_scan_body(d, r);
        else if (r - nscan < nred)
            vmax_reduce_body(d, nscan > 0, r - nscan);
        return;
    }
    __shared__ double s_buf[8];
    const int64_t k = blockIdx.x;
    const int ei = chunk_ens(d, k);
    const EnsC e = d.ens[ei];
    const int64_t N = e.ncells, nn = e.nnodes;
    const int64_t a = (k - e.chunk0) * kChunk;
    const int64_t j0 = a + (int64_t)threadIdx.x * kNodesPerThread;
    double loc = 0.0, sumpre = 0.0, totq = 0.0, n1 = 0.0, dd = 0.0, cnt = 0.0;
    // thread-local prefix of interior rho and its running sum
    double rho_loc[kNodesPerThread];
    double rho_first = 0.0;  // rho of the chunk's first node (thread 0), for the next chunk's solve
    // smoothing (R23): the chunk's raw densities and a halo of p nodes each side, folded
    // onto the grid, staged in LDS with coalesced loads; s_raw[i] is node a - p + i
    __shared__ double s_raw[kChunk + 2 * kMaxSmooth];
    const int p = e.smooth;
    double rq[kNodesPerThread];
    if (p > 0) {
        constexpr int kStage = (kChunk + 2 * kMaxSmooth + kSolveThreads - 1) / kSolveThreads;
        int64_t jm[kStage];
        bool ok[kStage];
        double rr[kStage];
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int i = threadIdx.x + u * kSolveThreads;
            const int64_t m = a - p + i;
            ok[u] = i < kChunk + 2 * p && m <= nn - 1 + p;
            jm[u] = ok[u] ? smooth_fold(e, m) : 0;
        }
        node_rho_raw<F64, kStage>(d, e, jm, ok, rr);
#pragma unroll
        for (int u = 0; u < kStage; ++u) {
            const int i = threadIdx.x + u * kSolveThreads;
            if (i < kChunk + 2 * p) s_raw[i] = rr[u];
        }
        __syncthreads();
        const double pscale = 1.0 / (double)(1 << (2 * p));
#pragma unroll
        for (int q = 0; q < kNodesPerThread; ++q) {
            double r = 0.0;
            double c = 1.0;  // C(2p, k), exact in binary64
            const int i0 = (int)(j0 + q - a);
            for (int k = 0; k <= 2 * p; ++k) {
                r += c * s_raw[i0 + k];
                c = c * (double)(2 * p - k) / (double)(k + 1);
            }
            rq[q] = r * pscale;
        }
    } else {
        int64_t jq[kNodesPerThread];
        bool ok[kNodesPerThread];
#pragma unroll
        for (int q = 0; q < kNodesPerThread; ++q) {
            jq[q] = j0 + q;
            ok[q] = jq[q] < nn;
        }
        node_rho_raw<F64, kNodesPerThread>(d, e, jq, ok, rq);
    }
#pragma unroll
    for (int q = 0; q < kNodesPerThread; ++q) {
        const int64_t j = j0 + q;
        double r = 0.0;
        if (j < nn) {
            r = rq[q];
            d.rho[e.gbase + j] = r;
            totq += r * node_vol(e, j);
        }
        if (q == 0) rho_first = r;
        rho_loc[q] = (j >= 1 && j <= N - 1) ? r : 0.0;
        loc += rho_loc[q];
    }
    const double excl = block_incl_scan(loc, s_buf) - loc;
    // integer counts in this thread's node range: interior nodes and the prefix weights
    double run = excl;
    int64_t c1_before = 0;  // interior nodes in [a, j0)
    {
        const int64_t lo = max(a, (int64_t)1), hi = min(j0, N);  // [lo, hi) interior, i < j0
        c1_before = hi > lo ? hi - lo : 0;
    }
    int64_t c1 = c1_before;
#pragma unroll
    for (int q = 0; q < kNodesPerThread; ++q) {
        const int64_t j = j0 + q;
        run += rho_loc[q];
        if (j >= 1 && j <= N - 1) {
            ++c1;
            n1 += 1.0;
        }
        if (j < N) {  // m in [0, N-1]
            sumpre += run;
            dd += (double)c1;
            cnt += 1.0;
        }
    }
    // the ensemble's max |E| is accumulated by the second pass's blocks (atomic max)
    if (k == e.chunk0 && threadIdx.x == 0) d.emax[ei] = 0.0;
    __shared__ double s_red[6 * 16];
    double v[6] = {loc, sumpre, totq, n1, dd, cnt};
    block_sums<6>(v, s_red);
    if (threadIdx.x == 0) {
        double *g = d.agg + k * A_NAGG;
        g[A_SUMRHO] = v[0];
        g[A_SUMPRE] = v[1];
        g[A_TOTQ] = v[2];
        g[A_N1] = v[3];
        g[A_D] = v[4];
        g[A_CNT] = v[5];
        g[A_RHO0] = rho_first;
    }
}

// Reading R11: per-segment null-collision bound from the current max speed and max field.
// One wave per segment (lanes read the striped speed maxima); every lane gets the result.
__device__ void compute_params(const Dev &d)
{
    const int nw = blockDim.x / kWave, w = threadIdx.x / kWave;
    const int half = *d.vcur;
    for (int sg = w; sg < d.nseg; sg += nw) {
        double numax, pnull;
        seg_params(d, sg, half, d.emax[d.seg[sg].ens], numax, pnull);
        if (lane_id() == 0) {
            d.numax[sg] = numax;
            d.pnull[sg] = pnull;
        }
    }
}

// The same bound in the last block of the second solve kernel, one thread per segment from
// the maxima the first kernel reduced: max |E| was accumulated by other blocks of the same
// launch, so it is read with an atomic, which sees every block's atomic update without a
// fence, and every segment's loads go out at once.
__device__ void compute_params_reduced(const Dev &d)
{
    for (int sg = threadIdx.x; sg < d.nseg; sg += blockDim.x) {
        const SegC &S = d.seg[sg];
        const double m2 = d.vmred[sg];
        const double emax =
            __longlong_as_double((long long)atomicMax((unsigned long long *)(d.emax + S.ens), 0ull));
        double numax, pnull;
        seg_bound(S, d.ens[S.ens], m2, emax, numax, pnull);
        d.numax[sg] = numax;
        d.pnull[sg] = pnull;
    }
}

__global__ void k_params(Dev d) { compute_params(d); }

// Inclusive prefix sum over the 64 lanes of a wave (FP64).
__device__ __forceinline__ double wave_incl_scan_f64(double v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double n = __shfl_up(v, o);
        if (lane >= o) v += n;
    }
    return v;
}

template <bool F64>
__device__ void solve2_body(const Dev &d, int zero_q)
{
    __shared__ double s_buf[8];
    __shared__ double s_E[F64 ? 1 : kChunk + 1];  // the chunk's node E, for the gather table
    __shared__ double s_C0, s_F0, s_Eh, s_bg, s_Ctot;
    const int64_t k = blockIdx.x;
    const int ei = chunk_ens(d, k);
    const EnsC e = d.ens[ei];
    const int64_t N = e.ncells, nn = e.nnodes;
    const int64_t a = (k - e.chunk0) * kChunk;
    const double dx = e.dx, ce = e.dx / e.eps0;
    const int64_t j0 = a + (int64_t)threadIdx.x * kNodesPerThread;
    // this thread's densities (written by the first pass), loaded before the chunk scan so
    // the two round trips overlap
    double rv[kNodesPerThread];
#pragma unroll
    for (int q = 0; q < kNodesPerThread; ++q) {
        const bool in = j0 + q < nn;
        const double v = d.rho[e.gbase + (in ? j0 + q : 0)];
        rv[q] = in ? v : 0.0;
    }
    // Scan of the ensemble's chunk aggregates by the first wave, in parallel: lane l owns
    // the contiguous chunk range [l R, (l+1) R).  C_pre(c) = sum_{c'<c} A'(c') and
    // F_pre(c) = sum_{c'<c} (cnt(c') C_pre(c') + B'(c')) are two nested exclusive scans.
    // (Wave shuffles only: no block barrier inside the scan.)
    if (threadIdx.x < kWave) {
        const int lane = (int)threadIdx.x;
        const int64_t nc = e.nchunks;
        const int64_t R = (nc + kWave - 1) / kWave;
        const int64_t c0 = (int64_t)lane * R, c1 = min(c0 + R, nc);
        // floating walls (R22): the particles absorbed so far at the left wall, per
        // species, from the exact striped wall counts (sums < 2^53: exact in binary64)
        // (species loops run over the two array entries with constant indices, so that the
        // local copy of the ensemble stays in registers)
        double nabs[2] = {0.0, 0.0};
        if (e.floating)
            for (int st = lane; st < kCntStripes; st += kWave) {
#pragma unroll
                for (int s = 0; s < 2; ++s)
                    if (s < e.nspecies)
                        nabs[s] += (double)d.cnt[((int64_t)st * d.nseg + e.seg[s]) * C_NCNT + C_WALL_L];
            }
        double tq = 0.0;
        for (int64_t c = c0; c < c1; ++c) tq += d.agg[(e.chunk0 + c) * A_NAGG + A_TOTQ];
        const double tqs = wave_sum_f64(tq);
        const double bg = e.periodic ? -tqs / e.L : 0.0;
        double a = 0.0, g = 0.0, n = 0.0;  // local A sum, local sum of cnt*Cpre_local + B, cnt sum
        for (int64_t c = c0; c < c1; ++c) {
            const double *gg = d.agg + (e.chunk0 + c) * A_NAGG;
            const double A = gg[A_SUMRHO] + bg * gg[A_N1];
            const double B = gg[A_SUMPRE] + bg * gg[A_D];
            g += gg[A_CNT] * a + B;
            n += gg[A_CNT];
            a += A;
        }
        const double apre = wave_incl_scan_f64(a) - a;  // C_pre at c0
        const double fin = n * apre + g;                // this range's sum of C over m
        const double fpre = wave_incl_scan_f64(fin) - fin;
        const double Stot = wave_sum_f64(fin), Ctot = wave_sum_f64(a);
        const double nab0 = wave_sum_f64(nabs[0]), nab1 = wave_sum_f64(nabs[1]);
        const int64_t me = k - e.chunk0;
        if (me >= c0 && me < c1) {
            double ca = apre, fa = fpre;
            for (int64_t c = c0; c < me; ++c) {
                const double *gg = d.agg + (e.chunk0 + c) * A_NAGG;
                const double A = gg[A_SUMRHO] + bg * gg[A_N1];
                const double B = gg[A_SUMPRE] + bg * gg[A_D];
                fa += gg[A_CNT] * ca + B;
                ca += A;
            }
            s_C0 = ca;
            s_F0 = fa;
        }
        // Reading R22: floating walls fix E_{1/2} by Gauss's law over the left wall (the
        // charge absorbed there, q w per particle) and the half cell in front of it;
        // otherwise phi_N = 0 (or periodicity) fixes it.
        const double sigL = e.qw[0] * nab0 + (e.nspecies > 1 ? e.qw[1] * nab1 : 0.0);
        if (lane == 0) {
            s_bg = bg;
            s_Ctot = Ctot;
            if (e.floating)
                s_Eh = (sigL + d.agg[e.chunk0 * A_NAGG + A_RHO0] * node_vol(e, 0)) / e.eps0;
            else
                s_Eh = -ce * Stot / (double)N;
        }
    }
    __syncthreads();
    const double bg = s_bg, Eh = s_Eh;
    // local inclusive prefix of interior rho' (with background) -> C_j
    double rl[kNodesPerThread + 1];
    double loc = 0.0;
#pragma unroll
    for (int q = 0; q < kNodesPerThread; ++q) {
        const int64_t j = j0 + q;
        double r = 0.0;
        if (j < nn) {
            const double rj = rv[q] + bg;
            if (e.periodic) d.rho[e.gbase + j] = rj;  // report rho with the background
            if (j >= 1 && j <= N - 1) r = rj;
        }
        rl[q] = r;
        loc += r;
    }
    const double cex = block_incl_scan(loc, s_buf) - loc;
    double Cj[kNodesPerThread];
    double c = s_C0 + cex;
    double csum = 0.0;
#pragma unroll
    for (int q = 0; q < kNodesPerThread; ++q) {
        c += rl[q];
        Cj[q] = c;
        csum += (j0 + q < N) ? c : 0.0;
    }
    // exclusive prefix of C over m < j (m in [0, N-1])
    const double fex = block_incl_scan(csum, s_buf) - csum;
    double F = s_F0 + fex;
    double emax = 0.0, phisum = 0.0, fe = 0.0;
    int nonfin = 0;
    // C_{j-1} for the first node of the thread
    double Cprev = (j0 == 0) ? 0.0 : (Cj[0] - rl[0]);
#pragma unroll
    for (int q = 0; q < kNodesPerThread; ++q) {
        const int64_t j = j0 + q;
        if (j >= nn) break;
        double phi = -dx * ((double)j * Eh + ce * F);
        if (!e.periodic && !e.floating && j == N) phi = 0.0;
        if (j == 0) phi = 0.0;
        d.phi[e.gbase + j] = phi;
        phisum += phi;
        // face fields around node j
        const double Em = Eh + ce * Cprev;  // E_{j-1/2} (j >= 1)
        const double Ep = Eh + ce * Cj[q];  // E_{j+1/2} (j <= N-1)
        double Ej;
        if (e.periodic) {
            if (j == 0) {
                const double Elast = Eh + ce * s_Ctot;  // E_{N-1/2}
                Ej = 0.5 * (Elast + Ep);
            } else {
                Ej = 0.5 * (Em + Ep);
            }
        } else if (j == 0) {
            Ej = Eh - d.rho[e.gbase] * node_vol(e, 0) / e.eps0;
        } else if (j == N) {
            Ej = Em + d.rho[e.gbase + N] * node_vol(e, N) / e.eps0;
        } else {
            Ej = 0.5 * (Em + Ep);
        }
        d.E[e.gbase + j] = Ej;
        if constexpr (!F64) s_E[j - a] = Ej;
        if (!isfinite(Ej)) nonfin = 1;
        emax = fmax(emax, fabs(Ej));
        fe += Ej * Ej * node_vol(e, j);
        if (j < N) F += Cj[q];
        Cprev = Cj[q];
    }
    if constexpr (!F64) {
        // Gather table of the chunk's cells, (E_j, E_{j+1} - E_j) in binary32.  The node
        // after the chunk's last cell is the periodic wrap E_0, or the next chunk's first
        // node, computed here from this chunk's last C and that node's rho (kept by the
        // first solve pass, since the next chunk rewrites it with the background).
        const int64_t L = min((int64_t)kChunk, N - a);
        if (L > 0) {
            if (e.periodic && a + L == N) {
                if (threadIdx.x == 0) s_E[L] = 0.5 * ((Eh + ce * s_Ctot) + (Eh + ce * 0.0));
            } else if (L == kChunk && threadIdx.x == blockDim.x - 1) {
                const int64_t jn = a + kChunk;
                const double rn = d.agg[(k + 1) * A_NAGG + A_RHO0];
                const double Cl = Cj[kNodesPerThread - 1];  // C_{jn-1}
                const double Em = Eh + ce * Cl;
                if (!e.periodic && jn == N) {
                    s_E[L] = Em + rn * node_vol(e, N) / e.eps0;
                } else {
                    const double Cn = Cl + (rn + bg);
                    s_E[L] = 0.5 * (Em + (Eh + ce * Cn));
                }
            }
        }
        __syncthreads();
        for (int64_t j = a + threadIdx.x; j < a + L; j += blockDim.x) {
            const double E0 = s_E[j - a], E1 = s_E[j - a + 1];
            d.Ecell[e.gbase + j] = make_float2((float)E0, (float)(E1 - E0));
        }
    }
    // zero the deposit for the next pass when asked (fused step)
    if (zero_q) {
        for (int q = 0; q < kNodesPerThread; ++q) {
            const int64_t j = j0 + q;
            if (j >= nn) break;
            for (int s = 0; s < e.nspecies; ++s) {
                if constexpr (!F64)
                    d.Qi[(int64_t)s * d.nodes_tot + e.gbase + j] = 0ull;
                else
                    d.Qd[(int64_t)s * d.nodes_tot + e.gbase + j] = 0.0;
            }
        }
    }
    // chunk partials
    {
        double em = wave_max_f64(emax);
        __shared__ double s_em[8];
        if (lane_id() == 0) s_em[threadIdx.x / kWave] = em;
        __syncthreads();
        if (threadIdx.x == 0) {
            for (int i = 1; i < (int)(blockDim.x / kWave); ++i) em = fmax(em, s_em[i]);
            s_em[0] = em;
        }
        __syncthreads();
        em = s_em[0];
        __shared__ double s_red3[3 * 16];
        double fv[3] = {phisum, (double)nonfin, fe};
        block_sums<3>(fv, s_red3);
        if (threadIdx.x == 0) {
            d.part[k * P_NPART + P_PHISUM] = fv[0];
            d.part[k * P_NPART + P_FE] = 0.5 * e.eps0 * fv[2];  // this chunk's field energy
            // |E| >= 0: its bit pattern orders as an unsigned integer
            atomicMax((unsigned long long *)(d.emax + ei), dbits(em));
            if (fv[1] > 0.0) atomicOr(d.err, (int)E_NONFINITE);
        }
    }
}

// Blocks [0, nchunks) solve; blocks beyond place the previous step's births (they touch
// particle slots beyond the ones in use, the id and slot counters, the birth lists, the
// speed-maximum halves and the step counter, none of which the solve reads or writes).
// With `params`, the last block to finish computes the next pass's null-collision bound
// (R11) from this solve's max |E| and the speed maxima the first kernel reduced, in place of
// a kernel of its own; it reads max |E|, which other blocks of this launch updated, through
// an atomic, which needs no fence.
template <bool F64>
__global__ void __launch_bounds__(kSolveThreads) k_solve2(Dev d, int zero_q, int nchunks, int params)
{
    if ((int)blockIdx.x >= nchunks)
        birth_place_body<F64>(d, 1, 1, (int)blockIdx.x - nchunks, (int)gridDim.x - nchunks);
    else
        solve2_body<F64>(d, zero_q);
    if (!params) return;
    __shared__ bool s_last;
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(d.ticket + 6, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last) return;
    compute_params_reduced(d);
    if (threadIdx.x == 0) d.ticket[6] = 0u;
}

// Periodic only: subtract the mean of phi and build the gather table.
__global__ void __launch_bounds__(kSolveThreads) k_phi_shift(Dev d)
{
    const int64_t k = blockIdx.x;
    const int ei = chunk_ens(d, k);
    const EnsC e = d.ens[ei];
    __shared__ double s_mean;
    if (threadIdx.x < kWave) {
        double ps = 0.0;
        for (int64_t c = threadIdx.x; c < e.nchunks; c += kWave) ps += d.part[(e.chunk0 + c) * P_NPART + P_PHISUM];
        ps = wave_sum_f64(ps);
        if (threadIdx.x == 0) s_mean = ps / (double)e.ncells;
    }
    __syncthreads();
    const int64_t a = (k - e.chunk0) * kChunk;
    for (int64_t j = a + threadIdx.x; j < min(a + kChunk, e.nnodes); j += blockDim.x)
        d.phi[e.gbase + j] -= s_mean;
}

// Gather table: per cell (E_j, E_{j+1} - E_j) in float.
__global__ void k_ecell(Dev d)
{
    const int64_t k = blockIdx.x;
    const int ei = chunk_ens(d, k);
    const EnsC e = d.ens[ei];
    const int64_t a = (k - e.chunk0) * kChunk;
    for (int64_t j = a + threadIdx.x; j < min(a + kChunk, e.ncells); j += blockDim.x) {
        const int64_t j1 = (e.periodic && j + 1 == e.ncells) ? 0 : j + 1;
        const double E0 = d.E[e.gbase + j], E1 = d.E[e.gbase + j1];
        d.Ecell[e.gbase + j] = make_float2((float)E0, (float)(E1 - E0));
    }
}

// Field energy 1/2 eps0 sum_j E_j^2 V_j of every ensemble (for the diagnostics and the
// adjoint objective; one wave per ensemble).
__global__ void __launch_bounds__(1024) k_field_energy(Dev d)
{
    __shared__ double s_buf[16];
    const EnsC e = d.ens[blockIdx.x];  // one block per ensemble
    double f = 0.0;
    for (int64_t j = threadIdx.x; j < e.nnodes; j += blockDim.x) {
        const double E = d.E[e.gbase + j];
        f += E * E * node_vol(e, j);
    }
    double v[1] = {f};
    block_sums<1>(v, s_buf);
    if (threadIdx.x == 0) d.fe[blockIdx.x] = 0.5 * e.eps0 * v[0];
}

// Max |E| and field energy of a field set from the host (test hook).
__global__ void __launch_bounds__(kSolveThreads) k_field_stats(Dev d)
{
    __shared__ double s_buf[8];
    for (int en = 0; en < d.nens; ++en) {
        const EnsC &e = d.ens[en];
        double em = 0.0, fe = 0.0;
        for (int64_t j = threadIdx.x; j < e.nnodes; j += blockDim.x) {
            const double E = d.E[e.gbase + j];
            em = fmax(em, fabs(E));
            fe += E * E * node_vol(e, j);
        }
        em = wave_max_f64(em);
        __shared__ double s_em[8];
        if (lane_id() == 0) s_em[threadIdx.x / kWave] = em;
        __syncthreads();
        const double f = block_sum(fe, s_buf);
        if (threadIdx.x == 0) {
            for (int i = 1; i < (int)(blockDim.x / kWave); ++i) em = fmax(em, s_em[i]);
            d.emax[en] = em;
            d.fe[en] = 0.5 * e.eps0 * f;
        }
        __syncthreads();
    }
}

template <bool F64>
__global__ void k_zero_q(Dev d)
{
    const int64_t n = 2 * d.nodes_tot;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if constexpr (!F64)
            d.Qi[i] = 0ull;
        else
            d.Qd[i] = 0.0;
    }
}

// =======================================================================================
// Generic exclusive scan of u32 (three kernels: block sums, scan of sums, down-sweep).
// =======================================================================================
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ uint32_t block_excl_scan_u32(uint32_t v, uint32_t *s_buf, uint32_t &total)
{
    const int lane = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t n = __shfl_up(x, o);
        if (lane >= o) x += n;
    }
    if (lane == kWave - 1) s_buf[w] = x;
    __syncthreads();
    uint32_t add = 0, tot = 0;
    for (int i = 0; i < nw; ++i) {
        if (i < w) add += s_buf[i];
        tot += s_buf[i];
    }
    __syncthreads();
    total = tot;
    return x - v + add;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_sums(const uint32_t *in, int64_t n, uint32_t *part,
                                                          const int64_t *parity_step)
{
    if (parity_step) in += (int64_t)(*parity_step & 1) * n;
    __shared__ uint32_t s_buf[16];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        const int64_t i = base + (int64_t)q * kScanBlock + threadIdx.x;
        if (i < n) s += in[i];
    }
    uint32_t tot;
    block_excl_scan_u32(s, s_buf, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_part(uint32_t *part, int64_t nb)
{
    __shared__ uint32_t s_buf[16];
    __shared__ uint32_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (int64_t c = 0; c < nb; c += blockDim.x) {
        const int64_t i = c + threadIdx.x;
        const uint32_t v = i < nb ? part[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan_u32(v, s_buf, tot);
        if (i < nb) part[i] = ex + s_carry;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_down(uint32_t *in, uint32_t *out, int64_t n,
                                                          const uint32_t *part, int zero_in,
                                                          const int64_t *parity_step)
{
    if (parity_step) in += (int64_t)(*parity_step & 1) * n;
    __shared__ uint32_t s_buf[16];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // each thread owns kScanItems consecutive elements
    const int64_t i0 = base + (int64_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = (i0 + q < n) ? in[i0 + q] : 0u;
        s += v[q];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan_u32(s, s_buf, tot) + part[blockIdx.x];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (i0 + q < n) {
            out[i0 + q] = ex;
            if (zero_in) in[i0 + q] = 0u;
        }
        ex += v[q];
    }
}

// =======================================================================================
// Births: a birth's rank among its ensemble's births of the step is the scanned count of
// the id groups below its own plus the bits below it in its group's 128 bitmap words.  The
// new electron and ion go to slot n_slots + rank with id next_id + rank.  The last block
// updates the counters.
// =======================================================================================
__device__ __forceinline__ void birth_locate(const Dev &d, int64_t k, int &st, uint32_t &idx,
                                             const uint32_t *s_pre)
{
    int lo = 0, hi = kStripes;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((int64_t)s_pre[mid] <= k)
            lo = mid;
        else
            hi = mid;
    }
    st = lo;
    idx = (uint32_t)(k - s_pre[lo]);
}

// Exclusive prefix of the per-stripe birth counts (clamped to the stripe capacity), with the
// total in s_pre[kStripes].  Called by the first wave of the block.
__device__ __forceinline__ void stripe_prefix(const BirthBuf &bb, int64_t cap, uint32_t *s_pre)
{
    const int lane = lane_id();
    const uint32_t v = lane < kStripes ? (uint32_t)min((int64_t)bb.nbirth[lane], cap) : 0u;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t n = __shfl_up(inc, o);
        if (lane >= o) inc += n;
    }
    if (lane < kStripes) s_pre[lane] = inc - v;
    if (lane == kStripes - 1) s_pre[kStripes] = inc;
}

// Bits of the group's bitmap below `pid` (the group's words are 128-byte aligned); the
// words are read as independent 16-byte loads four at a time.
__device__ __forceinline__ uint32_t rank_in_group(const uint32_t *group, uint32_t pid)
{
    static_assert(kGroupWords % 64 == 0, "whole batches of 64 words per group");
    const int wp = (int)((pid % kGroupIds) >> 5);  // words wholly below pid
    const uint4 *v = (const uint4 *)group;
    uint32_t r = __popc(group[wp] & ((1u << (pid & 31)) - 1u));
    // batches of 64 words, each batch's sixteen 16-byte loads in flight at once; words at
    // or above wp are masked
    for (int w0 = 0; w0 < wp; w0 += 64) {
        uint4 a[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) a[u] = v[w0 / 4 + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int w = w0 + 4 * u;
            r += (w < wp ? __popc(a[u].x) : 0u) + (w + 1 < wp ? __popc(a[u].y) : 0u) +
                 (w + 2 < wp ? __popc(a[u].z) : 0u) + (w + 3 < wp ? __popc(a[u].w) : 0u);
        }
    }
    return r;
}

// Exclusive scan of the current half's group counts, one tile of kGroupTile groups per block:
// gpre gets each group's prefix within its tile and gtile the tile's total (the placement
// adds the tiles' bases).  Wave w owns the w-th contiguous share of the tile, whole rows of
// 64 16-byte vectors, and reads it row by row, lane l taking the row's l-th vector, so every
// load instruction reads 1 KB of consecutive bytes; the share's rows are all loaded before
// any is used (one round trip), summed, the shares' bases exchanged in LDS, and each row
// scanned across the wave and written.  (One block over every group, per-thread runs read
// four vectors at a time, had taken 60 us for the 64 batched ensembles' 1.3e5 groups.)
constexpr int kTileVec = kGroupTile / 4;  // uint4 per tile

// (a block of 256 threads: four waves of kRows rows each)
__device__ void group_tile_scan_body(const Dev &d, int t)
{
    constexpr int kRows = kTileVec / (kWave * 4);
    __shared__ uint32_t s_w[4];
    const int p = (int)(*d.step & 1);
    const int w = (int)threadIdx.x / kWave, lane = lane_id();
    const int64_t v0 = (int64_t)t * kTileVec + (int64_t)w * kRows * kWave;
    const uint4 *in = (const uint4 *)(d.gcnt + (int64_t)p * d.g_tot) + v0;
    uint4 *out = (uint4 *)d.gpre + v0;
    uint4 v[kRows];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kRows; ++r) v[r] = in[r * kWave + lane];
#pragma unroll
    for (int r = 0; r < kRows; ++r) sum += v[r].x + v[r].y + v[r].z + v[r].w;
    sum = wave_sum_u32(sum);
    if (lane == 0) s_w[w] = sum;
    __syncthreads();
    uint32_t carry = 0;  // counts of the tile before this wave's share, then before the row
    for (int i = 0; i < w; ++i) carry += s_w[i];
    if (threadIdx.x == 0) d.gtile[t] = s_w[0] + s_w[1] + s_w[2] + s_w[3];
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
        const uint32_t ls = v[r].x + v[r].y + v[r].z + v[r].w;
        uint32_t inc = ls;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t n = __shfl_up(inc, o);
            if (lane >= o) inc += n;
        }
        const uint32_t ex = carry + inc - ls;
        out[r * kWave + lane] = make_uint4(ex, ex + v[r].x, ex + v[r].x + v[r].y, ex + v[r].x + v[r].y + v[r].z);
        carry += __shfl(inc, kWave - 1);
    }
}

__global__ void __launch_bounds__(256) k_group_scan(Dev d) { group_tile_scan_body(d, (int)blockIdx.x); }

// Place the births of this step (half p = step & 1).  With `deferred`, also clear the
// bitmap bits and group counts of half 1 - p (the previous step's births) and reset its
// birth counts, so the next step starts on a clean half.  The last block updates the
// counters, makes the freshly accumulated speed maxima current and (with `advance`)
// advances the step counter.
// The constants a birth's placement needs, staged in LDS by every placing block (one round
// trip, beside the stripe counts), so that a birth's chain of dependent loads is its record
// and then its rank: per ensemble the birth-ranking bases, id capacity and segments, per
// segment the slot base and capacity and the slots and ids in use before the placement.
struct PlaceEns {
    int64_t bm_base, grp_base, idcap;
    int32_t seg[2];
    int32_t nspecies;
};
struct PlaceSeg {
    int64_t base, cap, n_slots;
    uint32_t next_id;
};

// Bases of the group-count tiles (exclusive prefix of gtile) in LDS, by the whole block of
// 256 threads (four tiles each); all zero when the global scan ran (ngt = 0).
static_assert(kSolveThreads == 256, "the solve kernels' births blocks have 256 threads, as k_birth_place");
__device__ void stage_tile_bases(const Dev &d, uint32_t *s_tb)
{
    __shared__ uint32_t s_buf[16];
    constexpr int kPer = kMaxGroupTiles / 256;
    const int i0 = (int)threadIdx.x * kPer;
    uint32_t v[kPer], sum = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        v[u] = (i0 + u < d.ngt) ? d.gtile[i0 + u] : 0u;
        sum += v[u];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan_u32(sum, s_buf, tot);
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        s_tb[i0 + u] = ex;
        ex += v[u];
    }
}

// The births' scanned group count at group index i (global over every ensemble's groups).
__device__ __forceinline__ uint32_t group_prefix(const Dev &d, const uint32_t *s_tb, int64_t i)
{
    return s_tb[i / kGroupTile] + d.gpre[i];
}

template <bool F64>
__device__ void birth_place_body(const Dev &d, int deferred, int advance, int bid, int nblk)
{
    __shared__ uint32_t s_pre[kStripes + 1];
    __shared__ uint32_t s_old[kStripes + 1];
    __shared__ uint32_t s_tb[kMaxGroupTiles];
    __shared__ bool s_last;
    __shared__ PlaceEns s_pe[PIC_MAX_ENSEMBLES];
    __shared__ PlaceSeg s_ps[2 * PIC_MAX_ENSEMBLES];
    const int64_t step = *d.step;
    const int vc = *d.vcur;
    const int p = (int)(step & 1);
    const BirthBuf bb = birth_buf(d, p), ob = birth_buf(d, 1 - p);
    if (threadIdx.x < kWave) {
        stripe_prefix(bb, d.birth_stripe_cap, s_pre);
        if (deferred) stripe_prefix(ob, d.birth_stripe_cap, s_old);
    }
    for (int en = threadIdx.x; en < d.nens; en += blockDim.x) {
        const EnsC &e = d.ens[en];
        s_pe[en] = PlaceEns{e.bm_base, e.grp_base, e.idcap, {e.seg[0], e.seg[1]}, e.nspecies};
    }
    for (int sg = threadIdx.x; sg < d.nseg; sg += blockDim.x) {
        const SegC &S = d.seg[sg];
        s_ps[sg] = PlaceSeg{S.base, S.cap, d.n_slots[sg], d.next_id[sg]};
    }
    stage_tile_bases(d, s_tb);
    __syncthreads();
    const int64_t M = s_pre[kStripes], Mo = deferred ? (int64_t)s_old[kStripes] : 0;
    const int b = *d.cur;
    // this step's births (k < M) and, with `deferred`, the previous step's (k < Mo), whose
    // bits and group counts are cleared; both records are loaded before either is used
    for (int64_t k = (int64_t)bid * blockDim.x + threadIdx.x; k < max(M, Mo);
         k += (int64_t)nblk * blockDim.x) {
        const bool nw = k < M, od = k < Mo;
        int st = 0, sto = 0;
        uint32_t idx = 0, idxo = 0;
        if (nw) birth_locate(d, k, st, idx, s_pre);
        if (od) birth_locate(d, k, sto, idxo, s_old);
        // copies: the particle stores below cannot alias them, so nothing is read twice
        Birth B{};
        uint2 okey = make_uint2(0u, 0u);
        if (nw) B = bb.births[(int64_t)st * d.birth_stripe_cap + idx];
        if (od) okey = *(const uint2 *)&ob.births[(int64_t)sto * d.birth_stripe_cap + idxo];
        if (od) {
            const PlaceEns &E = s_pe[okey.y];
            ob.bitmap[E.bm_base + (okey.x >> 5)] = 0u;
            ob.gcnt[E.grp_base + okey.x / kGroupIds] = 0u;
        }
        if (!nw) continue;
        const PlaceEns &E = s_pe[B.ens];
        const uint32_t pid = B.pid;
        const int64_t g = pid / kGroupIds;
        const uint32_t r = group_prefix(d, s_tb, E.grp_base + g) - group_prefix(d, s_tb, E.grp_base) +
                           rank_in_group(bb.bitmap + E.bm_base + g * kGroupWords, pid);
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            if (s >= E.nspecies) break;
            const PlaceSeg &P = s_ps[E.seg[s]];
            const int64_t slot = P.n_slots + r;
            if (slot >= P.cap) {
                atomicOr(d.err, (int)E_CAP_PART);
                continue;
            }
            if ((int64_t)P.next_id + r >= E.idcap) {
                atomicOr(d.err, (int)E_CAP_ID);
                continue;
            }
            const int64_t i = P.base + slot;
            const double v0 = s == 0 ? B.ve[0] : B.vi[0];
            const double v1 = s == 0 ? B.ve[1] : B.vi[1];
            const double v2 = s == 0 ? B.ve[2] : B.vi[2];
            if constexpr (!F64) {
                d.cell[b][i] = B.cell;
                d.off[b][i] = B.off;
                d.fvx[b][i] = (float)v0;
                d.fvy[b][i] = (float)v1;
                d.fvz[b][i] = (float)v2;
            } else {
                d.x[b][i] = B.x;
                d.dvx[b][i] = v0;
                d.dvy[b][i] = v1;
                d.dvz[b][i] = v2;
            }
            d.id[b][i] = P.next_id + r;
        }
    }
    // The last block only updates counters that no block of this launch reads after taking
    // its ticket (each block staged them before its first barrier), and the next kernel
    // sees every write, so no device-scope fence is needed here; on gfx950 such a fence
    // writes back the XCD's L2 and costs microseconds per block.
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(d.ticket + 1, 1u) == (unsigned)(nblk - 1));
    __syncthreads();
    if (!s_last) return;
    for (int en = threadIdx.x; en < d.nens; en += blockDim.x) {
        const PlaceEns &E = s_pe[en];
        const int64_t ngrp = (E.idcap + kGroupIds - 1) / kGroupIds;
        const uint32_t m = group_prefix(d, s_tb, E.grp_base + ngrp) - group_prefix(d, s_tb, E.grp_base);
        for (int s = 0; s < E.nspecies; ++s) {
            const int sg = E.seg[s];
            const PlaceSeg &P = s_ps[sg];
            d.n_slots[sg] = min(P.n_slots + (int64_t)m, P.cap);
            d.next_id[sg] = P.next_id + m;
            if (m) atomicAdd(d.cnt + ((int64_t)0 * d.nseg + sg) * C_NCNT + C_CREATED, (unsigned long long)m);
        }
    }
    if (deferred)
        for (int i = threadIdx.x; i < kStripes; i += blockDim.x) ob.nbirth[i] = 0u;
    if (threadIdx.x == 0) {
        d.ticket[1] = 0u;
        atomicExch(d.vcur, 1 - vc);  // atomic: the bound may be computed in this launch
    }
    // the half that held the current maxima accumulates the next step's, and the step
    // tallies of that half restart
    for (int64_t i = threadIdx.x; i < (int64_t)kCntStripes * d.nseg; i += blockDim.x)
        d.vmax2[(int64_t)vc * kCntStripes * d.nseg + i] = 0ull;
    for (int64_t i = threadIdx.x; i < (int64_t)kCntStripes * d.nseg * T_NSTEP; i += blockDim.x)
        d.ssum[(int64_t)vc * kCntStripes * d.nseg * T_NSTEP + i] = 0.0;
    if (threadIdx.x == 0 && advance) *d.step = step + 1;
}

template <bool F64>
__global__ void __launch_bounds__(256) k_birth_place(Dev d, int deferred, int advance)
{
    birth_place_body<F64>(d, deferred, advance, (int)blockIdx.x, (int)gridDim.x);
}

// Clear one half (parity -1: the current step's): its bits and counts, then its birth counts.
__global__ void k_birth_clear(Dev d, int parity)
{
    __shared__ uint32_t s_pre[kStripes + 1];
    __shared__ bool s_last;
    const int p = parity < 0 ? (int)(*d.step & 1) : parity;
    const BirthBuf bb = birth_buf(d, p);
    if (threadIdx.x < kWave) stripe_prefix(bb, d.birth_stripe_cap, s_pre);
    __syncthreads();
    const int64_t M = s_pre[kStripes];
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < M;
         k += (int64_t)gridDim.x * blockDim.x) {
        int st;
        uint32_t idx;
        birth_locate(d, k, st, idx, s_pre);
        const Birth &B = bb.births[(int64_t)st * d.birth_stripe_cap + idx];
        birth_unmark(bb, d.ens[B.ens], B.pid);
    }
    // as in the placement: the last block only resets the counts (no fence needed)
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(d.ticket + 2, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last) return;
    for (int i = threadIdx.x; i < kStripes; i += blockDim.x) bb.nbirth[i] = 0u;
    if (threadIdx.x == 0) d.ticket[2] = 0u;
}

__global__ void k_advance(Dev d)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *d.step += 1;
}

// =======================================================================================
// Counting sort by cell of the FP64 form (the FP32 form runs in k_sort32): the histogram
// is in cellcnt, scanned into cursor (global positions over the concatenated segments).
// Each tile ranks its particles per cell in LDS (wave-leader reservation), reserves one
// run per cell with one HBM atomic, and scatters into the other buffer.  Absorbed slots
// are dropped.
// =======================================================================================
template <int PPT>
__global__ void __launch_bounds__(256) k_sort_scatter(Dev d, int W)
{
    extern __shared__ unsigned long long s_dyn[];
    uint32_t *sCnt = (uint32_t *)s_dyn;   // [W] counts, then bases
    __shared__ int64_t s_tpre[kMaxSeg + 1];
    __shared__ int64_t s_lim[2 * kMaxSeg];
    __shared__ int s_min;
    __shared__ bool s_last;
    const int BLOCK = blockDim.x;
    const int64_t TILE = (int64_t)BLOCK * PPT;
    sched_prefix(d, TILE, s_tpre, s_lim);
    const int64_t T = s_tpre[d.nseg];
    int64_t t0, t1;
    block_run(T, t0, t1);
    const int b = *d.cur, nb = 1 - b;
    const int lane = lane_id();
    for (int i = threadIdx.x; i < W; i += BLOCK) sCnt[i] = 0u;
    __syncthreads();
    for (int64_t t = t0; t < t1; ++t) {
        const int sg = __builtin_amdgcn_readfirstlane(seg_of_tile(s_tpre, d.nseg, t));
        const SegC &S = d.seg[sg];
        const int64_t lt = t - s_tpre[sg];
        const int64_t first = s_lim[2 * sg] + lt * TILE;
        const int64_t last = min(first + TILE, s_lim[2 * sg + 1]);
        // the whole particle is loaded up front (every load in flight at once) and kept in
        // registers until its store to the other buffer
        double xv[PPT], vx[PPT], vy[PPT], vz[PPT];
        uint32_t idv[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int64_t i = first + (int64_t)k * BLOCK + threadIdx.x;
            xv[k] = -1.0;
            if (i < last) {
                xv[k] = d.x[b][i];
                vx[k] = d.dvx[b][i];
                vy[k] = d.dvy[b][i];
                vz[k] = d.dvz[b][i];
                idv[k] = d.id[b][i];
            }
        }
        const Seg64 G = seg64(S, d.ens[S.ens]);
        const int64_t sbase = S.base, scap = S.cap, scb = S.cbase, sstart = d.segstart[sg];
        int cell[PPT];
        uint32_t rank[PPT];
        int mn = INT32_MAX;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            double f;
            cell[k] = (xv[k] >= 0.0) ? (int)cell_of_x64(G, xv[k], f) : kDead;
            if (cell[k] != kDead) mn = min(mn, cell[k]);
        }
        mn = wave_min_i32(mn);
        if (threadIdx.x == 0) s_min = INT32_MAX;
        __syncthreads();
        if (lane == 0) atomicMin(&s_min, mn);
        __syncthreads();
        const int base = s_min;
        // local ranks
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int rel = (cell[k] != kDead) ? cell[k] - base : -1;
            const int key = (rel >= 0 && rel < W) ? rel : -1;
            rank[k] = 0xFFFFFFFFu;
            unsigned long long act = __ballot(key >= 0);
            int it = 0;
            while (act != 0ull && it < 8) {
                const int leader = __ffsll((long long)act) - 1;
                const int kk = __shfl(key, leader);
                const bool mine = (key == kk) && ((act >> lane) & 1ull);
                const unsigned long long m = __ballot(mine);
                uint32_t r0 = 0;
                if (lane == leader) r0 = atomicAdd(&sCnt[kk], (uint32_t)__popcll(m));
                r0 = __shfl(r0, leader);
                if (mine) rank[k] = r0 + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                act &= ~m;
                ++it;
            }
            if ((act >> lane) & 1ull) rank[k] = atomicAdd(&sCnt[key], 1u);
        }
        __syncthreads();
        // reserve runs: counts -> global bases
        for (int i = threadIdx.x; i < W; i += BLOCK) {
            const uint32_t c = sCnt[i];
            if (c) sCnt[i] = atomicAdd(d.cursor + scb + base + i, c);
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (cell[k] == kDead) continue;
            uint32_t pos;
            if (rank[k] != 0xFFFFFFFFu)
                pos = sCnt[cell[k] - base] + rank[k];
            else
                pos = atomicAdd(d.cursor + scb + cell[k], 1u);
            const int64_t o = sbase + (int64_t)pos - sstart;
            if (o < sbase || o >= sbase + scap) {  // histogram and slots disagree
                atomicOr(d.err, (int)E_CAP_PART);
                continue;
            }
            d.x[nb][o] = xv[k];
            d.dvx[nb][o] = vx[k];
            d.dvy[nb][o] = vy[k];
            d.dvz[nb][o] = vz[k];
            d.id[nb][o] = idv[k];
        }
        __syncthreads();
        for (int i = threadIdx.x; i < W; i += BLOCK) sCnt[i] = 0u;
        __syncthreads();
    }
    // The last block sets the slot counts from the cursors, which the other blocks changed
    // with atomics; it reads them with device-scope atomic loads (which see every block's
    // atomics across the XCDs), so no block needs a device-scope fence: on gfx950 each such
    // fence writes back its XCD's L2, which cost this kernel more the more blocks it had.
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(d.ticket + 3, 1u) == gridDim.x - 1);
    __syncthreads();
    if (!s_last) return;
    for (int sg = threadIdx.x; sg < d.nseg; sg += BLOCK) {
        const SegC &S = d.seg[sg];
        const uint32_t end =
            __hip_atomic_load(d.cursor + S.cbase + S.ncells - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int64_t n = (int64_t)end - d.segstart[sg];
        d.n_slots[sg] = min(max(n, (int64_t)0), S.cap);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        *d.cur = nb;
        d.ticket[3] = 0u;
    }
}

// After the scan of cellcnt into cursor: the first global position of each segment.
__global__ void k_segstart(Dev d)
{
    for (int sg = threadIdx.x; sg < d.nseg; sg += blockDim.x) d.segstart[sg] = d.cursor[d.seg[sg].cbase];
}

// =======================================================================================
// Diagnostics: alive count and sum |v|^2 per segment (FP64, fixed order per block, then
// striped into a small array reduced on the host).
// =======================================================================================
template <bool F64>
__global__ void k_diag(Dev d, int sg, double *out /* [grid][2] */)
{
    __shared__ double s_buf[8];
    const SegC &S = d.seg[sg];
    const int b = *d.cur;
    const int64_t n = d.n_slots[sg];
    double c = 0.0, v2 = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
         p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = S.base + p;
        if constexpr (!F64) {
            if (d.cell[b][i] == kDead) continue;
            v2 += speed2_rn(d.fvx[b][i], d.fvy[b][i], d.fvz[b][i]);
        } else {
            if (!(d.x[b][i] >= 0.0)) continue;
            v2 += speed2_rn(d.dvx[b][i], d.dvy[b][i], d.dvz[b][i]);
        }
        c += 1.0;
    }
    c = block_sum(c, s_buf);
    v2 = block_sum(v2, s_buf);
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = c;
        out[2 * blockIdx.x + 1] = v2;
    }
}

// =======================================================================================
// Host launchers.
// =======================================================================================
#define LAUNCH_CHECK()                                          \
    do {                                                        \
        hipError_t _e = hipGetLastError();                      \
        if (_e != hipSuccess) return _e;                        \
    } while (0)

// The persistent FP64 pass: stages that push or collide run on half the grid, the deposit
// and histogram on all of it (on the 4e7-particle slab, push and collide were fastest at two
// blocks per CU and the deposit at three to four; more blocks slowed every stage).
template <int STAGES>
static hipError_t launch_particles_t(const Dev &d, const Launch &L, hipStream_t s, int hist)
{
    const int grid = (STAGES & (ST_PUSH | ST_COLLIDE)) ? std::max(8, L.grid / 16 * 8) : L.grid;
    switch (L.ppt) {
    case 1:
        hipLaunchKernelGGL((k_particles<STAGES, 1>), dim3(grid), dim3(L.block), 0, s, d, hist);
        break;
    case 2:
        hipLaunchKernelGGL((k_particles<STAGES, 2>), dim3(grid), dim3(L.block), 0, s, d, hist);
        break;
    case 8:
        hipLaunchKernelGGL((k_particles<STAGES, 8>), dim3(grid), dim3(L.block), 0, s, d, hist);
        break;
    default:
        hipLaunchKernelGGL((k_particles<STAGES, 4>), dim3(grid), dim3(L.block), 0, s, d, hist);
        break;
    }
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_particles(const Dev &d, const Launch &L, hipStream_t s, bool f64, int stages, int hist,
                            bool with_params)
{
    // the null-collision bound of every segment from this step's speed and field maxima
    if ((stages & SB_COLLIDE) && with_params) {
        hipLaunchKernelGGL(k_params, dim3(1), dim3(256), 0, s, d);
        LAUNCH_CHECK();
    }
    if (!f64) return launch_pass32(d, L.ppt, L.window, s, stages, hist, d.cap_tot, L.nt != 0);
#define PIC_CASE(ST) \
    case ST:         \
        return launch_particles_t<ST>(d, L, s, hist);
    switch (stages) {
        PIC_CASE(ST_PUSH)
        PIC_CASE(ST_COLLIDE)
        PIC_CASE(ST_DEPOSIT)
        PIC_CASE(ST_HIST)
        PIC_CASE(ST_PUSH | ST_COLLIDE | ST_DEPOSIT)
        PIC_CASE(ST_PUSH | ST_DEPOSIT)
    default:
        return hipErrorInvalidValue;
    }
#undef PIC_CASE
}

hipError_t launch_candidates(const Dev &d, const Launch &L, hipStream_t s, bool f64, int hist)
{
    if (f64) return hipSuccess;
    return launch_cand32(d, L.ppt, s, hist, d.cap_tot);
}

hipError_t launch_init(const Dev &d, bool f64, int sg, int64_t n, int64_t ppc, int init_mode,
                       double vth, double amp, int mode, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int B = 256;
    const int64_t G = (n + B - 1) / B;
    if (f64)
        hipLaunchKernelGGL(k_init<true>, dim3(G), dim3(B), 0, s, d, sg, n, ppc, init_mode, vth, amp, mode);
    else
        hipLaunchKernelGGL(k_init<false>, dim3(G), dim3(B), 0, s, d, sg, n, ppc, init_mode, vth, amp, mode);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_vmax(const Dev &d, bool f64, hipStream_t s)
{
    dim3 g(256, d.nseg);
    if (f64)
        hipLaunchKernelGGL(k_vmax<true>, g, dim3(256), 0, s, d);
    else
        hipLaunchKernelGGL(k_vmax<false>, g, dim3(256), 0, s, d);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_zero_q(const Dev &d, bool f64, hipStream_t s)
{
    if (f64)
        hipLaunchKernelGGL(k_zero_q<true>, dim3(512), dim3(256), 0, s, d);
    else
        hipLaunchKernelGGL(k_zero_q<false>, dim3(512), dim3(256), 0, s, d);
    LAUNCH_CHECK();
    return hipSuccess;
}

bool births_fit_solve(const Dev &d) { return d.ngt > 0; }

hipError_t launch_solve(const Dev &d, bool f64, int64_t nchunks, bool zero_q, hipStream_t s,
                        bool with_births, bool with_params)
{
    const int nc = (int)nchunks, zq = zero_q ? 1 : 0;
    const int nscan = with_births ? d.ngt : 0;
    const int nred = with_params ? (d.nseg + kSolveThreads / kWave - 1) / (kSolveThreads / kWave) : 0;
    const int par = with_params ? 1 : 0;
    const dim3 g1(nc + nscan + nred), g2(nc + (with_births ? place_blocks(d) : 0));
    if (f64) {
        hipLaunchKernelGGL(k_solve1<true>, g1, dim3(kSolveThreads), 0, s, d, nc, nscan, nred);
        hipLaunchKernelGGL(k_solve2<true>, g2, dim3(kSolveThreads), 0, s, d, zq, nc, par);
    } else {
        hipLaunchKernelGGL(k_solve1<false>, g1, dim3(kSolveThreads), 0, s, d, nc, nscan, nred);
        hipLaunchKernelGGL(k_solve2<false>, g2, dim3(kSolveThreads), 0, s, d, zq, nc, par);
    }
    LAUNCH_CHECK();
    if (d.periodic) {
        hipLaunchKernelGGL(k_phi_shift, dim3(nchunks), dim3(kSolveThreads), 0, s, d);
        LAUNCH_CHECK();
    }
    return hipSuccess;
}

hipError_t launch_field_stats(const Dev &d, bool f64, int64_t nchunks, hipStream_t s)
{
    hipLaunchKernelGGL(k_field_stats, dim3(1), dim3(kSolveThreads), 0, s, d);
    LAUNCH_CHECK();
    if (!f64) {
        hipLaunchKernelGGL(k_ecell, dim3(nchunks), dim3(kSolveThreads), 0, s, d);
        LAUNCH_CHECK();
    }
    return hipSuccess;
}

hipError_t launch_field_energy(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_field_energy, dim3(d.nens), dim3(1024), 0, s, d);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_params(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_params, dim3(1), dim3(256), 0, s, d);
    LAUNCH_CHECK();
    return hipSuccess;
}

static hipError_t launch_scan_sel(uint32_t *in, uint32_t *out, int64_t n, uint32_t *part, bool zero_in,
                                  const int64_t *parity_step, hipStream_t s)
{
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan_sums, dim3(nb), dim3(kScanBlock), 0, s, in, n, part, parity_step);
    hipLaunchKernelGGL(k_scan_part, dim3(1), dim3(1024), 0, s, part, nb);
    hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kScanBlock), 0, s, in, out, n, part, zero_in ? 1 : 0,
                       parity_step);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_scan(uint32_t *in, uint32_t *out, int64_t n, uint32_t *part, bool zero_in, hipStream_t s)
{
    return launch_scan_sel(in, out, n, part, zero_in, nullptr, s);
}

int64_t scan_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

hipError_t launch_births(const Dev &d, bool f64, bool in_step, bool advance, hipStream_t s)
{
    hipError_t e;
    // the group-count scan: one block per tile up to kMaxGroupTiles tiles, the global
    // three-kernel scan above that
    if (d.ngt > 0) {
        hipLaunchKernelGGL(k_group_scan, dim3(d.ngt), dim3(256), 0, s, d);
        LAUNCH_CHECK();
    } else if ((e = launch_scan_sel(d.gcnt, d.gpre, d.g_tot, d.scanpart, false, d.step, s)) != hipSuccess) {
        return e;
    }
    const int deferred = in_step ? 1 : 0, adv = advance ? 1 : 0;
    if (f64)
        hipLaunchKernelGGL(k_birth_place<true>, dim3(place_blocks(d)), dim3(256), 0, s, d, deferred, adv);
    else
        hipLaunchKernelGGL(k_birth_place<false>, dim3(place_blocks(d)), dim3(256), 0, s, d, deferred, adv);
    LAUNCH_CHECK();
    if (!in_step) {
        hipLaunchKernelGGL(k_birth_clear, dim3(64), dim3(256), 0, s, d, -1);
        LAUNCH_CHECK();
    }
    return hipSuccess;
}

hipError_t launch_births_clear_all(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_birth_clear, dim3(64), dim3(256), 0, s, d, 0);
    hipLaunchKernelGGL(k_birth_clear, dim3(64), dim3(256), 0, s, d, 1);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_advance(const Dev &d, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, d);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_sort_prepare(const Dev &d, hipStream_t s)
{
    hipError_t e = launch_scan(d.cellcnt, d.cursor, d.cells_tot, d.scanpart, true, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_segstart, dim3(1), dim3(256), 0, s, d);
    return hipGetLastError();
}

hipError_t launch_sort(const Dev &d, bool f64, const Launch &L, hipStream_t s)
{
    hipError_t e = launch_sort_prepare(d, s);
    if (e != hipSuccess) return e;
    if (!f64) return launch_sort32_scatter(d, L.sort_ppt, L.window, s, d.cap_tot, L.sort_nt != 0);
    // the scatter's static runs of tiles are short: 8x the pass's persistent grid (a sweep
    // from 1/2x to 8x on the 4e7-particle slab: 1.33, 1.07, 0.92, 0.85, 0.83 ms)
    const size_t lds = (size_t)L.window * 4;
    hipLaunchKernelGGL((k_sort_scatter<4>), dim3(8 * L.grid), dim3(L.block), lds, s, d, L.window);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_diag(const Dev &d, bool f64, int sg, double *out, int grid, hipStream_t s)
{
    if (f64)
        hipLaunchKernelGGL(k_diag<true>, dim3(grid), dim3(256), 0, s, d, sg, out);
    else
        hipLaunchKernelGGL(k_diag<false>, dim3(grid), dim3(256), 0, s, d, sg, out);
    LAUNCH_CHECK();
    return hipSuccess;
}

}  // namespace pic
