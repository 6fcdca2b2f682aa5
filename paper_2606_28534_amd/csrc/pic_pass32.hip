// pic_pass32.hip -- the FP32 cell+offset particle pass and counting sort for gfx950.
//
// One block = one tile of 256 x PPT consecutive slots of one segment; thread t owns the
// PPT consecutive slots t*PPT .. t*PPT+PPT-1 and moves them with 16-byte vector loads and
// stores (each wave touches 64 x 16 B contiguous bytes per array).  Because particles are
// sorted by cell every K steps, a thread's slots almost always sit in one cell: the thread
// merges them into runs of equal cell before touching shared memory, so the cloud-in-cell
// deposit costs one LDS atomic pair per run and one HBM atomic per window node and block.
// Tiles are mapped to blocks XCD-major: blocks are dispatched round-robin over the 8 XCDs,
// so block b takes tile (b % 8) * (G / 8) + b / 8 and each XCD streams one contiguous
// eighth of the slots (and, sorted, of the cells), keeping its L2 share of the gather table
// and of the deposit nodes local.
#include "pic_device.h"
#include "pic_kernels.h"
#include "pic_particle.h"

namespace pic {

enum : int { PS_PUSH = 1, PS_COLLIDE = 2, PS_DEPOSIT = 4, PS_HIST = 8 };

__device__ __forceinline__ int seg_of_slot(const Dev &d, int64_t slot)
{
    int lo = 0, hi = d.nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (d.seg[mid].base <= slot)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int64_t xcd_tile()
{
    const int64_t G = gridDim.x;  // a multiple of 8
    return (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
}

template <int PPT, typename T, typename V>
__device__ __forceinline__ void vload(const T *p, T (&v)[PPT])
{
#pragma unroll
    for (int q = 0; q < PPT; q += 4) {
        const V t = *(const V *)(p + q);
        v[q] = t.x;
        v[q + 1] = t.y;
        v[q + 2] = t.z;
        v[q + 3] = t.w;
    }
}

template <int PPT, typename T, typename V>
__device__ __forceinline__ void vstore(T *p, const T (&v)[PPT])
{
#pragma unroll
    for (int q = 0; q < PPT; q += 4) {
        V t;
        t.x = v[q];
        t.y = v[q + 1];
        t.z = v[q + 2];
        t.w = v[q + 3];
        *(V *)(p + q) = t;
    }
}

// One run of equal cells into the LDS window (or straight to HBM outside it).
__device__ __forceinline__ void emit_run(const Dev &d, const SegC &S, int s, int cell, uint32_t cnt,
                                         uint32_t sum, int wbase, int W, bool depo, bool hist,
                                         unsigned long long *sQ, uint32_t *sH)
{
    if (cnt == 0) return;
    const int rel = cell - wbase;
    if (rel >= 0 && rel < W) {
        if (depo) {
            atomicAdd(&sQ[rel], (unsigned long long)cnt * 16777216ull - (unsigned long long)sum);
            atomicAdd(&sQ[rel + 1], (unsigned long long)sum);
        }
        if (hist) atomicAdd(&sH[rel], cnt);
        return;
    }
    if (depo) {
        int j1 = cell + 1;
        if (S.periodic && j1 == S.ncells) j1 = 0;
        unsigned long long *Q = d.Qi + (int64_t)s * d.nodes_tot + S.gbase;
        atomicAdd(Q + cell, (unsigned long long)cnt * 16777216ull - (unsigned long long)sum);
        atomicAdd(Q + j1, (unsigned long long)sum);
    }
    if (hist) atomicAdd(d.cellcnt + S.cbase + cell, cnt);
}

template <int STAGES, int PPT>
__global__ void __launch_bounds__(256) k_pass32(Dev d, int W, int hist_rt, int64_t T)
{
    constexpr bool PUSH = STAGES & PS_PUSH;
    constexpr bool COLL = STAGES & PS_COLLIDE;
    constexpr bool DEPO = STAGES & PS_DEPOSIT;
    constexpr bool HISTC = STAGES & PS_HIST;
    constexpr bool WIN = DEPO || HISTC;
    constexpr bool NEED_V = PUSH || COLL;
    constexpr int TILE = 256 * PPT;
    static_assert(PPT % 4 == 0, "PPT must be a multiple of 4");

    extern __shared__ unsigned long long s_dyn[];
    unsigned long long *sQ = s_dyn;                // [W + 1]
    uint32_t *sH = (uint32_t *)(s_dyn + (W + 1));  // [W]
    __shared__ unsigned long long s_v2;
    __shared__ uint32_t s_c[C_NCNT];
    __shared__ double s_ke[2];
    __shared__ int s_c0;

    const int64_t t = xcd_tile();
    if (t >= T) return;
    const int64_t first = t * TILE;
    const int sg = seg_of_slot(d, first);
    const SegC &S = d.seg[sg];
    const int64_t last = min(first + TILE, S.base + d.n_slots[sg]);
    if (first >= last) return;
    const EnsC &e = d.ens[S.ens];
    const int s = S.species;
    const int b = *d.cur;
    const bool hist = HISTC || (hist_rt != 0);
    const int tid = threadIdx.x;

    const int64_t i0 = first + (int64_t)tid * PPT;
    const bool full = (i0 + PPT <= last);
    int cell[PPT];
    float off[PPT], vx[PPT], vy[PPT], vz[PPT];
    uint32_t id[PPT];
    if (full) {
        vload<PPT, int32_t, int4>(d.cell[b] + i0, cell);
        vload<PPT, float, float4>(d.off[b] + i0, off);
        if (NEED_V) {
            vload<PPT, float, float4>(d.fvx[b] + i0, vx);
            vload<PPT, float, float4>(d.fvy[b] + i0, vy);
            vload<PPT, float, float4>(d.fvz[b] + i0, vz);
        }
        if (COLL) vload<PPT, uint32_t, uint4>(d.id[b] + i0, id);
    } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int64_t i = i0 + k;
            cell[k] = kDead;
            if (i < last) {
                cell[k] = d.cell[b][i];
                off[k] = d.off[b][i];
                if (NEED_V) {
                    vx[k] = d.fvx[b][i];
                    vy[k] = d.fvy[b][i];
                    vz[k] = d.fvz[b][i];
                }
                if (COLL) id[k] = d.id[b][i];
            }
        }
    }

    if (WIN) {
        for (int i = tid; i <= W; i += 256) {
            sQ[i] = 0ull;
            if (i < W) sH[i] = 0u;
        }
    }
    if (tid < C_NCNT) s_c[tid] = 0u;
    if (tid < 2) s_ke[tid] = 0.0;
    if (tid == 0) {
        s_v2 = 0ull;
        s_c0 = cell[0];
    }
    __syncthreads();
    // deposit window [wbase, wbase + W) around the tile's first cell (pre-push)
    const int c0 = s_c0;
    const int wbase = (c0 == kDead) ? 0 : max(c0 - W / 4, 0);

    uint32_t npush = 0;
    double v2m = 0.0;
    const double numax = COLL ? d.numax[sg] : 0.0;
    const double pnull = COLL ? d.pnull[sg] : 0.0;
    const uint32_t tag = COLL ? (uint32_t)(*d.step) : 0u;
    const int st = stripe_of_block();

#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (cell[k] == kDead) continue;
        PS<false> p;
        p.cell = cell[k];
        p.off = off[k];
        if (NEED_V) {
            p.vx = vx[k];
            p.vy = vy[k];
            p.vz = vz[k];
        }
        if (PUSH) {
            ++npush;
            const int wall = p_push<false>(d, S, e, p);
            if (wall) {
                if (wall != 3) {
                    const double v2 = speed2_rn(p.vx, p.vy, p.vz);
                    atomicAdd(&s_c[wall == 1 ? C_WALL_L : C_WALL_R], 1u);
                    atomicAdd(&s_ke[wall - 1], S.halfmw * v2);
                }
                cell[k] = kDead;
                continue;
            }
            cell[k] = p.cell;
            off[k] = p.off;
            vx[k] = p.vx;
            vy[k] = p.vy;
            vz[k] = p.vz;
        }
        if (COLL) {
            p.id = id[k];
            double ve[3], vi[3];
            const int ch = p_collide<false>(e, S, s, numax, pnull, tag, p, ve, vi);
            if (ch >= 0) {
                atomicAdd(&s_c[C_EL + ch], 1u);
                vx[k] = p.vx;
                vy[k] = p.vy;
                vz[k] = p.vz;
            }
            if (ch == 1) {
                const uint32_t slot = atomicAdd(d.nbirth + st, 1u);
                if ((int64_t)slot < d.birth_stripe_cap) {
                    Birth &B = d.births[(int64_t)st * d.birth_stripe_cap + slot];
                    B.pid = p.id;
                    B.ens = S.ens;
                    B.cell = p.cell;
                    B.off = p.off;
                    B.x = ((double)p.cell + (double)p.off) * S.dx;
                    for (int q = 0; q < 3; ++q) {
                        B.ve[q] = ve[q];
                        B.vi[q] = vi[q];
                    }
                    atomicOr(d.bitmap + e.bm_base + (p.id >> 5), 1u << (p.id & 31));
                    atomicAdd(d.l1cnt + e.l1_base + (p.id >> 10), 1u);
                } else {
                    atomicOr(d.err, (int)E_CAP_BIRTH);
                }
                v2m = fmax(v2m, speed2_rn(ve[0], ve[1], ve[2]));
                if (S.other >= 0) {
                    const int half = 1 - *d.vcur;
                    atomicMax(d.vmax2 + ((int64_t)half * kStripes + st) * d.nseg + S.other,
                              dbits(speed2_rn(vi[0], vi[1], vi[2])));
                }
                if (DEPO) {
                    global_deposit32(d, S, s, p.cell, p.off, hist);
                    if (S.other >= 0) global_deposit32(d, d.seg[S.other], 1, p.cell, p.off, hist);
                }
            }
            v2m = fmax(v2m, speed2_rn(vx[k], vy[k], vz[k]));
        }
    }

    // write back
    if (PUSH || COLL) {
        if (full) {
            if (PUSH) {
                vstore<PPT, int32_t, int4>(d.cell[b] + i0, cell);
                vstore<PPT, float, float4>(d.off[b] + i0, off);
            }
            vstore<PPT, float, float4>(d.fvx[b] + i0, vx);
            vstore<PPT, float, float4>(d.fvy[b] + i0, vy);
            vstore<PPT, float, float4>(d.fvz[b] + i0, vz);
        } else {
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                const int64_t i = i0 + k;
                if (i >= last) continue;
                if (PUSH) {
                    d.cell[b][i] = cell[k];
                    d.off[b][i] = off[k];
                }
                if (cell[k] != kDead) {
                    d.fvx[b][i] = vx[k];
                    d.fvy[b][i] = vy[k];
                    d.fvz[b][i] = vz[k];
                }
            }
        }
    }

    // deposit / histogram by runs of equal cell
    if (WIN) {
        int rk = kDead;
        uint32_t rc = 0, rs = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (cell[k] == kDead) continue;
            if (cell[k] != rk) {
                if (rk != kDead) emit_run(d, S, s, rk, rc, rs, wbase, W, DEPO, hist, sQ, sH);
                rk = cell[k];
                rc = 0;
                rs = 0;
            }
            ++rc;
            if (DEPO) rs += fixed_share(off[k]);
        }
        if (rk != kDead) emit_run(d, S, s, rk, rc, rs, wbase, W, DEPO, hist, sQ, sH);
    }

    // block tallies
    if (PUSH) {
        const uint32_t np = wave_sum_u32(npush);
        if (lane_id() == 0 && np) atomicAdd(&s_c[C_PUSH], np);
    }
    if (COLL) {
        const double m = wave_max_f64(v2m);
        if (lane_id() == 0 && m > 0.0) atomicMax(&s_v2, dbits(m));
    }
    __syncthreads();
    if (WIN) {
        const int nn = S.periodic ? S.ncells : S.ncells + 1;
        unsigned long long *Q = d.Qi + (int64_t)s * d.nodes_tot + S.gbase;
        for (int i = tid; i <= W; i += 256) {
            if (DEPO) {
                const unsigned long long v = sQ[i];
                if (v) {
                    int node = wbase + i;
                    if (S.periodic && node >= S.ncells) node -= S.ncells;
                    if (node < nn) atomicAdd(Q + node, v);
                }
            }
            if (hist && i < W) {
                const uint32_t c = sH[i];
                const int cl = wbase + i;
                if (c && cl < S.ncells) atomicAdd(d.cellcnt + S.cbase + cl, c);
            }
        }
    }
    if (tid == 0 && (PUSH || COLL)) {
        unsigned long long *c = d.cnt + ((int64_t)st * d.nseg + sg) * C_NCNT;
        for (int k = 0; k < C_NCNT; ++k)
            if (s_c[k]) atomicAdd(c + k, (unsigned long long)s_c[k]);
        double *sm = d.sums + ((int64_t)st * d.nseg + sg) * S_NSUM;
        if (s_ke[0] != 0.0) unsafeAtomicAdd(sm + S_KE_L, s_ke[0]);
        if (s_ke[1] != 0.0) unsafeAtomicAdd(sm + S_KE_R, s_ke[1]);
        if (COLL && s_v2) {
            const int half = 1 - *d.vcur;
            atomicMax(d.vmax2 + ((int64_t)half * kStripes + st) * d.nseg + sg, s_v2);
        }
    }
}

// =======================================================================================
// Counting sort scatter (FP32 form): thread runs are ranked inside the tile with one LDS
// atomic each, every cell of the tile reserves its output run with one HBM atomic on the
// cursor, and the particles are written into the other buffer.  Absorbed slots drop out.
// =======================================================================================
template <int PPT>
__global__ void __launch_bounds__(256) k_sort32(Dev d, int W, int64_t T)
{
    constexpr int TILE = 256 * PPT;
    extern __shared__ unsigned long long s_dyn[];
    uint32_t *sCnt = (uint32_t *)s_dyn;  // [W]
    __shared__ int s_min;
    const int64_t t = xcd_tile();
    if (t >= T) return;
    const int64_t first = t * TILE;
    const int sg = seg_of_slot(d, first);
    const SegC &S = d.seg[sg];
    const int64_t last = min(first + TILE, S.base + d.n_slots[sg]);
    if (first >= last) return;
    const int b = *d.cur, nb = 1 - b;
    const int tid = threadIdx.x;
    const int64_t i0 = first + (int64_t)tid * PPT;
    const bool full = (i0 + PPT <= last);
    int cell[PPT];
    float off[PPT], vx[PPT], vy[PPT], vz[PPT];
    uint32_t id[PPT];
    if (full) {
        vload<PPT, int32_t, int4>(d.cell[b] + i0, cell);
        vload<PPT, float, float4>(d.off[b] + i0, off);
        vload<PPT, float, float4>(d.fvx[b] + i0, vx);
        vload<PPT, float, float4>(d.fvy[b] + i0, vy);
        vload<PPT, float, float4>(d.fvz[b] + i0, vz);
        vload<PPT, uint32_t, uint4>(d.id[b] + i0, id);
    } else {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int64_t i = i0 + k;
            cell[k] = kDead;
            if (i < last) {
                cell[k] = d.cell[b][i];
                off[k] = d.off[b][i];
                vx[k] = d.fvx[b][i];
                vy[k] = d.fvy[b][i];
                vz[k] = d.fvz[b][i];
                id[k] = d.id[b][i];
            }
        }
    }
    int mn = INT32_MAX;
#pragma unroll
    for (int k = 0; k < PPT; ++k)
        if (cell[k] != kDead) mn = min(mn, cell[k]);
    mn = wave_min_i32(mn);
    if (tid == 0) s_min = INT32_MAX;
    for (int i = tid; i < W; i += 256) sCnt[i] = 0u;
    __syncthreads();
    if (lane_id() == 0 && mn != INT32_MAX) atomicMin(&s_min, mn);
    __syncthreads();
    const int base = s_min;
    // rank runs: pos[k] is the rank inside the tile's run of that cell (in window) or the
    // final global position (outside it)
    uint32_t pos[PPT];
    bool inwin[PPT];
    {
        int rk = kDead, rstart = 0;
        uint32_t rc = 0;
        auto flush = [&](int kend) {
            if (rk == kDead || rc == 0) return;
            const int rel = rk - base;
            const bool w = rel >= 0 && rel < W;
            const uint32_t r0 = w ? atomicAdd(&sCnt[rel], rc) : atomicAdd(d.cursor + S.cbase + rk, rc);
            uint32_t r = r0;
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if (k >= rstart && k < kend && cell[k] == rk) {
                    pos[k] = r++;
                    inwin[k] = w;
                }
            }
        };
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (cell[k] == kDead) continue;
            if (cell[k] != rk) {
                flush(k);
                rk = cell[k];
                rc = 0;
                rstart = k;
            }
            ++rc;
        }
        flush(PPT);
    }
    __syncthreads();
    for (int i = tid; i < W; i += 256) {
        const uint32_t c = sCnt[i];
        if (c) sCnt[i] = atomicAdd(d.cursor + S.cbase + base + i, c);
    }
    __syncthreads();
    const int64_t sbase = S.base - d.segstart[sg];
    const int64_t send = S.base + S.cap;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (cell[k] == kDead) continue;
        const uint32_t P = inwin[k] ? sCnt[cell[k] - base] + pos[k] : pos[k];
        const int64_t o = sbase + (int64_t)P;
        if (o < S.base || o >= send) {
            atomicOr(d.err, (int)E_CAP_PART);
            continue;
        }
        d.cell[nb][o] = cell[k];
        d.off[nb][o] = off[k];
        d.fvx[nb][o] = vx[k];
        d.fvy[nb][o] = vy[k];
        d.fvz[nb][o] = vz[k];
        d.id[nb][o] = id[k];
    }
}

__global__ void k_sort_finish(Dev d)
{
    for (int sg = threadIdx.x; sg < d.nseg; sg += blockDim.x) {
        const SegC &S = d.seg[sg];
        const int64_t n = (int64_t)d.cursor[S.cbase + S.ncells - 1] - d.segstart[sg];
        d.n_slots[sg] = min(max(n, (int64_t)0), S.cap);
    }
    __syncthreads();
    if (threadIdx.x == 0) *d.cur = 1 - *d.cur;
}

// =======================================================================================
template <int STAGES>
static hipError_t launch_pass32_t(const Dev &d, int ppt, int W, hipStream_t s, int hist, int64_t cap_tot)
{
    const size_t lds = (size_t)(W + 1) * 8 + (size_t)W * 4;
    if (ppt == 4) {
        const int64_t T = cap_tot / (256 * 4);
        const int64_t G = (T + 7) / 8 * 8;
        hipLaunchKernelGGL((k_pass32<STAGES, 4>), dim3(G), dim3(256), lds, s, d, W, hist, T);
    } else {
        const int64_t T = cap_tot / (256 * 8);
        const int64_t G = (T + 7) / 8 * 8;
        hipLaunchKernelGGL((k_pass32<STAGES, 8>), dim3(G), dim3(256), lds, s, d, W, hist, T);
    }
    return hipGetLastError();
}

hipError_t launch_pass32(const Dev &d, int ppt, int W, hipStream_t s, int stages, int hist, int64_t cap_tot)
{
    switch (stages) {
    case PS_PUSH:
        return launch_pass32_t<PS_PUSH>(d, ppt, W, s, hist, cap_tot);
    case PS_COLLIDE:
        return launch_pass32_t<PS_COLLIDE>(d, ppt, W, s, hist, cap_tot);
    case PS_DEPOSIT:
        return launch_pass32_t<PS_DEPOSIT>(d, ppt, W, s, hist, cap_tot);
    case PS_HIST:
        return launch_pass32_t<PS_HIST>(d, ppt, W, s, hist, cap_tot);
    case PS_PUSH | PS_COLLIDE | PS_DEPOSIT:
        return launch_pass32_t<PS_PUSH | PS_COLLIDE | PS_DEPOSIT>(d, ppt, W, s, hist, cap_tot);
    case PS_PUSH | PS_DEPOSIT:
        return launch_pass32_t<PS_PUSH | PS_DEPOSIT>(d, ppt, W, s, hist, cap_tot);
    default:
        return hipErrorInvalidValue;
    }
}

hipError_t launch_sort32_scatter(const Dev &d, int ppt, int W, hipStream_t s, int64_t cap_tot)
{
    const size_t lds = (size_t)W * 4;
    if (ppt == 4) {
        const int64_t T = cap_tot / (256 * 4);
        hipLaunchKernelGGL((k_sort32<4>), dim3((T + 7) / 8 * 8), dim3(256), lds, s, d, W, T);
    } else {
        const int64_t T = cap_tot / (256 * 8);
        hipLaunchKernelGGL((k_sort32<8>), dim3((T + 7) / 8 * 8), dim3(256), lds, s, d, W, T);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(256), 0, s, d);
    return hipGetLastError();
}

}  // namespace pic
