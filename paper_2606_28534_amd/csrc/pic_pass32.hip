// pic_pass32.hip -- the FP32 cell+offset particle pass and counting sort for gfx950.
//
// One block = one tile of 256 x PPT consecutive slots of one segment; thread t owns the
// PPT consecutive slots t*PPT .. t*PPT+PPT-1 and moves them with 16-byte vector loads and
// stores (each wave touches 64 x 16 B contiguous bytes per array).  Because particles are
// sorted by cell every K steps, a thread's slots almost always sit in one cell: the thread
// merges them into runs of equal cell before touching shared memory, so the cloud-in-cell
// deposit costs one LDS atomic pair per run and one HBM atomic per window node and block.
// The window spans the tile's own cells (pre-push, plus a margin for the step's motion), up
// to the launch's maximum: a sorted tile clears and flushes a few nodes, a tile of freshly
// appended particles spread over many cells still deposits through LDS.
// Block b takes tile b (see tile_of_block for why not an XCD-major order).
#include <algorithm>

#include "pic_device.h"
#include "pic_kernels.h"
#include "pic_particle.h"

namespace pic {

enum : int { PS_PUSH = 1, PS_COLLIDE = 2, PS_DEPOSIT = 4, PS_HIST = 8 };
// collision-candidate records staged in LDS per tile (more go straight to HBM)
constexpr uint32_t kRecLds = 256;

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

// Block b takes tile b.  Workgroups go to the XCDs round-robin, so the tiles in use are
// spread evenly over the eight XCDs however much of the slot capacity is filled.  (Giving
// each XCD a contiguous eighth of the capacity instead, for L2 locality, left the XCDs that
// own the unused tail of each segment idle: 1.8x slower on a quarter-filled slab and no
// faster on the benchmark slab, whose gather table and charge fit every XCD's L2.)
__device__ __forceinline__ int64_t tile_of_block() { return (int64_t)blockIdx.x; }

typedef uint32_t word4 __attribute__((ext_vector_type(4)));

// PPT consecutive 32-bit values as 16-byte vectors, optionally with the non-temporal hint
// (the particle arrays are streamed once per step).
template <int PPT, bool NT, typename T>
__device__ __forceinline__ void vload(const T *p, T (&v)[PPT])
{
    static_assert(sizeof(T) == 4, "32-bit words");
#pragma unroll
    for (int q = 0; q < PPT; q += 4) {
        word4 t;
        if constexpr (NT)
            t = __builtin_nontemporal_load((const word4 *)(p + q));
        else
            t = *(const word4 *)(p + q);
        // copy the lanes out first: a bit_cast of a vector-element lvalue reads element 0
        const uint32_t e[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
        for (int u = 0; u < 4; ++u) v[q + u] = __builtin_bit_cast(T, e[u]);
    }
}

template <int PPT, bool NT, typename T>
__device__ __forceinline__ void vstore(T *p, const T (&v)[PPT])
{
    static_assert(sizeof(T) == 4, "32-bit words");
#pragma unroll
    for (int q = 0; q < PPT; q += 4) {
        word4 t;
        t.x = __builtin_bit_cast(uint32_t, v[q]);
        t.y = __builtin_bit_cast(uint32_t, v[q + 1]);
        t.z = __builtin_bit_cast(uint32_t, v[q + 2]);
        t.w = __builtin_bit_cast(uint32_t, v[q + 3]);
        if constexpr (NT)
            __builtin_nontemporal_store(t, (word4 *)(p + q));
        else
            *(word4 *)(p + q) = t;
    }
}

// A segment's grid placement and shape, held in registers by the pass (read before its first
// global store, so no store can force them to be read again).
struct SegGrid {
    int64_t gbase, cbase;
    int ncells;
    bool periodic;
};

// Cells a particle may move in one step and still deposit through the tile's window.
constexpr int kWinMargin = 2;

// The LDS window holds one 64-bit word per cell: the count of the cell's particles in the
// high 24 bits and the sum of their right-node shares (R15) in the low 40, so one LDS
// atomic per run serves the deposit and the sort histogram alike.  A tile holds at most
// 2048 particles, so the count stays below 2^12 and the share sum below 2^35.  The flush
// gives node j the left shares of cell j, count x 2^24 - sum, plus the right shares of
// cell j - 1.
constexpr int kWinShift = 40;
constexpr unsigned long long kWinSumMask = (1ull << kWinShift) - 1ull;

// One run of equal cells into the LDS window (or straight to HBM outside it).
__device__ __forceinline__ void emit_run(const Dev &d, const SegGrid &G, int s, int cell, uint32_t cnt,
                                         uint32_t sum, int wbase, int W, bool depo, bool hist,
                                         unsigned long long *sA)
{
    if (cnt == 0) return;
    const int rel = cell - wbase;
    if (rel >= 0 && rel < W) {
        if (depo || hist) atomicAdd(&sA[rel], ((unsigned long long)cnt << kWinShift) | (unsigned long long)sum);
        return;
    }
    if (depo) {
        int j1 = cell + 1;
        if (G.periodic && j1 == G.ncells) j1 = 0;
        unsigned long long *Q = d.Qi + (int64_t)s * d.nodes_tot + G.gbase;
        atomicAdd(Q + cell, (unsigned long long)cnt * 16777216ull - (unsigned long long)sum);
        atomicAdd(Q + j1, (unsigned long long)sum);
    }
    if (hist) atomicAdd(d.cellcnt + G.cbase + cell, cnt);
}

// Counting-sort ranking of one tile.  A particle whose cell lies in the window
// [base, base + Ws) gets its rank inside the tile's run of that cell; any other live
// particle takes its final position from the global cursor of its cell at once.  With
// AGGREGATE a wave ranks each distinct cell with one LDS atomic (leader election, a chain of
// dependent steps per cell); without, every particle adds 1 with an LDS atomic of its own
// (independent instructions, serialised by the LDS only where lanes share a cell).  The
// sort scatter measured faster aggregated (535 against 555 us), the sorting pass direct
// (572 against 625 us).
template <int PPT, bool AGGREGATE>
__device__ __forceinline__ void tile_rank(const int (&cell)[PPT], int base, int Ws, uint32_t *sCnt,
                                          uint32_t *cursor, uint32_t (&pos)[PPT], bool (&inwin)[PPT])
{
    if constexpr (!AGGREGATE) {
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int rel = (cell[k] != kDead) ? cell[k] - base : -1;
            inwin[k] = rel >= 0 && rel < Ws;
            if (inwin[k])
                pos[k] = atomicAdd(&sCnt[rel], 1u);
            else if (cell[k] != kDead)
                pos[k] = atomicAdd(cursor + cell[k], 1u);
        }
        return;
    }
    const int lane = lane_id();
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int rel = (cell[k] != kDead) ? cell[k] - base : -1;
        const int key = (rel >= 0 && rel < Ws) ? rel : -1;
        inwin[k] = key >= 0;
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
            if (mine) pos[k] = r0 + (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
            act &= ~m;
            ++it;
        }
        if ((act >> lane) & 1ull) pos[k] = atomicAdd(&sCnt[key], 1u);
        if (cell[k] != kDead && key < 0) pos[k] = atomicAdd(cursor + cell[k], 1u);
    }
}

// After tile_rank and a barrier: one run per window cell is reserved in the global order,
// turning the tile's counts in sCnt into the runs' first positions (a barrier must follow).
__device__ __forceinline__ void tile_reserve(uint32_t *sCnt, int Ws, uint32_t *cursor, int base)
{
    for (int i = threadIdx.x; i < Ws; i += blockDim.x) {
        const uint32_t c = sCnt[i];
        if (c) sCnt[i] = atomicAdd(cursor + base + i, c);
    }
}

// With SORT (a fused pass on the step after a histogram step) every live particle is written
// to the other buffer at its place in cell order instead of in place: the tile ranks its
// particles by their cell before the push (the cells the previous pass counted) in LDS and
// reserves one run per cell, as the sort scatter does, so the pass also sorts and compacts.
template <int STAGES, int PPT, bool NT = false, bool SORT = false>
__global__ void __launch_bounds__(256) k_pass32(Dev d, int W, int hist_rt, int64_t T)
{
    constexpr bool PUSH = STAGES & PS_PUSH;
    constexpr bool COLL = STAGES & PS_COLLIDE;
    constexpr bool DEPO = STAGES & PS_DEPOSIT;
    constexpr bool HISTC = STAGES & PS_HIST;
    constexpr bool WIN = DEPO || HISTC;
    constexpr bool NEED_V = PUSH || COLL;
    constexpr bool NEED_ID = COLL || SORT;
    constexpr int TILE = 256 * PPT;
    static_assert(PPT % 4 == 0, "PPT must be a multiple of 4");
    static_assert(!SORT || (PUSH && DEPO && !HISTC), "the sorting pass is a fused pass");

    extern __shared__ unsigned long long s_dyn[];
    unsigned long long *sA = s_dyn;             // [W]: count and right-share sum per cell
    uint32_t *sCnt = (uint32_t *)(s_dyn + W);   // [W], the sorting pass's tile ranking
    __shared__ unsigned long long s_v2;
    __shared__ uint32_t s_c[C_NCNT];
    __shared__ double s_ke[2];
    __shared__ double s_kes;   // fused step: sum |v|^2 of the block's particles alive after the push
    __shared__ uint32_t s_nal;  // and their count
    __shared__ int s_wmn[4], s_wmx[4];
    __shared__ uint32_t s_nc;
    __shared__ uint4 s_rec[COLL ? 2 * kRecLds : 1];

    const int64_t t = tile_of_block();
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
        vload<PPT, NT>(d.cell[b] + i0, cell);
        vload<PPT, NT>(d.off[b] + i0, off);
        if (NEED_V) {
            vload<PPT, NT>(d.fvx[b] + i0, vx);
            vload<PPT, NT>(d.fvy[b] + i0, vy);
            vload<PPT, NT>(d.fvz[b] + i0, vz);
        }
        if (NEED_ID) vload<PPT, NT>(d.id[b] + i0, id);
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
                if (NEED_ID) id[k] = d.id[b][i];
            }
        }
    }

    // Issue the gather loads and draw the collision test's random word for every particle
    // before anything waits on shared memory, so the Philox arithmetic (which needs only the
    // id) runs while the particle and gather-table loads are still in flight.
    float2 ec[PUSH ? PPT : 1];
    if (PUSH) {
        const float2 *__restrict__ Ecs = d.Ecell + S.gbase;
        // dead slots (cell = kDead < 0) read entry 0 and are masked in the push
#pragma unroll
        for (int k = 0; k < PPT; ++k) ec[k] = Ecs[cell[k] < 0 ? 0u : (uint32_t)cell[k]];
    }
    uint32_t rmask = 0;  // bit k: particle k's first Philox word passes R1 < P_null
    if (COLL) {
        // Reading R12 decision R1 < P_null, taken exactly as the integer test
        // (r >> 9) < ceil(P_null 2^23 - 1/2) on the first Philox word of block 0.
        const double X = d.pnull[sg] * 8388608.0 - 0.5;
        const uint32_t thr = X <= 0.0 ? 0u : (X >= 8388608.0 ? 8388608u : (uint32_t)ceil(X));
        const uint32_t tag = (uint32_t)(*d.step);
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const uint4 w = philox(id[k], tag, 0u, 0u, S.seed, (uint32_t)s);
            rmask |= ((w.x >> 9) < thr ? 1u : 0u) << k;
        }
    }

    if (WIN) {
        // the tile's live cells before the push, per wave
        int mn = INT32_MAX, mx = -1;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            if (cell[k] != kDead) {
                mn = min(mn, cell[k]);
                mx = max(mx, cell[k]);
            }
        }
        mn = wave_min_i32(mn);
        mx = wave_max_i32(mx);
        if (lane_id() == 0) {
            s_wmn[tid / kWave] = mn;
            s_wmx[tid / kWave] = mx;
        }
    }
    if (tid < C_NCNT) s_c[tid] = 0u;
    if (tid < 2) s_ke[tid] = 0.0;
    if (tid == 0) {
        s_v2 = 0ull;
        s_nc = 0u;
        s_kes = 0.0;
        s_nal = 0u;
    }
    __syncthreads();
    // deposit window: cells [wbase, wbase + Wt) and nodes [wbase, wbase + Wt], covering the
    // tile's cells and kWinMargin more on each side, at most W cells
    int wbase = 0, Wt = 0;
    if (WIN) {
        const int mn = min(min(s_wmn[0], s_wmn[1]), min(s_wmn[2], s_wmn[3]));
        const int mx = max(max(s_wmx[0], s_wmx[1]), max(s_wmx[2], s_wmx[3]));
        if (mx >= 0) {
            wbase = max(mn - kWinMargin, 0);
            Wt = min(mx + kWinMargin + 1 - wbase, W);
            for (int i = tid; i < Wt; i += 256) sA[i] = 0ull;
        }
    }
    // The segment constants of the push and of the bounds below, read into registers before
    // any global store or atomic (after one, a read through the segment reference would be
    // repeated, since the store might alias it).
    const float h = (float)S.h, dtdx = (float)S.dtdx, eext = (float)e.E_ext;
    const float tv[3] = {(float)S.t[0], (float)S.t[1], (float)S.t[2]};
    const float sv[3] = {(float)S.s[0], (float)S.s[1], (float)S.s[2]};
    const int N = S.ncells;
    const bool per = S.periodic != 0;
    const int64_t seg_lo = S.base, seg_hi = S.base + S.cap;
    const SegGrid G{S.gbase, S.cbase, N, per};
    // the tile's candidate count goes out tagged with its segment and ensemble (cand_tag)
    const uint32_t ctag = COLL ? cand_tag(sg, S.ens) : 0u;
    // sorting pass: destinations in the other buffer (-1: none)
    int64_t dst[SORT ? PPT : 1];
    if constexpr (SORT) {
        const int mn = min(min(s_wmn[0], s_wmn[1]), min(s_wmn[2], s_wmn[3]));
        const int mx = max(max(s_wmx[0], s_wmx[1]), max(s_wmx[2], s_wmx[3]));
        const int Ws = mx >= 0 ? min(mx - mn + 1, W) : 0;
        for (int i = tid; i < Ws; i += 256) sCnt[i] = 0u;
        __syncthreads();
        uint32_t *cursor = d.cursor + S.cbase;
        uint32_t pos[PPT];
        bool inwin[PPT];
        tile_rank<PPT, false>(cell, mn, Ws, sCnt, cursor, pos, inwin);
        __syncthreads();
        tile_reserve(sCnt, Ws, cursor, mn);
        __syncthreads();
        const int64_t sbase = S.base - d.segstart[sg];
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            dst[k] = -1;
            if (cell[k] == kDead) continue;
            const int64_t o = sbase + (int64_t)(inwin[k] ? sCnt[cell[k] - mn] + pos[k] : pos[k]);
            if (o < seg_lo || o >= seg_hi)
                atomicOr(d.err, (int)E_CAP_PART);
            else
                dst[k] = o;
        }
    }

    uint32_t npush = 0;
    uint32_t cchg = 0;  // bit k: particle k's cell changed in the push (or it died)
    double v2m = 0.0;
    // the fused step's scalar diagnostics: |v|^2 and count of the particles alive after the
    // push (|v|^2 per particle and the thread's few particles summed in binary32, FP64 from
    // the wave sum on; the count is the pushes less the absorptions); the candidate kernel
    // adds what collisions and births change
    float kes = 0.f;
    uint32_t nwl = 0, nwr = 0;
    const int st = stripe_of_block();

    if (PUSH) {
        // the loop below is straight-line code apart from the rare wall branch
        uint32_t bad = 0;
        double kel = 0.0, ker = 0.0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const bool alive = cell[k] != kDead;
            npush += alive ? 1u : 0u;
            const float Ep = fmaf(off[k], ec[k].y, ec[k].x) + eext;
            boris<float>(h, tv, sv, Ep, vx[k], vy[k], vz[k]);
            float o = off[k] + vx[k] * dtdx;
            // a non-finite field or velocity makes o NaN or infinite (and a step of 2^30
            // cells is no valid motion): such a particle is dropped and the step reports
            // PIC_ENONFINITE; o is replaced before its conversion to a cell shift
            const bool fin = fabsf(o) < 1073741824.0f;
            o = fin ? o : 0.0f;
            bad |= (alive && !fin) ? 1u : 0u;
            const float fl = floorf(o);
            int c = ((alive && fin) ? cell[k] : 0) + (int)fl;
            o -= fl;
            const bool up = o >= 1.0f;
            off[k] = up ? o - 1.0f : o;
            c += up ? 1 : 0;
            if (per) {
                c = (c < 0) ? c + N : ((c >= N) ? c - N : c);
                const bool inv = alive && (c < 0 || c >= N);  // moved more than a period
                bad |= inv ? 1u : 0u;
                const int cn = (alive && fin && !inv) ? c : kDead;
                cchg |= (cn != cell[k] ? 1u : 0u) << k;
                cell[k] = cn;
            } else {
                const bool out = alive && fin && (c < 0 || c >= N);
                if (out) {
                    const double v2 = speed2_rn(vx[k], vy[k], vz[k]);
                    if (c < 0) {
                        ++nwl;
                        kel += S.halfmw * v2;
                    } else {
                        ++nwr;
                        ker += S.halfmw * v2;
                    }
                    if (S.recycle) {
                        // reading R24: list the absorbed ion; it returns as a neutral
                        const uint32_t pid = NEED_ID ? id[k] : d.id[b][i0 + k];
                        const uint32_t r = atomicAdd(d.nrec, 1u);
                        if ((int64_t)r < d.rec_cap)
                            d.recs[r] = make_uint2(pid, ((uint32_t)S.ens << 1) | (c < 0 ? 0u : 1u));
                        else
                            atomicOr(d.err, (int)E_CAP_PART);
                    }
                }
                const int cn = (out || !fin) ? kDead : cell[k] == kDead ? kDead : c;
                cchg |= (cn != cell[k] ? 1u : 0u) << k;
                cell[k] = cn;
            }
        }
        if (nwl) {
            atomicAdd(&s_c[C_WALL_L], nwl);
            atomicAdd(&s_ke[0], kel);
        }
        if (nwr) {
            atomicAdd(&s_c[C_WALL_R], nwr);
            atomicAdd(&s_ke[1], ker);
        }
        if (bad) atomicOr(d.err, (int)E_NONFINITE);
    }

    if (COLL) {
        // Candidates (the particles still alive after the push whose test passed, about
        // P_null of them) are listed for k_cand32, which draws the rest of the block, picks
        // the channel and scatters; all others keep their velocity.
        float v2f = 0.f;
        uint32_t cmask = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const bool alive = cell[k] != kDead;
            const bool cand = alive && ((rmask >> k) & 1u) && (!SORT || dst[SORT ? k : 0] >= 0);
            cmask |= (cand ? 1u : 0u) << k;
            // |v|^2 of a live particle, 0 for a dead slot (whose velocity is stale): the
            // energy tally and, for the particles that keep their velocity, the speed bound
            const float vv = alive ? speed2_f32(vx[k], vy[k], vz[k]) : 0.f;
            v2f = cand ? v2f : fmaxf(v2f, vv);
            if constexpr (PUSH) kes += vv;
        }
        if (cmask) {
            // one 32-byte record per candidate with its post-push state, so the candidate
            // kernel reads contiguous records instead of six scattered words; records are
            // staged in LDS (the first kRecLds of the tile) and flushed coalesced below
            uint32_t q = atomicAdd(&s_nc, (uint32_t)__popc(cmask));
#pragma unroll
            for (int k = 0; k < PPT; ++k) {
                if ((cmask >> k) & 1u) {
                    const uint32_t slot = SORT ? (uint32_t)dst[SORT ? k : 0] : (uint32_t)(i0 + k);
                    const uint4 r0 = make_uint4(slot, (uint32_t)cell[k], __float_as_uint(off[k]), id[k]);
                    const uint4 r1 = make_uint4(__float_as_uint(vx[k]), __float_as_uint(vy[k]),
                                                __float_as_uint(vz[k]), (uint32_t)sg);
                    if (q < kRecLds) {
                        s_rec[2 * q] = r0;
                        s_rec[2 * q + 1] = r1;
                    } else {
                        d.crec[2 * (first + q)] = r0;
                        d.crec[2 * (first + q) + 1] = r1;
                    }
                    ++q;
                }
            }
        }
        // the speed bound of the next step carries a 2^-16 margin, far above the binary32
        // rounding of |v|^2 here; candidates report their post-collision speed themselves
        v2m = (double)v2f * (1.0 + 0x1p-20);
    }

    // write back
    if constexpr (SORT) {
        const int nb = 1 - b;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int64_t o = dst[SORT ? k : 0];
            if (o < 0) continue;
            d.cell[nb][o] = cell[k];
            d.off[nb][o] = off[k];
            d.fvx[nb][o] = vx[k];
            d.fvy[nb][o] = vy[k];
            d.fvz[nb][o] = vz[k];
            d.id[nb][o] = id[k];
        }
    } else if (PUSH || COLL) {
        if (full) {
            if (PUSH) {
                // a group of four cells is stored only if one of them changed (the heavy
                // ions almost never leave their cell in one step)
#pragma unroll
                for (int q = 0; q < PPT; q += 4) {
                    if ((cchg >> q) & 0xFu) {
                        int c4[4] = {cell[q], cell[q + 1], cell[q + 2], cell[q + 3]};
                        vstore<4, NT>(d.cell[b] + i0 + q, c4);
                    }
                }
                vstore<PPT, NT>(d.off[b] + i0, off);
            }
            vstore<PPT, NT>(d.fvx[b] + i0, vx);
            vstore<PPT, NT>(d.fvy[b] + i0, vy);
            vstore<PPT, NT>(d.fvz[b] + i0, vz);
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
        __syncthreads();  // the window is cleared
        int rk = kDead;
        uint32_t rc = 0, rs = 0;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const bool alive = cell[k] != kDead;
            if (alive && cell[k] != rk) {
                if (rk != kDead) emit_run(d, G, s, rk, rc, rs, wbase, Wt, DEPO, hist, sA);
                rk = cell[k];
                rc = 0;
                rs = 0;
            }
            rc += alive ? 1u : 0u;
            if (DEPO) rs += alive ? fixed_share(off[k]) : 0u;
        }
        if (rk != kDead) emit_run(d, G, s, rk, rc, rs, wbase, Wt, DEPO, hist, sA);
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
    if (PUSH && COLL) {
        const double ks = wave_sum_f64((double)kes);
        const uint32_t na = wave_sum_u32(npush - nwl - nwr);
        if (lane_id() == 0 && na) {
            atomicAdd(&s_kes, ks);
            atomicAdd(&s_nal, na);
        }
    }
    __syncthreads();
    if (WIN) {
        const int nn = G.periodic ? G.ncells : G.ncells + 1;
        unsigned long long *Q = d.Qi + (int64_t)s * d.nodes_tot + G.gbase;
        for (int i = tid; Wt > 0 && i <= Wt; i += 256) {
            const unsigned long long a = i < Wt ? sA[i] : 0ull;       // cell wbase + i
            const unsigned long long am = i > 0 ? sA[i - 1] : 0ull;   // cell wbase + i - 1
            const unsigned long long c = a >> kWinShift;
            if (DEPO) {
                const unsigned long long v = (c << 24) - (a & kWinSumMask) + (am & kWinSumMask);
                if (v) {
                    int node = wbase + i;
                    if (G.periodic && node >= G.ncells) node -= G.ncells;
                    if (node < nn) atomicAdd(Q + node, v);
                }
            }
            if (hist && c) {
                const int cl = wbase + i;
                if (cl < G.ncells) atomicAdd(d.cellcnt + G.cbase + cl, (uint32_t)c);
            }
        }
    }
    if (COLL) {
        const uint32_t nl = 2 * min(s_nc, (uint32_t)kRecLds);
        for (uint32_t i = tid; i < nl; i += 256) d.crec[2 * first + i] = s_rec[i];
        if (tid == 0) d.ctile[t] = s_nc | ctag;
    }
    if (tid == 0 && (PUSH || COLL)) {
        unsigned long long *c = d.cnt + ((int64_t)st * d.nseg + sg) * C_NCNT;
        for (int k = 0; k < C_NCNT; ++k)
            if (s_c[k]) atomicAdd(c + k, (unsigned long long)s_c[k]);
        double *sm = d.sums + ((int64_t)st * d.nseg + sg) * S_NSUM;
        if (s_ke[0] != 0.0) unsafeAtomicAdd(sm + S_KE_L, s_ke[0]);
        if (s_ke[1] != 0.0) unsafeAtomicAdd(sm + S_KE_R, s_ke[1]);
        if (COLL && (s_v2 || s_nal)) {
            const int half = 1 - *d.vcur;
            if (s_v2) atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + sg, s_v2);
            if (PUSH && s_nal) {
                double *ts = step_sums(d, half, st, sg);
                unsafeAtomicAdd(ts + T_V2, s_kes);
                unsafeAtomicAdd(ts + T_N, (double)s_nal);
            }
        }
    }
}

// =======================================================================================
// Counting sort scatter (FP32 form).  Thread t owns slots t, t + 256, ... of the tile, so a
// wave holds 64 consecutive (sorted, so mostly same-cell) particles.  Within a wave the
// lanes of one cell take consecutive ranks from one LDS atomic of their leader; each cell
// of the tile then reserves its output run with one HBM atomic on its cursor.  Lanes of
// one cell thus write consecutive output slots and every store instruction is coalesced.
// Absorbed slots drop out.
// =======================================================================================
template <bool NT, typename T>
__device__ __forceinline__ T ld_nt(const T *p)
{
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}


template <int PPT, bool NT>
__global__ void __launch_bounds__(256) k_sort32(Dev d, int W, int64_t T)
{
    constexpr int TILE = 256 * PPT;
    extern __shared__ unsigned long long s_dyn[];
    uint32_t *sCnt = (uint32_t *)s_dyn;  // [W]
    __shared__ int s_wmn[4], s_wmx[4];
    const int64_t t = tile_of_block();
    if (t >= T) return;
    const int64_t first = t * TILE;
    const int sg = seg_of_slot(d, first);
    const SegC &S = d.seg[sg];
    const int64_t last = min(first + TILE, S.base + d.n_slots[sg]);
    if (first >= last) return;
    const int b = *d.cur, nb = 1 - b;
    const int tid = threadIdx.x, lane = lane_id();
    const int32_t *__restrict__ icell = d.cell[b];
    const float *__restrict__ ioff = d.off[b];
    const float *__restrict__ ivx = d.fvx[b];
    const float *__restrict__ ivy = d.fvy[b];
    const float *__restrict__ ivz = d.fvz[b];
    const uint32_t *__restrict__ iid = d.id[b];
    int cell[PPT];
    float off[PPT], vx[PPT], vy[PPT], vz[PPT];
    uint32_t id[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int64_t i = first + (int64_t)k * 256 + tid;
        cell[k] = kDead;
        if (i < last) {
            cell[k] = ld_nt<NT>(icell + i);
            off[k] = ld_nt<NT>(ioff + i);
            vx[k] = ld_nt<NT>(ivx + i);
            vy[k] = ld_nt<NT>(ivy + i);
            vz[k] = ld_nt<NT>(ivz + i);
            id[k] = ld_nt<NT>(iid + i);
        }
    }
    // the counting window spans the tile's live cells, at most W of them
    int mn = INT32_MAX, mx = -1;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (cell[k] != kDead) {
            mn = min(mn, cell[k]);
            mx = max(mx, cell[k]);
        }
    }
    mn = wave_min_i32(mn);
    mx = wave_max_i32(mx);
    if (lane == 0) {
        s_wmn[tid / kWave] = mn;
        s_wmx[tid / kWave] = mx;
    }
    __syncthreads();
    const int base = min(min(s_wmn[0], s_wmn[1]), min(s_wmn[2], s_wmn[3]));
    const int top = max(max(s_wmx[0], s_wmx[1]), max(s_wmx[2], s_wmx[3]));
    const int Wt = top >= 0 ? min(top - base + 1, W) : 0;
    for (int i = tid; i < Wt; i += 256) sCnt[i] = 0u;
    __syncthreads();
    uint32_t *__restrict__ cursor = d.cursor + S.cbase;
    uint32_t pos[PPT];
    bool inwin[PPT];
    tile_rank<PPT, true>(cell, base, Wt, sCnt, cursor, pos, inwin);
    __syncthreads();
    tile_reserve(sCnt, Wt, cursor, base);
    __syncthreads();
    const int64_t sbase = S.base - d.segstart[sg];
    const int64_t send = S.base + S.cap;
    int32_t *__restrict__ ocell = d.cell[nb];
    float *__restrict__ ooff = d.off[nb];
    float *__restrict__ ovx = d.fvx[nb];
    float *__restrict__ ovy = d.fvy[nb];
    float *__restrict__ ovz = d.fvz[nb];
    uint32_t *__restrict__ oid = d.id[nb];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        if (cell[k] == kDead) continue;
        const uint32_t P = inwin[k] ? sCnt[cell[k] - base] + pos[k] : pos[k];
        const int64_t o = sbase + (int64_t)P;
        if (o < S.base || o >= send) {
            atomicOr(d.err, (int)E_CAP_PART);
            continue;
        }
        // the output runs are scattered: ordinary stores (non-temporal ones measured slower)
        ocell[o] = cell[k];
        ooff[o] = off[k];
        ovx[o] = vx[k];
        ovy[o] = vy[k];
        ovz[o] = vz[k];
        oid[o] = id[k];
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
hipError_t launch_pass32_stages(const Dev &d, int ppt, int W, hipStream_t s, int stages, int hist,
                                int64_t cap_tot, bool nt);

// The sorting pass ranks its tile in 4 more bytes of LDS per window cell; its window span
// is capped so that its LDS stays within what the plain pass's occupancy allows (12 B per
// cell x 1024 cells + the static LDS, seven blocks per CU).  Cells outside the window go
// to HBM atomics, so the cap changes no result.  (Counting cells costs no LDS of its own:
// the window's words carry the counts.)
constexpr int kCountWindowMax = 1024;

template <int STAGES, bool NT = false, bool SORT = false>
static hipError_t launch_pass32_t(const Dev &d, int ppt, int W, hipStream_t s, int hist, int64_t cap_tot)
{
    if (SORT) W = std::min(W, kCountWindowMax);
    const size_t lds = (size_t)W * 8 + (SORT ? (size_t)W * 4 : 0);
    if (ppt == 4) {
        const int64_t T = cap_tot / (256 * 4);
        const int64_t G = (T + 7) / 8 * 8;
        hipLaunchKernelGGL((k_pass32<STAGES, 4, NT, SORT>), dim3(G), dim3(256), lds, s, d, W, hist, T);
    } else {
        const int64_t T = cap_tot / (256 * 8);
        const int64_t G = (T + 7) / 8 * 8;
        hipLaunchKernelGGL((k_pass32<STAGES, 8, NT, SORT>), dim3(G), dim3(256), lds, s, d, W, hist, T);
    }
    return hipGetLastError();
}

// The fused pass that also sorts (after launch_sort_prepare on the previous step's
// histogram), then the new slot counts and the buffer flip.
hipError_t launch_pass32_sort(const Dev &d, int ppt, int W, hipStream_t s, bool coll, int64_t cap_tot, bool nt)
{
    hipError_t e;
    if (coll && nt)
        e = launch_pass32_t<PS_PUSH | PS_COLLIDE | PS_DEPOSIT, true, true>(d, ppt, W, s, 0, cap_tot);
    else if (coll)
        e = launch_pass32_t<PS_PUSH | PS_COLLIDE | PS_DEPOSIT, false, true>(d, ppt, W, s, 0, cap_tot);
    else
        e = launch_pass32_t<PS_PUSH | PS_DEPOSIT, false, true>(d, ppt, W, s, 0, cap_tot);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(256), 0, s, d);
    return hipGetLastError();
}

// A plain copy with the pass's access pattern (256 threads a block, four consecutive 32-bit
// words a thread, one 16-byte load and store each, optionally non-temporal): the measured
// bandwidth and traffic counters of the pass's own kind of stream, for reference.
template <bool NT>
__global__ void __launch_bounds__(256) k_stream_copy(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst,
                                                     int64_t nwords)
{
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
    if (i0 + 4 > nwords) return;  // nwords is a multiple of 4
    uint32_t v[4];
    vload<4, NT>(src + i0, v);
    vstore<4, NT>(dst + i0, v);
}

hipError_t launch_stream_copy(const void *src, void *dst, int64_t nwords, bool nt, hipStream_t s)
{
    const int64_t G = (nwords / 4 + 255) / 256;
    if (G == 0) return hipSuccess;
    if (nt)
        hipLaunchKernelGGL(k_stream_copy<true>, dim3((unsigned)G), dim3(256), 0, s, (const uint32_t *)src,
                           (uint32_t *)dst, nwords);
    else
        hipLaunchKernelGGL(k_stream_copy<false>, dim3((unsigned)G), dim3(256), 0, s, (const uint32_t *)src,
                           (uint32_t *)dst, nwords);
    return hipGetLastError();
}


hipError_t launch_pass32(const Dev &d, int ppt, int W, hipStream_t s, int stages, int hist, int64_t cap_tot,
                         bool nt)
{
    return launch_pass32_stages(d, ppt, W, s, stages, hist, cap_tot, nt);
}

hipError_t launch_pass32_stages(const Dev &d, int ppt, int W, hipStream_t s, int stages, int hist, int64_t cap_tot,
                                bool nt)
{
    if (nt && stages == (PS_PUSH | PS_COLLIDE | PS_DEPOSIT))
        return launch_pass32_t<PS_PUSH | PS_COLLIDE | PS_DEPOSIT, true>(d, ppt, W, s, hist, cap_tot);
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

template <bool NT>
static void launch_sort32_t(const Dev &d, int ppt, int W, hipStream_t s, int64_t cap_tot)
{
    const size_t lds = (size_t)W * 4;
    if (ppt == 4) {
        const int64_t T = cap_tot / (256 * 4);
        hipLaunchKernelGGL((k_sort32<4, NT>), dim3((T + 7) / 8 * 8), dim3(256), lds, s, d, W, T);
    } else {
        const int64_t T = cap_tot / (256 * 8);
        hipLaunchKernelGGL((k_sort32<8, NT>), dim3((T + 7) / 8 * 8), dim3(256), lds, s, d, W, T);
    }
}

hipError_t launch_sort32_scatter(const Dev &d, int ppt, int W, hipStream_t s, int64_t cap_tot, bool nt)
{
    if (nt)
        launch_sort32_t<true>(d, ppt, W, s, cap_tot);
    else
        launch_sort32_t<false>(d, ppt, W, s, cap_tot);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(256), 0, s, d);
    return hipGetLastError();
}

}  // namespace pic
