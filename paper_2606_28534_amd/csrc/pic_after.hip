// pic_after.hip -- the FP32 form's kernels that follow the particle pass: the collision
// candidates (the ~1% of particles whose null-collision test passed), the recycled
// neutrals (reading R24) and the volumetric pair source (reading R25) of the paper's two
// sheath cases (its table of sheath cases: absorbed D+ ions recycled into D neutrals at the
// walls; an initially empty slab filled by a plasma source in its left half).  The three
// read only what the pass wrote and touch disjoint state, so the fused step runs them as
// one launch whose block ranges take one body each (k_after); the separate stages launch
// them one by one.
//
// Neutrals carry no charge: they need no gather, deposit or collision, only a free-streaming
// position update and the wall test, so they live in a compact set of their own (24 B per
// neutral, two buffers) that one kernel streams per step, instead of a third segment of the
// charged pass.  Their order is free (nothing they compute depends on it), so survivors and
// new neutrals are appended with wave-aggregated atomics.
#include <algorithm>

#include "pic_kernels.h"
#include "pic_particle.h"

namespace pic {

#define LAUNCH_CHECK()                     \
    do {                                   \
        hipError_t _e = hipGetLastError(); \
        if (_e != hipSuccess) return _e;   \
    } while (0)

constexpr int kNeutralBlocks = 128;  // blocks per ensemble of the neutral kernel (each takes a ticket)

// =======================================================================================
// Null-collision candidates of the FP32 pass.  A block takes cand_tiles(T) consecutive tiles;
// their candidate records (post-push state and slot, written by the pass) are concatenated
// through a prefix of the tile counts, one candidate per thread.  Each candidate draws the
// full Philox block 0 again, picks its channel (in FP64, the same decision in both
// precisions), scatters, writes its velocity back to its slot, and on ionisation appends
// the new pair.  Collision counts and the largest post-collision speed are gathered in LDS
// per segment and go out once per block and segment.
//
// The block's critical path is a chain of dependent global round trips, so it is kept
// short: the tile counts carry their tile's segment and ensemble (cand_tag), so one load
// gives the block what it needs to stage those segments' constants and collision bounds
// in LDS, in the same round trip as the candidate records; then the birth reservation.
// =======================================================================================
// Tiles per block: a block's time is a chain of round trips per round of 256 candidates,
// so the kernel is fastest when its blocks fit one wave of resident blocks (four per CU at
// its registers, 1024 on the chip) without making each block's rounds many: the
// 4e7-particle slab's 4.9e4 tiles take 48 per block, 1018 blocks (16: 29.6 us, 24: 25.3 us,
// 32: 24.5 us, 40: 23.7 us, 48: 23.3 us, 64: 27.7 us); the 64 batched ensembles' 5e5 tiles
// take the most, 64 (156 us at 32, 124 us at 64).
constexpr int kCandTilesMax = 64;  // one lane of the first wave per tile
__host__ __forceinline__ int cand_tiles(int64_t T)
{
    return (int)std::min<int64_t>(kCandTilesMax, std::max<int64_t>(32, (T + 1023) / 1024));
}
constexpr int kCandSegs = 12;  // segments a block stages (more: read from global memory)

// Block `bid` (a kernel of its own, or the first blocks of the kernel that follows the pass).
template <bool CXREL>
__device__ void cand_body(const Dev &d, int tile, int64_t T, int hist, int bid, int ct)
{
    __shared__ uint32_t s_pre[kCandTilesMax + 1];
    __shared__ int s_tj[kCandTilesMax];  // staged entry of each tile's segment (-1: not staged)
    // staged segment constants: entry j is segment s_sg[j] of ensemble s_en[j]
    __shared__ SegC s_seg[kCandSegs];
    __shared__ EnsC s_ens[kCandSegs];
    __shared__ double s_nu[kCandSegs][2];  // nu_max, P_null
    __shared__ int s_sg[kCandSegs], s_en[kCandSegs];
    __shared__ int s_ns;
    // block tallies per staged entry (segments that are not staged send theirs with
    // atomics of their own)
    __shared__ uint32_t s_n[kCandSegs][3];
    __shared__ unsigned long long s_v[kCandSegs];
    // scalar diagnostics of the step: the change of sum |v|^2 from collisions and births,
    // and the births per segment
    __shared__ double s_dk[kCandSegs];
    __shared__ uint32_t s_dn[kCandSegs];
    // births of one round of the block: counted in LDS, then one reservation in the list
    __shared__ uint32_t s_nb, s_bbase;
    const int64_t t0 = (int64_t)bid * ct;
    // per-launch values, read with the tile counts
    const int b = *d.cur;
    const uint32_t tag = (uint32_t)(*d.step);
    const int half = 1 - *d.vcur;
    if (threadIdx.x < kWave) {
        // the first wave loads the tile counts in parallel, resets them, scans, and lists
        // the distinct segments of the tiles that hold candidates
        const int k = threadIdx.x;
        const int64_t t = t0 + k;
        uint32_t w = 0;
        if (k < ct && t < T) {
            w = d.ctile[t];
            d.ctile[t] = 0u;
        }
        const uint32_t c = w & kCandCountMask;
        uint32_t inc = c;
#pragma unroll
        for (int o = 1; o < kCandTilesMax; o <<= 1) {
            const uint32_t n = __shfl_up(inc, o);
            if (k >= o) inc += n;
        }
        // a tile opens a new entry when it holds candidates and its segment differs from
        // that of the last earlier tile with candidates (segments grow with the slot, so
        // the keys of such tiles never decrease: the previous one is the running maximum
        // over the lanes below)
        const int key = c ? (int)((w >> 12) & 0x3FFu) : -1;
        int pm = key;
#pragma unroll
        for (int o = 1; o < kCandTilesMax; o <<= 1) {
            const int n = __shfl_up(pm, o);
            if (k >= o) pm = max(pm, n);
        }
        int before = __shfl_up(pm, 1);
        if (k == 0) before = -1;
        const bool head = key >= 0 && key != before;
        const unsigned long long hm = __ballot(head);
        const int hidx = __popcll(hm & ((1ull << k) - 1ull)) - (head ? 0 : 1);  // entry of the run k is in
        if (k < ct) {
            s_pre[k] = inc - c;
            s_tj[k] = (key >= 0 && hidx < kCandSegs) ? hidx : -1;
        }
        if (k == ct - 1) s_pre[ct] = inc;
        if (head && hidx < kCandSegs) {
            s_sg[hidx] = key;
            s_en[hidx] = (int)(w >> 22);
        }
        if (k == 0) s_ns = min(__popcll(hm), kCandSegs);
        if (k < kCandSegs) {
            s_n[k][0] = s_n[k][1] = s_n[k][2] = 0u;
            s_v[k] = 0ull;
            s_dk[k] = 0.0;
            s_dn[k] = 0u;
        }
    }
    __syncthreads();
    const uint32_t m = s_pre[ct];
    if (m == 0) return;
    {
        // stage the segments' constants (word copies; all loads in one round trip)
        const int ns = s_ns;
        constexpr int WS = sizeof(SegC) / 4, WE = sizeof(EnsC) / 4;
        static_assert(sizeof(SegC) % 4 == 0 && sizeof(EnsC) % 4 == 0, "word copies");
        for (int i = threadIdx.x; i < ns * (WS + WE + 2); i += blockDim.x) {
            const int j = i / (WS + WE + 2), o = i % (WS + WE + 2);
            if (o < WS)
                ((uint32_t *)&s_seg[j])[o] = ((const uint32_t *)(d.seg + s_sg[j]))[o];
            else if (o < WS + WE)
                ((uint32_t *)&s_ens[j])[o - WS] = ((const uint32_t *)(d.ens + s_en[j]))[o - WS];
            else if (o == WS + WE)
                s_nu[j][0] = d.numax[s_sg[j]];
            else
                s_nu[j][1] = d.pnull[s_sg[j]];
        }
    }
    const BirthBuf bb = birth_buf(d, (int)(tag & 1u));
    const int st = stripe_of_block();          // counters and speed maxima
    const int bst = bid & (kStripes - 1);  // birth list
    for (uint32_t q0 = 0; q0 < m; q0 += blockDim.x) {
        const uint32_t q = q0 + threadIdx.x;
        const bool act = q < m;
        // this candidate's tile: the last k with s_pre[k] <= q (tiles without candidates
        // share their prefix with the next tile, which this picks)
        int k = 0;
        uint4 r0 = make_uint4(0u, 0u, 0u, 0u), r1 = r0;
        if (act) {
            int lo = 0, hi = ct;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_pre[mid] <= q)
                    lo = mid;
                else
                    hi = mid;
            }
            k = lo;
            const uint4 *r = d.crec + 2 * ((t0 + k) * (int64_t)tile + (q - s_pre[k]));
            r0 = r[0];
            r1 = r[1];
        }
        if (q0 == 0) __syncthreads();  // the staged constants are in place
        int ch = -1, sg = 0, j = -1;
        PS<false> p;
        double ve[3], vi[3];
        int64_t i = 0;
        int oth = -1;  // the ion segment of an electron segment (births)
        if (act) {
            j = s_tj[k];
            i = (int64_t)r0.x;
            sg = (int)r1.w;
            p.cell = (int)r0.y;
            p.off = __uint_as_float(r0.z);
            p.id = r0.w;
            p.vx = __uint_as_float(r1.x);
            p.vy = __uint_as_float(r1.y);
            p.vz = __uint_as_float(r1.z);
            if (j >= 0) {
                const SegC &S = s_seg[j];
                const EnsC &e = s_ens[j];
                oth = S.other;
                ch = p_collide<false, CXREL>(e, S, S.species, s_nu[j][0], s_nu[j][1], tag, p, ve, vi);
            } else {
                const SegC S = d.seg[sg];
                const EnsC e = d.ens[S.ens];
                oth = S.other;
                ch = p_collide<false, CXREL>(e, S, S.species, d.numax[sg], d.pnull[sg], tag, p, ve, vi);
            }
        }
        if (ch >= 0) {
            d.fvx[b][i] = p.vx;
            d.fvy[b][i] = p.vy;
            d.fvz[b][i] = p.vz;
            // the particle's |v|^2 after the collision replaces the one the pass tallied
            // (taken off exactly as the pass computed it); an ionisation adds the new
            // electron here and the new ion below (as stored, in binary32)
            double dk = speed2_rn(p.vx, p.vy, p.vz) -
                        (double)speed2_f32(__uint_as_float(r1.x), __uint_as_float(r1.y), __uint_as_float(r1.z));
            if (ch == 1) dk += speed2_rn((float)ve[0], (float)ve[1], (float)ve[2]);
            if (j >= 0) {
                atomicAdd(&s_n[j][ch], 1u);
                atomicAdd(&s_dk[j], dk);
                if (ch == 1) atomicAdd(&s_dn[j], 1u);
            } else {
                unsigned long long *c = d.cnt + ((int64_t)st * d.nseg + sg) * C_NCNT;
                atomicAdd(c + (ch == 0 ? C_EL : ch == 1 ? C_IZ : C_CX), 1ull);
                double *ts = step_sums(d, half, st, sg);
                unsafeAtomicAdd(ts + T_V2, dk);
                if (ch == 1) unsafeAtomicAdd(ts + T_N, 1.0);
            }
        }
        if (act) {
            double v2m = speed2_rn(p.vx, p.vy, p.vz);
            if (ch == 1) {
                v2m = fmax(v2m, speed2_rn(ve[0], ve[1], ve[2]));
                if (oth >= 0) {
                    // the new ion: its speed bound and diagnostics go to the ion segment
                    // directly (one of a few per block)
                    const double ki = speed2_rn((float)vi[0], (float)vi[1], (float)vi[2]);
                    double *ts = step_sums(d, half, st, oth);
                    unsafeAtomicAdd(ts + T_V2, ki);
                    unsafeAtomicAdd(ts + T_N, 1.0);
                    atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + oth,
                              dbits(speed2_rn(vi[0], vi[1], vi[2])));
                }
            }
            if (j >= 0) {
                if (v2m > 0.0) atomicMax(&s_v[j], dbits(v2m));
            } else if (v2m > 0.0) {
                atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + sg, dbits(v2m));
            }
        }
        // births of this round: one list reservation for the whole block
        if (threadIdx.x == 0) s_nb = 0u;
        __syncthreads();
        uint32_t lb = 0;
        if (ch == 1) lb = atomicAdd(&s_nb, 1u);
        __syncthreads();
        if (threadIdx.x == 0 && s_nb) s_bbase = atomicAdd(bb.nbirth + bst, s_nb);
        // the deposit of the new pair (the fused step's; the separate stages deposit all
        // particles afresh), while the reservation is in flight
        if (ch == 1) {
            const SegC Se = j >= 0 ? s_seg[j] : d.seg[sg];
            global_deposit32(d, Se, Se.species, p.cell, p.off, hist != 0);
            if (oth >= 0) {
                const SegC So = d.seg[oth];
                global_deposit32(d, So, 1, p.cell, p.off, hist != 0);
            }
        }
        __syncthreads();
        if (ch == 1) {
            const uint32_t slot = s_bbase + lb;
            if ((int64_t)slot < d.birth_stripe_cap) {
                const int ens = j >= 0 ? s_seg[j].ens : d.seg[sg].ens;
                const double dx = j >= 0 ? s_seg[j].dx : d.seg[sg].dx;
                Birth &B = bb.births[(int64_t)bst * d.birth_stripe_cap + slot];
                B.pid = p.id;
                B.ens = ens;
                B.cell = p.cell;
                B.off = p.off;
                B.x = ((double)p.cell + (double)p.off) * dx;
                for (int c = 0; c < 3; ++c) {
                    B.ve[c] = ve[c];
                    B.vi[c] = vi[c];
                }
                if (j >= 0)
                    birth_mark(bb, s_ens[j], p.id);
                else
                    birth_mark(bb, d.ens[ens], p.id);
            } else {
                atomicOr(d.err, (int)E_CAP_BIRTH);
            }
        }
        __syncthreads();  // s_nb and s_bbase are reused by the next round
    }
    // one set of counter atomics per block and staged segment
    if ((int)threadIdx.x < s_ns) {
        const int j = threadIdx.x, sgj = s_sg[j];
        unsigned long long *c = d.cnt + ((int64_t)st * d.nseg + sgj) * C_NCNT;
        if (s_n[j][0]) atomicAdd(c + C_EL, (unsigned long long)s_n[j][0]);
        if (s_n[j][1]) atomicAdd(c + C_IZ, (unsigned long long)s_n[j][1]);
        if (s_n[j][2]) atomicAdd(c + C_CX, (unsigned long long)s_n[j][2]);
        if (s_v[j]) atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + sgj, s_v[j]);
        if (s_dk[j] != 0.0 || s_dn[j]) {
            double *ts = step_sums(d, half, st, sgj);
            if (s_dk[j] != 0.0) unsafeAtomicAdd(ts + T_V2, s_dk[j]);
            if (s_dn[j]) unsafeAtomicAdd(ts + T_N, (double)s_dn[j]);
        }
    }
}

template <bool CXREL>
__global__ void __launch_bounds__(256) k_cand32(Dev d, int tile, int64_t T, int hist, int ct)
{
    cand_body<CXREL>(d, tile, T, hist, (int)blockIdx.x, ct);
}


// x in [0, L) (FP64) to the FP32 form's cell and offset, as the host upload converts it; a
// value that rounds up to L stays in the last cell.
__device__ __forceinline__ void x_to_celloff(double x, double dx, int N, int &cell, float &off)
{
    const double g = x / dx;
    const double jf = floor(g);
    int cl = (int)jf;
    float o = (float)(g - jf);
    if (o >= 1.0f) {
        o = 0.0f;
        cl += 1;
    }
    if (cl >= N) {
        cl = N - 1;
        o = 0x1.fffffep-1f;
    }
    if (cl < 0) {
        cl = 0;
        o = 0.0f;
    }
    cell = cl;
    off = o;
}

// Append this lane's neutral (if `keep`) to buffer `nb` of ensemble e: one atomic per wave.
__device__ __forceinline__ void neutral_append(const Dev &d, const EnsC &e, int en, int nb, bool keep,
                                               int c, float o, float vx, float vy, float vz,
                                               uint32_t id)
{
    const unsigned long long m = __ballot(keep);
    if (m == 0ull) return;
    const int lane = lane_id();
    unsigned long long base = 0;
    if (lane == __ffsll((long long)m) - 1)
        base = atomicAdd(d.nneu + (int64_t)nb * d.nens + en, (unsigned long long)__popcll(m));
    base = __shfl(base, __ffsll((long long)m) - 1);
    if (!keep) return;
    const unsigned long long below = m & ((1ull << lane) - 1ull);
    const int64_t pos = (int64_t)(base + (unsigned long long)__popcll(below));
    if (pos >= e.ncap) {
        atomicOr(d.err, (int)E_CAP_PART);
        return;
    }
    const int64_t i = e.nbase + pos;
    d.ncell[nb][i] = c;
    d.noff[nb][i] = o;
    d.nvx[nb][i] = vx;
    d.nvy[nb][i] = vy;
    d.nvz[nb][i] = vz;
    d.nid[nb][i] = id;
}

// Reading R24, per step: blocks (x, en) for en < nens stream ensemble en's neutrals (free
// flight x += v_x dt, the same binary32 cell+offset arithmetic as the charged push; those
// that leave are counted per wall); blocks (x, nens) turn the ions the pass listed as
// absorbed into neutrals.  Philox block 0 of key (seed, 2), counter (ion id, step): u1 the
// inward normal speed v_w sqrt(-2 ln u1) (flux-weighted half-Maxwellian at T_n), (u2, u3)
// the tangential components by Box-Muller, u4 the fraction of dt |v_x| it has flown.
// The last block to finish makes the streamed buffer current, empties the other one and
// clears the absorbed-ion list.
// Block (bx, by) of an nbx x nby arrangement (a kernel of its own, or a range of blocks of
// the kernel that follows the pass).
__device__ void neutrals_body(const Dev &d, int bx, int by, int nbx, int nby)
{
    __shared__ unsigned long long s_n[2];  // left and right exits
    __shared__ bool s_last;
    if (threadIdx.x < 2) s_n[threadIdx.x] = 0ull;
    __syncthreads();
    const int cur = *d.ncur, nb = 1 - cur;
    const int en = by;
    const int64_t stride = (int64_t)nbx * blockDim.x;
    int ion_seg = -1;
    if (en < d.nens && d.ens[en].recycle) {
        const EnsC &e = d.ens[en];
        ion_seg = e.seg[1];
        const int64_t n = min((int64_t)d.nneu[(int64_t)cur * d.nens + en], e.ncap);
        const float dtdx = (float)(e.dt / e.dx);
        const int N = (int)e.ncells;
        uint32_t wl = 0, wr = 0;
        for (int64_t k0 = (int64_t)bx * blockDim.x; k0 < n; k0 += stride) {
            const int64_t k = k0 + threadIdx.x;
            bool keep = false;
            int c = 0;
            float o = 0.f, vx = 0.f, vy = 0.f, vz = 0.f;
            uint32_t id = 0;
            if (k < n) {
                const int64_t i = e.nbase + k;
                c = d.ncell[cur][i];
                o = d.noff[cur][i];
                vx = d.nvx[cur][i];
                vy = d.nvy[cur][i];
                vz = d.nvz[cur][i];
                id = d.nid[cur][i];
                float q = o + vx * dtdx;
                const float fl = floorf(q);
                c += (int)fl;
                q -= fl;
                const bool up = q >= 1.0f;
                o = up ? q - 1.0f : q;
                c += up ? 1 : 0;
                if (c < 0)
                    ++wl;
                else if (c >= N)
                    ++wr;
                else
                    keep = true;
            }
            neutral_append(d, e, en, nb, keep, c, o, vx, vy, vz, id);
        }
        if (wl) atomicAdd(&s_n[0], (unsigned long long)wl);
        if (wr) atomicAdd(&s_n[1], (unsigned long long)wr);
    } else if (en == d.nens) {
        const int64_t nr = min((int64_t)*d.nrec, d.rec_cap);
        const uint32_t tag = (uint32_t)(*d.step);
        for (int64_t r0 = (int64_t)bx * blockDim.x; r0 < nr; r0 += stride) {
            const int64_t r = r0 + threadIdx.x;
            if (r >= nr) break;
            const uint2 rec = d.recs[r];
            const int re = (int)(rec.y >> 1), wall = (int)(rec.y & 1u);
            const EnsC &e = d.ens[re];
            const uint4 w = draw(e.seed, 2, rec.x, tag, 0u);
            const double vw = e.vn;
            const double vn = vw * sqrt(-2.0 * log(u01d(w.x)));
            double ty, tz;
            {
                const double rad = sqrt(-2.0 * log(u01d(w.y)));
                double sn, cs;
                sincos(6.283185307179586476925286766559 * u01d(w.z), &sn, &cs);
                ty = rad * cs;
                tz = rad * sn;
            }
            const double depth = u01d(w.w) * e.dt * vn;
            const double x = wall == 0 ? depth : e.L - depth;
            int c;
            float o;
            x_to_celloff(x, e.dx, (int)e.ncells, c, o);
            const float vx = (float)(wall == 0 ? vn : -vn);
            // records of one wave may belong to different ensembles: one append per lane
            const unsigned long long pos = atomicAdd(d.nneu + (int64_t)nb * d.nens + re, 1ull);
            if ((int64_t)pos >= e.ncap) {
                atomicOr(d.err, (int)E_CAP_PART);
                continue;
            }
            const int64_t i = e.nbase + (int64_t)pos;
            d.ncell[nb][i] = c;
            d.noff[nb][i] = o;
            d.nvx[nb][i] = vx;
            d.nvy[nb][i] = (float)(vw * ty);
            d.nvz[nb][i] = (float)(vw * tz);
            d.nid[nb][i] = rec.x;
            atomicAdd(d.cnt + ((int64_t)stripe_of_block() * d.nseg + e.seg[1]) * C_NCNT + C_RECYCLED, 1ull);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && ion_seg >= 0) {
        unsigned long long *c = d.cnt + ((int64_t)stripe_of_block() * d.nseg + ion_seg) * C_NCNT;
        if (s_n[0]) atomicAdd(c + C_NWALL_L, s_n[0]);
        if (s_n[1]) atomicAdd(c + C_NWALL_R, s_n[1]);
    }
    // The last block only empties the buffer every block has finished reading and flips;
    // no block of this launch reads what it writes, so no device-scope fence is needed
    // (on gfx950 one writes back the XCD's L2 and costs microseconds per block).
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(d.ticket + 5, 1u) == (unsigned)(nbx * nby - 1));
    __syncthreads();
    if (!s_last) return;
    for (int e2 = threadIdx.x; e2 < d.nens; e2 += blockDim.x) d.nneu[(int64_t)cur * d.nens + e2] = 0ull;
    __syncthreads();
    if (threadIdx.x == 0) {
        *d.ncur = nb;
        *d.nrec = 0u;
        d.ticket[5] = 0u;
    }
}

__global__ void __launch_bounds__(256) k_neutrals(Dev d)
{
    neutrals_body(d, (int)blockIdx.x, (int)blockIdx.y, (int)gridDim.x, (int)gridDim.y);
}

// Reading R25: pair k of ensemble e in step n (tag n).  Position: stratified, in the k-th of
// the src_pairs equal parts of [0, src_x), at the fraction given by word 0 of Philox block 4
// of key (seed, 0), counter (k, n), so a step's pairs come out in cell order (their tiles
// deposit through the LDS window like sorted particles); electron velocity: three normals of block 5 of key
// (seed, 0) at v_th,e; ion velocity: three normals of block 5 of key (seed, 1) at v_th,i.
// The pair takes slot and id n_slots + k, next_id + k of its species (before the step's
// ionisation births, which the placement numbers from the advanced counters), deposits its
// charge, enters the sort histogram on sort steps and the speed maxima of the next step's
// null-collision bound.  The last block advances the slot and id counters.
// Block `bid` of `nblk` (a kernel of its own, or a range of blocks of the kernel that
// follows the pass).
__device__ void source_body(const Dev &d, int hist, int bid, int nblk)
{
    __shared__ bool s_last;
    const int64_t g = (int64_t)bid * blockDim.x + threadIdx.x;
    const int b = *d.cur;
    const uint32_t tag = (uint32_t)(*d.step);
    const int half = 1 - *d.vcur;
    const int st = stripe_of_block();
    double v2e = 0.0, v2i = 0.0;
    uint32_t made = 0;  // bit s: the pair member of species s was created
    int en = -1;
    if (g < d.src_tot) {
        int lo = 0, hi = d.nens;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (d.ens[mid].src_base <= g)
                lo = mid;
            else
                hi = mid;
        }
        en = lo;  // the last ensemble whose range starts at or before g holds it
        const EnsC &e = d.ens[en];
        const int64_t k = g - e.src_base;
        const uint4 w = draw(e.seed, 0, (uint32_t)k, tag, 4u);
        const double x = e.src_x * (((double)k + u01d(w.x)) / (double)e.src_pairs);
        int c;
        float o;
        x_to_celloff(x, e.dx, (int)e.ncells, c, o);
        for (int s = 0; s < 2; ++s) {
            const int sg = e.seg[s];
            const SegC &S = d.seg[sg];
            double z[3];
            three_normals<double>(draw(e.seed, s, (uint32_t)k, tag, 5u), z);
            const float vx = (float)(S.vth * z[0]), vy = (float)(S.vth * z[1]), vz = (float)(S.vth * z[2]);
            const int64_t slot = d.n_slots[sg] + k;
            if (slot >= S.cap) {
                atomicOr(d.err, (int)E_CAP_PART);
                continue;
            }
            if ((int64_t)d.next_id[sg] + k >= e.idcap) {
                atomicOr(d.err, (int)E_CAP_ID);
                continue;
            }
            const int64_t i = S.base + slot;
            d.cell[b][i] = c;
            d.off[b][i] = o;
            d.fvx[b][i] = vx;
            d.fvy[b][i] = vy;
            d.fvz[b][i] = vz;
            d.id[b][i] = d.next_id[sg] + (uint32_t)k;
            global_deposit32(d, S, s, c, o, hist != 0);
            const double v2 = speed2_rn((double)vx, (double)vy, (double)vz);
            if (s == 0)
                v2e = v2;
            else
                v2i = v2;
            made |= 1u << s;
        }
    }
    // the fused step's scalar diagnostics: the new particles' |v|^2 and count
    {
        const int en0s = __shfl(en, 0);
        if (__all(en == en0s || en < 0)) {
            const double ke = wave_sum_f64(v2e), ki = wave_sum_f64(v2i);
            const uint32_t ne = wave_sum_u32(made & 1u), ni = wave_sum_u32((made >> 1) & 1u);
            if (lane_id() == 0 && en0s >= 0) {
                const EnsC &e = d.ens[en0s];
                if (ne) {
                    double *ts = step_sums(d, half, st, e.seg[0]);
                    unsafeAtomicAdd(ts + T_V2, ke);
                    unsafeAtomicAdd(ts + T_N, (double)ne);
                }
                if (ni) {
                    double *ts = step_sums(d, half, st, e.seg[1]);
                    unsafeAtomicAdd(ts + T_V2, ki);
                    unsafeAtomicAdd(ts + T_N, (double)ni);
                }
            }
        } else if (en >= 0) {
            const EnsC &e = d.ens[en];
            for (int s = 0; s < 2; ++s) {
                if (!((made >> s) & 1u)) continue;
                double *ts = step_sums(d, half, st, e.seg[s]);
                unsafeAtomicAdd(ts + T_V2, s == 0 ? v2e : v2i);
                unsafeAtomicAdd(ts + T_N, 1.0);
            }
        }
    }
    // the new speeds enter the half of the speed maxima this step accumulates: one atomic
    // per wave when the wave's pairs share an ensemble
    const int en0 = __shfl(en, 0);
    if (__all(en == en0 || en < 0)) {
        const double me = wave_max_f64(v2e), mi = wave_max_f64(v2i);
        if (lane_id() == 0 && en0 >= 0) {
            const EnsC &e = d.ens[en0];
            atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + e.seg[0], dbits(me));
            atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + e.seg[1], dbits(mi));
        }
    } else if (en >= 0) {
        const EnsC &e = d.ens[en];
        atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + e.seg[0], dbits(v2e));
        atomicMax(d.vmax2 + ((int64_t)half * kCntStripes + st) * d.nseg + e.seg[1], dbits(v2i));
    }
    // the last block advances counters every block read before taking its ticket (no fence
    // needed, as in the neutral kernel)
    __syncthreads();
    if (threadIdx.x == 0) s_last = (atomicAdd(d.ticket + 4, 1u) == (unsigned)(nblk - 1));
    __syncthreads();
    if (!s_last) return;
    for (int e2 = threadIdx.x; e2 < d.nens; e2 += blockDim.x) {
        const EnsC &e = d.ens[e2];
        if (e.src_pairs == 0) continue;
        for (int s = 0; s < 2; ++s) {
            const int sg = e.seg[s];
            d.n_slots[sg] = min(d.n_slots[sg] + e.src_pairs, d.seg[sg].cap);
            d.next_id[sg] += (uint32_t)e.src_pairs;
        }
        atomicAdd(d.cnt + (int64_t)e.seg[0] * C_NCNT + C_SOURCED, (unsigned long long)e.src_pairs);
    }
    __syncthreads();
    if (threadIdx.x == 0) d.ticket[4] = 0u;
}

__global__ void __launch_bounds__(256) k_source(Dev d, int hist) { source_body(d, hist, (int)blockIdx.x, (int)gridDim.x); }

hipError_t launch_neutrals(const Dev &d, hipStream_t s)
{
    if (d.ncap_tot == 0) return hipSuccess;
    hipLaunchKernelGGL(k_neutrals, dim3(kNeutralBlocks, d.nens + 1), dim3(256), 0, s, d);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_source(const Dev &d, int hist, hipStream_t s)
{
    if (d.src_tot == 0) return hipSuccess;
    const int64_t blocks = (d.src_tot + 255) / 256;
    hipLaunchKernelGGL(k_source, dim3((unsigned)blocks), dim3(256), 0, s, d, hist);
    LAUNCH_CHECK();
    return hipSuccess;
}

hipError_t launch_cand32(const Dev &d, int ppt, hipStream_t s, int hist, int64_t cap_tot)
{
    const int tile = 256 * ppt;
    const int64_t T = cap_tot / tile;
    const int ct = cand_tiles(T);
    const dim3 g((unsigned)((T + ct - 1) / ct));
    if (d.any_cx_rel)
        hipLaunchKernelGGL(k_cand32<true>, g, dim3(256), 0, s, d, tile, T, hist, ct);
    else
        hipLaunchKernelGGL(k_cand32<false>, g, dim3(256), 0, s, d, tile, T, hist, ct);
    return hipGetLastError();
}

// The fused step's kernel after the pass: blocks [0, nc) take the candidate tiles, the next
// nn = kNeutralBlocks x (nens + 1) the neutrals, the rest the source pairs.  Each range runs
// the body its own kernel would, so the results are those of the three launches.
template <bool CXREL>
__global__ void __launch_bounds__(256) k_after(Dev d, int tile, int64_t T, int hist, int nc, int nn, int ct)
{
    const int b = (int)blockIdx.x;
    if (b < nc) {
        cand_body<CXREL>(d, tile, T, hist, b, ct);
    } else if (b < nc + nn) {
        const int k = b - nc;
        neutrals_body(d, k % kNeutralBlocks, k / kNeutralBlocks, kNeutralBlocks, d.nens + 1);
    } else {
        source_body(d, hist, b - nc - nn, (int)gridDim.x - nc - nn);
    }
}

hipError_t launch_after(const Dev &d, int ppt, hipStream_t s, int hist, int64_t cap_tot, bool coll)
{
    const int tile = 256 * ppt;
    const int64_t T = cap_tot / tile;
    const int ct = cand_tiles(T);
    const int nc = coll ? (int)((T + ct - 1) / ct) : 0;
    const int nn = d.ncap_tot ? kNeutralBlocks * (d.nens + 1) : 0;
    const int ns = d.src_tot ? (int)((d.src_tot + 255) / 256) : 0;
    if (nc + nn + ns == 0) return hipSuccess;
    const dim3 g((unsigned)(nc + nn + ns));
    if (d.any_cx_rel)
        hipLaunchKernelGGL(k_after<true>, g, dim3(256), 0, s, d, tile, T, hist, nc, nn, ct);
    else
        hipLaunchKernelGGL(k_after<false>, g, dim3(256), 0, s, d, tile, T, hist, nc, nn, ct);
    return hipGetLastError();
}

}  // namespace pic
