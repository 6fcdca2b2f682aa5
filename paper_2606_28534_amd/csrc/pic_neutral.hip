// pic_neutral.hip -- recycled neutrals (reading R24) and the volumetric pair source
// (reading R25) of the FP32 form, for the paper's two sheath cases (its table of sheath
// cases: absorbed D+ ions recycled into D neutrals at the walls; an initially empty slab
// filled by a plasma source in its left half).
//
// Neutrals carry no charge: they need no gather, deposit or collision, only a free-streaming
// position update and the wall test, so they live in a compact set of their own (24 B per
// neutral, two buffers) that one kernel streams per step, instead of a third segment of the
// charged pass.  Their order is free (nothing they compute depends on it), so survivors and
// new neutrals are appended with wave-aggregated atomics.
#include "pic_kernels.h"
#include "pic_particle.h"

namespace pic {

#define LAUNCH_CHECK()                     \
    do {                                   \
        hipError_t _e = hipGetLastError(); \
        if (_e != hipSuccess) return _e;   \
    } while (0)

constexpr int kNeutralBlocks = 128;  // blocks per ensemble of the neutral kernel (each takes a ticket)

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
__global__ void __launch_bounds__(256) k_neutrals(Dev d)
{
    __shared__ unsigned long long s_n[2];  // left and right exits
    __shared__ bool s_last;
    if (threadIdx.x < 2) s_n[threadIdx.x] = 0ull;
    __syncthreads();
    const int cur = *d.ncur, nb = 1 - cur;
    const int en = (int)blockIdx.y;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int ion_seg = -1;
    if (en < d.nens && d.ens[en].recycle) {
        const EnsC &e = d.ens[en];
        ion_seg = e.seg[1];
        const int64_t n = min((int64_t)d.nneu[(int64_t)cur * d.nens + en], e.ncap);
        const float dtdx = (float)(e.dt / e.dx);
        const int N = (int)e.ncells;
        uint32_t wl = 0, wr = 0;
        for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x; k0 < n; k0 += stride) {
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
        for (int64_t r0 = (int64_t)blockIdx.x * blockDim.x; r0 < nr; r0 += stride) {
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
    if (threadIdx.x == 0) s_last = (atomicAdd(d.ticket + 5, 1u) == gridDim.x * gridDim.y - 1);
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

// Reading R25: pair k of ensemble e in step n (tag n).  Position: stratified, in the k-th of
// the src_pairs equal parts of [0, src_x), at the fraction given by word 0 of Philox block 4
// of key (seed, 0), counter (k, n), so a step's pairs come out in cell order (their tiles
// deposit through the LDS window like sorted particles); electron velocity: three normals of block 5 of key
// (seed, 0) at v_th,e; ion velocity: three normals of block 5 of key (seed, 1) at v_th,i.
// The pair takes slot and id n_slots + k, next_id + k of its species (before the step's
// ionisation births, which the placement numbers from the advanced counters), deposits its
// charge, enters the sort histogram on sort steps and the speed maxima of the next step's
// null-collision bound.  The last block advances the slot and id counters.
__global__ void __launch_bounds__(256) k_source(Dev d, int hist)
{
    __shared__ bool s_last;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    if (threadIdx.x == 0) s_last = (atomicAdd(d.ticket + 4, 1u) == gridDim.x - 1);
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

}  // namespace pic
