// pic_particle.h -- per-particle device code shared by the particle kernels: register
// state, gather + Boris push + walls, null-collision decision and kinematics, and the
// direct (HBM atomic) cloud-in-cell deposit of a single particle.
#pragma once
#include <type_traits>

#include "pic_device.h"

namespace pic {

// =======================================================================================
// Particle state in registers.
// =======================================================================================
template <bool F64>
struct PS;
template <>
struct PS<false> {
    int cell;
    float off, vx, vy, vz;
    uint32_t id;
};
template <>
struct PS<true> {
    double x, vx, vy, vz;
    uint32_t id;
};

template <bool F64>
__device__ __forceinline__ void p_load(const Dev &d, int b, int64_t i, PS<F64> &p, bool need_v,
                                       bool need_id)
{
    if constexpr (!F64) {
        p.cell = d.cell[b][i];
        if (p.cell == kDead) return;
        p.off = d.off[b][i];
        if (need_v) {
            p.vx = d.fvx[b][i];
            p.vy = d.fvy[b][i];
            p.vz = d.fvz[b][i];
        }
    } else {
        // every load is issued at once (a dead slot's velocity is read and not used), so a
        // tile waits for memory once
        p.x = d.x[b][i];
        if (need_v) {
            p.vx = d.dvx[b][i];
            p.vy = d.dvy[b][i];
            p.vz = d.dvz[b][i];
        }
    }
    if (need_id) p.id = d.id[b][i];
}

template <bool F64>
__device__ __forceinline__ bool p_alive(const PS<F64> &p)
{
    if constexpr (!F64)
        return p.cell != kDead;
    else
        return p.x >= 0.0;
}

template <bool F64>
__device__ __forceinline__ void p_kill(PS<F64> &p)
{
    if constexpr (!F64)
        p.cell = kDead;
    else
        p.x = -1.0;
}

// Cell index and fraction of an absolute position in [0, L): x / dx may round up to N
// for x just below L, which is folded back into the last cell.
__device__ __forceinline__ int64_t cell_of_x(const SegC &S, double x, double &f)
{
    const double g = x / S.dx;
    double jf = floor(g);
    if (jf > (double)(S.ncells - 1)) jf = (double)(S.ncells - 1);
    if (!(jf >= 0.0)) jf = 0.0;
    f = g - jf;
    return (int64_t)jf;
}

// Cell index and in-cell fraction.
template <bool F64>
__device__ __forceinline__ int p_cell(const SegC &S, const PS<F64> &p, double &f)
{
    if constexpr (!F64) {
        f = (double)p.off;
        return p.cell;
    } else {
        return (int)cell_of_x(S, p.x, f);
    }
}

// Boris rotation in the given precision: half kick, v' = v- + v- x t, v+ = v- + v' x s,
// half kick.
template <typename T>
__device__ __forceinline__ void boris(T h, const T t[3], const T s[3], T Ep, T &vx, T &vy, T &vz)
{
    T ax = vx + h * Ep, ay = vy, az = vz;
    const T px = ax + (ay * t[2] - az * t[1]);
    const T py = ay + (az * t[0] - ax * t[2]);
    const T pz = az + (ax * t[1] - ay * t[0]);
    ax += py * s[2] - pz * s[1];
    ay += pz * s[0] - px * s[2];
    az += px * s[1] - py * s[0];
    vx = ax + h * Ep;
    vy = ay;
    vz = az;
}

// The segment constants of the FP64 gather, push and deposit, copied into registers once
// per tile: after a particle store or atomic, a read through a reference into global
// memory would be repeated, since the store might alias it.
struct Seg64 {
    int64_t gbase, cbase;
    int32_t ncells, periodic;
    double dx, dt, h, t[3], s[3], L, E_ext;
    double rdx;  // 1 / dx when dx is a power of two (x / dx = x * rdx exactly), else 0
};

__device__ __forceinline__ Seg64 seg64(const SegC &S, const EnsC &e)
{
    int ex;
    const bool pow2 = frexp(S.dx, &ex) == 0.5;  // dx = 2^(ex - 1)
    return Seg64{S.gbase, S.cbase, S.ncells, S.periodic, S.dx, S.dt, S.h,
                 {S.t[0], S.t[1], S.t[2]}, {S.s[0], S.s[1], S.s[2]}, e.L, e.E_ext,
                 pow2 ? ldexp(1.0, 1 - ex) : 0.0};
}

// Cell index and fraction of x (as cell_of_x; the division is a multiplication, with the
// same result, when dx is a power of two).
__device__ __forceinline__ int64_t cell_of_x64(const Seg64 &G, double x, double &f)
{
    const double g = G.rdx != 0.0 ? x * G.rdx : x / G.dx;
    double jf = floor(g);
    if (jf > (double)(G.ncells - 1)) jf = (double)(G.ncells - 1);
    if (!(jf >= 0.0)) jf = 0.0;
    f = g - jf;
    return (int64_t)jf;
}

// FP64 gather of PPT particles, every load issued before any is used: the field at each
// particle (linear weighting of node E, plus E_ext).  A dead slot (x < 0) reads node 0.
template <int PPT>
__device__ __forceinline__ void gather64(const Dev &d, const Seg64 &G, const PS<true> (&p)[PPT], double (&Ep)[PPT])
{
    double f[PPT], E0[PPT], E1[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int64_t j = cell_of_x64(G, p[k].x, f[k]);
        int64_t j1 = j + 1;
        if (G.periodic && j1 == G.ncells) j1 = 0;
        E0[k] = d.E[G.gbase + j];
        E1[k] = d.E[G.gbase + j1];
    }
#pragma unroll
    for (int k = 0; k < PPT; ++k) Ep[k] = (1.0 - f[k]) * E0[k] + f[k] * E1[k] + G.E_ext;
}

// FP64 Boris push, position update and walls with the gathered field.
__device__ __forceinline__ int p_push64(const Dev &d, const Seg64 &G, PS<true> &p, double Ep)
{
    boris<double>(G.h, G.t, G.s, Ep, p.vx, p.vy, p.vz);
    double x = p.x + G.dt * p.vx;
    const double L = G.L;
    if (G.periodic) {
        if (x < 0.0)
            x += L;
        else if (x >= L)
            x -= L;
        if (x >= L) x -= L;  // x + L rounded up to L
        p.x = x;
        if (!(x >= 0.0 && x < L)) {
            atomicOr(d.err, (int)E_NONFINITE);
            return 3;
        }
        return 0;
    }
    p.x = x;
    if (x >= 0.0 && x < L) return 0;
    // a non-finite position (from a non-finite field) leaves at the right wall and the
    // step reports PIC_ENONFINITE
    if (!(fabs(x) <= 1.0e300)) atomicOr(d.err, (int)E_NONFINITE);
    return (x < 0.0) ? 1 : 2;
}

// Gather (linear weighting of node E), Boris push, position update, walls.
// Returns 0 alive, 1 absorbed at the left wall, 2 at the right wall.
template <bool F64>
__device__ __forceinline__ int p_push(const Dev &d, const SegC &S, const EnsC &e, PS<F64> &p)
{
    if constexpr (!F64) {
        const float2 ec = d.Ecell[S.gbase + p.cell];
        const float Ep = fmaf(p.off, ec.y, ec.x) + (float)e.E_ext;
        const float h = (float)S.h;
        const float t[3] = {(float)S.t[0], (float)S.t[1], (float)S.t[2]};
        const float s[3] = {(float)S.s[0], (float)S.s[1], (float)S.s[2]};
        boris<float>(h, t, s, Ep, p.vx, p.vy, p.vz);
        float o = p.off + p.vx * (float)S.dtdx;
        const float fl = floorf(o);
        int c = p.cell + (int)fl;
        o -= fl;
        if (o >= 1.0f) {
            o -= 1.0f;
            c += 1;
        }
        p.off = o;
        if (S.periodic) {
            if (c < 0)
                c += S.ncells;
            else if (c >= S.ncells)
                c -= S.ncells;
            p.cell = c;
            if (c < 0 || c >= S.ncells) {  // moved more than a period: not a valid state
                atomicOr(d.err, (int)E_NONFINITE);
                return 3;
            }
            return 0;
        }
        p.cell = c;
        if (c < 0) return 1;
        if (c >= S.ncells) return 2;
        return 0;
    } else {
        const Seg64 G = seg64(S, e);
        PS<true> q[1] = {p};
        double Ep[1];
        gather64<1>(d, G, q, Ep);
        const int w = p_push64(d, G, q[0], Ep[0]);
        p = q[0];
        return w;
    }
}

__device__ __forceinline__ void sc(float a, float *s, float *c) { sincosf(a, s, c); }
__device__ __forceinline__ void sc(double a, double *s, double *c) { sincos(a, s, c); }
__device__ __forceinline__ float msqrt(float a) { return sqrtf(a); }
__device__ __forceinline__ double msqrt(double a) { return sqrt(a); }
__device__ __forceinline__ float mlog(float a) { return logf(a); }
__device__ __forceinline__ double mlog(double a) { return log(a); }

template <typename T>
__device__ __forceinline__ void iso_dir(T ua, T ub, T d[3])
{
    const T c = (T)1 - (T)2 * ua;
    const T s2 = (T)1 - c * c;
    const T sn = s2 > (T)0 ? msqrt(s2) : (T)0;
    T sp, cp;
    sc((T)6.283185307179586476925286766559 * ub, &sp, &cp);
    d[0] = c;
    d[1] = sn * cp;
    d[2] = sn * sp;
}

template <typename T>
__device__ __forceinline__ void three_normals(uint4 w, T z[3])
{
    T u1 = (T)u01d(w.x), u2 = (T)u01d(w.y), u3 = (T)u01d(w.z), u4 = (T)u01d(w.w);
    const T r1 = msqrt((T)-2 * mlog(u1)), r2 = msqrt((T)-2 * mlog(u3));
    T s1, c1, s2, c2;
    sc((T)6.283185307179586476925286766559 * u2, &s1, &c1);
    sc((T)6.283185307179586476925286766559 * u4, &s2, &c2);
    z[0] = r1 * c1;
    z[1] = r1 * s1;
    z[2] = r2 * c2;
}

// Null-collision decision (FP64, no contraction: fixed by the inputs and the rounding, R12)
// and scattering kinematics (in the particle precision).  Returns the channel
// (-1 none, 0 elastic, 1 ionisation, 2 CX); on ionisation fills the new pair.  CXREL = false
// compiles the relative-speed charge exchange (R26) out, which keeps the FP32 candidate
// kernel's registers (and so its occupancy) to what the other channels need.
template <bool F64, bool CXREL = true>
__device__ __forceinline__ int p_collide(const EnsC &e, const SegC &S, int s, double numax,
                                         double pnull, uint32_t tag, PS<F64> &p, double ve[3],
                                         double vi[3])
{
    using T = typename std::conditional<F64, double, float>::type;
    const uint4 w = draw(S.seed, s, p.id, tag, 0u);
    if (!(u01d(w.x) < pnull)) return -1;
    const double v2 = speed2_rn((double)p.vx, (double)p.vy, (double)p.vz);
    const double spd = __dsqrt_rn(v2);
    const double thr = __dmul_rn(u01d(w.y), numax);
    int chan = -1;
    if (s == 0) {
        const double nu_el = __dmul_rn(e.ngs_el, spd);
        const double nu_iz =
            (__dmul_rn(__dmul_rn(0.5, S.m), v2) >= e.eps_iz) ? __dmul_rn(e.ngs_iz, spd) : 0.0;
        if (thr < nu_el)
            chan = 0;
        else if (thr < __dadd_rn(nu_el, nu_iz))
            chan = 1;
    } else if (CXREL && e.cx_rel) {
        // reading R26: the target neutral (block 2) is drawn first; the rate takes the
        // relative speed, and a charge exchange hands the ion the neutral's velocity
        double zn[3];
        three_normals<double>(draw(S.seed, s, p.id, tag, 2u), zn);
        const double gx = __dsub_rn((double)p.vx, __dmul_rn(e.vn, zn[0]));
        const double gy = __dsub_rn((double)p.vy, __dmul_rn(e.vn, zn[1]));
        const double gz = __dsub_rn((double)p.vz, __dmul_rn(e.vn, zn[2]));
        if (thr < __dmul_rn(e.ngs_cx, __dsqrt_rn(speed2_rn(gx, gy, gz)))) {
            p.vx = (T)(e.vn * zn[0]);
            p.vy = (T)(e.vn * zn[1]);
            p.vz = (T)(e.vn * zn[2]);
            return 2;
        }
        return -1;
    } else {
        if (thr < __dmul_rn(e.ngs_cx, spd)) chan = 2;
    }
    if (chan < 0) return -1;
    if (chan == 0) {
        T dd[3];
        iso_dir<T>((T)u01d(w.z), (T)u01d(w.w), dd);
        const T vs = (T)spd;
        const T cth = ((T)p.vx * dd[0] + (T)p.vy * dd[1] + (T)p.vz * dd[2]) / vs;
        const T f2 = (T)1 - (T)(2.0 * S.m / e.m_n) * ((T)1 - cth);
        const T sp2 = msqrt((T)v2 * f2);
        p.vx = sp2 * dd[0];
        p.vy = sp2 * dd[1];
        p.vz = sp2 * dd[2];
    } else if (chan == 1) {
        const uint4 w1 = draw(S.seed, s, p.id, tag, 1u);
        const uint4 w2 = draw(S.seed, s, p.id, tag, 2u);
        const T erem = (T)(0.5 * S.m * v2 - e.eps_iz);
        const T u = (T)u01d(w1.x);
        const T e1 = u * erem, e2 = ((T)1 - u) * erem;
        T d1[3], d2[3], z[3];
        iso_dir<T>((T)u01d(w.z), (T)u01d(w.w), d1);
        iso_dir<T>((T)u01d(w1.y), (T)u01d(w1.z), d2);
        const T s1 = msqrt((T)2 * e1 / (T)S.m), s2 = msqrt((T)2 * e2 / (T)S.m);
        p.vx = s1 * d1[0];
        p.vy = s1 * d1[1];
        p.vz = s1 * d1[2];
        three_normals<T>(w2, z);
        const T vn = (T)e.vn;
        for (int k = 0; k < 3; ++k) {
            ve[k] = (double)(s2 * d2[k]);
            vi[k] = (double)(vn * z[k]);
        }
    } else {
        const uint4 w2 = draw(S.seed, s, p.id, tag, 2u);
        T z[3];
        three_normals<T>(w2, z);
        const T vn = (T)e.vn;
        p.vx = vn * z[0];
        p.vy = vn * z[1];
        p.vz = vn * z[2];
    }
    return chan;
}

// =======================================================================================
// Deposit helpers of the FP32 form: the 2^-24 fixed-point share of the right node, and the
// direct HBM deposit of one particle.
// =======================================================================================
__device__ __forceinline__ uint32_t fixed_share(float off)
{
    return (uint32_t)__float2uint_rn(off * 16777216.0f);
}

// Direct HBM deposit of one particle (outside the window, or another segment).
__device__ __forceinline__ void global_deposit32(const Dev &d, const SegC &S, int s, int cell,
                                                 float off, bool hist)
{
    const uint32_t fq = fixed_share(off);
    int j1 = cell + 1;
    if (S.periodic && j1 == S.ncells) j1 = 0;
    unsigned long long *Q = d.Qi + (int64_t)s * d.nodes_tot + S.gbase;
    atomicAdd(Q + cell, 16777216ull - fq);
    atomicAdd(Q + j1, (unsigned long long)fq);
    if (hist) atomicAdd(d.cellcnt + S.cbase + cell, 1u);
}

__device__ __forceinline__ void global_deposit64(const Dev &d, const SegC &S, int s, double x,
                                                 bool hist)
{
    double f;
    const int j = (int)cell_of_x(S, x, f);
    int j1 = j + 1;
    if (S.periodic && j1 == S.ncells) j1 = 0;
    double *Q = d.Qd + (int64_t)s * d.nodes_tot + S.gbase;
    unsafeAtomicAdd(Q + j, 1.0 - f);
    unsafeAtomicAdd(Q + j1, f);
    if (hist) atomicAdd(d.cellcnt + S.cbase + j, 1u);
}

// The FP64 deposit window of one tile: nodes [base, base + n) accumulate in LDS (FP64 LDS
// atomics) and are added to the node array once per tile; n = 0 sends every share to HBM.
struct Win64 {
    double *w;
    int base, n;
};

// Cloud-in-cell deposit of one particle per lane (FP64 form), called by every lane of the
// wave with the lane's cell (key < 0: none) and in-cell fraction: lanes hold consecutive
// slots, which after a sort mostly share a cell, so the wave first sums the shares of each
// run of consecutive lanes with the same cell (a segmented scan over the lanes) and the
// last lane of each run adds the run's two shares, into the tile's LDS window when both
// nodes lie in it and with one FP64 atomic per node otherwise, and its count to the sort
// histogram.  `cnt_only` skips the shares.
__device__ __forceinline__ void wave_deposit64(const Dev &d, const Seg64 &S, int s, int key, double f,
                                               bool hist, bool cnt_only, const Win64 &W = Win64{nullptr, 0, 0})
{
    const int lane = lane_id();
    const bool live = key >= 0;
    double a = live ? 1.0 - f : 0.0, c = f;
    uint32_t n = live ? 1u : 0u;
    const int prev = __shfl_up(key, 1);
    const bool head = lane == 0 || prev != key;
    const unsigned long long heads = __ballot(head);
    // first lane of this lane's run: the highest head at or below it
    const unsigned long long below = heads & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
    const int start = 63 - __clzll((long long)below);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double ta = __shfl_up(a, o), tc = __shfl_up(c, o);
        const uint32_t tn = __shfl_up(n, o);
        if (lane - o >= start) {
            a += ta;
            c += tc;
            n += tn;
        }
    }
    const bool tail = lane == kWave - 1 || ((heads >> (lane + 1)) & 1ull);
    if (!tail || key < 0) return;
    if (!cnt_only) {
        const int r = key - W.base;
        if (r >= 0 && r + 1 < W.n) {
            // node wbase + r + 1 may be N of a periodic grid: the flush wraps it to node 0
            unsafeAtomicAdd(W.w + r, a);
            unsafeAtomicAdd(W.w + r + 1, c);
        } else {
            int j1 = key + 1;
            if (S.periodic && j1 == S.ncells) j1 = 0;
            double *Q = d.Qd + (int64_t)s * d.nodes_tot + S.gbase;
            unsafeAtomicAdd(Q + key, a);
            unsafeAtomicAdd(Q + j1, c);
        }
    }
    if (hist) {
        const int r = key - W.base;
        if (cnt_only && r >= 0 && r < W.n)
            unsafeAtomicAdd(W.w + r, (double)n);  // a count window: small exact integers
        else
            atomicAdd(d.cellcnt + S.cbase + key, n);
    }
}

// Deposit of one FP64 tile through an LDS window over the nodes of its cells (at most
// kWin64 nodes from the lowest cell of the tile; shares beyond it go to HBM atomics): the
// window is cleared, the waves add their merged runs into it, and each nonzero node is
// added to the node array with one FP64 atomic.  With COUNT the window holds the sort
// histogram's counts per cell instead (the histogram-only pass), each touched cell added
// with one atomic.  Called by every thread of the block; `s_mm` holds 8 ints.  The next
// call's barriers order its clearing after this flush.
constexpr int kWin64 = 1024;

template <int PPT, bool COUNT = false>
__device__ __forceinline__ void tile_deposit64(const Dev &d, const Seg64 &S, int s, const bool (&live)[PPT],
                                               const PS<true> (&p)[PPT], bool hist, double *s_win, int *s_mm)
{
    int mn = INT32_MAX, mx = -1;
    int key[PPT];
    double f[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        f[k] = 0.0;
        key[k] = live[k] ? (int)cell_of_x64(S, p[k].x, f[k]) : -1;
        if (live[k]) {
            mn = min(mn, key[k]);
            mx = max(mx, key[k]);
        }
    }
    mn = wave_min_i32(mn);
    mx = wave_max_i32(mx);
    const int w = threadIdx.x / kWave, nw = blockDim.x / kWave;
    if (lane_id() == 0) {
        s_mm[w] = mn;
        s_mm[4 + w] = mx;
    }
    __syncthreads();
    mn = s_mm[0];
    mx = s_mm[4];
    for (int i = 1; i < nw; ++i) {
        mn = min(mn, s_mm[i]);
        mx = max(mx, s_mm[4 + i]);
    }
    // nodes mn .. mx + 1 (cells mn .. mx for the counts)
    const int n = mx >= 0 ? min(mx - mn + (COUNT ? 1 : 2), kWin64) : 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s_win[i] = 0.0;
    __syncthreads();
    const Win64 W{s_win, mn, n};
#pragma unroll
    for (int k = 0; k < PPT; ++k) wave_deposit64(d, S, s, key[k], f[k], COUNT || hist, COUNT, W);
    __syncthreads();
    double *Q = d.Qd + (int64_t)s * d.nodes_tot + S.gbase;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = s_win[i];
        if (v == 0.0) continue;
        if constexpr (COUNT) {
            atomicAdd(d.cellcnt + S.cbase + mn + i, (uint32_t)v);
        } else {
            int node = mn + i;
            if (S.periodic && node >= S.ncells) node -= S.ncells;
            unsafeAtomicAdd(Q + node, v);
        }
    }
}

}  // namespace pic
