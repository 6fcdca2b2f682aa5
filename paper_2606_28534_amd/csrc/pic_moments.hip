// pic_moments.hip -- node moments of one species (reading R27), on demand for pic_diag.
//
// Per node j the cloud-in-cell shares S_j of the particles give W_j = sum S_j,
// sum S_j v (three components) and sum S_j |v|^2, accumulated in FP64; a second kernel
// turns them into the number density n_j = w W_j / V_j, the mean velocity
// u_j = sum S_j v / W_j and the temperature T_j = (m/3)(sum S_j |v|^2 / W_j - |u_j|^2).
// These are the plasma profiles (density, flow, temperature per species) whose
// time-averaged output the paper's input table switches on and whose in-situ plots its
// results section shows.
//
// Accumulation: a block takes a tile of 1024 consecutive slots.  Once sorted, a tile's
// particles sit in a few cells, so the block adds its shares into an LDS window over the
// tile's node span (LDS FP64 atomics) and flushes each touched node with one HBM FP64
// atomic per quantity; a tile spanning more than the window (unsorted slots, a sparse
// region) adds straight to HBM.  FP64 atomics make the last bits order-dependent, which
// the moments' tolerance (rel 1e-4) does not see.
#include <algorithm>

#include "pic_device.h"
#include "pic_kernels.h"
#include "pic_particle.h"

namespace pic {

constexpr int kMomThreads = 256;
constexpr int kMomPpt = 4;
constexpr int kMomTile = kMomThreads * kMomPpt;
constexpr int kMomWin = 512;  // nodes of the LDS window
constexpr int kMomQ = 5;      // W, W vx, W vy, W vz, W |v|^2

// acc: [kMomQ][nn] of this segment's ensemble, zeroed by the caller.
template <bool F64>
__global__ void __launch_bounds__(kMomThreads) k_moments(Dev d, int sg, double *acc, int64_t nn)
{
    __shared__ double s_acc[kMomQ][kMomWin];
    __shared__ int s_lo[kMomThreads / kWave], s_hi[kMomThreads / kWave];
    const SegC S = d.seg[sg];
    const int b = *d.cur;
    const int64_t n = d.n_slots[sg];
    const int64_t ntiles = (n + kMomTile - 1) / kMomTile;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        int cell[kMomPpt];
        double f[kMomPpt], v[kMomPpt][3];
        bool live[kMomPpt];
        int lo = INT32_MAX, hi = INT32_MIN;
#pragma unroll
        for (int k = 0; k < kMomPpt; ++k) {
            const int64_t p = t * kMomTile + (int64_t)k * kMomThreads + threadIdx.x;
            live[k] = false;
            cell[k] = 0;
            f[k] = 0.0;
            v[k][0] = v[k][1] = v[k][2] = 0.0;
            if (p < n) {
                const int64_t i = S.base + p;
                if constexpr (!F64) {
                    const int c = d.cell[b][i];
                    if (c != kDead) {
                        live[k] = true;
                        cell[k] = c;
                        f[k] = (double)d.off[b][i];
                        v[k][0] = d.fvx[b][i];
                        v[k][1] = d.fvy[b][i];
                        v[k][2] = d.fvz[b][i];
                    }
                } else {
                    const double x = d.x[b][i];
                    if (x >= 0.0) {
                        live[k] = true;
                        double ff;
                        cell[k] = (int)cell_of_x(S, x, ff);
                        f[k] = ff;
                        v[k][0] = d.dvx[b][i];
                        v[k][1] = d.dvy[b][i];
                        v[k][2] = d.dvz[b][i];
                    }
                }
            }
            if (live[k]) {
                lo = min(lo, cell[k]);
                hi = max(hi, cell[k]);
            }
        }
        lo = wave_min_i32(lo);
        hi = wave_max_i32(hi);
        if (lane_id() == 0) {
            s_lo[threadIdx.x / kWave] = lo;
            s_hi[threadIdx.x / kWave] = hi;
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < kMomThreads / kWave; ++w) {
            lo = min(lo, s_lo[w]);
            hi = max(hi, s_hi[w]);
        }
        // nodes lo .. hi + 1 of the tile (node N of a periodic grid is node 0)
        const int span = (lo <= hi) ? hi - lo + 2 : 0;
        const bool in_lds = span > 0 && span <= kMomWin;
        if (in_lds) {
            for (int i = threadIdx.x; i < span; i += kMomThreads)
#pragma unroll
                for (int q = 0; q < kMomQ; ++q) s_acc[q][i] = 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kMomPpt; ++k) {
            if (!live[k]) continue;
            const double v2 = v[k][0] * v[k][0] + v[k][1] * v[k][1] + v[k][2] * v[k][2];
            const double val[kMomQ] = {1.0, v[k][0], v[k][1], v[k][2], v2};
            const double sh[2] = {1.0 - f[k], f[k]};
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                int j = cell[k] + a;
                if (in_lds) {
#pragma unroll
                    for (int q = 0; q < kMomQ; ++q) atomicAdd(&s_acc[q][j - lo], sh[a] * val[q]);
                } else {
                    if (S.periodic && j == S.ncells) j = 0;
#pragma unroll
                    for (int q = 0; q < kMomQ; ++q) unsafeAtomicAdd(acc + (int64_t)q * nn + j, sh[a] * val[q]);
                }
            }
        }
        __syncthreads();
        if (in_lds) {
            for (int i = threadIdx.x; i < span; i += kMomThreads) {
                if (s_acc[0][i] == 0.0 && s_acc[1][i] == 0.0 && s_acc[2][i] == 0.0 && s_acc[3][i] == 0.0 &&
                    s_acc[4][i] == 0.0)
                    continue;
                int j = lo + i;
                if (S.periodic && j == S.ncells) j = 0;
#pragma unroll
                for (int q = 0; q < kMomQ; ++q) unsafeAtomicAdd(acc + (int64_t)q * nn + j, s_acc[q][i]);
            }
        }
        __syncthreads();
    }
}

// Sums -> (n, ux, uy, uz, T) in place, node by node.
__global__ void k_moments_finish(Dev d, int sg, double *acc, int64_t nn)
{
    const SegC S = d.seg[sg];
    const EnsC e = d.ens[S.ens];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nn; j += (int64_t)gridDim.x * blockDim.x) {
        const double W = acc[j];
        double u[3] = {0.0, 0.0, 0.0}, T = 0.0;
        if (W > 0.0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) u[k] = acc[(int64_t)(1 + k) * nn + j] / W;
            T = (S.m / 3.0) * (acc[4 * nn + j] / W - (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
        }
        const double V = (!e.periodic && (j == 0 || j == e.ncells)) ? 0.5 * e.dx : e.dx;
        acc[j] = S.w * W / V;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[(int64_t)(1 + k) * nn + j] = u[k];
        acc[4 * nn + j] = T;
    }
}

__global__ void k_fill_zero(double *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_moments(const Dev &d, bool f64, int sg, int64_t nn, double *out, hipStream_t s)
{
    const int64_t n5 = (int64_t)kMomQ * nn;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<int64_t>((n5 + 255) / 256, 4096)), dim3(256), 0, s,
                       out, n5);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned grid = 2048;  // grid-stride over the segment's tiles
    if (f64)
        hipLaunchKernelGGL(k_moments<true>, dim3(grid), dim3(kMomThreads), 0, s, d, sg, out, nn);
    else
        hipLaunchKernelGGL(k_moments<false>, dim3(grid), dim3(kMomThreads), 0, s, d, sg, out, nn);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_moments_finish, dim3((unsigned)std::min<int64_t>((nn + 255) / 256, 4096)), dim3(256), 0,
                       s, d, sg, out, nn);
    return hipGetLastError();
}

}  // namespace pic
