// pic_adjoint.hip -- discrete adjoint of the collisionless push + deposit + Poisson window
// (FP32 cell+offset forward, one periodic species on a fixed neutralising background,
// B = 0).  The floor of the cell index is treated as locally constant, so each step's
// adjoint is exact for the discrete forward:
//   x^{n+1} = x^n + dt v^{n+1/2},  v^{n+1/2} = v^{n-1/2} + dt (q/m) (E^n(x^n) + E_ext),
//   E^n = -D phi,  phi = S rho',  rho' = (q w / dx) P Q(x^n)
// with D the centred difference, S the zero-mean periodic Poisson solve (symmetric) and P
// the projection that removes the mean (the neutralising background).  Backwards:
//   lv += dt lx;  la = dt (q/m) lv;  lE_j += w_j(x) la;  lx += la (E_{j+1} - E_j) / dx;
//   lEext += la;  lQ = (q w / dx) S D lE;  lx += (lQ_{j+1} - lQ_j) / dx.
// Adjoint accumulators are FP64.
#include <algorithm>

#include "pic_device.h"
#include "pic_kernels.h"

namespace pic {

// Per particle, first half of the step adjoint: pass-through of lx into lv, the gather
// adjoint (a scatter into lE) and the interpolation derivative.
template <int PPT>
__global__ void __launch_bounds__(256) k_adj_a(Dev d, const int32_t *xc, const float *xo,
                                                  const double *E, double *lx, double *lv,
                                                  double *lE, double *lEext, int64_t n, double dt,
                                                  double qm, double dx, int N)
{
    __shared__ double s_red[4];
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * PPT;
    double ext = 0.0;
    int rk = -1;
    double r0 = 0.0, r1 = 0.0;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int64_t i = i0 + k;
        if (i >= n) break;
        const int j = xc[i];
        const double f = (double)xo[i];
        const int j1 = (j + 1 == N) ? 0 : j + 1;
        const double lvn = lv[i] + dt * lx[i];
        const double la = dt * qm * lvn;
        lv[i] = lvn;
        lx[i] += la * (E[j1] - E[j]) / dx;
        ext += la;
        if (j != rk) {
            if (rk >= 0) {
                unsafeAtomicAdd(lE + rk, r0);
                unsafeAtomicAdd(lE + ((rk + 1 == N) ? 0 : rk + 1), r1);
            }
            rk = j;
            r0 = r1 = 0.0;
        }
        r0 += (1.0 - f) * la;
        r1 += f * la;
    }
    if (rk >= 0) {
        unsafeAtomicAdd(lE + rk, r0);
        unsafeAtomicAdd(lE + ((rk + 1 == N) ? 0 : rk + 1), r1);
    }
    ext = wave_sum_f64(ext);
    if (lane_id() == 0) s_red[threadIdx.x / kWave] = ext;
    __syncthreads();
    if (threadIdx.x == 0) unsafeAtomicAdd(lEext, s_red[0] + s_red[1] + s_red[2] + s_red[3]);
}

// Second half: the deposit adjoint (a gather of lQ's difference).
template <int PPT>
__global__ void __launch_bounds__(256) k_adj_b(const int32_t *xc, const double *lQ, double *lx,
                                                  int64_t n, double dx, int N)
{
    const int64_t i0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * PPT;
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int64_t i = i0 + k;
        if (i >= n) break;
        const int j = xc[i];
        const int j1 = (j + 1 == N) ? 0 : j + 1;
        lx[i] += (lQ[j1] - lQ[j]) / dx;
    }
}

// Block-wide inclusive scan of a double per thread (1024 threads).
__device__ double adj_block_scan(double v, double *s_w)
{
    const int lane = lane_id(), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const double t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    if (lane == kWave - 1) s_w[w] = v;
    __syncthreads();
    double add = 0.0;
    for (int i = 0; i < w; ++i) add += s_w[i];
    double tot = 0.0;
    for (int i = 0; i < nw; ++i) tot += s_w[i];
    __syncthreads();
    s_w[16] = tot;  // read by the caller after the next barrier
    return v + add;
}

// Grid adjoint (one block): lphi = D lE; lrho = S lphi; lQ = (q w / dx) lrho; lE = 0.
// S is the zero-mean periodic solve of (phi_{j-1} - 2 phi_j + phi_{j+1}) / dx^2 = -r_j / eps0,
// computed as in the forward solve by two prefix sums with phi_0 = phi_N = 0, then the mean
// removed.  `tmp` holds N doubles of scratch.
__global__ void __launch_bounds__(1024) k_adj_grid(double *lE, double *lQ, double *tmp, int N,
                                                   double dx, double eps0, double qw)
{
    __shared__ double s_w[17];
    __shared__ double s_carry, s_tot;
    const int T = blockDim.x;
    // r = D lE (zero-sum by construction)
    for (int j = threadIdx.x; j < N; j += T) {
        const int jp = (j + 1 == N) ? 0 : j + 1, jm = (j == 0) ? N - 1 : j - 1;
        tmp[j] = (lE[jp] - lE[jm]) / (2.0 * dx);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += T) lE[j] = 0.0;
    // the source used by the solve: r_j on the interior nodes 1..N-1; remove the mean of r
    // (zero up to rounding) as the forward background does
    double loc = 0.0;
    for (int j = threadIdx.x; j < N; j += T) loc += tmp[j];
    loc = wave_sum_f64(loc);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = loc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < T / kWave; ++i) t += s_w[i];
        s_tot = t / N;
    }
    __syncthreads();
    const double mean_r = s_tot;
    const double ce = dx / eps0;
    // pass 1: C_m = sum_{i=1..m} r_i stored in lQ (as scratch), S = sum_{m<N} C_m
    if (threadIdx.x == 0) s_carry = 0.0;
    __syncthreads();
    double Ssum = 0.0;
    for (int base = 0; base < N; base += T) {
        const int j = base + threadIdx.x;
        const double r = (j >= 1 && j < N) ? tmp[j] - mean_r : 0.0;
        const double inc = adj_block_scan(r, s_w);
        __syncthreads();
        const double tot = s_w[16];
        const double C = s_carry + inc;
        if (j < N) lQ[j] = C;
        Ssum += (j < N) ? C : 0.0;
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
    Ssum = wave_sum_f64(Ssum);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = Ssum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < T / kWave; ++i) t += s_w[i];
        s_tot = t;
        s_carry = 0.0;
    }
    __syncthreads();
    const double Eh = -ce * s_tot / (double)N;
    // pass 2: phi_j = -dx (j Eh + ce F_j), F_j = sum_{m<j} C_m; accumulate the mean
    double phisum = 0.0;
    for (int base = 0; base < N; base += T) {
        const int j = base + threadIdx.x;
        const double C = (j < N) ? lQ[j] : 0.0;
        const double inc = adj_block_scan(C, s_w);
        __syncthreads();
        const double tot = s_w[16];
        const double F = s_carry + inc - C;
        if (j < N) {
            const double phi = -dx * ((double)j * Eh + ce * F);
            tmp[j] = phi;
            phisum += phi;
        }
        __syncthreads();
        if (threadIdx.x == 0) s_carry += tot;
        __syncthreads();
    }
    phisum = wave_sum_f64(phisum);
    if (lane_id() == 0) s_w[threadIdx.x / kWave] = phisum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < T / kWave; ++i) t += s_w[i];
        s_tot = t / N;
    }
    __syncthreads();
    const double mphi = s_tot;
    for (int j = threadIdx.x; j < N; j += T) lQ[j] = (qw / dx) * (tmp[j] - mphi);
}

// Seed of the reverse sweep: lE = d W / d E = eps0 dx E.
__global__ void k_adj_seed(const double *E, double *lE, int N, double eps0, double dx)
{
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < N; j += gridDim.x * blockDim.x)
        lE[j] = eps0 * dx * E[j];
}

// Gradient by particle id: out[id_i] = lv_i for the n slots (ids at or above `len` set the
// error flag instead).
__global__ void k_adj_by_id(const double *lv, const uint32_t *id, double *out, int64_t n, int64_t len,
                            int32_t *err)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = id[i];
        if ((int64_t)k < len)
            out[k] = lv[i];
        else
            atomicOr(err, 1);
    }
}

hipError_t launch_adj_by_id(const double *lv, const uint32_t *id, double *out, int64_t n, int64_t len,
                            int32_t *err, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t G = std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_adj_by_id, dim3((unsigned)G), dim3(256), 0, s, lv, id, out, n, len, err);
    return hipGetLastError();
}

hipError_t launch_adj_seed(const double *E, double *lE, int N, double eps0, double dx, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_seed, dim3(8), dim3(256), 0, s, E, lE, N, eps0, dx);
    return hipGetLastError();
}

hipError_t launch_adj_a(const Dev &d, const int32_t *xc, const float *xo, const double *E, double *lx,
                        double *lv, double *lE, double *lEext, int64_t n, double dt, double qm,
                        double dx, int N, hipStream_t s)
{
    const int64_t G = (n + 256 * 8 - 1) / (256 * 8);
    if (G == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_a<8>, dim3(G), dim3(256), 0, s, d, xc, xo, E, lx, lv, lE, lEext, n, dt, qm, dx, N);
    return hipGetLastError();
}

hipError_t launch_adj_grid(double *lE, double *lQ, double *tmp, int N, double dx, double eps0, double qw,
                           hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_grid, dim3(1), dim3(1024), 0, s, lE, lQ, tmp, N, dx, eps0, qw);
    return hipGetLastError();
}

hipError_t launch_adj_b(const int32_t *xc, const double *lQ, double *lx, int64_t n, double dx, int N,
                        hipStream_t s)
{
    const int64_t G = (n + 256 * 8 - 1) / (256 * 8);
    if (G == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_b<8>, dim3(G), dim3(256), 0, s, xc, lQ, lx, n, dx, N);
    return hipGetLastError();
}

}  // namespace pic
