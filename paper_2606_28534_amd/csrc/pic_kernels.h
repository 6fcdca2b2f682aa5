// pic_kernels.h -- host-side launchers of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "pic_device.h"

namespace pic {

// Launch shape of the particle kernels.
struct Launch {
    int block;   // threads per block of the FP64 kernels (64, 128 or 256)
    int ppt;     // particles per thread per tile (FP32 pass: 4 or 8)
    int grid;    // persistent blocks of the FP64 kernels (multiple of 8 for the XCD-aware mapping)
    int window;  // widest LDS window span, in cells, of the FP32 pass and of the sorts
    int sort_ppt;  // particles per thread of the FP32 sort scatter
    int nt;        // fused FP32 pass: non-temporal particle loads and stores
    int sort_nt;   // FP32 sort scatter: non-temporal loads
};

enum StageBits : int { SB_PUSH = 1, SB_COLLIDE = 2, SB_DEPOSIT = 4, SB_HIST = 8 };

// With the COLLIDE stage the null-collision bound kernel runs first unless `with_params`
// is false (the caller launched it).
hipError_t launch_particles(const Dev &d, const Launch &L, hipStream_t s, bool f64, int stages, int hist,
                            bool with_params = true);
hipError_t launch_field_energy(const Dev &d, hipStream_t s);
// After a pass with the COLLIDE stage: the FP32 form's candidate kernel (no-op for FP64,
// whose pass scatters in place).
hipError_t launch_candidates(const Dev &d, const Launch &L, hipStream_t s, bool f64, int hist);
hipError_t launch_init(const Dev &d, bool f64, int sg, int64_t n, int64_t ppc, int init_mode,
                       double vth, double amp, int mode, hipStream_t s);
hipError_t launch_vmax(const Dev &d, bool f64, hipStream_t s);
hipError_t launch_zero_q(const Dev &d, bool f64, hipStream_t s);
// The field solve; with `with_births` its two kernels also scan and place the previous
// step's births in extra blocks (needs births_fit_solve: the one-block group scan); with
// `with_params` extra blocks of the first kernel reduce the striped speed maxima per segment
// and the second kernel's last block computes the null-collision bound from them.
hipError_t launch_solve(const Dev &d, bool f64, int64_t nchunks, bool zero_q, hipStream_t s,
                        bool with_births = false, bool with_params = false);
bool births_fit_solve(const Dev &d);
hipError_t launch_field_stats(const Dev &d, bool f64, int64_t nchunks, hipStream_t s);
hipError_t launch_params(const Dev &d, hipStream_t s);
hipError_t launch_scan(uint32_t *in, uint32_t *out, int64_t n, uint32_t *part, bool zero_in, hipStream_t s);
int64_t scan_blocks(int64_t n);
hipError_t launch_births(const Dev &d, bool f64, bool in_step, bool advance, hipStream_t s);
hipError_t launch_advance(const Dev &d, hipStream_t s);
hipError_t launch_births_clear_all(const Dev &d, hipStream_t s);
hipError_t launch_sort(const Dev &d, bool f64, const Launch &L, hipStream_t s);
// The first half of a sort: the histogram's scan into run cursors and the segment starts.
hipError_t launch_sort_prepare(const Dev &d, hipStream_t s);
// FP32 fused pass that also scatters into cell order (after launch_sort_prepare), then the
// slot counts and the buffer flip.
hipError_t launch_pass32_sort(const Dev &d, int ppt, int W, hipStream_t s, bool coll, int64_t cap_tot, bool nt);
hipError_t launch_pass32(const Dev &d, int ppt, int W, hipStream_t s, int stages, int hist, int64_t cap_tot,
                         bool nt);
hipError_t launch_cand32(const Dev &d, int ppt, hipStream_t s, int hist, int64_t cap_tot);
// the fused step's candidates, neutrals and source as one launch (FP32 form)
hipError_t launch_after(const Dev &d, int ppt, hipStream_t s, int hist, int64_t cap_tot, bool coll);
hipError_t launch_stream_copy(const void *src, void *dst, int64_t nwords, bool nt, hipStream_t s);
hipError_t launch_sort32_scatter(const Dev &d, int ppt, int W, hipStream_t s, int64_t cap_tot, bool nt);
hipError_t launch_adj_seed(const double *E, double *lE, int N, double eps0, double dx, hipStream_t s);
hipError_t launch_adj_a(const Dev &d, const int32_t *xc, const float *xo, const double *E, double *lx,
                        double *lv, double *lE, double *lEext, int64_t n, double dt, double qm,
                        double dx, int N, hipStream_t s);
hipError_t launch_adj_grid(double *lE, double *lQ, double *tmp, int N, double dx, double eps0, double qw,
                           hipStream_t s);
hipError_t launch_adj_b(const int32_t *xc, const double *lQ, double *lx, int64_t n, double dx, int N,
                        hipStream_t s);
// out[id_i] = lv_i for n slots; ids >= len set *err (device int).
hipError_t launch_adj_by_id(const double *lv, const uint32_t *id, double *out, int64_t n, int64_t len,
                            int32_t *err, hipStream_t s);
hipError_t launch_diag(const Dev &d, bool f64, int sg, double *out, int grid, hipStream_t s);
// Node moments of segment sg (reading R27) into out[5][nn] (n, ux, uy, uz, T); nn is the
// node count of the segment's ensemble.  `out` is device memory the launch overwrites.
hipError_t launch_moments(const Dev &d, bool f64, int sg, int64_t nn, double *out, hipStream_t s);
// Recycled neutrals of the step (stream, recycle the absorbed ions the pass listed, flip
// buffers) and the volumetric source pairs (FP32 form; no-ops when unused).
hipError_t launch_neutrals(const Dev &d, hipStream_t s);
hipError_t launch_source(const Dev &d, int hist, hipStream_t s);

}  // namespace pic
