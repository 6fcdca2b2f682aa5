// pic_device.h -- device-side data layout and helpers of the gfx950 PIC MC library.
//
// Layout in HBM (all carved from the caller's workspace):
//   particles   SoA per precision, two buffers (the sort scatters from one into the other);
//               segment = (ensemble, species) owns slots [base, base + cap) in every array.
//               FP32 form: cell:i32 | off:f32 | vx,vy,vz:f32 | id:u32  (24 B per particle)
//               FP64 form: x:f64 | vx,vy,vz:f64 | id:u32                  (36 B per particle)
//   grid        per ensemble, nodes [gbase, gbase + nnodes): Q_s (int64 fixed point or f64),
//               rho, phi, E (f64) and per cell (E_j, E_{j+1} - E_j) as float2 for the gather.
//   tallies     striped counters [stripe][segment][k] so that at most grid/STRIPES blocks
//               ever hit one address with an atomic.
//   births      ionisation births of one step, striped, plus a per-ensemble bitmap over
//               electron ids and per-1024-id counts used to rank births by parent id.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pic {

constexpr int kStripes = 32;          // stripes of the birth list
constexpr int kCntStripes = 256;      // stripes of the counters, sums and speed maxima
constexpr int kWave = 64;             // CDNA wavefront
constexpr int32_t kDead = INT32_MIN;  // FP32 form: cell of an absorbed slot
constexpr int kChunk = 1024;          // nodes per block in the field solve
constexpr int kSolveThreads = 256;
constexpr int kMaxEns = 256;          // ensembles per context
constexpr int kMaxSmooth = 4;         // passes of the density filter
// Birth ranking: a bit per parent id and a count per group of kGroupIds ids (a birth's rank
// among its ensemble's births is the scanned count of the groups below its own plus the
// bits below it in its group).
constexpr int kGroupIds = 4096;
constexpr int kGroupWords = kGroupIds / 32;
constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;        // elements per thread in the generic scan
constexpr double kFix = 16777216.0;   // 2^24 fixed-point scale of the deposit
constexpr double kNuSafety = 1.0 + 1.0 / 65536.0;
// births' group counts are scanned in tiles of kGroupTile groups (one block each); the
// placement adds the tiles' bases, staged in LDS, so at most kMaxGroupTiles tiles
constexpr int kGroupTile = 4096;
constexpr int kMaxGroupTiles = 1024;
constexpr int64_t kSlotAlign = 4096;  // segment slot ranges are multiples of the largest tile

// Counter slots per (stripe, segment).
enum Cnt : int {
    C_PUSH = 0, C_WALL_L, C_WALL_R, C_EL, C_IZ, C_CX, C_CREATED,
    C_RECYCLED, C_NWALL_L, C_NWALL_R,  // ion segment: recycled neutrals (R24)
    C_SOURCED,                         // electron segment: source pairs (R25)
    C_NCNT
};
enum Sum : int { S_KE_L = 0, S_KE_R, S_NSUM };
// Per-step scalar tallies: sum |v|^2 and count of the particles alive after the step.
enum StepSum : int { T_V2 = 0, T_N, T_NSTEP };
// Per-chunk solve aggregates.
enum Agg : int { A_SUMRHO = 0, A_SUMPRE, A_TOTQ, A_N1, A_D, A_CNT, A_RHO0, A_NAGG };
enum Part : int { P_EMAX = 0, P_FE, P_PHISUM, P_NONFIN, P_NPART };
// Error flags (bit mask).
enum Err : int { E_CAP_PART = 1, E_CAP_BIRTH = 2, E_CAP_ID = 4, E_NONFINITE = 8 };

// Constant per segment.
struct SegC {
    int64_t base, cap;        // slots
    int64_t cbase;            // first entry in per-cell arrays (sort counts)
    int64_t gbase;            // first node of the ensemble grid
    int32_t ens, species, ncells, periodic;
    double h, t[3], s[3];     // (q/m) dt/2 and the Boris rotation vectors
    double dt, dx, dtdx;
    double qw, halfmw, m;
    double ngsT, qm_abs;      // n_g sigma_total, |q/m|
    uint32_t seed;
    int32_t other;            // ion segment of this ensemble (electron segments), else -1
    int32_t recycle;          // ion segment of a recycling ensemble (R24)
    double vth;               // sqrt(T / m): the source's Maxwellian (R25)
    double w;                 // macro-particle weight
};

// Constant per ensemble.
struct EnsC {
    int64_t ncells, nnodes, gbase;
    int64_t chunk0, nchunks;  // solve chunks [chunk0, chunk0 + nchunks)
    int64_t idcap;            // ids stay below this (2 x electron capacity, rounded)
    int64_t bm_base, grp_base;  // birth ranking: first bitmap word, first id-group count
    double dx, dt, eps0, E_ext, L;
    double qw[2];
    double ngs_el, ngs_iz, ngs_cx, eps_iz, vn, m_e, m_n;
    int32_t seg[2];
    uint32_t seed;
    int32_t periodic, nspecies;
    int32_t floating;         // bounded walls keep their absorbed charge (R22)
    int32_t smooth;           // passes of the 1-2-1 density filter (R23)
    int32_t recycle;          // absorbed ions return as neutrals (R24)
    int64_t nbase, ncap;      // neutral slots [nbase, nbase + ncap) in each neutral buffer
    int64_t src_pairs;        // volumetric source pairs per step (R25)
    int64_t src_base;         // first of this ensemble's pairs in the source launch
    double src_x;             // the source fills [0, src_x)
    int32_t cx_rel;           // CX at the speed relative to a sampled neutral (R26)
    double vn_max;            // bound on a sampled neutral's speed when cx_rel, else 0
};

struct Birth {
    uint32_t pid;
    int32_t ens;
    int32_t cell;
    float off;
    double x;
    double ve[3];
    double vi[3];
};
// the birth placement reads (pid, ens) as one 8-byte key
static_assert(__builtin_offsetof(Birth, pid) == 0 && __builtin_offsetof(Birth, ens) == 4, "Birth key layout");

// Everything a kernel may touch; passed by value.
struct Dev {
    int32_t nseg, nens, nspecies, periodic, collisions;
    int32_t any_cx_rel;       // some ensemble uses relative-speed charge exchange (R26)
    const SegC *seg;
    const EnsC *ens;
    // particles (buffer b in {0,1}); FP32 and FP64 forms
    int32_t *cell[2];
    float *off[2], *fvx[2], *fvy[2], *fvz[2];
    double *x[2], *dvx[2], *dvy[2], *dvz[2];
    uint32_t *id[2];
    int64_t cap_tot;          // total slots (a multiple of kSlotAlign)
    int32_t *cur;             // [1] current particle buffer
    int64_t *n_slots;         // [nseg] slots in use (alive + absorbed-not-yet-compacted)
    uint32_t *next_id;        // [nseg]
    int64_t *step;            // [1]
    // grid
    int64_t nodes_tot, cells_tot;
    unsigned long long *Qi;   // [2][nodes_tot] (int64 fixed point, two's complement)
    double *Qd;               // [2][nodes_tot]
    double *rho, *phi, *E;    // [nodes_tot]
    float2 *Ecell;            // [nodes_tot]
    double *agg;              // [nchunks_tot][A_NAGG]
    double *part;             // [nchunks_tot][P_NPART]
    double *emax, *fe;        // [nens]
    double *numax, *pnull;    // [nseg]
    // the largest |v|^2 of each segment over the stripes of the speed maxima the next bound
    // uses, reduced by extra blocks of the first solve kernel of the fused step
    double *vmred;            // [nseg]
    // tallies
    unsigned long long *vmax2;  // [2][kCntStripes][nseg] max |v|^2 as double bits
    int32_t *vcur;            // [1] which vmax2 half holds the current maxima
    unsigned long long *cnt;  // [kCntStripes][nseg][C_NCNT]
    double *sums;             // [kCntStripes][nseg][S_NSUM]
    // scalar diagnostics of the fused FP32 step, per step: [2][kCntStripes][nseg][T_NSTEP],
    // half 1 - *vcur accumulates the step under way and becomes current at the birth
    // placement, which clears the other half (as for vmax2)
    double *ssum;
    // births, double-buffered by step parity: step n appends to half n & 1 and its
    // placement clears half (n + 1) & 1, which step n - 1 used
    Birth *births;            // [2][kStripes][birth_stripe_cap]
    uint32_t *nbirth;         // [2][kStripes]
    int64_t birth_stripe_cap;
    uint32_t *bitmap;         // [2][bm_words] per-ensemble bit per parent id
    int64_t bm_words;
    uint32_t *gcnt;           // [2][g_tot] per-ensemble births per group of kGroupIds ids
    uint32_t *gpre;           // [g_tot] exclusive scan of the current half's gcnt, per tile
                              // of kGroupTile groups when ngt > 0 (global otherwise)
    uint32_t *gtile;          // [max(ngt, 1)] group-count total of each tile
    int32_t ngt;              // tiles of the tiled scan (0: the global three-kernel scan)
    int64_t g_tot;            // a multiple of 4096
    // null-collision candidates of the FP32 pass: tile t keeps its candidate slots in
    // cand[t * tile .. t * tile + ctile[t])
    uint4 *crec;              // [2 * cap_tot] collision-candidate records, per tile
    uint32_t *ctile;          // [cap_tot / 1024]
    // sort
    uint32_t *cellcnt, *cursor;  // [cells_tot] over all segments (SegC::cbase)
    int64_t *segstart;        // [nseg]
    // recycled neutrals (R24): two buffers; a step streams buffer *ncur into the other,
    // appends the neutrals born from the absorbed ions listed by the pass, then flips
    int32_t *ncell[2];
    float *noff[2], *nvx[2], *nvy[2], *nvz[2];
    uint32_t *nid[2];
    int64_t ncap_tot;
    int32_t *ncur;            // [1]
    unsigned long long *nneu; // [2][nens] neutrals per ensemble in each buffer
    uint2 *recs;              // [rec_cap] absorbed ions of the step: (id, ens << 1 | wall)
    int64_t rec_cap;
    uint32_t *nrec;           // [1]
    int64_t src_tot;          // source pairs per step over all ensembles (R25)
    // scan scratch, tickets, errors
    uint32_t *scanpart;       // [<= 1 << 16]
    uint32_t *ticket;         // [8]
    uint32_t *tq;             // [16]: the FP64 pass's eight tile queues and its exit ticket
    int32_t *err;             // [1]
};

// ---------------------------------------------------------------------------------------
// Philox4x32 (Salmon et al., SC'11) with kPhiloxRounds = 7 rounds (reading R17: the
// paper's smallest Crush-resistant count for this generator): each round multiplies counter
// words 0 and 2 by the published constants, xors the high halves with the other counter
// words and the round key, and bumps the key by the published Weyl increments between
// rounds.
constexpr int kPhiloxRounds = 7;
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < kPhiloxRounds; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // one 32x32 -> 64-bit product per word (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    return make_uint4(c0, c1, c2, c3);
}

// Uniform in (0,1): an odd multiple of 2^-24, exact in both float and double.
__device__ __forceinline__ double u01d(uint32_t r) { return ((double)(r >> 9) + 0.5) * 0x1p-23; }
__device__ __forceinline__ float u01f(uint32_t r) { return ((float)(r >> 9) + 0.5f) * 0x1p-23f; }

// Key and counter layout of the random streams: key = (seed, species),
// counter = (particle id, step tag, block, 0).  Tag 0xFFFFFFFF is the particle load.
constexpr uint32_t kInitTag = 0xFFFFFFFFu;
__device__ __forceinline__ uint4 draw(uint32_t seed, int species, uint32_t id, uint32_t tag,
                                      uint32_t blk)
{
    return philox(id, tag, blk, 0u, seed, (uint32_t)species);
}

// ---------------------------------------------------------------------------------------
// Wave-level helpers (64 lanes).
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}
__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    return v;
}
__device__ __forceinline__ double wave_max_f64(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
    return v;
}
__device__ __forceinline__ int wave_min_i32(int v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m));
    return v;
}
__device__ __forceinline__ int wave_max_i32(int v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m));
    return v;
}

// Double bits of a non-negative value order like unsigned integers.
__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

// |v|^2 in FP64 from the stored components, summed left to right with no fused
// multiply-add, so the collision decision is a function of the stored values alone: the
// same in both precisions and in any implementation that rounds this way.
__device__ __forceinline__ double speed2_rn(double a, double b, double c)
{
    return __dadd_rn(__dadd_rn(__dmul_rn(a, a), __dmul_rn(b, b)), __dmul_rn(c, c));
}

// |v|^2 in binary32 (two fused multiply-adds): the FP32 pass's per-particle speed for its
// collision bound and its kinetic-energy tally; the candidate kernel takes the same
// expression off for a particle that collides, so the two cancel exactly.
__device__ __forceinline__ float speed2_f32(float a, float b, float c) { return fmaf(a, a, fmaf(b, b, c * c)); }

// A tile's candidate count (at most 2048) as the pass writes it, tagged with the tile's
// segment (< 1024) and ensemble (< 1024), so the candidate kernel learns all three from one
// load.
constexpr uint32_t kCandCountMask = 0xFFFu;
__device__ __forceinline__ uint32_t cand_tag(int sg, int ens) { return ((uint32_t)sg << 12) | ((uint32_t)ens << 22); }

__device__ __forceinline__ int stripe_of_block() { return (int)(blockIdx.x & (kCntStripes - 1)); }

// The per-step scalar tallies of segment sg in stripe st of half `half`.
__device__ __forceinline__ double *step_sums(const Dev &d, int half, int st, int sg)
{
    return d.ssum + (((int64_t)half * kCntStripes + st) * d.nseg + sg) * T_NSTEP;
}

// One half of the birth buffers.
struct BirthBuf {
    Birth *births;
    uint32_t *nbirth, *bitmap, *gcnt;
};
__device__ __forceinline__ BirthBuf birth_buf(const Dev &d, int parity)
{
    return {d.births + (int64_t)parity * kStripes * d.birth_stripe_cap, d.nbirth + parity * kStripes,
            d.bitmap + (int64_t)parity * d.bm_words, d.gcnt + (int64_t)parity * d.g_tot};
}

// Reading R11, the null-collision bound of segment `sg` from the current striped speed
// maxima and the ensemble's max |E|: nu_max = n_g sigma_T (vmax + |q/m| dt (max|E| +
// |E_ext|)) (1 + 2^-16) and P_null = 1 - exp(-nu_max dt).  Called by a whole wave (lanes
// read the stripes); every lane gets the result.
// `half` is the vmax2 half holding the current maxima and `emax` the ensemble's max |E|.
// The largest |v|^2 of segment `sg` in one half of the striped speed maxima (a whole wave
// reads the stripes; every lane gets the result).
__device__ __forceinline__ double seg_vmax2(const Dev &d, int sg, int half)
{
    double m2 = 0.0;  // squared speeds are non-negative: bit patterns order as integers
    for (int st = lane_id(); st < kCntStripes; st += kWave)
        m2 = fmax(m2, __longlong_as_double((long long)d.vmax2[((int64_t)half * kCntStripes + st) * d.nseg + sg]));
    return wave_max_f64(m2);
}

// The bound itself, from the largest |v|^2 and the max |E| (one thread suffices).
__device__ __forceinline__ void seg_bound(const SegC &S, const EnsC &e, double m2, double emax, double &numax,
                                          double &pnull)
{
    const double vmax = __dsqrt_rn(m2);
    double Vb = __dadd_rn(vmax, __dmul_rn(__dmul_rn(S.qm_abs, e.dt), __dadd_rn(emax, fabs(e.E_ext))));
    // reading R26: the relative speed to a sampled neutral exceeds the ion's by at most vn_max
    if (S.species == 1) Vb = __dadd_rn(Vb, e.vn_max);
    numax = __dmul_rn(__dmul_rn(S.ngsT, Vb), kNuSafety);
    pnull = 1.0 - exp(-__dmul_rn(numax, e.dt));
}

__device__ __forceinline__ void seg_params(const Dev &d, int sg, int half, double emax, double &numax,
                                           double &pnull)
{
    const SegC &S = d.seg[sg];
    seg_bound(S, d.ens[S.ens], seg_vmax2(d, sg, half), emax, numax, pnull);
}

// Record a birth of parent `pid` (its bit and its group count) in one half.
__device__ __forceinline__ void birth_mark(const BirthBuf &bb, const EnsC &e, uint32_t pid)
{
    atomicOr(bb.bitmap + e.bm_base + (pid >> 5), 1u << (pid & 31));
    atomicAdd(bb.gcnt + e.grp_base + pid / kGroupIds, 1u);
}

__device__ __forceinline__ void birth_unmark(const BirthBuf &bb, const EnsC &e, uint32_t pid)
{
    bb.bitmap[e.bm_base + (pid >> 5)] = 0u;
    bb.gcnt[e.grp_base + pid / kGroupIds] = 0u;
}

}  // namespace pic
