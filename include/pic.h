/*
 * pic.h -- C ABI of the MI355X (gfx950) electrostatic 1D3V PIC Monte Carlo hot path.
 *
 * The library computes the per-step particle cycle that the paper's Background section
 * names for its 1D3V electrostatic PIC MC code (particle load, mover, deposition to the
 * grid, field solve, force interpolation, Monte Carlo collisions) plus the "natural
 * sorting" of particles by cell the same section describes, for the magnetised
 * double-bounded plasma layer of the paper's sheath-case table (absorbing walls, uniform
 * neutral background).  The paper fixes no equations for these steps; the method each
 * entry point implements is stated at its declaration.
 *
 * Conventions for every entry point:
 *   - Return value: PIC_OK (0) or a negative PIC_E* code; nothing throws across the ABI.
 *     pic_last_error(ctx) returns a message for the last failing call on that context.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every call that
 *     only enqueues GPU work is asynchronous on that stream; calls that return host data
 *     (pic_diag, pic_get_*) and pic_set_* synchronise it.
 *   - Device memory: the caller allocates ONE workspace of the size pic_query_workspace
 *     reports and keeps it alive until pic_free; the library carves every particle, grid
 *     and scratch array out of it and never allocates or frees device memory itself,
 *     except the small per-context HIP graph objects.  Host pointers are only read during
 *     the call.
 *   - Normalised units: eps0 = e = m_e = n0 = T_e = 1 (omega_pe = v_th,e = lambda_D = 1).
 *   - Sticky device error flags (capacity overflow, non-finite field) are checked at the
 *     end of pic_step and in pic_diag; a non-zero flag turns into the matching PIC_E* code.
 *
 * Readings.  Where the paper leaves a choice open, the sources follow these readings and
 * cite them by tag:
 *   R1  normalised units (eps0 = e = m_e = n0 = T_e = 1), dx = lambda_D / 2, omega_pe dt = 0.1.
 *   R2  state (x^n, v^{n-1/2}, Q^n); a step is solve, gather + Boris push, walls,
 *       null-collision MC, births, deposit of Q^{n+1}, and a sort every K steps; v^{-1/2}
 *       is loaded directly.
 *   R3  bounded walls are grounded (phi_0 = phi_N = 0); absorbed charge is tallied only.
 *   R4  periodic grids: a uniform background cancels the deposited charge, phi_0 = 0, then
 *       phi is shifted to zero mean.
 *   R5  the three-point Poisson stencil; the GPU solves it exactly with two prefix sums.
 *   R6  node E is the centred difference, with the half-cell Gauss law at bounded walls;
 *       E_ext is added at the gather.
 *   R7  sheath workloads: B = 2 (cos 80 deg, sin 80 deg, 0), i.e. |q_e| B / m_e = 2 omega_pe.
 *   R8  a particle is absorbed iff x < 0 or x >= L (cell < 0 or cell >= N in the FP32 form);
 *       count, charge and kinetic energy are tallied per wall and species.
 *   R9  channels: electron elastic (n_g sigma = 0.01), electron ionisation (0.005 above
 *       eps_iz = 1.576), ion charge exchange (1.0); T_n = T_i, m_n = m_i = 73440.
 *   R10 nu_k = n_g sigma_k |v| with the lab-frame speed.
 *   R11 null-collision bound nu_max = n_g sigma_T (v_max + |q/m| dt (max|E| + |E_ext|))
 *       (1 + 2^-16) from the speeds at the start of the step, so it holds before the push.
 *   R12 candidate iff R1 < P_null (Philox block 0 of the step); channel = first k with
 *       R2 nu_max < sum_{i<=k} nu_i; compared in FP64 without fused multiply-add.
 *   R13 lab-frame isotropic scattering: elastic energy loss 2 m_e / m_n (1 - cos theta);
 *       ionisation splits the energy above threshold; new and exchanged ions at T_n.
 *   R14 births are ranked by parent id and take ids next_id + rank, after the slots in use.
 *   R15 deposit shares (2^24 - f_q, f_q), f_q = rint(f 2^24), summed in int64.
 *   R16 sort every K = 20 steps (10 for the 1e9-particle workload); K = 0 still compacts
 *       every 20 steps.
 *   R17 Philox4x32-7 (seven rounds), key (seed, species), counter (id, tag, block, 0);
 *       u = ((r >> 9) + 1/2) 2^-23; normals by Box-Muller.
 *   R18 batched ensembles: sizes, ppc and temperatures come from the input generator;
 *       ensemble seed = index + 1.
 *   R19 quiet start x0 = (p + 1/2) L / P displaced by (A/k) sin(k x0), A = 0.01, cold
 *       electrons on a fixed background.
 *   R20 adjoint objective W = 1/2 eps0 dx sum_j E_j^2 after a collisionless periodic
 *       window, differentiated with respect to every initial v_x and E_ext (the exact
 *       transpose of the FP32 forward with cells held fixed).
 *   R21 adjoint window: the Langmuir workload, 200 steps, a checkpoint every 20.
 *   R22 floating walls keep the charge absorbed; E_{1/2} = (sigma_L + rho_0 V_0) / eps0
 *       with phi_0 = 0, and the right wall floats.
 *   R23 smoothing: p passes of the 1-2-1 filter on rho before the solve (periodic grids
 *       wrap, bounded grids mirror at the walls).
 *   R24 recycling: an absorbed ion returns from its wall as a neutral with the ion's id and
 *       a wall-flux Maxwellian velocity; neutrals stream freely and leave at the walls.
 *   R25 volumetric source: src_pairs electron-ion pairs per step, both at one x, stratified
 *       over [0, src_frac L); their ids precede the step's births.
 *   R26 relative-speed charge exchange: the rate uses the speed relative to a sampled
 *       neutral, and an exchanged ion takes that neutral's velocity.
 *   R27 node moments per species from the cloud-in-cell shares S_j of the deposit:
 *       n_j = w sum S_j / V_j, u_j = sum S_j v / sum S_j, T_j = (m/3)(sum S_j |v|^2 /
 *       sum S_j - |u_j|^2), zero mean and temperature at nodes no particle touches.
 */
#ifndef PIC_H
#define PIC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIC_OK 0
#define PIC_EINVAL (-1)      /* bad configuration, index or size                          */
#define PIC_ECAPACITY (-2)   /* particle, birth or id capacity exceeded: state undefined  */
#define PIC_ENONFINITE (-3)  /* NaN or Inf in the field solve or a particle's motion       */
#define PIC_EHIP (-4)        /* HIP runtime error; message in pic_last_error               */
#define PIC_ESTATE (-5)      /* call not valid in the current state                        */

#define PIC_FP64_PLAIN 0     /* particles as x:f64, v:f64x3, id:u32                        */
#define PIC_FP32_CELLOFF 1   /* particles as cell:i32, offset:f32 in [0,1), v:f32x3, id:u32 */

#define PIC_ABSORBING 0      /* grounded absorbing walls at x = 0 and x = L               */
#define PIC_PERIODIC 1
#define PIC_FLOATING 2       /* absorbing walls that keep the charge they absorb: no field
                              * left of x = 0, phi_0 = 0, the right wall floats (R22)      */

#define PIC_MAX_ENSEMBLES 256

typedef struct pic_ctx pic_ctx;

typedef struct {
    double q, m, w;      /* charge, mass, macro-particle weight (n0 L / P)                 */
    double T;            /* temperature of the initial Maxwellian                          */
    int64_t ppc;         /* initial particles per cell                                     */
    int64_t capacity;    /* slots reserved for this species (>= ppc * ncells)             */
} pic_species_desc;

/* One independent plasma (an "ensemble"); a run holds 1 .. PIC_MAX_ENSEMBLES of them. */
typedef struct {
    int64_t ncells;      /* N >= 2 cells of width dx; N+1 nodes bounded, N periodic       */
    double dx, dt, eps0;
    double B[3];         /* uniform magnetic field                                         */
    double E_ext;        /* uniform external field along x, added at the gather            */
    uint32_t seed;       /* Philox key word 0 (word 1 is the species index)                */
    int32_t init_mode;   /* 0: ppc per cell, Philox offsets + Maxwellian (R17);
                            1: quiet start with a sine displacement (R19)                  */
    pic_species_desc sp[2];                    /* 0 = electrons, 1 = ions                 */
    double ngs_el, ngs_iz, ngs_cx;             /* n_g sigma: e-elastic, e-ionisation, CX  */
    double eps_iz;                             /* ionisation energy                        */
    double T_n, m_n;                           /* neutral temperature and mass             */
    double perturb_amp;                        /* quiet start displacement amplitude A     */
    int32_t perturb_mode;                      /* quiet start mode number                  */
    /* The paper's sheath cases (its table of sheath cases): FP32 form and two species only. */
    int32_t recycle;          /* bounded walls: every absorbed ion returns from its wall as a
                                 neutral (species index 2 in pic_get/set_particles), reading
                                 R24; 0 = off                                              */
    int64_t neutral_capacity; /* neutrals held when recycling                              */
    int64_t src_pairs;        /* volumetric source: electron-ion pairs created per step
                                 uniformly over [0, src_frac L) (R25); 0 = off              */
    double src_frac;          /* in (0, 1]                                                 */
    int32_t cx_relative;      /* ion charge exchange at the speed relative to a neutral drawn
                                 from the background Maxwellian (R26), which then becomes the
                                 ion's velocity; 0 = the lab-frame ion speed (R10)          */
} pic_ensemble_desc;

typedef struct {
    int32_t n_ensembles;
    int32_t precision;   /* PIC_FP64_PLAIN or PIC_FP32_CELLOFF                              */
    int32_t boundary;    /* PIC_ABSORBING, PIC_PERIODIC or PIC_FLOATING (all ensembles)      */
    int32_t nspecies;    /* 1: electrons on a fixed neutralising background; 2: e + ions   */
    int32_t collisions;  /* 0: collisionless                                               */
    int32_t sort_every;  /* K in [0, 4096]: counting sort (which also compacts absorbed
                            slots) when the step count reaches a multiple of K; 0 =
                            compaction-only sort every 20 steps, physics unchanged either
                            way                                                             */
    int32_t fused;       /* 0: one kernel per stage; 1: fused particle pass + HIP graph    */
    int32_t block;       /* threads per block of the FP64 particle kernels (64, 128 or
                            256); 0 = default 256                                           */
    int32_t grid;        /* blocks of the FP64 particle kernels: the deposit and histogram
                            take this many, push and collide half, the sort scatter eight
                            times as many; 0 = default (1024)                              */
    int32_t window;      /* widest span of cells a tile deposits (and, on sort steps,
                            counts) through LDS, in [16, 4096]; a tile's window covers only
                            its own cells, so this bounds LDS per block; 0 = default 2048   */
    int32_t ppt;         /* particles per thread of the FP32 pass (4 or 8); 0 = default    */
    int32_t sort_ppt;    /* particles per thread of the FP32 sort scatter; 0 = default     */
    int32_t nontemporal; /* bit 0: the fused FP32 pass streams particles with non-temporal
                          * loads and stores; bit 1: the FP32 sort scatter reads its input
                          * with non-temporal loads;
                          * 0 = ordinary cached accesses (default)                         */
    int32_t smooth;      /* passes (0..4) of the 1-2-1 density filter applied to rho before
                          * every solve (R23): periodic grids wrap, bounded grids mirror at
                          * the walls; 0 = off                                              */
    const pic_ensemble_desc *ens;              /* [n_ensembles], copied by pic_init       */
} pic_config;

/* Scalars of one ensemble.  Counts are exact; sums are FP64. */
typedef struct {
    int64_t count[2];            /* alive particles per species                            */
    double charge;               /* sum_s q_s w_s count_s                                  */
    double ke[2];                /* 1/2 m_s w_s sum |v|^2 (current velocities)             */
    double field_energy;         /* 1/2 eps0 sum_j E_j^2 V_j of the last solved field      */
    int64_t wall_count[2][2];    /* [left, right][species] particles absorbed (cumulative)  */
    double wall_charge[2][2];    /* absorbed q w                                            */
    double wall_ke[2][2];        /* absorbed 1/2 m w |v|^2                                  */
    int64_t coll[3];             /* e-elastic, e-ionisation, ion CX events (cumulative)     */
    int64_t created[2];          /* particles created per species (cumulative)              */
    int64_t pushes;              /* particles pushed, summed over steps (cumulative)        */
    int64_t step;                /* steps taken                                             */
    double numax[2];             /* null-collision frequency bound of the last collide     */
    double emax;                 /* max |E| of the last solved / set field                  */
    int64_t neutral_count;       /* recycled neutrals alive (R24)                           */
    int64_t neutral_wall[2];     /* neutrals that left through the left / right wall        */
    int64_t recycled;            /* neutrals created from absorbed ions (cumulative)        */
    int64_t sourced;             /* pairs created by the volumetric source (cumulative)     */
} pic_diag_out;

/* Host-side particle exchange: absolute position x in [0, L), velocity, id. */
typedef struct {
    double *x, *vx, *vy, *vz;
    uint32_t *id;
} pic_particles;

/* Bytes of device workspace a configuration needs (256-byte aligned). */
int pic_query_workspace(const pic_config *cfg, size_t *bytes);

/* Create a context on `workspace` (>= the queried size, device memory) and load the
 * particles: reading R17 (random load) or R19 (quiet start) per ensemble, then the
 * cloud-in-cell deposit Q^0.  The step counter starts at 0.  This is the particle load
 * that opens the cycle of the paper's Background section, at the particles per cell of
 * its sheath-case table (experimental setup). */
int pic_init(const pic_config *cfg, void *workspace, size_t bytes, void *stream, pic_ctx **out);

/* Cloud-in-cell deposit (Birdsall-Langdon linear weighting) of every alive particle into
 * the per-species node sums Q_s (FP32 form: int64 fixed point, 2^24 per particle, R15;
 * FP64 form: FP64 sums).  Replaces the previous Q.  The "deposition to the grid" step of
 * the cycle in the paper's Background section. */
int pic_deposit(pic_ctx *ctx, void *stream);

/* Field solve from Q: rho_j = sum_s q_s w_s Q_{s,j} / V_j, optionally smoothed (R23), the
 * three-point Poisson stencil with grounded walls (R3), a neutralising background and
 * zero-mean phi (R4), or floating walls (R22: E_{1/2} = (sigma_L + rho_0 V_0) / eps0 with
 * sigma_L the charge absorbed so far at the left wall, phi_0 = 0), solved exactly by two
 * prefix sums (equivalent to the Thomas solve, R5), node E from the centred difference
 * with the half-cell Gauss rule at walls (R6).  FP64.  The density smoothing and wall
 * boundary conditions follow the cycle of the paper's Background section and the
 * charge-depositing walls of its sheath cases (experimental setup). */
int pic_solve(pic_ctx *ctx, void *stream);

/* Gather E at each particle (linear), Boris push in E + E_ext along x and uniform B,
 * position update, absorbing walls (R8: absorbed slots are marked dead and tallied; the
 * next sort compacts them) or periodic wrap.  With recycling (R24) the neutrals stream
 * freely, leave through the walls, and the ions absorbed in this push return as neutrals.
 * The "force interpolation" and "mover" steps of the cycle in the paper's Background
 * section (the mover is where its profiles put most of the time: performance results), in
 * the magnetised layer between absorbing walls of its sheath cases (experimental setup). */
int pic_push(pic_ctx *ctx, void *stream);

/* Null-collision Monte Carlo (R9-R14): per-particle Philox decision against the bound
 * nu_max, channel choice, scattering kinematics, ionisation births appended with ids
 * next_id + rank of the parent id.  The step's volumetric source pairs (R25) are created
 * here too, numbered before the births.  The "Monte Carlo collisions" step of the cycle in
 * the paper's Background section, against the uniform neutral background of its sheath
 * cases (experimental setup). */
int pic_collide(pic_ctx *ctx, void *stream);

/* Counting sort of each species by cell (histogram, exclusive scan, scatter); drops the
 * absorbed slots, so it is also the stream compaction.  Order inside a cell is unspecified.
 * The "natural sorting" of particles by cell that the paper's Background section credits
 * for faster collision operators (its arranger, the other large item of its profiles:
 * performance results). */
int pic_sort(pic_ctx *ctx, void *stream);

/* nsteps full steps (R2 order): solve, push + walls, collide, deposit, and a sort when
 * the new step count is a multiple of K: the whole cycle of the paper's Background
 * section, once per time step.  With cfg.fused = 1 the particle stages run as
 * one pass per step and the steps replay captured HIP graphs (see pic_graph_prepare);
 * in the FP32 form with
 * K >= 2 the step before a sort step also counts the cells, and the sort step's pass
 * writes the particles in the order of the cells they held before its push (so the
 * particles are ordered by cell up to that push, and the sort costs no kernel of its
 * own).  Synchronises the stream once at the end to read the sticky error flags. */
int pic_step(pic_ctx *ctx, int32_t nsteps, void *stream);

/* Instantiate, without running them, the HIP graphs that pic_step(ctx, nsteps) would
 * replay from the current state, so that a later pic_step of that many steps spends no
 * time on capture (e.g. before a timed or latency-bound loop).  A fused run replays one
 * graph per window of up to K steps: whole sort cycles from whatever phase of the cycle
 * the run is in, then a shorter tail, which replays from a graph only if this call
 * prepared it (otherwise those steps run eagerly).  Graphs stay valid until pic_load,
 * pic_autotune or pic_free.  A no-op for cfg.fused = 0. */
int pic_graph_prepare(pic_ctx *ctx, int32_t nsteps);

/* Number of graph replays pic_step has made on this context (so a caller can tell that a
 * run went through the graph path). */
int pic_graph_launches(const pic_ctx *ctx, int64_t *launches);

/* Diagnostics of ensemble `ens` (synchronises `stream`).  `out` receives the scalars.
 * `moments_dev` is NULL or device memory of 5 x nspecies x nnodes doubles (nnodes from
 * pic_nnodes), laid out [species][quantity][node] with the quantities, per node j, of
 * reading R27 computed from the cloud-in-cell shares S_j of the deposit: number density
 * n_j = w sum S_j / V_j (V_j = dx, dx/2 at bounded walls), mean velocity
 * u_j = sum S_j v / sum S_j (x, y, z) and temperature
 * T_j = (m/3)(sum S_j |v|^2 / sum S_j - |u_j|^2), with u_j = T_j = 0 at nodes no particle
 * touches.  These are the per-species density, flow and temperature profiles that the
 * paper's input-parameter table switches on as time-averaged output and its in-situ
 * analysis plots (results section).  Sums in FP64 atomics: the last bits depend on order.
 * The library overwrites the whole array; the caller owns it. */
int pic_diag(pic_ctx *ctx, int32_t ens, pic_diag_out *out, double *moments_dev, void *stream);

/* Copy the alive particles of (ens, species) to host arrays of length >= `cap`; `count`
 * receives the number written.  Order unspecified (compare by id).  Species 2 is the
 * recycled neutral set (R24). */
int pic_get_particles(pic_ctx *ctx, int32_t ens, int32_t species, pic_particles out,
                      int64_t cap, int64_t *count, void *stream);

/* Raw slots [first, first + count) of (ens, species) in the current buffer, absorbed slots
 * included (their x is -1), without compaction: a cheap sampled read-back for runs too
 * large to copy whole.  Slot order is the load order until the first sort. */
int pic_get_slots(pic_ctx *ctx, int32_t ens, int32_t species, int64_t first, int64_t count,
                  pic_particles out, void *stream);

/* Replace the particles of (ens, species) with `count` host particles (x in [0, L); in the
 * FP32 form an x whose x / dx rounds up to N goes to the top of the last cell);
 * next_id is the id the next created particle of this species receives (ignored for the
 * neutral set, species 2, whose ids are those of the ions they came from). */
int pic_set_particles(pic_ctx *ctx, int32_t ens, int32_t species, pic_particles in,
                      int64_t count, uint32_t next_id, void *stream);

/* Copy node arrays of ensemble `ens` to host (each may be NULL; length = node count):
 * Q_s as particle units, rho, phi, E (self-consistent part). */
int pic_get_grid(pic_ctx *ctx, int32_t ens, double *Q0, double *Q1, double *rho, double *phi,
                 double *E, void *stream);

/* Copy the FP32 form's gather table of ensemble `ens` to host: per cell j the binary32
 * pair (E_j, E_{j+1} - E_j) the push interpolates from (E_N is E_0 when periodic);
 * `out` holds 2 x ncells floats.  PIC_EINVAL for the FP64 form (it gathers from E). */
int pic_get_gather_table(pic_ctx *ctx, int32_t ens, float *out, void *stream);

/* Replace the self-consistent node field of ensemble `ens` with host values (test hook:
 * push in a given field, e.g. zero). */
int pic_set_fields(pic_ctx *ctx, int32_t ens, const double *E, void *stream);

/* Set the step counter (the collision random-number tag of the next collide). */
int pic_set_step(pic_ctx *ctx, int64_t step);

/* Node count of ensemble `ens` (N+1 bounded, N periodic), or a negative error. */
int64_t pic_nnodes(const pic_ctx *ctx, int32_t ens);

/* Set the uniform external field E_ext of ensemble `ens` (added at the gather). */
int pic_set_external_field(pic_ctx *ctx, int32_t ens, double E_ext);

/* Scratch bytes pic_adjoint_window needs for `nsteps` steps with a checkpoint every
 * `ckpt_every` steps (caller-allocated device memory). */
int pic_adjoint_query(pic_ctx *ctx, int32_t nsteps, int32_t ckpt_every, size_t *bytes);

/* Hand-written discrete adjoint of the collisionless push + deposit + Poisson window
 * (reading R20): runs `nsteps` steps from the current state, computes the field energy
 * W = 1/2 eps0 dx sum_j E_j^2 at the final positions, and the exact gradients of that
 * discrete forward (cell index held locally constant) with respect to the initial x
 * velocities and to the uniform external field.  Checkpoints every `ckpt_every` steps and
 * recomputes each segment forward before its reverse sweep.  Requires one ensemble, one
 * periodic species, no collisions, B = 0 and the FP32 form; no sort runs inside the
 * window.  dW_dvx (host, length >= particle count) is indexed by particle id.  On return
 * the particle state is the final state of the window.  Synchronises `stream`. */
int pic_adjoint_window(pic_ctx *ctx, int32_t nsteps, int32_t ckpt_every, void *scratch,
                       size_t bytes, double *W, double *dW_dvx, int64_t dvx_len,
                       double *dW_dEext, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving or optimisation loops, harnesses that forbid hipMalloc): pic_adjoint_window with
 * no scratch argument.  Its scratch (the window's checkpoints, recorded positions and fields,
 * adjoint arrays, then dvx_len doubles for the by-id gradient) lives in a static device
 * array of 160 MiB that the library holds on every GPU it runs on until the process ends;
 * pic_init looks up its address on the context's device.  Calls that need more return
 * PIC_EINVAL with the size in pic_last_error (the 2048-cell, 409,600-particle, 200-step
 * window at a checkpoint every 20 steps needs about 127 MiB).  The call allocates nothing
 * (no hipMalloc, hipFree or allocating library routine); it clears what must start at zero.
 * Every call on one GPU shares that GPU's array, so calls that overlap on one GPU (two
 * contexts on two host threads or two streams) race: serialise them.  Arguments, results,
 * requirements and errors are otherwise those of pic_adjoint_window; synchronises `stream`. */
int pic_adjoint_window_noalloc(pic_ctx *ctx, int32_t nsteps, int32_t ckpt_every, double *W,
                               double *dW_dvx, int64_t dvx_len, double *dW_dEext, void *stream);

/* The library's autotuner: times the particle pass over `trial_steps` steps for every
 * candidate launch shape (particles per thread x widest LDS window span x, for the fused
 * pass, non-temporal streaming) and the sort scatter for each particles-per-thread and
 * non-temporal-load choice, all with HIP events on `stream`, keeps the fastest, and
 * writes {ppt, window, sort_ppt, pass non-temporal, sort non-temporal} to `shape`
 * (5 ints, may be NULL).  The trial steps advance the
 * run like pic_step (the sort is repeated on already-sorted data, which leaves the state
 * unchanged apart from slot order). */
int pic_autotune(pic_ctx *ctx, int32_t trial_steps, int32_t *shape, void *stream);

/* Device-state checkpoint of the run at a step boundary: the particles in use (in slot
 * order), the deposited charge, the per-segment slot counts and id counters, the step,
 * the current speed maxima and the diagnostic counters.  A context created with the same
 * configuration and loaded from it continues bit for bit as the saved run would have
 * (random numbers are keyed by particle id and step).  pic_checkpoint_size gives the
 * bytes of the host buffer pic_save fills (it depends on the slots in use, so query it
 * right before saving); both synchronise `stream`.  pic_load returns PIC_EINVAL for a
 * buffer written by a different configuration. */
int pic_checkpoint_size(pic_ctx *ctx, size_t *bytes, void *stream);
int pic_save(pic_ctx *ctx, void *host_buf, size_t bytes, void *stream);
int pic_load(pic_ctx *ctx, const void *host_buf, size_t bytes, void *stream);

/* Measurement hook: with `enable` != 0, pic_step runs its steps without the graph and
 * brackets every particle-pass launch with HIP events recorded on the caller's stream
 * (up to 65536 launches), except the fused FP32 passes that also sort (one per K steps,
 * a kernel of their own); pic_timing_read synchronises that stream and returns the summed
 * kernel time in milliseconds and the number of timed launches.  Enabling again resets. */
int pic_timing(pic_ctx *ctx, int32_t enable);
int pic_timing_read(pic_ctx *ctx, double *ms_total, int64_t *launches, void *stream);

/* Measurement hook: copy `bytes` (a multiple of 16) of device memory from `src` to `dst`
 * (not overlapping) with the particle pass's access pattern: 256 threads a block, four
 * consecutive 32-bit words a thread, one 16-byte load and one 16-byte store, non-temporal
 * when `nontemporal` is non-zero.  Its bandwidth and its traffic counters are the
 * reference the pass is read against (the counters' scale, the achievable stream rate).
 * Asynchronous on `stream`; PIC_EINVAL for a null pointer or a size not a multiple of 16. */
int pic_stream_copy(const void *src, void *dst, size_t bytes, int32_t nontemporal, void *stream);

void pic_free(pic_ctx *ctx);
const char *pic_last_error(const pic_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
