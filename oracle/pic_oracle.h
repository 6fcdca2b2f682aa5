/*
 * pic_oracle.h -- plain FP64 CPU oracle of the electrostatic 1D3V PIC Monte Carlo step.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously-correct reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it; the product path never does.  It shares no code, header,
 * table or constant generator with the GPU library.
 *
 * What it computes follows the PIC cycle the paper names in its Background section
 * (particle load, mover, deposition to the grid, electrostatic field solve, force
 * interpolation, Monte Carlo collisions) for the 1D3V electrostatic code described there.
 * The paper gives no equations for these steps, so each one is the textbook method it
 * names implicitly (Birdsall-Langdon cloud-in-cell, a three-point Poisson stencil solved
 * by the Thomas algorithm, the Boris rotation, the Vahedi-Surendra null-collision method),
 * with every unstated choice fixed by a written reading (the R-tags in the comments).
 *
 * Units are normalised: eps0 = e = m_e = n0 = T_e = 1, so omega_pe = v_th,e = lambda_D = 1.
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
#ifndef PIC_ORACLE_H
#define PIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One charged species. */
typedef struct {
    double q, m, w;      /* charge, mass, macro-particle weight (real particles per area)   */
    double T;            /* temperature of the initial Maxwellian                            */
    int64_t ppc;         /* initial particles per cell                                       */
    int64_t capacity;    /* maximum particles held                                           */
} orc_species;

typedef struct {
    int64_t ncells;      /* N cells; N+1 nodes when bounded, N nodes when periodic            */
    int32_t periodic;    /* 0 = absorbing grounded walls, 1 = periodic                        */
    int32_t nspecies;    /* 1 (electrons on a fixed neutralising background) or 2 (e, ion)    */
    int32_t collisions;  /* 0 = collisionless                                                 */
    int32_t init_mode;   /* 0 = random cell load + Maxwellian, 1 = cold quiet start + sine    */
    double dx, dt, eps0;
    double B[3];         /* uniform magnetic field                                            */
    double E_ext;        /* uniform external field along x                                    */
    uint32_t seed;       /* Philox key word 0                                                 */
    int32_t sort_every;  /* K; 0 = never                                                      */
    orc_species sp[2];   /* 0 = electrons, 1 = ions                                           */
    double ngs_el, ngs_iz, ngs_cx;  /* n_g * sigma for e-elastic, e-ionisation, ion CX       */
    double eps_iz;       /* ionisation energy                                                 */
    double T_n, m_n;     /* neutral temperature and mass                                      */
    double perturb_amp;  /* quiet start: displacement amplitude A (density ~ 1 - A cos kx)    */
    int32_t perturb_mode;
    int32_t floating;    /* bounded only: 1 = the walls keep the charge they absorb (R22)     */
    int32_t smooth;      /* passes of the 1-2-1 filter on rho before the solve (R23), 0 = off */
    int32_t recycle;     /* bounded, two species: ions absorbed at a wall return as neutrals
                            (R24), held in a neutral set of `neutral_capacity` particles      */
    int64_t neutral_capacity;
    int64_t src_pairs;   /* electron-ion pairs created per step by the volumetric source (R25) */
    double src_frac;     /* the source fills [0, src_frac L)                                  */
    int32_t cx_relative; /* ion CX rate from the speed relative to a sampled neutral (R26)    */
} orc_config;

/* Cumulative diagnostics (reset only by orc_create / orc_init). */
typedef struct {
    int64_t count[2];            /* particles alive per species                              */
    double charge;               /* sum_s q_s w_s n_s                                        */
    double ke[2];                /* 1/2 m_s w_s sum |v|^2                                    */
    double field_energy;         /* 1/2 eps0 sum_j E_j^2 V_j of the self-consistent field    */
    int64_t wall_count[2][2];    /* [wall 0=left,1=right][species] absorbed particles        */
    double wall_charge[2][2];    /* absorbed q w                                             */
    double wall_ke[2][2];        /* absorbed 1/2 m w |v|^2                                   */
    int64_t coll[3];             /* e-elastic, e-ionisation, ion charge exchange             */
    int64_t created[2];          /* particles created per species                            */
    int64_t pushes;              /* sum over steps of the particles pushed                   */
    int64_t step;
    int64_t neutral_count;       /* recycled neutrals alive (R24)                            */
    int64_t neutral_wall[2];     /* neutrals that left through the left / right wall         */
    int64_t recycled;            /* neutrals created from absorbed ions                      */
    int64_t sourced;             /* pairs created by the volumetric source (R25)             */
} orc_diag;

typedef struct orc_state orc_state;

/* Threads the particle loops use: 1 in the default build; the OpenMP team size in the
 * OpenMP build, which exists only to time the oracle on all host cores (its deposit adds
 * per-thread partial sums, so its last bits differ from the default build's). */
int orc_threads(void);

orc_state *orc_create(const orc_config *cfg);
void orc_free(orc_state *st);
/* Non-zero after a capacity overflow (1, 3) or a particle outside the grid (2). */
int orc_error(const orc_state *st);

/* Particle load (R17 init / R19 quiet start), then deposit of Q^0 and the speed bound. */
void orc_init(orc_state *st);

/* The load of one particle p of species s (the same recipe as orc_init), for checking
 * sampled particles of runs too large to load whole on the CPU. */
void orc_init_particle(const orc_config *cfg, int s, int64_t p, double *x, double *vx, double *vy,
                       double *vz);

/* Inject / read back a species' particles: absolute x, velocity, id.  Species 2 is the
 * recycled neutral set (R24; its next_id argument is ignored).                           */
int orc_set_particles(orc_state *st, int s, int64_t n, const double *x, const double *vx,
                      const double *vy, const double *vz, const uint32_t *id, uint32_t next_id);
int64_t orc_get_particles(const orc_state *st, int s, double *x, double *vx, double *vy,
                          double *vz, uint32_t *id);
uint32_t orc_next_id(const orc_state *st, int s);

/* The stages of one step, callable one by one. */
void orc_deposit(orc_state *st);                 /* particles -> Q_s (FP64 CIC shares)    */
void orc_solve(orc_state *st);                   /* Q -> rho -> phi -> E (Thomas)         */
void orc_set_fields(orc_state *st, const double *E);  /* replace E (self part)           */
void orc_push(orc_state *st);                    /* gather + Boris + position update      */
void orc_walls(orc_state *st);                   /* absorb (bounded) or wrap (periodic)   */
void orc_collide(orc_state *st);                 /* null-collision MC, volumetric source
                                                    pairs (R25) and ionisation births      */
void orc_sort(orc_state *st);                    /* stable counting sort by cell          */
void orc_step(orc_state *st, int64_t nsteps);    /* full steps, including the step count  */

/* Read-outs. */
int64_t orc_nnodes(const orc_state *st);
void orc_get_grid(const orc_state *st, double *Q0, double *Q1, double *rho, double *phi,
                  double *E);
void orc_get_diag(orc_state *st, orc_diag *out);
/* Collision bookkeeping of the last orc_collide call: per alive particle (post-wall order)
 * the channel taken (-1 none, 0 elastic, 1 ionisation, 2 CX), and nu_max per species. */
/* Node moments of species s from the cloud-in-cell shares (reading R27): number density
 * n_j = w W_j / V_j, mean velocity u_j and temperature T_j = (m/3)(<|v|^2>_j - |u_j|^2),
 * each an array of nnodes (NULL skips it). */
void orc_moments(const orc_state *st, int s, double *n, double *ux, double *uy, double *uz,
                 double *T);
int64_t orc_last_channels(const orc_state *st, int s, int32_t *chan, uint32_t *ids);
void orc_last_numax(const orc_state *st, double *numax, double *pnull);
void orc_set_step(orc_state *st, int64_t step);

/* Philox4x32 block (ORC_PHILOX_ROUNDS rounds) and the derived variates, exposed for
 * pinning. */
#define ORC_PHILOX_ROUNDS 7
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* n independent blocks: ctr[4n], key[2n] -> out[4n]. */
void orc_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out);
double orc_uniform(uint32_t r);
void orc_boxmuller(double u1, double u2, double *z0, double *z1);

/* Reading R23: `passes` of the 1-2-1 filter on node densities rho[0 .. nn), in place:
 * periodic wraps, bounded mirrors at the walls (rho_{-1} = rho_1, rho_{N+1} = rho_{N-1}).
 * Exposed for pinning. */
void orc_smooth_nodes(int64_t nn, int32_t periodic, int32_t passes, double *rho);

/* Tridiagonal (Thomas) solve of a_i x_{i-1} + b_i x_i + c_i x_{i+1} = d_i, exposed for pinning. */
void orc_thomas(int64_t n, const double *a, const double *b, const double *c, const double *d,
                double *x);

#ifdef __cplusplus
}
#endif
#endif
