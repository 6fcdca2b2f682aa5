/*
 * pic_oracle.c -- plain FP64 CPU oracle of the electrostatic 1D3V PIC Monte Carlo step.
 *
 * TEST INFRASTRUCTURE ONLY (see pic_oracle.h).  Single-threaded, no blocking, no fusion:
 * each stage is one loop over particles or nodes, written to be checked against the
 * textbook definition by eye.  Built with -ffp-contract=off so that no multiply-add is
 * fused behind the reader's back.
 *
 * Step order (one step n -> n+1), reading R2 (Birdsall-Langdon leapfrog levels: the state
 * is x^n, v^{n-1/2} and the deposited charge Q^n):
 *   solve (Q^n -> rho -> phi -> E^n), push (gather E^n at x^n, Boris -> v^{n+1/2},
 *   x^{n+1}), walls, null-collision MC, deposit Q^{n+1}, sort when (n+1) % K == 0.
 * The paper's Background section lists mover, deposition, field solve and force
 * interpolation plus MC collisions as the cycle; it does not fix their order or levels.
 */
#include "pic_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define ORC_TWO_PI 6.283185307179586476925286766559
/* Inflation of the null-collision frequency bound (reading R11). */
#define ORC_NU_SAFETY (1.0 + 1.0 / 65536.0)
/* Reading R26: a Box-Muller radius is at most sqrt(-2 ln 2^-24) (the smallest uniform is
 * 2^-24), and a neutral velocity's first two normals share one radius, so
 * |v_n| <= sqrt(2) sqrt(48 ln 2) v_tn = sqrt(96 ln 2) v_tn.                               */
#define ORC_VN_BOUND (sqrt(96.0 * log(2.0)))
#define ORC_INIT_TAG 0xFFFFFFFFu

struct orc_state {
    orc_config cfg;
    int64_t nnodes;
    int64_t n[2], cap[2];
    double *x[2], *vx[2], *vy[2], *vz[2];
    uint32_t *id[2];
    uint32_t next_id[2];
    double *Q[2], *rho, *phi, *E;
    double vmax[2];       /* max |v| over the particles present at the start of a step */
    double Emax;          /* max |E_self| over nodes from the last solve / set_fields   */
    int64_t step;
    orc_diag d;
    int32_t *last_chan[2];
    uint32_t *last_id[2];
    int64_t last_n[2];
    double numax[2], pnull[2];
    /* recycled neutrals (R24): absolute x, velocity, id (the id of the ion they came from) */
    double *nx, *nvx, *nvy, *nvz;
    uint32_t *nid;
    int64_t nneu, ncap;
    int err;
};

/* ------------------------------------------------------------------------------------ */
/* Philox4x32 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11) with ORC_PHILOX_ROUNDS rounds (reading R17: seven, the smallest round count the
 * paper finds Crush-resistant for this generator): each round takes two 32x32->64
 * multiplies on counter words 0 and 2 with the published multipliers, xors the high halves
 * with the other counter words and the round key, and the key is bumped by the published
 * Weyl constants between rounds.                                                         */
void orc_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < ORC_PHILOX_ROUNDS; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

void orc_philox_batch(int64_t n, const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    for (int64_t i = 0; i < n; i++) orc_philox4x32(ctr + 4 * i, key + 2 * i, out + 4 * i);
}

/* Reading R17: u = ((r >> 9) + 1/2) * 2^-23, an odd multiple of 2^-24 in (0, 1); exactly
 * representable in binary32 and binary64, so both precisions see the same number.        */
double orc_uniform(uint32_t r) { return ((double)(r >> 9) + 0.5) * 0x1p-23; }

/* Box-Muller: two independent standard normals from two uniforms. */
void orc_boxmuller(double u1, double u2, double *z0, double *z1)
{
    double rad = sqrt(-2.0 * log(u1));
    *z0 = rad * cos(ORC_TWO_PI * u2);
    *z1 = rad * sin(ORC_TWO_PI * u2);
}

static void draw_block(const orc_state *st, int s, uint32_t id, uint32_t tag, uint32_t blk,
                       uint32_t w[4])
{
    uint32_t ctr[4] = {id, tag, blk, 0u};
    uint32_t key[2] = {st->cfg.seed, (uint32_t)s};
    orc_philox4x32(ctr, key, w);
}

/* Three standard normals from one Philox block: (w0, w1) -> z0, z1 and (w2, w3) -> z2. */
static void three_normals(const uint32_t w[4], double z[3])
{
    double dummy;
    orc_boxmuller(orc_uniform(w[0]), orc_uniform(w[1]), &z[0], &z[1]);
    orc_boxmuller(orc_uniform(w[2]), orc_uniform(w[3]), &z[2], &dummy);
}

/* Isotropic unit vector from two uniforms: cos(chi) = 1 - 2 ua, azimuth = 2 pi ub. */
static void iso_dir(double ua, double ub, double d[3])
{
    double c = 1.0 - 2.0 * ua;
    double s2 = 1.0 - c * c;
    double sn = s2 > 0.0 ? sqrt(s2) : 0.0;
    double ph = ORC_TWO_PI * ub;
    d[0] = c;
    d[1] = sn * cos(ph);
    d[2] = sn * sin(ph);
}

/* ------------------------------------------------------------------------------------ */
/* Thomas algorithm (forward elimination, back substitution) for a tridiagonal system.  */
void orc_thomas(int64_t n, const double *a, const double *b, const double *c, const double *d,
                double *x)
{
    if (n <= 0) return;
    double *cp = (double *)malloc((size_t)n * sizeof(double));
    double *dp = (double *)malloc((size_t)n * sizeof(double));
    cp[0] = c[0] / b[0];
    dp[0] = d[0] / b[0];
    for (int64_t i = 1; i < n; i++) {
        double den = b[i] - a[i] * cp[i - 1];
        cp[i] = c[i] / den;
        dp[i] = (d[i] - a[i] * dp[i - 1]) / den;
    }
    x[n - 1] = dp[n - 1];
    for (int64_t i = n - 2; i >= 0; i--) x[i] = dp[i] - cp[i] * x[i + 1];
    free(cp);
    free(dp);
}

/* ------------------------------------------------------------------------------------ */
static double dlen(const orc_state *st) { return (double)st->cfg.ncells * st->cfg.dx; }

static double node_volume(const orc_state *st, int64_t j)
{
    if (!st->cfg.periodic && (j == 0 || j == st->cfg.ncells)) return 0.5 * st->cfg.dx;
    return st->cfg.dx;
}

static double speed2(double vx, double vy, double vz) { return vx * vx + vy * vy + vz * vz; }

/* Cell j = floor(x / dx) and fraction f = x / dx - j of a position inside the grid.
 * Reading R8 keeps every x < L inside, but for a dx that is not a power of two x / dx can
 * round up to N for x just below L: such a particle belongs to the last cell (f = 1).
 * Returns -1 for a position outside [0, L).                                              */
static int64_t cell_index(const orc_state *st, double x, double *f)
{
    const orc_config *c = &st->cfg;
    double g = x / c->dx;
    double jf = floor(g);
    if (!(x >= 0.0) || !(x < dlen(st))) return -1;
    if (jf > (double)(c->ncells - 1)) jf = (double)(c->ncells - 1);
    *f = g - jf;
    return (int64_t)jf;
}

static void recompute_vmax(orc_state *st, int s)
{
    double m2 = 0.0;
#pragma omp parallel for schedule(static) reduction(max : m2)
    for (int64_t p = 0; p < st->n[s]; p++) {
        double v2 = speed2(st->vx[s][p], st->vy[s][p], st->vz[s][p]);
        if (v2 > m2) m2 = v2;
    }
    st->vmax[s] = sqrt(m2);
}

orc_state *orc_create(const orc_config *cfg)
{
    orc_state *st = (orc_state *)calloc(1, sizeof(orc_state));
    st->cfg = *cfg;
    st->nnodes = cfg->periodic ? cfg->ncells : cfg->ncells + 1;
    for (int s = 0; s < cfg->nspecies; s++) {
        int64_t cap = cfg->sp[s].capacity;
        st->cap[s] = cap;
        st->x[s] = (double *)calloc((size_t)cap + 1, sizeof(double));
        st->vx[s] = (double *)calloc((size_t)cap + 1, sizeof(double));
        st->vy[s] = (double *)calloc((size_t)cap + 1, sizeof(double));
        st->vz[s] = (double *)calloc((size_t)cap + 1, sizeof(double));
        st->id[s] = (uint32_t *)calloc((size_t)cap + 1, sizeof(uint32_t));
        st->last_chan[s] = (int32_t *)calloc((size_t)cap + 1, sizeof(int32_t));
        st->last_id[s] = (uint32_t *)calloc((size_t)cap + 1, sizeof(uint32_t));
        st->Q[s] = (double *)calloc((size_t)st->nnodes + 1, sizeof(double));
    }
    st->rho = (double *)calloc((size_t)st->nnodes + 1, sizeof(double));
    st->phi = (double *)calloc((size_t)st->nnodes + 1, sizeof(double));
    st->E = (double *)calloc((size_t)st->nnodes + 1, sizeof(double));
    st->ncap = cfg->recycle ? cfg->neutral_capacity : 0;
    st->nx = (double *)calloc((size_t)st->ncap + 1, sizeof(double));
    st->nvx = (double *)calloc((size_t)st->ncap + 1, sizeof(double));
    st->nvy = (double *)calloc((size_t)st->ncap + 1, sizeof(double));
    st->nvz = (double *)calloc((size_t)st->ncap + 1, sizeof(double));
    st->nid = (uint32_t *)calloc((size_t)st->ncap + 1, sizeof(uint32_t));
    return st;
}

void orc_free(orc_state *st)
{
    if (!st) return;
    for (int s = 0; s < 2; s++) {
        free(st->x[s]);
        free(st->vx[s]);
        free(st->vy[s]);
        free(st->vz[s]);
        free(st->id[s]);
        free(st->last_chan[s]);
        free(st->last_id[s]);
        free(st->Q[s]);
    }
    free(st->rho);
    free(st->phi);
    free(st->E);
    free(st->nx);
    free(st->nvx);
    free(st->nvy);
    free(st->nvz);
    free(st->nid);
    free(st);
}

int orc_error(const orc_state *st) { return st->err; }

/* Threads the particle loops run on: 1, or the OpenMP team size when the oracle is built
 * with OpenMP (a timing build only; its deposit sums in a different order). */
int orc_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------ */
/* Particle load.
 * Reading R17 (init_mode 0): particle p of species s has id p and sits in cell p / ppc;
 *   Philox block 0 of the init tag gives its in-cell offset, block 1 three normals that
 *   scale to a Maxwellian at T_s.
 * Reading R19 (init_mode 1): quiet start x0 = (p + 1/2) L / P displaced by
 *   (A / k) sin(k x0) with k = 2 pi mode / L, which gives density ~ 1 - A cos(k x) to first
 *   order; velocities Maxwellian at T_s (cold when T_s = 0).                              */
void orc_init_particle(const orc_config *c, int s, int64_t p, double *xo, double *vx, double *vy,
                       double *vz)
{
    int64_t ppc = c->sp[s].ppc;
    int64_t P = ppc * c->ncells;
    double L = (double)c->ncells * c->dx;
    double vth = sqrt(c->sp[s].T / c->sp[s].m);
    uint32_t w[4];
    uint32_t key[2] = {c->seed, (uint32_t)s};
    double z[3];
    double x;
    if (c->init_mode == 0) {
        int64_t cell = p / ppc;
        uint32_t ctr[4] = {(uint32_t)p, ORC_INIT_TAG, 0u, 0u};
        orc_philox4x32(ctr, key, w);
        x = ((double)cell + orc_uniform(w[0])) * c->dx;
    } else {
        double k = ORC_TWO_PI * (double)c->perturb_mode / L;
        double x0 = ((double)p + 0.5) * L / (double)P;
        x = x0 + (c->perturb_amp / k) * sin(k * x0);
        while (x < 0.0) x += L;
        while (x >= L) x -= L;
    }
    uint32_t ctr1[4] = {(uint32_t)p, ORC_INIT_TAG, 1u, 0u};
    orc_philox4x32(ctr1, key, w);
    three_normals(w, z);
    *xo = x;
    *vx = vth * z[0];
    *vy = vth * z[1];
    *vz = vth * z[2];
}

void orc_init(orc_state *st)
{
    const orc_config *c = &st->cfg;
    for (int s = 0; s < c->nspecies; s++) {
        int64_t ppc = c->sp[s].ppc;
        int64_t P = ppc * c->ncells;
        if (P > st->cap[s]) {
            st->err = 1;
            P = st->cap[s];
        }
        for (int64_t p = 0; p < P; p++) {
            orc_init_particle(c, s, p, &st->x[s][p], &st->vx[s][p], &st->vy[s][p], &st->vz[s][p]);
            st->id[s][p] = (uint32_t)p;
        }
        st->n[s] = P;
        st->next_id[s] = (uint32_t)P;
        recompute_vmax(st, s);
    }
    st->step = 0;
    st->nneu = 0;
    memset(&st->d, 0, sizeof(st->d));
    orc_deposit(st);
}

int orc_set_particles(orc_state *st, int s, int64_t n, const double *x, const double *vx,
                      const double *vy, const double *vz, const uint32_t *id, uint32_t next_id)
{
    if (s == 2) {
        if (n < 0 || n > st->ncap) return -1;
        memcpy(st->nx, x, (size_t)n * sizeof(double));
        memcpy(st->nvx, vx, (size_t)n * sizeof(double));
        memcpy(st->nvy, vy, (size_t)n * sizeof(double));
        memcpy(st->nvz, vz, (size_t)n * sizeof(double));
        memcpy(st->nid, id, (size_t)n * sizeof(uint32_t));
        st->nneu = n;
        return 0;
    }
    if (s < 0 || s >= st->cfg.nspecies || n > st->cap[s] || n < 0) return -1;
    memcpy(st->x[s], x, (size_t)n * sizeof(double));
    memcpy(st->vx[s], vx, (size_t)n * sizeof(double));
    memcpy(st->vy[s], vy, (size_t)n * sizeof(double));
    memcpy(st->vz[s], vz, (size_t)n * sizeof(double));
    memcpy(st->id[s], id, (size_t)n * sizeof(uint32_t));
    st->n[s] = n;
    st->next_id[s] = next_id;
    recompute_vmax(st, s);
    return 0;
}

int64_t orc_get_particles(const orc_state *st, int s, double *x, double *vx, double *vy,
                          double *vz, uint32_t *id)
{
    if (s == 2) {
        int64_t m = st->nneu;
        if (x) memcpy(x, st->nx, (size_t)m * sizeof(double));
        if (vx) memcpy(vx, st->nvx, (size_t)m * sizeof(double));
        if (vy) memcpy(vy, st->nvy, (size_t)m * sizeof(double));
        if (vz) memcpy(vz, st->nvz, (size_t)m * sizeof(double));
        if (id) memcpy(id, st->nid, (size_t)m * sizeof(uint32_t));
        return m;
    }
    int64_t n = st->n[s];
    if (x) memcpy(x, st->x[s], (size_t)n * sizeof(double));
    if (vx) memcpy(vx, st->vx[s], (size_t)n * sizeof(double));
    if (vy) memcpy(vy, st->vy[s], (size_t)n * sizeof(double));
    if (vz) memcpy(vz, st->vz[s], (size_t)n * sizeof(double));
    if (id) memcpy(id, st->id[s], (size_t)n * sizeof(uint32_t));
    return n;
}

uint32_t orc_next_id(const orc_state *st, int s) { return (s >= 0 && s < 2) ? st->next_id[s] : 0u; }
int64_t orc_nnodes(const orc_state *st) { return st->nnodes; }
void orc_set_step(orc_state *st, int64_t step) { st->step = step; }

/* ------------------------------------------------------------------------------------ */
/* Cloud-in-cell deposit (Birdsall-Langdon linear weighting): a particle at
 * x = (j + f) dx gives share 1 - f to node j and f to node j+1 (node N wraps to 0 when
 * periodic).  Q_s holds the share sums; charge density follows in the solve.             */
void orc_deposit(orc_state *st)
{
    const orc_config *c = &st->cfg;
    for (int s = 0; s < c->nspecies; s++) {
        double *Q = st->Q[s];
        int64_t nq = st->nnodes + 1;
        memset(Q, 0, (size_t)nq * sizeof(double));
#pragma omp parallel for schedule(static) reduction(+ : Q[:nq])
        for (int64_t p = 0; p < st->n[s]; p++) {
            double f = 0.0;
            int64_t j = cell_index(st, st->x[s][p], &f);
            if (j < 0) {
                st->err = 2;
                continue;
            }
            int64_t j1 = j + 1;
            if (c->periodic && j1 == c->ncells) j1 = 0;
            Q[j] += 1.0 - f;
            Q[j1] += f;
        }
    }
}

/* Field solve.
 * rho_j = sum_s q_s w_s Q_{s,j} / V_j with V_j = dx inside and dx/2 at bounded walls.
 * Reading R3 (bounded): grounded walls phi_0 = phi_N = 0.
 * Reading R4 (periodic): a uniform background cancels the net deposited charge; phi_0 = 0
 *   fixes the free constant, then the mean of phi is removed.
 * Reading R5: the three-point stencil (phi_{j-1} - 2 phi_j + phi_{j+1}) / dx^2 = -rho_j/eps0
 *   on the interior nodes, solved by Thomas.
 * Reading R6: E_j = (phi_{j-1} - phi_{j+1}) / (2 dx) inside (and everywhere when periodic);
 *   at a bounded wall Gauss's law over the half cell gives
 *   E_0 = (phi_0 - phi_1)/dx - sigma_0/eps0 and E_N = (phi_{N-1} - phi_N)/dx + sigma_N/eps0
 *   with sigma_j = rho_j V_j.
 * Reading R22 (bounded, floating): the walls keep the charge of the particles they absorb
 *   (the sheath cases of the paper's experimental setup deposit charge on the walls).  The
 *   system of plasma and walls is isolated, so no field exists left of the left wall, and
 *   the left wall is the potential reference.  Gauss's law over the left wall and the half
 *   cell in front of it gives E_{1/2} = (sigma_L + rho_0 V_0)/eps0, with sigma_L = the
 *   absorbed charge sum_s q_s w_s (particles of s absorbed there); each further cell adds
 *   rho_j dx / eps0 to the face field, and phi_{j+1} = phi_j - dx E_{j+1/2}.  The right
 *   wall's potential floats.  R6 gives the wall nodes' E as before.
 * Reading R23: the density smoothing that the paper's Background section lists in the
 *   cycle is applied to rho (after the deposit, before the background and the solve).     */
void orc_smooth_nodes(int64_t nn, int32_t periodic, int32_t passes, double *rho)
{
    double *t = (double *)malloc((size_t)nn * sizeof(double));
    for (int k = 0; k < passes; k++) {
        memcpy(t, rho, (size_t)nn * sizeof(double));
        for (int64_t j = 0; j < nn; j++) {
            double left, right;
            if (periodic) {
                left = t[j == 0 ? nn - 1 : j - 1];
                right = t[j == nn - 1 ? 0 : j + 1];
            } else {
                /* a wall node's missing neighbour is its mirror image across the wall */
                left = t[j == 0 ? 1 : j - 1];
                right = t[j == nn - 1 ? nn - 2 : j + 1];
            }
            rho[j] = 0.25 * left + 0.5 * t[j] + 0.25 * right;
        }
    }
    free(t);
}

void orc_solve(orc_state *st)
{
    const orc_config *c = &st->cfg;
    int64_t N = c->ncells, nn = st->nnodes;
    double dx = c->dx, L = dlen(st);
    for (int64_t j = 0; j < nn; j++) {
        double q = 0.0;
        for (int s = 0; s < c->nspecies; s++) q += c->sp[s].q * c->sp[s].w * st->Q[s][j];
        st->rho[j] = q / node_volume(st, j);
    }
    if (c->smooth > 0) orc_smooth_nodes(nn, c->periodic, c->smooth, st->rho);
    if (c->periodic) {
        double tot = 0.0;
        for (int64_t j = 0; j < nn; j++) tot += st->rho[j] * node_volume(st, j);
        double bg = -tot / L;
        for (int64_t j = 0; j < nn; j++) st->rho[j] += bg;
    }
    int64_t m = N - 1; /* interior unknowns phi_1 .. phi_{N-1} */
    st->phi[0] = 0.0;
    if (!c->periodic) st->phi[N] = 0.0;
    if (!c->periodic && c->floating) {
        double sigL = 0.0;
        for (int s = 0; s < c->nspecies; s++)
            sigL += c->sp[s].q * c->sp[s].w * (double)st->d.wall_count[0][s];
        double Eface = (sigL + st->rho[0] * node_volume(st, 0)) / c->eps0; /* E_{1/2} */
        for (int64_t j = 1; j <= N; j++) {
            st->phi[j] = st->phi[j - 1] - dx * Eface;
            if (j < N) Eface += st->rho[j] * dx / c->eps0;
        }
    } else if (m > 0) {
        double *a = (double *)malloc((size_t)m * sizeof(double));
        double *b = (double *)malloc((size_t)m * sizeof(double));
        double *cc = (double *)malloc((size_t)m * sizeof(double));
        double *d = (double *)malloc((size_t)m * sizeof(double));
        for (int64_t i = 0; i < m; i++) {
            a[i] = 1.0;
            b[i] = -2.0;
            cc[i] = 1.0;
            d[i] = -st->rho[i + 1] * dx * dx / c->eps0;
        }
        orc_thomas(m, a, b, cc, d, st->phi + 1);
        free(a);
        free(b);
        free(cc);
        free(d);
    }
    if (c->periodic) {
        double mean = 0.0;
        for (int64_t j = 0; j < N; j++) mean += st->phi[j];
        mean /= (double)N;
        for (int64_t j = 0; j < N; j++) st->phi[j] -= mean;
        for (int64_t j = 0; j < N; j++) {
            int64_t jm = (j == 0) ? N - 1 : j - 1;
            int64_t jp = (j == N - 1) ? 0 : j + 1;
            st->E[j] = (st->phi[jm] - st->phi[jp]) / (2.0 * dx);
        }
    } else {
        for (int64_t j = 1; j < N; j++) st->E[j] = (st->phi[j - 1] - st->phi[j + 1]) / (2.0 * dx);
        double sig0 = st->rho[0] * node_volume(st, 0);
        double sigN = st->rho[N] * node_volume(st, N);
        st->E[0] = (st->phi[0] - st->phi[1]) / dx - sig0 / c->eps0;
        st->E[N] = (st->phi[N - 1] - st->phi[N]) / dx + sigN / c->eps0;
    }
    double em = 0.0;
    for (int64_t j = 0; j < nn; j++)
        if (fabs(st->E[j]) > em) em = fabs(st->E[j]);
    st->Emax = em;
}

void orc_set_fields(orc_state *st, const double *E)
{
    double em = 0.0;
    for (int64_t j = 0; j < st->nnodes; j++) {
        st->E[j] = E[j];
        if (fabs(E[j]) > em) em = fabs(E[j]);
    }
    st->Emax = em;
}

/* ------------------------------------------------------------------------------------ */
/* Gather + Boris push (Boris 1970).  E_p = (1 - f) E_j + f E_{j+1} + E_ext along x;
 * half kick, rotation t = (q/m)(dt/2) B, s = 2 t / (1 + |t|^2), v' = v- + v- x t,
 * v+ = v- + v' x s, half kick, then x += dt v_x.                                          */
void orc_push(orc_state *st)
{
    const orc_config *c = &st->cfg;
    for (int s = 0; s < c->nspecies; s++) {
        double h = c->sp[s].q / c->sp[s].m * 0.5 * c->dt;
        double t[3] = {h * c->B[0], h * c->B[1], h * c->B[2]};
        double tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
        double sf = 2.0 / (1.0 + tt);
        double sv[3] = {sf * t[0], sf * t[1], sf * t[2]};
#pragma omp parallel for schedule(static)
        for (int64_t p = 0; p < st->n[s]; p++) {
            double f = 0.0;
            int64_t j = cell_index(st, st->x[s][p], &f);
            if (j < 0) {
                st->err = 2;
                continue;
            }
            int64_t j1 = j + 1;
            if (c->periodic && j1 == c->ncells) j1 = 0;
            double Ep = (1.0 - f) * st->E[j] + f * st->E[j1] + c->E_ext;
            double vm[3] = {st->vx[s][p] + h * Ep, st->vy[s][p], st->vz[s][p]};
            double vp_[3] = {vm[0] + (vm[1] * t[2] - vm[2] * t[1]),
                             vm[1] + (vm[2] * t[0] - vm[0] * t[2]),
                             vm[2] + (vm[0] * t[1] - vm[1] * t[0])};
            double vpl[3] = {vm[0] + (vp_[1] * sv[2] - vp_[2] * sv[1]),
                             vm[1] + (vp_[2] * sv[0] - vp_[0] * sv[2]),
                             vm[2] + (vp_[0] * sv[1] - vp_[1] * sv[0])};
            st->vx[s][p] = vpl[0] + h * Ep;
            st->vy[s][p] = vpl[1];
            st->vz[s][p] = vpl[2];
            st->x[s][p] += c->dt * st->vx[s][p];
        }
        st->d.pushes += st->n[s];
    }
    /* recycled neutrals carry no charge: they stream freely */
    for (int64_t p = 0; p < st->nneu; p++) st->nx[p] += c->dt * st->nvx[p];
}

/* Reading R24: an ion absorbed at a wall returns from that wall as a D neutral (the
 * sheath cases recycle D+ ions into D neutrals at the walls), with recycling coefficient
 * one.  The neutral keeps the ion's id and draws Philox block 0 of key (seed, 2) with the
 * step tag: u1 gives the inward normal speed from the flux-weighted half-Maxwellian at the
 * neutral temperature T_n, v_w sqrt(-2 ln u1) with v_w = sqrt(T_n / m_n); (u2, u3) give
 * the two tangential components (Box-Muller, times v_w); it leaves the wall during the
 * step, so it starts u4 dt |v_x| inside the wall it came from.                            */
static void emit_neutral(orc_state *st, uint32_t ion_id, int wall)
{
    const orc_config *c = &st->cfg;
    if (st->nneu >= st->ncap) {
        st->err = 3;
        return;
    }
    uint32_t w[4];
    draw_block(st, 2, ion_id, (uint32_t)st->step, 0u, w);
    double vw = sqrt(c->T_n / c->m_n);
    double vn = vw * sqrt(-2.0 * log(orc_uniform(w[0])));
    double vy, vz;
    orc_boxmuller(orc_uniform(w[1]), orc_uniform(w[2]), &vy, &vz);
    double depth = orc_uniform(w[3]) * c->dt * vn;
    int64_t k = st->nneu++;
    st->nx[k] = wall == 0 ? depth : dlen(st) - depth;
    st->nvx[k] = wall == 0 ? vn : -vn;
    st->nvy[k] = vw * vy;
    st->nvz[k] = vw * vz;
    st->nid[k] = ion_id;
    st->d.recycled += 1;
}

/* Reading R8: bounded walls absorb every particle with x < 0 or x >= L (count, charge and
 * kinetic energy tallied per wall); survivors keep their order.  Periodic: wrap into
 * [0, L).  Neutrals leave through either wall (counted); then the ions absorbed in this
 * call return as neutrals (R24).                                                           */
void orc_walls(orc_state *st)
{
    const orc_config *c = &st->cfg;
    double L = dlen(st);
    uint32_t *rec_id = NULL;
    int *rec_wall = NULL;
    int64_t nrec = 0, reccap = 0;
    for (int s = 0; s < c->nspecies; s++) {
        const orc_species *sp = &c->sp[s];
        if (c->periodic) {
            for (int64_t p = 0; p < st->n[s]; p++) {
                double x = st->x[s][p];
                while (x < 0.0) x += L;
                while (x >= L) x -= L;
                st->x[s][p] = x;
            }
            continue;
        }
        int64_t k = 0;
        for (int64_t p = 0; p < st->n[s]; p++) {
            double x = st->x[s][p];
            if (x < 0.0 || x >= L) {
                int wall = x < 0.0 ? 0 : 1;
                double v2 = speed2(st->vx[s][p], st->vy[s][p], st->vz[s][p]);
                st->d.wall_count[wall][s] += 1;
                st->d.wall_charge[wall][s] += sp->q * sp->w;
                st->d.wall_ke[wall][s] += 0.5 * sp->m * sp->w * v2;
                if (c->recycle && s == 1) {
                    if (nrec == reccap) {
                        reccap = reccap ? 2 * reccap : 1024;
                        rec_id = (uint32_t *)realloc(rec_id, (size_t)reccap * sizeof(uint32_t));
                        rec_wall = (int *)realloc(rec_wall, (size_t)reccap * sizeof(int));
                    }
                    rec_id[nrec] = st->id[s][p];
                    rec_wall[nrec] = wall;
                    nrec++;
                }
                continue;
            }
            st->x[s][k] = x;
            st->vx[s][k] = st->vx[s][p];
            st->vy[s][k] = st->vy[s][p];
            st->vz[s][k] = st->vz[s][p];
            st->id[s][k] = st->id[s][p];
            k++;
        }
        st->n[s] = k;
    }
    int64_t k = 0;
    for (int64_t p = 0; p < st->nneu; p++) {
        double x = st->nx[p];
        if (x < 0.0 || x >= L) {
            st->d.neutral_wall[x < 0.0 ? 0 : 1] += 1;
            continue;
        }
        st->nx[k] = x;
        st->nvx[k] = st->nvx[p];
        st->nvy[k] = st->nvy[p];
        st->nvz[k] = st->nvz[p];
        st->nid[k] = st->nid[p];
        k++;
    }
    st->nneu = k;
    for (int64_t r = 0; r < nrec; r++) emit_neutral(st, rec_id[r], rec_wall[r]);
    free(rec_id);
    free(rec_wall);
}

/* ------------------------------------------------------------------------------------ */
/* Null-collision Monte Carlo (Vahedi & Surendra 1995) against a uniform neutral
 * background with constant n_g sigma per channel (reading R9), rates nu_k = n_g sigma_k |v|
 * in the lab frame (R10).
 * Reading R11: the bound nu_max,s = n_g sigma_T,s (vmax_s + |q_s/m_s| dt (Emax + |E_ext|))
 *   times a 2^-16 inflation, where vmax_s is the largest speed present at the start of the
 *   step; a push changes a speed by at most |q/m| dt |E_p|, so the bound holds for every
 *   pushed particle.  P_null = 1 - exp(-nu_max dt).
 * Reading R12: each particle draws Philox block 0 (tag = step n) -> (R1..R4); it is a
 *   candidate iff R1 < P_null; the channel is the first k with R2 nu_max < sum_{i<=k} nu_i,
 *   channel order (elastic, ionisation) for electrons and (CX) for ions.
 * Reading R13: kinematics with isotropic lab-frame directions (see iso_dir); elastic keeps
 *   |v'|^2 = |v|^2 (1 - (2 m_e / m_n)(1 - cos theta)); ionisation shares the energy above
 *   threshold by a uniform fraction (block 1 word 0) between the scattered electron
 *   (direction R3, R4) and the new electron (direction block 1 words 1-2); the new ion and a
 *   charge-exchanged ion take neutral velocities, three normals of block 2 at T_n.
 * Reading R14: created particles are ordered by parent id and numbered next_id, next_id+1,
 *   ... in that order, then appended after the survivors of each species.
 * Reading R25: the volumetric source of the non-uniform sheath case creates src_pairs
 *   electron-ion pairs per step, spread uniformly over [0, src_frac L) by stratified
 *   sampling: pair k of step n lies in the k-th of src_pairs equal sub-intervals, at the
 *   fraction u of it given by word 0 of Philox block 4 of key (seed, 0) with counter (k, n); the
 *   electron three normals of block 5 of key (seed, 0) at T_e and the ion three normals of
 *   block 5 of key (seed, 1) at T_i.  Both members sit at the same x.  A step's source
 *   pairs take the ids (and slots) before its ionisation births: next_id + k for pair k,
 *   the births follow from next_id + src_pairs.  Like births they are pushed from the next
 *   step on.                                                                              */
typedef struct {
    uint32_t pid;
    double x;
    double ve[3];
    double vi[3];
} orc_birth;

static int birth_cmp(const void *a, const void *b)
{
    uint32_t pa = ((const orc_birth *)a)->pid, pb = ((const orc_birth *)b)->pid;
    return (pa > pb) - (pa < pb);
}

void orc_collide(orc_state *st)
{
    const orc_config *c = &st->cfg;
    uint32_t tag = (uint32_t)st->step;
    orc_birth *births = NULL;
    int64_t nb = 0, nbcap = 0;
    for (int s = 0; s < c->nspecies; s++) {
        const orc_species *sp = &c->sp[s];
        double ngsT = (s == 0) ? c->ngs_el + c->ngs_iz : c->ngs_cx;
        double qm = fabs(sp->q / sp->m);
        double Vb = st->vmax[s] + qm * c->dt * (st->Emax + fabs(c->E_ext));
        if (s == 1 && c->cx_relative) Vb += ORC_VN_BOUND * sqrt(c->T_n / c->m_n);
        double numax = ngsT * Vb * ORC_NU_SAFETY;
        double pnull = 1.0 - exp(-numax * c->dt);
        st->numax[s] = numax;
        st->pnull[s] = pnull;
        st->last_n[s] = st->n[s];
        double vn = sqrt(c->T_n / c->m_n);
        int64_t ncoll[3] = {0, 0, 0};
#pragma omp parallel for schedule(static) reduction(+ : ncoll[:3])
        for (int64_t p = 0; p < st->n[s]; p++) {
            uint32_t pid = st->id[s][p];
            st->last_id[s][p] = pid;
            st->last_chan[s][p] = -1;
            if (!c->collisions || ngsT <= 0.0) continue;
            uint32_t w[4];
            draw_block(st, s, pid, tag, 0u, w);
            double R1 = orc_uniform(w[0]), R2 = orc_uniform(w[1]);
            double R3 = orc_uniform(w[2]), R4 = orc_uniform(w[3]);
            if (!(R1 < pnull)) continue;
            double vx = st->vx[s][p], vy = st->vy[s][p], vz = st->vz[s][p];
            double v2 = speed2(vx, vy, vz);
            double spd = sqrt(v2);
            double thr = R2 * numax;
            int chan = -1;
            if (s == 0) {
                double nu_el = c->ngs_el * spd;
                double nu_iz = (0.5 * sp->m * v2 >= c->eps_iz) ? c->ngs_iz * spd : 0.0;
                if (thr < nu_el)
                    chan = 0;
                else if (thr < nu_el + nu_iz)
                    chan = 1;
            } else if (c->cx_relative) {
                /* R26: the target neutral is drawn first (block 2) and the rate uses the
                 * relative speed; a charge exchange hands the ion that neutral's velocity */
                uint32_t w2[4];
                double z[3];
                draw_block(st, s, pid, tag, 2u, w2);
                three_normals(w2, z);
                double gx = vx - vn * z[0], gy = vy - vn * z[1], gz = vz - vn * z[2];
                double g = sqrt(gx * gx + gy * gy + gz * gz);
                if (thr < c->ngs_cx * g) chan = 2;
            } else {
                if (thr < c->ngs_cx * spd) chan = 2;
            }
            st->last_chan[s][p] = chan;
            if (chan < 0) continue;
            ncoll[chan] += 1;
            if (chan == 0) {
                double d[3];
                iso_dir(R3, R4, d);
                double cth = (vx * d[0] + vy * d[1] + vz * d[2]) / spd;
                double f2 = 1.0 - (2.0 * sp->m / c->m_n) * (1.0 - cth);
                double sp2 = sqrt(v2 * f2);
                st->vx[s][p] = sp2 * d[0];
                st->vy[s][p] = sp2 * d[1];
                st->vz[s][p] = sp2 * d[2];
            } else if (chan == 1) {
                uint32_t w1[4], w2[4];
                draw_block(st, s, pid, tag, 1u, w1);
                draw_block(st, s, pid, tag, 2u, w2);
                double erem = 0.5 * sp->m * v2 - c->eps_iz;
                double u = orc_uniform(w1[0]);
                double e1 = u * erem, e2 = (1.0 - u) * erem;
                double d1[3], d2[3], z[3];
                iso_dir(R3, R4, d1);
                iso_dir(orc_uniform(w1[1]), orc_uniform(w1[2]), d2);
                double s1 = sqrt(2.0 * e1 / sp->m), s2 = sqrt(2.0 * e2 / sp->m);
                st->vx[s][p] = s1 * d1[0];
                st->vy[s][p] = s1 * d1[1];
                st->vz[s][p] = s1 * d1[2];
                three_normals(w2, z);
                /* births are ordered by parent id below, so the order of appending here
                 * does not matter */
#pragma omp critical(orc_births)
                {
                    if (nb == nbcap) {
                        nbcap = nbcap ? 2 * nbcap : 1024;
                        births = (orc_birth *)realloc(births, (size_t)nbcap * sizeof(orc_birth));
                    }
                    orc_birth *b = &births[nb++];
                    b->pid = pid;
                    b->x = st->x[s][p];
                    b->ve[0] = s2 * d2[0];
                    b->ve[1] = s2 * d2[1];
                    b->ve[2] = s2 * d2[2];
                    b->vi[0] = vn * z[0];
                    b->vi[1] = vn * z[1];
                    b->vi[2] = vn * z[2];
                }
            } else {
                uint32_t w2[4];
                double z[3];
                draw_block(st, s, pid, tag, 2u, w2);
                three_normals(w2, z);
                st->vx[s][p] = vn * z[0];
                st->vy[s][p] = vn * z[1];
                st->vz[s][p] = vn * z[2];
            }
        }
        for (int k = 0; k < 3; k++) st->d.coll[k] += ncoll[k];
    }
    for (int64_t k = 0; k < c->src_pairs && c->nspecies > 1; k++) {
        uint32_t w[4], z0w[4], z1w[4];
        double z[3];
        draw_block(st, 0, (uint32_t)k, tag, 4u, w);
        double x = c->src_frac * dlen(st) * (((double)k + orc_uniform(w[0])) / (double)c->src_pairs);
        draw_block(st, 0, (uint32_t)k, tag, 5u, z0w);
        draw_block(st, 1, (uint32_t)k, tag, 5u, z1w);
        for (int s = 0; s < 2; s++) {
            int64_t j = st->n[s];
            if (j >= st->cap[s]) {
                st->err = 3;
                continue;
            }
            double vt = sqrt(c->sp[s].T / c->sp[s].m);
            three_normals(s == 0 ? z0w : z1w, z);
            st->x[s][j] = x;
            st->vx[s][j] = vt * z[0];
            st->vy[s][j] = vt * z[1];
            st->vz[s][j] = vt * z[2];
            st->id[s][j] = st->next_id[s]++;
            st->n[s] = j + 1;
        }
        st->d.sourced += 1;
    }
    if (nb > 0) {
        qsort(births, (size_t)nb, sizeof(orc_birth), birth_cmp);
        int ns = c->nspecies;
        for (int64_t r = 0; r < nb; r++) {
            for (int s = 0; s < ns && s < 2; s++) {
                int64_t k = st->n[s];
                if (k >= st->cap[s]) {
                    st->err = 3;
                    continue;
                }
                const double *v = (s == 0) ? births[r].ve : births[r].vi;
                st->x[s][k] = births[r].x;
                st->vx[s][k] = v[0];
                st->vy[s][k] = v[1];
                st->vz[s][k] = v[2];
                st->id[s][k] = st->next_id[s]++;
                st->n[s] = k + 1;
                st->d.created[s] += 1;
            }
        }
    }
    free(births);
    for (int s = 0; s < c->nspecies; s++) recompute_vmax(st, s);
}

/* ------------------------------------------------------------------------------------ */
/* Stable counting sort of each species by cell index floor(x / dx) (folded into the last
 * cell when it rounds up to N): histogram, exclusive scan, scatter in input order.                                                           */
void orc_sort(orc_state *st)
{
    const orc_config *c = &st->cfg;
    int64_t N = c->ncells;
    int64_t *start = (int64_t *)malloc((size_t)(N + 1) * sizeof(int64_t));
    for (int s = 0; s < c->nspecies; s++) {
        int64_t n = st->n[s];
        int64_t *cellof = (int64_t *)malloc((size_t)(n + 1) * sizeof(int64_t));
        memset(start, 0, (size_t)(N + 1) * sizeof(int64_t));
        for (int64_t p = 0; p < n; p++) {
            double f = 0.0;
            cellof[p] = cell_index(st, st->x[s][p], &f);
            if (cellof[p] < 0) {  /* not a valid state: keep the particle, first cell */
                st->err = 2;
                cellof[p] = 0;
            }
            start[cellof[p] + 1] += 1;
        }
        for (int64_t j = 0; j < N; j++) start[j + 1] += start[j];
        double *nx = (double *)malloc((size_t)(n + 1) * sizeof(double));
        double *nvx = (double *)malloc((size_t)(n + 1) * sizeof(double));
        double *nvy = (double *)malloc((size_t)(n + 1) * sizeof(double));
        double *nvz = (double *)malloc((size_t)(n + 1) * sizeof(double));
        uint32_t *nid = (uint32_t *)malloc((size_t)(n + 1) * sizeof(uint32_t));
        for (int64_t p = 0; p < n; p++) {
            int64_t k = start[cellof[p]]++;
            nx[k] = st->x[s][p];
            nvx[k] = st->vx[s][p];
            nvy[k] = st->vy[s][p];
            nvz[k] = st->vz[s][p];
            nid[k] = st->id[s][p];
        }
        memcpy(st->x[s], nx, (size_t)n * sizeof(double));
        memcpy(st->vx[s], nvx, (size_t)n * sizeof(double));
        memcpy(st->vy[s], nvy, (size_t)n * sizeof(double));
        memcpy(st->vz[s], nvz, (size_t)n * sizeof(double));
        memcpy(st->id[s], nid, (size_t)n * sizeof(uint32_t));
        free(nx);
        free(nvx);
        free(nvy);
        free(nvz);
        free(nid);
        free(cellof);
    }
    free(start);
}

/* ------------------------------------------------------------------------------------ */
void orc_step(orc_state *st, int64_t nsteps)
{
    const orc_config *c = &st->cfg;
    for (int64_t it = 0; it < nsteps; it++) {
        orc_solve(st);
        orc_push(st);
        orc_walls(st);
        if (c->collisions || c->src_pairs > 0) orc_collide(st);
        else
            for (int s = 0; s < c->nspecies; s++) recompute_vmax(st, s);
        orc_deposit(st);
        st->step += 1;
        if (c->sort_every > 0 && st->step % c->sort_every == 0) orc_sort(st);
    }
}

/* ------------------------------------------------------------------------------------ */
void orc_get_grid(const orc_state *st, double *Q0, double *Q1, double *rho, double *phi,
                  double *E)
{
    size_t nb = (size_t)st->nnodes * sizeof(double);
    if (Q0) memcpy(Q0, st->Q[0], nb);
    if (Q1 && st->cfg.nspecies > 1) memcpy(Q1, st->Q[1], nb);
    if (rho) memcpy(rho, st->rho, nb);
    if (phi) memcpy(phi, st->phi, nb);
    if (E) memcpy(E, st->E, nb);
}

/* Diagnostics: FP64 sums over the current state plus the cumulative tallies.  Field
 * energy is 1/2 eps0 sum_j E_j^2 V_j of the self-consistent field (no external part).   */
void orc_get_diag(orc_state *st, orc_diag *out)
{
    const orc_config *c = &st->cfg;
    orc_diag d = st->d;
    d.charge = 0.0;
    for (int s = 0; s < 2; s++) {
        d.count[s] = 0;
        d.ke[s] = 0.0;
    }
    for (int s = 0; s < c->nspecies; s++) {
        const orc_species *sp = &c->sp[s];
        double sum = 0.0;
        for (int64_t p = 0; p < st->n[s]; p++)
            sum += speed2(st->vx[s][p], st->vy[s][p], st->vz[s][p]);
        d.count[s] = st->n[s];
        d.ke[s] = 0.5 * sp->m * sp->w * sum;
        d.charge += sp->q * sp->w * (double)st->n[s];
    }
    double fe = 0.0;
    for (int64_t j = 0; j < st->nnodes; j++) fe += st->E[j] * st->E[j] * node_volume(st, j);
    d.field_energy = 0.5 * c->eps0 * fe;
    d.step = st->step;
    d.neutral_count = st->nneu;
    *out = d;
}

/* Node moments of species s (reading R27): with the cloud-in-cell shares S_j(x_p) of the
 * deposit, W_j = sum_p S_j, the number density n_j = w_s W_j / V_j, the mean velocity
 * u_j = sum_p S_j v_p / W_j (three components) and the temperature
 * T_j = (m_s / 3) (sum_p S_j |v_p|^2 / W_j - |u_j|^2); u_j = T_j = 0 where W_j = 0.
 * Output arrays of length nnodes: n, ux, uy, uz, T (any may be NULL).                     */
void orc_moments(const orc_state *st, int s, double *n, double *ux, double *uy, double *uz,
                 double *T)
{
    const orc_config *c = &st->cfg;
    int64_t nn = st->nnodes;
    double *W = (double *)calloc((size_t)nn + 1, sizeof(double));
    double *Wv[3];
    for (int k = 0; k < 3; k++) Wv[k] = (double *)calloc((size_t)nn + 1, sizeof(double));
    double *Wv2 = (double *)calloc((size_t)nn + 1, sizeof(double));
    if (s >= 0 && s < c->nspecies) {
        for (int64_t p = 0; p < st->n[s]; p++) {
            double f = 0.0;
            int64_t j = cell_index(st, st->x[s][p], &f);
            if (j < 0) continue;
            int64_t j1 = j + 1;
            if (c->periodic && j1 == c->ncells) j1 = 0;
            double v[3] = {st->vx[s][p], st->vy[s][p], st->vz[s][p]};
            double v2 = speed2(v[0], v[1], v[2]);
            double sh[2] = {1.0 - f, f};
            int64_t nd[2] = {j, j1};
            for (int a = 0; a < 2; a++) {
                W[nd[a]] += sh[a];
                for (int k = 0; k < 3; k++) Wv[k][nd[a]] += sh[a] * v[k];
                Wv2[nd[a]] += sh[a] * v2;
            }
        }
    }
    double w = (s >= 0 && s < c->nspecies) ? c->sp[s].w : 0.0;
    double m = (s >= 0 && s < c->nspecies) ? c->sp[s].m : 0.0;
    for (int64_t j = 0; j < nn; j++) {
        double u[3] = {0.0, 0.0, 0.0}, t = 0.0;
        if (W[j] > 0.0) {
            for (int k = 0; k < 3; k++) u[k] = Wv[k][j] / W[j];
            t = (m / 3.0) * (Wv2[j] / W[j] - speed2(u[0], u[1], u[2]));
        }
        if (n) n[j] = w * W[j] / node_volume(st, j);
        if (ux) ux[j] = u[0];
        if (uy) uy[j] = u[1];
        if (uz) uz[j] = u[2];
        if (T) T[j] = t;
    }
    free(W);
    for (int k = 0; k < 3; k++) free(Wv[k]);
    free(Wv2);
}

int64_t orc_last_channels(const orc_state *st, int s, int32_t *chan, uint32_t *ids)
{
    int64_t n = st->last_n[s];
    if (chan) memcpy(chan, st->last_chan[s], (size_t)n * sizeof(int32_t));
    if (ids) memcpy(ids, st->last_id[s], (size_t)n * sizeof(uint32_t));
    return n;
}

void orc_last_numax(const orc_state *st, double *numax, double *pnull)
{
    for (int s = 0; s < 2; s++) {
        if (numax) numax[s] = st->numax[s];
        if (pnull) pnull[s] = st->pnull[s];
    }
}
