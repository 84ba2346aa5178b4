/*
 * lsm_oracle.c -- plain FP64 CPU oracle of the lattice spring model (LSM).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only callers.  Nothing here is shared
 * with the GPU path (no headers, tables or helpers), and the product never
 * calls into this library.
 *
 * What it computes, in the paper's order and notation (arXiv 2201.04565):
 *   - image -> particles on a triangular (2D) or simple-cubic (3D) packing,
 *     one particle per non-void pixel/voxel, springs to nearest (2D) or
 *     face + edge-diagonal (3D) neighbours, typed by the phases of the two
 *     end particles (Introduction: Img2Particle; Section 2.3: particle masses
 *     and spring parameters are assigned by type; Table "Constants of linear
 *     fracture spring").
 *   - truncated harmonic potential U = sum 1/2 k (r - r0)^2 (1 - H(r - rc))
 *     (Eq. 1) and the pair force obtained from its gradient (Eq. 2).
 *   - irreversible critical-stretch breaking: a spring whose length exceeds
 *     rc is switched off for good and contributes no force in the step that
 *     detects it (Section 2.3 force routine; Section 4 keeps broken springs in
 *     the list with zero stiffness).
 *   - velocity Verlet (Eq. 3-5) in the half-step velocity form (Section 2.2),
 *     with an optional viscous damping force -gamma v evaluated with the
 *     half-step velocity (damping is not in the paper; gamma = 0 recovers
 *     Eq. 3-5 exactly).
 *   - displacement-controlled uniaxial loading of boundary particles along x
 *     (Section 3.1), applied as strain increments followed by relaxation.
 *   - virial stress (Eq. 7), kinetic and potential energy (Section 2.3).
 *
 * Readings where the paper is silent (shared with the GPU path as
 * definitions, never as code): breaking uses the strict test r > rc; spring
 * ids follow the canonical enumeration below; grips are the first and last
 * image columns, clamped in all components; interface springs without an
 * explicit value use the series rule k_ab = 2 k_a k_b / (k_a + k_b) and
 * s_ab = min(s_a k_a, s_b k_b) / k_ab.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EUNSTABLE (-4)

typedef struct {
    int32_t inc;
    int32_t step;
    int64_t id;
    double margin;
} orc_event;

typedef struct {
    double eps;
    double sigma[9];
    double ke;
    double pe;
    int64_t n_broken;
    int32_t inc;
    int32_t step;
    int32_t status;
    int32_t pad;
} orc_record;

typedef struct orc_net {
    int dim;
    int64_t n, m;
    /* particles (Section 2.3: flattened position/velocity/acceleration vectors) */
    double *X0, *x, *v, *a, *F, *mass, *c;
    uint8_t *grip; /* 0 free, 1 left grip, 2 right grip */
    /* springs (Eq. 1: the set M of unique pairs) */
    int64_t *sp, *sq;
    double *k, *r0, *rc;
    uint8_t *broken;
    double omega; /* reference volume of Eq. 7 */
    /* spring law (0 linear, 1 recoverable in compression, 2 cubic) and the
       cubic coefficient */
    int law;
    double law_c;
    /* dynamics */
    double dt, gamma;
    int predictor; /* 0 affine, 1 grips only */
    double eps;
    /* constant strain-rate loading: grips at eps0 + s (rate dt) at the s-th
       step since the rate was set or the last increment */
    double rate, rate_eps0;
    int64_t rate_steps;
    int32_t inc, step;
    orc_event *ev;
    int64_t nev, evcap;
} orc_net;

/* ------------------------------------------------------------------ memory */

static void net_free(orc_net *N)
{
    if (!N) return;
    free(N->X0); free(N->x); free(N->v); free(N->a); free(N->F);
    free(N->mass); free(N->c); free(N->grip);
    free(N->sp); free(N->sq); free(N->k); free(N->r0); free(N->rc);
    free(N->broken); free(N->ev);
    free(N);
}

static orc_net *net_alloc(int dim, int64_t n, int64_t m)
{
    orc_net *N = (orc_net *)calloc(1, sizeof(orc_net));
    if (!N) return NULL;
    N->dim = dim;
    N->n = n;
    N->m = m;
    size_t nd = (size_t)(n > 0 ? n : 1) * (size_t)dim;
    size_t nn = (size_t)(n > 0 ? n : 1);
    size_t mm = (size_t)(m > 0 ? m : 1);
    N->X0 = (double *)calloc(nd, sizeof(double));
    N->x = (double *)calloc(nd, sizeof(double));
    N->v = (double *)calloc(nd, sizeof(double));
    N->a = (double *)calloc(nd, sizeof(double));
    N->F = (double *)calloc(nd, sizeof(double));
    N->mass = (double *)calloc(nn, sizeof(double));
    N->c = (double *)calloc(nn, sizeof(double));
    N->grip = (uint8_t *)calloc(nn, 1);
    N->sp = (int64_t *)calloc(mm, sizeof(int64_t));
    N->sq = (int64_t *)calloc(mm, sizeof(int64_t));
    N->k = (double *)calloc(mm, sizeof(double));
    N->r0 = (double *)calloc(mm, sizeof(double));
    N->rc = (double *)calloc(mm, sizeof(double));
    N->broken = (uint8_t *)calloc(mm, 1);
    N->evcap = 1024;
    N->ev = (orc_event *)malloc((size_t)N->evcap * sizeof(orc_event));
    if (!N->X0 || !N->x || !N->v || !N->a || !N->F || !N->mass || !N->c || !N->grip ||
        !N->sp || !N->sq || !N->k || !N->r0 || !N->rc || !N->broken || !N->ev) {
        net_free(N);
        return NULL;
    }
    N->dt = 0.01;
    N->gamma = 0.0;
    N->omega = 1.0;
    return N;
}

static int log_event(orc_net *N, int64_t id, double margin)
{
    if (N->nev == N->evcap) {
        int64_t cap = N->evcap * 2;
        orc_event *e = (orc_event *)realloc(N->ev, (size_t)cap * sizeof(orc_event));
        if (!e) return ORC_ENOMEM;
        N->ev = e;
        N->evcap = cap;
    }
    N->ev[N->nev].inc = N->inc;
    N->ev[N->nev].step = N->step;
    N->ev[N->nev].id = id;
    N->ev[N->nev].margin = margin;
    N->nev++;
    return ORC_OK;
}

/* -------------------------------------------------------- explicit network */

/* A network given particle by particle and spring by spring.  Used for the
 * two-particle oscillator of Section 3.1 and other hand-made cases. */
orc_net *orc_network(int dim, int64_t n, const double *X0, const double *mass,
                     const double *c, const uint8_t *grip, int64_t m,
                     const int64_t *sp, const int64_t *sq, const double *k,
                     const double *r0, const double *rc, double omega)
{
    if ((dim != 2 && dim != 3) || n < 0 || m < 0) return NULL;
    for (int64_t s = 0; s < m; ++s)
        if (sp[s] < 0 || sp[s] >= n || sq[s] < 0 || sq[s] >= n || sp[s] == sq[s]) return NULL;
    orc_net *N = net_alloc(dim, n, m);
    if (!N) return NULL;
    memcpy(N->X0, X0, (size_t)n * dim * sizeof(double));
    memcpy(N->x, X0, (size_t)n * dim * sizeof(double));
    memcpy(N->mass, mass, (size_t)n * sizeof(double));
    memcpy(N->c, c, (size_t)n * sizeof(double));
    memcpy(N->grip, grip, (size_t)n);
    memcpy(N->sp, sp, (size_t)m * sizeof(int64_t));
    memcpy(N->sq, sq, (size_t)m * sizeof(int64_t));
    memcpy(N->k, k, (size_t)m * sizeof(double));
    memcpy(N->r0, r0, (size_t)m * sizeof(double));
    memcpy(N->rc, rc, (size_t)m * sizeof(double));
    N->omega = omega;
    return N;
}

/* ----------------------------------------------------- image -> lattice */

/* Spring constant and critical stretch of a pair of phases.  An explicit
 * table entry wins; a non-finite entry falls back to two half-springs in
 * series, which break when the weaker half reaches its own stretch limit. */
static void pair_params(int P, const double *kpp, const double *spp, int pa, int pb,
                        double *k_out, double *s_out)
{
    int lo = pa < pb ? pa : pb, hi = pa < pb ? pb : pa;
    double k = kpp[lo * P + hi];
    double s = spp[lo * P + hi];
    double ka = kpp[lo * P + lo], kb = kpp[hi * P + hi];
    double sa = spp[lo * P + lo], sb = spp[hi * P + hi];
    if (!isfinite(k)) k = (ka + kb) > 0.0 ? 2.0 * ka * kb / (ka + kb) : 0.0;
    if (!isfinite(s)) {
        double la = sa * ka, lb = sb * kb;
        s = k > 0.0 ? (la < lb ? la : lb) / k : 0.0;
    }
    *k_out = k;
    *s_out = s;
}

/* Forward neighbour offsets in canonical order.  2D: east, then the two
 * sites of the next row (left one first); which grid columns those are
 * depends on the row parity because odd rows are shifted by half a spacing.
 * 3D: the 3 face and 6 edge directions with a positive leading component. */
static const int fwd2_even[3][2] = {{1, 0}, {-1, 1}, {0, 1}};
static const int fwd2_odd[3][2] = {{1, 0}, {0, 1}, {1, 1}};
static const int fwd3[9][3] = {{1, 0, 0},  {0, 1, 0},  {0, 0, 1},
                               {1, 1, 0},  {-1, 1, 0}, {1, 0, 1},
                               {-1, 0, 1}, {0, 1, 1},  {0, -1, 1}};

static void site_position(int kind, int64_t i, int64_t j, int64_t kk, double a, double *X)
{
    if (kind == 0) {
        X[0] = ((double)i + 0.5 * (double)(j % 2)) * a;
        X[1] = (double)j * (sqrt(3.0) / 2.0) * a;
    } else {
        X[0] = (double)i * a;
        X[1] = (double)j * a;
        X[2] = (double)kk * a;
    }
}

/* Builds the particle-spring network of a phase image.
 * kind 0: 2D triangular packing, image (ny, nx); kind 1: 3D simple cubic,
 * image (nz, ny, nx).  Pixel value = phase index, void_value (if >= 0) marks
 * empty sites.  Particles are numbered in raster order (x fastest) over the
 * non-void sites; springs are numbered by owner particle, then by forward
 * direction in canonical order. */
orc_net *orc_lattice(int kind, const uint8_t *img, int64_t nx, int64_t ny, int64_t nz,
                     double a, int P, const double *kpp, const double *spp,
                     double k_face, double k_diag, const double *mass_of_phase,
                     int void_value)
{
    if ((kind != 0 && kind != 1) || nx <= 0 || ny <= 0 || nz <= 0 || P <= 0 || P > 16) return NULL;
    if (kind == 0 && nz != 1) return NULL;
    int dim = kind == 0 ? 2 : 3;
    int64_t ns = nx * ny * nz;
    int64_t *id = (int64_t *)malloc((size_t)ns * sizeof(int64_t));
    if (!id) return NULL;
    int64_t n = 0;
    for (int64_t g = 0; g < ns; ++g) {
        int v = img[g];
        if (void_value >= 0 && v == void_value) {
            id[g] = -1;
        } else {
            if (v >= P) { free(id); return NULL; }
            id[g] = n++;
        }
    }
    /* pass 1: count springs; pass 2: fill */
    int64_t m = 0;
    orc_net *N = NULL;
    for (int pass = 0; pass < 2; ++pass) {
        int64_t s = 0;
        for (int64_t kk = 0; kk < nz; ++kk)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    int64_t g = i + nx * (j + ny * kk);
                    int64_t p = id[g];
                    if (p < 0) continue;
                    int nf = kind == 0 ? 3 : 9;
                    for (int d = 0; d < nf; ++d) {
                        int64_t qi, qj, qk;
                        int geom_face = 1;
                        if (kind == 0) {
                            const int *o = (j % 2 == 0) ? fwd2_even[d] : fwd2_odd[d];
                            qi = i + o[0]; qj = j + o[1]; qk = kk;
                        } else {
                            qi = i + fwd3[d][0]; qj = j + fwd3[d][1]; qk = kk + fwd3[d][2];
                            geom_face = d < 3;
                        }
                        if (qi < 0 || qi >= nx || qj < 0 || qj >= ny || qk < 0 || qk >= nz) continue;
                        int64_t gq = qi + nx * (qj + ny * qk);
                        int64_t q = id[gq];
                        if (q < 0) continue;
                        if (pass == 1) {
                            double Xp[3], Xq[3], r2 = 0.0;
                            site_position(kind, i, j, kk, a, Xp);
                            site_position(kind, qi, qj, qk, a, Xq);
                            for (int e = 0; e < dim; ++e) r2 += (Xq[e] - Xp[e]) * (Xq[e] - Xp[e]);
                            double kab, sab;
                            pair_params(P, kpp, spp, img[g], img[gq], &kab, &sab);
                            if (kind == 1) kab *= geom_face ? k_face : k_diag;
                            N->sp[s] = p;
                            N->sq[s] = q;
                            N->k[s] = kab;
                            N->r0[s] = sqrt(r2);
                            N->rc[s] = N->r0[s] * (1.0 + sab);
                        }
                        s++;
                    }
                }
        if (pass == 0) {
            m = s;
            N = net_alloc(dim, n, m);
            if (!N) { free(id); return NULL; }
        }
    }
    /* particles */
    for (int64_t kk = 0; kk < nz; ++kk)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t g = i + nx * (j + ny * kk);
                int64_t p = id[g];
                if (p < 0) continue;
                site_position(kind, i, j, kk, a, &N->X0[p * dim]);
                for (int e = 0; e < dim; ++e) N->x[p * dim + e] = N->X0[p * dim + e];
                N->mass[p] = mass_of_phase[img[g]];
                N->c[p] = (double)i * a;
                N->grip[p] = (i == 0) ? 1 : (i == nx - 1 ? 2 : 0);
            }
    N->omega = (double)n * (kind == 0 ? (sqrt(3.0) / 2.0) * a * a : a * a * a);
    free(id);
    return N;
}

/* ------------------------------------------------------------- dynamics */

/* Spring laws.  The linear truncated spring of Eq. 1-2 is law 0.  The
 * paper's closing section names extensions of it; two are built:
 *   law 1, recoverable stiffness: a broken spring still resists compression,
 *     with its intact stiffness, while shorter than its rest length
 *     (U = k (r - r0)^2 / 2 for r < r0, nothing otherwise);
 *   law 2, cubic (non-linear) elasticity: U = k d^2 / 2 + k c d^4 / (4 r0^2)
 *     with d = r - r0, so the force magnitude is k d (1 + c d^2 / r0^2).
 * The break rule (an intact spring longer than rc breaks) is the same for
 * all laws. */
static int spring_acts(const orc_net *N, int64_t s, double r)
{
    if (!N->broken[s]) return 1;
    return N->law == 1 && r < N->r0[s];
}

static double spring_coef(const orc_net *N, int64_t s, double r)
{
    double dl = r - N->r0[s];
    if (N->law == 2) return N->k[s] * dl * (1.0 + N->law_c * dl * dl / (N->r0[s] * N->r0[s])) / r;
    return N->k[s] * dl / r;
}

static double spring_energy(const orc_net *N, int64_t s, double r)
{
    double dl = r - N->r0[s];
    double u = 0.5 * N->k[s] * dl * dl;
    if (N->law == 2) u += 0.25 * N->k[s] * N->law_c * dl * dl * dl * dl / (N->r0[s] * N->r0[s]);
    return u;
}

/* Eq. 2 with the break rule: loops the spring list in id order, skipping
 * broken springs (unless the law lets them act).  An intact spring longer
 * than rc is (if commit) marked broken and logged, and gives no force in
 * this evaluation either way. */
static int forces(orc_net *N, double *F, int commit)
{
    const int dim = N->dim;
    memset(F, 0, (size_t)N->n * dim * sizeof(double));
    for (int64_t s = 0; s < N->m; ++s) {
        if (N->broken[s] && N->law != 1) continue;
        int64_t p = N->sp[s], q = N->sq[s];
        double d[3] = {0.0, 0.0, 0.0};
        double r2 = 0.0;
        for (int e = 0; e < dim; ++e) {
            d[e] = N->x[q * dim + e] - N->x[p * dim + e];
            r2 += d[e] * d[e];
        }
        double r = sqrt(r2);
        if (!N->broken[s] && r > N->rc[s]) {
            if (commit) {
                N->broken[s] = 1;
                if (log_event(N, s, (r - N->rc[s]) / N->rc[s]) != ORC_OK) return ORC_ENOMEM;
            }
            continue;
        }
        if (!spring_acts(N, s, r)) continue;
        /* force on p from q is +coef d with d = x_q - x_p (Eq. 2 for law 0) */
        double coef = spring_coef(N, s, r);
        for (int e = 0; e < dim; ++e) {
            F[p * dim + e] += coef * d[e];
            F[q * dim + e] -= coef * d[e];
        }
    }
    return ORC_OK;
}

/* a = (F - gamma v) / m for free particles; grips carry no acceleration. */
static void accelerations(orc_net *N)
{
    const int dim = N->dim;
    for (int64_t p = 0; p < N->n; ++p) {
        for (int e = 0; e < dim; ++e) {
            if (N->grip[p])
                N->a[p * dim + e] = 0.0;
            else
                N->a[p * dim + e] = (N->F[p * dim + e] - N->gamma * N->v[p * dim + e]) / N->mass[p];
        }
    }
}

/* Spring law of the network (see spring_acts); 0 linear by default. */
int orc_set_spring_law(orc_net *N, int law, double c)
{
    if (law < 0 || law > 2 || !isfinite(c)) return ORC_EINVAL;
    N->law = law;
    N->law_c = c;
    return ORC_OK;
}

void orc_set_dynamics(orc_net *N, double dt, double gamma, int predictor)
{
    N->dt = dt;
    N->gamma = gamma;
    N->predictor = predictor;
}

/* One displacement-controlled increment (Section 3.1 boundary displacement,
 * recast as a strain increment).  Grips are placed at X0_x + eps * c and
 * clamped; free particles optionally receive the affine predictor
 * d_eps * c along x.  Then step 0: forces with the break test and the
 * accelerations from the current full-step velocity. */
int orc_apply_increment(orc_net *N, double d_eps)
{
    const int dim = N->dim;
    N->inc += 1;
    N->step = 0;
    N->eps += d_eps;
    N->rate_eps0 = N->eps;
    N->rate_steps = 0;
    for (int64_t p = 0; p < N->n; ++p) {
        if (N->grip[p]) {
            N->x[p * dim + 0] = N->X0[p * dim + 0] + N->eps * N->c[p];
            for (int e = 1; e < dim; ++e) N->x[p * dim + e] = N->X0[p * dim + e];
            for (int e = 0; e < dim; ++e) N->v[p * dim + e] = 0.0;
        } else if (N->predictor == 0) {
            N->x[p * dim + 0] += d_eps * N->c[p];
        }
    }
    int rc = forces(N, N->F, 1);
    if (rc != ORC_OK) return rc;
    accelerations(N);
    return ORC_OK;
}

/* Constant strain-rate loading, the paper's protocol (Section 3.1: the
 * boundary particles move apart along x at a fixed strain rate; Section 2.3:
 * the boundary displacement is the first operation of every time step).
 * rate is per unit time.  From the next step on, the s-th step since this
 * call (or since the last increment) first places the grips at
 * X0_x + (eps0 + s (rate dt)) c, eps0 being the strain at that point; rate
 * 0 stops them.  Free particles are only moved by the integrator. */
void orc_set_strain_rate(orc_net *N, double rate)
{
    N->rate = rate;
    N->rate_eps0 = N->eps;
    N->rate_steps = 0;
}

/* grips to the strain of the next step of the constant-rate protocol */
static void move_grips(orc_net *N)
{
    const int dim = N->dim;
    N->rate_steps += 1;
    N->eps = N->rate_eps0 + (double)N->rate_steps * (N->rate * N->dt);
    for (int64_t p = 0; p < N->n; ++p) {
        if (!N->grip[p]) continue;
        N->x[p * dim + 0] = N->X0[p * dim + 0] + N->eps * N->c[p];
        for (int e = 1; e < dim; ++e) N->x[p * dim + e] = N->X0[p * dim + e];
    }
}

/* nsteps of velocity Verlet in the half-step form (Eq. 3-5, Section 2.2):
 * (grips moved first under constant-rate loading) v += dt/2 a; x += dt v;
 * F(x) with the break test; a = (F - gamma v)/m; v += dt/2 a.  Grips are
 * not integrated. */
int orc_relax(orc_net *N, int64_t nsteps)
{
    const int dim = N->dim;
    const double h = 0.5 * N->dt;
    for (int64_t it = 0; it < nsteps; ++it) {
        N->step += 1;
        if (N->rate != 0.0) move_grips(N);
        for (int64_t p = 0; p < N->n; ++p) {
            if (N->grip[p]) continue;
            for (int e = 0; e < dim; ++e) {
                N->v[p * dim + e] += h * N->a[p * dim + e];
                N->x[p * dim + e] += N->dt * N->v[p * dim + e];
            }
        }
        int rc = forces(N, N->F, 1);
        if (rc != ORC_OK) return rc;
        accelerations(N);
        for (int64_t p = 0; p < N->n; ++p) {
            if (N->grip[p]) continue;
            for (int e = 0; e < dim; ++e) N->v[p * dim + e] += h * N->a[p * dim + e];
        }
    }
    return ORC_OK;
}

/* Virial stress (Eq. 7) over the whole specimen with f^{kl} the force on k
 * from l: each intact spring contributes d_a f_b once (the two ordered pairs
 * of the double sum carry 1/2 each), the kinetic term m v_a v_b is
 * subtracted, and the sum is divided by the reference volume.  Tension is
 * positive.  Also the kinetic energy, Eq. 1 potential energy and the number
 * of broken springs. */
int orc_record_state(orc_net *N, orc_record *R)
{
    const int dim = N->dim;
    double S[9] = {0}, K[9] = {0};
    double pe = 0.0, ke = 0.0;
    int64_t nb = 0;
    for (int64_t s = 0; s < N->m; ++s) {
        if (N->broken[s]) {
            nb++;
            if (N->law != 1) continue;
        }
        int64_t p = N->sp[s], q = N->sq[s];
        double d[3] = {0.0, 0.0, 0.0}, r2 = 0.0;
        for (int e = 0; e < dim; ++e) {
            d[e] = N->x[q * dim + e] - N->x[p * dim + e];
            r2 += d[e] * d[e];
        }
        double r = sqrt(r2);
        if (!N->broken[s] && r > N->rc[s]) continue; /* Heaviside factor of Eq. 1 */
        if (!spring_acts(N, s, r)) continue;
        double coef = spring_coef(N, s, r);
        for (int aa = 0; aa < dim; ++aa)
            for (int bb = 0; bb < dim; ++bb) S[aa * 3 + bb] += d[aa] * (coef * d[bb]);
        pe += spring_energy(N, s, r);
    }
    for (int64_t p = 0; p < N->n; ++p) {
        for (int aa = 0; aa < dim; ++aa) {
            for (int bb = 0; bb < dim; ++bb)
                K[aa * 3 + bb] += N->mass[p] * N->v[p * dim + aa] * N->v[p * dim + bb];
            ke += 0.5 * N->mass[p] * N->v[p * dim + aa] * N->v[p * dim + aa];
        }
    }
    memset(R, 0, sizeof(*R));
    R->eps = N->eps;
    int finite = isfinite(ke) && isfinite(pe);
    for (int i = 0; i < 9; ++i) {
        R->sigma[i] = (S[i] - K[i]) / N->omega;
        finite = finite && isfinite(R->sigma[i]);
    }
    R->ke = ke;
    R->pe = pe;
    R->n_broken = nb;
    R->inc = N->inc;
    R->step = N->step;
    R->status = finite ? ORC_OK : ORC_EUNSTABLE;
    return R->status;
}

/* Full protocol: n_inc increments of d_eps, each relaxed for steps_per_inc
 * steps, one record per increment.  Stops early (returning ORC_EUNSTABLE)
 * when a record is not finite. */
int orc_run(orc_net *N, int32_t n_inc, int64_t steps_per_inc, double d_eps, orc_record *out)
{
    for (int32_t it = 0; it < n_inc; ++it) {
        int rc = orc_apply_increment(N, d_eps);
        if (rc != ORC_OK) return rc;
        rc = orc_relax(N, steps_per_inc);
        if (rc != ORC_OK) return rc;
        rc = orc_record_state(N, &out[it]);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------ accessors */

void orc_free(orc_net *N) { net_free(N); }

void orc_counts(const orc_net *N, int64_t *n, int64_t *m, int32_t *dim)
{
    *n = N->n;
    *m = N->m;
    *dim = N->dim;
}

double orc_omega(const orc_net *N) { return N->omega; }

void orc_get_x(const orc_net *N, double *out) { memcpy(out, N->x, (size_t)N->n * N->dim * sizeof(double)); }
void orc_set_x(orc_net *N, const double *in) { memcpy(N->x, in, (size_t)N->n * N->dim * sizeof(double)); }
void orc_get_v(const orc_net *N, double *out) { memcpy(out, N->v, (size_t)N->n * N->dim * sizeof(double)); }
void orc_set_v(orc_net *N, const double *in) { memcpy(N->v, in, (size_t)N->n * N->dim * sizeof(double)); }
void orc_get_a(const orc_net *N, double *out) { memcpy(out, N->a, (size_t)N->n * N->dim * sizeof(double)); }
void orc_get_X0(const orc_net *N, double *out) { memcpy(out, N->X0, (size_t)N->n * N->dim * sizeof(double)); }

void orc_get_particles(const orc_net *N, double *mass, double *c, uint8_t *grip)
{
    memcpy(mass, N->mass, (size_t)N->n * sizeof(double));
    memcpy(c, N->c, (size_t)N->n * sizeof(double));
    memcpy(grip, N->grip, (size_t)N->n);
}

void orc_get_springs(const orc_net *N, int64_t *sp, int64_t *sq, double *k, double *r0,
                     double *rc, uint8_t *broken)
{
    memcpy(sp, N->sp, (size_t)N->m * sizeof(int64_t));
    memcpy(sq, N->sq, (size_t)N->m * sizeof(int64_t));
    memcpy(k, N->k, (size_t)N->m * sizeof(double));
    memcpy(r0, N->r0, (size_t)N->m * sizeof(double));
    memcpy(rc, N->rc, (size_t)N->m * sizeof(double));
    memcpy(broken, N->broken, (size_t)N->m);
}

void orc_set_broken(orc_net *N, const uint8_t *broken) { memcpy(N->broken, broken, (size_t)N->m); }

/* Forces at the current positions (Eq. 2); commit != 0 applies the break
 * rule to the state and logs events at the current (increment, step). */
int orc_forces(orc_net *N, double *F, int commit) { return forces(N, F, commit); }

/* Eq. 1 at the current positions, skipping broken springs. */
double orc_potential_energy(const orc_net *N)
{
    const int dim = N->dim;
    double pe = 0.0;
    for (int64_t s = 0; s < N->m; ++s) {
        if (N->broken[s] && N->law != 1) continue;
        int64_t p = N->sp[s], q = N->sq[s];
        double r2 = 0.0;
        for (int e = 0; e < dim; ++e) {
            double d = N->x[q * dim + e] - N->x[p * dim + e];
            r2 += d * d;
        }
        double r = sqrt(r2);
        if (!N->broken[s] && r > N->rc[s]) continue;
        if (!spring_acts(N, s, r)) continue;
        pe += spring_energy(N, s, r);
    }
    return pe;
}

int64_t orc_n_events(const orc_net *N) { return N->nev; }

void orc_get_events(const orc_net *N, int32_t *inc, int32_t *step, int64_t *id, double *margin)
{
    for (int64_t e = 0; e < N->nev; ++e) {
        inc[e] = N->ev[e].inc;
        step[e] = N->ev[e].step;
        id[e] = N->ev[e].id;
        margin[e] = N->ev[e].margin;
    }
}

void orc_get_clock(const orc_net *N, int32_t *inc, int32_t *step, double *eps)
{
    *inc = N->inc;
    *step = N->step;
    *eps = N->eps;
}

/* ------------------------------------------------ run to failure (derived) */

/* Uniaxial test to failure: increments of d_eps, each relaxed for steps
 * steps, until the first increment after the stress peak whose sigma_xx
 * falls below drop * peak, a non-finite state, or max_inc increments.
 * Returns per-increment sigma_xx and broken counts, the number of
 * increments run, the strength (peak sigma_xx) and the modulus: the least
 * squares slope through the origin of sigma_xx against strain over the
 * increments that ended with no broken spring (at least the first one). */
int orc_run_to_failure(orc_net *N, double d_eps, int64_t steps, int32_t max_inc, double drop,
                       double *sxx, double *eps_out, int64_t *nbroken, int32_t *n_inc,
                       double *modulus, double *strength)
{
    double peak = -INFINITY;
    int32_t peak_inc = 0, n = 0;
    int status = ORC_OK;
    orc_record R;
    for (int32_t it = 1; it <= max_inc; ++it) {
        int rc = orc_apply_increment(N, d_eps);
        if (rc == ORC_OK) rc = orc_relax(N, steps);
        if (rc != ORC_OK) return rc;
        status = orc_record_state(N, &R);
        sxx[it - 1] = R.sigma[0];
        eps_out[it - 1] = R.eps;
        nbroken[it - 1] = R.n_broken;
        n = it;
        if (status != ORC_OK) break;
        if (R.sigma[0] > peak) {
            peak = R.sigma[0];
            peak_inc = it;
        }
        if (it > peak_inc && R.sigma[0] < drop * peak) break;
    }
    *n_inc = n;
    *strength = peak;
    int32_t k = 0;
    while (k < n && nbroken[k] == 0) ++k;
    if (k == 0) k = 1;
    double num = 0.0, den = 0.0;
    for (int32_t i = 0; i < k && i < n; ++i) {
        num += eps_out[i] * sxx[i];
        den += eps_out[i] * eps_out[i];
    }
    *modulus = den > 0.0 ? num / den : 0.0;
    return status;
}
