/*
 * FP64 CPU ORACLE of the magneto-elastic MLS-MPM time step and of its discrete
 * adjoint.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product (the HIP library and its
 * Python binding) links, loads or calls this file; it exists so that tests, the
 * smoke check and the CPU baseline of the benchmark have an independent,
 * obviously-correct reference. It shares no code, header or constant table with
 * the GPU path.
 *
 * What it computes (paper section 2, "Differentiable dynamic simulation"):
 *   - constitutive model: neo-Hookean energy (Eq. 4) plus ideal hard-magnetic
 *     potential (Eq. 5); first Piola-Kirchhoff stress (Eq. 7); SIMP-style
 *     interpolation of both energies by the projected density (Eq. 31) and a
 *     mass linear in the density (Eq. 33);
 *   - one MLS-MPM step: P2G mass and momentum transfer with quadratic B-spline
 *     weights (Eqs. 14-15), grid velocity with damping and gravity (Eqs. 16-17),
 *     separating Coulomb contact, no-slip and attached boundaries (Eq. 18 and the
 *     text after it), G2P velocity, affine matrix, position and deformation
 *     gradient update (Eqs. 19-22);
 *   - the losses of Sec. 4 (Eqs. 36-40) and the exact reverse-mode derivative of
 *     the discrete rollout (Sec. 2.3: gradients obtained by running the chain
 *     rule backwards through every step), here derived by hand.
 *
 * Readings of the text that is silent or garbled (all listed in the design notes):
 *   - Eq. 15 omits the time step and Eqs. 15/20/22 disagree in sign; the standard
 *     MLS-MPM form is used: dpos = x_i - x_p, affine term m C dpos, stress term
 *     -(4 dt / dx^2) V P F^T dpos, C = (4/dx^2) sum w v_i dpos^T, F <- (I + dt C) F.
 *   - 2D is plane strain: F is embedded in 3x3 with F33 = 1, so I1 = tr(F^T F) + 1.
 *   - G = E / (2 (1 + nu)), K = E / (3 (1 - 2 nu)).
 *   - Eq. 17's damping acts on the transferred velocity p/m with rate c.
 *   - Floor contact is node based: nodes with y_i <= y_floor apply Eq. 18 when
 *     the node moves into the floor (normal +y, static floor). |v_t| = 0 gives 0.
 *     Domain walls (b cells) zero the component pointing out of the domain.
 *     Attached (clamped) nodes x_i <= clamp_xmax get v = 0 (applied last).
 *   - Obstacles (the solid boundaries of Eq. 18 beyond the floor): analytic
 *     shapes (half-space, sphere, axis-aligned box) translating with a constant
 *     velocity v_b, at position a + v_b t_n during step n. A node lies on the
 *     boundary when the shape's signed distance at the node is <= 0; the normal
 *     is the distance's gradient. Such a node whose velocity relative to v_b
 *     points into the shape applies Eq. 18 relative to v_b (no-slip: v = v_b);
 *     an attached obstacle sets v = v_b whatever the velocity. Obstacles act
 *     after the floor, in order, before walls and clamp.
 *   - Piecewise-constant field: segment k(n) = n / L (periodic: mod S, else
 *     clamped to S-1), B evaluated at the start of the step.
 *
 * Arithmetic: IEEE double, no fast-math. Particle and node loops run on the
 * host's cores with OpenMP; a scatter to the grid adds into one private grid
 * per thread, and the private grids are summed node by node in thread order
 * (see "host parallelism" below). Built without OpenMP the loops run serially
 * in particle order. Particle data is stored with three components and 3x3
 * matrices in 2D too (z parts zero, F33 = 1).
 */
#include <limits.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
    ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 2,
    ORC_EDOMAIN = 4, ORC_EINVERT = 5, ORC_ENONFINITE = 6
};
enum { ORC_LOSS_FINAL_MSE = 0, ORC_LOSS_COM_DISP = 1, ORC_LOSS_TRAJ_VEL = 2, ORC_LOSS_TIP_DISP = 3 };

enum { ORC_MAX_OBST = 4 };
enum { ORC_OBST_NONE = 0, ORC_OBST_HALFSPACE = 1, ORC_OBST_SPHERE = 2, ORC_OBST_BOX = 3 };

typedef struct {
    int kind, attached;
    double a[3];     /* half-space: a point of its plane; sphere, box: centre at t = 0 */
    double b[3];     /* half-space: outward normal; sphere: b[0] radius; box: half extents */
    double mu;       /* friction; INFINITY: no-slip */
    double vel[3];   /* v_b */
} orc_obstacle;

typedef struct {
    int dim, n_grid;
    double dt;
    int n_steps;
    double E, nu, rho, mu0, simp_eps, simp_q, damping;
    double gravity[3];
    int wall_cells;
    double clamp_xmax;
    int floor_on;
    double floor_y, floor_mu;
    double particle_volume;
    int n_segments, seg_steps, periodic;
    int loss_kind;
    double loss_dir[3];
    int n_obstacles;
    orc_obstacle obst[ORC_MAX_OBST];
    double mass_eps;   /* floor of the mass interpolation: m = (eps + (1 - eps) phi) rho V; 0 gives Eq. 33 */
} orc_params;

typedef struct {
    double x[3], v[3], C[9], F[9];
} orc_particle;

/* ------------------------------------------------------------------------- */
/* 3x3 helpers (row-major)                                                   */
/* ------------------------------------------------------------------------- */

static double det3(const double A[9])
{
    return A[0] * (A[4] * A[8] - A[5] * A[7])
         - A[1] * (A[3] * A[8] - A[5] * A[6])
         + A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* inverse transpose A^{-T} via the cofactor matrix: A^{-T} = cof(A) / det(A) */
static void inv_transpose3(const double A[9], double H[9])
{
    double d = det3(A);
    H[0] = (A[4] * A[8] - A[5] * A[7]) / d;
    H[1] = -(A[3] * A[8] - A[5] * A[6]) / d;
    H[2] = (A[3] * A[7] - A[4] * A[6]) / d;
    H[3] = -(A[1] * A[8] - A[2] * A[7]) / d;
    H[4] = (A[0] * A[8] - A[2] * A[6]) / d;
    H[5] = -(A[0] * A[7] - A[1] * A[6]) / d;
    H[6] = (A[1] * A[5] - A[2] * A[4]) / d;
    H[7] = -(A[0] * A[5] - A[2] * A[3]) / d;
    H[8] = (A[0] * A[4] - A[1] * A[3]) / d;
}

static void matmul3(const double A[9], const double B[9], double out[9])
{
    double t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = 0.0;
            for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(out, t, sizeof t);
}

static void transpose3(const double A[9], double T[9])
{
    double t[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) t[3 * i + j] = A[3 * j + i];
    memcpy(T, t, sizeof t);
}

static double ddot9(const double A[9], const double B[9])
{
    double s = 0.0;
    for (int k = 0; k < 9; ++k) s += A[k] * B[k];
    return s;
}

/* ------------------------------------------------------------------------- */
/* host parallelism                                                          */
/* ------------------------------------------------------------------------- */

static int max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* Threads of the oracle's parallel loops; n <= 0 restores the OpenMP default
 * (all host cores unless OMP_NUM_THREADS says otherwise). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    static int initial = 0;
    if (!initial) initial = omp_get_max_threads();
    omp_set_num_threads(n > 0 ? n : initial);
#else
    (void)n;
#endif
}

int orc_get_threads(void) { return max_threads(); }

/*
 * Private scatter grids. A particle loop that adds into grid nodes gives each
 * thread a contiguous block of particles (static schedule) and its own copy of
 * the grid, 4 values per node. The copies are then summed node by node in
 * thread order 0, 1, 2, ...: a run repeats exactly, and the result differs
 * from the serial particle-order sum only in the order of the additions. A
 * copy holds zeros outside the range of node indices [lo, hi] its thread
 * touched; the sum skips it there, and the range is cleared afterwards.
 */
typedef struct {
    int nt, G;
    double* buf;   /* [nt][G][4] */
    int* lo;       /* [nt] */
    int* hi;       /* [nt] */
} orc_scatter;

static int scatter_alloc(orc_scatter* ws, int G)
{
    ws->nt = max_threads();
    ws->G = G;
    ws->buf = calloc((size_t)ws->nt * (size_t)(G > 0 ? G : 1) * 4, sizeof(double));
    ws->lo = malloc(sizeof(int) * ws->nt);
    ws->hi = malloc(sizeof(int) * ws->nt);
    if (!ws->buf || !ws->lo || !ws->hi) {
        free(ws->buf); free(ws->lo); free(ws->hi);
        ws->buf = NULL; ws->lo = ws->hi = NULL;
        return ORC_ENOMEM;
    }
    return 0;
}

static void scatter_free(orc_scatter* ws)
{
    free(ws->buf); free(ws->lo); free(ws->hi);
    ws->buf = NULL; ws->lo = ws->hi = NULL;
}

/* no node touched yet */
static void scatter_begin(orc_scatter* ws)
{
    for (int t = 0; t < ws->nt; ++t) {
        ws->lo[t] = ws->G;
        ws->hi[t] = -1;
    }
}

static double* scatter_copy(const orc_scatter* ws, int t) { return ws->buf + (size_t)t * ws->G * 4; }

/* sum of the private copies at node g, in thread order */
static void scatter_node(const orc_scatter* ws, int g, double acc[4])
{
    acc[0] = acc[1] = acc[2] = acc[3] = 0.0;
    for (int t = 0; t < ws->nt; ++t) {
        if (g < ws->lo[t] || g > ws->hi[t]) continue;
        const double* c = scatter_copy(ws, t) + (size_t)g * 4;
        for (int k = 0; k < 4; ++k) acc[k] += c[k];
    }
}

/* zero what each thread touched, so every copy is zero again */
static void scatter_clear(orc_scatter* ws)
{
    for (int t = 0; t < ws->nt; ++t)
        if (ws->hi[t] >= ws->lo[t])
            memset(scatter_copy(ws, t) + (size_t)ws->lo[t] * 4, 0,
                   sizeof(double) * 4 * (size_t)(ws->hi[t] - ws->lo[t] + 1));
}

/* Error of a parallel particle loop. The serial loop stops at the first
 * particle whose stencil cannot be formed, and otherwise reports the first
 * particle whose new state is flagged; keys index * 8 + code keep that order
 * under a minimum. */
#define ERR_KEY(q, code) ((long long)(q) * 8 + (long long)(code))
#define ERR_NONE LLONG_MAX
static int err_code(long long first_in, long long first_out)
{
    if (first_in != ERR_NONE) return (int)(first_in % 8);
    if (first_out != ERR_NONE) return (int)(first_out % 8);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* constitutive model                                                        */
/* ------------------------------------------------------------------------- */

void orc_moduli(double E, double nu, double* G, double* K)
{
    *G = E / (2.0 * (1.0 + nu));
    *K = E / (3.0 * (1.0 - 2.0 * nu));
}

/* Eq. 4: W_e = G/2 (J^{-2/3} I1 - 3) + K/2 (J - 1)^2 */
double orc_energy_elastic(const double F[9], double G, double K)
{
    double J = det3(F);
    double I1 = ddot9(F, F);
    return 0.5 * G * (pow(J, -2.0 / 3.0) * I1 - 3.0) + 0.5 * K * (J - 1.0) * (J - 1.0);
}

/* elastic part of Eq. 7: P_e = G J^{-2/3} (F - I1/3 F^{-T}) + K J (J - 1) F^{-T} */
void orc_stress_elastic(const double F[9], double G, double K, double P[9])
{
    double H[9];
    double J = det3(F);
    double I1 = ddot9(F, F);
    inv_transpose3(F, H);
    double a = G * pow(J, -2.0 / 3.0);
    double b = K * J * (J - 1.0);
    for (int k = 0; k < 9; ++k) P[k] = a * (F[k] - I1 / 3.0 * H[k]) + b * H[k];
}

/*
 * Directional derivative dP_e = (d P_e / d F)[dF] of the elastic stress, from
 * dJ = J H:dF, dI1 = 2 F:dF, dH = -H dF^T H, d(J^{-2/3}) = -2/3 J^{-2/3} H:dF.
 * The tangent is the Hessian of W_e, hence symmetric: it is its own transpose.
 */
void orc_stress_elastic_dir(const double F[9], double G, double K, const double dF[9], double dP[9])
{
    double H[9], dFt[9], T[9];
    double J = det3(F);
    double I1 = ddot9(F, F);
    inv_transpose3(F, H);
    double a = G * pow(J, -2.0 / 3.0);
    double HdF = ddot9(H, dF);
    double FdF = ddot9(F, dF);
    transpose3(dF, dFt);
    matmul3(H, dFt, T);
    matmul3(T, H, T); /* T = H dF^T H */
    for (int k = 0; k < 9; ++k) {
        double dev = dF[k] - (2.0 / 3.0) * HdF * (F[k] - I1 / 3.0 * H[k])
                   - (2.0 / 3.0) * FdF * H[k] + (I1 / 3.0) * T[k];
        dP[k] = a * dev + K * ((2.0 * J - 1.0) * J * HdF * H[k] - J * (J - 1.0) * T[k]);
    }
}

/* magnetic part of Eq. 7: P_m = -(1/mu0) B_applied (x) Br_ref */
static void stress_magnetic(const double B[3], const double Br[3], double mu0, double P[9])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) P[3 * i + j] = -B[i] * Br[j] / mu0;
}

/* Eq. 31 scalings and their derivatives w.r.t. the density */
static double simp_e(const orc_params* P, double phi)
{
    return P->simp_eps + (1.0 - P->simp_eps) * pow(phi, P->simp_q);
}
static double simp_m(const orc_params* P, double phi) { return pow(phi, P->simp_q); }
static double simp_e_d(const orc_params* P, double phi)
{
    return (1.0 - P->simp_eps) * P->simp_q * pow(phi, P->simp_q - 1.0);
}
static double simp_m_d(const orc_params* P, double phi)
{
    return P->simp_q * pow(phi, P->simp_q - 1.0);
}

/* total stress of one particle: P = s_e P_e(F) + s_m P_m; also returns the parts */
static void particle_stress(const orc_params* P, const double F[9], double phi, const double Br[3],
                            const double B[3], double Ptot[9], double Pe[9], double Pm[9])
{
    double G, K;
    orc_moduli(P->E, P->nu, &G, &K);
    orc_stress_elastic(F, G, K, Pe);
    stress_magnetic(B, Br, P->mu0, Pm);
    double se = simp_e(P, phi), sm = simp_m(P, phi);
    for (int k = 0; k < 9; ++k) Ptot[k] = se * Pe[k] + sm * Pm[k];
}

/* ------------------------------------------------------------------------- */
/* quadratic B-spline stencil                                                */
/* ------------------------------------------------------------------------- */

typedef struct {
    int base[3];
    double f[3];        /* x / dx - base, in [1/2, 3/2) */
    double w[3][3];     /* w[axis][node] */
    double dw[3][3];    /* d w / d x (already divided by dx) */
} orc_stencil;

/* 1-D quadratic B-spline weights of nodes base, base+1, base+2 and their
 * derivatives with respect to the particle position (in units of f) */
void orc_bspline(double f, double w[3], double dwdf[3])
{
    w[0] = 0.5 * (1.5 - f) * (1.5 - f);
    w[1] = 0.75 - (f - 1.0) * (f - 1.0);
    w[2] = 0.5 * (f - 0.5) * (f - 0.5);
    dwdf[0] = -(1.5 - f);
    dwdf[1] = -2.0 * (f - 1.0);
    dwdf[2] = f - 0.5;
}

/* returns 0 or ORC_EDOMAIN / ORC_ENONFINITE when the 3^d stencil leaves the grid */
static int make_stencil(const orc_params* P, const double x[3], orc_stencil* S)
{
    double dx = 1.0 / P->n_grid;
    for (int k = 0; k < 3; ++k) {
        if (k >= P->dim) {
            S->base[k] = 0;
            S->f[k] = 0.0;
            S->w[k][0] = 1.0; S->w[k][1] = 0.0; S->w[k][2] = 0.0;
            S->dw[k][0] = S->dw[k][1] = S->dw[k][2] = 0.0;
            continue;
        }
        if (!isfinite(x[k])) return ORC_ENONFINITE;
        double xs = x[k] / dx;
        double b = floor(xs - 0.5);
        if (b < 0.0 || b > (double)(P->n_grid - 3)) return ORC_EDOMAIN;
        S->base[k] = (int)b;
        S->f[k] = xs - b;
        double dwdf[3];
        orc_bspline(S->f[k], S->w[k], dwdf);
        for (int a = 0; a < 3; ++a) S->dw[k][a] = dwdf[a] / dx;
    }
    return 0;
}

static int n_nodes(const orc_params* P)
{
    return P->dim == 2 ? P->n_grid * P->n_grid : P->n_grid * P->n_grid * P->n_grid;
}

/* one stencil node: flat grid index, weight, weight gradient, dpos = x_i - x_p */
typedef struct {
    int idx;
    double w, gw[3], dpos[3];
} orc_node;

static void stencil_node(const orc_params* P, const orc_stencil* S, int a0, int a1, int a2, orc_node* nd)
{
    double dx = 1.0 / P->n_grid;
    int a[3] = {a0, a1, a2};
    int n = P->n_grid;
    nd->idx = (S->base[0] + a0) + n * (S->base[1] + a1) + n * n * (S->base[2] + a2);
    nd->w = S->w[0][a0] * S->w[1][a1] * S->w[2][a2];
    nd->gw[0] = S->dw[0][a0] * S->w[1][a1] * S->w[2][a2];
    nd->gw[1] = S->w[0][a0] * S->dw[1][a1] * S->w[2][a2];
    nd->gw[2] = S->w[0][a0] * S->w[1][a1] * S->dw[2][a2];
    for (int k = 0; k < 3; ++k)
        nd->dpos[k] = (k < P->dim) ? ((double)a[k] - S->f[k]) * dx : 0.0;
}

#define FOR_STENCIL(P, a0, a1, a2) \
    for (int a2 = 0; a2 < ((P)->dim == 3 ? 3 : 1); ++a2) \
        for (int a1 = 0; a1 < 3; ++a1) \
            for (int a0 = 0; a0 < 3; ++a0)

/* field program: segment of step n */
int orc_segment(const orc_params* P, int n)
{
    int L = P->seg_steps > 0 ? P->seg_steps : (P->n_steps + P->n_segments - 1) / P->n_segments;
    int k = n / L;
    if (P->periodic) k %= P->n_segments;
    else if (k > P->n_segments - 1) k = P->n_segments - 1;
    return k;
}

static void field_at(const orc_params* P, const double* bprog, int n, double B[3])
{
    int k = orc_segment(P, n);
    for (int j = 0; j < 3; ++j) B[j] = j < P->dim ? bprog[k * P->dim + j] : 0.0;
}

/* Eq. 33, m = phi rho V, with a floor for void particles: m = (eps_m + (1 -
 * eps_m) phi) rho V, linear in phi like the stiffness interpolation of Eq. 31
 * (its eps); eps_m = 0 is Eq. 33 itself. */
static double particle_mass(const orc_params* P, double phi)
{
    return (P->mass_eps + (1.0 - P->mass_eps) * phi) * P->rho * P->particle_volume;
}
/* d m / d phi */
static double particle_mass_d(const orc_params* P) { return (1.0 - P->mass_eps) * P->rho * P->particle_volume; }

/* ------------------------------------------------------------------------- */
/* forward pieces                                                            */
/* ------------------------------------------------------------------------- */

/* Eqs. 14-15: grid mass m[G] and momentum p[G][3], through the private
 * scatter grids ws (copy slot 0: mass, slots 1-3: momentum) */
static int p2g_into(const orc_params* P, int N, const orc_particle* s, const double* phi, const double* br3,
                    const double B[3], double* m, double* p, orc_scatter* ws)
{
    int G = n_nodes(P);
    double dx = 1.0 / P->n_grid;
    double kappa = 4.0 * P->dt / (dx * dx);
    long long first_err = ERR_NONE;
    scatter_begin(ws);
#pragma omp parallel num_threads(ws->nt) reduction(min : first_err)
    {
        const int t = thread_id();
        double* mine = scatter_copy(ws, t);
        int lo = G, hi = -1;
#pragma omp for schedule(static)
        for (int q = 0; q < N; ++q) {
            orc_stencil S;
            int e = make_stencil(P, s[q].x, &S);
            if (e) {
                if (ERR_KEY(q, e) < first_err) first_err = ERR_KEY(q, e);
                continue;
            }
            double Pt[9], Pe[9], Pm[9], PFt[9], Ft[9], A[9];
            particle_stress(P, s[q].F, phi[q], br3 + 3 * q, B, Pt, Pe, Pm);
            transpose3(s[q].F, Ft);
            matmul3(Pt, Ft, PFt);
            double mp = particle_mass(P, phi[q]);
            double V = P->particle_volume;
            for (int k = 0; k < 9; ++k) A[k] = mp * s[q].C[k] - kappa * V * PFt[k];
            FOR_STENCIL(P, a0, a1, a2) {
                orc_node nd;
                stencil_node(P, &S, a0, a1, a2, &nd);
                double* c = mine + (size_t)nd.idx * 4;
                c[0] += nd.w * mp;
                for (int i = 0; i < 3; ++i) {
                    double Ad = 0.0;
                    for (int j = 0; j < 3; ++j) Ad += A[3 * i + j] * nd.dpos[j];
                    c[1 + i] += nd.w * (mp * s[q].v[i] + Ad);
                }
                if (nd.idx < lo) lo = nd.idx;
                if (nd.idx > hi) hi = nd.idx;
            }
        }
        ws->lo[t] = lo;
        ws->hi[t] = hi;
    }
#pragma omp parallel for schedule(static) num_threads(ws->nt)
    for (int g = 0; g < G; ++g) {
        double acc[4];
        scatter_node(ws, g, acc);
        m[g] = acc[0];
        for (int i = 0; i < 3; ++i) p[3 * g + i] = acc[1 + i];
    }
    scatter_clear(ws);
    return err_code(first_err, ERR_NONE);
}

int orc_p2g(const orc_params* P, int N, const orc_particle* s, const double* phi, const double* br3,
            const double B[3], double* m, double* p)
{
    orc_scatter ws;
    if (scatter_alloc(&ws, n_nodes(P))) return ORC_ENOMEM;
    int e = p2g_into(P, N, s, phi, br3, B, m, p, &ws);
    scatter_free(&ws);
    return e;
}

static void node_coords(const orc_params* P, int g, int ijk[3])
{
    int n = P->n_grid;
    ijk[0] = g % n;
    ijk[1] = (g / n) % n;
    ijk[2] = P->dim == 3 ? g / (n * n) : 0;
}

/* floor contact (Eq. 18) on one node velocity u; returns the branch taken:
 * 0 untouched, 1 set to zero (no-slip, |v_t| = 0 or friction exceeds slip), 2 sliding.
 * force >= 0 applies that branch instead of deciding it (branch replay); a
 * forced slide keeps the slide map v_t (1 - mu |v_n| / |v_t|), v_n -> 0. */
static int floor_contact(const orc_params* P, double u[3], int force)
{
    double vn = u[1];
    double vt[3] = {u[0], 0.0, u[2]};
    double t = sqrt(vt[0] * vt[0] + vt[2] * vt[2]);
    double s = t - P->floor_mu * (-vn);
    int br = force;
    if (br < 0) {
        if (!(vn < 0.0)) br = 0;
        else if (isinf(P->floor_mu) || t == 0.0 || s <= 0.0) br = 1;
        else br = 2;
    }
    if (br == 1 || (br == 2 && (isinf(P->floor_mu) || t == 0.0))) {
        u[0] = u[1] = u[2] = 0.0;
    } else if (br == 2) {
        u[0] = s / t * vt[0];
        u[1] = 0.0;
        u[2] = s / t * vt[2];
    }
    return br;
}

/* Signed distance of obstacle O at node position x during step n, and its
 * outward normal; <= 0 on and inside the solid. */
static double obstacle_sdf(const orc_params* P, const orc_obstacle* O, int n, const double x[3], double nrm[3])
{
    double t = n * P->dt;
    double y[3];
    for (int k = 0; k < 3; ++k) y[k] = (k < P->dim) ? x[k] - (O->a[k] + O->vel[k] * t) : 0.0;
    nrm[0] = nrm[1] = nrm[2] = 0.0;
    if (O->kind == ORC_OBST_HALFSPACE) {
        double len = 0.0;
        for (int k = 0; k < P->dim; ++k) len += O->b[k] * O->b[k];
        len = sqrt(len);
        double d = 0.0;
        for (int k = 0; k < P->dim; ++k) {
            nrm[k] = O->b[k] / len;
            d += y[k] * nrm[k];
        }
        return d;
    }
    if (O->kind == ORC_OBST_SPHERE) {
        double r = 0.0;
        for (int k = 0; k < P->dim; ++k) r += y[k] * y[k];
        r = sqrt(r);
        if (r > 0.0)
            for (int k = 0; k < P->dim; ++k) nrm[k] = y[k] / r;
        else
            nrm[1] = 1.0;
        return r - O->b[0];
    }
    if (O->kind == ORC_OBST_BOX) {
        double best = -INFINITY;
        int kb = 0;
        for (int k = 0; k < P->dim; ++k) {
            double q = fabs(y[k]) - O->b[k];
            if (q > best) { best = q; kb = k; }
        }
        nrm[kb] = y[kb] < 0.0 ? -1.0 : 1.0;
        return best;   /* exact inside (<= 0), a lower bound outside */
    }
    return INFINITY;
}

/* contact of Eq. 18 against a boundary with velocity vb and outward normal
 * nrm on node velocity u (3 components) of a node on the boundary; returns 0
 * untouched, 1 set to vb, 2 sliding. force >= 0 applies that branch instead
 * of deciding it (branch replay). */
static int obstacle_contact(const orc_params* P, const orc_obstacle* O, const double nrm[3], double u[3], int force)
{
    double r[3], vn = 0.0;
    for (int k = 0; k < 3; ++k) {
        r[k] = (k < P->dim) ? u[k] - O->vel[k] : 0.0;
        vn += r[k] * nrm[k];
    }
    double tv[3], t = 0.0;
    for (int k = 0; k < 3; ++k) {
        tv[k] = r[k] - vn * nrm[k];
        t += tv[k] * tv[k];
    }
    t = sqrt(t);
    double sl = t + O->mu * vn;
    int br = force;
    if (br < 0) {
        if (O->attached) br = 1;
        else if (!(vn < 0.0)) br = 0;
        else if (isinf(O->mu) || t == 0.0 || sl <= 0.0) br = 1;
        else br = 2;
    }
    if (br == 1 || (br == 2 && (isinf(O->mu) || t == 0.0))) {
        for (int k = 0; k < 3; ++k) u[k] = (k < P->dim) ? O->vel[k] : 0.0;
    } else if (br == 2) {
        for (int k = 0; k < 3; ++k) u[k] = (k < P->dim) ? O->vel[k] + sl / t * tv[k] : 0.0;
    }
    return br;
}

/* ------------------------------------------------------------------------- */
/* branch decisions of the grid operation                                    */
/* ------------------------------------------------------------------------- */

/*
 * The grid operation decides, per node and step, whether the node has mass
 * (Eq. 16 applies only then), which branch of Eq. 18 the floor and each
 * obstacle take, and which velocity components the domain walls zero. These
 * integer decisions are taken from floating-point velocities, so a run in
 * another precision can decide a near-tie the other way; the adjoint then
 * follows the other branch (the Jacobian of the branch the forward took). For
 * comparing such a run's arithmetic with the oracle's, the decisions can be
 * replayed: with a replay table set, every node takes its decisions from the
 * table instead of deciding them, in the forward steps and in the transpose
 * alike. A record table receives the decisions taken. Tables hold one code per
 * step and node, [n_steps][n_nodes] (nodes x fastest), packed as
 *   bit 0      the node has mass
 *   bits 1-2   floor branch (0 untouched, 1 zero, 2 slide)
 *   bits 3-5   the walls zero the x, y, z component
 *   bits 6+2j  obstacle j's branch (0 untouched, 1 v_b, 2 slide)
 * Test instrumentation: the tables are process-wide, set with
 * orc_set_branch_trace and cleared with NULL.
 */
static const uint16_t* g_replay;
static uint16_t* g_record;
static int64_t g_trace_nodes;
static long long g_mass_mismatch;   /* replayed "has mass" where the oracle's mass is 0 */

void orc_set_branch_trace(const uint16_t* replay, uint16_t* record, int64_t n_nodes)
{
    g_replay = replay;
    g_record = record;
    g_trace_nodes = n_nodes;
    g_mass_mismatch = 0;
}

long long orc_branch_mass_mismatches(void) { return g_mass_mismatch; }

/* Eqs. 16-18 on one node in step n with every decision kept for the
 * transpose. Returns 0 (and v = 0) for a node without mass. */
typedef struct {
    double vh[3], u0[3];                  /* p/m; after damping and gravity (Eq. 17) */
    int floor_br;
    double ob_in[ORC_MAX_OBST][3], ob_n[ORC_MAX_OBST][3];
    int ob_br[ORC_MAX_OBST];
    int wall[3], clamped;
    double v[3];                          /* the node velocity */
} orc_node_bc;

static int node_bc(const orc_params* P, int g, int n, double m, const double p[3], orc_node_bc* s)
{
    memset(s, 0, sizeof *s);
    const int64_t slot = (int64_t)n * g_trace_nodes + g;
    const int code = g_replay ? (int)g_replay[slot] : -1;
    int has_mass = m > 0.0;
    if (code >= 0) {
        if ((code & 1) && !has_mass) {
#pragma omp atomic
            ++g_mass_mismatch;
        }
        has_mass = has_mass && (code & 1);
    }
    if (!has_mass) {
        if (g_record) g_record[slot] = 0;
        return 0;
    }
    int ijk[3];
    node_coords(P, g, ijk);
    double dx = 1.0 / P->n_grid;
    double c = P->damping;
    double u[3];
    for (int k = 0; k < 3; ++k) {
        s->vh[k] = p[k] / m;
        s->u0[k] = (k < P->dim) ? s->vh[k] + P->dt * (P->gravity[k] - c * s->vh[k]) : 0.0;
        u[k] = s->u0[k];
    }
    if (P->floor_on && ijk[1] * dx <= P->floor_y)
        s->floor_br = floor_contact(P, u, code >= 0 ? (code >> 1) & 3 : -1);
    double xi[3] = {ijk[0] * dx, ijk[1] * dx, ijk[2] * dx};
    for (int j = 0; j < P->n_obstacles; ++j) {
        for (int k = 0; k < 3; ++k) s->ob_in[j][k] = u[k];
        const int on = obstacle_sdf(P, &P->obst[j], n, xi, s->ob_n[j]) <= 0.0;
        const int force = code >= 0 ? (code >> (6 + 2 * j)) & 3 : (on ? -1 : 0);
        s->ob_br[j] = obstacle_contact(P, &P->obst[j], s->ob_n[j], u, force);
    }
    int b = P->wall_cells;
    for (int k = 0; k < P->dim; ++k) {
        s->wall[k] = code >= 0 ? (code >> (3 + k)) & 1
                               : ((ijk[k] < b && u[k] < 0.0) || (ijk[k] >= P->n_grid - b && u[k] > 0.0));
        if (s->wall[k]) u[k] = 0.0;
    }
    s->clamped = P->clamp_xmax >= 0.0 && ijk[0] * dx <= P->clamp_xmax;
    if (s->clamped) u[0] = u[1] = u[2] = 0.0;
    for (int k = 0; k < 3; ++k) s->v[k] = u[k];
    if (g_record) {
        int out = 1 | (s->floor_br << 1);
        for (int k = 0; k < 3; ++k) out |= s->wall[k] << (3 + k);
        for (int j = 0; j < P->n_obstacles; ++j) out |= s->ob_br[j] << (6 + 2 * j);
        g_record[slot] = (uint16_t)out;
    }
    return 1;
}

/* Eqs. 16-18 for one node during step n: returns v */
static void grid_node(const orc_params* P, int g, int n, double m, const double p[3], double v[3])
{
    orc_node_bc s;
    node_bc(P, g, n, m, p, &s);
    for (int k = 0; k < 3; ++k) v[k] = s.v[k];
}

void orc_grid(const orc_params* P, int n, const double* m, const double* p, double* v)
{
    int G = n_nodes(P);
#pragma omp parallel for schedule(static)
    for (int g = 0; g < G; ++g) grid_node(P, g, n, m[g], p + 3 * g, v + 3 * g);
}

/* Eqs. 19-22: new particle state from grid velocities v[G][3] */
int orc_g2p(const orc_params* P, int N, const orc_particle* s, const double* v, orc_particle* out)
{
    double dx = 1.0 / P->n_grid;
    double lam = 4.0 / (dx * dx);
    long long first_in = ERR_NONE, first_out = ERR_NONE;
#pragma omp parallel for schedule(static) reduction(min : first_in, first_out)
    for (int q = 0; q < N; ++q) {
        orc_stencil S;
        int e = make_stencil(P, s[q].x, &S);
        if (e) {
            if (ERR_KEY(q, e) < first_in) first_in = ERR_KEY(q, e);
            continue;
        }
        double vn[3] = {0, 0, 0}, Bm[9] = {0};
        FOR_STENCIL(P, a0, a1, a2) {
            orc_node nd;
            stencil_node(P, &S, a0, a1, a2, &nd);
            const double* vi = v + 3 * nd.idx;
            for (int i = 0; i < 3; ++i) {
                vn[i] += nd.w * vi[i];
                for (int j = 0; j < 3; ++j) Bm[3 * i + j] += nd.w * vi[i] * nd.dpos[j];
            }
        }
        orc_particle r;
        double IdC[9];
        for (int k = 0; k < 9; ++k) r.C[k] = lam * Bm[k];
        for (int i = 0; i < 3; ++i) {
            r.v[i] = vn[i];
            r.x[i] = s[q].x[i] + P->dt * vn[i];
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) IdC[3 * i + j] = (i == j ? 1.0 : 0.0) + P->dt * r.C[3 * i + j];
        matmul3(IdC, s[q].F, r.F);
        out[q] = r;
        /* error flags on the new state */
        int err = 0;
        for (int k = 0; k < 9 && !err; ++k)
            if (!isfinite(r.F[k]) || !isfinite(r.C[k])) err = ORC_ENONFINITE;
        for (int k = 0; k < 3 && !err; ++k)
            if (!isfinite(r.x[k]) || !isfinite(r.v[k])) err = ORC_ENONFINITE;
        if (!err && !(det3(r.F) > 0.0)) err = ORC_EINVERT;
        if (!err) {
            orc_stencil S2;
            int e2 = make_stencil(P, r.x, &S2);
            if (e2) err = e2;
        }
        if (err && ERR_KEY(q, err) < first_out) first_out = ERR_KEY(q, err);
    }
    return err_code(first_in, first_out);
}

/* one full step n: P2G, grid update, G2P. Work arrays m[G], p[3G], v[3G]. */
static int step_forward(const orc_params* P, int N, int n, const orc_particle* s, const double* phi,
                        const double* br3, const double B[3], double* m, double* p, double* v,
                        orc_particle* out, orc_scatter* ws)
{
    int e = p2g_into(P, N, s, phi, br3, B, m, p, ws);
    if (e) return e;
    orc_grid(P, n, m, p, v);
    return orc_g2p(P, N, s, v, out);
}

/* ------------------------------------------------------------------------- */
/* adjoint pieces                                                            */
/* ------------------------------------------------------------------------- */

/*
 * Transpose of G2P. Inputs: state n (x, F), grid velocities v, adjoints of the
 * new state (xb1, vb1, Cb1, Fb1). Outputs: the grid velocity adjoint vbar[G][3]
 * (overwritten) and the G2P share of the adjoint of state n: xb0, Fb0
 * (overwritten; the P2G transpose adds its share later).
 */
static int g2p_adj_into(const orc_params* P, int N, const orc_particle* s, const double* v,
                        const orc_particle* adj1, double* vbar, orc_particle* adj0, orc_scatter* ws)
{
    int G = n_nodes(P);
    double dx = 1.0 / P->n_grid;
    double lam = 4.0 / (dx * dx);
    double dt = P->dt;
    long long first_err = ERR_NONE;
    scatter_begin(ws);
#pragma omp parallel num_threads(ws->nt) reduction(min : first_err)
    {
        const int t = thread_id();
        double* mine = scatter_copy(ws, t);
        int lo = G, hi = -1;
#pragma omp for schedule(static)
        for (int q = 0; q < N; ++q) {
            orc_stencil S;
            int e = make_stencil(P, s[q].x, &S);
            if (e) {
                if (ERR_KEY(q, e) < first_err) first_err = ERR_KEY(q, e);
                continue;
            }
            /* recompute the new affine matrix C' */
            double Bm[9] = {0};
            FOR_STENCIL(P, a0, a1, a2) {
                orc_node nd;
                stencil_node(P, &S, a0, a1, a2, &nd);
                const double* vi = v + 3 * nd.idx;
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) Bm[3 * i + j] += nd.w * vi[i] * nd.dpos[j];
            }
            double Cn[9], IdC[9], IdCt[9], Ft[9], FbFt[9];
            for (int k = 0; k < 9; ++k) Cn[k] = lam * Bm[k];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) IdC[3 * i + j] = (i == j ? 1.0 : 0.0) + dt * Cn[3 * i + j];
            const orc_particle* a1p = &adj1[q];
            orc_particle* a0p = &adj0[q];
            /* F' = (I + dt C') F */
            transpose3(IdC, IdCt);
            matmul3(IdCt, a1p->F, a0p->F);
            transpose3(s[q].F, Ft);
            matmul3(a1p->F, Ft, FbFt);
            double Cbt[9], vbt[3];
            for (int k = 0; k < 9; ++k) Cbt[k] = a1p->C[k] + dt * FbFt[k];
            /* x' = x + dt v' */
            for (int i = 0; i < 3; ++i) {
                vbt[i] = a1p->v[i] + dt * a1p->x[i];
                a0p->x[i] = a1p->x[i];
                a0p->v[i] = 0.0;
            }
            for (int k = 0; k < 9; ++k) a0p->C[k] = 0.0;
            /* v' = sum w v_i ; C' = lam sum w v_i dpos^T */
            FOR_STENCIL(P, a0, a1, a2) {
                orc_node nd;
                stencil_node(P, &S, a0, a1, a2, &nd);
                const double* vi = v + 3 * nd.idx;
                double u[3];
                for (int i = 0; i < 3; ++i) {
                    double Cd = 0.0;
                    for (int j = 0; j < 3; ++j) Cd += Cbt[3 * i + j] * nd.dpos[j];
                    u[i] = vbt[i] + lam * Cd;
                    mine[(size_t)nd.idx * 4 + i] += nd.w * u[i];
                }
                if (nd.idx < lo) lo = nd.idx;
                if (nd.idx > hi) hi = nd.idx;
                double vu = vi[0] * u[0] + vi[1] * u[1] + vi[2] * u[2];
                for (int k = 0; k < 3; ++k) {
                    double CtV = 0.0;
                    for (int i = 0; i < 3; ++i) CtV += Cbt[3 * i + k] * vi[i];
                    a0p->x[k] += vu * nd.gw[k] - lam * nd.w * CtV;
                }
            }
            if (P->dim == 2) {
                a0p->x[2] = 0.0;
                for (int k = 0; k < 9; ++k)
                    if (k / 3 == 2 || k % 3 == 2) a0p->F[k] = 0.0;
            }
        }
        ws->lo[t] = lo;
        ws->hi[t] = hi;
    }
#pragma omp parallel for schedule(static) num_threads(ws->nt)
    for (int g = 0; g < G; ++g) {
        double acc[4];
        scatter_node(ws, g, acc);
        for (int i = 0; i < 3; ++i) vbar[3 * g + i] = acc[i];
    }
    scatter_clear(ws);
    return err_code(first_err, ERR_NONE);
}

int orc_g2p_adj(const orc_params* P, int N, const orc_particle* s, const double* v,
                const orc_particle* adj1, double* vbar, orc_particle* adj0)
{
    orc_scatter ws;
    if (scatter_alloc(&ws, n_nodes(P))) return ORC_ENOMEM;
    int e = g2p_adj_into(P, N, s, v, adj1, vbar, adj0, &ws);
    scatter_free(&ws);
    return e;
}

/* transpose of the floor slide map at input u (vn < 0, |v_t| > 0, slide branch) */
static void floor_slide_adj(const orc_params* P, const double u[3], double gbar[3])
{
    double mu = P->floor_mu;
    double vn = u[1];
    double vt[3] = {u[0], 0.0, u[2]};
    double t = sqrt(vt[0] * vt[0] + vt[2] * vt[2]);
    double Ptg[3] = {gbar[0], 0.0, gbar[2]};          /* tangential projection of gbar */
    double vtg = vt[0] * gbar[0] + vt[2] * gbar[2];   /* v_t . gbar */
    double out[3];
    for (int k = 0; k < 3; ++k) {
        double nk = (k == 1) ? 1.0 : 0.0;
        out[k] = Ptg[k] + (mu / t) * (nk * vtg + vn * Ptg[k] - vn * vt[k] * vtg / (t * t));
    }
    for (int k = 0; k < 3; ++k) gbar[k] = out[k];
}

/* transpose of the obstacle slide map u -> vb + (1 + mu vn / t) P (u - vb) at
 * input u (P = I - n n^T, vn = n . (u - vb), t = |P (u - vb)|):
 * J^T g = (1 + mu vn / t) P g + mu (n / t - vn tv / t^3) (tv . g) */
static void obstacle_slide_adj(const orc_params* P, const orc_obstacle* O, const double nrm[3], const double u[3],
                               double g[3])
{
    double r[3], vn = 0.0;
    for (int k = 0; k < 3; ++k) {
        r[k] = (k < P->dim) ? u[k] - O->vel[k] : 0.0;
        vn += r[k] * nrm[k];
    }
    double tv[3], t = 0.0, ng = 0.0, tg = 0.0;
    for (int k = 0; k < 3; ++k) {
        tv[k] = r[k] - vn * nrm[k];
        t += tv[k] * tv[k];
        ng += nrm[k] * g[k];
        tg += tv[k] * g[k];
    }
    t = sqrt(t);
    double out[3];
    for (int k = 0; k < 3; ++k) {
        double pg = g[k] - ng * nrm[k];
        out[k] = (1.0 + O->mu * vn / t) * pg + O->mu * (nrm[k] / t - vn * tv[k] / (t * t * t)) * tg;
    }
    for (int k = 0; k < 3; ++k) g[k] = out[k];
}

/* transpose of Eqs. 16-18 for one node during step n: vbar -> (pbar, mbar) */
static void grid_node_adj(const orc_params* P, int g, int n, double m, const double p[3], const double vbar[3],
                          double pbar[3], double* mbar)
{
    pbar[0] = pbar[1] = pbar[2] = 0.0;
    *mbar = 0.0;
    orc_node_bc s;
    if (!node_bc(P, g, n, m, p, &s)) return;
    /* reverse order: clamp, walls, obstacles (last first), floor */
    double gb[3] = {vbar[0], vbar[1], vbar[2]};
    if (s.clamped) gb[0] = gb[1] = gb[2] = 0.0;
    for (int k = 0; k < P->dim; ++k)
        if (s.wall[k]) gb[k] = 0.0;
    for (int j = P->n_obstacles - 1; j >= 0; --j) {
        if (s.ob_br[j] == 1) gb[0] = gb[1] = gb[2] = 0.0;
        else if (s.ob_br[j] == 2) obstacle_slide_adj(P, &P->obst[j], s.ob_n[j], s.ob_in[j], gb);
    }
    if (s.floor_br == 1) gb[0] = gb[1] = gb[2] = 0.0;
    else if (s.floor_br == 2) floor_slide_adj(P, s.u0, gb);
    if (P->dim == 2) gb[2] = 0.0;
    double sc = 1.0 - P->damping * P->dt;
    double vhb[3];
    for (int k = 0; k < 3; ++k) vhb[k] = sc * gb[k];
    for (int k = 0; k < 3; ++k) pbar[k] = vhb[k] / m;
    *mbar = -(vhb[0] * s.vh[0] + vhb[1] * s.vh[1] + vhb[2] * s.vh[2]) / m;
}

void orc_grid_adj(const orc_params* P, int n, const double* m, const double* p, const double* vbar,
                  double* pbar, double* mbar)
{
    int G = n_nodes(P);
#pragma omp parallel for schedule(static)
    for (int g = 0; g < G; ++g) grid_node_adj(P, g, n, m[g], p + 3 * g, vbar + 3 * g, pbar + 3 * g, mbar + g);
}

/*
 * Transpose of P2G (a gather over each particle's stencil). Adds into adj
 * (x and F already hold the G2P share; v and C are overwritten here), and
 * accumulates into the design adjoints gphi[N], gbr[N][3] and gB[3].
 */
int orc_p2g_adj(const orc_params* P, int N, const orc_particle* s, const double* phi, const double* br3,
                const double B[3], const double* pbar, const double* mbar, orc_particle* adj,
                double* gphi, double* gbr3, double gB[3])
{
    double dx = 1.0 / P->n_grid;
    double kappa = 4.0 * P->dt / (dx * dx);
    double V = P->particle_volume;
    double G, K;
    orc_moduli(P->E, P->nu, &G, &K);
    /* the field gradient sums over all particles: one partial sum per thread
     * (its contiguous block of particles, in order), added in thread order */
    const int nt = max_threads();
    double* gB_part = calloc((size_t)nt * 3, sizeof(double));
    if (!gB_part) return ORC_ENOMEM;
    long long first_err = ERR_NONE;
#pragma omp parallel num_threads(nt) reduction(min : first_err)
    {
        double* gB_t = gB_part + 3 * thread_id();
#pragma omp for schedule(static)
        for (int q = 0; q < N; ++q) {
            orc_stencil S;
            int e = make_stencil(P, s[q].x, &S);
            if (e) {
                if (ERR_KEY(q, e) < first_err) first_err = ERR_KEY(q, e);
                continue;
            }
            double Pt[9], Pe[9], Pm[9], PFt[9], Ft[9], A[9];
            particle_stress(P, s[q].F, phi[q], br3 + 3 * q, B, Pt, Pe, Pm);
            transpose3(s[q].F, Ft);
            matmul3(Pt, Ft, PFt);
            double mp = particle_mass(P, phi[q]);
            for (int k = 0; k < 9; ++k) A[k] = mp * s[q].C[k] - kappa * V * PFt[k];
            double mb = 0.0, vb[3] = {0, 0, 0}, Ab[9] = {0}, xb[3] = {0, 0, 0};
            FOR_STENCIL(P, a0, a1, a2) {
                orc_node nd;
                stencil_node(P, &S, a0, a1, a2, &nd);
                const double* pb = pbar + 3 * nd.idx;
                double mbi = mbar[nd.idx];
                double Ad[3], Atp[3];
                for (int i = 0; i < 3; ++i) {
                    Ad[i] = 0.0;
                    Atp[i] = 0.0;
                    for (int j = 0; j < 3; ++j) {
                        Ad[i] += A[3 * i + j] * nd.dpos[j];
                        Atp[i] += A[3 * j + i] * pb[j];
                    }
                }
                double pv = pb[0] * s[q].v[0] + pb[1] * s[q].v[1] + pb[2] * s[q].v[2];
                double pmom = 0.0;
                for (int i = 0; i < 3; ++i) pmom += pb[i] * (mp * s[q].v[i] + Ad[i]);
                mb += nd.w * (mbi + pv);
                for (int i = 0; i < 3; ++i) {
                    vb[i] += nd.w * mp * pb[i];
                    for (int j = 0; j < 3; ++j) Ab[3 * i + j] += nd.w * pb[i] * nd.dpos[j];
                }
                for (int k = 0; k < 3; ++k)
                    xb[k] += (mbi * mp + pmom) * nd.gw[k] - nd.w * Atp[k];
            }
            /* A = m C - kappa V P F^T */
            mb += ddot9(Ab, s[q].C);
            double Pb[9], AbF[9], Abt[9], AbtP[9], dP[9];
            matmul3(Ab, s[q].F, AbF);
            for (int k = 0; k < 9; ++k) Pb[k] = -kappa * V * AbF[k];
            transpose3(Ab, Abt);
            matmul3(Abt, Pt, AbtP);
            if (P->dim == 2)
                for (int k = 0; k < 9; ++k)
                    if (k / 3 == 2 || k % 3 == 2) Pb[k] = 0.0;
            orc_stress_elastic_dir(s[q].F, G, K, Pb, dP);
            double se = simp_e(P, phi[q]), sm = simp_m(P, phi[q]);
            orc_particle* a = &adj[q];
            for (int k = 0; k < 9; ++k) {
                a->C[k] = mp * Ab[k];
                a->F[k] += -kappa * V * AbtP[k] + se * dP[k];
            }
            for (int k = 0; k < 3; ++k) {
                a->v[k] = vb[k];
                a->x[k] += xb[k];
            }
            if (P->dim == 2) {
                a->x[2] = a->v[2] = 0.0;
                for (int k = 0; k < 9; ++k)
                    if (k / 3 == 2 || k % 3 == 2) { a->F[k] = 0.0; a->C[k] = 0.0; }
            }
            /* P = s_e(phi) P_e + s_m(phi) P_m ; m = phi rho V */
            gphi[q] += particle_mass_d(P) * mb + simp_e_d(P, phi[q]) * ddot9(Pb, Pe) + simp_m_d(P, phi[q]) * ddot9(Pb, Pm);
            /* P_m = -(1/mu0) B (x) Br */
            for (int j = 0; j < 3; ++j) {
                double PtB = 0.0, PBr = 0.0;
                for (int i = 0; i < 3; ++i) {
                    PtB += Pb[3 * i + j] * B[i];
                    PBr += Pb[3 * j + i] * br3[3 * q + i];
                }
                gbr3[3 * q + j] += -sm / P->mu0 * PtB;
                gB_t[j] += -sm / P->mu0 * PBr;
            }
        }
    }
    for (int t = 0; t < nt; ++t)
        for (int j = 0; j < 3; ++j) gB[j] += gB_part[3 * t + j];
    free(gB_part);
    return err_code(first_err, ERR_NONE);
}

/* ------------------------------------------------------------------------- */
/* rollout, loss and reverse rollout                                         */
/* ------------------------------------------------------------------------- */

static void init_state(const orc_params* P, int N, const double* x0, const double* v0, orc_particle* s)
{
    for (int q = 0; q < N; ++q) {
        memset(&s[q], 0, sizeof(orc_particle));
        for (int k = 0; k < P->dim; ++k) {
            s[q].x[k] = x0[q * P->dim + k];
            s[q].v[k] = v0 ? v0[q * P->dim + k] : 0.0;
        }
        s[q].F[0] = s[q].F[4] = s[q].F[8] = 1.0;
    }
}

static void expand3(const orc_params* P, int N, const double* a, double* a3)
{
    for (int q = 0; q < N; ++q)
        for (int k = 0; k < 3; ++k) a3[3 * q + k] = k < P->dim ? a[q * P->dim + k] : 0.0;
}

/* losses of Sec. 4 (Eqs. 36-40). vsum = sum over steps of v(t_{n+1}) per particle
 * (needed only by the trajectory loss, Eq. 39). */
static double loss_value(const orc_params* P, int N, const orc_particle* sT, const double* x0,
                         const double* phi, const double* target, const unsigned char* mask,
                         double traj_acc)
{
    int d = P->dim;
    const double* e = P->loss_dir;
    if (P->loss_kind == ORC_LOSS_FINAL_MSE) {
        if (!target) return 0.0;   /* no target given: no loss */
        double s = 0.0;
        int cnt = 0;
        for (int q = 0; q < N; ++q) {
            if (mask && !mask[q]) continue;
            ++cnt;
            for (int k = 0; k < d; ++k) {
                double r = sT[q].x[k] - target[q * d + k];
                s += r * r;
            }
        }
        return cnt ? s / cnt : 0.0;
    }
    if (P->loss_kind == ORC_LOSS_TIP_DISP) {
        double s = 0.0;
        int cnt = 0;
        for (int q = 0; q < N; ++q) {
            if (mask && !mask[q]) continue;
            ++cnt;
            for (int k = 0; k < d; ++k) s += e[k] * (sT[q].x[k] - x0[q * d + k]);
        }
        return cnt ? -s / cnt : 0.0;
    }
    /* Eq. 40 sums the mass-averaged velocity over the steps, i.e. the centre
     * of mass's displacement: summed here from each particle's displacement
     * x(T) - x(0), not as a difference of two centres of mass (which would
     * cancel nearly all digits of a small displacement) */
    double M = 0.0, s = 0.0;
    for (int q = 0; q < N; ++q) {
        double mq = particle_mass(P, phi[q]);
        M += mq;
        for (int k = 0; k < d; ++k) s += mq * e[k] * (sT[q].x[k] - x0[q * d + k]);
    }
    if (P->loss_kind == ORC_LOSS_COM_DISP) return -s / M;
    /* trajectory loss: -dt sum_n e . (sum_p m_p v_p(t_{n+1})) / M, accumulated */
    return traj_acc;
}

static double total_mass(const orc_params* P, int N, const double* phi)
{
    double M = 0.0;
    for (int q = 0; q < N; ++q) M += particle_mass(P, phi[q]);
    return M;
}

static double traj_step(const orc_params* P, int N, const orc_particle* s1, const double* phi, double M)
{
    double acc = 0.0;
    for (int q = 0; q < N; ++q) {
        double mq = particle_mass(P, phi[q]);
        for (int k = 0; k < P->dim; ++k) acc += mq * P->loss_dir[k] * s1[q].v[k];
    }
    return -P->dt * acc / M;
}

/*
 * Forward rollout of n_steps steps from x0 (v0 optional, else 0), C = 0, F = I.
 * x0, v0, br: [N][dim]; bprog: [S][dim]; target: [N][dim] or NULL; mask: [N] or NULL.
 * Outputs (each optional): final state as 3-component / 3x3 arrays
 * x_out[N][3], v_out[N][3], C_out[N][9], F_out[N][9]; loss_out;
 * traj_x[(n_steps+1)][N][3] positions at every step.
 */
int orc_rollout(const orc_params* P, int N, const double* x0, const double* v0, const double* phi,
                const double* br, const double* bprog, const double* target, const unsigned char* mask,
                double* x_out, double* v_out, double* C_out, double* F_out, double* loss_out,
                double* traj_x)
{
    if (!P || N < 0 || (P->dim != 2 && P->dim != 3) || P->n_grid < 4) return ORC_EINVAL;
    int G = n_nodes(P);
    orc_particle* s = malloc(sizeof(orc_particle) * (N ? N : 1));
    orc_particle* t = malloc(sizeof(orc_particle) * (N ? N : 1));
    double* br3 = malloc(sizeof(double) * 3 * (N ? N : 1));
    double* m = malloc(sizeof(double) * G);
    double* p = malloc(sizeof(double) * 3 * G);
    double* v = malloc(sizeof(double) * 3 * G);
    orc_scatter ws;
    int err = scatter_alloc(&ws, G);
    if (!s || !t || !br3 || !m || !p || !v || err) { err = ORC_ENOMEM; goto done; }
    init_state(P, N, x0, v0, s);
    expand3(P, N, br, br3);
    double M = total_mass(P, N, phi);
    double traj = 0.0;
    if (traj_x)
        for (int q = 0; q < N; ++q)
            for (int k = 0; k < 3; ++k) traj_x[3 * q + k] = s[q].x[k];
    for (int n = 0; n < P->n_steps; ++n) {
        double B[3];
        field_at(P, bprog, n, B);
        err = step_forward(P, N, n, s, phi, br3, B, m, p, v, t, &ws);
        if (err) goto done;
        orc_particle* tmp = s; s = t; t = tmp;
        if (P->loss_kind == ORC_LOSS_TRAJ_VEL && N) traj += traj_step(P, N, s, phi, M);
        if (traj_x)
            for (int q = 0; q < N; ++q)
                for (int k = 0; k < 3; ++k) traj_x[(size_t)(n + 1) * 3 * N + 3 * q + k] = s[q].x[k];
    }
    for (int q = 0; q < N; ++q) {
        if (x_out) memcpy(x_out + 3 * q, s[q].x, sizeof(double) * 3);
        if (v_out) memcpy(v_out + 3 * q, s[q].v, sizeof(double) * 3);
        if (C_out) memcpy(C_out + 9 * q, s[q].C, sizeof(double) * 9);
        if (F_out) memcpy(F_out + 9 * q, s[q].F, sizeof(double) * 9);
    }
    if (loss_out) *loss_out = N ? loss_value(P, N, s, x0, phi, target, mask, traj) : 0.0;
done:
    free(s); free(t); free(br3); free(m); free(p); free(v);
    scatter_free(&ws);
    return err;
}

/* one reverse step n: state sn (state at step n), adjoint of state n+1 in adj
 * (overwritten with the adjoint of state n). */
static int reverse_step(const orc_params* P, int N, int n, const orc_particle* sn, const double* phi,
                        const double* br3, const double* bprog, double* m, double* p, double* v,
                        double* vbar, double* pbar, double* mbar, orc_particle* adj, orc_particle* adj0,
                        double* gphi, double* gbr3, double* gprog, double traj_seed, double M,
                        orc_scatter* ws)
{
    double B[3];
    field_at(P, bprog, n, B);
    int e = p2g_into(P, N, sn, phi, br3, B, m, p, ws);
    if (e) return e;
    orc_grid(P, n, m, p, v);
    if (P->loss_kind == ORC_LOSS_TRAJ_VEL)
        for (int q = 0; q < N; ++q) {
            double mq = particle_mass(P, phi[q]);
            for (int k = 0; k < P->dim; ++k) adj[q].v[k] += traj_seed * (-P->dt * mq * P->loss_dir[k] / M);
        }
    e = g2p_adj_into(P, N, sn, v, adj, vbar, adj0, ws);
    if (e) return e;
    orc_grid_adj(P, n, m, p, vbar, pbar, mbar);
    double gB[3] = {0, 0, 0};
    e = orc_p2g_adj(P, N, sn, phi, br3, B, pbar, mbar, adj0, gphi, gbr3, gB);
    if (e) return e;
    int k = orc_segment(P, n);
    for (int j = 0; j < P->dim; ++j) gprog[k * P->dim + j] += gB[j];
    memcpy(adj, adj0, sizeof(orc_particle) * N);
    return 0;
}

/*
 * Reverse-mode gradient of the loss of one instance with respect to the design
 * density phi[N], the reference remanence br[N][dim] and the field program
 * bprog[S][dim], scaled by dloss. Checkpoints every ckpt_every steps (1 = keep
 * every state); each segment is recomputed forward once, then reversed.
 */
int orc_backward(const orc_params* P, int N, const double* x0, const double* phi, const double* br,
                 const double* bprog, const double* target, const unsigned char* mask, double dloss,
                 int ckpt_every, double* loss_out, double* gphi, double* gbr, double* gprog)
{
    if (!P || N <= 0 || (P->dim != 2 && P->dim != 3) || P->n_grid < 4) return ORC_EINVAL;
    int T = P->n_steps, d = P->dim;
    int K = ckpt_every > 0 ? ckpt_every : 1;
    int nck = (T + K - 1) / K;
    if (nck < 1) nck = 1;
    int G = n_nodes(P);
    size_t ps = sizeof(orc_particle) * N;
    orc_particle* ck = malloc(ps * nck);
    orc_particle* seg = malloc(ps * (K + 1));
    orc_particle* adj = calloc(N, sizeof(orc_particle));
    orc_particle* adj0 = calloc(N, sizeof(orc_particle));
    double* br3 = malloc(sizeof(double) * 3 * N);
    double* gbr3 = calloc(3 * (size_t)N, sizeof(double));
    double* vsum = calloc(3 * (size_t)N, sizeof(double));
    double* m = malloc(sizeof(double) * G);
    double* p = malloc(sizeof(double) * 3 * G);
    double* v = malloc(sizeof(double) * 3 * G);
    double* vbar = malloc(sizeof(double) * 3 * G);
    double* pbar = malloc(sizeof(double) * 3 * G);
    double* mbar = malloc(sizeof(double) * G);
    orc_scatter ws;
    int err = scatter_alloc(&ws, G);
    if (!ck || !seg || !adj || !adj0 || !br3 || !gbr3 || !vsum || !m || !p || !v || !vbar || !pbar || !mbar || err) {
        err = ORC_ENOMEM;
        goto done;
    }
    expand3(P, N, br, br3);
    for (int q = 0; q < N; ++q) gphi[q] = 0.0;
    for (int j = 0; j < P->n_segments * d; ++j) gprog[j] = 0.0;

    /* forward, keeping checkpoints */
    orc_particle* cur = seg;
    orc_particle* nxt = seg + N;
    init_state(P, N, x0, NULL, cur);
    double M = total_mass(P, N, phi);
    double traj = 0.0;
    for (int n = 0; n < T; ++n) {
        if (n % K == 0) memcpy(ck + (size_t)(n / K) * N, cur, ps);
        double B[3];
        field_at(P, bprog, n, B);
        err = step_forward(P, N, n, cur, phi, br3, B, m, p, v, nxt, &ws);
        if (err) goto done;
        orc_particle* tmp = cur; cur = nxt; nxt = tmp;
        if (P->loss_kind == ORC_LOSS_TRAJ_VEL) {
            traj += traj_step(P, N, cur, phi, M);
            for (int q = 0; q < N; ++q)
                for (int k = 0; k < 3; ++k) vsum[3 * q + k] += cur[q].v[k];
        }
    }
    if (T == 0) memcpy(ck, cur, ps);
    double L = loss_value(P, N, cur, x0, phi, target, mask, traj);
    if (loss_out) *loss_out = L;

    /* adjoint seed at the final state and the direct density terms */
    const double* e = P->loss_dir;
    if (P->loss_kind == ORC_LOSS_FINAL_MSE || P->loss_kind == ORC_LOSS_TIP_DISP) {
        int cnt = 0;
        for (int q = 0; q < N; ++q) cnt += (!mask || mask[q]) ? 1 : 0;
        for (int q = 0; q < N; ++q) {
            if (mask && !mask[q]) continue;
            for (int k = 0; k < d; ++k) {
                if (P->loss_kind == ORC_LOSS_FINAL_MSE)
                    adj[q].x[k] = dloss * 2.0 * (cur[q].x[k] - target[q * d + k]) / cnt;
                else
                    adj[q].x[k] = -dloss * e[k] / cnt;
            }
        }
    } else if (P->loss_kind == ORC_LOSS_COM_DISP) {
        /* L = -(S1 - S0) / M with S = sum m_q e.x_q ; m_q = phi_q rho V */
        for (int q = 0; q < N; ++q) {
            double mq = particle_mass(P, phi[q]);
            double dxe = 0.0;
            for (int k = 0; k < d; ++k) {
                adj[q].x[k] = -dloss * mq * e[k] / M;
                dxe += e[k] * (cur[q].x[k] - x0[q * d + k]);
            }
            gphi[q] += dloss * particle_mass_d(P) * (-dxe / M - L / M);
        }
    } else {
        /* trajectory loss: per-step velocity seeds are injected in reverse_step */
        for (int q = 0; q < N; ++q) {
            double ve = 0.0;
            for (int k = 0; k < d; ++k) ve += e[k] * vsum[3 * q + k];
            gphi[q] += dloss * particle_mass_d(P) * (-P->dt * ve / M - L / M);
        }
    }

    /* reverse over the checkpoint segments, last first */
    for (int c = nck - 1; c >= 0; --c) {
        int s0 = c * K;
        int s1 = s0 + K < T ? s0 + K : T;
        memcpy(seg, ck + (size_t)c * N, ps);
        for (int n = s0; n < s1 - 1; ++n) {
            double B[3];
            field_at(P, bprog, n, B);
            err = step_forward(P, N, n, seg + (size_t)(n - s0) * N, phi, br3, B, m, p, v,
                               seg + (size_t)(n - s0 + 1) * N, &ws);
            if (err) goto done;
        }
        for (int n = s1 - 1; n >= s0; --n) {
            err = reverse_step(P, N, n, seg + (size_t)(n - s0) * N, phi, br3, bprog, m, p, v, vbar, pbar,
                               mbar, adj, adj0, gphi, gbr3, gprog, dloss, M, &ws);
            if (err) goto done;
        }
    }
    for (int q = 0; q < N; ++q)
        for (int k = 0; k < d; ++k) gbr[q * d + k] = gbr3[3 * q + k];
done:
    free(ck); free(seg); free(adj); free(adj0); free(br3); free(gbr3); free(vsum);
    free(m); free(p); free(v); free(vbar); free(pbar); free(mbar);
    scatter_free(&ws);
    return err;
}

/* ------------------------------------------------------------------------- */
/* flat-array entry points for the per-phase tests                           */
/* ------------------------------------------------------------------------- */

static void pack(int N, const double* x, const double* v, const double* C, const double* F, orc_particle* s)
{
    for (int q = 0; q < N; ++q) {
        memcpy(s[q].x, x + 3 * q, sizeof(double) * 3);
        memcpy(s[q].v, v + 3 * q, sizeof(double) * 3);
        memcpy(s[q].C, C + 9 * q, sizeof(double) * 9);
        memcpy(s[q].F, F + 9 * q, sizeof(double) * 9);
    }
}

static void unpack(int N, const orc_particle* s, double* x, double* v, double* C, double* F)
{
    for (int q = 0; q < N; ++q) {
        if (x) memcpy(x + 3 * q, s[q].x, sizeof(double) * 3);
        if (v) memcpy(v + 3 * q, s[q].v, sizeof(double) * 3);
        if (C) memcpy(C + 9 * q, s[q].C, sizeof(double) * 9);
        if (F) memcpy(F + 9 * q, s[q].F, sizeof(double) * 9);
    }
}

/* P2G on flat arrays: x,v [N][3]; C,F [N][9]; br3 [N][3]; B[3] -> m[G], p[G][3] */
int orc_p2g_flat(const orc_params* P, int N, const double* x, const double* v, const double* C,
                 const double* F, const double* phi, const double* br3, const double* B, double* m, double* p)
{
    orc_particle* s = malloc(sizeof(orc_particle) * (N ? N : 1));
    if (!s) return ORC_ENOMEM;
    pack(N, x, v, C, F, s);
    int e = orc_p2g(P, N, s, phi, br3, B, m, p);
    free(s);
    return e;
}

int orc_g2p_flat(const orc_params* P, int N, const double* x, const double* F, const double* vgrid,
                 double* x1, double* v1, double* C1, double* F1)
{
    orc_particle* s = calloc(N ? N : 1, sizeof(orc_particle));
    orc_particle* o = calloc(N ? N : 1, sizeof(orc_particle));
    if (!s || !o) { free(s); free(o); return ORC_ENOMEM; }
    for (int q = 0; q < N; ++q) {
        memcpy(s[q].x, x + 3 * q, sizeof(double) * 3);
        memcpy(s[q].F, F + 9 * q, sizeof(double) * 9);
    }
    int e = orc_g2p(P, N, s, vgrid, o);
    unpack(N, o, x1, v1, C1, F1);
    free(s); free(o);
    return e;
}

int orc_g2p_adj_flat(const orc_params* P, int N, const double* x, const double* F, const double* vgrid,
                     const double* xb1, const double* vb1, const double* Cb1, const double* Fb1,
                     double* vbar, double* xb0, double* Fb0)
{
    orc_particle* s = calloc(N ? N : 1, sizeof(orc_particle));
    orc_particle* a1 = calloc(N ? N : 1, sizeof(orc_particle));
    orc_particle* a0 = calloc(N ? N : 1, sizeof(orc_particle));
    if (!s || !a1 || !a0) { free(s); free(a1); free(a0); return ORC_ENOMEM; }
    for (int q = 0; q < N; ++q) {
        memcpy(s[q].x, x + 3 * q, sizeof(double) * 3);
        memcpy(s[q].F, F + 9 * q, sizeof(double) * 9);
    }
    pack(N, xb1, vb1, Cb1, Fb1, a1);
    int e = orc_g2p_adj(P, N, s, vgrid, a1, vbar, a0);
    unpack(N, a0, xb0, NULL, NULL, Fb0);
    free(s); free(a1); free(a0);
    return e;
}

int orc_p2g_adj_flat(const orc_params* P, int N, const double* x, const double* v, const double* C,
                     const double* F, const double* phi, const double* br3, const double* B,
                     const double* pbar, const double* mbar, double* xb, double* vb, double* Cb, double* Fb,
                     double* gphi, double* gbr3, double* gB)
{
    orc_particle* s = malloc(sizeof(orc_particle) * (N ? N : 1));
    orc_particle* a = calloc(N ? N : 1, sizeof(orc_particle));
    if (!s || !a) { free(s); free(a); return ORC_ENOMEM; }
    pack(N, x, v, C, F, s);
    int e = orc_p2g_adj(P, N, s, phi, br3, B, pbar, mbar, a, gphi, gbr3, gB);
    unpack(N, a, xb, vb, Cb, Fb);
    free(s); free(a);
    return e;
}

int orc_num_nodes(const orc_params* P) { return n_nodes(P); }
