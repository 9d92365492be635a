/*
 * Host driver for sanitizer runs of the FP64 oracle (test infrastructure):
 * built together with the oracle's source under AddressSanitizer and
 * UndefinedBehaviorSanitizer, it runs 2D and 3D rollouts and backward passes
 * with floor contact, a clamp and obstacles (a sphere, a moving half-space and
 * an attached box), for every loss kind. Exit status 0 and "ok" when every call
 * succeeds with finite results.
 */
#include "mpm_oracle.c"

#include <stdio.h>

static int check_finite(const double* a, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int run_case(int dim, int loss_kind)
{
    orc_params P;
    memset(&P, 0, sizeof P);
    P.dim = dim;
    P.n_grid = 16;
    P.dt = 2e-3;
    P.n_steps = 12;
    P.E = 1.0;
    P.nu = 0.3;
    P.rho = 1.0;
    P.mu0 = 1.0;
    P.simp_eps = 1e-3;
    P.simp_q = 3.0;
    P.damping = 0.1;
    P.gravity[1] = -1.0;
    P.wall_cells = 3;
    P.clamp_xmax = 0.33;
    P.floor_on = 1;
    P.floor_y = 0.4;
    P.floor_mu = 0.5;
    P.particle_volume = pow(1.0 / 32, dim);
    P.n_segments = 3;
    P.seg_steps = 4;
    P.loss_kind = loss_kind;
    P.loss_dir[0] = 0.8;
    P.loss_dir[1] = 0.6;
    P.n_obstacles = 3;
    P.obst[0].kind = ORC_OBST_SPHERE;
    P.obst[0].a[0] = 0.5; P.obst[0].a[1] = 0.35; P.obst[0].a[2] = 0.5;
    P.obst[0].b[0] = 0.06;
    P.obst[0].mu = 0.3;
    P.obst[1].kind = ORC_OBST_HALFSPACE;
    P.obst[1].a[0] = 0.62;
    P.obst[1].b[0] = -1.0; P.obst[1].b[1] = 0.2;
    P.obst[1].mu = INFINITY;
    P.obst[1].vel[0] = -0.1;
    P.obst[2].kind = ORC_OBST_BOX;
    P.obst[2].a[0] = 0.45; P.obst[2].a[1] = 0.55; P.obst[2].a[2] = 0.5;
    P.obst[2].b[0] = 0.02; P.obst[2].b[1] = 0.02; P.obst[2].b[2] = 0.02;
    P.obst[2].attached = 1;
    P.obst[2].vel[1] = 0.05;
    const int side = 6, N = dim == 2 ? side * side : side * side * side;
    double *x0 = calloc((size_t)N * dim, sizeof(double)), *phi = calloc(N, sizeof(double));
    double *br = calloc((size_t)N * dim, sizeof(double)), *tgt = calloc((size_t)N * dim, sizeof(double));
    double *bprog = calloc((size_t)P.n_segments * dim, sizeof(double));
    unsigned char* mask = calloc(N, 1);
    for (int q = 0; q < N; ++q) {
        int c[3] = {q % side, (q / side) % side, q / (side * side)};
        for (int k = 0; k < dim; ++k) {
            x0[q * dim + k] = 0.4 + (c[k] + 0.5) / 32.0 + (k == 1 ? 0.02 : 0.0);
            br[q * dim + k] = (k == 0) ? 1.0 : 0.2;
            tgt[q * dim + k] = x0[q * dim + k] + 0.01 * k;
        }
        phi[q] = 0.3 + 0.7 * (q % 5) / 4.0;
        mask[q] = (unsigned char)(q % 3 != 0);
    }
    for (int s = 0; s < P.n_segments * dim; ++s) bprog[s] = 0.2 * ((s % 3) - 1);
    double *xo = calloc((size_t)N * 3, sizeof(double)), *vo = calloc((size_t)N * 3, sizeof(double));
    double *Co = calloc((size_t)N * 9, sizeof(double)), *Fo = calloc((size_t)N * 9, sizeof(double));
    double loss = 0, loss2 = 0;
    double *gphi = calloc(N, sizeof(double)), *gbr = calloc((size_t)N * dim, sizeof(double));
    double* gprog = calloc((size_t)P.n_segments * dim, sizeof(double));
    int e = orc_rollout(&P, N, x0, NULL, phi, br, bprog, tgt, mask, xo, vo, Co, Fo, &loss, NULL);
    if (!e) e = orc_backward(&P, N, x0, phi, br, bprog, tgt, mask, 1.0, 5, &loss2, gphi, gbr, gprog);
    int ok = !e && isfinite(loss) && check_finite(xo, N * 3) && check_finite(gphi, N) &&
             check_finite(gbr, N * dim) && check_finite(gprog, P.n_segments * dim);
    if (!ok) fprintf(stderr, "dim %d loss %d: status %d\n", dim, loss_kind, e);
    free(x0); free(phi); free(br); free(tgt); free(bprog); free(mask);
    free(xo); free(vo); free(Co); free(Fo); free(gphi); free(gbr); free(gprog);
    return ok;
}

int main(void)
{
    int ok = 1;
    for (int dim = 2; dim <= 3; ++dim)
        for (int kind = ORC_LOSS_FINAL_MSE; kind <= ORC_LOSS_TIP_DISP; ++kind) ok = run_case(dim, kind) && ok;
    puts(ok ? "ok" : "failed");
    return ok ? 0 : 1;
}
