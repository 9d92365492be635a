/*
 * mpm_mag_design.h: the design front end of the magneto-elastic MPM library.
 * (The harmonic stimulus of Eqs. 29-30 is at the end of this file.)
 *
 * Maps the design variables of Sec. 3.1 to the per-particle inputs of
 * mpm_mag_rollout, and maps the gradients mpm_mag_backward returns back to
 * the design variables:
 *   density filter (Eqs. 23-24)  phit_p = sum_q w_pq phi_q / sum_q w_pq over the
 *                                particles q with |x_q(0) - x_p(0)| < R (p itself
 *                                included), w_pq = 1 - |x_q(0) - x_p(0)| / R
 *   Heaviside projection (Eq. 25) density_p = (tanh(beta/2) + tanh(beta (phit_p - 1/2)))
 *                                             / (2 tanh(beta/2))
 *   magnetization (Eqs. 26-27)  br_p = Br_max Br_m zeta_m / sqrt(|zeta_m|^2 + delta)
 *   region sharing (Eq. 28)     m = region[p]; without a region map every
 *                                particle is its own region (n_m = N)
 *
 * All array pointers are HIP device pointers owned by the caller, contiguous,
 * of the handle's element type (float for precision 4, double for 8) unless
 * stated. Work is ordered on the given stream (a hipStream_t, NULL for the
 * default stream). Status codes are those of mpm_mag.h; no call aborts or
 * throws. A handle is not thread-safe.
 */
#ifndef MPM_MAG_DESIGN_H
#define MPM_MAG_DESIGN_H

#include <stdint.h>

#include "mpm_mag.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_mag_design mpm_mag_design;

/*
 * Build the filter's neighbour matrix from the initial positions, once.
 *   dim         2 or 3
 *   n_particles N >= 1 (at most 2^30)
 *   x0          [N][dim] initial positions (copied into the matrix; not kept)
 *   radius      filter radius R > 0
 *   region      [N] int32 region of each particle, in [0, n_regions), or NULL
 *   n_regions   region count (ignored when region is NULL)
 *   precision   4 (float) or 8 (double)
 * Synchronizes the stream (the matrix size is read back). Returns EINVAL for
 * bad sizes or a region outside [0, n_regions), ENONFINITE for a non-finite
 * position, ENOMEM when the matrix would exceed 2^31 - 1 entries or memory.
 * *out is set only on success.
 */
int mpm_mag_design_create(int dim, int64_t n_particles, const void* x0, double radius, const int32_t* region,
                          int n_regions, int precision, void* stream, mpm_mag_design** out);

/*
 * Forward map.
 *   phi         [N]          topology variables (Sec. 3.1)
 *   beta        projection sharpness, > 0
 *   br_mag      [n_m]        normalized magnetization magnitudes
 *   zeta        [n_m][dim]   magnetization orientation vectors
 *   br_max      Br_max of Eq. 26
 *   delta       delta of Eq. 27, >= 0 (|zeta_m|^2 + delta must be > 0)
 *   copies      1..4096: the outputs hold this many consecutive copies of the
 *               design, one per task instance that shares it (Eq. 35)
 *   density_out [copies][N]      projected density (output, overwritten)
 *   br_out      [copies][N][dim] remanent flux density (output, overwritten)
 * The handle keeps phit, beta, br_mag, zeta, br_max and delta for backward.
 */
int mpm_mag_design_forward(mpm_mag_design* h, void* stream, const void* phi, double beta, const void* br_mag,
                           const void* zeta, double br_max, double delta, int copies, void* density_out,
                           void* br_out);

/*
 * Transpose of the forward map's Jacobian at the last forward call; the
 * gradients of the copies are summed (Eq. 35's shared design).
 *   copies    1..4096
 *   g_density [copies][N]      gradient with respect to density (e.g. from mpm_mag_backward)
 *   g_br      [copies][N][dim] gradient with respect to br
 *   g_phi     [N]        output, overwritten, or NULL
 *   g_br_mag  [n_m]      output, overwritten, or NULL
 *   g_zeta    [n_m][dim] output, overwritten, or NULL
 * Returns ESTATE before a successful forward call.
 */
int mpm_mag_design_backward(mpm_mag_design* h, void* stream, int copies, const void* g_density, const void* g_br,
                            void* g_phi, void* g_br_mag, void* g_zeta);

/* Stored entries of the neighbour matrix (pairs within the radius, self included). */
int64_t mpm_mag_design_nnz(const mpm_mag_design* h);

/* Detail of the last failure on this handle, or of the last failed create when h is NULL. */
const char* mpm_mag_design_last_error(const mpm_mag_design* h);

/* Release the handle and its device memory. NULL is accepted. */
void mpm_mag_design_destroy(mpm_mag_design* h);

/*
 * Harmonic stimulus (Sec. 3.1.2, Eqs. 29-30) as a field program of one row per
 * step, for instances created with n_segments = n_steps and seg_steps = 1
 * (non-periodic), whose step n then takes row n, the field at t_n = n dt:
 *   B(t_n) = B_max B_a sin(2 pi fbar t_n) b,  fbar = (f_max - f_min) f + f_min,
 *   b = eta / sqrt(|eta|^2 + delta).
 * Instance k has its own (B_a[k], f[k], eta[k]); all share the descriptor.
 * Evaluated in double whatever the element type. No handle and no state.
 */
typedef struct {
    int dim;                 /* 2 or 3 */
    int n_inst;              /* >= 1 */
    int n_steps;             /* >= 1; n_inst * n_steps <= 2^31 - 1 */
    double dt;               /* > 0 */
    double b_max;            /* B_max */
    double f_min, f_max;     /* frequency range (finite) */
    double delta;            /* >= 0; |eta|^2 + delta must be > 0 */
} mpm_mag_harmonic_desc;

/*
 *   b_a    [n_inst]                    normalized magnitudes
 *   f      [n_inst]                    normalized frequencies
 *   eta    [n_inst][dim]               orientation vectors
 *   b_prog [n_inst * n_steps][dim]     output, overwritten (instance-major)
 * Returns EINVAL for a bad descriptor, precision or null pointer.
 */
int mpm_mag_harmonic_program(const mpm_mag_harmonic_desc* d, int precision, void* stream, const void* b_a,
                             const void* f, const void* eta, void* b_prog);

/*
 * Transpose at (b_a, f, eta): from g_b_prog [n_inst * n_steps][dim] (e.g. the
 * program gradient of mpm_mag_backward) to g_b_a [n_inst], g_f [n_inst] and
 * g_eta [n_inst][dim] (outputs, overwritten; each may be NULL).
 */
int mpm_mag_harmonic_backward(const mpm_mag_harmonic_desc* d, int precision, void* stream, const void* b_a,
                              const void* f, const void* eta, const void* g_b_prog, void* g_b_a, void* g_f,
                              void* g_eta);

/*
 * Optimizer update of the co-design loop (Sec. 3.2): one Adam step (Kingma and
 * Ba, 2015) at step >= 1 on n variables, then the variables mapped back into
 * [lo, hi] (Eqs. 34c-d, 35c-d):
 *   m = beta1 m + (1 - beta1) g,  v = beta2 v + (1 - beta2) g^2,
 *   param = clamp(param - lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps), lo, hi)
 *   param [n] in/out; grad [n]; m, v [n] in/out, zero before the first step.
 * Element type by precision (4 float, 8 double). Returns EINVAL for bad
 * hyper-parameters (0 <= beta < 1, eps >= 0, lr >= 0, lo <= hi) or null arrays.
 */
int mpm_mag_adam_step(int precision, void* stream, int64_t n, void* param, const void* grad, void* m, void* v,
                      int step, double lr, double beta1, double beta2, double eps, double lo, double hi);

#ifdef __cplusplus
}
#endif

#endif /* MPM_MAG_DESIGN_H */
