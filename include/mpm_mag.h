/*
 * mpm_mag.h -- C ABI of the MI355X magneto-elastic MLS-MPM rollout and its adjoint.
 *
 * The library advances particle-represented hard-magnetic soft bodies through
 * time with the moving-least-squares material point method of the paper's
 * Sec. 2.2 (P2G Eqs. 14-15, grid operation Eqs. 16-18, G2P Eqs. 19-22), using
 * the magneto-elastic first Piola-Kirchhoff stress of Sec. 2.1 (Eq. 7) scaled by
 * the design density as in Sec. 3.1.3 (Eqs. 31-33). It evaluates the task losses
 * of Sec. 4 (Eqs. 36-40) and returns their gradient with respect to the design
 * density, the reference remanence and the applied-field program, i.e. the
 * sensitivities of the optimisation problems Eq. 34 / Eq. 35, obtained by
 * running the chain rule backwards through every time step (Sec. 2.3).
 *
 * Conventions shared by every entry point:
 *  - Array arguments are HIP DEVICE pointers owned by the caller, contiguous,
 *    with elements of the handle's precision (float when created with
 *    precision 4, double with precision 8) unless stated otherwise. Vectors per
 *    particle are row-major [N][dim] (AoS), per field segment [S][dim].
 *  - Several instances ("design instances" or "tasks") live in one handle; their
 *    particles are concatenated in instance order (N = sum of n_particles[k]),
 *    and their field programs likewise (S_tot = sum of n_segments[k]).
 *  - All device work is ordered on the HIP stream passed as `stream` (a
 *    hipStream_t; NULL is the null stream). rollout and backward synchronise
 *    that stream once, at the end, to read the device error word.
 *  - Functions return an mpm_mag_status; they never abort or throw across the
 *    ABI. On failure mpm_mag_last_error() holds a human-readable detail.
 *  - A handle is not thread safe; calls on one handle must not overlap.
 */
#ifndef MPM_MAG_H
#define MPM_MAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpm_mag mpm_mag;

typedef enum {
    MPM_MAG_OK = 0,
    MPM_MAG_EINVAL = 1,      /* bad argument or descriptor                                  */
    MPM_MAG_ENOMEM = 2,      /* device allocation failed                                    */
    MPM_MAG_EHIP = 3,        /* a HIP runtime call or kernel launch failed                  */
    MPM_MAG_EDOMAIN = 4,     /* a particle's 3^d stencil left the grid [0, n_grid)^d         */
    MPM_MAG_EINVERT = 5,     /* det F <= 0 for some particle                                */
    MPM_MAG_ENONFINITE = 6,  /* NaN or Inf in the inputs or the particle state              */
    MPM_MAG_ESTATE = 7       /* backward without a preceding successful record=1 rollout    */
} mpm_mag_status;

typedef enum {
    MPM_MAG_LOSS_FINAL_MSE = 0,  /* (1/|S|) sum_{p in S} |x_p(T) - target_p|^2   (Eq. 38)          */
    MPM_MAG_LOSS_COM_DISP = 1,   /* -e . (com(T) - com(0)), mass-weighted      (Eq. 40)          */
    MPM_MAG_LOSS_TRAJ_VEL = 2,   /* -dt sum_n e . vbar(t_{n+1}), vbar mass-averaged (Eq. 39)     */
    MPM_MAG_LOSS_TIP_DISP = 3    /* -(1/|S|) sum_{p in S} e . (x_p(T) - x_p(0))  (Eqs. 36-37)     */
} mpm_mag_loss_kind;

/*
 * A solid boundary of Eq. 18 beyond the floor: an analytic shape translating
 * with the constant velocity vel (v_b), at position a + vel t_n during step n
 * (t_n = n dt). A grid node lies on the boundary when the shape's signed
 * distance at the node is <= 0; the outward normal is the distance's gradient.
 * Such a node whose velocity relative to v_b points into the shape applies
 * Eq. 18 relative to v_b (mu = INFINITY: v = v_b); an attached obstacle sets
 * v = v_b whatever the velocity. Obstacles act after the floor, in order,
 * before the walls and the clamp.
 */
#define MPM_MAG_MAX_OBSTACLES 4
typedef enum {
    MPM_MAG_OBSTACLE_HALFSPACE = 1,  /* a: a point of the plane; b: outward normal (any length > 0) */
    MPM_MAG_OBSTACLE_SPHERE = 2,     /* a: centre at t = 0; b[0]: radius > 0                        */
    MPM_MAG_OBSTACLE_BOX = 3         /* axis-aligned; a: centre at t = 0; b: half extents > 0       */
} mpm_mag_obstacle_kind;

typedef struct {
    int kind;                /* mpm_mag_obstacle_kind                                          */
    int attached;            /* 1: nodes inside take v_b whatever their velocity              */
    double a[3], b[3];       /* shape parameters (components beyond dim ignored)              */
    double mu;               /* Coulomb friction of Eq. 18, >= 0; INFINITY: no-slip            */
    double vel[3];           /* v_b                                                           */
} mpm_mag_obstacle;

/*
 * One design instance. The domain is the unit square/cube with n_grid nodes per
 * axis (dx = 1 / n_grid, node i at i dx). Units are the caller's (the
 * workloads use nondimensional E = 1, mu0 = 1).
 */
typedef struct {
    int dim;                 /* 2 (plane strain) or 3                                         */
    int n_grid;              /* nodes per axis, 8..1024                                        */
    double dt;               /* time step                                                     */
    int n_steps;             /* steps per rollout; equal for all instances of a handle        */
    double E, nu;            /* Young's modulus, Poisson ratio -> G, K of Eq. 4               */
    double rho;              /* reference mass density rho_0 (Eq. 33)                         */
    double mu0;              /* permeability in Eq. 5                                          */
    double simp_eps, simp_q; /* Eq. 31: s_e = eps + (1-eps) phi^q, s_m = phi^q                 */
    double damping;          /* c of Eq. 17, a rate: v <- v + dt (g - c v)                     */
    double gravity[3];       /* g of Eq. 17 (components beyond dim ignored)                   */
    int wall_cells;          /* separating frictionless walls, this many cells from each face  */
    double clamp_xmax;       /* attached boundary: nodes with x_i <= clamp_xmax keep v = 0;
                                negative disables                                              */
    int floor_on;            /* separating Coulomb floor (Eq. 18), normal +y                   */
    double floor_y;          /* nodes with y_i <= floor_y are floor nodes                      */
    double floor_mu;         /* friction coefficient; INFINITY gives the no-slip rule          */
    double particle_volume;  /* V_p, equal for all particles of the instance                   */
    int n_segments;          /* S: segments of the piecewise-constant field program           */
    int seg_steps;           /* steps per segment L (0: ceil(n_steps / S))                     */
    int periodic;            /* segment of step n: periodic ? (n/L) mod S : min(n/L, S-1)      */
    int loss_kind;           /* mpm_mag_loss_kind                                              */
    double loss_dir[3];      /* e of the displacement / velocity losses                        */
    int ckpt_every;          /* checkpoint spacing K of the recorded rollout (0: auto ~ sqrt(T)) */
    int n_obstacles;         /* 0..MPM_MAG_MAX_OBSTACLES                                      */
    mpm_mag_obstacle obstacles[MPM_MAG_MAX_OBSTACLES];
    int64_t ckpt_budget_bytes; /* device bytes the recorded rollout may hold for the reverse
                                  sweep (checkpoints, segment stash, grid ring, grid stores);
                                  0: no bound. The handle takes the smallest positive value
                                  over its instances (or the "ckpt_budget" option).        */
    double mass_eps;         /* floor of the mass interpolation for void particles, in [0, 1]:
                                m_p = (mass_eps + (1 - mass_eps) phi_p) rho V_p; 0 is Eq. 33  */
} mpm_mag_instance_desc;

/*
 * Create a handle for n_inst instances with n_particles[k] particles each
 * (host arrays). precision: 4 (FP32) or 8 (FP64). All instances must share dim
 * and n_steps. Allocates every device buffer of the plain rollout; checkpoint
 * storage of the recorded rollout is allocated on its first use.
 * Returns EINVAL for inconsistent descriptors or for grids that hold more than
 * 2^31 - 1 nodes together (each instance's n_grid^dim rounded up to a multiple
 * of 512: two 3D instances at n_grid = 1024 fit, three do not), ENOMEM/EHIP on
 * allocation failure; *out is set only on success.
 */
int mpm_mag_create(const mpm_mag_instance_desc* descs, int n_inst, const int64_t* n_particles,
                   int precision, mpm_mag** out);

/*
 * Forward rollout of n_steps MPM steps (Sec. 2.2, repeated until T) from
 * x(0) = x0, v = 0, C = 0, F = I, for every instance, then the loss of each.
 *   x0          [N][dim]  initial positions
 *   density     [N]       projected design density phi_p in [0, 1] (Eq. 31, 33)
 *   br          [N][dim]  reference remanent flux density Br_p (Eq. 5, 26)
 *   b_prog      [S_tot][dim] applied flux density per field segment (B_applied)
 *   loss_target [N][dim]  target positions (FINAL_MSE instances), or NULL
 *   loss_mask   [N] uint8 particle subset S of FINAL_MSE / TIP_DISP, or NULL = all
 *   x_final     [N][dim]  final positions (output, overwritten), or NULL
 *   loss_out    [n_inst]  loss of each instance (output, overwritten), or NULL
 *   record      0: plain forward; 1: also keep step checkpoints for backward
 * Inputs are copied; the caller may free them after the call. Returns EDOMAIN,
 * EINVERT or ENONFINITE when the corresponding condition occurred: the earliest
 * one by step (a failure can cause others later, e.g. an inverted F gives a
 * non-finite stress one step on), and within a step a non-finite value before
 * det F <= 0 before a stencil outside the grid; mpm_mag_last_error names the
 * step. Non-finite inputs are ENONFINITE at step 0.
 */
int mpm_mag_rollout(mpm_mag* h, void* stream, const void* x0, const void* density, const void* br,
                    const void* b_prog, const void* loss_target, const uint8_t* loss_mask,
                    void* x_final, void* loss_out, int record);

/*
 * Reverse-mode gradient of sum_k dloss[k] * loss_k + sum_p dx_final_p . x_p(T)
 * over the last record=1 rollout (Sec. 2.3; Eq. 35 when instances share a
 * design): the hand-derived transpose of every step, replayed segment by
 * segment from the checkpoints. The second term lets a caller's own function
 * g of the final positions (Eq. 34) be differentiated through the rollout.
 *   dloss     [n_inst]      upstream gradient of each instance's loss
 *   dx_final  [N][dim]      upstream gradient of the final positions, or NULL (zero)
 *   g_density [N]           d/d density   (output, overwritten), or NULL
 *   g_br      [N][dim]      d/d br        (output, overwritten), or NULL
 *   g_b_prog  [S_tot][dim]  d/d b_prog    (output, overwritten), or NULL
 * dx_final and the gradients are in the caller's particle order. Returns
 * ESTATE without a recorded rollout.
 */
int mpm_mag_backward(mpm_mag* h, void* stream, const void* dloss, const void* dx_final, void* g_density,
                     void* g_br, void* g_b_prog);

/* Release every device buffer and the handle. NULL is accepted. */
void mpm_mag_destroy(mpm_mag* h);

/* Static text for a status code. */
const char* mpm_mag_strerror(int status);

/* Detail of the last failure on this handle ("" if none); valid until the next call. */
const char* mpm_mag_last_error(const mpm_mag* h);

/*
 * Tuning and instrumentation switches (key = value):
 *   "graph"         1: capture the step loop of a rollout and the reverse sweep of
 *                   backward once into HIP graphs and replay them on the stream;
 *                   0: direct launches (default). Ignored while kernel_timing is on.
 *   "kernel_timing" 1: bracket every kernel launch with HIP events on the stream
 *   "p2g_lds"       1: LDS-staged scatter (default), 0: direct global atomics
 *   "sort_curve"    particle order by cell: 0 Hilbert (default), 1 Morton, 2 row major;
 *                   takes effect at the next rollout
 *   "box_cap"       largest per-block staging box in grid nodes, 64..1024 (default 1024);
 *                   larger boxes are staged per wave or fall back to global atomics
 *   "grid_wgs"      workgroups of the grid kernels, 16..2^20 (default 2048)
 *   "grid_threads"  threads per workgroup of the grid update and its transpose, a
 *                   multiple of 64 in 256..1024; 0 (default): 256 when instance groups
 *                   run on several streams, 1024 on one
 *   "grid_parts"    workgroups that share one coarse grid block in the grid update and
 *                   its transpose, each taking a slab of the block along its last axis
 *                   (1, 2, 4 or 8; 0 (default): 2 in 3D when instance groups run on
 *                   several streams, else 1); results do not depend on it
 *   "streams"       instance groups advanced on separate streams, 0..8 (0: min(3, instances));
 *                   consecutive instances form a group; 1 runs everything on the call's stream
 *   "fuse_fwd"      1: G2P of step n and P2G of step n+1 in one kernel (default), 0: separate
 *   "fuse_adj"      1: P2G transpose of step n and G2P transpose of step n-1 in one
 *                   kernel (default), 0: separate
 *   "lane_sort"     1: at the start of every checkpoint segment, group the lanes of each
 *                   chunk of the forward kernels by the particles' current stencil base
 *                   cell (default), so the scatter's lanes that share a base stay
 *                   adjacent; 0: slot order. Results do not depend on it.
 *   "ckpt_every"    checkpoint spacing K (0: automatic); takes effect at the next recorded rollout
 *   "ckpt_budget"   device bytes the recorded rollout may hold for the reverse sweep
 *                   (checkpoints, segment stash, grid ring, grid and segment stores);
 *                   a positive value replaces the instances' ckpt_budget_bytes, 0
 *                   (default) keeps theirs. A budget below what the checkpoints,
 *                   the stash and the ring need at spacing K makes the recorded
 *                   rollout fail with ENOMEM; the grid store takes what is left.
 *                   Takes effect at the next recorded rollout.
 *   "grid_store"    device memory for the grid store, in MiB: a recorded rollout keeps
 *                   each step's active coarse grid blocks (summed momentum and mass,
 *                   4 values per node), and backward rebuilds a checkpoint segment's
 *                   grids from it (the node velocity by the same grid operation) and
 *                   recomputes only the segment's G2P instead of the whole step.
 *                   Segments the store cannot hold are recomputed in full, their
 *                   grids kept in a segment store. -1 (default): sized from the last
 *                   recorded rollout's block count plus a tenth (an estimate from the
 *                   particle counts before the first), within the checkpoint budget
 *                   when there is one, else within the free device memory less an
 *                   eighth of the total; a positive value caps it further; 0: off.
 *                   Takes effect at the next recorded rollout; results do not depend
 *                   on it beyond summation order.
 * Returns EINVAL for an unknown key or value.
 */
int mpm_mag_set_option(mpm_mag* h, const char* key, int64_t value);

/*
 * Accumulated kernel statistics since the last reset (kernel_timing must be on
 * for the times): launches, total milliseconds, and the algorithmic bytes one
 * launch moves summed over launches. Kernel ids run 0..mpm_mag_num_kernels()-1.
 * Passing kernel = -1 resets all counters.
 */
int mpm_mag_num_kernels(void);
const char* mpm_mag_kernel_name(int kernel);
int mpm_mag_kernel_stats(mpm_mag* h, int kernel, int64_t* launches, double* total_ms, double* bytes);

/*
 * Algorithmic floating-point operations of the launches counted by
 * mpm_mag_kernel_stats (add or multiply 1, fused multiply-add 2), from the
 * per-particle arithmetic of the method that each kernel class performs.
 * EINVAL for a bad kernel id or a NULL output.
 */
int mpm_mag_kernel_flops(mpm_mag* h, int kernel, double* flops);

/* Device bytes currently held by the handle (state, grids, checkpoints). */
int64_t mpm_mag_device_bytes(const mpm_mag* h);

/*
 * Allocation-free plain rollout, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same forward rollout and losses as
 * mpm_mag_create + mpm_mag_rollout(record = 0) + mpm_mag_destroy, with the
 * same arguments, computed by the same kernels, but every device buffer of
 * the rollout (particle state, grids, staging boxes, sort keys, tables) is
 * carved from a static device array of mpm_mag_noalloc_scratch_bytes() (64 MiB)
 * that each GPU the library runs on holds until the process ends. It calls no
 * hipMalloc, hipFree or other allocating routine; the caller passes the inputs
 * and outputs (device arrays as for mpm_mag_rollout). Returns ENOMEM with a
 * message (mpm_mag_last_error(NULL)) when the problem needs more scratch than
 * that. All calls on one GPU share its array: calls that overlap on one GPU
 * (other threads, other streams) race; the call returns after its stream has
 * finished with the array.
 */
int mpm_mag_rollout_noalloc(const mpm_mag_instance_desc* descs, int n_inst, const int64_t* n_particles,
                            int precision, void* stream, const void* x0, const void* density, const void* br,
                            const void* b_prog, const void* loss_target, const uint8_t* loss_mask, void* x_final,
                            void* loss_out);
int64_t mpm_mag_noalloc_scratch_bytes(void);

/*
 * Branch trace (instrumentation for parity checks). The grid operation of
 * Eqs. 16-18 takes integer decisions from floating-point node velocities:
 * whether the node has mass, which branch of Eq. 18 the floor and each
 * obstacle take, and which velocity components the domain walls zero. A
 * reference computed in another precision may decide a near-tie the other
 * way; to compare the arithmetic on equal branches it can replay these.
 * With a trace set, every forward step of the following rollouts writes one
 * code per grid node to trace[n * T_nodes + node_off_k + node], where T_nodes =
 * mpm_mag_trace_nodes(h) (the sum of the instances' n_grid^dim), node_off_k the
 * sum over the instances before k, and node = i + n_grid (j + n_grid l). Codes:
 *   bit 0      the node has mass
 *   bits 1-2   floor branch: 0 untouched, 1 velocity zeroed, 2 sliding
 *   bits 3-5   the walls zero the x, y, z component
 *   bits 6+2j  obstacle j: 0 untouched, 1 set to v_b, 2 sliding
 * Nodes outside the step's active blocks read 0. The rollout clears the trace
 * first. trace: a caller-owned DEVICE buffer of at least n_steps * T_nodes
 * uint16 (EINVAL if smaller), kept until the trace is reset with NULL.
 */
int mpm_mag_set_branch_trace(mpm_mag* h, uint16_t* trace, int64_t elems);
int64_t mpm_mag_trace_nodes(const mpm_mag* h);

/*
 * Scatter fallback counts (instrumentation; the P2G scatter of Eqs. 14-15 and
 * its transpose). A block of 256 particles sums its stencils in an LDS box and
 * registers the box with the coarse grid blocks it overlaps; when the block's
 * box is too large, each wave stages its own box, and when a wave's box is
 * too large as well, or a coarse block's list of boxes is full, values go to
 * global atomics instead. The paths differ in speed, and in results only by
 * rounding: the global atomics add in no fixed order, so a run that takes them
 * need not repeat bit for bit. Fills counts[k] for k < n with the counts of the last
 * rollout or backward on h (0 for k >= 3):
 *   counts[0]  waves that staged their own box (their block's was too large)
 *   counts[1]  waves that added their values with global atomics
 *   counts[2]  box registrations past a coarse block's list capacity
 * The counts are read back when that call finished. EINVAL when h or counts
 * is NULL or n < 0.
 */
int mpm_mag_scatter_stats(const mpm_mag* h, int64_t* counts, int n);

#ifdef __cplusplus
}
#endif

#endif /* MPM_MAG_H */
