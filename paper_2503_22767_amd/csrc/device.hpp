// Device-side building blocks of the magneto-elastic MLS-MPM step for gfx950:
// per-instance parameter record, quadratic B-spline stencil, neo-Hookean and
// hard-magnetic stress (Eq. 7) with its directional derivative, small DxD
// matrix algebra and wave64 / block reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpm {

constexpr int kBlock = 256;       // threads per particle block = particles per chunk
constexpr int kWaves = kBlock / 64;
constexpr int kGridBlock = 512;   // threads of the grid kernels (and grid padding unit)
constexpr int kGridThreadsMax = 1024;   // largest workgroup of the grid update and its transpose

// device error word bits
constexpr int kErrDomain = 1;
constexpr int kErrInvert = 2;
constexpr int kErrNonFinite = 4;
constexpr int kErrStore = 8;   // a grid store entry to be read was not kept (internal)

// The error word of a call keeps its earliest failure, as the key
// (2 n + phase) * 4 + rank: phase 0 is step n's input (the stencils of the
// state it starts from), phase 1 its G2P output (the new state); rank 0 a
// non-finite value, 1 det F <= 0, 2 a stencil outside the grid, 3 a grid store
// entry to be read that was not kept (an internal failure). A key of all
// ones means no failure. (After a first failure later steps can fail as its
// consequence, e.g. an inverted F gives a non-finite stress one step later; the
// earliest one is the cause reported.)
constexpr unsigned long long kNoError = ~0ull;
constexpr int kScatStats = 3;   // scatter fallback counters kept after the error word
__device__ __forceinline__ void report_error(unsigned long long* word, int step, int phase, int flags)
{
    const unsigned long long rank = (flags & kErrNonFinite) ? 0ull
                                  : (flags & kErrInvert)    ? 1ull
                                  : (flags & kErrDomain)    ? 2ull : 3ull;
    atomicMin(word, ((unsigned long long)(2 * step + phase) << 2) | rank);
}

enum LossKind { kFinalMse = 0, kComDisp = 1, kTrajVel = 2, kTipDisp = 3 };

// per-instance loss accumulators (double)
enum Acc { kAccMass = 0, kAccS0, kAccS1, kAccSq, kAccCnt, kAccTip, kAccTraj, kAccCount = 8 };

constexpr int kMaxObst = 4;   // obstacles per instance

template <typename real>
struct InstDev {
    int n_grid, grid_off, n_nodes, n_steps;
    int seg_off, n_seg, seg_steps, periodic;
    int floor_on, wall_cells, loss_kind, clamp_on;
    int floor_noslip, floor_jmax, clamp_imax, chunk_off;
    int n_particles, cb_off, nb;         // first coarse block, coarse blocks per axis
    int trace_off;                       // first node of the instance in a branch trace step
    real dx, inv_dx, dt, kappa_vol;      // kappa_vol = 4 dt / dx^2 * V
    real lam;                            // 4 / dx^2
    real G, K;
    real mass_a, mass_b;                 // particle mass m = mass_a + mass_b phi (Eq. 33 with its floor)
    real inv_mu0, simp_eps, simp_q, damp; // damp = 1 - c dt
    real gdt[3];                         // g dt
    real floor_mu;
    real loss_dir[3];
    // obstacles: solid boundaries of Eq. 18 beyond the floor, at a + vel t
    int n_obst;
    int obst_kind[kMaxObst];             // 1 half-space, 2 sphere, 3 axis-aligned box
    int obst_mode[kMaxObst];             // 0 sliding (Coulomb), 1 no-slip, 2 attached
    real obst_a[kMaxObst][3];            // point of the plane / centre at t = 0
    real obst_b[kMaxObst][3];            // unit outward normal / radius in [0] / half extents
    real obst_vel[kMaxObst][3];          // v_b
    real obst_mu[kMaxObst];
};

struct ChunkDev {
    int inst;   // instance of this chunk
    int count;  // active particles in it (1..kBlock)
};

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------

template <typename real> __device__ __forceinline__ real rfloor(real v);
template <> __device__ __forceinline__ float rfloor<float>(float v) { return floorf(v); }
template <> __device__ __forceinline__ double rfloor<double>(double v) { return floor(v); }

template <typename real> __device__ __forceinline__ bool rfinite(real v) { return isfinite(v); }

// Powers for J^{-2/3} and the SIMP factors. In single precision a^b is taken
// as 2^(b log2 a) with the hardware base-2 logarithm and exponential (about one
// ulp each; J and phi stay near [0.1, 10]); double precision uses pow.
template <typename real> __device__ __forceinline__ real rpow(real a, real b);
template <> __device__ __forceinline__ float rpow<float>(float a, float b)
{
    return __builtin_amdgcn_exp2f(b * __builtin_amdgcn_logf(a));
}
template <> __device__ __forceinline__ double rpow<double>(double a, double b) { return pow(a, b); }

// J^{-2/3}
template <typename real> __device__ __forceinline__ real jpow_m23(real J) { return rpow<real>(J, real(-2) / real(3)); }

// phi^q and q phi^(q-1), with the common q = 3 spelled out
template <typename real>
__device__ __forceinline__ void simp_pow(real phi, real q, real& pq, real& dpq)
{
    if (q == real(3)) {
        pq = phi * phi * phi;
        dpq = real(3) * phi * phi;
    } else {
        pq = rpow(phi, q);
        dpq = q * rpow(phi, q - real(1));
    }
}

template <typename real>
__device__ __forceinline__ void atomic_add(real* p, real v) { unsafeAtomicAdd(p, v); }

// --------------------------------------------------------------------------
// quadratic B-spline stencil (3 nodes per axis from base = floor(x/dx - 1/2))
// --------------------------------------------------------------------------

template <typename real, int D>
struct Stencil {
    int base[D];
    real f[D];      // x/dx - base in [1/2, 3/2)
    real w[D][3];   // weights per axis
    real dw[D][3];  // d w / d x per axis
};

// Builds the stencil of a particle stored relative to its chunk origin: x is
// the position minus org * dx, org the chunk's origin cell. Keeping positions
// small keeps FP32 resolution near 1e-9 of the unit domain instead of 3e-8.
// The base is clamped so the 3^D nodes always lie in the grid; a clamped or
// non-finite coordinate sets the returned error bits.
template <typename real, int D>
__device__ __forceinline__ int make_stencil(const real* x, const int* org, real inv_dx, int n_grid,
                                            Stencil<real, D>& S)
{
    int err = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        real xs = x[k] * inv_dx - real(0.5);
        real f;
        int base;
        if (!rfinite(xs)) {
            err |= kErrNonFinite;
            base = org[k];
            f = real(1);
        } else {
            real b = rfloor(xs);
            base = org[k] + (int)b;
            f = xs - b + real(0.5);
        }
        if (base < 0 || base > n_grid - 3) {
            err |= kErrDomain;
            base = min(max(base, 0), n_grid - 3);
        }
        S.base[k] = base;
        real t0 = real(1.5) - f, t1 = f - real(1), t2 = f - real(0.5);
        S.f[k] = f;
        S.w[k][0] = real(0.5) * t0 * t0;
        S.w[k][1] = real(0.75) - t1 * t1;
        S.w[k][2] = real(0.5) * t2 * t2;
        S.dw[k][0] = -t0 * inv_dx;
        S.dw[k][1] = real(-2) * t1 * inv_dx;
        S.dw[k][2] = t2 * inv_dx;
    }
    return err;
}

// select one of three values by a runtime index 0..2 (register-resident)
template <typename real>
__device__ __forceinline__ real sel3(const real* v, int a)
{
    return a == 0 ? v[0] : (a == 1 ? v[1] : v[2]);
}

// stencil offset o in [0, 3^D) -> per-axis offsets (x fastest)
template <int D>
__device__ __forceinline__ void offset_split(int o, int a[D])
{
    a[0] = o % 3;
    if (D == 2) {
        a[1] = o / 3;
    } else {
        a[1] = (o / 3) % 3;
        a[D - 1] = o / 9;
    }
}

// --------------------------------------------------------------------------
// DxD matrices (row major, registers)
// --------------------------------------------------------------------------

template <typename real, int D>
__device__ __forceinline__ real det(const real F[D][D])
{
    if (D == 2) return F[0][0] * F[1][1] - F[0][1] * F[1][0];
    return F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1])
         - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0])
         + F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
}

// H = F^{-T} (cofactor matrix over det)
template <typename real, int D>
__device__ __forceinline__ void inv_transpose(const real F[D][D], real J, real H[D][D])
{
    real r = real(1) / J;
    if (D == 2) {
        H[0][0] = F[1][1] * r;
        H[0][1] = -F[1][0] * r;
        H[1][0] = -F[0][1] * r;
        H[1][1] = F[0][0] * r;
    } else {
        H[0][0] = (F[1][1] * F[2][2] - F[1][2] * F[2][1]) * r;
        H[0][1] = -(F[1][0] * F[2][2] - F[1][2] * F[2][0]) * r;
        H[0][2] = (F[1][0] * F[2][1] - F[1][1] * F[2][0]) * r;
        H[1][0] = -(F[0][1] * F[2][2] - F[0][2] * F[2][1]) * r;
        H[1][1] = (F[0][0] * F[2][2] - F[0][2] * F[2][0]) * r;
        H[1][2] = -(F[0][0] * F[2][1] - F[0][1] * F[2][0]) * r;
        H[2][0] = (F[0][1] * F[1][2] - F[0][2] * F[1][1]) * r;
        H[2][1] = -(F[0][0] * F[1][2] - F[0][2] * F[1][0]) * r;
        H[2][2] = (F[0][0] * F[1][1] - F[0][1] * F[1][0]) * r;
    }
}

template <typename real, int D>
__device__ __forceinline__ real ddot(const real A[D][D], const real B[D][D])
{
    real s = 0;
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) s += A[i][j] * B[i][j];
    return s;
}

// Elastic stress of Eq. 7: P_e = G J^{-2/3} (F - I1/3 H) + K J (J-1) H, H = F^{-T}.
// 2D is plane strain (F embedded with F33 = 1): I1 = tr(F^T F) + 1, the
// in-plane block is returned. Also returns the pieces the tangent reuses.
template <typename real, int D>
struct StressCtx {
    real J, I1, a;   // a = G J^{-2/3}
    real H[D][D];
};

template <typename real, int D>
__device__ __forceinline__ void elastic_stress(const real F[D][D], real G, real K, real Pe[D][D],
                                               StressCtx<real, D>& c)
{
    c.J = det<real, D>(F);
    inv_transpose<real, D>(F, c.J, c.H);
    c.I1 = ddot<real, D>(F, F) + (D == 2 ? real(1) : real(0));
    c.a = G * jpow_m23(c.J);
    real b = K * c.J * (c.J - real(1));
    real i3 = c.I1 * real(1.0 / 3.0);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) Pe[i][j] = c.a * (F[i][j] - i3 * c.H[i][j]) + b * c.H[i][j];
}

// Directional derivative of P_e along dF (the Hessian of W_e applied to dF;
// symmetric, so it is also its own transpose):
// dP = a [dF - 2/3 (H:dF)(F - I1/3 H) - 2/3 (F:dF) H + I1/3 H dF^T H]
//    + K [(2J-1) J (H:dF) H - J (J-1) H dF^T H]
template <typename real, int D>
__device__ __forceinline__ void elastic_stress_dir(const real F[D][D], real K, const StressCtx<real, D>& c,
                                                   const real dF[D][D], real dP[D][D])
{
    real HdF = ddot<real, D>(c.H, dF);
    real FdF = ddot<real, D>(F, dF);
    real T1[D][D], T[D][D];
    // T = H dF^T H
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            real s = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) s += c.H[i][k] * dF[j][k];
            T1[i][j] = s;
        }
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            real s = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) s += T1[i][k] * c.H[k][j];
            T[i][j] = s;
        }
    real i3 = c.I1 * real(1.0 / 3.0);
    real t23 = real(2.0 / 3.0);
    real kb1 = K * (real(2) * c.J - real(1)) * c.J * HdF;
    real kb2 = K * c.J * (c.J - real(1));
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            real dev = dF[i][j] - t23 * HdF * (F[i][j] - i3 * c.H[i][j]) - t23 * FdF * c.H[i][j] + i3 * T[i][j];
            dP[i][j] = c.a * dev + kb1 * c.H[i][j] - kb2 * T[i][j];
        }
}

// --------------------------------------------------------------------------
// reductions (wave64)
// --------------------------------------------------------------------------

template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Reductions over the 64 lanes of a wave: DPP moves inside each row of 16
// lanes (pairs, quads, half rows, rows; every source lane is in the row, so
// no old value is kept), after which every lane holds its row's result; the
// four rows are then combined on values read from lanes 0, 16, 32 and 48.
// The result is returned to every lane. Every lane must take part.
template <typename Op>
__device__ __forceinline__ int wave_reduce(int v, Op op)
{
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, true));    // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, true));    // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x141, 0xF, 0xF, true));   // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(0, v, 0x140, 0xF, 0xF, true));   // row_mirror
    const int r0 = __builtin_amdgcn_readlane(v, 0), r1 = __builtin_amdgcn_readlane(v, 16);
    const int r2 = __builtin_amdgcn_readlane(v, 32), r3 = __builtin_amdgcn_readlane(v, 48);
    return op(op(r0, r1), op(r2, r3));
}

__device__ __forceinline__ int wave_min(int v)
{
    return wave_reduce(v, [](int a, int b) { return min(a, b); });
}

__device__ __forceinline__ int wave_max(int v)
{
    return wave_reduce(v, [](int a, int b) { return max(a, b); });
}

// maximum of non-negative floats (their bit patterns order like the values)
__device__ __forceinline__ float wave_max_nonneg(float v)
{
    return __int_as_float(wave_max(__float_as_int(v)));
}

// Per-axis minimum and maximum of the stencil bases c[] over the active lanes
// of the wave (every lane must call). The bases lie in [0, 1021], so they are
// reduced as packed 16-bit integers: (x, y), (z, -x), (-y, -z) by minimum,
// three DPP reductions for the six bounds. With no active lane lo = 0x3fffffff
// and hi = -0x3fffffff.
typedef short short2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ int pk_min16(int a, int b)
{
    return __builtin_bit_cast(int, __builtin_elementwise_min(__builtin_bit_cast(short2v, a),
                                                              __builtin_bit_cast(short2v, b)));
}

__device__ __forceinline__ int pack16(int lo, int hi) { return (int)(((unsigned)hi << 16) | ((unsigned)lo & 0xFFFFu)); }

template <int D>
__device__ __forceinline__ void wave_bounds(const int c[D], bool active, int lo[D], int hi[D])
{
    constexpr int kNone = 0x3fff;
    auto mn = [](int a, int b) { return pk_min16(a, b); };
    const int x = active ? c[0] : kNone, nx = active ? -c[0] : kNone;
    const int y = active ? c[1] : kNone, ny = active ? -c[1] : kNone;
    if (D == 3) {
        const int z = active ? c[D - 1] : kNone, nz = active ? -c[D - 1] : kNone;
        const int p0 = wave_reduce(pack16(x, y), mn);
        const int p1 = wave_reduce(pack16(z, nx), mn);
        const int p2 = wave_reduce(pack16(ny, nz), mn);
        lo[0] = (short)(p0 & 0xFFFF);
        lo[1] = p0 >> 16;
        lo[D - 1] = (short)(p1 & 0xFFFF);
        hi[0] = -(p1 >> 16);
        hi[1] = -(short)(p2 & 0xFFFF);
        hi[D - 1] = -(p2 >> 16);
    } else {
        const int p0 = wave_reduce(pack16(x, y), mn);
        const int p1 = wave_reduce(pack16(nx, ny), mn);
        lo[0] = (short)(p0 & 0xFFFF);
        lo[1] = p0 >> 16;
        hi[0] = -(short)(p1 & 0xFFFF);
        hi[1] = -(p1 >> 16);
    }
    if (lo[0] == kNone) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            lo[k] = 0x3fffffff;
            hi[k] = -0x3fffffff;
        }
    }
}

// origin cell of chunk c (particle positions are stored relative to it)
__device__ __forceinline__ void chunk_origin(const int4* corig, int c, int org[3])
{
    const int4 o = corig[c];
    org[0] = o.x;
    org[1] = o.y;
    org[2] = o.z;
}

// field segment of step n
__device__ __forceinline__ int segment_of(int n, int L, int S, int periodic)
{
    int k = n / L;
    return periodic ? k % S : min(k, S - 1);
}

}  // namespace mpm
