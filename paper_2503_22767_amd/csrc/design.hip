// Design front end (Sec. 3.1, Eqs. 23-28): density filter over a neighbour
// matrix built once from the initial positions, Heaviside projection,
// magnetization parametrization with region sharing, and the transpose of
// their Jacobian; and the harmonic stimulus (Sec. 3.1.2, Eqs. 29-30) as a
// one-row-per-step field program with its transpose. C ABI in mpm_mag_design.h.
//
// Layout: the filter's weights form a CSR matrix whose rows follow the
// caller's particle order (row p: the particles within R of p, ordered by cell,
// then by index). Its weights are symmetric bit for bit (the same difference,
// squared and summed in the same order, from both ends), so the transpose of
// the normalized filter is the same matrix applied to g / s. Rows are reduced
// by groups of kRowLanes lanes reading consecutive entries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "mpm_mag_design.h"
#include "sort.hpp"

namespace mpm {
namespace fe {

constexpr int kRowLanes = 4;                     // lanes per matrix row
constexpr int kRowsPerBlock = kBlock / kRowLanes;
constexpr int kMaxCellBits = 24;                 // cell keys of the binning
constexpr int kBoxBlocks = 1024;                 // blocks of the bounding-box pass
constexpr int kChunk = 2048;                     // members per workgroup of the chunked region sums
constexpr int kChunkedMinMean = 2048;            // mean region size from which region sums are chunked
constexpr int kMaxCopies = 4096;                 // design copies (tasks sharing the design)

enum { kBadNonFinite = 1, kBadRegion = 2 };

// --------------------------------------------------------------- build passes

// per-block min and max of every coordinate; non-finite coordinates set a flag
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_bbox(const real* x0, int64_t n, real* part, int* bad)
{
    __shared__ real s_lo[D][kBlock], s_hi[D][kBlock];
    const int t = threadIdx.x;
    real lo[D], hi[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lo[k] = INFINITY;
        hi[k] = -INFINITY;
    }
    bool fin = true;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + t; i < n; i += (int64_t)gridDim.x * kBlock)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const real v = x0[i * D + k];
            fin = fin && isfinite(v);
            lo[k] = fmin(lo[k], v);
            hi[k] = fmax(hi[k], v);
        }
    if (!fin) atomicOr(bad, kBadNonFinite);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        s_lo[k][t] = lo[k];
        s_hi[k][t] = hi[k];
    }
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if (t < off)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                s_lo[k][t] = fmin(s_lo[k][t], s_lo[k][t + off]);
                s_hi[k][t] = fmax(s_hi[k][t], s_hi[k][t + off]);
            }
        __syncthreads();
    }
    if (t == 0)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            part[(int64_t)blockIdx.x * 2 * D + k] = s_lo[k][0];
            part[(int64_t)blockIdx.x * 2 * D + D + k] = s_hi[k][0];
        }
}

// Binning grid. Cells are computed in double whatever the element type, so
// that the cell edge's margin over R (1e-5) exceeds the rounding even with
// millions of cells along one axis.
struct Cells {
    double lo[3];
    double inv_c;   // 1 / cell edge
    int nc[3];      // cells per axis
};

template <typename real, int D>
__device__ __forceinline__ void cell_of(const Cells& cg, const real* x, int c[3])
{
    c[2] = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double v = floor(((double)x[k] - cg.lo[k]) * cg.inv_c);
        c[k] = v < 0 ? 0 : (v >= cg.nc[k] ? cg.nc[k] - 1 : (int)v);
    }
}

template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_cell_keys(const real* x0, int64_t n, Cells cg, uint32_t* keys,
                                                      uint32_t* vals)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    real x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = x0[i * D + k];
    int c[3];
    cell_of<real, D>(cg, x, c);
    keys[i] = (uint32_t)c[0] + (uint32_t)cg.nc[0] * ((uint32_t)c[1] + (uint32_t)cg.nc[1] * (uint32_t)c[2]);
    vals[i] = (uint32_t)i;
}

// first and one-past-last sorted position of every occupied cell (the arrays
// start zeroed, so empty cells are empty ranges)
__global__ __launch_bounds__(kBlock) void k_cell_ranges(const uint32_t* keys, int64_t n, int* cell_lo, int* cell_hi)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint32_t k = keys[j];
    if (j == 0 || keys[j - 1] != k) cell_lo[k] = (int)j;
    if (j == n - 1 || keys[j + 1] != k) cell_hi[k] = (int)(j + 1);
}

// positions in sorted order, so the neighbour scans read them coalesced
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_sorted_pos(const real* x0, const uint32_t* vals, int64_t n, real* xs)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int64_t i = vals[j];
#pragma unroll
    for (int k = 0; k < D; ++k) xs[j * D + k] = x0[i * D + k];
}

// Visits the particles within the radius of sorted particle j, cells in a
// fixed order, sorted order within a cell: fn(k, d2).
template <typename real, int D, typename Fn>
__device__ __forceinline__ void for_neighbours(const real* xs, const uint32_t* keys, const int* cell_lo,
                                               const int* cell_hi, const Cells& cg, real r2, int64_t j, Fn fn)
{
    real xj[D];
#pragma unroll
    for (int k = 0; k < D; ++k) xj[k] = xs[j * D + k];
    const uint32_t key = keys[j];
    int c[3];
    c[0] = (int)(key % (uint32_t)cg.nc[0]);
    c[1] = (int)((key / (uint32_t)cg.nc[0]) % (uint32_t)cg.nc[1]);
    c[2] = (int)(key / ((uint32_t)cg.nc[0] * (uint32_t)cg.nc[1]));
    for (int dz = (D == 3 ? -1 : 0); dz <= (D == 3 ? 1 : 0); ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int cx = c[0] + dx, cy = c[1] + dy, cz = c[2] + dz;
                if (cx < 0 || cy < 0 || cz < 0 || cx >= cg.nc[0] || cy >= cg.nc[1] || cz >= cg.nc[2]) continue;
                const uint32_t nk = (uint32_t)cx + (uint32_t)cg.nc[0] * ((uint32_t)cy + (uint32_t)cg.nc[1] * (uint32_t)cz);
                const int e = cell_hi[nk];
                for (int k = cell_lo[nk]; k < e; ++k) {
                    real d2 = 0;
#pragma unroll
                    for (int q = 0; q < D; ++q) {
                        const real d = xs[(int64_t)k * D + q] - xj[q];
                        d2 += d * d;
                    }
                    if (d2 < r2) fn(k, d2);
                }
            }
}

template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_count(const real* xs, const uint32_t* keys, const uint32_t* vals,
                                                  const int* cell_lo, const int* cell_hi, Cells cg, real r2,
                                                  int64_t n, uint32_t* cnt, unsigned long long* total)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t c = 0;
    if (j < n) {
        for_neighbours<real, D>(xs, keys, cell_lo, cell_hi, cg, r2, j, [&](int, real) { ++c; });
        cnt[vals[j]] = c;
    }
    // one 64-bit total per wave, to refuse matrices beyond 32-bit offsets
    unsigned long long s = c;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(total, s);
}

template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_fill(const real* xs, const uint32_t* keys, const uint32_t* vals,
                                                 const int* cell_lo, const int* cell_hi, Cells cg, real r2,
                                                 real inv_r, int64_t n, const uint32_t* row_ptr, int* col, real* w,
                                                 real* inv_s)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const int64_t p = vals[j];
    int64_t o = row_ptr[p];
    real s = 0;
    for_neighbours<real, D>(xs, keys, cell_lo, cell_hi, cg, r2, j, [&](int k, real d2) {
        const real wk = real(1) - sqrt(d2) * inv_r;
        col[o] = (int)vals[k];
        w[o] = wk;
        ++o;
        s += wk;
    });
    inv_s[p] = real(1) / s;   // the particle itself weighs 1, so s >= 1
}

__global__ __launch_bounds__(kBlock) void k_region_keys(const int32_t* region, int64_t n, int n_regions,
                                                        uint32_t* keys, uint32_t* vals, int* bad)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int32_t r = region[i];
    if (r < 0 || r >= n_regions) atomicOr(bad, kBadRegion);
    keys[i] = (uint32_t)min(max(r, 0), n_regions - 1);
    vals[i] = (uint32_t)i;
}

// ------------------------------------------------------------ forward, backward

// sum over row p of w_pq v_q, reduced over the row's kRowLanes lanes (all of
// them call it; lanes of rows past the end pass p = -1)
template <typename real>
__device__ __forceinline__ real row_dot(const uint32_t* row_ptr, const int* col, const real* w, const real* v,
                                        int64_t p, int g)
{
    real acc = 0;
    if (p >= 0) {
        const int64_t e = row_ptr[p + 1];
        for (int64_t k = row_ptr[p] + g; k < e; k += kRowLanes) acc += w[k] * v[col[k]];
    }
#pragma unroll
    for (int off = kRowLanes / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kRowLanes);
    return acc;
}

template <typename real>
struct FwdParams {
    real beta;
    real inv_2t;    // 1 / (2 tanh(beta / 2))
    real t_half;    // tanh(beta / 2)
    real br_max;
    real delta;
};

template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_forward(const uint32_t* row_ptr, const int* col, const real* w,
                                                    const real* inv_s, int64_t n, const real* phi,
                                                    const int32_t* region, const real* br_mag, const real* zeta,
                                                    FwdParams<real> fp, int copies, real* phit, real* density,
                                                    real* br)
{
    const int g = threadIdx.x % kRowLanes;
    const int64_t p0 = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kRowLanes;
    const int64_t p = p0 < n ? p0 : -1;
    const real acc = row_dot<real>(row_ptr, col, w, phi, p, g);
    if (p < 0) return;
    if (g == 0) {
        const real pt = acc * inv_s[p];
        phit[p] = pt;
        const real dp = (fp.t_half + tanh(fp.beta * (pt - real(0.5)))) * fp.inv_2t;
        for (int c = 0; c < copies; ++c) density[c * n + p] = dp;
    }
    if (g < D) {
        const int64_t m = region ? (int64_t)region[p] : p;
        real z2 = fp.delta;
#pragma unroll
        for (int k = 0; k < D; ++k) z2 += zeta[m * D + k] * zeta[m * D + k];
        const real b = fp.br_max * br_mag[m] * zeta[m * D + g] / sqrt(z2);
        for (int c = 0; c < copies; ++c) br[(c * n + p) * D + g] = b;
    }
}

// gradient of particle p summed over the copies of the design (tasks that
// share it, Eq. 35): component k of [copies][n][D]
template <typename real, int D>
__device__ __forceinline__ double copies_sum(const real* g, int64_t n, int copies, int64_t p, int k)
{
    double s = 0.0;
    for (int c = 0; c < copies; ++c) s += (double)g[(c * n + p) * D + k];
    return s;
}

// u_p = g_density_p H'(phit_p) / s_p
template <typename real>
__global__ __launch_bounds__(kBlock) void k_scale(const real* g_density, const real* phit, const real* inv_s,
                                                  int64_t n, int copies, FwdParams<real> fp, real* u)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    const real th = tanh(fp.beta * (phit[p] - real(0.5)));
    const real gd = (real)copies_sum<real, 1>(g_density, n, copies, p, 0);
    u[p] = gd * fp.beta * (real(1) - th * th) * fp.inv_2t * inv_s[p];
}

// g_phi = W u (W symmetric)
template <typename real>
__global__ __launch_bounds__(kBlock) void k_spmv(const uint32_t* row_ptr, const int* col, const real* w, int64_t n,
                                                 const real* u, real* out)
{
    const int g = threadIdx.x % kRowLanes;
    const int64_t p0 = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kRowLanes;
    const int64_t p = p0 < n ? p0 : -1;
    const real acc = row_dot<real>(row_ptr, col, w, u, p, g);
    if (p >= 0 && g == 0) out[p] = acc;
}

// region sums G_m of g_br over the members, sorted by region (many small
// regions): each wave sums its runs of equal region and the run tails add them
// to the accumulators
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_region_sums(const uint32_t* reg_sorted, const uint32_t* members,
                                                        int64_t n, int copies, const real* g_br, double* G)
{
    const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = j < n;
    const int r = valid ? (int)reg_sorted[j] : -1;
    double v[D];
    const int64_t p = valid ? (int64_t)members[j] : 0;
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = valid ? copies_sum<real, D>(g_br, n, copies, p, k) : 0.0;
    // inclusive scan inside runs of equal r
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int ro = __shfl_up(r, off, 64);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double vo = __shfl_up(v[k], off, 64);
            if (lane >= off && ro == r) v[k] += vo;
        }
    }
    const int rn = __shfl_down(r, 1, 64);
    const bool tail = valid && (lane == 63 || rn != r);
    if (tail)
#pragma unroll
        for (int k = 0; k < D; ++k) atomicAdd(&G[(int64_t)r * D + k], v[k]);
}

// Chunked region sums (few, large regions): chunk c covers sorted members
// [c_lo[c], c_hi[c]) of one region; one workgroup sums it in double and writes
// its partial, with no atomics.
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_region_chunks(const uint32_t* members, const int64_t* c_lo,
                                                          const int64_t* c_hi, int64_t n, int copies,
                                                          const real* g_br, double* part)
{
    __shared__ double s_w[kWaves][D];
    const int t = threadIdx.x;
    const int64_t lo = c_lo[blockIdx.x], hi = c_hi[blockIdx.x];
    double v[D];
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = 0.0;
    for (int c = 0; c < copies; ++c) {   // copies outermost: the inner loop stays a plain gather
        const real* gc = g_br + (int64_t)c * n * D;
        for (int64_t j = lo + t; j < hi; j += kBlock) {
            const int64_t p = members[j];
#pragma unroll
            for (int k = 0; k < D; ++k) v[k] += (double)gc[p * D + k];
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
    if ((t & 63) == 0)
#pragma unroll
        for (int k = 0; k < D; ++k) s_w[t >> 6][k] = v[k];
    __syncthreads();
    if (t < D) {
        double a = 0.0;
        for (int w2 = 0; w2 < kWaves; ++w2) a += s_w[w2][t];
        part[(int64_t)blockIdx.x * D + t] = a;
    }
}

// region gradients from G_m: g_mag = Br_max b . G, g_zeta = Br_max Br_m (G / r - zeta (zeta . G) / r^3)
template <typename real, int D>
__device__ __forceinline__ void region_grad(const real* br_mag, const real* zeta, real br_max, real delta,
                                            int64_t m, const double G[D], real* g_mag, real* g_zeta)
{
    double z[D], z2 = (double)delta, zg = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        z[k] = (double)zeta[m * D + k];
        z2 += z[k] * z[k];
        zg += z[k] * G[k];
    }
    const double r = sqrt(z2), ir = 1.0 / r, ir3 = ir * ir * ir;
    if (g_mag) g_mag[m] = (real)((double)br_max * zg * ir);
    if (g_zeta) {
        const double a = (double)br_max * (double)br_mag[m];
#pragma unroll
        for (int k = 0; k < D; ++k) g_zeta[m * D + k] = (real)(a * (G[k] * ir - z[k] * zg * ir3));
    }
}

// region gradients from the accumulated G_m (atomic path)
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_region_grads(const double* G, int64_t n_m, const real* br_mag,
                                                         const real* zeta, real br_max, real delta, real* g_mag,
                                                         real* g_zeta)
{
    const int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (m >= n_m) return;
    double g[D];
#pragma unroll
    for (int k = 0; k < D; ++k) g[k] = G[m * D + k];
    region_grad<real, D>(br_mag, zeta, br_max, delta, m, g, g_mag, g_zeta);
}

// region gradients from the chunk partials [m_chunk[m], m_chunk[m + 1]) of each
// region (chunked path): one wave per region, lanes striding over the
// partials, a fixed reduction order
template <typename real, int D>
__global__ __launch_bounds__(64) void k_region_chunk_grads(const double* part, const int* m_chunk, int64_t n_m,
                                                           const real* br_mag, const real* zeta, real br_max,
                                                           real delta, real* g_mag, real* g_zeta)
{
    const int64_t m = blockIdx.x;
    const int lane = threadIdx.x;
    double g[D];
#pragma unroll
    for (int k = 0; k < D; ++k) g[k] = 0.0;
    for (int c = m_chunk[m] + lane; c < m_chunk[m + 1]; c += 64)
#pragma unroll
        for (int k = 0; k < D; ++k) g[k] += part[(int64_t)c * D + k];
#pragma unroll
    for (int k = 0; k < D; ++k)
        for (int off = 32; off > 0; off >>= 1) g[k] += __shfl_xor(g[k], off, 64);
    if (lane != 0) return;
    region_grad<real, D>(br_mag, zeta, br_max, delta, m, g, g_mag, g_zeta);
}

// every particle its own region: G_p = g_br_p
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_particle_grads(const real* g_br, int64_t n, int copies,
                                                           const real* br_mag, const real* zeta, real br_max,
                                                           real delta, real* g_mag, real* g_zeta)
{
    const int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (p >= n) return;
    double g[D];
#pragma unroll
    for (int k = 0; k < D; ++k) g[k] = copies_sum<real, D>(g_br, n, copies, p, k);
    region_grad<real, D>(br_mag, zeta, br_max, delta, p, g, g_mag, g_zeta);
}

static int grid_of(int64_t n, int per = kBlock) { return (int)((n + per - 1) / per); }

// ------------------------------------------------------ harmonic stimulus

struct Harm {
    int n_inst, T;
    double dt, b_max, f_min, f_max, delta;
};

template <int D, typename real>
__device__ __forceinline__ double orient(const real* eta, int k, double delta, double b[D], double* r)
{
    double r2 = delta;
#pragma unroll
    for (int c = 0; c < D; ++c) {
        b[c] = (double)eta[k * D + c];
        r2 += b[c] * b[c];
    }
    *r = sqrt(r2);
#pragma unroll
    for (int c = 0; c < D; ++c) b[c] /= *r;
    return r2;
}

// row (k, n) of the program: B_max B_a sin(2 pi fbar t_n) b (Eqs. 29-30)
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_harmonic(const real* b_a, const real* f, const real* eta, Harm hp,
                                                     real* prog)
{
    const int64_t idx = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (int64_t)hp.n_inst * hp.T) return;
    const int k = (int)(idx / hp.T), n = (int)(idx % hp.T);
    double b[D], r;
    orient<D>(eta, k, hp.delta, b, &r);
    const double fbar = (hp.f_max - hp.f_min) * (double)f[k] + hp.f_min;
    const double a = hp.b_max * (double)b_a[k] * sin(2.0 * M_PI * fbar * ((double)n * hp.dt));
#pragma unroll
    for (int c = 0; c < D; ++c) prog[idx * D + c] = (real)(a * b[c]);
}

// one workgroup per instance: sums over the steps of s_n q_n, c_n t_n q_n and
// s_n G_n (q_n = b . G_n), reduced in a fixed order
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_harmonic_t(const real* b_a, const real* f, const real* eta, Harm hp,
                                                       const real* g, real* g_ba, real* g_f, real* g_eta)
{
    constexpr int NV = 2 + D;
    __shared__ double s_w[kWaves][NV];
    const int k = blockIdx.x, t = threadIdx.x;
    double b[D], r;
    orient<D>(eta, k, hp.delta, b, &r);
    const double w = 2.0 * M_PI * ((hp.f_max - hp.f_min) * (double)f[k] + hp.f_min);
    double acc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = 0.0;
    for (int n = t; n < hp.T; n += kBlock) {
        const double tn = (double)n * hp.dt;
        const double sn = sin(w * tn), cn = cos(w * tn);
        const real* G = g + ((int64_t)k * hp.T + n) * D;
        double q = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) {
            const double gc = (double)G[c];
            q += b[c] * gc;
            acc[2 + c] += sn * gc;
        }
        acc[0] += sn * q;
        acc[1] += cn * tn * q;
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
        for (int off = 32; off > 0; off >>= 1) acc[v] += __shfl_xor(acc[v], off, 64);
    if ((t & 63) == 0)
#pragma unroll
        for (int v = 0; v < NV; ++v) s_w[t >> 6][v] = acc[v];
    __syncthreads();
    if (t != 0) return;
    double tot[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        tot[v] = 0.0;
        for (int w2 = 0; w2 < kWaves; ++w2) tot[v] += s_w[w2][v];
    }
    const double ba = (double)b_a[k];
    if (g_ba) g_ba[k] = (real)(hp.b_max * tot[0]);
    if (g_f) g_f[k] = (real)(hp.b_max * ba * 2.0 * M_PI * (hp.f_max - hp.f_min) * tot[1]);
    if (g_eta) {
        // J_b^T S with J_b = I / r - eta eta^T / r^3, eta = r b
        double bs = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) bs += b[c] * tot[2 + c];
#pragma unroll
        for (int c = 0; c < D; ++c) g_eta[k * D + c] = (real)(hp.b_max * ba * (tot[2 + c] - b[c] * bs) / r);
    }
}

template <typename real, int D>
int harmonic_launch(const mpm_mag_harmonic_desc* d, hipStream_t s, const void* b_a, const void* f, const void* eta,
                    const void* g, void* out0, void* out1, void* out2, bool backward)
{
    Harm hp{d->n_inst, d->n_steps, d->dt, d->b_max, d->f_min, d->f_max, d->delta};
    if (backward)
        hipLaunchKernelGGL((k_harmonic_t<real, D>), dim3(d->n_inst), dim3(kBlock), 0, s, (const real*)b_a,
                           (const real*)f, (const real*)eta, hp, (const real*)g, (real*)out0, (real*)out1,
                           (real*)out2);
    else
        hipLaunchKernelGGL((k_harmonic<real, D>), dim3((unsigned)grid_of((int64_t)d->n_inst * d->n_steps)),
                           dim3(kBlock), 0, s, (const real*)b_a, (const real*)f, (const real*)eta, hp, (real*)out0);
    return hipGetLastError() == hipSuccess ? MPM_MAG_OK : MPM_MAG_EHIP;
}

// ------------------------------------------------------- optimizer update

// One Adam step (Kingma and Ba 2015) on n variables, then the bound map:
// m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
// p = clamp(p - lr (m c1) / (sqrt(v c2) + eps), lo, hi), c1, c2 the bias
// corrections. 1 - b1 and 1 - b2 come from the host in double: formed in FP32
// from b2 = 0.999 the difference would be off by 1e-5.
template <typename real>
__global__ __launch_bounds__(kBlock) void k_adam(int64_t n, real* p, const real* g, real* m, real* v, real lr,
                                                 real b1, real b2, real one_b1, real one_b2, real eps, real c1,
                                                 real c2, real lo, real hi)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const real gi = g[i];
    const real mi = b1 * m[i] + one_b1 * gi;
    const real vi = b2 * v[i] + one_b2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const real q = p[i] - lr * (mi * c1) / (sqrt(vi * c2) + eps);
    p[i] = q < lo ? lo : (q > hi ? hi : q);
}

// ------------------------------------------------------------------- handle

struct Base {
    virtual ~Base() = default;
    virtual int forward(hipStream_t s, const void* phi, double beta, const void* br_mag, const void* zeta,
                        double br_max, double delta, int copies, void* density, void* br) = 0;
    virtual int backward(hipStream_t s, int copies, const void* g_density, const void* g_br, void* g_phi,
                         void* g_mag, void* g_zeta) = 0;
    int64_t nnz = 0;
    std::string err;
};

#define FE_HIP(expr)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(MPM_MAG_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)


template <typename real, int D>
struct Design final : Base {
    int64_t N = 0, n_m = 0;
    bool has_region = false;
    uint32_t* row_ptr = nullptr;   // [N + 1]
    int* col = nullptr;            // [nnz]
    real* w = nullptr;             // [nnz]
    real* inv_s = nullptr;         // [N]
    int32_t* region = nullptr;     // [N] copy, or null
    uint32_t* reg_sorted = nullptr, *members = nullptr;   // [N] by region
    real* phit = nullptr;          // [N] of the last forward
    real* mag = nullptr;           // [n_m] and [n_m][D] of the last forward
    real* zeta = nullptr;
    real* u = nullptr;             // [N] scratch of backward
    double* G = nullptr;           // [n_m][D] region sums, or [n_chunks][D] chunk partials
    int64_t *c_lo = nullptr, *c_hi = nullptr;   // chunked region sums: member range of each chunk
    int* m_chunk = nullptr;        // [n_m + 1] first chunk of each region
    int n_chunks = 0;
    FwdParams<real> fp{};
    bool have_fwd = false;
    std::vector<void*> allocs;
    std::vector<void*> scratch;    // build-only buffers, released at the end of init

    ~Design() override
    {
        for (void* p : allocs) (void)hipFree(p);
    }

    int fail(int code, const std::string& m)
    {
        err = m;
        return code;
    }

    template <typename T>
    int dalloc(T** p, size_t count)
    {
        if (hipMalloc((void**)p, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return fail(MPM_MAG_ENOMEM, "device allocation");
        }
        allocs.push_back(*p);
        return MPM_MAG_OK;
    }

    // stable radix sort of (keys, vals) over `bits` key bits; the result ends in k[0], v[0]
    int radix_sort(hipStream_t s, uint32_t* k[2], uint32_t* v[2], int64_t n, int bits)
    {
        const int nb = grid_of(n, kSortTile);
        uint32_t* hist = nullptr;
        int st = dalloc(&hist, (size_t)256 * nb);
        if (st) return st;
        scratch.push_back(hist);
        int cur = 0;
        for (int shift = 0; shift < bits; shift += 8) {
            hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kBlock), 0, s, (const uint32_t*)k[cur], n, shift, hist, nb);
            hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, s, hist, (int64_t)256 * nb);
            hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kBlock), 0, s, (const uint32_t*)k[cur],
                               (const uint32_t*)v[cur], k[1 - cur], v[1 - cur], n, shift, (const uint32_t*)hist, nb);
            cur = 1 - cur;
        }
        FE_HIP(hipGetLastError());
        if (cur == 1) {
            FE_HIP(hipMemcpyAsync(k[0], k[1], sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
            FE_HIP(hipMemcpyAsync(v[0], v[1], sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
        }
        return MPM_MAG_OK;
    }

    int init(int64_t n, const real* x0, double radius, const int32_t* reg, int n_regions, hipStream_t s)
    {
        N = n;
        has_region = reg != nullptr;
        n_m = has_region ? n_regions : n;
        int* bad = nullptr;
        int st = dalloc(&bad, 1);
        if (st) return st;
        FE_HIP(hipMemsetAsync(bad, 0, sizeof(int), s));
        // bounding box
        const int nbb = (int)std::min<int64_t>(kBoxBlocks, grid_of(n));
        real* part = nullptr;
        if ((st = dalloc(&part, (size_t)nbb * 2 * D))) return st;
        hipLaunchKernelGGL((k_bbox<real, D>), dim3(nbb), dim3(kBlock), 0, s, x0, n, part, bad);
        FE_HIP(hipGetLastError());
        std::vector<real> ph((size_t)nbb * 2 * D);
        int bad_h = 0;
        FE_HIP(hipMemcpyAsync(ph.data(), part, sizeof(real) * ph.size(), hipMemcpyDeviceToHost, s));
        FE_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
        FE_HIP(hipStreamSynchronize(s));
        if (bad_h & kBadNonFinite) return fail(MPM_MAG_ENONFINITE, "non-finite initial position");
        double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
        for (int k = 0; k < D; ++k) {
            lo[k] = INFINITY;
            hi[k] = -INFINITY;
            for (int b = 0; b < nbb; ++b) {
                lo[k] = std::min(lo[k], (double)ph[(size_t)b * 2 * D + k]);
                hi[k] = std::max(hi[k], (double)ph[(size_t)b * 2 * D + D + k]);
            }
        }
        // cells of edge >= R (slightly above it, so a pair within R never lies
        // two cells apart after rounding), grown until the keys fit
        double c = radius * (1.0 + 1e-5);
        Cells cg{};
        for (;;) {
            double cells = 1;
            for (int k = 0; k < 3; ++k) {
                cg.nc[k] = k < D ? (int)std::min(1e9, std::floor((hi[k] - lo[k]) / c) + 1) : 1;
                cells *= cg.nc[k];
            }
            if (cells <= (double)(1u << kMaxCellBits)) break;
            c *= 1.25;
        }
        for (int k = 0; k < 3; ++k) cg.lo[k] = k < D ? lo[k] : 0.0;
        cg.inv_c = 1.0 / c;
        const uint32_t n_cells = (uint32_t)cg.nc[0] * cg.nc[1] * cg.nc[2];
        int bits = 8;
        while (bits < 32 && ((uint64_t)1 << bits) < n_cells) bits += 8;
        // bin and sort by cell
        uint32_t *k[2], *v[2];
        for (int b = 0; b < 2; ++b) {
            if ((st = dalloc(&k[b], n)) || (st = dalloc(&v[b], n))) return st;
        }
        hipLaunchKernelGGL((k_cell_keys<real, D>), dim3(grid_of(n)), dim3(kBlock), 0, s, x0, n, cg, k[0], v[0]);
        FE_HIP(hipGetLastError());
        if ((st = radix_sort(s, k, v, n, bits))) return st;
        int *cell_lo = nullptr, *cell_hi = nullptr;
        if ((st = dalloc(&cell_lo, n_cells)) || (st = dalloc(&cell_hi, n_cells))) return st;
        FE_HIP(hipMemsetAsync(cell_lo, 0, sizeof(int) * n_cells, s));
        FE_HIP(hipMemsetAsync(cell_hi, 0, sizeof(int) * n_cells, s));
        hipLaunchKernelGGL(k_cell_ranges, dim3(grid_of(n)), dim3(kBlock), 0, s, (const uint32_t*)k[0], n, cell_lo,
                           cell_hi);
        real* xs = nullptr;
        if ((st = dalloc(&xs, (size_t)n * D))) return st;
        hipLaunchKernelGGL((k_sorted_pos<real, D>), dim3(grid_of(n)), dim3(kBlock), 0, s, x0, (const uint32_t*)v[0],
                           n, xs);
        // rows: count, offsets, fill
        unsigned long long* total = nullptr;
        if ((st = dalloc(&row_ptr, n + 1)) || (st = dalloc(&total, 1))) return st;
        FE_HIP(hipMemsetAsync(row_ptr, 0, sizeof(uint32_t) * (n + 1), s));
        FE_HIP(hipMemsetAsync(total, 0, sizeof(unsigned long long), s));
        const real r2 = (real)(radius * radius);
        hipLaunchKernelGGL((k_count<real, D>), dim3(grid_of(n)), dim3(kBlock), 0, s, (const real*)xs,
                           (const uint32_t*)k[0], (const uint32_t*)v[0], (const int*)cell_lo, (const int*)cell_hi, cg,
                           r2, n, row_ptr, total);
        FE_HIP(hipGetLastError());
        unsigned long long tot = 0;
        FE_HIP(hipMemcpyAsync(&tot, total, sizeof(tot), hipMemcpyDeviceToHost, s));
        FE_HIP(hipStreamSynchronize(s));
        if (tot > 0x7fffffffull) return fail(MPM_MAG_ENOMEM, "neighbour matrix beyond 2^31 - 1 entries");
        nnz = (int64_t)tot;
        hipLaunchKernelGGL(k_scan_exclusive, dim3(1), dim3(1024), 0, s, row_ptr, n + 1);
        if ((st = dalloc(&col, nnz)) || (st = dalloc(&w, nnz)) || (st = dalloc(&inv_s, n))) return st;
        hipLaunchKernelGGL((k_fill<real, D>), dim3(grid_of(n)), dim3(kBlock), 0, s, (const real*)xs,
                           (const uint32_t*)k[0], (const uint32_t*)v[0], (const int*)cell_lo, (const int*)cell_hi, cg,
                           r2, (real)(1.0 / radius), n, (const uint32_t*)row_ptr, col, w, inv_s);
        FE_HIP(hipGetLastError());
        // regions: a copy of the map and the members sorted by region
        if (has_region) {
            if ((st = dalloc(&region, n))) return st;
            FE_HIP(hipMemcpyAsync(region, reg, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
            hipLaunchKernelGGL(k_region_keys, dim3(grid_of(n)), dim3(kBlock), 0, s, (const int32_t*)region, n,
                               n_regions, k[0], v[0], bad);
            FE_HIP(hipGetLastError());
            int rbits = 8;
            while (rbits < 32 && ((uint64_t)1 << rbits) < (uint64_t)n_regions) rbits += 8;
            if ((st = radix_sort(s, k, v, n, rbits))) return st;
            if ((st = dalloc(&reg_sorted, n)) || (st = dalloc(&members, n))) return st;
            FE_HIP(hipMemcpyAsync(reg_sorted, k[0], sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
            FE_HIP(hipMemcpyAsync(members, v[0], sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
            if (n / n_m >= kChunkedMinMean) {
                // few large regions: chunks of at most kChunk members inside each region
                std::vector<uint32_t> rs((size_t)n);
                FE_HIP(hipMemcpyAsync(rs.data(), reg_sorted, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, s));
                FE_HIP(hipStreamSynchronize(s));
                std::vector<int64_t> lo_h, hi_h;
                std::vector<int> mc((size_t)n_m + 1, 0);
                int64_t j = 0;
                for (int64_t m = 0; m < n_m; ++m) {
                    mc[m] = (int)lo_h.size();
                    int64_t e = j;
                    while (e < n && rs[e] == (uint32_t)m) ++e;
                    for (int64_t a = j; a < e; a += kChunk) {
                        lo_h.push_back(a);
                        hi_h.push_back(std::min<int64_t>(e, a + kChunk));
                    }
                    j = e;
                }
                mc[n_m] = (int)lo_h.size();
                n_chunks = (int)lo_h.size();
                if ((st = dalloc(&c_lo, std::max(1, n_chunks))) || (st = dalloc(&c_hi, std::max(1, n_chunks))) ||
                    (st = dalloc(&m_chunk, n_m + 1)) || (st = dalloc(&G, (size_t)std::max(1, n_chunks) * D)))
                    return st;
                FE_HIP(hipMemcpy(c_lo, lo_h.data(), sizeof(int64_t) * n_chunks, hipMemcpyHostToDevice));
                FE_HIP(hipMemcpy(c_hi, hi_h.data(), sizeof(int64_t) * n_chunks, hipMemcpyHostToDevice));
                FE_HIP(hipMemcpy(m_chunk, mc.data(), sizeof(int) * (n_m + 1), hipMemcpyHostToDevice));
            } else if ((st = dalloc(&G, (size_t)n_m * D))) {
                return st;
            }
        }
        if ((st = dalloc(&phit, n)) || (st = dalloc(&u, n)) || (st = dalloc(&mag, n_m)) ||
            (st = dalloc(&zeta, (size_t)n_m * D)))
            return st;
        FE_HIP(hipMemcpyAsync(&bad_h, bad, sizeof(int), hipMemcpyDeviceToHost, s));
        FE_HIP(hipStreamSynchronize(s));
        if (bad_h & kBadRegion) return fail(MPM_MAG_EINVAL, "a region id outside [0, n_regions)");
        // the build's scratch goes back now
        for (void* p : {(void*)part, (void*)k[0], (void*)k[1], (void*)v[0], (void*)v[1], (void*)cell_lo,
                        (void*)cell_hi, (void*)xs, (void*)total, (void*)bad})
            release(p);
        for (void* p : scratch) release(p);
        scratch.clear();
        return MPM_MAG_OK;
    }

    void release(void* p)
    {
        for (auto& a : allocs)
            if (a == p) {
                (void)hipFree(a);
                a = allocs.back();
                allocs.pop_back();
                return;
            }
    }

    int forward(hipStream_t s, const void* phi, double beta, const void* br_mag, const void* zeta_in,
                double br_max, double delta, int copies, void* density, void* br) override
    {
        err.clear();
        have_fwd = false;
        if (!phi || !br_mag || !zeta_in || !density || !br) return fail(MPM_MAG_EINVAL, "null array");
        if (copies < 1 || copies > kMaxCopies) return fail(MPM_MAG_EINVAL, "copies must be in [1, 4096]");
        if (!(beta > 0) || !std::isfinite(beta)) return fail(MPM_MAG_EINVAL, "beta must be positive");
        if (!(delta >= 0) || !std::isfinite(br_max)) return fail(MPM_MAG_EINVAL, "bad br_max or delta");
        const double th = std::tanh(0.5 * beta);
        fp.beta = (real)beta;
        fp.t_half = (real)th;
        fp.inv_2t = (real)(1.0 / (2.0 * th));
        fp.br_max = (real)br_max;
        fp.delta = (real)delta;
        FE_HIP(hipMemcpyAsync(mag, br_mag, sizeof(real) * n_m, hipMemcpyDeviceToDevice, s));
        FE_HIP(hipMemcpyAsync(zeta, zeta_in, sizeof(real) * n_m * D, hipMemcpyDeviceToDevice, s));
        hipLaunchKernelGGL((k_forward<real, D>), dim3(grid_of(N, kRowsPerBlock)), dim3(kBlock), 0, s,
                           (const uint32_t*)row_ptr, (const int*)col, (const real*)w, (const real*)inv_s, N,
                           (const real*)phi, (const int32_t*)region, (const real*)mag, (const real*)zeta, fp, copies,
                           phit, (real*)density, (real*)br);
        FE_HIP(hipGetLastError());
        have_fwd = true;
        return MPM_MAG_OK;
    }

    int backward(hipStream_t s, int copies, const void* g_density, const void* g_br, void* g_phi, void* g_mag,
                 void* g_zeta) override
    {
        err.clear();
        if (!have_fwd) return fail(MPM_MAG_ESTATE, "backward needs a forward call");
        if (copies < 1 || copies > kMaxCopies) return fail(MPM_MAG_EINVAL, "copies must be in [1, 4096]");
        if ((g_phi && !g_density) || ((g_mag || g_zeta) && !g_br)) return fail(MPM_MAG_EINVAL, "null gradient input");
        if (g_phi) {
            hipLaunchKernelGGL((k_scale<real>), dim3(grid_of(N)), dim3(kBlock), 0, s, (const real*)g_density,
                               (const real*)phit, (const real*)inv_s, N, copies, fp, u);
            hipLaunchKernelGGL((k_spmv<real>), dim3(grid_of(N, kRowsPerBlock)), dim3(kBlock), 0, s,
                               (const uint32_t*)row_ptr, (const int*)col, (const real*)w, N, (const real*)u,
                               (real*)g_phi);
            FE_HIP(hipGetLastError());
        }
        if (g_mag || g_zeta) {
            if (has_region) {
                if (m_chunk) {
                    if (n_chunks > 0)
                        hipLaunchKernelGGL((k_region_chunks<real, D>), dim3(n_chunks), dim3(kBlock), 0, s,
                                           (const uint32_t*)members, (const int64_t*)c_lo, (const int64_t*)c_hi,
                                           N, copies, (const real*)g_br, G);
                } else {
                    FE_HIP(hipMemsetAsync(G, 0, sizeof(double) * n_m * D, s));
                    hipLaunchKernelGGL((k_region_sums<real, D>), dim3(grid_of(N)), dim3(kBlock), 0, s,
                                       (const uint32_t*)reg_sorted, (const uint32_t*)members, N, copies,
                                       (const real*)g_br, G);
                }
                if (m_chunk)
                    hipLaunchKernelGGL((k_region_chunk_grads<real, D>), dim3((unsigned)n_m), dim3(64), 0, s,
                                       (const double*)G, (const int*)m_chunk, n_m, (const real*)mag,
                                       (const real*)zeta, fp.br_max, fp.delta, (real*)g_mag, (real*)g_zeta);
                else
                    hipLaunchKernelGGL((k_region_grads<real, D>), dim3(grid_of(n_m)), dim3(kBlock), 0, s,
                                       (const double*)G, n_m, (const real*)mag, (const real*)zeta, fp.br_max,
                                       fp.delta, (real*)g_mag, (real*)g_zeta);
            } else {
                hipLaunchKernelGGL((k_particle_grads<real, D>), dim3(grid_of(N)), dim3(kBlock), 0, s,
                                   (const real*)g_br, N, copies, (const real*)mag, (const real*)zeta, fp.br_max,
                                   fp.delta, (real*)g_mag, (real*)g_zeta);
            }
            FE_HIP(hipGetLastError());
        }
        return MPM_MAG_OK;
    }
};

template <typename real, int D>
Base* make(int64_t n, const void* x0, double radius, const int32_t* region, int n_regions, hipStream_t s,
           int* status, std::string* msg)
{
    auto* d = new (std::nothrow) Design<real, D>();
    if (!d) {
        *status = MPM_MAG_ENOMEM;
        return nullptr;
    }
    *status = d->init(n, (const real*)x0, radius, region, n_regions, s);
    if (*status != MPM_MAG_OK) {
        *msg = d->err;
        (void)hipStreamSynchronize(s);   // no build pass may still use the memory freed below
        delete d;
        return nullptr;
    }
    return d;
}

}  // namespace fe
}  // namespace mpm

struct mpm_mag_design {
    mpm::fe::Base* d = nullptr;
    std::string last;
};

namespace {
thread_local std::string g_design_create_error;
}

extern "C" {

int mpm_mag_design_create(int dim, int64_t n_particles, const void* x0, double radius, const int32_t* region,
                          int n_regions, int precision, void* stream, mpm_mag_design** out)
{
    if (!out) return MPM_MAG_EINVAL;
    *out = nullptr;
    g_design_create_error.clear();
    if ((dim != 2 && dim != 3) || (precision != 4 && precision != 8) || !x0 || n_particles < 1 ||
        n_particles > ((int64_t)1 << 30) || !(radius > 0) || !std::isfinite(radius) ||
        (region && (n_regions < 1 || n_regions > (1 << 30)))) {
        g_design_create_error = "bad dim, precision, size, radius or region count";
        return MPM_MAG_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    int st = MPM_MAG_OK;
    std::string msg;
    mpm::fe::Base* d = nullptr;
    try {
        if (precision == 4)
            d = dim == 2 ? mpm::fe::make<float, 2>(n_particles, x0, radius, region, n_regions, s, &st, &msg)
                         : mpm::fe::make<float, 3>(n_particles, x0, radius, region, n_regions, s, &st, &msg);
        else
            d = dim == 2 ? mpm::fe::make<double, 2>(n_particles, x0, radius, region, n_regions, s, &st, &msg)
                         : mpm::fe::make<double, 3>(n_particles, x0, radius, region, n_regions, s, &st, &msg);
    } catch (...) {
        return MPM_MAG_ENOMEM;
    }
    if (!d) {
        g_design_create_error = msg;
        return st ? st : MPM_MAG_ENOMEM;
    }
    auto* h = new (std::nothrow) mpm_mag_design();
    if (!h) {
        delete d;
        return MPM_MAG_ENOMEM;
    }
    h->d = d;
    *out = h;
    return MPM_MAG_OK;
}

int mpm_mag_design_forward(mpm_mag_design* h, void* stream, const void* phi, double beta, const void* br_mag,
                           const void* zeta, double br_max, double delta, int copies, void* density_out,
                           void* br_out)
{
    if (!h) return MPM_MAG_EINVAL;
    const int st =
        h->d->forward((hipStream_t)stream, phi, beta, br_mag, zeta, br_max, delta, copies, density_out, br_out);
    h->last = st ? h->d->err : std::string();
    return st;
}

int mpm_mag_design_backward(mpm_mag_design* h, void* stream, int copies, const void* g_density, const void* g_br,
                            void* g_phi, void* g_br_mag, void* g_zeta)
{
    if (!h) return MPM_MAG_EINVAL;
    const int st = h->d->backward((hipStream_t)stream, copies, g_density, g_br, g_phi, g_br_mag, g_zeta);
    h->last = st ? h->d->err : std::string();
    return st;
}

int64_t mpm_mag_design_nnz(const mpm_mag_design* h) { return h ? h->d->nnz : 0; }

const char* mpm_mag_design_last_error(const mpm_mag_design* h)
{
    return h ? h->last.c_str() : g_design_create_error.c_str();
}

static int harmonic_check(const mpm_mag_harmonic_desc* d, int precision)
{
    if (!d || (d->dim != 2 && d->dim != 3) || (precision != 4 && precision != 8) || d->n_inst < 1 ||
        d->n_steps < 1 || (int64_t)d->n_inst * d->n_steps > 0x7fffffffLL || !(d->dt > 0) || !std::isfinite(d->dt) ||
        !std::isfinite(d->b_max) || !std::isfinite(d->f_min) || !std::isfinite(d->f_max) || !(d->delta >= 0))
        return MPM_MAG_EINVAL;
    return MPM_MAG_OK;
}

static int harmonic_dispatch(const mpm_mag_harmonic_desc* d, int precision, hipStream_t s, const void* b_a,
                             const void* f, const void* eta, const void* g, void* o0, void* o1, void* o2, bool bwd)
{
    if (precision == 4)
        return d->dim == 2 ? mpm::fe::harmonic_launch<float, 2>(d, s, b_a, f, eta, g, o0, o1, o2, bwd)
                           : mpm::fe::harmonic_launch<float, 3>(d, s, b_a, f, eta, g, o0, o1, o2, bwd);
    return d->dim == 2 ? mpm::fe::harmonic_launch<double, 2>(d, s, b_a, f, eta, g, o0, o1, o2, bwd)
                       : mpm::fe::harmonic_launch<double, 3>(d, s, b_a, f, eta, g, o0, o1, o2, bwd);
}

int mpm_mag_harmonic_program(const mpm_mag_harmonic_desc* d, int precision, void* stream, const void* b_a,
                             const void* f, const void* eta, void* b_prog)
{
    const int st = harmonic_check(d, precision);
    if (st) return st;
    if (!b_a || !f || !eta || !b_prog) return MPM_MAG_EINVAL;
    return harmonic_dispatch(d, precision, (hipStream_t)stream, b_a, f, eta, nullptr, b_prog, nullptr, nullptr, false);
}

int mpm_mag_harmonic_backward(const mpm_mag_harmonic_desc* d, int precision, void* stream, const void* b_a,
                              const void* f, const void* eta, const void* g_b_prog, void* g_b_a, void* g_f,
                              void* g_eta)
{
    const int st = harmonic_check(d, precision);
    if (st) return st;
    if (!b_a || !f || !eta || !g_b_prog) return MPM_MAG_EINVAL;
    return harmonic_dispatch(d, precision, (hipStream_t)stream, b_a, f, eta, g_b_prog, g_b_a, g_f, g_eta, true);
}

int mpm_mag_adam_step(int precision, void* stream, int64_t n, void* param, const void* grad, void* m, void* v,
                      int step, double lr, double beta1, double beta2, double eps, double lo, double hi)
{
    if ((precision != 4 && precision != 8) || n < 0 || step < 1 || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps >= 0) || !(lo <= hi))
        return MPM_MAG_EINVAL;
    if (n == 0) return MPM_MAG_OK;
    if (!param || !grad || !m || !v) return MPM_MAG_EINVAL;
    const double c1 = 1.0 / (1.0 - std::pow(beta1, step)), c2 = 1.0 / (1.0 - std::pow(beta2, step));
    hipStream_t s = (hipStream_t)stream;
    const dim3 grid((unsigned)mpm::fe::grid_of(n));
    if (precision == 4)
        hipLaunchKernelGGL(mpm::fe::k_adam<float>, grid, dim3(mpm::kBlock), 0, s, n, (float*)param,
                           (const float*)grad, (float*)m, (float*)v, (float)lr, (float)beta1, (float)beta2,
                           (float)(1.0 - beta1), (float)(1.0 - beta2), (float)eps, (float)c1, (float)c2, (float)lo,
                           (float)hi);
    else
        hipLaunchKernelGGL(mpm::fe::k_adam<double>, grid, dim3(mpm::kBlock), 0, s, n, (double*)param,
                           (const double*)grad, (double*)m, (double*)v, lr, beta1, beta2, 1.0 - beta1, 1.0 - beta2,
                           eps, c1, c2, lo, hi);
    return hipGetLastError() == hipSuccess ? MPM_MAG_OK : MPM_MAG_EHIP;
}

void mpm_mag_design_destroy(mpm_mag_design* h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();   // queued forward/backward work may still read the handle's arrays
    delete h->d;
    delete h;
}

}  // extern "C"
