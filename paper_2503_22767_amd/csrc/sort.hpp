// Cell binning of particles: spatial keys (instance, Hilbert, Morton or
// row-major index of the particle's cell) and a stable LSD radix sort of (key, caller index) pairs with
// 8-bit digits. One block histograms / scatters kSortTile consecutive items;
// ranks inside a wave come from ballots, waves of a block take their turn.
#pragma once

#include "device.hpp"

namespace mpm {

constexpr int kSortItems = 16;
constexpr int kSortTile = kBlock * kSortItems;

struct KeyParams {
    int n_inst;
    int cell_bits;      // bits of the per-instance cell key (dim * axis_bits)
    int axis_bits;      // bits per axis: ceil(log2(n_grid)) over the instances
    int curve;          // cell order: 0 Hilbert, 1 Morton (Z order), 2 row major (x fastest)
};

// Morton index: bits of the axes interleaved, x least significant.
__device__ __forceinline__ uint32_t morton_index(const int c[3], int dim, int bits)
{
    uint32_t key = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = dim - 1; i >= 0; --i) key = (key << 1) | (((uint32_t)c[i] >> b) & 1u);
    return key;
}

// Hilbert index of a cell (dim 2 or 3, `bits` bits per axis) by Skilling's
// transpose method ("Programming the Hilbert curve", AIP Conf. Proc. 707,
// 2004): undo the excess work per bit level, Gray-encode, then interleave the
// transposed coordinates, most significant bit first. Consecutive indices are
// face-adjacent cells, so any run of particles sorted by it covers a connected
// set of cells.
__device__ __forceinline__ uint32_t hilbert_index(const int c[3], int dim, int bits)
{
    uint32_t X[3] = {(uint32_t)c[0], (uint32_t)c[1], (uint32_t)c[2]};
    const uint32_t M = 1u << (bits - 1);
    for (uint32_t Q = M; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int i = 0; i < dim; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    for (int i = 1; i < dim; ++i) X[i] ^= X[i - 1];
    uint32_t t = 0;
    for (uint32_t Q = M; Q > 1; Q >>= 1)
        if (X[dim - 1] & Q) t ^= Q - 1;
    for (int i = 0; i < dim; ++i) X[i] ^= t;
    uint32_t key = 0;
    for (int b = bits - 1; b >= 0; --b)
        for (int i = 0; i < dim; ++i) key = (key << 1) | ((X[i] >> b) & 1u);
    return key;
}

// key of caller particle q: (instance << cell_bits) | hilbert(cell of its stencil base)
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_sort_keys(const InstDev<real>* inst, const int64_t* caller_start,
                                                      KeyParams kp, const real* x0, int64_t n, uint32_t* keys,
                                                      uint32_t* vals)
{
    int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= n) return;
    int lo = 0, hi = kp.n_inst - 1;
    while (lo < hi) {  // last instance whose start <= q
        int mid = (lo + hi + 1) >> 1;
        if (caller_start[mid] <= q) lo = mid; else hi = mid - 1;
    }
    const InstDev<real>& I = inst[lo];
    int c[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        real xs = x0[q * D + k] * I.inv_dx - real(0.5);
        int b = (xs >= real(0)) ? (int)xs : 0;
        c[k] = min(max(b, 0), I.n_grid - 3);
    }
    uint32_t cell;
    if (kp.curve == 1) {
        cell = morton_index(c, D, kp.axis_bits);
    } else if (kp.curve == 2) {
        cell = (uint32_t)c[0] | ((uint32_t)c[1] << kp.axis_bits) | (D == 3 ? ((uint32_t)c[2] << (2 * kp.axis_bits)) : 0u);
    } else {
        cell = hilbert_index(c, D, kp.axis_bits);
    }
    keys[q] = ((uint32_t)lo << kp.cell_bits) | cell;
    vals[q] = (uint32_t)q;
}

static __global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* keys, int64_t n, int shift, uint32_t* hist,
                                                       int nblocks)
{
    __shared__ uint32_t h[256];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t start = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        int64_t j = start + (int64_t)r * kBlock + t;
        if (j < n) atomicAdd(&h[(keys[j] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)t * nblocks + blockIdx.x] = h[t];
}

// exclusive scan in place, single block of 1024 threads
static __global__ __launch_bounds__(1024) void k_scan_exclusive(uint32_t* a, int64_t n)
{
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int64_t per = (n + 1023) / 1024;
    const int64_t b = (int64_t)t * per;
    const int64_t e = min(n, b + per);
    uint32_t s = 0;
    for (int64_t j = b; j < e; ++j) s += a[j];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int64_t j = b; j < e; ++j) {
        uint32_t v = a[j];
        a[j] = run;
        run += v;
    }
}

static __global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t* kin, const uint32_t* vin, uint32_t* kout,
                                                          uint32_t* vout, int64_t n, int shift,
                                                          const uint32_t* hist, int nblocks)
{
    __shared__ uint32_t base[256];
    const int t = threadIdx.x;
    const int wave = t >> 6, lane = t & 63;
    base[t] = hist[(int64_t)t * nblocks + blockIdx.x];
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t start = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        int64_t j = start + (int64_t)r * kBlock + t;
        bool valid = j < n;
        uint32_t key = valid ? kin[j] : 0u;
        uint32_t val = valid ? vin[j] : 0u;
        uint32_t d = (key >> shift) & 255u;
        uint64_t match = __ballot(valid);
        if (!valid) match = ~match;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t bb = __ballot((d >> b) & 1u);
            match &= ((d >> b) & 1u) ? bb : ~bb;
        }
        int rank = __popcll(match & lt);
        int cnt = __popcll(match);
        for (int w = 0; w < kWaves; ++w) {
            if (w == wave && valid) {
                uint32_t pos = base[d] + (uint32_t)rank;
                kout[pos] = key;
                vout[pos] = val;
            }
            __syncthreads();
            if (w == wave && valid && rank == cnt - 1) base[d] += (uint32_t)cnt;
            __syncthreads();
        }
    }
}

}  // namespace mpm
