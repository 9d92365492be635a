// HIP kernels of the magneto-elastic MLS-MPM step (Sec. 2.2) and of its
// transpose (Sec. 2.3), templated on the precision and the dimension.
//
// Layout in HBM:
//  - particle state: structure of arrays, component c of particle slot i at
//    st[c * nalloc + i]; components u[D], v[D], C[DxD], F[DxD] (row major),
//    where u = x - x(0) is the displacement; the initial position x0s is kept
//    read-only relative to the chunk's origin cell (x_abs = org dx + x0s + u),
//    so FP32 resolves displacements to their own precision and positions to
//    ~1e-9 of the domain; the adjoint state uses the same layout (ubar = xbar);
//  - particles are stored per instance in chunks of kBlock slots (one block per
//    chunk), sorted once per rollout into spatial tiles so a chunk's stencils
//    cover a compact box of nodes;
//  - grids: per instance n^D nodes (x fastest), 4 values per node
//    (p_0..p_{D-1} or v, and the mass in slot 3), instances concatenated.
#pragma once

#include "device.hpp"

namespace mpm {

template <int D> struct Comp {
    static constexpr int NC = 2 * D + 2 * D * D;
    static constexpr int X = 0, V = D, C = 2 * D, F = 2 * D + D * D;
    static constexpr int S3 = D == 2 ? 9 : 27;
};

// Staging box capacity (nodes).
constexpr int kBoxCap = 1024;

// LDS accumulator of the staged boxes. On gfx950 the single-precision LDS add
// runs more than an order of magnitude slower than the integer and the
// double-precision ones, so FP32 contributions are summed as 32-bit fixed point
// (scaled per block so that 256 contributions of the block's largest magnitude
// fit in 2^30: rounding comparable to FP32 summation, and order independent),
// FP64 contributions in double.
template <typename real> struct LdsAcc;
template <> struct LdsAcc<float> {
    using T = int;
    static constexpr float range = 1073741824.0f / (float)kBlock;   // 2^30 / contributions per node
    // w u + 1.5 2^23 leaves w u rounded to the nearest integer in the low
    // mantissa bits (|w u| <= 2^22); subtracting the bits of 1.5 2^23 yields it
    static constexpr float magic = 12582912.0f;
    static constexpr unsigned magic_bits = 0x4B400000u;
    __device__ static T enc(float w, float u)
    {
        return (int)((unsigned)__float_as_int(__fmaf_rn(w, u, magic)) - magic_bits);
    }
    __device__ static float dec(T a, float inv) { return (float)a * inv; }
};
template <> struct LdsAcc<double> {
    using T = double;
    static constexpr double range = 0.0;
    __device__ static T enc(double w, double u) { return w * u; }
    __device__ static double dec(T a, double) { return a; }
};
// coarse blocks of the grid used to hand staged boxes to the grid update
template <int D> struct Coarse {
    static constexpr int edge = D == 2 ? 16 : 8;                    // nodes per axis
    static constexpr int nodes = D == 2 ? 256 : 512;
    static constexpr int cap = 256;                                  // registered boxes per coarse block
};
static_assert(Coarse<2>::cap <= kGridBlock && Coarse<3>::cap <= kGridBlock, "grid scan assumes cap <= block");

// The field-program gradient and the per-instance loss sums are accumulated
// by FP64 atomics, one per workgroup (and step). Every workgroup of an
// instance adds to the same few values, so the atomics are spread over
// kGbCopies copies (by chunk index) and the copies are summed in a fixed order
// at the end: a single copy serialized several thousand atomics per value at
// the L2, a quarter of the fused adjoint kernel's time.
constexpr int kGbCopies = 64;


template <typename real>
struct Args {
    const InstDev<real>* inst;
    const ChunkDev* chunks;
    const int* gblock_inst;
    int64_t nalloc;
    const real* phi;     // [nalloc]
    const real* br;      // [D][nalloc]
    const real* bprog;   // [S_tot][D]
    real* gm;            // [4 G] momentum / mass
    real* gv;            // [4 G] velocity after the grid operation
    real* gbar;          // [4 G] adjoint grid values
    unsigned long long* err;   // device error word (earliest failure; report_error)
    unsigned long long* scat_stats;   // [3] scatter fallbacks: waves staged alone, waves on global atomics,
                                      // box registrations past a coarse block's list
    double* acc;         // [kGbCopies][n_inst][kAccCount] per-instance sums; k_loss_finalize leaves the totals in copy 0
    int64_t acc_stride;  // n_inst * kAccCount: distance between copies
    double* loss_val;    // [n_inst]
    double* gB;          // [kGbCopies][S_tot][D] field-program gradient, summed over the copies at the end
    int64_t gB_stride;   // S_tot * D: distance between copies
    real* gphi;          // [nalloc]
    real* gbr;           // [D][nalloc]
    const int4* corig;   // [n_chunks] origin cell of each chunk (positions are stored relative to it)
    const real* x0s;     // [D][nalloc] initial positions relative to the chunk origin
    real* part;          // [n_chunks][kBoxCap][4] staged box of each chunk
    int4* box;           // [n_chunks][2]: lo (xyz), ext (xyz); ext = 0 when the box was not staged
    int* reg_count;      // [n_coarse] boxes registered with each coarse block this phase
    int* reg_list;       // [n_coarse][cap] chunk ids
    int* fb_used;        // [n_coarse] nonzero when the dense fallback accumulator holds values of the block
    int* part_done;      // [n_coarse] parts of the block whose gather has finished (grid kernels)
    const int* cb_inst;  // [n_coarse] instance of each coarse block
    int* active;         // [4]: coarse blocks activated per scatter list (P2G: 0, 3; G2P transpose: 1, 2)
    int* active_list;    // [4][n_coarse]
    int n_coarse;
    int use_lds;
    int chunk_base;      // first chunk of the launch (launches may cover a range of instances)
    int box_cap;         // largest block staging box (nodes, <= kBoxCap)
    int grid_parts;      // workgroups sharing one coarse block in the grid kernels (slabs along its last axis)
    const uint8_t* lperm;  // [nalloc]: lane t of chunk c works on slot c * kBlock + lperm[c * kBlock + t]
    uint16_t* trace;       // [n_steps][trace_nodes] branch decisions of the grid update, or nullptr
    int64_t trace_nodes;   // nodes of all instances (sum of n_grid^D)
};

// copy of the per-instance accumulators that chunk c adds to
template <typename real>
__device__ __forceinline__ double* acc_copy(const Args<real>& a, int c, int inst)
{
    return a.acc + (int64_t)(c % kGbCopies) * a.acc_stride + (int64_t)inst * kAccCount;
}

// Grid store: a step's active coarse blocks, each node's summed (momentum,
// mass) record (4 values), packed step after step, so that the reverse sweep
// can rebuild a step's grid without recomputing its P2G; the node velocity is
// recomputed from the record by the same grid operation. Entry idx of one
// chain owns the slots [base[idx], base[idx + 1]); blk names the coarse block
// in each slot. base keeps counting past cap (and counts even without data),
// so an entry is stored iff base[idx + 1] <= cap. The recorded forward keeps
// the whole rollout (idx = step); the recompute of a segment the forward could
// not keep writes its own steps to a segment store (idx = step in segment).
constexpr int kStoreCountMax = 1 << 30;
template <typename real>
struct GridStore {
    real* data;   // [cap][Coarse<D>::nodes][4], nullptr: only counted
    int* blk;     // [cap]
    int* base;    // [entries + 1], nullptr: neither kept nor counted
    int cap;      // slots
    int idx;      // entry of this launch
    int step;     // time step (moving obstacles)
};

// Slot of the particle that lane t of this block works on. The forward
// particle kernels take a chunk's particles grouped by their current stencil
// base cell (k_lane_sort), so that lanes sharing a base are adjacent and the
// scatter's segments stay long after particles change cells; every order gives
// the same sums. The transposed kernels keep slot order: they move more data
// per particle, and for them the permuted loads cost more than the longer
// segments save.
template <typename real>
__device__ __forceinline__ int64_t lane_slot(const Args<real>& a, int t)
{
    const int64_t c0 = (int64_t)(a.chunk_base + blockIdx.x) * kBlock;
    return c0 + a.lperm[c0 + t];
}

// --------------------------------------------------------------------------
// block scatter through LDS
// --------------------------------------------------------------------------

// slot of value c in a node record: momenta / velocities first, mass in slot 3
template <int D, int NV>
__device__ __forceinline__ int value_slot(int c) { return (NV == D + 1 && c == D) ? 3 : c; }

constexpr int kWaveBoxCap = kBoxCap / kWaves;   // staging box of one wave when the block's box is too big

// storage offset (nodes) of staged box `id` = chunk * kWaves + wave inside `part`
__device__ __forceinline__ int64_t box_offset(int id) { return (int64_t)(id / kWaves) * kBoxCap + (id % kWaves) * kWaveBoxCap; }

// Node records of a staged box. In FP32 the P2G scatter (momentum and mass)
// sums its values in pairs with 64-bit LDS atomics: word 0 holds the mass and
// word 1 the first momentum component of one 64-bit integer (the mass sum is
// never negative, so word 1 is that component's sum); in 3D words 2 and 3 hold
// the second and third components of another, whose high word carries the
// sign of the low one; in 2D word 2 is the second component alone. Otherwise
// word q is record slot q.
template <typename real, int D, bool kPacked>
__device__ __forceinline__ void decode_node(const typename LdsAcc<real>::T* w, const real inv[4], real out[4])
{
    using Acc = LdsAcc<real>;
    if constexpr (kPacked) {
        out[0] = Acc::dec(w[1], inv[0]);
        out[1] = Acc::dec(w[2], inv[1]);
        out[2] = D == 3 ? Acc::dec(w[3] + (w[2] < 0 ? 1 : 0), inv[2]) : Acc::dec(w[3], inv[2]);
        out[3] = Acc::dec(w[0], inv[3]);
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = Acc::dec(w[q], inv[q]);
    }
}

// Registers box `id` (node range lo .. lo + ext - 1) with every coarse block it
// overlaps; the lanes lane0, lane0 + stride, ... share the work. A coarse block
// whose list is full gets the staged values of its part of the box added to
// the dense accumulator fb instead.
template <typename real, int D, bool kPacked>
__device__ __forceinline__ void register_box(const Args<real>& a, const InstDev<real>& I, int id, const int lo[3],
                                             const int ext[3], const typename LdsAcc<real>::T* box_lds,
                                             const real inv[4], bool staged, real* fb, int phase, int lane0,
                                             int stride)
{
    using CB = Coarse<D>;
    int b0[3] = {0, 0, 0}, nbk[3] = {1, 1, 1};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        b0[k] = lo[k] / CB::edge;
        nbk[k] = (lo[k] + ext[k] - 1) / CB::edge - b0[k] + 1;
    }
    const int n_ov = nbk[0] * nbk[1] * nbk[2];
    for (int j = lane0; j < n_ov; j += stride) {
        int jj[3] = {j % nbk[0], (j / nbk[0]) % nbk[1], j / (nbk[0] * nbk[1])};
        int cb = I.cb_off + (b0[0] + jj[0]) + I.nb * ((b0[1] + jj[1]) + (D == 3 ? I.nb * (b0[2] + jj[2]) : 0));
        int slot = atomicAdd(&a.reg_count[cb], 1);
        if (slot == 0) a.active_list[phase * a.n_coarse + atomicAdd(&a.active[phase], 1)] = cb;
        if (!staged || slot >= CB::cap) a.fb_used[cb] = 1;   // values of this block go to fb
        if (slot >= CB::cap) atomicAdd(&a.scat_stats[2], 1ull);
        if (slot < CB::cap) {
            a.reg_list[cb * CB::cap + slot] = id;
        } else if (staged) {
            int clo[3] = {0, 0, 0}, chi[3] = {1, 1, 1};
#pragma unroll
            for (int k = 0; k < D; ++k) {
                int cs = (b0[k] + jj[k]) * CB::edge;
                clo[k] = max(cs, lo[k]) - lo[k];
                chi[k] = min(cs + CB::edge, lo[k] + ext[k]) - lo[k];
            }
            for (int z = clo[2]; z < chi[2]; ++z)
                for (int y = clo[1]; y < chi[1]; ++y)
                    for (int x = clo[0]; x < chi[0]; ++x) {
                        int l = x + ext[0] * (y + ext[1] * z);
                        int64_t g = (int64_t)I.grid_off + (int64_t)(lo[0] + x) +
                                    (int64_t)I.n_grid * ((lo[1] + y) + (D == 3 ? (int64_t)I.n_grid * (lo[D - 1] + z) : 0));
                        real rec[4];
                        decode_node<real, D, kPacked>(box_lds + 4 * l, inv, rec);
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            if (rec[q] != real(0)) atomic_add(&fb[4 * g + q], rec[q]);
                    }
        }
    }
}

// Lanes of one 16-lane row that share a stencil base form contiguous segments
// (particles are sorted along a Hilbert curve of their cells). Four DPP
// shift-right steps leave in the last lane of each segment the sum of the
// segment's values (exact for the fixed-point integers).
__device__ __forceinline__ int dpp_shr(int v, int off)
{
    switch (off) {
    case 1: return __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);
    case 2: return __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);
    case 4: return __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);
    default: return __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);
    }
}

// one step of the segmented sum: add the value of lane l - off when the mask
// (all ones or zero) says that lane is in the same segment
__device__ __forceinline__ int seg_step(int v, int off, int m) { return v + (dpp_shr(v, off) & m); }

__device__ __forceinline__ double seg_step(double v, int off, int m)
{
    const int lo = dpp_shr(__double2loint(v), off) & m;
    const int hi = dpp_shr(__double2hiint(v), off) & m;
    return v + __hiloint2double(hi, lo);
}

// segmented sums of NV values at once (steps interleaved over the values so
// the DPP reads do not wait on the adds just issued)
template <int NV, typename T>
__device__ __forceinline__ void seg_row_sums(T (&e)[NV], const int (&m)[4])
{
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < NV; ++q) e[q] = seg_step(e[q], 1 << j, m[j]);
}

// inclusive prefix sums within each 16-lane row (integers, modulo 2^32)
template <int NV>
__device__ __forceinline__ void row_prefix_sums(int (&e)[NV])
{
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int q = 0; q < NV; ++q) e[q] = (int)((unsigned)e[q] + (unsigned)dpp_shr(e[q], 1 << j));
}

// Adds NV values per stencil node of every active particle of the block to the
// instance grid. The block's stencils are summed in LDS over their bounding
// box: as 32-bit fixed point with a per-block scale per value slot (FP32
// build), the lanes of a 16-lane row that share a stencil base combined first
// by row prefix sums so that one lane per segment adds to a node; as doubles
// (FP64 build), by segmented row sums. The box is then written with plain
// stores to this chunk's slot of `part` and registered (one integer atomic per
// coarse block it overlaps) so the grid update can gather it; no float atomics
// touch HBM. When the block's box exceeds kBoxCap every wave stages its own box
// (at most kWaveBoxCap nodes); a wave whose box is larger still, or a coarse
// block whose list is full, falls back to float atomics into the dense
// accumulator fb, which the grid update also reads. Must be reached by every
// thread of the block.
template <typename real, int D, int NV, typename ValFn>
__device__ __forceinline__ void scatter_box(const Args<real>& a, const InstDev<real>& I,
                                            typename LdsAcc<real>::T* lds, bool active, const int base[D],
                                            const real bound[NV], real* fb, int phase, ValFn vals)
{
    using Acc = LdsAcc<real>;
    using acc_t = typename Acc::T;
    constexpr int S3 = Comp<D>::S3;
    constexpr bool kPacked = NV == D + 1 && sizeof(acc_t) == 4;   // see decode_node
    __shared__ int s_bb[kWaves][6];
    __shared__ float s_bmax[kWaves][4];
    const int t = threadIdx.x;
    const int w = t >> 6;
    const int c = a.chunk_base + blockIdx.x;
    const int n_grid = I.n_grid;
    // bounding boxes of the wave and of the block
    int wlo[3] = {0, 0, 0}, wext[3] = {1, 1, 1};
    int whi[D];
    wave_bounds<D>(base, active, wlo, whi);
    const bool wave_live = wlo[0] != 0x3fffffff;
    int wvol = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        wext[k] = wave_live ? whi[k] - wlo[k] + 3 : 1;
        wvol *= wext[k];
    }
    float bmax[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        bmax[q] = wave_max_nonneg(active ? (float)fabs(bound[q]) : 0.0f);
    }
    if ((t & 63) == 0) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            s_bb[w][k] = wlo[k];
            s_bb[w][3 + k] = whi[k];
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) s_bmax[w][q] = bmax[q];
    }
    __syncthreads();
    // fixed-point scales of the value slots (FP32 build)
    real scl[4], inv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        scl[q] = real(1);
        inv[q] = real(1);
    }
    if (Acc::range > 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            float m = s_bmax[0][q];
#pragma unroll
            for (int ww = 1; ww < kWaves; ++ww) m = fmaxf(m, s_bmax[ww][q]);
            const int sl = value_slot<D, NV>(q);
            scl[sl] = m > 0.0f ? (real)(Acc::range / m) : real(0);
            inv[sl] = m > 0.0f ? (real)(m / Acc::range) : real(0);
        }
    }
    int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
    int vol = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        int l = s_bb[0][k], h = s_bb[0][3 + k];
#pragma unroll
        for (int ww = 1; ww < kWaves; ++ww) {
            l = min(l, s_bb[ww][k]);
            h = max(h, s_bb[ww][3 + k]);
        }
        lo[k] = l;
        ext[k] = h - l + 3;
        vol *= ext[k];
    }
    const bool block_mode = a.use_lds && vol <= a.box_cap;
    // this lane's staging box: the block's, or its wave's
    const bool staged = block_mode || (a.use_lds && wave_live && wvol <= kWaveBoxCap);
    if (!block_mode && wave_live && (t & 63) == 0) atomicAdd(&a.scat_stats[staged ? 0 : 1], 1ull);
    int blo[3], bext[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        blo[k] = block_mode ? lo[k] : wlo[k];
        bext[k] = block_mode ? ext[k] : wext[k];
    }
    acc_t* blds = block_mode ? lds : lds + w * 4 * kWaveBoxCap;
    const int id = c * kWaves + (block_mode ? 0 : w);
    // zero the staging boxes
    if (block_mode) {
        for (int i = t; i < vol; i += kBlock)
#pragma unroll
            for (int q = 0; q < 4; ++q) blds[4 * i + q] = acc_t(0);
    } else if (staged) {
        for (int i = t & 63; i < wvol; i += 64)
#pragma unroll
            for (int q = 0; q < 4; ++q) blds[4 * i + q] = acc_t(0);
    }
    __syncthreads();
    // segments of lanes sharing a stencil base within each 16-lane row
    int seg_d, seg_tail;
    {
        const int lane = t & 63;
        const int key = active ? (base[0] + n_grid * (base[1] + (D == 3 ? n_grid * base[D - 1] : 0))) : -1 - lane;
        const int prev = __shfl_up(key, 1, 64);
        const bool head = (lane & 15) == 0 || prev != key;
        const uint64_t H = __ballot(head);
        const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
        seg_d = lane - (63 - __clzll(H & upto));
        seg_tail = (lane & 15) == 15 || ((H >> (lane + 1)) & 1ull);
    }
    if (staged) {
        int rel[D];
#pragma unroll
        for (int k = 0; k < D; ++k) rel[k] = active ? base[k] - blo[k] : 0;
        const int lrel = rel[0] + bext[0] * (rel[1] + (D == 3 ? bext[1] * rel[D - 1] : 0));
        const bool emit = active && seg_tail;
        int msk[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) msk[j] = seg_d >= (1 << j) ? -1 : 0;
        // FP32 (integer sums): a segment's sum is the row prefix at its tail
        // minus the row prefix just before its head, which is the prefix of
        // the previous segment's tail. So every tail adds its prefix at its
        // own node and, unless it ends the row or the active lanes, subtracts
        // the same prefix at the next lane's node (exact in modular
        // arithmetic); the next lane's node offset comes by one row shift
        const int next_active = __builtin_amdgcn_update_dpp(0, active ? 1 : 0, 0x101, 0xF, 0xF, true);   // row_shl:1
        const bool sub_next = emit && (t & 15) != 15 && next_active != 0;
        const int lrel_next = __builtin_amdgcn_update_dpp(0, lrel, 0x101, 0xF, 0xF, true);
        real sq[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) sq[q] = scl[value_slot<D, NV>(q)];
#pragma unroll
        for (int o = 0; o < S3; ++o) {
            int oa[D];
            oa[0] = o % 3;
            oa[1] = (o / 3) % 3;
            if (D == 3) oa[D - 1] = o / 9;
            real wgt, u[NV];
            vals(oa, sq, wgt, u);
            acc_t e[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) e[q] = Acc::enc(wgt, u[q]);
            const int li = lrel + oa[0] + bext[0] * (oa[1] + (D == 3 ? bext[1] * oa[D - 1] : 0));
            if constexpr (kPacked) {
                row_prefix_sums<NV>(e);
                // (mass | momentum 0) and, in 3D, (momentum 1 | momentum 2)
                // with the sign of the low word carried into the high one
                const uint64_t pa = ((uint64_t)(uint32_t)e[0] << 32) | (uint32_t)e[D];
                uint64_t pb = 0;
                if constexpr (D == 3) pb = ((uint64_t)(uint32_t)(e[2] + (e[1] >> 31)) << 32) | (uint32_t)e[1];
                if (emit) {
                    atomicAdd(reinterpret_cast<unsigned long long*>(&blds[4 * li]), (unsigned long long)pa);
                    if constexpr (D == 3) atomicAdd(reinterpret_cast<unsigned long long*>(&blds[4 * li + 2]), (unsigned long long)pb);
                    else atomicAdd(&blds[4 * li + 2], e[1]);
                }
                if (sub_next) {
                    const int ln = li - lrel + lrel_next;
                    __hip_atomic_fetch_sub(reinterpret_cast<unsigned long long*>(&blds[4 * ln]), (unsigned long long)pa,
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if constexpr (D == 3)
                        __hip_atomic_fetch_sub(reinterpret_cast<unsigned long long*>(&blds[4 * ln + 2]), (unsigned long long)pb,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    else
                        __hip_atomic_fetch_sub(&blds[4 * ln + 2], e[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            } else if constexpr (sizeof(acc_t) == 4) {
                row_prefix_sums<NV>(e);
                if (emit) {
#pragma unroll
                    for (int q = 0; q < NV; ++q) atomicAdd(&blds[4 * li + value_slot<D, NV>(q)], e[q]);
                }
                if (sub_next) {
                    const int ln = li - lrel + lrel_next;
#pragma unroll
                    for (int q = 0; q < NV; ++q)
                        __hip_atomic_fetch_sub(&blds[4 * ln + value_slot<D, NV>(q)], e[q], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_WORKGROUP);
                }
            } else {
                seg_row_sums<NV>(e, msk);
                if (emit) {
#pragma unroll
                    for (int q = 0; q < NV; ++q) atomicAdd(&blds[4 * li + value_slot<D, NV>(q)], e[q]);
                }
            }
        }
    } else if (active) {
        for (int o = 0; o < S3; ++o) {
            int oa[D];
            offset_split<D>(o, oa);
            int64_t g = (int64_t)I.grid_off + (int64_t)(base[0] + oa[0]) +
                        (int64_t)n_grid * ((base[1] + oa[1]) + (D == 3 ? (int64_t)n_grid * (base[D - 1] + oa[D - 1]) : 0));
            real one[NV], wgt, u[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) one[q] = real(1);
            vals(oa, one, wgt, u);
#pragma unroll
            for (int q = 0; q < NV; ++q) atomic_add(&fb[4 * g + value_slot<D, NV>(q)], wgt * u[q]);
        }
    }
    __syncthreads();
    // write the staged boxes and their descriptors
    real* dst = a.part + box_offset(id) * 4;
    if (block_mode || staged) {
        const int n_write = block_mode ? vol : wvol, l0 = block_mode ? t : (t & 63), step = block_mode ? kBlock : 64;
        for (int l = l0; l < n_write; l += step) {
            real rec[4];
            decode_node<real, D, kPacked>(blds + 4 * l, inv, rec);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[4 * l + q] = rec[q];
        }
    }
    // one writer per descriptor: thread t < kWaves in block mode, lane 0 of each wave otherwise
    if (block_mode ? (t < kWaves) : ((t & 63) == 0)) {
        const int slot = block_mode ? t : w;
        const int bid = c * kWaves + slot;
        int4 blo4 = make_int4(0, 0, 0, 0), bext4 = make_int4(0, 0, 0, 0);
        if (block_mode ? (slot == 0) : staged) {
            blo4 = make_int4(blo[0], blo[1], blo[2], 0);
            bext4 = make_int4(bext[0], bext[1], bext[2], 0);
        }
        a.box[2 * bid] = blo4;
        a.box[2 * bid + 1] = bext4;
    }
    // register the boxes (also the ranges of waves that fell back, so the
    // grid update visits their coarse blocks)
    if (block_mode) {
        register_box<real, D, kPacked>(a, I, id, lo, ext, blds, inv, true, fb, phase, t, kBlock);
    } else if (wave_live) {
        register_box<real, D, kPacked>(a, I, id, wlo, wext, blds, inv, staged, fb, phase, t & 63, 64);
    }
}

// Gathers the boxes registered with coarse block b into the records of the
// nodes of its slab `part` (of a.grid_parts slabs along the block's last axis),
// plus the dense fallback accumulator fb, which is cleared, then calls
// node_fn(global node index, grid coords, block-local index, summed[4]) for
// every node of the slab inside the grid. The (box, node) pairs of all
// registered boxes are enumerated flat across the workgroup so their loads are
// independent; sums go through LDS in double. The workgroups of one block's
// slabs run independently (a heavy block's pairs no longer wait on one
// workgroup); the last of them to finish resets the block's registration.
template <typename real, int D, typename NodeFn>
__device__ __forceinline__ void gather_coarse(const Args<real>& a, const InstDev<real>& I, int b, int part,
                                              real* fb, NodeFn node_fn)
{
    using CB = Coarse<D>;
    constexpr int U = 4;   // pairs in flight per thread
    __shared__ int s_id[CB::cap];
    __shared__ int s_ilo[CB::cap][3];    // intersection origin (grid coords)
    __shared__ int s_iext[CB::cap][3];   // intersection extent
    __shared__ int s_blo[CB::cap][3];    // box origin and extent (for the box-local index)
    __shared__ int s_bext[CB::cap][2];
    __shared__ int s_off[CB::cap + 1];
    __shared__ double s_acc[4][CB::nodes];
    const int t = threadIdx.x;
    __syncthreads();   // the previous coarse block of this workgroup is done with the shared arrays
    const int cnt_raw = a.reg_count[b];
    if (cnt_raw == 0) return;
    const bool fb_any = a.fb_used[b] != 0;   // otherwise fb is zero over the block
    const int cnt = min(cnt_raw, CB::cap);
    const int lb = b - I.cb_off;
    const int bc[3] = {lb % I.nb, D == 3 ? (lb / I.nb) % I.nb : lb / I.nb, D == 3 ? lb / (I.nb * I.nb) : 0};
    int co[3] = {bc[0] * CB::edge, bc[1] * CB::edge, D == 3 ? bc[2] * CB::edge : 0};
    // the slab: layers [sl0, sl0 + sl_n) of the last axis, block-local nodes [ln0, ln0 + n_slab)
    const int sl_n = CB::edge / a.grid_parts, sl0 = part * sl_n;
    const int n_slab = CB::nodes / a.grid_parts, ln0 = part * n_slab;
    int clo[3], chi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        clo[k] = k == D - 1 ? co[k] + sl0 : co[k];
        chi[k] = k == D - 1 ? co[k] + sl0 + sl_n : co[k] + CB::edge;
    }
    for (int j = t; j < cnt; j += blockDim.x) {
        const int id = a.reg_list[b * CB::cap + j];
        const int4 lo = a.box[2 * id], ex = a.box[2 * id + 1];
        const int blo[3] = {lo.x, lo.y, lo.z}, bex[3] = {ex.x, ex.y, ex.z};
        int sz = 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            int l = k < D ? max(blo[k], clo[k]) : 0;
            int h = k < D ? min(blo[k] + bex[k], chi[k]) : 1;
            int e = bex[k] > 0 ? max(0, h - l) : 0;
            s_ilo[j][k] = l;
            s_iext[j][k] = e;
            s_blo[j][k] = blo[k];
            sz *= e;
        }
        s_bext[j][0] = bex[0];
        s_bext[j][1] = bex[1];
        s_id[j] = id;
        s_off[j + 1] = sz;
    }
    for (int i = ln0 + t; i < ln0 + n_slab; i += blockDim.x)
#pragma unroll
        for (int q = 0; q < 4; ++q) s_acc[q][i] = 0.0;
    if (t == 0) s_off[0] = 0;
    __syncthreads();
    // inclusive scan of s_off[1..cnt] (cnt <= blockDim.x): wave scans, then wave totals
    {
        __shared__ int s_wsum[kGridThreadsMax / 64];
        const int lane = t & 63, wv = t >> 6;
        int v = (t < cnt) ? s_off[t + 1] : 0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            int y = __shfl_up(v, off, 64);
            if (lane >= off) v += y;
        }
        if (lane == 63) s_wsum[wv] = v;
        __syncthreads();
        int add = 0;
        for (int w2 = 0; w2 < wv; ++w2) add += s_wsum[w2];
        if (t < cnt) s_off[t + 1] = v + add;
    }
    __syncthreads();
    const int P = s_off[cnt];
    for (int k0 = t; k0 < P; k0 += blockDim.x * U) {
        const real* src[U];
        int nl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * blockDim.x;
            src[u] = nullptr;
            nl[u] = 0;
            if (k < P) {
                int lo = 0, hi = cnt - 1;   // last j with s_off[j] <= k
                while (lo < hi) {
                    int mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= k) lo = mid; else hi = mid - 1;
                }
                const int j = lo;
                int r = k - s_off[j];
                const int ex0 = s_iext[j][0], ex1 = s_iext[j][1];
                int g3[3];
                g3[0] = s_ilo[j][0] + r % ex0;
                r /= ex0;
                g3[1] = s_ilo[j][1] + r % ex1;
                g3[2] = s_ilo[j][2] + r / ex1;
                const int l = (g3[0] - s_blo[j][0]) +
                              s_bext[j][0] * ((g3[1] - s_blo[j][1]) + s_bext[j][1] * (g3[2] - s_blo[j][2]));
                src[u] = a.part + (box_offset(s_id[j]) + l) * 4;
                nl[u] = (g3[0] - co[0]) + CB::edge * ((g3[1] - co[1]) + CB::edge * (g3[2] - co[2]));
            }
        }
        real v[U][4];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) v[u][q] = src[u] ? src[u][q] : real(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (src[u])
#pragma unroll
                for (int q = 0; q < 4; ++q) atomicAdd(&s_acc[q][nl[u]], (double)v[u][q]);
    }
    __syncthreads();
    for (int ln = ln0 + t; ln < ln0 + n_slab; ln += blockDim.x) {
        int g3[3];
        g3[0] = co[0] + ln % CB::edge;
        g3[1] = co[1] + (ln / CB::edge) % CB::edge;
        g3[2] = D == 3 ? co[2] + ln / (CB::edge * CB::edge) : 0;
        bool inside = g3[0] < I.n_grid && g3[1] < I.n_grid && (D == 2 || g3[2] < I.n_grid);
        if (!inside) continue;
        const int64_t local = (int64_t)g3[0] + (int64_t)I.n_grid * (g3[1] + (D == 3 ? (int64_t)I.n_grid * g3[2] : 0));
        const int64_t g = (int64_t)I.grid_off + local;
        real acc[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = (real)s_acc[q][ln];
        if (fb_any)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                acc[q] += fb[4 * g + q];
                fb[4 * g + q] = real(0);
            }
        node_fn(g, g3, ln, acc);
    }
    __syncthreads();
    if (t == 0) {
        // every slab has consumed the registration (its loads have returned)
        // before it counts itself done, so the last one may reset the block;
        // the reset is read only by later kernels. Relaxed: an agent-scope
        // release here would write back the L2 after every block.
        const int done = __hip_atomic_fetch_add(&a.part_done[b], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (done == a.grid_parts - 1) {
            a.part_done[b] = 0;
            a.reg_count[b] = 0;
            if (fb_any) a.fb_used[b] = 0;
        }
    }
}

// Box of grid nodes covering the active particles' stencils, copied from a
// grid array (4 values per node) into LDS for the block's gathers.
template <int D>
struct NodeBox {
    int lo[3], ext[3];
    bool staged;
};

// Block-wide: reduces the bounding box of the active lanes' stencil bases and,
// when it holds at most `cap` nodes, loads those node records of the instance
// grid `src` into lds[4 * node] with coalesced loads. Every thread must call it.
template <typename real, int D>
__device__ __forceinline__ NodeBox<D> stage_nodes(const InstDev<real>& I, bool active, const int base[D],
                                                  const real* src, real* lds, int cap)
{
    __shared__ int s_nb[kWaves][6];
    const int t = threadIdx.x;
    NodeBox<D> nb;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        nb.lo[k] = 0;
        nb.ext[k] = 1;
    }
    int lo[D], hi[D];
    wave_bounds<D>(base, active, lo, hi);
    __syncthreads();   // s_nb may still be read by a previous call
    if ((t & 63) == 0)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            s_nb[t >> 6][k] = lo[k];
            s_nb[t >> 6][3 + k] = hi[k];
        }
    __syncthreads();
    int vol = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        int l = s_nb[0][k], h = s_nb[0][3 + k];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            l = min(l, s_nb[w][k]);
            h = max(h, s_nb[w][3 + k]);
        }
        nb.lo[k] = l;
        nb.ext[k] = h - l + 3;
        vol *= nb.ext[k];
    }
    nb.staged = vol > 0 && vol <= cap;
    if (nb.staged) {
        // walk l = t, t + kBlock, ... keeping its box coordinates (x, y, z)
        // up to date with carries instead of dividing every step
        const int e0 = nb.ext[0], e1 = D == 3 ? nb.ext[1] : 1 << 30;
        int x = t % e0, r = t / e0;
        int y = D == 3 ? r % e1 : r, z = D == 3 ? r / e1 : 0;
        const int sx = kBlock % e0, sr = kBlock / e0;
        const int sy = D == 3 ? sr % e1 : sr, sz = D == 3 ? sr / e1 : 0;
        for (int l = t; l < vol; l += kBlock) {
            int64_t g = (int64_t)(nb.lo[0] + x) +
                        (int64_t)I.n_grid * ((nb.lo[1] + y) + (D == 3 ? (int64_t)I.n_grid * (nb.lo[D - 1] + z) : 0));
#pragma unroll
            for (int q = 0; q < 4; ++q) lds[4 * l + q] = src[4 * g + q];
            x += sx;
            y += sy;
            if (x >= e0) {
                x -= e0;
                ++y;
            }
            if (D == 3) {
                z += sz;
                if (y >= e1) {
                    y -= e1;
                    ++z;
                }
            }
        }
    }
    __syncthreads();
    return nb;
}

__device__ constexpr int kZero3[3] = {0, 0, 0};

// Calls body(g0, sy, sz) with the record of the particle's first stencil node
// and the strides (values) of one node step along y and z: in the staged box
// when there is one, else in the instance grid. The two calls are separate
// instantiations, so the staged one reads with LDS instructions rather than
// generic (flat) loads, and every node of a stencil row sits at a constant
// offset (4, 8) from the row's first.
template <typename real, int D, typename Body>
__device__ __forceinline__ void with_stencil_rows(const NodeBox<D>& nb, const real* lds, const real* src,
                                                  const int base[D], int n, Body body)
{
    if (nb.staged) {
        const int l = (base[0] - nb.lo[0]) +
                      nb.ext[0] * ((base[1] - nb.lo[1]) + (D == 3 ? nb.ext[1] * (base[D - 1] - nb.lo[D - 1]) : 0));
        body(lds + 4 * l, 4 * nb.ext[0], 4 * nb.ext[0] * nb.ext[1]);
    } else {
        body(src + 4 * ((int64_t)base[0] + (int64_t)n * (base[1] + (D == 3 ? (int64_t)n * base[D - 1] : 0))), 4 * n,
             4 * n * n);
    }
}

template <typename real, int D>
__device__ __forceinline__ int64_t node_index(const int base[D], const int a[D], int n)
{
    return (int64_t)(base[0] + a[0]) + (int64_t)n * ((base[1] + a[1]) + (D == 3 ? (int64_t)n * (base[D - 1] + a[D - 1]) : 0));
}

template <typename real, int D>
__device__ __forceinline__ void load_vec(const real* g, real v[D])
{
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = g[k];
}

// block sum of up to 8 doubles; thread 0 of the block gets the totals
template <int NV>
__device__ __forceinline__ void block_sum(double v[NV])
{
    __shared__ double s_red[kWaves][NV > 0 ? NV : 1];
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] = wave_sum(v[c]);
    if ((t & 63) == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) s_red[t >> 6][c] = v[c];
    __syncthreads();
    if (t == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double s = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) s += s_red[w][c];
            v[c] = s;
        }
}

// --------------------------------------------------------------------------
// particle loads
// --------------------------------------------------------------------------

template <typename real, int D>
struct Particle {
    real x[D], v[D], C[D][D], F[D][D];
};

// position x = x0s + u and deformation gradient of slot i
template <typename real, int D>
__device__ __forceinline__ void load_xF(const real* st, const real* x0s, int64_t S, int64_t i, real x[D],
                                        real F[D][D])
{
    using Cp = Comp<D>;
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = x0s[k * S + i] + st[(Cp::X + k) * S + i];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) F[a][b] = st[(Cp::F + a * D + b) * S + i];
}

// full state of slot i with q.x the position x0s + u
template <typename real, int D>
__device__ __forceinline__ void load_particle(const real* st, const real* x0s, int64_t S, int64_t i,
                                              Particle<real, D>& q)
{
    using Cp = Comp<D>;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        q.x[k] = x0s[k * S + i] + st[(Cp::X + k) * S + i];
        q.v[k] = st[(Cp::V + k) * S + i];
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            q.C[a][b] = st[(Cp::C + a * D + b) * S + i];
            q.F[a][b] = st[(Cp::F + a * D + b) * S + i];
        }
}

// stores q with q.x holding the displacement u
template <typename real, int D>
__device__ __forceinline__ void store_particle(real* st, int64_t S, int64_t i, const Particle<real, D>& q)
{
    using Cp = Comp<D>;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        st[(Cp::X + k) * S + i] = q.x[k];
        st[(Cp::V + k) * S + i] = q.v[k];
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            st[(Cp::C + a * D + b) * S + i] = q.C[a][b];
            st[(Cp::F + a * D + b) * S + i] = q.F[a][b];
        }
}

// the same with non-temporal stores, for states written long before they are
// read (the segment stash: a quadruped step's state is 330 MB)
template <typename real, int D>
__device__ __forceinline__ void stream_particle(real* st, int64_t S, int64_t i, const Particle<real, D>& q)
{
    using Cp = Comp<D>;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        __builtin_nontemporal_store(q.x[k], &st[(Cp::X + k) * S + i]);
        __builtin_nontemporal_store(q.v[k], &st[(Cp::V + k) * S + i]);
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) {
            __builtin_nontemporal_store(q.C[a][b], &st[(Cp::C + a * D + b) * S + i]);
            __builtin_nontemporal_store(q.F[a][b], &st[(Cp::F + a * D + b) * S + i]);
        }
}

// --------------------------------------------------------------------------
// per-particle stress and affine momentum matrix (Eqs. 7, 15, 31-33)
// --------------------------------------------------------------------------

template <typename real, int D>
struct P2GTerms {
    real m;            // particle mass phi rho V
    real se, sm;       // SIMP scalings
    real dse, dsm;     // their derivatives w.r.t. phi
    real Pe[D][D];     // elastic stress
    real P[D][D];      // total stress
    real A[D][D];      // m C - (4 dt / dx^2) V P F^T
    StressCtx<real, D> ctx;
};

template <typename real, int D>
__device__ __forceinline__ void p2g_terms(const InstDev<real>& I, const Particle<real, D>& q, real phi,
                                          const real br[D], const real B[D], P2GTerms<real, D>& T)
{
    real pq, dpq;
    simp_pow(phi, I.simp_q, pq, dpq);
    T.se = I.simp_eps + (real(1) - I.simp_eps) * pq;
    T.sm = pq;
    T.dse = (real(1) - I.simp_eps) * dpq;
    T.dsm = dpq;
    T.m = I.mass_a + phi * I.mass_b;
    elastic_stress<real, D>(q.F, I.G, I.K, T.Pe, T.ctx);
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) T.P[i][j] = T.se * T.Pe[i][j] - T.sm * I.inv_mu0 * B[i] * br[j];
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
        for (int j = 0; j < D; ++j) {
            real s = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) s += T.P[i][k] * q.F[j][k];
            T.A[i][j] = T.m * q.C[i][j] - I.kappa_vol * s;
        }
}

template <typename real, int D>
__device__ __forceinline__ void field_at(const InstDev<real>& I, const real* bprog, int step, real B[D])
{
    int seg = segment_of(step, I.seg_steps, I.n_seg, I.periodic);
#pragma unroll
    for (int k = 0; k < D; ++k) B[k] = bprog[(int64_t)(I.seg_off + seg) * D + k];
}

// weight and dpos of one stencil node
template <typename real, int D>
__device__ __forceinline__ real node_weight(const Stencil<real, D>& S, const int a[D], real dx, real dpos[D])
{
    real w = real(1);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        w *= sel3(S.w[k], a[k]);
        dpos[k] = (real(a[k]) - S.f[k]) * dx;
    }
    return w;
}

// the same weight with the product taken over the outer axes first, so that
// stencil nodes sharing their (y, z) offsets share that partial product
template <typename real, int D>
__device__ __forceinline__ real node_weight_outer(const Stencil<real, D>& S, const int a[D], real dx, real dpos[D])
{
    real w = sel3(S.w[D - 1], a[D - 1]);
#pragma unroll
    for (int k = D - 2; k >= 0; --k) w = sel3(S.w[k], a[k]) * w;
#pragma unroll
    for (int k = 0; k < D; ++k) dpos[k] = (real(a[k]) - S.f[k]) * dx;
    return w;
}

template <typename real, int D>
__device__ __forceinline__ void node_grad(const Stencil<real, D>& S, const int a[D], real gw[D])
{
    real wk[D], dk[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        wk[k] = sel3(S.w[k], a[k]);
        dk[k] = sel3(S.dw[k], a[k]);
    }
    if (D == 2) {
        gw[0] = dk[0] * wk[1];
        gw[1] = wk[0] * dk[1];
    } else {
        gw[0] = dk[0] * wk[1] * wk[D - 1];
        gw[1] = wk[0] * dk[1] * wk[D - 1];
        gw[D - 1] = wk[0] * wk[1] * dk[D - 1];
    }
}

// --------------------------------------------------------------------------
// P2G (Eqs. 14-15)
// --------------------------------------------------------------------------

// P2G (Eqs. 14-15) of this block's particles from their state in registers
// (positions relative to the chunk origin): stress, affine momentum, and the
// scatter of (p, m) into staging list `list`. Inactive lanes carry a neutral
// state (zero mass).
template <typename real, int D>
__device__ __forceinline__ void p2g_scatter(const Args<real>& a, const InstDev<real>& I, bool active, int64_t i,
                                            const Particle<real, D>& q, int step, int list,
                                            typename LdsAcc<real>::T* lds)
{
    const int64_t S = a.nalloc;
    real phi = 0, br[D];
    if (active) {
        phi = a.phi[i];
#pragma unroll
        for (int k = 0; k < D; ++k) br[k] = a.br[k * S + i];
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) br[k] = real(0);
    }
    real B[D];
    field_at<real, D>(I, a.bprog, step, B);
    int org[3];
    chunk_origin(a.corig, a.chunk_base + blockIdx.x, org);
    Stencil<real, D> Sx;
    int err = make_stencil<real, D>(q.x, org, I.inv_dx, I.n_grid, Sx);
    if (active && err) report_error(a.err, step, 0, err);
    P2GTerms<real, D> T;
    p2g_terms<real, D>(I, q, phi, br, B, T);
    real mv[D];
#pragma unroll
    for (int k = 0; k < D; ++k) mv[k] = T.m * q.v[k];
    const real dx = I.dx;
    // magnitude bound of one contribution (weights <= 1, |dpos| <= 1.5 dx)
    real bnd[D + 1];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        real s = fabs(mv[r]);
#pragma unroll
        for (int c = 0; c < D; ++c) s += fabs(T.A[r][c]) * real(1.5) * dx;
        bnd[r] = s;
    }
    bnd[D] = T.m;
    scatter_box<real, D, D + 1>(a, I, lds, active, Sx.base, bnd, a.gm, list,
        [&](const int o[D], const real sq[D + 1], real& w, real u[D + 1]) {
            real dpos[D];
            w = node_weight_outer<real, D>(Sx, o, dx, dpos);
#pragma unroll
            for (int r = 0; r < D; ++r) {
                real s = mv[r] * sq[r];
#pragma unroll
                for (int c = D - 1; c >= 0; --c) s += (T.A[r][c] * sq[r]) * dpos[c];
                u[r] = s;
            }
            u[D] = T.m * sq[D];
        });
}

template <typename real, int D>
__device__ __forceinline__ void neutral_particle(Particle<real, D>& q)
{
#pragma unroll
    for (int k = 0; k < D; ++k) {
        q.x[k] = real(0.5);
        q.v[k] = real(0);
#pragma unroll
        for (int b = 0; b < D; ++b) {
            q.C[k][b] = real(0);
            q.F[k][b] = k == b ? real(1) : real(0);
        }
    }
}

// Orders the lanes of each chunk so that particles sharing their current
// stencil base cell are adjacent, moving as few as possible: a particle's
// group is led by the first slot of the chunk with the same base cell, groups
// keep the order of their leaders and members their slot order. While the
// particles of each cell are contiguous (as the initial sort leaves them) the
// order is the identity. Groups are found in an LDS table over the chunk's box
// of base cells; a chunk whose box exceeds the table keeps slot order. Writes
// the lane order used by the particle kernels. st: the particle state.
constexpr int kLaneSortCells = 2048;
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_lane_sort(Args<real> a, const real* st, uint8_t* lperm)
{
    __shared__ int lead[kLaneSortCells];   // first slot of each cell of the box
    __shared__ int cnt[kLaneSortCells];    // particles per cell
    __shared__ int cellof[kBlock];         // box cell of each slot
    __shared__ int scan[kBlock];
    __shared__ int s_bb[kWaves][6];
    const int c = a.chunk_base + blockIdx.x;
    const ChunkDev ch = a.chunks[c];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    const int n = ch.count;
    const bool active = t < n;
    const int64_t c0 = (int64_t)c * kBlock;
    const int64_t S = a.nalloc;
    int base[D];
    {
        int org[3];
        chunk_origin(a.corig, c, org);
        real x[D];
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = active ? a.x0s[k * S + c0 + t] + st[(Comp<D>::X + k) * S + c0 + t] : real(0.5);
        Stencil<real, D> Sx;
        make_stencil<real, D>(x, org, I.inv_dx, I.n_grid, Sx);
#pragma unroll
        for (int k = 0; k < D; ++k) base[k] = Sx.base[k];
    }
    // the block's box of base cells
    int wlo[D], whi[D];
    wave_bounds<D>(base, active, wlo, whi);
    if ((t & 63) == 0)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            s_bb[t >> 6][k] = wlo[k];
            s_bb[t >> 6][3 + k] = whi[k];
        }
    __syncthreads();
    int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
    int vol = 1;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        int l = s_bb[0][k], h = s_bb[0][3 + k];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) {
            l = min(l, s_bb[w][k]);
            h = max(h, s_bb[w][3 + k]);
        }
        lo[k] = l;
        ext[k] = max(h - l + 1, 1);
        vol *= ext[k];
    }
    if (vol > kLaneSortCells) {   // block-uniform
        lperm[c0 + t] = (uint8_t)t;
        return;
    }
    for (int j = t; j < vol; j += kBlock) {
        lead[j] = kBlock;
        cnt[j] = 0;
    }
    __syncthreads();
    int li = -1;
    if (active) {
        li = (base[0] - lo[0]) + ext[0] * ((base[1] - lo[1]) + (D == 3 ? ext[1] * (base[D - 1] - lo[D - 1]) : 0));
        atomicMin(&lead[li], t);
        atomicAdd(&cnt[li], 1);
    }
    cellof[t] = li;
    __syncthreads();
    const int first = active ? lead[li] : t;
    // offsets of the groups: exclusive prefix over slots of the leaders' group sizes
    int v = (active && first == t) ? cnt[li] : 0;
    scan[t] = v;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
        const int u = t >= d ? scan[t - d] : 0;
        __syncthreads();
        scan[t] += u;
        __syncthreads();
    }
    if (active) {
        // members of the group at slots first .. t - 1 come before this one
        int rank = scan[first] - cnt[li];
        for (int j = first; j < t; ++j) rank += cellof[j] == li ? 1 : 0;
        lperm[c0 + rank] = (uint8_t)t;
    } else {
        lperm[c0 + t] = (uint8_t)t;
    }
}

template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_p2g(Args<real> a, const real* __restrict__ st, int step, int list)
{
    __shared__ typename LdsAcc<real>::T lds[4 * kBoxCap];
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    const bool active = t < ch.count;
    const int64_t i = lane_slot(a, t);
    Particle<real, D> q;
    if (active)
        load_particle<real, D>(st, a.x0s, a.nalloc, i, q);
    else
        neutral_particle(q);
    p2g_scatter<real, D>(a, I, active, i, q, step, list, lds);
}

// --------------------------------------------------------------------------
// grid operation (Eqs. 16-18 plus walls and clamp)
// --------------------------------------------------------------------------

template <typename real, int D>
__device__ __forceinline__ void node_ijk(const InstDev<real>& I, int local, int ijk[D])
{
    int n = I.n_grid;
    ijk[0] = local % n;
    if (D == 2) {
        ijk[1] = local / n;
    } else {
        ijk[1] = (local / n) % n;
        ijk[D - 1] = local / (n * n);
    }
}

// Signed distance of obstacle j at node position xi at time t (the shape sits
// at a + vel t) and its outward normal; <= 0 on and inside the solid. The box's
// distance is exact inside, a lower bound outside.
template <typename real, int D>
__device__ __forceinline__ real obstacle_sdf(const InstDev<real>& I, int j, const real xi[D], real t, real nrm[D])
{
    real y[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        y[k] = xi[k] - (I.obst_a[j][k] + I.obst_vel[j][k] * t);
        nrm[k] = real(0);
    }
    const int kind = I.obst_kind[j];
    if (kind == 1) {
        real d = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            nrm[k] = I.obst_b[j][k];
            d += y[k] * nrm[k];
        }
        return d;
    }
    if (kind == 2) {
        real r2 = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) r2 += y[k] * y[k];
        const real r = sqrt(r2);
        if (r > real(0)) {
#pragma unroll
            for (int k = 0; k < D; ++k) nrm[k] = y[k] / r;
        } else {
            nrm[1] = real(1);
        }
        return r - I.obst_b[j][0];
    }
    real best = -INFINITY;
    int kb = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const real q = fabs(y[k]) - I.obst_b[j][k];
        if (q > best) {
            best = q;
            kb = k;
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k)
        if (k == kb) nrm[k] = y[k] < real(0) ? real(-1) : real(1);
    return best;
}

// Eq. 18 against obstacle j (normal nrm) on node velocity u: 0 untouched,
// 1 set to v_b (no-slip, attached, no tangential motion or friction exceeding
// it), 2 sliding
template <typename real, int D>
__device__ __forceinline__ int obstacle_contact(const InstDev<real>& I, int j, const real nrm[D], real u[D])
{
    const int mode = I.obst_mode[j];
    if (mode == 2) {
#pragma unroll
        for (int k = 0; k < D; ++k) u[k] = I.obst_vel[j][k];
        return 1;
    }
    real r[D], vn = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        r[k] = u[k] - I.obst_vel[j][k];
        vn += r[k] * nrm[k];
    }
    if (!(vn < real(0))) return 0;
    real tv[D], t2 = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        tv[k] = r[k] - vn * nrm[k];
        t2 += tv[k] * tv[k];
    }
    const real t = sqrt(t2);
    const real sl = t + I.obst_mu[j] * vn;
    if (mode == 1 || t == real(0) || sl <= real(0)) {
#pragma unroll
        for (int k = 0; k < D; ++k) u[k] = I.obst_vel[j][k];
        return 1;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) u[k] = I.obst_vel[j][k] + sl / t * tv[k];
    return 2;
}

// What the grid transpose needs of each obstacle: its input velocity, normal
// and branch.
template <typename real, int D>
struct ObstTrace {
    real in[kMaxObst][D], nrm[kMaxObst][D];
    int br[kMaxObst];
};

// Transpose of the sliding map u -> v_b + (1 + mu vn / t) P (u - v_b) at input u:
// g <- (1 + mu vn / t) P g + mu (n / t - vn tv / t^3) (tv . g)
template <typename real, int D>
__device__ __forceinline__ void obstacle_slide_adj(const InstDev<real>& I, int j, const real nrm[D], const real u[D],
                                                   real g[D])
{
    real r[D], vn = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        r[k] = u[k] - I.obst_vel[j][k];
        vn += r[k] * nrm[k];
    }
    real tv[D], t2 = 0, ng = 0, tg = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        tv[k] = r[k] - vn * nrm[k];
        t2 += tv[k] * tv[k];
        ng += nrm[k] * g[k];
        tg += tv[k] * g[k];
    }
    const real t = sqrt(t2), mu = I.obst_mu[j];
    real o[D];
#pragma unroll
    for (int k = 0; k < D; ++k)
        o[k] = (real(1) + mu * vn / t) * (g[k] - ng * nrm[k]) + mu * (nrm[k] / t - vn * tv[k] / (t2 * t)) * tg;
#pragma unroll
    for (int k = 0; k < D; ++k) g[k] = o[k];
}

// Velocity of one node with mass m > 0 and momentum p at time t. Returns the
// floor branch (0 untouched, 1 zeroed, 2 sliding) and the intermediates the
// transpose needs: vh = p/m, u0 after damping and gravity, u1 after the floor,
// v final; tr (if given) records the obstacles.
template <typename real, int D>
__device__ __forceinline__ int node_velocity(const InstDev<real>& I, const int ijk[D], real m, const real p[D],
                                             real vh[D], real u0[D], real u1[D], real v[D], int wallz[D],
                                             bool& clamped, real t, ObstTrace<real, D>* tr, int* ocode = nullptr)
{
    const real rm = real(1) / m;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        vh[k] = p[k] * rm;
        u0[k] = I.damp * vh[k] + I.gdt[k];
        u1[k] = u0[k];
    }
    int branch = 0;
    if (I.floor_on && ijk[1] <= I.floor_jmax) {
        real vn = u0[1];
        if (vn < real(0)) {
            real t2 = 0;
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (k != 1) t2 += u0[k] * u0[k];
            real tn = sqrt(t2);
            real s = tn + I.floor_mu * vn;
            if (I.floor_noslip || tn == real(0) || s <= real(0)) {
                branch = 1;
#pragma unroll
                for (int k = 0; k < D; ++k) u1[k] = real(0);
            } else {
                branch = 2;
                real f = s / tn;
#pragma unroll
                for (int k = 0; k < D; ++k) u1[k] = (k == 1) ? real(0) : f * u0[k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) v[k] = u1[k];
    if (I.n_obst > 0) {
        real xi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) xi[k] = (real)ijk[k] * I.dx;
        for (int j = 0; j < I.n_obst; ++j) {
            real nrm[D];
            int ob = 0;
            if (tr)
#pragma unroll
                for (int k = 0; k < D; ++k) tr->in[j][k] = v[k];
            if (obstacle_sdf<real, D>(I, j, xi, t, nrm) <= real(0)) ob = obstacle_contact<real, D>(I, j, nrm, v);
            if (ocode) *ocode |= ob << (6 + 2 * j);
            if (tr) {
                tr->br[j] = ob;
#pragma unroll
                for (int k = 0; k < D; ++k) tr->nrm[j][k] = nrm[k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        wallz[k] = 0;
        if (ijk[k] < I.wall_cells && v[k] < real(0)) wallz[k] = 1;
        if (ijk[k] >= I.n_grid - I.wall_cells && v[k] > real(0)) wallz[k] = 1;
        if (wallz[k]) v[k] = real(0);
    }
    clamped = I.clamp_on && ijk[0] <= I.clamp_imax;
    if (clamped)
#pragma unroll
        for (int k = 0; k < D; ++k) v[k] = real(0);
    return branch;
}

// Grid-stride over the coarse blocks the P2G registered: gathers the staged
// boxes, applies Eqs. 16-18 and writes the node velocity to gv_out. When gmd_out
// is given (reverse sweep) the summed (momentum, mass) records are kept there
// for the grid transpose. When gs.data is given (recorded forward) the step's
// blocks also go to the grid store, if they fit (GridStore).
// The FP32 build is held to 64 VGPRs (8 waves per SIMD; 4 pairs in flight per
// thread instead of 8), so its workgroups fit beside the particle kernels of
// other instance groups sooner (measured 2% more steps per second on three
// streams; no change on one).
template <typename real, int D>
__global__ __launch_bounds__(kGridThreadsMax) __attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 ? 8 : 1)))
void k_grid(Args<real> a, real* gv_out, real* gmd_out, int list, GridStore<real> gs)
{
  const int n_act = a.active[list];
  int sbase = -1;   // first store slot of this step, -1 when not kept
  if (gs.base) {
      const int s0 = gs.idx == 0 ? 0 : gs.base[gs.idx];
      if (gs.data && (int64_t)s0 + n_act <= gs.cap) sbase = s0;
      if (blockIdx.x == 0 && threadIdx.x == 0) {
          if (gs.idx == 0) gs.base[0] = 0;
          const int64_t s1 = (int64_t)s0 + n_act;
          gs.base[gs.idx + 1] = s1 < kStoreCountMax ? (int)s1 : kStoreCountMax;
      }
  }
  for (int wi = blockIdx.x; wi < n_act * a.grid_parts; wi += gridDim.x) {
    const int ai = wi / a.grid_parts, part = wi - ai * a.grid_parts;
    const int b = a.active_list[list * a.n_coarse + ai];
    const InstDev<real>& I = a.inst[a.cb_inst[b]];
    real* keep = sbase >= 0 ? gs.data + (size_t)(sbase + ai) * Coarse<D>::nodes * 4 : nullptr;
    if (keep && part == 0 && threadIdx.x == 0) gs.blk[sbase + ai] = b;
    gather_coarse<real, D>(a, I, b, part, a.gm, [&](int64_t g, const int g3[3], int ln, const real node[4]) {
        real v[D];
        int code = 0;   // branch decisions (the layout of mpm_mag_set_branch_trace)
        if (node[3] > real(0)) {
            int ijk[D];
#pragma unroll
            for (int k = 0; k < D; ++k) ijk[k] = g3[k];
            real vh[D], u0[D], u1[D];
            int wz[D];
            bool cl;
            const int br = node_velocity<real, D>(I, ijk, node[3], node, vh, u0, u1, v, wz, cl,
                                                  (real)gs.step * I.dt, (ObstTrace<real, D>*)nullptr,
                                                  a.trace ? &code : (int*)nullptr);
            code |= 1 | (br << 1);
#pragma unroll
            for (int k = 0; k < D; ++k) code |= wz[k] << (3 + k);
        } else {
#pragma unroll
            for (int k = 0; k < D; ++k) v[k] = real(0);
        }
        if (a.trace) a.trace[(int64_t)gs.step * a.trace_nodes + I.trace_off + (g - I.grid_off)] = (uint16_t)code;
#pragma unroll
        for (int k = 0; k < D; ++k) gv_out[4 * g + k] = v[k];
        if (gmd_out)
#pragma unroll
            for (int q = 0; q < 4; ++q) gmd_out[4 * g + q] = node[q];
        if (keep) {
            real* o = keep + (size_t)ln * 4;
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = node[q];
        }
    });
  }
}

// Rebuilds one step's grid from a store entry into the dense velocity and
// (momentum, mass) arrays of the reverse sweep: the same nodes, with the same
// values, that k_grid writes there when it recomputes the step (the velocity
// from the kept record by the same grid operation).
template <typename real, int D>
__global__ __launch_bounds__(kGridBlock) void k_grid_restore(Args<real> a, GridStore<real> gs, real* gv_out,
                                                             real* gmd_out)
{
  using CB = Coarse<D>;
  const int s0 = gs.idx == 0 ? 0 : gs.base[gs.idx];
  const int s1 = gs.base[gs.idx + 1];
  if (s1 > gs.cap) {   // not kept: nothing to read (the host sizes stores so this does not happen)
      if (blockIdx.x == 0 && threadIdx.x == 0) report_error(a.err, gs.step, 1, kErrStore);
      return;
  }
  for (int sl = s0 + blockIdx.x; sl < s1; sl += gridDim.x) {
    const int b = gs.blk[sl];
    const InstDev<real>& I = a.inst[a.cb_inst[b]];
    const int lb = b - I.cb_off;
    const int co[3] = {(lb % I.nb) * CB::edge, (D == 3 ? (lb / I.nb) % I.nb : lb / I.nb) * CB::edge,
                       D == 3 ? (lb / (I.nb * I.nb)) * CB::edge : 0};
    const real* src = gs.data + (size_t)sl * CB::nodes * 4;
    for (int ln = threadIdx.x; ln < CB::nodes; ln += blockDim.x) {
        const int g3[3] = {co[0] + ln % CB::edge, co[1] + (ln / CB::edge) % CB::edge,
                           D == 3 ? co[2] + ln / (CB::edge * CB::edge) : 0};
        if (g3[0] >= I.n_grid || g3[1] >= I.n_grid || (D == 3 && g3[2] >= I.n_grid)) continue;
        const int64_t g = (int64_t)I.grid_off + g3[0] +
                          (int64_t)I.n_grid * (g3[1] + (D == 3 ? (int64_t)I.n_grid * g3[2] : 0));
        real node[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) node[q] = src[(size_t)ln * 4 + q];
        real v[D];
        if (node[3] > real(0)) {
            int ijk[D];
#pragma unroll
            for (int k = 0; k < D; ++k) ijk[k] = g3[k];
            real vh[D], u0[D], u1[D];
            int wz[D];
            bool cl;
            node_velocity<real, D>(I, ijk, node[3], node, vh, u0, u1, v, wz, cl, (real)gs.step * I.dt,
                                   (ObstTrace<real, D>*)nullptr);
        } else {
#pragma unroll
            for (int k = 0; k < D; ++k) v[k] = real(0);
        }
#pragma unroll
        for (int k = 0; k < D; ++k) gv_out[4 * g + k] = v[k];
#pragma unroll
        for (int q = 0; q < 4; ++q) gmd_out[4 * g + q] = node[q];
    }
  }
}

// --------------------------------------------------------------------------
// G2P (Eqs. 19-22)
// --------------------------------------------------------------------------

// G2P (Eqs. 19-22) of one active particle from the velocities of its stencil's
// nodes, node (base + a) at g0 + 4 a_x + sy a_y + sz a_z (the instance grid,
// or a box of it in LDS): update v, C, F and the displacement (stored in q.x);
// x1 gets the new position relative to the chunk origin. Returns the error flags.
template <typename real, int D>
__device__ __forceinline__ int g2p_from_nodes(const Args<real>& a, const InstDev<real>& I, int64_t i,
                                              const Stencil<real, D>& Sx, const real* g0, int sy, int sz,
                                              const real F[D][D], const real u[D], const int org[3],
                                              Particle<real, D>& q, real x1[D])
{
    const int64_t S = a.nalloc;
    // sums over the 3^D nodes (all unrolled, by rows along x) of w v and of
    // w v b_c with centred node offsets b_c = a_c - 1 in {-1, 0, 1}; with
    // dpos = (a - f) dx, sum w v dpos_c = dx (sum w v b_c - (f_c - 1) sum w v),
    // where |f_c - 1| <= 1/2 keeps the cancellation small in FP32
    real vn[D], Ba[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        vn[r] = 0;
#pragma unroll
        for (int c = 0; c < D; ++c) Ba[r][c] = 0;
    }
    const real wx0 = Sx.w[0][0], wx1 = Sx.w[0][1], wx2 = Sx.w[0][2];
#pragma unroll
    for (int a2 = 0; a2 < (D == 3 ? 3 : 1); ++a2)
#pragma unroll
        for (int a1 = 0; a1 < 3; ++a1) {
            const real wyz = Sx.w[1][a1] * (D == 3 ? Sx.w[D - 1][a2] : real(1));
            const real* row = g0 + sy * a1 + (D == 3 ? sz * a2 : 0);
            real v0[D], v1[D], v2[D];
            load_vec<real, D>(row, v0);
            load_vec<real, D>(row + 4, v1);
            load_vec<real, D>(row + 8, v2);
#pragma unroll
            for (int r = 0; r < D; ++r) {
                const real p0 = wx0 * v0[r], p2 = wx2 * v2[r];
                const real sw = wyz * fma(wx1, v1[r], p0 + p2);      // row sum of w v
                vn[r] += sw;
                Ba[r][0] = fma(wyz, p2 - p0, Ba[r][0]);
                if (a1 == 0) Ba[r][1] -= sw;
                if (a1 == 2) Ba[r][1] += sw;
                if (D == 3 && a2 == 0) Ba[r][D - 1] -= sw;
                if (D == 3 && a2 == 2) Ba[r][D - 1] += sw;
            }
        }
    real Bm[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int c = 0; c < D; ++c) Bm[r][c] = I.dx * fma(real(1) - Sx.f[c], vn[r], Ba[r][c]);
    real IdC[D][D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        q.v[r] = vn[r];
        q.x[r] = u[r] + I.dt * vn[r];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            q.C[r][c] = I.lam * Bm[r][c];
            IdC[r][c] = (r == c ? real(1) : real(0)) + I.dt * q.C[r][c];
        }
    }
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            real s = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) s += IdC[r][k] * F[k][c];
            q.F[r][c] = s;
        }
#pragma unroll
    for (int r = 0; r < D; ++r) x1[r] = a.x0s[r * S + i] + q.x[r];
    int err = 0;
    bool fin = true;
#pragma unroll
    for (int r = 0; r < D; ++r) {
        fin = fin && rfinite(q.x[r]) && rfinite(q.v[r]);
#pragma unroll
        for (int c = 0; c < D; ++c) fin = fin && rfinite(q.F[r][c]) && rfinite(q.C[r][c]);
    }
    if (!fin) {
        err |= kErrNonFinite;
    } else {
        if (!(det<real, D>(q.F) > real(0))) err |= kErrInvert;
        Stencil<real, D> S1;
        err |= make_stencil<real, D>(x1, org, I.inv_dx, I.n_grid, S1);
    }
    return err;
}

// G2P of one active particle, gathering from the instance grid
template <typename real, int D>
__device__ __forceinline__ int g2p_update(const Args<real>& a, const InstDev<real>& I, int64_t i,
                                          const real* __restrict__ gv_in, const real* sin, const int org[3],
                                          Particle<real, D>& q, real x1[D])
{
    const int64_t S = a.nalloc;
    real x[D], F[D][D], u[D];
    load_xF<real, D>(sin, a.x0s, S, i, x, F);
#pragma unroll
    for (int k = 0; k < D; ++k) u[k] = sin[(Comp<D>::X + k) * S + i];
    Stencil<real, D> Sx;
    make_stencil<real, D>(x, org, I.inv_dx, I.n_grid, Sx);
    // the stencil's first node; the others are at small 32-bit offsets
    const int n = I.n_grid;
    const real* g0 = gv_in + 4 * ((int64_t)I.grid_off + node_index<real, D>(Sx.base, kZero3, n));
    return g2p_from_nodes<real, D>(a, I, i, Sx, g0, 4 * n, 4 * n * n, F, u, org, q, x1);
}

// mass-weighted velocity along the loss direction (trajectory loss, Eq. 39),
// summed over the block into the instance accumulator
template <typename real, int D>
__device__ __forceinline__ void traj_accumulate(const Args<real>& a, const InstDev<real>& I, int inst, bool active,
                                                int64_t i, const Particle<real, D>& q)
{
    double traj = 0.0;
    if (active) {
        real ve = 0;
#pragma unroll
        for (int r = 0; r < D; ++r) ve += I.loss_dir[r] * q.v[r];
        traj = (double)(I.mass_a + a.phi[i] * I.mass_b) * (double)ve;
    }
    double v1[1] = {traj};
    block_sum<1>(v1);
    if (threadIdx.x == 0) unsafeAtomicAdd(&acc_copy(a, a.chunk_base + blockIdx.x, inst)[kAccTraj], v1[0]);
}

// G2P of one step (no scatter follows): the recompute of a stored segment,
// and the forward's last step. slot_order: lanes take their own slots rather
// than the lane order, which serves only the scatter of the forward kernels.
// The new state is streamed out with non-temporal stores (a stashed state is
// read back only after the rest of its segment), and the kernel is bound to
// 6 waves per SIMD: it waits on memory more than it computes.
template <typename real, int D>
__global__ __launch_bounds__(kBlock, 6) void k_g2p(Args<real> a, const real* __restrict__ gv_in, const real* sin,
                                                real* sout, int step, int traj_on, int list_done, int slot_order)
{
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    const bool active = t < ch.count;
    const int64_t i = slot_order ? (int64_t)(a.chunk_base + blockIdx.x) * kBlock + t : lane_slot(a, t);
    if (blockIdx.x == 0 && t == 0) a.active[list_done] = 0;   // the grid update has consumed this list
    // the chunk's box of stencil nodes is staged in LDS once, so the 3^D node
    // reads of every particle hit LDS rather than the L2
    __shared__ real s_box[4 * kBoxCap];
    const int64_t S = a.nalloc;
    int org[3];
    chunk_origin(a.corig, a.chunk_base + blockIdx.x, org);
    real x[D], F[D][D], u[D];
    if (active) {
        load_xF<real, D>(sin, a.x0s, S, i, x, F);
#pragma unroll
        for (int k = 0; k < D; ++k) u[k] = sin[(Comp<D>::X + k) * S + i];
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) x[k] = real(0.5);
    }
    Stencil<real, D> Sx;
    make_stencil<real, D>(x, org, I.inv_dx, I.n_grid, Sx);
    const real* gv = gv_in + 4 * (int64_t)I.grid_off;
    const NodeBox<D> nb = stage_nodes<real, D>(I, active, Sx.base, gv, s_box, kBoxCap);
    Particle<real, D> q;
    if (active) {
        real x1[D];
        int err;
        if (nb.staged) {
            const int l = (Sx.base[0] - nb.lo[0]) +
                          nb.ext[0] * ((Sx.base[1] - nb.lo[1]) + (D == 3 ? nb.ext[1] * (Sx.base[D - 1] - nb.lo[D - 1]) : 0));
            err = g2p_from_nodes<real, D>(a, I, i, Sx, s_box + 4 * l, 4 * nb.ext[0], 4 * nb.ext[0] * nb.ext[1], F, u,
                                          org, q, x1);
        } else {
            const int n = I.n_grid;
            err = g2p_from_nodes<real, D>(a, I, i, Sx, gv + 4 * node_index<real, D>(Sx.base, kZero3, n), 4 * n,
                                          4 * n * n, F, u, org, q, x1);
        }
        if (err) report_error(a.err, step, 1, err);
        stream_particle<real, D>(sout, a.nalloc, i, q);
    }
    if (traj_on && I.loss_kind == kTrajVel) traj_accumulate<real, D>(a, I, ch.inst, active, i, q);
}

// G2P of step n and P2G of step n + 1 in one pass: the new state stays in
// registers for the scatter. x and F are always stored; v and C only when a
// later pass reads them (checkpoints, stashed states).
template <typename real, int D>
__global__ __launch_bounds__(kBlock, 6) void k_g2p2g(Args<real> a, const real* __restrict__ gv_in, const real* sin,
                                                  real* sout, int step, int traj_on, int store_vc, int list_done,
                                                  int list_next)
{
    using Cp = Comp<D>;
    __shared__ typename LdsAcc<real>::T lds[4 * kBoxCap];
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    const bool active = t < ch.count;
    const int64_t i = lane_slot(a, t);
    const int64_t S = a.nalloc;
    if (blockIdx.x == 0 && t == 0) a.active[list_done] = 0;
    Particle<real, D> q;
    if (active) {
        int org[3];
        chunk_origin(a.corig, a.chunk_base + blockIdx.x, org);
        real x1[D];
        const int err = g2p_update<real, D>(a, I, i, gv_in, sin, org, q, x1);
        if (err) report_error(a.err, step, 1, err);
#pragma unroll
        for (int r = 0; r < D; ++r) {
            sout[(Cp::X + r) * S + i] = q.x[r];
#pragma unroll
            for (int c = 0; c < D; ++c) sout[(Cp::F + r * D + c) * S + i] = q.F[r][c];
        }
        if (store_vc) {
#pragma unroll
            for (int r = 0; r < D; ++r) {
                sout[(Cp::V + r) * S + i] = q.v[r];
#pragma unroll
                for (int c = 0; c < D; ++c) sout[(Cp::C + r * D + c) * S + i] = q.C[r][c];
            }
        }
#pragma unroll
        for (int r = 0; r < D; ++r) q.x[r] = x1[r];
    } else {
        neutral_particle(q);
    }
    if (traj_on && I.loss_kind == kTrajVel) traj_accumulate<real, D>(a, I, ch.inst, active, i, q);
    p2g_scatter<real, D>(a, I, active, i, q, step + 1, list_next, lds);
}

// --------------------------------------------------------------------------
// losses (Eqs. 36-40)
// --------------------------------------------------------------------------

// sums per instance: total mass, sum m e.(x - x0), masked squared distance,
// mask count, masked e.(x - x0)
template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_loss_sums(Args<real> a, const real* st, const real* x0s,
                                                      const real* target, const uint8_t* mask, int has_target)
{
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    const int64_t i = (int64_t)(a.chunk_base + blockIdx.x) * kBlock + t;
    const int64_t S = a.nalloc;
    double v[5] = {0, 0, 0, 0, 0};
    if (t < ch.count) {
        double m = (double)I.mass_a + (double)a.phi[i] * (double)I.mass_b;
        int mk = mask ? mask[i] : 1;
        double de = 0, sq = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double uk = st[(Comp<D>::X + k) * S + i];
            de += (double)I.loss_dir[k] * uk;
            if (has_target) {
                double r = uk - (double)target[k * S + i];
                sq += r * r;
            }
        }
        v[0] = m;
        v[1] = m * de;
        v[2] = mk ? sq : 0.0;
        v[3] = mk ? 1.0 : 0.0;
        v[4] = mk ? de : 0.0;
    }
    block_sum<5>(v);
    if (t == 0) {
        double* acc = acc_copy(a, a.chunk_base + blockIdx.x, ch.inst);
        unsafeAtomicAdd(&acc[kAccMass], v[0]);
        unsafeAtomicAdd(&acc[kAccS1], v[1]);
        unsafeAtomicAdd(&acc[kAccSq], v[2]);
        unsafeAtomicAdd(&acc[kAccCnt], v[3]);
        unsafeAtomicAdd(&acc[kAccTip], v[4]);
    }
}

template <typename real>
__global__ void k_loss_finalize(Args<real> a, int n_inst, real* loss_out)
{
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_inst) return;
    const InstDev<real>& I = a.inst[k];
    // sum the copies in copy order and leave the totals in copy 0, where the
    // seed and the adjoint read them
    double acc[kAccCount];
    double* acc0 = a.acc + (int64_t)k * kAccCount;
#pragma unroll
    for (int j = 0; j < kAccCount; ++j) {
        double s = 0.0;
        for (int r = 0; r < kGbCopies; ++r) s += acc0[(int64_t)r * a.acc_stride + j];
        acc[j] = s;
    }
#pragma unroll
    for (int j = 0; j < kAccCount; ++j) acc0[j] = acc[j];
    double L = 0;
    switch (I.loss_kind) {
    case kFinalMse: L = acc[kAccCnt] > 0 ? acc[kAccSq] / acc[kAccCnt] : 0.0; break;
    case kComDisp: L = -acc[kAccS1] / acc[kAccMass]; break;
    case kTrajVel: L = -(double)I.dt * acc[kAccTraj] / acc[kAccMass]; break;
    default: L = acc[kAccCnt] > 0 ? -acc[kAccTip] / acc[kAccCnt] : 0.0; break;
    }
    a.loss_val[k] = L;
    if (loss_out) loss_out[k] = (real)L;
}

// --------------------------------------------------------------------------
// adjoint seeds at the final state and direct density terms
// --------------------------------------------------------------------------

template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_seed(Args<real> a, const real* st, real* adj, const real* x0s,
                                                 const real* target, const uint8_t* mask, const real* dloss,
                                                 const int* __restrict__ id, const real* __restrict__ dx_final)
{
    using Cp = Comp<D>;
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    if (t >= ch.count) return;
    const int64_t i = (int64_t)(a.chunk_base + blockIdx.x) * kBlock + t;
    const int64_t S = a.nalloc;
    const double* acc = a.acc + ch.inst * kAccCount;
    const double dl = (double)dloss[ch.inst];
    const double M = acc[kAccMass];
    const double L = a.loss_val[ch.inst];
    const double m = (double)I.mass_a + (double)a.phi[i] * (double)I.mass_b;
    const int mk = mask ? mask[i] : 1;
    double gphi = 0, de = 0;
    real xb[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        double uk = st[(Cp::X + k) * S + i];
        double e = I.loss_dir[k];
        de += e * uk;
        double s = 0;
        switch (I.loss_kind) {
        case kFinalMse: s = mk ? dl * 2.0 * (uk - (double)target[k * S + i]) / acc[kAccCnt] : 0.0; break;
        case kTipDisp: s = mk ? -dl * e / acc[kAccCnt] : 0.0; break;
        case kComDisp: s = -dl * m * e / M; break;
        default: s = 0.0; break;
        }
        // an upstream gradient on the final positions (the caller's order)
        if (dx_final) s += (double)dx_final[(int64_t)id[i] * D + k];
        xb[k] = (real)s;
    }
    if (I.loss_kind == kComDisp || I.loss_kind == kTrajVel)
        gphi = dl * (double)I.mass_b * (-de / M - L / M);
#pragma unroll
    for (int c = 0; c < Cp::NC; ++c) adj[c * S + i] = real(0);
#pragma unroll
    for (int k = 0; k < D; ++k) adj[(Cp::X + k) * S + i] = xb[k];
    a.gphi[i] = (real)gphi;
#pragma unroll
    for (int k = 0; k < D; ++k) a.gbr[k * S + i] = real(0);
}

// --------------------------------------------------------------------------
// G2P transpose: adjoint of state n+1 -> grid velocity adjoint (scatter) and
// the G2P share of the adjoint of state n
// --------------------------------------------------------------------------

// adjoint of one particle's state (x, v, C, F)
template <typename real, int D>
struct AdjState {
    real x[D], v[D], C[D][D], F[D][D];
};

template <typename real, int D>
__device__ __forceinline__ void adj_zero(AdjState<real, D>& A)
{
#pragma unroll
    for (int r = 0; r < D; ++r) {
        A.x[r] = A.v[r] = real(0);
#pragma unroll
        for (int c = 0; c < D; ++c) A.C[r][c] = A.F[r][c] = real(0);
    }
}

// Transpose of the G2P of step n for the particles of this block: from the
// adjoint A1 of state n+1 (registers), state n (st) and the v and C of state
// n+1 (st_next: the sums over the stencil that the G2P produced), scatter the
// grid velocity adjoint (list `list` of the scatter phases) and store the G2P
// share of the adjoint of state n (x and F parts) in adj. lds: 4 kBoxCap words.
template <typename real, int D>
__device__ __forceinline__ void g2p_adj_phase(const Args<real>& a, const InstDev<real>& I, int inst, bool active,
                                              int64_t i, const real* __restrict__ gv_in, const real* st,
                                              const real* st_next, AdjState<real, D>& A1, real* adj,
                                              const real* dloss, int list, typename LdsAcc<real>::T* lds)
{
    using Cp = Comp<D>;
    const int64_t S = a.nalloc;
    real x[D], F[D][D];
    if (active) {
        load_xF<real, D>(st, a.x0s, S, i, x, F);
        if (I.loss_kind == kTrajVel) {
            const double M = a.acc[inst * kAccCount + kAccMass];
            const double sc = -(double)dloss[inst] * (double)I.dt *
                              ((double)I.mass_a + (double)a.phi[i] * (double)I.mass_b) / M;
#pragma unroll
            for (int k = 0; k < D; ++k) A1.v[k] += (real)(sc * (double)I.loss_dir[k]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            x[k] = real(0.5);
#pragma unroll
            for (int c = 0; c < D; ++c) F[k][c] = k == c ? real(1) : real(0);
        }
    }
    int org[3];
    chunk_origin(a.corig, a.chunk_base + blockIdx.x, org);
    Stencil<real, D> Sx;
    make_stencil<real, D>(x, org, I.inv_dx, I.n_grid, Sx);
    const real* gv = gv_in + 4 * (int64_t)I.grid_off;
    // the velocity box is staged in the LDS that later holds the scatter box
    real* glds = reinterpret_cast<real*>(lds);
    const NodeBox<D> nbx = stage_nodes<real, D>(I, active, Sx.base, gv, glds, kBoxCap);
    // x' = x + dt v' and F' = (I + dt C') F give vbt = vb' + dt xb' and
    // Cbt = Cb' + dt Fb' F^T, neither of which depends on C'
    real Cbt[D][D], vbt[D], xb[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        vbt[r] = A1.v[r] + I.dt * A1.x[r];
        xb[r] = A1.x[r];
#pragma unroll
        for (int c = 0; c < D; ++c) {
            real u = A1.C[r][c];
#pragma unroll
            for (int k = 0; k < D; ++k) u += I.dt * A1.F[r][k] * F[c][k];
            Cbt[r][c] = u;
        }
    }
    const real lam = I.lam, dx = I.dx;
    // one gather pass: C' of the forward G2P, and the share of xbar through the
    // weights and dpos, which needs the grid velocity:
    // xb += (v_i . u_i) grad w - lam w Cbt^T v_i,  u_i = vbt + lam Cbt dpos_i
    // (the last term is lam Cbt^T v', with v' = sum w v_i the velocity of
    // state n+1)
    if (active) {
        // lam Cbt, and dpos_x and the x factors of the weights of the three
        // x offsets (the weights factor as in the P2G transpose)
        real lC[D][D], d0[3], wx[3], dwx[3];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) lC[r][c] = lam * Cbt[r][c];
#pragma unroll
        for (int a0 = 0; a0 < 3; ++a0) {
            d0[a0] = (real(a0) - Sx.f[0]) * dx;
            wx[a0] = Sx.w[0][a0];
            dwx[a0] = Sx.dw[0][a0];
        }
        with_stencil_rows<real, D>(nbx, glds, gv, Sx.base, I.n_grid, [&](const real* g0, int sy, int sz) {
#pragma unroll 1
            for (int a2 = 0; a2 < (D == 3 ? 3 : 1); ++a2)
#pragma unroll 1
                for (int a1 = 0; a1 < 3; ++a1) {
                    const real* row = g0 + sy * a1 + (D == 3 ? sz * a2 : 0);
                    const real d1 = (real(a1) - Sx.f[1]) * dx;
                    const real d2 = D == 3 ? (real(a2) - Sx.f[D - 1]) * dx : real(0);
                    const real wz = D == 3 ? sel3(Sx.w[D - 1], a2) : real(1);
                    const real dwz = D == 3 ? sel3(Sx.dw[D - 1], a2) : real(0);
                    const real wy = sel3(Sx.w[1], a1), dwy = sel3(Sx.dw[1], a1);
                    const real wyz = wy * wz, dwyz = dwy * wz, wydz = wy * dwz;
                    real h[D];   // u_i = vbt + lam Cbt dpos_i without its x term
#pragma unroll
                    for (int r = 0; r < D; ++r) {
                        real u = vbt[r];
                        if (D == 3) u += lC[r][D - 1] * d2;
                        h[r] = u + lC[r][1] * d1;
                    }
                    real cdx = 0, cwx = 0;   // row sums of (v_i . u_i) dwx and (v_i . u_i) wx
#pragma unroll
                    for (int a0 = 0; a0 < 3; ++a0) {
                        real vi[D];
                        load_vec<real, D>(row + 4 * a0, vi);
                        real vh = 0, vc = 0;
#pragma unroll
                        for (int r = 0; r < D; ++r) {
                            vh += vi[r] * h[r];
                            vc += vi[r] * lC[r][0];
                        }
                        const real vu = vh + d0[a0] * vc;
                        cdx += vu * dwx[a0];
                        cwx += vu * wx[a0];
                    }
                    xb[0] += wyz * cdx;
                    xb[1] += dwyz * cwx;
                    if (D == 3) xb[D - 1] += wydz * cwx;
                }
        });
        real v1[D];
#pragma unroll
        for (int r = 0; r < D; ++r) v1[r] = st_next[(Cp::V + r) * S + i];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            real ctv = 0;
#pragma unroll
            for (int r = 0; r < D; ++r) ctv += Cbt[r][k] * v1[r];
            xb[k] -= lam * ctv;
        }
    }
    // F' = (I + dt C') F  ->  Fb = (I + dt C')^T Fb', C' from state n+1
    real Fb[D][D];
    {
        real C1[D][D];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) C1[r][c] = active ? st_next[(Cp::C + r * D + c) * S + i] : real(0);
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
                real s = A1.F[r][c];
#pragma unroll
                for (int k = 0; k < D; ++k) s += I.dt * C1[k][r] * A1.F[k][c];
                Fb[r][c] = s;
            }
    }
    // scatter w u_i to the grid velocity adjoint (registers only)
    real bnd[D];
#pragma unroll
    for (int r = 0; r < D; ++r) {
        real s = fabs(vbt[r]);
#pragma unroll
        for (int c = 0; c < D; ++c) s += lam * fabs(Cbt[r][c]) * real(1.5) * dx;
        bnd[r] = s;
    }
    scatter_box<real, D, D>(a, I, lds, active, Sx.base, bnd, a.gbar, list,
        [&](const int o[D], const real sq[D], real& w, real u[D]) {
            real dpos[D];
            w = node_weight_outer<real, D>(Sx, o, dx, dpos);
#pragma unroll
            for (int r = 0; r < D; ++r) {
                real s = vbt[r] * sq[r];
#pragma unroll
                for (int c = D - 1; c >= 0; --c) s += (lam * Cbt[r][c] * sq[r]) * dpos[c];
                u[r] = s;
            }
        });
    if (active) {
#pragma unroll
        for (int k = 0; k < D; ++k) adj[(Cp::X + k) * S + i] = xb[k];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) adj[(Cp::F + r * D + c) * S + i] = Fb[r][c];
    }
}

template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_g2p_adj(Args<real> a, const real* __restrict__ gv_in, const real* st,
                                                    const real* st_next, real* adj, const real* dloss, int list,
                                                    int list_fwd_done)
{
    using Cp = Comp<D>;
    __shared__ typename LdsAcc<real>::T lds[4 * kBoxCap];
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    const bool active = t < ch.count;
    const int64_t i = (int64_t)(a.chunk_base + blockIdx.x) * kBlock + t;
    const int64_t S = a.nalloc;
    if (blockIdx.x == 0 && t == 0) a.active[list_fwd_done] = 0;   // the grid update has consumed this P2G list
    AdjState<real, D> A1;
    adj_zero(A1);
    if (active) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            A1.x[k] = adj[(Cp::X + k) * S + i];
            A1.v[k] = adj[(Cp::V + k) * S + i];
        }
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
                A1.C[r][c] = adj[(Cp::C + r * D + c) * S + i];
                A1.F[r][c] = adj[(Cp::F + r * D + c) * S + i];
            }
    }
    g2p_adj_phase<real, D>(a, I, ch.inst, active, i, gv_in, st, st_next, A1, adj, dloss, list, lds);
}

// --------------------------------------------------------------------------
// grid transpose: vbar -> (pbar, mbar), in place in gbar; clears gm
// --------------------------------------------------------------------------

template <typename real, int D>
__global__ __launch_bounds__(kGridThreadsMax) __attribute__((amdgpu_waves_per_eu(sizeof(real) == 4 ? 8 : 1)))
void k_grid_adj(Args<real> a, const real* __restrict__ gmd_in, real* __restrict__ gpm_out, int list, int step)
{
  const int n_act = a.active[list];
  for (int wi = blockIdx.x; wi < n_act * a.grid_parts; wi += gridDim.x) {
    const int ai = wi / a.grid_parts, part = wi - ai * a.grid_parts;
    const int b = a.active_list[list * a.n_coarse + ai];
    const InstDev<real>& I = a.inst[a.cb_inst[b]];
    gather_coarse<real, D>(a, I, b, part, a.gbar, [&](int64_t g, const int g3[3], int, const real vb[4]) {
        real node[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) node[q] = gmd_in[4 * g + q];
        real out[4] = {0, 0, 0, 0};
        if (node[3] > real(0)) {
            int ijk[D];
#pragma unroll
            for (int k = 0; k < D; ++k) ijk[k] = g3[k];
            real vh[D], u0[D], u1[D], v[D], gb[D];
            int wz[D];
            bool cl;
            ObstTrace<real, D> tr;
            int br = node_velocity<real, D>(I, ijk, node[3], node, vh, u0, u1, v, wz, cl, (real)step * I.dt,
                                            I.n_obst > 0 ? &tr : (ObstTrace<real, D>*)nullptr);
#pragma unroll
            for (int k = 0; k < D; ++k) gb[k] = cl ? real(0) : vb[k];
#pragma unroll
            for (int k = 0; k < D; ++k)
                if (wz[k]) gb[k] = real(0);
            for (int j = I.n_obst - 1; j >= 0; --j) {
                if (tr.br[j] == 1) {
#pragma unroll
                    for (int k = 0; k < D; ++k) gb[k] = real(0);
                } else if (tr.br[j] == 2) {
                    obstacle_slide_adj<real, D>(I, j, tr.nrm[j], tr.in[j], gb);
                }
            }
            if (br == 1) {
#pragma unroll
                for (int k = 0; k < D; ++k) gb[k] = real(0);
            } else if (br == 2) {
                // transpose of v_t (1 + mu vn / |v_t|), n = e_y, at u0
                real vn = u0[1];
                real t2 = 0, vtg = 0;
#pragma unroll
                for (int k = 0; k < D; ++k)
                    if (k != 1) {
                        t2 += u0[k] * u0[k];
                        vtg += u0[k] * gb[k];
                    }
                real tn = sqrt(t2);
                real mu_t = I.floor_mu / tn;
                real o[D];
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    real ptg = (k == 1) ? real(0) : gb[k];
                    real vt = (k == 1) ? real(0) : u0[k];
                    o[k] = ptg + mu_t * ((k == 1 ? vtg : real(0)) + vn * ptg - vn * vt * vtg / t2);
                }
#pragma unroll
                for (int k = 0; k < D; ++k) gb[k] = o[k];
            }
            const real rm = real(1) / node[3];
            real mb = 0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                real vhb = I.damp * gb[k];
                out[k] = vhb * rm;
                mb -= vhb * vh[k];
            }
            out[3] = mb * rm;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) gpm_out[4 * g + q] = out[q];
    });
  }
}

// --------------------------------------------------------------------------
// P2G transpose: gather (pbar, mbar) -> adjoint of state n and design
// --------------------------------------------------------------------------

// Transpose of the P2G of step n for the particles of this block: gather
// (pbar, mbar) of the grid transpose, accumulate the design gradients, and
// return the full adjoint A0 of state n (the G2P share of its x and F parts is
// read from adj). lds: 4 kBoxCap words.
template <typename real, int D>
__device__ __forceinline__ void p2g_adj_phase(const Args<real>& a, const InstDev<real>& I, int inst, bool active,
                                              int64_t i, const real* __restrict__ gpm_in, const real* st,
                                              const real* adj, int step, AdjState<real, D>& A0, real* lds)
{
    using Cp = Comp<D>;
    const int t = threadIdx.x;
    const int64_t S = a.nalloc;
    adj_zero(A0);   // inactive lanes keep a zero adjoint
    real B[D];
    field_at<real, D>(I, a.bprog, step, B);
    double gBl[D];
#pragma unroll
    for (int k = 0; k < D; ++k) gBl[k] = 0.0;
    Particle<real, D> q;
    real phi = 0, br[D];
    int org[3];
    chunk_origin(a.corig, a.chunk_base + blockIdx.x, org);
    Stencil<real, D> Sx;
    if (active) {
        load_particle<real, D>(st, a.x0s, S, i, q);
        phi = a.phi[i];
#pragma unroll
        for (int k = 0; k < D; ++k) br[k] = a.br[k * S + i];
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) q.x[k] = real(0.5);
    }
    make_stencil<real, D>(q.x, org, I.inv_dx, I.n_grid, Sx);
    const real* gsrc = gpm_in + 4 * (int64_t)I.grid_off;
    const NodeBox<D> nbx = stage_nodes<real, D>(I, active, Sx.base, gsrc, lds, kBoxCap);
    if (active) {
        P2GTerms<real, D> T;
        p2g_terms<real, D>(I, q, phi, br, B, T);
        // Sums over the stencil; the terms linear in a per-particle factor are
        // summed first and multiplied once after the loop:
        //   mb = sum w mbar_i + v . S0 + Ab : C,  vb = m S0,  xb -= A^T S0,
        //   S0 = sum w pbar_i,  Ab = sum w pbar_i dpos_i^T
        real smb = 0, S0[D], Ab[D][D], xb[D], mv[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            S0[r] = 0;
            xb[r] = 0;
            mv[r] = T.m * q.v[r];
#pragma unroll
            for (int c = 0; c < D; ++c) Ab[r][c] = 0;
        }
        // Outer (z, y) offsets run-time, x offsets unrolled. Every weight
        // factors into its x part and its (y, z) part, so the three nodes of a
        // row sum with their x factors only and the (y, z) factor multiplies
        // the row sums once: xb += coef grad w splits into
        // wyz sum coef dwx, dwyz sum coef wx and wydz sum coef wx.
        real d0[3], wx[3], dwx[3], wd0[3];
#pragma unroll
        for (int a0 = 0; a0 < 3; ++a0) {
            d0[a0] = (real(a0) - Sx.f[0]) * I.dx;
            wx[a0] = Sx.w[0][a0];
            dwx[a0] = Sx.dw[0][a0];
            wd0[a0] = wx[a0] * d0[a0];
        }
        with_stencil_rows<real, D>(nbx, lds, gsrc, Sx.base, I.n_grid, [&](const real* g0, int sy, int sz) {
#pragma unroll 1
            for (int a2 = 0; a2 < (D == 3 ? 3 : 1); ++a2)
#pragma unroll 1
                for (int a1 = 0; a1 < 3; ++a1) {
                    const real* row = g0 + sy * a1 + (D == 3 ? sz * a2 : 0);
                    const real d1 = (real(a1) - Sx.f[1]) * I.dx;
                    const real d2 = D == 3 ? (real(a2) - Sx.f[D - 1]) * I.dx : real(0);
                    const real wz = D == 3 ? sel3(Sx.w[D - 1], a2) : real(1);
                    const real dwz = D == 3 ? sel3(Sx.dw[D - 1], a2) : real(0);
                    const real wy = sel3(Sx.w[1], a1), dwy = sel3(Sx.dw[1], a1);
                    const real wyz = wy * wz, dwyz = dwy * wz, wydz = wy * dwz;
                    real h[D];   // m v + A dpos without its x term
#pragma unroll
                    for (int r = 0; r < D; ++r) {
                        real u = mv[r];
                        if (D == 3) u += T.A[r][D - 1] * d2;
                        h[r] = u + T.A[r][1] * d1;
                    }
                    // row sums with the x factors of the weights
                    real cdx = 0, cwx = 0, smw = 0, U[D], V[D];
#pragma unroll
                    for (int r = 0; r < D; ++r) U[r] = V[r] = real(0);
#pragma unroll
                    for (int a0 = 0; a0 < 3; ++a0) {
                        const real* nd = row + 4 * a0;
                        real pb[D];
                        load_vec<real, D>(nd, pb);
                        const real mbi = nd[3];
                        // pb . (h + A[:, 0] dpos_x), as two dots so no product
                        // of A with the x offsets has to stay live
                        real ph = 0, pa = 0;
#pragma unroll
                        for (int r = 0; r < D; ++r) {
                            ph += pb[r] * h[r];
                            pa += pb[r] * T.A[r][0];
                        }
                        const real coef = mbi * T.m + (ph + d0[a0] * pa);
                        cdx += coef * dwx[a0];
                        cwx += coef * wx[a0];
                        smw += wx[a0] * mbi;
#pragma unroll
                        for (int r = 0; r < D; ++r) {
                            U[r] += wx[a0] * pb[r];
                            V[r] += wd0[a0] * pb[r];
                        }
                    }
                    xb[0] += wyz * cdx;
                    xb[1] += dwyz * cwx;
                    if (D == 3) xb[D - 1] += wydz * cwx;
                    smb += wyz * smw;
#pragma unroll
                    for (int r = 0; r < D; ++r) {
                        const real uw = wyz * U[r];
                        S0[r] += uw;
                        Ab[r][0] += wyz * V[r];
                        Ab[r][1] += d1 * uw;
                        if (D == 3) Ab[r][D - 1] += d2 * uw;
                    }
                }
        });
        real mb = smb + ddot<real, D>(Ab, q.C), vb[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            mb += q.v[r] * S0[r];
            vb[r] = T.m * S0[r];
#pragma unroll
            for (int c = 0; c < D; ++c) xb[r] -= T.A[c][r] * S0[c];
        }
        // Recompute the stress here rather than keeping it live through the
        // gather loop (the empty asm hides F's value so the compiler does not
        // reuse the copy from before the loop); this halves register pressure.
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) asm volatile("" : "+v"(q.F[r][c]));
        p2g_terms<real, D>(I, q, phi, br, B, T);
        // A = m C - kappa V P F^T
        real Pb[D][D], Fbp[D][D], dP[D][D];
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
                real s = 0, u = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    s += Ab[r][k] * q.F[k][c];
                    u += Ab[k][r] * T.P[k][c];
                }
                Pb[r][c] = -I.kappa_vol * s;
                Fbp[r][c] = -I.kappa_vol * u;
            }
        elastic_stress_dir<real, D>(q.F, I.K, T.ctx, Pb, dP);
        // P = s_e P_e + s_m P_m, P_m = -(1/mu0) B (x) br ; m = phi rho V
        real PbPe = ddot<real, D>(Pb, T.Pe);
        real PbBBr = 0;
        real PtB[D], PBr[D];
#pragma unroll
        for (int r = 0; r < D; ++r) {
            PtB[r] = 0;
            PBr[r] = 0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                PtB[r] += Pb[c][r] * B[c];
                PBr[r] += Pb[r][c] * br[c];
                PbBBr += Pb[r][c] * B[r] * br[c];
            }
        }
        real gphi = I.mass_b * mb + T.dse * PbPe - T.dsm * I.inv_mu0 * PbBBr;
        a.gphi[i] += gphi;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            a.gbr[k * S + i] += -T.sm * I.inv_mu0 * PtB[k];
            gBl[k] = (double)(-T.sm * I.inv_mu0 * PBr[k]);
        }
        // adjoint of state n: x and F add to the G2P share, v and C are set
#pragma unroll
        for (int k = 0; k < D; ++k) {
            A0.x[k] = adj[(Cp::X + k) * S + i] + xb[k];
            A0.v[k] = vb[k];
        }
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
                A0.C[r][c] = T.m * Ab[r][c];
                A0.F[r][c] = adj[(Cp::F + r * D + c) * S + i] + Fbp[r][c] + T.se * dP[r][c];
            }
    }
    block_sum<D>(gBl);
    if (t == 0) {
        int seg = segment_of(step, I.seg_steps, I.n_seg, I.periodic);
#pragma unroll
        for (int k = 0; k < D; ++k)
            unsafeAtomicAdd(&a.gB[(int64_t)((a.chunk_base + blockIdx.x) % kGbCopies) * a.gB_stride +
                                  (int64_t)(I.seg_off + seg) * D + k],
                            gBl[k]);
    }
}

template <typename real, int D>
__global__ __launch_bounds__(kBlock, sizeof(real) == 4 ? 3 : 2) void k_p2g_adj(Args<real> a, const real* __restrict__ gpm_in,
                                                                             const real* st, real* adj, int step,
                                                                             int list_done)
{
    using Cp = Comp<D>;
    __shared__ real lds[4 * kBoxCap];
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    const bool active = t < ch.count;
    const int64_t i = (int64_t)(a.chunk_base + blockIdx.x) * kBlock + t;
    const int64_t S = a.nalloc;
    if (blockIdx.x == 0 && t == 0) a.active[list_done] = 0;   // the grid transpose has consumed this list
    AdjState<real, D> A0;
    p2g_adj_phase<real, D>(a, I, ch.inst, active, i, gpm_in, st, adj, step, A0, lds);
    if (active) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            adj[(Cp::X + k) * S + i] = A0.x[k];
            adj[(Cp::V + k) * S + i] = A0.v[k];
        }
#pragma unroll
        for (int r = 0; r < D; ++r)
#pragma unroll
            for (int c = 0; c < D; ++c) {
                adj[(Cp::C + r * D + c) * S + i] = A0.C[r][c];
                adj[(Cp::F + r * D + c) * S + i] = A0.F[r][c];
            }
    }
}

// Transposes of P2G at step n and of G2P at step n - 1 in one pass: the
// adjoint of state n stays in registers between them. Resets the scatter list
// the grid transpose of step n consumed and fills the other one for step n - 1.
template <typename real, int D>
__global__ __launch_bounds__(kBlock, sizeof(real) == 4 ? 4 : 2) void k_adj_fused(
    Args<real> a, const real* __restrict__ gpm_in, const real* st_n, int step, const real* __restrict__ gv_prev,
    const real* st_prev, real* adj, const real* dloss, int list_done, int list_next)
{
    __shared__ typename LdsAcc<real>::T lds[4 * kBoxCap];
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    const bool active = t < ch.count;
    const int64_t i = (int64_t)(a.chunk_base + blockIdx.x) * kBlock + t;
    if (blockIdx.x == 0 && t == 0) a.active[list_done] = 0;
    AdjState<real, D> A;
    p2g_adj_phase<real, D>(a, I, ch.inst, active, i, gpm_in, st_n, adj, step, A, reinterpret_cast<real*>(lds));
    __syncthreads();   // the LDS node box of the gather is reused below
    g2p_adj_phase<real, D>(a, I, ch.inst, active, i, gv_prev, st_prev, st_n, A, adj, dloss, list_next, lds);
}

// --------------------------------------------------------------------------
// input gather (caller order -> sorted slots) and output scatter
// --------------------------------------------------------------------------

template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_gather(Args<real> a, const int* __restrict__ sorted_ids,
                                                   const int64_t* __restrict__ caller_start, real* st, real* x0s,
                                                   real* phi, real* br, real* tgt, uint8_t* mask, int* id,
                                                   int4* corig, const real* x0_in, const real* phi_in,
                                                   const real* br_in, const real* tgt_in, const uint8_t* mask_in,
                                                   int64_t n_prog)
{
    using Cp = Comp<D>;
    __shared__ int s_min[kWaves][3];
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const InstDev<real>& I = a.inst[ch.inst];
    const int t = threadIdx.x;
    const bool active = t < ch.count;
    const int64_t i = (int64_t)(a.chunk_base + blockIdx.x) * kBlock + t;
    const int64_t S = a.nalloc;
    const int64_t local = (int64_t)(a.chunk_base + blockIdx.x - I.chunk_off) * kBlock + t;
    const int q = active ? sorted_ids[caller_start[ch.inst] + local] : 0;
    // origin cell of the chunk: lowest cell index over its particles per axis
    double xa[D];
    int cmin[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        xa[k] = active ? (double)x0_in[(int64_t)q * D + k] : 0.0;
        double c = floor(xa[k] * (double)I.n_grid);
        int ci = (active && c > -1e9 && c < 1e9) ? (int)c : 0x3fffffff;
        cmin[k] = wave_min(ci);
    }
    if ((t & 63) == 0)
#pragma unroll
        for (int k = 0; k < D; ++k) s_min[t >> 6][k] = cmin[k];
    __syncthreads();
    int org[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < D; ++k) {
        int m = s_min[0][k];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) m = min(m, s_min[w][k]);
        org[k] = (m == 0x3fffffff) ? 0 : m;
    }
    if (t == 0) corig[a.chunk_base + blockIdx.x] = make_int4(org[0], org[1], org[2], 0);
    // inputs must be finite: a NaN mass would otherwise read as an empty node
    if (blockIdx.x == 0)
        for (int64_t j = t; j < n_prog; j += kBlock)
            if (!rfinite(a.bprog[j])) report_error(a.err, 0, 0, kErrNonFinite);
    if (!active) return;
    {
        bool fin = rfinite(phi_in[q]);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            fin = fin && isfinite(xa[k]) && rfinite(br_in[(int64_t)q * D + k]);
            if (tgt_in) fin = fin && rfinite(tgt_in[(int64_t)q * D + k]);
        }
        if (!fin) report_error(a.err, 0, 0, kErrNonFinite);
    }
    id[i] = q;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const double o = (double)org[k] / (double)I.n_grid;
        st[(Cp::X + k) * S + i] = real(0);
        st[(Cp::V + k) * S + i] = real(0);
        x0s[k * S + i] = (real)(xa[k] - o);
        br[k * S + i] = br_in[(int64_t)q * D + k];
        // FINAL_MSE target as a displacement from the initial position
        if (tgt_in) tgt[k * S + i] = (real)((double)tgt_in[(int64_t)q * D + k] - xa[k]);
    }
#pragma unroll
    for (int r = 0; r < D; ++r)
#pragma unroll
        for (int c = 0; c < D; ++c) {
            st[(Cp::C + r * D + c) * S + i] = real(0);
            st[(Cp::F + r * D + c) * S + i] = r == c ? real(1) : real(0);
        }
    phi[i] = phi_in[q];
    mask[i] = mask_in ? mask_in[q] : 1;
}

template <typename real, int D>
__global__ __launch_bounds__(kBlock) void k_scatter_out(Args<real> a, const int* __restrict__ id, const real* st,
                                                        real* x_out, real* g_phi, real* g_br)
{
    const ChunkDev ch = a.chunks[a.chunk_base + blockIdx.x];
    const int t = threadIdx.x;
    if (t >= ch.count) return;
    const int64_t i = (int64_t)(a.chunk_base + blockIdx.x) * kBlock + t;
    const int64_t S = a.nalloc;
    const int64_t q = id[i];
    const InstDev<real>& I = a.inst[ch.inst];
    int org[3];
    chunk_origin(a.corig, a.chunk_base + blockIdx.x, org);
    if (x_out)
#pragma unroll
        for (int k = 0; k < D; ++k)
            x_out[q * D + k] = (real)((double)org[k] / (double)I.n_grid + (double)a.x0s[k * S + i] +
                                      (double)st[(Comp<D>::X + k) * S + i]);
    if (g_phi) g_phi[q] = a.gphi[i];
    if (g_br)
#pragma unroll
        for (int k = 0; k < D; ++k) g_br[q * D + k] = a.gbr[k * S + i];
}

// dst[k] = sum over the kGbCopies copies of src[k] (copies n apart), in copy order
template <typename real>
__global__ void k_sum_copies_out(const double* src, real* dst, int64_t n)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double s = 0.0;
    for (int r = 0; r < kGbCopies; ++r) s += src[(int64_t)r * n + k];
    dst[k] = (real)s;
}

}  // namespace mpm
