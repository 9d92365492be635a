// Host engine behind the C ABI: buffer plan in HBM, instance / chunk / grid
// tables, the per-rollout cell sort, the step loop with checkpoints, the
// reverse sweep over checkpoint segments (recompute, then transpose of every
// step), optional HIP-graph replay of step sequences and per-kernel timing.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "mpm_mag.h"
#include "kernels.hpp"
#include "sort.hpp"

namespace mpm {

enum KernelId {
    K_SORT = 0, K_GATHER, K_P2G, K_GRID, K_G2P, K_LOSS, K_CKPT, K_SEED,
    K_G2P_ADJ, K_GRID_ADJ, K_P2G_ADJ, K_OUT, K_ADJ_FUSED, K_G2P2G, K_RESTORE, K_COUNT
};

inline const char* kernel_name(int k)
{
    static const char* names[K_COUNT] = {"sort", "gather", "p2g", "grid_update", "g2p", "loss", "checkpoint",
                                         "seed", "g2p_adj", "grid_adj", "p2g_adj", "output",
                                         "p2g_g2p_adj", "g2p_p2g", "grid_restore"};
    return (k >= 0 && k < K_COUNT) ? names[k] : "";
}

struct KernelStat {
    int64_t launches = 0;
    double ms = 0.0;
    double bytes = 0.0;
    double flops = 0.0;
};

class EngineBase {
public:
    virtual ~EngineBase() = default;
    virtual int rollout(hipStream_t s, const void* x0, const void* density, const void* br, const void* b_prog,
                        const void* target, const uint8_t* mask, void* x_final, void* loss_out, int record) = 0;
    virtual int backward(hipStream_t s, const void* dloss, const void* dx_final, void* g_density, void* g_br,
                         void* g_b_prog) = 0;
    virtual int set_option(const char* key, int64_t value) = 0;
    virtual int64_t device_bytes() const = 0;
    virtual int set_trace(uint16_t* trace, int64_t elems) = 0;
    virtual int64_t trace_nodes() const = 0;
    // scatter fallback counts of the last rollout or backward (kScatStats values)
    virtual int scatter_stats(int64_t* out, int n) const = 0;
    int kernel_stats(int k, int64_t* launches, double* ms, double* bytes)
    {
        if (k == -1) {
            for (auto& s : stats_) s = KernelStat();
            return MPM_MAG_OK;
        }
        if (k < 0 || k >= K_COUNT) return MPM_MAG_EINVAL;
        if (launches) *launches = stats_[k].launches;
        if (ms) *ms = stats_[k].ms;
        if (bytes) *bytes = stats_[k].bytes;
        return MPM_MAG_OK;
    }
    int kernel_flops(int k, double* flops)
    {
        if (k < 0 || k >= K_COUNT || !flops) return MPM_MAG_EINVAL;
        *flops = stats_[k].flops;
        return MPM_MAG_OK;
    }
    std::string err;

protected:
    KernelStat stats_[K_COUNT];
};

#define MPM_HIP(call)                                                               \
    do {                                                                            \
        hipError_t e_ = (call);                                                     \
        if (e_ != hipSuccess) {                                                     \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                \
            return MPM_MAG_EHIP;                                                    \
        }                                                                           \
    } while (0)

template <typename real, int D>
class Engine : public EngineBase {
    using Cp = Comp<D>;

public:
    ~Engine() override { release(); }

    // ------------------------------------------------------------------ setup
    // ws: a device range the handle's buffers are carved from instead of being
    // allocated (the allocation-free entry point); the handle then runs plain
    // rollouts only, on the call's stream, and allocates no device memory.
    int init(const mpm_mag_instance_desc* descs, int n_inst, const int64_t* np, void* ws = nullptr,
             size_t ws_bytes = 0)
    {
        ws_ = (uint8_t*)ws;
        ws_bytes_ = ws ? ws_bytes : 0;
        ws_used_ = 0;
        if (!descs || !np || n_inst < 1 || n_inst > 4096) return fail(MPM_MAG_EINVAL, "bad instance list");
        n_inst_ = n_inst;
        T_ = descs[0].n_steps;
        int64_t chunk = 0, grid = 0, seg = 0, caller = 0;
        int max_axis_bits = 1;
        for (int k = 0; k < n_inst; ++k) {
            const mpm_mag_instance_desc& d = descs[k];
            if (d.dim != D) return fail(MPM_MAG_EINVAL, "all instances must share dim");
            if (d.n_steps != T_ || d.n_steps < 0) return fail(MPM_MAG_EINVAL, "all instances must share n_steps >= 0");
            if (d.n_grid < 8 || d.n_grid > 1024) return fail(MPM_MAG_EINVAL, "n_grid must be in [8, 1024]");
            if (np[k] < 1 || np[k] > (int64_t)1 << 30) return fail(MPM_MAG_EINVAL, "n_particles must be in [1, 2^30]");
            if (d.n_segments < 1) return fail(MPM_MAG_EINVAL, "n_segments must be >= 1");
            if (!(d.dt > 0) || !(d.particle_volume > 0) || !(d.mu0 > 0) || !(d.rho > 0))
                return fail(MPM_MAG_EINVAL, "dt, particle_volume, mu0 and rho must be positive");
            if (!(d.nu > -1.0 && d.nu < 0.5)) return fail(MPM_MAG_EINVAL, "nu must be in (-1, 1/2)");
            if (d.loss_kind < 0 || d.loss_kind > 3) return fail(MPM_MAG_EINVAL, "unknown loss_kind");
            if (d.wall_cells < 0 || d.wall_cells > d.n_grid / 2) return fail(MPM_MAG_EINVAL, "bad wall_cells");
            InstDev<real> I;
            std::memset(&I, 0, sizeof I);
            const double dx = 1.0 / d.n_grid;
            I.n_grid = d.n_grid;
            I.n_nodes = D == 2 ? d.n_grid * d.n_grid : d.n_grid * d.n_grid * d.n_grid;
            I.grid_off = (int)grid;
            I.n_steps = d.n_steps;
            I.seg_off = (int)seg;
            I.n_seg = d.n_segments;
            I.seg_steps = d.seg_steps > 0 ? d.seg_steps : (d.n_steps + d.n_segments - 1) / d.n_segments;
            if (I.seg_steps < 1) I.seg_steps = 1;
            I.periodic = d.periodic ? 1 : 0;
            I.floor_on = d.floor_on ? 1 : 0;
            I.wall_cells = d.wall_cells;
            I.loss_kind = d.loss_kind;
            I.clamp_on = d.clamp_xmax >= 0.0 ? 1 : 0;
            I.clamp_imax = -1;
            for (int i = 0; i < d.n_grid; ++i)
                if (i * dx <= d.clamp_xmax) I.clamp_imax = i;
            I.floor_jmax = -1;
            for (int j = 0; j < d.n_grid; ++j)
                if (j * dx <= d.floor_y) I.floor_jmax = j;
            I.floor_noslip = std::isinf(d.floor_mu) ? 1 : 0;
            I.chunk_off = (int)chunk;
            I.n_particles = (int)np[k];
            I.nb = (d.n_grid + Coarse<D>::edge - 1) / Coarse<D>::edge;
            I.cb_off = (int)n_cb_;
            I.trace_off = (int)trace_nodes_;
            trace_nodes_ += I.n_nodes;
            const int ncb = D == 2 ? I.nb * I.nb : I.nb * I.nb * I.nb;
            for (int b = 0; b < ncb; ++b) cb_inst_h_.push_back(k);
            n_cb_ += ncb;
            I.dx = (real)dx;
            I.inv_dx = (real)d.n_grid;
            I.dt = (real)d.dt;
            I.kappa_vol = (real)(4.0 * d.dt / (dx * dx) * d.particle_volume);
            I.lam = (real)(4.0 / (dx * dx));
            I.G = (real)(d.E / (2.0 * (1.0 + d.nu)));
            I.K = (real)(d.E / (3.0 * (1.0 - 2.0 * d.nu)));
            if (!(d.mass_eps >= 0.0 && d.mass_eps <= 1.0)) return fail(MPM_MAG_EINVAL, "mass_eps must be in [0, 1]");
            I.mass_a = (real)(d.mass_eps * d.rho * d.particle_volume);
            I.mass_b = (real)((1.0 - d.mass_eps) * d.rho * d.particle_volume);
            I.inv_mu0 = (real)(1.0 / d.mu0);
            I.simp_eps = (real)d.simp_eps;
            I.simp_q = (real)d.simp_q;
            I.damp = (real)(1.0 - d.damping * d.dt);
            for (int c = 0; c < 3; ++c) {
                I.gdt[c] = (real)(d.gravity[c] * d.dt);
                I.loss_dir[c] = (real)d.loss_dir[c];
            }
            I.floor_mu = I.floor_noslip ? (real)0 : (real)d.floor_mu;
            if (d.n_obstacles < 0 || d.n_obstacles > kMaxObst) return fail(MPM_MAG_EINVAL, "n_obstacles must be in [0, 4]");
            I.n_obst = d.n_obstacles;
            for (int j = 0; j < d.n_obstacles; ++j) {
                const mpm_mag_obstacle& o = d.obstacles[j];
                if (o.kind < MPM_MAG_OBSTACLE_HALFSPACE || o.kind > MPM_MAG_OBSTACLE_BOX)
                    return fail(MPM_MAG_EINVAL, "unknown obstacle kind");
                if (!(o.mu >= 0)) return fail(MPM_MAG_EINVAL, "obstacle friction must be >= 0");
                double len = 0;
                for (int k = 0; k < D; ++k) len += o.b[k] * o.b[k];
                len = std::sqrt(len);
                bool ok = std::isfinite(len);
                if (o.kind == MPM_MAG_OBSTACLE_HALFSPACE) ok = ok && len > 0;
                if (o.kind == MPM_MAG_OBSTACLE_SPHERE) ok = ok && o.b[0] > 0;
                if (o.kind == MPM_MAG_OBSTACLE_BOX)
                    for (int k = 0; k < D; ++k) ok = ok && o.b[k] > 0;
                for (int k = 0; k < D; ++k) ok = ok && std::isfinite(o.a[k]) && std::isfinite(o.vel[k]);
                if (!ok) return fail(MPM_MAG_EINVAL, "bad obstacle shape");
                I.obst_kind[j] = o.kind;
                I.obst_mode[j] = o.attached ? 2 : (std::isinf(o.mu) ? 1 : 0);
                I.obst_mu[j] = std::isinf(o.mu) ? (real)0 : (real)o.mu;
                for (int k = 0; k < 3; ++k) {
                    // the half-space's normal is stored unit length (divided in double)
                    const double bk = (o.kind == MPM_MAG_OBSTACLE_HALFSPACE) ? (k < D ? o.b[k] / len : 0.0) : o.b[k];
                    I.obst_a[j][k] = (real)o.a[k];
                    I.obst_b[j][k] = (real)bk;
                    I.obst_vel[j][k] = (real)o.vel[k];
                }
            }
            inst_h_.push_back(I);
            {
                // grid-store sizing before the first recorded rollout: coarse
                // blocks a step may touch, from the cells the particles fill
                const double cells = (double)np[k] * d.particle_volume / std::pow(dx, (double)D);
                const double est = 4.0 * std::ceil(cells / Coarse<D>::nodes) + 27.0;
                est_cb_inst_.push_back((int64_t)std::min<double>(est, (double)ncb));
            }
            caller_start_h_.push_back(caller);
            int n_ch = (int)((np[k] + kBlock - 1) / kBlock);
            for (int c = 0; c < n_ch; ++c) {
                ChunkDev ch;
                ch.inst = k;
                ch.count = (int)std::min<int64_t>(kBlock, np[k] - (int64_t)c * kBlock);
                chunks_h_.push_back(ch);
            }
            int n_gb = (I.n_nodes + kGridBlock - 1) / kGridBlock;
            for (int b = 0; b < n_gb; ++b) gblock_h_.push_back(k);
            chunk += n_ch;
            grid += (int64_t)n_gb * kGridBlock;
            // the instance grid offsets (InstDev::grid_off) and the coarse-block and
            // trace tables are 32-bit; node indices in the kernels are 64-bit
            if (grid > (int64_t)INT32_MAX)
                return fail(MPM_MAG_EINVAL, "the instances' grids hold more than 2^31 - 1 nodes together");
            seg += d.n_segments;
            caller += np[k];
            int abits = 1;
            while ((1 << abits) < d.n_grid) ++abits;
            max_axis_bits = std::max(max_axis_bits, abits);
            ckpt_desc_ = d.ckpt_every;
            if (d.ckpt_budget_bytes < 0) return fail(MPM_MAG_EINVAL, "ckpt_budget_bytes must be >= 0");
            if (d.ckpt_budget_bytes > 0 && (budget_desc_ == 0 || d.ckpt_budget_bytes < budget_desc_))
                budget_desc_ = d.ckpt_budget_bytes;
        }
        caller_start_h_.push_back(caller);
        N_ = caller;
        n_chunks_ = (int)chunk;
        nalloc_ = chunk * kBlock;
        G_ = grid;
        S_tot_ = (int)seg;
        int inst_bits = 0;
        while ((1 << inst_bits) < n_inst) ++inst_bits;
        const int max_cell_bits = D * max_axis_bits;
        kp_.n_inst = n_inst;
        kp_.cell_bits = max_cell_bits;
        kp_.axis_bits = max_axis_bits;
        kp_.curve = 0;
        if (max_cell_bits + inst_bits > 32) return fail(MPM_MAG_EINVAL, "too many grid cells x instances for the sort key");
        sort_passes_ = (max_cell_bits + inst_bits + 7) / 8;
        sort_blocks_ = (int)((N_ + kSortTile - 1) / kSortTile);
        int st_alloc = allocate();
        if (st_alloc) return st_alloc;
        plan_chains();
        return MPM_MAG_OK;
    }

    int set_option(const char* key, int64_t value) override
    {
        if (!key) return fail(MPM_MAG_EINVAL, "null option key");
        std::string k(key);
        if (k == "graph") {
            if (value != 0 && value != 1) return fail(MPM_MAG_EINVAL, "graph must be 0 or 1");
            graph_ = value != 0;
            return MPM_MAG_OK;
        }
        if (k == "kernel_timing") { timing_ = value != 0; return MPM_MAG_OK; }
        if (k == "streams") {
            if (value < 0 || value > kMaxChains) return fail(MPM_MAG_EINVAL, "streams must be in [0, 8]");
            streams_opt_ = (int)value;
            plan_chains();
            gs_valid_ = false;   // the store is laid out per chain
            ++plan_gen_;
            return MPM_MAG_OK;
        }
        if (k == "fuse_fwd") {
            fuse_fwd_ = value != 0;
            ++plan_gen_;
            return MPM_MAG_OK;
        }
        if (k == "fuse_adj") {
            fuse_adj_ = value != 0;
            ++plan_gen_;   // changes the captured launch sequence
            return MPM_MAG_OK;
        }
        if (k == "lane_sort") {
            lane_sort_ = value != 0;
            ++plan_gen_;   // changes the captured launch sequence
            if (!lane_sort_) {
                // back to the identity order, once queued work has finished with it
                MPM_HIP(hipDeviceSynchronize());
                std::vector<uint8_t> ident((size_t)nalloc_);
                for (size_t j = 0; j < ident.size(); ++j) ident[j] = (uint8_t)(j % kBlock);
                MPM_HIP(hipMemcpy(lperm_, ident.data(), ident.size(), hipMemcpyHostToDevice));
            }
            return MPM_MAG_OK;
        }
        if (k == "p2g_lds") {
            use_lds_ = value != 0;
            ++plan_gen_;   // kernel arguments of captured launches
            return MPM_MAG_OK;
        }
        if (k == "sort_curve") {
            if (value < 0 || value > 2) return fail(MPM_MAG_EINVAL, "sort_curve must be 0, 1 or 2");
            kp_.curve = (int)value;
            return MPM_MAG_OK;
        }
        if (k == "box_cap") {
            if (value < 64 || value > kBoxCap) return fail(MPM_MAG_EINVAL, "box_cap must be in [64, 1024]");
            box_cap_ = (int)value;
            ++plan_gen_;   // kernel arguments of captured launches
            return MPM_MAG_OK;
        }
        if (k == "grid_wgs") {
            if (value < 16 || value > (1 << 20)) return fail(MPM_MAG_EINVAL, "grid_wgs must be in [16, 2^20]");
            grid_wgs_ = (int)value;
            ++plan_gen_;   // baked into captured launches
            return MPM_MAG_OK;
        }
        if (k == "grid_threads") {
            if (value != 0 && (value < Coarse<D>::cap || value > kGridThreadsMax || value % 64))
                return fail(MPM_MAG_EINVAL, "grid_threads must be 0 or a multiple of 64 in [256, 1024]");
            grid_threads_ = (int)value;
            ++plan_gen_;   // baked into captured launches
            return MPM_MAG_OK;
        }
        if (k == "grid_parts") {
            if (value != 0 && (value < 1 || value > 8 || (value & (value - 1))))
                return fail(MPM_MAG_EINVAL, "grid_parts must be 0, 1, 2, 4 or 8");
            grid_parts_ = (int)value;
            ++plan_gen_;   // baked into captured launches
            return MPM_MAG_OK;
        }
        if (k == "grid_store") {
            if (value < -1 || value > ((int64_t)1 << 30)) return fail(MPM_MAG_EINVAL, "grid_store must be -1, 0 or MiB");
            gs_budget_mib_ = value;   // applied at the next recorded rollout
            return MPM_MAG_OK;
        }
        if (k == "ckpt_budget") {
            if (value < 0) return fail(MPM_MAG_EINVAL, "ckpt_budget must be >= 0 bytes");
            budget_opt_ = value;   // applied at the next recorded rollout
            return MPM_MAG_OK;
        }
        if (k == "ckpt_every") {
            if (value < 0 || value > (1 << 30)) return fail(MPM_MAG_EINVAL, "bad ckpt_every");
            ckpt_opt_ = (int)value;
            return MPM_MAG_OK;
        }
        return fail(MPM_MAG_EINVAL, "unknown option " + k);
    }

    int64_t device_bytes() const override { return bytes_; }

    // Branch trace: the forward steps of the following rollouts write every
    // node's grid-update decisions to trace[n][node] (see mpm_mag.h).
    int set_trace(uint16_t* trace, int64_t elems) override
    {
        if (trace && elems < (int64_t)std::max(1, T_) * trace_nodes_)
            return fail(MPM_MAG_EINVAL, "branch trace smaller than n_steps x trace nodes");
        trace_ = trace;
        ++plan_gen_;   // the pointer is baked into captured launches
        return MPM_MAG_OK;
    }
    int64_t trace_nodes() const override { return trace_nodes_; }
    int scatter_stats(int64_t* out, int n) const override
    {
        if (!out || n < 0) return MPM_MAG_EINVAL;
        for (int k = 0; k < n; ++k) out[k] = (k < kScatStats && err_h_) ? (int64_t)err_h_[1 + k] : 0;
        return MPM_MAG_OK;
    }

    // --------------------------------------------------------------- rollout
    int rollout(hipStream_t s, const void* x0, const void* density, const void* br, const void* b_prog,
                const void* target, const uint8_t* mask, void* x_final, void* loss_out, int record) override
    {
        err.clear();
        recorded_ = false;
        if (!x0 || !density || !br || !b_prog) return fail(MPM_MAG_EINVAL, "x0, density, br and b_prog are required");
        bool need_target = false;
        for (auto& I : inst_h_) need_target |= I.loss_kind == kFinalMse;
        if (need_target && !target) return fail(MPM_MAG_EINVAL, "a FINAL_MSE instance needs loss_target");
        has_target_ = target != nullptr;
        if (record && ws_) return fail(MPM_MAG_EINVAL, "a handle on static scratch runs plain rollouts (record = 0)");
        if (record) {
            int st = ensure_checkpoints();
            if (st) return st;
            st = ensure_store();
            if (st) return st;
        }
        MPM_HIP(hipMemsetAsync(err_d_, 0xff, sizeof(*err_d_), s));   // kNoError
        MPM_HIP(hipMemsetAsync(err_d_ + 1, 0, sizeof(*err_d_) * kScatStats, s));
        MPM_HIP(hipMemsetAsync(acc_, 0, sizeof(double) * kAccCount * n_inst_ * kGbCopies, s));
        MPM_HIP(hipMemsetAsync(gm_, 0, sizeof(real) * 4 * G_, s));
        MPM_HIP(hipMemsetAsync(reg_count_, 0, sizeof(int) * n_cb_, s));
        MPM_HIP(hipMemsetAsync(part_done_, 0, sizeof(int) * n_cb_, s));
        MPM_HIP(hipMemsetAsync(fb_used_, 0, sizeof(int) * n_cb_, s));
        MPM_HIP(hipMemsetAsync(active_, 0, sizeof(int) * 4 * kMaxChains, s));
        MPM_HIP(hipMemcpyAsync(bprog_, b_prog, sizeof(real) * S_tot_ * D, hipMemcpyDeviceToDevice, s));
        if (trace_) MPM_HIP(hipMemsetAsync(trace_, 0, sizeof(uint16_t) * (size_t)T_ * trace_nodes_, s));
        int st = sort_and_gather(s, (const real*)x0, (const real*)density, (const real*)br, (const real*)target, mask);
        if (st) return st;
        auto steps = [&](hipStream_t cs) -> int {
            int r = fork(cs);
            if (r) return r;
            for (int n = 0; n < T_; ++n)
                for (int q = 0; q < n_chains(); ++q) {
                    r = fwd_step(q, stream_of(q, cs), n, record != 0);
                    if (r) return r;
                }
            return join(cs);
        };
        auto steps_of = [&](int q, hipStream_t cs) -> int {
            for (int n = 0; n < T_; ++n) {
                int r = fwd_step(q, cs, n, record != 0);
                if (r) return r;
            }
            return MPM_MAG_OK;
        };
        if (use_graph() && n_chains() > 1)
            st = replay_chains(s, gfwd_c_[record ? 1 : 0], steps_of, plan_gen_);
        else
            st = use_graph() ? replay(s, gfwd_[record ? 1 : 0], steps) : steps(s);
        if (st) return st;
        Args<real> a = args();
        st = launch(K_LOSS, s, n_chunks_, kBlock, k_loss_sums<real, D>, a, (const real*)st_, (const real*)x0s_,
                    (const real*)tgt_, (const uint8_t*)mask_, has_target_ ? 1 : 0);
        if (st) return st;
        st = launch(K_LOSS, s, (n_inst_ + 63) / 64, 64, k_loss_finalize<real>, a, n_inst_, (real*)loss_out);
        if (st) return st;
        if (x_final) {
            st = launch(K_OUT, s, n_chunks_, kBlock, k_scatter_out<real, D>, a, (const int*)id_, (const real*)st_,
                        (real*)x_final, (real*)nullptr, (real*)nullptr);
            if (st) return st;
        }
        st = finish(s);
        if (st) return st;
        if (record && T_ > 0) {
            // per-step active block counts of every chain (and which steps the store kept)
            gs_base_h_.assign((size_t)n_chains() * (T_ + 1), 0);
            MPM_HIP(hipMemcpy(gs_base_h_.data(), gs_base_, sizeof(int) * gs_base_h_.size(), hipMemcpyDeviceToHost));
            gs_count_chains_ = n_chains();
            gs_valid_ = true;
        }
        recorded_ = record != 0;
        return MPM_MAG_OK;
    }

    // -------------------------------------------------------------- backward
    int backward(hipStream_t s, const void* dloss, const void* dx_final, void* g_density, void* g_br,
                 void* g_b_prog) override
    {
        err.clear();
        if (!recorded_) return fail(MPM_MAG_ESTATE, "backward needs a successful record=1 rollout");
        if (!dloss) return fail(MPM_MAG_EINVAL, "dloss is required");
        MPM_HIP(hipMemsetAsync(err_d_, 0xff, sizeof(*err_d_), s));   // kNoError
        MPM_HIP(hipMemsetAsync(err_d_ + 1, 0, sizeof(*err_d_) * kScatStats, s));
        MPM_HIP(hipMemsetAsync(gB_, 0, sizeof(double) * S_tot_ * D * kGbCopies, s));
        MPM_HIP(hipMemcpyAsync(dloss_, dloss, sizeof(real) * n_inst_, hipMemcpyDeviceToDevice, s));
        MPM_HIP(hipMemsetAsync(active_, 0, sizeof(int) * 4 * kMaxChains, s));
        int st = ensure_seg_store();
        if (st) return st;
        Args<real> a = args();
        st = launch(K_SEED, s, n_chunks_, kBlock, k_seed<real, D>, a, (const real*)st_, adj_,
                        (const real*)x0s_, (const real*)tgt_, (const uint8_t*)mask_, (const real*)dloss_,
                        (const int*)id_, (const real*)dx_final);
        if (st) return st;
        auto sweep = [&](hipStream_t cs) -> int {
            int r = fork(cs);
            if (r) return r;
            for (int c = nck_ - 1; c >= 0; --c) {
                const int s0 = c * K_;
                const int s1 = std::min(T_, s0 + K_);
                if (s1 <= s0) continue;   // no step to reverse (T = 0)
                // recompute the segment, keeping every step's grid (sparse: only
                // the active coarse blocks are written)
                for (int n = s0; n < s1; ++n)
                    for (int q = 0; q < n_chains(); ++q) {
                        r = recompute_step(q, stream_of(q, cs), c, n);
                        if (r) return r;
                    }
                // transpose of every step, last first
                for (int q = 0; q < n_chains(); ++q) {
                    r = reverse_first(q, stream_of(q, cs), c);
                    if (r) return r;
                }
                for (int n = s1 - 1; n >= s0; --n)
                    for (int q = 0; q < n_chains(); ++q) {
                        r = reverse_step(q, stream_of(q, cs), c, n);
                        if (r) return r;
                    }
            }
            return join(cs);
        };
        std::vector<char> sig;
        for (int c = 0; c < nck_; ++c)
            for (int q = 0; q < n_chains(); ++q) sig.push_back(seg_stored(q, c) ? 1 : 0);
        if (sig != bwd_sig_) {
            bwd_sig_ = sig;
            ++bwd_gen_;   // another mix of stored and recomputed segments
        }
        auto sweep_of = [&](int q, hipStream_t cs) -> int {
            for (int c = nck_ - 1; c >= 0; --c) {
                const int s0 = c * K_;
                const int s1 = std::min(T_, s0 + K_);
                if (s1 <= s0) continue;
                int r;
                for (int n = s0; n < s1; ++n)
                    if ((r = recompute_step(q, cs, c, n))) return r;
                if ((r = reverse_first(q, cs, c))) return r;
                for (int n = s1 - 1; n >= s0; --n)
                    if ((r = reverse_step(q, cs, c, n))) return r;
            }
            return MPM_MAG_OK;
        };
        const int64_t bkey = (plan_gen_ << 24) ^ bwd_gen_;
        if (use_graph() && n_chains() > 1)
            st = replay_chains(s, gbwd_c_, sweep_of, bkey);
        else
            st = use_graph() ? replay(s, gbwd_, sweep, bkey) : sweep(s);
        if (st) return st;
        if (g_density || g_br) {
            st = launch(K_OUT, s, n_chunks_, kBlock, k_scatter_out<real, D>, a, (const int*)id_, (const real*)st_,
                        (real*)nullptr, (real*)g_density, (real*)g_br);
            if (st) return st;
        }
        if (g_b_prog) {
            int64_t nb = (int64_t)S_tot_ * D;
            st = launch(K_OUT, s, (int)((nb + 255) / 256), 256, k_sum_copies_out<real>, (const double*)gB_,
                        (real*)g_b_prog, nb);
            if (st) return st;
        }
        return finish(s);
    }

private:
    // ---------------------------------------------------------------- chains
    // Instances are split into up to kMaxChains groups of consecutive
    // instances (balanced by particle count). Each group advances on its own
    // stream with its own scatter lists, so one group's latency-bound grid
    // kernels overlap another group's particle kernels. One group runs on the
    // caller's stream directly.
    static constexpr int kMaxChains = 8;
    struct Chain {
        int c0 = 0, nc = 0;     // chunk range
        int ncb = 0;            // coarse blocks of its instances
        int64_t p0 = 0, np = 0; // particle slots (chunks * kBlock)
        hipStream_t s = nullptr;
        hipEvent_t done = nullptr;
    };

    int n_chains() const { return (int)chains_.size(); }

    void plan_chains()
    {
        const int n_inst = n_inst_;
        int want = streams_opt_ > 0 ? streams_opt_ : std::min(3, n_inst);
        if (ws_) want = 1;   // no streams of its own
        want = std::max(1, std::min({want, n_inst, kMaxChains}));
        std::vector<int> inst_chunks(n_inst), inst_cb(n_inst);
        for (int k = 0; k < n_inst; ++k) {
            const int next = k + 1 < n_inst ? inst_h_[k + 1].chunk_off : n_chunks_;
            inst_chunks[k] = next - inst_h_[k].chunk_off;
            const int nb = inst_h_[k].nb;
            inst_cb[k] = D == 2 ? nb * nb : nb * nb * nb;
        }
        std::vector<Chain> ch;
        int k = 0, done_chunks = 0;
        for (int q = 0; q < want && k < n_inst; ++q) {
            Chain c;
            c.c0 = inst_h_[k].chunk_off;
            const double target = (double)(n_chunks_ - done_chunks) / (double)(want - q);
            do {
                c.nc += inst_chunks[k];
                c.ncb += inst_cb[k];
                ++k;
            } while (k < n_inst && (q == want - 1 || c.nc + inst_chunks[k] / 2 < target));
            done_chunks += c.nc;
            c.p0 = (int64_t)c.c0 * kBlock;
            c.np = (int64_t)c.nc * kBlock;
            ch.push_back(c);
        }
        // keep existing streams and events
        for (size_t q = 0; q < ch.size() && q < chains_.size(); ++q) {
            ch[q].s = chains_[q].s;
            ch[q].done = chains_[q].done;
        }
        for (size_t q = ch.size(); q < chains_.size(); ++q) {
            if (chains_[q].s) (void)hipStreamDestroy(chains_[q].s);
            if (chains_[q].done) (void)hipEventDestroy(chains_[q].done);
        }
        chains_ = ch;
    }

    hipStream_t stream_of(int q, hipStream_t cs) const { return n_chains() > 1 ? chains_[q].s : cs; }

    // the chain streams start after the work queued on cs, and cs continues
    // after theirs
    int fork(hipStream_t cs)
    {
        if (n_chains() <= 1) return MPM_MAG_OK;
        if (!fork_ev_) MPM_HIP(hipEventCreateWithFlags(&fork_ev_, hipEventDisableTiming));
        for (auto& c : chains_) {
            if (!c.s) MPM_HIP(hipStreamCreateWithFlags(&c.s, hipStreamNonBlocking));
            if (!c.done) MPM_HIP(hipEventCreateWithFlags(&c.done, hipEventDisableTiming));
        }
        MPM_HIP(hipEventRecord(fork_ev_, cs));
        for (auto& c : chains_) MPM_HIP(hipStreamWaitEvent(c.s, fork_ev_, 0));
        return MPM_MAG_OK;
    }

    int join(hipStream_t cs)
    {
        if (n_chains() <= 1) return MPM_MAG_OK;
        for (auto& c : chains_) {
            MPM_HIP(hipEventRecord(c.done, c.s));
            MPM_HIP(hipStreamWaitEvent(cs, c.done, 0));
        }
        return MPM_MAG_OK;
    }

    Args<real> args_of(int q)
    {
        Args<real> a = args();
        a.chunk_base = chains_[q].c0;
        a.active = active_ + 4 * q;
        a.active_list = active_list_ + (size_t)4 * q * n_cb_;
        return a;
    }

    // Threads per workgroup of the grid update and its transpose. On one
    // stream the largest workgroup gathers a coarse block's boxes in the fewest
    // rounds (quadruped: 38 us per launch at 1024 threads, 41 at 512, 59 at
    // 256); when instance groups overlap on several streams, one-wave-per-SIMD
    // workgroups fit beside the particle kernels' blocks sooner (quadruped,
    // three streams: 4.76e9 particle-steps/s at 256 threads, 4.65e9 at 512,
    // 4.44e9 at 1024).
    int grid_threads() const { return grid_threads_ > 0 ? grid_threads_ : (n_chains() > 1 ? 256 : kGridThreadsMax); }

    int grid_blocks_of(int q) const { return (int)std::min<int64_t>(chains_[q].ncb, grid_wgs_); }
    // workgroups sharing one coarse block in the grid gathers
    int grid_parts() const { return grid_parts_ > 0 ? grid_parts_ : (D == 3 && n_chains() > 1 ? 2 : 1); }
    int gather_blocks_of(int q) const { return (int)std::min<int64_t>(chains_[q].ncb * grid_parts(), grid_wgs_); }

    // copy of the chain's particle state (all components) from src to dst
    int copy_state(int q, hipStream_t cs, real* dst, const real* src)
    {
        const Chain& c = chains_[q];
        const size_t pitch = sizeof(real) * (size_t)nalloc_;
        MPM_HIP(hipMemcpy2DAsync(dst + c.p0, pitch, src + c.p0, pitch, sizeof(real) * (size_t)c.np, Cp::NC,
                                 hipMemcpyDeviceToDevice, cs));
        count(K_CKPT, 2.0 * sizeof(real) * (double)c.np * Cp::NC);
        return MPM_MAG_OK;
    }

    // step n of the forward for chain q (checkpoints taken before steps
    // 0, K, 2K, ... when recording)
    int fwd_step(int q, hipStream_t cs, int n, bool record)
    {
        Args<real> a = args_of(q);
        a.trace = trace_;
        const int nc = chains_[q].nc;
        int r;
        if (n % lane_every() == 0) {
            r = sort_lanes(q, cs, st_);
            if (r) return r;
        }
        if (n == 0 || !fuse_fwd_) {
            if (record && n % K_ == 0) {
                r = copy_state(q, cs, ckpt_slot(n / K_), st_);
                if (r) return r;
            }
            r = launch(K_P2G, cs, nc, kBlock, k_p2g<real, D>, a, (const real*)st_, n, lf(n));
            if (r) return r;
        }
        r = launch(K_GRID, cs, gather_blocks_of(q), grid_threads(), k_grid<real, D>, a, gv_, (real*)nullptr, lf(n),
                   store_of(q, n, record));
        if (r) return r;
        if (n + 1 < T_ && fuse_fwd_) {
            // G2P of step n with P2G of step n + 1; v and C are stored only for
            // the checkpoint taken before step n + 1
            const bool ck1 = record && (n + 1) % K_ == 0;
            r = launch(K_G2P2G, cs, nc, kBlock, k_g2p2g<real, D>, a, (const real*)gv_, (const real*)st_, st_, n, 1,
                       ck1 ? 1 : 0, lf(n), lf(n + 1));
            if (r) return r;
            if (ck1) return copy_state(q, cs, ckpt_slot((n + 1) / K_), st_);
            return MPM_MAG_OK;
        }
        return launch(K_G2P, cs, nc, kBlock, k_g2p<real, D>, a, (const real*)gv_, (const real*)st_, st_, n, 1, lf(n), 0);
    }

    // step n of segment c, recomputed from its checkpoint for chain q, keeping
    // the step's grid (v, (p, m)) and the next state. When the recorded forward
    // stored the segment's grids, they are copied back and only the G2P runs.
    int recompute_step(int q, hipStream_t cs, int c, int n)
    {
        Args<real> a = args_of(q);
        const int nc = chains_[q].nc;
        const int s0 = c * K_, s1 = std::min(T_, s0 + K_), j = n - s0;
        int r;
        const bool stored = seg_stored(q, c);
        if (!stored && n == s0 && s0 % lane_every() == 0) {   // the lane order serves the fused forward only
            r = sort_lanes(q, cs, seg_state(c, 0));
            if (r) return r;
        }
        if (stored) {
            r = restore(q, cs, c, n);
            if (r || n + 1 >= s1) return r;
            return launch(K_G2P, cs, nc, kBlock, k_g2p<real, D>, a, (const real*)gv_slot(j),
                          (const real*)seg_state(c, j), seg_state(c, j + 1), n, 0, lf(n), 1);
        }
        if (n == s0 || !fuse_fwd_) {
            r = launch(K_P2G, cs, nc, kBlock, k_p2g<real, D>, a, (const real*)seg_state(c, j), n, lf(n));
            if (r) return r;
        }
        // the step's grid goes to the dense ring for this pass and to the
        // segment store for the transposed steps
        r = launch(K_GRID, cs, gather_blocks_of(q), grid_threads(), k_grid<real, D>, a, gv_slot(j), gm_slot(j), lf(n),
                   seg_store_of(q, j, n));
        if (r) return r;
        if (n + 1 >= s1) return MPM_MAG_OK;
        if (fuse_fwd_)
            return launch(K_G2P2G, cs, nc, kBlock, k_g2p2g<real, D>, a, (const real*)gv_slot(j),
                          (const real*)seg_state(c, j), seg_state(c, j + 1), n, 0, 1, lf(n), lf(n + 1));
        return launch(K_G2P, cs, nc, kBlock, k_g2p<real, D>, a, (const real*)gv_slot(j), (const real*)seg_state(c, j),
                      seg_state(c, j + 1), n, 0, lf(n), 0);
    }

    // Lane order of chain q's chunks by the stencil base cells of state st,
    // used by the forward particle kernels. It is refreshed every lane_every()
    // steps: in the forward pass, and in the recompute of the reverse sweep
    // at the segments that start on those steps (the other segments use the
    // last order made, which is as valid: every order gives the same sums).
    // steps between lane sorts: the smallest multiple of the checkpoint
    // spacing that is at least kLaneSortSteps (an order stays useful for a few
    // hundred steps; a sort is one more launch)
    static constexpr int kLaneSortSteps = 128;
    int lane_every() const
    {
        const int k = K_ > 0 ? K_ : std::max(1, (int)std::ceil(std::sqrt((double)std::max(1, T_))));
        return k * ((kLaneSortSteps + k - 1) / k);
    }

    int sort_lanes(int q, hipStream_t cs, const real* st)
    {
        if (!lane_sort_) return MPM_MAG_OK;
        return launch(K_SORT, cs, chains_[q].nc, kBlock, k_lane_sort<real, D>, args_of(q), st, lperm_);
    }

    // scatter lists of the G2P transpose alternate between consecutive steps
    static int lst(int n) { return 1 + (n & 1); }

    // transpose of the G2P of the last step of segment c
    int reverse_first(int q, hipStream_t cs, int c)
    {
        Args<real> a = args_of(q);
        const int s0 = c * K_, s1 = std::min(T_, s0 + K_), j = s1 - 1 - s0;
        return launch(K_G2P_ADJ, cs, chains_[q].nc, kBlock, k_g2p_adj<real, D>, a, (const real*)gv_slot(j),
                      (const real*)seg_state(c, j), (const real*)next_state(c, j), adj_, (const real*)dloss_,
                      lst(s1 - 1), lf(s1 - 1));
    }

    // grid transpose of step n, then the P2G transpose of step n (fused with
    // the G2P transpose of step n - 1 inside the segment)
    int reverse_step(int q, hipStream_t cs, int c, int n)
    {
        Args<real> a = args_of(q);
        const int nc = chains_[q].nc;
        const int s0 = c * K_, s1 = std::min(T_, s0 + K_), j = n - s0;
        int r = launch(K_GRID_ADJ, cs, gather_blocks_of(q), grid_threads(), k_grid_adj<real, D>, a, (const real*)gm_slot(j),
                       gpm_, lst(n), n);
        if (r) return r;
        // the G2P transpose of step n - 1 needs its grid: the ring still holds
        // the segment's last two steps from the recompute, earlier ones are
        // rebuilt from their store (their ring slot's previous step, n + 1, is
        // done with)
        if (n > s0 && j - 1 < (s1 - s0) - 2) {
            r = restore(q, cs, c, n - 1);
            if (r) return r;
        }
        if (n > s0 && fuse_adj_)
            return launch(K_ADJ_FUSED, cs, nc, kBlock, k_adj_fused<real, D>, a, (const real*)gpm_,
                          (const real*)seg_state(c, j), n, (const real*)gv_slot(j - 1), (const real*)seg_state(c, j - 1),
                          adj_, (const real*)dloss_, lst(n), lst(n - 1));
        r = launch(K_P2G_ADJ, cs, nc, kBlock, k_p2g_adj<real, D>, a, (const real*)gpm_, (const real*)seg_state(c, j),
                   adj_, n, lst(n));
        if (r || n == s0) return r;
        return launch(K_G2P_ADJ, cs, nc, kBlock, k_g2p_adj<real, D>, a, (const real*)gv_slot(j - 1),
                      (const real*)seg_state(c, j - 1), (const real*)seg_state(c, j), adj_, (const real*)dloss_,
                      lst(n - 1), lf(s1 - 1));
    }

    // workgroups of the grid kernels, which stride over the active coarse blocks
    int grid_blocks() const { return (int)std::min<int64_t>(n_cb_, grid_wgs_); }
    size_t state_elems() const { return (size_t)Cp::NC * nalloc_; }
    size_t state_bytes() const { return sizeof(real) * state_elems(); }
    real* ckpt_slot(int c) { return ckpt_ + (size_t)c * state_elems(); }
    // state of step s0 + j inside checkpoint segment c (slot 0 is the checkpoint)
    real* seg_state(int c, int j) { return j == 0 ? ckpt_slot(c) : stash_ + (size_t)(j - 1) * state_elems(); }
    // state after step s0 + j of segment c: the next stashed state, the next
    // segment's checkpoint, or the final state
    real* next_state(int c, int j)
    {
        if (c * K_ + j + 1 < std::min(T_, (c + 1) * K_)) return seg_state(c, j + 1);
        return c + 1 < nck_ ? ckpt_slot(c + 1) : st_;
    }
    // grid velocity / (momentum, mass) of step s0 + j of the segment being
    // reversed: a ring of two dense grids, steps of equal parity sharing one
    real* gv_slot(int j) { return ring_ + (size_t)(2 * (j & 1)) * 4 * G_; }
    real* gm_slot(int j) { return ring_ + (size_t)(2 * (j & 1) + 1) * 4 * G_; }

    // step n of segment c's grid, rebuilt in its ring slot from the store that
    // holds it (the recorded forward's, or the segment store of its recompute)
    int restore(int q, hipStream_t cs, int c, int n)
    {
        const int j = n - c * K_;
        const GridStore<real> g = seg_stored(q, c) ? store_of(q, n, true) : seg_store_of(q, j, n);
        return launch(K_RESTORE, cs, grid_blocks_of(q), kGridBlock, k_grid_restore<real, D>, args_of(q), g,
                      gv_slot(j), gm_slot(j));
    }

    int fail(int code, const std::string& msg)
    {
        err = msg;
        return code;
    }

    Args<real> args()
    {
        Args<real> a;
        a.inst = inst_d_;
        a.chunks = chunks_d_;
        a.gblock_inst = gblock_d_;
        a.nalloc = nalloc_;
        a.phi = phi_;
        a.br = br_;
        a.bprog = bprog_;
        a.gm = gm_;
        a.gv = gv_;
        a.gbar = gbar_;
        a.err = err_d_;
        a.scat_stats = err_d_ + 1;
        a.acc = acc_;
        a.acc_stride = (int64_t)n_inst_ * kAccCount;
        a.loss_val = loss_val_;
        a.gB = gB_;
        a.gB_stride = (int64_t)S_tot_ * D;
        a.gphi = gphi_;
        a.gbr = gbr_;
        a.corig = corig_;
        a.x0s = x0s_;
        a.part = part_;
        a.box = box_;
        a.reg_count = reg_count_;
        a.part_done = part_done_;
        a.grid_parts = grid_parts();
        a.reg_list = reg_list_;
        a.fb_used = fb_used_;
        a.cb_inst = cb_inst_d_;
        a.active = active_;
        a.active_list = active_list_;
        a.n_coarse = (int)n_cb_;

        a.use_lds = use_lds_ ? 1 : 0;
        a.box_cap = box_cap_;
        a.chunk_base = 0;
        a.lperm = lperm_;
        a.trace = nullptr;
        a.trace_nodes = trace_nodes_;
        return a;
    }

    // bytes a launch of each kernel class must move (for the roofline report)
    double algo_bytes(int kid) const
    {
        const double r = sizeof(real);
        const double n = (double)N_;
        switch (kid) {
        case K_P2G: return n * r * (D + D + 2 * D * D + 1 + D);                 // x v C F phi br
        case K_G2P: return n * r * ((D + D * D) + (2 * D + 2 * D * D));         // read x F, write x v C F
        case K_GRID: return 0.0;        // touches only the active coarse blocks; not priced
        case K_G2P_ADJ: return n * r * ((D + D * D) + (2 * D + 2 * D * D) + (D + D * D));
        case K_GRID_ADJ: return 0.0;
        case K_P2G_ADJ: return n * r * ((2 * D + 2 * D * D) + 1 + D + (2 * D + 2 * D * D) + (D + D * D) + 2 * (1 + D));
        // P2G transpose of step n (state n, phi, br, G2P share of the adjoint,
        // gradient read-modify-write) and G2P transpose of step n-1 (x, F of
        // state n-1, store of its G2P share)
        // G2P of step n with P2G of step n+1: read x, F, phi, br; write x, F
        // (v and C only at checkpoints and in the segment recompute, not priced)
        case K_G2P2G: return n * r * (2 * (D + D * D) + 1 + D);
        case K_ADJ_FUSED: return n * r * ((2 * D + 2 * D * D) + 1 + D + (D + D * D) + 2 * (1 + D) + (D + D * D) + (D + D * D));
        default: return 0.0;
        }
    }

    void count(int kid, double bytes, double flops = 0.0)
    {
        stats_[kid].launches += 1;
        stats_[kid].bytes += bytes;
        stats_[kid].flops += flops;
    }

    // Floating-point operations a launch of each kernel class must perform
    // (add or multiply 1, fused multiply-add 2), counted from the arithmetic of
    // the method per particle: the stencil weights, the stress of Eq. 7 with the
    // SIMP factors, the 3^D-node transfers of Eqs. 14-15 and 19-22, and for the
    // transposed kernels their adjoints with the stress tangent. Encoding,
    // indexing and reduction bookkeeping are not counted.
    double algo_flops(int kid) const
    {
        const double n = (double)N_;
        const double S3 = D == 2 ? 9.0 : 27.0;
        // per-node work: P2G, G2P, P2G transpose, G2P transpose (its sums of
        // w v_i and w v_i dpos^T are the v and C of the next state, read back)
        const double p2g_node = 2 * D * D + 3 * D + 1, g2p_node = 2 * D * D + 3 * D - 1;
        const double p2ga_node = 5 * D * D + 5 * D + 2, g2pa_node = 3 * D * D + 7 * D - 2;
        // per-particle work outside the node loops
        const double stress = D == 2 ? 95.0 : 237.0;          // Eq. 7 with SIMP, A = m C - k V P F^T
        const double fwd_rest = D == 2 ? 154.0 : 374.0;       // stencil, stress, C, x, F updates, det F
        const double adj_rest = D == 2 ? 445.0 : 1027.0;      // both stencils, stress, tangent, design terms
        switch (kid) {
        case K_P2G: return n * (12.0 * D + stress + S3 * p2g_node);
        case K_G2P: return n * ((fwd_rest - stress) + S3 * g2p_node);
        case K_G2P2G: return n * (fwd_rest + S3 * (p2g_node + g2p_node));
        case K_ADJ_FUSED: return n * (adj_rest + S3 * (p2ga_node + g2pa_node));
        case K_P2G_ADJ: return n * (0.6 * adj_rest + S3 * p2ga_node);
        case K_G2P_ADJ: return n * (0.4 * adj_rest + S3 * g2pa_node);
        default: return 0.0;
        }
    }

    template <typename Kern, typename... A>
    int launch(int kid, hipStream_t s, int grid, int block, Kern k, A... args)
    {
        if (grid <= 0) return MPM_MAG_OK;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (timing_) {
            e0 = event();
            MPM_HIP(hipEventRecord(e0, s));
        }
        hipLaunchKernelGGL(k, dim3(grid), dim3(block), 0, s, args...);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) {
            err = std::string("launch of ") + kernel_name(kid) + ": " + hipGetErrorString(e);
            return MPM_MAG_EHIP;
        }
        if (timing_) {
            e1 = event();
            MPM_HIP(hipEventRecord(e1, s));
            pending_.push_back({kid, e0, e1});
        }
        count(kid, algo_bytes(kid), algo_flops(kid));
        return MPM_MAG_OK;
    }

    hipEvent_t event()
    {
        if (ev_used_ == events_.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            events_.push_back(e);
        }
        return events_[ev_used_++];
    }

    // ------------------------------------------------------------ graphs
    // The step loop of a rollout and the reverse sweep of backward touch only
    // buffers the handle owns, so each is captured once into a HIP graph and
    // replayed on the caller's stream. A graph is rebuilt when the checkpoint
    // plan (and with it the buffer addresses) changes. Per-kernel launch and
    // byte counters recorded during capture are re-added on every replay.
    struct Graph {
        hipGraphExec_t exec = nullptr;
        int64_t key = -1;
        KernelStat delta[K_COUNT];
    };

    bool use_graph() const { return graph_ && !timing_; }

    void drop(Graph& g)
    {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g.exec = nullptr;
        g.key = -1;
    }

    template <typename Body>
    int replay(hipStream_t s, Graph& g, Body body, int64_t key = -2)
    {
        if (key == -2) key = plan_gen_;
        if (!g.exec || g.key != key) {
            drop(g);
            if (!cap_) MPM_HIP(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
            KernelStat before[K_COUNT];
            for (int k = 0; k < K_COUNT; ++k) before[k] = stats_[k];
            MPM_HIP(hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal));
            const int st = body(cap_);
            hipGraph_t graph = nullptr;
            const hipError_t e = hipStreamEndCapture(cap_, &graph);
            for (int k = 0; k < K_COUNT; ++k) {
                g.delta[k].launches = stats_[k].launches - before[k].launches;
                g.delta[k].bytes = stats_[k].bytes - before[k].bytes;
                g.delta[k].ms = 0.0;
                stats_[k] = before[k];
            }
            if (st) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return fail(MPM_MAG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
            const hipError_t ei = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ei != hipSuccess) {
                g.exec = nullptr;
                return fail(MPM_MAG_EHIP, std::string("graph instantiation: ") + hipGetErrorString(ei));
            }
            g.key = key;
        }
        MPM_HIP(hipGraphLaunch(g.exec, s));
        for (int k = 0; k < K_COUNT; ++k) {
            stats_[k].launches += g.delta[k].launches;
            stats_[k].bytes += g.delta[k].bytes;
        }
        return MPM_MAG_OK;
    }

    // Several instance groups: each group's sequence is captured into a graph
    // of its own and replayed on the group's stream between the fork and the
    // join. (One graph holding a branch per group ran the quadruped's three
    // groups 37% slower than direct launches on their streams.)
    template <typename BodyQ>
    int replay_chains(hipStream_t s, Graph* gq, BodyQ body_q, int64_t key)
    {
        int r = fork(s);
        if (r) return r;
        for (int q = 0; q < n_chains(); ++q) {
            r = replay(chains_[q].s, gq[q], [&](hipStream_t cs) { return body_q(q, cs); }, key);
            if (r) return r;
        }
        return join(s);
    }

    // scatter list of the forward P2G of step n (alternating, so a fused
    // G2P + P2G pass can reset the list its grid update consumed)
    static int lf(int n) { return (n & 1) ? 3 : 0; }

    int sort_and_gather(hipStream_t s, const real* x0, const real* phi, const real* br, const real* tgt,
                        const uint8_t* mask)
    {
        int st = launch(K_SORT, s, (int)((N_ + kBlock - 1) / kBlock), kBlock, k_sort_keys<real, D>,
                        (const InstDev<real>*)inst_d_, (const int64_t*)caller_start_d_, kp_, x0, (int64_t)N_,
                        keys_[0], vals_[0]);
        if (st) return st;
        int cur = 0;
        for (int p = 0; p < sort_passes_; ++p) {
            int shift = 8 * p;
            st = launch(K_SORT, s, sort_blocks_, kBlock, k_radix_hist, (const uint32_t*)keys_[cur], (int64_t)N_, shift,
                        hist_, sort_blocks_);
            if (st) return st;
            st = launch(K_SORT, s, 1, 1024, k_scan_exclusive, hist_, (int64_t)256 * sort_blocks_);
            if (st) return st;
            st = launch(K_SORT, s, sort_blocks_, kBlock, k_radix_scatter, (const uint32_t*)keys_[cur],
                        (const uint32_t*)vals_[cur], keys_[cur ^ 1], vals_[cur ^ 1], (int64_t)N_, shift,
                        (const uint32_t*)hist_, sort_blocks_);
            if (st) return st;
            cur ^= 1;
        }
        Args<real> a = args();
        return launch(K_GATHER, s, n_chunks_, kBlock, k_gather<real, D>, a, (const int*)vals_[cur],
                      (const int64_t*)caller_start_d_, st_, x0s_, phi_, br_, tgt_, mask_, id_, corig_, x0, phi, br, tgt,
                      mask, (int64_t)S_tot_ * D);
    }

    int finish(hipStream_t s)
    {
        MPM_HIP(hipMemcpyAsync(err_h_, err_d_, sizeof(*err_d_) * (1 + kScatStats), hipMemcpyDeviceToHost, s));
        MPM_HIP(hipStreamSynchronize(s));
        if (timing_) {
            for (auto& p : pending_) {
                float ms = 0.f;
                MPM_HIP(hipEventElapsedTime(&ms, p.e0, p.e1));
                stats_[p.kid].ms += ms;
            }
        }
        pending_.clear();
        ev_used_ = 0;
        const unsigned long long e = *err_h_;
        if (e != kNoError) {
            // the earliest failure (report_error)
            const int step = (int)((e >> 2) / 2), rank = (int)(e & 3);
            const std::string at = " (first at step " + std::to_string(step) + ")";
            if (rank == 0) return fail(MPM_MAG_ENONFINITE, "non-finite particle state" + at);
            if (rank == 1) return fail(MPM_MAG_EINVERT, "det F <= 0" + at);
            if (rank == 2) return fail(MPM_MAG_EDOMAIN, "a particle stencil left the grid" + at);
            return fail(MPM_MAG_EHIP, "grid store entry not kept" + at);
        }
        return MPM_MAG_OK;
    }

    // ------------------------------------------------------------ grid store
    // The recorded forward keeps every step's active coarse blocks (GridStore:
    // each node's summed (momentum, mass), the velocity being recomputed from
    // it) in one arena, split between the chains; steps beyond it are not kept
    // and their segments are recomputed in full by the reverse sweep, which
    // then writes their grids to a segment store. The arena's size comes from
    // the block counts of the last recorded rollout (a particle-count estimate
    // before the first), within the memory bound: the checkpoint budget when
    // one is set (it also covers the checkpoints, the segment stash, the grid
    // ring and the segment store), else the grid_store option in MiB, else the
    // free device memory less an eighth of the total.
    size_t store_block_bytes() const { return sizeof(real) * 4 * Coarse<D>::nodes; }

    // the handle's checkpoint budget in bytes, 0: none
    int64_t budget() const { return budget_opt_ > 0 ? budget_opt_ : budget_desc_; }

    // bytes of the checkpoints, the segment stash and the grid ring
    int64_t ckpt_plan_bytes(int K) const
    {
        const int nck = std::max(1, (T_ + K - 1) / K);
        return (int64_t)state_bytes() * (nck + std::max(1, K - 1)) + (int64_t)sizeof(real) * 2 * 2 * 4 * G_;
    }

    GridStore<real> store_of(int q, int n, bool on) const
    {
        GridStore<real> g;
        g.data = nullptr;
        g.blk = nullptr;
        g.base = nullptr;
        g.cap = 0;
        g.idx = n;
        g.step = n;
        if (!on || !gs_base_) return g;
        g.base = gs_base_ + (size_t)q * (T_ + 1);   // counted whenever recording
        if (!gstore_ || q >= gs_chains_) return g;
        g.data = gstore_ + (size_t)gs_off_[q] * 4 * Coarse<D>::nodes;
        g.blk = gs_blk_ + gs_off_[q];
        g.cap = (int)gs_cap_[q];
        return g;
    }

    // step n = s0 + j of a segment recomputed in full: its entry j of chain q's
    // segment store
    GridStore<real> seg_store_of(int q, int j, int n) const
    {
        GridStore<real> g;
        g.data = seg_data_ ? seg_data_ + (size_t)seg_off_[q] * 4 * Coarse<D>::nodes : nullptr;
        g.blk = seg_blk_ ? seg_blk_ + seg_off_[q] : nullptr;
        g.base = seg_base_ ? seg_base_ + (size_t)q * (K_ + 1) : nullptr;
        g.cap = (int)seg_cap_[q];
        g.idx = j;
        g.step = n;
        return g;
    }

    // the last recorded rollout kept every step of segment c for chain q
    bool seg_stored(int q, int c) const
    {
        if (!gs_valid_ || !gstore_ || q >= gs_chains_) return false;
        const int s1 = std::min(T_, (c + 1) * K_);
        return gs_base_h_[(size_t)q * (T_ + 1) + s1] <= gs_cap_[q];
    }

    // active blocks of segment c of chain q in the last recorded rollout
    int64_t seg_blocks(int q, int c) const
    {
        const int s0 = c * K_, s1 = std::min(T_, s0 + K_);
        const int* b = gs_base_h_.data() + (size_t)q * (T_ + 1);
        return (int64_t)b[s1] - (s0 == 0 ? 0 : b[s0]);
    }

    void free_store()
    {
        if (gstore_) (void)hipFree(gstore_);
        if (gs_blk_) (void)hipFree(gs_blk_);
        bytes_ -= gstore_bytes_;
        gstore_ = nullptr;
        gs_blk_ = nullptr;
        gstore_bytes_ = 0;
        gs_chains_ = 0;
        gs_valid_ = false;
        ++plan_gen_;   // store addresses are baked into captured launches
    }

    void free_seg_store()
    {
        if (seg_data_) (void)hipFree(seg_data_);
        if (seg_blk_) (void)hipFree(seg_blk_);
        bytes_ -= seg_bytes_;
        seg_data_ = nullptr;
        seg_blk_ = nullptr;
        seg_bytes_ = 0;
        for (int q = 0; q < kMaxChains; ++q) seg_off_[q] = seg_cap_[q] = 0;
        ++plan_gen_;
    }

    // allocate slots for chain-split arenas; false when the device is out of memory
    bool alloc_arena(real** data, int** blk, int64_t slots)
    {
        if (hipMalloc(data, store_block_bytes() * (size_t)slots) != hipSuccess) {
            (void)hipGetLastError();
            *data = nullptr;
            return false;
        }
        if (hipMalloc(blk, sizeof(int) * (size_t)slots) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipFree(*data);
            *data = nullptr;
            *blk = nullptr;
            return false;
        }
        return true;
    }

    int ensure_store()
    {
        gs_valid_ = false;
        const int nq = n_chains();
        if (T_ == 0) {
            if (gstore_) free_store();
            return MPM_MAG_OK;
        }
        if (!gs_base_) {
            if (hipMalloc(&gs_base_, sizeof(int) * (size_t)kMaxChains * (T_ + 1)) != hipSuccess) {
                gs_base_ = nullptr;
                return fail(MPM_MAG_ENOMEM, "grid store counters");
            }
            bytes_ += sizeof(int) * (size_t)kMaxChains * (T_ + 1);
        }
        const int64_t B = budget();
        if (gs_budget_mib_ == 0) {   // option: no store
            if (gstore_) free_store();
            return MPM_MAG_OK;
        }
        // slots wanted per chain: the last count with a tenth more, else the
        // estimate; and the largest segment, for the segment store
        const bool known = !gs_base_h_.empty() && gs_count_chains_ == nq;
        std::vector<int64_t> want(nq, 0), seg_want(nq, 0);
        int64_t total = 0, seg_total = 0;
        for (int q = 0; q < nq; ++q) {
            if (known) {
                const int64_t need = gs_base_h_[(size_t)q * (T_ + 1) + T_];
                want[q] = need + need / 10 + 8;
                for (int c = 0; c < nck_; ++c) seg_want[q] = std::max(seg_want[q], seg_blocks(q, c));
            } else {
                int64_t per_step = 0;
                for (int k = 0; k < n_inst_; ++k)
                    if (inst_h_[k].chunk_off >= chains_[q].c0 && inst_h_[k].chunk_off < chains_[q].c0 + chains_[q].nc)
                        per_step += est_cb_inst_[k];
                want[q] = per_step * T_;
                seg_want[q] = per_step * K_;
            }
            seg_want[q] += seg_want[q] / 10 + 8;
            want[q] = std::min<int64_t>(want[q], kStoreCountMax);
            total += want[q];
            seg_total += seg_want[q];
        }
        const size_t bb = store_block_bytes();
        int64_t avail;   // bytes the arena may take
        if (B > 0) {
            avail = B - ckpt_plan_bytes(K_) - (int64_t)sizeof(int) * kMaxChains * (T_ + 1);
            // a store short of the whole rollout leaves segments to recompute,
            // whose grids go to the segment store: keep room for it
            if (avail < (int64_t)(bb + sizeof(int)) * total) avail -= (int64_t)(bb + sizeof(int)) * seg_total;
            if (gs_budget_mib_ > 0) avail = std::min<int64_t>(avail, gs_budget_mib_ << 20);
        } else if (gs_budget_mib_ > 0) {
            avail = gs_budget_mib_ << 20;
        } else {
            size_t fr = 0, tot = 0;
            if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
                (void)hipGetLastError();
                fr = tot = 0;
            }
            avail = (int64_t)fr + (int64_t)gstore_bytes_ - (int64_t)(tot / 8);
        }
        const int64_t max_slots = std::max<int64_t>(0, avail) / (int64_t)(bb + sizeof(int));
        if (total > max_slots) {
            int64_t t2 = 0;
            for (int q = 0; q < nq; ++q) {
                want[q] = (int64_t)((double)want[q] * (double)max_slots / (double)total);
                t2 += want[q];
            }
            total = t2;
        }
        // keep the arena when it fits every chain and is not more than twice the
        // need (and, under a budget, within it)
        bool keep = gstore_ && gs_chains_ == nq;
        int64_t cur = 0;
        for (int q = 0; keep && q < nq; ++q) {
            keep = gs_cap_[q] >= want[q];
            cur += gs_cap_[q];
        }
        if (keep && cur <= 2 * total + 64 && cur <= max_slots) return MPM_MAG_OK;
        if (gstore_) free_store();
        if (total <= 0) return MPM_MAG_OK;
        if (!alloc_arena(&gstore_, &gs_blk_, total)) return MPM_MAG_OK;   // no arena: every segment is recomputed
        gstore_bytes_ = (bb + sizeof(int)) * (size_t)total;
        bytes_ += gstore_bytes_;
        int64_t off = 0;
        for (int q = 0; q < nq; ++q) {
            gs_off_[q] = off;
            gs_cap_[q] = want[q];
            off += want[q];
        }
        gs_chains_ = nq;
        ++plan_gen_;
        return MPM_MAG_OK;
    }

    // Segment store for the segments the recorded forward could not keep,
    // sized from the last recorded rollout's largest such segment per chain.
    int ensure_seg_store()
    {
        const int nq = n_chains();
        std::vector<int64_t> need(nq, 0);
        int64_t total = 0;
        const bool counted = gs_valid_ && gs_count_chains_ == nq;
        for (int q = 0; q < nq; ++q) {
            for (int c = 0; c < nck_; ++c) {
                if (seg_stored(q, c)) continue;
                need[q] = std::max(need[q], counted ? seg_blocks(q, c) : (int64_t)n_cb_ * K_);
            }
            if (need[q] > 0) need[q] += need[q] / 10 + 8;
            total += need[q];
        }
        if (!seg_base_) {
            if (hipMalloc(&seg_base_, sizeof(int) * (size_t)kMaxChains * (K_ + 1)) != hipSuccess) {
                seg_base_ = nullptr;
                return fail(MPM_MAG_ENOMEM, "segment store counters");
            }
            seg_base_k_ = K_;
            bytes_ += sizeof(int) * (size_t)kMaxChains * (K_ + 1);
        }
        bool fits = seg_base_k_ >= K_;
        for (int q = 0; fits && q < nq; ++q) fits = seg_cap_[q] >= need[q];
        if (fits) return MPM_MAG_OK;
        if (seg_base_k_ < K_) {
            (void)hipFree(seg_base_);
            bytes_ -= sizeof(int) * (size_t)kMaxChains * (seg_base_k_ + 1);
            if (hipMalloc(&seg_base_, sizeof(int) * (size_t)kMaxChains * (K_ + 1)) != hipSuccess) {
                seg_base_ = nullptr;
                return fail(MPM_MAG_ENOMEM, "segment store counters");
            }
            seg_base_k_ = K_;
            bytes_ += sizeof(int) * (size_t)kMaxChains * (K_ + 1);
        }
        free_seg_store();
        if (!alloc_arena(&seg_data_, &seg_blk_, total)) return fail(MPM_MAG_ENOMEM, "segment store");
        seg_bytes_ = (store_block_bytes() + sizeof(int)) * (size_t)total;
        bytes_ += seg_bytes_;
        int64_t off = 0;
        for (int q = 0; q < nq; ++q) {
            seg_off_[q] = off;
            seg_cap_[q] = need[q];
            off += need[q];
        }
        return MPM_MAG_OK;
    }

    int ensure_checkpoints()
    {
        int K = ckpt_opt_ > 0 ? ckpt_opt_ : (ckpt_desc_ > 0 ? ckpt_desc_ : 0);
        if (K <= 0) K = std::max(1, (int)std::ceil(std::sqrt((double)std::max(1, T_))));
        if (T_ == 0) K = 1;
        K = std::max(1, std::min(K, std::max(1, T_)));
        int nck = std::max(1, (T_ + K - 1) / K);
        const int64_t B = budget();
        if (B > 0 && ckpt_plan_bytes(K) > B)
            return fail(MPM_MAG_ENOMEM, "checkpoint budget of " + std::to_string(B) + " bytes is below the " +
                                            std::to_string(ckpt_plan_bytes(K)) + " the checkpoints, segment stash " +
                                            "and grid ring need at spacing " + std::to_string(K));
        if (ckpt_ && K == K_ && nck == nck_) return MPM_MAG_OK;
        if (ckpt_) { (void)hipFree(ckpt_); bytes_ -= ckpt_bytes_; ckpt_ = nullptr; }
        if (stash_) { (void)hipFree(stash_); bytes_ -= stash_bytes_; stash_ = nullptr; }
        if (ring_) { (void)hipFree(ring_); bytes_ -= ring_bytes_; ring_ = nullptr; }
        ckpt_bytes_ = state_bytes() * nck;
        stash_bytes_ = state_bytes() * std::max(1, K - 1);
        ring_bytes_ = sizeof(real) * (size_t)2 * 2 * 4 * G_;
        if (hipMalloc(&ring_, ring_bytes_) != hipSuccess) { ring_ = nullptr; return fail(MPM_MAG_ENOMEM, "grid ring"); }
        bytes_ += ring_bytes_;
        if (hipMalloc(&ckpt_, ckpt_bytes_) != hipSuccess) { ckpt_ = nullptr; return fail(MPM_MAG_ENOMEM, "checkpoint pool"); }
        if (hipMalloc(&stash_, stash_bytes_) != hipSuccess) {
            (void)hipFree(ckpt_); ckpt_ = nullptr;
            return fail(MPM_MAG_ENOMEM, "segment stash");
        }
        bytes_ += ckpt_bytes_ + stash_bytes_;
        K_ = K;
        nck_ = nck;
        gs_valid_ = false;   // segment boundaries moved
        ++plan_gen_;
        return MPM_MAG_OK;
    }

    template <typename T>
    int dalloc(T** p, size_t n)
    {
        size_t b = sizeof(T) * std::max<size_t>(n, 1);
        if (ws_) {   // carved from the workspace, 256-byte aligned
            const size_t off = (ws_used_ + 255) & ~(size_t)255;
            if (off + b > ws_bytes_) {
                *p = nullptr;
                return fail(MPM_MAG_ENOMEM, "the problem needs more than the " + std::to_string(ws_bytes_ >> 20) +
                                                " MiB of static scratch");
            }
            *p = (T*)(ws_ + off);
            ws_used_ = off + b;
            bytes_ += b;
            return MPM_MAG_OK;
        }
        if (hipMalloc((void**)p, b) != hipSuccess) { *p = nullptr; return fail(MPM_MAG_ENOMEM, "device allocation"); }
        allocs_.push_back((void*)*p);
        bytes_ += b;
        return MPM_MAG_OK;
    }

    int allocate()
    {
        int st = 0;
        st |= dalloc(&inst_d_, inst_h_.size());
        st |= dalloc(&chunks_d_, chunks_h_.size());
        st |= dalloc(&gblock_d_, gblock_h_.size());
        st |= dalloc(&caller_start_d_, caller_start_h_.size());
        st |= dalloc(&st_, state_elems());
        st |= dalloc(&adj_, state_elems());
        st |= dalloc(&x0s_, (size_t)D * nalloc_);
        st |= dalloc(&tgt_, (size_t)D * nalloc_);
        st |= dalloc(&br_, (size_t)D * nalloc_);
        st |= dalloc(&phi_, (size_t)nalloc_);
        st |= dalloc(&gphi_, (size_t)nalloc_);
        st |= dalloc(&gbr_, (size_t)D * nalloc_);
        st |= dalloc(&mask_, (size_t)nalloc_);
        st |= dalloc(&lperm_, (size_t)nalloc_);
        st |= dalloc(&id_, (size_t)nalloc_);
        st |= dalloc(&corig_, (size_t)n_chunks_);
        st |= dalloc(&part_, (size_t)n_chunks_ * kBoxCap * 4);
        st |= dalloc(&box_, (size_t)n_chunks_ * kWaves * 2);
        st |= dalloc(&reg_count_, (size_t)n_cb_);
        st |= dalloc(&part_done_, (size_t)n_cb_);
        st |= dalloc(&reg_list_, (size_t)n_cb_ * Coarse<D>::cap);
        st |= dalloc(&fb_used_, (size_t)n_cb_);
        st |= dalloc(&cb_inst_d_, (size_t)n_cb_);
        st |= dalloc(&active_, 4 * kMaxChains);
        st |= dalloc(&active_list_, (size_t)4 * kMaxChains * n_cb_);
        st |= dalloc(&gpm_, (size_t)4 * G_);
        st |= dalloc(&gm_, (size_t)4 * G_);
        st |= dalloc(&gv_, (size_t)4 * G_);
        st |= dalloc(&gbar_, (size_t)4 * G_);
        st |= dalloc(&bprog_, (size_t)S_tot_ * D);
        // the program gradient's copies (a handle on static scratch runs no backward)
        st |= dalloc(&gB_, ws_ ? (size_t)1 : (size_t)S_tot_ * D * kGbCopies);
        st |= dalloc(&acc_, (size_t)kAccCount * n_inst_ * kGbCopies);
        st |= dalloc(&loss_val_, (size_t)n_inst_);
        st |= dalloc(&dloss_, (size_t)n_inst_);
        st |= dalloc(&err_d_, 1 + kScatStats);   // error word, then the scatter fallback counts
        for (int b = 0; b < 2; ++b) {
            st |= dalloc(&keys_[b], (size_t)N_);
            st |= dalloc(&vals_[b], (size_t)N_);
        }
        st |= dalloc(&hist_, (size_t)256 * sort_blocks_);
        if (st) return ws_ ? MPM_MAG_ENOMEM : fail(MPM_MAG_ENOMEM, "device allocation failed");
        if (ws_)
            err_h_ = err_host_;   // pageable words: no host allocation either
        else if (hipHostMalloc((void**)&err_h_, sizeof(*err_h_) * (1 + kScatStats)) != hipSuccess)
            return fail(MPM_MAG_ENOMEM, "pinned error word");
        MPM_HIP(hipMemcpy(inst_d_, inst_h_.data(), sizeof(InstDev<real>) * inst_h_.size(), hipMemcpyHostToDevice));
        MPM_HIP(hipMemcpy(chunks_d_, chunks_h_.data(), sizeof(ChunkDev) * chunks_h_.size(), hipMemcpyHostToDevice));
        MPM_HIP(hipMemcpy(gblock_d_, gblock_h_.data(), sizeof(int) * gblock_h_.size(), hipMemcpyHostToDevice));
        MPM_HIP(hipMemcpy(caller_start_d_, caller_start_h_.data(), sizeof(int64_t) * caller_start_h_.size(),
                          hipMemcpyHostToDevice));
        MPM_HIP(hipMemcpy(cb_inst_d_, cb_inst_h_.data(), sizeof(int) * cb_inst_h_.size(), hipMemcpyHostToDevice));
        MPM_HIP(hipMemset(reg_count_, 0, sizeof(int) * n_cb_));
        MPM_HIP(hipMemset(part_done_, 0, sizeof(int) * n_cb_));
        MPM_HIP(hipMemset(fb_used_, 0, sizeof(int) * n_cb_));
        MPM_HIP(hipMemset(active_, 0, sizeof(int) * 4 * kMaxChains));
        MPM_HIP(hipMemset(gm_, 0, sizeof(real) * 4 * G_));
        MPM_HIP(hipMemset(gv_, 0, sizeof(real) * 4 * G_));
        MPM_HIP(hipMemset(gbar_, 0, sizeof(real) * 4 * G_));
        MPM_HIP(hipMemset(st_, 0, state_bytes()));
        MPM_HIP(hipMemset(adj_, 0, state_bytes()));
        MPM_HIP(hipMemset(tgt_, 0, sizeof(real) * D * nalloc_));
        {
            // identity lane order until the first rollout sorts the lanes
            std::vector<uint8_t> ident((size_t)nalloc_);
            for (size_t j = 0; j < ident.size(); ++j) ident[j] = (uint8_t)(j % kBlock);
            MPM_HIP(hipMemcpy(lperm_, ident.data(), ident.size(), hipMemcpyHostToDevice));
        }
        MPM_HIP(hipDeviceSynchronize());
        return MPM_MAG_OK;
    }

    void release()
    {
        drop(gfwd_[0]);
        drop(gfwd_[1]);
        drop(gbwd_);
        for (int q = 0; q < kMaxChains; ++q) {
            drop(gfwd_c_[0][q]);
            drop(gfwd_c_[1][q]);
            drop(gbwd_c_[q]);
        }
        if (cap_) (void)hipStreamDestroy(cap_);
        cap_ = nullptr;
        for (auto& c : chains_) {
            if (c.s) (void)hipStreamDestroy(c.s);
            if (c.done) (void)hipEventDestroy(c.done);
        }
        chains_.clear();
        if (fork_ev_) (void)hipEventDestroy(fork_ev_);
        fork_ev_ = nullptr;
        for (void* p : allocs_) (void)hipFree(p);
        allocs_.clear();
        if (ckpt_) (void)hipFree(ckpt_);
        if (stash_) (void)hipFree(stash_);
        if (ring_) (void)hipFree(ring_);
        ckpt_ = stash_ = ring_ = nullptr;
        if (seg_data_) (void)hipFree(seg_data_);
        if (seg_blk_) (void)hipFree(seg_blk_);
        if (seg_base_) (void)hipFree(seg_base_);
        seg_data_ = nullptr;
        seg_blk_ = seg_base_ = nullptr;
        if (gstore_) (void)hipFree(gstore_);
        if (gs_blk_) (void)hipFree(gs_blk_);
        if (gs_base_) (void)hipFree(gs_base_);
        gstore_ = nullptr;
        gs_blk_ = gs_base_ = nullptr;
        if (err_h_ && !ws_) (void)hipHostFree(err_h_);
        err_h_ = nullptr;
        for (auto e : events_) (void)hipEventDestroy(e);
        events_.clear();
    }

    struct Pending {
        int kid;
        hipEvent_t e0, e1;
    };

    // tables
    int n_inst_ = 0, T_ = 0, n_chunks_ = 0, S_tot_ = 0;
    int64_t N_ = 0, nalloc_ = 0, G_ = 0;
    std::vector<InstDev<real>> inst_h_;
    std::vector<ChunkDev> chunks_h_;
    std::vector<int> gblock_h_;
    std::vector<int64_t> caller_start_h_;
    KeyParams kp_;
    int sort_passes_ = 0, sort_blocks_ = 0;
    // device buffers
    InstDev<real>* inst_d_ = nullptr;
    ChunkDev* chunks_d_ = nullptr;
    int* gblock_d_ = nullptr;
    int64_t* caller_start_d_ = nullptr;
    real *st_ = nullptr, *adj_ = nullptr, *x0s_ = nullptr, *tgt_ = nullptr, *br_ = nullptr, *phi_ = nullptr;
    real *gphi_ = nullptr, *gbr_ = nullptr, *gm_ = nullptr, *gv_ = nullptr, *gbar_ = nullptr, *bprog_ = nullptr;
    uint8_t* mask_ = nullptr;
    uint8_t* lperm_ = nullptr;   // lane order of the particle kernels (k_lane_sort)
    int* id_ = nullptr;
    int4* corig_ = nullptr;
    real* part_ = nullptr;
    int4* box_ = nullptr;
    int* reg_count_ = nullptr;
    int* part_done_ = nullptr;
    int* reg_list_ = nullptr;
    int* fb_used_ = nullptr;
    int* cb_inst_d_ = nullptr;
    int* active_ = nullptr;
    int* active_list_ = nullptr;
    real* gpm_ = nullptr;      // (pbar, mbar) of the grid transpose
    real* ring_ = nullptr;     // two dense grids (v, (p, m)) of the segment being reversed
    size_t ring_bytes_ = 0;
    // segment store: chain q owns slots [seg_off_[q], seg_off_[q] + seg_cap_[q])
    real* seg_data_ = nullptr;
    int* seg_blk_ = nullptr;
    int* seg_base_ = nullptr;         // [kMaxChains][seg_base_k_ + 1]
    int seg_base_k_ = 0;
    size_t seg_bytes_ = 0;
    int64_t seg_off_[kMaxChains] = {}, seg_cap_[kMaxChains] = {};
    int64_t budget_desc_ = 0, budget_opt_ = 0;   // checkpoint budget (bytes): descriptors, option
    // grid store: chain q owns slots [gs_off_[q], gs_off_[q] + gs_cap_[q])
    real* gstore_ = nullptr;
    int* gs_blk_ = nullptr;
    int* gs_base_ = nullptr;          // [kMaxChains][T + 1]
    size_t gstore_bytes_ = 0;
    int64_t gs_off_[kMaxChains] = {}, gs_cap_[kMaxChains] = {};
    int gs_chains_ = 0;               // chains the arena is laid out for
    int gs_count_chains_ = 0;         // chains of the counts in gs_base_h_
    std::vector<int> gs_base_h_;      // step bases of the last recorded rollout
    bool gs_valid_ = false;           // they describe the recorded rollout
    int64_t gs_budget_mib_ = -1;      // option grid_store
    std::vector<int64_t> est_cb_inst_;
    std::vector<char> bwd_sig_;       // stored segments of the captured reverse sweep
    int64_t bwd_gen_ = 0;
    std::vector<int> cb_inst_h_;
    int64_t n_cb_ = 0;
    int64_t trace_nodes_ = 0;       // sum of the instances' node counts
    uint16_t* trace_ = nullptr;     // caller's branch trace, or nullptr
    double *gB_ = nullptr, *acc_ = nullptr, *loss_val_ = nullptr;
    real* dloss_ = nullptr;   // copy of the upstream loss gradient (stable address for graphs)
    unsigned long long* err_d_ = nullptr;   // earliest failure of the call (report_error)
    unsigned long long* err_h_ = nullptr;
    unsigned long long err_host_[1 + kScatStats] = {};   // error word and counts of a handle on a workspace
    uint8_t* ws_ = nullptr;             // workspace the buffers are carved from, or nullptr
    size_t ws_bytes_ = 0, ws_used_ = 0;
    uint32_t* keys_[2] = {nullptr, nullptr};
    uint32_t* vals_[2] = {nullptr, nullptr};
    uint32_t* hist_ = nullptr;
    std::vector<void*> allocs_;
    int64_t bytes_ = 0;
    // checkpoints
    real* ckpt_ = nullptr;
    real* stash_ = nullptr;
    size_t ckpt_bytes_ = 0, stash_bytes_ = 0;
    int K_ = 0, nck_ = 0, ckpt_desc_ = 0, ckpt_opt_ = 0;
    bool recorded_ = false, has_target_ = false;
    // options
    bool graph_ = false, timing_ = false, use_lds_ = true;
    int box_cap_ = kBoxCap, grid_wgs_ = 2048, grid_threads_ = 0, grid_parts_ = 0;
    bool fuse_adj_ = true, fuse_fwd_ = true, lane_sort_ = true;
    std::vector<hipEvent_t> events_;
    size_t ev_used_ = 0;
    // captured graphs: forward step loop (plain, recorded) and reverse sweep
    Graph gfwd_[2], gbwd_;
    Graph gfwd_c_[2][kMaxChains], gbwd_c_[kMaxChains];   // per instance group, with several
    hipStream_t cap_ = nullptr;
    std::vector<Chain> chains_;
    hipEvent_t fork_ev_ = nullptr;
    int streams_opt_ = 0;
    int64_t plan_gen_ = 0;
    std::vector<Pending> pending_;
};

// ws / ws_bytes: carve the engine's buffers from that device range (plain
// rollouts only) instead of allocating them
EngineBase* make_engine_f2(const mpm_mag_instance_desc*, int, const int64_t*, int*, std::string*, void* ws = nullptr,
                           size_t ws_bytes = 0);
EngineBase* make_engine_f3(const mpm_mag_instance_desc*, int, const int64_t*, int*, std::string*, void* ws = nullptr,
                           size_t ws_bytes = 0);
EngineBase* make_engine_d2(const mpm_mag_instance_desc*, int, const int64_t*, int*, std::string*, void* ws = nullptr,
                           size_t ws_bytes = 0);
EngineBase* make_engine_d3(const mpm_mag_instance_desc*, int, const int64_t*, int*, std::string*, void* ws = nullptr,
                           size_t ws_bytes = 0);

}  // namespace mpm
