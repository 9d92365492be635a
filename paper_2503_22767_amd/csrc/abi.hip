// C ABI of the library: argument checks, dispatch to the engine instantiation
// for (precision, dim), status strings. No exception crosses this boundary.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <string>

#include "mpm_mag.h"
#include "engine.hpp"

struct mpm_mag {
    mpm::EngineBase* eng = nullptr;
    std::string last;
};

namespace {
thread_local std::string g_create_error;

// Static scratch of mpm_mag_rollout_noalloc: every device buffer of its plain
// rollout is carved from this array (one copy per GPU, held until the process
// ends). Host code must not pass the array's name to kernels or copies (it is
// a host-side stand-in); the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int record(mpm_mag* h, int st)
{
    if (h) h->last = st ? h->eng->err : std::string();
    return st;
}
}  // namespace

extern "C" {

int mpm_mag_create(const mpm_mag_instance_desc* descs, int n_inst, const int64_t* n_particles, int precision,
                   mpm_mag** out)
{
    if (!out || !descs || !n_particles || n_inst < 1) return MPM_MAG_EINVAL;
    *out = nullptr;
    if (precision != 4 && precision != 8) return MPM_MAG_EINVAL;
    int dim = descs[0].dim;
    if (dim != 2 && dim != 3) return MPM_MAG_EINVAL;
    int st = MPM_MAG_OK;
    std::string msg;
    mpm::EngineBase* e = nullptr;
    try {
        if (precision == 4)
            e = dim == 2 ? mpm::make_engine_f2(descs, n_inst, n_particles, &st, &msg)
                         : mpm::make_engine_f3(descs, n_inst, n_particles, &st, &msg);
        else
            e = dim == 2 ? mpm::make_engine_d2(descs, n_inst, n_particles, &st, &msg)
                         : mpm::make_engine_d3(descs, n_inst, n_particles, &st, &msg);
    } catch (...) {
        return MPM_MAG_ENOMEM;
    }
    if (!e) {
        g_create_error = msg;
        return st ? st : MPM_MAG_ENOMEM;
    }
    mpm_mag* h = new (std::nothrow) mpm_mag();
    if (!h) {
        delete e;
        return MPM_MAG_ENOMEM;
    }
    h->eng = e;
    *out = h;
    return MPM_MAG_OK;
}

int mpm_mag_rollout(mpm_mag* h, void* stream, const void* x0, const void* density, const void* br,
                    const void* b_prog, const void* loss_target, const uint8_t* loss_mask, void* x_final,
                    void* loss_out, int record_flag)
{
    if (!h) return MPM_MAG_EINVAL;
    try {
        return record(h, h->eng->rollout((hipStream_t)stream, x0, density, br, b_prog, loss_target, loss_mask,
                                         x_final, loss_out, record_flag));
    } catch (...) {
        h->last = "unexpected host exception";
        return MPM_MAG_ENOMEM;
    }
}

int mpm_mag_backward(mpm_mag* h, void* stream, const void* dloss, const void* dx_final, void* g_density,
                     void* g_br, void* g_b_prog)
{
    if (!h) return MPM_MAG_EINVAL;
    try {
        return record(h, h->eng->backward((hipStream_t)stream, dloss, dx_final, g_density, g_br, g_b_prog));
    } catch (...) {
        h->last = "unexpected host exception";
        return MPM_MAG_ENOMEM;
    }
}

void mpm_mag_destroy(mpm_mag* h)
{
    if (!h) return;
    delete h->eng;
    delete h;
}

const char* mpm_mag_strerror(int status)
{
    switch (status) {
    case MPM_MAG_OK: return "ok";
    case MPM_MAG_EINVAL: return "invalid argument";
    case MPM_MAG_ENOMEM: return "out of device memory";
    case MPM_MAG_EHIP: return "HIP runtime error";
    case MPM_MAG_EDOMAIN: return "particle stencil left the grid";
    case MPM_MAG_EINVERT: return "deformation gradient inverted (det F <= 0)";
    case MPM_MAG_ENONFINITE: return "non-finite particle state";
    case MPM_MAG_ESTATE: return "backward without a recorded rollout";
    default: return "unknown status";
    }
}

const char* mpm_mag_last_error(const mpm_mag* h)
{
    if (!h) return g_create_error.c_str();
    return h->last.c_str();
}

int mpm_mag_set_option(mpm_mag* h, const char* key, int64_t value)
{
    if (!h) return MPM_MAG_EINVAL;
    return record(h, h->eng->set_option(key, value));
}

int mpm_mag_num_kernels(void) { return mpm::K_COUNT; }

const char* mpm_mag_kernel_name(int kernel) { return mpm::kernel_name(kernel); }

int mpm_mag_kernel_flops(mpm_mag* h, int kernel, double* flops)
{
    if (!h) return MPM_MAG_EINVAL;
    return h->eng->kernel_flops(kernel, flops);
}

int mpm_mag_kernel_stats(mpm_mag* h, int kernel, int64_t* launches, double* total_ms, double* bytes)
{
    if (!h) return MPM_MAG_EINVAL;
    return h->eng->kernel_stats(kernel, launches, total_ms, bytes);
}

int64_t mpm_mag_device_bytes(const mpm_mag* h) { return h ? h->eng->device_bytes() : 0; }

int mpm_mag_rollout_noalloc(const mpm_mag_instance_desc* descs, int n_inst, const int64_t* n_particles,
                            int precision, void* stream, const void* x0, const void* density, const void* br,
                            const void* b_prog, const void* loss_target, const uint8_t* loss_mask, void* x_final,
                            void* loss_out)
{
    g_create_error.clear();
    if (!descs || !n_particles || n_inst < 1 || (precision != 4 && precision != 8)) return MPM_MAG_EINVAL;
    const int dim = descs[0].dim;
    if (dim != 2 && dim != 3) return MPM_MAG_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        g_create_error = "no current HIP device (or more than 64)";
        return MPM_MAG_EHIP;
    }
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                g_create_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
                return MPM_MAG_EHIP;
            }
            g_scratch_ptr[dev] = p;
        }
        ws = g_scratch_ptr[dev];
    }
    int st = MPM_MAG_OK;
    std::string msg;
    mpm::EngineBase* e = nullptr;
    try {
        if (precision == 4)
            e = dim == 2 ? mpm::make_engine_f2(descs, n_inst, n_particles, &st, &msg, ws, kScratchBytes)
                         : mpm::make_engine_f3(descs, n_inst, n_particles, &st, &msg, ws, kScratchBytes);
        else
            e = dim == 2 ? mpm::make_engine_d2(descs, n_inst, n_particles, &st, &msg, ws, kScratchBytes)
                         : mpm::make_engine_d3(descs, n_inst, n_particles, &st, &msg, ws, kScratchBytes);
    } catch (...) {
        g_create_error = "unexpected host exception";
        return MPM_MAG_ENOMEM;
    }
    if (!e) {
        g_create_error = msg;
        return st ? st : MPM_MAG_ENOMEM;
    }
    try {
        st = e->rollout((hipStream_t)stream, x0, density, br, b_prog, loss_target, loss_mask, x_final, loss_out, 0);
    } catch (...) {
        st = MPM_MAG_ENOMEM;
        e->err = "unexpected host exception";
    }
    if (st) g_create_error = e->err;
    delete e;
    return st;
}

int64_t mpm_mag_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }

int mpm_mag_set_branch_trace(mpm_mag* h, uint16_t* trace, int64_t elems)
{
    if (!h) return MPM_MAG_EINVAL;
    return record(h, h->eng->set_trace(trace, elems));
}

int64_t mpm_mag_trace_nodes(const mpm_mag* h) { return h ? h->eng->trace_nodes() : 0; }

int mpm_mag_scatter_stats(const mpm_mag* h, int64_t* counts, int n)
{
    if (!h || !counts || n < 0) return MPM_MAG_EINVAL;
    return h->eng->scatter_stats(counts, n);
}

}  // extern "C"
