// One instantiation of the engine, selected at compile time by MPM_REAL
// (float or double) and MPM_DIM (2 or 3); the build compiles this file once
// per combination so the four variants build in parallel.
#include "engine.hpp"

#ifndef MPM_REAL
#error "define MPM_REAL"
#endif
#ifndef MPM_DIM
#error "define MPM_DIM"
#endif
#ifndef MPM_FACTORY
#error "define MPM_FACTORY"
#endif

namespace mpm {

EngineBase* MPM_FACTORY(const mpm_mag_instance_desc* d, int n, const int64_t* np, int* status, std::string* msg,
                        void* ws, size_t ws_bytes)
{
    auto* e = new (std::nothrow) Engine<MPM_REAL, MPM_DIM>();
    if (!e) {
        *status = MPM_MAG_ENOMEM;
        return nullptr;
    }
    *status = e->init(d, n, np, ws, ws_bytes);
    if (*status != MPM_MAG_OK) {
        *msg = e->err;
        delete e;
        return nullptr;
    }
    return e;
}

}  // namespace mpm
