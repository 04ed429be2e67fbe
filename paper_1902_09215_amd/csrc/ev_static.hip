// Evaluation without allocation: ev_eval_fitness_static.
//
// Every buffer its kernels use besides the population's plan and the
// caller's outputs (the work counters, each plan level's intermediate
// result slots and the spill slabs of the interpreter's waves) is carved
// from `scratch`, a static device array of EV_STATIC_SCRATCH_BYTES that
// each device the library runs on holds until the process ends.  In host
// code the array's name is only a host-side stand-in: the device address of
// each device's copy is looked up once per device, with that device current,
// when a context is created there (static_scratch_init), and only that
// address is ever handed to a kernel.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ev_runtime.h"

namespace ev {

static __device__ __align__(256) uint8_t scratch[EV_STATIC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static constexpr int MAX_DEVICES = 64;
static void* g_scratch_ptr[MAX_DEVICES] = {};

// Called by ev_create with `device` current.
ev_status static_scratch_init(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return fail(EV_EINVAL, "device %d out of range", device);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return EV_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return fail(EV_EDEVICE, "static scratch of device %d: %s", device, hipGetErrorString(e));
    }
    g_scratch_ptr[device] = ptr;
    return EV_OK;
}

static void* static_scratch(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace ev

using namespace ev;

extern "C" ev_status ev_eval_fitness_static(ev_ctx* c, ev_pop pop, int32_t table, float* fitness, float* per_case,
                                            int32_t* hits)
{
    if (!c || !fitness) return fail(EV_EINVAL, "ev_eval_fitness_static: bad arguments");
    Pop* P = pop_get(c, pop);
    if (!P) return fail(EV_ENOTFOUND, "no population %d", pop);
    const hipError_t e = hipSetDevice(c->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    uint8_t* base = (uint8_t*)static_scratch(c->device);
    if (!base) return fail(EV_EDEVICE, "static scratch of device %d not set up", c->device);
    return eval_in_scratch(c, P, table, fitness, per_case, hits, base, EV_STATIC_SCRATCH_BYTES);
}
