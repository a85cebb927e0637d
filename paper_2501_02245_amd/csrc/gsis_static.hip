// gsis_static.hip -- binding a case to a static device workspace, for callers
// that cannot allocate device memory (code under HIP graph capture, serving
// loops that must not call the allocator, harnesses that forbid it).
//
// The workspace is one file-scope device array, `scratch`, of a fixed size.
// Each GPU the library runs on holds its own copy until the process ends.
// Its device address is taken once per device with hipGetSymbolAddress (the
// array's name in host code is a host-side stand-in, not a device address)
// and kept per device; only that address is handed to the kernels.
//
// One case at a time owns a device's array: binding another case to it takes
// the array over and leaves the previous owner unbound (its calls then fail
// with E_STATE), and calls on two cases that overlap in time on one GPU would
// race on the same memory.  Everything a case needs zeroed is cleared by the
// bind, exactly as for a caller-owned workspace.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "gsis_impl.hpp"

namespace {

constexpr size_t SCRATCH_BYTES = (size_t)256 << 20;   // 256 MiB per device
constexpr int MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex g_mu;
void *g_addr[MAX_DEVICES];          // device address of scratch, per device
gsis_case g_owner[MAX_DEVICES];     // case bound to the device's scratch

}  // namespace

namespace gsis {

void static_release(gsis_case c)
{
    std::lock_guard<std::mutex> lock(g_mu);
    for (int d = 0; d < MAX_DEVICES; ++d)
        if (g_owner[d] == c) g_owner[d] = nullptr;
}

}  // namespace gsis

extern "C" gsis_status gsis_case_bind_static(gsis_case c, int64_t kinetic_capacity, void *stream)
{
    if (!c) return gsis::set_error(GSIS_E_ARG, "null case");
    size_t need = 0;
    gsis_status st = gsis_case_footprint(c, kinetic_capacity, &need);
    if (st) return st;
    if (need > SCRATCH_BYTES) {
        char msg[160];
        snprintf(msg, sizeof msg, "footprint of %zu bytes exceeds the static workspace of %zu bytes", need,
                 SCRATCH_BYTES);
        return gsis::set_error(GSIS_E_NOMEM, msg);
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gsis::set_error(GSIS_E_HIP, hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return gsis::set_error(GSIS_E_ARG, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_addr[dev]) {
        // first use on this device (current): the array's device address
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return gsis::set_error(GSIS_E_HIP, "hipGetSymbolAddress(scratch) failed");
        g_addr[dev] = p;
    }
    if (g_owner[dev] && g_owner[dev] != c) gsis::unbind_case(g_owner[dev]);
    g_owner[dev] = nullptr;
    st = gsis::bind_impl(c, g_addr[dev], SCRATCH_BYTES, kinetic_capacity, stream, false);
    if (st == GSIS_OK) g_owner[dev] = c;
    return st;
}
