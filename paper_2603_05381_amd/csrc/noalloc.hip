// bpm_decode_noalloc: bpm_decode with its workspace in a fixed array of
// device memory inside the library, for callers that cannot allocate.
//
// The array is a file-scope __device__ variable, so every device the library
// runs on holds one copy of it (kNoallocScratchBytes) from the time the
// library's code is loaded there until the process ends.  Its device address
// is looked up once per device, with that device current, and kept; host
// code uses only that address, never the variable's name (which on the host
// is a stand-in, not device memory).  Every call on a device shares that
// device's array: calls that overlap on one device race.  The decode clears
// what must start at zero itself (its work-queue counters) with a fill
// kernel, and writes every other workspace entry before reading it, so the
// previous call's contents do not matter.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "bpm.h"
#include "graph_internal.hpp"

namespace {

constexpr size_t kNoallocScratchBytes = (size_t)BPM_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

std::mutex g_lock;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's array (looked up on first use).
bpm_status scratch_ptr(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return bpm::set_last_error(BPM_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return bpm::set_last_error(BPM_EUNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return bpm::set_last_error(BPM_EDEVICE, std::string("hipGetSymbolAddress of the scratch array: ") +
                                                        hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return BPM_OK;
}

}  // namespace

extern "C" {

bpm_status bpm_decode_noalloc(const bpm_graph *g, const uint64_t *syn, const uint64_t *obs, uint64_t n_shots,
                              const bpm_decode_opts *opts, const bpm_decode_out *out, void *stream) {
    if (!g || !opts || !out) return bpm::set_last_error(BPM_EINVAL, "NULL argument");
    if (opts->class_streams > 1)
        return bpm::set_last_error(BPM_EUNSUPPORTED,
                                   "bpm_decode_noalloc runs every kernel on the caller's stream: class_streams must be 0 or 1");
    size_t need = 0;
    bpm_status st = bpm_decode_workspace_size(g, n_shots, opts, &need);
    if (st != BPM_OK) return st;
    if (need > kNoallocScratchBytes)
        return bpm::set_last_error(BPM_EINVAL, "bpm_decode_noalloc: these shots and options need " + std::to_string(need) +
                                                   " bytes of workspace, more than the " +
                                                   std::to_string(kNoallocScratchBytes) +
                                                   "-byte scratch array; use fewer shots or a smaller s_cap");
    if (n_shots == 0) return bpm_decode(g, syn, obs, n_shots, opts, out, nullptr, 0, stream);
    void *ws = nullptr;
    st = scratch_ptr(&ws);
    if (st != BPM_OK) return st;
    return bpm_decode(g, syn, obs, n_shots, opts, out, ws, kNoallocScratchBytes, stream);
}

}  // extern "C"
