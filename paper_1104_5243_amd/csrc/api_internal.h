// Host-side helpers shared by the C-ABI entry points (defined in api.hip):
// the per-thread error message, the per-device staging buffer and the
// kernel-timing hooks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>
#include <string>

namespace fdk {
namespace host {

extern thread_local std::string g_err;
// sets the calling thread's error message, returns code
int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// One grow-only device buffer per device for a call's staged planes,
// matrices and tables; its users are ordered by the last_use event.
struct Staging {
    void* ptr = nullptr;
    size_t bytes = 0;
    hipEvent_t last_use = nullptr;  // recorded after the last call's kernels
    // the folded matrices of a call: written on the host into pinned
    // memory, copied once to the end of the staging buffer
    float* host_mats = nullptr;
    size_t host_floats = 0;
    hipEvent_t mats_copied = nullptr;  // recorded after the last such copy
    // the fused backprojection's second stream, on which the next pass's
    // views are staged into the other half of the buffer while the current
    // pass runs (default priority, non-blocking; created on first use)
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr;                // the call's start, on its stream
    hipEvent_t staged[2] = {nullptr, nullptr};  // a half filled (side stream)
    hipEvent_t freed[2] = {nullptr, nullptr};   // a half's pass done (call's stream)
};
extern std::mutex g_stage_mu;
// The calling device's staging buffer with at least `bytes`, `stream`
// ordered after its previous user.  Caller holds g_stage_mu.
int acquire_staging(size_t bytes, hipStream_t stream, Staging** out);

// HIP events around a call's kernels while fdk_profile_begin is active
int timed_begin(hipStream_t s, hipEvent_t* e0);
int timed_end(hipStream_t s, hipEvent_t e0);

}  // namespace host
}  // namespace fdk
