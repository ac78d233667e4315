// Copy of a device state (structure of arrays) to host records, shared by
// state export (sim_export_state) and the server's result copies.
//
// A device-to-host copy into pageable memory goes through the runtime's own
// staging and serialises across host threads; here each calling thread owns a
// pinned staging buffer, copies a chunk of the state into it at DMA speed and
// interleaves the chunk into the caller's (lo, hi) key records and amplitudes.
// Several threads can do this at once (the server copies the states of
// several finished requests in parallel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "host_pool.h"
#include "sim_internal.h"

namespace sparsesim {

namespace {

constexpr size_t kStageBytes = 16u << 20;   // per host thread, kept for the process's lifetime

struct Stage {
  char* p = nullptr;
};

// The calling thread's staging buffer (allocated on first use, never freed:
// host threads of the library live as long as the process).
hipError_t stage_of_thread(char** out) {
  static thread_local Stage st;
  if (!st.p) {
    void* p = nullptr;
    const hipError_t e = hipHostMalloc(&p, kStageBytes, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    st.p = static_cast<char*>(p);
  }
  *out = st.p;
  return hipSuccess;
}

}  // namespace

namespace {

// Chunks of the state through the staging buffer; emit(b, m, s_lo, s_hi,
// s_amp, pb, pe) writes entries [pb, pe) of the chunk that starts at entry b.
template <class Emit>
hipError_t staged_copy(const uint64_t* lo, const uint64_t* hi, const double2* amp, uint64_t n, Emit&& emit) {
  if (!n) return hipSuccess;
  char* stage = nullptr;
  hipError_t e = stage_of_thread(&stage);
  if (e != hipSuccess) return e;
  const size_t per_entry = hi ? 32 : 24;
  const uint64_t chunk = kStageBytes / per_entry;
  for (uint64_t b = 0; b < n; b += chunk) {
    const uint64_t m = std::min<uint64_t>(chunk, n - b);
    auto* s_lo = reinterpret_cast<const uint64_t*>(stage);
    auto* s_hi = reinterpret_cast<const uint64_t*>(stage + 8 * m);
    auto* s_amp = reinterpret_cast<const double2*>(stage + (hi ? 16 : 8) * m);
    e = hipMemcpy(stage, lo + b, 8 * m, hipMemcpyDeviceToHost);
    if (e == hipSuccess && hi) e = hipMemcpy(stage + 8 * m, hi + b, 8 * m, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(const_cast<double2*>(s_amp), amp + b, 16 * m, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    // On the host thread pool (on this thread alone when it is itself one of
    // the pool's tasks).
    parallel_parts(m, 1u << 16, [&](size_t pb, size_t pe, size_t) { emit(b, s_lo, hi ? s_hi : nullptr, s_amp, pb, pe); });
  }
  return hipSuccess;
}

}  // namespace

hipError_t copy_state_to_host(const uint64_t* lo, const uint64_t* hi, const double2* amp, uint64_t n, sim_key* keys,
                              sim_c64* amps) {
  return staged_copy(lo, hi, amp, n,
                     [&](uint64_t b, const uint64_t* s_lo, const uint64_t* s_hi, const double2* s_amp, size_t pb, size_t pe) {
                       for (size_t k = pb; k < pe; ++k) keys[b + k] = sim_key{s_lo[k], s_hi ? s_hi[k] : 0};
                       std::memcpy(amps + b + pb, s_amp + pb, 16 * (pe - pb));
                     });
}

hipError_t copy_state_to_host_soa(const uint64_t* lo, const uint64_t* hi, const double2* amp, uint64_t n,
                                  uint64_t* key_lo, uint64_t* key_hi, sim_c64* amps) {
  return staged_copy(lo, hi, amp, n,
                     [&](uint64_t b, const uint64_t* s_lo, const uint64_t* s_hi, const double2* s_amp, size_t pb, size_t pe) {
                       std::memcpy(key_lo + b + pb, s_lo + pb, 8 * (pe - pb));
                       if (key_hi) {
                         if (s_hi) std::memcpy(key_hi + b + pb, s_hi + pb, 8 * (pe - pb));
                         else std::memset(key_hi + b + pb, 0, 8 * (pe - pb));
                       }
                       std::memcpy(amps + b + pb, s_amp + pb, 16 * (pe - pb));
                     });
}

}  // namespace sparsesim
