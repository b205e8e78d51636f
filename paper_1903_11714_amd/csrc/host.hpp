// host.hpp — host-side helpers shared by the library's translation units (defined in ising.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace ising_host {

int hip_failed(hipError_t e, const char* what);  // records the text for ising_last_error; ISING_EHIP
int check_launch(const char* what);              // ISING_OK, or hip_failed on hipGetLastError
bool valid_beta(double beta);                    // finite >= 0 or +inf
bool aligned16(const void* p);
bool xcd_remap();                                // option "xcd_remap"
int64_t option(const char* name);                // current value of a launch-shape option
int zero_trace(int64_t* p, int64_t n, hipStream_t stream);  // n int64 set to 0 by a kernel

// Spread sets of a traced sweep loop.  Up to 64 traced launches take a set each: 64 cache lines of
// 128 bytes, a workgroup adding (M, E) into line blockIdx.x % 64 (spread_line), so that the
// workgroups' atomics do not queue on one address.  A fold then writes each set's sums into its
// trace entries and clears the set.  The sets come from a per-device stream-ordered pool, or from
// memory the caller passes.
class SpreadTrace {
  public:
    SpreadTrace() = default;
    SpreadTrace(const SpreadTrace&) = delete;
    SpreadTrace& operator=(const SpreadTrace&) = delete;
    ~SpreadTrace();
    // n_launches: traced launches to come (the sets to clear); given: 512 KiB of device memory for
    // the sets, or null to take them from the pool (returned at destruction, in stream order)
    int begin(int64_t* given, int64_t n_launches, hipStream_t s);
    // The set of the next traced launch, whose n (<= 4) values belong at dst.  The launches between
    // two folds write consecutive trace entries; a launch that does not continue them folds first.
    int next(int64_t* dst, uint32_t n, int64_t** set);
    // the sums of the sets taken since the last fold into their trace entries
    int fold();

  private:
    int64_t* sets_ = nullptr;
    bool owned_ = false;
    hipStream_t s_ = nullptr;
    int64_t* dst0_ = nullptr;
    uint32_t n_ = 0, used_ = 0;
};

}  // namespace ising_host
