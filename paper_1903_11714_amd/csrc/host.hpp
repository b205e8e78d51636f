// host.hpp — host-side helpers shared by the library's translation units (defined in ising.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace ising_host {

int hip_failed(hipError_t e, const char* what);  // records the text for ising_last_error; ISING_EHIP
int check_launch(const char* what);              // ISING_OK, or hip_failed on hipGetLastError
bool valid_beta(double beta);                    // finite >= 0 or +inf
bool aligned16(const void* p);
bool xcd_remap();                                // option "xcd_remap"
int64_t option(const char* name);                // current value of a launch-shape option
int zero_trace(int64_t* p, int64_t n, hipStream_t stream);  // n int64 set to 0 by a kernel

}  // namespace ising_host
