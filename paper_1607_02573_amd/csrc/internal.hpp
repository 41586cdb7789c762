// Internal interface between the C ABI's source files (not part of mw.h):
// error handling of the entry points and access to a problem's device,
// stream and byte budget for the code that drives problems through the ABI
// (invert.hip).
#pragma once

#include <functional>

#include "kernels.hpp"

namespace mw {

// Runs f; an exception becomes the returned status and the calling thread's
// mw_last_error() text.
mw_status guarded(const std::function<void()>& f);

// Makes `dev` the current device for the lifetime of the object.
struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    MW_HIP(hipGetDevice(&prev));
    if (prev != dev) MW_HIP(hipSetDevice(dev));
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

hipStream_t problem_stream(mw_problem* p);
int problem_device(mw_problem* p);
// device memory counted against the problem's context budget (MW_ENOMEM beyond it)
DevBuf problem_alloc(mw_problem* p, int64_t bytes);
DevBuf problem_upload(mw_problem* p, const void* host, int64_t bytes);
// Y = A X (Bsub NULL) or Y = Bsub - A X for nc columns (leading dimensions ld), on the problem's stream
void problem_spmm(mw_problem* p, const double2* X, double2* Y, int nc, int64_t ld, const double2* Bsub);
// objects that drive a problem (an inversion) register themselves, so that
// mw_destroy_problem refuses while they exist
void problem_retain(mw_problem* p);
void problem_release(mw_problem* p);

}  // namespace mw
