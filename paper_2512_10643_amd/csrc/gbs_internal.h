// Library-internal entry points shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/gbs_mps.h"

// gbs_mps_build with an explicit stream.  ordered_keep: the handle's own
// buffers are stream-ordered allocations on `stream` and are released in
// order on it by gbs_mps_free (the stream must outlive the handle).
int gbs_build_handle(const double* gamma, int M, const gbs_build_opts* opt, hipStream_t stream, bool ordered_keep,
                     gbs_mps* out, int only_site);

// Record `msg` as this thread's gbs_last_error() text and return `code`.
int gbs_fail(int code, const std::string& msg);

// Sampling (as gbs_mps_sample) on buffers carved from a device region of
// `cap` bytes the caller provides; allocates nothing.
int gbs_sample_in_region(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, hipStream_t st, void* region,
                         size_t cap);
