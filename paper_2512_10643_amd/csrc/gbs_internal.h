// Library-internal entry points shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/gbs_mps.h"
#include "gbs_sampler.h"

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

// Batched sampling of several handles (the server's sampling engine): a
// handle qualifies when it has the MFMA sampler operand and shots <= 2^20.
bool gbs_batch_supported(gbs_mps h, int64_t shots);
// Device bytes of one request's sweep buffers.
int64_t gbs_batch_bytes(gbs_mps h, int64_t shots);
// Carve the request's buffers from `region` (cap bytes), start its left
// vectors on `st`, and fill its descriptor at site 1.
int gbs_batch_prepare(gbs_mps h, int64_t shots, uint64_t seed, int32_t* out, hipStream_t st, void* region, size_t cap,
                      SampleBatchDesc* d);
// Accumulator tiles the handle's site needs (8, 16, 24 or 32).
int gbs_batch_site_nt(gbs_mps h, int site);
// Device bytes a handle holds.
int64_t gbs_mps_device_bytes(gbs_mps h);
