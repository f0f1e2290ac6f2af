// Internal declarations shared by the host files of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "weno_fwd.h"
#include "weno_zoom.h"

// Device-resident table of a batched call, written into the caller's
// workspace by weno_zoom2x_batched_plan:
//   [0, 256)                 BatchTable header
//   [256, ...)               FwdJob jobs[count]       (largest image first)
//   then                     int64_t prefix[count+1]  (first queue item of each image)
//   then                     FwdParams params[count]
struct BatchTable {
    unsigned long long counter;  // queue head, zeroed by a kernel before every run
    int64_t total_items;
    int32_t count;
    int32_t pad0;
    int64_t params_offset;
};

__host__ __device__ constexpr size_t batch_jobs_offset() { return 256; }
__host__ __device__ constexpr size_t batch_prefix_offset(int count)
{
    return batch_jobs_offset() + (size_t)count * sizeof(wz::FwdJob);
}
__host__ __device__ constexpr size_t batch_params_offset(int count)
{
    return (batch_prefix_offset(count) + (size_t)(count + 1) * sizeof(int64_t) + 15) / 16 * 16;
}
__host__ __device__ constexpr size_t batch_table_bytes(int count)
{
    return (batch_params_offset(count) + (size_t)count * sizeof(wz::FwdParams) + 255) / 256 * 256;
}
__host__ __device__ inline const wz::FwdJob* batch_jobs(const BatchTable* t)
{
    return (const wz::FwdJob*)((const uint8_t*)t + batch_jobs_offset());
}
__host__ __device__ inline const int64_t* batch_prefix(const BatchTable* t)
{
    return (const int64_t*)((const uint8_t*)t + batch_prefix_offset(t->count));
}
__host__ __device__ inline const wz::FwdParams* batch_params(const BatchTable* t)
{
    return (const wz::FwdParams*)((const uint8_t*)t + t->params_offset);
}

// host helpers (weno_api.hip)
int wz_hip_error(hipError_t e, const char* what);
int wz_esize(int32_t dtype);
int wz_check_tensor(const weno_tensor_t* t);
int wz_check_params(const weno_params_t* p);
int wz_check_pair(const weno_tensor_t* src, const weno_tensor_t* dst, int factor);
void wz_byte_range(const weno_tensor_t* t, uintptr_t* lo, uintptr_t* hi);
bool wz_overlap(const weno_tensor_t* a, const weno_tensor_t* b);
int64_t wz_plane_extent(const weno_tensor_t* t);
double wz_nbw(const weno_params_t* p);
int wz_beta_mode(float beta);
