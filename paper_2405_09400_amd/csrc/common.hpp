// Shared host/device helpers of the gfx950 domain-decomposition library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/domdec.h"

namespace dd {

// Log-domain "zero mass" sentinel: finite so that sums and differences of
// sentinels never produce inf - inf; exp(sentinel - finite) underflows to 0.
constexpr float kNegF = -1.0e30f;
constexpr double kNegD = -1.0e30;
// entries at or below this are treated as zero mass
constexpr double kZeroMassLog = -1.0e29;

template <typename T>
__host__ __device__ constexpr T neg_sentinel();
template <>
__host__ __device__ constexpr float neg_sentinel<float>() { return kNegF; }
template <>
__host__ __device__ constexpr double neg_sentinel<double>() { return kNegD; }

__device__ __forceinline__ float fexp(float x) { return __expf(x); }
__device__ __forceinline__ double fexp(double x) { return exp(x); }
__device__ __forceinline__ float flog(float x) { return __logf(x); }
__device__ __forceinline__ double flog(double x) { return log(x); }

// Wave64 reduction of a double (all lanes receive the sum).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ int wave_min_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide sum of a double; `scratch` holds >= blockDim.x/64 doubles.  The
// result is returned to every thread.  Fixed reduction order (deterministic).
__device__ __forceinline__ double block_sum(double v, double* scratch) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) scratch[wid] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += scratch[w];
    __syncthreads();
    return t;
}

struct Status {
    dd_status code = DD_OK;
    std::string msg;
};

// Thread-local message of the last context-free error.
void set_global_error(const std::string& m);
const char* global_error();

#define DD_HIP(call, st_ret)                                                              \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            char b_[256];                                                                 \
            snprintf(b_, sizeof b_, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                     __FILE__, __LINE__);                                                 \
            st_ret.code = e_ == hipErrorOutOfMemory ? DD_ENOMEM : DD_EDEVICE;              \
            st_ret.msg = b_;                                                              \
            return st_ret;                                                                \
        }                                                                                 \
    } while (0)

// Device-memory supplier of a context: the caller's hooks (dd_params.dev_alloc / dev_free)
// when both are set, else hipMalloc / hipFree.  A hook allocation that returns NULL is
// reported as out of memory.  Buffers are released only after every kernel that touches them
// has been ordered before the release on the context's stream.
struct Mem {
    void* (*alloc)(size_t, void*) = nullptr;
    void (*release)(void*, void*) = nullptr;
    void* ud = nullptr;

    template <typename P>
    hipError_t get(P** p, size_t bytes) const {
        if (!alloc) return hipMalloc(p, bytes);
        *p = static_cast<P*>(alloc(bytes, ud));
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    void put(void* p) const {
        if (!p) return;
        if (alloc)
            release(p, ud);
        else
            (void)hipFree(p);
    }
};

}  // namespace dd
