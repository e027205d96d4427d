// microbench.hip -- throughput probes of the GPU's LDS atomics and vector
// ALU (measurement support: the peaks that the brick kernels' counter
// figures are compared with).  Built into its own library
// (libcsg_microbench.so); nothing in the operator library calls it.
//
// LDS atomics: every lane of a 256-thread block adds to its own LDS word
// (address lane * stride, so stride 1 gives each wave 64 consecutive words),
// `reps` times, with the result unused by the loop (ds_add without return).
// Blocks per CU and LDS per block are chosen by the caller through `blocks`.
// VALU: every lane runs 8 independent FMA chains, `reps` iterations each.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr int kWords = 1024;

template <typename T>
__global__ __launch_bounds__(256) void lds_add_kernel(T *out, int reps, int stride) {
    __shared__ T acc[kWords];
    const int t = threadIdx.x;
    for (int i = t; i < kWords; i += 256) acc[i] = (T)0;
    __syncthreads();
    const int a = (t * stride) & (kWords - 1);
    for (int r = 0; r < reps; ++r) atomicAdd(&acc[a], (T)(1 + (r & 1)));
    __syncthreads();
    if (t == 0) {
        T s = (T)0;
        for (int i = 0; i < kWords; ++i) s += acc[i];
        out[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(256) void valu_fma_kernel(float *out, int reps, float a, float b) {
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (float)(threadIdx.x + j);
    for (int r = 0; r < reps; ++r) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = fmaf(x[j], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

template <typename T>
float time_lds(void *out, int blocks, int reps, int stride) {
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipLaunchKernelGGL(lds_add_kernel<T>, dim3(blocks), dim3(256), 0, 0, (T *)out, reps, stride);  // warm
    hipEventRecord(e0, 0);
    hipLaunchKernelGGL(lds_add_kernel<T>, dim3(blocks), dim3(256), 0, 0, (T *)out, reps, stride);
    hipEventRecord(e1, 0);
    hipEventSynchronize(e1);
    float ms = -1.f;
    if (hipGetLastError() == hipSuccess) hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return ms;
}

}  // namespace

extern "C" {

// Duration (ms) of one launch of `blocks` blocks x 256 lanes x `reps` LDS
// atomic adds of type kind (0 u32, 1 u64, 2 f32, 3 f64); `out` is a device
// buffer of at least 8 * blocks bytes.  Returns a negative value on error.
float csg_mb_lds_add(int kind, void *out, int blocks, int reps, int stride) {
    switch (kind) {
        case 0: return time_lds<uint32_t>(out, blocks, reps, stride);
        case 1: return time_lds<unsigned long long>(out, blocks, reps, stride);
        case 2: return time_lds<float>(out, blocks, reps, stride);
        case 3: return time_lds<double>(out, blocks, reps, stride);
        default: return -1.f;
    }
}

// Duration (ms) of `blocks` x 256 lanes x reps x 8 FMAs; out: device float
// [blocks * 256].
float csg_mb_valu_fma(float *out, int blocks, int reps) {
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipLaunchKernelGGL(valu_fma_kernel, dim3(blocks), dim3(256), 0, 0, out, reps, 0.999f, 0.5f);
    hipEventRecord(e0, 0);
    hipLaunchKernelGGL(valu_fma_kernel, dim3(blocks), dim3(256), 0, 0, out, reps, 0.999f, 0.5f);
    hipEventRecord(e1, 0);
    hipEventSynchronize(e1);
    float ms = -1.f;
    if (hipGetLastError() == hipSuccess) hipEventElapsedTime(&ms, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return ms;
}

}  // extern "C"
