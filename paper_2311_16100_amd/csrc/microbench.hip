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

// Scatter probe: the accumulation of one complex contribution into a
// voxel of an LDS accumulator, at effectively random voxels (as a row of
// pixels scatters into a brick).  Every lane keeps 16 random word indices
// in registers; repetition r uses index ^ c(r), c the same for all lanes, so
// the pattern of bank coincidences stays random from one repetition to the
// next.  Designs of one contribution:
//   0: two ds_add_u64 (64-bit fixed point per component)
//   1: one ds_add_u64 (both components packed as 32-bit halves)
//   2: two ds_add_rtn_u32 (32-bit low words) with the signed-overflow carry
//      into separate high words taken from the returned old values
//   3: two ds_add_u32 (32-bit words without return; the carry-free bound)
//   4: one ds_add_rtn_u64 of both components packed as 32-bit halves, with
//      the wraps of the low half and of the high half counted in separate
//      words from the returned old value
constexpr int kScatterWords = 2048;

__device__ __forceinline__ uint32_t mb_hash(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <int DESIGN>
__global__ __launch_bounds__(256) void lds_scatter_kernel(unsigned long long *out, int reps) {
    __shared__ unsigned long long acc64[DESIGN <= 1 || DESIGN == 4 ? 2 * kScatterWords : 1];
    __shared__ int lo[DESIGN >= 2 ? 2 * kScatterWords : 1];
    __shared__ int hi[DESIGN == 2 ? 2 * kScatterWords : 1];
    const int t = threadIdx.x;
    for (int i = t; i < 2 * kScatterWords; i += 256) {
        if (DESIGN <= 1 || DESIGN == 4) acc64[i] = 0ull;
        if (DESIGN >= 2) lo[i] = 0;
        if (DESIGN == 2) hi[i] = 0;
    }
    __syncthreads();
    uint32_t base[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) base[j] = mb_hash((blockIdx.x * 256u + t) * 16u + j) & (kScatterWords - 1);
    // contributions of either sign, about 2^20 in size (the carry path is
    // exercised when a sum leaves the 31-bit range)
    const int q0 = (int)(mb_hash(t * 7u + 3u) & 0x1FFFFF) - 0x100000;
    uint32_t ovf_any = 0;
    for (int r = 0; r < reps; r += 16) {
        const uint32_t c = ((uint32_t)r * 0x9E3779B1u >> 21) & (kScatterWords - 1);
        const int q = q0 + r;
        if (DESIGN == 2) {
            // all 32 atomics first, one test of the returned values after
            // them, the exact overflow test only when a sum may have left
            // [-2^30, 2^30)
            int o_re[16], o_im[16];
            uint32_t f = 0;
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const uint32_t i = base[j] ^ c;
                o_re[j] = atomicAdd(&lo[i], q);
                o_im[j] = atomicAdd(&lo[i + kScatterWords], -q);
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) f |= (uint32_t)(o_re[j] + 0x40000000) | (uint32_t)(o_im[j] + 0x40000000);
            ovf_any |= f;
            if ((int)f < 0) {
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const uint32_t i = base[j] ^ c;
                    const int n_re = (int)((uint32_t)o_re[j] + (uint32_t)q);
                    const int n_im = (int)((uint32_t)o_im[j] - (uint32_t)q);
                    if (((o_re[j] ^ n_re) & (q ^ n_re)) < 0) atomicAdd(&hi[i], n_re < 0 ? 1 : -1);
                    if (((o_im[j] ^ n_im) & (-q ^ n_im)) < 0) atomicAdd(&hi[i + kScatterWords], n_im < 0 ? 1 : -1);
                }
            }
            continue;
        }
        if (DESIGN == 4) {
            // lo[i]: wraps of the low halves, lo[i + words]: of the high halves
            unsigned long long o[16];
            uint32_t f = 0;
            const unsigned long long P = (unsigned long long)(long long)q + ((unsigned long long)(unsigned)(-q) << 32);
#pragma unroll
            for (int j = 0; j < 16; ++j) o[j] = atomicAdd(&acc64[base[j] ^ c], P);
#pragma unroll
            for (int j = 0; j < 16; ++j)
                f |= ((uint32_t)o[j] + 0x40000000u) | ((uint32_t)(o[j] >> 32) + 0x40000000u);
            ovf_any |= f;
            if ((int)f < 0) {
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const uint32_t i = base[j] ^ c;
                    const int lo_old = (int)(uint32_t)o[j];
                    const long long lo_new = (long long)lo_old + q;
                    const int dl = lo_new >= 0x80000000ll ? 1 : (lo_new < -0x80000000ll ? -1 : 0);
                    const int h_old = (int)((uint32_t)(o[j] >> 32) + (lo_old < 0 ? 1u : 0u));
                    const long long h_new = (long long)h_old - q + dl;
                    const int dh = h_new >= 0x80000000ll ? 1 : (h_new < -0x80000000ll ? -1 : 0);
                    if (dl) atomicAdd(&lo[i], dl);
                    if (dh) atomicAdd(&lo[i + kScatterWords], dh);
                }
            }
            continue;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const uint32_t i = base[j] ^ c;
            if (DESIGN == 0) {
                atomicAdd(&acc64[i], (unsigned long long)(long long)q);
                atomicAdd(&acc64[i + kScatterWords], (unsigned long long)(long long)(-q));
            } else if (DESIGN == 1) {
                atomicAdd(&acc64[i], (unsigned long long)(long long)q + ((unsigned long long)(unsigned)(-q) << 32));
            } else if (DESIGN == 3) {
                atomicAdd((unsigned *)&lo[i], (unsigned)q);
                atomicAdd((unsigned *)&lo[i + kScatterWords], (unsigned)(-q));
            }
        }
    }
    __syncthreads();
    if (t == 0) {
        unsigned long long s = ovf_any;
        for (int i = 0; i < 2 * kScatterWords; ++i) {
            if (DESIGN <= 1 || DESIGN == 4) s += acc64[i];
            if (DESIGN >= 2) s += (unsigned)lo[i];
            if (DESIGN == 2) s += (unsigned long long)(unsigned)hi[i] << 32;
        }
        out[blockIdx.x] = s;
    }
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

template <int DESIGN>
float time_scatter(void *out, int blocks, int reps) {
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    auto *o = (unsigned long long *)out;
    hipLaunchKernelGGL(lds_scatter_kernel<DESIGN>, dim3(blocks), dim3(256), 0, 0, o, reps);  // warm
    hipEventRecord(e0, 0);
    hipLaunchKernelGGL(lds_scatter_kernel<DESIGN>, dim3(blocks), dim3(256), 0, 0, o, reps);
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

// Duration (ms) of one launch of `blocks` blocks x 256 lanes x `reps`
// complex contributions scattered to random voxels with accumulator design
// `design` (0..4, see lds_scatter_kernel); `out`: device buffer of at least
// 8 * blocks bytes; reps a multiple of 16.  Negative on error.
float csg_mb_lds_scatter(int design, void *out, int blocks, int reps) {
    if (reps <= 0 || reps % 16) return -1.f;
    switch (design) {
        case 0: return time_scatter<0>(out, blocks, reps);
        case 1: return time_scatter<1>(out, blocks, reps);
        case 2: return time_scatter<2>(out, blocks, reps);
        case 3: return time_scatter<3>(out, blocks, reps);
        case 4: return time_scatter<4>(out, blocks, reps);
        default: return -1.f;
    }
}


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
