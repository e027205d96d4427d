// noise.hip -- seeded complex Gaussian noise for synthetic images, made on
// the device, for data sets whose images are regenerated batch by batch (too
// many to keep in device memory).  Pure input synthesis: nothing of the
// method is computed here.
//
// The noise of pixel (ky, kx) of data-set image i is a function of
// (seed, i, ky, kx) only, so an image receives the same noise whenever it is
// regenerated, in any batch and at any position in it.  Counter-based
// generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC 2011) with counter (pixel, i low, i high,
// stream tag) and key (seed low, seed high); two of its four words give a
// standard normal pair by the Box-Muller transform.  Real and imaginary
// parts are N(0, sigma^2 / 2); only the pixels of the disk
// kx^2 + ky^2 <= k2max receive noise.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace {

constexpr uint32_t kPhiloxM0 = 0xD2511F53u, kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u, kPhiloxW1 = 0xBB67AE85u;
constexpr uint32_t kNoiseTag = 0x4E4F4953u;  // stream tag of image noise

__device__ inline void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = kPhiloxM0 * c[0], hi0 = __umulhi(kPhiloxM0, c[0]);
        const uint32_t lo1 = kPhiloxM1 * c[2], hi1 = __umulhi(kPhiloxM1, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += kPhiloxW0;
        k1 += kPhiloxW1;
    }
}

// grid: x over the pixels of an image, y over the batch's images
__global__ __launch_bounds__(256) void add_disk_noise_kernel(float2 *x, const int64_t *idx, int M, int k2max,
                                                             float sd, uint32_t s_lo, uint32_t s_hi) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= M * M) return;
    const int ky = p / M - M / 2, kx = p % M - M / 2;
    if (kx * kx + ky * ky > k2max) return;
    const int64_t b = blockIdx.y;
    const uint64_t i = (uint64_t)idx[b];
    uint32_t c[4] = {(uint32_t)p, (uint32_t)i, (uint32_t)(i >> 32), kNoiseTag};
    philox10(c, s_lo, s_hi);
    // u1 in (0, 1], u2 in [0, 1)
    const float u1 = ((float)(c[0] >> 8) + 1.0f) * 0x1p-24f;
    const float u2 = (float)(c[1] >> 8) * 0x1p-24f;
    const float rad = sd * sqrtf(-2.0f * logf(u1));
    float s, co;
    sincospif(2.0f * u2, &s, &co);
    float2 *q = x + b * (int64_t)M * M + p;
    float2 v = *q;
    v.x += rad * co;
    v.y += rad * s;
    *q = v;
}

}  // namespace

extern "C" {

// x: device complex64 [n][M][M] (row-major, DC at M/2); idx: device int64
// [n], the data-set index of each image.  sigma2: noise variance (per
// complex pixel).  Returns 0, or -1 for invalid sizes, or the HIP error code.
int synth_add_disk_noise(void *x, const void *idx, int64_t n, int M, int k2max, double sigma2, uint64_t seed,
                         void *stream) {
    if (n < 0 || n > 65535 || M <= 0 || M > 4096 || !(sigma2 >= 0.0)) return -1;
    if (n == 0) return 0;
    const float sd = (float)sqrt(sigma2 / 2.0);
    dim3 grid((unsigned)((M * M + 255) / 256), (unsigned)n);
    hipLaunchKernelGGL(add_disk_noise_kernel, grid, dim3(256), 0, (hipStream_t)stream, (float2 *)x,
                       (const int64_t *)idx, M, k2max, sd, (uint32_t)seed, (uint32_t)(seed >> 32));
    return (int)hipGetLastError();
}

}  // extern "C"
