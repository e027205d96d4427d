// volume_kernels.hip -- streaming kernels over whole volumes: initialisation
// of gradient / HVP outputs, Rademacher probes, Hutchinson accumulation and
// the preconditioned SGD update of Algorithm 1.  All are HBM-bound
// grid-stride loops in which consecutive lanes touch consecutive voxels, so
// every wavefront access is fully coalesced.
#include "csg_device.h"
#include "csg_internal.h"

namespace csg {

static inline unsigned stream_blocks(int64_t units) {
    int64_t b = (units + kBlock - 1) / kBlock;
    if (b > 8192) b = 8192;  // grid-stride beyond 32 blocks per CU
    if (b < 1) b = 1;
    return (unsigned)b;
}

// Kernels that end in a double-precision atomic per block use fewer, longer
// blocks (16 waves per CU) to keep those atomics few.
static inline unsigned reduce_blocks(int64_t units) {
    int64_t b = (units + kBlock - 1) / kBlock;
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return (unsigned)b;
}

// out = lam * in (complex), norm2 += sum |in|^2 (norm2 may be NULL).
__global__ __launch_bounds__(kBlock) void scaled_copy_kernel(float2 *__restrict__ out, const float2 *__restrict__ in,
                                                              float lam, int64_t nvox, double *norm2) {
    __shared__ double red[16];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nvox; k += stride) {
        const float2 v = in[k];
        out[k] = make_float2(lam * v.x, lam * v.y);
        s += (double)v.x * v.x + (double)v.y * v.y;
    }
    if (norm2) {
        const double t = block_sum(s, red);
        if (threadIdx.x == 0) atomicAdd(norm2, t);
    }
}

// The same over pairs of voxels (16-byte accesses; pointers 16-byte aligned,
// nvox even).
__global__ __launch_bounds__(kBlock) void scaled_copy2_kernel(float4 *__restrict__ out, const float4 *__restrict__ in,
                                                               float lam, int64_t npair, double *norm2) {
    __shared__ double red[16];
    double s = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npair; k += stride) {
        const float4 v = in[k];
        out[k] = make_float4(lam * v.x, lam * v.y, lam * v.z, lam * v.w);
        s += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
    }
    if (norm2) {
        const double t = block_sum(s, red);
        if (threadIdx.x == 0) atomicAdd(norm2, t);
    }
}

__global__ void fill_f64_kernel(double *p, int n, double v) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = v;
}

__global__ __launch_bounds__(kBlock) void fill_f32_kernel(float *__restrict__ p, int64_t n, float v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}

// loss = scale * data + lam/2 * norm2 (all device scalars)
__global__ void finish_loss_kernel(double *loss_out, const double *data, const double *norm2, float scale, float lam) {
    if (threadIdx.x == 0) *loss_out = (double)scale * data[0] + 0.5 * (double)lam * norm2[0];
}

// Rademacher entries: thread t writes voxels 4t..4t+3, all inside one 128-bit
// Philox block (k/128), using bits (k mod 128).
__device__ __forceinline__ float4 rademacher4(uint64_t seed, uint64_t probe, int64_t k4) {
    const int64_t k = k4 * 4;
    const U4 r = rademacher_block(seed, probe, (uint32_t)(k >> 7));
    const int bit = (int)(k & 127);
    const uint32_t word = (bit < 32) ? r.x : (bit < 64) ? r.y : (bit < 96) ? r.z : r.w;
    const uint32_t b = word >> (bit & 31);
    return make_float4((b & 1u) ? -1.f : 1.f, (b & 2u) ? -1.f : 1.f, (b & 4u) ? -1.f : 1.f, (b & 8u) ? -1.f : 1.f);
}

__global__ __launch_bounds__(kBlock) void rademacher_kernel(float *__restrict__ z, int64_t nvox, uint64_t seed,
                                                             uint64_t probe) {
    const int64_t n4 = (nvox + 3) / 4;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n4; t += stride) {
        const float4 v = rademacher4(seed, probe, t);
        const int64_t k = t * 4;
        if (k + 3 < nvox) {
            *reinterpret_cast<float4 *>(z + k) = v;
        } else {
            const float vv[4] = {v.x, v.y, v.z, v.w};
            for (int e = 0; e < 4 && k + e < nvox; ++e) z[k + e] = vv[e];
        }
    }
}

// Start of the product of a probe pair z = z_pa + i z_pb: hz = lam z, and z
// itself only where a kernel must read it (z may be NULL: the brick kernel
// and the accumulation below regenerate it).  Voxel k takes bit k mod 128 of Philox block k / 128 (rademacher_block).
// A wave covers 8192 consecutive voxels: each lane evaluates one Philox block
// per probe into LDS, then the wave writes the voxels two per lane and store,
// consecutive lanes at consecutive 16-byte addresses.  nvox is even and hz is
// 16-byte aligned.
constexpr int kProbeWaves = kBlock / 64;

// the bits of probe pair (pa, pb) for the 8192 voxels of chunk c, into
// words[probe][word][block of the chunk] of the calling wave
__device__ __forceinline__ void probe_chunk_bits(uint32_t (*words)[4][64], int64_t c, int lane, uint64_t seed,
                                                 uint64_t pa, uint64_t pb, int has_b) {
    const uint32_t blk = (uint32_t)(c * 64 + lane);
    const U4 ra = rademacher_block(seed, pa, blk);
    const U4 rb = has_b ? rademacher_block(seed, pb, blk) : U4{0u, 0u, 0u, 0u};
    words[0][0][lane] = ra.x;
    words[0][1][lane] = ra.y;
    words[0][2][lane] = ra.z;
    words[0][3][lane] = ra.w;
    words[1][0][lane] = rb.x;
    words[1][1][lane] = rb.y;
    words[1][2][lane] = rb.z;
    words[1][3][lane] = rb.w;
    // the words were written by this wave: its LDS accesses complete in
    // order, and the barrier keeps the compiler from moving them
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// voxels 2 q and 2 q + 1 of chunk c (q = c 4096 + 64 j + lane) take bits
// 2 lane and 2 lane + 1 of block c 64 + j: the pair (a0 + i b0, a1 + i b1)
__device__ __forceinline__ float4 probe_pair_values(uint32_t (*words)[4][64], int j, int lane, int has_b) {
    const int w = lane >> 4, sh = (2 * lane) & 31;
    const uint32_t ba = words[0][w][j] >> sh, bb = words[1][w][j] >> sh;
    const float a0 = (ba & 1u) ? -1.f : 1.f, a1 = (ba & 2u) ? -1.f : 1.f;
    const float b0 = has_b ? ((bb & 1u) ? -1.f : 1.f) : 0.f;
    const float b1 = has_b ? ((bb & 2u) ? -1.f : 1.f) : 0.f;
    return make_float4(a0, b0, a1, b1);
}

__global__ __launch_bounds__(kBlock) void probe_init_kernel(float4 *__restrict__ z_out, float4 *__restrict__ hz,
                                                             int64_t nvox, uint64_t seed, uint64_t pa, uint64_t pb,
                                                             int has_b, float lam) {
    __shared__ uint32_t words[kProbeWaves][2][4][64];  // [wave][probe][word][block of the chunk]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nchunk = (nvox + 8191) / 8192;
    const int64_t npair = nvox / 2;
    for (int64_t c = (int64_t)blockIdx.x * kProbeWaves + wv; c < nchunk; c += (int64_t)gridDim.x * kProbeWaves) {
        probe_chunk_bits(words[wv], c, lane, seed, pa, pb, has_b);
        for (int j = 0; j < 64; ++j) {
            const int64_t q = c * 4096 + (int64_t)j * 64 + lane;
            if (q >= npair) break;
            const float4 z = probe_pair_values(words[wv], j, lane, has_b);
            if (z_out) z_out[q] = z;
            hz[q] = make_float4(lam * z.x, lam * z.y, lam * z.z, lam * z.w);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// diag += w (Re z Re hz + Im z Im hz) with z regenerated as above; with
// `first` the sum starts here (diag is not read).  nvox even, hz 16-byte
// aligned; diag is written as float pairs when it is 8-byte aligned.
__global__ __launch_bounds__(kBlock) void zhz_hash_kernel(float *__restrict__ diag, const float4 *__restrict__ hz,
                                                           int64_t nvox, uint64_t seed, uint64_t pa, uint64_t pb,
                                                           int has_b, float w, int first) {
    __shared__ uint32_t words[kProbeWaves][2][4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t nchunk = (nvox + 8191) / 8192;
    const int64_t npair = nvox / 2;
    const bool pairs = ((uintptr_t)diag & 7u) == 0;
    for (int64_t c = (int64_t)blockIdx.x * kProbeWaves + wv; c < nchunk; c += (int64_t)gridDim.x * kProbeWaves) {
        probe_chunk_bits(words[wv], c, lane, seed, pa, pb, has_b);
        // eight pairs per step, their loads issued together (addresses
        // clamped into the volume; pairs past its end are not stored)
        constexpr int U = 8;
        for (int j0 = 0; j0 < 64; j0 += U) {
            float4 h[U];
            float2 d[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = min(c * 4096 + (int64_t)(j0 + u) * 64 + lane, npair - 1);
                h[u] = hz[q];
                d[u] = make_float2(0.f, 0.f);
                if (!first) d[u] = pairs ? reinterpret_cast<const float2 *>(diag)[q] : make_float2(diag[2 * q], diag[2 * q + 1]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = c * 4096 + (int64_t)(j0 + u) * 64 + lane;
                if (q >= npair) break;
                const float4 z = probe_pair_values(words[wv], j0 + u, lane, has_b);
                const float s0 = fmaf(z.x, h[u].x, z.y * h[u].y), s1 = fmaf(z.z, h[u].z, z.w * h[u].w);
                const float2 r = make_float2(fmaf(w, s0, d[u].x), fmaf(w, s1, d[u].y));
                if (pairs) {
                    reinterpret_cast<float2 *>(diag)[q] = r;
                } else {
                    diag[2 * q] = r.x;
                    diag[2 * q + 1] = r.y;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// Algorithm 1: running mean / exponential average of the diagonal,
// thresholding and the preconditioned step, with the two reductions the line
// search needs.
__global__ __launch_bounds__(kBlock) void precond_step_kernel(int64_t nvox, const float2 *__restrict__ v,
                                                               const float2 *__restrict__ g, float *D, float *D_avg,
                                                               const float *__restrict__ zHz, float wk_old, float wk_new,
                                                               float beta, float alpha, float eta, float2 *v_out,
                                                               float *Dhat_out, double *stats) {
    __shared__ double red[16];
    double s0 = 0.0, s1 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nvox; k += stride) {
        float dh = 1.0f;
        if (D) {
            float d = D[k];
            if (zHz) {
                const float da = fmaf(wk_old, D_avg[k], wk_new * zHz[k]);
                D_avg[k] = da;
                d = fmaf(beta, d, (1.0f - beta) * da);
                D[k] = d;
            }
            dh = fmaxf(fabsf(d), alpha);
        }
        if (Dhat_out) Dhat_out[k] = dh;
        if (!v_out) continue;  // the diagonal update alone
        const float2 gk = g[k], vk = v[k];
        // the hardware reciprocal (1 ulp); each voxel's terms of the two
        // sums are formed in float (a few ulp) and summed in double
        const float inv = __builtin_amdgcn_rcpf(dh);
        const float2 o = make_float2(vk.x - eta * gk.x * inv, vk.y - eta * gk.y * inv);
        v_out[k] = o;
        s0 += (double)(fmaf(gk.x, gk.x, gk.y * gk.y) * inv);
        s1 += (double)fmaf(o.x, o.x, o.y * o.y);
    }
    if (!v_out) return;
    const double t0 = block_sum(s0, red);
    const double t1 = block_sum(s1, red);
    if (threadIdx.x == 0) {
        atomicAdd(&stats[0], t0);
        atomicAdd(&stats[1], t1);
    }
}

// The same over pairs of voxels (complex arrays 16-byte aligned, real arrays
// 8-byte aligned, nvox even).
__global__ __launch_bounds__(kBlock) void precond_step2_kernel(int64_t npair, const float4 *__restrict__ v,
                                                                const float4 *__restrict__ g, float2 *D, float2 *D_avg,
                                                                const float2 *__restrict__ zHz, float wk_old,
                                                                float wk_new, float beta, float alpha, float eta,
                                                                float4 *v_out, float2 *Dhat_out, double *stats) {
    __shared__ double red[16];
    double s0 = 0.0, s1 = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < npair; k += stride) {
        float2 dh = make_float2(1.0f, 1.0f);
        if (D) {
            float2 d = D[k];
            if (zHz) {
                const float2 za = zHz[k], av = D_avg[k];
                const float2 da = make_float2(fmaf(wk_old, av.x, wk_new * za.x), fmaf(wk_old, av.y, wk_new * za.y));
                D_avg[k] = da;
                d = make_float2(fmaf(beta, d.x, (1.0f - beta) * da.x), fmaf(beta, d.y, (1.0f - beta) * da.y));
                D[k] = d;
            }
            dh = make_float2(fmaxf(fabsf(d.x), alpha), fmaxf(fabsf(d.y), alpha));
        }
        if (Dhat_out) Dhat_out[k] = dh;
        if (!v_out) continue;  // the diagonal update alone
        const float4 gk = g[k], vk = v[k];
        const float i0 = __builtin_amdgcn_rcpf(dh.x), i1 = __builtin_amdgcn_rcpf(dh.y);
        const float4 o = make_float4(vk.x - eta * gk.x * i0, vk.y - eta * gk.y * i0, vk.z - eta * gk.z * i1,
                                     vk.w - eta * gk.w * i1);
        v_out[k] = o;
        s0 += (double)(fmaf(gk.x, gk.x, gk.y * gk.y) * i0) + (double)(fmaf(gk.z, gk.z, gk.w * gk.w) * i1);
        s1 += (double)fmaf(o.x, o.x, o.y * o.y) + (double)fmaf(o.z, o.z, o.w * o.w);
    }
    if (!v_out) return;
    const double t0 = block_sum(s0, red);
    const double t1 = block_sum(s1, red);
    if (threadIdx.x == 0) {
        atomicAdd(&stats[0], t0);
        atomicAdd(&stats[1], t1);
    }
}

// sum_i C_i(R)^2 over the defocus values of all N images (one block,
// fixed-order reduction), then alpha = ratio * sum + lambda.
__global__ __launch_bounds__(kBlock) void ctf2_sum_kernel(Geom g, const float *__restrict__ defocus, int64_t n, int k2,
                                                           double ratio, float lam, double *alpha_out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const float c = ctf_value(g, g.ctf_a * (double)defocus[i], k2);
        s += (double)c * c;
    }
    const double t = block_sum(s, red);
    if (threadIdx.x == 0) *alpha_out = ratio * t + (double)lam;
}

// Per-shell sums of two volumes, shells round(|k|) = s < nsh (the Fourier
// shells of the shell correlation):
//   out[s] = sum Re(u conj v),  out[nsh + s] = sum |u|^2,  out[2 nsh + s] = sum |v|^2.
// One thread walks one row of kx, accumulating while the shell is unchanged;
// block partials in LDS, then one global double atomic per block and entry.
// out must be zero on entry.
__global__ __launch_bounds__(kBlock) void shell_sums_kernel(const float2 *__restrict__ u,
                                                            const float2 *__restrict__ v, int M, int nsh,
                                                            double *out) {
    extern __shared__ double part[];  // [3][nsh]
    for (int i = threadIdx.x; i < 3 * nsh; i += blockDim.x) part[i] = 0.0;
    __syncthreads();
    const int half = M / 2;
    const int64_t rows = (int64_t)M * M;
    for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < rows;
         row += (int64_t)gridDim.x * blockDim.x) {
        const int ky = (int)(row % M) - half, kz = (int)(row / M) - half;
        const int base2 = ky * ky + kz * kz;
        const float2 *pu = u + row * M, *pv = v + row * M;
        int cur = -1;
        double a = 0.0, b = 0.0, c = 0.0;
        for (int x = 0; x < M; ++x) {
            const int kx = x - half;
            const int k2 = base2 + kx * kx;
            // round(sqrt(k2)) with integers: s^2 - s < k2 <= s^2 + s
            int sh = (int)sqrtf((float)k2);
            while (sh * sh + sh < k2) ++sh;
            while (sh > 0 && sh * sh - sh >= k2) --sh;
            if (sh != cur) {
                if (cur >= 0 && cur < nsh) {
                    atomicAdd(&part[cur], a);
                    atomicAdd(&part[nsh + cur], b);
                    atomicAdd(&part[2 * nsh + cur], c);
                }
                cur = sh;
                a = b = c = 0.0;
            }
            const float2 U = pu[x], V = pv[x];
            a += (double)U.x * V.x + (double)U.y * V.y;
            b += (double)U.x * U.x + (double)U.y * U.y;
            c += (double)V.x * V.x + (double)V.y * V.y;
        }
        if (cur >= 0 && cur < nsh) {
            atomicAdd(&part[cur], a);
            atomicAdd(&part[nsh + cur], b);
            atomicAdd(&part[2 * nsh + cur], c);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * nsh; i += blockDim.x)
        if (part[i] != 0.0) atomicAdd(&out[i], part[i]);
}

hipError_t launch_shell_sums(const float2 *u, const float2 *v, int M, double *out, hipStream_t st) {
    const int nsh = M / 2;
    hipLaunchKernelGGL(fill_f32_kernel, dim3(stream_blocks(6 * nsh)), dim3(kBlock), 0, st, (float *)out,
                       (int64_t)6 * nsh, 0.0f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t rows = (int64_t)M * M;
    int64_t blocks = (rows + kBlock - 1) / kBlock;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(shell_sums_kernel, dim3((unsigned)blocks), dim3(kBlock), (size_t)3 * nsh * sizeof(double), st,
                       u, v, M, nsh, out);
    return hipGetLastError();
}

hipError_t launch_alpha(const Geom &g, const float *defocus, int64_t n, int k2, double ratio, float lam,
                        double *alpha_out, hipStream_t st) {
    hipLaunchKernelGGL(ctf2_sum_kernel, dim3(1), dim3(kBlock), 0, st, g, defocus, n, k2, ratio, lam, alpha_out);
    return hipGetLastError();
}

static inline bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

hipError_t launch_scaled_copy(float2 *out, const float2 *in, float lam, int64_t nvox, double *norm2, hipStream_t st) {
    if (nvox % 2 == 0 && aligned(out, 16) && aligned(in, 16)) {
        const int64_t np = nvox / 2;
        hipLaunchKernelGGL(scaled_copy2_kernel, dim3(norm2 ? reduce_blocks(np) : stream_blocks(np)), dim3(kBlock), 0,
                           st, (float4 *)out, (const float4 *)in, lam, np, norm2);
    } else {
        hipLaunchKernelGGL(scaled_copy_kernel, dim3(norm2 ? reduce_blocks(nvox) : stream_blocks(nvox)), dim3(kBlock),
                           0, st, out, in, lam, nvox, norm2);
    }
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int n, double v, hipStream_t st) {
    hipLaunchKernelGGL(fill_f64_kernel, dim3(1), dim3(64), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st) {
    hipLaunchKernelGGL(fill_f32_kernel, dim3(stream_blocks(n)), dim3(kBlock), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_finish_loss(double *loss_out, const double *data, const double *norm2, float scale, float lam,
                              hipStream_t st) {
    hipLaunchKernelGGL(finish_loss_kernel, dim3(1), dim3(64), 0, st, loss_out, data, norm2, scale, lam);
    return hipGetLastError();
}

hipError_t launch_rademacher(float *z, int64_t nvox, uint64_t seed, uint64_t probe, hipStream_t st) {
    hipLaunchKernelGGL(rademacher_kernel, dim3(stream_blocks((nvox + 3) / 4)), dim3(kBlock), 0, st, z, nvox, seed,
                       probe);
    return hipGetLastError();
}

hipError_t launch_probe_init(float2 *z, float2 *hz, int64_t nvox, uint64_t seed, uint64_t pa, uint64_t pb, int has_b,
                             float lam, hipStream_t st) {
    // z and hz live in the (256-byte aligned) workspace and nvox = M^3 is even
    if (nvox % 2 != 0 || !aligned(hz, 16) || !aligned(z, 16)) return hipErrorInvalidValue;
    // one wave per 8192 voxels, four waves per block
    int64_t blocks = ((nvox + 8191) / 8192 + kProbeWaves - 1) / kProbeWaves;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(probe_init_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, (float4 *)z, (float4 *)hz, nvox,
                       seed, pa, pb, has_b, lam);
    return hipGetLastError();
}

hipError_t launch_zhz_hash(float *diag, const float2 *hz, int64_t nvox, uint64_t seed, uint64_t pa, uint64_t pb,
                           int has_b, float w, bool first, hipStream_t st) {
    if (nvox % 2 != 0 || !aligned(hz, 16)) return hipErrorInvalidValue;
    int64_t blocks = ((nvox + 8191) / 8192 + kProbeWaves - 1) / kProbeWaves;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(zhz_hash_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, diag, (const float4 *)hz, nvox,
                       seed, pa, pb, has_b, w, first ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_precond_step(int64_t nvox, const float2 *v, const float2 *g, float *D, float *D_avg,
                               const float *zHz, int64_t k, float beta, float alpha, float eta, float2 *v_out,
                               float *Dhat_out, double *stats, hipStream_t st) {
    const float wk_old = k > 0 ? (float)((double)(k - 1) / (double)k) : 0.f;
    const float wk_new = k > 0 ? (float)(1.0 / (double)k) : 0.f;
    if (stats) {
        hipError_t e = launch_fill_f64(stats, 2, 0.0, st);
        if (e != hipSuccess) return e;
    }
    if (nvox % 2 == 0 && aligned(v, 16) && aligned(g, 16) && aligned(v_out, 16) && aligned(D, 8) &&
        aligned(D_avg, 8) && aligned(zHz, 8) && aligned(Dhat_out, 8)) {
        const int64_t np = nvox / 2;
        hipLaunchKernelGGL(precond_step2_kernel, dim3(reduce_blocks(np)), dim3(kBlock), 0, st, np, (const float4 *)v,
                           (const float4 *)g, (float2 *)D, (float2 *)D_avg, (const float2 *)zHz, wk_old, wk_new, beta,
                           alpha, eta, (float4 *)v_out, (float2 *)Dhat_out, stats);
    } else {
        hipLaunchKernelGGL(precond_step_kernel, dim3(reduce_blocks(nvox)), dim3(kBlock), 0, st, nvox, v, g, D, D_avg,
                           zHz, wk_old, wk_new, beta, alpha, eta, v_out, Dhat_out, stats);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Deterministic adjoint (fixed point, see FxScale)
// ---------------------------------------------------------------------------

// Largest |re| + |im| over n complex values, as float bits with the sign
// cleared: for non-negative floats the bit patterns order like the values,
// and a NaN orders above every finite value and infinity, so it is not lost.
__device__ __forceinline__ unsigned absmax_bits(const float2 *p, int64_t n, int64_t tid, int64_t stride) {
    unsigned m = 0u;
    if (((uintptr_t)p & 15u) == 0) {
        const float4 *q = (const float4 *)p;
        const int64_t np = n / 2;
        for (int64_t k = tid; k < np; k += stride) {
            const float4 v = q[k];
            m = max(m, __float_as_uint(fabsf(v.x) + fabsf(v.y)) & 0x7fffffffu);
            m = max(m, __float_as_uint(fabsf(v.z) + fabsf(v.w)) & 0x7fffffffu);
        }
        if ((n & 1) && tid == 0) {
            const float2 v = p[n - 1];
            m = max(m, __float_as_uint(fabsf(v.x) + fabsf(v.y)) & 0x7fffffffu);
        }
    } else {
        for (int64_t k = tid; k < n; k += stride) {
            const float2 v = p[k];
            m = max(m, __float_as_uint(fabsf(v.x) + fabsf(v.y)) & 0x7fffffffu);
        }
    }
    return m;
}

__device__ __forceinline__ void block_max_to(unsigned m, unsigned *lds /* >= 16 */, unsigned *dst) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, 64));
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned t = 0u;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = max(t, lds[i]);
        // most blocks cannot raise the maximum: skip their atomics
        if (t > __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMax(dst, t);
    }
    __syncthreads();
}

// *maxbits = bound of a[0..na) (a may be NULL; *maxbits zero on entry); the
// fixed-point volume fx[0..nvox) is zeroed.
__global__ __launch_bounds__(kBlock) void fx_prep_kernel(const float2 *a, int64_t na, unsigned *maxbits,
                                                          ulonglong2 *fx, int64_t nvox) {
    __shared__ unsigned red[16];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = tid; k < nvox; k += stride) fx[k] = make_ulonglong2(0ull, 0ull);
    if (a) block_max_to(absmax_bits(a, na, tid, stride), red, maxbits);
}

// *dst = max(*dst, bound of the disk pixels of n images [n][M][M]): the
// pixels the operators read.  One block per image; each wave takes every
// fourth disk row, four rows per step with all their loads issued before the
// first maximum (up to 16 loads in flight per lane).
// floor(sqrt(k2max - ky^2)) for |ky| <= floor(sqrt(k2max)) (k2max < 2^20:
// the float square root is off by at most one)
__device__ __forceinline__ int disk_half_width(int k2max, int ky) {
    const int rem = k2max - ky * ky;
    int kxm = (int)sqrtf((float)rem);
    kxm -= kxm * kxm > rem ? 1 : 0;
    kxm += (kxm + 1) * (kxm + 1) <= rem ? 1 : 0;
    return kxm;
}

__global__ __launch_bounds__(kBlock) void img_absmax_kernel(const float2 *__restrict__ img, int M, int half,
                                                             int k2max, int kymax, unsigned *dst) {
    __shared__ unsigned red[16];
    constexpr int NW = kBlock / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const float2 *im = img + (int64_t)blockIdx.x * M * M + (int64_t)half * M + half;  // pixel (0, 0)
    unsigned m = 0u;
    for (int ky0 = -kymax + wv; ky0 <= kymax; ky0 += 4 * NW) {
        // the loads are unconditional (addresses clamped into the row, rows
        // past the disk replaced by its last row) so that all sixteen are
        // issued before the first wait; the values outside are masked
        float2 v[4][4];
        bool in[4][4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int ky = ky0 + j * NW;
            const bool row_in = ky <= kymax;
            const int kyc = row_in ? ky : kymax;
            const int kxm = disk_half_width(k2max, kyc);
            const float2 *p = im + (int64_t)kyc * M;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int x = lane - kxm + 64 * k;
                v[j][k] = p[min(x, kxm)];
                in[j][k] = row_in && x <= kxm;
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const unsigned bv = __float_as_uint(fabsf(v[j][k].x) + fabsf(v[j][k].y)) & 0x7fffffffu;
                m = max(m, in[j][k] ? bv : 0u);
            }
    }
    // rows longer than 256 pixels (M > 512)
    for (int ky = -kymax + wv; ky <= kymax; ky += NW) {
        const int kxm = disk_half_width(k2max, ky);
        const float2 *p = im + (int64_t)ky * M;
        for (int x = lane - kxm + 256; x <= kxm; x += 64) {
            const float2 w = p[x];
            m = max(m, __float_as_uint(fabsf(w.x) + fabsf(w.y)) & 0x7fffffffu);
        }
    }
    block_max_to(m, red, dst);
}

// The same over 16-byte pairs of pixels (image base 16-byte aligned; M is
// even, so a pair never straddles two rows): blockIdx.y is the image,
// blockIdx.x a range of kImgPairs pairs, strided by the block size so that
// each wave load covers 1 KB of consecutive pixels.  A pair with no pixel in
// the disk loads the image's centre pair instead (always cached), so only
// lines that hold disk pixels are fetched while every load stays
// unconditional (all are issued before the first wait).
constexpr int kImgPairs = 8;  // pairs per thread
__global__ __launch_bounds__(kBlock) void img_absmax2_kernel(const float4 *__restrict__ img, int M, int half,
                                                              int k2max, int pairs, unsigned *dst) {
    __shared__ unsigned red[16];
    const float4 *im = img + (int64_t)blockIdx.y * pairs;
    const float invM = 1.0f / (float)M;
    const int centre = (half * M + half) >> 1;
    float4 v[kImgPairs];
    int inside[kImgPairs];  // bit 0: first pixel, bit 1: second
#pragma unroll
    for (int u = 0; u < kImgPairs; ++u) {
        const int q = (blockIdx.x * kImgPairs + u) * kBlock + threadIdx.x;
        const int p = 2 * q;  // first pixel (p < M^2 <= 2^20: the float quotient is off by at most one)
        int y = (int)((float)p * invM);
        y += (y + 1) * M <= p ? 1 : 0;
        y -= y * M > p ? 1 : 0;
        const int kx = p - y * M - half, ky = y - half;
        const int r2 = kx * kx + ky * ky;
        const int in = (q < pairs ? 1 : 0) * ((r2 <= k2max ? 1 : 0) | (r2 + 2 * kx + 1 <= k2max ? 2 : 0));
        inside[u] = in;
        v[u] = im[in ? q : centre];
    }
    unsigned m = 0u;
#pragma unroll
    for (int u = 0; u < kImgPairs; ++u) {
        const unsigned b0 = __float_as_uint(fabsf(v[u].x) + fabsf(v[u].y)) & 0x7fffffffu;
        const unsigned b1 = __float_as_uint(fabsf(v[u].z) + fabsf(v[u].w)) & 0x7fffffffu;
        m = max(m, (inside[u] & 1) ? b0 : 0u);
        m = max(m, (inside[u] & 2) ? b1 : 0u);
    }
    block_max_to(m, red, dst);
}

// out += fx / S per component, in double precision with one rounding to
// float; every voxel becomes NaN when an input was not finite.
__global__ __launch_bounds__(kBlock) void fx_finish_kernel(float2 *__restrict__ out,
                                                            const ulonglong2 *__restrict__ fx, int64_t nvox,
                                                            const unsigned *maxbits, float scale, int64_t n) {
    const FxScale f = fx_scale(maxbits, scale, n);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nvox; k += stride) {
        const ulonglong2 q = fx[k];
        float2 o = out[k];
        if (f.ok) {
            o.x = (float)fma((double)(long long)q.x, f.invS, (double)o.x);
            o.y = (float)fma((double)(long long)q.y, f.invS, (double)o.y);
        } else {
            o = make_float2(__builtin_nanf(""), __builtin_nanf(""));
        }
        out[k] = o;
    }
}

hipError_t launch_fx_prep(const float2 *a, int64_t na, unsigned *maxbits, unsigned long long *fx, int64_t nvox,
                          hipStream_t st) {
    hipError_t e = launch_fill_f32((float *)maxbits, 2, 0.0f, st);  // zero bits
    if (e != hipSuccess) return e;
    const int64_t units = na > nvox ? na : nvox;
    if (units == 0) return hipSuccess;
    hipLaunchKernelGGL(fx_prep_kernel, dim3(reduce_blocks(units)), dim3(kBlock), 0, st, a, na, maxbits,
                       (ulonglong2 *)fx, nvox);
    return hipGetLastError();
}

hipError_t launch_img_absmax(const Geom &g, const float2 *img, int64_t n, unsigned *dst, hipStream_t st) {
    int kymax = (int)sqrt((double)g.k2max);
    while ((kymax + 1) * (kymax + 1) <= g.k2max) ++kymax;
    while (kymax > 0 && kymax * kymax > g.k2max) --kymax;
    if (aligned(img, 16)) {
        const int pairs = g.M * g.M / 2;
        const unsigned bx = (unsigned)((pairs + kImgPairs * kBlock - 1) / (kImgPairs * kBlock));
        for (int64_t i0 = 0; i0 < n; i0 += 65535) {
            const int64_t cnt = n - i0 < 65535 ? n - i0 : 65535;
            hipLaunchKernelGGL(img_absmax2_kernel, dim3(bx, (unsigned)cnt), dim3(kBlock), 0, st,
                               (const float4 *)(img + i0 * (int64_t)g.M * g.M), g.M, g.half, g.k2max, pairs, dst);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    for (int64_t i0 = 0; i0 < n; i0 += (int64_t)1 << 30) {  // one block per image
        const int64_t cnt = n - i0 < ((int64_t)1 << 30) ? n - i0 : ((int64_t)1 << 30);
        hipLaunchKernelGGL(img_absmax_kernel, dim3((unsigned)cnt), dim3(kBlock), 0, st,
                           img + i0 * (int64_t)g.M * g.M, g.M, g.half, g.k2max, kymax, dst);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fx_finish(float2 *out, const unsigned long long *fx, int64_t nvox, const unsigned *maxbits,
                            float scale, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(fx_finish_kernel, dim3(stream_blocks(nvox)), dim3(kBlock), 0, st, out, (const ulonglong2 *)fx,
                       nvox, maxbits, scale, n);
    return hipGetLastError();
}

}  // namespace csg
