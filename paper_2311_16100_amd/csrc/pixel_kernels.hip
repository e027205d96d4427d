// pixel_kernels.hip -- pixel-parallel kernels: one thread per image pixel.
//
// Each block owns 256 consecutive pixels of one image (for M = 256, one
// image row), so a wavefront reads and writes 64 adjacent pixels of a row
// with coalesced accesses, and the rotation and defocus of the image are
// uniform over the block.  The sample point and the CTF are computed in
// registers.  Block ids are remapped so that each XCD processes a contiguous
// range of images: adjacent rows of an image reuse the same volume cache
// lines, and that reuse stays inside one XCD's L2.
//
// Modes (template parameter):
//   kProject     y = C P v (optionally - x), written and/or squared into a loss
//   kBackproject accum += scale C^p x, scattered with float atomics
//   kGradient    r = C P v - x; loss += |r|^2/2; accum += scale C r
//   kHvp         accum += scale C^2 P z
//   kSqDiag      diag  += scale C^2 w^2 (real, exact Hessian diagonal)
#include "csg_device.h"
#include "csg_internal.h"

namespace csg {

enum PixelMode { kProject = 0, kBackproject = 1, kGradient = 2, kHvp = 3, kSqDiag = 4 };

struct PixelArgs {
    Geom g;
    const float *rot;
    const float *defocus;
    const float *shift;  // [n][2] in-plane shifts or NULL
    int64_t n;
    const float2 *src;   // gathered volume (project / gradient / hvp)
    const float2 *img;   // image stack read (subtract, backproject input, data x)
    float2 *out;         // projected images (project)
    float2 *accum;       // scatter target (backproject / gradient / hvp)
    float *accum_real;   // scatter target (sq diag)
    double *loss;        // += 1/2 sum |r|^2 (project / gradient)
    float scale;
    int ctf_power;
    int chunks;          // blocks per image
    int64_t nblocks;     // n * chunks
    int64_t nblocks_pad; // rounded up to a multiple of 8
};

__device__ __forceinline__ void atomic_add_c(float2 *p, float2 v) {
    atomicAdd(&p->x, v.x);
    atomicAdd(&p->y, v.y);
}

template <int MODE, int INTERP>
__global__ __launch_bounds__(kBlock) void pixel_kernel(PixelArgs a) {
    __shared__ double red[16];
    const int64_t L = xcd_logical_block(blockIdx.x, a.nblocks, a.nblocks_pad);
    if (L < 0) return;  // whole padding block: uniform exit before any barrier
    const int64_t i = L / a.chunks;
    const int chunk = (int)(L - i * a.chunks);
    const Geom &g = a.g;
    const int M = g.M;
    const int pix = chunk * kBlock + threadIdx.x;
    const bool valid = pix < M * M;
    const int ky = pix / M - g.half;
    const int kx = pix % M - g.half;
    const int k2 = kx * kx + ky * ky;
    const bool in_disk = valid && k2 <= g.k2max;
    const int64_t j = i * (int64_t)M * M + pix;

    float e1[3], e2[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        e1[d] = a.rot[i * 9 + d];
        e2[d] = a.rot[i * 9 + 3 + d];
    }
    const double a_i = g.ctf_a * (double)a.defocus[i];

    double lsum = 0.0;
    if (in_disk) {
        const float C = ctf_value(g, a_i, k2);
        Stencil s;
        if (INTERP == 0) {
            int q[3];
            sample_nearest(g, e1, e2, kx, ky, q);
            const bool ok = in_grid(q[0], M) && in_grid(q[1], M) && in_grid(q[2], M);
            s.idx[0] = ok ? (q[2] * M + q[1]) * M + q[0] : 0;
            s.w[0] = ok ? 1.0f : 0.0f;
        } else {
            s = make_stencil(g, e1, e2, kx, ky);
        }
        constexpr int NC = INTERP == 0 ? 1 : 8;
        float2 acc = make_float2(0.f, 0.f);
        if (MODE == kProject || MODE == kGradient || MODE == kHvp) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const float2 v = a.src[s.idx[c]];
                acc.x = fmaf(s.w[c], v.x, acc.x);
                acc.y = fmaf(s.w[c], v.y, acc.y);
            }
        }
        // in-plane shift: T on the forward value, conj(T) on the adjoint input
        float2 T = make_float2(1.f, 0.f);
        if (a.shift && (MODE == kProject || MODE == kBackproject || MODE == kGradient))
            T = shift_phase(a.shift, i, M, kx, ky);
        if (MODE == kProject || MODE == kGradient) acc = cmul(acc, T);
        float2 val = make_float2(0.f, 0.f);
        if (MODE == kProject) {
            float2 y = make_float2(C * acc.x, C * acc.y);
            if (a.img) {
                const float2 x = a.img[j];
                y.x -= x.x;
                y.y -= x.y;
            }
            if (a.out) a.out[j] = y;
            lsum = 0.5 * ((double)y.x * y.x + (double)y.y * y.y);
        } else if (MODE == kBackproject) {
            const float2 x = cmul_conj(a.img[j], T);
            const float f = a.scale * ctf_pow(C, a.ctf_power);
            val = make_float2(f * x.x, f * x.y);
        } else if (MODE == kGradient) {
            const float2 x = a.img[j];
            const float2 r = make_float2(fmaf(C, acc.x, -x.x), fmaf(C, acc.y, -x.y));
            lsum = 0.5 * ((double)r.x * r.x + (double)r.y * r.y);
            const float f = a.scale * C;
            const float2 rt = cmul_conj(r, T);
            val = make_float2(f * rt.x, f * rt.y);
        } else if (MODE == kHvp) {
            const float f = a.scale * C * C;
            val = make_float2(f * acc.x, f * acc.y);
        }
        if (MODE == kBackproject || MODE == kGradient || MODE == kHvp) {
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                atomic_add_c(&a.accum[s.idx[c]], make_float2(s.w[c] * val.x, s.w[c] * val.y));
            }
        } else if (MODE == kSqDiag) {
            const float f = a.scale * C * C;
#pragma unroll
            for (int c = 0; c < NC; ++c) atomicAdd(&a.accum_real[s.idx[c]], f * s.w[c] * s.w[c]);
        }
    } else if (MODE == kProject && valid && a.out) {
        a.out[j] = make_float2(0.f, 0.f);
    }
    if ((MODE == kProject || MODE == kGradient) && a.loss) {
        const double t = block_sum(lsum, red);
        if (threadIdx.x == 0 && t != 0.0) atomicAdd(a.loss, t);
    }
}

template <int MODE>
static hipError_t launch_mode(const PixelArgs &a0, hipStream_t st) {
    PixelArgs a = a0;
    const int64_t pix = (int64_t)a.g.M * a.g.M;
    a.chunks = (int)((pix + kBlock - 1) / kBlock);
    a.nblocks = a.n * a.chunks;
    a.nblocks_pad = (a.nblocks + 7) / 8 * 8;
    if (a.nblocks == 0) return hipSuccess;
    if (a.nblocks_pad > 0x7FFFFFFFLL) return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)a.nblocks_pad), block(kBlock);
    if (a.g.interp == 0)
        hipLaunchKernelGGL((pixel_kernel<MODE, 0>), grid, block, 0, st, a);
    else
        hipLaunchKernelGGL((pixel_kernel<MODE, 1>), grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_project(const Geom &g, const float *rot, const float *defocus, const float *shift, int64_t n,
                          const float2 *vol, const float2 *subtract, float2 *out, double *loss, hipStream_t st) {
    PixelArgs a{};
    a.g = g; a.rot = rot; a.defocus = defocus; a.shift = shift; a.n = n;
    a.src = vol; a.img = subtract; a.out = out; a.loss = loss;
    return launch_mode<kProject>(a, st);
}

hipError_t launch_backproject_atomic(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                     int64_t n, const float2 *img, int ctf_power, float scale, float2 *accum,
                                     hipStream_t st) {
    PixelArgs a{};
    a.g = g; a.rot = rot; a.defocus = defocus; a.shift = shift; a.n = n;
    a.img = img; a.accum = accum; a.ctf_power = ctf_power; a.scale = scale;
    return launch_mode<kBackproject>(a, st);
}

hipError_t launch_gradient_atomic(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                  int64_t n, const float2 *vol, const float2 *x, float scale, float2 *accum,
                                  double *loss, hipStream_t st) {
    PixelArgs a{};
    a.g = g; a.rot = rot; a.defocus = defocus; a.shift = shift; a.n = n;
    a.src = vol; a.img = x; a.accum = accum; a.scale = scale; a.loss = loss;
    return launch_mode<kGradient>(a, st);
}

hipError_t launch_hvp_atomic(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *z,
                             float scale, float2 *accum, hipStream_t st) {
    PixelArgs a{};
    a.g = g; a.rot = rot; a.defocus = defocus; a.n = n;
    a.src = z; a.accum = accum; a.scale = scale;
    return launch_mode<kHvp>(a, st);
}

hipError_t launch_sq_diag(const Geom &g, const float *rot, const float *defocus, int64_t n, float scale,
                          float *accum, hipStream_t st) {
    PixelArgs a{};
    a.g = g; a.rot = rot; a.defocus = defocus; a.n = n;
    a.accum_real = accum; a.scale = scale;
    return launch_mode<kSqDiag>(a, st);
}

}  // namespace csg
