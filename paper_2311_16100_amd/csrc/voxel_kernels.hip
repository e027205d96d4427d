// voxel_kernels.hip -- voxel-parallel ("owner computes") adjoint kernels.
//
// One thread owns one voxel of an 8 x 8 x 4 brick and sums every
// contribution to that voxel itself, image by image in index order and, per
// image, pixel by pixel in a fixed order; the result is therefore bitwise
// reproducible, and no atomic operation is used.  A block first culls the
// images whose slice plane cannot reach its brick, keeping the survivors in
// index order in LDS.  For a surviving image, the pixels whose trilinear cell
// has the voxel q as a corner satisfy |p - q|_inf < 1 with p on the plane, so
// they lie within distance sqrt(3 - h^2) of the projection of q onto the
// plane (h = distance of q to the plane); those few lattice candidates are
// enumerated and each is confirmed with exactly the same cell computation the
// pixel kernels use, so both families agree on every weight bit for bit.
//
// Modes:
//   kVoxBackproject  accum[q] += scale * sum_ij w_ijq C_ij^p img_ij
//   kVoxFeatures     ctf2[q] += sum_ij w_ijq C_ij^2 ; cover[q] += #{i : some w_ijq > 0}
#include "csg_device.h"
#include "csg_internal.h"

namespace csg {

enum VoxMode { kVoxBackproject = 0, kVoxFeatures = 1 };

constexpr int BX = 8, BY = 8, BZ = 4;  // brick = one voxel per thread
static_assert(BX * BY * BZ == kBlock, "brick must match the block size");

struct VoxArgs {
    Geom g;
    const float *rot;
    const float *defocus;
    const float *shift;  // [n][2] in-plane shifts or NULL (backprojection)
    int64_t n;
    const float2 *img;
    float2 *accum;
    float *ctf2;
    float *cover;
    float scale;
    int ctf_power;
    int nbx, nby, nbz;  // bricks per axis
};

struct ImgEntry {
    float e1[3], e2[3], e3[3];
    float l1;  // |e3|_1, the reach of the plane into the L-infinity unit ball
    double a;  // CTF defocus term of the image
    int64_t idx;
    float sx, sy;  // in-plane shift (pixels)
};

template <int MODE, int INTERP>
__global__ __launch_bounds__(kBlock) void voxel_kernel(VoxArgs a) {
    __shared__ ImgEntry list[kBlock];
    __shared__ int wave_count[kBlock / 64];
    __shared__ int list_len;

    const Geom &g = a.g;
    const int M = g.M;
    const int bid = blockIdx.x;
    const int bxi = bid % a.nbx, byi = (bid / a.nbx) % a.nby, bzi = bid / (a.nbx * a.nby);
    const int tx = threadIdx.x % BX, ty = (threadIdx.x / BX) % BY, tz = threadIdx.x / (BX * BY);
    const int qx = bxi * BX + tx, qy = byi * BY + ty, qz = bzi * BZ + tz;
    const bool owner = qx < M && qy < M && qz < M;
    // centred coordinates of the voxel and of the culling box
    // [b0 - 1, b0 + S) per axis (the cells that have a corner in the brick)
    const float cx = (float)(qx - g.half), cy = (float)(qy - g.half), cz = (float)(qz - g.half);
    const float bc[3] = {(float)(bxi * BX - g.half) + 0.5f * (BX - 1), (float)(byi * BY - g.half) + 0.5f * (BY - 1),
                         (float)(bzi * BZ - g.half) + 0.5f * (BZ - 1)};
    const float bh[3] = {0.5f * (BX + 1), 0.5f * (BY + 1), 0.5f * (BZ + 1)};

    float accx = 0.f, accy = 0.f, f2 = 0.f, ncov = 0.f;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;

    for (int64_t base = 0; base < a.n; base += kBlock) {
        // ---- cull: images whose plane meets the brick's box, kept in order
        const int64_t ii = base + threadIdx.x;
        bool keep = false;
        ImgEntry e;
        if (ii < a.n) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                e.e1[d] = a.rot[ii * 9 + d];
                e.e2[d] = a.rot[ii * 9 + 3 + d];
                e.e3[d] = a.rot[ii * 9 + 6 + d];
            }
            e.l1 = fabsf(e.e3[0]) + fabsf(e.e3[1]) + fabsf(e.e3[2]);
            const float h = e.e3[0] * bc[0] + e.e3[1] * bc[1] + e.e3[2] * bc[2];
            const float reach = fabsf(e.e3[0]) * bh[0] + fabsf(e.e3[1]) * bh[1] + fabsf(e.e3[2]) * bh[2];
            keep = fabsf(h) <= reach + 1e-3f;
            e.a = g.ctf_a * (double)a.defocus[ii];
            e.idx = ii;
            e.sx = a.shift ? a.shift[2 * ii] : 0.f;
            e.sy = a.shift ? a.shift[2 * ii + 1] : 0.f;
        }
        const uint64_t mask = __ballot(keep);
        if (lane == 0) wave_count[wv] = __popcll(mask);
        __syncthreads();
        int off = 0;
        for (int w = 0; w < wv; ++w) off += wave_count[w];
        if (keep) list[off + __popcll(mask & ((1ull << lane) - 1ull))] = e;
        if (threadIdx.x == 0) {
            int t = 0;
            for (int w = 0; w < kBlock / 64; ++w) t += wave_count[w];
            list_len = t;
        }
        __syncthreads();
        const int len = list_len;

        // ---- gather the contributions of each surviving image, in order
        for (int l = 0; l < len; ++l) {
            const ImgEntry &E = list[l];
            if (!owner) continue;
            const float h = E.e3[0] * cx + E.e3[1] * cy + E.e3[2] * cz;
            const float reach = INTERP == 0 ? 0.5f * E.l1 : E.l1;
            if (!(fabsf(h) < reach + 1e-4f)) continue;
            const float u0 = E.e1[0] * cx + E.e1[1] * cy + E.e1[2] * cz;
            const float v0 = E.e2[0] * cx + E.e2[1] * cy + E.e2[2] * cz;
            const float r2 = (INTERP == 0 ? 0.75f : 3.0f) - h * h + 1e-3f;
            const float r = sqrtf(fmaxf(r2, 0.f));
            // candidate pixels, clamped to the image so that no input can
            // make these loops long (r <= sqrt(3): at most 4 x 4 candidates)
            const float lo_k = (float)(-g.half), hi_k = (float)(g.half - 1);
            const int kx0 = (int)fmaxf(ceilf(u0 - r), lo_k), kx1 = (int)fminf(floorf(u0 + r), hi_k);
            const int ky0 = (int)fmaxf(ceilf(v0 - r), lo_k), ky1 = (int)fminf(floorf(v0 + r), hi_k);
            bool hit = false;
            for (int ky = ky0; ky <= ky1; ++ky) {
                for (int kx = kx0; kx <= kx1; ++kx) {
                    const float du = (float)kx - u0, dv = (float)ky - v0;
                    if (du * du + dv * dv > r2) continue;
                    const int k2 = kx * kx + ky * ky;
                    if (k2 > g.k2max) continue;
                    float w;
                    if (INTERP == 0) {
                        int q[3];
                        sample_nearest(g, E.e1, E.e2, kx, ky, q);
                        if (q[0] != qx || q[1] != qy || q[2] != qz) continue;
                        w = 1.0f;
                    } else {
                        const Cell c = sample_cell(g, E.e1, E.e2, kx, ky);
                        const int dx = qx - c.f[0], dy = qy - c.f[1], dz = qz - c.f[2];
                        if ((unsigned)dx > 1u || (unsigned)dy > 1u || (unsigned)dz > 1u) continue;
                        w = (dx ? c.t[0] : 1.0f - c.t[0]) * (dy ? c.t[1] : 1.0f - c.t[1]) *
                            (dz ? c.t[2] : 1.0f - c.t[2]);
                    }
                    const float C = ctf_value(g, E.a, k2);
                    if (MODE == kVoxBackproject) {
                        const int64_t j = (E.idx * M + (ky + g.half)) * (int64_t)M + (kx + g.half);
                        float2 x = a.img[j];
                        if (a.shift) {
                            // conj(T) of the in-plane shift (exact zero shift: T = 1)
                            const float sh[2] = {E.sx, E.sy};
                            x = cmul_conj(x, shift_phase(sh, 0, M, kx, ky));
                        }
                        const float f = a.scale * ctf_pow(C, a.ctf_power);
                        const float fx = f * x.x, fy = f * x.y;
                        accx = fmaf(w, fx, accx);
                        accy = fmaf(w, fy, accy);
                    } else {
                        f2 = fmaf(w, C * C, f2);
                        hit = hit || w > 0.f;
                    }
                }
            }
            if (MODE == kVoxFeatures && hit) ncov += 1.0f;  // distinct images
        }
        __syncthreads();  // list is rewritten by the next chunk
    }
    if (!owner) return;
    const int64_t q = ((int64_t)qz * M + qy) * M + qx;
    if (MODE == kVoxBackproject) {
        float2 o = a.accum[q];
        o.x += accx;
        o.y += accy;
        a.accum[q] = o;
    } else {
        a.ctf2[q] += f2;
        a.cover[q] += ncov;
    }
}

static VoxArgs vox_grid(VoxArgs a, dim3 &grid) {
    a.nbx = (a.g.M + BX - 1) / BX;
    a.nby = (a.g.M + BY - 1) / BY;
    a.nbz = (a.g.M + BZ - 1) / BZ;
    grid = dim3((unsigned)(a.nbx * a.nby * a.nbz));
    return a;
}

template <int MODE>
static hipError_t launch_vox(const VoxArgs &a0, hipStream_t st) {
    dim3 grid;
    VoxArgs a = vox_grid(a0, grid);
    if (a.g.interp == 0)
        hipLaunchKernelGGL((voxel_kernel<MODE, 0>), grid, dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL((voxel_kernel<MODE, 1>), grid, dim3(kBlock), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_backproject_owner(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                    int64_t n, const float2 *img, int ctf_power, float scale, float2 *accum,
                                    hipStream_t st) {
    VoxArgs a{};
    a.g = g; a.rot = rot; a.defocus = defocus; a.shift = shift; a.n = n;
    a.img = img; a.accum = accum; a.ctf_power = ctf_power; a.scale = scale;
    return launch_vox<kVoxBackproject>(a, st);
}

hipError_t launch_features(const Geom &g, const float *rot, const float *defocus, int64_t n, float *ctf2,
                           float *cover, hipStream_t st) {
    VoxArgs a{};
    a.g = g; a.rot = rot; a.defocus = defocus; a.n = n;
    a.ctf2 = ctf2; a.cover = cover;
    return launch_vox<kVoxFeatures>(a, st);
}

}  // namespace csg
