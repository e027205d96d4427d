// brick_kernels.hip -- brick-binned forward projection and adjoint.
//
// The volume is cut into 12^3 bricks.  A cull kernel lists, per brick and in
// image order, the images whose slice plane reaches the brick.  A work item is
// one brick and up to 256 of its images; its block
//   - stages the brick plus a one-voxel halo of the gathered volume in LDS
//     (14^3 complex values), so every trilinear gather is 8 LDS reads;
//   - accumulates the adjoint into an LDS copy of the brick with double-
//     precision LDS atomics, and writes it to HBM once per voxel at the end (a
//     plain read-modify-write when the brick has a single work item, global
//     atomics only for the few central bricks that more than 256 images
//     cross).  On gfx950 the LDS double atomic add sustains about 20x the lane
//     rate of the single-precision one, so the wider accumulator is also the
//     faster one.
// The pixels of an image that matter for a brick are found row by row: for
// image row ky the sample points form a line, and the pixels whose cell
// reaches the brick's box form an interval of kx, computed by clipping the
// line against the box.  Eight images x 32 rows fill the 256 lanes; a block
// scan turns the row intervals into one flat pixel range that the lanes walk
// together, so neighbouring lanes take neighbouring pixels of a row (coalesced
// image reads and writes).
//
// A pixel is "touching" a brick when one of its eight cell corners lies in
// the brick, and "owned" by the brick that contains its base corner
// floor(g).  The adjoint adds, for every touching pixel, the corners inside
// the brick -- so each (pixel, corner) contribution is added exactly once over
// all bricks; forward outputs and loss terms are produced by the owner only.
//
// Modes:
//   kBProject      out = C P v (- x) for owned pixels; loss
//   kBBackproject  accum += scale C^p img
//   kBGradient     r = C P v - x; loss (owner); accum += scale C r
//   kBHvp          accum += scale C^2 P z
//   kBFeatures     accum += (C^2, 1) w: the CTF^2 weight and the plain weight
//                  sum of every voxel (no image is read)
//   kBSqDiag       diag += scale C^2 w^2: the exact diagonal of the data
//                  Hessian (real accumulator; no image is read)
#include "csg_device.h"
#include "csg_internal.h"

namespace csg {

#ifndef CSG_BRICK_SIDE
#define CSG_BRICK_SIDE 12
#endif
constexpr int BS = CSG_BRICK_SIDE;  // brick side
constexpr int BH = BS + 2;       // staged side: one halo voxel below and above
// LDS strides are odd (in elements) so that lanes stepping along any axis of
// the brick fall into different banks.
constexpr int AR = BS + 1;       // accumulator row stride
constexpr int AP = AR * AR;      // accumulator plane stride (289)
constexpr int VR = BH + 1;       // staged-volume row stride (19)
constexpr int VP = VR * VR;      // staged-volume plane stride (361)
constexpr int kBT = 512;         // threads per brick block (8 waves)
constexpr int ROWS = 32;         // row slots per image (a brick spans <= 24 rows)
constexpr int GIMG = kBT / ROWS; // images per group
constexpr int CHUNK_ADJ = 256;   // images per work item of the adjoint modes
constexpr int CHUNK_FWD = 64;    // images per work item of the forward mode (no flush)
constexpr float kClipEps = 1e-2f;

enum BrickMode { kBProject = 0, kBBackproject = 1, kBGradient = 2, kBHvp = 3, kBFeatures = 4, kBSqDiag = 5 };

struct BrickArgs {
    Geom g;
    const float *rot;
    const float *defocus;
    int64_t n;          // images of this sub-batch
    const float2 *src;  // gathered volume
    const float2 *img;  // x (project subtract / gradient) or adjoint input
    float2 *out;        // projected images
    float2 *accum;      // adjoint target
    float *accum_real;  // real target (squared-weight diagonal)
    double *loss;
    float scale;
    int ctf_power;
    const int *counts;  // [nb]
    const int *lists;   // [nb][stride]
    int stride;
    int nbx, nb;
    int nchunks;        // work items per brick at most
};

__device__ __forceinline__ void brick_origin(int b, int nbx, int o[3]) {
    o[0] = (b % nbx) * BS;
    o[1] = ((b / nbx) % nbx) * BS;
    o[2] = (b / (nbx * nbx)) * BS;
}

// ---------------------------------------------------------------------------
// Cull: lists[b] = images whose plane meets the box of cells touching brick b
// (grid coordinates [b0 - 1, b0 + BS]^3), in increasing image order.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void brick_cull_kernel(Geom g, const float *rot, int64_t n, int nbx,
                                                             int *counts, int *lists, int stride) {
    __shared__ int wave_count[kBlock / 64];
    const int b = blockIdx.x;
    int o[3];
    brick_origin(b, nbx, o);
    float c[3], hw[3];
    float dist2 = 0.f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float lo = (float)(o[d] - 1 - g.half), hi = (float)(o[d] + BS - g.half);
        c[d] = 0.5f * (lo + hi);
        hw[d] = 0.5f * (hi - lo);
        const float near = fmaxf(fmaxf(lo, -hi), 0.f);  // distance of the box to the origin along d
        dist2 += near * near;
    }
    // sample points lie within |p| <= r_max; the box must come that close
    const float rmax = sqrtf((float)g.k2max) + 2.0f;
    const bool reachable = dist2 <= rmax * rmax;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int total = 0;
    for (int64_t base = 0; base < n; base += kBlock) {
        const int64_t i = base + threadIdx.x;
        bool keep = false;
        if (reachable && i < n) {
            const float e0 = rot[i * 9 + 6], e1 = rot[i * 9 + 7], e2 = rot[i * 9 + 8];
            const float h = e0 * c[0] + e1 * c[1] + e2 * c[2];
            const float reach = fabsf(e0) * hw[0] + fabsf(e1) * hw[1] + fabsf(e2) * hw[2];
            keep = fabsf(h) <= reach + kClipEps;
        }
        const uint64_t mask = __ballot(keep);
        if (lane == 0) wave_count[wv] = __popcll(mask);
        __syncthreads();
        int off = total;
        for (int w = 0; w < wv; ++w) off += wave_count[w];
        if (keep) lists[(int64_t)b * stride + off + __popcll(mask & ((1ull << lane) - 1ull))] = (int)i;
        for (int w = 0; w < kBlock / 64; ++w) total += wave_count[w];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[b] = total;
}

// Exclusive scan of one int per thread over the block; returns the prefix and
// writes the total to *total.
__device__ __forceinline__ int block_exclusive_scan(int v, int *wave_sums, int *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    constexpr int NW = kBT / 64;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wave_sums[wv] = x;
    __syncthreads();
    int base = 0, tot = 0;
    for (int w = 0; w < NW; ++w) {
        if (w < wv) base += wave_sums[w];
        tot += wave_sums[w];
    }
    *total = tot;
    return base + x - v;
}

// Interval of kx for which the sample point of row ky lies in the box
// [lo, hi) (grid coordinates) on every axis, widened by kClipEps.
__device__ __forceinline__ void clip_row(const float e1[3], const float e2[3], float half, int ky, const float lo[3],
                                         const float hi[3], int &kx0, int &kx1) {
    float a = -1e30f, b = 1e30f;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float c = fmaf((float)ky, e2[d], half);
        if (fabsf(e1[d]) < 1e-7f) {
            if (c < lo[d] - kClipEps || c >= hi[d] + kClipEps) {
                a = 1e30f;
                b = -1e30f;
            }
        } else {
            const float inv = 1.0f / e1[d];
            const float t0 = (lo[d] - c) * inv, t1 = (hi[d] - c) * inv;
            a = fmaxf(a, fminf(t0, t1));
            b = fminf(b, fmaxf(t0, t1));
        }
    }
    kx0 = (int)fmaxf(ceilf(a - kClipEps), -1e6f);
    kx1 = (int)fminf(floorf(b + kClipEps), 1e6f);
}

// Per-image constants of a group, kept in LDS in double precision so the
// pixel loop needs no conversions: the rows of R and the folded CTF term.
struct ImgSlot {
    double e1[3];
    double e2[3];
    double ctfA;  // (lambda df / 2) / (M pixel)^2: chi / 2pi = k2 (ctfA - ctfB k2)
    double pad;
};

constexpr int PIXCAP = 4096;  // pixels per window of the pixel -> segment table

template <int MODE>
__global__ __launch_bounds__(kBT) void brick_kernel(BrickArgs a) {
    constexpr bool GATHER = MODE == kBProject || MODE == kBGradient || MODE == kBHvp;
    constexpr bool SCATTER = MODE != kBProject;
    constexpr bool OWNER_ONLY = MODE == kBProject;
    constexpr int CHUNK = OWNER_ONLY ? CHUNK_FWD : CHUNK_ADJ;
    __shared__ float2 vh[GATHER ? BH * VP : 1];
    __shared__ double acc_re[SCATTER ? BS * AP : 1];
    __shared__ double acc_im[SCATTER ? BS * AP : 1];
    // segment record: x = first flat pixel, y = kx of that pixel,
    // z = (ky + 512) | image slot << 16, w = pixel index of (kx = 0, ky)
    __shared__ int4 seg[kBT];
    __shared__ unsigned short pix2seg[PIXCAP];
    __shared__ ImgSlot slot[GIMG];
    __shared__ int wave_sums[kBT / 64];
    __shared__ double red[16];

    const Geom &g = a.g;
    const int M = g.M;
    // highest chunk index first: the extra work items of the heavily crossed
    // central bricks start before the single items of the outer bricks
    const int brick = blockIdx.x % a.nb;
    const int chunk = a.nchunks - 1 - (int)(blockIdx.x / a.nb);
    const int count = a.counts[brick];
    const int first = chunk * CHUNK;
    if (first >= count) return;  // uniform: no work item here
    const int n_img = min(CHUNK, count - first);
    const bool single = count <= CHUNK;
    int o[3];
    brick_origin(brick, a.nbx, o);

    if (GATHER) {
        for (int t = threadIdx.x; t < BH * BH * BH; t += kBT) {
            const int hx = t % BH, hy = (t / BH) % BH, hz = t / (BH * BH);
            const int qx = o[0] - 1 + hx, qy = o[1] - 1 + hy, qz = o[2] - 1 + hz;
            float2 v = make_float2(0.f, 0.f);
            if (in_grid(qx, M) && in_grid(qy, M) && in_grid(qz, M)) v = a.src[((int64_t)qz * M + qy) * M + qx];
            vh[(hz * VR + hy) * VR + hx] = v;
        }
    }
    if (SCATTER) {
        for (int t = threadIdx.x; t < BS * AP; t += kBT) {
            acc_re[t] = 0.0;
            acc_im[t] = 0.0;
        }
    }
    // enumeration box (grid coordinates): owned pixels have floor(g) in the
    // brick, touching pixels have floor(g) in [b0 - 1, b0 + BS - 1]
    float lo[3], hi[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = (float)(OWNER_ONLY ? o[d] : o[d] - 1);
        hi[d] = (float)(o[d] + BS);
    }
    const float halff = (float)g.half;
    const double halfd = (double)g.half;
    const int kymax = (int)floorf(sqrtf((float)g.k2max) + 1e-4f);
    const int *list = a.lists + (int64_t)brick * a.stride + first;
    const double ctfB = g.ctf_b * g.inv_s2 * g.inv_s2;
    const uint32_t MM = (uint32_t)M * (uint32_t)M;
    double lsum = 0.0;
    __syncthreads();

    for (int gi = 0; gi < n_img; gi += GIMG) {
        // every wave has finished with the previous group's scan, segments
        // and image slots before they are rewritten
        __syncthreads();
        // ---- row segments of GIMG images x ROWS rows, one per thread
        const int s = threadIdx.x / ROWS, r = threadIdx.x % ROWS;
        int len = 0, kx0 = 0, ky = 0;
        uint32_t img_base = 0;
        if (gi + s < n_img) {
            const int ii = list[gi + s];
            img_base = (uint32_t)ii * MM;
            float e1[3], e2[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                e1[d] = a.rot[(int64_t)ii * 9 + d];
                e2[d] = a.rot[(int64_t)ii * 9 + 3 + d];
            }
            if (r == 0) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    slot[s].e1[d] = (double)e1[d];
                    slot[s].e2[d] = (double)e2[d];
                }
                slot[s].ctfA = g.ctf_a * (double)a.defocus[ii] * g.inv_s2;
            }
            // rows: range of e2 . (g - half) over the box
            float ylo = 0.f, yhi = 0.f;
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const float u = e2[d] * (lo[d] - halff), w = e2[d] * (hi[d] - halff);
                ylo += fminf(u, w);
                yhi += fmaxf(u, w);
            }
            const int ky_lo = max((int)ceilf(ylo - kClipEps), -kymax);
            const int ky_hi = min((int)floorf(yhi + kClipEps), kymax);
            ky = ky_lo + r;
            if (ky <= ky_hi) {
                int x0, x1;
                clip_row(e1, e2, halff, ky, lo, hi, x0, x1);
                // the disk: |kx| <= floor(sqrt(k2max - ky^2))
                const int rem = g.k2max - ky * ky;
                int kxm = (int)sqrtf((float)rem);
                while ((kxm + 1) * (kxm + 1) <= rem) ++kxm;
                while (kxm * kxm > rem) --kxm;
                x0 = max(x0, -kxm);
                x1 = min(x1, kxm);
                if (x1 >= x0) {
                    len = x1 - x0 + 1;
                    kx0 = x0;
                }
            }
        }
        int T;
        const int pre = block_exclusive_scan(len, wave_sums, &T);
        seg[threadIdx.x] = make_int4(pre, kx0, (ky + 512) | (s << 16),
                                     (int)(img_base + (uint32_t)(ky + g.half) * (uint32_t)M + (uint32_t)g.half));

        for (int wbase = 0; wbase < T; wbase += PIXCAP) {
            // ---- pixel -> segment table of this window
            {
                const int b0 = max(pre, wbase), b1 = min(pre + len, wbase + PIXCAP);
                for (int q = b0; q < b1; ++q) pix2seg[q - wbase] = (unsigned short)threadIdx.x;
            }
            __syncthreads();
            const int wend = min(T, wbase + PIXCAP);
            for (int f = wbase + threadIdx.x; f < wend; f += kBT) {
                const int sl = pix2seg[f - wbase];
                const int4 rec = seg[sl];
                const int pkx = rec.y + (f - rec.x);
                const int pky = (rec.z & 0xFFFF) - 512;
                const ImgSlot &I = slot[rec.z >> 16];
                const double dkx = (double)pkx, dky = (double)pky;
                double rel[3];
                float t[3];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const double gd = fma(dkx, I.e1[d], fma(dky, I.e2[d], halfd));
                    const double fl = floor(gd);
                    rel[d] = fl - (double)o[d];  // base corner relative to the brick
                    t[d] = (float)(gd - fl);
                }
                // range tests in floating point (NaN fails them), so only
                // in-range values are converted to int
                const bool owned = rel[0] >= 0.0 && rel[0] <= BS - 1.0 && rel[1] >= 0.0 && rel[1] <= BS - 1.0 &&
                                   rel[2] >= 0.0 && rel[2] <= BS - 1.0;
                const bool inside = rel[0] >= -1.0 && rel[0] <= BS - 1.0 && rel[1] >= -1.0 &&
                                    rel[1] <= BS - 1.0 && rel[2] >= -1.0 && rel[2] <= BS - 1.0;
                if (OWNER_ONLY ? !owned : !inside) continue;
                const int l[3] = {(int)rel[0], (int)rel[1], (int)rel[2]};
                float C = 1.0f;
                if (g.ctf_on) {
                    const double k2 = (double)(pkx * pkx + pky * pky);
                    const double turns = fma(fma(-ctfB, k2, I.ctfA), k2, g.phase0);
                    C = -__builtin_amdgcn_sinf((float)(turns - rint(turns)));
                }
                const uint32_t j = (uint32_t)rec.w + (uint32_t)pkx;
                const float wx[2] = {1.0f - t[0], t[0]};
                const float wy[2] = {1.0f - t[1], t[1]};
                const float wz[2] = {1.0f - t[2], t[2]};
                float2 acc = make_float2(0.f, 0.f);
                if (GATHER) {
                    // halo index of the base corner: l + 1 in [0, BS]; halo
                    // voxels outside the grid hold zeros, which drops those
                    // corners
                    const int hb = ((l[2] + 1) * VR + (l[1] + 1)) * VR + (l[0] + 1);
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int ax = c & 1, ay = (c >> 1) & 1, az = (c >> 2) & 1;
                        const float w = wx[ax] * wy[ay] * wz[az];
                        const float2 v = vh[hb + az * VP + ay * VR + ax];
                        acc.x = fmaf(w, v.x, acc.x);
                        acc.y = fmaf(w, v.y, acc.y);
                    }
                }
                float2 val = make_float2(0.f, 0.f);
                if (MODE == kBProject) {
                    float2 y = make_float2(C * acc.x, C * acc.y);
                    if (a.img) {
                        const float2 x = a.img[j];
                        y.x -= x.x;
                        y.y -= x.y;
                    }
                    if (a.out) a.out[j] = y;
                    lsum += 0.5 * ((double)y.x * y.x + (double)y.y * y.y);
                } else if (MODE == kBBackproject) {
                    const float2 x = a.img[j];
                    const float fct = a.scale * ctf_pow(C, a.ctf_power);
                    val = make_float2(fct * x.x, fct * x.y);
                } else if (MODE == kBGradient) {
                    const float2 x = a.img[j];
                    const float2 rr = make_float2(fmaf(C, acc.x, -x.x), fmaf(C, acc.y, -x.y));
                    if (owned) lsum += 0.5 * ((double)rr.x * rr.x + (double)rr.y * rr.y);
                    const float fct = a.scale * C;
                    val = make_float2(fct * rr.x, fct * rr.y);
                } else if (MODE == kBHvp) {
                    const float fct = a.scale * C * C;
                    val = make_float2(fct * acc.x, fct * acc.y);
                } else if (MODE == kBFeatures) {
                    val = make_float2(C * C, 1.0f);
                } else if (MODE == kBSqDiag) {
                    val = make_float2(a.scale * C * C, 0.0f);
                }
                if (SCATTER) {
                    // corners inside the brick; a corner beyond the grid edge
                    // lands in an LDS slot that is never written back
                    const int lb = l[2] * AP + l[1] * AR + l[0];
#pragma unroll
                    for (int c = 0; c < 8; ++c) {
                        const int ax = c & 1, ay = (c >> 1) & 1, az = (c >> 2) & 1;
                        const int lx = l[0] + ax, ly = l[1] + ay, lz = l[2] + az;
                        if ((unsigned)lx < (unsigned)BS && (unsigned)ly < (unsigned)BS &&
                            (unsigned)lz < (unsigned)BS) {
                            const float w = wx[ax] * wy[ay] * wz[az];
                            const int li = lb + az * AP + ay * AR + ax;
                            if (MODE == kBSqDiag) {
                                atomicAdd(&acc_re[li], (double)(w * w * val.x));
                            } else {
                                atomicAdd(&acc_re[li], (double)(w * val.x));
                                atomicAdd(&acc_im[li], (double)(w * val.y));
                            }
                        }
                    }
                }
            }
            __syncthreads();  // the table (and, after the last window, the segments) are rebuilt
        }
    }

    if (SCATTER) {
        for (int t = threadIdx.x; t < BS * BS * BS; t += kBT) {
            const int tx = t % BS, ty = (t / BS) % BS, tz = t / (BS * BS);
            const int qx = o[0] + tx, qy = o[1] + ty, qz = o[2] + tz;
            if (!(qx < M && qy < M && qz < M)) continue;
            const int li = tz * AP + ty * AR + tx;
            const float re = (float)acc_re[li], im = (float)acc_im[li];
            if (MODE == kBSqDiag) {
                float *pr = a.accum_real + ((int64_t)qz * M + qy) * M + qx;
                if (single) *pr += re;
                else if (re != 0.f) atomicAdd(pr, re);
                continue;
            }
            float2 *p = a.accum + ((int64_t)qz * M + qy) * M + qx;
            if (single) {
                float2 v = *p;
                v.x += re;
                v.y += im;
                *p = v;
            } else if (re != 0.f || im != 0.f) {
                atomicAdd(&p->x, re);
                atomicAdd(&p->y, im);
            }
        }
    }
    if ((MODE == kBProject || MODE == kBGradient) && a.loss) {
        const double t = block_sum(lsum, red);
        if (threadIdx.x == 0 && t != 0.0) atomicAdd(a.loss, t);
    }
}

// Zero the pixels outside the disk (the brick kernels write only the disk).
// One thread per (image row, pixel); only the pixels outside the disk are
// stored.
__global__ __launch_bounds__(kBlock) void zero_outside_disk_kernel(float2 *out, int64_t n, int M, int half,
                                                                    int k2max) {
    const int64_t rows = n * (int64_t)M;
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int ky = (int)(row % M) - half;
        for (int x = threadIdx.x; x < M; x += blockDim.x) {
            const int kx = x - half;
            if (kx * kx + ky * ky > k2max) out[row * M + x] = make_float2(0.f, 0.f);
        }
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int brick_count(int M) {
    const int nbx = (M + BS - 1) / BS;
    return nbx * nbx * nbx;
}

size_t brick_workspace_bytes(int M, int64_t n) {
    const int64_t sub = n < kBrickSubBatch ? n : kBrickSubBatch;
    const size_t nb = (size_t)brick_count(M);
    const size_t counts = (nb * 4 + 255) / 256 * 256;
    return counts + nb * (size_t)(sub > 0 ? sub : 1) * 4;
}

template <int MODE>
static hipError_t run_brick_mode(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *src,
                                 const float2 *img, float2 *out, float2 *accum, double *loss, float scale,
                                 int ctf_power, void *ws, hipStream_t st, float *accum_real = nullptr) {
    const int M = g.M;
    const int nbx = (M + BS - 1) / BS;
    const int nb = nbx * nbx * nbx;
    int *counts = (int *)ws;
    int *lists = (int *)((char *)ws + ((size_t)nb * 4 + 255) / 256 * 256);
    const int64_t img_stride = (int64_t)M * M;
    for (int64_t s0 = 0; s0 < n; s0 += kBrickSubBatch) {
        const int64_t ns = (n - s0) < kBrickSubBatch ? (n - s0) : kBrickSubBatch;
        const int stride = (int)ns;
        hipLaunchKernelGGL(brick_cull_kernel, dim3(nb), dim3(kBlock), 0, st, g, rot + s0 * 9, ns, nbx, counts, lists,
                           stride);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        BrickArgs a{};
        a.g = g;
        a.rot = rot + s0 * 9;
        a.defocus = defocus + s0;
        a.n = ns;
        a.src = src;
        a.img = img ? img + s0 * img_stride : nullptr;
        a.out = out ? out + s0 * img_stride : nullptr;
        a.accum = accum;
        a.accum_real = accum_real;
        a.loss = loss;
        a.scale = scale;
        a.ctf_power = ctf_power;
        a.counts = counts;
        a.lists = lists;
        a.stride = stride;
        a.nbx = nbx;
        a.nb = nb;
        const int chunk = MODE == kBProject ? CHUNK_FWD : CHUNK_ADJ;
        const int64_t chunks = (ns + chunk - 1) / chunk;
        a.nchunks = (int)chunks;
        hipEvent_t t0 = timing_begin(MODE, st);
        hipLaunchKernelGGL((brick_kernel<MODE>), dim3((unsigned)(chunks * nb)), dim3(kBT), 0, st, a);
        e = hipGetLastError();
        timing_end(MODE, t0, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The brick kernels implement trilinear interpolation; nearest-neighbour
// grids (the exact-pin mode of Sec. 3.1) use the pixel-parallel kernels.
hipError_t launch_brick_project(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *vol,
                                const float2 *subtract, float2 *out, double *loss, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_project(g, rot, defocus, n, vol, subtract, out, loss, st);
    hipError_t e = run_brick_mode<kBProject>(g, rot, defocus, n, vol, subtract, out, nullptr, loss, 1.0f, 0, ws, st);
    if (e != hipSuccess || !out) return e;
    int64_t blocks = n * (int64_t)g.M;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(zero_outside_disk_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, out, n, g.M, g.half,
                       g.k2max);
    return hipGetLastError();
}

hipError_t launch_brick_backproject(const Geom &g, const float *rot, const float *defocus, int64_t n,
                                    const float2 *img, int ctf_power, float scale, float2 *accum, void *ws,
                                    hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_backproject_atomic(g, rot, defocus, n, img, ctf_power, scale, accum, st);
    return run_brick_mode<kBBackproject>(g, rot, defocus, n, nullptr, img, nullptr, accum, nullptr, scale, ctf_power,
                                         ws, st);
}

hipError_t launch_brick_gradient(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *vol,
                                 const float2 *x, float scale, float2 *accum, double *loss, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_gradient_atomic(g, rot, defocus, n, vol, x, scale, accum, loss, st);
    return run_brick_mode<kBGradient>(g, rot, defocus, n, vol, x, nullptr, accum, loss, scale, 1, ws, st);
}

hipError_t launch_brick_feature_sums(const Geom &g, const float *rot, const float *defocus, int64_t n,
                                     float2 *accum, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return hipErrorInvalidValue;  // trilinear stencils only
    return run_brick_mode<kBFeatures>(g, rot, defocus, n, nullptr, nullptr, nullptr, accum, nullptr, 1.0f, 0, ws, st);
}

hipError_t launch_brick_sq_diag(const Geom &g, const float *rot, const float *defocus, int64_t n, float scale,
                                float *diag, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_sq_diag(g, rot, defocus, n, scale, diag, st);
    return run_brick_mode<kBSqDiag>(g, rot, defocus, n, nullptr, nullptr, nullptr, nullptr, nullptr, scale, 2, ws, st,
                                    diag);
}

hipError_t launch_brick_hvp(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *z,
                            float scale, float2 *accum, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_hvp_atomic(g, rot, defocus, n, z, scale, accum, st);
    return run_brick_mode<kBHvp>(g, rot, defocus, n, z, nullptr, nullptr, accum, nullptr, scale, 2, ws, st);
}

}  // namespace csg
