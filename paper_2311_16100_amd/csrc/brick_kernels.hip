// brick_kernels.hip -- brick-binned forward projection and adjoint.
//
// The volume is cut into 12^3 bricks.  A cull kernel lists, per brick and in
// image order, the images whose slice plane reaches the brick; a plan kernel
// turns the lists into work items (one brick and chunks of its images),
// ordered by size, largest first.  One wave of resident blocks takes the items from
// that list with an atomic counter.  For each item the block takes the
// brick's images in chunks (64 for the forward mode, 128 for the adjoint
// modes; up to eight chunks per item for the gradient and HVP) and
//   - stages the brick and the voxels one step above it on each axis (13^3
//     complex values of the gathered volume) in LDS once, so every trilinear
//     gather is 8 LDS reads;
//   - accumulates the adjoint into an LDS array of the same extent as exact
//     fixed-point integers: in the gradient and the HVP both components
//     of a contribution in one 64-bit word with wrap counters (CarryScale),
//     elsewhere one 64-bit integer per component (ItemScale; the
//     deterministic mode: FxScale; the probe modes keep one 32-bit sum of
//     z (.) H z per voxel, see PackedScale: flushed after every chunk), and
//     adds it to HBM
//     once per voxel at the end with global
//     atomics (the upper faces of the extent belong to the neighbouring
//     bricks, which other blocks may be flushing at the same time).  On gfx950
//     the LDS single-precision atomic add sustains about a twentieth of the
//     lane rate of the 64-bit ones, and in these kernels the integer add is
//     cheaper than the double one, so the wide integer accumulator is also
//     the fastest; the scatter to effectively random voxels of the extent
//     is bound by LDS bank conflicts, which cost per atomic instruction, so
//     one instruction per contribution beats two.
// The pixels of an image that matter for a brick are found row by row: for
// image row ky the sample points form a line, and the pixels whose cell
// reaches the brick's box form an interval of kx, computed by clipping the
// line against the box.  Each image of a window owns a fixed block of row
// records, a block scan turns their intervals into one flat range of runs (one or two
// consecutive pixels of a row), and the lanes walk that range together, so
// neighbouring lanes take neighbouring pixels of a row (coalesced image reads
// and writes).  Within a run the sample point advances in exact fixed-point
// arithmetic (see ImgSlot), so every brick sees identical cells.
//
// A pixel is handled by exactly one brick: the one that contains its base
// corner floor(g).  Its eight corners lie in that brick's extended extent
// (the brick plus one voxel above on each axis), so the gather, the forward
// value, the loss term and all eight adjoint contributions of the pixel are
// computed once, with no per-corner bounds tests.
//
// Modes:
//   kBProject      out = C P v (- x) for owned pixels; loss
//   kBBackproject  accum += scale C^p img
//   kBGradient     r = C P v - x; loss (owner); accum += scale C r
//   kBHvp          accum += scale C^2 P z
//   kBHvpProbe     diag += z (.) scale C^2 P z for a Rademacher probe pair z
//                  (Hutchinson), generated from its hash while the brick is
//                  staged and kept as two halves per voxel; each contribution
//                  is multiplied by the receiving voxel's probe signs at once,
//                  so the accumulator holds z (.) H z itself, one 32-bit
//                  fixed-point number per voxel (see PackedScale), added to
//                  the diagonal after every chunk of images
//   kBFeatures     accum += (C^2, 1) w: the CTF^2 weight and the plain weight
//                  sum of every voxel (no image is read)
//   kBSqDiag       diag += scale C^2 w^2: the exact diagonal of the data
//                  Hessian (real accumulator; no image is read)
//   kBGradProbe    kBGradient and kBHvpProbe of the same images in one pass
//                  (the Hessian does not depend on v, so both visit the same
//                  pixels with the same cells, weights and CTF values; no
//                  in-plane shifts)
#include <type_traits>

#include "carry.h"
#include "csg_device.h"
#include "csg_internal.h"

namespace csg {

#ifndef CSG_BRICK_SIDE
#define CSG_BRICK_SIDE 12
#endif
constexpr int BS = CSG_BRICK_SIDE;  // brick side
constexpr int BX = BS + 1;       // extended side: the brick and one voxel above
// LDS strides are odd (in elements) so that lanes stepping along any axis of
// the brick fall into different banks.
constexpr int XR = BX | 1;       // row stride of the staged volume and the accumulator (13)
constexpr int XP = XR * XR;      // plane stride (169)
constexpr int XN = BX * XP;      // elements of one staged array
constexpr int kBT = 512;         // threads per brick block (8 waves)
// Tuning constants (measured at 256^3 with 1024 images); each may be set at
// compile time.
#ifndef CSG_CHUNK_ADJ
#define CSG_CHUNK_ADJ 128
#endif
#ifndef CSG_CHUNK_FWD
#define CSG_CHUNK_FWD 64
#endif
#ifndef CSG_RUN_ADJ
#define CSG_RUN_ADJ 2
#endif
#ifndef CSG_RUN_GRAD
#define CSG_RUN_GRAD 2
#endif
#ifndef CSG_RUN_GP
#define CSG_RUN_GP 1
#endif
#ifndef CSG_WI_ADJ
#define CSG_WI_ADJ 32
#endif
#ifndef CSG_WI_GH
#define CSG_WI_GH 64
#endif
#ifndef CSG_RUN_FWD
#define CSG_RUN_FWD 1
#endif
#ifndef CSG_WI_FWD
#define CSG_WI_FWD 64
#endif
// run-table entries of the gradient and HVP modes: as many as fit beside
// their other LDS at two blocks per CU (80 KB).  The fast modes' carry
// accumulator needs half the counter space of the two-word accumulator of
// the deterministic modes and takes 4352 more; the gradient with in-plane
// shifts keeps two image constants more per image and takes 384 fewer
#ifndef CSG_RUNCAP_GH
#define CSG_RUNCAP_GH 3584
#endif
#ifndef CSG_RUNCAP_ADJ
#define CSG_RUNCAP_ADJ 2048
#endif
#ifndef CSG_RUNCAP_CARRY_EXTRA
#define CSG_RUNCAP_CARRY_EXTRA 4352
#endif
#ifndef CSG_RUNCAP_SHIFT_CUT
#define CSG_RUNCAP_SHIFT_CUT 384
#endif
// the probe HVP, which stages only the probe pair and keeps one 32-bit sum
// per voxel, takes this many more run-table entries
#ifndef CSG_RUNCAP_PROBE_EXTRA
#define CSG_RUNCAP_PROBE_EXTRA 4608
#endif
#ifndef CSG_BRICK_WAVES_GH
#define CSG_BRICK_WAVES_GH 4
#endif
// the fused gradient and probe mode: images per window and run-table
// entries (as many as fit beside its two accumulators at two blocks per CU)
#ifndef CSG_WI_GP
#define CSG_WI_GP 32
#endif
#ifndef CSG_RUNCAP_GP
#define CSG_RUNCAP_GP 3584
#endif
constexpr int CHUNK_ADJ = CSG_CHUNK_ADJ;  // images per work item of the adjoint modes
constexpr int CHUNK_FWD = CSG_CHUNK_FWD;  // images per work item of the forward mode (no flush)
constexpr float kClipEps = 1e-2f;

enum BrickMode { kBProject = 0, kBBackproject = 1, kBGradient = 2, kBHvp = 3, kBFeatures = 4, kBSqDiag = 5,
                 kBHvpProbe = 6, kBGradProbe = 7 };
constexpr bool is_hvp(int mode) { return mode == kBHvp || mode == kBHvpProbe; }
constexpr bool is_grad(int mode) { return mode == kBGradient || mode == kBGradProbe; }
// the most chunks of a brick's images per work item (staged and flushed once
// for all of them): eight for the gradient and HVP modes (two blocks per CU),
// two for the modes with three blocks per CU (measured: a whole brick per
// item leaves those with a long tail); the plan lowers it for small batches
constexpr int max_chunks_per_item(int mode) { return (is_grad(mode) || is_hvp(mode)) ? 8 : 2; }

struct BrickArgs {
    Geom g;
    const float *rot;
    const float *defocus;
    const float *shift; // [n][2] in-plane shifts or NULL (project, backproject, gradient)
    int64_t n;          // images of this sub-batch
    const float2 *src;  // gathered volume
    const float2 *img;  // x (project subtract / gradient) or adjoint input
    float2 *out;        // projected images
    float2 *accum;      // adjoint target
    float *accum_real;  // real target (squared-weight diagonal)
    double *loss;
    float scale;
    float scale2;       // fused gradient and probe: the probe product's factor
    int ctf_power;
    const int *counts;  // [nb]
    const int *lists;   // [nb][stride]
    int stride;
    int nbx, nb;
    const int2 *items;  // work items, heaviest first: (brick | first chunk << 20, images of the brick)
    const int *n_items; // number of work items
    int *next_item;     // work counter (zero at launch)
    const int *per_item; // chunks of images per work item
    // deterministic adjoint (fixed point, see FxScale): the 64-bit volume
    // [M^3][re, im], the input bounds and the images of the whole launch
    unsigned long long *fx;
    const unsigned *fx_max;
    int64_t n_total;
    // probe HVP: the Rademacher pair z = z_a + i z_b (z_b = 0 without has_b),
    // generated while the bricks are staged (rademacher_block)
    uint64_t probe_seed, probe_a, probe_b;
    int probe_has_b;
};

__device__ __forceinline__ void brick_origin(int b, int nbx, int o[3]) {
    o[0] = (b % nbx) * BS;
    o[1] = ((b / nbx) % nbx) * BS;
    o[2] = (b / (nbx * nbx)) * BS;
}

// ---------------------------------------------------------------------------
// Cull: lists[b] = images whose plane meets the box of sample points whose
// base corner lies in brick b (grid coordinates [b0, b0 + BS]^3), in
// increasing image order.  One wave per brick, eight bricks per block: the
// block stages the third rows of R for a chunk of images in LDS once, and each
// wave tests them against its brick.
// ---------------------------------------------------------------------------
constexpr int kCullWaves = 8;
constexpr int kCullThreads = kCullWaves * 64;

__global__ __launch_bounds__(kCullThreads) void brick_cull_kernel(Geom g, const float *rot, int64_t n, int nbx, int nb,
                                                                   int *counts, int *lists, int stride) {
    __shared__ float se[kCullThreads][3];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = blockIdx.x * kCullWaves + wv;
    float c[3] = {0.f, 0.f, 0.f}, hw[3] = {0.f, 0.f, 0.f};
    bool reachable = false;
    if (b < nb) {
        int o[3];
        brick_origin(b, nbx, o);
        float dist2 = 0.f;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const float lo = (float)(o[d] - g.half), hi = (float)(o[d] + BS - g.half);
            c[d] = 0.5f * (lo + hi);
            hw[d] = 0.5f * (hi - lo);
            const float near = fmaxf(fmaxf(lo, -hi), 0.f);  // distance of the box to the origin along d
            dist2 += near * near;
        }
        // sample points lie within |p| <= r_max; the box must come that close
        const float rmax = sqrtf((float)g.k2max) + 2.0f;
        reachable = dist2 <= rmax * rmax;
    }
    const uint64_t below = (1ull << lane) - 1ull;
    int total = 0;
    for (int64_t base = 0; base < n; base += kCullThreads) {
        const int64_t i = base + threadIdx.x;
        if (i < n) {
            se[threadIdx.x][0] = rot[i * 9 + 6];
            se[threadIdx.x][1] = rot[i * 9 + 7];
            se[threadIdx.x][2] = rot[i * 9 + 8];
        }
        __syncthreads();
        const int cnt = (int)min((int64_t)kCullThreads, n - base);
        if (reachable) {
            for (int s0 = 0; s0 < cnt; s0 += 64) {
                const int ii = s0 + lane;
                bool keep = false;
                if (ii < cnt) {
                    const float e0 = se[ii][0], e1 = se[ii][1], e2 = se[ii][2];
                    const float h = e0 * c[0] + e1 * c[1] + e2 * c[2];
                    const float reach = fabsf(e0) * hw[0] + fabsf(e1) * hw[1] + fabsf(e2) * hw[2];
                    keep = fabsf(h) <= reach + kClipEps;
                }
                const uint64_t mask = __ballot(keep);
                if (keep) lists[(int64_t)b * stride + total + __popcll(mask & below)] = (int)(base + ii);
                total += __popcll(mask);
            }
        }
        __syncthreads();
    }
    if (b < nb && lane == 0) counts[b] = total;
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

// ---------------------------------------------------------------------------
// Plan: one work item per brick and run of up to `per` consecutive chunks of
// `chunk` images of its list (the block that takes the item stages the brick
// once for all of them), ordered by the number of images, largest first, so
// that the long items start first: the key is ceil(images / per), at most
// `chunk`.  `per` is the largest value up to `max_per` that leaves at least
// `min_items` items (about ceil(chunks / per) of them), so that small batches
// keep every resident block busy; it is stored in *per_out for the kernel.
// Each wave counts into its own histogram copy (fewer colliding LDS atomics).
// Resets the work counter.  One block.
// ---------------------------------------------------------------------------
constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;
constexpr int kMaxChunk = 128;
static_assert(CHUNK_ADJ <= kMaxChunk && CHUNK_FWD <= kMaxChunk, "plan histogram too small");

__global__ __launch_bounds__(kPlanThreads) void brick_plan_kernel(const int *counts, int nb, int chunk, int max_per,
                                                                   int min_items, int2 *items, int *n_items,
                                                                   int *next_item, int *per_out) {
    __shared__ int hist[kPlanWaves][kMaxChunk + 1];
    __shared__ int base[kMaxChunk + 1];
    __shared__ int s_chunks;
    const int wv = threadIdx.x >> 6;
    // the batch's chunks, then chunks per item
    if (threadIdx.x == 0) s_chunks = 0;
    __syncthreads();
    {
        int nc = 0;
        for (int b = threadIdx.x; b < nb; b += kPlanThreads) nc += (counts[b] + chunk - 1) / chunk;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) nc += __shfl_xor(nc, off, 64);
        if ((threadIdx.x & 63) == 0 && nc) atomicAdd(&s_chunks, nc);
    }
    __syncthreads();
    const int per = max(1, min(max_per, s_chunks / max(min_items, 1)));
    if (threadIdx.x == 0) *per_out = per;
    const int span = chunk * per;  // images of a full item
    for (int k = threadIdx.x; k < kPlanWaves * (kMaxChunk + 1); k += kPlanThreads) (&hist[0][0])[k] = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kPlanThreads) {
        const int c = counts[b], full = c / span, rem = c - full * span;
        if (full) atomicAdd(&hist[wv][chunk], full);
        if (rem) atomicAdd(&hist[wv][(rem + per - 1) / per], 1);
    }
    __syncthreads();
    // bucket starts (largest key first), then per-wave cursors inside each
    // bucket (in place of the counts)
    if ((int)threadIdx.x <= chunk) {
        const int k = threadIdx.x;
        int tot = 0;
        for (int w = 0; w < kPlanWaves; ++w) tot += hist[w][k];
        base[k] = tot;
    }
    __syncthreads();
    // bucket starts in the order chunk, chunk - 1, ..., 1: an exclusive scan
    // over the first chunk threads (thread r holds bucket chunk - r)
    {
        __shared__ int wsum[kPlanWaves];
        const int r = threadIdx.x, lane = r & 63;
        const int val = r < chunk ? base[chunk - r] : 0;
        int x = val;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wsum[wv] = x;
        __syncthreads();
        int pre = 0;
        for (int w = 0; w < wv; ++w) pre += wsum[w];
        if (r < chunk) base[chunk - r] = pre + x - val;
        if (r == chunk - 1) {
            *n_items = pre + x;
            *next_item = 0;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x <= chunk) {
        const int k = threadIdx.x;
        int run = base[k];
        for (int w = 0; w < kPlanWaves; ++w) {
            const int t = hist[w][k];
            hist[w][k] = run;
            run += t;
        }
    }
    __syncthreads();
    // item record: (brick | first chunk << 20, images of the brick)
    for (int b = threadIdx.x; b < nb; b += kPlanThreads) {
        const int c = counts[b], full = c / span, rem = c - full * span;
        if (full) {
            const int p = atomicAdd(&hist[wv][chunk], full);
            for (int k = 0; k < full; ++k) items[p + k] = make_int2(b | ((k * per) << 20), c);
        }
        if (rem) items[atomicAdd(&hist[wv][(rem + per - 1) / per], 1)] = make_int2(b | ((full * per) << 20), c);
    }
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

// Per-image constants of a window, in LDS.  The sample point of pixel
// (kx, ky) is kept in fixed point with 32 fractional bits:
//   G = kx E1 + ky E2 + (M/2) 2^32,  E = rint(e 2^32)  (e a row of R),
// an exact integer (|G| < 2^53), formed in double precision at the first
// pixel of a run and advanced by the integer E1 from pixel to pixel.  Every
// brick therefore obtains bit-identical cells and offsets for a pixel, so
// ownership is decided consistently, and the point differs from
// kx e1 + ky e2 + M/2 by at most (|kx| + |ky|) 2^-33 grid units.
struct ImgSlot {
    double E1[3];      // rint(e1 2^32), exact integers
    double E2[3];
    int64_t E1i[3];    // the same as integers (the per-pixel step)
    double ctfA;       // (lambda df / 2) / (M pixel)^2: chi / 2pi = k2 (ctfA - ctfB k2)
    uint32_t img_base; // index of pixel (0, 0) of the image: i M^2
    short ky_lo;       // first row that can reach the box
    unsigned short nrows; // rows that can reach the box (at most MAXROWS)
    float sx, sy;      // in-plane shift (pixels)
};

// rows of one image that reach a brick's box (side BS): the box's extent
// along e2 is at most BS sqrt(3), plus the clipping margins
constexpr int MAXROWS = (int)(BS * 1.7321f) + 2;
constexpr int MAXLEN = MAXROWS + 8;  // bound on a row interval (same argument along e1)

// Window sizes per mode: images per window (a whole forward chunk; 64 for
// gradient and HVP, whose LDS footprint allows two blocks per CU either way;
// 32 for the other adjoint modes, which keeps them at three blocks per CU)
// and runs per pass of the run -> row table.
template <int MODE>
struct Win {
    // consecutive pixels of a row per lane (measured fastest): one for the
    // forward mode and the fused gradient and probe mode (whose two
    // accumulators leave no registers for a second pixel's state), two for
    // the adjoint modes, the gradient among them
    static constexpr int RUN = MODE == kBProject ? CSG_RUN_FWD : MODE == kBGradProbe ? CSG_RUN_GP
                             : MODE == kBGradient ? CSG_RUN_GRAD : CSG_RUN_ADJ;
    static constexpr int WI = MODE == kBProject ? CSG_WI_FWD : MODE == kBGradProbe ? CSG_WI_GP
                            : (MODE == kBGradient || is_hvp(MODE)) ? CSG_WI_GH : CSG_WI_ADJ;
    static constexpr int ROWCAP = WI * MAXROWS;          // row records per window
    static constexpr int RPT = (ROWCAP + kBT - 1) / kBT; // rows per thread
    static constexpr int RUNCAP = MODE == kBProject ? 7168 : MODE == kBGradProbe ? CSG_RUNCAP_GP
                                : (MODE == kBGradient || is_hvp(MODE)) ? CSG_RUNCAP_GH : CSG_RUNCAP_ADJ;
};

__device__ __forceinline__ double rint_scaled(float e) {
    return rint((double)fminf(fmaxf(e, -2.0f), 2.0f) * 0x1p32);
}

// Fixed-point scale of the probe modes' LDS accumulator of z (.) H z for a
// Rademacher pair z = z_a + i z_b.  The pixel's value is val = scale C^2
// (P z)_pixel, and corner c of its stencil receives w_c (z_a(c) val.x +
// z_b(c) val.y), the contribution to z (.) H z of the voxel it lands in,
// rounded to an integer multiple of 1/S and added to that voxel's signed
// 32-bit integer.
//
// The bound: |z_a(c) val.x + z_b(c) val.y| <= |val.x| + |val.y| <= V =
// |scale| (|z_a| + |z_b|) = 2 |scale| (|C| <= 1 and the trilinear weights
// sum to 1), and w_c <= 1.  A voxel receives from one image at most the
// pixels of the plane lattice inside its 2x2x2 neighbourhood, whose section
// has area at most 4 sqrt(2): at most 13 pixels (Pick's theorem; 16 is
// used).  Over a chunk of at most 128 images (the probe modes flush after
// each) a voxel's sum is therefore below 2048 V = B, and S = 2^e with
// B S <= 2^30 keeps every sum (and every rounded contribution) below 2^30.
// The rounding error is at most 1/(2S) per contribution, i.e. 2^-31 B
// (relative 5e-10 of B).  Because B is a worst case, the result is about
// 1e-5 relative (measured), well below the noise of a two-probe Hutchinson
// estimate; the gradient and the general HVP, whose sums need float
// accuracy, keep exact 64-bit sums.
// x rounded to an integer, halves upwards (floor(x + 0.5) in one
// instruction; |x| < 2^31)
__device__ __forceinline__ int round_half_up(float x) {
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

struct PackedScale {
    float S = 1.f, invS = 1.f;
    static __device__ __forceinline__ PackedScale make(float V) {
        static_assert(CHUNK_ADJ <= 128, "the fixed-point bound assumes at most 128 images per item");
        PackedScale p;
        const float B = 2048.f * V;
        int e = 0;
        if (B > 0.f && B < 3.0e38f) {
            int k;
            (void)frexpf(B, &k);  // B < 2^k
            e = min(max(30 - k, -126), 100);
        }
        p.S = ldexpf(1.f, e);
        p.invS = ldexpf(1.f, -e);
        return p;
    }
};

// Per-item fixed-point scale of the 64-bit LDS accumulator of the fast
// adjoint modes.  A contribution is w val with w <= 1 and |val| <= V; an item
// holds at most one sub-batch of 2048 images and a voxel receives
// at most 32 pixels of one image (see FxScale), so every LDS sum stays below
// 2^16 V.  S = 2^e is the largest power of two with 2^16 V S <= 2^61 and
// V S <= 2^50: the sums are exact, each contribution is rounded by at most
// 2^-46 V (about 2^-22 of a float ulp of V), and the flush converts each
// voxel's sum to float once.
#ifndef CSG_LDS_FIXED
#define CSG_LDS_FIXED 1
#endif
// ok = 0 when an input is not finite (the flush then writes NaN).
struct ItemScale {
    double S = 1.0, invS = 1.0;
    int ok = 1;
    static __device__ __forceinline__ ItemScale make(double V) {
        static_assert(kBrickSubBatch <= 2048, "the LDS bound assumes at most 2048 images per item");
        ItemScale q;
        q.ok = isfinite(V) ? 1 : 0;
        if (q.ok && V > 0.0) {
            int kt, kv;
            (void)frexp(65536.0 * V, &kt);
            (void)frexp(V, &kv);
            const int e = min(61 - kt, 50 - kv);
            q.S = ldexp(1.0, e);
            q.invS = ldexp(1.0, -e);
        }
        return q;
    }
};

// Packed accumulator with wrap counters (gradient and HVP).  A
// contribution (w val.x, w val.y) is rounded to integers (qr, qi) at a
// per-item power-of-two scale S with |val| S <= 2^29, so every integer fits
// in 30 bits.  One 64-bit LDS atomic adds qr + 2^32 qi to the voxel's word
// W, whose low half then holds the real sum R and whose high half the
// imaginary sum I, each modulo 2^32: R = lo + 2^32 c_lo, I = H - c_lo +
// 2^32 c_hi, with lo the low half as a signed number, H the high half plus
// one where lo is negative, and c_lo, c_hi the net count of signed wraps of
// lo and of H.  The atomic returns the word it added to; from that old value
// the lane that made a half wrap sees it happen (the exact test runs only
// when an old half lies outside [-2^30, 2^30), where a 30-bit addend can
// wrap it) and adds +-1 to the counter (both counters of a voxel share one
// 32-bit word, see carry.h).  Every addition is exact, so the sums are exact
// 64-bit integers (as with one 64-bit word per component) while each
// contribution costs one LDS atomic instead of two; each contribution is
// rounded by at most half a step 2^-e <= 2^-28 V, V the item's bound, and
// the flush converts each sum to float once.
struct CarryScale {
    float S = 1.f;
    double invS = 1.0;
    int ok = 1;
    static __device__ __forceinline__ CarryScale make(double V) {
        CarryScale q;
        q.ok = isfinite(V) ? 1 : 0;
        if (q.ok && V > 0.0) {
            int kv;
            (void)frexp(V, &kv);  // V < 2^kv
            int e = 29 - kv;
            if (e < -126) q.ok = 0;
            e = min(max(e, -126), 127);
            q.S = ldexpf(1.f, e);
            q.invS = ldexp(1.0, -e);
        }
        return q;
    }
};

// corners whose atomics are issued before their old words are looked at
// (measured at 256^3 with 1024 images: 2 beats 1, 4 and 8, where the held
// words spill)
#ifndef CSG_CARRY_GROUP
#define CSG_CARRY_GROUP 2
#endif
constexpr int CARRY_GROUP = CSG_CARRY_GROUP;

// the lane's wraps go to the voxel's counters
__device__ __forceinline__ void carry_fix(unsigned long long old, int qr, int qi, int *counters) {
    int dl, dh;
    carry_wraps(old, qr, qi, dl, dh);
    if (dl | dh) atomicAdd(counters, carry_counter_step(dl, dh));
}

// IEEE half-precision bits of 0, 1 or -1, and the two halves of a word as floats
__device__ __forceinline__ uint32_t half_bits(float x) {
    return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)x);
}
__device__ __forceinline__ float half_lo(uint32_t u) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(u & 0xFFFFu));
}
__device__ __forceinline__ float half_hi(uint32_t u) {
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(u >> 16));
}

// Probe signs of row `row` (row = y + BX z of the extended brick) and probe p
// (0: z_a, 1: z_b): bit x is set where the probe is -1 at voxel x of the row
// (at most 13 consecutive voxels, which fall in one or two Philox blocks),
// bit 16 + x where that voxel lies in the grid.
__device__ __forceinline__ uint32_t probe_row_mask(const BrickArgs &a, const int o[3], int M, int row, int p) {
    const int qy = o[1] + row % BX, qz = o[2] + row / BX;
    const int nx = min(BX, M - o[0]);
    uint32_t m = 0u;
    if (qy < M && qz < M && (p == 0 || a.probe_has_b)) {
        const int64_t g0 = ((int64_t)qz * M + qy) * M + o[0];
        const uint64_t probe = p ? a.probe_b : a.probe_a;
        const uint32_t b0 = (uint32_t)(g0 >> 7);
        const U4 r0 = rademacher_block(a.probe_seed, probe, b0);
        const bool next_block = (uint32_t)((g0 + nx - 1) >> 7) != b0;
        const U4 r1 = next_block ? rademacher_block(a.probe_seed, probe, b0 + 1) : r0;
        // the 13 bits from bit (g0 mod 128) on, in the words r0.x .. r0.w
        // r1.x r1.y (a run of 13 spans at most two consecutive words)
        const int start = (int)(g0 & 127), wi = start >> 5, sh = start & 31;
        const uint32_t lo = wi == 0 ? r0.x : wi == 1 ? r0.y : wi == 2 ? r0.z : r0.w;
        const uint32_t hi = wi == 0 ? r0.y : wi == 1 ? r0.z : wi == 2 ? r0.w : r1.x;
        const uint64_t two = ((uint64_t)hi << 32) | lo;
        m = (uint32_t)(two >> sh) & ((1u << nx) - 1u);
        m |= ((1u << nx) - 1u) << 16;
    }
    return m;
}

// z_a + i z_b at voxel x of a row from the row's masks (0 outside the grid;
// z_b = 0 without the second probe)
__device__ __forceinline__ float2 probe_value(const uint32_t m[2], int x, int has_b) {
    float2 z = make_float2(0.f, 0.f);
    if ((m[0] >> (16 + x)) & 1u) {
        z.x = ((m[0] >> x) & 1u) ? -1.f : 1.f;
        if (has_b) z.y = ((m[1] >> x) & 1u) ? -1.f : 1.f;
    }
    return z;
}

#ifndef CSG_BRICK_WAVES
#define CSG_BRICK_WAVES 6
#endif
// waves per SIMD the register allocation must allow: three blocks per CU
// where the LDS footprint permits it (project, backproject, features,
// squared weights), two for gradient and HVP
// FX: the deterministic adjoint (backproject, gradient, HVP): contributions
// are accumulated as 64-bit fixed-point integers (see FxScale), in LDS and in
// the fixed-point volume a.fx, so the result does not depend on the order in
// which blocks and lanes add them.
template <int MODE, bool SHIFT, bool FX>
__global__ __launch_bounds__(kBT, (is_grad(MODE) || is_hvp(MODE)) ? CSG_BRICK_WAVES_GH : CSG_BRICK_WAVES) void brick_kernel(BrickArgs a) {
    static_assert(!FX || MODE == kBBackproject || MODE == kBGradient || MODE == kBHvp,
                  "fixed-point accumulation is built for backproject, gradient and HVP");
    static_assert(!(MODE == kBGradProbe && SHIFT), "the fused gradient and probe mode takes no in-plane shifts");
    // the fused mode: the gradient of kBGradient and, in the same pass over the
    // pixels, the probe product of kBHvpProbe (the probe pair staged beside the
    // gathered volume; z (.) H z in an accumulator of its own, flushed after
    // every chunk)
    constexpr bool PROBE2 = MODE == kBGradProbe;
    // the probe modes (probe HVP, fused): the Rademacher pair staged as two
    // halves per voxel, z (.) H z accumulated as one signed 32-bit
    // fixed-point number per voxel (each contribution multiplied by the
    // receiving voxel's probe signs), flushed into the diagonal after every
    // chunk of images
    constexpr bool PSIGNED = MODE == kBHvpProbe || PROBE2;
    // the modes that gather a staged volume (the probe HVP gathers only the pair)
    constexpr bool GATHER = MODE == kBProject || is_grad(MODE) || MODE == kBHvp;
    constexpr bool SCATTER = MODE != kBProject;
    constexpr bool READS_IMG = MODE == kBProject || MODE == kBBackproject || is_grad(MODE);
    // the in-plane shift is compiled in only where a launch carries shifts
    constexpr bool SHIFTED = SHIFT && READS_IMG;
    constexpr int IMGDAT = SHIFTED ? 10 : 8;
    constexpr int CHUNK = MODE == kBProject ? CHUNK_FWD : CHUNK_ADJ;
    // fixed-point LDS accumulators: the deterministic modes (one 64-bit
    // integer per component, one launch-wide scale, FxScale) and the fast
    // modes other than the probe HVP (a scale per work item: the carry
    // accumulator of CarryScale in gradient and HVP, one 64-bit integer per
    // component with ItemScale in the backproject, features and
    // squared-weight modes; the flush adds floats).  On gfx950 the LDS 64-bit integer atomic
    // add is cheaper than the double one.
    constexpr bool QLDS = FX || (CSG_LDS_FIXED && SCATTER && MODE != kBHvpProbe);
    constexpr bool QITEM = QLDS && !FX;
    // the packed accumulator with wrap counters (see CarryScale)
    // (gradient and HVP; in backproject, with its 80-register budget, the
    // held old words cost spills that ate the gain)
    constexpr bool QCARRY = QITEM && (is_grad(MODE) || MODE == kBHvp);
    using QScale = typename std::conditional<QCARRY, CarryScale, ItemScale>::type;
    // the item bound needs the largest staged volume value (gradient, HVP)
    // and, where images are read (backproject, gradient), a bound on their
    // values: a guess, checked against every value read; an item that meets
    // a larger one is redone with its exact maximum (see the retry below)
    constexpr bool STAGE_MAX = QITEM && GATHER;
    constexpr bool XRETRY = QITEM && READS_IMG;
    // the complex volume accumulator (all adjoint modes but the probe HVP)
    constexpr bool ACC = SCATTER && MODE != kBHvpProbe;
    __shared__ float2 vh[GATHER ? XN : 1];
    __shared__ double acc_re[ACC ? XN : 1];
    // (the carry accumulator keeps one 32-bit counter word per voxel here)
    constexpr int XN_IM = QCARRY ? (XN + 1) / 2 : XN;
    __shared__ double acc_im[ACC ? XN_IM : 1];
    // the fixed-point accumulators of the deterministic mode share the
    // storage (zero bits are zero in both)
    unsigned long long *const acc_qre = reinterpret_cast<unsigned long long *>(acc_re);
    unsigned long long *const acc_qim = reinterpret_cast<unsigned long long *>(acc_im);
    // and the carry accumulator: its words in acc_re, its counters in acc_im
    unsigned long long *const acc_w = reinterpret_cast<unsigned long long *>(acc_re);
    int *const c_word = reinterpret_cast<int *>(acc_im);
    __shared__ unsigned s_wmax[kBT / 64];
    __shared__ unsigned s_xmax[kBT / 64];
    // probe modes: the staged probe pair (z_a, z_b as two halves, exact for
    // 0 and +-1) and the sums of z (.) H z, one fixed-point integer per voxel
    // (the probe signs of the receiving voxel are applied to each
    // contribution, so the flush needs no signs)
    __shared__ uint32_t zq[PSIGNED ? XN : 1];
    __shared__ int acc_d[PSIGNED ? XN : 1];
    constexpr int WI = Win<MODE>::WI, ROWCAP = Win<MODE>::ROWCAP, RPT = Win<MODE>::RPT;
    constexpr int RUNCAP = Win<MODE>::RUNCAP + (QCARRY && !PROBE2 ? CSG_RUNCAP_CARRY_EXTRA : 0) +
                           (MODE == kBHvpProbe ? CSG_RUNCAP_PROBE_EXTRA : 0) -
                           (SHIFTED && MODE == kBGradient ? CSG_RUNCAP_SHIFT_CUT : 0);
    constexpr int RUN = Win<MODE>::RUN;
    __shared__ ImgSlot slot[WI];
    // the item's images: index (as int bits), rows 0 and 1 of R, defocus,
    // in-plane shift
    __shared__ float imgdat[CHUNK][IMGDAT];
    // row record: x = first run | len << 16 | image slot << 24,
    //             y = (kx0 + 32768) | (ky + 32768) << 16
    __shared__ int2 seg[ROWCAP];
    __shared__ __align__(8) unsigned short run2row[RUNCAP];
    // probe modes: the signs of the staged rows ([row][probe]; see
    // probe_row_mask) live only while a brick is staged, when the run table
    // is unused (barriers separate the two uses)
    static_assert(!PSIGNED || RUNCAP * sizeof(unsigned short) >= BX * BX * 2 * sizeof(uint32_t), "run table too small");
    uint32_t(*const s_zmask)[2] = reinterpret_cast<uint32_t(*)[2]>(run2row);
    __shared__ int wave_sums[kBT / 64];
    __shared__ int s_item;
    __shared__ double red[16];

    const Geom &g = a.g;
    const int M = g.M;
    const int total = *a.n_items;
    const int per_item = *a.per_item;  // chunks per work item (from the plan)
    double lsum = 0.0;
    double fxS = 1.0;
    if (FX) fxS = fx_scale(a.fx_max, a.scale, a.n_total).S;
    // the block's largest |re| + |im| of image values so far (float bits with
    // the sign cleared, which order like the values and keep a NaN), started
    // from a sample of disk pixels: per thread one of the 5 x 5 lowest
    // frequencies (where the largest values of a Fourier-space image sit) of
    // one image and one pixel spread over the disk of another
    // (in LDS, to keep registers for the pixel loop: s_xseen is thread 0's,
    // s_guess the item's guess, written by thread 0 and read after a barrier)
    __shared__ unsigned s_xseen, s_guess;
    if (XRETRY) {
        int rr = (int)sqrtf(0.5f * (float)g.k2max);  // |kx|, |ky| <= rr lies in the disk
        while (rr > 0 && 2 * rr * rr > g.k2max) --rr;
        const int side = 2 * rr + 1, t = (int)threadIdx.x;
        const int rc = min(rr, 2), sc = 2 * rc + 1;
        const int cx = t % sc - rc, cy = (t / sc) % sc - rc;
        const int kx = (t * 13 + (int)blockIdx.x) % side - rr, ky = (t * 7 + 3 * (int)blockIdx.x) % side - rr;
        const int64_t i0 = ((int64_t)blockIdx.x * (kBT / (sc * sc) + 1) + t / (sc * sc)) % a.n;
        const int64_t i1 = ((int64_t)blockIdx.x * kBT + t) % a.n;
        const float2 u = a.img[(i0 * M + (cy + g.half)) * (int64_t)M + (cx + g.half)];
        const float2 v = a.img[(i1 * M + (ky + g.half)) * (int64_t)M + (kx + g.half)];
        unsigned b = max(__float_as_uint(fabsf(u.x) + fabsf(u.y)) & 0x7fffffffu,
                         __float_as_uint(fabsf(v.x) + fabsf(v.y)) & 0x7fffffffu);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) b = max(b, (unsigned)__shfl_xor((int)b, off, 64));
        if ((threadIdx.x & 63) == 0) s_wmax[threadIdx.x >> 6] = b;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned m = 0u;
            for (int w = 0; w < kBT / 64; ++w) m = max(m, s_wmax[w]);
            s_xseen = m;
        }
    }

    // work items are taken from the planned list (heaviest first) until it
    // is exhausted
    for (;;) {
        // the previous item is done with every LDS table and accumulator
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(a.next_item, 1);
        __syncthreads();
        // uniform values read from LDS are moved to scalar registers
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= total) break;
        // an item is a brick and up to per_item chunks of CHUNK of its images:
        // images first0 .. last - 1 of its list
        const int2 rec = a.items[item];
        const int brick = rec.x & 0xFFFFF;
        const int count = rec.y;
        const int first0 = (rec.x >> 20) * CHUNK;
        const int last = min(count, first0 + per_item * CHUNK);
        int o[3];
        brick_origin(brick, a.nbx, o);

        const int *list = a.lists + (int64_t)brick * a.stride;
        // a chunk's images are staged in LDS by threads t < n_img; the first
        // chunk's loads are issued together with the halo loads so that the
        // latencies overlap
        const bool holds_img = (int)threadIdx.x < min(CHUNK, last - first0);
        int my_ii = 0;
        if (holds_img) my_ii = list[first0 + threadIdx.x];
        if (GATHER || PSIGNED) {
            // the extended brick of the gathered volume; every load is issued
            // before the first LDS store
            constexpr int HALO = BX * BX * BX;
            constexpr int HPT = (HALO + kBT - 1) / kBT;
            float2 hv[GATHER ? HPT : 1];
            if constexpr (GATHER) {
#pragma unroll
                for (int k = 0; k < HPT; ++k) {
                    int t = threadIdx.x + k * kBT;
                    // recomputed per item instead of being kept live across
                    // the item loop, where the pixel loop's registers are
                    // short (kept live, these coordinates were spilled and
                    // reloaded from scratch memory per item)
                    asm volatile("" : "+v"(t));
                    const int hx = t % BX, hy = (t / BX) % BX, hz = t / (BX * BX);
                    const int qx = o[0] + hx, qy = o[1] + hy, qz = o[2] + hz;
                    hv[k] = make_float2(0.f, 0.f);
                    if (t < HALO && qx < M && qy < M && qz < M) hv[k] = a.src[((int64_t)qz * M + qy) * M + qx];
                }
            }
            if (PSIGNED) {
                // the probe pair is generated, not loaded: row masks (while
                // the volume's loads are in flight), then the values
                if ((int)threadIdx.x < 2 * BX * BX)
                    s_zmask[threadIdx.x >> 1][threadIdx.x & 1] = probe_row_mask(a, o, M, threadIdx.x >> 1, threadIdx.x & 1);
                __syncthreads();
#pragma unroll
                for (int k = 0; k < HPT; ++k) {
                    int t = threadIdx.x + k * kBT;
                    asm volatile("" : "+v"(t));
                    if (t < HALO) {
                        const int hx = t % BX, hy = (t / BX) % BX, hz = t / (BX * BX);
                        const float2 z = probe_value(s_zmask[t / BX], hx, a.probe_has_b);
                        zq[(hz * XR + hy) * XR + hx] = half_bits(z.x) | (half_bits(z.y) << 16);
                    }
                }
            }
            if constexpr (GATHER) {
#pragma unroll
                for (int k = 0; k < HPT; ++k) {
                    int t = threadIdx.x + k * kBT;
                    asm volatile("" : "+v"(t));
                    const int hx = t % BX, hy = (t / BX) % BX, hz = t / (BX * BX);
                    if (t < HALO) vh[(hz * XR + hy) * XR + hx] = hv[k];
                }
            }
            if constexpr (STAGE_MAX) {
                // bound on |z| over the staged brick (|re| + |im| >= modulus),
                // per wave; combined after the next barrier.  The maximum is
                // taken over the float bits with the sign cleared, which
                // order like the values and keep a NaN.
                unsigned zb = 0u;
#pragma unroll
                for (int k = 0; k < HPT; ++k)
                    zb = max(zb, __float_as_uint(fabsf(hv[k].x) + fabsf(hv[k].y)) & 0x7fffffffu);
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) zb = max(zb, (unsigned)__shfl_xor((int)zb, off, 64));
                if ((threadIdx.x & 63) == 0) s_wmax[threadIdx.x >> 6] = zb;
            }
        }
        // one image of a chunk into LDS (thread t: the chunk's image t)
        auto stage_image = [&](int ii) {
            float e[9];
#pragma unroll
            for (int d = 0; d < 6; ++d) e[d] = a.rot[(int64_t)ii * 9 + d];
            e[6] = a.defocus[ii];
            if (SHIFTED) {
                e[7] = a.shift[2 * ii];
                e[8] = a.shift[2 * ii + 1];
            }
            imgdat[threadIdx.x][0] = __int_as_float(ii);
#pragma unroll
            for (int d = 0; d < IMGDAT - 1; ++d) imgdat[threadIdx.x][1 + d] = e[d];
        };
        if (holds_img) stage_image(my_ii);
        if (SCATTER) {
            for (int t = threadIdx.x; t < XN; t += kBT) {
                if (ACC) {
                    acc_re[t] = 0.0;
                    if (t < XN_IM) acc_im[t] = 0.0;
                }
                if (PSIGNED) acc_d[t] = 0;
            }
        }
        // the probe modes' fixed-point scale: |z_a| + |z_b| <= 2 (1 without z_b)
        const PackedScale pk = PSIGNED ? PackedScale::make(fabsf(PROBE2 ? a.scale2 : a.scale) *
                                                           (a.probe_has_b ? 2.f : 1.f))
                                       : PackedScale{};
        QScale qs;       // likewise
        // the image-value guess of the item: twice the block's maximum so far
        // (the exponent raised by one, at most the largest float; a NaN or an
        // infinity stays and gives a NaN flush)
        if (XRETRY && threadIdx.x == 0) {
            const unsigned xs = s_xseen;
            s_guess = xs >= 0x7f800000u ? xs : min(xs + (1u << 23), 0x7f7fffffu);
        }
        // enumeration box (grid coordinates): the brick's pixels have floor(g)
        // in the brick
        float lo[3], hi[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            lo[d] = (float)o[d];
            hi[d] = (float)(o[d] + BS);
        }
        const float halff = (float)g.half;
        const double halfG = (double)g.half * 0x1p32;
        const int kymax = (int)floorf(sqrtf((float)g.k2max) + 1e-4f);
        const double ctfB = g.ctf_b * g.inv_s2 * g.inv_s2;
        const uint32_t MM = (uint32_t)M * (uint32_t)M;
        const uint32_t pix_off = (uint32_t)g.half * (uint32_t)M + (uint32_t)g.half;

        // flush: every voxel of the extended brick that lies in the grid is
        // added to HBM with global atomics (voxels that received nothing are
        // skipped)
        auto flush_voxels = [&]() {
            constexpr int NV = BX * BX * BX;
            for (int t = threadIdx.x; t < NV; t += kBT) {
                const int tx = t % BX, ty = (t / BX) % BX, tz = t / (BX * BX);
                const int li = (tz * XR + ty) * XR + tx;
                if (o[0] + tx >= M || o[1] + ty >= M || o[2] + tz >= M) continue;
                const int64_t gi = ((int64_t)(o[2] + tz) * M + (o[1] + ty)) * M + (o[0] + tx);
                if (FX) {
                    const unsigned long long qr = acc_qre[li], qi = acc_qim[li];
                    if (qr) atomicAdd(&a.fx[2 * gi], qr);
                    if (qi) atomicAdd(&a.fx[2 * gi + 1], qi);
                    continue;
                }
                if (QCARRY) {
                    long long R, I;
                    int c_lo, c_hi;
                    carry_counters(c_word[li], c_lo, c_hi);
                    carry_decode(acc_w[li], c_lo, c_hi, R, I);
                    if (!qs.ok) {
                        atomicAdd(&a.accum[gi].x, __builtin_nanf(""));
                        atomicAdd(&a.accum[gi].y, __builtin_nanf(""));
                    } else {
                        if (R) atomicAdd(&a.accum[gi].x, (float)((double)R * qs.invS));
                        if (I) atomicAdd(&a.accum[gi].y, (float)((double)I * qs.invS));
                    }
                    continue;
                }
                if (QITEM && MODE == kBSqDiag) {
                    const long long qr = (long long)acc_qre[li];
                    if (!qs.ok) atomicAdd(a.accum_real + gi, __builtin_nanf(""));
                    else if (qr) atomicAdd(a.accum_real + gi, (float)((double)qr * qs.invS));
                    continue;
                }
                if (QITEM) {
                    const long long qr = (long long)acc_qre[li], qi = (long long)acc_qim[li];
                    if (!qs.ok) {
                        atomicAdd(&a.accum[gi].x, __builtin_nanf(""));
                        atomicAdd(&a.accum[gi].y, __builtin_nanf(""));
                    } else {
                        if (qr) atomicAdd(&a.accum[gi].x, (float)((double)qr * qs.invS));
                        if (qi) atomicAdd(&a.accum[gi].y, (float)((double)qi * qs.invS));
                    }
                    continue;
                }
                const float re = (float)acc_re[li];
                if (MODE == kBSqDiag) {
                    if (re != 0.f) atomicAdd(a.accum_real + gi, re);
                } else {
                    const float im = (float)acc_im[li];
                    if (re != 0.f) atomicAdd(&a.accum[gi].x, re);
                    if (im != 0.f) atomicAdd(&a.accum[gi].y, im);
                }
            }
        };
        // probe modes: the sums of z (.) H z of one chunk into the diagonal,
        // cleared for the next chunk
        auto flush_probe = [&]() {
            constexpr int NV = BX * BX * BX;
            for (int t = threadIdx.x; t < NV; t += kBT) {
                const int tx = t % BX, ty = (t / BX) % BX, tz = t / (BX * BX);
                const int li = (tz * XR + ty) * XR + tx;
                const int q = acc_d[li];
                acc_d[li] = 0;
                if (o[0] + tx >= M || o[1] + ty >= M || o[2] + tz >= M) continue;
                const int64_t gi = ((int64_t)(o[2] + tz) * M + (o[1] + ty)) * M + (o[0] + tx);
                if (q) atomicAdd(a.accum_real + gi, (float)q * pk.invS);
            }
        };

        for (int attempt = 0;; ++attempt) {
            unsigned xmax_item = 0u;  // this thread's largest image value of the item
            // modes without a gathered value: the bound is known before the item
            // (features: C^2 w <= 1 and w <= 1; squared weights: |scale| C^2 w^2;
            // backproject: |scale| times the image guess, set in the first window)
            if (QITEM && !GATHER && !READS_IMG)
                qs = QScale::make(MODE == kBFeatures ? 1.0 : fabs((double)a.scale));
            for (int first = first0; first < last; first += CHUNK) {
                const int n_img = min(CHUNK, last - first);
                if (first > first0 || attempt > 0) {
                    // the chunk's images (the first chunk's were staged with the
                    // brick); every wave is done with the previous chunk's
                    __syncthreads();
                    if ((int)threadIdx.x < n_img) stage_image(list[first + threadIdx.x]);
                }
                for (int w0 = 0; w0 < n_img; w0 += WI) {
                    const int nw = min(WI, n_img - w0);
                    // every wave has finished with the previous window's tables
                    __syncthreads();
                    if (STAGE_MAX && w0 == 0) {
                        unsigned zbits = 0u;
#pragma unroll
                        for (int w = 0; w < kBT / 64; ++w) zbits = max(zbits, s_wmax[w]);
                        const float zb = __uint_as_float(__builtin_amdgcn_readfirstlane(zbits));
                        if (QITEM) {
                            const unsigned gb = __builtin_amdgcn_readfirstlane(s_guess);
                            const double xg = READS_IMG ? (double)__uint_as_float(gb) : 0.0;
                            qs = QScale::make(fabs((double)a.scale) * ((double)zb + xg));
                        }
                    }
                    if (QITEM && !GATHER && READS_IMG && w0 == 0)
                        qs = QScale::make(fabs((double)a.scale) *
                                             (double)__uint_as_float(__builtin_amdgcn_readfirstlane(s_guess)));
                    // ---- the window's images (one thread each): constants, first row,
                    // row count.  Image s owns row records s MAXROWS .. s MAXROWS +
                    // MAXROWS - 1 of the window; those past its row count stay empty.
                    const int t = (int)threadIdx.x;
                    if (t < nw) {
                        {
                            ImgSlot &S = slot[t];
                            const float *D = imgdat[w0 + t];
#pragma unroll
                            for (int d = 0; d < 3; ++d) {
                                S.E1[d] = rint_scaled(D[1 + d]);
                                S.E2[d] = rint_scaled(D[4 + d]);
                                S.E1i[d] = (int64_t)S.E1[d];
                            }
                            S.ctfA = g.ctf_a * (double)D[7] * g.inv_s2;
                            S.img_base = (uint32_t)__float_as_int(D[0]) * MM;
                            if (SHIFTED) {
                                S.sx = D[IMGDAT - 2];
                                S.sy = D[IMGDAT - 1];
                            }
                            // rows: range of e2 . (g - half) over the box
                            float ylo = 0.f, yhi = 0.f;
#pragma unroll
                            for (int d = 0; d < 3; ++d) {
                                const float u = D[4 + d] * (lo[d] - halff), w = D[4 + d] * (hi[d] - halff);
                                ylo += fminf(u, w);
                                yhi += fmaxf(u, w);
                            }
                            // range tests in floating point first, so only bounded values
                            // are converted
                            const float fl = fmaxf(ceilf(ylo - kClipEps), (float)-kymax);
                            const float fh = fminf(floorf(yhi + kClipEps), (float)kymax);
                            if (fl <= fh) {
                                S.ky_lo = (short)(int)fl;
                                S.nrows = (unsigned short)min((int)fh - (int)fl + 1, MAXROWS);
                            } else {
                                S.ky_lo = 0;
                                S.nrows = 0;
                            }
                        }
                    }

                    __syncthreads();
                    const int n_rows = nw * MAXROWS;
                    // ---- row intervals (kx range whose cells reach the box), runs per row
                    int rlen[RPT], rkx0[RPT], rky[RPT], rsl[RPT];
                    int myruns = 0;
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        const int r = threadIdx.x + k * kBT;
                        rlen[k] = 0;
                        rkx0[k] = 0;
                        rky[k] = 0;
                        rsl[k] = 0;
                        const int s = r / MAXROWS;
                        const int q = r - s * MAXROWS;
                        if (r < n_rows && q < (int)slot[s].nrows) {
                            const ImgSlot &S = slot[s];
                            const int ky = S.ky_lo + q;
                            const float *D = imgdat[w0 + s];
                            const float e1f[3] = {D[1], D[2], D[3]}, e2f[3] = {D[4], D[5], D[6]};
                            int x0, x1;
                            clip_row(e1f, e2f, halff, ky, lo, hi, x0, x1);
                            // the disk: |kx| <= floor(sqrt(k2max - ky^2))
                            const int rem = g.k2max - ky * ky;
                            int kxm = (int)sqrtf((float)max(rem, 0));
                            while ((kxm + 1) * (kxm + 1) <= rem) ++kxm;
                            while (kxm > 0 && kxm * kxm > rem) --kxm;
                            x0 = max(x0, -kxm);
                            x1 = min(x1, kxm);
                            if (rem >= 0 && x1 >= x0) {
                                rlen[k] = min(x1 - x0 + 1, MAXLEN);
                                rkx0[k] = x0;
                            }
                            rky[k] = ky;
                            rsl[k] = s;
                        }
                        myruns += (rlen[k] + RUN - 1) / RUN;
                    }
                    int T;
                    {
                        int p = block_exclusive_scan(myruns, wave_sums, &T);
                        T = __builtin_amdgcn_readfirstlane(T);
#pragma unroll
                        for (int k = 0; k < RPT; ++k) {
                            const int r = threadIdx.x + k * kBT;
                            if (r < n_rows)
                                seg[r] = make_int2(p | (rlen[k] << 16) | (rsl[k] << 24),
                                                   (rkx0[k] + 32768) | ((rky[k] + 32768) << 16));
                            p += (rlen[k] + RUN - 1) / RUN;
                        }
                    }

                    for (int wbase = 0; wbase < T; wbase += RUNCAP) {
                        // ---- run -> row table of this pass (each thread fills the runs
                        // of its own rows, read back from their records)
#pragma unroll
                        for (int k = 0; k < RPT; ++k) {
                            const int r = threadIdx.x + k * kBT;
                            if (r < n_rows) {
                                const int x = seg[r].x;
                                const int rs = x & 0xFFFF, nr = (((x >> 16) & 0xFF) + RUN - 1) / RUN;
                                const int b0 = max(rs, wbase), b1 = min(rs + nr, wbase + RUNCAP);
                                for (int q = b0; q < b1; ++q) run2row[q - wbase] = (unsigned short)r;
                            }
                        }
                        __syncthreads();
                        const int wend = min(T, wbase + RUNCAP);
                        for (int u = wbase + threadIdx.x; u < wend; u += kBT) {
                            const int2 rec = seg[run2row[u - wbase]];
                            const int rs = rec.x & 0xFFFF;
                            const int len = (rec.x >> 16) & 0xFF;
                            const ImgSlot &I = slot[(unsigned)rec.x >> 24];
                            const int kx0 = (rec.y & 0xFFFF) - 32768;
                            const int ky = (int)((unsigned)rec.y >> 16) - 32768;
                            const int j0 = (u - rs) * RUN;
                            const int kxs = kx0 + j0;
                            const int cnt = min(RUN, len - j0);
                            const uint32_t jrun = I.img_base + pix_off + (uint32_t)(ky * M) + (uint32_t)kxs;
                            // the run's image values are requested first, so that their
                            // latency overlaps the sample-point arithmetic (every pixel of
                            // a run lies in the disk, hence inside its image)
                            float2 xin[RUN];
#pragma unroll
                            for (int jj = 0; jj < RUN; ++jj) {
                                xin[jj] = make_float2(0.f, 0.f);
                                if (READS_IMG && a.img && jj < cnt) xin[jj] = a.img[jrun + jj];
                            }
                            // fixed-point sample point of the run's first pixel (exact)
                            int64_t G[3];
#pragma unroll
                            for (int d = 0; d < 3; ++d) {
                                const double gd = fma((double)kxs, I.E1[d], fma((double)ky, I.E2[d], halfG));
                                const double h = floor(gd * 0x1p-32);
                                const uint32_t l32 = (uint32_t)fma(-h, 0x1p32, gd);
                                G[d] = (int64_t)(((uint64_t)(uint32_t)(int)h << 32) | l32);
                            }
                            const int64_t E1i[3] = {I.E1i[0], I.E1i[1], I.E1i[2]};
                            const double ctfA = I.ctfA;
                            const int ky2 = ky * ky;
#pragma unroll
                            for (int jj = 0; jj < RUN; ++jj) {
                                if (jj < cnt) {
                                    int l[3];
                                    float t[3];
#pragma unroll
                                    for (int d = 0; d < 3; ++d) {
                                        l[d] = (int)(G[d] >> 32) - o[d];  // base corner relative to the brick
                                        t[d] = (float)(uint32_t)G[d] * 0x1p-32f;
                                    }
                                    const bool owned = (unsigned)l[0] < (unsigned)BS && (unsigned)l[1] < (unsigned)BS &&
                                                       (unsigned)l[2] < (unsigned)BS;
                                    if (owned) {
                                        const int kx = kxs + jj;
                                        float C = 1.0f;
                                        if (g.ctf_on) {
                                            const double k2 = (double)(kx * kx + ky2);
                                            const double turns = fma(fma(-ctfB, k2, ctfA), k2, g.phase0);
                                            C = -__builtin_amdgcn_sinf((float)(turns - rint(turns)));
                                        }
                                        const uint32_t j = jrun + (uint32_t)jj;
                                        const float wx[2] = {1.0f - t[0], t[0]};
                                        const float wy[2] = {1.0f - t[1], t[1]};
                                        const float wz[2] = {1.0f - t[2], t[2]};
                                        float2 acc = make_float2(0.f, 0.f);
                                        // index of the base corner in the extended brick; the
                                        // eight corners lie in it
                                        const int lb = (l[2] * XR + l[1]) * XR + l[0];
                                        // probe modes: the probe pair at the corners and P z
                                        uint32_t zc[PSIGNED ? 8 : 1];
                                        float2 pz = make_float2(0.f, 0.f);
                                        if (GATHER || PSIGNED) {
                                            // staged voxels outside the grid hold zeros, which
                                            // drops those corners
#pragma unroll
                                            for (int c = 0; c < 8; ++c) {
                                                const int ax = c & 1, ay = (c >> 1) & 1, az = (c >> 2) & 1;
                                                const float w = wx[ax] * wy[ay] * wz[az];
                                                if (GATHER) {
                                                    const float2 v = vh[lb + az * XP + ay * XR + ax];
                                                    acc.x = fmaf(w, v.x, acc.x);
                                                    acc.y = fmaf(w, v.y, acc.y);
                                                }
                                                if (PSIGNED) {
                                                    zc[c] = zq[lb + az * XP + ay * XR + ax];
                                                    pz.x = fmaf(w, half_lo(zc[c]), pz.x);
                                                    pz.y = fmaf(w, half_hi(zc[c]), pz.y);
                                                }
                                            }
                                        }
                                        // in-plane shift: T on the forward value, conj(T)
                                        // on the adjoint input
                                        float2 T = make_float2(1.f, 0.f);
                                        if (SHIFTED) {
                                            const double tt = -((double)kx * (double)I.sx + (double)ky * (double)I.sy) /
                                                              (double)M;
                                            const float fr = (float)(tt - rint(tt));
                                            T = make_float2(__builtin_amdgcn_cosf(fr), __builtin_amdgcn_sinf(fr));
                                            if (GATHER) acc = cmul(acc, T);
                                        }
                                        float2 val = make_float2(0.f, 0.f);
                                        if (MODE == kBProject) {
                                            float2 y = make_float2(C * acc.x, C * acc.y);
                                            if (a.img) {
                                                y.x -= xin[jj].x;
                                                y.y -= xin[jj].y;
                                            }
                                            if (a.out) a.out[j] = y;
                                            lsum += 0.5 * ((double)y.x * y.x + (double)y.y * y.y);
                                        }
                                        if (XRETRY) {
                                            const float xa = fabsf(xin[jj].x) + fabsf(xin[jj].y);
                                            xmax_item = max(xmax_item, __float_as_uint(xa) & 0x7fffffffu);
                                        }
                                        if (MODE == kBBackproject) {
                                            const float2 x = cmul_conj(xin[jj], T);
                                            const float fct = a.scale * ctf_pow(C, a.ctf_power);
                                            val = make_float2(fct * x.x, fct * x.y);
                                        } else if (is_grad(MODE)) {
                                            const float2 x = xin[jj];
                                            const float2 rr = make_float2(fmaf(C, acc.x, -x.x), fmaf(C, acc.y, -x.y));
                                            lsum += 0.5 * ((double)rr.x * rr.x + (double)rr.y * rr.y);
                                            const float fct = a.scale * C;
                                            const float2 rt = cmul_conj(rr, T);
                                            val = make_float2(fct * rt.x, fct * rt.y);
                                        } else if (MODE == kBHvp) {
                                            const float fct = a.scale * C * C;
                                            val = make_float2(fct * acc.x, fct * acc.y);
                                        } else if (MODE == kBFeatures) {
                                            val = make_float2(C * C, 1.0f);
                                        } else if (MODE == kBSqDiag) {
                                            val = make_float2(a.scale * C * C, 0.0f);
                                        }
                                        if (QCARRY) {
                                            // the packed atomics of CARRY_GROUP corners, then one
                                            // look at their old words (see CarryScale)
                                            const float2 vs = make_float2(val.x * qs.S, val.y * qs.S);
                                            // corner (ax, ayz): (wx vs) times (wy wz)
                                            const float ur[2] = {wx[0] * vs.x, wx[1] * vs.x};
                                            const float ui[2] = {wx[0] * vs.y, wx[1] * vs.y};
                                            const float wyz[4] = {wy[0] * wz[0], wy[1] * wz[0], wy[0] * wz[1],
                                                                  wy[1] * wz[1]};
#pragma unroll
                                            for (int c0 = 0; c0 < 8; c0 += CARRY_GROUP) {
                                                unsigned long long old[CARRY_GROUP];
#pragma unroll
                                                for (int k = 0; k < CARRY_GROUP; ++k) {
                                                    const int c = c0 + k;
                                                    const int ax = c & 1, ay = (c >> 1) & 1, az = (c >> 2) & 1;
                                                    const int li = lb + az * XP + ay * XR + ax;
                                                    old[k] = atomicAdd(&acc_w[li],
                                                                       carry_pack(round_half_up(ur[ax] * wyz[c >> 1]),
                                                                                  round_half_up(ui[ax] * wyz[c >> 1])));
                                                }
                                                uint32_t f = 0u;
#pragma unroll
                                                for (int k = 0; k < CARRY_GROUP; ++k) f |= carry_may_wrap(old[k]);
                                                if ((int)f < 0) {
#pragma unroll
                                                    for (int k = 0; k < CARRY_GROUP; ++k) {
                                                        const int c = c0 + k;
                                                        const int ax = c & 1, ay = (c >> 1) & 1, az = (c >> 2) & 1;
                                                        const int li = lb + az * XP + ay * XR + ax;
                                                        carry_fix(old[k], round_half_up(ur[ax] * wyz[c >> 1]),
                                                                  round_half_up(ui[ax] * wyz[c >> 1]), c_word + li);
                                                    }
                                                }
                                            }
                                        } else if (ACC) {
                                            // all eight corners; a corner beyond the grid edge
                                            // lands in a slot that is never written back
#pragma unroll
                                            for (int c = 0; c < 8; ++c) {
                                                const int ax = c & 1, ay = (c >> 1) & 1, az = (c >> 2) & 1;
                                                const float w = wx[ax] * wy[ay] * wz[az];
                                                const int li = lb + az * XP + ay * XR + ax;
                                                if (MODE == kBSqDiag && QLDS) {
                                                    atomicAdd(&acc_qre[li], fx_quant(w * w * val.x, qs.S));
                                                } else if (MODE == kBSqDiag) {
                                                    atomicAdd(&acc_re[li], (double)(w * w * val.x));
                                                } else if (QLDS) {
                                                    const double S = FX ? fxS : qs.S;
                                                    atomicAdd(&acc_qre[li], fx_quant(w * val.x, S));
                                                    atomicAdd(&acc_qim[li], fx_quant(w * val.y, S));
                                                } else {
                                                    atomicAdd(&acc_re[li], (double)(w * val.x));
                                                    atomicAdd(&acc_im[li], (double)(w * val.y));
                                                }
                                            }
                                        }
                                        if (PSIGNED && attempt == 0) {
                                            // probe modes (in the fused mode after the
                                            // gradient's atomics): the probe pair's product
                                            // scale C^2 P z at this pixel; corner c receives
                                            // w_c (z_a(c) re + z_b(c) im) of z (.) H z, one
                                            // fixed-point integer (the bound of PackedScale); a
                                            // retried item (attempt > 0) has its probe sums
                                            // flushed already
                                            const float fz = (PROBE2 ? a.scale2 : a.scale) * C * C;
                                            const float px = fz * pz.x * pk.S, py = fz * pz.y * pk.S;
#pragma unroll
                                            for (int c = 0; c < 8; ++c) {
                                                const int ax = c & 1, ay = (c >> 1) & 1, az = (c >> 2) & 1;
                                                const float w = wx[ax] * wy[ay] * wz[az];
                                                const float d = fmaf(half_lo(zc[c]), px, half_hi(zc[c]) * py);
                                                atomicAdd(&acc_d[lb + az * XP + ay * XR + ax], round_half_up(w * d));
                                            }
                                        }
                                    }
                                }
#pragma unroll
                                for (int d = 0; d < 3; ++d) G[d] += E1i[d];
                            }
                        }
                        __syncthreads();  // the table is rebuilt (and, after the last pass, the window)
                    }
                }
                // the probe modes' 32-bit sums hold one chunk (see PackedScale)
                if (PSIGNED && attempt == 0) flush_probe();
            }  // chunks
            if (!XRETRY) break;
            // the item's largest image value; above the guess, a fixed-point sum
            // may have overflowed, and the item is redone with that maximum as
            // its bound (which no value of the item can exceed, so once at most)
            {
                unsigned m = xmax_item;
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off, 64));
                if ((threadIdx.x & 63) == 0) s_xmax[threadIdx.x >> 6] = m;
                const unsigned guess = __builtin_amdgcn_readfirstlane(s_guess);  // read before thread 0 may change it
                __syncthreads();
                unsigned im = 0u;
#pragma unroll
                for (int w = 0; w < kBT / 64; ++w) im = max(im, s_xmax[w]);
                im = __builtin_amdgcn_readfirstlane(im);
                if (threadIdx.x == 0) s_xseen = max(s_xseen, im);
                if (im <= guess || attempt > 0) {
                    // the item's loss terms, added once the item is accepted
                    if (is_grad(MODE) && a.loss) {
                        const double t = block_sum(lsum, red);
                        if (threadIdx.x == 0 && t != 0.0) atomicAdd(a.loss, t);
                    }
                    lsum = 0.0;
                    break;
                }
                if (threadIdx.x == 0) s_guess = im;  // read after the next window's barrier
                lsum = 0.0;
                for (int t = threadIdx.x; t < XN; t += kBT) {
                    acc_re[t] = 0.0;
                    if (t < XN_IM) acc_im[t] = 0.0;
                }
            }
        }  // attempts

        if (ACC) {
            __syncthreads();
            flush_voxels();
        }
    }  // work items

    // (the gradient with the retry adds its loss per item)
    if ((MODE == kBProject || (is_grad(MODE) && !XRETRY)) && a.loss) {
        const double t = block_sum(lsum, red);
        if (threadIdx.x == 0 && t != 0.0) atomicAdd(a.loss, t);
    }
}

// Zero the pixels outside the disk (the brick kernels write only the disk).
// One wave per image row: it stores the columns left and right of the row's
// disk interval (the whole row where the disk does not reach it).
__global__ __launch_bounds__(kBlock) void zero_outside_disk_kernel(float2 *out, int64_t n, int M, int half,
                                                                    int k2max) {
    const int64_t rows = n * (int64_t)M;
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t row = wave; row < rows; row += waves) {
        const int ky = (int)(row % M) - half;
        const int rem = k2max - ky * ky;
        int left = M, right = M;  // columns [0, left) and [right, M) are outside
        if (rem >= 0) {
            int kxm = (int)sqrtf((float)rem);
            while ((kxm + 1) * (kxm + 1) <= rem) ++kxm;
            while (kxm > 0 && kxm * kxm > rem) --kxm;
            left = half - kxm;
            right = half + kxm + 1;
        }
        float2 *p = out + row * M;
        for (int x = lane; x < left; x += 64) p[x] = make_float2(0.f, 0.f);
        for (int x = right + lane; x < M; x += 64) p[x] = make_float2(0.f, 0.f);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int brick_count(int M) {
    const int nbx = (M + BS - 1) / BS;
    return nbx * nbx * nbx;
}

// Workspace of the brick kernels for a batch of n images (256-byte aligned
// regions): per-brick image counts, per-brick image lists of one sub-batch,
// the work items of one launch, and the three work-list scalars.
static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static size_t brick_items_cap(int M, int64_t sub) {
    const int64_t per = (sub + CHUNK_FWD - 1) / CHUNK_FWD;  // the smallest chunk gives the most items
    return (size_t)brick_count(M) * (size_t)(per > 0 ? per : 1);
}

// (sub = images per launch: the sub-batch the per-brick lists hold)
size_t brick_workspace_bytes_sub(int M, int64_t sub) {
    const size_t nb = (size_t)brick_count(M);
    return align256(nb * 4) + align256(nb * (size_t)(sub > 0 ? sub : 1) * 4) + align256(brick_items_cap(M, sub) * 8) +
           256;
}

size_t brick_workspace_bytes(int M, int64_t n) {
    return brick_workspace_bytes_sub(M, n < kBrickSubBatch ? n : kBrickSubBatch);
}

// Resident blocks of one brick-kernel mode on the current device (one wave
// of blocks that then fetch work items until the list is exhausted).
template <int MODE, bool FX>
static int resident_blocks() {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, brick_kernel<MODE, false, FX>, kBT, 0) != hipSuccess || per <= 0)
        per = 1;
    return cus * per;
}

// The Rademacher probe pair of the probe HVP mode (seed, pa, pb, has_b) and,
// in the fused gradient and probe mode, the factor of its product.
struct ProbePair {
    uint64_t seed, pa, pb;
    int has_b;
    float scale = 0.f;
};

template <int MODE, bool FX = false>
static hipError_t run_brick_mode(const Geom &g, const float *rot, const float *defocus, const float *shift, int64_t n,
                                 const float2 *src, const float2 *img, float2 *out, float2 *accum, double *loss,
                                 float scale, int ctf_power, void *ws, hipStream_t st, float *accum_real = nullptr,
                                 const FxBuf *fb = nullptr, const ProbePair *probe = nullptr,
                                 int64_t sub_cap = kBrickSubBatch, bool timed = true) {
    const int M = g.M;
    const int nbx = (M + BS - 1) / BS;
    const int nb = nbx * nbx * nbx;
    if (sub_cap < 1 || sub_cap > kBrickSubBatch) sub_cap = kBrickSubBatch;
    const int64_t sub = n < sub_cap ? n : sub_cap;
    char *w = (char *)ws;
    int *counts = (int *)w;
    w += align256((size_t)nb * 4);
    int *lists = (int *)w;
    w += align256((size_t)nb * (size_t)sub * 4);
    int2 *items = (int2 *)w;
    w += align256(brick_items_cap(M, sub) * 8);
    int *scalars = (int *)w;  // [0] number of work items, [1] work counter, [2] chunks per item
    const int64_t img_stride = (int64_t)M * M;
    constexpr int chunk = MODE == kBProject ? CHUNK_FWD : CHUNK_ADJ;
    const int64_t max_items = (int64_t)nb * ((sub + chunk - 1) / chunk);
    const int grid = (int)(resident_blocks<MODE, FX>() < max_items ? resident_blocks<MODE, FX>() : max_items);
    for (int64_t s0 = 0; s0 < n; s0 += sub) {
        const int64_t ns = (n - s0) < sub ? (n - s0) : sub;
        const int stride = (int)ns;
        hipLaunchKernelGGL(brick_cull_kernel, dim3((unsigned)((nb + kCullWaves - 1) / kCullWaves)), dim3(kCullThreads), 0,
                           st, g, rot + s0 * 9, ns, nbx, nb, counts, lists, stride);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        // at least two items per resident block
        hipLaunchKernelGGL(brick_plan_kernel, dim3(1), dim3(kPlanThreads), 0, st, counts, nb, chunk,
                           max_chunks_per_item(MODE), 2 * grid, items, scalars, scalars + 1, scalars + 2);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        BrickArgs a{};
        a.g = g;
        a.rot = rot + s0 * 9;
        a.defocus = defocus + s0;
        a.shift = shift ? shift + s0 * 2 : nullptr;
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
        a.items = items;
        a.n_items = scalars;
        a.next_item = scalars + 1;
        a.per_item = scalars + 2;
        if (FX) {
            a.fx = fb->fx;
            a.fx_max = fb->maxbits;
            a.n_total = n;
        }
        if (probe) {
            a.probe_seed = probe->seed;
            a.probe_a = probe->pa;
            a.probe_b = probe->pb;
            a.probe_has_b = probe->has_b;
            a.scale2 = probe->scale;
        }
        // the probe HVP is timed with the HVP, the fused mode under index 6
        constexpr int TMODE = MODE == kBHvpProbe ? kBHvp : MODE == kBGradProbe ? kTimedGradProbe : MODE;
        hipEvent_t t0 = timed ? timing_begin(TMODE, st) : nullptr;
        if constexpr (MODE == kBGradProbe) {
            hipLaunchKernelGGL((brick_kernel<MODE, false, FX>), dim3((unsigned)grid), dim3(kBT), 0, st, a);
        } else {
            if (shift)
                hipLaunchKernelGGL((brick_kernel<MODE, true, FX>), dim3((unsigned)grid), dim3(kBT), 0, st, a);
            else
                hipLaunchKernelGGL((brick_kernel<MODE, false, FX>), dim3((unsigned)grid), dim3(kBT), 0, st, a);
        }
        e = hipGetLastError();
        timing_end(TMODE, t0, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The brick kernels implement trilinear interpolation; nearest-neighbour
// grids (the exact-pin mode of Sec. 3.1) use the pixel-parallel kernels.
hipError_t launch_brick_project(const Geom &g, const float *rot, const float *defocus, const float *shift, int64_t n,
                                const float2 *vol, const float2 *subtract, float2 *out, double *loss, void *ws,
                                hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_project(g, rot, defocus, shift, n, vol, subtract, out, loss, st);
    hipError_t e = run_brick_mode<kBProject>(g, rot, defocus, shift, n, vol, subtract, out, nullptr, loss, 1.0f, 0, ws,
                                             st);
    if (e != hipSuccess || !out) return e;
    int64_t blocks = (n * (int64_t)g.M + 3) / 4;  // four waves (rows) per block
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(zero_outside_disk_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, st, out, n, g.M, g.half,
                       g.k2max);
    return hipGetLastError();
}

hipError_t launch_brick_backproject(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                    int64_t n, const float2 *img, int ctf_power, float scale, float2 *accum,
                                    void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_backproject_atomic(g, rot, defocus, shift, n, img, ctf_power, scale, accum, st);
    return run_brick_mode<kBBackproject>(g, rot, defocus, shift, n, nullptr, img, nullptr, accum, nullptr, scale,
                                         ctf_power, ws, st);
}

hipError_t launch_brick_gradient(const Geom &g, const float *rot, const float *defocus, const float *shift, int64_t n,
                                 const float2 *vol, const float2 *x, float scale, float2 *accum, double *loss,
                                 void *ws, hipStream_t st, int64_t sub_cap, bool timed) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_gradient_atomic(g, rot, defocus, shift, n, vol, x, scale, accum, loss, st);
    return run_brick_mode<kBGradient>(g, rot, defocus, shift, n, vol, x, nullptr, accum, loss, scale, 1, ws, st,
                                      nullptr, nullptr, nullptr, sub_cap, timed);
}

hipError_t launch_brick_feature_sums(const Geom &g, const float *rot, const float *defocus, int64_t n,
                                     float2 *accum, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return hipErrorInvalidValue;  // trilinear stencils only
    return run_brick_mode<kBFeatures>(g, rot, defocus, nullptr, n, nullptr, nullptr, nullptr, accum, nullptr, 1.0f, 0,
                                      ws, st);
}

hipError_t launch_brick_sq_diag(const Geom &g, const float *rot, const float *defocus, int64_t n, float scale,
                                float *diag, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_sq_diag(g, rot, defocus, n, scale, diag, st);
    return run_brick_mode<kBSqDiag>(g, rot, defocus, nullptr, n, nullptr, nullptr, nullptr, nullptr, nullptr, scale, 2,
                                    ws, st, diag);
}

hipError_t launch_brick_hvp(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *z,
                            float scale, float2 *accum, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return launch_hvp_atomic(g, rot, defocus, n, z, scale, accum, st);
    return run_brick_mode<kBHvp>(g, rot, defocus, nullptr, n, z, nullptr, nullptr, accum, nullptr, scale, 2, ws, st);
}

// Gradient (as launch_brick_gradient, no in-plane shifts) and the probe
// pair's z (.) scale2 P^T C^2 P z added to diag, in one pass over the pixels.
hipError_t launch_brick_gradient_probe(const Geom &g, const float *rot, const float *defocus, int64_t n,
                                       const float2 *vol, const float2 *x, float scale, float2 *accum, double *loss,
                                       uint64_t seed, uint64_t pa, uint64_t pb, int has_b, float scale2, float *diag,
                                       void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return hipErrorInvalidValue;  // trilinear stencils only
    const ProbePair pp{seed, pa, pb, has_b, scale2};
    return run_brick_mode<kBGradProbe>(g, rot, defocus, nullptr, n, vol, x, nullptr, accum, loss, scale, 1, ws, st,
                                       diag, nullptr, &pp);
}

hipError_t launch_brick_hvp_probe(const Geom &g, const float *rot, const float *defocus, int64_t n, uint64_t seed,
                                  uint64_t pa, uint64_t pb, int has_b, float scale, float *diag, void *ws,
                                  hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return hipErrorInvalidValue;  // the pixel kernels read a stored probe
    const ProbePair pp{seed, pa, pb, has_b};
    return run_brick_mode<kBHvpProbe>(g, rot, defocus, nullptr, n, nullptr, nullptr, nullptr, nullptr, nullptr, scale, 2,
                                      ws, st, diag, nullptr, &pp);
}

// Deterministic adjoint: input bounds and a zeroed fixed-point volume, the
// fixed-point brick kernel, then one conversion pass that adds the volume to
// the float target.
hipError_t launch_brick_backproject_fx(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                       int64_t n, const float2 *img, int ctf_power, float scale, float2 *accum,
                                       const FxBuf &fb, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return hipErrorInvalidValue;  // trilinear stencils only
    const int64_t nv = (int64_t)g.M * g.M * g.M;
    hipError_t e = launch_fx_prep(nullptr, 0, fb.maxbits, fb.fx, nv, st);
    if (e == hipSuccess) e = launch_img_absmax(g, img, n, fb.maxbits, st);
    if (e != hipSuccess) return e;
    e = run_brick_mode<kBBackproject, true>(g, rot, defocus, shift, n, nullptr, img, nullptr, accum, nullptr, scale,
                                            ctf_power, ws, st, nullptr, &fb);
    if (e != hipSuccess) return e;
    return launch_fx_finish(accum, fb.fx, nv, fb.maxbits, scale, n, st);
}

hipError_t launch_brick_gradient_fx(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                    int64_t n, const float2 *vol, const float2 *x, float scale, float2 *accum,
                                    double *loss, const FxBuf &fb, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return hipErrorInvalidValue;
    const int64_t nv = (int64_t)g.M * g.M * g.M;
    hipError_t e = launch_fx_prep(vol, nv, fb.maxbits, fb.fx, nv, st);
    if (e == hipSuccess) e = launch_img_absmax(g, x, n, fb.maxbits + 1, st);
    if (e != hipSuccess) return e;
    e = run_brick_mode<kBGradient, true>(g, rot, defocus, shift, n, vol, x, nullptr, accum, loss, scale, 1, ws, st,
                                         nullptr, &fb);
    if (e != hipSuccess) return e;
    return launch_fx_finish(accum, fb.fx, nv, fb.maxbits, scale, n, st);
}

hipError_t launch_brick_hvp_fx(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *z,
                               float scale, float2 *accum, const FxBuf &fb, void *ws, hipStream_t st) {
    if (n == 0) return hipSuccess;
    if (g.interp == 0) return hipErrorInvalidValue;
    const int64_t nv = (int64_t)g.M * g.M * g.M;
    hipError_t e = launch_fx_prep(z, nv, fb.maxbits, fb.fx, nv, st);
    if (e != hipSuccess) return e;
    e = run_brick_mode<kBHvp, true>(g, rot, defocus, nullptr, n, z, nullptr, nullptr, accum, nullptr, scale, 2, ws, st,
                                    nullptr, &fb);
    if (e != hipSuccess) return e;
    return launch_fx_finish(accum, fb.fx, nv, fb.maxbits, scale, n, st);
}

}  // namespace csg
