// mlp_kernels.hip -- the per-voxel preconditioner network: inference and
// training (forward, backward, Adam).  MLP 3 -> 64 -> 64 -> 1 with GELU;
// weights are float32 masters rounded to bfloat16 when used, layer inputs
// are rounded to bfloat16, products accumulate in float32.  The 64 x 64
// layer and the two GEMMs of its backward pass run on the matrix cores
// (v_mfma_f32_32x32x8_bf16): one wavefront handles a tile of 32 samples.
//
// MFMA 32x32x8 operand layout (wave64), lane l = 32 h + c:
//   A (32 x 8):  lane l holds A[c][4h + q], q = 0..3
//   B (8 x 32):  lane l holds B[4h + q][c]
//   D (32 x 32): lane l holds D[8 (r/4) + 4h + (r%4)][c] in register r = 0..15
//
// Parameter vector (float32): W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3.
#include <math.h>

#include "csg_device.h"
#include "csg_internal.h"

namespace csg {

constexpr int H = 64;
// LDS row stride (bfloat16 entries) of the staged W2 and of the tile copies
// read along rows: 68 entries = 34 words, so the 8-byte reads of 32 lanes
// from 32 consecutive rows fall into distinct bank pairs (a stride of 64
// entries would put all of them into one bank)
constexpr int W2S = H + 4;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + 3 * H, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
              OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H, NPARAM = OFF_B3 + 1;

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return (unsigned short)(u >> 16);  // inf / nan
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float bfr(float f) { return bf2f(f2bf(f)); }

// The normal distribution function Phi(x) = (1 + erf(x / sqrt 2)) / 2 from
// the erfc approximation of Abramowitz & Stegun, Handbook of Mathematical
// Functions, formula 7.1.26 (Hastings): erfc(u) = t (a1 + t (a2 + t (a3 + t (a4 +
// t a5)))) exp(-u^2), t = 1 / (1 + p u), u >= 0, absolute error below 1.5e-7;
// Phi(x) = 1 - erfc(|x| / sqrt 2) / 2 for x >= 0 and erfc(|x| / sqrt 2) / 2
// below (no cancellation in the lower tail).  Branch-free; the hardware
// reciprocal and exponential are accurate to about one ulp, far below the
// bfloat16 rounding that follows every activation.  *pdf receives
// phi(x) = exp(-x^2 / 2) / sqrt(2 pi).
// (constants: p / sqrt 2, a_i / 2, and -log2(e) / 2 for exp(-x^2 / 2) = 2^(c x^2))
__device__ __forceinline__ float half_erfc_scaled(float x, float *e_out) {
    const float t = __builtin_amdgcn_rcpf(fmaf(0.23164188827f, fabsf(x), 1.0f));
    const float poly =
        t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 0.5307027145f, -0.7265760135f), 0.7107068705f), -0.142248368f),
                 0.127414796f);
    const float e = __builtin_amdgcn_exp2f(x * x * -0.72134752044448170f);
    *e_out = e;
    return poly * e;  // erfc(|x| / sqrt 2) / 2
}
__device__ __forceinline__ float normal_cdf(float x, float *pdf) {
    float e;
    const float h = half_erfc_scaled(x, &e);
    if (pdf) *pdf = e * 0.39894228040143268f;
    return x >= 0.f ? 1.0f - h : h;
}
// x Phi(x): x - x h above zero, x h below
__device__ __forceinline__ float gelu(float x) {
    float e;
    const float xh = x * half_erfc_scaled(x, &e);
    return x >= 0.f ? x - xh : xh;
}
__device__ __forceinline__ float gelu_grad(float x) {
    float pdf;
    const float c = normal_cdf(x, &pdf);
    return fmaf(x, pdf, c);
}

// Two floats to bfloat16 (round to nearest even, v_cvt_pk_bf16_f32): the
// low half holds a, the high half b.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pack2(float a, float b) {
    const f32x2_t f = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2_t));
}

// Parameters staged in LDS for a block.
struct MlpShared {
    unsigned short w2[H * W2S];  // bf16 W2[j][k] at j W2S + k
    float w1[H * 3];           // bf16-rounded W1
    float b1[H];
    float b2[H];
    float w3[H];               // bf16-rounded W3
    float b3;
    float4 l1[H];              // unit k of layer 1: (W1[k][0..2] bf16-rounded, b1[k])
};

__device__ void stage_params(const float *p, MlpShared &s) {
    for (int t = threadIdx.x; t < H * H; t += blockDim.x) s.w2[(t / H) * W2S + t % H] = f2bf(p[OFF_W2 + t]);
    for (int t = threadIdx.x; t < H * 3; t += blockDim.x) s.w1[t] = bfr(p[OFF_W1 + t]);
    for (int t = threadIdx.x; t < H; t += blockDim.x) {
        s.b1[t] = p[OFF_B1 + t];
        s.b2[t] = p[OFF_B2 + t];
        s.w3[t] = bfr(p[OFF_W3 + t]);
    }
    if (threadIdx.x == 0) s.b3 = p[OFF_B3];
    for (int t = threadIdx.x; t < H; t += blockDim.x)
        s.l1[t] = make_float4(bfr(p[OFF_W1 + 3 * t]), bfr(p[OFF_W1 + 3 * t + 1]), bfr(p[OFF_W1 + 3 * t + 2]),
                              p[OFF_B1 + t]);
}

// Layer 1 for the lane's sample and its 32 hidden units k = 8 st + 4 h + q;
// returns the bf16 A operands of layer 2 and (optionally) the pre-activations.
__device__ __forceinline__ void layer1(const MlpShared &s, const float x0[3], int hh, s16x4 a[8], float *z1) {
#pragma unroll
    for (int st = 0; st < 8; ++st) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = 8 * st + 4 * hh + q;
            const float z = fmaf(s.w1[k * 3 + 2], x0[2], fmaf(s.w1[k * 3 + 1], x0[1], fmaf(s.w1[k * 3], x0[0], s.b1[k])));
            if (z1) z1[st * 4 + q] = z;
            a[st][q] = (short)f2bf(gelu(z));
        }
    }
}

// Layer 2: D_nb = H1 (32 x 64) . W2^T restricted to output columns 32 nb + c.
__device__ __forceinline__ void layer2(const MlpShared &s, const s16x4 a[8], int hh, int c, f32x16 &acc0,
                                       f32x16 &acc1) {
    acc0 = f32x16{0.f};
    acc1 = f32x16{0.f};
#pragma unroll
    for (int st = 0; st < 8; ++st) {
        const int k = 8 * st + 4 * hh;
        s16x4 b0, b1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            b0[q] = (short)s.w2[c * W2S + k + q];
            b1[q] = (short)s.w2[(32 + c) * W2S + k + q];
        }
        acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a[st], b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a[st], b1, acc1, 0, 0, 0);
    }
}

// Sum over the 32 lanes of one half-wave (lanes with the same l / 32).
__device__ __forceinline__ float half_sum(float v) {
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Inputs of one voxel for the fused (volume) mode: |k| / (M/2),
// log(ctf2 M / N), log(cover M / N) (the chance that an image reaches a voxel
// at a given fraction of the maximum radius falls like 1/M, so the M / N
// scaling makes the inputs comparable across grid sizes); returns false for
// voxels no image reaches.
__device__ __forceinline__ bool voxel_inputs(int64_t v, int M, float scale, const float *ctf2, const float *cover,
                                             float x0[3]) {
    const int half = M / 2;
    const int kx = (int)(v % M) - half, ky = (int)((v / M) % M) - half, kz = (int)(v / ((int64_t)M * M)) - half;
    const float cv = cover[v];
    x0[0] = sqrtf((float)(kx * kx + ky * ky + kz * kz)) / (float)half;
    x0[1] = logf(fmaxf(ctf2[v] * scale, 1e-30f));
    x0[2] = logf(fmaxf(cv * scale, 1e-30f));
    return cv > 0.f;
}

// One halving exchange of a reduction over lanes: the lane keeps the sums of
// values j (lower lanes of the pair, bit OFF of c clear) or j + K (upper) of
// its 2K values with its partner's.
template <int K, int OFF>
__device__ __forceinline__ void halve(float *v, int c) {
    const bool upper = (c & OFF) != 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float send = upper ? v[j] : v[j + K];
        const float keep = upper ? v[j + K] : v[j];
        v[j] = keep + __shfl_xor(send, OFF, 64);
    }
}

// The network on one tile of 32 samples, one wave: lane l = 32 h + c holds the
// (bfloat16-rounded) inputs of sample c.  Layer 1 is formed block by block of
// eight hidden units (the lane's four of them, 8 st + 4 h + q) and fed
// straight into the two 32 x 32 x 8 products of layer 2, so no layer-1
// activations are kept.  The output layer's dot products over the 64 units
// are reduced over the 32 lanes of each half-wave by halving exchanges (16,
// 8, 4, 2 values kept, then a pair sum).  Returns the output of sample
// 8 (r / 4) + 4 h + r % 4, r = c / 2, in every lane (lanes 2r and 2r + 1 agree).
struct TileConst {
    float b2a, b2b, w3a, w3b, b3;
};

__device__ __forceinline__ float mlp_tile(const MlpShared &s, const TileConst &tc, const float x0[3], int hh, int c) {
    f32x16 acc0 = f32x16{0.f}, acc1 = f32x16{0.f};
    // the weight reads are redone per tile rather than kept live across
    // tiles (which would need 160 more registers)
    int kh = 4 * hh;
    asm volatile("" : "+v"(kh));
#pragma unroll
    for (int st = 0; st < 8; ++st) {
        const int k = 8 * st + kh;
        float h[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float4 w = s.l1[k + q];
            h[q] = gelu(fmaf(w.z, x0[2], fmaf(w.y, x0[1], fmaf(w.x, x0[0], w.w))));
        }
        const uint32_t p01 = bf16_pack2(h[0], h[1]), p23 = bf16_pack2(h[2], h[3]);
        const s16x4 a = __builtin_bit_cast(s16x4, ((uint64_t)p23 << 32) | p01);
        const s16x4 b0 = *reinterpret_cast<const s16x4 *>(&s.w2[c * W2S + k]);
        const s16x4 b1 = *reinterpret_cast<const s16x4 *>(&s.w2[(32 + c) * W2S + k]);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b0, acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b1, acc1, 0, 0, 0);
    }
    // output layer: partial dot products of the lane's two units
    float v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const uint32_t hp = bf16_pack2(gelu(acc0[r] + tc.b2a), gelu(acc1[r] + tc.b2b));
        v[r] = fmaf(tc.w3a, __uint_as_float(hp << 16), tc.w3b * __uint_as_float(hp & 0xFFFF0000u));
    }
    // halving exchanges over lane bits 4 .. 1 of c, then the pair sum
    halve<8, 16>(v, c);
    halve<4, 8>(v, c);
    halve<2, 4>(v, c);
    halve<1, 2>(v, c);
    return v[0] + __shfl_xor(v[0], 1, 64) + tc.b3;
}

// sample index within its tile of the output that lane c holds
__device__ __forceinline__ int tile_out_index(int hh, int c) {
    const int r = c >> 1;
    return 8 * (r / 4) + 4 * hh + (r % 4);
}

__device__ __forceinline__ TileConst tile_const(const MlpShared &s, int c) {
    return TileConst{s.b2[c], s.b2[32 + c], s.w3[c], s.w3[32 + c], s.b3};
}

// y[s] = mlp(X[s]) for n samples, one wave per tile of 32.
__global__ __launch_bounds__(256, 2) void mlp_infer_kernel(const float *params, const float *X, float *y, int64_t n) {
    __shared__ MlpShared s;
    stage_params(params, s);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int hh = lane >> 5, c = lane & 31;
    const TileConst tc = tile_const(s, c);
    const int64_t ntiles = (n + 31) / 32;
#pragma unroll 1
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wv; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t smp = tile * 32 + c;
        float x0[3] = {0.f, 0.f, 0.f};
        if (smp < n) {
#pragma unroll
            for (int d = 0; d < 3; ++d) x0[d] = bfr(X[smp * 3 + d]);
        }
        const float out = mlp_tile(s, tc, x0, hh, c);
        const int64_t t = tile * 32 + tile_out_index(hh, c);
        if ((c & 1) == 0 && t < n) y[t] = out;
    }
}

// Over the M^3 voxels: D[v] = lambda + (N / M) exp(mlp(inputs(v))) where some
// image reaches v, else lambda.  One wave per grid row (fixed kz, ky; rows
// interleaved over the waves): the row's reached voxels span [x_first,
// x_last] (found with one ballot per 64 voxels of cover); the network runs
// on that span in tiles of 32, and the rest of the row is written lambda.
__global__ __launch_bounds__(256, 2) void learned_diag_kernel(const float *params, int M, float N, float lambda,
                                                             const float *ctf2, const float *cover, float *D) {
    __shared__ MlpShared s;
    stage_params(params, s);
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int hh = lane >> 5, c = lane & 31;
    const TileConst tc = tile_const(s, c);
    const float scale = (float)M / N;
    const int64_t rows = (int64_t)M * M;
#pragma unroll 1
    for (int64_t row = (int64_t)blockIdx.x * 4 + wv; row < rows; row += (int64_t)gridDim.x * 4) {
        const int64_t base = row * M;
        int x_first = M, x_last = -1;
        for (int xs = 0; xs < M; xs += 64) {
            const int x = xs + lane;
            const uint64_t m = __ballot(x < M && cover[base + x] > 0.f);
            if (m) {
                x_first = min(x_first, xs + (int)__builtin_ctzll(m));
                x_last = max(x_last, xs + 63 - (int)__builtin_clzll(m));
            }
        }
        x_first = __builtin_amdgcn_readfirstlane(x_first);
        x_last = __builtin_amdgcn_readfirstlane(x_last);
        for (int xs = 0; xs < M; xs += 64) {
            const int x = xs + lane;
            if (x < M && (x < x_first || x > x_last)) D[base + x] = lambda;
        }
#pragma unroll 1
        for (int xt = x_first; xt <= x_last; xt += 32) {
            float x0[3] = {0.f, 0.f, 0.f};
            if (xt + c <= x_last) {
                voxel_inputs(base + xt + c, M, scale, ctf2, cover, x0);
#pragma unroll
                for (int d = 0; d < 3; ++d) x0[d] = bfr(x0[d]);
            }
            const float out = mlp_tile(s, tc, x0, hh, c);
            const int x = xt + tile_out_index(hh, c);
            if ((c & 1) == 0 && x <= x_last) {
                const float cv = cover[base + x];
                D[base + x] = cv > 0.f ? lambda + expf(out) / scale : lambda;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Training: gradient of L = 1/n sum (y - t)^2 over a batch (straight-through
// for the bfloat16 roundings), accumulated into grad[NPARAM]; loss += L.
// ---------------------------------------------------------------------------
constexpr int TW = 4;  // waves per training block

struct TrainShared {
    MlpShared p;
    unsigned short h1t[TW][32][H];  // bf16 H1 of the tile, [sample][k]
    unsigned short dzt[TW][32][W2S];  // bf16 dZ2 of the tile, [sample][j] (padded rows)
    float dh[TW][32][H + 1];        // dH1, then dZ1, [sample][k]
    float x0[TW][32][3];
    float g[NPARAM];                // block gradient
    double red[16];
};

__global__ __launch_bounds__(TW * 64) void mlp_grad_kernel(const float *params, const float *X, const float *T,
                                                           int64_t n, float inv_n, float *part, double *part_loss) {
    __shared__ TrainShared s;
    stage_params(params, s.p);
    for (int t = threadIdx.x; t < NPARAM; t += blockDim.x) s.g[t] = 0.f;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int hh = lane >> 5, c = lane & 31;
    // per-lane accumulators kept across tiles
    f32x16 dw2[2][2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int kb = 0; kb < 2; ++kb) dw2[jb][kb] = f32x16{0.f};
    float dw1[3] = {0.f, 0.f, 0.f}, db1 = 0.f;  // hidden unit k = lane
    float dw3[2] = {0.f, 0.f}, db2[2] = {0.f, 0.f}, db3 = 0.f;
    double lsum = 0.0;

    // the loop runs the same number of times in every wave of the block (it
    // contains barriers); tiles past the end hold no valid sample and add zero
    const int64_t ntiles = (n + 31) / 32;
    for (int64_t bt = blockIdx.x; bt * TW < ntiles; bt += gridDim.x) {
        const int64_t tile = bt * TW + wv;
        const int64_t smp = tile * 32 + c;
        const bool valid = smp < n;
        float x0[3] = {0.f, 0.f, 0.f};
        if (valid) {
            x0[0] = X[smp * 3];
            x0[1] = X[smp * 3 + 1];
            x0[2] = X[smp * 3 + 2];
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) x0[d] = bfr(x0[d]);
        if (hh == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) s.x0[wv][c][d] = x0[d];
        }
        // ---- forward
        s16x4 a[8];
        float z1[32];
        layer1(s.p, x0, hh, a, z1);
#pragma unroll
        for (int st = 0; st < 8; ++st)
#pragma unroll
            for (int q = 0; q < 4; ++q) s.h1t[wv][c][8 * st + 4 * hh + q] = (unsigned short)a[st][q];
        f32x16 acc0, acc1;
        layer2(s.p, a, hh, c, acc0, acc1);
        float h2[2][16], z2[2][16], out[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            z2[0][r] = acc0[r] + s.p.b2[c];
            z2[1][r] = acc1[r] + s.p.b2[32 + c];
            h2[0][r] = bfr(gelu(z2[0][r]));
            h2[1][r] = bfr(gelu(z2[1][r]));
            out[r] = half_sum(fmaf(s.p.w3[c], h2[0][r], s.p.w3[32 + c] * h2[1][r])) + s.p.b3;
        }
        // ---- output layer and its gradient
        float dy[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = 8 * (r / 4) + 4 * hh + (r % 4);
            const int64_t t = tile * 32 + i;
            const float res = t < n ? out[r] - T[t] : 0.f;
            dy[r] = t < n ? 2.0f * res * inv_n : 0.f;
            if (c == 0) lsum += (double)res * res * inv_n;
            dw3[0] = fmaf(dy[r], h2[0][r], dw3[0]);
            dw3[1] = fmaf(dy[r], h2[1][r], dw3[1]);
            if (c == 0) db3 += dy[r];
        }
        // dZ2 = dy W3 gelu'(z2), D layout; its bf16 copy feeds two GEMMs
        float dz2[2][16];
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                dz2[jb][r] = dy[r] * s.p.w3[32 * jb + c] * gelu_grad(z2[jb][r]);
                db2[jb] += dz2[jb][r];
                const int i = 8 * (r / 4) + 4 * hh + (r % 4);
                s.dzt[wv][i][32 * jb + c] = f2bf(dz2[jb][r]);
            }
        __syncthreads();  // h1t / dzt / x0 of every wave written
        // ---- dW2 += dZ2^T H1: rows j (A from dZ2 in D layout), K = samples
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                s16x4 av;
#pragma unroll
                for (int q = 0; q < 4; ++q) av[q] = (short)f2bf(dz2[jb][4 * s4 + q]);
#pragma unroll
                for (int kb = 0; kb < 2; ++kb) {
                    s16x4 bv;
#pragma unroll
                    for (int q = 0; q < 4; ++q) bv[q] = (short)s.h1t[wv][8 * s4 + 4 * hh + q][32 * kb + c];
                    dw2[jb][kb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, dw2[jb][kb], 0, 0, 0);
                }
            }
        }
        // ---- dH1 = dZ2 W2: rows = samples (A from dzt), K = j
        f32x16 dh[2];
        dh[0] = f32x16{0.f};
        dh[1] = f32x16{0.f};
#pragma unroll
        for (int st = 0; st < 8; ++st) {
            s16x4 av;
#pragma unroll
            for (int q = 0; q < 4; ++q) av[q] = (short)s.dzt[wv][c][8 * st + 4 * hh + q];
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                s16x4 bv;
#pragma unroll
                for (int q = 0; q < 4; ++q) bv[q] = (short)s.p.w2[(8 * st + 4 * hh + q) * W2S + 32 * kb + c];
                dh[kb] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, dh[kb], 0, 0, 0);
            }
        }
#pragma unroll
        for (int kb = 0; kb < 2; ++kb)
#pragma unroll
            for (int r = 0; r < 16; ++r) s.dh[wv][8 * (r / 4) + 4 * hh + (r % 4)][32 * kb + c] = dh[kb][r];
        __syncthreads();
        // dZ1 = dH1 gelu'(z1) in the layer-1 layout, written back in place
#pragma unroll
        for (int st = 0; st < 8; ++st)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = 8 * st + 4 * hh + q;
                s.dh[wv][c][k] *= gelu_grad(z1[st * 4 + q]);
            }
        __syncthreads();
        // dW1[k][.] and db1[k] for k = lane, summed over the tile's samples
        for (int i = 0; i < 32; ++i) {
            const float d = s.dh[wv][i][lane];
            db1 += d;
#pragma unroll
            for (int e = 0; e < 3; ++e) dw1[e] = fmaf(d, s.x0[wv][i][e], dw1[e]);
        }
        __syncthreads();  // LDS tile buffers are rewritten by the next tile
    }
    // ---- fold the per-lane accumulators into the block gradient, wave by
    // wave in order (every entry is held by one lane of a wave once the two
    // half-waves' partial sums of the output layer are combined), so the
    // block's sums do not depend on timing
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
        dw3[jb] += __shfl_xor(dw3[jb], 32, 64);
        db2[jb] += __shfl_xor(db2[jb], 32, 64);
    }
    db3 += __shfl_xor(db3, 32, 64);
    lsum += __shfl_xor(lsum, 32, 64);
    for (int w = 0; w < TW; ++w) {
        __syncthreads();
        if (wv != w) continue;
#pragma unroll
        for (int jb = 0; jb < 2; ++jb)
#pragma unroll
            for (int kb = 0; kb < 2; ++kb)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int j = 32 * jb + 8 * (r / 4) + 4 * hh + (r % 4);
                    s.g[OFF_W2 + j * H + 32 * kb + c] += dw2[jb][kb][r];
                }
#pragma unroll
        for (int e = 0; e < 3; ++e) s.g[OFF_W1 + lane * 3 + e] += dw1[e];
        s.g[OFF_B1 + lane] += db1;
        if (hh == 0) {
#pragma unroll
            for (int jb = 0; jb < 2; ++jb) {
                s.g[OFF_W3 + 32 * jb + c] += dw3[jb];
                s.g[OFF_B2 + 32 * jb + c] += db2[jb];
            }
            if (c == 0) {
                s.g[OFF_B3] += db3;
                s.red[0] = (w == 0 ? 0.0 : s.red[0]) + lsum;
            }
        }
    }
    __syncthreads();
    // the block's partial sums; mlp_grad_sum_kernel adds them in block order
    float *pg = part + (size_t)blockIdx.x * NPARAM;
    for (int t = threadIdx.x; t < NPARAM; t += blockDim.x) pg[t] = s.g[t];
    if (threadIdx.x == 0) part_loss[blockIdx.x] = s.red[0];
}

// grad[t] = sum over the blocks' partials in block order; loss likewise.
__global__ __launch_bounds__(256) void mlp_grad_sum_kernel(const float *part, const double *part_loss, int nblocks,
                                                           float *grad, double *loss) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < NPARAM) {
        float g = 0.f;
        for (int b = 0; b < nblocks; ++b) g += part[(size_t)b * NPARAM + t];
        grad[t] = g;
    }
    if (t == 0) {
        double l = 0.0;
        for (int b = 0; b < nblocks; ++b) l += part_loss[b];
        *loss = l;
    }
}

// Adam (Kingma & Ba) on the float32 master parameters.
__global__ void mlp_adam_kernel(float *params, float *m, float *v, const float *grad, int step, float lr, float beta1,
                                float beta2, float eps) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NPARAM) return;
    const float g = grad[t];
    const float mt = beta1 * m[t] + (1.0f - beta1) * g;
    const float vt = beta2 * v[t] + (1.0f - beta2) * g * g;
    m[t] = mt;
    v[t] = vt;
    const float mh = mt / (1.0f - powf(beta1, (float)step));
    const float vh = vt / (1.0f - powf(beta2, (float)step));
    params[t] -= lr * mh / (sqrtf(vh) + eps);
}

int mlp_param_count() { return NPARAM; }

hipError_t launch_mlp_forward(const float *params, const float *X, float *y, int64_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    int64_t blocks = ((n + 31) / 32 + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(mlp_infer_kernel, dim3((unsigned)blocks), dim3(256), 0, st, params, X, y, n);
    return hipGetLastError();
}

hipError_t launch_learned_diag(const float *params, int M, float N, float lambda, const float *ctf2,
                               const float *cover, float *D, hipStream_t st) {
    const int64_t rows = (int64_t)M * M;
    int64_t blocks = (rows + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(learned_diag_kernel, dim3((unsigned)blocks), dim3(256), 0, st, params, M, N, lambda, ctf2,
                       cover, D);
    return hipGetLastError();
}

// Blocks of the gradient kernel for n samples: about four tiles of 32 per
// wave, at most kMlpGradBlocks.
constexpr int kMlpGradBlocks = 64;
static int mlp_grad_blocks(int64_t n) {
    int64_t blocks = ((n + 31) / 32 + TW * 4 - 1) / (TW * 4);
    if (blocks > kMlpGradBlocks) blocks = kMlpGradBlocks;
    if (blocks < 1) blocks = 1;
    return (int)blocks;
}

size_t mlp_grad_workspace_bytes(int64_t n) {
    const size_t b = (size_t)mlp_grad_blocks(n);
    return (b * NPARAM * sizeof(float) + 255) / 256 * 256 + b * sizeof(double);
}

hipError_t launch_mlp_grad(const float *params, const float *X, const float *T, int64_t n, float *grad,
                           double *loss, void *ws, hipStream_t st) {
    if (n == 0) {
        hipError_t e = launch_fill_f32(grad, NPARAM, 0.0f, st);
        if (e != hipSuccess) return e;
        return launch_fill_f64(loss, 1, 0.0, st);
    }
    const int blocks = mlp_grad_blocks(n);
    float *part = (float *)ws;
    double *part_loss = (double *)((char *)ws + ((size_t)blocks * NPARAM * sizeof(float) + 255) / 256 * 256);
    hipLaunchKernelGGL(mlp_grad_kernel, dim3((unsigned)blocks), dim3(TW * 64), 0, st, params, X, T, n,
                       1.0f / (float)n, part, part_loss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_grad_sum_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, part, part_loss, blocks,
                       grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *params, float *m, float *v, const float *grad, int step, float lr, float beta1,
                           float beta2, float eps, hipStream_t st) {
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((NPARAM + 255) / 256), dim3(256), 0, st, params, m, v, grad, step, lr,
                       beta1, beta2, eps);
    return hipGetLastError();
}

}  // namespace csg
