// csg_device.h -- device-side building blocks shared by the HIP kernels of
// libcryosgd: launch parameters, the sample point of a pixel, the CTF and the
// Philox4x32-10 generator.  Internal to the library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace csg {

constexpr int kBlock = 256;  // threads per block of the pixel kernels (4 waves)

// Per-launch constants of the discretisation and the CTF.
struct Geom {
    int M;         // grid side
    int half;      // M / 2
    int interp;    // 0 nearest neighbour, 1 trilinear
    int k2max;     // floor(r_max^2): pixel used iff kx^2 + ky^2 <= k2max
    int ctf_on;
    double ctf_a;  // lambda / 2   (chi / 2pi per Angstrom of defocus per s^2)
    double ctf_b;  // Cs lambda^3 / 4 (chi / 2pi per s^4)
    double inv_s2; // 1 / (M pixel)^2: s^2 = k2 * inv_s2
    double phase0; // asin(A) / 2pi
};

// CTF at squared integer radius k2 for an image whose defocus term is
// a_i = ctf_a * defocus.  C = -(sqrt(1-A^2) sin chi + A cos chi) =
// -sin(chi + asin A).  The phase is formed in double precision in units of
// turns and reduced to [-1/2, 1/2]; the hardware sine takes its argument in
// turns (v_sin_f32, measured max error 1.3e-7 on [-1/2, 1/2]), so the result
// keeps full float accuracy even where chi is hundreds of radians.
__device__ __forceinline__ float ctf_value(const Geom &g, double a_i, int k2) {
    if (!g.ctf_on) return 1.0f;
    const double s2 = (double)k2 * g.inv_s2;
    const double turns = s2 * (a_i - g.ctf_b * s2) + g.phase0;
    const float fr = (float)(turns - rint(turns));
    return -__builtin_amdgcn_sinf(fr);
}

// In-plane shift of image i (Definition "Projection operator"): the phase
// T = exp(-2 pi i (kx sx + ky sy) / M) of a translation by (sx, sy) pixels,
// returned as (cos, sin).  The angle is formed in double precision in turns
// and reduced to [-1/2, 1/2] for the hardware turn-sine and turn-cosine.
__device__ __forceinline__ float2 shift_phase(const float *shift, int64_t i, int M, int kx, int ky) {
    const double t = -((double)kx * (double)shift[2 * i] + (double)ky * (double)shift[2 * i + 1]) / (double)M;
    const float fr = (float)(t - rint(t));
    return make_float2(__builtin_amdgcn_cosf(fr), __builtin_amdgcn_sinf(fr));
}

// a * t and a * conj(t) for complex values held as float2
__device__ __forceinline__ float2 cmul(float2 a, float2 t) {
    return make_float2(a.x * t.x - a.y * t.y, a.x * t.y + a.y * t.x);
}
__device__ __forceinline__ float2 cmul_conj(float2 a, float2 t) {
    return make_float2(a.x * t.x + a.y * t.y, a.y * t.x - a.x * t.y);
}

__device__ __forceinline__ float ctf_pow(float c, int p) {
    return p == 0 ? 1.0f : (p == 1 ? c : c * c);
}

// Sample point of pixel (kx,ky) in grid units: g = R^T (kx,ky,0) + M/2.
// kx*R and ky*R are exact in double (a float times a small integer), so g
// is the exact value rounded once or twice to 53 bits; the cell index and
// the fractional offsets then agree with any double-precision evaluation.
struct Cell {
    int f[3];    // floor(g) per axis (x, y, z), clamped into [-1, M]
    float t[3];  // g - floor(g)
};

__device__ __forceinline__ Cell sample_cell(const Geom &g, const float e1[3], const float e2[3], int kx, int ky) {
    Cell c;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double gd = fma((double)kx, (double)e1[d], fma((double)ky, (double)e2[d], (double)g.half));
        const double fl = floor(gd);
        // clamp so that absurd rotations cannot produce wild indices; such
        // corners are dropped below exactly like corners outside the grid
        const double flc = fmin(fmax(fl, -1.0), (double)g.M);
        c.f[d] = (int)flc;
        c.t[d] = (float)(gd - fl);
    }
    return c;
}

// Nearest grid point floor(g + 1/2) per axis, clamped into [-1, M].
__device__ __forceinline__ void sample_nearest(const Geom &g, const float e1[3], const float e2[3], int kx, int ky,
                                               int q[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double gd = fma((double)kx, (double)e1[d], fma((double)ky, (double)e2[d], (double)g.half));
        q[d] = (int)fmin(fmax(floor(gd + 0.5), -1.0), (double)g.M);
    }
}

__device__ __forceinline__ bool in_grid(int q, int M) { return (unsigned)q < (unsigned)M; }

// The up-to-eight (index, weight) pairs of a pixel.  Corners outside the grid
// get weight 0 and a clamped (valid) index, so callers may use every slot.
struct Stencil {
    int idx[8];
    float w[8];
};

__device__ __forceinline__ Stencil make_stencil(const Geom &g, const float e1[3], const float e2[3], int kx, int ky) {
    Stencil s;
    const int M = g.M;
    if (g.interp == 0) {
        int q[3];
        sample_nearest(g, e1, e2, kx, ky, q);
        const bool ok = in_grid(q[0], M) && in_grid(q[1], M) && in_grid(q[2], M);
        s.idx[0] = ok ? (q[2] * M + q[1]) * M + q[0] : 0;
        s.w[0] = ok ? 1.0f : 0.0f;
#pragma unroll
        for (int c = 1; c < 8; ++c) {
            s.idx[c] = 0;
            s.w[c] = 0.0f;
        }
        return s;
    }
    const Cell cl = sample_cell(g, e1, e2, kx, ky);
    int ix[2], iy[2], iz[2];
    float wx[2], wy[2], wz[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int qx = cl.f[0] + a, qy = cl.f[1] + a, qz = cl.f[2] + a;
        const bool okx = in_grid(qx, M), oky = in_grid(qy, M), okz = in_grid(qz, M);
        ix[a] = okx ? qx : 0;
        iy[a] = oky ? qy : 0;
        iz[a] = okz ? qz : 0;
        wx[a] = okx ? (a ? cl.t[0] : 1.0f - cl.t[0]) : 0.0f;
        wy[a] = oky ? (a ? cl.t[1] : 1.0f - cl.t[1]) : 0.0f;
        wz[a] = okz ? (a ? cl.t[2] : 1.0f - cl.t[2]) : 0.0f;
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int a = c & 1, b = (c >> 1) & 1, e = (c >> 2) & 1;
        s.idx[c] = (iz[e] * M + iy[b]) * M + ix[a];
        s.w[c] = wx[a] * wy[b] * wz[e];
    }
    return s;
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two
// 32x32->64-bit products of the even words by fixed multipliers, a swap and an
// xor with the odd words and the key; the key is bumped by the Weyl constants
// between rounds.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c.x, hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z, hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    }
    return c;
}

constexpr uint32_t kRademacherTag = 0x52414431u;  // counter word 3 of the probe stream

// The 128 random bits of Rademacher probe `probe` for voxels 128 blk ..
// 128 blk + 127: voxel k takes bit k mod 128 (word (k mod 128) / 32 of the
// output, bit k mod 32 of that word); a set bit means -1, a clear one +1.
__device__ __forceinline__ U4 rademacher_block(uint64_t seed, uint64_t probe, uint32_t blk) {
    return philox4x32_10(U4{blk, (uint32_t)probe, (uint32_t)(probe >> 32), kRademacherTag}, (uint32_t)seed,
                         (uint32_t)(seed >> 32));
}

// Wave-wide sum of a double (64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum (blockDim.x a multiple of 64, at most 1024); every thread
// must call it.  Returns the total in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds /* >= 16 */) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) lds[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += lds[i];
    }
    __syncthreads();
    return t;
}

// Fixed-point scale of the deterministic adjoint.  Every contribution w val to
// a component of a voxel is rounded to an integer multiple of 1/S and the
// multiples are summed as 64-bit integers: exact, hence independent of the
// order of summation.  The bound: w <= 1 and |val| <= V, where V = |scale| (m0
// + m1) with m0, m1 the largest |re| + |im| of the operator's inputs (|C| <= 1,
// |T| = 1 and the trilinear weights of a gathered value sum to 1).  A voxel
// receives from one image only the lattice pixels inside its 2x2x2
// neighbourhood: a plane cuts that cube in area at most 4 sqrt(2), so by
// Pick's theorem at most 13 pixels (32 is used as margin), and every partial
// sum over n images stays below 32 n V.  S = 2^e is the largest power of two with
// 32 n V S <= 2^61 (no 64-bit overflow) and V S <= 2^50 (fx_quant is exact).
// ok = 0 when an input is not finite.
struct FxScale {
    double S, invS;
    int ok;
};
__device__ __forceinline__ FxScale fx_scale(const unsigned *maxbits, float scale, int64_t n) {
    const double m = (double)__uint_as_float(maxbits[0]) + (double)__uint_as_float(maxbits[1]);
    const double V = fabs((double)scale) * m * (1.0 + 0x1p-20);
    FxScale f;
    f.S = 1.0;
    f.invS = 1.0;
    f.ok = isfinite(V) ? 1 : 0;
    if (f.ok && V > 0.0) {
        int kt, kv;
        (void)frexp(32.0 * (double)n * V, &kt);  // 32 n V < 2^kt
        (void)frexp(V, &kv);
        const int e = min(61 - kt, 50 - kv);
        f.S = ldexp(1.0, e);
        f.invS = ldexp(1.0, -e);
    }
    return f;
}

// round(x S) as a two's-complement 64-bit integer, for |x S| <= 2^50: adding
// 1.5 2^52 rounds the product to an integer (the spacing of doubles there is
// 1), and the sum's bit pattern is that of 1.5 2^52 plus the integer.
__device__ __forceinline__ unsigned long long fx_quant(float x, double S) {
    const double q = fma((double)x, S, 0x1.8p52);
    return (unsigned long long)__double_as_longlong(q) - 0x4338000000000000ull;
}

// Map a linear block id to a logical one so that the blocks placed on one XCD
// (ids congruent modulo 8) take a contiguous range of logical ids; returns -1
// for padding blocks.  nb_pad is the grid size rounded up to a multiple of 8.
__device__ __forceinline__ int64_t xcd_logical_block(int64_t bid, int64_t nb, int64_t nb_pad) {
    const int64_t per = nb_pad >> 3;
    const int64_t L = (bid & 7) * per + (bid >> 3);
    return L < nb ? L : -1;
}

}  // namespace csg
