/*
 * oracle.c -- plain, slow, double-precision CPU oracle for the known-pose
 * Fourier-slice operators of Toader, Brubaker & Lederman, "Efficient
 * high-resolution refinement in cryo-EM with stochastic gradient descent"
 * (arXiv:2311.16100).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this file's library.  It shares
 * no code, header, table or constant with the HIP library: every formula here
 * is written out again from the paper (and, where the paper is silent, from
 * the textbook definition named in the comment).
 *
 * Conventions (the paper leaves them open; Sec. 2.1 says the ordering is
 * "without loss of generality"):
 *   - Fourier grid k in {-M/2, ..., M/2-1} per axis, M even.
 *   - Volume element (kx,ky,kz) is stored at ((kz+M/2)*M + (ky+M/2))*M + (kx+M/2).
 *   - Image element (kx,ky) of image i is stored at (i*M + ky+M/2)*M + kx+M/2.
 *   - Rotations are 3x3 row-major float32, promoted to double here.
 *   - Complex data is double complex (numpy complex128).
 *
 * Everything is double precision; inputs that the GPU receives as float32
 * (rotations, defocus) are taken as float32 and promoted, so both sides see
 * the same numbers.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,       */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11).  Each round takes  */
/* the two 32x32->64 products of the even counter words with the round       */
/* multipliers, swaps the halves and xors in the odd words and the key; the  */
/* key is bumped by the Weyl constants between rounds.                       */
/* ------------------------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/*
 * Rademacher(0.5) probe entries for Hutchinson's estimator (Sec. 3.2,
 * eq. (hutch)): z_k = +1 or -1 with equal probability.  The bits come from
 * Philox4x32-10 with key = (seed low word, seed high word) and counter =
 * (k / 128, probe low word, probe high word, 0x52414431); entry k uses bit
 * (k mod 128) of the 128-bit output, word (k mod 128) / 32, bit (k mod 32),
 * and z_k = 1 - 2 * bit.
 */
void or_rademacher(uint64_t seed, uint64_t probe, int64_t nvox, double *z)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4] = {0, 0, 0, 0};
    int64_t block = -1;
    for (int64_t k = 0; k < nvox; ++k) {
        int64_t b = k / 128;
        if (b != block) {
            uint32_t ctr[4] = {(uint32_t)b, (uint32_t)probe, (uint32_t)(probe >> 32), 0x52414431u};
            or_philox4x32_10(ctr, key, out);
            block = b;
        }
        int bit_index = (int)(k % 128);
        uint32_t bit = (out[bit_index / 32] >> (bit_index % 32)) & 1u;
        z[k] = bit ? -1.0 : 1.0;
    }
}

/* ------------------------------------------------------------------------ */
/* Contrast transfer function.  The paper (Sec. 2.1) states only that the    */
/* CTF is a known, real, radially symmetric diagonal with per-image          */
/* parameters such as defocus.  The oracle uses the textbook weak-phase CTF: */
/*   C(s) = -( sqrt(1 - A^2) sin(chi) + A cos(chi) ),                         */
/*   chi(s) = pi * lambda * df * s^2 - (pi/2) * Cs * lambda^3 * s^4,           */
/* s = |k| / (M * pixel) in 1/Angstrom, df > 0 underfocus (Angstrom),        */
/* Cs in Angstrom, lambda the relativistic electron wavelength.              */
/* ------------------------------------------------------------------------ */
typedef struct {
    double kv;           /* accelerating voltage, kV */
    double cs_mm;        /* spherical aberration, mm */
    double amp_contrast; /* amplitude contrast fraction A */
    double pixel_A;      /* pixel size, Angstrom */
    int32_t ctf_on;      /* 0: C == 1 (the CTF-free setting of Sec. 3.1) */
} or_optics;

/* lambda = h / sqrt(2 m0 e V (1 + e V / (2 m0 c^2))), returned in Angstrom
   (CODATA 2018 constants). */
double or_wavelength_A(double kv)
{
    const double h = 6.62607015e-34, m0 = 9.1093837015e-31, e = 1.602176634e-19, c = 299792458.0;
    double V = kv * 1.0e3;
    double lam_m = h / sqrt(2.0 * m0 * e * V * (1.0 + e * V / (2.0 * m0 * c * c)));
    return lam_m * 1.0e10;
}

/* C_i at integer squared radius k2 = kx^2 + ky^2 on an M grid. */
double or_ctf(const or_optics *o, int M, double defocus_A, double k2)
{
    if (!o->ctf_on) return 1.0;
    double lam = or_wavelength_A(o->kv);
    double cs = o->cs_mm * 1.0e7;
    double s2 = k2 / ((double)M * o->pixel_A * (double)M * o->pixel_A);
    double chi = M_PI * lam * defocus_A * s2 - 0.5 * M_PI * cs * lam * lam * lam * s2 * s2;
    double A = o->amp_contrast;
    return -(sqrt(1.0 - A * A) * sin(chi) + A * cos(chi));
}

/* ------------------------------------------------------------------------ */
/* Projection operators (Definition "Projection operator", Sec. 2.1).       */
/* Pixel j at (kx,ky) is sent to p = R^T (kx,ky,0) = kx R[0,:] + ky R[1,:],  */
/* since the rotated volume is read at R^T r (Sec. 2.1).  Only pixels in the */
/* disk kx^2+ky^2 <= r_max^2 are used; the rest of the image is zero.        */
/*   interp = 0: nearest neighbour, eq. (def nn interp); the nearest grid   */
/*               point is floor(p + 1/2) per axis.                            */
/*   interp = 1: trilinear, eq. (def tri interp); the eight corners of the  */
/*               cell of p, weights prod_d (t_d or 1 - t_d).                  */
/* A corner outside the M^3 grid is dropped (its value is taken as zero).    */
/* The shift T of the definition is the identity here (no shifts).           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t M;
    double r_max;
    int32_t interp;
} or_grid;

/* Enumerate the (voxel index, weight) pairs of one pixel; returns the count. */
static int pixel_stencil(const or_grid *g, const double R[9], int kx, int ky,
                         int64_t vox[8], double w[8])
{
    int M = g->M;
    double pos[3];
    for (int d = 0; d < 3; ++d) pos[d] = (double)kx * R[0 * 3 + d] + (double)ky * R[1 * 3 + d] + (double)(M / 2);
    int count = 0;
    if (g->interp == 0) {
        int64_t q[3];
        for (int d = 0; d < 3; ++d) q[d] = (int64_t)floor(pos[d] + 0.5);
        for (int d = 0; d < 3; ++d)
            if (q[d] < 0 || q[d] >= M) return 0;
        vox[0] = (q[2] * M + q[1]) * M + q[0];
        w[0] = 1.0;
        return 1;
    }
    int64_t f[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
        double fl = floor(pos[d]);
        f[d] = (int64_t)fl;
        t[d] = pos[d] - fl;
    }
    for (int c = 0; c < 8; ++c) {
        int a[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        int64_t q[3];
        double wt = 1.0;
        int inside = 1;
        for (int d = 0; d < 3; ++d) {
            q[d] = f[d] + a[d];
            wt *= a[d] ? t[d] : 1.0 - t[d];
            if (q[d] < 0 || q[d] >= M) inside = 0;
        }
        if (!inside) continue;
        vox[count] = (q[2] * M + q[1]) * M + q[0];
        w[count] = wt;
        ++count;
    }
    return count;
}

static void load_rotation(const float *rot, int64_t i, double R[9])
{
    for (int e = 0; e < 9; ++e) R[e] = (double)rot[i * 9 + e];
}

static int in_disk(const or_grid *g, int kx, int ky)
{
    double k2 = (double)kx * kx + (double)ky * ky;
    return k2 <= g->r_max * g->r_max;
}

/*
 * In-plane shift of image i, the diagonal T_i of Definition "Projection
 * operator" (Sec. 2.1): translating the image by (sx, sy) pixels multiplies
 * pixel (kx, ky) of its discrete Fourier transform by
 *   T_jj = exp(-2 pi i (kx sx + ky sy) / M).
 * shift == NULL means T = I.
 */
static double complex shift_phase(const float *shift, int64_t i, int M, int kx, int ky)
{
    if (!shift) return 1.0;
    double t = -((double)kx * (double)shift[2 * i] + (double)ky * (double)shift[2 * i + 1]) / (double)M;
    double a = 2.0 * M_PI * t;
    return cos(a) + I * sin(a);
}

/*
 * Forward model without noise, eq. (fwd model): out_i = C_i T_i P_i v.
 * out is [n][M][M]; pixels outside the disk are set to zero.
 */
void or_project(const or_grid *g, const or_optics *o, int64_t n, const float *rot,
                const float *defocus, const float *shift, const double complex *vol, double complex *out)
{
    int M = g->M, h = M / 2;
    for (int64_t i = 0; i < n; ++i) {
        double R[9];
        load_rotation(rot, i, R);
        for (int ky = -h; ky < h; ++ky) {
            for (int kx = -h; kx < h; ++kx) {
                int64_t j = (i * M + (ky + h)) * M + (kx + h);
                out[j] = 0.0;
                if (!in_disk(g, kx, ky)) continue;
                int64_t vox[8];
                double w[8];
                int cnt = pixel_stencil(g, R, kx, ky, vox, w);
                double complex acc = 0.0;
                for (int c = 0; c < cnt; ++c) acc += w[c] * vol[vox[c]];
                double C = or_ctf(o, M, (double)defocus[i], (double)kx * kx + (double)ky * ky);
                out[j] = C * shift_phase(shift, i, M, kx, ky) * acc;
            }
        }
    }
}

/*
 * Adjoint (backprojection), the operator P_i^* C_i^p that appears in the
 * M-step (eq. (em v)) and in b = sum_i P_i^* x_i (Sec. 3.1):
 *   vol_accum += scale * sum_i P_i^T conj(T_i) C_i^p img_i
 * (the adjoint of the real interpolation matrix is its transpose; T_i is
 * unitary and diagonal).
 */
void or_backproject(const or_grid *g, const or_optics *o, int64_t n, const float *rot,
                    const float *defocus, const float *shift, const double complex *img, int ctf_power,
                    double scale, double complex *vol_accum)
{
    int M = g->M, h = M / 2;
    for (int64_t i = 0; i < n; ++i) {
        double R[9];
        load_rotation(rot, i, R);
        for (int ky = -h; ky < h; ++ky) {
            for (int kx = -h; kx < h; ++kx) {
                if (!in_disk(g, kx, ky)) continue;
                int64_t j = (i * M + (ky + h)) * M + (kx + h);
                double C = or_ctf(o, M, (double)defocus[i], (double)kx * kx + (double)ky * ky);
                double Cp = 1.0;
                for (int e = 0; e < ctf_power; ++e) Cp *= C;
                int64_t vox[8];
                double w[8];
                int cnt = pixel_stencil(g, R, kx, ky, vox, w);
                double complex x = conj(shift_phase(shift, i, M, kx, ky)) * img[j];
                for (int c = 0; c < cnt; ++c) vol_accum[vox[c]] += scale * w[c] * Cp * x;
            }
        }
    }
}

/*
 * Exact diagonal of the data part of the Hessian, eq. (hessian) with the CTF
 * re-inserted as in eq. (em v): diag(sum_i P_i^T C_i^2 P_i)_k
 *   = sum_i sum_j C_ij^2 (P_i)_{jk}^2, i.e. a backprojection of C^2 with the
 * interpolation weights squared.  diag_accum += scale * that.
 */
void or_sq_backproject(const or_grid *g, const or_optics *o, int64_t n, const float *rot,
                       const float *defocus, double scale, double *diag_accum)
{
    int M = g->M, h = M / 2;
    for (int64_t i = 0; i < n; ++i) {
        double R[9];
        load_rotation(rot, i, R);
        for (int ky = -h; ky < h; ++ky) {
            for (int kx = -h; kx < h; ++kx) {
                if (!in_disk(g, kx, ky)) continue;
                double C = or_ctf(o, M, (double)defocus[i], (double)kx * kx + (double)ky * ky);
                int64_t vox[8];
                double w[8];
                int cnt = pixel_stencil(g, R, kx, ky, vox, w);
                for (int c = 0; c < cnt; ++c) diag_accum[vox[c]] += scale * C * C * w[c] * w[c];
            }
        }
    }
}

/*
 * Per-voxel features of the learned preconditioner:
 *   ctf2_accum[k]  += sum_i sum_j C_ij^2 w_ijk   (CTF^2 backprojected with
 *                     the plain interpolation weights, i.e. the row sums of
 *                     sum_i P_i^T C_i^2 P_i);
 *   cover_accum[k] += |{ i : some pixel j of image i has w_ijk > 0 }|, the
 *                     size of the voxel mapping set Omega_k (Definition
 *                     "Voxel mapping set", Sec. 3.1) extended to trilinear
 *                     stencils.
 */
void or_features(const or_grid *g, const or_optics *o, int64_t n, const float *rot,
                 const float *defocus, double *ctf2_accum, double *cover_accum)
{
    int M = g->M, h = M / 2;
    int64_t nvox = (int64_t)M * M * M;
    unsigned char *hit = (unsigned char *)calloc((size_t)nvox, 1);
    if (!hit) return;
    for (int64_t i = 0; i < n; ++i) {
        double R[9];
        load_rotation(rot, i, R);
        memset(hit, 0, (size_t)nvox);
        for (int ky = -h; ky < h; ++ky) {
            for (int kx = -h; kx < h; ++kx) {
                if (!in_disk(g, kx, ky)) continue;
                double C = or_ctf(o, M, (double)defocus[i], (double)kx * kx + (double)ky * ky);
                int64_t vox[8];
                double w[8];
                int cnt = pixel_stencil(g, R, kx, ky, vox, w);
                for (int c = 0; c < cnt; ++c) {
                    ctf2_accum[vox[c]] += C * C * w[c];
                    if (w[c] > 0.0) hit[vox[c]] = 1;
                }
            }
        }
        for (int64_t k = 0; k < nvox; ++k) cover_accum[k] += hit[k];
    }
    free(hit);
}
