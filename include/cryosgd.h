/*
 * cryosgd.h -- C ABI of the MI355X (gfx950) implementation of the known-pose
 * Fourier-slice refinement of Toader, Brubaker & Lederman, "Efficient
 * high-resolution refinement in cryo-EM with stochastic gradient descent"
 * (arXiv:2311.16100).
 *
 * General rules for every entry point
 * -----------------------------------
 *  - Pointers to volumes, images, rotations, defocus values, probes and
 *    results are DEVICE pointers owned by the caller.  Descriptors
 *    (csg_grid, csg_optics, csg_poses) are HOST structs read during the call.
 *    The library keeps no pointer after a call returns.
 *  - Complex data is complex64 stored interleaved (re, im) as float pairs:
 *    a "complex [K]" argument points to 2*K floats.
 *  - Volumes are [M][M][M] complex, index ((kz+M/2)*M + ky+M/2)*M + kx+M/2
 *    for frequencies k in {-M/2, ..., M/2-1} (DC at index M/2 on each axis).
 *    Images are [n][M][M] complex, index (i*M + ky+M/2)*M + kx+M/2.
 *  - Rotations are [n][3][3] float, row-major.  Pixel (kx,ky) of image i
 *    samples the volume at p = R_i^T (kx,ky,0) = kx R_i[0,:] + ky R_i[1,:]
 *    (the rotated volume is read at R^T r, Sec. 2.1).
 *  - Only pixels with kx^2 + ky^2 <= r_max^2 are used ("the disk"); the
 *    projector writes 0 elsewhere and the adjoint and the loss ignore them.
 *    An interpolation corner outside the grid counts as zero.
 *  - All work is enqueued on `stream` (a hipStream_t, NULL = the null
 *    stream); calls are asynchronous unless stated.  Nothing is allocated:
 *    scratch memory comes from the caller's `workspace` (size from
 *    csg_workspace_bytes), or, for csg_gradient_noalloc only, from a static
 *    device array that the library holds per GPU.
 *  - Return value: CSG_OK, or a negative code; csg_last_error() then holds
 *    a message (per thread).  No C++ exception crosses the ABI.
 */
#ifndef CRYOSGD_H
#define CRYOSGD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CSG_OK 0
#define CSG_EINVAL (-1)     /* invalid argument (shape, null pointer, range) */
#define CSG_EHIP (-2)       /* HIP launch or runtime error */
#define CSG_EWORKSPACE (-3) /* workspace missing or too small */

/* Discretisation (Sec. 2.1 and Definition "Projection operator").
 * M: grid side, even, 4 <= M <= 1024.
 * r_max: disk radius in pixels, 0 <= r_max <= M/2 - 1.
 * interp: 0 nearest neighbour (eq. (def nn interp), nearest point
 *         floor(p + 1/2) per axis), 1 trilinear (eq. (def tri interp)). */
typedef struct csg_grid {
    int32_t M;
    float r_max;
    int32_t interp;
} csg_grid;

/* CTF C_i (Sec. 2.1: real, radially symmetric, per-image defocus).  Weak-
 * phase model C(s) = -(sqrt(1-A^2) sin chi + A cos chi), chi = pi lambda df
 * s^2 - (pi/2) Cs lambda^3 s^4, s = |k| / (M pixel_A), lambda the
 * relativistic wavelength at kv.  ctf_on = 0 gives C == 1 (the CTF-free
 * setting of Sec. 3.1). */
typedef struct csg_optics {
    float kv;           /* accelerating voltage, kV (> 0 if ctf_on) */
    float cs_mm;        /* spherical aberration, mm */
    float amp_contrast; /* amplitude contrast A, 0 <= A < 1 */
    float pixel_A;      /* pixel size, Angstrom (> 0 if ctf_on) */
    int32_t ctf_on;
} csg_optics;

/* Known poses phi_i (Definition "Projection operator", Sec. 2.1): rotation
 * R_i, CTF defocus and the in-plane shift T_i.  Pixel (kx, ky) of image i
 * samples the volume at kx R_i[0,:] + ky R_i[1,:] (rows of R_i span the image
 * plane) and is multiplied by
 *   T_jj = exp(-2 pi i (kx sx_i + ky sy_i) / M),
 * the phase of a real-space translation of the image by (sx_i, sy_i) pixels.
 * shift_px == NULL means T = I.  T is unitary and diagonal, so the Hessian
 * (csg_hvp, csg_hutchinson_diag, csg_exact_diag) and the preconditioner
 * features do not depend on it; csg_project, csg_backproject and csg_gradient
 * apply it. */
typedef struct csg_poses {
    int64_t n;
    const float *rot;       /* device [n][3][3] */
    const float *defocus_A; /* device [n], Angstrom, underfocus > 0 */
    const float *shift_px;  /* device [n][2] (sx, sy) in pixels, or NULL */
} csg_poses;

/* Forward model without noise, eq. (fwd model): y_i = C_i T_i P_i v.
 *   vol      device complex [M^3]
 *   subtract device complex [n][M][M] or NULL: if given, out = C T P v - x
 *   out      device complex [n][M][M] or NULL (then loss_accum is required)
 *   loss_accum device double scalar or NULL: += 1/2 sum_disk |C T P v - x|^2
 *            (x = 0 when subtract is NULL).  Not zeroed by the call.
 *   workspace >= csg_workspace_bytes(grid, n, CSG_WS_PROJECT) bytes.
 * out and vol must not overlap. */
int csg_project(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                const float *vol, const float *subtract, float *out, double *loss_accum,
                void *workspace, size_t workspace_bytes, void *stream);

/* Adjoint / backprojection, the operator P_i^* C_i that appears in the M step
 * (eq. (em v)) and in b = sum_i P_i^* x_i (eq. (lin sys)):
 *   vol_accum += scale * sum_i P_i^T T_i^* C_i^p img_i,  p = ctf_power in {0,1,2}.
 *   img        device complex [n][M][M] (pixels outside the disk ignored)
 *   vol_accum  device complex [M^3], accumulated into
 *   deterministic 0: fast scatter (the floating-point summation order
 *                 varies between runs; within a work item the sums are exact
 *                 64-bit fixed point bounded by the largest |re| + |im| of
 *                 img, so a non-finite img value gives NaN).
 *                 1: bitwise reproducible.  On trilinear grids every
 *                 contribution is rounded to a multiple of 2^-e (64-bit fixed
 *                 point, with 2^e the largest power of two for which
 *                 32 n |scale| max(|re| + |im|) of img stays below 2^61) and
 *                 the integers are summed exactly, so the order of summation
 *                 cannot matter; the rounding is far below float precision.
 *                 A non-finite img value makes every voxel NaN.
 *                 Nearest-neighbour grids sum each voxel in a fixed order.
 *   workspace  device scratch of at least csg_workspace_bytes(grid, n,
 *              CSG_WS_BACKPROJECT or CSG_WS_BACKPROJECT_DETERMINISTIC) bytes
 *              (may be NULL when that is 0). */
int csg_backproject(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                    const float *img, int32_t ctf_power, float scale, float *vol_accum,
                    int32_t deterministic, void *workspace, size_t workspace_bytes, void *stream);

/* Minibatch gradient and loss of the known-pose least-squares problem,
 * eq. (optim cp) with the CTF re-inserted (eq. (em v)) and the batch scaled
 * by `scale` (N/B for an unbiased estimate of the full objective):
 *   f(v)     = scale * 1/2 sum_i ||C_i T_i P_i v - x_i||^2 + lambda/2 ||v||^2
 *   grad_out = scale * sum_i P_i^T T_i^* C_i (C_i T_i P_i v - x_i) + lambda v
 * (complex gradient convention d/dRe + i d/dIm).  The residual images are
 * never written to memory.
 *   vol       device complex [M^3];  x device complex [n][M][M]
 *   grad_out  device complex [M^3], overwritten (must not alias vol)
 *   loss_out  device double scalar or NULL, overwritten with f(v).
 *   deterministic as in csg_backproject (for the fixed-point bound, img is
 *             replaced by the largest |re| + |im| of vol plus that of x); the
 *             gradient is bitwise reproducible, the loss is a double sum
 *             whose order may vary.
 *   workspace >= csg_workspace_bytes(grid, n, CSG_WS_GRADIENT or
 *             CSG_WS_GRADIENT_DETERMINISTIC). */
int csg_gradient(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                 const float *vol, const float *x, float scale, float lambda, float *grad_out,
                 double *loss_out, int32_t deterministic, void *workspace, size_t workspace_bytes,
                 void *stream);

/* Allocation-free form of csg_gradient (deterministic = 0), for callers that
 * cannot allocate device memory or pass a workspace: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and error codes as csg_gradient with deterministic = 0,
 * without the workspace.  The call allocates nothing (no hipMalloc, hipFree,
 * events or library allocations); its scratch (device scalars and the
 * per-brick image tables) is a static device array of
 * CSG_STATIC_SCRATCH_BYTES bytes per GPU, which the library holds from its
 * first use on that GPU until the process ends.  The array of the CURRENT
 * device is used, so `stream` must belong to the current device.  Batches
 * whose brick tables exceed the array are processed in sub-batches (as many
 * images per launch as fit; at most 2048 as in csg_gradient); a grid too
 * large for the tables of one image returns CSG_EWORKSPACE.
 * Every call on one GPU shares that GPU's array and every call overwrites
 * it: calls that overlap in time on one GPU (different streams, or threads
 * without ordering) race and give wrong results.  Calls in order on one
 * stream are safe. */
#define CSG_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
int csg_gradient_noalloc(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                         const float *vol, const float *x, float scale, float lambda, float *grad_out,
                         double *loss_out, void *stream);

/* Hessian-vector product of the same objective (eq. (hessian)); H is real and
 * independent of v, so a complex z carries two real products:
 *   hz_out = scale * sum_i P_i^T C_i^2 P_i z + lambda z
 *   z, hz_out device complex [M^3] (hz_out overwritten, must not alias z).
 *   deterministic, workspace: as in csg_gradient. */
int csg_hvp(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
            const float *z, float scale, float lambda, float *hz_out, int32_t deterministic,
            void *workspace, size_t workspace_bytes, void *stream);

/* Rademacher(0.5) probe of Hutchinson's estimator (eq. (hutch)), entries
 * +1/-1: z_k = 1 - 2 b, b = bit (k mod 128) of Philox4x32-10 (Salmon et al.,
 * SC'11) with key (seed lo, seed hi) and counter (k/128, probe lo, probe hi,
 * 0x52414431); within the 128-bit block bit j is bit (j mod 32) of word j/32.
 *   z_out device float [nvox], overwritten. */
int csg_rademacher(int64_t nvox, uint64_t seed, int64_t probe, float *z_out, void *stream);

/* Hutchinson's diagonal estimate D = mean_p z_p (.) H z_p (eq. (hutch)) over
 * the probes probe0 .. probe0 + n_probe - 1 (as csg_rademacher), with H the
 * minibatch Hessian of csg_hvp.  Two probes share one complex product.  The
 * probes are regenerated from their hash wherever they are read and never
 * stored; on trilinear grids each contribution to z (.) H z is formed where
 * the product is scattered (multiplied by the receiving voxel's probe
 * signs) and summed in 32-bit fixed point per voxel with a scale from a
 * worst-case bound (the probe entries are +-1), so no volume of H z is
 * stored either: the estimate matches the one formed with csg_hvp to about
 * 1e-5 relative, far below its own sampling noise (on nearest-neighbour
 * grids the pair and its product are stored in the workspace).
 *   diag_out device float [M^3], overwritten.
 *   workspace >= csg_workspace_bytes(grid, n, CSG_WS_HUTCHINSON). */
int csg_hutchinson_diag(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                        int32_t n_probe, uint64_t seed, int64_t probe0, float scale, float lambda,
                        float *diag_out, void *workspace, size_t workspace_bytes, void *stream);

/* The two minibatch quantities of one iteration of Algorithm 1 (Sec. 3.4) on
 * the same batch: the gradient and loss of csg_gradient (deterministic = 0)
 * and the Hutchinson diagonal of csg_hutchinson_diag.  The Hessian does not
 * depend on v (eq. (hessian)), so the probe product and the gradient visit
 * the same pixels with the same sample points, CTF values and weights; on
 * trilinear grids without in-plane shifts one brick kernel computes the
 * gradient and the first probe pair's product in one pass over the pixels
 * (further pairs, nearest-neighbour grids and shifted poses take the two
 * separate paths).  Results equal those of the two calls up to rounding:
 * the gradient and loss up to the order of float additions, the diagonal to
 * about 1e-5 relative (its 32-bit fixed-point sums take each contribution
 * after the receiving voxel's probe signs are applied, as one number).
 *   Arguments as in csg_gradient and csg_hutchinson_diag; grad_out and
 *   diag_out must not alias vol or each other.
 *   workspace >= csg_workspace_bytes(grid, n, CSG_WS_GRADIENT_HUTCHINSON). */
int csg_gradient_hutchinson(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                            const float *vol, const float *x, float scale, float lambda,
                            float *grad_out, double *loss_out, int32_t n_probe, uint64_t seed,
                            int64_t probe0, float *diag_out, void *workspace, size_t workspace_bytes,
                            void *stream);

/* Exact diagonal of the minibatch Hessian: diag_out = scale * sum_ij C_ij^2
 * w_ijk^2 + lambda (squared interpolation weights; eq. (hessian) with eq.
 * (def tri interp)).  diag_out device float [M^3], overwritten; workspace as for
 * csg_backproject. */
int csg_exact_diag(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                   float scale, float lambda, float *diag_out, void *workspace,
                   size_t workspace_bytes, void *stream);

/* One preconditioned SGD step of Algorithm 1 (Sec. 3.4), elementwise over
 * nvox voxels:
 *   if zHz != NULL (probe sample of this iteration k >= 1):
 *       D_avg = (k-1)/k D_avg + zHz / k ;  D = beta D + (1-beta) D_avg
 *   D_hat  = max(|D|, alpha)                (eq. (thresh)); D == NULL: D_hat = 1
 *   v_out  = v - eta g / D_hat              (eq. (sgd step))
 *   stats_out[0] = sum |g|^2 / D_hat        (the norm of eq. (stochastic armijo))
 *   stats_out[1] = sum |v_out|^2
 *   v, g, v_out device complex [nvox] (v_out may alias v only if g does not)
 *   D, D_avg device float [nvox] updated in place (D_avg may be NULL when
 *            zHz is NULL); Dhat_out device float [nvox] or NULL
 *   stats_out device double [2], overwritten.
 * With v, g, v_out and stats_out all NULL (and D, D_avg, zHz given) only the
 * diagonal estimate is updated (eq. (diag est rule) with the running mean
 * of Algorithm 1) and D_hat written if asked for: the precomputation of a
 * preconditioner over many epochs before SGD starts (Sec. 4.1). */
int csg_precond_sgd_step(int64_t nvox, const float *v, const float *g, float *D, float *D_avg,
                         const float *zHz, int64_t k, float beta, float alpha, float eta,
                         float *v_out, float *Dhat_out, double *stats_out, void *stream);

/* Fast per-voxel sums for the learned preconditioner, one pass over the
 * images (trilinear grids only):
 *   accum[k].re += sum_i sum_j C_ij^2 w_ijk   (as ctf2_accum of csg_features)
 *   accum[k].im += sum_i sum_j w_ijk          (interpolation weight reaching
 *                  k: for nearest-neighbour stencils without repeated hits
 *                  this is the size of the voxel mapping set |Omega_k|)
 *   accum device complex [M^3]; workspace as for csg_backproject. */
int csg_feature_sums(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                     float *accum, void *workspace, size_t workspace_bytes, void *stream);

/* Threshold of the preconditioner, eq. (thresh value) (Sec. 3.3): the
 * expected Hessian entry at the maximum radius R = round(r_max),
 *   alpha = (P_x(R) / P_v(R)) * sum_{i=1}^N C_i(R)^2 + lambda,
 * with P_x(R), P_v(R) the numbers of pixels / voxels of the grid whose radius
 * rounds to R, and the sum over all N images of `poses` (the whole data set).
 *   alpha_out device double scalar, overwritten. */
int csg_threshold_alpha(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                        float lambda, double *alpha_out, void *stream);

/* Per-voxel inputs of the learned preconditioner:
 *   ctf2_accum[k]  += sum_i sum_j C_ij^2 w_ijk   (CTF^2 weight)
 *   cover_accum[k] += |{i : some pixel of image i has w_ijk > 0}| (the size of
 *                     the voxel mapping set Omega_k, Definition "Voxel mapping
 *                     set", over trilinear stencils)
 * both device float [M^3]. */
int csg_features(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses,
                 float *ctf2_accum, float *cover_accum, void *stream);

/* ------------------------------------------------------------------------
 * Learned preconditioner (not part of the paper's method: a regression of
 * the Hessian diagonal of Sec. 3.2 from per-voxel features, trained on
 * Hutchinson estimates, with Hutchinson as its judge and fallback).
 * Network: MLP 3 -> 64 -> 64 -> 1, GELU activations, float32 master
 * weights used as bfloat16 (round to nearest even), layer inputs rounded to
 * bfloat16, float32 accumulation (the 64 x 64 products on the matrix cores).
 * Parameter vector, float32, csg_mlp_param_count() entries:
 *   W1[64][3], b1[64], W2[64][64], b2[64], W3[64], b3.
 * ------------------------------------------------------------------------ */
int32_t csg_mlp_param_count(void);

/* y[s] = mlp(X[s]) for n samples; X device float [n][3], y device float [n]. */
int csg_mlp_forward(const float *params, const float *X, int64_t n, float *y, void *stream);

/* Gradient of the mean squared error L = 1/n sum_s (mlp(X[s]) - T[s])^2 with
 * respect to the parameter vector (bfloat16 roundings passed straight
 * through).  grad device float [param_count] and loss_out device double [1]
 * are overwritten.  The sums run in a fixed order (per-block partials in the
 * workspace, added in block order), so equal inputs give bitwise equal
 * results.  workspace: device, 256-byte aligned, at least
 * csg_mlp_grad_workspace_bytes(n) bytes (NULL allowed for n = 0). */
size_t csg_mlp_grad_workspace_bytes(int64_t n);
int csg_mlp_grad(const float *params, const float *X, const float *T, int64_t n, float *grad,
                 double *loss_out, void *workspace, size_t workspace_bytes, void *stream);

/* One Adam step (Kingma & Ba) on params with moment buffers m, v (device
 * float [param_count], zero before step 1); step >= 1 counts the updates. */
int csg_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr,
                 float beta1, float beta2, float eps, void *stream);

/* Predicted Hessian diagonal over the M^3 grid of `grid`:
 *   diag_out[k] = lambda + (N/M) exp(mlp(|k| / (M/2), log(ctf2[k] M/N), log(cover[k] M/N)))
 * where cover[k] > 0, and lambda where no image reaches voxel k (there the
 * data part of the diagonal is exactly zero).  ctf2 and cover are per-voxel
 * sums over the N = n_images images of the data set, the same kind the
 * network was trained on (csg_feature_sums: real and imaginary parts). */
int csg_learned_diag(const csg_grid *grid, int64_t n_images, float lambda, const float *params,
                     const float *ctf2, const float *cover, float *diag_out, void *stream);

/* Workspace sizes (bytes) for a batch of n images:
 *   CSG_WS_PROJECT                 csg_project
 *   CSG_WS_BACKPROJECT             csg_backproject, deterministic = 0
 *   CSG_WS_BACKPROJECT_DETERMINISTIC  csg_backproject, deterministic = 1
 *                                  (trilinear grids: adds the 64-bit
 *                                  fixed-point volume, 16 M^3 bytes)
 *   CSG_WS_HUTCHINSON              csg_hutchinson_diag: the brick tables
 *                                  (nearest-neighbour grids: two complex
 *                                  volumes)
 *   CSG_WS_GRADIENT                csg_gradient / csg_hvp, deterministic = 0
 *   CSG_WS_GRADIENT_DETERMINISTIC  csg_gradient / csg_hvp, deterministic = 1
 *                                  (trilinear grids: the fixed-point volume;
 *                                  nearest neighbour: one complex image per
 *                                  batch image)
 *   CSG_WS_GRADIENT_HUTCHINSON     csg_gradient_hutchinson: the larger of
 *                                  CSG_WS_GRADIENT and CSG_WS_HUTCHINSON
 * Workspaces must be 256-byte aligned.  Returns 0 for an invalid grid. */
#define CSG_WS_BACKPROJECT 0
#define CSG_WS_HUTCHINSON 1
#define CSG_WS_GRADIENT 2
#define CSG_WS_GRADIENT_DETERMINISTIC 3
#define CSG_WS_PROJECT 4
#define CSG_WS_BACKPROJECT_DETERMINISTIC 5
#define CSG_WS_GRADIENT_HUTCHINSON 6
size_t csg_workspace_bytes(const csg_grid *grid, int64_t n, int32_t which);

/* Per-shell sums of two volumes over the Fourier shells round(|k|) = s,
 * s = 0 .. M/2 - 1 (the shells of the shell correlation, eq. (fsc), Sec. 4.1):
 *   sums_out[s]         = sum Re(u_k conj(v_k))
 *   sums_out[M/2 + s]   = sum |u_k|^2
 *   sums_out[M + s]     = sum |v_k|^2
 * so FSC(s) = sums_out[s] / sqrt(sums_out[M/2 + s] sums_out[M + s]).
 * u, v: device complex64 [M][M][M] (centred); sums_out: device double
 * [3 M/2], overwritten.  Voxels beyond the last full shell are ignored. */
int csg_shell_sums(const csg_grid *grid, const float *u, const float *v, double *sums_out, void *stream);

/* ------------------------------------------------------------------------
 * Kernel timing (measurement support, not part of the method).  While
 * enabled, every launch of a brick-binned operator kernel is bracketed by two
 * HIP events recorded on the stream the kernel is launched on (timing-only
 * events, without the system-scope cache write-back on record).
 * csg_timing_read waits for the recorded events of one kernel, returns the
 * summed duration (ms) and the number of launches recorded since the last
 * read of that kernel, and forgets them.  At most 8192 launches per kernel
 * are kept between reads; later ones are not recorded.  Launches of the
 * nearest-neighbour path (other kernels) are not timed; the fixed-point
 * brick kernels of the deterministic mode are timed under the same index as
 * the fast ones.
 * Results of the operators do not depend on the setting.
 *   kernel: CSG_KERNEL_PROJECT     forward projection (csg_project)
 *           CSG_KERNEL_BACKPROJECT adjoint (csg_backproject, fast mode)
 *           CSG_KERNEL_GRADIENT    fused residual + adjoint (csg_gradient)
 *           CSG_KERNEL_HVP         gather + scatter of H z (csg_hvp,
 *                                  csg_hutchinson_diag)
 *           CSG_KERNEL_FEATURES    csg_feature_sums
 *           CSG_KERNEL_SQ_DIAG     csg_exact_diag
 *           CSG_KERNEL_GRADIENT_PROBE  gradient with the first probe pair
 *                                  (csg_gradient_hutchinson)
 * ------------------------------------------------------------------------ */
#define CSG_KERNEL_PROJECT 0
#define CSG_KERNEL_BACKPROJECT 1
#define CSG_KERNEL_GRADIENT 2
#define CSG_KERNEL_HVP 3
#define CSG_KERNEL_FEATURES 4
#define CSG_KERNEL_SQ_DIAG 5
#define CSG_KERNEL_GRADIENT_PROBE 6
int csg_timing_enable(int32_t on);
int csg_timing_read(int32_t kernel, double *total_ms, int64_t *launches);

/* Message for the last nonzero return on the calling thread. */
const char *csg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CRYOSGD_H */
