// csg_internal.h -- host-side launchers of the kernels, called by the C ABI
// layer (api.hip).  Internal to the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "csg_device.h"

namespace csg {

// Images per launch of the brick kernels; larger batches are processed in
// sub-batches of this size (it bounds the per-brick image lists).
constexpr int64_t kBrickSubBatch = 2048;

// optional kernel timing (timing.hip): brick kernel modes 0..kTimedKernels-1
constexpr int kTimedKernels = 7;
constexpr int kTimedGradProbe = 6;  // the fused gradient and probe kernel
void timing_set(int on);
hipEvent_t timing_begin(int kernel, hipStream_t st);  // nullptr when not timing
void timing_end(int kernel, hipEvent_t start, hipStream_t st);
hipError_t timing_read(int kernel, double *total_ms, int64_t *launches);

// brick-binned kernels (brick_kernels.hip)
int brick_count(int M);
size_t brick_workspace_bytes(int M, int64_t n);
// the same for launches of at most `sub` images each
size_t brick_workspace_bytes_sub(int M, int64_t sub);
hipError_t launch_brick_project(const Geom &g, const float *rot, const float *defocus, const float *shift, int64_t n,
                                const float2 *vol, const float2 *subtract, float2 *out, double *loss, void *ws,
                                hipStream_t st);
hipError_t launch_brick_backproject(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                    int64_t n, const float2 *img, int ctf_power, float scale, float2 *accum,
                                    void *ws, hipStream_t st);
// sub_cap: images per launch (the brick tables in ws hold that many);
// timed = false keeps the launches out of the optional kernel timing, which
// creates events
hipError_t launch_brick_gradient(const Geom &g, const float *rot, const float *defocus, const float *shift, int64_t n,
                                 const float2 *vol, const float2 *x, float scale, float2 *accum, double *loss,
                                 void *ws, hipStream_t st, int64_t sub_cap = kBrickSubBatch, bool timed = true);
hipError_t launch_brick_feature_sums(const Geom &g, const float *rot, const float *defocus, int64_t n,
                                     float2 *accum, void *ws, hipStream_t st);
hipError_t launch_brick_sq_diag(const Geom &g, const float *rot, const float *defocus, int64_t n, float scale,
                                float *diag, void *ws, hipStream_t st);
hipError_t launch_brick_hvp(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *z,
                            float scale, float2 *accum, void *ws, hipStream_t st);
// the same for the Rademacher probe pair (seed, pa, pb, has_b) of
// launch_probe_init, generated while the bricks are staged; its entries are
// 0 or +-1 per component, which allows the packed fixed-point accumulator.
// It adds z_a (.) (H z_a) + z_b (.) (H z_b) (H = scale P^T C^2 P, no lambda
// term) to the real diag, with float atomics
hipError_t launch_brick_hvp_probe(const Geom &g, const float *rot, const float *defocus, int64_t n, uint64_t seed,
                                  uint64_t pa, uint64_t pb, int has_b, float scale, float *diag, void *ws,
                                  hipStream_t st);
// launch_brick_gradient (no in-plane shifts) and launch_brick_hvp_probe with
// factor scale2 in one pass over the pixels (trilinear grids)
hipError_t launch_brick_gradient_probe(const Geom &g, const float *rot, const float *defocus, int64_t n,
                                       const float2 *vol, const float2 *x, float scale, float2 *accum, double *loss,
                                       uint64_t seed, uint64_t pa, uint64_t pb, int has_b, float scale2, float *diag,
                                       void *ws, hipStream_t st);
// the deterministic adjoint (fixed point; trilinear grids): scratch of
// 16 M^3 bytes (the 64-bit fixed-point volume, 16-byte aligned) and two words
// (input bounds), both in device memory
struct FxBuf {
    unsigned long long *fx;
    unsigned *maxbits;
};
hipError_t launch_brick_backproject_fx(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                       int64_t n, const float2 *img, int ctf_power, float scale, float2 *accum,
                                       const FxBuf &fb, void *ws, hipStream_t st);
hipError_t launch_brick_gradient_fx(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                    int64_t n, const float2 *vol, const float2 *x, float scale, float2 *accum,
                                    double *loss, const FxBuf &fb, void *ws, hipStream_t st);
hipError_t launch_brick_hvp_fx(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *z,
                               float scale, float2 *accum, const FxBuf &fb, void *ws, hipStream_t st);

// pixel-parallel kernels (pixel_kernels.hip)
hipError_t launch_project(const Geom &g, const float *rot, const float *defocus, const float *shift, int64_t n,
                          const float2 *vol, const float2 *subtract, float2 *out, double *loss, hipStream_t st);
hipError_t launch_backproject_atomic(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                     int64_t n, const float2 *img, int ctf_power, float scale, float2 *accum,
                                     hipStream_t st);
hipError_t launch_gradient_atomic(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                  int64_t n, const float2 *vol, const float2 *x, float scale, float2 *accum,
                                  double *loss, hipStream_t st);
hipError_t launch_hvp_atomic(const Geom &g, const float *rot, const float *defocus, int64_t n, const float2 *z,
                             float scale, float2 *accum, hipStream_t st);
hipError_t launch_sq_diag(const Geom &g, const float *rot, const float *defocus, int64_t n, float scale,
                          float *accum, hipStream_t st);

// voxel-parallel (owner computes) kernels (voxel_kernels.hip)
hipError_t launch_backproject_owner(const Geom &g, const float *rot, const float *defocus, const float *shift,
                                    int64_t n, const float2 *img, int ctf_power, float scale, float2 *accum,
                                    hipStream_t st);
hipError_t launch_features(const Geom &g, const float *rot, const float *defocus, int64_t n, float *ctf2,
                           float *cover, hipStream_t st);

// volume-wise kernels (volume_kernels.hip)
hipError_t launch_scaled_copy(float2 *out, const float2 *in, float lam, int64_t nvox, double *norm2, hipStream_t st);
hipError_t launch_fill_f64(double *p, int n, double v, hipStream_t st);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t st);
hipError_t launch_finish_loss(double *loss_out, const double *data, const double *norm2, float scale, float lam,
                              hipStream_t st);
hipError_t launch_rademacher(float *z, int64_t nvox, uint64_t seed, uint64_t probe, hipStream_t st);
// Rademacher probe pair z = z_pa + i z_pb (z_pb = 0 without has_b; voxel k
// takes bit k mod 128 of rademacher_block k / 128), never stored:
// probe_init writes hz = lam z; zhz_hash adds w (Re z Re hz + Im z Im hz) to
// diag (first: the sum starts with this pair, diag is written, not read).
// probe_init also writes z where z is not NULL (the nearest-neighbour
// kernels read it).  z and hz 16-byte aligned, nvox even.
hipError_t launch_probe_init(float2 *z, float2 *hz, int64_t nvox, uint64_t seed, uint64_t pa, uint64_t pb, int has_b,
                             float lam, hipStream_t st);
hipError_t launch_zhz_hash(float *diag, const float2 *hz, int64_t nvox, uint64_t seed, uint64_t pa, uint64_t pb,
                           int has_b, float w, bool first, hipStream_t st);
// fixed-point adjoint: maxbits[0..1] zeroed, then the bound of a (may be
// NULL) into maxbits[0] and a zeroed fx[0..2 nvox); img_absmax raises *dst
// to the bound of the images' disk pixels; finish adds fx / S to accum
hipError_t launch_fx_prep(const float2 *a, int64_t na, unsigned *maxbits, unsigned long long *fx, int64_t nvox,
                          hipStream_t st);
hipError_t launch_img_absmax(const Geom &g, const float2 *img, int64_t n, unsigned *dst, hipStream_t st);
hipError_t launch_fx_finish(float2 *out, const unsigned long long *fx, int64_t nvox, const unsigned *maxbits,
                            float scale, int64_t n, hipStream_t st);
hipError_t launch_shell_sums(const float2 *u, const float2 *v, int M, double *out, hipStream_t st);
hipError_t launch_alpha(const Geom &g, const float *defocus, int64_t n, int k2, double ratio, float lam,
                        double *alpha_out, hipStream_t st);
hipError_t launch_precond_step(int64_t nvox, const float2 *v, const float2 *g, float *D, float *D_avg,
                               const float *zHz, int64_t k, float beta, float alpha, float eta, float2 *v_out,
                               float *Dhat_out, double *stats, hipStream_t st);

// preconditioner network (mlp_kernels.hip)
int mlp_param_count();
hipError_t launch_mlp_forward(const float *params, const float *X, float *y, int64_t n, hipStream_t st);
hipError_t launch_learned_diag(const float *params, int M, float N, float lambda, const float *ctf2,
                               const float *cover, float *D, hipStream_t st);
size_t mlp_grad_workspace_bytes(int64_t n);
hipError_t launch_mlp_grad(const float *params, const float *X, const float *T, int64_t n, float *grad,
                           double *loss, void *ws, hipStream_t st);
hipError_t launch_mlp_adam(float *params, float *m, float *v, const float *grad, int step, float lr, float beta1,
                           float beta2, float eps, hipStream_t st);

}  // namespace csg
