// api.hip -- the C ABI of libcryosgd (declared in include/cryosgd.h):
// argument validation, workspace carving and kernel sequencing.  Every entry
// point only enqueues work on the caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <mutex>
#include <string>

#include "../../include/cryosgd.h"
#include "csg_internal.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return CSG_OK;
    return fail(CSG_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define CSG_TRY(expr, what)                         \
    do {                                            \
        int _rc = hip_check((expr), (what));        \
        if (_rc != CSG_OK) return _rc;              \
    } while (0)

// Relativistic electron wavelength in Angstrom:
// lambda = h / sqrt(2 m0 e V (1 + e V / (2 m0 c^2))), CODATA 2018 constants.
double electron_wavelength_A(double kv) {
    const double planck = 6.62607015e-34, electron_mass = 9.1093837015e-31;
    const double charge = 1.602176634e-19, light = 299792458.0;
    const double volts = kv * 1.0e3;
    const double p2 = 2.0 * electron_mass * charge * volts * (1.0 + charge * volts / (2.0 * electron_mass * light * light));
    return planck / sqrt(p2) * 1.0e10;
}

int make_geom(const csg_grid *grid, const csg_optics *optics, csg::Geom *g) {
    if (!grid) return fail(CSG_EINVAL, "grid descriptor is NULL");
    if (!optics) return fail(CSG_EINVAL, "optics descriptor is NULL");
    const int M = grid->M;
    if (M < 4 || M > 1024 || (M & 1)) return fail(CSG_EINVAL, "grid side M=%d must be even and in [4, 1024]", M);
    if (!(grid->r_max >= 0.0f) || grid->r_max > (float)(M / 2 - 1))
        return fail(CSG_EINVAL, "r_max=%g must lie in [0, M/2-1=%d]", (double)grid->r_max, M / 2 - 1);
    if (grid->interp != 0 && grid->interp != 1) return fail(CSG_EINVAL, "interp=%d must be 0 or 1", grid->interp);
    g->M = M;
    g->half = M / 2;
    g->interp = grid->interp;
    g->k2max = (int)floor((double)grid->r_max * (double)grid->r_max);
    g->ctf_on = optics->ctf_on ? 1 : 0;
    g->ctf_a = g->ctf_b = g->inv_s2 = g->phase0 = 0.0;
    if (g->ctf_on) {
        const double kv = optics->kv, cs = optics->cs_mm, A = optics->amp_contrast, px = optics->pixel_A;
        if (!(kv > 0.0) || !isfinite(kv)) return fail(CSG_EINVAL, "kv=%g must be positive", kv);
        if (!(px > 0.0) || !isfinite(px)) return fail(CSG_EINVAL, "pixel_A=%g must be positive", px);
        if (!(A >= 0.0 && A < 1.0)) return fail(CSG_EINVAL, "amp_contrast=%g must lie in [0, 1)", A);
        if (!(cs >= 0.0) || !isfinite(cs)) return fail(CSG_EINVAL, "cs_mm=%g must be non-negative", cs);
        const double lam = electron_wavelength_A(kv);
        g->ctf_a = 0.5 * lam;                          // chi/2pi = (lambda df / 2) s^2 ...
        g->ctf_b = 0.25 * cs * 1.0e7 * lam * lam * lam; // ... - (Cs lambda^3 / 4) s^4
        g->inv_s2 = 1.0 / ((double)M * px * (double)M * px);
        g->phase0 = asin(A) / (2.0 * M_PI);
    }
    return CSG_OK;
}

int check_poses(const csg_poses *p) {
    if (!p) return fail(CSG_EINVAL, "poses descriptor is NULL");
    if (p->n < 0) return fail(CSG_EINVAL, "n=%lld must be non-negative", (long long)p->n);
    if (p->n > 0 && (!p->rot || !p->defocus_A)) return fail(CSG_EINVAL, "rot and defocus_A must be non-NULL");
    return CSG_OK;
}

int64_t nvox_of(const csg::Geom &g) { return (int64_t)g.M * g.M * g.M; }

constexpr size_t kScalarBytes = 256;  // device scalars at the start of a workspace

size_t image_bytes(int M, int64_t n) { return (size_t)n * (size_t)M * (size_t)M * 8u; }

int need_workspace(void *ws, size_t have, size_t need, const char *who) {
    if (need == 0) return CSG_OK;
    if (!ws) return fail(CSG_EWORKSPACE, "%s: workspace of %zu bytes required, got NULL", who, need);
    if (have < need) return fail(CSG_EWORKSPACE, "%s: workspace of %zu bytes required, got %zu", who, need, have);
    if (((uintptr_t)ws & 255u) != 0) return fail(CSG_EWORKSPACE, "%s: workspace must be 256-byte aligned", who);
    return CSG_OK;
}

// The fixed-point scratch of the deterministic adjoint inside a workspace of
// kind CSG_WS_*_DETERMINISTIC: the input bounds in the scalar area, then the
// brick tables, then the fixed-point volume.
csg::FxBuf fx_buffers(void *ws, int M, int64_t n, void **brick_ws) {
    char *w = (char *)ws;
    *brick_ws = w + kScalarBytes;
    csg::FxBuf fb;
    fb.maxbits = (unsigned *)(w + 16);  // after the two double scalars
    fb.fx = (unsigned long long *)(w + kScalarBytes + csg::brick_workspace_bytes(M, n));
    return fb;
}

}  // namespace

extern "C" {

const char *csg_last_error(void) { return g_last_error.c_str(); }

size_t csg_workspace_bytes(const csg_grid *grid, int64_t n, int32_t which) {
    if (!grid || grid->M < 4 || grid->M > 1024 || (grid->M & 1) || n < 0) return 0;
    const int M = grid->M;
    const size_t vol = (size_t)M * M * M * 8u;
    const size_t bricks = csg::brick_workspace_bytes(M, n);
    // the deterministic adjoint: the fixed-point volume (two 64-bit integers
    // per voxel) beside the brick tables; the nearest-neighbour grids use the
    // owner-computes kernel instead (plus one image per batch image for the
    // gradient and the HVP)
    const bool trilinear = grid->interp != 0;
    const size_t fixed = kScalarBytes + bricks + 2 * vol;
    switch (which) {
        case CSG_WS_PROJECT: return bricks;
        case CSG_WS_BACKPROJECT: return bricks;
        case CSG_WS_BACKPROJECT_DETERMINISTIC: return trilinear ? fixed : 0;
        case CSG_WS_GRADIENT: return kScalarBytes + bricks;
        case CSG_WS_GRADIENT_DETERMINISTIC: return trilinear ? fixed : kScalarBytes + image_bytes(M, n);
        // trilinear: the brick tables (the probe pair is regenerated from its
        // hash in the staged bricks and z (.) H z goes straight into the
        // output); nearest neighbour: the product of a probe pair and the
        // stored pair
        case CSG_WS_HUTCHINSON: return kScalarBytes + (trilinear ? bricks : 2 * vol);
        // the larger of the two (nearest-neighbour grids run the two calls)
        case CSG_WS_GRADIENT_HUTCHINSON: return kScalarBytes + (trilinear || bricks > 2 * vol ? bricks : 2 * vol);
        default: return 0;
    }
}

int csg_project(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, const float *vol,
                const float *subtract, float *out, double *loss_accum, void *workspace, size_t workspace_bytes,
                void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (poses->n == 0) return CSG_OK;
    if (!vol) return fail(CSG_EINVAL, "csg_project: vol is NULL");
    if (!out && !loss_accum) return fail(CSG_EINVAL, "csg_project: need out or loss_accum");
    if (out && out == vol) return fail(CSG_EINVAL, "csg_project: out must not alias vol");
    const size_t need = csg_workspace_bytes(grid, poses->n, CSG_WS_PROJECT);
    if ((rc = need_workspace(workspace, workspace_bytes, need, "csg_project"))) return rc;
    CSG_TRY(csg::launch_brick_project(g, poses->rot, poses->defocus_A, poses->shift_px, poses->n,
                                      (const float2 *)vol, (const float2 *)subtract, (float2 *)out, loss_accum,
                                      workspace, (hipStream_t)stream),
            "csg_project");
    return CSG_OK;
}

int csg_backproject(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, const float *img,
                    int32_t ctf_power, float scale, float *vol_accum, int32_t deterministic, void *workspace,
                    size_t workspace_bytes, void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (ctf_power < 0 || ctf_power > 2) return fail(CSG_EINVAL, "ctf_power=%d must be 0, 1 or 2", ctf_power);
    if (poses->n == 0) return CSG_OK;
    if (!img || !vol_accum) return fail(CSG_EINVAL, "csg_backproject: img and vol_accum must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    if (deterministic && g.interp == 0) {
        CSG_TRY(csg::launch_backproject_owner(g, poses->rot, poses->defocus_A, poses->shift_px, poses->n,
                                              (const float2 *)img, ctf_power, scale, (float2 *)vol_accum, st),
                "csg_backproject");
    } else if (deterministic) {
        const size_t need = csg_workspace_bytes(grid, poses->n, CSG_WS_BACKPROJECT_DETERMINISTIC);
        if ((rc = need_workspace(workspace, workspace_bytes, need, "csg_backproject"))) return rc;
        void *bws;
        const csg::FxBuf fb = fx_buffers(workspace, g.M, poses->n, &bws);
        CSG_TRY(csg::launch_brick_backproject_fx(g, poses->rot, poses->defocus_A, poses->shift_px, poses->n,
                                                 (const float2 *)img, ctf_power, scale, (float2 *)vol_accum, fb, bws,
                                                 st),
                "csg_backproject");
    } else {
        const size_t need = csg_workspace_bytes(grid, poses->n, CSG_WS_BACKPROJECT);
        if ((rc = need_workspace(workspace, workspace_bytes, need, "csg_backproject"))) return rc;
        CSG_TRY(csg::launch_brick_backproject(g, poses->rot, poses->defocus_A, poses->shift_px, poses->n,
                                              (const float2 *)img, ctf_power, scale, (float2 *)vol_accum, workspace,
                                              st),
                "csg_backproject");
    }
    return CSG_OK;
}

int csg_gradient(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, const float *vol,
                 const float *x, float scale, float lambda, float *grad_out, double *loss_out, int32_t deterministic,
                 void *workspace, size_t workspace_bytes, void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (!vol || !grad_out || (poses->n > 0 && !x))
        return fail(CSG_EINVAL, "csg_gradient: vol, x and grad_out must be non-NULL");
    if (vol == grad_out) return fail(CSG_EINVAL, "csg_gradient: grad_out must not alias vol");
    const size_t need = csg_workspace_bytes(grid, poses->n, deterministic ? CSG_WS_GRADIENT_DETERMINISTIC : CSG_WS_GRADIENT);
    if ((rc = need_workspace(workspace, workspace_bytes, need, "csg_gradient"))) return rc;
    hipStream_t st = (hipStream_t)stream;
    double *sc = (double *)workspace;  // sc[0] = 1/2 sum |r|^2, sc[1] = ||v||^2
    const int64_t nv = nvox_of(g);
    CSG_TRY(csg::launch_fill_f64(sc, 2, 0.0, st), "csg_gradient");
    CSG_TRY(csg::launch_scaled_copy((float2 *)grad_out, (const float2 *)vol, lambda, nv, sc + 1, st), "csg_gradient");
    if (poses->n > 0) {
        if (!deterministic) {
            CSG_TRY(csg::launch_brick_gradient(g, poses->rot, poses->defocus_A, poses->shift_px, poses->n,
                                               (const float2 *)vol, (const float2 *)x, scale, (float2 *)grad_out, sc,
                                               (char *)workspace + kScalarBytes, st),
                    "csg_gradient");
        } else if (g.interp != 0) {
            void *bws;
            const csg::FxBuf fb = fx_buffers(workspace, g.M, poses->n, &bws);
            CSG_TRY(csg::launch_brick_gradient_fx(g, poses->rot, poses->defocus_A, poses->shift_px, poses->n,
                                                  (const float2 *)vol, (const float2 *)x, scale, (float2 *)grad_out,
                                                  sc, fb, bws, st),
                    "csg_gradient");
        } else {
            float2 *resid = (float2 *)((char *)workspace + kScalarBytes);
            CSG_TRY(csg::launch_project(g, poses->rot, poses->defocus_A, poses->shift_px, poses->n,
                                        (const float2 *)vol, (const float2 *)x, resid, sc, st),
                    "csg_gradient");
            CSG_TRY(csg::launch_backproject_owner(g, poses->rot, poses->defocus_A, poses->shift_px, poses->n, resid,
                                                  1, scale, (float2 *)grad_out, st),
                    "csg_gradient");
        }
    }
    if (loss_out) CSG_TRY(csg::launch_finish_loss(loss_out, sc, sc + 1, scale, lambda, st), "csg_gradient");
    return CSG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free gradient: the scratch of csg_gradient (device scalars and
// the brick tables) in a static device array, one per GPU, held until the
// process ends.  Host code uses the array only through the device address
// that hipGetSymbolAddress returns for the current device.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kStaticScratchBytes = CSG_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch, looked up on the first call
// on that device.
int static_scratch(void **out) {
    int dev = -1;
    CSG_TRY(hipGetDevice(&dev), "csg_gradient_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(CSG_EINVAL, "csg_gradient_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        CSG_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "csg_gradient_noalloc: hipGetSymbolAddress(scratch)");
        if (!p || ((uintptr_t)p & 255u) != 0)
            return fail(CSG_EHIP, "csg_gradient_noalloc: scratch address %p is not 256-byte aligned", p);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CSG_OK;
}

}  // namespace

extern "C" {

int csg_gradient_noalloc(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, const float *vol,
                         const float *x, float scale, float lambda, float *grad_out, double *loss_out, void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (!vol || !grad_out || (poses->n > 0 && !x))
        return fail(CSG_EINVAL, "csg_gradient_noalloc: vol, x and grad_out must be non-NULL");
    if (vol == grad_out) return fail(CSG_EINVAL, "csg_gradient_noalloc: grad_out must not alias vol");
    // images per launch: all of them, or the most whose brick tables fit (the
    // table size grows with the images per launch)
    int64_t sub = poses->n < csg::kBrickSubBatch ? poses->n : csg::kBrickSubBatch;
    if (sub < 1) sub = 1;
    if (g.interp != 0) {
        auto fits = [&](int64_t s) { return kScalarBytes + csg::brick_workspace_bytes_sub(g.M, s) <= kStaticScratchBytes; };
        if (!fits(sub)) {
            int64_t lo = 0, hi = sub;  // fits(lo) or lo == 0; !fits(hi)
            while (hi - lo > 1) {
                const int64_t mid = lo + (hi - lo) / 2;
                if (fits(mid)) lo = mid;
                else hi = mid;
            }
            sub = lo;
        }
        if (sub < 1)
            return fail(CSG_EWORKSPACE,
                        "csg_gradient_noalloc: grid M=%d needs %zu bytes of scratch for one image per launch; the "
                        "static scratch holds %zu",
                        g.M, kScalarBytes + csg::brick_workspace_bytes_sub(g.M, 1), kStaticScratchBytes);
    }
    void *ws = nullptr;
    if ((rc = static_scratch(&ws))) return rc;
    hipStream_t st = (hipStream_t)stream;
    double *sc = (double *)ws;  // sc[0] = 1/2 sum |r|^2, sc[1] = ||v||^2 (cleared by a kernel)
    const int64_t nv = nvox_of(g);
    CSG_TRY(csg::launch_fill_f64(sc, 2, 0.0, st), "csg_gradient_noalloc");
    CSG_TRY(csg::launch_scaled_copy((float2 *)grad_out, (const float2 *)vol, lambda, nv, sc + 1, st),
            "csg_gradient_noalloc");
    if (poses->n > 0)
        CSG_TRY(csg::launch_brick_gradient(g, poses->rot, poses->defocus_A, poses->shift_px, poses->n,
                                           (const float2 *)vol, (const float2 *)x, scale, (float2 *)grad_out, sc,
                                           (char *)ws + kScalarBytes, st, sub, /*timed=*/false),
                "csg_gradient_noalloc");
    if (loss_out) CSG_TRY(csg::launch_finish_loss(loss_out, sc, sc + 1, scale, lambda, st), "csg_gradient_noalloc");
    return CSG_OK;
}

int csg_hvp(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, const float *z, float scale,
            float lambda, float *hz_out, int32_t deterministic, void *workspace, size_t workspace_bytes,
            void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (!z || !hz_out) return fail(CSG_EINVAL, "csg_hvp: z and hz_out must be non-NULL");
    if (z == hz_out) return fail(CSG_EINVAL, "csg_hvp: hz_out must not alias z");
    {
        const size_t need = csg_workspace_bytes(grid, poses->n, deterministic ? CSG_WS_GRADIENT_DETERMINISTIC
                                                                              : CSG_WS_GRADIENT);
        if ((rc = need_workspace(workspace, workspace_bytes, need, "csg_hvp"))) return rc;
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t nv = nvox_of(g);
    CSG_TRY(csg::launch_scaled_copy((float2 *)hz_out, (const float2 *)z, lambda, nv, nullptr, st), "csg_hvp");
    if (poses->n == 0) return CSG_OK;
    if (!deterministic) {
        CSG_TRY(csg::launch_brick_hvp(g, poses->rot, poses->defocus_A, poses->n, (const float2 *)z, scale,
                                      (float2 *)hz_out, (char *)workspace + kScalarBytes, st),
                "csg_hvp");
    } else if (g.interp != 0) {
        void *bws;
        const csg::FxBuf fb = fx_buffers(workspace, g.M, poses->n, &bws);
        CSG_TRY(csg::launch_brick_hvp_fx(g, poses->rot, poses->defocus_A, poses->n, (const float2 *)z, scale,
                                         (float2 *)hz_out, fb, bws, st),
                "csg_hvp");
    } else {
        float2 *img = (float2 *)((char *)workspace + kScalarBytes);
        // T^* T = I: the Hessian does not involve the in-plane shifts
        CSG_TRY(csg::launch_project(g, poses->rot, poses->defocus_A, nullptr, poses->n, (const float2 *)z, nullptr,
                                    img, nullptr, st),
                "csg_hvp");
        CSG_TRY(csg::launch_backproject_owner(g, poses->rot, poses->defocus_A, nullptr, poses->n, img, 1, scale,
                                              (float2 *)hz_out, st),
                "csg_hvp");
    }
    return CSG_OK;
}

int csg_rademacher(int64_t nvox, uint64_t seed, int64_t probe, float *z_out, void *stream) {
    if (nvox < 0) return fail(CSG_EINVAL, "csg_rademacher: nvox must be non-negative");
    if (nvox == 0) return CSG_OK;
    if (!z_out) return fail(CSG_EINVAL, "csg_rademacher: z_out is NULL");
    CSG_TRY(csg::launch_rademacher(z_out, nvox, seed, (uint64_t)probe, (hipStream_t)stream), "csg_rademacher");
    return CSG_OK;
}

int csg_hutchinson_diag(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, int32_t n_probe,
                        uint64_t seed, int64_t probe0, float scale, float lambda, float *diag_out, void *workspace,
                        size_t workspace_bytes, void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (n_probe < 1) return fail(CSG_EINVAL, "csg_hutchinson_diag: n_probe=%d must be >= 1", n_probe);
    if (!diag_out) return fail(CSG_EINVAL, "csg_hutchinson_diag: diag_out is NULL");
    const size_t need = csg_workspace_bytes(grid, poses->n, CSG_WS_HUTCHINSON);
    if ((rc = need_workspace(workspace, workspace_bytes, need, "csg_hutchinson_diag"))) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int64_t nv = nvox_of(g);
    const float w = 1.0f / (float)n_probe;
    if (g.interp != 0) {
        // Trilinear grids: z (.) H z summed over the probes in place.  The
        // lambda term of every probe is lambda z (.) z = lambda, so the mean
        // over the probes starts from lambda; each pair's brick kernel then
        // adds w z (.) (scale P^T C^2 P z) with the pair regenerated from its
        // hash in the staged bricks (the workspace holds the brick tables).
        void *bws = (char *)workspace + kScalarBytes;
        CSG_TRY(csg::launch_fill_f32(diag_out, nv, lambda, st), "csg_hutchinson_diag");
        for (int32_t p = 0; p < n_probe && poses->n > 0; p += 2) {
            const int has_b = (p + 1 < n_probe) ? 1 : 0;
            CSG_TRY(csg::launch_brick_hvp_probe(g, poses->rot, poses->defocus_A, poses->n, seed,
                                                (uint64_t)(probe0 + p), (uint64_t)(probe0 + p + 1), has_b, scale * w,
                                                diag_out, bws, st),
                    "csg_hutchinson_diag");
        }
        return CSG_OK;
    }
    // nearest neighbour: hz = H z of each pair in the workspace (beside the
    // stored pair z), then z (.) hz
    float2 *hz = (float2 *)((char *)workspace + kScalarBytes);
    float2 *z = hz + nv;
    for (int32_t p = 0; p < n_probe; p += 2) {
        const int has_b = (p + 1 < n_probe) ? 1 : 0;
        const uint64_t pa = (uint64_t)(probe0 + p), pb = (uint64_t)(probe0 + p + 1);
        // hz = lambda z (and z itself for the nearest-neighbour kernels)
        CSG_TRY(csg::launch_probe_init(z, hz, nv, seed, pa, pb, has_b, lambda, st), "csg_hutchinson_diag");
        if (poses->n > 0)
            CSG_TRY(csg::launch_brick_hvp(g, poses->rot, poses->defocus_A, poses->n, z, scale, hz, nullptr, st),
                    "csg_hutchinson_diag");
        CSG_TRY(csg::launch_zhz_hash(diag_out, hz, nv, seed, pa, pb, has_b, w, /*first=*/p == 0, st),
                "csg_hutchinson_diag");
    }
    return CSG_OK;
}

int csg_gradient_hutchinson(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, const float *vol,
                            const float *x, float scale, float lambda, float *grad_out, double *loss_out,
                            int32_t n_probe, uint64_t seed, int64_t probe0, float *diag_out, void *workspace,
                            size_t workspace_bytes, void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (n_probe < 1) return fail(CSG_EINVAL, "csg_gradient_hutchinson: n_probe=%d must be >= 1", n_probe);
    if (!vol || !grad_out || !diag_out || (poses->n > 0 && !x))
        return fail(CSG_EINVAL, "csg_gradient_hutchinson: vol, x, grad_out and diag_out must be non-NULL");
    if (vol == grad_out || (const void *)vol == (const void *)diag_out || (void *)grad_out == (void *)diag_out)
        return fail(CSG_EINVAL, "csg_gradient_hutchinson: vol, grad_out and diag_out must not alias");
    const size_t need = csg_workspace_bytes(grid, poses->n, CSG_WS_GRADIENT_HUTCHINSON);
    if ((rc = need_workspace(workspace, workspace_bytes, need, "csg_gradient_hutchinson"))) return rc;
    if (g.interp == 0 || poses->shift_px || poses->n == 0) {
        // the two separate paths (their workspaces are no larger than this one)
        rc = csg_gradient(grid, optics, poses, vol, x, scale, lambda, grad_out, loss_out, 0, workspace,
                          workspace_bytes, stream);
        if (rc) return rc;
        return csg_hutchinson_diag(grid, optics, poses, n_probe, seed, probe0, scale, lambda, diag_out, workspace,
                                   workspace_bytes, stream);
    }
    hipStream_t st = (hipStream_t)stream;
    double *sc = (double *)workspace;  // sc[0] = 1/2 sum |r|^2, sc[1] = ||v||^2
    void *bws = (char *)workspace + kScalarBytes;
    const int64_t nv = nvox_of(g);
    const float w = 1.0f / (float)n_probe;
    CSG_TRY(csg::launch_fill_f64(sc, 2, 0.0, st), "csg_gradient_hutchinson");
    CSG_TRY(csg::launch_scaled_copy((float2 *)grad_out, (const float2 *)vol, lambda, nv, sc + 1, st),
            "csg_gradient_hutchinson");
    // the lambda term of every probe is lambda z (.) z = lambda (as in csg_hutchinson_diag)
    CSG_TRY(csg::launch_fill_f32(diag_out, nv, lambda, st), "csg_gradient_hutchinson");
    CSG_TRY(csg::launch_brick_gradient_probe(g, poses->rot, poses->defocus_A, poses->n, (const float2 *)vol,
                                             (const float2 *)x, scale, (float2 *)grad_out, sc, seed,
                                             (uint64_t)probe0, (uint64_t)(probe0 + 1), n_probe > 1 ? 1 : 0,
                                             scale * w, diag_out, bws, st),
            "csg_gradient_hutchinson");
    for (int32_t p = 2; p < n_probe; p += 2) {
        const int has_b = (p + 1 < n_probe) ? 1 : 0;
        CSG_TRY(csg::launch_brick_hvp_probe(g, poses->rot, poses->defocus_A, poses->n, seed, (uint64_t)(probe0 + p),
                                            (uint64_t)(probe0 + p + 1), has_b, scale * w, diag_out, bws, st),
                "csg_gradient_hutchinson");
    }
    if (loss_out)
        CSG_TRY(csg::launch_finish_loss(loss_out, sc, sc + 1, scale, lambda, st), "csg_gradient_hutchinson");
    return CSG_OK;
}

int csg_exact_diag(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, float scale, float lambda,
                   float *diag_out, void *workspace, size_t workspace_bytes, void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (!diag_out) return fail(CSG_EINVAL, "csg_exact_diag: diag_out is NULL");
    const size_t need = csg_workspace_bytes(grid, poses->n, CSG_WS_BACKPROJECT);
    if ((rc = need_workspace(workspace, workspace_bytes, need, "csg_exact_diag"))) return rc;
    hipStream_t st = (hipStream_t)stream;
    CSG_TRY(csg::launch_fill_f32(diag_out, nvox_of(g), lambda, st), "csg_exact_diag");
    if (poses->n > 0)
        CSG_TRY(csg::launch_brick_sq_diag(g, poses->rot, poses->defocus_A, poses->n, scale, diag_out, workspace, st),
                "csg_exact_diag");
    return CSG_OK;
}

int csg_features(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, float *ctf2_accum,
                 float *cover_accum, void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (!ctf2_accum || !cover_accum) return fail(CSG_EINVAL, "csg_features: outputs must be non-NULL");
    if (poses->n == 0) return CSG_OK;
    CSG_TRY(csg::launch_features(g, poses->rot, poses->defocus_A, poses->n, ctf2_accum, cover_accum,
                                 (hipStream_t)stream),
            "csg_features");
    return CSG_OK;
}

int csg_threshold_alpha(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, float lambda,
                        double *alpha_out, void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (!alpha_out) return fail(CSG_EINVAL, "csg_threshold_alpha: alpha_out is NULL");
    const int R = (int)lrint((double)grid->r_max);
    if (R < 1) return fail(CSG_EINVAL, "csg_threshold_alpha: r_max must round to at least 1");
    // Shell counts: round(|k|) == R  <=>  R^2 - R + 1 <= |k|^2 <= R^2 + R
    // (|k|^2 is an integer and |k| is never exactly R + 1/2).
    const int64_t lo = (int64_t)R * R - R + 1, hi = (int64_t)R * R + R;
    const int h = g.half;
    int64_t px = 0, pv = 0;
    for (int y = -h; y < h; ++y)
        for (int x = -h; x < h; ++x) {
            const int64_t r2 = (int64_t)x * x + (int64_t)y * y;
            if (r2 >= lo && r2 <= hi) ++px;
        }
    for (int z = -h; z < h; ++z) {
        const int64_t z2 = (int64_t)z * z;
        if (z2 > hi) continue;
        for (int y = -h; y < h; ++y) {
            const int64_t yz = z2 + (int64_t)y * y;
            if (yz > hi) continue;
            for (int x = -h; x < h; ++x) {
                const int64_t r2 = yz + (int64_t)x * x;
                if (r2 >= lo && r2 <= hi) ++pv;
            }
        }
    }
    if (pv == 0) return fail(CSG_EINVAL, "csg_threshold_alpha: empty voxel shell");
    const double ratio = (double)px / (double)pv;
    CSG_TRY(csg::launch_alpha(g, poses->defocus_A, poses->n, R * R, ratio, lambda, alpha_out, (hipStream_t)stream),
            "csg_threshold_alpha");
    return CSG_OK;
}

int csg_feature_sums(const csg_grid *grid, const csg_optics *optics, const csg_poses *poses, float *accum,
                     void *workspace, size_t workspace_bytes, void *stream) {
    csg::Geom g;
    int rc = make_geom(grid, optics, &g);
    if (rc) return rc;
    if ((rc = check_poses(poses))) return rc;
    if (g.interp != 1) return fail(CSG_EINVAL, "csg_feature_sums: trilinear grids only");
    if (!accum) return fail(CSG_EINVAL, "csg_feature_sums: accum is NULL");
    if (poses->n == 0) return CSG_OK;
    const size_t need = csg_workspace_bytes(grid, poses->n, CSG_WS_BACKPROJECT);
    if ((rc = need_workspace(workspace, workspace_bytes, need, "csg_feature_sums"))) return rc;
    CSG_TRY(csg::launch_brick_feature_sums(g, poses->rot, poses->defocus_A, poses->n, (float2 *)accum, workspace,
                                           (hipStream_t)stream),
            "csg_feature_sums");
    return CSG_OK;
}

int csg_precond_sgd_step(int64_t nvox, const float *v, const float *g, float *D, float *D_avg, const float *zHz,
                         int64_t k, float beta, float alpha, float eta, float *v_out, float *Dhat_out,
                         double *stats_out, void *stream) {
    if (nvox < 0) return fail(CSG_EINVAL, "csg_precond_sgd_step: nvox must be non-negative");
    const bool d_only = !v && !g && !v_out && !stats_out;
    if (d_only && !(D && zHz))
        return fail(CSG_EINVAL, "csg_precond_sgd_step: the diagonal update alone needs D, D_avg and zHz");
    if (!d_only && (!v || !g || !v_out || !stats_out))
        return fail(CSG_EINVAL, "csg_precond_sgd_step: v, g, v_out and stats_out must be non-NULL");
    if (zHz && (!D || !D_avg)) return fail(CSG_EINVAL, "csg_precond_sgd_step: a probe sample needs D and D_avg");
    if (zHz && k < 1) return fail(CSG_EINVAL, "csg_precond_sgd_step: iteration k=%lld must be >= 1", (long long)k);
    if (!d_only && v_out == g) return fail(CSG_EINVAL, "csg_precond_sgd_step: v_out must not alias g");
    if (!(eta >= 0.0f)) return fail(CSG_EINVAL, "csg_precond_sgd_step: eta must be non-negative");
    if (D && !(alpha >= 0.0f)) return fail(CSG_EINVAL, "csg_precond_sgd_step: alpha must be non-negative");
    CSG_TRY(csg::launch_precond_step(nvox, (const float2 *)v, (const float2 *)g, D, D_avg, zHz, k, beta, alpha, eta,
                                     (float2 *)v_out, Dhat_out, stats_out, (hipStream_t)stream),
            "csg_precond_sgd_step");
    return CSG_OK;
}

int32_t csg_mlp_param_count(void) { return (int32_t)csg::mlp_param_count(); }

int csg_mlp_forward(const float *params, const float *X, int64_t n, float *y, void *stream) {
    if (n < 0) return fail(CSG_EINVAL, "csg_mlp_forward: n must be non-negative");
    if (n == 0) return CSG_OK;
    if (!params || !X || !y) return fail(CSG_EINVAL, "csg_mlp_forward: params, X and y must be non-NULL");
    CSG_TRY(csg::launch_mlp_forward(params, X, y, n, (hipStream_t)stream), "csg_mlp_forward");
    return CSG_OK;
}

size_t csg_mlp_grad_workspace_bytes(int64_t n) { return n < 0 ? 0 : csg::mlp_grad_workspace_bytes(n); }

int csg_mlp_grad(const float *params, const float *X, const float *T, int64_t n, float *grad, double *loss_out,
                 void *workspace, size_t workspace_bytes, void *stream) {
    if (n < 0) return fail(CSG_EINVAL, "csg_mlp_grad: n must be non-negative");
    if (!params || !grad || !loss_out || (n > 0 && (!X || !T)))
        return fail(CSG_EINVAL, "csg_mlp_grad: params, X, T, grad and loss_out must be non-NULL");
    int rc;
    if (n > 0 && (rc = need_workspace(workspace, workspace_bytes, csg::mlp_grad_workspace_bytes(n), "csg_mlp_grad")))
        return rc;
    CSG_TRY(csg::launch_mlp_grad(params, X, T, n, grad, loss_out, workspace, (hipStream_t)stream), "csg_mlp_grad");
    return CSG_OK;
}

int csg_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr, float beta1,
                 float beta2, float eps, void *stream) {
    if (!params || !m || !v || !grad) return fail(CSG_EINVAL, "csg_mlp_adam: buffers must be non-NULL");
    if (step < 1) return fail(CSG_EINVAL, "csg_mlp_adam: step must be >= 1");
    if (!(lr >= 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(CSG_EINVAL, "csg_mlp_adam: invalid hyper-parameters");
    CSG_TRY(csg::launch_mlp_adam(params, m, v, grad, step, lr, beta1, beta2, eps, (hipStream_t)stream),
            "csg_mlp_adam");
    return CSG_OK;
}

int csg_learned_diag(const csg_grid *grid, int64_t n_images, float lambda, const float *params, const float *ctf2,
                     const float *cover, float *diag_out, void *stream) {
    if (!grid || grid->M < 4 || grid->M > 1024 || (grid->M & 1))
        return fail(CSG_EINVAL, "csg_learned_diag: invalid grid");
    if (n_images < 1) return fail(CSG_EINVAL, "csg_learned_diag: n_images must be >= 1");
    if (!params || !ctf2 || !cover || !diag_out) return fail(CSG_EINVAL, "csg_learned_diag: NULL buffer");
    CSG_TRY(csg::launch_learned_diag(params, grid->M, (float)n_images, lambda, ctf2, cover, diag_out,
                                     (hipStream_t)stream),
            "csg_learned_diag");
    return CSG_OK;
}

}  // extern "C"

extern "C" int csg_timing_enable(int32_t on) {
    csg::timing_set(on);
    return CSG_OK;
}

extern "C" int csg_timing_read(int32_t kernel, double *total_ms, int64_t *launches) {
    if (kernel < 0 || kernel >= csg::kTimedKernels) return fail(CSG_EINVAL, "timing: kernel %d out of range", kernel);
    if (!total_ms || !launches) return fail(CSG_EINVAL, "timing: NULL output pointer");
    CSG_TRY(csg::timing_read(kernel, total_ms, launches), "csg_timing_read");
    return CSG_OK;
}

extern "C" int csg_shell_sums(const csg_grid *grid, const float *u, const float *v, double *sums_out, void *stream) {
    if (!grid || grid->M < 4 || grid->M > 1024 || (grid->M & 1)) return fail(CSG_EINVAL, "csg_shell_sums: invalid grid");
    if (!u || !v || !sums_out) return fail(CSG_EINVAL, "csg_shell_sums: NULL buffer");
    CSG_TRY(csg::launch_shell_sums((const float2 *)u, (const float2 *)v, grid->M, sums_out, (hipStream_t)stream),
            "csg_shell_sums");
    return CSG_OK;
}

