"""Thin ctypes binding of libcryosgd (include/cryosgd.h).

Argument marshalling only: every call hands device pointers of torch tensors
and the current HIP stream to the C ABI; all arithmetic runs in the library's
HIP kernels.  If the library is missing the import of any function here fails
loudly -- there is no fallback.

Tensors: volumes complex64 [M,M,M]; images complex64 [n,M,M]; rotations
float32 [n,3,3]; defocus float32 [n] (Angstrom); all on the same CUDA (HIP)
device and contiguous.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcryosgd.so")

CSG_WS_BACKPROJECT = 0
CSG_WS_HUTCHINSON = 1
CSG_WS_GRADIENT = 2
CSG_WS_GRADIENT_DETERMINISTIC = 3
CSG_WS_PROJECT = 4
CSG_WS_BACKPROJECT_DETERMINISTIC = 5
CSG_WS_GRADIENT_HUTCHINSON = 6


class CsgError(RuntimeError):
    pass


class _Grid(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("r_max", ctypes.c_float), ("interp", ctypes.c_int32)]


class _Optics(ctypes.Structure):
    _fields_ = [("kv", ctypes.c_float), ("cs_mm", ctypes.c_float), ("amp_contrast", ctypes.c_float),
                ("pixel_A", ctypes.c_float), ("ctf_on", ctypes.c_int32)]


class _Poses(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rot", ctypes.c_void_p), ("defocus_A", ctypes.c_void_p),
                ("shift_px", ctypes.c_void_p)]


EXPORTS = {
    "csg_project": [ctypes.c_void_p] * 7 + [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "csg_backproject": [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_float, ctypes.c_void_p, ctypes.c_int32,
                                                 ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "csg_gradient": [ctypes.c_void_p] * 5 + [ctypes.c_float, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "csg_gradient_noalloc": [ctypes.c_void_p] * 5 + [ctypes.c_float, ctypes.c_float, ctypes.c_void_p,
                                                     ctypes.c_void_p, ctypes.c_void_p],
    "csg_hvp": [ctypes.c_void_p] * 4 + [ctypes.c_float, ctypes.c_float, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "csg_rademacher": [ctypes.c_int64, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
    "csg_hutchinson_diag": [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_float,
                                                    ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                                    ctypes.c_size_t, ctypes.c_void_p],
    "csg_gradient_hutchinson": [ctypes.c_void_p] * 5 + [ctypes.c_float, ctypes.c_float, ctypes.c_void_p,
                                                        ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint64,
                                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                                        ctypes.c_size_t, ctypes.c_void_p],
    "csg_exact_diag": [ctypes.c_void_p] * 3 + [ctypes.c_float, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                               ctypes.c_size_t, ctypes.c_void_p],
    "csg_features": [ctypes.c_void_p] * 5 + [ctypes.c_void_p],
    "csg_precond_sgd_step": [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                             ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "csg_threshold_alpha": [ctypes.c_void_p] * 3 + [ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p],
    "csg_feature_sums": [ctypes.c_void_p] * 4 + [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "csg_mlp_param_count": [],
    "csg_mlp_forward": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
    "csg_mlp_grad": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
    "csg_mlp_grad_workspace_bytes": [ctypes.c_int64],
    "csg_mlp_adam": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                     ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_void_p],
    "csg_learned_diag": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "csg_workspace_bytes": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32],
    "csg_shell_sums": [ctypes.c_void_p] * 4 + [ctypes.c_void_p],
    "csg_timing_enable": [ctypes.c_int32],
    "csg_timing_read": [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p],
    "csg_last_error": [],
}

_lib = None


def lib() -> ctypes.CDLL:
    """Load libcryosgd.so (built in-tree by paper_2311_16100_amd/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise CsgError("libcryosgd.so is not built (%s); run `python paper_2311_16100_amd/build.py`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, args in EXPORTS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.csg_workspace_bytes.restype = ctypes.c_size_t
        L.csg_mlp_grad_workspace_bytes.restype = ctypes.c_size_t
        L.csg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().csg_last_error().decode(errors="replace")
        raise CsgError("%s failed (%d): %s" % (what, rc, msg))


@dataclass(frozen=True)
class Grid:
    M: int
    r_max: float | None = None
    interp: int = 1

    @property
    def rmax(self) -> float:
        return float(self.M // 2 - 1) if self.r_max is None else float(self.r_max)

    def c(self) -> _Grid:
        return _Grid(int(self.M), float(self.rmax), int(self.interp))


@dataclass(frozen=True)
class Optics:
    kv: float = 300.0
    cs_mm: float = 2.7
    amp_contrast: float = 0.1
    pixel_A: float = 1.0
    ctf_on: bool = True

    def c(self) -> _Optics:
        return _Optics(self.kv, self.cs_mm, self.amp_contrast, self.pixel_A, int(self.ctf_on))


NO_CTF = Optics(ctf_on=False)


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise CsgError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise CsgError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _poses(rot: torch.Tensor, defocus: torch.Tensor, shift: torch.Tensor | None = None) -> _Poses:
    if rot.dtype != torch.float32 or defocus.dtype != torch.float32:
        raise CsgError("rotations and defocus must be float32")
    n = rot.shape[0] if rot.dim() == 3 else rot.numel() // 9
    if rot.numel() != 9 * n or defocus.numel() != n:
        raise CsgError("rot must be [n,3,3] and defocus [n]")
    if shift is not None and (shift.dtype != torch.float32 or shift.numel() != 2 * n):
        raise CsgError("shift must be float32 [n,2]")
    return _Poses(n, _ptr(rot), _ptr(defocus), _ptr(shift))


def _cplx(t: torch.Tensor, shape, name):
    if t.dtype != torch.complex64:
        raise CsgError("%s must be complex64" % name)
    if tuple(t.shape) != tuple(shape):
        raise CsgError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    return _ptr(t)


def workspace_bytes(grid: Grid, n: int, which: int) -> int:
    g = grid.c()
    return int(lib().csg_workspace_bytes(ctypes.byref(g), int(n), int(which)))


def alloc_workspace(grid: Grid, n: int, which: int, device=None) -> torch.Tensor | None:
    nb = workspace_bytes(grid, n, which)
    if nb == 0:
        return None
    ws = torch.empty(nb, dtype=torch.uint8, device=device or "cuda")
    if ws.data_ptr() % 256:
        raise CsgError("workspace allocation is not 256-byte aligned")
    return ws


def _ws(ws):
    return (None, 0) if ws is None else (_ptr(ws), ws.numel())


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI without the csg_ prefix)
# ---------------------------------------------------------------------------
def project(grid: Grid, optics: Optics, rot, defocus, vol, subtract=None, out=None, loss=None,
            want_out: bool = True, workspace=None, stream=None, shift=None):
    """C T P v (- subtract) for each image; returns `out` (allocated if None).
    `shift`: float32 [n,2] in-plane shifts in pixels (None: no shift)."""
    M = grid.M
    p = _poses(rot, defocus, shift)
    if want_out and out is None:
        out = torch.empty((p.n, M, M), dtype=torch.complex64, device=vol.device)
    if workspace is None:
        workspace = alloc_workspace(grid, p.n, CSG_WS_PROJECT, vol.device)
    g, o = grid.c(), optics.c()
    wp, wn = _ws(workspace)
    _check(lib().csg_project(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), _cplx(vol, (M, M, M), "vol"),
                             None if subtract is None else _cplx(subtract, (p.n, M, M), "subtract"),
                             None if out is None else _cplx(out, (p.n, M, M), "out"),
                             None if loss is None else _ptr(loss), wp, wn, _stream(stream)), "csg_project")
    return out


def backproject(grid: Grid, optics: Optics, rot, defocus, img, ctf_power: int = 1, scale: float = 1.0,
                accum=None, deterministic: bool = False, workspace=None, stream=None, shift=None):
    """accum += scale P^T T^* C^p img; returns accum (zeros if None)."""
    M = grid.M
    p = _poses(rot, defocus, shift)
    if accum is None:
        accum = torch.zeros((M, M, M), dtype=torch.complex64, device=img.device)
    if workspace is None:
        workspace = alloc_workspace(grid, p.n, CSG_WS_BACKPROJECT_DETERMINISTIC if deterministic else CSG_WS_BACKPROJECT,
                                    img.device)
    g, o = grid.c(), optics.c()
    wp, wn = _ws(workspace)
    _check(lib().csg_backproject(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p),
                                 _cplx(img, (p.n, M, M), "img"), int(ctf_power), float(scale),
                                 _cplx(accum, (M, M, M), "accum"), int(bool(deterministic)), wp, wn,
                                 _stream(stream)), "csg_backproject")
    return accum


def gradient(grid: Grid, optics: Optics, rot, defocus, vol, x, scale: float, lam: float, grad_out=None,
             loss_out=None, deterministic: bool = False, workspace=None, stream=None, shift=None):
    """grad = scale P^T T^* C (C T P v - x) + lam v; loss_out (device float64 [1]) = f(v)."""
    M = grid.M
    p = _poses(rot, defocus, shift)
    if grad_out is None:
        grad_out = torch.empty((M, M, M), dtype=torch.complex64, device=vol.device)
    if workspace is None:
        workspace = alloc_workspace(grid, p.n, CSG_WS_GRADIENT_DETERMINISTIC if deterministic else CSG_WS_GRADIENT,
                                    vol.device)
    g, o = grid.c(), optics.c()
    wp, wn = _ws(workspace)
    _check(lib().csg_gradient(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), _cplx(vol, (M, M, M), "vol"),
                              _cplx(x, (p.n, M, M), "x"), float(scale), float(lam),
                              _cplx(grad_out, (M, M, M), "grad_out"),
                              None if loss_out is None else _ptr(loss_out), int(bool(deterministic)), wp, wn,
                              _stream(stream)), "csg_gradient")
    return grad_out


def gradient_noalloc(grid: Grid, optics: Optics, rot, defocus, vol, x, scale: float, lam: float, grad_out,
                     loss_out=None, stream=None, shift=None):
    """csg_gradient (fast mode) with the library's static per-GPU scratch
    instead of a workspace; grad_out (and loss_out, if wanted) are passed in,
    so nothing is allocated on either side of the call."""
    M = grid.M
    p = _poses(rot, defocus, shift)
    g, o = grid.c(), optics.c()
    _check(lib().csg_gradient_noalloc(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), _cplx(vol, (M, M, M), "vol"),
                                      _cplx(x, (p.n, M, M), "x"), float(scale), float(lam),
                                      _cplx(grad_out, (M, M, M), "grad_out"),
                                      None if loss_out is None else _ptr(loss_out), _stream(stream)),
           "csg_gradient_noalloc")
    return grad_out


def hvp(grid: Grid, optics: Optics, rot, defocus, z, scale: float, lam: float, hz_out=None,
        deterministic: bool = False, workspace=None, stream=None):
    """hz = scale P^T C^2 P z + lam z."""
    M = grid.M
    p = _poses(rot, defocus)
    if hz_out is None:
        hz_out = torch.empty((M, M, M), dtype=torch.complex64, device=z.device)
    if workspace is None:
        workspace = alloc_workspace(grid, p.n, CSG_WS_GRADIENT_DETERMINISTIC if deterministic else CSG_WS_GRADIENT,
                                    z.device)
    g, o = grid.c(), optics.c()
    wp, wn = _ws(workspace)
    _check(lib().csg_hvp(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), _cplx(z, (M, M, M), "z"), float(scale),
                         float(lam), _cplx(hz_out, (M, M, M), "hz_out"), int(bool(deterministic)), wp, wn,
                         _stream(stream)), "csg_hvp")
    return hz_out


def rademacher(nvox: int, seed: int, probe: int, out=None, device=None, stream=None):
    if out is None:
        out = torch.empty(nvox, dtype=torch.float32, device=device or "cuda")
    _check(lib().csg_rademacher(int(nvox), int(seed), int(probe), _ptr(out), _stream(stream)), "csg_rademacher")
    return out


def hutchinson_diag(grid: Grid, optics: Optics, rot, defocus, n_probe: int, seed: int, scale: float, lam: float,
                    probe0: int = 0, diag_out=None, workspace=None, stream=None):
    M = grid.M
    p = _poses(rot, defocus)
    if diag_out is None:
        diag_out = torch.empty((M, M, M), dtype=torch.float32, device=rot.device)
    if workspace is None:
        workspace = alloc_workspace(grid, p.n, CSG_WS_HUTCHINSON, rot.device)
    g, o = grid.c(), optics.c()
    wp, wn = _ws(workspace)
    _check(lib().csg_hutchinson_diag(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), int(n_probe), int(seed),
                                     int(probe0), float(scale), float(lam), _ptr(diag_out), wp, wn,
                                     _stream(stream)), "csg_hutchinson_diag")
    return diag_out


def gradient_hutchinson(grid: Grid, optics: Optics, rot, defocus, vol, x, scale: float, lam: float, n_probe: int,
                        seed: int, probe0: int = 0, grad_out=None, loss_out=None, diag_out=None, workspace=None,
                        stream=None, shift=None):
    """gradient(...) and hutchinson_diag(...) of one batch in one call
    (csg_gradient_hutchinson); returns (grad_out, diag_out)."""
    M = grid.M
    p = _poses(rot, defocus, shift)
    if grad_out is None:
        grad_out = torch.empty((M, M, M), dtype=torch.complex64, device=vol.device)
    if diag_out is None:
        diag_out = torch.empty((M, M, M), dtype=torch.float32, device=vol.device)
    if diag_out.dtype != torch.float32 or diag_out.numel() != M ** 3:
        raise CsgError("diag_out must be float32 with M^3 = %d elements" % M ** 3)
    if workspace is None:
        workspace = alloc_workspace(grid, p.n, CSG_WS_GRADIENT_HUTCHINSON, vol.device)
    g, o = grid.c(), optics.c()
    wp, wn = _ws(workspace)
    _check(lib().csg_gradient_hutchinson(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p),
                                         _cplx(vol, (M, M, M), "vol"), _cplx(x, (p.n, M, M), "x"), float(scale),
                                         float(lam), _cplx(grad_out, (M, M, M), "grad_out"),
                                         None if loss_out is None else _ptr(loss_out), int(n_probe), int(seed),
                                         int(probe0), _ptr(diag_out), wp, wn, _stream(stream)),
           "csg_gradient_hutchinson")
    return grad_out, diag_out


def exact_diag(grid: Grid, optics: Optics, rot, defocus, scale: float, lam: float, diag_out=None, workspace=None,
               stream=None):
    M = grid.M
    p = _poses(rot, defocus)
    if diag_out is None:
        diag_out = torch.empty((M, M, M), dtype=torch.float32, device=rot.device)
    if workspace is None:
        workspace = alloc_workspace(grid, p.n, CSG_WS_BACKPROJECT, rot.device)
    g, o = grid.c(), optics.c()
    wp, wn = _ws(workspace)
    _check(lib().csg_exact_diag(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), float(scale), float(lam),
                                _ptr(diag_out), wp, wn, _stream(stream)), "csg_exact_diag")
    return diag_out


def features(grid: Grid, optics: Optics, rot, defocus, ctf2=None, cover=None, stream=None):
    M = grid.M
    p = _poses(rot, defocus)
    if ctf2 is None:
        ctf2 = torch.zeros((M, M, M), dtype=torch.float32, device=rot.device)
    if cover is None:
        cover = torch.zeros((M, M, M), dtype=torch.float32, device=rot.device)
    g, o = grid.c(), optics.c()
    _check(lib().csg_features(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), _ptr(ctf2), _ptr(cover),
                              _stream(stream)), "csg_features")
    return ctf2, cover


def threshold_alpha(grid: Grid, optics: Optics, rot, defocus, lam: float, alpha_out=None, stream=None):
    """alpha of eq. (thresh value) over all images given; device float64 [1]."""
    p = _poses(rot, defocus)
    if alpha_out is None:
        alpha_out = torch.empty(1, dtype=torch.float64, device=defocus.device)
    g, o = grid.c(), optics.c()
    _check(lib().csg_threshold_alpha(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), float(lam), _ptr(alpha_out),
                                     _stream(stream)), "csg_threshold_alpha")
    return alpha_out


def feature_sums(grid: Grid, optics: Optics, rot, defocus, accum=None, workspace=None, stream=None):
    """accum.real += sum C^2 w, accum.imag += sum w (complex64 [M,M,M])."""
    M = grid.M
    p = _poses(rot, defocus)
    if accum is None:
        accum = torch.zeros((M, M, M), dtype=torch.complex64, device=rot.device)
    if workspace is None:
        workspace = alloc_workspace(grid, p.n, CSG_WS_BACKPROJECT, rot.device)
    g, o = grid.c(), optics.c()
    wp, wn = _ws(workspace)
    _check(lib().csg_feature_sums(ctypes.byref(g), ctypes.byref(o), ctypes.byref(p), _cplx(accum, (M, M, M), "accum"),
                                  wp, wn, _stream(stream)), "csg_feature_sums")
    return accum


def precond_sgd_step(v, g, D, D_avg, zHz, k: int, beta: float, alpha: float, eta: float, v_out=None,
                     Dhat_out=None, stats_out=None, stream=None):
    """One step of Algorithm 1 (see include/cryosgd.h); returns (v_out, stats_out[2])."""
    nvox = v.numel()
    if v_out is None:
        v_out = torch.empty_like(v)
    if stats_out is None:
        stats_out = torch.empty(2, dtype=torch.float64, device=v.device)
    _check(lib().csg_precond_sgd_step(int(nvox), _ptr(v), _ptr(g), _ptr(D), _ptr(D_avg), _ptr(zHz), int(k),
                                      float(beta), float(alpha), float(eta), _ptr(v_out), _ptr(Dhat_out),
                                      _ptr(stats_out), _stream(stream)), "csg_precond_sgd_step")
    return v_out, stats_out


def diag_update(D, D_avg, zHz, k: int, beta: float, alpha: float = 0.0, Dhat_out=None, stream=None):
    """The diagonal estimate's update alone (csg_precond_sgd_step with no
    step): D_avg = (k-1)/k D_avg + zHz/k, D = beta D + (1-beta) D_avg, and
    D_hat = max(|D|, alpha) into Dhat_out if given."""
    _check(lib().csg_precond_sgd_step(int(D.numel()), None, None, _ptr(D), _ptr(D_avg), _ptr(zHz), int(k),
                                      float(beta), float(alpha), 0.0, None, _ptr(Dhat_out), None, _stream(stream)),
           "csg_precond_sgd_step")
    return D


# ---------------------------------------------------------------------------
# Learned preconditioner network
# ---------------------------------------------------------------------------
def mlp_param_count() -> int:
    return int(lib().csg_mlp_param_count())


def _f32(t, name, numel=None):
    if t.dtype != torch.float32:
        raise CsgError("%s must be float32" % name)
    if numel is not None and t.numel() != numel:
        raise CsgError("%s must have %d elements" % (name, numel))
    return _ptr(t)


def mlp_forward(params, X, y=None, stream=None):
    """y = mlp(X) for X float32 [n, 3]."""
    n = X.shape[0]
    if y is None:
        y = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(lib().csg_mlp_forward(_f32(params, "params", mlp_param_count()), _f32(X, "X", 3 * n), int(n),
                                 _f32(y, "y", n), _stream(stream)), "csg_mlp_forward")
    return y


def mlp_grad_workspace(n: int, device=None) -> torch.Tensor | None:
    nb = int(lib().csg_mlp_grad_workspace_bytes(int(n)))
    return None if nb == 0 else torch.empty(nb, dtype=torch.uint8, device=device or "cuda")


def mlp_grad(params, X, T, grad=None, loss=None, workspace=None, stream=None):
    """Gradient (and value) of the mean squared error of mlp(X) against T
    (bitwise reproducible: fixed-order sums)."""
    n = X.shape[0]
    if grad is None:
        grad = torch.empty(mlp_param_count(), dtype=torch.float32, device=X.device)
    if loss is None:
        loss = torch.empty(1, dtype=torch.float64, device=X.device)
    if workspace is None:
        workspace = mlp_grad_workspace(n, X.device)
    wp, wn = _ws(workspace)
    _check(lib().csg_mlp_grad(_f32(params, "params", mlp_param_count()), _f32(X, "X", 3 * n), _f32(T, "T", n),
                              int(n), _f32(grad, "grad", mlp_param_count()), _ptr(loss), wp, wn, _stream(stream)),
           "csg_mlp_grad")
    return grad, loss


def mlp_adam(params, m, v, grad, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
             eps: float = 1e-8, stream=None):
    _check(lib().csg_mlp_adam(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step), float(lr), float(beta1),
                              float(beta2), float(eps), _stream(stream)), "csg_mlp_adam")


def learned_diag(grid: Grid, n_images: int, lam: float, params, ctf2, cover, out=None, stream=None):
    M = grid.M
    if out is None:
        out = torch.empty((M, M, M), dtype=torch.float32, device=params.device)
    g = grid.c()
    _check(lib().csg_learned_diag(ctypes.byref(g), int(n_images), float(lam), _ptr(params), _ptr(ctf2),
                                  _ptr(cover), _ptr(out), _stream(stream)), "csg_learned_diag")
    return out


def shell_sums(grid: Grid, u, v, out=None, stream=None):
    """Per-shell (Re sum u conj v, sum |u|^2, sum |v|^2), each [M/2], as a
    device float64 tensor [3, M/2]."""
    M = grid.M
    g = grid.c()
    pu = _cplx(u, (M, M, M), "u")
    pv = _cplx(v, (M, M, M), "v")
    if out is None:
        out = torch.empty((3, M // 2), dtype=torch.float64, device=u.device)
    _check(lib().csg_shell_sums(ctypes.byref(g), pu, pv, _ptr(out), _stream(stream)), "csg_shell_sums")
    return out


def fsc(grid: Grid, u, v):
    """Fourier shell correlation per shell s = 0 .. M/2 - 1 (eq. (fsc)); shells
    where either volume vanishes give 0."""
    s = shell_sums(grid, u, v)
    den = torch.sqrt(s[1] * s[2])
    return torch.where(den > 0, s[0] / torch.where(den > 0, den, torch.ones_like(den)), torch.zeros_like(den))


KERNELS = {"project": 0, "backproject": 1, "gradient": 2, "hvp": 3, "features": 4, "sq_diag": 5,
           "gradient_probe": 6}


def timing_enable(on: bool = True):
    """Bracket every brick-kernel launch with HIP events on its stream."""
    _check(lib().csg_timing_enable(1 if on else 0), "csg_timing_enable")


def timing_read(kernel: str):
    """(summed milliseconds, launches) of one kernel since its last read."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().csg_timing_read(KERNELS[kernel], ctypes.byref(ms), ctypes.byref(n)), "csg_timing_read")
    return ms.value, n.value

