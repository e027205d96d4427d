"""Algorithm 1 of the paper (Sec. 3.4): SGD preconditioned by the estimated,
thresholded Hessian diagonal, with the stochastic Armijo line search of
eq. (stochastic armijo).

This module is a host-side loop over the C-ABI calls of libcryosgd; every
arithmetic step (gradient, Hessian-vector probes, the running mean and
exponential average of the diagonal, thresholding, the step, the line-search
losses) runs in the library's kernels.  The only host work is the line
search's decision, which needs one read-back of four device scalars per trial.
The device keeps working while the host decides, on the next batch's work
queued behind that read-back when the caller names that batch:
  - the Hutchinson probe product does not depend on v (the Hessian of the
    least-squares loss is constant), so it needs only the next poses (the
    one-call form forms it with the gradient and needs the images too);
  - the gradient and loss, given the next images, are formed at the first
    trial point v'.  The first trial is usually accepted, and then v' is the
    next iterate and the queued gradient is the next iteration's; after a
    rejected first trial it is discarded and the next iteration forms its
    own.

Arms (same loop, same step-size rule):
  "hutchinson"  D estimated on the fly from Rademacher probes (Algorithm 1)
  "fixed"       a given diagonal D held fixed (precomputed / learned / exact)
  "plain"       D_hat = 1 (no preconditioner)

Line search bounds (the same rule as the oracle's iteration): after
max_halvings failed halvings the last trial step is kept and the iteration
is counted in `capped`; a loss or gradient norm that is not finite raises
CsgError before any step is taken.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from . import binding as B


@dataclass
class Alg1Config:
    beta: float = 0.9        # exponential-average weight of eq. (exp avg update)
    c: float = 0.1           # sufficient-decrease constant of eq. (stochastic armijo)
    eta0: float = 1.0        # initial step size
    n_probe: int = 2         # Rademacher probes per iteration (one complex product)
    max_halvings: int = 30
    probe_seed: int = 4
    deterministic: bool = False
    # Hutchinson arm, fast gradient: the gradient and the iteration's probe
    # product in one call (csg_gradient_hutchinson); otherwise two calls, the
    # probe product of the next batch queued behind the line search
    fused: bool = True


@dataclass
class Alg1State:
    v: torch.Tensor                 # complex64 [M,M,M]
    D: torch.Tensor | None          # float32 [M,M,M] (None: plain SGD)
    D_avg: torch.Tensor | None
    eta: float
    k: int = 0
    halvings: list = field(default_factory=list)
    capped: int = 0  # iterations whose line search hit max_halvings


class Alg1Runner:
    """Owns the device buffers of one run; `iteration` performs one k."""

    def __init__(self, grid: B.Grid, optics: B.Optics, arm: str, scale: float, lam: float, alpha: float,
                 cfg: Alg1Config, v0: torch.Tensor, D_fixed: torch.Tensor | None = None, batch: int = 0):
        assert arm in ("hutchinson", "fixed", "plain")
        self.grid, self.optics, self.arm = grid, optics, arm
        self.scale, self.lam, self.alpha, self.cfg = float(scale), float(lam), float(alpha), cfg
        M = grid.M
        dev = v0.device
        if arm == "hutchinson":
            D = torch.ones((M, M, M), dtype=torch.float32, device=dev)
            Da = torch.zeros((M, M, M), dtype=torch.float32, device=dev)
        elif arm == "fixed":
            D, Da = D_fixed.contiguous(), None
        else:
            D, Da = None, None
        self.state = Alg1State(v=v0.clone(), D=D, D_avg=Da, eta=cfg.eta0)
        self.fused = arm == "hutchinson" and cfg.fused and not cfg.deterministic
        self.g = torch.empty_like(v0)
        self.v_new = torch.empty_like(v0)
        self.zHz = torch.empty((M, M, M), dtype=torch.float32, device=dev) if arm == "hutchinson" else None
        self.zHz_next = torch.empty_like(self.zHz) if arm == "hutchinson" else None
        # the next batch's gradient, formed at the first trial point
        self.g_next = torch.empty_like(v0)
        # (rot, defocus, images or None, k, probe) of the next batch's queued
        # results: the gradient and f(v) in g_next and sc[4 - f_at] when images
        # are named, the probe product in zHz_next when probe is true
        self._queued = None
        # scalars: [f_at] f(v), [1] sum |g|^2 / D_hat, [2] ||v'||^2, [3] data
        # term of f(v'), [4 - f_at] f of the queued next batch (f_at is 0 or 4)
        self.f_at = 0
        self.sc = torch.zeros(5, dtype=torch.float64, device=dev)
        self.sc_host = torch.zeros(5, dtype=torch.float64, pin_memory=v0.is_cuda)
        self.sc_ready = torch.cuda.Event()
        self.ws_grad = B.alloc_workspace(grid, batch, B.CSG_WS_GRADIENT_DETERMINISTIC if cfg.deterministic
                                         else B.CSG_WS_GRADIENT_HUTCHINSON if self.fused else B.CSG_WS_GRADIENT, dev)
        self.ws_hutch = (B.alloc_workspace(grid, batch, B.CSG_WS_HUTCHINSON, dev)
                         if arm == "hutchinson" and not self.fused else None)
        self.ws_proj = B.alloc_workspace(grid, batch, B.CSG_WS_PROJECT, dev)

    def state_dict(self) -> dict:
        """The iteration state (v, D, D_avg, eta, k and the line-search
        counters) as host arrays and numbers, for a checkpoint."""
        st = self.state
        arrays = {"v": st.v.cpu().numpy()}
        if st.D is not None:
            arrays["D"] = st.D.cpu().numpy()
        if st.D_avg is not None:
            arrays["D_avg"] = st.D_avg.cpu().numpy()
        return {"arrays": arrays, "eta": st.eta, "k": st.k, "capped": st.capped, "halvings": list(st.halvings)}

    def load_state_dict(self, sd: dict):
        """Restore what state_dict returned (same arm and grid); a probe
        product queued for the next batch is dropped and recomputed."""
        st = self.state
        st.v.copy_(torch.from_numpy(sd["arrays"]["v"]))
        if st.D is not None and "D" in sd["arrays"]:
            st.D.copy_(torch.from_numpy(sd["arrays"]["D"]))
        if st.D_avg is not None and "D_avg" in sd["arrays"]:
            st.D_avg.copy_(torch.from_numpy(sd["arrays"]["D_avg"]))
        st.eta, st.k, st.capped = float(sd["eta"]), int(sd["k"]), int(sd["capped"])
        st.halvings = list(sd["halvings"])
        self._queued = None

    def iteration(self, rot_I, df_I, x_I, next_poses=None, next_images=None) -> int:
        """One iteration on the batch (rot_I, df_I, x_I).  `next_poses` =
        (rot, defocus) of the next call's batch and `next_images` its images,
        if known: during this line search the Hutchinson arm computes that
        batch's probe product (needs the poses; in the one-call form also the
        images), and every arm given the images computes that batch's
        gradient and loss at the first trial point.  The next call uses them
        when it is given the same tensors (and, for the gradient, when the
        first trial was accepted)."""
        st, cfg, g, o = self.state, self.cfg, self.grid, self.optics
        st.k += 1
        q, self._queued = self._queued, None
        match = q is not None and q[0] is rot_I and q[1] is df_I and q[3] == st.k
        have_probe = match and q[4]
        have_grad = match and q[2] is x_I
        if have_probe:
            self.zHz, self.zHz_next = self.zHz_next, self.zHz
        if have_grad:
            # gradient and f(v) of this batch at v, queued by the previous
            # call at its accepted first trial point
            self.g, self.g_next = self.g_next, self.g
            self.f_at = 4 - self.f_at
        if self.arm == "hutchinson" and not have_probe:
            if self.fused:
                # a queued gradient of the one-call form comes with its probe product
                assert not have_grad
                # the gradient and z (.) H_I z for this iteration's probes
                # (Algorithm 1: gradient and running-mean line) in one pass
                B.gradient_hutchinson(g, o, rot_I, df_I, st.v, x_I, self.scale, self.lam, cfg.n_probe,
                                      cfg.probe_seed, probe0=(st.k - 1) * cfg.n_probe, grad_out=self.g,
                                      loss_out=self.sc[self.f_at:self.f_at + 1], diag_out=self.zHz,
                                      workspace=self.ws_grad)
                have_grad = True
            else:
                # z (.) H_I z for this iteration's probes (Algorithm 1, running-mean line)
                B.hutchinson_diag(g, o, rot_I, df_I, cfg.n_probe, cfg.probe_seed, self.scale, self.lam,
                                  probe0=(st.k - 1) * cfg.n_probe, diag_out=self.zHz, workspace=self.ws_hutch)
        if not have_grad:
            B.gradient(g, o, rot_I, df_I, st.v, x_I, self.scale, self.lam, grad_out=self.g,
                       loss_out=self.sc[self.f_at:self.f_at + 1], deterministic=cfg.deterministic,
                       workspace=self.ws_grad)
        eta = st.eta
        halvings = 0
        first = True
        while True:
            B.precond_sgd_step(st.v, self.g, st.D, st.D_avg, self.zHz if first else None, st.k, cfg.beta,
                               self.alpha if st.D is not None else 0.0, eta, v_out=self.v_new,
                               stats_out=self.sc[1:3])
            self.sc[3:4].zero_()
            B.project(g, o, rot_I, df_I, self.v_new, subtract=x_I, out=None, loss=self.sc[3:4], want_out=False,
                      workspace=self.ws_proj)
            self.sc_host.copy_(self.sc, non_blocking=True)
            self.sc_ready.record()
            if first and next_poses is not None:
                self._queue_next(next_poses, next_images)
            elif not first and self._queued is not None and self._queued[2] is not None:
                # the first trial was rejected: the queued gradient is not at
                # the next iterate; a queued probe product does not depend on
                # v and is kept
                qn = self._queued
                self._queued = (qn[0], qn[1], None, qn[3], True) if qn[4] else None
            first = False
            self.sc_ready.synchronize()
            sc = self.sc_host.tolist()
            f0, gn, vn2, l1 = sc[self.f_at], sc[1], sc[2], sc[3]
            f1 = self.scale * l1 + 0.5 * self.lam * vn2
            if not (math.isfinite(f0) and math.isfinite(f1) and math.isfinite(gn)):
                # v is left as it was (the trial went to v_new)
                self._queued = None
                raise B.CsgError("Armijo line search at iteration %d: f(v) = %r, f(v') = %r, |g|^2_D^-1 = %r "
                                 "(non-finite input or preconditioner)" % (st.k, f0, f1, gn))
            if f1 <= f0 - cfg.c * eta * gn:
                break
            if halvings >= cfg.max_halvings:
                # the decrease is below the resolution of the minibatch loss:
                # keep the (tiny) step rather than loop on rounding noise
                st.capped += 1
                break
            eta *= 0.5
            halvings += 1
        st.v, self.v_new = self.v_new, st.v
        st.eta = eta
        st.halvings.append(halvings)
        return halvings

    def _queue_next(self, next_poses, next_images):
        """Enqueue the next batch's work behind the first trial's read-back:
        the probe product (Hutchinson arm) and, given the images, the
        gradient and loss at the trial point v_new.  Stream order: the
        read-back is taken before this writes sc[4 - f_at], and a later
        trial's step writes v_new only after this has read it."""
        st, cfg, g, o = self.state, self.cfg, self.grid, self.optics
        rn, dn = next_poses
        probe = self.arm == "hutchinson"
        if self.fused:
            if next_images is None:
                return
            B.gradient_hutchinson(g, o, rn, dn, self.v_new, next_images, self.scale, self.lam, cfg.n_probe,
                                  cfg.probe_seed, probe0=st.k * cfg.n_probe, grad_out=self.g_next,
                                  loss_out=self.sc[4 - self.f_at:5 - self.f_at], diag_out=self.zHz_next,
                                  workspace=self.ws_grad)
        else:
            if probe:
                B.hutchinson_diag(g, o, rn, dn, cfg.n_probe, cfg.probe_seed, self.scale, self.lam,
                                  probe0=st.k * cfg.n_probe, diag_out=self.zHz_next, workspace=self.ws_hutch)
            if next_images is not None:
                B.gradient(g, o, rn, dn, self.v_new, next_images, self.scale, self.lam, grad_out=self.g_next,
                           loss_out=self.sc[4 - self.f_at:5 - self.f_at], deterministic=cfg.deterministic,
                           workspace=self.ws_grad)
            elif not probe:
                return
        self._queued = (rn, dn, next_images, st.k + 1, probe)
