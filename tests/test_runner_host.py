"""CPU checks of the Algorithm 1 runner's host logic (`sgd.Alg1Runner`) with
a stand-in for the library: every library call the runner makes is replaced
by a few lines of torch on the CPU for an element-wise quadratic loss, so the
line search, the probe-product queue and the next batch's queued gradient
run without a GPU.  What is checked is the runner's bookkeeping, not the
library's arithmetic (that is the GPU tests' part):
  - the next batch's work is enqueued after the first trial's read-back and
    before the host waits for it;
  - a queued gradient is used exactly when the first trial was accepted, a
    queued probe product also after a rejected first trial;
  - queueing does not change the trajectory (bit for bit here);
  - results queued for other tensors are not used.

Stand-in loss of batch I: f_I(v) = s/2 sum |c_I v - x_I|^2 + lam/2 |v|^2 with
c_I = 1 + rot_I[0], so H = s c_I^2 + lam on every voxel (the probe product is
that value, as one probe gives exactly for a diagonal H)."""
import types

import pytest
import torch

from paper_2311_16100_amd import binding, sgd

M, SCALE, LAM, ALPHA = 4, 12.0, 0.05, 0.5


class FakeLib:
    def __init__(self):
        self.log = []

    @staticmethod
    def _c(rot):
        return 1.0 + float(rot[0])

    def _grad(self, rot, v, x, scale, lam, grad_out, loss_out):
        c = self._c(rot)
        r = c * v - x
        grad_out.copy_(scale * c * r + lam * v)
        loss_out[0] = 0.5 * scale * float((r.abs() ** 2).sum()) + 0.5 * lam * float((v.abs() ** 2).sum())

    def gradient(self, g, o, rot, df, v, x, scale, lam, grad_out=None, loss_out=None, deterministic=False,
                 workspace=None):
        self.log.append(("gradient", rot, v.clone()))
        self._grad(rot, v, x, scale, lam, grad_out, loss_out)

    def gradient_hutchinson(self, g, o, rot, df, v, x, scale, lam, n_probe, seed, probe0=0, grad_out=None,
                            loss_out=None, diag_out=None, workspace=None):
        self.log.append(("gradient_hutchinson", rot, v.clone()))
        self._grad(rot, v, x, scale, lam, grad_out, loss_out)
        diag_out.fill_(scale * self._c(rot) ** 2 + lam)

    def hutchinson_diag(self, g, o, rot, df, n_probe, seed, scale, lam, probe0=0, diag_out=None, workspace=None):
        self.log.append(("hutchinson_diag", rot, None))
        diag_out.fill_(scale * self._c(rot) ** 2 + lam)

    def precond_sgd_step(self, v, g, D, D_avg, zHz, k, beta, alpha, eta, v_out=None, stats_out=None):
        dh = torch.ones(v.shape)
        if D is not None:
            if zHz is not None:
                D_avg.mul_((k - 1) / k).add_(zHz / k)
                D.mul_(beta).add_((1 - beta) * D_avg)
            dh = torch.clamp(D.abs(), min=alpha)
        v_out.copy_(v - eta * g / dh)
        stats_out[0] = float(((g.abs() ** 2) / dh).sum())
        stats_out[1] = float((v_out.abs() ** 2).sum())
        self.log.append(("step", None, v_out.clone()))

    def project(self, g, o, rot, df, v, subtract=None, out=None, loss=None, want_out=False, workspace=None):
        self.log.append(("project", rot, None))
        loss[0] += 0.5 * float(((self._c(rot) * v - subtract).abs() ** 2).sum())


class FakeEvent:
    def __init__(self, lib):
        self.lib = lib

    def record(self):
        self.lib.log.append(("record", None, None))

    def synchronize(self):
        self.lib.log.append(("sync", None, None))


@pytest.fixture
def fake(monkeypatch):
    lib = FakeLib()
    for name in ("gradient", "gradient_hutchinson", "hutchinson_diag", "precond_sgd_step", "project"):
        monkeypatch.setattr(binding, name, getattr(lib, name))
    monkeypatch.setattr(binding, "alloc_workspace", lambda *a, **k: None)
    monkeypatch.setattr(sgd.torch.cuda, "Event", lambda *a, **k: FakeEvent(lib))
    return lib


def batches(n=6, seed=3):
    gen = torch.Generator().manual_seed(seed)
    out = []
    for _ in range(n):
        rot = 0.3 * torch.rand(9, generator=gen, dtype=torch.float32)
        df = torch.rand(1, generator=gen, dtype=torch.float32)
        x = torch.complex(torch.randn(M, M, M, generator=gen), torch.randn(M, M, M, generator=gen))
        out.append((rot, df, x))
    return out


def run(fake, arm, fused, queue_probe, queue_grad, copies=False):
    cfg = sgd.Alg1Config(eta0=1.0, n_probe=2, fused=fused)
    D_fixed = torch.full((M, M, M), 3.0) if arm == "fixed" else None
    runner = sgd.Alg1Runner(types.SimpleNamespace(M=M), None, arm, SCALE, LAM, ALPHA, cfg,
                            torch.zeros((M, M, M), dtype=torch.complex64), D_fixed=D_fixed, batch=1)
    bs = batches()
    traj = []
    for k, (rot, df, x) in enumerate(bs):
        nxt, nxt_x = None, None
        if k + 1 < len(bs):
            rn, dn, xn = bs[k + 1]
            if copies:
                rn, dn, xn = rn.clone(), dn.clone(), xn.clone()
            nxt = (rn, dn) if (queue_probe or queue_grad) else None
            nxt_x = xn if queue_grad else None
        h = runner.iteration(rot, df, x, next_poses=nxt, next_images=nxt_x)
        traj.append((h, runner.state.eta, runner.state.v.clone()))
    return traj, bs


FORMS = [("hutchinson", True), ("hutchinson", False), ("plain", False), ("fixed", False)]


@pytest.mark.parametrize("arm,fused", FORMS, ids=["one-call", "two-call", "plain", "fixed"])
def test_queued_gradient_leaves_the_trajectory_unchanged(fake, arm, fused):
    base, _ = run(fake, arm, fused, False, False)
    hs = [h for h, _, _ in base]
    # the stand-in problem has both kinds of line search: a rejected first
    # trial at the start and accepted first trials later
    assert hs[0] > 0 and 0 in hs[:-1]
    fake.log.clear()
    got, bs = run(fake, arm, fused, True, True)
    for (h0, e0, v0), (h1, e1, v1) in zip(base, got):
        assert h0 == h1 and e0 == e1
        assert torch.equal(v0, v1)
    # gradient launches: one queued per iteration but the last, plus an own
    # one for the first iteration and after every rejected first trial
    grads = [e for e in fake.log if e[0] in ("gradient", "gradient_hutchinson")]
    assert len(grads) == (len(bs) - 1) + 1 + sum(1 for h in hs[:-1] if h > 0)


@pytest.mark.parametrize("arm,fused", FORMS, ids=["one-call", "two-call", "plain", "fixed"])
def test_next_batch_work_follows_the_read_back(fake, arm, fused):
    """The next batch's launches sit between the first trial's read-back
    event and the host's wait on it, once per iteration but the last, and a
    queued gradient takes the trial point as v."""
    _, bs = run(fake, arm, fused, True, True)
    log = fake.log
    launches = ("gradient", "gradient_hutchinson", "hutchinson_diag")
    queued = 0
    for i, e in enumerate(log):
        if e[0] not in launches:
            continue
        prev = next((x for x in reversed(log[:i]) if x[0] not in launches), ("start",))
        if prev[0] != "record":
            # an own launch: at the start or after the previous iteration's wait
            assert prev[0] in ("start", "sync")
            continue
        queued += 1
        # before the wait on that read-back and before any further step
        nxt = next(x for x in log[i + 1:] if x[0] not in launches)
        assert nxt[0] == "sync"
        if e[2] is not None:
            trial = next(x for x in reversed(log[:i]) if x[0] == "step")[2]
            assert torch.equal(e[2], trial)
    expect = len(bs) - 1
    if arm == "hutchinson" and not fused:
        expect *= 2  # the probe product and the gradient
    assert queued == expect


def test_rejected_first_trial_keeps_only_the_probe_product(fake):
    """After the first iteration's rejected first trial the next iteration
    uses the queued probe product and launches only csg_gradient (two-call
    and one-call forms)."""
    for fused in (False, True):
        fake.log.clear()
        traj, bs = run(fake, "hutchinson", fused, True, True)
        assert traj[0][0] > 0
        steps = [i for i, e in enumerate(fake.log) if e[0] == "step"]
        last_of_first = steps[traj[0][0]]  # the first iteration's last trial
        first_of_second = steps[traj[0][0] + 1]
        own = [e[0] for e in fake.log[last_of_first + 1:first_of_second]
               if e[0] not in ("project", "record", "sync")]
        assert own == ["gradient"], own


def test_results_queued_for_other_tensors_are_not_used(fake):
    for arm, fused in FORMS:
        base, _ = run(fake, arm, fused, False, False)
        fake.log.clear()
        got, bs = run(fake, arm, fused, True, True, copies=True)
        for (h0, e0, v0), (h1, e1, v1) in zip(base, got):
            assert h0 == h1 and e0 == e1 and torch.equal(v0, v1)
        # every iteration launches its own gradient
        own = [e for e in fake.log if e[0] in ("gradient", "gradient_hutchinson") and any(e[1] is b[0] for b in bs)]
        assert len(own) == len(bs)
