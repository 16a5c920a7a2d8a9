"""Learned closure for under-resolved k = 1 runs: data, training, evaluation.

Not part of the paper's method: a k = 1 solution on a coarse mesh is corrected
toward high-resolution DG (k = 2 on twice the cells per axis) restricted to the
coarse mesh.  With P the exact L2 restriction (linear), the coarse state
y_c = P y_f evolves exactly as dy_c/dt = -P R_f(y_f); the coarse operator gives
-R_c(P y_f).  The network learns the difference c = R_c(P y_f) - P R_f(y_f)
from the coarse state's neighbourhood, and the corrected scheme is
dy/dt = -R_c(y) + c (dg_set_closure).

Every arithmetic step runs in libdgmi.so's kernels (restriction, features,
targets, statistics, standardisation, forward/backward products, Adam, the DG
solvers); this module only orders the calls, draws the seeded batch indices and
keeps the device buffers.
"""
import math
import time

import numpy as np

from . import dg, synth

SHAPE = (140, 128, 128, 20)


class Config:
    """Workload of the closure experiment (defaults: k=2 128^3 -> k=1 64^3)."""

    def __init__(self, nc=64, mach=0.3, ic_seed=9079, forcing=True, precision="fp32", t_spin=0.05, dt_snap=0.02,
                 nsnap=16, t_gap=0.1, horizon=0.2, batch=4096, iters=3000, lr=1e-3, init_seed=4, batch_seed=17):
        self.nc = nc
        self.nf = 2 * nc
        self.mach = mach
        self.ic_seed = ic_seed
        self.forcing = forcing
        self.precision = precision
        self.t_spin = t_spin       # time run before the first training snapshot
        self.dt_snap = dt_snap     # time between snapshots
        self.nsnap = nsnap         # training snapshots
        self.t_gap = t_gap         # time between the last training snapshot and the held-out start
        self.horizon = horizon     # length of the held-out comparison runs
        self.batch = batch
        self.iters = iters
        self.lr = lr
        self.init_seed = init_seed
        self.batch_seed = batch_seed


def driving(a0=0.03, seed=1602):
    """The benchmark's driving table: one OU update of the 1 <= |n| <= 3 modes."""
    nvec = synth.forcing_modes(1.0, 3.0)
    th = synth.ou_stationary_start(seed, len(nvec))
    z = synth.ou_normals(seed, len(nvec), 1)[0]
    _, ahat = dg.ou_update(nvec, th, z, math.exp(-0.1), 1.0, a0, 1.0, 3.0)
    return nvec, ahat


def _advance(s, y, T, t_now):
    """Advance solver s by exactly T with CFL-limited equal steps; returns the new time."""
    if T <= 0:
        return t_now
    h = s.dt(y)
    n = max(1, int(math.ceil(T / h)))
    s.step(y, n, T / n)
    return t_now + T


class Experiment:
    def __init__(self, cfg, log=print):
        import torch
        self.cfg = cfg
        self.log = log
        self.torch = torch
        fl = dict(forcing=cfg.forcing, precision=cfg.precision)
        self.fine = dg.Solver(2, cfg.nf, **fl)
        self.coarse = dg.Solver(1, cfg.nc, **fl)
        self.coarse_cl = dg.Solver(1, cfg.nc, closure=True, **fl)
        if cfg.forcing:
            nvec, ahat = driving()
            for s in (self.fine, self.coarse, self.coarse_cl):
                s.set_forcing(nvec, ahat)
        x = dg.gauss_nodes(3)
        qp = synth.turbulence(cfg.nf, x, seed=cfg.ic_seed, mach=cfg.mach, device="cuda", dtype=self.fine.dtype)
        self.yf = self.fine.project(qp)
        del qp
        self.t = 0.0

    # ------------------------------------------------------------ data
    def sample(self):
        """(features, targets) of the current fine state: raw, [cells][140], [cells][20]."""
        c, f = self.coarse, self.fine
        yc = c.restrict(2, self.yf)
        rf = f.rhs(self.yf)
        prf = c.restrict(2, rf)
        rc = c.rhs(yc)
        return c.closure_features(yc), c.closure_targets(rc, prf)

    def generate(self):
        cfg = self.cfg
        t0 = time.perf_counter()
        self.t = _advance(self.fine, self.yf, cfg.t_spin, self.t)
        feats, targs = [], []
        for j in range(cfg.nsnap):
            if j:
                self.t = _advance(self.fine, self.yf, cfg.dt_snap, self.t)
            fx, tx = self.sample()
            feats.append(fx)
            targs.append(tx)
        self.X = self.torch.cat(feats)
        self.T = self.torch.cat(targs)
        del feats, targs
        self.torch.cuda.synchronize()
        self.log(f"[closure] {cfg.nsnap} snapshots to t={self.t:.3f}, {self.X.shape[0]} samples "
                 f"({time.perf_counter() - t0:.1f} s)")

    # ------------------------------------------------------------ training
    def train(self):
        torch = self.torch
        cfg = self.cfg
        fmean, fstd, _, _ = dg.column_stats(self.X)
        _, _, trms, _ = dg.column_stats(self.T)
        fstd = torch.where(fstd > 0, fstd, torch.ones_like(fstd))
        trms = torch.where(trms > 0, trms, torch.ones_like(trms))
        zero = torch.zeros_like(trms)
        dg.standardize(self.X, fmean, fstd)
        dg.standardize(self.T, zero, trms)
        _, _, _, tmax = dg.column_stats(self.T)
        self.norm = dict(feat_mean=fmean.cpu().numpy(), feat_std=fstd.cpu().numpy(), out_scale=trms.cpu().numpy(),
                         out_bound=tmax.cpu().numpy())
        params = torch.tensor(synth.xavier_params(SHAPE, seed=cfg.init_seed), dtype=torch.float32, device="cuda")
        m = torch.zeros_like(params)
        v = torch.zeros_like(params)
        net = dg.MLP(SHAPE, cfg.batch)
        rng = np.random.default_rng(cfg.batch_seed)
        ns = self.X.shape[0]
        grad = torch.empty_like(params)
        loss = torch.empty((), dtype=torch.float64, device="cuda")
        hist = []
        t0 = time.perf_counter()
        perm = rng.permutation(ns)
        pos = 0
        for it in range(1, cfg.iters + 1):
            if pos + cfg.batch > ns:
                perm = rng.permutation(ns)
                pos = 0
            rows = torch.from_numpy(perm[pos:pos + cfg.batch].astype(np.int32)).to("cuda", non_blocking=True)
            pos += cfg.batch
            net.loss_grad(params, self.X, self.T, rows=rows, grad=grad, loss=loss)
            net.adam(params, grad, m, v, it, lr=cfg.lr)
            if it == 1 or it % 250 == 0 or it == cfg.iters:
                hist.append((it, float(loss.item())))
        torch.cuda.synchronize()
        self.params = params
        self.net = net
        self.loss_history = hist
        self.log(f"[closure] trained {cfg.iters} Adam steps in {time.perf_counter() - t0:.1f} s, "
                 f"loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}")
        self.coarse_cl.set_closure(params.cpu().numpy(), **self.norm)
        return hist

    # ------------------------------------------------------------ evaluation
    def evaluate(self):
        """Held-out comparison: start both coarse runs from P y_f(t0) at a later
        time, run for the horizon, compare with P y_f(t0 + horizon)."""
        torch = self.torch
        cfg = self.cfg
        self.t = _advance(self.fine, self.yf, cfg.t_gap, self.t)
        c = self.coarse
        # instantaneous: how much of the coarse operator's error the closure removes
        fx, tx = self.sample()
        yc0 = c.restrict(2, self.yf)
        rf = self.fine.rhs(self.yf)
        prf = c.restrict(2, rf)
        r_plain = c.rhs(yc0)
        r_clos = self.coarse_cl.rhs(yc0)
        self.coarse_cl.closure_fallbacks()
        e_rhs_plain = _rel_l2(r_plain, prf)
        e_rhs_clos = _rel_l2(r_clos, prf)
        # integrated over the horizon
        y_plain = yc0.clone()
        y_clos = yc0.clone()
        t0 = self.t
        h = min(c.dt(y_plain), self.coarse_cl.dt(y_clos))
        n = max(1, int(math.ceil(cfg.horizon / h)))
        c.step(y_plain, n, cfg.horizon / n)
        self.coarse_cl.closure_fallbacks()
        self.coarse_cl.step(y_clos, n, cfg.horizon / n)
        fb = self.coarse_cl.closure_fallbacks()
        self.t = _advance(self.fine, self.yf, cfg.horizon, self.t)
        ref = c.restrict(2, self.yf)
        e_plain = _rel_l2(y_plain, ref)
        e_clos = _rel_l2(y_clos, ref)
        # the deviation from the start isolates the evolution the schemes must capture
        d_ref = ref - yc0
        e_plain_dev = _rel_l2(y_plain - yc0, d_ref)
        e_clos_dev = _rel_l2(y_clos - yc0, d_ref)
        ncells = cfg.nc ** 3
        out = dict(t0=t0, horizon=cfg.horizon, coarse_steps=n,
                   rhs_err_plain=e_rhs_plain.tolist(), rhs_err_closure=e_rhs_clos.tolist(),
                   err_plain=e_plain.tolist(), err_closure=e_clos.tolist(),
                   dev_err_plain=e_plain_dev.tolist(), dev_err_closure=e_clos_dev.tolist(),
                   fallback_rate=fb / float(ncells * 3 * n),
                   totals_plain=c.totals(y_plain).tolist(), totals_closure=c.totals(y_clos).tolist(),
                   totals_start=c.totals(yc0).tolist())
        self.log(f"[closure] held-out RHS error plain {np.round(e_rhs_plain, 4)} closure {np.round(e_rhs_clos, 4)}")
        self.log(f"[closure] after {cfg.horizon} ({n} steps): evolution error plain {np.round(e_plain_dev, 4)} "
                 f"closure {np.round(e_clos_dev, 4)}; fallback rate {out['fallback_rate']:.2e}")
        return out


def _rel_l2(a, b):
    """Per-field relative L2 of state-shaped tensors ([z][y][i][l][x])."""
    a = a.double()
    b = b.double()
    num = ((a - b) ** 2).sum(dim=(0, 1, 3, 4)).sqrt()
    den = (b ** 2).sum(dim=(0, 1, 3, 4)).sqrt()
    return (num / den.clamp_min(1e-300)).cpu().numpy()


def run(cfg=None, log=print):
    cfg = cfg or Config()
    ex = Experiment(cfg, log=log)
    ex.generate()
    ex.train()
    res = ex.evaluate()
    res["loss_history"] = ex.loss_history
    return res
