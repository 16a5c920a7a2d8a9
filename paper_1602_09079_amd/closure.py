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
                 nsnap=16, t_gap=0.1, horizon=0.1, batch=4096, iters=3000, lr=1e-3, init_seed=4, batch_seed=17,
                 noise=0.1, noise_seed=29, alphas=(1.0, 0.5, 0.25)):
        self.nc = nc
        self.nf = 2 * nc
        self.mach = mach
        self.ic_seed = ic_seed
        self.forcing = forcing
        self.precision = precision
        self.t_spin = t_spin       # time run before the first training snapshot
        self.dt_snap = dt_snap     # time between snapshots
        self.nsnap = nsnap         # training snapshots
        self.t_gap = t_gap         # time before each held-out window
        self.horizon = horizon     # length of the held-out comparison runs
        self.batch = batch
        self.iters = iters
        self.lr = lr
        self.init_seed = init_seed
        self.batch_seed = batch_seed
        self.noise = noise         # std of the input noise during training (standardised units)
        self.noise_seed = noise_seed
        self.alphas = alphas       # correction scales tried on the validation window


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
        self.plain2 = dg.Solver(1, cfg.nf, **fl)  # the plain scheme with 8x the cells (DOF ladder)
        if cfg.forcing:
            nvec, ahat = driving()
            for s in (self.fine, self.coarse, self.coarse_cl, self.plain2):
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
            net.loss_grad(params, self.X, self.T, rows=rows, grad=grad, loss=loss, noise=cfg.noise,
                          seed=cfg.noise_seed * 1000003 + it)
            net.adam(params, grad, m, v, it, lr=cfg.lr)
            if it == 1 or it % 250 == 0 or it == cfg.iters:
                hist.append((it, float(loss.item())))
        torch.cuda.synchronize()
        self.params = params
        self.net = net
        self.loss_history = hist
        self.log(f"[closure] trained {cfg.iters} Adam steps in {time.perf_counter() - t0:.1f} s, "
                 f"loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}")
        return hist

    def install(self, alpha):
        """The trained network with its correction scaled by alpha."""
        n = dict(self.norm)
        n["out_scale"] = n["out_scale"] * alpha
        self.coarse_cl.set_closure(self.params.cpu().numpy(), **n)

    # ------------------------------------------------------------ evaluation
    def window(self, alphas):
        """A held-out window at a later time: both coarse runs start from P y_f(t0)
        and run for the horizon; the errors are relative to P y_f(t0 + horizon).
        Returns the a-priori operator errors and, per correction scale, the error
        of the evolution (y(T) - y(0) against the restricted fine evolution)."""
        cfg = self.cfg
        c, cl = self.coarse, self.coarse_cl
        self.t = _advance(self.fine, self.yf, cfg.t_gap, self.t)
        t0 = self.t
        yc0 = c.restrict(2, self.yf)
        # plain k = 1 on the fine mesh from the fine state's degree-1 modes (the L2 projection: the
        # basis is orthonormal and graded by degree), for the ladder
        y2 = self.yf[:, :, :, :dg.nmodes(1), :].contiguous()
        prf = c.restrict(2, self.fine.rhs(self.yf))
        self.t = _advance(self.fine, self.yf, cfg.horizon, self.t)
        ref = c.restrict(2, self.yf)
        d_ref = ref - yc0
        h = c.dt(yc0)
        n = max(1, int(math.ceil(cfg.horizon / h)))
        out = dict(t0=t0, horizon=cfg.horizon, coarse_steps=n)
        y = yc0.clone()
        c.step(y, n, cfg.horizon / n)
        out["plain"] = dict(rhs_err=_rel_l2(c.rhs(yc0), prf).tolist(), err=_rel_l2(y - yc0, d_ref).tolist())
        h2 = self.plain2.dt(y2)
        n2 = max(1, int(math.ceil(cfg.horizon / h2)))
        self.plain2.step(y2, n2, cfg.horizon / n2)
        out["plain_8x_dof"] = dict(cells=cfg.nf ** 3, err=_rel_l2(c.restrict(1, y2) - yc0, d_ref).tolist())
        for a in alphas:
            self.install(a)
            cl.closure_fallbacks()
            r = _rel_l2(cl.rhs(yc0), prf).tolist()
            cl.closure_fallbacks()
            y = yc0.clone()
            cl.step(y, n, cfg.horizon / n)
            fb = cl.closure_fallbacks()
            out[f"alpha={a}"] = dict(alpha=a, rhs_err=r, err=_rel_l2(y - yc0, d_ref).tolist(),
                                     fallback_rate=fb / float(cfg.nc ** 3 * 3 * n),
                                     totals_drift=(np.abs(c.totals(y) - c.totals(yc0))).tolist())
        return out

    def evaluate(self):
        """Choose the correction scale on a validation window, then compare with
        the plain scheme on a later test window."""
        val = self.window(self.cfg.alphas)
        best = min(self.cfg.alphas, key=lambda a: float(np.mean(val[f"alpha={a}"]["err"])))
        test = self.window([best])
        res = dict(validation=val, alpha=best, test=test)
        p, cl = test["plain"], test[f"alpha={best}"]
        res["effective_dof_gain"] = effective_dof_gain(p["err"], test["plain_8x_dof"]["err"], cl["err"])
        self.log(f"[closure] alpha={best}; test window t0={test['t0']:.3f}, {test['coarse_steps']} steps")
        self.log(f"[closure] operator error plain {np.round(p['rhs_err'], 3)} closure {np.round(cl['rhs_err'], 3)}")
        self.log(f"[closure] evolution error plain {np.round(p['err'], 3)} closure {np.round(cl['err'], 3)}; "
                 f"fallback rate {cl['fallback_rate']:.2e}")
        self.log(f"[closure] plain with 8x the cells {np.round(test['plain_8x_dof']['err'], 3)}; effective DOF gain "
                 f"of the closure per field {np.round(res['effective_dof_gain'], 2)}")
        return res


def effective_dof_gain(e1, e8, ec):
    """Per field: the DOF factor at which the plain scheme would reach the closure's error, read off
    the plain runs at 1x and 8x the cells (error taken as a power of the DOF between them).  Not
    clipped: a value below 1 means the closure is worse than the plain scheme on that field (a
    coarser plain mesh would match it), above 8 is extrapolated past the ladder."""
    out = []
    for a, b, c in zip(e1, e8, ec):
        if not (b < a) or not (c > 0):
            out.append(float("nan"))
        else:
            out.append(float(8.0 ** (math.log(a / c) / math.log(a / b))))
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
