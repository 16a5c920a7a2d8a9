"""FP64 CPU oracle for the modal DG Euler scheme (arXiv 1602.09079, Sec. 2-3).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It is independent of the GPU library:
no shared code, tables or constants.  See dg_oracle.c for the readings of the
paper that it follows.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

NF = 5

c_double_p = ctypes.POINTER(ctypes.c_double)
c_int_p = ctypes.POINTER(ctypes.c_int32)


class Cfg(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("box", ctypes.c_double * 3),
                ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("riemann", ctypes.c_int32)]


class Forcing(ctypes.Structure):
    _fields_ = [("nmodes", ctypes.c_int32), ("nvec", c_int_p), ("ahat", c_double_p)]


def lib():
    global _lib
    if _lib is None:
        # DG_ORACLE_LIB: an instrumented build of the same source (the sanitizer test uses it)
        path = os.environ.get("DG_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
        src = os.path.join(_HERE, "dg_oracle.c")
        if "DG_ORACLE_LIB" not in os.environ and (
                not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src)):
            _build.build()
        L = ctypes.CDLL(path)
        L.orc_nmodes.restype = ctypes.c_int
        L.orc_pleg.restype = ctypes.c_double
        L.orc_dpleg.restype = ctypes.c_double
        L.orc_dt.restype = ctypes.c_double
        L.orc_mlp_loss_grad.restype = ctypes.c_double
        _lib = L
    return _lib


def _d(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(c_double_p)


def _i(a):
    assert a.dtype == np.int32 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(c_int_p)


def make_cfg(k, n, box=(1.0, 1.0, 1.0), gamma=5.0 / 3.0, cfl=0.3, riemann="hllc"):
    if isinstance(n, int):
        n = (n, n, n)
    c = Cfg()
    c.k = k
    for a in range(3):
        c.n[a] = n[a]
        c.box[a] = box[a]
    c.gamma = gamma
    c.cfl = cfl
    c.riemann = {"hllc": 0, "exact": 1}[riemann]
    return c


class ForcingTable:
    """Keeps the numpy arrays alive behind an orc_forcing struct."""

    def __init__(self, nvec, ahat):
        self.nvec = np.ascontiguousarray(nvec, dtype=np.int32).reshape(-1, 3)
        self.ahat = np.ascontiguousarray(ahat, dtype=np.float64).reshape(-1, 3, 2)
        self.s = Forcing(len(self.nvec), _i(self.nvec), _d(self.ahat))

    def ptr(self):
        return ctypes.byref(self.s)


def _fptr(frc):
    return None if frc is None else frc.ptr()


def nmodes(k):
    return lib().orc_nmodes(k)


def mode_list(k):
    out = np.zeros((nmodes(k), 3), dtype=np.int32)
    lib().orc_mode_list(k, _i(out))
    return out


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    lib().orc_gauss_legendre(n, _d(x), _d(w))
    return x, w


def pleg(u, x):
    return lib().orc_pleg(u, ctypes.c_double(x))


def dpleg(u, x):
    return lib().orc_dpleg(u, ctypes.c_double(x))


def basis(k, xi):
    out = np.zeros(nmodes(k))
    lib().orc_basis(k, _d(np.ascontiguousarray(xi, dtype=np.float64)), _d(out))
    return out


def basis_grad(k, xi):
    out = np.zeros((3, nmodes(k)))
    lib().orc_basis_grad(k, _d(np.ascontiguousarray(xi, dtype=np.float64)), _d(out))
    return out


def state_shape(cfg):
    return (NF, nmodes(cfg.k), cfg.n[2], cfg.n[1], cfg.n[0])


def project(cfg, qp):
    qp = np.ascontiguousarray(qp, dtype=np.float64)
    n = cfg.k + 1
    assert qp.size == NF * n ** 3 * cfg.n[0] * cfg.n[1] * cfg.n[2]
    y = np.zeros(state_shape(cfg))
    lib().orc_project(ctypes.byref(cfg), _d(qp), _d(y))
    return y


def euler_flux(q, axis, gamma):
    F = np.zeros(5)
    lib().orc_euler_flux(_d(np.ascontiguousarray(q, dtype=np.float64)), axis, ctypes.c_double(gamma), _d(F))
    return F


def hllc(qL, qR, axis, gamma):
    F = np.zeros(5)
    lib().orc_hllc(_d(np.ascontiguousarray(qL, dtype=np.float64)), _d(np.ascontiguousarray(qR, dtype=np.float64)),
                   axis, ctypes.c_double(gamma), _d(F))
    return F


def exact_riemann(qL, qR, axis, gamma):
    F = np.zeros(5)
    lib().orc_exact_riemann(_d(np.ascontiguousarray(qL, dtype=np.float64)),
                            _d(np.ascontiguousarray(qR, dtype=np.float64)), axis, ctypes.c_double(gamma), _d(F))
    return F


def rhs(cfg, y, frc=None):
    y = np.ascontiguousarray(y, dtype=np.float64)
    r = np.zeros_like(y)
    lib().orc_rhs(ctypes.byref(cfg), _d(y), _fptr(frc), _d(r))
    return r


def rhs_cells(cfg, y, cells, frc=None):
    """R at the listed cells (flat index (z*ny + y)*nx + x); returns [len(cells)][5][N]."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    r = np.zeros((len(cells), NF, nmodes(cfg.k)))
    lib().orc_rhs_cells(ctypes.byref(cfg), _d(y), _fptr(frc), ctypes.c_int64(len(cells)),
                        cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _d(r))
    return r


def dt(cfg, y):
    return lib().orc_dt(ctypes.byref(cfg), _d(np.ascontiguousarray(y, dtype=np.float64)))


def stage(cfg, y0, yin, a, b, h, frc=None):
    y0 = np.ascontiguousarray(y0, dtype=np.float64)
    yin = np.ascontiguousarray(yin, dtype=np.float64)
    out = np.zeros_like(yin)
    lib().orc_stage(ctypes.byref(cfg), _d(y0), _d(yin), ctypes.c_double(a), ctypes.c_double(b),
                    ctypes.c_double(h), _fptr(frc), _d(out))
    return out


def step(cfg, y, h=0.0, nsteps=1, t=0.0, frc=None):
    """Returns (y_new, t_new); y is not modified."""
    y = np.array(y, dtype=np.float64, copy=True, order="C")
    tt = ctypes.c_double(t)
    lib().orc_step(ctypes.byref(cfg), _d(y), ctypes.c_double(h), nsteps, ctypes.byref(tt), _fptr(frc))
    return y, tt.value


def totals(cfg, y):
    out = np.zeros(5)
    lib().orc_totals(ctypes.byref(cfg), _d(np.ascontiguousarray(y, dtype=np.float64)), _d(out))
    return out


def accel(frc, box, x):
    a = np.zeros(3)
    lib().orc_accel(frc.ptr(), _d(np.ascontiguousarray(box, dtype=np.float64)),
                    _d(np.ascontiguousarray(x, dtype=np.float64)), _d(a))
    return a


def ou_update(nvec, theta, z, f, sigma, a0, kmin, kmax):
    """Returns (theta_new, ahat)."""
    nvec = np.ascontiguousarray(nvec, dtype=np.int32)
    th = np.array(theta, dtype=np.float64, copy=True, order="C")
    z = np.ascontiguousarray(z, dtype=np.float64)
    ahat = np.zeros_like(th)
    lib().orc_ou_update(len(nvec), _i(nvec), _d(th), _d(z), ctypes.c_double(f), ctypes.c_double(sigma),
                        ctypes.c_double(a0), ctypes.c_double(kmin), ctypes.c_double(kmax), _d(ahat))
    return th, ahat


def restrict(kf, kc, nc, yf):
    if isinstance(nc, int):
        nc = (nc, nc, nc)
    ncv = np.array(nc, dtype=np.int32)
    yf = np.ascontiguousarray(yf, dtype=np.float64)
    yc = np.zeros((NF, nmodes(kc), nc[2], nc[1], nc[0]))
    lib().orc_restrict(kf, kc, _i(ncv), _d(yf), _d(yc))
    return yc


MLP_SHAPE = (140, 128, 128, 20)


def mlp_nparams(nin, nh1, nh2, nout):
    return nh1 * nin + nh1 + nh2 * nh1 + nh2 + nout * nh2 + nout


def mlp_forward(params, x, shape=MLP_SHAPE):
    nin, nh1, nh2, nout = shape
    x = np.ascontiguousarray(x, dtype=np.float64)
    B = x.shape[0]
    h1 = np.zeros((B, nh1))
    h2 = np.zeros((B, nh2))
    y = np.zeros((B, nout))
    lib().orc_mlp_forward(nin, nh1, nh2, nout, _d(np.ascontiguousarray(params, dtype=np.float64)), B,
                          _d(x), _d(h1), _d(h2), _d(y))
    return h1, h2, y


def mlp_loss_grad(params, x, target, shape=MLP_SHAPE):
    nin, nh1, nh2, nout = shape
    x = np.ascontiguousarray(x, dtype=np.float64)
    target = np.ascontiguousarray(target, dtype=np.float64)
    g = np.zeros(mlp_nparams(*shape))
    loss = lib().orc_mlp_loss_grad(nin, nh1, nh2, nout, _d(np.ascontiguousarray(params, dtype=np.float64)),
                                   x.shape[0], _d(x), _d(target), _d(g))
    return loss, g


def adam(params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of params, m, v (float64 arrays)."""
    lib().orc_adam(len(params), _d(params), _d(np.ascontiguousarray(grad, dtype=np.float64)), _d(m), _d(v),
                   step, ctypes.c_double(lr), ctypes.c_double(beta1), ctypes.c_double(beta2), ctypes.c_double(eps))


def rel_l2(a, b):
    """Per-field relative L2 error ||a - b|| / ||b|| over all (mode, cell)."""
    a = np.asarray(a, dtype=np.float64).reshape(NF, -1)
    b = np.asarray(b, dtype=np.float64).reshape(NF, -1)
    nb = np.linalg.norm(b, axis=1)
    return np.linalg.norm(a - b, axis=1) / np.where(nb > 0, nb, 1.0)


class Closure(ctypes.Structure):
    _fields_ = [("nin", ctypes.c_int32), ("nh1", ctypes.c_int32), ("nh2", ctypes.c_int32), ("nout", ctypes.c_int32),
                ("params", c_double_p), ("feat_mean", c_double_p), ("feat_std", c_double_p),
                ("out_scale", c_double_p), ("out_bound", c_double_p)]


class ClosureParams:
    """Keeps the arrays alive behind an orc_closure struct."""

    def __init__(self, params, feat_mean, feat_std, out_scale, out_bound, shape=MLP_SHAPE):
        f = lambda a: np.ascontiguousarray(a, dtype=np.float64)
        self.arrays = [f(params), f(feat_mean), f(feat_std), f(out_scale), f(out_bound)]
        self.s = Closure(*shape, *[_d(a) for a in self.arrays])

    def ptr(self):
        return ctypes.byref(self.s)


def closure_features(cfg, y):
    """[ncells][7][5][N] features (self, -x, +x, -y, +y, -z, +z)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    N = nmodes(cfg.k)
    nc = cfg.n[0] * cfg.n[1] * cfg.n[2]
    out = np.zeros((nc, 7, NF, N))
    lib().orc_closure_features(ctypes.byref(cfg), _d(y), _d(out))
    return out


def closure_correction(cfg, y, clo):
    """Returns (corr in state layout, number of cells that fell back)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    corr = np.zeros_like(y)
    L = lib()
    L.orc_closure_correction.restype = ctypes.c_int64
    nfb = L.orc_closure_correction(ctypes.byref(cfg), _d(y), clo.ptr(), _d(corr))
    return corr, int(nfb)


LIMIT_EPS = 1e-13


def gll(m):
    x = np.zeros(m)
    w = np.zeros(m)
    lib().orc_gll(m, _d(x), _d(w))
    return x, w


def limiter_points(k):
    pts = np.zeros((3 * 4 * (k + 1) ** 2, 3))
    n = lib().orc_limiter_points(k, _d(pts))
    return pts[:n]


LIMIT_REL_FP32 = 2.0 ** -20


def limit(cfg, y, eps=LIMIT_EPS, rel=0.0):
    """Returns (limited copy of y, theta [cells][2]).  rel: see orc_limit (2^-20 for FP32 storage)."""
    y = np.array(y, dtype=np.float64, copy=True, order="C")
    th = np.zeros((cfg.n[0] * cfg.n[1] * cfg.n[2], 2))
    lib().orc_limit(ctypes.byref(cfg), _d(y), ctypes.c_double(eps), ctypes.c_double(rel), _d(th))
    return y, th


def dt_limited(cfg, y):
    L = lib()
    L.orc_dt_limited.restype = ctypes.c_double
    return L.orc_dt_limited(ctypes.byref(cfg), _d(np.ascontiguousarray(y, dtype=np.float64)))


def step_limited(cfg, y, h=0.0, nsteps=1, t=0.0, frc=None, eps=LIMIT_EPS):
    y = np.array(y, dtype=np.float64, copy=True, order="C")
    tt = ctypes.c_double(t)
    lib().orc_step_limited(ctypes.byref(cfg), _d(y), ctypes.c_double(h), nsteps, ctypes.byref(tt), _fptr(frc),
                           ctypes.c_double(eps))
    return y, tt.value


def isothermal_reset(cfg, y, cs=1.0, rho0=1.0):
    """Sec. 3.2.  Returns (copy of y with the energy weights reset, dissipated energy)."""
    y = np.array(y, dtype=np.float64, copy=True, order="C")
    L = lib()
    L.orc_isothermal_reset.restype = ctypes.c_double
    d = L.orc_isothermal_reset(ctypes.byref(cfg), _d(y), ctypes.c_double(cs), ctypes.c_double(rho0))
    return y, d


def step_isothermal(cfg, y, h=0.0, nsteps=1, t=0.0, frc=None, cs=1.0, rho0=1.0, limit=False, eps=LIMIT_EPS):
    """nsteps steps each followed by the reset (and the limiter with limit=True).
    Returns (y, t, dissipated energy summed over the steps)."""
    y = np.array(y, dtype=np.float64, copy=True, order="C")
    tt = ctypes.c_double(t)
    dis = ctypes.c_double(0.0)
    lib().orc_step_isothermal(ctypes.byref(cfg), _d(y), ctypes.c_double(h), nsteps, ctypes.byref(tt), _fptr(frc),
                              ctypes.c_double(cs), ctypes.c_double(rho0), int(bool(limit)), ctypes.c_double(eps),
                              ctypes.byref(dis))
    return y, tt.value, dis.value
