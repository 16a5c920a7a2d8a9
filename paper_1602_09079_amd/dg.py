"""ctypes binding of libdgmi.so (include/dg.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.  PyTorch supplies
device memory and the current stream.

The library must have been built (``__graft_entry__.build()``); importing this
module without it raises, there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# DGMI_LIB: another build of the same library to load (the tests use it for an instrumented build)
LIB_PATH = os.environ.get("DGMI_LIB") or os.path.join(HERE, "libdgmi.so")

DG_OK, DG_ERR_ARG, DG_ERR_UNSUPPORTED, DG_ERR_HIP, DG_ERR_RANGE, DG_ERR_STATE = range(6)
PRECISIONS = {"fp64": 0, "fp32": 1, "bf16": 2, "bf16x3": 3}
DG_FORCING = 1
DG_CLOSURE = 2
DG_CHECK_RANGE = 4
DG_LIMIT = 8
DG_ISOTHERMAL = 16
DG_EXACT_RIEMANN = 32
DG_ZHALO = 64
STATUS_NAMES = {0: "DG_OK", 1: "DG_ERR_ARG", 2: "DG_ERR_UNSUPPORTED", 3: "DG_ERR_HIP", 4: "DG_ERR_RANGE",
                5: "DG_ERR_STATE"}

# every entry point declared in include/dg.h
EXPORTS = ["dg_init", "dg_destroy", "dg_state_count", "dg_workspace_bytes", "dg_project", "dg_rhs", "dg_stage",
           "dg_dt", "dg_step", "dg_totals", "dg_set_forcing", "dg_ou_update", "dg_nmodes", "dg_gauss_nodes",
           "dg_error_string", "dg_set_closure", "dg_closure_fallbacks", "dg_closure_features", "dg_closure_targets",
           "dg_restrict", "dg_mlp_nparams", "dg_mlp_workspace_bytes", "dg_mlp_forward", "dg_mlp_loss_grad", "dg_adam",
           "dg_column_stats_workspace_bytes", "dg_column_stats", "dg_column_stats_noalloc", "dg_standardize", "dg_limiter_stats",
           "dg_set_isothermal", "dg_isothermal_reset", "dg_dissipated", "dg_sample",
           "dg_spectrum_workspace_bytes", "dg_velocity_spectrum", "dg_density_pdf", "dg_rms_mach",
           "dg_plane_count", "dg_set_halo", "dg_set_slab", "dg_set_zchunk", "dg_state_import", "dg_state_export"]


class DGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("box", ctypes.c_double * 3),
                ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_fp = ctypes.POINTER(ctypes.c_float)


def hip_runtimes():
    """Distinct libamdhip64 files mapped into this process (Linux; empty elsewhere)."""
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # torch's HIP runtime first: the library's libamdhip64 dependency then resolves to the
        # copy already mapped (same soname).  Loaded the other way round, the process holds two
        # HIP runtimes and torch's streams and buffers are foreign to the library's.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        runtimes = hip_runtimes()
        if len(runtimes) > 1:
            raise RuntimeError(f"{LIB_PATH} loaded a second HIP runtime beside torch's: {runtimes}")
        sig = {
            "dg_init": (ctypes.c_int, [ctypes.POINTER(Config), _vp, ctypes.POINTER(_vp)]),
            "dg_destroy": (ctypes.c_int, [_vp]),
            "dg_state_count": (ctypes.c_size_t, [_vp]),
            "dg_workspace_bytes": (ctypes.c_size_t, [_vp]),
            "dg_project": (ctypes.c_int, [_vp, _vp, _vp]),
            "dg_state_import": (ctypes.c_int, [_vp, _vp, _vp]),
            "dg_state_export": (ctypes.c_int, [_vp, _vp, _vp]),
            "dg_rhs": (ctypes.c_int, [_vp, _vp, _vp]),
            "dg_stage": (ctypes.c_int, [_vp, _vp, _vp, _vp, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
            "dg_dt": (ctypes.c_int, [_vp, _vp, _dp]),
            "dg_step": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_int32, _dp]),
            "dg_totals": (ctypes.c_int, [_vp, _vp, _dp]),
            "dg_set_forcing": (ctypes.c_int, [_vp, ctypes.c_int32, _ip, _dp]),
            "dg_ou_update": (ctypes.c_int, [ctypes.c_int32, _ip, _dp, _dp, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]),
            "dg_nmodes": (ctypes.c_int32, [ctypes.c_int32]),
            "dg_gauss_nodes": (ctypes.c_int, [ctypes.c_int32, _dp]),
            "dg_error_string": (ctypes.c_char_p, [_vp]),
            "dg_set_closure": (ctypes.c_int, [_vp, _fp, _fp, _fp, _fp, _fp]),
            "dg_closure_fallbacks": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)]),
            "dg_closure_features": (ctypes.c_int, [_vp, _vp, _vp]),
            "dg_closure_targets": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
            "dg_restrict": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp]),
            "dg_mlp_nparams": (ctypes.c_size_t, [_ip]),
            "dg_mlp_workspace_bytes": (ctypes.c_size_t, [_ip, ctypes.c_int32]),
            "dg_mlp_forward": (ctypes.c_int, [_ip, _vp, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp]),
            "dg_mlp_loss_grad": (ctypes.c_int, [_ip, _vp, ctypes.c_int32, _vp, _vp, _vp, ctypes.c_float,
                                                ctypes.c_uint64, _vp, _vp, _vp, _vp]),
            "dg_adam": (ctypes.c_int, [ctypes.c_int64, _vp, _vp, _vp, _vp, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double, _vp]),
            "dg_column_stats_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32]),
            "dg_column_stats": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp, _vp, _vp]),
            "dg_column_stats_noalloc": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp, _vp,
                                                       _vp]),
            "dg_standardize": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int32, _vp, _vp, _vp]),
            "dg_limiter_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64)]),
            "dg_set_isothermal": (ctypes.c_int, [_vp, ctypes.c_double, ctypes.c_double]),
            "dg_isothermal_reset": (ctypes.c_int, [_vp, _vp]),
            "dg_dissipated": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double)]),
            "dg_sample": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, _vp]),
            "dg_spectrum_workspace_bytes": (ctypes.c_size_t, [_vp, ctypes.c_int32]),
            "dg_velocity_spectrum": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp, _vp]),
            "dg_density_pdf": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_int32, _vp]),
            "dg_rms_mach": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
            "dg_plane_count": (ctypes.c_size_t, [_vp]),
            "dg_set_halo": (ctypes.c_int, [_vp, _vp, _vp]),
            "dg_set_slab": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32]),
            "dg_set_zchunk": (ctypes.c_int, [_vp, ctypes.c_int32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def nmodes(k):
    return lib().dg_nmodes(k)


def gauss_nodes(n):
    import numpy as np
    x = np.zeros(max(n, 1))
    st = lib().dg_gauss_nodes(n, x.ctypes.data_as(_dp))
    if st != DG_OK:
        raise DGError(st, f"dg_gauss_nodes({n})")
    return x


def ou_update(nvec, theta, z, f, sigma, a0, kmin, kmax):
    """Host-only OU driving update; returns (theta_new, ahat) as float64 arrays [m][3][2]."""
    import numpy as np
    nvec = np.ascontiguousarray(nvec, dtype=np.int32)
    th = np.array(theta, dtype=np.float64, copy=True, order="C")
    z = np.ascontiguousarray(z, dtype=np.float64)
    ahat = np.zeros_like(th)
    st = lib().dg_ou_update(len(nvec), nvec.ctypes.data_as(_ip), th.ctypes.data_as(_dp), z.ctypes.data_as(_dp),
                            f, sigma, a0, kmin, kmax, ahat.ctypes.data_as(_dp))
    if st != DG_OK:
        raise DGError(st, "dg_ou_update")
    return th, ahat


def make_config(k, n, box=(1.0, 1.0, 1.0), gamma=5.0 / 3.0, cfl=0.3, precision="fp32", flags=0):
    if isinstance(n, int):
        n = (n, n, n)
    c = Config()
    c.k = k
    for a in range(3):
        c.n[a] = n[a]
        c.box[a] = box[a]
    c.gamma = gamma
    c.cfl = cfl
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    c.flags = flags
    return c


def init_status(cfg):
    """dg_init's status for cfg, destroying any context it made (used to test validation)."""
    ctx = _vp()
    st = lib().dg_init(ctypes.byref(cfg), None, ctypes.byref(ctx))
    if st == DG_OK:
        lib().dg_destroy(ctx)
    return st


class Solver:
    """One DG context on the current CUDA (HIP) device and stream."""

    def __init__(self, k, n, box=(1.0, 1.0, 1.0), gamma=5.0 / 3.0, cfl=0.3, precision="fp32", flags=0,
                 forcing=False, check_range=False, closure=False, limit=False, isothermal=False, riemann="hllc",
                 zhalo=False, stream=None):
        import torch
        if zhalo:
            flags |= DG_ZHALO
        if riemann not in ("hllc", "exact"):
            raise ValueError("riemann must be 'hllc' or 'exact'")
        if riemann == "exact":
            flags |= DG_EXACT_RIEMANN
        if isothermal:
            flags |= DG_ISOTHERMAL
        if forcing:
            flags |= DG_FORCING
        if limit:
            flags |= DG_LIMIT
        if closure:
            flags |= DG_CLOSURE
        if check_range:
            flags |= DG_CHECK_RANGE
        self.cfg = make_config(k, n, box, gamma, cfl, precision, flags)
        self.k = k
        self.n = tuple(self.cfg.n)
        self.precision = precision
        self.dtype = torch.float64 if self.cfg.precision == 0 else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._ctx = _vp()
        st = lib().dg_init(ctypes.byref(self.cfg), _vp(self.stream.cuda_stream), ctypes.byref(self._ctx))
        if st != DG_OK:
            why = lib().dg_error_string(None)
            raise DGError(st, f"dg_init failed ({why.decode() if why else ''})")
        self.N = nmodes(k)
        self.nq = k + 1
        self._work = None

    def __del__(self):
        try:
            if self._ctx:
                lib().dg_destroy(self._ctx)
                self._ctx = _vp()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def _check(self, st, what):
        if st != DG_OK:
            msg = lib().dg_error_string(self._ctx)
            raise DGError(st, f"{what}: {msg.decode() if msg else ''}")

    def state_shape(self):
        """[z][y][i][l][x]: each row of cells holds its 5 N rows of weights contiguously."""
        return (self.n[2], self.n[1], 5, self.N, self.n[0])

    def canonical_shape(self):
        """[i][l][z][y][x]: one plane of cells per (field, mode)."""
        return (5, self.N, self.n[2], self.n[1], self.n[0])

    def empty_state(self):
        import torch
        return torch.empty(self.state_shape(), dtype=self.dtype, device=self.device)

    def _ptr(self, t, shape=None):
        if t.dtype != self.dtype or not t.is_contiguous() or t.device.type != "cuda":
            raise ValueError(f"expected a contiguous {self.dtype} CUDA tensor")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return _vp(t.data_ptr())

    def workspace(self):
        import torch
        if self._work is None:
            nb = lib().dg_workspace_bytes(self._ctx)
            self._work = torch.empty(nb, dtype=torch.uint8, device=self.device)
        return self._work

    # ------------------------------------------------------------ entry points
    def project(self, qp, out=None):
        """qp: [5][n][n][n][nz][ny][nx] point values at the Gauss offsets."""
        q = self.nq
        shape = (5, q, q, q, self.n[2], self.n[1], self.n[0])
        y = self.empty_state() if out is None else out
        self._check(lib().dg_project(self._ctx, self._ptr(qp, shape), self._ptr(y, self.state_shape())),
                    "dg_project")
        return y

    def import_state(self, canon, out=None):
        """State from the canonical order [i][l][z][y][x] into the library's order."""
        y = self.empty_state() if out is None else out
        self._check(lib().dg_state_import(self._ctx, self._ptr(canon, self.canonical_shape()),
                                          self._ptr(y, self.state_shape())), "dg_state_import")
        return y

    def export_state(self, y, out=None):
        """The library's state in the canonical order [i][l][z][y][x]."""
        import torch
        c = torch.empty(self.canonical_shape(), dtype=self.dtype, device=self.device) if out is None else out
        self._check(lib().dg_state_export(self._ctx, self._ptr(y, self.state_shape()),
                                          self._ptr(c, self.canonical_shape())), "dg_state_export")
        return c

    def rhs(self, y, out=None):
        r = self.empty_state() if out is None else out
        self._check(lib().dg_rhs(self._ctx, self._ptr(y, self.state_shape()), self._ptr(r, self.state_shape())),
                    "dg_rhs")
        return r

    def stage(self, y0, yin, out, a, b, dt):
        p0 = self._ptr(y0, self.state_shape()) if y0 is not None else _vp()
        self._check(lib().dg_stage(self._ctx, p0, self._ptr(yin, self.state_shape()),
                                   self._ptr(out, self.state_shape()), a, b, dt), "dg_stage")
        return out

    def dt(self, y):
        v = ctypes.c_double()
        self._check(lib().dg_dt(self._ctx, self._ptr(y, self.state_shape()), ctypes.byref(v)), "dg_dt")
        return v.value

    def step(self, y, nsteps=1, dt=0.0, t=0.0):
        """Advance y in place; returns the new time (synchronises when dt <= 0)."""
        tt = ctypes.c_double(t)
        w = self.workspace()
        self._check(lib().dg_step(self._ctx, self._ptr(y, self.state_shape()), _vp(w.data_ptr()), dt, nsteps,
                                  ctypes.byref(tt)), "dg_step")
        return tt.value

    def step_async(self, y, nsteps=1, dt=0.0):
        """Advance y in place without reading back the time (no host synchronisation)."""
        w = self.workspace()
        self._check(lib().dg_step(self._ctx, self._ptr(y, self.state_shape()), _vp(w.data_ptr()), dt, nsteps,
                                  None), "dg_step")

    def totals(self, y):
        import numpy as np
        out = np.zeros(5)
        self._check(lib().dg_totals(self._ctx, self._ptr(y, self.state_shape()), out.ctypes.data_as(_dp)),
                    "dg_totals")
        return out

    def set_forcing(self, nvec, ahat):
        import numpy as np
        nvec = np.ascontiguousarray(nvec, dtype=np.int32).reshape(-1, 3)
        ahat = np.ascontiguousarray(ahat, dtype=np.float64).reshape(-1, 3, 2)
        self._check(lib().dg_set_forcing(self._ctx, len(nvec), nvec.ctypes.data_as(_ip), ahat.ctypes.data_as(_dp)),
                    "dg_set_forcing")

    # ------------------------------------------------------------ closure
    def set_closure(self, params, feat_mean, feat_std, out_scale, out_bound):
        """Host arrays (any float dtype), copied as float32."""
        import numpy as np
        a = [np.ascontiguousarray(np.asarray(v, dtype=np.float64).astype(np.float32))
             for v in (params, feat_mean, feat_std, out_scale, out_bound)]
        self._check(lib().dg_set_closure(self._ctx, *[v.ctypes.data_as(_fp) for v in a]), "dg_set_closure")

    def limiter_stats(self):
        """Cells the positivity limiter changed since the previous call."""
        v = ctypes.c_int64()
        self._check(lib().dg_limiter_stats(self._ctx, ctypes.byref(v)), "dg_limiter_stats")
        return v.value

    def set_isothermal(self, cs=1.0, rho0=1.0):
        """Sound speed and reference density of the isothermal reset."""
        self._check(lib().dg_set_isothermal(self._ctx, ctypes.c_double(cs), ctypes.c_double(rho0)),
                    "dg_set_isothermal")

    def isothermal_reset(self, y):
        """One reset of y in place (its dissipated energy goes to dissipated())."""
        self._check(lib().dg_isothermal_reset(self._ctx, self._ptr(y, self.state_shape())), "dg_isothermal_reset")
        return y

    def dissipated(self):
        """Dissipated energy of the resets since the previous call."""
        v = ctypes.c_double()
        self._check(lib().dg_dissipated(self._ctx, ctypes.byref(v)), "dg_dissipated")
        return v.value

    # ------------------------------------------------------------ z slabs
    def set_halo(self, lo, hi):
        """Halo planes [y][i][l][x] (device tensors of the storage type, kept alive by the caller)."""
        shape = (self.n[1], 5, self.N, self.n[0])
        self._halo = (lo, hi)
        self._check(lib().dg_set_halo(self._ctx, self._ptr(lo, shape), self._ptr(hi, shape)), "dg_set_halo")

    def set_slab(self, z0, nz_global):
        self._check(lib().dg_set_slab(self._ctx, z0, nz_global), "dg_set_slab")

    def set_zchunk(self, length):
        """z-chunk length of the stage sweep (0: the automatic choice); results are independent of it."""
        self._check(lib().dg_set_zchunk(self._ctx, length), "dg_set_zchunk")

    # ------------------------------------------------------------ diagnostics (Sec. 3.3, 4.1, 4.4)
    def sample(self, y, S=4):
        """The five conserved fields on the sub-cell grid: [5][S nz][S ny][S nx]."""
        import torch
        out = torch.empty((5, S * self.n[2], S * self.n[1], S * self.n[0]), dtype=self.dtype, device=self.device)
        self._check(lib().dg_sample(self._ctx, self._ptr(y, self.state_shape()), S, _vp(out.data_ptr())),
                    "dg_sample")
        return out

    def velocity_spectrum(self, y, S=4, nbins=None, work=None):
        """Shell powers P(s), s < nbins (default S n), summed over the velocity components."""
        import numpy as np
        import torch
        nbins = S * self.n[0] if nbins is None else nbins
        if work is None:
            work = torch.empty(lib().dg_spectrum_workspace_bytes(self._ctx, S), dtype=torch.uint8, device=self.device)
        out = np.zeros(nbins)
        self._check(lib().dg_velocity_spectrum(self._ctx, self._ptr(y, self.state_shape()), S, nbins,
                                               out.ctypes.data_as(_dp), _vp(work.data_ptr())), "dg_velocity_spectrum")
        return out

    def density_pdf(self, y, S=4, lo=-1.0, hi=1.0, nbins=100):
        """Counts of log10(rho): [below lo, nbins bins of [lo, hi), at or above hi]."""
        import numpy as np
        out = np.zeros(nbins + 2, dtype=np.int64)
        self._check(lib().dg_density_pdf(self._ctx, self._ptr(y, self.state_shape()), S, lo, hi, nbins,
                                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))), "dg_density_pdf")
        return out

    def rms_mach(self, y, S=4):
        v = ctypes.c_double()
        self._check(lib().dg_rms_mach(self._ctx, self._ptr(y, self.state_shape()), S, ctypes.byref(v)),
                    "dg_rms_mach")
        return v.value

    def closure_fallbacks(self):
        v = ctypes.c_int64()
        self._check(lib().dg_closure_fallbacks(self._ctx, ctypes.byref(v)), "dg_closure_fallbacks")
        return v.value

    def closure_features(self, y, out=None):
        import torch
        nc = self.n[0] * self.n[1] * self.n[2]
        f = torch.empty((nc, 7 * 5 * self.N), dtype=torch.float32, device=self.device) if out is None else out
        self._check(lib().dg_closure_features(self._ctx, self._ptr(y, self.state_shape()), _vp(f.data_ptr())),
                    "dg_closure_features")
        return f

    def closure_targets(self, r_coarse, r_fine_restricted, out=None):
        import torch
        nc = self.n[0] * self.n[1] * self.n[2]
        t = torch.empty((nc, 5 * self.N), dtype=torch.float32, device=self.device) if out is None else out
        self._check(lib().dg_closure_targets(self._ctx, self._ptr(r_coarse, self.state_shape()),
                                             self._ptr(r_fine_restricted, self.state_shape()), _vp(t.data_ptr())),
                    "dg_closure_targets")
        return t

    def restrict(self, kf, yf, out=None):
        """yf: a degree-kf state on the mesh with twice the cells per axis (same storage type)."""
        yc = self.empty_state() if out is None else out
        fshape = (2 * self.n[2], 2 * self.n[1], 5, nmodes(kf), 2 * self.n[0])
        self._check(lib().dg_restrict(self._ctx, kf, self._ptr(yf, fshape), self._ptr(yc, self.state_shape())),
                    "dg_restrict")
        return yc


# ---------------------------------------------------------------- dense networks (closure training)

def _f32ptr(t):
    import torch
    if t.dtype != torch.float32 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("expected a contiguous float32 CUDA tensor")
    return _vp(t.data_ptr())


def _shape_arr(shape):
    return (ctypes.c_int32 * 4)(*shape)


def mlp_nparams(shape):
    return lib().dg_mlp_nparams(_shape_arr(shape))


class MLP:
    """Device-side tanh network of the closure: forward, loss gradient, Adam."""

    def __init__(self, shape, batch, stream=None):
        import torch
        self.shape = tuple(shape)
        self.batch = batch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nb = lib().dg_mlp_workspace_bytes(_shape_arr(shape), batch)
        if nb == 0:
            raise ValueError("invalid network shape or batch")
        self.work = torch.empty(nb, dtype=torch.uint8, device="cuda")
        self.nparams = mlp_nparams(shape)

    def _s(self):
        return _vp(self.stream.cuda_stream)

    def forward(self, params, x, rows=None, batch=None):
        import torch
        B = batch or (len(rows) if rows is not None else x.shape[0])
        if B > self.batch:
            raise ValueError("batch larger than the workspace")
        y = torch.empty((B, self.shape[3]), dtype=torch.float32, device="cuda")
        rp = _vp(rows.data_ptr()) if rows is not None else _vp()
        st = lib().dg_mlp_forward(_shape_arr(self.shape), _f32ptr(params), B, _f32ptr(x), rp, _f32ptr(y),
                                  _vp(self.work.data_ptr()), self._s())
        if st != DG_OK:
            raise DGError(st, "dg_mlp_forward")
        return y

    def loss_grad(self, params, x, target, rows=None, grad=None, loss=None, batch=None, noise=0.0, seed=0):
        """Returns (grad, loss) device tensors; loss is a float64 scalar tensor.  noise > 0 perturbs
        the batch inputs with noise * N(0,1) drawn from the counter-based generator keyed by seed."""
        import torch
        B = batch or (len(rows) if rows is not None else x.shape[0])
        if B > self.batch:
            raise ValueError("batch larger than the workspace")
        g = torch.empty(self.nparams, dtype=torch.float32, device="cuda") if grad is None else grad
        lo = torch.empty((), dtype=torch.float64, device="cuda") if loss is None else loss
        rp = _vp(rows.data_ptr()) if rows is not None else _vp()
        st = lib().dg_mlp_loss_grad(_shape_arr(self.shape), _f32ptr(params), B, _f32ptr(x), _f32ptr(target), rp,
                                    noise, seed, _f32ptr(g), _vp(lo.data_ptr()), _vp(self.work.data_ptr()),
                                    self._s())
        if st != DG_OK:
            raise DGError(st, "dg_mlp_loss_grad")
        return g, lo

    def adam(self, params, grad, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        st = lib().dg_adam(self.nparams, _f32ptr(params), _f32ptr(grad), _f32ptr(m), _f32ptr(v), step, lr, beta1,
                           beta2, eps, self._s())
        if st != DG_OK:
            raise DGError(st, "dg_adam")


def column_stats(x, stream=None):
    """(mean, std, rms, maxabs) float64 device tensors of the columns of a float32 [rows][cols] tensor."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    rows, cols = x.shape
    out = [torch.empty(cols, dtype=torch.float64, device="cuda") for _ in range(4)]
    work = torch.empty(lib().dg_column_stats_workspace_bytes(cols), dtype=torch.uint8, device="cuda")
    st = lib().dg_column_stats(_f32ptr(x), rows, cols, *[_vp(o.data_ptr()) for o in out], _vp(work.data_ptr()),
                               _vp(s.cuda_stream))
    if st != DG_OK:
        raise DGError(st, "dg_column_stats")
    return tuple(out)


def standardize(x, shift, scale, stream=None):
    """x = (x - shift) / scale in place, per column (shift, scale: float64 device tensors)."""
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    rows, cols = x.shape
    st = lib().dg_standardize(_f32ptr(x), rows, cols, _vp(shift.data_ptr()), _vp(scale.data_ptr()),
                              _vp(s.cuda_stream))
    if st != DG_OK:
        raise DGError(st, "dg_standardize")
    return x
