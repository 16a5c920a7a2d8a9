"""Seeded synthetic inputs shared by the GPU library's callers and the oracle.

This module holds none of the method's arithmetic: it only produces point
values of prescribed fields, random draws and integer mode lists.  The
quadrature offsets at which fields are sampled are passed in by the caller, so
each side uses its own Gauss nodes.

Point-value layout (what ``dg_project`` and the oracle's projection take):
    qp[i][c][b][a][z][y][x]
i = conserved field (rho, m_x, m_y, m_z, E); a, b, c = Gauss index along
x, y, z; the sample point of Gauss index a in cell ix is
x = (ix + (1 + xi_a) / 2) * box / n.

Workloads (stand-ins for the paper's own turbulence runs, whose data is not
public):
  * ``advected_wave``: rho = 1 + 0.1 sin(2 pi (x + y + z)), v = (1, 1, 1),
    p = 1; exact solution rho(x - v t).
  * ``turbulence``: rho = 1, p = 1 and a solenoidal Gaussian random velocity
    with a k^(-5/3) shell spectrum on 1 <= |n| <= 16 (capped below the
    grid's Nyquist mode), rescaled to a given rms Mach number.  This mimics
    developed subsonic turbulence with an inertial range, as in the paper's
    driven runs.
"""
import math

import numpy as np

NF = 5


def _axis_points(nc, box, nodes):
    """Physical coordinates [len(nodes), nc] of the sample points along one axis."""
    dx = box / nc
    nodes = np.asarray(nodes, dtype=np.float64)
    return (np.arange(nc)[None, :] + 0.5 * (1.0 + nodes[:, None])) * dx


def advected_wave(ncells, nodes, box=(1.0, 1.0, 1.0), gamma=5.0 / 3.0, t=0.0, amp=0.1,
                  vel=(1.0, 1.0, 1.0), p0=1.0):
    """Point values [5][n][n][n][nz][ny][nx] of the advected density wave at time t."""
    if isinstance(ncells, int):
        ncells = (ncells, ncells, ncells)
    nx, ny, nz = ncells
    n = len(nodes)
    X = _axis_points(nx, box[0], nodes)  # [a, ix]
    Y = _axis_points(ny, box[1], nodes)
    Z = _axis_points(nz, box[2], nodes)
    ph = (X[None, None, :, None, None, :] - vel[0] * t) / box[0] \
        + (Y[None, :, None, None, :, None] - vel[1] * t) / box[1] \
        + (Z[:, None, None, :, None, None] - vel[2] * t) / box[2]
    rho = 1.0 + amp * np.sin(2.0 * np.pi * ph)
    shape = (NF, n, n, n, nz, ny, nx)
    out = np.empty(shape)
    out[0] = rho
    out[1] = rho * vel[0]
    out[2] = rho * vel[1]
    out[3] = rho * vel[2]
    out[4] = p0 / (gamma - 1.0) + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    return out


def uniform_state(ncells, nodes, rho=1.0, vel=(0.3, -0.2, 0.1), p=1.0, gamma=5.0 / 3.0):
    if isinstance(ncells, int):
        ncells = (ncells, ncells, ncells)
    nx, ny, nz = ncells
    n = len(nodes)
    out = np.empty((NF, n, n, n, nz, ny, nx))
    out[0] = rho
    for a in range(3):
        out[1 + a] = rho * vel[a]
    out[4] = p / (gamma - 1.0) + 0.5 * rho * sum(v * v for v in vel)
    return out


def turbulence_spectrum(ncells, seed, kmax=16, slope=-5.0 / 3.0):
    """Complex solenoidal velocity coefficients uhat[3][nz][ny][nx] on the FFT grid.

    |uhat(n)|^2 is proportional to E(|n|) / |n|^2 with E(k) ~ k^slope, on
    1 <= |n| <= kmax; kmax is capped below the Nyquist mode of the grid."""
    if isinstance(ncells, int):
        ncells = (ncells, ncells, ncells)
    nx, ny, nz = ncells
    kcap = min(kmax, (min(ncells) - 1) // 2)
    rng = np.random.default_rng(seed)
    kx = np.fft.fftfreq(nx, 1.0 / nx)[None, None, :]
    ky = np.fft.fftfreq(ny, 1.0 / ny)[None, :, None]
    kz = np.fft.fftfreq(nz, 1.0 / nz)[:, None, None]
    kk = kx * kx + ky * ky + kz * kz
    kn = np.sqrt(kk)
    band = (kn >= 1.0) & (kn <= kcap)
    amp = np.where(band, np.power(np.where(band, kn, 1.0), 0.5 * (slope - 2.0)), 0.0)
    g = rng.standard_normal((3, nz, ny, nx)) + 1j * rng.standard_normal((3, nz, ny, nx))
    g *= amp[None]
    # solenoidal projection of the random vector field: (I - n n^T / |n|^2) g
    kv = [np.broadcast_to(kx, kk.shape), np.broadcast_to(ky, kk.shape), np.broadcast_to(kz, kk.shape)]
    safe = np.where(kk > 0, kk, 1.0)
    dot = (kv[0] * g[0] + kv[1] * g[1] + kv[2] * g[2]) / safe
    for c in range(3):
        g[c] = g[c] - kv[c] * dot
    return g


def turbulence(ncells, nodes, seed=9079, mach=0.3, gamma=5.0 / 3.0, rho0=1.0, p0=1.0, kmax=16,
               device="cpu", dtype=None):
    """Point values [5][n][n][n][nz][ny][nx] of the turbulence surrogate.

    The field is sampled at the Gauss offsets by one phase-shifted inverse FFT
    per offset and component.  Returned as a torch tensor on ``device``."""
    import torch

    if isinstance(ncells, int):
        ncells = (ncells, ncells, ncells)
    nx, ny, nz = ncells
    n = len(nodes)
    dtype = dtype or torch.float64
    cdt = torch.complex128
    uhat = torch.from_numpy(turbulence_spectrum(ncells, seed, kmax)).to(device=device, dtype=cdt)
    kx = torch.fft.fftfreq(nx, 1.0 / nx, dtype=torch.float64, device=device)[None, None, :]
    ky = torch.fft.fftfreq(ny, 1.0 / ny, dtype=torch.float64, device=device)[None, :, None]
    kz = torch.fft.fftfreq(nz, 1.0 / nz, dtype=torch.float64, device=device)[:, None, None]
    # shifts of the Gauss offsets relative to the cell's left edge, in cell widths
    off = [0.5 * (1.0 + float(x)) for x in nodes]
    out = torch.empty((NF, n, n, n, nz, ny, nx), dtype=dtype, device=device)
    scale = float(nx * ny * nz)
    sumsq = 0.0
    vel = torch.empty((3, n, n, n, nz, ny, nx), dtype=torch.float64, device=device)
    for c in range(n):
        pz = torch.exp(2j * math.pi * kz * (off[c] / nz))
        for b in range(n):
            py = torch.exp(2j * math.pi * ky * (off[b] / ny))
            for a in range(n):
                px = torch.exp(2j * math.pi * kx * (off[a] / nx))
                phase = pz * py * px
                for comp in range(3):
                    v = torch.fft.ifftn(uhat[comp] * phase).real * scale
                    vel[comp, c, b, a] = v
    vrms = torch.sqrt((vel * vel).sum(0).mean() / 3.0).item() * math.sqrt(3.0)
    cs = math.sqrt(gamma * p0 / rho0)
    vel *= (mach * cs) / vrms
    out[0] = rho0
    for comp in range(3):
        out[1 + comp] = (rho0 * vel[comp]).to(dtype)
    out[4] = (p0 / (gamma - 1.0) + 0.5 * rho0 * (vel * vel).sum(0)).to(dtype)
    del vel, sumsq
    return out


# ---------------------------------------------------------------- driving

def forcing_modes(kmin=1.0, kmax=3.0):
    """Integer wave vectors with kmin < |n| < kmax, one of each +-n pair (first
    non-zero component positive).  These are the modes whose paraboloid
    amplitude is non-zero; each entry stands for the pair n, -n."""
    out = []
    r = int(math.ceil(kmax))
    for nz in range(-r, r + 1):
        for ny in range(-r, r + 1):
            for nx in range(-r, r + 1):
                v = (nx, ny, nz)
                kk = nx * nx + ny * ny + nz * nz
                if kk == 0:
                    continue
                kn = math.sqrt(kk)
                if not (kmin < kn < kmax):
                    continue
                first = next(c for c in v if c != 0)
                if first < 0:
                    continue
                out.append(v)
    return np.array(out, dtype=np.int32)


def ou_normals(seed, nmodes, nupdates):
    """Standard normal draws [nupdates][nmodes][3][2] for the OU driving process."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nupdates, nmodes, 3, 2))


def ou_stationary_start(seed, nmodes):
    """OU state drawn from its stationary distribution (unit variance)."""
    rng = np.random.default_rng(seed + 7919)
    return rng.standard_normal((nmodes, 3, 2))


# ---------------------------------------------------------------- closure inputs

def xavier_params(shape, seed=4):
    """Xavier-uniform weights, zero biases, packed as W1 b1 W2 b2 W3 b3 (row-major W[out][in])."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in zip(shape[:-1], shape[1:]):
        lim = math.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, size=(fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)


def random_batch(seed, batch, nin, nout):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((batch, nin)), rng.standard_normal((batch, nout))
