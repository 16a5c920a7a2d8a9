"""FP64 oracle of the turbulence diagnostics (arXiv 1602.09079, Sec. 3.3, 4.1, 4.4).

TEST INFRASTRUCTURE ONLY (like the rest of this package): only the tests, the
smoke check and the benchmark's CPU-baseline leg may use it.

Readings (the paper states the ideas, not every convention):
* Sub-cell sampling (Sec. 4, the slices and the PDFs): each cell is split into
  S equal parts per axis (S = 4 in the paper) and the DG polynomial is
  evaluated at the part centres xi_j = -1 + (2j+1)/S.  The M = S n points per
  axis form a uniform grid, point X at x = (X + 1/2) L / M.  Velocity v = m/rho
  at each point.
* Power spectrum (Sec. 3.3): w_hat(n) = sum_X w_X exp(-2 pi i n.X / M) over
  the grid, n the integer wave vector (FFT frequencies, |n_a| <= M/2); the
  shell of n is the integer nearest to |n|; the shell power
  P(s) = sum_{n in shell s} |w_hat(n)|^2 / M^6, summed over the three velocity
  components, so that sum_s P(s) is the grid mean of |v|^2 (the paper's
  normalisation: the integral of the spectrum is the total).  E(k_s) =
  P(s) L / (2 pi) at k_s = 2 pi s / L.
* Density PDF (Sec. 4.4): histogram of log10(rho) over the sampled points in
  nbins equal bins of [lo, hi); bin 0 counts points below lo (and rho <= 0 or
  non-finite), bin nbins + 1 points at or above hi.
* rms Mach number (Sec. 4.1): sqrt of the grid mean of |v|^2 / c^2 with the
  local sound speed c^2 = gamma p / rho at each sampled point.
"""
import numpy as np

from . import NF, basis, nmodes


def sub_points(S):
    """Centres of the S equal parts of [-1, 1]."""
    return -1.0 + (2.0 * np.arange(S) + 1.0) / S


def _table(k, S):
    """phi_l at the S^3 sub-points, point index (c S + b) S + a (a along x)."""
    xs = sub_points(S)
    T = np.zeros((S, S, S, nmodes(k)))
    for c in range(S):
        for b in range(S):
            for a in range(S):
                T[c, b, a] = basis(k, np.array([xs[a], xs[b], xs[c]]))
    return T


def sample(cfg, y, S=4):
    """Point values of the five conserved fields on the M^3 sub-cell grid:
    returns [5][Mz][My][Mx] (oracle state layout [i][l][z][y][x] in)."""
    k = cfg.k
    nx, ny, nz = cfg.n[0], cfg.n[1], cfg.n[2]
    T = _table(k, S)
    y = np.asarray(y, dtype=np.float64).reshape(NF, nmodes(k), nz, ny, nx)
    # q[i][z][y][x][c][b][a] = sum_l y[i][l][z][y][x] T[c][b][a][l]
    q = np.einsum("ilzyx,cbal->izcybxa", y, T)
    return q.reshape(NF, nz * S, ny * S, nx * S)


def velocity_grid(cfg, y, S=4):
    q = sample(cfg, y, S)
    return q[0], q[1:4] / q[0]


def shell_power(w, nbins):
    """Shell powers P(s), s < nbins, of one real grid w[M][M][M] (see the module notes)."""
    M = w.shape[0]
    assert w.shape == (M, M, M)
    wh = np.fft.fftn(w)
    f = np.fft.fftfreq(M, d=1.0 / M)  # integer frequencies
    n2 = f[:, None, None] ** 2 + f[None, :, None] ** 2 + f[None, None, :] ** 2
    s = np.floor(np.sqrt(n2) + 0.5).astype(np.int64)
    p = np.abs(wh) ** 2 / float(M) ** 6
    out = np.zeros(nbins)
    keep = s < nbins
    np.add.at(out, s[keep], p[keep])
    return out


def velocity_spectrum(cfg, y, S=4, nbins=None):
    """P(s) summed over the velocity components."""
    _, v = velocity_grid(cfg, y, S)
    M = v.shape[1]
    if nbins is None:
        nbins = M
    return sum(shell_power(v[i], nbins) for i in range(3))


def density_pdf(cfg, y, S, lo, hi, nbins):
    """Counts of log10(rho) per bin; [0] below lo (or rho <= 0, non-finite), [nbins+1] >= hi."""
    rho = sample(cfg, y, S)[0].ravel()
    counts = np.zeros(nbins + 2, dtype=np.int64)
    for r in rho:
        if not (r > 0.0) or not np.isfinite(r):
            counts[0] += 1
            continue
        x = np.log10(r)
        if x < lo:
            counts[0] += 1
        elif x >= hi:
            counts[nbins + 1] += 1
        else:
            b = int(np.floor((x - lo) / (hi - lo) * nbins))
            counts[1 + min(b, nbins - 1)] += 1
    return counts


def rms_mach(cfg, y, S=4):
    q = sample(cfg, y, S)
    rho = q[0]
    v2 = (q[1] ** 2 + q[2] ** 2 + q[3] ** 2) / rho ** 2
    p = (cfg.gamma - 1.0) * (q[4] - 0.5 * rho * v2)
    c2 = cfg.gamma * p / rho
    return float(np.sqrt(np.mean(v2 / c2)))
