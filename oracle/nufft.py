"""FP64 measurement operator Phi = Theta G F Z (Sec. 2, eq. of the discrete
inverse problem) -- test infrastructure only, see ``oracle/__init__``.

Conventions (readings of what the paper leaves open):

* image x[r, c], r < Ny along v, c < Nx along u; centred pixel indices
  n_c = c - Nx/2, n_r = r - Ny/2; continuous model (Sec. 2, measurement
  equation, negative exponent):  y_e = theta_e sum x[r,c] exp(-i(wu_e n_c + wv_e n_r));
* oversampled grid Kx = 2 Nx, Ky = 2 Ny (the paper's n = 4 counts grid
  points, i.e. 2x per axis, Sec. 5);
* G: 8x8 Kaiser-Bessel interpolation (Sec. 5, after Fessler & Sutton 2003),
  phi(d) = I0(beta sqrt(1 - (2d/J)^2)) for |d| <= J/2, J = 8, with
  beta = pi sqrt((J/s)^2 (s - 1/2)^2 - 0.8), s = 2 (Beatty, Nishimura & Pauly
  2005); per axis t = K w / (2 pi), taps k = floor(t)-3 .. floor(t)+4, weight
  phi(t - k), grid index k mod K; 2D weight = product of the axis weights;
* Z: zero padding plus division by the continuous Fourier transform of phi,
  phi_hat(xi) = J sinh(sqrt(beta^2 - (pi J xi)^2)) / sqrt(beta^2 - (pi J xi)^2),
  at xi = n / K, the pixel placed at (n_r mod Ky, n_c mod Kx);
* F: unnormalised forward 2D DFT (numpy.fft.fft2); F^H = Kx Ky ifft2;
* the adjoint for a real image is Re(Z^H F^H G^H Theta^H v).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse
import scipy.special

J = 8  # interpolation kernel width per axis (Sec. 5: 8x8 kernels)


def kb_beta(J: int = J, sigma: float = 2.0) -> float:
    """Kaiser-Bessel shape for width J and oversampling sigma (Beatty et al. 2005)."""
    return math.pi * math.sqrt((J / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def kb(d, beta: float, J: int = J) -> np.ndarray:
    """Kaiser-Bessel kernel phi(d), zero outside |d| <= J/2 (Sec. 5, G)."""
    d = np.asarray(d, dtype=np.float64)
    arg = 1.0 - (2.0 * d / J) ** 2
    return np.where(arg >= 0.0, scipy.special.i0(beta * np.sqrt(np.maximum(arg, 0.0))), 0.0)


def kb_ft(xi, beta: float, J: int = J) -> np.ndarray:
    """Continuous Fourier transform of ``kb`` (valid for pi J |xi| < beta)."""
    xi = np.asarray(xi, dtype=np.float64)
    z = np.sqrt(beta * beta - (math.pi * J * xi) ** 2)
    return J * np.sinh(z) / z


def grid_shape(ny: int, nx: int):
    return 2 * ny, 2 * nx


def axis_taps(omega, K: int, beta: float):
    """Per-axis taps of the interpolation G (Sec. 2): returns (cells[M, 8] in
    [0, K), weights[M, 8]) for frequencies omega (radians per pixel)."""
    t = K * np.asarray(omega, dtype=np.float64) / (2.0 * math.pi)
    k = np.floor(t)[:, None] + np.arange(-3, 5, dtype=np.float64)[None, :]
    w = kb(t[:, None] - k, beta)
    return np.mod(k, K).astype(np.int64), w


def build_G(wu, wv, ny: int, nx: int, beta: float) -> scipy.sparse.csr_matrix:
    """Sparse interpolation matrix G (M x Ky*Kx), 64 non-zeros per row (Sec. 2, 5)."""
    Ky, Kx = grid_shape(ny, nx)
    cu, gu = axis_taps(wu, Kx, beta)
    cv, gv = axis_taps(wv, Ky, beta)
    M = cu.shape[0]
    cols = (cv[:, :, None] * Kx + cu[:, None, :]).reshape(M, 64)
    vals = (gv[:, :, None] * gu[:, None, :]).reshape(M, 64)
    rows = np.repeat(np.arange(M, dtype=np.int64), 64)
    return scipy.sparse.csr_matrix((vals.ravel(), (rows, cols.ravel())), shape=(M, Ky * Kx))


def deapod(ny: int, nx: int, beta: float):
    """1D scaling factors 1/phi_hat(n/K) of Z for the centred pixel indices."""
    Ky, Kx = grid_shape(ny, nx)
    nr = np.arange(ny) - ny // 2
    nc = np.arange(nx) - nx // 2
    return 1.0 / kb_ft(nr / Ky, beta), 1.0 / kb_ft(nc / Kx, beta)


class Nufft:
    """Phi = Theta G F Z for one coverage, FP64 (Sec. 2; block rows of Sec. 3.1).

    ``workers`` > 1 (used only to time the oracle on several host cores):
    the sparse products G a and G^T v run as row ranges on a thread pool
    (each output entry is the same dot product as in the single product, so
    the values are identical) and the FFTs are scipy.fft's with that many
    workers (the same transform; rounding may differ in the last bits)."""

    def __init__(self, wu, wv, ny: int, nx: int, theta=None, beta: float | None = None,
                 workers: int | None = None):
        self.ny, self.nx = ny, nx
        self.Ky, self.Kx = grid_shape(ny, nx)
        self.beta = kb_beta() if beta is None else beta
        self.G = build_G(wu, wv, ny, nx, self.beta)
        self.GT = self.G.T.tocsr()
        self.M = self.G.shape[0]
        self.theta = None if theta is None else np.asarray(theta, dtype=np.float64)
        sr, sc = deapod(ny, nx, self.beta)
        self.scale = sr[:, None] * sc[None, :]
        self.rows = np.mod(np.arange(ny) - ny // 2, self.Ky)
        self.cols = np.mod(np.arange(nx) - nx // 2, self.Kx)
        self.workers = workers if workers and workers > 1 else None
        if self.workers:
            from concurrent.futures import ThreadPoolExecutor
            self._pool = ThreadPoolExecutor(self.workers)
            self._Gp = self._row_parts(self.G)
            self._GTp = self._row_parts(self.GT)

    def _row_parts(self, A):
        cuts = np.linspace(0, A.shape[0], self.workers + 1).astype(np.int64)
        return [A[cuts[i]:cuts[i + 1]] for i in range(self.workers)]

    def _matvec(self, A, parts, v):
        if not self.workers:
            return A @ v
        return np.concatenate(list(self._pool.map(lambda B: B @ v, parts)))

    def _fft2(self, g):
        if not self.workers:
            return np.fft.fft2(g)
        import scipy.fft
        return scipy.fft.fft2(g, workers=self.workers)

    def _ifft2(self, g):
        if not self.workers:
            return np.fft.ifft2(g)
        import scipy.fft
        return scipy.fft.ifft2(g, workers=self.workers)

    # Z: oversample and scale
    def Z(self, x):
        g = np.zeros((self.Ky, self.Kx), dtype=np.complex128)
        g[np.ix_(self.rows, self.cols)] = x * self.scale
        return g

    def ZH(self, g):
        return g[np.ix_(self.rows, self.cols)] * self.scale

    def fft_grid(self, x):
        """F Z x: the oversampled spectrum of the scaled image."""
        return self._fft2(self.Z(x))

    def degrid(self, grid):
        """Theta G a for a spectrum a (Ky x Kx)."""
        y = self._matvec(self.G, getattr(self, "_Gp", None), grid.ravel())
        return y if self.theta is None else self.theta * y

    def grid(self, v):
        """G^H Theta^H v onto the oversampled grid."""
        v = np.asarray(v, dtype=np.complex128)
        if self.theta is not None:
            v = self.theta * v
        return self._matvec(self.GT, getattr(self, "_GTp", None), v).reshape(self.Ky, self.Kx)

    def ifft_grid_real(self, g):
        """Re Z^H F^H g with F^H = Kx Ky ifft2."""
        return np.real(self.ZH(self._ifft2(g) * (self.Kx * self.Ky)))

    def phi(self, x):
        return self.degrid(self.fft_grid(x))

    def phit(self, v):
        return self.ifft_grid_real(self.grid(v))


def nudft(x, wu, wv, theta=None):
    """Direct evaluation of the discrete measurement model (brute force)."""
    ny, nx = x.shape
    nr = np.arange(ny) - ny // 2
    nc = np.arange(nx) - nx // 2
    wu = np.asarray(wu, dtype=np.float64)
    wv = np.asarray(wv, dtype=np.float64)
    Eu = np.exp(-1j * np.outer(wu, nc))        # M x nx
    Ev = np.exp(-1j * np.outer(wv, nr))        # M x ny
    y = np.einsum("mr,rc,mc->m", Ev, x.astype(np.complex128), Eu)
    return y if theta is None else np.asarray(theta) * y
