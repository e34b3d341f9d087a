"""FP64 SARA sparsity dictionary (Sec. 5.1: a Dirac basis concatenated with
the first eight Daubechies wavelet bases) -- test infrastructure only.

Readings of what the paper leaves open:

* Psi = (1/3) [Psi_0 .. Psi_8], Psi_0 = I, Psi_p the orthonormal periodised
  2D DWT with the Daubechies-p filter (length 2p); the 1/sqrt(9) factor makes
  Psi Psi^H = I so that ||Psi||_S = 1 and zeta = 1 (Sec. 5.1 parameter choice);
* L decomposition levels (3 for every workload here);
* filters by spectral factorisation (Daubechies 1988): |m0|^2 =
  cos^{2p}(w/2) P(sin^2(w/2)), P(y) = sum_{k<p} C(p-1+k, k) y^k, minimum-phase
  root choice, normalised to sum sqrt(2); high-pass g_n = (-1)^n h_{2p-1-n};
* 1D analysis a[k] = sum_n h[n] s[(2k+n) mod L] (periodisation), synthesis is
  its transpose;
* 2D: filter along columns (axis 0), then rows (axis 1), recurse on the
  low-low band; coefficients in the Mallat pyramid layout of the image size:
  [LL | lo-col/hi-row ; hi-col/lo-row | HH] at each level.
"""
from __future__ import annotations

import math

import numpy as np

N_BASES = 9  # Dirac + db1..db8


def daubechies_lowpass(p: int) -> np.ndarray:
    """Minimum-phase Daubechies-p scaling filter h[0..2p-1], sum = sqrt(2)."""
    # roots of P(y), polished by Newton steps, then mapped through
    # y = (2 - z - 1/z)/4, i.e. z + 1/z = 2 - 4y, keeping the root |z| < 1
    coef = np.array([math.comb(p - 1 + k, k) for k in range(p)], dtype=np.float64)
    P = np.polynomial.Polynomial(coef)
    dP = P.deriv()
    yroots = P.roots().astype(np.complex128) if p > 1 else np.array([], dtype=np.complex128)
    for _ in range(5):
        yroots = yroots - P(yroots) / dP(yroots)
    inside = []
    for yr in yroots:
        b = 1.0 - 2.0 * yr                                # z + 1/z = 2b
        z1 = b + np.sqrt(b * b - 1.0)
        z2 = b - np.sqrt(b * b - 1.0)
        inside.append(z1 if abs(z1) < 1.0 else z2)
    h = np.array([1.0 + 0j])
    for _ in range(p):
        h = np.convolve(h, [1.0, 1.0])                   # (1 + z^-1)^p
    for r in inside:
        h = np.convolve(h, [1.0, -r])                    # (1 - r z^-1)
    h = np.real(h)
    return h * (math.sqrt(2.0) / h.sum())


def highpass(h: np.ndarray) -> np.ndarray:
    L = h.size
    return np.array([(-1) ** n * h[L - 1 - n] for n in range(L)])


def _analysis_1d(s: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    """Periodised one-level analysis along ``axis``: (approx, detail)."""
    s = np.moveaxis(s, axis, 0)
    L = s.shape[0]
    k = np.arange(L // 2)
    a = np.zeros((L // 2,) + s.shape[1:])
    d = np.zeros((L // 2,) + s.shape[1:])
    for n in range(h.size):
        idx = (2 * k + n) % L
        a += h[n] * s[idx]
        d += g[n] * s[idx]
    return np.moveaxis(a, 0, axis), np.moveaxis(d, 0, axis)


def _synthesis_1d(a: np.ndarray, d: np.ndarray, h: np.ndarray, g: np.ndarray, axis: int):
    """Transpose of ``_analysis_1d``."""
    a = np.moveaxis(a, axis, 0)
    d = np.moveaxis(d, axis, 0)
    L = 2 * a.shape[0]
    k = np.arange(L // 2)
    s = np.zeros((L,) + a.shape[1:])
    for n in range(h.size):
        idx = (2 * k + n) % L
        np.add.at(s, idx, h[n] * a + g[n] * d)
    return np.moveaxis(s, 0, axis)


def dwt2(x: np.ndarray, p: int, levels: int) -> np.ndarray:
    """Orthonormal periodised 2D DWT, Mallat layout, same shape as x."""
    h = daubechies_lowpass(p)
    g = highpass(h)
    c = np.array(x, dtype=np.float64, copy=True)
    hh, ww = c.shape
    for _ in range(levels):
        s = c[:hh, :ww]
        A, D = _analysis_1d(s, h, g, axis=0)
        LL, LH = _analysis_1d(A, h, g, axis=1)
        HL, HH = _analysis_1d(D, h, g, axis=1)
        c[: hh // 2, : ww // 2] = LL
        c[: hh // 2, ww // 2: ww] = LH
        c[hh // 2: hh, : ww // 2] = HL
        c[hh // 2: hh, ww // 2: ww] = HH
        hh, ww = hh // 2, ww // 2
    return c


def idwt2(c: np.ndarray, p: int, levels: int) -> np.ndarray:
    """Inverse (= transpose) of ``dwt2``."""
    h = daubechies_lowpass(p)
    g = highpass(h)
    x = np.array(c, dtype=np.float64, copy=True)
    H, W = x.shape
    for lev in reversed(range(levels)):
        hh, ww = H >> lev, W >> lev
        LL = x[: hh // 2, : ww // 2]
        LH = x[: hh // 2, ww // 2: ww]
        HL = x[hh // 2: hh, : ww // 2]
        HH = x[hh // 2: hh, ww // 2: ww]
        A = _synthesis_1d(LL, LH, h, g, axis=1)
        D = _synthesis_1d(HL, HH, h, g, axis=1)
        x[:hh, :ww] = _synthesis_1d(A, D, h, g, axis=0)
    return x


def analysis(x: np.ndarray, levels: int = 3) -> np.ndarray:
    """Psi^H x: (9, Ny, Nx) coefficients [x, dwt_1 x, .., dwt_8 x] / 3."""
    out = np.empty((N_BASES,) + x.shape)
    out[0] = x
    for p in range(1, N_BASES):
        out[p] = dwt2(x, p, levels)
    return out / 3.0


def synthesis(u: np.ndarray, levels: int = 3) -> np.ndarray:
    """Psi u = (u_0 + sum_p idwt_p u_p) / 3 for u of shape (9, Ny, Nx)."""
    x = np.array(u[0], dtype=np.float64, copy=True)
    for p in range(1, N_BASES):
        x += idwt2(u[p], p, levels)
    return x / 3.0
