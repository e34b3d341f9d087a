"""FP64 problem assembly for synthetic workloads -- test infrastructure only.

* visibilities y = Phi x_true + n (Sec. 2, discrete inverse problem), with the
  noise power set from the input SNR relative to the noise-free signal power
  (Sec. 5): sigma^2 = ||Phi x_true||^2 / M * 10^(-iSNR/10); y is stored as
  complex64 (the data precision of the GPU path) and used at that precision;
* l2 bounds: eps^2 two standard deviations above the mean of the chi-square
  distribution of ||n||^2 (Sec. 5.1), per block: eps_j^2 = sigma^2 (M_j + 2 sqrt(M_j));
* U: the inverse of the sampling density near each point (Sec. 4.3, 5):
  points counted on an Ny x Nx u-v cell grid, cell floor((w + pi) N / (2 pi))
  clamped to N - 1, U_e = c_min / c_e so that max U = 1;
* eta = 1 / ||U^1/2 Phi||_S^2 (Sec. 5.1) by power iteration on the real
  operator x -> Re Phi^H (U Phi x).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

from .nufft import Nufft


def uniform_weights(wu, wv, ny: int, nx: int) -> np.ndarray:
    """Diagonal of U: inverse local sampling density, normalised to max 1."""
    w_u = np.asarray(wu, dtype=np.float64)
    w_v = np.asarray(wv, dtype=np.float64)
    iu = np.floor((w_u + np.pi) * nx / (2.0 * np.pi)).astype(np.int64)
    iv = np.floor((w_v + np.pi) * ny / (2.0 * np.pi)).astype(np.int64)
    iu = np.clip(iu, 0, nx - 1)
    iv = np.clip(iv, 0, ny - 1)
    cell = iv * nx + iu
    counts = np.bincount(cell, minlength=ny * nx)
    c = counts[cell].astype(np.float64)
    return c.min() / c


def l2_bounds(sigma: float, block_off) -> np.ndarray:
    Mj = np.diff(np.asarray(block_off, dtype=np.float64))
    return sigma * np.sqrt(Mj + 2.0 * np.sqrt(Mj))


def power_norm(op: Nufft, U, x0, tol: float = 1e-10, max_iter: int = 1000):
    """Largest eigenvalue of x -> Re Phi^H (U Phi x), i.e. ||U^1/2 Phi||_S^2."""
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    lam_prev = 0.0
    lam = 0.0
    for k in range(max_iter):
        b = op.phit(U * op.phi(x))
        lam = float(np.linalg.norm(b))
        x = b / lam
        if k > 0 and abs(lam - lam_prev) <= tol * lam:
            break
        lam_prev = lam
    return lam


@dataclasses.dataclass
class Problem:
    op: Nufft
    x_true: np.ndarray
    y: np.ndarray            # complex128 holding complex64 values
    U: np.ndarray
    eps: np.ndarray
    block_off: np.ndarray
    sigma: float
    eta: float
    eta_pd: float            # 1 / ||Phi||^2 (U = 1)


def make_problem(x_true, wu, wv, block_off, noise, isnr_db: float, power_start,
                 theta=None, power_tol: float = 1e-10, power_max_iter: int = 1000,
                 with_eta: bool = True) -> Problem:
    ny, nx = x_true.shape
    op = Nufft(wu, wv, ny, nx, theta=theta)
    y0 = op.phi(x_true)
    M = y0.size
    sigma = math.sqrt(np.sum(np.abs(y0) ** 2) / M * 10.0 ** (-isnr_db / 10.0))
    y = (y0 + sigma * np.asarray(noise)).astype(np.complex64).astype(np.complex128)
    U = uniform_weights(wu, wv, ny, nx)
    eps = l2_bounds(sigma, block_off)
    eta = eta_pd = float("nan")
    if with_eta:
        eta = 1.0 / power_norm(op, U, power_start, power_tol, power_max_iter)
        eta_pd = 1.0 / power_norm(op, np.ones_like(U), power_start, power_tol, power_max_iter)
    return Problem(op, x_true, y, U, eps, np.asarray(block_off), sigma, eta, eta_pd)


def problem_from_inputs(inp, channel: int = 0, **kw) -> Problem:
    w = inp.workload
    return make_problem(inp.x_true, inp.wu[channel], inp.wv[channel], inp.block_off,
                        inp.noise[channel], w.isnr_db, inp.power_start, **kw)
