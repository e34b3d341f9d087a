"""FP64 proximity operators (Sec. 3.3) and the metric-U proximity operator of
the data-fidelity term (Sec. 4.1) -- test infrastructure only.
"""
from __future__ import annotations

import numpy as np


def proj_C(z):
    """Projection onto the positive real orthant (Sec. 3.3, eq. proj-plus):
    Re z where Re z > 0, else 0."""
    r = np.real(np.asarray(z))
    return np.where(r > 0.0, r, 0.0)


def soft(z, alpha: float):
    """Soft-thresholding S_alpha (Sec. 3.3, eq. prox-L1):
    z (|z| - alpha)_+ / |z| for |z| > 0, and 0 for |z| = 0."""
    z = np.asarray(z)
    mag = np.abs(z)
    safe = np.where(mag > 0.0, mag, 1.0)
    return np.where(mag > 0.0, z * np.maximum(mag - alpha, 0.0) / safe, 0.0 * z)


def clip_dual(z, alpha: float):
    """(I - S_alpha)(z), the clip of the l1 dual update of Algorithm 3."""
    z = np.asarray(z)
    return z - soft(z, alpha)


def proj_B(z, y, eps: float):
    """Projection onto the l2 ball {||z - y|| <= eps} (Sec. 3.3, eq. proj-L2)."""
    r = np.linalg.norm(z - y)
    if r > eps:
        return eps * (z - y) / r + y
    return np.array(z, copy=True)


def fb_ellipsoid(w, y, eps: float, U, mu: float, n_itr: int, z0):
    """Algorithm 2: forward-backward iterations for prox^U_h(w), h the
    indicator of the l2 ball around y (Sec. 4.1, eq. elip-proj-1):
    z <- P_B(z - mu U (z - w)), n_itr times from the start z0."""
    z = np.array(z0, dtype=np.complex128, copy=True)
    for _ in range(n_itr):
        z = proj_B(z - mu * U * (z - w), y, eps)
    return z


def prox_metric_exact(w, y, eps: float, U, tol: float = 1e-15):
    """Exact argmin_{||z - y|| <= eps} (w - z)^H U (w - z) / 2 for diagonal U > 0.

    KKT: U (z - w) + nu (z - y) = 0, so z(nu) = (U w + nu y) / (U + nu) and
    ||z(nu) - y|| = ||U (w - y) / (U + nu)|| decreases in nu >= 0; nu = 0 when
    w is feasible, otherwise the root of ||z(nu) - y|| = eps is bracketed in
    [0, max(U) ||w - y|| / eps] and found by bisection."""
    w = np.asarray(w, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    U = np.asarray(U, dtype=np.float64)
    r = np.abs(w - y)
    if np.linalg.norm(w - y) <= eps:
        return w.copy()

    def dist(nu):
        return np.sqrt(np.sum((U * r / (U + nu)) ** 2))

    lo, hi = 0.0, float(U.max() * np.linalg.norm(w - y) / eps)
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if dist(mid) > eps:
            lo = mid
        else:
            hi = mid
        if hi - lo <= tol * max(hi, 1e-300):
            break
    nu = hi
    return (U * w + nu * y) / (U + nu)
