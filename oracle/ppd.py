"""FP64 Algorithm 3 (preconditioned forward-backward primal-dual, PPD) --
test infrastructure only.

No randomisation (the paper's simulations update every block and basis each
iteration, Sec. 5.1), so the active sets are all data blocks and all bases.
With U = 1, mu = 1 and one sub-iteration the data dual step is the Euclidean
l2-ball step of the non-preconditioned PD algorithm.

Reading of the data-dual update (whose printed form mixes dual and data scales):
  w_j   = U_j^{-1} v_j + Theta_j G_j M_j a
  vbar_j = U_j (w_j - prox^{U_j}_{h_j}(w_j)),
the generalised Moreau decomposition (Sec. 4.1) with alpha = 1, where the
proximity operator is approximated by ``n_itr`` iterations of Algorithm 2
warm-started from the block's previous iterate (which starts at y_j).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import prox, sara


@dataclasses.dataclass
class State:
    """Primal and dual variables of Algorithm 3 plus the Algorithm 2 iterate."""
    x: np.ndarray        # (Ny, Nx) primal image
    xt: np.ndarray       # (Ny, Nx) x tilde
    v: np.ndarray        # (M,) complex data duals
    u: np.ndarray        # (9, Ny, Nx) sparsity duals
    z: np.ndarray        # (M,) complex Algorithm 2 iterate (warm start)
    it: int = 0

    def copy(self):
        return State(self.x.copy(), self.xt.copy(), self.v.copy(), self.u.copy(),
                     self.z.copy(), self.it)


def init_state(ny: int, nx: int, y: np.ndarray) -> State:
    """Zeros for x, x tilde, u, v; the Algorithm 2 iterate starts at y."""
    M = y.size
    return State(np.zeros((ny, nx)), np.zeros((ny, nx)), np.zeros(M, np.complex128),
                 np.zeros((sara.N_BASES, ny, nx)), np.asarray(y, np.complex128).copy(), 0)


def snr_db(x_true: np.ndarray, x: np.ndarray) -> float:
    """SNR = 20 log10(||x_true|| / ||x_true - x||) (Sec. 5)."""
    return 20.0 * np.log10(np.linalg.norm(x_true) / np.linalg.norm(x_true - x))


@dataclasses.dataclass
class Params:
    tau: float = 0.49       # Sec. 5.1
    eta: float = 1.0        # 1 / ||U^1/2 Phi||_S^2
    zeta: float = 1.0       # 1 / ||Psi W||_S^2 = 1 with the 1/3-normalised SARA
    lam: float = 1.0        # relaxation (Sec. 5.1)
    alpha: float = 1e-4     # kappa ||Psi W||_S^2 with kappa = 1e-4 (Sec. 5.1)
    mu: float = 1.0         # Algorithm 2 step, 1 / max(U)
    n_itr: int = 1          # Algorithm 2 iterations per outer iteration
    levels: int = 3
    prox: str = "fb"        # "fb": Algorithm 2 (n_itr steps); "exact": prox^U_h itself


def iterate(op, y, U, eps, block_off, params: Params, state: State, T: int,
            x_true: Optional[np.ndarray] = None, W: Optional[np.ndarray] = None,
            trace: Optional[list] = None, active=None):
    """Run T iterations of Algorithm 3 in place on ``state``.

    op: ``oracle.nufft.Nufft``; y, U: (M,) data and preconditioner; eps: (d,)
    l2 bounds; block_off: (d+1,) contiguous block offsets; W: optional (9, Ny,
    Nx) re-weights (identity when None).  Returns a list of per-iteration
    records: SNR when x_true is given, the relative change
    ||x_t - x_{t-1}|| / ||x_t||, ||x_t||, and the block residuals
    ||Phi_j x~ - y_j|| at the x~ the iteration started from.
    If ``trace`` is a list, each iteration appends what decides its active
    sets -- the clip margins |u + Psi^H x~| - alpha, the arguments of P_C and
    which Algorithm 2 steps project -- i.e. the pieces on which the iteration
    is smooth.
    ``active`` (randomised Algorithm 3): None (every block and basis each
    iteration) or a sequence of T pairs (block_mask (d,), basis_mask (9,)):
    an inactive block keeps v_j (and its Algorithm 2 iterate), an inactive
    basis keeps u_i; the random draws are inputs."""
    p = params
    y = np.asarray(y, np.complex128)
    U = np.asarray(U, np.float64)
    hist = []
    for t in range(T):
        bmask, pmask = (None, None) if active is None else active[t]
        a = op.fft_grid(state.xt)                          # a = F Z x tilde
        Ga = op.degrid(a)                                  # Theta_j G_j M_j a, all j
        v_new = state.v.copy()
        z_new = state.z.copy()
        res = []
        sets_proj = []
        for j in range(len(block_off) - 1):                # every data block
            s = slice(int(block_off[j]), int(block_off[j + 1]))
            res.append(np.linalg.norm(Ga[s] - y[s]))
            if bmask is not None and not bmask[j]:         # inactive: v_j, z_j kept
                sets_proj.append(())
                continue
            w = state.v[s] / U[s] + Ga[s]
            if p.prox == "exact":                          # eq. elip-proj-1 solved exactly
                z = prox.prox_metric_exact(w, y[s], eps[j], U[s])
            else:
                z = prox.fb_ellipsoid(w, y[s], eps[j], U[s], p.mu, p.n_itr, state.z[s])
            if trace is not None and p.prox == "exact":
                sets_proj.append((bool(np.linalg.norm(w - y[s]) > eps[j]),))
            elif trace is not None:
                zz, proj = state.z[s], []
                for _ in range(p.n_itr):
                    q = zz - p.mu * U[s] * (zz - w)
                    proj.append(bool(np.linalg.norm(q - y[s]) > eps[j]))
                    zz = prox.proj_B(q, y[s], eps[j])
                sets_proj.append(tuple(proj))
            vbar = U[s] * (w - z)                          # generalised Moreau identity
            v_new[s] = state.v[s] + p.lam * (vbar - state.v[s])   # relaxation
            z_new[s] = z
        vt = op.grid(v_new)                                # G^H Theta^H v, summed over j
        coef = sara.analysis(state.xt, p.levels)           # Psi_i^H x tilde
        if W is not None:
            coef = W * coef
        ubar = prox.clip_dual(state.u + coef, p.alpha)     # (I - S_alpha)
        u_new = state.u + p.lam * (ubar - state.u)         # relaxation
        if pmask is not None:                              # inactive bases: u_i kept
            keep = ~np.asarray(pmask, dtype=bool)
            u_new[keep] = state.u[keep]
        ut = sara.synthesis(u_new if W is None else W * u_new, p.levels)  # Psi W u, summed
        arg = state.x - p.tau * (p.eta * op.ifft_grid_real(vt) + p.zeta * ut)
        xbar = prox.proj_C(arg)                            # P_C of the primal step
        if trace is not None:
            trace.append({"clip": np.abs(state.u + coef) - p.alpha, "pos": arg,
                          "proj": tuple(sets_proj)})
        x_prev = state.x
        x_new = x_prev + p.lam * (xbar - x_prev)           # relaxation
        xt_new = 2.0 * xbar - x_prev                       # x tilde
        state.x, state.xt, state.v, state.u, state.z = x_new, xt_new, v_new, u_new, z_new
        state.it += 1
        x_norm = float(np.linalg.norm(x_new))
        rec = {"it": state.it,
               "rel_change": float(np.linalg.norm(x_new - x_prev) / max(x_norm, 1e-300)),
               "x_norm": x_norm,
               "residual": res}
        if x_true is not None:
            rec["snr"] = float(snr_db(x_true, x_new))
        hist.append(rec)
    return hist


def reweights(x: np.ndarray, omega: float, levels: int = 3) -> np.ndarray:
    """Re-weights of Sec. 3.2 (eq. reweighting): omega / (omega + |Psi_i^H x|)."""
    return omega / (omega + np.abs(sara.analysis(x, levels)))


def reweighted(op, y, U, eps, block_off, params: Params, state: State, n_reweights: int,
               iters_per_solve: int, omega0: float = 1e-2, decay: float = 0.25,
               x_true: Optional[np.ndarray] = None):
    """Algorithm 1: Algorithm 3 solves warm-started from the previous state;
    after solve k the weight parameter becomes omega^(k) = decay^k omega0 and
    the weights are recomputed from the latest image (the reading of the
    index of x in the re-weighting equation).  The first solve uses W = I.
    Returns the per-solve histories and the last weights."""
    W = None
    omega = omega0
    hists = []
    for k in range(n_reweights + 1):
        hists.append(iterate(op, y, U, eps, block_off, params, state, iters_per_solve, x_true=x_true, W=W))
        if k < n_reweights:
            omega *= decay
            W = reweights(state.x, omega, params.levels)
    return hists, W
