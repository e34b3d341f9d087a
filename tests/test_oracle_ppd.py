"""Pins for the FP64 Algorithm 3 oracle and the problem assembly."""
import math

import numpy as np
import pytest

import synth
from oracle import nufft as nf
from oracle import ppd as O
from oracle import problem as P
from oracle import prox, sara


@pytest.fixture(scope="module")
def small():
    """A 32x32 problem with 3 radial blocks, built with a short power iteration."""
    x, wu, wv, off = synth.small_case(32, 3000, seed=11, d=3)
    noise = synth.noise_unit(wu.size, 211)
    pb = P.make_problem(x, wu, wv, off, noise, 30.0, np.ones((32, 32)), power_tol=1e-9)
    return pb


def _params(pb, U, eta, n_itr=1):
    return O.Params(eta=eta, mu=1.0 / U.max(), n_itr=n_itr)


def test_first_iteration_closed_form(small):
    pb = small
    prm = _params(pb, pb.U, pb.eta, n_itr=1)
    st = O.init_state(32, 32, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, st, 1)
    # from zeros: z = P_B((1 - mu U) y) per block, v = -U z, u = 0,
    # x = max(0, tau eta Re Phi^H (U z)), x tilde = 2 x
    z = np.empty_like(pb.y)
    for j in range(len(pb.eps)):
        s = slice(pb.block_off[j], pb.block_off[j + 1])
        z[s] = prox.proj_B((1 - prm.mu * pb.U[s]) * pb.y[s], pb.y[s], pb.eps[j])
    x1 = np.maximum(prm.tau * prm.eta * pb.op.phit(pb.U * z), 0.0)
    assert np.allclose(st.z, z, rtol=1e-13, atol=0)
    assert np.allclose(st.v, -pb.U * z, rtol=1e-13, atol=0)
    assert np.abs(st.u).max() == 0.0
    assert np.abs(st.x - x1).max() <= 1e-13 * np.abs(x1).max()
    assert np.abs(st.xt - 2 * x1).max() <= 1e-13 * np.abs(x1).max()


def _pd_reference(pb, eta, T, lam=1.0):
    """Non-preconditioned PD written independently: vbar = w - P_B(w)."""
    op = pb.op
    ny, nx = pb.x_true.shape
    x = np.zeros((ny, nx)); xt = np.zeros((ny, nx))
    v = np.zeros(pb.y.size, complex); u = np.zeros((9, ny, nx))
    for _ in range(T):
        g = op.phi(xt)
        for j in range(len(pb.eps)):
            s = slice(pb.block_off[j], pb.block_off[j + 1])
            w = v[s] + g[s]
            v[s] = (1 - lam) * v[s] + lam * (w - prox.proj_B(w, pb.y[s], pb.eps[j]))
        u = (1 - lam) * u + lam * np.clip(u + sara.analysis(xt), -1e-4, 1e-4)
        xb = np.maximum(x - 0.49 * (eta * op.phit(v) + sara.synthesis(u)), 0.0)
        xt = 2 * xb - x
        x = (1 - lam) * x + lam * xb
    return x


@pytest.mark.parametrize("lam", [1.0, 0.7])
def test_identity_preconditioner_gives_pd(small, lam):
    pb = small
    U = np.ones_like(pb.U)
    st = O.init_state(32, 32, pb.y)
    prm = _params(pb, U, pb.eta_pd)
    prm.lam = lam
    O.iterate(pb.op, pb.y, U, pb.eps, pb.block_off, prm, st, 8)
    xr = _pd_reference(pb, pb.eta_pd, 8, lam)
    assert np.abs(st.x - xr).max() <= 1e-11 * np.abs(xr).max()


def test_preconditioner_scale_invariance(small):
    pb = small
    a = O.init_state(32, 32, pb.y)
    b = O.init_state(32, 32, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, _params(pb, pb.U, pb.eta, 2), a, 6)
    U2 = 2.0 * pb.U
    O.iterate(pb.op, pb.y, U2, pb.eps, pb.block_off, _params(pb, U2, pb.eta / 2.0, 2), b, 6)
    assert np.array_equal(a.x, b.x)          # power-of-2 scaling: bitwise
    assert np.array_equal(2.0 * a.v, b.v)


def test_resume_is_bitwise(small):
    pb = small
    prm = _params(pb, pb.U, pb.eta, 2)
    a = O.init_state(32, 32, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, a, 6)
    b = O.init_state(32, 32, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, b, 3)
    c = b.copy()
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, c, 3)
    assert np.array_equal(a.x, c.x) and np.array_equal(a.v, c.v) and np.array_equal(a.u, c.u)


def test_ppd_and_pd_converge_on_workload():
    inp = synth.make_inputs(synth.WORKLOADS["ppd64"])
    pb = P.problem_from_inputs(inp, power_tol=1e-8)
    out = {}
    for name, U, eta in [("ppd", pb.U, pb.eta), ("pd", np.ones_like(pb.U), pb.eta_pd)]:
        st = O.init_state(64, 64, pb.y)
        h = O.iterate(pb.op, pb.y, U, pb.eps, pb.block_off, _params(pb, U, eta), st, 150,
                      x_true=pb.x_true)
        out[name] = h
        assert h[-1]["snr"] > 15.0
        assert h[-1]["snr"] > h[9]["snr"]
        assert h[-1]["residual"][0] <= 1.05 * pb.eps[0]
        assert np.all(st.x >= 0)
    # both approach the same solution of the same problem
    assert abs(out["ppd"][-1]["snr"] - out["pd"][-1]["snr"]) < 1.5


def test_uniform_weights_brute_force():
    rng = np.random.default_rng(3)
    M, ny, nx = 500, 8, 16
    wu = rng.uniform(-math.pi, math.pi, M).astype(np.float32)
    wv = (rng.standard_normal(M) * 0.5).clip(-3.14, 3.14).astype(np.float32)
    U = P.uniform_weights(wu, wv, ny, nx)
    cu = [min(nx - 1, int(math.floor((float(a) + math.pi) * nx / (2 * math.pi)))) for a in wu]
    cv = [min(ny - 1, int(math.floor((float(b) + math.pi) * ny / (2 * math.pi)))) for b in wv]
    counts = {}
    for k in zip(cv, cu):
        counts[k] = counts.get(k, 0) + 1
    c = np.array([counts[k] for k in zip(cv, cu)], dtype=float)
    assert np.array_equal(U, c.min() / c)
    assert U.max() == 1.0 and U.min() > 0


def test_power_norm_matches_dense_eigenvalue():
    x, wu, wv, _ = synth.small_case(8, 120, seed=13)
    op = nf.Nufft(wu, wv, 8, 8)
    U = P.uniform_weights(wu, wv, 8, 8)
    A = np.empty((64, 64))
    for k in range(64):
        e = np.zeros(64); e[k] = 1
        A[:, k] = op.phit(U * op.phi(e.reshape(8, 8))).ravel()
    lam = np.linalg.eigvalsh(0.5 * (A + A.T)).max()
    assert P.power_norm(op, U, np.ones((8, 8)), tol=1e-13, max_iter=5000) == pytest.approx(lam, rel=1e-9)


def test_l2_bound_is_chi_square_mean_plus_two_std():
    # ||n_j||^2 / sigma^2 ~ chi^2_{2 M_j} / 2: mean M_j, std sqrt(M_j)
    off = np.array([0, 1000, 5000])
    eps = P.l2_bounds(2.0, off)
    assert eps ** 2 == pytest.approx(4.0 * np.array([1000 + 2 * math.sqrt(1000), 4000 + 2 * math.sqrt(4000)]))
    draws = np.array([np.sum(np.abs(synth.noise_unit(4000, s)) ** 2) for s in range(200)])
    assert abs(draws.mean() - 4000) < 4 * math.sqrt(4000) / math.sqrt(200) * 3
    assert abs(draws.std() - math.sqrt(4000)) < 0.25 * math.sqrt(4000)


def test_input_snr_definition():
    x, wu, wv, off = synth.small_case(16, 2000, seed=21)
    noise = synth.noise_unit(2000, 5)
    pb = P.make_problem(x, wu, wv, off, noise, 20.0, np.ones((16, 16)), with_eta=False)
    y0 = pb.op.phi(x)
    assert pb.sigma ** 2 == pytest.approx(np.mean(np.abs(y0) ** 2) / 100.0, rel=1e-12)
    assert pb.y.dtype == np.complex128
    assert np.array_equal(pb.y, pb.y.astype(np.complex64).astype(np.complex128))


# ---- Algorithm 1 re-weighting (Sec. 3.2) ---------------------------------

def test_reweights_dirac_closed_form():
    """The Dirac basis analyses x to x / 3 under the 1/3-normalised SARA, so
    its re-weights are omega / (omega + |x| / 3) pixel by pixel."""
    rng = np.random.default_rng(71)
    x = rng.standard_normal((32, 32))
    W = O.reweights(x, 0.05)
    assert W.shape == (9, 32, 32)
    assert np.allclose(W[0], 0.05 / (0.05 + np.abs(x) / 3.0), rtol=1e-14, atol=0)
    assert np.all(W > 0) and np.all(W <= 1.0)


def test_reweights_constant_image():
    """An orthonormal periodised DWT maps a constant image c to zero details
    and approximation coefficients c 2^levels (sqrt 2 per axis per level):
    W = 1 at every detail coefficient and omega/(omega + 8c/3) on LL."""
    c, om = 0.7, 0.1
    W = O.reweights(np.full((64, 64), c), om)
    for b in range(1, 9):
        ll = W[b, :8, :8]
        assert np.allclose(ll, om / (om + 8.0 * c / 3.0), rtol=1e-12)
        det = W[b].copy()
        det[:8, :8] = 1.0
        assert np.allclose(det, 1.0, rtol=0, atol=1e-12)


def test_reweights_limits():
    rng = np.random.default_rng(72)
    x = np.abs(rng.standard_normal((32, 32)))
    assert np.array_equal(O.reweights(np.zeros((32, 32)), 1e-3), np.ones((9, 32, 32)))
    assert np.allclose(O.reweights(x, 1e12), 1.0, atol=1e-10)
    small = O.reweights(x, 1e-12)
    assert small.max() <= 1.0 and np.median(small) < 1e-9


def _weighted_problem(seed=73):
    n, M = 32, 1500
    x, wu, wv, off = synth.small_case(n, M, seed=seed, d=2)
    return P.make_problem(x, wu, wv, off, synth.noise_unit(M, seed), 25.0, np.ones((n, n)), power_tol=1e-8)


def test_weighted_iteration_identity_and_zero():
    """W = 1 reproduces the unweighted iteration bit for bit; W = 0 removes
    the sparsity term: u stays at zero and x follows the iteration with
    zeta = 0 exactly."""
    pb = _weighted_problem()
    n = pb.x_true.shape[0]
    prm = O.Params(eta=pb.eta)
    runs = {}
    for key, W, p in [("none", None, prm), ("ones", np.ones((9, n, n)), prm),
                      ("zero", np.zeros((9, n, n)), prm), ("zeta0", None, O.Params(eta=pb.eta, zeta=0.0))]:
        st = O.init_state(n, n, pb.y)
        O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, p, st, 6, W=W)
        runs[key] = st
    assert np.array_equal(runs["ones"].x, runs["none"].x)
    assert np.array_equal(runs["ones"].u, runs["none"].u)
    assert np.array_equal(runs["zero"].x, runs["zeta0"].x)
    assert np.abs(runs["zero"].u).max() == 0.0
    assert np.abs(runs["none"].u).max() > 0.0


def test_snr_db_closed_forms():
    """SNR = 20 log10(||x_true|| / ||x_true - x||) (Sec. 5) on cases with
    exact values: a 10% uniform error is 20 dB, an error as large as the
    image 0 dB, an error ten times the image -20 dB."""
    xt = np.ones((4, 4))
    assert abs(O.snr_db(xt, 0.9 * xt) - 20.0) < 1e-12
    assert abs(O.snr_db(np.array([[3.0, 4.0]]), np.array([[3.0, 4.5]])) - 20.0) < 1e-12
    assert abs(O.snr_db(xt, np.zeros((4, 4)))) < 1e-12
    assert abs(O.snr_db(xt, 2.0 * xt)) < 1e-12
    assert abs(O.snr_db(xt, -9.0 * xt) - (-20.0)) < 1e-12


def test_reweighted_schedule():
    """Algorithm 1 with two re-weightings: solve 0 with W = I; solve k uses
    W = omega_k / (omega_k + |Psi^H x|) from the image x (not x tilde) that
    solve k-1 ended with, omega_k = 0.25^k 1e-2 (Sec. 5.1: 2.5e-3, then
    6.25e-4); every solve warm-starts from the state the previous one left.
    Written out solve by solve and compared bit for bit; the readings a slip
    would produce (weights from x tilde, omega decayed one step late) are
    checked to differ, so the comparison can tell them apart."""
    pb = _weighted_problem(seed=75)
    n = pb.x_true.shape[0]
    prm = O.Params(eta=pb.eta)
    st = O.init_state(n, n, pb.y)
    hists, W = O.reweighted(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, st, 2, 4)
    assert len(hists) == 3 and all(len(h) == 4 for h in hists)
    ref = O.init_state(n, n, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ref, 4)
    W1 = 2.5e-3 / (2.5e-3 + np.abs(sara.analysis(ref.x)))
    W1_slip_xt = 2.5e-3 / (2.5e-3 + np.abs(sara.analysis(ref.xt)))
    W1_slip_omega = 1e-2 / (1e-2 + np.abs(sara.analysis(ref.x)))
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ref, 4, W=W1)
    W2 = 6.25e-4 / (6.25e-4 + np.abs(sara.analysis(ref.x)))
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ref, 4, W=W2)
    assert np.array_equal(W, W2)
    assert np.array_equal(st.x, ref.x) and np.array_equal(st.u, ref.u) and np.array_equal(st.v, ref.v)
    assert not np.allclose(W1, W1_slip_xt) and not np.allclose(W1, W1_slip_omega)


def test_reweighted_outer_loop_improves_snr():
    """Algorithm 1 on the 64x64 workload: each re-weighted solve, warm-started,
    ends at a higher SNR than the unweighted solve of the same total length
    (the effect the re-weighting is introduced for, Sec. 3.2)."""
    w = synth.WORKLOADS["ppd64"]
    pb = P.problem_from_inputs(synth.make_inputs(w), power_tol=1e-8)
    prm = O.Params(eta=pb.eta)
    st = O.init_state(64, 64, pb.y)
    hists, W = O.reweighted(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, st, 2, 150, x_true=pb.x_true)
    ref = O.init_state(64, 64, pb.y)
    h0 = O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, prm, ref, 450, x_true=pb.x_true)
    assert W.shape == (9, 64, 64) and W.max() <= 1.0
    assert hists[-1][-1]["snr"] > h0[-1]["snr"]


# ---- exact prox of eq. elip-proj-1 inside Algorithm 3 ----------------------

def test_exact_prox_with_identity_metric_is_pd():
    """U = I: the exact prox is the Euclidean projection P_B, which Algorithm 2
    also returns after one step from any start (mu = 1), so the exact-prox
    iteration reproduces PD."""
    pb = _weighted_problem(seed=74)
    n = pb.x_true.shape[0]
    U1 = np.ones_like(pb.U)
    a = O.init_state(n, n, pb.y)
    b = O.init_state(n, n, pb.y)
    O.iterate(pb.op, pb.y, U1, pb.eps, pb.block_off, O.Params(eta=pb.eta_pd, prox="exact"), a, 8)
    O.iterate(pb.op, pb.y, U1, pb.eps, pb.block_off, O.Params(eta=pb.eta_pd, n_itr=1), b, 8)
    assert np.allclose(a.x, b.x, rtol=0, atol=1e-11 * np.abs(b.x).max())
    assert np.allclose(a.v, b.v, rtol=0, atol=1e-11 * np.abs(b.v).max())


def test_exact_prox_is_limit_of_algorithm2():
    """With many Algorithm 2 steps per iteration the iterates approach the
    exact-prox iterates (Algorithm 2 converges to prox^U_h)."""
    pb = _weighted_problem(seed=75)
    n = pb.x_true.shape[0]
    a = O.init_state(n, n, pb.y)
    b = O.init_state(n, n, pb.y)
    mu = 1.0 / pb.U.max()
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=pb.eta, mu=mu, prox="exact"), a, 5)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=pb.eta, mu=mu, n_itr=3000), b, 5)
    assert np.linalg.norm(a.x - b.x) <= 1e-6 * np.linalg.norm(a.x)
    assert np.linalg.norm(a.z - b.z) <= 1e-6 * np.linalg.norm(a.z)


# ---- randomised active sets of blocks and bases (Algorithm 3) -------------

def test_all_active_masks_equal_full_iteration():
    pb = _weighted_problem(seed=76)
    n, d = pb.x_true.shape[0], len(pb.eps)
    T = 5
    a = O.init_state(n, n, pb.y)
    b = O.init_state(n, n, pb.y)
    masks = [(np.ones(d, np.uint8), np.ones(9, np.uint8))] * T
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=pb.eta), a, T, active=masks)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=pb.eta), b, T)
    for k in ("x", "xt", "v", "u", "z"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


def test_never_active_basis_equals_zero_weight():
    """A basis that is never active keeps u_i = 0, which is what a zero
    re-weight W_i does through the clip and the synthesis."""
    pb = _weighted_problem(seed=77)
    n, d = pb.x_true.shape[0], len(pb.eps)
    T = 6
    pm = np.ones(9, np.uint8)
    pm[4] = 0
    a = O.init_state(n, n, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=pb.eta), a, T,
              active=[(np.ones(d, np.uint8), pm)] * T)
    W = np.ones((9, n, n))
    W[4] = 0.0
    b = O.init_state(n, n, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, pb.block_off, O.Params(eta=pb.eta), b, T, W=W)
    assert np.array_equal(a.x, b.x)
    assert np.abs(a.u[4]).max() == 0.0


def test_never_active_block_equals_dropping_its_data():
    """A data block that is never active keeps v_j = 0: the run equals the
    one on the problem without that block's visibilities."""
    from oracle import nufft as onf
    pb = _weighted_problem(seed=78)
    n = pb.x_true.shape[0]
    off = pb.block_off
    T = 6
    a = O.init_state(n, n, pb.y)
    O.iterate(pb.op, pb.y, pb.U, pb.eps, off, O.Params(eta=pb.eta), a, T,
              active=[(np.array([1, 0], np.uint8), np.ones(9, np.uint8))] * T)
    keep = slice(int(off[0]), int(off[1]))
    _, wu, wv, _ = synth.small_case(32, 1500, seed=78, d=2)     # the coverage of _weighted_problem
    op0 = onf.Nufft(wu[keep], wv[keep], n, n)
    b = O.init_state(n, n, pb.y[keep])
    O.iterate(op0, pb.y[keep], pb.U[keep], pb.eps[:1], off[:2], O.Params(eta=pb.eta), b, T)
    assert np.allclose(a.x, b.x, rtol=0, atol=1e-12 * np.abs(b.x).max())
    assert np.abs(a.v[int(off[1]):]).max() == 0.0


def test_ggd_acceleration_with_concentrated_sampling():
    """Sec. 5.2: with Gaussian sampling (beta = 2) PPD and PD converge at a
    similar speed; with beta = 0.25 (a dense centre) PPD is about an order of
    magnitude faster.  On these synthetic skies that holds at 50 dB input
    SNR throughout and at 30 dB in the first iterations (later PD catches up
    there).  Read from the oracle trajectories in tests/golden (written by
    make_ggd256.py)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ggd256_snr.json")
    g = json.load(open(path))

    def ratio(name, frac):
        p, d = np.asarray(g[name]["ppd"]["snr_db"]), np.asarray(g[name]["pd"]["snr_db"])
        t = frac * max(p[-1], d[-1])
        first = lambda c: int(np.argmax(c >= t)) + 1 if (c >= t).any() else len(c) + 1
        return first(d) / first(p)

    assert ratio("ggd256_b025_50db", 0.9) >= 5.0
    assert ratio("ggd256_b025", 0.7) >= 3.0
    for frac in (0.7, 0.8, 0.9):
        assert 0.7 <= ratio("ggd256_b2", frac) <= 1.5
