"""Pins for the proximity operators and Algorithm 2 (Sec. 3.3, Sec. 4.1)."""
import numpy as np
import pytest

from oracle import prox


def test_proj_C_cases():
    z = np.array([2.0 + 3j, -1.0 + 5j, 0.0 - 1j, 1e-300 + 0j])
    assert np.array_equal(prox.proj_C(z), [2.0, 0.0, 0.0, 1e-300])
    assert np.array_equal(prox.proj_C(np.array([-0.0, 0.5])), [0.0, 0.5])


def test_soft_threshold_cases():
    a = 0.5
    z = np.array([0.0, 0.25, -0.5, 0.5, 2.0, -3.0])
    assert np.allclose(prox.soft(z, a), [0.0, 0.0, 0.0, 0.0, 1.5, -2.5], atol=0)
    zc = np.array([3 + 4j, 0j, 0.3 + 0.4j])
    assert np.allclose(prox.soft(zc, 1.0), [(3 + 4j) * 4 / 5, 0, 0], atol=1e-16)
    # (I - S_a) is the clip to [-a, a] for real inputs
    assert np.allclose(prox.clip_dual(z, a), np.clip(z, -a, a), atol=0)


def test_proj_B_cases():
    y = np.array([1.0 + 1j, -2.0 + 0j])
    z_in = y + np.array([0.1, 0.1j])
    assert np.array_equal(prox.proj_B(z_in, y, 1.0), z_in)           # inside: unchanged
    z_out = y + np.array([3.0, 4.0j])                                 # ||z - y|| = 5
    assert np.allclose(prox.proj_B(z_out, y, 1.0), y + np.array([0.6, 0.8j]), atol=1e-15)
    z_b = y + np.array([0.6, 0.8j])                                   # on the boundary
    assert np.allclose(prox.proj_B(z_b, y, 1.0), z_b, atol=1e-15)
    assert np.array_equal(prox.proj_B(y, y, 0.5), y)                  # q = y


def _rand_block(M, seed, eps_frac=0.5):
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    w = y + rng.standard_normal(M) + 1j * rng.standard_normal(M)
    U = rng.uniform(0.05, 1.0, M)
    U[rng.integers(M)] = 1.0
    eps = eps_frac * np.linalg.norm(w - y)
    return w, y, U, eps


def test_alg2_identity_metric_is_l2_projection():
    w, y, U, eps = _rand_block(200, 1)
    start = np.random.default_rng(9).standard_normal(200) + 0j
    z = prox.fb_ellipsoid(w, y, eps, np.ones(200), 1.0, 1, start)
    assert np.abs(z - prox.proj_B(w, y, eps)).max() < 1e-15 * np.abs(w).max() * 10


@pytest.mark.parametrize("seed", [2, 3, 4])
def test_alg2_converges_to_exact_metric_prox(seed):
    w, y, U, eps = _rand_block(300, seed)
    exact = prox.prox_metric_exact(w, y, eps, U)
    z = prox.fb_ellipsoid(w, y, eps, U, 1.0 / U.max(), 20000, y)
    assert np.linalg.norm(z - exact) / np.linalg.norm(exact) < 1e-8


def test_exact_metric_prox_is_minimiser():
    w, y, U, eps = _rand_block(50, 5)
    z = prox.prox_metric_exact(w, y, eps, U)
    f = lambda q: 0.5 * np.sum(U * np.abs(w - q) ** 2)
    assert np.linalg.norm(z - y) == pytest.approx(eps, rel=1e-12)
    rng = np.random.default_rng(6)
    for _ in range(200):                 # random feasible points never do better
        d = rng.standard_normal(50) + 1j * rng.standard_normal(50)
        q = y + (z - y + 0.05 * d)
        q = prox.proj_B(q, y, eps)
        assert f(q) >= f(z) * (1 - 1e-12)
    # feasible w is returned unchanged
    assert np.array_equal(prox.prox_metric_exact(w, y, 10 * eps, U), w)


@pytest.mark.parametrize("n_itr", [1, 2, 5, 50])
def test_alg2_iterates_stay_feasible(n_itr):
    w, y, U, eps = _rand_block(100, 7)
    z = prox.fb_ellipsoid(w, y, eps, U, 1.0, n_itr, y)
    assert np.linalg.norm(z - y) <= eps * (1 + 1e-12)


def test_alg2_reduces_to_closed_form_for_scalar_metric():
    # U = c I: prox^U_h is the Euclidean projection for any c > 0
    w, y, _, eps = _rand_block(100, 8)
    U = np.full(100, 0.25)
    z = prox.fb_ellipsoid(w, y, eps, U, 4.0, 1, np.zeros(100, complex))
    assert np.allclose(z, prox.proj_B(w, y, eps), atol=1e-14)
