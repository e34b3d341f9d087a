"""Pins for the FP64 measurement operator oracle (Sec. 2, Sec. 5)."""
import math

import numpy as np
import pytest
import scipy.integrate

import synth
from oracle import nufft as nf


def test_kb_beta_value():
    # Beatty et al. (2005) with J = 8, oversampling 2: beta = pi sqrt(35.2)
    assert nf.kb_beta() == pytest.approx(math.pi * math.sqrt(35.2), rel=1e-15)


@pytest.mark.parametrize("xi", [0.0, 0.05, 0.125, 0.2, 0.25])
def test_kb_fourier_transform_by_quadrature(xi):
    beta = nf.kb_beta()
    val, _ = scipy.integrate.quad(lambda d: float(nf.kb(d, beta)) * math.cos(2 * math.pi * xi * d),
                                  -4.0, 4.0, epsabs=0, epsrel=1e-13, limit=200)
    assert float(nf.kb_ft(xi, beta)) == pytest.approx(val, rel=1e-10)


def test_kernel_partition_of_unity():
    # Poisson summation: sum_k phi(t - k) = phi_hat(0) up to the aliased terms
    beta = nf.kb_beta()
    t = np.linspace(-3.0, 3.0, 101) + 0.123
    cells, w = nf.axis_taps(t * 2 * math.pi / 64, 64, beta)
    s = w.sum(axis=1)
    assert np.allclose(s, float(nf.kb_ft(0.0, beta)), rtol=1e-7, atol=0)


def test_taps_window_and_wrap():
    beta = nf.kb_beta()
    K = 32
    om = np.array([-math.pi, 0.0, 1.0, math.pi * (1 - 1e-7)])
    cells, w = nf.axis_taps(om, K, beta)
    t = K * om / (2 * math.pi)
    assert np.all((cells >= 0) & (cells < K))
    # taps k = floor(t)-3 .. floor(t)+4
    assert np.all(cells[:, 3] == np.mod(np.floor(t), K).astype(int))
    # at integer t the d = -4 tap is at the kernel edge, I0(0) = 1
    assert w[1, 7] == pytest.approx(1.0, rel=1e-14)
    assert w[1, 3] == pytest.approx(float(nf.kb(0.0, beta)), rel=1e-14)


@pytest.mark.parametrize("ny,nx,M", [(16, 16, 300), (32, 32, 300), (16, 32, 500), (32, 16, 257)])
def test_phi_matches_direct_nudft(ny, nx, M):
    x, wu, wv, _ = synth.small_case(ny, M, seed=ny + nx + M, nx=nx, coverage="uniform")
    op = nf.Nufft(wu, wv, ny, nx)
    y = op.phi(x)
    yd = nf.nudft(x, wu, wv)
    err = np.linalg.norm(y - yd) / np.linalg.norm(yd)
    assert err < 1e-7, err          # J = 8, 2x oversampling: measured ~3e-8


def test_delta_image_phase_convention():
    ny = nx = 16
    M = 64
    _, wu, wv, _ = synth.small_case(ny, M, seed=5, coverage="uniform")
    op = nf.Nufft(wu, wv, ny, nx)
    r, c = 3, 11
    x = np.zeros((ny, nx))
    x[r, c] = 1.0
    expect = np.exp(-1j * (wu.astype(np.float64) * (c - nx // 2) + wv.astype(np.float64) * (r - ny // 2)))
    assert np.abs(op.phi(x) - expect).max() < 5e-7


def test_centre_pixel_is_real_constant():
    ny = nx = 16
    _, wu, wv, _ = synth.small_case(ny, 50, seed=9, coverage="uniform")
    op = nf.Nufft(wu, wv, ny, nx)
    x = np.zeros((ny, nx))
    x[ny // 2, nx // 2] = 2.5
    assert np.abs(op.phi(x) - 2.5).max() < 5e-7 * 2.5   # per-point NUFFT error bound


@pytest.mark.parametrize("ny,nx", [(16, 16), (32, 64)])
def test_adjoint_dot_product(ny, nx):
    x, wu, wv, _ = synth.small_case(ny, 700, seed=1, nx=nx)
    rng = np.random.default_rng(2)
    theta = rng.uniform(0.5, 2.0, wu.size)
    op = nf.Nufft(wu, wv, ny, nx, theta=theta)
    v = rng.standard_normal(wu.size) + 1j * rng.standard_normal(wu.size)
    xr = rng.standard_normal((ny, nx))
    lhs = np.real(np.vdot(v, op.phi(xr)))
    rhs = float(np.sum(xr * op.phit(v)))
    assert abs(lhs - rhs) / (np.linalg.norm(op.phi(xr)) * np.linalg.norm(v)) < 1e-12


def test_theta_is_diagonal_weighting():
    x, wu, wv, _ = synth.small_case(16, 100, seed=4)
    theta = np.linspace(0.5, 1.5, 100)
    a = nf.Nufft(wu, wv, 16, 16).phi(x)
    b = nf.Nufft(wu, wv, 16, 16, theta=theta).phi(x)
    assert np.allclose(b, theta * a, rtol=1e-14, atol=0)


def test_oversampled_fft_is_unnormalised_dft():
    ny, nx = 8, 8
    x = np.random.default_rng(3).standard_normal((ny, nx))
    _, wu, wv, _ = synth.small_case(ny, 4, seed=3, coverage="uniform")
    op = nf.Nufft(wu, wv, ny, nx)
    a = op.fft_grid(x)
    Zx = op.Z(x)
    Ky, Kx = Zx.shape
    kv, ku = 5, 13
    direct = sum(Zx[i, j] * np.exp(-2j * np.pi * (kv * i / Ky + ku * j / Kx))
                 for i in range(Ky) for j in range(Kx))
    assert abs(a[kv, ku] - direct) < 1e-12 * np.abs(Zx).sum()


def test_G_has_64_nonzeros_per_row():
    _, wu, wv, _ = synth.small_case(32, 200, seed=6)
    G = nf.build_G(wu, wv, 32, 32, nf.kb_beta())
    assert np.all(np.diff(G.indptr) == 64)
    assert np.all(G.data > 0)


def test_threaded_operator_matches_single_threaded():
    """The oracle's multi-core option (used only to time it): row ranges of
    the sparse products give the same values bit for bit; scipy.fft's
    transforms agree with numpy's to rounding."""
    x, wu, wv, off = synth.small_case(32, 3000, seed=5)
    a = nf.Nufft(wu, wv, 32, 32)
    b = nf.Nufft(wu, wv, 32, 32, workers=4)
    g = a.fft_grid(x)
    assert np.array_equal(a.degrid(g), b.degrid(g))
    v = a.degrid(g)
    assert np.array_equal(a.grid(v), b.grid(v))
    assert np.abs(b.fft_grid(x) - g).max() <= 1e-13 * np.abs(g).max()
    assert np.abs(b.phit(v) - a.phit(v)).max() <= 1e-13 * np.abs(a.phit(v)).max()
