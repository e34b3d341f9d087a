"""Pins for the FP64 SARA oracle (Sec. 5.1: Dirac + Daubechies 1..8)."""
import math

import numpy as np
import pytest

from oracle import sara


def test_db1_is_haar():
    h = sara.daubechies_lowpass(1)
    assert np.allclose(h, [1 / math.sqrt(2), 1 / math.sqrt(2)], atol=1e-16)


def test_db2_closed_form():
    s3 = math.sqrt(3.0)
    expect = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * math.sqrt(2))
    assert np.allclose(sara.daubechies_lowpass(2), expect, atol=1e-15)


def test_db3_closed_form():
    r10 = math.sqrt(10.0)
    q = math.sqrt(5 + 2 * r10)
    expect = np.array([1 + r10 + q, 5 + r10 + 3 * q, 10 - 2 * r10 + 2 * q,
                       10 - 2 * r10 - 2 * q, 5 + r10 - 3 * q, 1 + r10 - q]) / (16 * math.sqrt(2))
    assert np.allclose(sara.daubechies_lowpass(3), expect, atol=1e-14)


@pytest.mark.parametrize("p", range(1, 9))
def test_filter_identities(p):
    h = sara.daubechies_lowpass(p)
    g = sara.highpass(h)
    assert h.size == 2 * p
    assert h.sum() == pytest.approx(math.sqrt(2.0), abs=1e-14)
    for m in range(p):                          # double-shift orthonormality
        assert np.dot(h[: h.size - 2 * m], h[2 * m:]) == pytest.approx(float(m == 0), abs=1e-14)
    n = np.arange(2 * p) / (2.0 * p)
    for q in range(p):                          # p vanishing moments
        assert abs(np.dot(n ** q, g)) < 1e-13
    # minimum phase: energy front-loaded relative to the reversed filter
    assert np.cumsum(h ** 2)[p - 1] >= np.cumsum(h[::-1] ** 2)[p - 1] - 1e-15


def test_haar_one_level_closed_form():
    x = np.random.default_rng(0).standard_normal((4, 6))
    c = sara.dwt2(x, 1, 1)
    a, b, cc, d = x[0::2, 0::2], x[0::2, 1::2], x[1::2, 0::2], x[1::2, 1::2]
    assert np.allclose(c[:2, :3], (a + b + cc + d) / 2, atol=1e-15)      # LL
    assert np.allclose(c[:2, 3:], (a - b + cc - d) / 2, atol=1e-15)      # lo-col, hi-row
    assert np.allclose(c[2:, :3], (a + b - cc - d) / 2, atol=1e-15)      # hi-col, lo-row
    assert np.allclose(c[2:, 3:], (a - b - cc + d) / 2, atol=1e-15)      # HH


@pytest.mark.parametrize("p", range(1, 9))
@pytest.mark.parametrize("shape,levels", [((64, 64), 3), ((16, 32), 3), ((8, 8), 3), ((32, 16), 1)])
def test_dwt_orthonormal(p, shape, levels):
    rng = np.random.default_rng(p)
    x = rng.standard_normal(shape)
    c = sara.dwt2(x, p, levels)
    assert np.linalg.norm(c) == pytest.approx(np.linalg.norm(x), rel=1e-13)
    assert np.abs(sara.idwt2(c, p, levels) - x).max() < 1e-12 * np.abs(x).max()
    # idwt2 is the transpose of dwt2 (independent of the inverse property)
    e = rng.standard_normal(shape)
    assert np.sum(c * e) == pytest.approx(np.sum(x * sara.idwt2(e, p, levels)), rel=1e-12)


@pytest.mark.parametrize("p", range(1, 9))
def test_constant_image_has_no_details(p):
    x = np.full((32, 32), 1.5)
    c = sara.dwt2(x, p, 3)
    assert np.allclose(c[:4, :4], 1.5 * 8.0, rtol=1e-12)       # (sum h)^2 = 2 per level
    c[:4, :4] = 0
    assert np.abs(c).max() < 1e-12


def test_shift_equivariance_level1():
    x = np.random.default_rng(4).standard_normal((16, 16))
    for p in (2, 5, 8):
        c = sara.dwt2(x, p, 1)
        cs = sara.dwt2(np.roll(x, (2, 4), axis=(0, 1)), p, 1)
        ll, lls = c[:8, :8], cs[:8, :8]
        assert np.allclose(lls, np.roll(ll, (1, 2), axis=(0, 1)), atol=1e-13)


def test_sara_parseval_frame():
    x = np.random.default_rng(7).standard_normal((32, 32))
    u = sara.analysis(x, 3)
    assert u.shape == (9, 32, 32)
    assert np.linalg.norm(u) == pytest.approx(np.linalg.norm(x), rel=1e-13)   # ||Psi^H x|| = ||x||
    assert np.abs(sara.synthesis(u, 3) - x).max() < 1e-12                    # Psi Psi^H = I
    assert np.allclose(u[0], x / 3.0, atol=0)                                # Dirac basis
    w = np.random.default_rng(8).standard_normal((9, 32, 32))
    assert np.sum(u * w) == pytest.approx(np.sum(x * sara.synthesis(w, 3)), rel=1e-12)
