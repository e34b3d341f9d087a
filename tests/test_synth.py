"""Host checks of the seeded input generators (no method arithmetic)."""
import math

import numpy as np

import synth


def test_active_sets_shapes_and_rates():
    bm, pm = synth.active_sets(2000, 16, 0.3, 0.7, seed=1)
    assert bm.shape == (2000, 16) and pm.shape == (2000, 9)
    assert bm.dtype == np.uint8 and set(np.unique(bm)) <= {0, 1}
    assert abs(bm.mean() - 0.3) < 0.02 and abs(pm.mean() - 0.7) < 0.02
    bm2, _ = synth.active_sets(2000, 16, 0.3, 0.7, seed=1)
    assert np.array_equal(bm, bm2)


def test_ggd_coverage_concentrates_as_beta_drops():
    """Equal standard deviation for every shape: the centre gets denser and
    the tails heavier as beta drops (Sec. 5.2's sampling family)."""
    frac = {}
    for beta in (2.0, 0.5, 0.25):
        wu, wv = synth.coverage_ggd(50000, seed=3, beta=beta)
        assert wu.dtype == np.float32 and np.all(np.abs(wu) < math.pi) and np.all(np.abs(wv) < math.pi)
        frac[beta] = float(np.mean(np.hypot(wu, wv) < 0.1))
    assert frac[0.25] > frac[0.5] > frac[2.0]


def test_crop_keeps_points_per_cell():
    """The crop problem keeps 1/keep of every block and an n_crop^2 image, so
    points per grid cell match the full problem's."""
    w = synth.Workload("t", n=256, M=64000, d=4, coverage="radial", isnr_db=30.0, seed_idx=9,
                       block_lo=8000, block_hi=30000)
    big = synth.make_inputs(w)
    c = synth.crop_inputs(big, 64, 16, seed=5)
    assert c.x_true.shape == (64, 64) and c.wu.shape[1] == c.block_off[-1]
    assert np.allclose(np.diff(c.block_off), np.diff(big.block_off) // 16)
    dens_big = w.M / (2 * w.n) ** 2
    dens_crop = c.block_off[-1] / (2 * 64) ** 2
    assert abs(dens_crop / dens_big - 1.0) < 0.01
    assert np.array_equal(c.x_true, big.x_true[96:160, 96:160])
