"""Seeded synthetic inputs shaped like the paper's simulated workloads.

This module is shared by the FP64 oracle (``oracle/``), the tests and the
benchmark.  It holds none of the imaging method's arithmetic: it only draws
random skies, u-v coverages, unit noise samples and data-block partitions.
Everything that depends on the measurement operator (visibilities, noise
level, l2 bounds, preconditioner, operator norms) is computed by whichever
side consumes these inputs.

The paper's own test images (a 512x512 galaxy cluster, a 477x1024 Cygnus A
image) and coverages (VLA, SKA, 3C129) are not available, so the recipes
below stand in for them (Sec. 5 of the paper describes the originals):

* sky: 3 Gaussian blobs plus 10 point sources, non-negative, FP64;
* coverage: frequencies normalised to [-pi, pi) (Sec. 5, coverage figure
  caption), drawn radially with areal density ~ 1/r, or along elliptical
  Earth-rotation-like tracks, or from a generalised Gaussian (Sec. 5.2);
* noise: zero-mean complex white Gaussian samples of unit variance, scaled
  later to a target input SNR (Sec. 5);
* blocks: visibilities sorted by radius and cut into contiguous radial
  bands, innermost first (the split of Sec. 3.1 with the rule unspecified).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Tuple

import numpy as np

# Largest float32 strictly below pi: coverage values stay inside [-pi, pi).
PI_F32_BELOW = float(np.nextafter(np.float32(np.pi), np.float32(0.0)))


@dataclasses.dataclass(frozen=True)
class Workload:
    """A named synthetic workload: sizes, coverage kind, noise level, seeds."""
    name: str
    n: int                      # image is n x n pixels
    M: int                      # visibilities per channel
    d: int                      # number of data blocks
    coverage: str               # "radial" | "tracks" | "ggd"
    isnr_db: float              # input SNR of the visibilities
    seed_idx: int               # seeds: sky k, coverage 100+k, noise 200+k, blocks 300+k
    block_sizes: Optional[Tuple[int, ...]] = None   # explicit sizes, else drawn
    block_lo: int = 0           # log-uniform block size range when drawn
    block_hi: int = 0
    n_chan: int = 1
    rmin_frac: float = 1e-3     # radial coverage: r ~ U[rmin_frac*pi, rmax]
    rmax: float = math.pi
    ggd_beta: float = 2.0
    iters: int = 200
    n_itr: int = 1


WORKLOADS = {
    # 64^2 image, 4096 points, one block, 20 dB: small enough for the oracle.
    "ppd64": Workload("ppd64", n=64, M=4096, d=1, coverage="radial", isnr_db=20.0,
                      seed_idx=1, iters=200, n_itr=1),
    # 256^2, 65536 points on 36 elliptical tracks, 4 uneven blocks, 30 dB.
    "tracks256": Workload("tracks256", n=256, M=65536, d=4, coverage="tracks",
                          isnr_db=30.0, seed_idx=2,
                          block_sizes=(8000, 12000, 20000, 25536), iters=500, n_itr=5),
    # 512^2, 1.3M points, 16 uneven blocks of 20k..200k, 30 dB.
    "ppd512": Workload("ppd512", n=512, M=1_300_000, d=16, coverage="radial",
                       isnr_db=30.0, seed_idx=3, block_lo=20_000, block_hi=200_000,
                       iters=200, n_itr=1),
    # 512^2, 1M points per channel, 8 channels scaled by nu/nu0 in [0.9, 1.1].
    "multichan512": Workload("multichan512", n=512, M=1_000_000, d=8, coverage="radial",
                             isnr_db=30.0, seed_idx=4, n_chan=8,
                             rmax=math.pi / 1.1, block_lo=60_000, block_hi=250_000),
    # 256^2, 65536 points drawn from a generalised Gaussian of shape beta in u
    # and v (Sec. 5.2: beta = 2, 0.5, 0.25; input SNR 30 and 50 dB), 4 blocks.
    "ggd256_b2": Workload("ggd256_b2", n=256, M=65536, d=4, coverage="ggd", isnr_db=30.0,
                          seed_idx=6, block_lo=8000, block_hi=30000, ggd_beta=2.0, iters=300),
    "ggd256_b05": Workload("ggd256_b05", n=256, M=65536, d=4, coverage="ggd", isnr_db=30.0,
                           seed_idx=7, block_lo=8000, block_hi=30000, ggd_beta=0.5, iters=300),
    "ggd256_b025": Workload("ggd256_b025", n=256, M=65536, d=4, coverage="ggd", isnr_db=30.0,
                            seed_idx=8, block_lo=8000, block_hi=30000, ggd_beta=0.25, iters=300),
    "ggd256_b025_50db": Workload("ggd256_b025_50db", n=256, M=65536, d=4, coverage="ggd", isnr_db=50.0,
                                 seed_idx=8, block_lo=8000, block_hi=30000, ggd_beta=0.25, iters=300),
    # 2048^2, 20M points, 64 uneven blocks, 1e3:1 density contrast.
    "ppd2048": Workload("ppd2048", n=2048, M=20_000_000, d=64, coverage="radial",
                        isnr_db=30.0, seed_idx=5,
                        block_lo=int(20_000_000 / 64 / math.sqrt(10)),
                        block_hi=int(20_000_000 / 64 * math.sqrt(10)), iters=200),
}


def sky(n: int, seed: int, nx: Optional[int] = None) -> np.ndarray:
    """Non-negative FP64 test sky of shape (n, nx): 3 Gaussian blobs + 10 points.

    Blob width sigma ~ U[2, 6] px scaled by n/64, peak ~ U[0.1, 1], centre
    ~ U[0.2n, 0.8n]^2; point sources at integer pixels ~ U[0.1n, 0.9n)^2 with
    amplitude log-uniform in [1e-2, 1].
    """
    ny = n
    nx = n if nx is None else nx
    rng = np.random.default_rng(seed)
    img = np.zeros((ny, nx), dtype=np.float64)
    rr, cc = np.meshgrid(np.arange(ny, dtype=np.float64),
                         np.arange(nx, dtype=np.float64), indexing="ij")
    scale = min(ny, nx) / 64.0
    for _ in range(3):
        sig = rng.uniform(2.0, 6.0) * scale
        peak = rng.uniform(0.1, 1.0)
        r0 = rng.uniform(0.2 * ny, 0.8 * ny)
        c0 = rng.uniform(0.2 * nx, 0.8 * nx)
        img += peak * np.exp(-((rr - r0) ** 2 + (cc - c0) ** 2) / (2.0 * sig * sig))
    rs = rng.integers(int(0.1 * ny), int(0.9 * ny), size=10)
    cs = rng.integers(int(0.1 * nx), int(0.9 * nx), size=10)
    amps = 10.0 ** rng.uniform(-2.0, 0.0, size=10)
    for r, c, a in zip(rs, cs, amps):
        img[r, c] += a
    return img


def _to_f32_coverage(wu: np.ndarray, wv: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    lo, hi = -PI_F32_BELOW, PI_F32_BELOW
    wu = np.clip(wu, lo, hi).astype(np.float32)
    wv = np.clip(wv, lo, hi).astype(np.float32)
    return wu, wv


def coverage_radial(M: int, seed: int, rmin: float = math.pi * 1e-3,
                    rmax: float = math.pi, jitter: float = 0.01 * math.pi):
    """Radius ~ U[rmin, rmax] (areal density ~ 1/r), angle ~ U[0, 2pi),
    Gaussian jitter per axis, clipped to [-pi, pi). Returns float32 (wu, wv)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(rmin, rmax, size=M)
    a = rng.uniform(0.0, 2.0 * math.pi, size=M)
    wu = r * np.cos(a) + rng.normal(0.0, jitter, size=M)
    wv = r * np.sin(a) + rng.normal(0.0, jitter, size=M)
    return _to_f32_coverage(wu, wv)


def coverage_tracks(M: int, seed: int, n_tracks: int = 36, jitter: float = 0.002 * math.pi):
    """Half-ellipse tracks: semi-major ~ U[0.02pi, 0.95pi], axis ratio
    ~ U[0.2, 1], rotation ~ U[0, pi), evenly spaced along the arc."""
    rng = np.random.default_rng(seed)
    counts = np.full(n_tracks, M // n_tracks, dtype=np.int64)
    counts[: M - counts.sum()] += 1
    us, vs = [], []
    for k in range(n_tracks):
        a = rng.uniform(0.02 * math.pi, 0.95 * math.pi)
        b = a * rng.uniform(0.2, 1.0)
        rot = rng.uniform(0.0, math.pi)
        s0 = rng.uniform(0.0, 2.0 * math.pi)
        s = s0 + math.pi * (np.arange(counts[k]) + 0.5) / counts[k]
        eu, ev = a * np.cos(s), b * np.sin(s)
        us.append(eu * math.cos(rot) - ev * math.sin(rot) + rng.normal(0.0, jitter, counts[k]))
        vs.append(eu * math.sin(rot) + ev * math.cos(rot) + rng.normal(0.0, jitter, counts[k]))
    return _to_f32_coverage(np.concatenate(us), np.concatenate(vs))


def coverage_ggd(M: int, seed: int, beta: float, std: float = math.pi / 3):
    """Zero-mean generalised Gaussian in u and v independently, shape beta
    (beta = 2 Gaussian; smaller beta = sharper centre and heavier tails),
    scale set so that the standard deviation is `std` for every beta:
    x = s * alpha * g^(1/beta), g ~ Gamma(1/beta), s = +-1, alpha =
    std * sqrt(Gamma(1/beta) / Gamma(3/beta)).  Samples outside [-pi, pi)
    are redrawn."""
    rng = np.random.default_rng(seed)
    alpha = std * math.exp(0.5 * (math.lgamma(1.0 / beta) - math.lgamma(3.0 / beta)))
    out = []
    for _ in range(2):
        vals = np.empty(0)
        while vals.size < M:
            g = rng.gamma(1.0 / beta, 1.0, size=2 * M)
            sgn = np.where(rng.uniform(size=2 * M) < 0.5, -1.0, 1.0)
            x = sgn * alpha * g ** (1.0 / beta)
            vals = np.concatenate([vals, x[np.abs(x) < PI_F32_BELOW]])
        out.append(vals[:M])
    return _to_f32_coverage(out[0], out[1])


def active_sets(T: int, d: int, p_block: float, p_basis: float, seed: int, n_bases: int = 9):
    """Random active sets of a randomised run (Sec. 4: independent, identically
    distributed draws with nonzero probability): T x d block masks and
    T x n_bases basis masks, Bernoulli(p_block) and Bernoulli(p_basis), uint8."""
    rng = np.random.default_rng(seed)
    blocks = (rng.uniform(size=(T, d)) < p_block).astype(np.uint8)
    bases = (rng.uniform(size=(T, n_bases)) < p_basis).astype(np.uint8)
    return blocks, bases


def noise_unit(M: int, seed: int) -> np.ndarray:
    """Complex white Gaussian noise with E|n|^2 = 1: (a + ib)/sqrt(2)."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(M)
    b = rng.standard_normal(M)
    return (a + 1j * b) / math.sqrt(2.0)


def block_sizes_loguniform(M: int, d: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """d block sizes drawn log-uniform in [lo, hi], rescaled to sum exactly to M."""
    if d == 1:
        return np.array([M], dtype=np.int64)
    rng = np.random.default_rng(seed)
    s = np.exp(rng.uniform(math.log(lo), math.log(hi), size=d))
    s = np.maximum(1, np.floor(s * (M / s.sum()))).astype(np.int64)
    s[int(np.argmax(s))] += M - int(s.sum())
    return s


def radial_blocks(wu: np.ndarray, wv: np.ndarray, sizes) -> Tuple[np.ndarray, np.ndarray, np.ndarray, np.ndarray]:
    """Order points by |omega| (stable) and cut contiguous radial bands of the
    given sizes, innermost first.  Returns (wu, wv, block_off[d+1], order)."""
    sizes = np.asarray(sizes, dtype=np.int64)
    assert int(sizes.sum()) == wu.size
    r2 = wu.astype(np.float64) ** 2 + wv.astype(np.float64) ** 2
    order = np.argsort(r2, kind="stable")
    off = np.zeros(sizes.size + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    return wu[order], wv[order], off, order


@dataclasses.dataclass
class Inputs:
    """Everything random a run needs, before any operator is applied."""
    workload: Workload
    x_true: np.ndarray          # (n, n) float64, non-negative
    wu: np.ndarray              # (n_chan, M) float32, blocks contiguous
    wv: np.ndarray
    block_off: np.ndarray       # (d+1,) int64 offsets into one channel
    noise: np.ndarray           # (n_chan, M) complex128, unit variance
    power_start: np.ndarray     # (n, n) float64 start vector for power iteration


def make_inputs(w: Workload) -> Inputs:
    k = w.seed_idx
    x = sky(w.n, seed=k)
    if w.block_sizes is not None:
        sizes = np.asarray(w.block_sizes, dtype=np.int64)
    else:
        sizes = block_sizes_loguniform(w.M, w.d, w.block_lo, w.block_hi, seed=300 + k)
    if w.coverage == "radial":
        wu, wv = coverage_radial(w.M, seed=100 + k, rmin=w.rmin_frac * math.pi, rmax=w.rmax)
    elif w.coverage == "tracks":
        wu, wv = coverage_tracks(w.M, seed=100 + k)
    elif w.coverage == "ggd":
        wu, wv = coverage_ggd(w.M, seed=100 + k, beta=w.ggd_beta)
    else:
        raise ValueError(w.coverage)
    wu, wv, off, _ = radial_blocks(wu, wv, sizes)
    if w.n_chan > 1:
        f = np.linspace(0.9, 1.1, w.n_chan, dtype=np.float64)
        base_u, base_v = wu.astype(np.float64), wv.astype(np.float64)
        scaled = [_to_f32_coverage(base_u * fi, base_v * fi) for fi in f]
        wu = np.stack([s[0] for s in scaled])
        wv = np.stack([s[1] for s in scaled])
    else:
        wu, wv = wu[None, :], wv[None, :]
    nz = np.stack([noise_unit(w.M, seed=200 + k + 1000 * c) for c in range(w.n_chan)])
    ps = np.random.default_rng(400 + k).standard_normal((w.n, w.n))
    return Inputs(w, x, wu, wv, off, nz, ps)


def crop_inputs(big: Inputs, n_crop: int, keep: int, seed: int) -> Inputs:
    """A smaller problem at the same visibilities-per-grid-cell density as a
    large workload: the central n_crop x n_crop part of its sky and a random
    1/keep subset of its points (frequencies in radians per pixel, so the
    same values index the smaller grid at the same relative place), with the
    block structure kept (each block subsampled alike) and fresh unit noise."""
    w = big.workload
    n = w.n
    r0 = (n - n_crop) // 2
    x = big.x_true[r0:r0 + n_crop, r0:r0 + n_crop].copy()
    rng = np.random.default_rng(seed)
    wu, wv, off = big.wu[0], big.wv[0], big.block_off
    idx, new_off = [], [0]
    for j in range(off.size - 1):
        pick = np.sort(rng.choice(np.arange(off[j], off[j + 1]), size=(off[j + 1] - off[j]) // keep,
                                  replace=False))
        idx.append(pick)
        new_off.append(new_off[-1] + pick.size)
    idx = np.concatenate(idx)
    M = idx.size
    cw = dataclasses.replace(w, name=f"{w.name}_crop{n_crop}", n=n_crop, M=M)
    nz = noise_unit(M, seed=seed + 1)[None, :]
    ps = np.random.default_rng(seed + 2).standard_normal((n_crop, n_crop))
    return Inputs(cw, x, wu[idx][None, :], wv[idx][None, :], np.asarray(new_off, dtype=np.int64), nz, ps)


def small_case(n: int, M: int, seed: int, nx: Optional[int] = None, d: int = 1,
               coverage: str = "radial"):
    """Tiny random problem for unit tests: (x, wu, wv, block_off)."""
    nx = n if nx is None else nx
    x = sky(n, seed=seed, nx=nx)
    if coverage == "uniform":
        rng = np.random.default_rng(100 + seed)
        wu, wv = _to_f32_coverage(rng.uniform(-math.pi, math.pi, M),
                                  rng.uniform(-math.pi, math.pi, M))
    else:
        wu, wv = coverage_radial(M, seed=100 + seed)
    if d == 1:
        off = np.array([0, M], dtype=np.int64)
    else:
        sizes = block_sizes_loguniform(M, d, max(1, M // (4 * d)), max(2, 4 * M // d), 300 + seed)
        wu, wv, off, _ = radial_blocks(wu, wv, sizes)
    return x, wu, wv, off
