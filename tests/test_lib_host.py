"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
its host-side helpers agree with the oracle, and argument validation rejects
bad plans before touching a device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from oracle import nufft as onf
from oracle import sara as osara

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ppd.h")


@pytest.fixture(scope="module")
def P():
    from paper_1701_01748_amd import ppd
    if not os.path.exists(ppd.LIB_PATH):
        pytest.fail("libppd.so not built (python -m paper_1701_01748_amd.build)")
    ppd.lib()
    return ppd


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ppd_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(P):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(P.lib(), n), n
        assert n in P._PROTOS, f"binding lacks a prototype for {n}"


def test_single_hip_runtime(P):
    assert len(P._hip_runtimes_mapped()) == 1


def test_status_strings(P):
    L = P.lib()
    assert L.ppd_strerror(0) == b"ok"
    assert b"invalid" in L.ppd_strerror(-1)


def test_kb_weights_match_oracle(P):
    beta = onf.kb_beta()
    s = np.linspace(0.0, 1.0, 4001, dtype=np.float32)[:-1]
    w = P.kb_weights_host(s).astype(np.float64)
    m = np.arange(8)
    ref = onf.kb(s.astype(np.float64)[:, None] + 3.0 - m[None, :], beta)
    peak = float(onf.kb(0.0, beta))
    assert np.abs(w - ref).max() / peak < 2e-7


@pytest.mark.parametrize("p", range(1, 9))
def test_daubechies_match_oracle(P, p):
    h = P.daubechies_host(p)
    assert np.allclose(h, osara.daubechies_lowpass(p), atol=1e-14)


def test_daubechies_db2_closed_form(P):
    s3 = math.sqrt(3.0)
    ref = np.array([1 + s3, 3 + s3, 3 - s3, 1 - s3]) / (4 * math.sqrt(2))
    assert np.allclose(P.daubechies_host(2), ref, atol=1e-15)


class _NoStream:
    cuda_stream = 0


@pytest.mark.parametrize("case", ["nx_not_pow2", "omega_out_of_range", "empty_block", "bad_offsets",
                                  "bad_tile", "bad_levels", "theta_nonpositive"])
def test_plan_validation_rejects_before_device_use(P, case):
    M = 64
    rng = np.random.default_rng(0)
    wu = rng.uniform(-3, 3, M).astype(np.float32)
    wv = rng.uniform(-3, 3, M).astype(np.float32)
    kw = dict(nx=32, ny=32, omega_u=wu, omega_v=wv, block_off=np.array([0, M]))
    if case == "nx_not_pow2":
        kw["nx"] = 48
    elif case == "omega_out_of_range":
        wu[5] = 3.2
    elif case == "empty_block":
        kw["block_off"] = np.array([0, 10, 10, M])
    elif case == "bad_offsets":
        kw["block_off"] = np.array([0, 10, M - 1])
    elif case == "bad_tile":
        kw["tile"] = 24
    elif case == "bad_levels":
        kw["levels"] = 7
    elif case == "theta_nonpositive":
        kw["theta"] = np.ones(M, np.float32)
        kw["theta"][3] = 0.0
    with pytest.raises(P.PPDError) as ei:
        P.Plan(stream=_NoStream(), **kw)
    assert ei.value.status in (P.PPD_EINVAL, P.PPD_EUNSUPPORTED)


def test_workspace_size_is_a_host_query(P):
    """The workspace query runs without a device, is reproducible, holds at
    least the two oversampled grids and grows with the number of points."""
    rng = np.random.default_rng(1)
    sizes = []
    for M in (64, 4096):
        wu = rng.uniform(-3, 3, M).astype(np.float32)
        wv = rng.uniform(-3, 3, M).astype(np.float32)
        off = np.array([0, M // 2, M])
        a = P.plan_workspace_size(32, 32, wu, wv, off)
        assert a == P.plan_workspace_size(32, 32, wu, wv, off)
        assert a % 256 == 0 and a >= 2 * 64 * 64 * 8
        sizes.append(a)
    assert sizes[1] > sizes[0]
    with pytest.raises(P.PPDError) as ei:
        P.plan_workspace_size(48, 32, wu, wv, off)
    assert ei.value.status == P.PPD_EUNSUPPORTED
