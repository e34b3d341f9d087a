"""Helpers shared by the GPU parity tests (no method arithmetic)."""
import sys

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_1701_01748_amd import ppd
    ppd.lib()
    return ppd


def announce(msg: str):
    """Name the GPU case before it runs (flushed, in case the device faults)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def peak_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# Operator outputs (float32 path against the float64 oracle): norm-wise and
# peak-relative element-wise bound of the stated parity tolerance.
OP_TOL = 1e-5


def assert_op_close(gpu, ref, tol=OP_TOL, what=""):
    r, p = rel_err(gpu, ref), peak_err(gpu, ref)
    assert r <= tol and p <= tol, f"{what}: rel {r:.3e}, peak-rel {p:.3e} > {tol:g}"
