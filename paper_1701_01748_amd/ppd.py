"""ctypes binding of libppd (include/ppd.h), argument marshalling only.

Torch tensors provide device memory and the stream; every operation runs in
the HIP kernels of ``libppd.so``.  There is no fallback: if the library is
missing, or no GPU is present, the calls raise.

Shapes and dtypes are checked here, on the host, before any launch, because
the C ABI takes plain pointers and cannot check buffer sizes itself.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libppd.so")

# status codes and flags (include/ppd.h)
PPD_OK, PPD_EINVAL, PPD_ENOMEM, PPD_EDEVICE, PPD_ENONFINITE, PPD_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
USER_TO_PLAN, PLAN_TO_USER = 0, 1
ORDER_PLAN, ORDER_USER = 0, 1
SARA_ANALYSIS, SARA_SYNTHESIS, SARA_DUAL = 0, 1, 2
FORM_FUSED, FORM_PLAIN = 0, 1
PROX_FB, PROX_EXACT = 0, 1
PERSIST_AUTO, PERSIST_OFF = 0, 1

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class PlanDesc(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("M", c_int64), ("d", c_int32),
                ("block_off", ctypes.POINTER(c_int64)), ("omega_u", c_void_p), ("omega_v", c_void_p),
                ("theta", c_void_p), ("kb_beta", c_double), ("levels", c_int32), ("tile", c_int32),
                ("chunk", c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("Kx", c_int32), ("Ky", c_int32), ("M", c_int64),
                ("d", c_int32), ("levels", c_int32), ("tile", c_int32), ("chunk", c_int32),
                ("n_chunks", c_int32), ("kb_beta", c_double), ("device_bytes", ctypes.c_size_t),
                ("persistent", c_int32), ("pad_", c_int32)]


class State(ctypes.Structure):
    _fields_ = [("x", c_void_p), ("xt", c_void_p), ("v", c_void_p), ("u", c_void_p), ("z", c_void_p),
                ("iter", c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("tau", c_double), ("eta", c_double), ("zeta", c_double), ("lambda_", c_double),
                ("alpha", c_double), ("mu", c_double), ("n_itr", c_int32), ("form", c_int32),
                ("use_graph", c_int32), ("pad_", c_int32), ("y", c_void_p), ("U", c_void_p),
                ("eps", ctypes.POINTER(c_double)), ("x_true", c_void_p), ("W", c_void_p),
                ("prox", c_int32), ("n_newton", c_int32), ("block_active", c_void_p),
                ("basis_active", c_void_p), ("persistent", c_int32), ("spin_limit", c_int32),
                ("stats_every", c_int32), ("pad2_", c_int32), ("stats_history", c_void_p)]


class Stats(ctypes.Structure):
    _fields_ = [("iter", c_int64), ("rel_change", c_double), ("x_norm", c_double), ("snr_db", c_double),
                ("residual_max", c_double)]


_PROTOS = {
    "ppd_strerror": (ctypes.c_char_p, [c_int32]),
    "ppd_last_error": (ctypes.c_char_p, []),
    "ppd_plan_create": (c_int32, [ctypes.POINTER(c_void_p), ctypes.POINTER(PlanDesc), c_void_p]),
    "ppd_plan_workspace_size": (c_int32, [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_size_t)]),
    "ppd_plan_create_ws": (c_int32, [ctypes.POINTER(c_void_p), ctypes.POINTER(PlanDesc), c_void_p,
                                     ctypes.c_size_t, c_void_p]),
    "ppd_plan_destroy": (c_int32, [c_void_p]),
    "ppd_plan_set_stream": (c_int32, [c_void_p, c_void_p]),
    "ppd_plan_get_info": (c_int32, [c_void_p, ctypes.POINTER(PlanInfo)]),
    "ppd_plan_permutation": (c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    "ppd_plan_permute": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_int32]),
    "ppd_phi": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32]),
    "ppd_phit": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32]),
    "ppd_sara": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, ctypes.c_float, ctypes.c_float]),
    "ppd_sara_w": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, ctypes.c_float,
                             ctypes.c_float]),
    "ppd_reweight": (c_int32, [c_void_p, c_void_p, ctypes.c_float, c_void_p]),
    "ppd_ellipsoid_proj": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double),
                                     c_int32, c_double, c_void_p]),
    "ppd_ellipsoid_proj_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, ctypes.POINTER(c_int64),
                                             ctypes.POINTER(c_double), c_int32, c_double, c_void_p, c_void_p]),
    "ppd_prox_metric": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double), c_int32,
                                  c_void_p, c_void_p]),
    "ppd_uniform_weights": (c_int32, [c_void_p, c_void_p]),
    "ppd_op_norm": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_double, ctypes.POINTER(c_double),
                              ctypes.POINTER(c_int32)]),
    "ppd_iterate": (c_int32, [c_void_p, ctypes.POINTER(State), ctypes.POINTER(Params), c_int32,
                              ctypes.POINTER(Stats), ctypes.POINTER(c_double)]),
    "ppd_reweighted": (c_int32, [c_void_p, ctypes.POINTER(State), ctypes.POINTER(Params), c_int32, c_int32,
                                 c_double, c_double, c_void_p, ctypes.POINTER(Stats)]),
    "ppd_dual_update": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double), c_void_p,
                                  c_void_p, c_int32, c_double, c_double, c_void_p, c_void_p, c_void_p]),
    "ppd_dual_update_vjp": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, ctypes.POINTER(c_double), c_void_p,
                                      c_void_p, c_int32, c_double, c_double, c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p, c_void_p, c_void_p]),
    "ppd_sparsity_update": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.c_float, ctypes.c_float, c_void_p]),
    "ppd_sparsity_update_vjp": (c_int32, [c_void_p, c_void_p, c_void_p, ctypes.c_float, ctypes.c_float, c_void_p,
                                          c_void_p, c_void_p]),
    "ppd_primal_update": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_double, c_double,
                                    c_void_p, c_void_p]),
    "ppd_primal_update_vjp": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_double, c_double, c_double,
                                        c_double, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "ppd_timing_enable": (c_int32, [c_void_p, c_int32]),
    "ppd_timing_reset": (c_int32, [c_void_p]),
    "ppd_timing_read": (c_int32, [c_void_p, c_int32, ctypes.POINTER(ctypes.c_char_p),
                                  ctypes.POINTER(c_int64), ctypes.POINTER(c_double), ctypes.POINTER(c_int32)]),
    "ppd_kb_weights_host": (c_int32, [c_double, c_int64, c_void_p, c_void_p]),
    "ppd_daubechies_host": (c_int32, [c_int32, ctypes.POINTER(c_double)]),
}

_lib = None


def _hip_runtimes_mapped():
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(line.split()[-1])
    return paths


def lib() -> ctypes.CDLL:
    """Load libppd.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  -- loads torch's HIP runtime first
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1701_01748_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _PROTOS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        rts = _hip_runtimes_mapped()
        if len(rts) > 1:
            raise RuntimeError(f"two HIP runtimes are mapped in this process: {sorted(rts)}")
        _lib = L
    return _lib


class PPDError(RuntimeError):
    def __init__(self, fn: str, status: int):
        L = lib()
        super().__init__(f"{fn}: {L.ppd_strerror(status).decode()} ({status}): {L.ppd_last_error().decode()}")
        self.status = status


def _check(fn: str, status: int):
    if status != PPD_OK:
        raise PPDError(fn, status)


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _need(t, dtype, numel: int, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, got {t.numel()}")


def plan_workspace_size(nx: int, ny: int, omega_u, omega_v, block_off, theta=None, kb_beta: float = 0.0,
                        levels: int = 3, tile: int = 0, chunk: int = 0) -> int:
    """Device bytes a plan of this coverage needs in a caller workspace (host
    only: validation and binning, no device call)."""
    L = lib()
    wu = np.ascontiguousarray(omega_u, dtype=np.float32)
    wv = np.ascontiguousarray(omega_v, dtype=np.float32)
    off = np.ascontiguousarray(block_off, dtype=np.int64)
    th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float32)
    desc = PlanDesc(nx, ny, wu.size, off.size - 1, off.ctypes.data_as(ctypes.POINTER(c_int64)),
                    wu.ctypes.data, wv.ctypes.data, None if th is None else th.ctypes.data,
                    kb_beta, levels, tile, chunk)
    size = ctypes.c_size_t(0)
    _check("ppd_plan_workspace_size", L.ppd_plan_workspace_size(ctypes.byref(desc), ctypes.byref(size)))
    return int(size.value)


class Plan:
    """A libppd plan for one coverage (HOST numpy inputs, see ppd_plan_desc).
    With `workspace` (the default) the plan's device buffers live in one
    uint8 tensor allocated here by PyTorch and kept with the plan; without
    it the library allocates them."""

    def __init__(self, nx: int, ny: int, omega_u, omega_v, block_off, theta=None, kb_beta: float = 0.0,
                 levels: int = 3, tile: int = 0, chunk: int = 0, stream=None, workspace: bool = True):
        import torch
        L = lib()
        self._wu = np.ascontiguousarray(omega_u, dtype=np.float32)
        self._wv = np.ascontiguousarray(omega_v, dtype=np.float32)
        self._off = np.ascontiguousarray(block_off, dtype=np.int64)
        self._th = None if theta is None else np.ascontiguousarray(theta, dtype=np.float32)
        if self._wu.shape != self._wv.shape or self._wu.ndim != 1:
            raise ValueError("omega_u and omega_v must be equal-length 1-D arrays")
        if self._th is not None and self._th.shape != self._wu.shape:
            raise ValueError("theta must match omega")
        desc = PlanDesc(nx, ny, self._wu.size, self._off.size - 1,
                        self._off.ctypes.data_as(ctypes.POINTER(c_int64)),
                        self._wu.ctypes.data, self._wv.ctypes.data,
                        None if self._th is None else self._th.ctypes.data,
                        kb_beta, levels, tile, chunk)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = c_void_p()
        self._ws = None
        if workspace:
            size = ctypes.c_size_t(0)
            _check("ppd_plan_workspace_size", L.ppd_plan_workspace_size(ctypes.byref(desc), ctypes.byref(size)))
            self._ws = torch.empty(size.value, dtype=torch.uint8, device="cuda")
            _check("ppd_plan_create_ws", L.ppd_plan_create_ws(ctypes.byref(h), ctypes.byref(desc),
                                                              c_void_p(self._ws.data_ptr()), size,
                                                              c_void_p(int(stream.cuda_stream))))
        else:
            _check("ppd_plan_create", L.ppd_plan_create(ctypes.byref(h), ctypes.byref(desc),
                                                        c_void_p(int(stream.cuda_stream))))
        self._h = h
        info = PlanInfo()
        _check("ppd_plan_get_info", L.ppd_plan_get_info(h, ctypes.byref(info)))
        self.info = info
        self.nx, self.ny, self.M, self.d = nx, ny, int(info.M), int(info.d)
        self.N = nx * ny

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            lib().ppd_plan_destroy(self._h)   # synchronises the plan's streams
            self._h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        _check("ppd_plan_set_stream", lib().ppd_plan_set_stream(self.handle, c_void_p(int(stream.cuda_stream))))
        self.stream = stream

    def permutation(self) -> np.ndarray:
        out = np.empty(self.M, dtype=np.int64)
        _check("ppd_plan_permutation", lib().ppd_plan_permutation(self.handle, out.ctypes.data_as(ctypes.POINTER(c_int64))))
        return out

    def permute(self, direction: int, t, out=None):
        import torch
        if t.numel() != self.M and t.dtype not in (torch.complex64, torch.complex128, torch.float64):
            raise ValueError("per-visibility array expected")
        eb = t.element_size()
        if out is None:
            out = torch.empty_like(t)
        _need(t, t.dtype, self.M, "in")
        _need(out, t.dtype, self.M, "out")
        _check("ppd_plan_permute", lib().ppd_plan_permute(self.handle, direction, _ptr(t), _ptr(out), eb))
        return out

    # ---- timing ------------------------------------------------------------
    def timing(self, on: bool):
        _check("ppd_timing_enable", lib().ppd_timing_enable(self.handle, int(on)))

    def timing_reset(self):
        _check("ppd_timing_reset", lib().ppd_timing_reset(self.handle))

    def timing_read(self) -> dict:
        cap = 32
        names = (ctypes.c_char_p * cap)()
        counts = (c_int64 * cap)()
        ms = (c_double * cap)()
        n = c_int32()
        _check("ppd_timing_read", lib().ppd_timing_read(self.handle, cap, names, counts, ms, ctypes.byref(n)))
        return {names[i].decode(): (int(counts[i]), float(ms[i])) for i in range(min(n.value, cap))}


def _alloc(shape, dtype, like=None):
    import torch
    return torch.empty(shape, dtype=dtype, device="cuda")


def ppd_phi(plan: Plan, x, y=None, order: int = ORDER_PLAN):
    """y = Theta G F Z x (complex64, plan or user order)."""
    import torch
    _need(x, torch.float32, plan.N, "x")
    if y is None:
        y = _alloc((plan.M,), torch.complex64)
    _need(y, torch.complex64, plan.M, "y")
    _check("ppd_phi", lib().ppd_phi(plan.handle, _ptr(x), _ptr(y), order))
    return y


def ppd_phit(plan: Plan, y, x=None, order: int = ORDER_PLAN):
    """x = Re Phi^H y (float32 image)."""
    import torch
    _need(y, torch.complex64, plan.M, "y")
    if x is None:
        x = _alloc((plan.ny, plan.nx), torch.float32)
    _need(x, torch.float32, plan.N, "x")
    _check("ppd_phit", lib().ppd_phit(plan.handle, _ptr(y), _ptr(x), order))
    return x


def ppd_sara(plan: Plan, op: int, inp, out=None, u=None, alpha: float = 0.0, lam: float = 1.0, W=None):
    """SARA analysis / synthesis / dual step (Sec. 5.1), optionally re-weighted (Algorithm 1)."""
    import torch
    if W is not None:
        _need(W, torch.float32, 9 * plan.N, "W")
    if op == SARA_ANALYSIS:
        _need(inp, torch.float32, plan.N, "in")
        if out is None:
            out = _alloc((9, plan.ny, plan.nx), torch.float32)
        _need(out, torch.float32, 9 * plan.N, "out")
    elif op == SARA_SYNTHESIS:
        _need(inp, torch.float32, 9 * plan.N, "in")
        if out is None:
            out = _alloc((plan.ny, plan.nx), torch.float32)
        _need(out, torch.float32, plan.N, "out")
    elif op == SARA_DUAL:
        _need(inp, torch.float32, plan.N, "in")
        _need(u, torch.float32, 9 * plan.N, "u")
        if out is None:
            out = _alloc((plan.ny, plan.nx), torch.float32)
        _need(out, torch.float32, plan.N, "out")
    else:
        raise ValueError("unknown SARA op")
    _check("ppd_sara", lib().ppd_sara_w(plan.handle, op, _ptr(inp), _ptr(out), _ptr(u), _ptr(W), float(alpha),
                                         float(lam)))
    return out


def ppd_reweight(plan: Plan, x, omega: float, W=None):
    """Algorithm 1 re-weights W = omega / (omega + |Psi^H x|) ([9][ny][nx])."""
    import torch
    _need(x, torch.float32, plan.N, "x")
    if W is None:
        W = _alloc((9, plan.ny, plan.nx), torch.float32)
    _need(W, torch.float32, 9 * plan.N, "W")
    _check("ppd_reweight", lib().ppd_reweight(plan.handle, _ptr(x), float(omega), _ptr(W)))
    return W


def _eps_arg(plan: Plan, eps):
    e = np.ascontiguousarray(eps, dtype=np.float64)
    if e.shape != (plan.d,):
        raise ValueError(f"eps must have shape ({plan.d},)")
    return e, e.ctypes.data_as(ctypes.POINTER(c_double))


def ppd_ellipsoid_proj(plan: Plan, w, y, U, eps, n_itr: int, mu: float, z):
    """n_itr Algorithm 2 iterations per block, in place on z (complex128)."""
    import torch
    _need(w, torch.complex128, plan.M, "w")
    _need(y, torch.complex64, plan.M, "y")
    _need(U, torch.float64, plan.M, "U")
    _need(z, torch.complex128, plan.M, "z")
    e, ep = _eps_arg(plan, eps)
    _check("ppd_ellipsoid_proj", lib().ppd_ellipsoid_proj(plan.handle, _ptr(w), _ptr(y), _ptr(U), ep,
                                                          int(n_itr), float(mu), _ptr(z)))
    return z


def ppd_ellipsoid_proj_noalloc(w, y, U, block_off, eps, n_itr: int, mu: float, z, stream=None):
    """ppd_ellipsoid_proj without a plan or any device allocation: blocks are
    the contiguous ranges of block_off (HOST); in place on z (complex128)."""
    import torch
    off = np.ascontiguousarray(block_off, dtype=np.int64)
    d = off.size - 1
    M = int(off[-1]) if d >= 1 else 0
    _need(w, torch.complex128, M, "w")
    _need(y, torch.complex64, M, "y")
    _need(U, torch.float64, M, "U")
    _need(z, torch.complex128, M, "z")
    e = np.ascontiguousarray(eps, dtype=np.float64)
    if e.shape != (d,):
        raise ValueError(f"eps must have shape ({d},)")
    if stream is None:
        stream = torch.cuda.current_stream()
    _check("ppd_ellipsoid_proj_noalloc",
           lib().ppd_ellipsoid_proj_noalloc(_ptr(w), _ptr(y), _ptr(U), d, off.ctypes.data_as(ctypes.POINTER(c_int64)),
                                            e.ctypes.data_as(ctypes.POINTER(c_double)), int(n_itr), float(mu),
                                            _ptr(z), c_void_p(int(stream.cuda_stream))))
    return z


def ppd_prox_metric(plan: Plan, w, y, U, eps, n_newton: int = 12, z=None, nu=None):
    """Exact prox of eq. elip-proj-1 per block (Newton on the secular equation)."""
    import torch
    _need(w, torch.complex128, plan.M, "w")
    _need(y, torch.complex64, plan.M, "y")
    _need(U, torch.float64, plan.M, "U")
    if z is None:
        z = _alloc((plan.M,), torch.complex128)
    _need(z, torch.complex128, plan.M, "z")
    if nu is not None:
        _need(nu, torch.float64, plan.d, "nu")
    e, ep = _eps_arg(plan, eps)
    _check("ppd_prox_metric", lib().ppd_prox_metric(plan.handle, _ptr(w), _ptr(y), _ptr(U), ep, int(n_newton),
                                                    _ptr(z), _ptr(nu)))
    return z


def ppd_uniform_weights(plan: Plan, U=None):
    import torch
    if U is None:
        U = _alloc((plan.M,), torch.float64)
    _need(U, torch.float64, plan.M, "U")
    _check("ppd_uniform_weights", lib().ppd_uniform_weights(plan.handle, _ptr(U)))
    return U


def ppd_op_norm(plan: Plan, U, x0, max_iter: int = 1000, tol: float = 1e-10):
    import torch
    if U is not None:
        _need(U, torch.float64, plan.M, "U")
    _need(x0, torch.float32, plan.N, "x0")
    out = c_double()
    it = c_int32()
    _check("ppd_op_norm", lib().ppd_op_norm(plan.handle, _ptr(U), _ptr(x0), int(max_iter), float(tol),
                                            ctypes.byref(out), ctypes.byref(it)))
    return float(out.value), int(it.value)


# ---- differentiable pieces of Algorithm 3 (forward and VJP) ---------------------

def ppd_dual_update(plan: Plan, g, y, U, eps, v, z, n_itr: int, mu: float, lam: float, keep: bool = False):
    """(v', z', zs) of the data-dual update; zs (n_itr x M complex128) only
    when keep (the VJP needs it)."""
    import torch
    for t, dt, name in ((g, torch.complex64, "g"), (y, torch.complex64, "y"), (v, torch.complex64, "v")):
        _need(t, dt, plan.M, name)
    _need(U, torch.float64, plan.M, "U")
    _need(z, torch.complex128, plan.M, "z")
    e, ep = _eps_arg(plan, eps)
    v_out = _alloc((plan.M,), torch.complex64)
    z_out = _alloc((plan.M,), torch.complex128)
    zs = _alloc((int(n_itr), plan.M), torch.complex128) if keep else None
    _check("ppd_dual_update", lib().ppd_dual_update(plan.handle, _ptr(g), _ptr(y), _ptr(U), ep, _ptr(v), _ptr(z),
                                                    int(n_itr), float(mu), float(lam), _ptr(v_out), _ptr(z_out),
                                                    _ptr(zs)))
    return v_out, z_out, zs


def ppd_dual_update_vjp(plan: Plan, g, y, U, eps, v, z, n_itr: int, mu: float, lam: float, zs, gv_out, gz_out):
    """Gradients (g_g, g_v, g_z, g_y) of the data-dual update."""
    import torch
    _need(zs, torch.complex128, int(n_itr) * plan.M, "zs")
    if gv_out is not None:
        _need(gv_out, torch.complex64, plan.M, "gv_out")
    if gz_out is not None:
        _need(gz_out, torch.complex128, plan.M, "gz_out")
    e, ep = _eps_arg(plan, eps)
    g_g = _alloc((plan.M,), torch.complex64)
    g_v = _alloc((plan.M,), torch.complex64)
    g_z = _alloc((plan.M,), torch.complex128)
    g_y = _alloc((plan.M,), torch.complex64)
    _check("ppd_dual_update_vjp", lib().ppd_dual_update_vjp(
        plan.handle, _ptr(g), _ptr(y), _ptr(U), ep, _ptr(v), _ptr(z), int(n_itr), float(mu), float(lam), _ptr(zs),
        _ptr(gv_out), _ptr(gz_out), _ptr(g_g), _ptr(g_v), _ptr(g_z), _ptr(g_y)))
    return g_g, g_v, g_z, g_y


def ppd_sparsity_update(plan: Plan, u, c, alpha: float, lam: float):
    import torch
    _need(u, torch.float32, 9 * plan.N, "u")
    _need(c, torch.float32, 9 * plan.N, "c")
    out = _alloc((9, plan.ny, plan.nx), torch.float32)
    _check("ppd_sparsity_update", lib().ppd_sparsity_update(plan.handle, _ptr(u), _ptr(c), float(alpha), float(lam),
                                                            _ptr(out)))
    return out


def ppd_sparsity_update_vjp(plan: Plan, u, c, alpha: float, lam: float, g_out):
    import torch
    _need(g_out, torch.float32, 9 * plan.N, "g_out")
    g_u = _alloc((9, plan.ny, plan.nx), torch.float32)
    g_c = _alloc((9, plan.ny, plan.nx), torch.float32)
    _check("ppd_sparsity_update_vjp", lib().ppd_sparsity_update_vjp(plan.handle, _ptr(u), _ptr(c), float(alpha),
                                                                    float(lam), _ptr(g_out), _ptr(g_u), _ptr(g_c)))
    return g_u, g_c


def ppd_primal_update(plan: Plan, x, a, b, tau: float, eta: float, zeta: float, lam: float):
    import torch
    for t, name in ((x, "x"), (a, "a"), (b, "b")):
        _need(t, torch.float32, plan.N, name)
    x_out = _alloc((plan.ny, plan.nx), torch.float32)
    xt_out = _alloc((plan.ny, plan.nx), torch.float32)
    _check("ppd_primal_update", lib().ppd_primal_update(plan.handle, _ptr(x), _ptr(a), _ptr(b), float(tau),
                                                        float(eta), float(zeta), float(lam), _ptr(x_out),
                                                        _ptr(xt_out)))
    return x_out, xt_out


def ppd_primal_update_vjp(plan: Plan, x, a, b, tau: float, eta: float, zeta: float, lam: float, gx_out, gxt_out):
    import torch
    for t, name in ((gx_out, "gx_out"), (gxt_out, "gxt_out")):
        if t is not None:
            _need(t, torch.float32, plan.N, name)
    g_x = _alloc((plan.ny, plan.nx), torch.float32)
    g_a = _alloc((plan.ny, plan.nx), torch.float32)
    g_b = _alloc((plan.ny, plan.nx), torch.float32)
    _check("ppd_primal_update_vjp", lib().ppd_primal_update_vjp(
        plan.handle, _ptr(x), _ptr(a), _ptr(b), float(tau), float(eta), float(zeta), float(lam), _ptr(gx_out),
        _ptr(gxt_out), _ptr(g_x), _ptr(g_a), _ptr(g_b)))
    return g_x, g_a, g_b


class PPDState:
    """Device state of Algorithm 3 (x, x tilde, v, u, z) owned by torch."""

    def __init__(self, plan: Plan, y=None):
        import torch
        self.x = torch.zeros((plan.ny, plan.nx), dtype=torch.float32, device="cuda")
        self.xt = torch.zeros_like(self.x)
        self.v = torch.zeros(plan.M, dtype=torch.complex64, device="cuda")
        self.u = torch.zeros((9, plan.ny, plan.nx), dtype=torch.float32, device="cuda")
        self.z = torch.zeros(plan.M, dtype=torch.complex128, device="cuda")
        if y is not None:
            self.z.copy_(y.to(torch.complex128))
        self.iter = 0

    def clone(self):
        c = object.__new__(PPDState)
        for k in ("x", "xt", "v", "u", "z"):
            setattr(c, k, getattr(self, k).clone())
        c.iter = self.iter
        return c


class Iteration:
    """Algorithm 3 on `state` with its arguments checked and marshalled once
    (see ppd_iterate for their meaning): run(n_iter) only calls the library,
    as a serving loop or a timed region would."""

    def __init__(self, plan: Plan, state: PPDState, y, U, eps, *, tau=0.49, eta=1.0, zeta=1.0, lam=1.0,
                 alpha=1e-4, mu=1.0, n_itr=1, form=FORM_FUSED, use_graph=False, x_true=None, prox=PROX_FB,
                 n_newton=0, block_active=None, basis_active=None, W=None, stats_every: int = 0,
                 stats_history=None, persistent: int = PERSIST_AUTO, spin_limit: int = 0):
        import torch
        _need(y, torch.complex64, plan.M, "y")
        _need(U, torch.float64, plan.M, "U")
        for k, dt, n in (("x", torch.float32, plan.N), ("xt", torch.float32, plan.N),
                         ("v", torch.complex64, plan.M), ("u", torch.float32, 9 * plan.N),
                         ("z", torch.complex128, plan.M)):
            _need(getattr(state, k), dt, n, k)
        if x_true is not None:
            _need(x_true, torch.float32, plan.N, "x_true")
        if W is not None:
            _need(W, torch.float32, 9 * plan.N, "W")
        if block_active is not None:
            _need(block_active, torch.uint8, plan.d, "block_active")
        if basis_active is not None:
            _need(basis_active, torch.uint8, 9, "basis_active")
        if stats_history is not None:
            if stats_every <= 0:
                raise ValueError("stats_history needs stats_every > 0")
            import torch as _t
            if not isinstance(stats_history, _t.Tensor) or not stats_history.is_cuda or \
                    stats_history.dtype != _t.float64 or not stats_history.is_contiguous():
                raise ValueError("stats_history must be a contiguous float64 CUDA tensor")
        self.plan, self.state = plan, state
        self._keep = (y, U, x_true, W, block_active, basis_active, stats_history)
        self._hist_rows = None if stats_history is None else stats_history.numel() // (8 + plan.d)
        self._stats_every = int(stats_every)
        self._eps, ep = _eps_arg(plan, eps)
        self._st = State(_ptr(state.x), _ptr(state.xt), _ptr(state.v), _ptr(state.u), _ptr(state.z), state.iter)
        self._prm = Params(tau, eta, zeta, lam, alpha, mu, n_itr, form, int(use_graph), 0, _ptr(y), _ptr(U), ep,
                           _ptr(x_true), _ptr(W), int(prox), int(n_newton), _ptr(block_active),
                           _ptr(basis_active), int(persistent), int(spin_limit), int(stats_every), 0,
                           _ptr(stats_history))
        self._out = Stats()
        self._res = (c_double * plan.d)()
        self._fn = lib().ppd_iterate

    def run(self, n_iter: int, stats: bool = True):
        """n_iter iterations; returns the last iteration's statistics (or None)."""
        if self._hist_rows is not None and self._hist_rows < n_iter // self._stats_every:
            raise ValueError(f"stats_history holds {self._hist_rows} rows, {n_iter // self._stats_every} needed")
        self._st.iter = self.state.iter
        _check("ppd_iterate", self._fn(self.plan.handle, ctypes.byref(self._st), ctypes.byref(self._prm),
                                       int(n_iter), ctypes.byref(self._out) if stats else None,
                                       self._res if stats else None))
        self.state.iter = int(self._st.iter)
        if not stats:
            return None
        o = self._out
        return {"iter": int(o.iter), "rel_change": o.rel_change, "x_norm": o.x_norm, "snr_db": o.snr_db,
                "residual_max": o.residual_max, "residual": np.array(self._res[:])}


def ppd_iterate(plan: Plan, state: PPDState, y, U, eps, n_iter: int, *, stats: bool = True, **kw):
    """Run n_iter iterations of Algorithm 3; returns a statistics dict (or None).
    Keywords: tau, eta, zeta, lam, alpha, mu, n_itr, form, use_graph, x_true,
    prox, n_newton, block_active, basis_active, W, stats_every, stats_history,
    persistent, spin_limit (see Iteration and ppd_params).  With stats_every > 0 the statistics of every
    stats_every-th iteration are also reduced on the device during the call,
    into stats_history (a float64 tensor of n_iter // stats_every rows of
    8 + d) if given."""
    hist = kw.get("stats_history")
    if hist is not None and kw.get("stats_every", 0) > 0:
        import torch
        _need(hist, torch.float64, (n_iter // kw["stats_every"]) * (8 + plan.d), "stats_history")
    return Iteration(plan, state, y, U, eps, **kw).run(n_iter, stats=stats)


def randomised_ppd(plan: Plan, state: PPDState, y, U, eps, block_masks, basis_masks, **kw):
    """Algorithm 3 with random active sets: iteration t updates the blocks
    with block_masks[t] != 0 and the bases with basis_masks[t] != 0 (HOST
    uint8 arrays T x d and T x 9).  The masks go to two device buffers that
    every call reads, so a captured graph replays with the current draw.
    Returns the statistics of the last iteration."""
    import torch
    bm = np.ascontiguousarray(block_masks, dtype=np.uint8)
    pm = np.ascontiguousarray(basis_masks, dtype=np.uint8)
    if bm.ndim != 2 or bm.shape[1] != plan.d or pm.shape != (bm.shape[0], 9):
        raise ValueError("block_masks must be T x d and basis_masks T x 9")
    dev_b = torch.empty(plan.d, dtype=torch.uint8, device="cuda")
    dev_p = torch.empty(9, dtype=torch.uint8, device="cuda")
    stats = kw.pop("stats", True)
    out = None
    for t in range(bm.shape[0]):
        dev_b.copy_(torch.from_numpy(bm[t]), non_blocking=False)
        dev_p.copy_(torch.from_numpy(pm[t]), non_blocking=False)
        last = t == bm.shape[0] - 1
        out = ppd_iterate(plan, state, y, U, eps, 1, block_active=dev_b, basis_active=dev_p,
                          stats=stats and last, **kw)
    return out


def reweighted_ppd(plan: Plan, state: PPDState, y, U, eps, n_reweights: int, iters_per_solve: int,
                   omega0: float = 1e-2, decay: float = 0.25, x_true=None, **kw):
    """Algorithm 1: solve with Algorithm 3 (warm-started from `state`), then
    omega <- decay * omega and W = omega / (omega + |Psi^H x|), repeated.
    The first solve uses W = I; the weights of solve k come from solve k-1's
    image with omega^(k) = decay^k omega0.  Returns per-solve statistics."""
    import torch
    W = _alloc((9, plan.ny, plan.nx), torch.float32) if n_reweights > 0 else None
    it = Iteration(plan, state, y, U, eps, x_true=x_true, **kw)
    st = (Stats * (n_reweights + 1))()
    it._st.iter = state.iter
    _check("ppd_reweighted", lib().ppd_reweighted(plan.handle, ctypes.byref(it._st), ctypes.byref(it._prm),
                                                   int(n_reweights), int(iters_per_solve), float(omega0),
                                                   float(decay), _ptr(W), st))
    state.iter = int(it._st.iter)
    out = [{"iter": int(o.iter), "rel_change": o.rel_change, "x_norm": o.x_norm, "snr_db": o.snr_db,
            "residual_max": o.residual_max} for o in st]
    return out, W


def kb_weights_host(s, kb_beta: float = 0.0) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.float32)
    w = np.empty((s.size, 8), dtype=np.float32)
    _check("ppd_kb_weights_host", lib().ppd_kb_weights_host(kb_beta, s.size, s.ctypes.data, w.ctypes.data))
    return w


def daubechies_host(p: int) -> np.ndarray:
    h = np.empty(2 * p, dtype=np.float64)
    _check("ppd_daubechies_host", lib().ppd_daubechies_host(p, h.ctypes.data_as(ctypes.POINTER(c_double))))
    return h
