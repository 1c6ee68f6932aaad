"""NTF with HER-accelerated A-HALS on MI355X (gfx950): thin Python binding of libntf.so.

Every function here marshals torch tensors (device memory, current stream) into the C ABI
declared in include/ntf.h and calls it; all arithmetic runs in the library's HIP kernels.
There is no CPU fallback: if libntf.so is missing the import of a call raises.

Functions carry the C names: ntf_norm2, ntf_cast_bf16, ntf_mttkrp, ntf_mttkrp_noalloc,
ntf_mttkrp_multi,
ntf_mttkrp_autotune,
ntf_tune_export, ntf_tune_import, ntf_gram, ntf_hals_update, ntf_pgd_update,
ntf_admm_update, ntf_her_step,
ntf_error,
ntf_solve, ntf_solve_apg, ntf_solve_ibpg, ntf_tucker_mttkrp, ntf_tucker_norm2,
ntf_solve_tucker, ntf_residual_norm2, ntf_cp_loss, ntf_cp_grad,
ntf_solve_batched, plus the
autograd loss `NTFLoss` / `ntf_loss` (module `autograd`) and a JSON file for the tuning
table (`save_tuning`, `load_tuning`).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _abi
from ._abi import NtfError, check, i64_array, lib, ptr_array

__all__ = [
    "Handle", "HerParams", "NtfError", "handle", "ntf_norm2", "ntf_cast_bf16", "ntf_mttkrp",
    "ntf_gram", "ntf_hals_update", "ntf_her_step", "ntf_error", "ntf_solve",
    "ntf_residual_norm2", "ntf_device_flags", "new_state", "state_dict", "ntf_cp_loss",
    "ntf_cp_grad", "NTFLoss", "ntf_loss", "ntf_solve_batched", "ntf_mttkrp_autotune",
    "ntf_tune_export", "ntf_tune_import", "save_tuning", "load_tuning", "ntf_mttkrp_multi",
    "ntf_pgd_update", "ntf_mttkrp_noalloc", "ntf_handle_set_wait_limit", "ntf_admm_update",
    "ntf_solve_apg", "ntf_solve_ibpg", "ntf_tucker_mttkrp", "ntf_tucker_norm2",
    "ntf_solve_tucker", "new_trace",
]

_DTYPES = {torch.float32: _abi.NTF_F32, torch.bfloat16: _abi.NTF_BF16}


class Handle:
    """Owns an ntf_handle on one device (workspace, cached graphs)."""

    def __init__(self, device: int = 0):
        h = C.c_void_p()
        check(lib().ntf_handle_create(C.byref(h), int(device)))
        self.ptr = h
        self.device = int(device)

    def close(self):
        if self.ptr:
            lib().ntf_handle_destroy(self.ptr)
            self.ptr = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_handles: dict[int, Handle] = {}


def handle(device: int | None = None) -> Handle:
    d = torch.cuda.current_device() if device is None else int(device)
    if d not in _handles:
        _handles[d] = Handle(d)
    return _handles[d]


def _stream(stream=None) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype=None) -> int:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


def _tensor_desc(T: torch.Tensor) -> _abi.NtfTensor:
    if T.dtype not in _DTYPES:
        raise ValueError(f"tensor dtype {T.dtype} not supported (float32 or bfloat16)")
    d = _abi.NtfTensor()
    d.order = T.dim()
    d.dtype = _DTYPES[T.dtype]
    for i, s in enumerate(T.shape):
        d.dims[i] = int(s)
    d.data = _dev(T, "T")
    return d


def _h(h):
    return (h or handle()).ptr


@dataclass
class HerParams:
    """HER parameters (defaults of the paper's experiments), the inner stopping rule and the
    block solver: "ahals" (default), "pgd" or "nesterov" (projected gradient steps; these
    run exactly max_inner steps and need inner_tol = 0), "admm" (ADMM steps with the
    stopping rule, max_inner <= 64); the extrapolation scheme: "her" (Algorithm 2) or "bro"
    (Bro's sequence in the block-wise form of Sec. 3.3, no projection)."""
    beta0: float = 0.5
    gamma: float = 1.05
    gamma_bar: float = 1.01
    eta: float = 1.5
    max_inner: int = 50
    inner_tol: float = 1e-2
    inner: str = "ahals"
    scheme: str = "her"

    def to_c(self) -> _abi.NtfHerParams:
        p = _abi.NtfHerParams()
        p.beta0, p.gamma, p.gamma_bar, p.eta = self.beta0, self.gamma, self.gamma_bar, self.eta
        p.max_inner, p.inner_tol = int(self.max_inner), float(self.inner_tol)
        p.inner_solver = {"ahals": 0, "pgd": 1, "nesterov": 2, "admm": 3}[self.inner]
        p.scheme = {"her": 0, "bro": 1}[self.scheme]
        return p


def new_state(device=None) -> torch.Tensor:
    """Device buffer holding one ntf_her_state (opaque bytes)."""
    n = C.sizeof(_abi.NtfHerState)
    return torch.zeros(n, dtype=torch.uint8, device=device or "cuda")


def state_dict(state: torch.Tensor) -> dict:
    raw = bytes(state.cpu().numpy().tobytes())
    s = _abi.NtfHerState.from_buffer_copy(raw)
    return {f: getattr(s, f) for f, _ in _abi.NtfHerState._fields_}


def ntf_norm2(T: torch.Tensor, out: torch.Tensor | None = None, h=None, stream=None):
    out = torch.empty((), dtype=torch.float64, device=T.device) if out is None else out
    d = _tensor_desc(T)
    check(lib().ntf_norm2(_h(h), C.byref(d), _dev(out, "out", torch.float64), _stream(stream)))
    return out


def ntf_cast_bf16(x: torch.Tensor, h=None, stream=None) -> torch.Tensor:
    out = torch.empty(x.shape, dtype=torch.bfloat16, device=x.device)
    check(lib().ntf_cast_bf16(_h(h), _dev(x, "x", torch.float32), out.data_ptr(), x.numel(),
                              _stream(stream)))
    return out


def _check_shape(t: torch.Tensor, shape, name: str) -> None:
    if tuple(t.shape) != tuple(int(x) for x in shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _check_factors(T: torch.Tensor, factors, skip=()) -> int:
    """The factor list matches T (one I_l x r float32 factor per mode, on T's device; modes
    in `skip` may be None) and the common rank r, which is returned. The C ABI receives raw
    pointers, so shapes can only be checked here."""
    factors = list(factors)
    if len(factors) != T.dim():
        raise ValueError(f"{len(factors)} factors for a {T.dim()}-way tensor")
    r = None
    for l, A in enumerate(factors):
        if A is None:
            if l in skip:
                continue
            raise ValueError(f"factor {l} is None")
        if A.dim() != 2:
            raise ValueError(f"factor {l} must be a matrix (I_{l} x r), got {A.dim()} dims")
        if r is None:
            r = int(A.shape[1])
        _check_shape(A, (T.shape[l], r), f"factor {l}")
        if A.device != T.device:
            raise ValueError(f"factor {l} is on {A.device}, the tensor on {T.device}")
    if r is None:
        raise ValueError("no factor given")
    return r


def _mttkrp_args(T, factors, mode, out):
    if not 0 <= int(mode) < T.dim():
        raise ValueError(f"mode {mode} outside [0, {T.dim()})")
    r = _check_factors(T, factors, skip=(int(mode),))
    if out is None:
        out = torch.empty((T.shape[mode], r), dtype=torch.float32, device=T.device)
    _check_shape(out, (T.shape[mode], r), "out")
    d = _tensor_desc(T)
    ptrs = ptr_array([(_dev(A, f"A[{l}]", torch.float32) if (A is not None and l != mode) else None)
                      for l, A in enumerate(factors)])
    return r, out, d, ptrs


def ntf_mttkrp(T: torch.Tensor, factors, mode: int, out: torch.Tensor | None = None, h=None,
               stream=None) -> torch.Tensor:
    r, out, d, ptrs = _mttkrp_args(T, factors, mode, out)
    check(lib().ntf_mttkrp(_h(h), C.byref(d), ptrs, r, int(mode), _dev(out, "P", torch.float32),
                           _stream(stream)))
    return out


def ntf_mttkrp_noalloc(T: torch.Tensor, factors, mode: int, out: torch.Tensor, h=None,
                       stream=None) -> torch.Tensor:
    """ntf_mttkrp without any device allocation in the library (the caller passes `out`)."""
    r, out, d, ptrs = _mttkrp_args(T, factors, mode, out)
    check(lib().ntf_mttkrp_noalloc(_h(h), C.byref(d), ptrs, r, int(mode),
                                   _dev(out, "P", torch.float32), _stream(stream)))
    return out


def ntf_pgd_update(W: torch.Tensor, P: torch.Tensor, G: torch.Tensor, steps: int,
                   accel: bool = False, h=None, stream=None) -> torch.Tensor:
    """Projected-gradient block solver in place on W; returns L = ||G||_2 (device double)."""
    L = torch.empty((), dtype=torch.float64, device=W.device)
    if W.dim() != 2:
        raise ValueError(f"W must be a matrix (I x r), got shape {tuple(W.shape)}")
    rows, r = int(W.shape[0]), int(W.shape[1])
    _check_shape(P, (rows, r), "P")
    _check_shape(G, (r, r), "G")
    check(lib().ntf_pgd_update(_h(h), _dev(W, "W", torch.float32), _dev(P, "P", torch.float32),
                               _dev(G, "G", torch.float32), rows, r, int(steps),
                               1 if accel else 0, L.data_ptr(), _stream(stream)))
    return L


def ntf_admm_update(W: torch.Tensor, P: torch.Tensor, G: torch.Tensor, max_steps: int = 50,
                    tol: float = 1e-2, steps: torch.Tensor | None = None, h=None,
                    stream=None) -> torch.Tensor:
    """ADMM block solver in place on W; returns a device int32 tensor with the steps done."""
    steps = torch.zeros((), dtype=torch.int32, device=W.device) if steps is None else steps
    if W.dim() != 2:
        raise ValueError(f"W must be a matrix (I x r), got shape {tuple(W.shape)}")
    rows, r = W.shape
    _check_shape(P, (rows, r), "P")
    _check_shape(G, (r, r), "G")
    check(lib().ntf_admm_update(_h(h), _dev(W, "W", torch.float32), _dev(P, "P", torch.float32),
                                _dev(G, "G", torch.float32), rows, r, int(max_steps),
                                float(tol), _dev(steps, "steps", torch.int32), _stream(stream)))
    return steps


def ntf_mttkrp_multi(T: torch.Tensor, factors, modes, h=None, stream=None) -> dict:
    """MTTKRPs of several modes with the same factors ({mode: P}); a 3-way tensor's first two
    modes share one pass over T."""
    N = T.dim()
    modes = sorted(set(int(m) for m in modes))
    if not modes or modes[0] < 0 or modes[-1] >= N:
        raise ValueError(f"modes {modes} must be a non-empty subset of [0, {N})")
    skip = (modes[0],) if len(modes) == 1 else ()
    r = _check_factors(T, factors, skip=skip)
    out = {n: torch.empty((T.shape[n], r), dtype=torch.float32, device=T.device) for n in modes}
    d = _tensor_desc(T)
    ptrs = ptr_array([(_dev(A, f"A[{l}]", torch.float32) if A is not None else None)
                      for l, A in enumerate(factors)])
    P = ptr_array([out[n].data_ptr() if n in out else None for n in range(N)])
    mask = sum(1 << n for n in modes)
    check(lib().ntf_mttkrp_multi(_h(h), C.byref(d), ptrs, r, mask, P, _stream(stream)))
    return out


def ntf_mttkrp_autotune(T: torch.Tensor, factors, mode: int, reps: int = 5,
                        out: torch.Tensor | None = None, h=None, stream=None):
    """Time the MTTKRP shapes for this mode and record the fastest in the handle's table.

    Returns (out, {"kernel": 1 row tiles | 2 row slab, "wm": waves along rows, "ms": ...}).
    Synchronizes the stream.
    """
    r, out, d, ptrs = _mttkrp_args(T, factors, mode, out)
    kern, wm, ms = C.c_int32(), C.c_int32(), C.c_float()
    check(lib().ntf_mttkrp_autotune(_h(h), C.byref(d), ptrs, r, int(mode),
                                    _dev(out, "P", torch.float32), int(reps), C.byref(kern),
                                    C.byref(wm), C.byref(ms), _stream(stream)))
    return out, {"kernel": kern.value, "wm": wm.value, "ms": ms.value}


def ntf_tune_export(h=None) -> str:
    """The handle's tuning table as text ("<key> <kernel> <wm>" per line)."""
    n = lib().ntf_tune_export(_h(h), None, 0)
    if n < 0:
        raise NtfError(1, "handle is NULL")
    buf = C.create_string_buffer(int(n))
    lib().ntf_tune_export(_h(h), buf, int(n))
    return buf.value.decode()


def ntf_tune_import(text: str, h=None) -> None:
    check(lib().ntf_tune_import(_h(h), text.encode()))


def save_tuning(path: str, h=None) -> None:
    """Write the handle's tuning table to a JSON file {key: [kernel, wm]}."""
    import json
    table = {}
    for ln in ntf_tune_export(h).splitlines():
        k, kern, wm = ln.split()
        table[k] = [int(kern), int(wm)]
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load_tuning(path: str, h=None) -> None:
    """Add the entries of a JSON file written by save_tuning to the handle's table."""
    import json
    with open(path) as f:
        table = json.load(f)
    ntf_tune_import("".join(f"{k} {int(v[0])} {int(v[1])}\n" for k, v in table.items()), h)


def ntf_gram(factors, exclude: int = -1, want32: bool = True, want64: bool = True, h=None,
             stream=None):
    factors = list(factors)
    if not factors or not -1 <= int(exclude) < len(factors):
        raise ValueError(f"exclude {exclude} outside [-1, {len(factors)})")
    r = int(factors[0].shape[1]) if exclude != 0 else int(factors[-1].shape[1])
    for l, A in enumerate(factors):
        if A.dim() != 2 or int(A.shape[1]) != r:
            raise ValueError(f"factor {l} has shape {tuple(A.shape)}; every factor needs r = {r} "
                             "columns")
    dev = factors[0].device
    G32 = torch.empty((r, r), dtype=torch.float32, device=dev) if want32 else None
    G64 = torch.empty((r, r), dtype=torch.float64, device=dev) if want64 else None
    ptrs = ptr_array([_dev(A, f"A[{l}]", torch.float32) for l, A in enumerate(factors)])
    rows = i64_array([A.shape[0] for A in factors])
    check(lib().ntf_gram(_h(h), ptrs, rows, len(factors), r, int(exclude),
                         G32.data_ptr() if G32 is not None else None,
                         G64.data_ptr() if G64 is not None else None, _stream(stream)))
    return G32, G64


def ntf_hals_update(W: torch.Tensor, P: torch.Tensor, G: torch.Tensor, max_sweeps: int = 50,
                    tol: float = 1e-2, sweeps: torch.Tensor | None = None, h=None, stream=None):
    """In-place A-HALS on W; returns a device int32 tensor with the sweeps done."""
    sweeps = torch.zeros((), dtype=torch.int32, device=W.device) if sweeps is None else sweeps
    if W.dim() != 2:
        raise ValueError(f"W must be a matrix (I x r), got shape {tuple(W.shape)}")
    rows, r = W.shape
    _check_shape(P, (rows, r), "P")
    _check_shape(G, (r, r), "G")
    if sweeps.numel() < 1:
        raise ValueError("sweeps must hold one int32")
    check(lib().ntf_hals_update(_h(h), _dev(W, "W", torch.float32), _dev(P, "P", torch.float32),
                                _dev(G, "G", torch.float32), rows, r, int(max_sweeps),
                                float(tol), _dev(sweeps, "sweeps", torch.int32),
                                _stream(stream)))
    return sweeps


def ntf_her_step(op: int, state: torch.Tensor, params: HerParams | None = None, A=(),
                 A_new=(), A_hat=(), block: int = 0, fhat: torch.Tensor | None = None,
                 h=None, stream=None):
    p = (params or HerParams()).to_c()
    nb = len(A)
    r = int(A[0].shape[1]) if nb else 1
    if nb and (len(A_new) != nb or len(A_hat) != nb):
        raise ValueError("A, A_new and A_hat need one entry per block")
    for b in range(nb):
        for nm, X in (("A", A[b]), ("A_new", A_new[b]), ("A_hat", A_hat[b])):
            _check_shape(X, (A[b].shape[0], r), f"{nm}[{b}]")
    if nb and not 0 <= int(block) < nb:
        raise ValueError(f"block {block} outside [0, {nb})")
    if state.numel() < C.sizeof(_abi.NtfHerState):
        raise ValueError("state buffer is smaller than one ntf_her_state")
    rows = i64_array([a.shape[0] for a in A]) if nb else None
    pa = ptr_array([_dev(a, "A", torch.float32) for a in A]) if nb else None
    pn = ptr_array([_dev(a, "A_new", torch.float32) for a in A_new]) if nb else None
    ph = ptr_array([_dev(a, "A_hat", torch.float32) for a in A_hat]) if nb else None
    check(lib().ntf_her_step(_h(h), int(op), _dev(state, "state"), C.byref(p), nb, rows, r,
                             pa, pn, ph, int(block),
                             _dev(fhat, "fhat", torch.float64) if fhat is not None else None,
                             _stream(stream)))


def ntf_error(normT2: torch.Tensor, P: torch.Tensor, A: torch.Tensor, G64: torch.Tensor,
              out: torch.Tensor | None = None, h=None, stream=None) -> torch.Tensor:
    out = torch.empty((), dtype=torch.float64, device=P.device) if out is None else out
    rows, r = A.shape
    _check_shape(P, (rows, r), "P")
    _check_shape(G64, (r, r), "G64")
    check(lib().ntf_error(_h(h), _dev(normT2, "normT2", torch.float64),
                          _dev(P, "P", torch.float32), _dev(A, "A", torch.float32),
                          _dev(G64, "G", torch.float64), rows, r, _dev(out, "fhat", torch.float64),
                          _stream(stream)))
    return out


def ntf_cp_loss(normT2: torch.Tensor, P: torch.Tensor, A: torch.Tensor, G64: torch.Tensor,
                out: torch.Tensor | None = None, h=None, stream=None) -> torch.Tensor:
    """||T - [[A]]||^2 by the float64 Gram trick from one mode's P, A and G (no 1/2)."""
    out = torch.empty((), dtype=torch.float64, device=P.device) if out is None else out
    rows, r = A.shape
    _check_shape(P, (rows, r), "P")
    _check_shape(G64, (r, r), "G64")
    check(lib().ntf_cp_loss(_h(h), _dev(normT2, "normT2", torch.float64),
                            _dev(P, "P", torch.float32), _dev(A, "A", torch.float32),
                            _dev(G64, "G", torch.float64), rows, r,
                            _dev(out, "loss", torch.float64), _stream(stream)))
    return out


def ntf_cp_grad(A: torch.Tensor, P: torch.Tensor, G64: torch.Tensor,
                scale: torch.Tensor | None = None, alpha: float = 2.0,
                out: torch.Tensor | None = None, h=None, stream=None) -> torch.Tensor:
    """alpha * scale * (A G - P): the loss gradient for one factor (scale: device double)."""
    out = torch.empty_like(A) if out is None else out
    rows, r = A.shape
    _check_shape(P, (rows, r), "P")
    _check_shape(G64, (r, r), "G64")
    _check_shape(out, (rows, r), "out")
    check(lib().ntf_cp_grad(_h(h), _dev(A, "A", torch.float32), _dev(P, "P", torch.float32),
                            _dev(G64, "G", torch.float64), rows, r,
                            _dev(scale, "scale", torch.float64) if scale is not None else None,
                            float(alpha), _dev(out, "grad", torch.float32), _stream(stream)))
    return out


def ntf_residual_norm2(T: torch.Tensor, factors, h=None, stream=None) -> torch.Tensor:
    out = torch.empty((), dtype=torch.float64, device=T.device)
    r = _check_factors(T, factors)
    d = _tensor_desc(T)
    ptrs = ptr_array([_dev(A, f"A[{l}]", torch.float32) for l, A in enumerate(factors)])
    check(lib().ntf_residual_norm2(_h(h), C.byref(d), ptrs, r,
                                   out.data_ptr(), _stream(stream)))
    return out


def ntf_solve(T: torch.Tensor, factors, iters: int, params: HerParams | None = None,
              state: torch.Tensor | None = None, resume: bool = False, trace=True,
              h=None, stream=None):
    """Run `iters` HER outer iterations in place on `factors` (list of float32 tensors).

    trace: True (new buffers), a dict from new_trace (reused), or False. Returns
    (state, trace) where trace is a dict of device tensors (or None).
    """
    p = (params or HerParams()).to_c()
    N = T.dim()
    r = _check_factors(T, factors)
    dev = T.device
    if state is None:
        state = new_state(dev)
    if state.numel() < C.sizeof(_abi.NtfHerState):
        raise ValueError("state buffer is smaller than one ntf_her_state")
    tr, ctr = _trace_buffers(trace, iters, N, dev)
    d = _tensor_desc(T)
    ptrs = ptr_array([_dev(A, f"A[{l}]", torch.float32) for l, A in enumerate(factors)])
    check(lib().ntf_solve(_h(h), C.byref(d), r, ptrs, C.byref(p), int(iters),
                          _dev(state, "state"), 1 if resume else 0,
                          C.byref(ctr) if ctr is not None else None, _stream(stream)))
    return state, tr


def _tucker_desc(core: torch.Tensor, bases, dims=None) -> _abi.NtfTucker:
    """Descriptor of T = (U^(1) (x) ... (x) U^(N)) core (float32 core, bases n_p x r_p)."""
    bases = list(bases)
    if core.dtype != torch.float32:
        raise ValueError("the Tucker core must be float32")
    if len(bases) != core.dim():
        raise ValueError(f"{len(bases)} bases for a {core.dim()}-way core")
    X = _abi.NtfTucker()
    X.core = _tensor_desc(core)
    for p, U in enumerate(bases):
        if U.dim() != 2 or int(U.shape[1]) != int(core.shape[p]):
            raise ValueError(f"basis {p} has shape {tuple(U.shape)}; it needs "
                             f"{int(core.shape[p])} columns")
        X.U[p] = _dev(U, f"U[{p}]", torch.float32)
        X.dims[p] = int(U.shape[0])
    return X


def _tucker_factors(X: _abi.NtfTucker, core, factors, skip=()) -> int:
    factors = list(factors)
    if len(factors) != core.dim():
        raise ValueError(f"{len(factors)} factors for a {core.dim()}-way tensor")
    r = None
    for l, A in enumerate(factors):
        if A is None and l in skip:
            continue
        if A is None or A.dim() != 2:
            raise ValueError(f"factor {l} must be a matrix")
        r = int(A.shape[1]) if r is None else r
        _check_shape(A, (X.dims[l], r), f"factor {l}")
    return r


def ntf_tucker_mttkrp(core: torch.Tensor, bases, factors, mode: int,
                      out: torch.Tensor | None = None, h=None, stream=None) -> torch.Tensor:
    """MTTKRP of mode `mode` of the Tucker-format tensor (Appendix A); T is never formed."""
    X = _tucker_desc(core, bases)
    if not 0 <= int(mode) < core.dim():
        raise ValueError(f"mode {mode} outside [0, {core.dim()})")
    r = _tucker_factors(X, core, factors, skip=(int(mode),))
    if out is None:
        out = torch.empty((X.dims[mode], r), dtype=torch.float32, device=core.device)
    _check_shape(out, (X.dims[mode], r), "out")
    ptrs = ptr_array([(_dev(A, f"A[{l}]", torch.float32) if (A is not None and l != mode) else None)
                      for l, A in enumerate(factors)])
    check(lib().ntf_tucker_mttkrp(_h(h), C.byref(X), ptrs, r, int(mode),
                                  _dev(out, "P", torch.float32), _stream(stream)))
    return out


def ntf_tucker_norm2(core: torch.Tensor, bases, h=None, stream=None) -> torch.Tensor:
    out = torch.empty((), dtype=torch.float64, device=core.device)
    X = _tucker_desc(core, bases)
    check(lib().ntf_tucker_norm2(_h(h), C.byref(X), out.data_ptr(), _stream(stream)))
    return out


def ntf_solve_tucker(core: torch.Tensor, bases, factors, iters: int,
                     params: HerParams | None = None, state: torch.Tensor | None = None,
                     resume: bool = False, trace=True, h=None, stream=None):
    """ntf_solve on a Tucker-format tensor (Appendix A); returns (state, trace)."""
    p = (params or HerParams()).to_c()
    X = _tucker_desc(core, bases)
    r = _tucker_factors(X, core, factors)
    N = core.dim()
    dev = core.device
    if state is None:
        state = new_state(dev)
    tr, ctr = _trace_buffers(trace, iters, N, dev)
    ptrs = ptr_array([_dev(A, f"A[{l}]", torch.float32) for l, A in enumerate(factors)])
    check(lib().ntf_solve_tucker(_h(h), C.byref(X), r, ptrs, C.byref(p), int(iters),
                                 _dev(state, "state"), 1 if resume else 0,
                                 C.byref(ctr) if ctr is not None else None, _stream(stream)))
    return state, tr


def new_trace(iters: int, order: int, device=None) -> dict:
    """Device buffers for the trace of up to `iters` outer iterations of an order-`order`
    problem. Passing the same dict (and state) to successive ntf_solve calls keeps their
    arguments equal, so the captured iteration graph is reused instead of captured again."""
    dev = device or "cuda"
    return dict(fhat=torch.zeros(iters, dtype=torch.float64, device=dev),
                beta=torch.zeros(iters, dtype=torch.float64, device=dev),
                beta_bar=torch.zeros(iters, dtype=torch.float64, device=dev),
                restart=torch.zeros(iters, dtype=torch.int32, device=dev),
                sweeps=torch.zeros((iters, order), dtype=torch.int32, device=dev))


def _trace_buffers(trace, iters: int, N: int, dev):
    """(trace dict, ntf_trace) for trace=True (new buffers), a dict from new_trace (reused;
    the call writes its first `iters` entries), or False/None (no trace)."""
    if not trace or iters <= 0:
        return None, None
    if isinstance(trace, dict):
        tr = trace
        if tr["fhat"].numel() < iters or tuple(tr["sweeps"].shape[1:]) != (N,):
            raise ValueError(f"trace buffers hold {tr['fhat'].numel()} iterations of order "
                             f"{tuple(tr['sweeps'].shape[1:])}; need {iters} of order {N}")
        for k, dt in (("fhat", torch.float64), ("beta", torch.float64),
                      ("beta_bar", torch.float64), ("restart", torch.int32),
                      ("sweeps", torch.int32)):
            _dev(tr[k], f"trace[{k}]", dt)
    else:
        tr = new_trace(iters, N, dev)
    ctr = _abi.NtfTrace(tr["fhat"].data_ptr(), tr["beta"].data_ptr(),
                        tr["beta_bar"].data_ptr(), tr["restart"].data_ptr(),
                        tr["sweeps"].data_ptr())
    return tr, ctr


def ntf_solve_apg(T: torch.Tensor, factors, iters: int, delta_w: float = 0.9999, h=None,
                  stream=None):
    """APG (the paper's comparison method, Sec. 2.2.1) in place on `factors`; synchronous.
    Returns (objective per iteration, restart flags) as numpy arrays."""
    import numpy as np
    r = _check_factors(T, factors)
    d = _tensor_desc(T)
    ptrs = ptr_array([_dev(A, f"A[{l}]", torch.float32) for l, A in enumerate(factors)])
    obj = np.zeros(max(iters, 1), dtype=np.float64)
    rst = np.zeros(max(iters, 1), dtype=np.int32)
    check(lib().ntf_solve_apg(_h(h), C.byref(d), r, ptrs, int(iters), float(delta_w),
                              obj.ctypes.data, rst.ctypes.data, _stream(stream)))
    return obj[:iters], rst[:iters].astype(bool)


def ntf_solve_ibpg(T: torch.Tensor, factors, iters: int, inner_steps: int = 50,
                   delta_w: float = 0.99, beta: float = 1.01, h=None, stream=None):
    """iBPG (the paper's comparison method, Sec. 2.2.2) in place on `factors`; synchronous.
    Returns the objective after each outer iteration (numpy)."""
    import numpy as np
    r = _check_factors(T, factors)
    d = _tensor_desc(T)
    ptrs = ptr_array([_dev(A, f"A[{l}]", torch.float32) for l, A in enumerate(factors)])
    obj = np.zeros(max(iters, 1), dtype=np.float64)
    check(lib().ntf_solve_ibpg(_h(h), C.byref(d), r, ptrs, int(iters), int(inner_steps),
                               float(delta_w), float(beta), obj.ctypes.data, _stream(stream)))
    return obj[:iters]


def ntf_solve_batched(tensors, factors, iters: int, params: HerParams | None = None,
                      states: torch.Tensor | None = None, resume: bool = False,
                      trace: bool = True, h=None, stream=None):
    """Algorithm 2 on many independent 3-way float32 problems in one persistent launch.

    tensors: list of float32 device tensors (I1, I2, I3); factors: list of [A1, A2, A3]
    (float32, I_n x r) updated in place. states: device uint8 tensor of
    len(tensors) * sizeof(ntf_her_state) bytes (allocated when None). Returns
    (states, trace) with trace = dict(fhat [B, iters], restart [B, iters],
    sweeps [B, iters, 3]) of device tensors, or None.
    """
    p = (params or HerParams()).to_c()
    B = len(tensors)
    if len(factors) != B:
        raise ValueError("one factor list per tensor")
    dev = tensors[0].device
    ss = C.sizeof(_abi.NtfHerState)
    if states is None:
        states = torch.zeros(B * ss, dtype=torch.uint8, device=dev)
    tr = None
    if trace and iters > 0:
        tr = dict(fhat=torch.zeros((B, iters), dtype=torch.float64, device=dev),
                  restart=torch.zeros((B, iters), dtype=torch.int32, device=dev),
                  sweeps=torch.zeros((B, iters, 3), dtype=torch.int32, device=dev))
    arr = (_abi.NtfProblem * B)()
    if states.numel() < B * ss:
        raise ValueError(f"states holds {states.numel()} bytes, {B} problems need {B * ss}")
    for b, (T, A) in enumerate(zip(tensors, factors)):
        if T.dim() != 3:
            raise ValueError(f"problem {b}: the batched solver takes 3-way tensors")
        q = arr[b]
        q.T = _tensor_desc(T)
        q.r = _check_factors(T, A)
        q.reserved = 0
        for n in range(3):
            q.A[n] = _dev(A[n], f"A[{b}][{n}]", torch.float32)
        q.state = states.data_ptr() + b * ss
        if tr is not None:
            q.trace_fhat = tr["fhat"][b].data_ptr()
            q.trace_restart = tr["restart"][b].data_ptr()
            q.trace_sweeps = tr["sweeps"][b].data_ptr()
    check(lib().ntf_solve_batched(_h(h), B, arr, C.byref(p), int(iters), 1 if resume else 0,
                                  _stream(stream)))
    return states, tr


def batched_state_dict(states: torch.Tensor, b: int) -> dict:
    ss = C.sizeof(_abi.NtfHerState)
    return state_dict(states[b * ss:(b + 1) * ss])


def ntf_device_flags(h=None, stream=None) -> int:
    v = C.c_uint32()
    check(lib().ntf_device_flags(_h(h), _stream(stream), C.byref(v)))
    return int(v.value)


def ntf_handle_set_wait_limit(seconds: float, h=None) -> None:
    """Time after which the A-HALS kernel's cross-workgroup waits give up (default 2 s)."""
    check(lib().ntf_handle_set_wait_limit(_h(h), float(seconds)))


from .autograd import NTFLoss, ntf_loss  # noqa: E402
