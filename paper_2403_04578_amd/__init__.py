"""MI355X batched fixed-point power flow (tensor power flow, arXiv 2403.04578).

Thin Python binding over ``libtpf.so``: it only marshals arguments.  Every step
of the solve runs in the library's HIP kernels; PyTorch supplies device memory
and the current stream.  There is no CPU fallback: if the library is missing the
import of a solve fails with an error that says how to build it.

    net = Network.from_feeder(workloads.make_feeder(100))
    V, iters, status = solve_timeseries(net, S_cuda, tol=1e-6, max_iter=100)
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtpf.so")

TPF_OK = 0
TPF_ERR_INVALID_ARG = -1
TPF_ERR_SINGULAR = -2
TPF_ERR_DEVICE = -3
TPF_ERR_OOM = -4
TPF_ERR_UNSUPPORTED = -5

TPF_C64, TPF_C128 = 0, 1
MODE_FP64, MODE_FP32, MODE_MIXED_BF16, MODE_MIXED_FP16, MODE_TREE_FP64, MODE_TREE_FP32 = 0, 1, 2, 3, 4, 5
ST_CONVERGED, ST_MAX_ITER, ST_NONFINITE = 0, 1, 2

_MODES = {"fp64": MODE_FP64, "fp32": MODE_FP32, "mixed_bf16": MODE_MIXED_BF16, "mixed_fp16": MODE_MIXED_FP16,
          "tree_fp64": MODE_TREE_FP64, "tree_fp32": MODE_TREE_FP32}


class TpfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tpf error {code}: {msg}")
        self.code = code


class _Options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("V0", ctypes.c_void_p),
                ("mismatch_out", ctypes.c_void_p), ("warm_start", ctypes.c_void_p), ("t_index", ctypes.c_void_p),
                ("reserved1", ctypes.c_double * 2)]


_lib = None


def load_library() -> ctypes.CDLL:
    """Loads libtpf.so (built in-tree by ``python -m paper_2403_04578_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_2403_04578_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "tpf_build_network": (ctypes.c_int, [I32, I32, P, P, P, P, I32, D, D, ctypes.POINTER(P)]),
        "tpf_build_network_zip": (ctypes.c_int, [I32, I32, P, P, P, P, I32, D, D, P, P, P, ctypes.POINTER(P)]),
        "tpf_build_network_3ph": (ctypes.c_int, [I32, I32, P, P, P, I32, P, ctypes.POINTER(P)]),
        "tpf_free_network": (None, [P]),
        "tpf_network_n_pq": (ctypes.c_int, [P]),
        "tpf_network_get_zw": (ctypes.c_int, [P, P, P]),
        "tpf_workspace_bytes": (ctypes.c_size_t, [P, I64, P]),
        "tpf_solve_timeseries": (ctypes.c_int, [P, P, I32, I64, D, I32, P, P, P, P, P, ctypes.c_size_t, P]),
        "tpf_solve_tensor": (ctypes.c_int, [P, P, I32, I64, I64, D, I32, P, P, P, P, P, ctypes.c_size_t, P]),
        "tpf_solve_timeseries_noalloc": (ctypes.c_int, [P, P, I32, I64, D, I32, P, P, P, P, P]),
        "tpf_mismatch": (ctypes.c_int, [P, P, P, I32, I64, P, P]),
        "tpf_last_error": (ctypes.c_char_p, []),
        "tpf_mlp_create": (ctypes.c_int, [I32, I32, I32, P, D, D, ctypes.POINTER(P)]),
        "tpf_mlp_free": (None, [P]),
        "tpf_mlp_num_params": (I64, [P]),
        "tpf_mlp_get_params": (ctypes.c_int, [P, P]),
        "tpf_mlp_set_params": (ctypes.c_int, [P, P]),
        "tpf_mlp_workspace_bytes": (ctypes.c_size_t, [P, I64]),
        "tpf_mlp_loss_grad": (ctypes.c_int, [P, P, I32, P, P, I64, P, P, P, ctypes.c_size_t, P]),
        "tpf_mlp_train_step": (ctypes.c_int, [P, P, I32, P, P, I64, ctypes.c_float, ctypes.c_float, P, P,
                                              ctypes.c_size_t, P]),
        "tpf_mlp_train": (ctypes.c_int, [P, P, I32, P, P, I64, I32, I32, I32, I32, ctypes.c_float,
                                         ctypes.c_float, ctypes.c_float, ctypes.c_uint64, P, P,
                                         ctypes.c_size_t, P]),
        "tpf_mlp_predict": (ctypes.c_int, [P, P, I32, P, I64, P, P, ctypes.c_size_t, P]),
        "tpf_mlp_save": (ctypes.c_int, [P, ctypes.c_char_p]),
        "tpf_mlp_load": (ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(P)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != TPF_OK:
        raise TpfError(rc, load_library().tpf_last_error().decode())


class Network:
    """A feeder prepared for the sweeps: Z = -Y_dd^-1 and w (Sec. II Eqs. (1)-(2)).

    With alpha_i / alpha_p (per PQ bus, or scalars) the loads follow Eq. (2)'s ZIP model
    with constant-current and constant-power shares; a non-zero constant-impedance share
    alpha_z makes B = diag(alpha_Z s*) + Y_dd differ per column, which the tree modes
    eliminate along the tree (radial, single-phase networks) and the dense modes carry as
    the current alpha_Z conj(S) V in the injection (the same fixed point)."""

    def __init__(self, n_bus: int, frm, to, r, x, slack: int = 0, vs: complex = 1.0 + 0.0j,
                 alpha_i=None, alpha_p=None, alpha_z=None):
        lib = load_library()
        self._keep = [np.ascontiguousarray(frm, np.int32), np.ascontiguousarray(to, np.int32),
                      np.ascontiguousarray(r, np.float64), np.ascontiguousarray(x, np.float64)]
        h = ctypes.c_void_p()
        f, t, rr, xx = self._keep
        if not (len(f) == len(t) == len(rr) == len(xx)):
            raise ValueError("branch arrays must have equal lengths")
        self.zip = alpha_i is not None or alpha_p is not None or alpha_z is not None
        if self.zip:
            n = int(n_bus) - 1
            shares = [np.ascontiguousarray(np.broadcast_to(np.asarray(a if a is not None else d, np.float64), (n,)))
                      for a, d in ((alpha_z, 0.0), (alpha_i, 0.0), (alpha_p, 1.0))]
            self._keep += shares
            rc = lib.tpf_build_network_zip(int(n_bus), len(f), f.ctypes.data, t.ctypes.data, rr.ctypes.data,
                                           xx.ctypes.data, int(slack), float(np.real(vs)), float(np.imag(vs)),
                                           shares[0].ctypes.data, shares[1].ctypes.data, shares[2].ctypes.data,
                                           ctypes.byref(h))
        else:
            rc = lib.tpf_build_network(int(n_bus), len(f), f.ctypes.data, t.ctypes.data, rr.ctypes.data,
                                       xx.ctypes.data, int(slack), float(np.real(vs)), float(np.imag(vs)),
                                       ctypes.byref(h))
        _check(rc)
        self._h = h
        self.n_bus = int(n_bus)
        self.n = lib.tpf_network_n_pq(h)

    @classmethod
    def three_phase(cls, n_bus: int, frm, to, zabc, slack: int = 0, vs_abc=None) -> "Network":
        """Three-phase network (Eq. (1) per phase node): zabc [n_branch, 3, 3] complex
        series impedance matrices, vs_abc the slack phase voltages (balanced by default).
        Demand node 3 k + p is phase p of the k-th non-slack bus."""
        lib = load_library()
        self = cls.__new__(cls)
        f, t = np.ascontiguousarray(frm, np.int32), np.ascontiguousarray(to, np.int32)
        z = np.ascontiguousarray(np.asarray(zabc, np.complex128).reshape(len(f), 3, 3))
        if vs_abc is None:
            vs_abc = np.exp(-2j * np.pi / 3 * np.arange(3))
        v = np.ascontiguousarray(np.asarray(vs_abc, np.complex128).reshape(3))
        if len(f) != len(t):
            raise ValueError("branch arrays must have equal lengths")
        self._keep = [f, t, z, v]
        h = ctypes.c_void_p()
        _check(lib.tpf_build_network_3ph(int(n_bus), len(f), f.ctypes.data, t.ctypes.data, z.ctypes.data,
                                         int(slack), v.ctypes.data, ctypes.byref(h)))
        self._h = h
        self.zip = False
        self.n_bus = int(n_bus)
        self.n = lib.tpf_network_n_pq(h)
        return self

    @classmethod
    def from_feeder_3ph(cls, feeder) -> "Network":
        return cls.three_phase(feeder.n_bus, feeder.frm, feeder.to, feeder.zabc, 0, feeder.vs_abc)

    @classmethod
    def from_feeder(cls, feeder, alpha_i=None, alpha_p=None, alpha_z=None) -> "Network":
        return cls(feeder.n_bus, feeder.frm, feeder.to, feeder.r, feeder.x, 0, feeder.vs, alpha_i, alpha_p, alpha_z)

    @property
    def handle(self):
        return self._h

    def zw(self):
        """(Z, w) as complex128 numpy arrays, copied out of the handle."""
        Z = np.empty((self.n, self.n), np.complex128)
        w = np.empty(self.n, np.complex128)
        _check(load_library().tpf_network_get_zw(self._h, Z.ctypes.data, w.ctypes.data))
        return Z, w

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tpf_free_network(h)
            self._h = None


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.complex128:
        return TPF_C128
    if t.dtype == torch.complex64:
        return TPF_C64
    raise TypeError("S must be complex64 or complex128")


def _stream_ptr(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def workspace_bytes(net: Network, tau: int, mode: int = MODE_FP64, warm_start=None) -> int:
    o = _Options(mode=_MODES[mode] if isinstance(mode, str) else int(mode))
    if warm_start is not None:
        o.warm_start = warm_start.handle.value
    return int(load_library().tpf_workspace_bytes(net.handle, int(tau), ctypes.byref(o)))


def solve_timeseries(net: Network, S, tol: float, max_iter: int, mode="fp64", V0=None,
                     mismatch: bool = False, out=None, warm_start=None, t_index=None):
    """Algorithm 1 over S [T, n] (CUDA complex tensor).  Returns (V, iters, status[, mismatch]).

    ``mode``: "fp64" | "fp32" | "mixed_bf16" | "mixed_fp16" | "tree_fp64" | "tree_fp32" (or the MODE_* ints).
    ``V0``: optional start voltages [T, n] (same dtype); guarded columns fall back to flat.
    ``warm_start``: a :class:`WarmStart` evaluated by the solve itself (instead of V0), with
    ``t_index`` (int64 [T] minute indices, default: the column index) for its calendar features.
    """
    return _solve(net, S, tol, max_iter, mode, V0, mismatch, out, tensor=False, warm_start=warm_start,
                  t_index=t_index)


def solve_tensor(net: Network, S, tol: float, max_iter: int, mode="fp64", V0=None,
                 mismatch: bool = False, out=None, warm_start=None, t_index=None):
    """Algorithm 1 over S [P, T, n]; outputs shaped [P, T, n], [P, T]."""
    return _solve(net, S, tol, max_iter, mode, V0, mismatch, out, tensor=True, warm_start=warm_start,
                  t_index=t_index)


def _solve(net, S, tol, max_iter, mode, V0, mismatch, out, tensor, warm_start=None, t_index=None):
    torch = _torch()
    lib = load_library()
    if not S.is_cuda:
        raise ValueError("S must be a device tensor")
    if not S.is_contiguous():
        raise ValueError("S must be contiguous")
    mode_i = _MODES[mode] if isinstance(mode, str) else int(mode)
    dt = _dtype_code(S)
    if tensor:
        if S.dim() != 3 or S.shape[2] != net.n:
            raise ValueError(f"S must be [P, T, {net.n}]")
        lead = tuple(S.shape[:2])
    else:
        if S.dim() != 2 or S.shape[1] != net.n:
            raise ValueError(f"S must be [T, {net.n}]")
        lead = (S.shape[0],)
    tau = int(np.prod(lead)) if lead else 0
    dev = S.device
    if out is None:
        V = torch.empty_like(S)
        iters = torch.empty(lead, dtype=torch.int32, device=dev)
        status = torch.empty(lead, dtype=torch.int8, device=dev)
        mm = torch.empty(lead, dtype=torch.float64, device=dev) if mismatch else None
        ws = torch.empty(max(workspace_bytes(net, tau, mode_i, warm_start), 256), dtype=torch.uint8, device=dev)
    else:
        V, iters, status, mm, ws = out
    opts = _Options(mode=mode_i)
    if warm_start is not None:
        opts.warm_start = warm_start.handle.value
        if t_index is not None:
            if t_index.dtype != torch.int64 or t_index.numel() != tau or not t_index.is_contiguous() \
                    or t_index.device != dev:
                raise ValueError("t_index must be a contiguous int64 tensor with one entry per column")
            opts.t_index = t_index.data_ptr()
    if V0 is not None:
        if V0.shape != S.shape or V0.dtype != S.dtype or not V0.is_contiguous() or V0.device != dev:
            raise ValueError("V0 must match S in shape, dtype and device and be contiguous")
        opts.V0 = V0.data_ptr()
    if mismatch:
        opts.mismatch_out = mm.data_ptr()
    with torch.cuda.device(dev):
        stream = _stream_ptr(dev)
        if tensor:
            rc = lib.tpf_solve_tensor(net.handle, S.data_ptr(), dt, lead[0], lead[1], float(tol), int(max_iter),
                                      ctypes.byref(opts), V.data_ptr(), iters.data_ptr(), status.data_ptr(),
                                      ws.data_ptr(), ws.numel(), stream)
        else:
            rc = lib.tpf_solve_timeseries(net.handle, S.data_ptr(), dt, tau, float(tol), int(max_iter),
                                          ctypes.byref(opts), V.data_ptr(), iters.data_ptr(), status.data_ptr(),
                                          ws.data_ptr(), ws.numel(), stream)
    _check(rc)
    if mismatch:
        return V, iters, status, mm
    return V, iters, status


def solve_timeseries_noalloc(net: Network, S, tol: float, max_iter: int, mode="fp64", V0=None, out=None,
                             mismatch: bool = False):
    """tpf_solve_timeseries_noalloc: the solve without a workspace (the library's static
    scratch; the network must already be resident on S's device).  ``out`` = (V, iters,
    status[, mismatch]) preallocated by the caller, or None (allocated here by torch)."""
    torch = _torch()
    lib = load_library()
    if not S.is_cuda or not S.is_contiguous() or S.dim() != 2 or S.shape[1] != net.n:
        raise ValueError(f"S must be a contiguous device tensor [T, {net.n}]")
    T = S.shape[0]
    dev = S.device
    if out is None:
        out = (torch.empty_like(S), torch.empty(T, dtype=torch.int32, device=dev),
               torch.empty(T, dtype=torch.int8, device=dev),
               torch.empty(T, dtype=torch.float64, device=dev) if mismatch else None)
    V, iters, status, mm = (tuple(out) + (None,))[:4]
    opts = _Options(mode=_MODES[mode] if isinstance(mode, str) else int(mode))
    if V0 is not None:
        opts.V0 = V0.data_ptr()
    if mm is not None:
        opts.mismatch_out = mm.data_ptr()
    with torch.cuda.device(dev):
        rc = lib.tpf_solve_timeseries_noalloc(net.handle, S.data_ptr(), _dtype_code(S), T, float(tol), int(max_iter),
                                              ctypes.byref(opts), V.data_ptr(), iters.data_ptr(), status.data_ptr(),
                                              _stream_ptr(dev))
    _check(rc)
    return (V, iters, status, mm) if mm is not None else (V, iters, status)


def alloc_outputs(net: Network, S, mode="fp64", mismatch: bool = False, tensor: bool = False, warm_start=None):
    """Pre-allocates (V, iters, status, mismatch, workspace) for repeated solves of S's shape."""
    torch = _torch()
    lead = tuple(S.shape[:2]) if tensor else (S.shape[0],)
    tau = int(np.prod(lead))
    mode_i = _MODES[mode] if isinstance(mode, str) else int(mode)
    dev = S.device
    return (torch.empty_like(S), torch.empty(lead, dtype=torch.int32, device=dev),
            torch.empty(lead, dtype=torch.int8, device=dev),
            torch.empty(lead, dtype=torch.float64, device=dev) if mismatch else None,
            torch.empty(max(workspace_bytes(net, tau, mode_i, warm_start), 256), dtype=torch.uint8, device=dev))


def mismatch(net: Network, S, V):
    """FP64 power-balance mismatch per column: max_i |S + V .* conj(Y_ds v_s + Y_dd V)|."""
    torch = _torch()
    lib = load_library()
    if S.shape != V.shape or S.dtype != V.dtype:
        raise ValueError("S and V must match")
    lead = tuple(S.shape[:-1])
    tau = int(np.prod(lead))
    out = torch.empty(lead, dtype=torch.float64, device=S.device)
    with torch.cuda.device(S.device):
        rc = lib.tpf_mismatch(net.handle, S.data_ptr(), V.data_ptr(), _dtype_code(S), tau, out.data_ptr(),
                              _stream_ptr(S.device))
    _check(rc)
    return out


class WarmStart:
    """Learned warm start (multilayer perceptron, trained and run by libtpf kernels).

    Maps a time step's loads and minute index to an estimate of its converged
    voltages; pass the result of :meth:`predict` as ``V0`` to the solve calls.
    Parameters: flat float32 [W_1 (out x in), b_1, ...]; see include/tpf.h.
    """

    def __init__(self, n_pq: int, hidden: int = 256, layers: int = 3, params=None, vs: complex = 1.0 + 0.0j,
                 _handle=None):
        lib = load_library()
        if _handle is not None:
            self._h = _handle
        else:
            h = ctypes.c_void_p()
            pp = None
            if params is not None:
                self._init = np.ascontiguousarray(params, np.float32)
                pp = self._init.ctypes.data
            _check(lib.tpf_mlp_create(int(n_pq), int(hidden), int(layers), pp, float(np.real(vs)),
                                      float(np.imag(vs)), ctypes.byref(h)))
            self._h = h
        self.n = int(n_pq)
        self.num_params = int(lib.tpf_mlp_num_params(self._h))
        self._ws = None

    @property
    def handle(self):
        return self._h

    def _workspace(self, rows, device):
        torch = _torch()
        need = int(load_library().tpf_mlp_workspace_bytes(self._h, int(rows)))
        if self._ws is None or self._ws.numel() < need or self._ws.device != device:
            self._ws = torch.empty(max(need, 256), dtype=torch.uint8, device=device)
        return self._ws

    def get_params(self) -> np.ndarray:
        out = np.empty(self.num_params, np.float32)
        _check(load_library().tpf_mlp_get_params(self._h, out.ctypes.data))
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, np.float32)
        if p.size != self.num_params:
            raise ValueError("wrong parameter count")
        _check(load_library().tpf_mlp_set_params(self._h, p.ctypes.data))

    @staticmethod
    def _rows(S, t_index):
        if S.dim() != 2 or not S.is_contiguous() or not t_index.is_contiguous():
            raise ValueError("S must be a contiguous [rows, n] tensor")
        torch = _torch()
        if t_index.dtype != torch.int64 or t_index.numel() != S.shape[0]:
            raise ValueError("t_index must be int64 [rows]")
        return S.shape[0]

    def loss_grad(self, S, t_index, V):
        """(loss [1], grad [num_params]) float32 device tensors for one batch."""
        torch = _torch()
        rows = self._rows(S, t_index)
        loss = torch.zeros(1, dtype=torch.float32, device=S.device)
        grad = torch.zeros(self.num_params, dtype=torch.float32, device=S.device)
        ws = self._workspace(rows, S.device)
        with torch.cuda.device(S.device):
            _check(load_library().tpf_mlp_loss_grad(self._h, S.data_ptr(), _dtype_code(S), t_index.data_ptr(),
                                                    V.data_ptr(), rows, loss.data_ptr(), grad.data_ptr(),
                                                    ws.data_ptr(), ws.numel(), _stream_ptr(S.device)))
        return loss, grad

    def train_step(self, S, t_index, V, lr: float, weight_decay: float = 1e-4):
        torch = _torch()
        rows = self._rows(S, t_index)
        loss = torch.zeros(1, dtype=torch.float32, device=S.device)
        ws = self._workspace(rows, S.device)
        with torch.cuda.device(S.device):
            _check(load_library().tpf_mlp_train_step(self._h, S.data_ptr(), _dtype_code(S), t_index.data_ptr(),
                                                     V.data_ptr(), rows, float(lr), float(weight_decay),
                                                     loss.data_ptr(), ws.data_ptr(), ws.numel(),
                                                     _stream_ptr(S.device)))
        return loss

    def predict(self, S, t_index, out=None):
        """V0 [rows, n] (same dtype as S) for the solve calls' warm start."""
        torch = _torch()
        rows = self._rows(S, t_index)
        V0 = torch.empty_like(S) if out is None else out
        ws = self._workspace(rows, S.device)
        with torch.cuda.device(S.device):
            _check(load_library().tpf_mlp_predict(self._h, S.data_ptr(), _dtype_code(S), t_index.data_ptr(), rows,
                                                  V0.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(S.device)))
        return V0

    def fit(self, S, t_index, V, epochs: int = 10, batch: int = 1024, lr: float = 1e-3, lr_min: float = 1e-5,
            weight_decay: float = 1e-4, seed: int = 0, first_epoch: int = 0, total_epochs: Optional[int] = None):
        """Mini-batch AdamW with a cosine learning-rate schedule (one tpf_mlp_train call):
        epochs first_epoch .. first_epoch + epochs - 1 of a run of total_epochs (default:
        first_epoch + epochs).  Returns the mean loss per epoch."""
        torch = _torch()
        rows = self._rows(S, t_index)
        if V.shape != S.shape or V.dtype != S.dtype or not V.is_contiguous():
            raise ValueError("V must match S")
        total = first_epoch + epochs if total_epochs is None else int(total_epochs)
        losses = torch.zeros(max(1, epochs), dtype=torch.float32, device=S.device)
        ws = self._workspace(min(int(batch), rows), S.device)
        with torch.cuda.device(S.device):
            _check(load_library().tpf_mlp_train(self._h, S.data_ptr(), _dtype_code(S), t_index.data_ptr(),
                                                V.data_ptr(), rows, int(first_epoch), int(epochs), total,
                                                int(batch), float(lr), float(lr_min), float(weight_decay),
                                                int(seed) & 0xFFFFFFFFFFFFFFFF, losses.data_ptr(), ws.data_ptr(),
                                                ws.numel(), _stream_ptr(S.device)))
        return [float(x) for x in losses[:epochs].cpu()]

    def save(self, path: str):
        _check(load_library().tpf_mlp_save(self._h, path.encode()))

    @classmethod
    def load(cls, path: str) -> "WarmStart":
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.tpf_mlp_load(path.encode(), ctypes.byref(h)))
        obj = cls.__new__(cls)
        obj._h = h
        obj.num_params = int(lib.tpf_mlp_num_params(h))
        obj._ws = None
        obj.n = None
        return obj

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.tpf_mlp_free(h)
            self._h = None
