"""CPU oracle of the batched fixed-point power flow -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never calls it and
shares no code with it; the two meet only on the seeded inputs drawn by
``paper_2403_04578_amd.workloads`` (which holds none of the method's arithmetic).

The arithmetic lives in ``tpf_oracle.c`` (plain FP64 C, one function per step of
the paper's method) and ``mlp_ref.py`` (plain FP64 numpy for the learned warm
start).  This module only compiles the C file with gcc and marshals arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tpf_oracle.c")
_LIB = os.path.join(_HERE, "libtpf_oracle.so")

ST_CONVERGED, ST_MAX_ITER, ST_NONFINITE = 0, 1, 2


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
               _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.oracle_build.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_int,
                                     ctypes.c_double, ctypes.c_double, P, P, P, P]
        lib.oracle_build.restype = ctypes.c_int
        lib.oracle_fpi.argtypes = [ctypes.c_int, P, P, ctypes.c_int64, P, ctypes.c_double,
                                   ctypes.c_int, P, P, P, P, P]
        lib.oracle_fpi.restype = None
        lib.oracle_mismatch.argtypes = [ctypes.c_int, P, P, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int64, P, P, P]
        lib.oracle_mismatch.restype = None
        lib.oracle_build_3ph.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, P, P]
        lib.oracle_build_3ph.restype = ctypes.c_int
        lib.oracle_fpi_zip.argtypes = [ctypes.c_int, P, P, ctypes.c_double, ctypes.c_double, P, P, ctypes.c_int64,
                                       P, ctypes.c_double, ctypes.c_int, P, P, P, P, P]
        lib.oracle_fpi_zip.restype = None
        lib.oracle_fpi_zipz.argtypes = [ctypes.c_int, P, P, ctypes.c_double, ctypes.c_double, P, P, P,
                                        ctypes.c_int64, P, ctypes.c_double, ctypes.c_int, P, P, P, P, P]
        lib.oracle_fpi_zipz.restype = None
        lib.oracle_mismatch_zip.argtypes = [ctypes.c_int, P, P, ctypes.c_double, ctypes.c_double, P, P, P,
                                            ctypes.c_int64, P, P, P]
        lib.oracle_mismatch_zip.restype = None
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__({-1: "invalid network", -2: "singular Y_dd", -4: "out of memory"}.get(code, str(code)))
        self.code = code


@dataclass
class OracleNetwork:
    n: int  # number of PQ buses
    Ydd: np.ndarray  # complex128 [n, n]
    Yds: np.ndarray  # complex128 [n]
    Z: np.ndarray  # complex128 [n, n]  (= -Y_dd^-1)
    w: np.ndarray  # complex128 [n]     (= -Y_dd^-1 Y_ds v_s)
    vs: complex


def build_network(n_bus, frm, to, r, x, slack=0, vs=1.0 + 0.0j) -> OracleNetwork:
    """Sec. II Eqs. (1)-(2): Y, its partition, Z = -Y_dd^-1 and w."""
    lib = _load()
    n = n_bus - 1
    frm = np.ascontiguousarray(frm, np.int32)
    to = np.ascontiguousarray(to, np.int32)
    r = np.ascontiguousarray(r, np.float64)
    x = np.ascontiguousarray(x, np.float64)
    Ydd = np.zeros((n, n), np.complex128)
    Yds = np.zeros(n, np.complex128)
    Z = np.zeros((n, n), np.complex128)
    w = np.zeros(n, np.complex128)
    rc = lib.oracle_build(n_bus, len(frm), _ptr(frm), _ptr(to), _ptr(r), _ptr(x), slack,
                          float(np.real(vs)), float(np.imag(vs)), _ptr(Ydd), _ptr(Yds), _ptr(Z), _ptr(w))
    if rc != 0:
        raise OracleError(rc)
    return OracleNetwork(n, Ydd, Yds, Z, w, complex(vs))


def build_network_3ph(n_bus, frm, to, zabc, slack=0, vs_abc=None) -> OracleNetwork:
    """Sec. II Eq. (1) per phase node of a three-phase network (zabc [n_branch, 3, 3]).
    The returned network holds Yds = Y_ds v_s (the slack block times the slack phase
    voltages) and vs = 1, so every function below applies unchanged."""
    lib = _load()
    n = 3 * (n_bus - 1)
    frm = np.ascontiguousarray(frm, np.int32)
    to = np.ascontiguousarray(to, np.int32)
    z = np.ascontiguousarray(np.asarray(zabc, np.complex128).reshape(len(frm), 3, 3))
    if vs_abc is None:
        vs_abc = np.exp(-2j * np.pi / 3 * np.arange(3))
    v = np.ascontiguousarray(np.asarray(vs_abc, np.complex128).reshape(3))
    Ydd = np.zeros((n, n), np.complex128)
    c = np.zeros(n, np.complex128)
    Z = np.zeros((n, n), np.complex128)
    w = np.zeros(n, np.complex128)
    rc = lib.oracle_build_3ph(n_bus, len(frm), _ptr(frm), _ptr(to), _ptr(z), slack, _ptr(v), _ptr(Ydd), _ptr(c),
                              _ptr(Z), _ptr(w))
    if rc != 0:
        raise OracleError(rc)
    return OracleNetwork(n, Ydd, c, Z, w, 1.0 + 0.0j)


def build_feeder_3ph(feeder) -> OracleNetwork:
    return build_network_3ph(feeder.n_bus, feeder.frm, feeder.to, feeder.zabc, 0, feeder.vs_abc)


def build_feeder(feeder) -> OracleNetwork:
    return build_network(feeder.n_bus, feeder.frm, feeder.to, feeder.r, feeder.x, 0, feeder.vs)


@dataclass
class FpiResult:
    V: np.ndarray  # complex128 [tau, n]
    iters: np.ndarray  # int32 [tau]
    status: np.ndarray  # int8 [tau]
    d: np.ndarray  # float64 [tau] last step size


def fpi(net: OracleNetwork, S: np.ndarray, tol: float, max_iter: int, V0: np.ndarray | None = None) -> FpiResult:
    """Algorithm 1 per column: flat start (or V0), V <- Z conj(S./V) + w until max|dV| < tol."""
    lib = _load()
    S = np.ascontiguousarray(np.asarray(S).reshape(-1, net.n), np.complex128)
    tau = S.shape[0]
    V = np.empty_like(S)
    iters = np.empty(tau, np.int32)
    status = np.empty(tau, np.int8)
    d = np.empty(tau, np.float64)
    v0p = None
    if V0 is not None:
        V0 = np.ascontiguousarray(np.asarray(V0).reshape(-1, net.n), np.complex128)
        assert V0.shape == S.shape
        v0p = _ptr(V0)
    lib.oracle_fpi(net.n, _ptr(np.ascontiguousarray(net.Z)), _ptr(np.ascontiguousarray(net.w)), tau, _ptr(S),
                   float(tol), int(max_iter), v0p, _ptr(V), _ptr(iters), _ptr(status), _ptr(d))
    return FpiResult(V, iters, status, d)


def mismatch(net: OracleNetwork, S: np.ndarray, V: np.ndarray) -> np.ndarray:
    """Per-column max |S + V .* conj(Y_ds v_s + Y_dd V)| (Eq. (1) power balance)."""
    lib = _load()
    S = np.ascontiguousarray(np.asarray(S).reshape(-1, net.n), np.complex128)
    V = np.ascontiguousarray(np.asarray(V).reshape(-1, net.n), np.complex128)
    out = np.empty(S.shape[0], np.float64)
    lib.oracle_mismatch(net.n, _ptr(np.ascontiguousarray(net.Ydd)), _ptr(np.ascontiguousarray(net.Yds)),
                        float(np.real(net.vs)), float(np.imag(net.vs)), S.shape[0], _ptr(S), _ptr(V), _ptr(out))
    return out


def _alphas(net: OracleNetwork, alpha_i, alpha_p):
    ai = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha_i, np.float64), (net.n,)))
    ap = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha_p, np.float64), (net.n,)))
    return ai, ap


def fpi_zip(net: OracleNetwork, S: np.ndarray, alpha_i, alpha_p, tol: float, max_iter: int,
            V0: np.ndarray | None = None, alpha_z=None) -> FpiResult:
    """Eq. (2) with ZIP loads (alpha_Z, alpha_I, alpha_P per PQ bus or scalars): per
    column F = -B^-1 diag(alpha_P s*), w = -B^-1 (Y_ds v_s + alpha_I s*) with
    B = diag(alpha_Z s*) + Y_dd, iterated as Algorithm 1.  Without alpha_Z, B = Y_dd and
    the network's Z = -Y_dd^-1 serves every column; with it, each column eliminates
    its own B."""
    lib = _load()
    S = np.ascontiguousarray(np.asarray(S).reshape(-1, net.n), np.complex128)
    ai, ap = _alphas(net, alpha_i, alpha_p)
    if alpha_z is not None:
        az = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha_z, np.float64), (net.n,)))
        return _fpi_zipz(lib, net, S, az, ai, ap, tol, max_iter, V0)
    tau = S.shape[0]
    V = np.empty_like(S)
    iters = np.empty(tau, np.int32)
    status = np.empty(tau, np.int8)
    d = np.empty(tau, np.float64)
    v0p = None
    if V0 is not None:
        V0 = np.ascontiguousarray(np.asarray(V0).reshape(-1, net.n), np.complex128)
        assert V0.shape == S.shape
        v0p = _ptr(V0)
    lib.oracle_fpi_zip(net.n, _ptr(np.ascontiguousarray(net.Z)), _ptr(np.ascontiguousarray(net.Yds)),
                       float(np.real(net.vs)), float(np.imag(net.vs)), _ptr(ai), _ptr(ap), tau, _ptr(S),
                       float(tol), int(max_iter), v0p, _ptr(V), _ptr(iters), _ptr(status), _ptr(d))
    return FpiResult(V, iters, status, d)


def _fpi_zipz(lib, net, S, az, ai, ap, tol, max_iter, V0):
    tau = S.shape[0]
    V = np.empty_like(S)
    iters = np.empty(tau, np.int32)
    status = np.empty(tau, np.int8)
    d = np.empty(tau, np.float64)
    v0p = None
    if V0 is not None:
        V0 = np.ascontiguousarray(np.asarray(V0).reshape(-1, net.n), np.complex128)
        assert V0.shape == S.shape
        v0p = _ptr(V0)
    lib.oracle_fpi_zipz(net.n, _ptr(np.ascontiguousarray(net.Ydd)), _ptr(np.ascontiguousarray(net.Yds)),
                        float(np.real(net.vs)), float(np.imag(net.vs)), _ptr(az), _ptr(ai), _ptr(ap), tau, _ptr(S),
                        float(tol), int(max_iter), v0p, _ptr(V), _ptr(iters), _ptr(status), _ptr(d))
    return FpiResult(V, iters, status, d)


def mismatch_zip(net: OracleNetwork, S: np.ndarray, V: np.ndarray, alpha_i, alpha_p, alpha_z=None) -> np.ndarray:
    """Per-column max |S .* (alpha_P + alpha_I .* V + alpha_Z .* |V|^2) + V .* conj(Y_ds v_s + Y_dd V)|."""
    lib = _load()
    S = np.ascontiguousarray(np.asarray(S).reshape(-1, net.n), np.complex128)
    V = np.ascontiguousarray(np.asarray(V).reshape(-1, net.n), np.complex128)
    ai, ap = _alphas(net, alpha_i, alpha_p)
    azp = None
    if alpha_z is not None:
        az = np.ascontiguousarray(np.broadcast_to(np.asarray(alpha_z, np.float64), (net.n,)))
        azp = _ptr(az)
    out = np.empty(S.shape[0], np.float64)
    lib.oracle_mismatch_zip(net.n, _ptr(np.ascontiguousarray(net.Ydd)), _ptr(np.ascontiguousarray(net.Yds)),
                            float(np.real(net.vs)), float(np.imag(net.vs)), azp, _ptr(ai), _ptr(ap), S.shape[0],
                            _ptr(S), _ptr(V), _ptr(out))
    return out


def num_threads() -> int:
    return int(_load().oracle_num_threads())
