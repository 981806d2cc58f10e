"""ctypes front end of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It loads `liboracle.so` (plain C, built by `oracle/build.py`) and
converts gate lists (objects with .kind, .targets, .controls, .control_states,
.params, .matrix) into the oracle's own operation records.  It shares nothing
with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")

KINDS = ["i", "x", "y", "z", "h", "s", "sdg", "t", "tdg", "sx", "rx", "ry", "rz", "p",
         "u2", "u3", "swap", "rxx", "ryy", "rzz", "givens", "dexc", "unitary"]
KIND_ID = {k: i for i, k in enumerate(KINDS)}


class OrcOp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_targets", C.c_int32), ("targets", C.c_int32 * 5),
                ("n_controls", C.c_int32), ("controls", C.c_int32 * 5),
                ("control_states", C.c_uint32), ("param_index", C.c_int32 * 3),
                ("matrix", C.POINTER(C.c_double))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"oracle library missing: {LIB_PATH} (run oracle/build.py)")
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        up = C.POINTER(C.c_uint64)
        op_p = C.POINTER(OrcOp)
        L.orc_apply.argtypes = [C.c_int, dp, op_p, C.c_int, dp]
        L.orc_run.argtypes = [C.c_int, dp, op_p, C.c_int, dp]
        L.orc_gate_matrix.argtypes = [op_p, dp, dp]
        L.orc_gate_dmatrix.argtypes = [op_p, dp, C.c_int, dp]
        L.orc_expect_pauli.argtypes = [C.c_int, dp, up, up, dp, C.c_int, dp, dp, dp]
        L.orc_apply_pauli_sum.argtypes = [C.c_int, dp, up, up, dp, C.c_int, dp]
        L.orc_adjoint_grad.argtypes = [C.c_int, op_p, C.c_int, dp, C.c_int, up, up, dp, C.c_int,
                                       dp, dp]
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_sample.argtypes = [C.c_int, dp, C.c_uint64, C.c_int64, C.POINTER(C.c_int32), C.c_int,
                                 up]
        L.orc_sample_prefix.argtypes = [C.c_int, dp, dp, dp]
        L.orc_fuse_greedy.argtypes = [C.c_int, op_p, C.c_int, C.POINTER(C.c_int32)]
        L.orc_threads.restype = C.c_int
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _up(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_uint64))


class OpArray:
    """Owns the ctypes op records and any user matrices they point to."""

    def __init__(self, ops: Sequence):
        self.arr = (OrcOp * max(1, len(ops)))()
        self.keep = []
        self.n = len(ops)
        for i, op in enumerate(ops):
            r = self.arr[i]
            r.kind = KIND_ID[op.kind]
            r.n_targets = len(op.targets)
            for j, q in enumerate(op.targets):
                r.targets[j] = int(q)
            r.n_controls = len(op.controls)
            for j, q in enumerate(op.controls):
                r.controls[j] = int(q)
            r.control_states = int(op.control_states)
            for j in range(3):
                r.param_index[j] = int(op.params[j]) if j < len(op.params) else -1
            if op.kind == "unitary":
                m = np.ascontiguousarray(np.asarray(op.matrix, dtype=np.complex128))
                flat = np.empty(m.size * 2, dtype=np.float64)
                flat[0::2] = m.real.reshape(-1)
                flat[1::2] = m.imag.reshape(-1)
                self.keep.append(flat)
                r.matrix = _dp(flat)

    def ptr(self):
        return C.cast(self.arr, C.POINTER(OrcOp))


def _params(params) -> np.ndarray:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    if p.size == 0:
        p = np.zeros(1)
    return p


def run(n: int, ops: Sequence, params, psi0: Optional[np.ndarray] = None) -> np.ndarray:
    """Return U(params)|psi0> (|0...0> by default) as complex128."""
    oa = OpArray(ops)
    p = _params(params)
    if psi0 is None:
        buf = np.zeros(2 << n, dtype=np.float64)
        rc = lib().orc_run(n, _dp(buf), oa.ptr(), oa.n, _dp(p))
    else:
        z = np.ascontiguousarray(np.asarray(psi0, dtype=np.complex128))
        buf = z.view(np.float64).copy()
        rc = lib().orc_apply(n, _dp(buf), oa.ptr(), oa.n, _dp(p))
    if rc != 0:
        raise ValueError(f"oracle rejected op {-rc - 1}")
    return buf.view(np.complex128)


def run_circuit(circ, psi0=None) -> np.ndarray:
    return run(circ.n, circ.ops, circ.params, psi0)


def gate_matrix(op, params) -> np.ndarray:
    oa = OpArray([op])
    p = _params(params)
    d = 1 << (len(op.targets))
    out = np.zeros(2 * d * d)
    if lib().orc_gate_matrix(oa.ptr(), _dp(p), _dp(out)):
        raise ValueError("bad op")
    return out.view(np.complex128).reshape(d, d)


def gate_dmatrix(op, params, which: int) -> np.ndarray:
    oa = OpArray([op])
    p = _params(params)
    d = 1 << (len(op.targets))
    out = np.zeros(2 * d * d)
    if lib().orc_gate_dmatrix(oa.ptr(), _dp(p), which, _dp(out)):
        raise ValueError("bad op")
    return out.view(np.complex128).reshape(d, d)


def expect(n: int, psi: np.ndarray, ham) -> Tuple[np.ndarray, float, np.ndarray]:
    """(per-term <P_j>, sum_j c_j <P_j>, per-term imaginary parts)."""
    z = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).view(np.float64)
    nt = len(ham)
    terms = np.zeros(max(1, nt))
    ims = np.zeros(max(1, nt))
    tot = np.zeros(1)
    x = np.ascontiguousarray(ham.x, dtype=np.uint64)
    zz = np.ascontiguousarray(ham.z, dtype=np.uint64)
    c = np.ascontiguousarray(ham.c, dtype=np.float64)
    if lib().orc_expect_pauli(n, _dp(z), _up(x), _up(zz), _dp(c), nt, _dp(terms), _dp(ims),
                              _dp(tot)):
        raise ValueError("mask out of range")
    return terms[:nt], float(tot[0]), ims[:nt]


def apply_pauli_sum(n: int, psi: np.ndarray, ham) -> np.ndarray:
    z = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).view(np.float64)
    out = np.zeros(2 << n)
    x = np.ascontiguousarray(ham.x, dtype=np.uint64)
    zz = np.ascontiguousarray(ham.z, dtype=np.uint64)
    c = np.ascontiguousarray(ham.c, dtype=np.float64)
    if lib().orc_apply_pauli_sum(n, _dp(z), _up(x), _up(zz), _dp(c), len(ham), _dp(out)):
        raise ValueError("mask out of range")
    return out.view(np.complex128)


def energy(circ, ham, params=None) -> float:
    p = circ.params if params is None else params
    psi = run(circ.n, circ.ops, p)
    return expect(circ.n, psi, ham)[1]


def adjoint_grad(circ, ham, params=None) -> Tuple[float, np.ndarray]:
    p = _params(circ.params if params is None else params)
    npar = int(circ.n_params)
    oa = OpArray(circ.ops)
    g = np.zeros(max(1, npar))
    e = np.zeros(1)
    x = np.ascontiguousarray(ham.x, dtype=np.uint64)
    zz = np.ascontiguousarray(ham.z, dtype=np.uint64)
    c = np.ascontiguousarray(ham.c, dtype=np.float64)
    rc = lib().orc_adjoint_grad(circ.n, oa.ptr(), oa.n, _dp(p), npar, _up(x), _up(zz), _dp(c),
                                len(ham), _dp(e), _dp(g))
    if rc:
        raise ValueError(f"oracle adjoint failed ({rc})")
    return float(e[0]), g[:npar]


def param_shift_grad(circ, ham, indices: Sequence[int]) -> np.ndarray:
    """Two-term shift rule (paper eq. for Pauli rotations): half the difference
    of the energies at theta +/- pi/2.  Exact for parameters read by exactly
    one Pauli-rotation gate."""
    out = []
    for i in indices:
        p = np.array(circ.params, dtype=np.float64)
        p[i] += math.pi / 2
        ep = energy(circ, ham, p)
        p[i] -= math.pi
        em = energy(circ, ham, p)
        out.append(0.5 * (ep - em))
    return np.array(out)


def finite_diff_grad(circ, ham, indices: Sequence[int], h: float = 1e-6) -> np.ndarray:
    out = []
    for i in indices:
        p = np.array(circ.params, dtype=np.float64)
        p[i] += h
        ep = energy(circ, ham, p)
        p[i] -= 2 * h
        em = energy(circ, ham, p)
        out.append((ep - em) / (2 * h))
    return np.array(out)


def splitmix64(seed: int, s: int) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(seed), C.c_uint64(s)))


def sample(n: int, psi: np.ndarray, seed: int, shots: int, qubits: Sequence[int]) -> np.ndarray:
    z = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).view(np.float64)
    q = np.ascontiguousarray(np.asarray(list(qubits), dtype=np.int32))
    if q.size == 0:
        q = np.zeros(1, dtype=np.int32)
        nq = 0
    else:
        nq = len(qubits)
    out = np.zeros(max(1, shots), dtype=np.uint64)
    if lib().orc_sample(n, _dp(z), C.c_uint64(seed), shots, q.ctypes.data_as(C.POINTER(C.c_int32)),
                        nq, _up(out)):
        raise ValueError("bad sample arguments")
    return out[:shots]


def sample_prefix(n: int, psi: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    z = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).view(np.float64)
    cb = min(n, 10)
    K = (1 << n) >> cb
    S = np.zeros(K)
    P = np.zeros(K + 1)
    lib().orc_sample_prefix(n, _dp(z), _dp(S), _dp(P))
    return S, P


def fuse_greedy(k: int, ops: Sequence) -> Tuple[int, np.ndarray]:
    oa = OpArray(ops)
    out = np.zeros(max(1, len(ops)), dtype=np.int32)
    nb = lib().orc_fuse_greedy(k, oa.ptr(), oa.n, out.ctypes.data_as(C.POINTER(C.c_int32)))
    return int(nb), out[:len(ops)]


def threads() -> int:
    return int(lib().orc_threads())
