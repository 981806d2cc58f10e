"""ctypes binding of libsv.so (include/sv.h).  Argument marshalling only:
every step of the path runs in the HIP library; torch supplies device memory
and the stream.  Importing this module loads the library and raises if it is
missing -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsv.so")

SV_C128, SV_C64 = 0, 1
SV_FUSE_AUTO = -1
SV_WS_ADJOINT = 1
STATUS = {0: "SV_OK", -1: "SV_EINVAL", -2: "SV_EDTYPE", -3: "SV_EUNBOUND", -4: "SV_ENOMEM",
          -5: "SV_EUNSUPPORTED", -6: "SV_EDEVICE"}

KINDS = ["i", "x", "y", "z", "h", "s", "sdg", "t", "tdg", "sx", "rx", "ry", "rz", "p", "u2",
         "u3", "swap", "rxx", "ryy", "rzz", "givens", "dexc", "unitary"]
KIND_ID = {k: i for i, k in enumerate(KINDS)}


class SvError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class SvOp(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_targets", C.c_int32), ("targets", C.c_int32 * 5),
                ("n_controls", C.c_int32), ("controls", C.c_int32 * 5),
                ("control_states", C.c_uint32), ("param_index", C.c_int32 * 3),
                ("matrix", C.POINTER(C.c_double))]


class SvPauliTerm(C.Structure):
    _fields_ = [("x_mask", C.c_uint64), ("z_mask", C.c_uint64), ("coeff", C.c_double)]


class SvCircuitDesc(C.Structure):
    _fields_ = [("n_qubits", C.c_int32), ("n_ops", C.c_int32), ("ops", C.POINTER(SvOp)),
                ("n_params", C.c_int32), ("n_terms", C.c_int32),
                ("terms", C.POINTER(SvPauliTerm))]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH}; run `python -m paper_2608_09733_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, dp, u64p = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)
    opp, tp = C.POINTER(SvOp), C.POINTER(SvPauliTerm)
    i32, i64, u64 = C.c_int32, C.c_int64, C.c_uint64
    sig = {
        "sv_workspace_bytes": (C.c_size_t, [i32, C.c_int, C.c_uint32]),
        "sv_alloc": (C.c_int, [i32, C.c_int, vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]),
        "sv_free": (C.c_int, [vp]),
        "sv_set_stream": (C.c_int, [vp, vp]),
        "sv_reset": (C.c_int, [vp]),
        "sv_apply_layer": (C.c_int, [vp, opp, i32, dp, i32, i32]),
        "sv_expect_pauli": (C.c_int, [vp, tp, i32, dp, dp]),
        "sv_expect_pauli_noalloc": (C.c_int, [vp, tp, i32, dp, dp]),
        "sv_adjoint_grad": (C.c_int, [vp, opp, i32, dp, i32, tp, i32, dp, dp, C.POINTER(i32)]),
        "sv_adjoint_grad_device": (C.c_int, [vp, opp, i32, dp, i32, tp, i32, vp]),
        "sv_sample": (C.c_int, [vp, u64, i64, C.POINTER(i32), i32, u64p]),
        "sv_sample_counts": (C.c_int, [vp, u64, i64, C.POINTER(i32), i32, u64p]),
        "sv_shot_estimate": (C.c_int, [vp, u64, i64, tp, i32, dp, dp, dp, C.POINTER(i32)]),
        "sv_dm_apply": (C.c_int, [vp, i32, opp, i32, dp, i32]),
        "sv_dm_apply_kraus": (C.c_int, [vp, i32, C.POINTER(i32), i32, dp, i32]),
        "sv_dm_expect_pauli": (C.c_int, [vp, i32, tp, i32, dp, dp]),
        "sv_dm_apply_kraus2": (C.c_int, [vp, i32, i32, i32, dp, i32]),
        "sv_copy_to_host": (C.c_int, [vp, vp, vp, u64, u64]),
        "sv_copy_from_host": (C.c_int, [vp, vp, vp, u64, u64]),
        "sv_last_error": (C.c_char_p, []),
        "sv_default_tiling": (C.c_int, [i32, C.c_int, i32, C.POINTER(i32), C.POINTER(i32),
                                        C.POINTER(i32)]),
        "sv_plan_stats": (C.c_int, [i32, opp, i32, i32, i32, i32, i32, C.POINTER(i32),
                                    C.POINTER(i32)]),
        "sv_adjoint_plan_stats": (C.c_int, [i32, opp, i32, i32, i32, i32, i32, C.POINTER(i32),
                                            C.POINTER(i32), C.POINTER(i32)]),
        "sv_set_tiling": (C.c_int, [vp, i32, i32, i32]),
        "sv_set_adjoint_tiling": (C.c_int, [vp, i32, i32, i32]),
        "sv_fuse_blocks": (C.c_int, [opp, i32, i32, C.POINTER(i32), C.POINTER(i32)]),
        "sv_version": (C.c_char_p, []),
        "sv_timing_enable": (C.c_int, [vp, i32]),
        "sv_timing_read": (C.c_int, [vp, dp, C.POINTER(i64), dp]),
        "sv_batch_plan": (C.c_int, [C.POINTER(SvCircuitDesc), i32, C.c_int, i32, i32, i32,
                                    C.POINTER(vp)]),
        "sv_batch_upload_params": (C.c_int, [vp, dp, i64]),
        "sv_batch_params_device": (vp, [vp]),
        "sv_batch_param_offset": (i64, [vp, i32]),
        "sv_batch_run": (C.c_int, [vp, vp]),
        "sv_batch_graph_launch": (C.c_int, [vp, vp]),
        "sv_batch_results_device": (vp, [vp]),
        "sv_batch_check": (C.c_int, [vp, vp]),
        "sv_batch_set_spin_limit": (C.c_int, [vp, i32]),
        "sv_batch_state": (C.c_int, [vp, i32, C.POINTER(vp), C.POINTER(vp)]),
        "sv_batch_stats": (C.c_int, [vp, C.POINTER(i64), C.POINTER(i64), dp, dp]),
        "sv_batch_free": (C.c_int, [vp]),
        "sv_batch_copy_results": (C.c_int, [vp, dp, vp]),
        "sv_batch_autotune": (C.c_int, [C.POINTER(SvCircuitDesc), i32, C.c_int, dp, i32, vp,
                                        C.POINTER(i32), C.POINTER(i32), C.POINTER(i32), dp]),
        "sv_batch_copy_state": (C.c_int, [vp, i32, vp, vp, vp]),
        "sv_serve_create": (C.c_int, [C.POINTER(vp)]),
        "sv_serve_max_qubits": (i32, []),
        "sv_serve_check": (C.c_int, [vp, C.POINTER(SvCircuitDesc)]),
        "sv_serve_submit": (C.c_int, [vp, C.POINTER(SvCircuitDesc), i32, dp, vp, vp]),
        "sv_serve_free": (C.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st: int):
    if st != 0:
        raise SvError(st, lib().sv_last_error().decode())


class OpArray:
    """sv_op records for a gate list (objects with .kind .targets .controls
    .control_states .params .matrix); keeps user matrices alive."""

    def __init__(self, ops: Sequence):
        self.n = len(ops)
        self.arr = (SvOp * max(1, self.n))()
        self.keep = []
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
                flat = np.ascontiguousarray(m.reshape(-1).view(np.float64))
                self.keep.append(flat)
                r.matrix = flat.ctypes.data_as(C.POINTER(C.c_double))

    def ptr(self):
        return C.cast(self.arr, C.POINTER(SvOp))


class TermArray:
    def __init__(self, ham):
        self.n = len(ham)
        self.arr = (SvPauliTerm * max(1, self.n))()
        for j in range(self.n):
            self.arr[j].x_mask = int(ham.x[j])
            self.arr[j].z_mask = int(ham.z[j])
            self.arr[j].coeff = float(ham.c[j])

    def ptr(self):
        return C.cast(self.arr, C.POINTER(SvPauliTerm))


def _params_ptr(params) -> Tuple[np.ndarray, int]:
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float64))
    n = int(p.size)
    if n == 0:
        p = np.zeros(1)
    return p, n


def _stream_ptr(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) or None


class State:
    """A 2^n-amplitude state held as two torch device planes (FP64 or FP32)."""

    def __init__(self, n: int, dtype: str = "c128", adjoint: bool = False, device: str = "cuda",
                 stream=None):
        import torch
        L = lib()
        self.n = int(n)
        self.dtype = dtype
        self.code = SV_C128 if dtype == "c128" else SV_C64
        tdt = torch.float64 if dtype == "c128" else torch.float32
        self.np_dtype = np.float64 if dtype == "c128" else np.float32
        N = 1 << self.n
        self.re = torch.empty(N, dtype=tdt, device=device)
        self.im = torch.empty(N, dtype=tdt, device=device)
        wsb = int(L.sv_workspace_bytes(self.n, self.code, SV_WS_ADJOINT if adjoint else 0))
        if wsb == 0:
            raise SvError(-1, f"bad state size n={n} dtype={dtype}")
        self.ws = torch.empty(wsb + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.stream = stream
        h = C.c_void_p()
        _check(L.sv_alloc(self.n, self.code, C.c_void_p(self.re.data_ptr()),
                          C.c_void_p(self.im.data_ptr()), C.c_void_p(base + off), wsb,
                          C.c_void_p(_stream_ptr(stream)), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().sv_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        _check(lib().sv_set_stream(self.h, C.c_void_p(_stream_ptr(stream))))

    def set_tiling(self, tile_bits: int = 0, low_bits: int = 0, group_bits: int = 0):
        _check(lib().sv_set_tiling(self.h, tile_bits, low_bits, group_bits))

    def set_adjoint_tiling(self, tile_bits: int = 0, low_bits: int = 0, group_bits: int = 0):
        _check(lib().sv_set_adjoint_tiling(self.h, tile_bits, low_bits, group_bits))

    def reset(self):
        _check(lib().sv_reset(self.h))

    def timing(self, on: bool = True):
        _check(lib().sv_timing_enable(self.h, 1 if on else 0))

    def timing_read(self) -> Tuple[float, int, float]:
        """(summed sweep-kernel ms, launches, algorithmic bytes) since the last read."""
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        by = C.c_double(0.0)
        _check(lib().sv_timing_read(self.h, C.byref(ms), C.byref(n), C.byref(by)))
        return float(ms.value), int(n.value), float(by.value)

    def apply(self, ops, params, fuse: int = SV_FUSE_AUTO, op_array: Optional[OpArray] = None):
        oa = op_array or OpArray(ops)
        p, npar = _params_ptr(params)
        _check(lib().sv_apply_layer(self.h, oa.ptr(), oa.n, p.ctypes.data_as(C.POINTER(C.c_double)),
                                    npar, int(fuse)))

    def run(self, circ, fuse: int = SV_FUSE_AUTO):
        self.reset()
        self.apply(circ.ops, circ.params, fuse)

    def expect(self, ham) -> Tuple[np.ndarray, float]:
        ta = TermArray(ham)
        out = np.zeros(max(1, ta.n))
        tot = C.c_double(0.0)
        _check(lib().sv_expect_pauli(self.h, ta.ptr(), ta.n,
                                     out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(tot)))
        return out[:ta.n], float(tot.value)

    def expect_noalloc(self, ham) -> Tuple[np.ndarray, float]:
        """As expect(), through the allocation-free entry point (fixed scratch)."""
        ta = TermArray(ham)
        out = np.zeros(max(1, ta.n))
        tot = C.c_double(0.0)
        _check(lib().sv_expect_pauli_noalloc(self.h, ta.ptr(), ta.n,
                                             out.ctypes.data_as(C.POINTER(C.c_double)),
                                             C.byref(tot)))
        return out[:ta.n], float(tot.value)

    def adjoint_grad(self, ops, params, ham, op_array: Optional[OpArray] = None
                     ) -> Tuple[float, np.ndarray]:
        oa = op_array or OpArray(ops)
        ta = TermArray(ham)
        p, npar = _params_ptr(params)
        g = np.zeros(max(1, npar))
        e = C.c_double(0.0)
        ne = C.c_int32(0)
        _check(lib().sv_adjoint_grad(self.h, oa.ptr(), oa.n, p.ctypes.data_as(C.POINTER(C.c_double)),
                                     npar, ta.ptr(), ta.n, C.byref(e),
                                     g.ctypes.data_as(C.POINTER(C.c_double)), C.byref(ne)))
        return float(e.value), g[:npar]

    def adjoint_grad_device(self, ops, params, ham, out_tensor, op_array=None):
        oa = op_array or OpArray(ops)
        ta = TermArray(ham)
        p, npar = _params_ptr(params)
        _check(lib().sv_adjoint_grad_device(self.h, oa.ptr(), oa.n,
                                            p.ctypes.data_as(C.POINTER(C.c_double)), npar,
                                            ta.ptr(), ta.n, C.c_void_p(out_tensor.data_ptr())))

    def sample(self, seed: int, shots: int, qubits: Sequence[int]) -> np.ndarray:
        q = np.ascontiguousarray(np.asarray(list(qubits), dtype=np.int32))
        nq = int(q.size)
        if nq == 0:
            q = np.zeros(1, dtype=np.int32)
        out = np.zeros(max(1, shots), dtype=np.uint64)
        _check(lib().sv_sample(self.h, C.c_uint64(seed), int(shots),
                               q.ctypes.data_as(C.POINTER(C.c_int32)), nq,
                               out.ctypes.data_as(C.POINTER(C.c_uint64))))
        return out[:shots]

    def sample_counts(self, seed: int, shots: int, qubits: Sequence[int]) -> np.ndarray:
        q = np.ascontiguousarray(np.asarray(list(qubits), dtype=np.int32))
        nq = int(q.size)
        if nq == 0:
            q = np.zeros(1, dtype=np.int32)
        out = np.zeros(1 << nq, dtype=np.uint64)
        _check(lib().sv_sample_counts(self.h, C.c_uint64(seed), int(shots),
                                      q.ctypes.data_as(C.POINTER(C.c_int32)), nq,
                                      out.ctypes.data_as(C.POINTER(C.c_uint64))))
        return out

    def shot_estimate(self, seed: int, shots: int, ham) -> Tuple[np.ndarray, float, float, int]:
        """(per-term values, energy, variance of the energy, number of groups)."""
        ta = TermArray(ham)
        vals = np.zeros(max(1, ta.n))
        e = C.c_double(0.0)
        v = C.c_double(0.0)
        g = C.c_int32(0)
        _check(lib().sv_shot_estimate(self.h, C.c_uint64(seed), int(shots), ta.ptr(), ta.n,
                                      vals.ctypes.data_as(C.POINTER(C.c_double)), C.byref(e),
                                      C.byref(v), C.byref(g)))
        return vals[:ta.n], float(e.value), float(v.value), int(g.value)

    # ---- density matrix of n = self.n / 2 qubits held as vec(rho)
    def dm_apply(self, ops, params, op_array: Optional[OpArray] = None):
        oa = op_array or OpArray(ops)
        p, npar = _params_ptr(params)
        _check(lib().sv_dm_apply(self.h, self.n // 2, oa.ptr(), oa.n,
                                 p.ctypes.data_as(C.POINTER(C.c_double)), npar))

    def dm_apply_kraus(self, qubits, kraus: Sequence[np.ndarray]):
        """One channel (the same Kraus set) on each qubit of `qubits` (an int or a sequence)."""
        q = np.ascontiguousarray(np.atleast_1d(np.asarray(qubits, dtype=np.int32)))
        k = np.ascontiguousarray(np.asarray(kraus, dtype=np.complex128).reshape(-1, 2, 2))
        buf = np.ascontiguousarray(k.view(np.float64).reshape(-1))
        _check(lib().sv_dm_apply_kraus(self.h, self.n // 2, q.ctypes.data_as(C.POINTER(C.c_int32)),
                                       int(q.size), buf.ctypes.data_as(C.POINTER(C.c_double)),
                                       int(k.shape[0])))

    def dm_apply_kraus2(self, q0: int, q1: int, kraus: Sequence[np.ndarray]):
        """A channel on the qubit pair (q0, q1): 4x4 Kraus matrices, local index bit(q0) + 2 bit(q1)."""
        k = np.ascontiguousarray(np.asarray(kraus, dtype=np.complex128).reshape(-1, 4, 4))
        buf = np.ascontiguousarray(k.view(np.float64).reshape(-1))
        _check(lib().sv_dm_apply_kraus2(self.h, self.n // 2, int(q0), int(q1),
                                        buf.ctypes.data_as(C.POINTER(C.c_double)), int(k.shape[0])))

    def dm_expect(self, ham) -> Tuple[np.ndarray, float]:
        ta = TermArray(ham)
        out = np.zeros(max(1, ta.n))
        tot = C.c_double(0.0)
        _check(lib().sv_dm_expect_pauli(self.h, self.n // 2, ta.ptr(), ta.n,
                                        out.ctypes.data_as(C.POINTER(C.c_double)), C.byref(tot)))
        return out[:ta.n], float(tot.value)

    def planes(self, offset: int = 0, count: Optional[int] = None,
               out: Optional[Tuple[np.ndarray, np.ndarray]] = None) -> Tuple[np.ndarray, np.ndarray]:
        """Copy amplitudes [offset, offset + count) of both planes to the host;
        `out` = (re, im) reuses caller buffers (e.g. numpy views of pinned
        tensors), each contiguous, of the state's element type and >= count long."""
        N = 1 << self.n
        if count is None:
            count = N - offset
        if out is None:
            re = np.empty(count, dtype=self.np_dtype)
            im = np.empty(count, dtype=self.np_dtype)
        else:
            re, im = out
            for a in (re, im):
                if a.dtype != self.np_dtype or a.size < count or not a.flags["C_CONTIGUOUS"]:
                    raise ValueError("out buffers must be contiguous, of the state's element "
                                     "type and at least count long")
        _check(lib().sv_copy_to_host(self.h, C.c_void_p(re.ctypes.data), C.c_void_p(im.ctypes.data),
                                     offset, count))
        return re, im

    def gather(self, idx, window: int = 1 << 22) -> np.ndarray:
        """Amplitudes at the basis indices `idx` (complex128), copied out window
        by window through pinned host buffers (sv_copy_to_host)."""
        import torch
        idx = np.asarray(idx, dtype=np.int64)
        order = np.argsort(idx, kind="stable")
        sidx = idx[order]
        N = 1 << self.n
        window = min(window, N)
        tdt = torch.float64 if self.dtype == "c128" else torch.float32
        bufs = (torch.empty(window, dtype=tdt, pin_memory=True).numpy(),
                torch.empty(window, dtype=tdt, pin_memory=True).numpy())
        out = np.empty(idx.size, dtype=np.complex128)
        k = 0
        while k < sidx.size:
            base = int(sidx[k]) // window * window
            cnt = min(window, N - base)
            re, im = self.planes(base, cnt, out=bufs)
            e = int(np.searchsorted(sidx, base + cnt, side="left"))
            loc = sidx[k:e] - base
            out[order[k:e]] = re[loc].astype(np.float64) + 1j * im[loc].astype(np.float64)
            k = e
        return out

    def to_numpy(self) -> np.ndarray:
        re, im = self.planes()
        return re.astype(np.float64) + 1j * im.astype(np.float64)

    def set_planes(self, re: np.ndarray, im: np.ndarray, offset: int = 0):
        re = np.ascontiguousarray(re, dtype=self.np_dtype)
        im = np.ascontiguousarray(im, dtype=self.np_dtype)
        _check(lib().sv_copy_from_host(self.h, C.c_void_p(re.ctypes.data), C.c_void_p(im.ctypes.data),
                                       offset, int(re.size)))


def default_tiling(n: int, dtype: str = "c128", backward: bool = False) -> Tuple[int, int, int]:
    """(tile_bits, low_bits, group_bits) a handle uses unless set_tiling overrides them."""
    t, c, r = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    code = SV_C128 if dtype == "c128" else SV_C64
    _check(lib().sv_default_tiling(n, code, 1 if backward else 0, C.byref(t), C.byref(c),
                                   C.byref(r)))
    return int(t.value), int(c.value), int(r.value)


def adjoint_plan_stats(n: int, ops, n_params: int, tile_bits: int = 0, low_bits: int = 0,
                       group_bits: int = 0) -> Tuple[int, int, int]:
    """(sweeps, register stages, gradient slots) of the adjoint's backward program."""
    oa = OpArray(ops)
    s, b, g = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    _check(lib().sv_adjoint_plan_stats(n, oa.ptr(), oa.n, n_params, tile_bits, low_bits, group_bits,
                                       C.byref(s), C.byref(b), C.byref(g)))
    return int(s.value), int(b.value), int(g.value)


def plan_stats(n: int, ops, fuse: int = SV_FUSE_AUTO, tile_bits: int = 0, low_bits: int = 0,
               group_bits: int = 0) -> Tuple[int, int]:
    oa = OpArray(ops)
    s = C.c_int32(0)
    b = C.c_int32(0)
    _check(lib().sv_plan_stats(n, oa.ptr(), oa.n, fuse, tile_bits, low_bits, group_bits,
                               C.byref(s), C.byref(b)))
    return int(s.value), int(b.value)


def fuse_blocks(ops, width: int) -> Tuple[int, np.ndarray]:
    oa = OpArray(ops)
    out = np.zeros(max(1, oa.n), dtype=np.int32)
    nb = C.c_int32(0)
    _check(lib().sv_fuse_blocks(oa.ptr(), oa.n, width, out.ctypes.data_as(C.POINTER(C.c_int32)),
                                C.byref(nb)))
    return int(nb.value), out[:oa.n]


def version() -> str:
    return lib().sv_version().decode()


_OPA_CACHE: dict = {}


def op_array_for(circuit) -> "OpArray":
    """The sv_op records of `circuit`, shared by every circuit with the same
    structure key (`circuit.key`, when set); built afresh otherwise."""
    key = getattr(circuit, "key", None)
    if key is None:
        return OpArray(circuit.ops)
    oa = _OPA_CACHE.get(key)
    if oa is None:
        if len(_OPA_CACHE) >= 512:
            _OPA_CACHE.clear()
        oa = _OPA_CACHE[key] = OpArray(circuit.ops)
    return oa


def _circuit_descs(circuits, observables):
    ops = [op_array_for(c) for c in circuits]
    terms = [TermArray(h) for h in observables]
    descs = (SvCircuitDesc * max(1, len(circuits)))()
    for k, c in enumerate(circuits):
        d = descs[k]
        d.n_qubits = int(c.n)
        d.n_ops = ops[k].n
        d.ops = ops[k].ptr()
        d.n_params = int(len(c.params))
        d.n_terms = terms[k].n
        d.terms = terms[k].ptr()
    return descs, (ops, terms)


def batch_autotune(circuits, observables, dtype: str = "c128", reps: int = 2, stream=None):
    """Measured choice of the batch tiling: {"tile_bits", "low_bits",
    "group_bits", "ms"} (sv_batch_autotune)."""
    if not isinstance(observables, (list, tuple)):
        observables = [observables] * len(circuits)
    descs, keep = _circuit_descs(circuits, observables)
    flat = np.concatenate([np.asarray(c.params, dtype=np.float64).reshape(-1) for c in circuits])
    p, _ = _params_ptr(flat)
    tb, lb, gb, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
    _check(lib().sv_batch_autotune(descs, len(circuits), SV_C128 if dtype == "c128" else SV_C64,
                                   p.ctypes.data_as(C.POINTER(C.c_double)), reps,
                                   _stream_ptr(stream), C.byref(tb), C.byref(lb), C.byref(gb),
                                   C.byref(ms)))
    del keep
    return {"tile_bits": tb.value, "low_bits": lb.value, "group_bits": gb.value, "ms": ms.value}


class Batch:
    """A ragged batch of independent circuits run as one persistent launch
    (sv_batch_*).  `circuits` are objects with .n .ops .params (a Circuit of
    paper_2608_09733_amd.inputs); `observables` one Hamiltonian per circuit
    (or one shared by all).  Results are sum_j c_j <P_j> per circuit."""

    def __init__(self, circuits, observables, dtype: str = "c128", tile_bits: int = 0,
                 low_bits: int = 0, group_bits: int = 0):
        L = lib()
        self.nc = len(circuits)
        if not isinstance(observables, (list, tuple)):
            observables = [observables] * self.nc
        if len(observables) != self.nc:
            raise ValueError("one observable per circuit")
        self.dtype = dtype
        descs, self._keep = _circuit_descs(circuits, observables)
        h = C.c_void_p()
        _check(L.sv_batch_plan(descs, self.nc, SV_C128 if dtype == "c128" else SV_C64,
                               tile_bits, low_bits, group_bits, C.byref(h)))
        self.h = h
        self.n_qubits = [int(c.n) for c in circuits]
        self.n_params = [int(len(c.params)) for c in circuits]
        self.set_params([c.params for c in circuits])

    def close(self):
        if getattr(self, "h", None):
            lib().sv_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params_per_circuit):
        flat = np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1)
                               for p in params_per_circuit]) if self.nc else np.zeros(0)
        p, n = _params_ptr(flat)
        _check(lib().sv_batch_upload_params(self.h, p.ctypes.data_as(C.POINTER(C.c_double)), n))

    def run(self, stream=None, graph: bool = False):
        f = lib().sv_batch_graph_launch if graph else lib().sv_batch_run
        _check(f(self.h, _stream_ptr(stream)))

    def check(self, stream=None):
        _check(lib().sv_batch_check(self.h, _stream_ptr(stream)))

    def set_spin_limit(self, polls: int):
        _check(lib().sv_batch_set_spin_limit(self.h, int(polls)))

    def results(self, stream=None) -> np.ndarray:
        """Synchronise, verify the run, return the per-circuit observables."""
        self.check(stream)
        out = np.zeros(max(1, self.nc), dtype=np.float64)
        _check(lib().sv_batch_copy_results(self.h, out.ctypes.data_as(C.POINTER(C.c_double)),
                                           _stream_ptr(stream)))
        return out[:self.nc]

    def state(self, k: int, stream=None) -> np.ndarray:
        N = 1 << self.n_qubits[k]
        dt = np.float64 if self.dtype == "c128" else np.float32
        r = np.zeros(N, dtype=dt)
        i = np.zeros(N, dtype=dt)
        _check(lib().sv_batch_copy_state(self.h, k, r.ctypes.data_as(C.c_void_p),
                                         i.ctypes.data_as(C.c_void_p), _stream_ptr(stream)))
        return r.astype(np.float64) + 1j * i.astype(np.float64)

    def stats(self) -> Tuple[int, int, float, float]:
        """(work units, sweeps, gate-amplitude updates, algorithmic HBM bytes) of one run."""
        u, s, up, by = C.c_int64(), C.c_int64(), C.c_double(), C.c_double()
        _check(lib().sv_batch_stats(self.h, C.byref(u), C.byref(s), C.byref(up), C.byref(by)))
        return u.value, s.value, up.value, by.value


class Serve:
    """Small adjoint requests run whole, one workgroup per request, in one
    persistent launch per submission (sv_serve_*).  A request is a circuit
    (.n .ops .params) and an observable; each returns E and dE/dtheta."""

    def __init__(self):
        h = C.c_void_p()
        _check(lib().sv_serve_create(C.byref(h)))
        self.h = h

    @staticmethod
    def max_qubits() -> int:
        return int(lib().sv_serve_max_qubits())

    def close(self):
        if getattr(self, "h", None):
            lib().sv_serve_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def supports(self, circuit, ham) -> bool:
        """True if the serving kernel takes this request (plans get cached);
        False if it must go through State.adjoint_grad."""
        descs, keep = _circuit_descs([circuit], [ham])
        st = lib().sv_serve_check(self.h, descs)
        del keep
        if st == -5:     # SV_EUNSUPPORTED
            return False
        _check(st)
        return True

    def submit(self, circuits, observables, out_tensor, stream=None):
        """Enqueue the requests on `stream`; `out_tensor` (FP64 device, at
        least sum(1 + n_params) elements) receives per request E then the
        gradient, concatenated in request order.  Returns the offsets."""
        descs, keep = _circuit_descs(circuits, observables)
        flat = (np.concatenate([np.asarray(c.params, dtype=np.float64).reshape(-1) for c in circuits])
                if circuits else np.zeros(0))
        p, _ = _params_ptr(flat)
        offs = np.zeros(len(circuits) + 1, dtype=np.int64)
        offs[1:] = np.cumsum([1 + len(c.params) for c in circuits])
        if out_tensor.numel() < offs[-1]:
            raise ValueError(f"output holds {out_tensor.numel()} values, {offs[-1]} needed")
        _check(lib().sv_serve_submit(self.h, descs, len(circuits),
                                     p.ctypes.data_as(C.POINTER(C.c_double)),
                                     C.c_void_p(out_tensor.data_ptr()), _stream_ptr(stream)))
        del keep
        return offs
