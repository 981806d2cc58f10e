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
        L.orc_sample_at.argtypes = [C.c_int, dp, dp, C.c_int64, up]
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


# Shift rules (Section 4.2: a gate's generator fixes its rule).  For one
# occurrence of a parameter in a gate U(theta) = exp(-i theta G / 2), the
# energy as a function of that occurrence is a trigonometric polynomial whose
# frequencies are half the differences of G's eigenvalues:
#   * G with eigenvalues {-1, +1} (Pauli rotations) or {0, -2} (phase gates):
#     frequency 1, and dE/dtheta = [E(theta + pi/2) - E(theta - pi/2)] / 2
#     (the paper's two-term rule, eq. 2);
#   * G with eigenvalues {-1, 0, +1} (single and double excitations, and any
#     rotation under a control, which adds the eigenvalue 0 on the
#     non-firing subspace): frequencies 1/2 and 1.  With
#     E(theta + x) = a + b1 sin(x/2) + b2 sin(x) + (even terms) the odd part
#     E(theta + x) - E(theta - x) = 2 b1 sin(x/2) + 2 b2 sin(x) at x = pi/2
#     and 3 pi/2 gives sqrt2 b1 + 2 b2 and sqrt2 b1 - 2 b2, so
#     dE/dtheta = b1/2 + b2 = c+ [E(+pi/2) - E(-pi/2)] + c- [E(+3pi/2) - E(-3pi/2)]
#     with c+ = (2 + sqrt2)/8 and c- = (sqrt2 - 2)/8: the four-term rule the
#     paper selects for excitation gates (published form: Anselmetti et al.
#     2021; Wierichs et al. 2022).
# A parameter read by several gates sums one such derivative per occurrence
# (each occurrence shifted alone through an extra parameter slot).
TWO_TERM = ((math.pi / 2, 0.5),)
FOUR_TERM = ((math.pi / 2, (2 + math.sqrt(2)) / 8), (3 * math.pi / 2, (math.sqrt(2) - 2) / 8))


def shift_rule(op, slot: int):
    """Shift rule of parameter slot `slot` of gate `op`: ((shift, weight), ...)
    with dE/dtheta = sum_k weight_k [E(theta + shift_k) - E(theta - shift_k)]."""
    if op.kind in ("givens", "dexc"):
        return FOUR_TERM
    if op.kind == "p" or (op.kind in ("u2", "u3") and not (op.kind == "u3" and slot == 0)):
        return TWO_TERM                   # phases: eigenvalues {0, -2}, controlled or not
    if op.kind in ("rx", "ry", "rz", "rxx", "ryy", "rzz", "u3"):
        return FOUR_TERM if op.controls else TWO_TERM
    raise ValueError(f"no shift rule for {op.kind}")


def param_shift_grad(circ, ham, indices: Sequence[int]) -> np.ndarray:
    """dE/dtheta_i for each i by the shift rules above, one occurrence at a time."""
    from dataclasses import replace
    base = np.array(circ.params, dtype=np.float64)
    extra = len(base)
    out = []
    for i in indices:
        g = 0.0
        for k, op in enumerate(circ.ops):
            for w, pi in enumerate(op.params):
                if pi != i:
                    continue
                pidx = list(op.params)
                pidx[w] = extra
                ops = list(circ.ops)
                ops[k] = replace(op, params=tuple(pidx))
                for shift, weight in shift_rule(op, w):
                    p = np.concatenate([base, [base[i] + shift]])
                    ep = energy(type(circ)(circ.n, ops, p), ham)
                    p[extra] = base[i] - shift
                    em = energy(type(circ)(circ.n, ops, p), ham)
                    g += weight * (ep - em)
        out.append(g)
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


def sample_at(n: int, psi: np.ndarray, t) -> np.ndarray:
    """Basis index drawn for each target value t (steps 5-6 of the sampling
    specification; the sampler itself uses t = u_s * T)."""
    z = np.ascontiguousarray(np.asarray(psi, dtype=np.complex128)).view(np.float64)
    tt = np.ascontiguousarray(np.atleast_1d(np.asarray(t, dtype=np.float64)))
    out = np.zeros(max(1, tt.size), dtype=np.uint64)
    if lib().orc_sample_at(n, _dp(z), _dp(tt), tt.size, _up(out)):
        raise ValueError("bad sample arguments")
    return out[:tt.size]


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


# ------------------------------------------------------------ shot readout
# Terminal readout with a finite number of shots (Section 4.4).  Readout at
# the end of a circuit gives counts of the drawn bit strings.  The estimator
# measures each Pauli term after a per-qubit basis change; terms that agree on
# every qubit they share are measured together, a fixed number of shots is
# divided among those groups, and the result is each term's value, the energy
# and an estimate of its variance.  The paper fixes neither the grouping rule, nor the split, nor the
# variance; the readings implemented here:
#   * terms are taken in order; an identity term is exact (value 1, no shots);
#     any other term joins the first group whose measurement basis agrees
#     with it on every qubit both act on, else it opens a new group;
#   * group g of G draws floor(S/G) shots, one more when g < S mod G, with
#     seed + g, from its rotated state by the sampling specification, reading
#     the group's qubits in increasing order;
#   * rotation into the Z basis: H on an X qubit; S^dagger, then H, on a Y qubit;
#   * a term's value is (N - 2*odd) / N, odd = the number of the group's N
#     shots whose bits on the term's qubits have odd parity;
#   * per group, y = sum_j c_j s_j over its terms (s_j = +-1 per shot) has the
#     empirical variance Var(y) = sum_j sum_k c_j c_k (v_jk - v_j v_k), v_jk the
#     value of the parity over the symmetric difference of the two terms'
#     qubits; the reported variance of the energy is sum_g Var(y_g) / N_g;
#   * energy = sum_j c_j v_j, in term order.


class _Gate:
    """Minimal gate record for the oracle's own basis rotations."""

    def __init__(self, kind, q):
        self.kind = kind
        self.targets = (q,)
        self.controls = ()
        self.control_states = 0
        self.params = ()
        self.matrix = None


def _letters(x: int, z: int, n: int):
    out = {}
    for q in range(n):
        bx, bz = (x >> q) & 1, (z >> q) & 1
        if bx or bz:
            out[q] = "Y" if (bx and bz) else ("X" if bx else "Z")
    return out


def qwc_groups(ham):
    """Greedy qubit-wise-commuting groups: list of (term indices, {qubit: letter})."""
    groups = []
    for j in range(len(ham)):
        let = _letters(int(ham.x[j]), int(ham.z[j]), ham.n)
        if not let:
            continue
        for ids, basis in groups:
            if all(basis.get(q, b) == b for q, b in let.items()):
                ids.append(j)
                basis.update(let)
                break
        else:
            groups.append(([j], dict(let)))
    return groups


def shot_counts(n: int, psi: np.ndarray, seed: int, shots: int, qubits: Sequence[int]) -> np.ndarray:
    """Bit-string counts of `shots` terminal samples of `qubits` (bit i = qubits[i])."""
    s = sample(n, psi, seed, shots, qubits)
    return np.bincount(s.astype(np.int64), minlength=1 << len(qubits)).astype(np.uint64)


def _odd_parity(samples: np.ndarray, mask: int) -> int:
    v = samples & np.uint64(mask)
    par = np.zeros(v.shape, dtype=np.uint64)
    for b in range(64):
        par ^= (v >> np.uint64(b)) & np.uint64(1)
    return int(par.sum())


def shot_estimate(n: int, psi: np.ndarray, seed: int, shots: int, ham):
    """(per-term values, energy, variance of the energy, number of groups)."""
    groups = qwc_groups(ham)
    G = len(groups)
    if G and shots < G:
        raise ValueError("fewer shots than measurement groups")
    values = np.ones(len(ham))
    variance = 0.0
    for g, (ids, basis) in enumerate(groups):
        N = shots // G + (1 if g < shots % G else 0)
        rot = []
        for q in sorted(basis):
            if basis[q] == "X":
                rot.append(_Gate("h", q))
            elif basis[q] == "Y":
                rot.append(_Gate("sdg", q))
                rot.append(_Gate("h", q))
        phi = run(n, rot, [], psi) if rot else np.asarray(psi, dtype=np.complex128)
        support = sorted(basis)
        pos = {q: i for i, q in enumerate(support)}
        smp = sample(n, phi, (seed + g) % (1 << 64), N, support)
        masks = []
        for j in ids:
            m = 0
            for q in _letters(int(ham.x[j]), int(ham.z[j]), n):
                m |= 1 << pos[q]
            masks.append(m)
        v = [(N - 2 * _odd_parity(smp, m)) / N for m in masks]
        for j, vj in zip(ids, v):
            values[j] = vj
        var = 0.0
        for a, j in enumerate(ids):
            for b, k in enumerate(ids):
                vjk = (N - 2 * _odd_parity(smp, masks[a] ^ masks[b])) / N
                var += ham.c[j] * ham.c[k] * (vjk - v[a] * v[b])
        variance += var / N
    energy = 0.0
    for j in range(len(ham)):
        energy += ham.c[j] * values[j]
    return values, energy, variance, G


# ------------------------------------------------------- density matrices
# rho of n qubits as a dense 2^n x 2^n matrix (Section 4.1 density-matrix
# state): gates act as U rho U^dagger, channels as sum_k K rho K^dagger, and
# <P> = Re Tr(rho P).  Written out densely for small n: the full U is built
# column by column with the state-vector oracle, one-qubit Kraus operators and
# Pauli strings by Kronecker products (qubit 0 is the least significant bit).

_PAULI = {"I": np.eye(2, dtype=complex), "X": np.array([[0, 1], [1, 0]], dtype=complex),
          "Y": np.array([[0, -1j], [1j, 0]]), "Z": np.diag([1.0 + 0j, -1.0])}


def dm_unitary(n: int, ops: Sequence, params) -> np.ndarray:
    N = 1 << n
    U = np.zeros((N, N), dtype=complex)
    for b in range(N):
        e = np.zeros(N, dtype=complex)
        e[b] = 1.0
        U[:, b] = run(n, ops, params, e)
    return U


def dm_run(n: int, ops: Sequence, params, rho0: Optional[np.ndarray] = None) -> np.ndarray:
    N = 1 << n
    if rho0 is None:
        rho0 = np.zeros((N, N), dtype=complex)
        rho0[0, 0] = 1.0
    U = dm_unitary(n, ops, params)
    return U @ rho0 @ U.conj().T


def _embed1(n: int, q: int, m: np.ndarray) -> np.ndarray:
    return np.kron(np.kron(np.eye(1 << (n - q - 1)), m), np.eye(1 << q))


def dm_kraus(n: int, rho: np.ndarray, qubit: int, kraus: Sequence[np.ndarray]) -> np.ndarray:
    out = np.zeros_like(rho)
    for K in kraus:
        Kf = _embed1(n, qubit, np.asarray(K, dtype=complex))
        out += Kf @ rho @ Kf.conj().T
    return out


def dm_expect(n: int, rho: np.ndarray, ham) -> Tuple[np.ndarray, float]:
    vals = np.zeros(len(ham))
    for j in range(len(ham)):
        x, z = int(ham.x[j]), int(ham.z[j])
        P = np.eye(1, dtype=complex)
        for q in range(n - 1, -1, -1):
            bx, bz = (x >> q) & 1, (z >> q) & 1
            P = np.kron(P, _PAULI["Y" if bx and bz else "X" if bx else "Z" if bz else "I"])
        vals[j] = np.trace(rho @ P).real
    e = 0.0
    for j in range(len(ham)):
        e += ham.c[j] * vals[j]
    return vals, e


def dm_kraus2(n: int, rho: np.ndarray, q0: int, q1: int, kraus: Sequence[np.ndarray]) -> np.ndarray:
    """sum_k K rho K^dagger for 4x4 Kraus operators on (q0, q1), local index
    bit(q0) + 2 bit(q1); each K is embedded column by column through the
    oracle's own user-matrix gate."""
    N = 1 << n
    out = np.zeros_like(rho)
    for K in kraus:
        g = _Gate("unitary", q0)
        g.targets = (q0, q1)
        g.matrix = np.asarray(K, dtype=complex)
        Kf = np.zeros((N, N), dtype=complex)
        for b in range(N):
            e = np.zeros(N, dtype=complex)
            e[b] = 1.0
            Kf[:, b] = run(n, [g], [], e)
        out += Kf @ rho @ Kf.conj().T
    return out
