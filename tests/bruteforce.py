"""Brute-force dense reference for n <= 6 (pins the oracle; test-only).

Every gate becomes a full 2^n x 2^n matrix built by Kronecker products and an
explicit qubit permutation; rotation and phase gates come from the matrix
exponential of their generators (scipy.linalg.expm), fixed gates from their
textbook matrices.  Nothing here shares code with the oracle or the HIP path.
"""
from __future__ import annotations

import math
from functools import reduce

import numpy as np
from scipy.linalg import expm, sqrtm

I2 = np.eye(2, dtype=complex)
PX = np.array([[0, 1], [1, 0]], dtype=complex)
PY = np.array([[0, -1j], [1j, 0]], dtype=complex)
PZ = np.array([[1, 0], [0, -1]], dtype=complex)
PAULI = {"I": I2, "X": PX, "Y": PY, "Z": PZ}


def kron_all(ms):
    return reduce(np.kron, ms)


def _embed_sub(d, a, b, m2):
    """Embed a 2x2 operator on the span of local basis states a, b."""
    g = np.zeros((d, d), dtype=complex)
    g[np.ix_([a, b], [a, b])] = m2
    return g


def local_matrix(kind: str, th) -> np.ndarray:
    """Matrix on the gate's targets; local index = sum_i bit(t_i) 2^i, so the
    first target is the rightmost Kronecker factor."""
    if kind == "i":
        return I2
    if kind == "x":
        return PX
    if kind == "y":
        return PY
    if kind == "z":
        return PZ
    if kind == "h":
        return (PX + PZ) / math.sqrt(2)
    if kind == "s":
        return expm(1j * math.pi / 4 * (I2 - PZ))
    if kind == "sdg":
        return expm(-1j * math.pi / 4 * (I2 - PZ))
    if kind == "t":
        return expm(1j * math.pi / 8 * (I2 - PZ))
    if kind == "tdg":
        return expm(-1j * math.pi / 8 * (I2 - PZ))
    if kind == "sx":
        return sqrtm(PX)
    if kind == "rx":
        return expm(-0.5j * th[0] * PX)
    if kind == "ry":
        return expm(-0.5j * th[0] * PY)
    if kind == "rz":
        return expm(-0.5j * th[0] * PZ)
    if kind == "p":
        return expm(0.5j * th[0] * (I2 - PZ))
    if kind in ("u3", "u2"):
        if kind == "u3":
            t, f, l = th
        else:
            t, f, l = math.pi / 2, th[0], th[1]
        # U3 = e^{i(f+l)/2} RZ(f) RY(t) RZ(l)
        return (np.exp(0.5j * (f + l)) * local_matrix("rz", [f]) @ local_matrix("ry", [t])
                @ local_matrix("rz", [l]))
    if kind == "swap":
        m = np.zeros((4, 4), dtype=complex)
        for j in range(4):
            m[((j & 1) << 1) | (j >> 1), j] = 1
        return m
    if kind == "rxx":
        return expm(-0.5j * th[0] * np.kron(PX, PX))
    if kind == "ryy":
        return expm(-0.5j * th[0] * np.kron(PY, PY))
    if kind == "rzz":
        return expm(-0.5j * th[0] * np.kron(PZ, PZ))
    if kind == "givens":
        return expm(-0.5j * th[0] * _embed_sub(4, 1, 2, PY))
    if kind == "dexc":
        return expm(-0.5j * th[0] * _embed_sub(16, 3, 12, PY))
    raise ValueError(kind)


def qubit_perm_matrix(n: int, order) -> np.ndarray:
    """Permutation matrix Q with (Q psi)[c] = psi[b] where bit i of c is bit
    order[i] of b (moves qubit order[i] to position i)."""
    N = 1 << n
    Q = np.zeros((N, N))
    for b in range(N):
        c = 0
        for i, q in enumerate(order):
            c |= ((b >> q) & 1) << i
        Q[c, b] = 1
    return Q


def full_matrix(n: int, op, params) -> np.ndarray:
    th = [params[i] for i in op.params]
    if op.kind == "unitary":
        U = np.asarray(op.matrix, dtype=complex)
    else:
        U = local_matrix(op.kind, th)
    k = len(op.targets)
    nc = len(op.controls)
    if nc:
        proj = np.zeros((1 << nc, 1 << nc))
        proj[op.control_states, op.control_states] = 1
        U = np.kron(proj, U) + np.kron(np.eye(1 << nc) - proj, np.eye(1 << k))
    qs = list(op.targets) + list(op.controls)
    rest = [q for q in range(n) if q not in qs]
    order = qs + rest
    Q = qubit_perm_matrix(n, order)
    big = np.kron(np.eye(1 << len(rest)), U)
    return Q.T @ big @ Q


def circuit_unitary(n: int, ops, params) -> np.ndarray:
    U = np.eye(1 << n, dtype=complex)
    for op in ops:
        U = full_matrix(n, op, params) @ U
    return U


def run(n: int, ops, params) -> np.ndarray:
    return circuit_unitary(n, ops, params)[:, 0]


def pauli_dense(n: int, x: int, z: int) -> np.ndarray:
    facs = []
    for q in range(n - 1, -1, -1):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        facs.append(PY if xb and zb else PX if xb else PZ if zb else I2)
    return kron_all(facs)


def ham_dense(n: int, ham) -> np.ndarray:
    H = np.zeros((1 << n, 1 << n), dtype=complex)
    for x, z, c in zip(ham.x, ham.z, ham.c):
        H += c * pauli_dense(n, int(x), int(z))
    return H
