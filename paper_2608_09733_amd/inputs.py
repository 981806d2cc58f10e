"""Seeded synthetic inputs shared by the GPU path, the oracle and the tests.

This module only *describes* workloads: gate lists (kind names, qubit indices,
parameter slots), parameter vectors, Pauli-term masks and request traces.  It
holds none of the method's arithmetic (no gate matrices, no amplitudes), so the
oracle and the HIP path can both consume it without sharing any computation.

Circuit model (paper, Section 4.2): an ordered list of typed operations; each
operation names its targets first, then its controls, with optional control
states (a control may fire on |0>).  Parameters are bound by index into one
dense vector in first-use order (paper, Section 4.2, parameter binding).

Qubit q is bit q of the basis index (little-endian).  For a multi-target gate
the first target is the least-significant bit of the gate's local index.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Gate vocabulary: name -> (number of targets, number of parameters).
# Each side (oracle, HIP library) maps these names to its own enum and its own
# matrices.
GATES = {
    "i": (1, 0), "x": (1, 0), "y": (1, 0), "z": (1, 0), "h": (1, 0),
    "s": (1, 0), "sdg": (1, 0), "t": (1, 0), "tdg": (1, 0), "sx": (1, 0),
    "rx": (1, 1), "ry": (1, 1), "rz": (1, 1), "p": (1, 1),
    "u2": (1, 2), "u3": (1, 3),
    "swap": (2, 0), "rxx": (2, 1), "ryy": (2, 1), "rzz": (2, 1),
    "givens": (2, 1),      # single excitation on the |01>,|10> pair
    "dexc": (4, 1),        # double excitation on the |0011>,|1100> pair
    "unitary": (None, 0),  # user matrix on 1..5 targets
}


@dataclass(frozen=True)
class Op:
    kind: str
    targets: Tuple[int, ...]
    controls: Tuple[int, ...] = ()
    cstate: Optional[int] = None          # bit i: control i fires on |1>; None = all |1>
    params: Tuple[int, ...] = ()          # indices into the parameter vector
    matrix: Optional[np.ndarray] = field(default=None, compare=False)  # "unitary" only

    @property
    def control_states(self) -> int:
        if self.cstate is None:
            return (1 << len(self.controls)) - 1
        return int(self.cstate)

    @property
    def qubits(self) -> Tuple[int, ...]:
        return tuple(self.targets) + tuple(self.controls)


@dataclass
class Circuit:
    n: int
    ops: List[Op]
    params: np.ndarray                     # float64, length n_params
    # structure key: circuits with equal non-None keys have identical op lists
    # (kinds, qubits, controls, parameter slots); only their angles differ
    key: Optional[Tuple] = None

    @property
    def n_params(self) -> int:
        return int(self.params.shape[0])

    def gate_count(self) -> int:
        return len(self.ops)


@dataclass
class Hamiltonian:
    """H = sum_j c_j P_j as (x_mask, z_mask, coeff) triples (paper eq. for the
    Pauli action: x marks X or Y, z marks Z or Y)."""
    n: int
    x: np.ndarray   # uint64
    z: np.ndarray   # uint64
    c: np.ndarray   # float64

    def __len__(self) -> int:
        return int(self.c.shape[0])


def pauli_term(spec: str, qubits: Sequence[int]) -> Tuple[int, int]:
    """Masks of a Pauli string given per-qubit letters, e.g. ("ZZ", [0, 3])."""
    x = z = 0
    for ch, q in zip(spec.upper(), qubits):
        if ch == "X":
            x |= 1 << q
        elif ch == "Z":
            z |= 1 << q
        elif ch == "Y":
            x |= 1 << q
            z |= 1 << q
        elif ch != "I":
            raise ValueError(f"bad Pauli letter {ch!r}")
    return x, z


def hamiltonian(n: int, terms: Sequence[Tuple[str, Sequence[int], float]]) -> Hamiltonian:
    xs, zs, cs = [], [], []
    for spec, qs, c in terms:
        x, z = pauli_term(spec, qs)
        xs.append(x)
        zs.append(z)
        cs.append(float(c))
    return Hamiltonian(n, np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64),
                       np.array(cs, dtype=np.float64))


# ---------------------------------------------------------------- workloads

def layered_structure(n: int, layers: int) -> List[Op]:
    """Layered ansatz: per layer RY then RZ on every qubit (interleaved per
    qubit), followed by the CNOT ladder control i -> target i+1, i = 0..n-2.
    Parameter slot of (layer l, qubit q, axis a) is l*2n + 2q + a."""
    ops: List[Op] = []
    for l in range(layers):
        for q in range(n):
            ops.append(Op("ry", (q,), params=(l * 2 * n + 2 * q,)))
            ops.append(Op("rz", (q,), params=(l * 2 * n + 2 * q + 1,)))
        for i in range(n - 1):
            ops.append(Op("x", (i + 1,), (i,)))
    return ops


def _layer_angles(rng: np.random.Generator, n: int, layers: int) -> np.ndarray:
    theta = rng.uniform(0.0, 2.0 * math.pi, (layers, n))
    phi = rng.uniform(0.0, 2.0 * math.pi, (layers, n))
    p = np.empty((layers, n, 2), dtype=np.float64)
    p[:, :, 0] = theta
    p[:, :, 1] = phi
    return p.reshape(-1)


def layered(n: int, layers: int, seed: int = 0) -> Circuit:
    rng = np.random.default_rng(seed)
    return Circuit(n, layered_structure(n, layers), _layer_angles(rng, n, layers))


def hea_structure(n: int, layers: int) -> List[Op]:
    """Hardware-efficient ansatz: per layer RY, RZ on every qubit (interleaved),
    then the CZ ring CZ(q, (q+1) mod n) for q = 0..n-1."""
    ops: List[Op] = []
    for l in range(layers):
        for q in range(n):
            ops.append(Op("ry", (q,), params=(l * 2 * n + 2 * q,)))
            ops.append(Op("rz", (q,), params=(l * 2 * n + 2 * q + 1,)))
        if n >= 2:
            for q in range(n):
                a, b = q, (q + 1) % n
                if n == 2 and q == 1:
                    break
                ops.append(Op("z", (b,), (a,)))
    return ops


def hea(n: int, layers: int, seed: int = 0) -> Circuit:
    rng = np.random.default_rng(seed)
    return Circuit(n, hea_structure(n, layers), _layer_angles(rng, n, layers))


def tfim(n: int, h: float = 0.7) -> Hamiltonian:
    """Open-chain transverse-field Ising model sum Z_i Z_{i+1} + h sum X_i."""
    terms = [("ZZ", (i, i + 1), 1.0) for i in range(n - 1)]
    terms += [("X", (i,), h) for i in range(n)]
    return hamiltonian(n, terms)


def ghz(n: int) -> Circuit:
    ops = [Op("h", (0,))] + [Op("x", (i + 1,), (i,)) for i in range(n - 1)]
    return Circuit(n, ops, np.zeros(0))


def qft(n: int) -> Circuit:
    """Swap-free QFT: for j = n-1..0: H(j), then controlled phases with control
    k and target j for k = j-1..0, angle 2*pi/2^(j-k+1).  n H + n(n-1)/2 CP."""
    ops: List[Op] = []
    params: List[float] = []
    for j in range(n - 1, -1, -1):
        ops.append(Op("h", (j,)))
        for k in range(j - 1, -1, -1):
            params.append(2.0 * math.pi / float(1 << (j - k + 1)))
            ops.append(Op("p", (j,), (k,), params=(len(params) - 1,)))
    return Circuit(n, ops, np.array(params, dtype=np.float64))


def batch_circuits(count: int = 512, seed: int = 0, n_lo: int = 8, n_hi: int = 22,
                   l_lo: int = 10, l_hi: int = 40) -> List[Circuit]:
    """Ragged batch: per circuit n ~ U{n_lo..n_hi}, L ~ U{l_lo..l_hi} drawn first
    for all circuits, then the angles in circuit order."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, count)
    ls = rng.integers(l_lo, l_hi + 1, count)
    out = []
    for n, L in zip(ns, ls):
        out.append(Circuit(int(n), layered_structure(int(n), int(L)),
                           _layer_angles(rng, int(n), int(L))))
    return out


def z0z1(n: int) -> Hamiltonian:
    return hamiltonian(n, [("ZZ", (0, 1), 1.0)])


@dataclass
class Request:
    rid: int
    arrival: float     # seconds from trace start
    circuit: Circuit
    ham: Hamiltonian


def serving_trace(rate: float, count: int = 2000, seed: int = 0, n_lo: int = 10,
                  n_hi: int = 28, l_lo: int = 4, l_hi: int = 30) -> List[Request]:
    """Poisson arrivals at `rate` req/s.  Per request n = clip(round(exp(U[ln n_lo,
    ln n_hi])), n_lo, n_hi), L ~ U{l_lo..l_hi}, angles U[0, 2pi), TFIM(h=0.7)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for i in range(count):
        n = int(np.clip(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))), n_lo, n_hi))
        L = int(rng.integers(l_lo, l_hi + 1))
        circ = Circuit(n, layered_structure(n, L), _layer_angles(rng, n, L), key=("layered", n, L))
        reqs.append(Request(i, float(t[i]), circ, tfim(n)))
    return reqs


def random_circuit(n: int, depth: int, seed: int = 0, kinds: Optional[Sequence[str]] = None,
                   max_controls: int = 2, allow_unitary: bool = True,
                   max_qubits: int = 5) -> Circuit:
    """Random circuit over the whole vocabulary, with random target/control
    orderings and random control states; every op gets fresh parameters.
    Each op touches at most `max_qubits` qubits (targets + controls)."""
    rng = np.random.default_rng(seed)
    if kinds is None:
        kinds = [k for k in GATES if k != "unitary" or allow_unitary]
    ops: List[Op] = []
    params: List[float] = []
    for _ in range(depth):
        kind = str(rng.choice(list(kinds)))
        nt, npar = GATES[kind]
        if kind == "unitary":
            nt = int(rng.integers(1, min(3, n) + 1))
        if nt > n or nt > max_qubits:
            continue
        perm = rng.permutation(n)
        targets = tuple(int(q) for q in perm[:nt])
        nc = int(rng.integers(0, max(0, min(max_controls, n - nt, max_qubits - nt)) + 1))
        controls = tuple(int(q) for q in perm[nt:nt + nc])
        cstate = int(rng.integers(0, 1 << nc)) if nc else None
        pidx = []
        for _ in range(npar):
            params.append(float(rng.uniform(-2 * math.pi, 2 * math.pi)))
            pidx.append(len(params) - 1)
        mat = None
        if kind == "unitary":
            d = 1 << nt
            a = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
            qm, r = np.linalg.qr(a)
            mat = qm * (np.diag(r) / np.abs(np.diag(r)))
        ops.append(Op(kind, targets, controls, cstate, tuple(pidx), mat))
    return Circuit(n, ops, np.array(params, dtype=np.float64))


def random_hamiltonian(n: int, n_terms: int, seed: int = 0) -> Hamiltonian:
    rng = np.random.default_rng(seed)
    terms = []
    for _ in range(n_terms):
        letters = rng.choice(list("IXYZ"), n)
        c = float(rng.normal())
        terms.append(("".join(letters), list(range(n)), c))
    return hamiltonian(n, terms)


def random_state(n: int, seed: int = 0) -> Tuple[np.ndarray, np.ndarray]:
    """A normalised random state as (re, im) float64 planes."""
    rng = np.random.default_rng(seed)
    re = rng.normal(size=1 << n)
    im = rng.normal(size=1 << n)
    s = math.sqrt(float(np.sum(re * re + im * im)))
    return re / s, im / s
