"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (FP64): max-abs <= 1e-12 per amplitude, expectation values and
gradients; complex64: <= 1e-5 per amplitude.  Every case prints its name
before it touches the GPU.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_09733_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL32 = 1e-5


@pytest.fixture(scope="module")
def sv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2608_09733_amd import sv as _sv
    _sv.lib()
    return _sv


def _say(*a):
    print("[case]", *a, flush=True)


def _forward(sv, circ, fuse, dtype="c128", tiling=None):
    st = sv.State(circ.n, dtype)
    if tiling:
        st.set_tiling(*tiling)
    st.apply(circ.ops, circ.params, fuse=fuse)
    out = st.to_numpy()
    st.close()
    return out


FUSES = [0, 2, 3, 5, -1]


@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 8])
@pytest.mark.parametrize("fuse", FUSES)
def test_random_circuits_all_kinds(sv, n, fuse):
    for seed in range(3):
        circ = I.random_circuit(n, 40, seed=100 * n + seed, max_controls=min(2, n - 1))
        _say("random", n, fuse, seed)
        psi = _forward(sv, circ, fuse)
        ref = O.run_circuit(circ)
        assert np.max(np.abs(psi - ref)) <= TOL, (n, fuse, seed)


@pytest.mark.parametrize("n", [14, 16])
@pytest.mark.parametrize("fuse", [0, 4, -1])
def test_random_circuits_multi_tile(sv, n, fuse):
    circ = I.random_circuit(n, 60, seed=7 + n, max_controls=2)
    _say("random multi-tile", n, fuse)
    psi = _forward(sv, circ, fuse)
    ref = O.run_circuit(circ)
    assert np.max(np.abs(psi - ref)) <= TOL


@pytest.mark.parametrize("fuse", FUSES)
def test_config1_layered_12q(sv, fuse):
    circ = I.layered(12, 20, seed=0)
    _say("cfg1", fuse)
    st = sv.State(12, "c128")
    st.apply(circ.ops, circ.params, fuse=fuse)
    psi = st.to_numpy()
    ref = O.run_circuit(circ)
    assert np.max(np.abs(psi - ref)) <= TOL
    ham = I.hamiltonian(12, [("Z", [q], 1.0) for q in range(12)])
    z, _ = st.expect(ham)
    zr, _, _ = O.expect(12, ref, ham)
    assert np.max(np.abs(z - zr)) <= TOL
    st.close()


@pytest.mark.parametrize("n,L", [(15, 3), (18, 4), (20, 2)])
@pytest.mark.parametrize("tiling", [(13, 3, 5), (12, 3, 5), (13, 4, 5), (12, 4, 4), (13, 3, 4),
                                    (11, 5, 5)])
def test_layered_tilings(sv, n, L, tiling):
    circ = I.layered(n, L, seed=n)
    _say("layered tiling", n, L, tiling)
    psi = _forward(sv, circ, -1, tiling=tiling)
    ref = O.run_circuit(circ)
    assert np.max(np.abs(psi - ref)) <= TOL


def test_hea_and_qft_and_ghz(sv):
    for circ in [I.hea(14, 3, seed=1), I.qft(12), I.ghz(17)]:
        _say("family", circ.n, len(circ.ops))
        for fuse in [0, -1]:
            psi = _forward(sv, circ, fuse)
            ref = O.run_circuit(circ)
            assert np.max(np.abs(psi - ref)) <= TOL


@pytest.mark.parametrize("n", [3, 10, 15])
def test_expectation_random_terms(sv, n):
    circ = I.random_circuit(n, 40, seed=n)
    ham = I.random_hamiltonian(n, 30, seed=n)
    _say("expect", n)
    st = sv.State(n)
    st.apply(circ.ops, circ.params, fuse=-1)
    t, e = st.expect(ham)
    ref = O.run_circuit(circ)
    tr, er, _ = O.expect(n, ref, ham)
    assert np.max(np.abs(t - tr)) <= TOL and abs(e - er) <= TOL
    st.close()


def test_expectation_tfim_many_passes(sv):
    n = 20
    circ = I.layered(n, 2, seed=3)
    ham = I.tfim(n)
    _say("expect tfim", n)
    st = sv.State(n)
    st.apply(circ.ops, circ.params, fuse=-1)
    t, e = st.expect(ham)
    ref = O.run_circuit(circ)
    tr, er, _ = O.expect(n, ref, ham)
    assert np.max(np.abs(t - tr)) <= TOL and abs(e - er) <= TOL
    st.close()


@pytest.mark.parametrize("n,L,seed", [(6, 3, 0), (12, 3, 1), (16, 2, 2)])
def test_adjoint_hea_tfim(sv, n, L, seed):
    circ = I.hea(n, L, seed=seed)
    ham = I.tfim(n)
    _say("adjoint hea", n, L, seed)
    st = sv.State(n, adjoint=True)
    e, g = st.adjoint_grad(circ.ops, circ.params, ham)
    er, gr = O.adjoint_grad(circ, ham)
    assert abs(e - er) <= TOL
    assert np.max(np.abs(g - gr)) <= TOL
    # the state holds U|0> on return
    psi = st.to_numpy()
    assert np.max(np.abs(psi - O.run_circuit(circ))) <= TOL
    st.close()


def test_adjoint_general_generators(sv):
    # every parameterised kind, with controls (control states included):
    # Pauli rotations, phases, U2 / U3 (split into P RY P under the same
    # controls), and the excitation gates, whose generator is the Pauli-Y of
    # the rotated pair of basis patterns
    n = 7
    kinds = ["rx", "ry", "rz", "p", "rxx", "ryy", "rzz", "u3", "u2", "givens", "dexc", "h", "x",
             "swap", "s", "t"]
    for seed in range(6):
        # ops on at most 4 qubits (targets and controls): the backward sweeps'
        # register groups hold 4
        circ = I.random_circuit(n, 50, seed=300 + seed, kinds=kinds, max_controls=2, max_qubits=4)
        # one of each controlled multi-angle kind and controlled excitation, for certain
        k = circ.n_params
        extra = [I.Op("u3", (seed % n,), ((seed + 3) % n,), 0, (k, k + 1, k + 2)),
                 I.Op("u2", ((seed + 1) % n,), ((seed + 4) % n, (seed + 5) % n), 2, (k + 3, k + 4)),
                 I.Op("givens", ((seed + 2) % n, (seed + 6) % n), ((seed + 1) % n,), 1, (k + 5,)),
                 I.Op("dexc", (0, 2, 4, 6), (), None, (k + 6,))]
        rng = np.random.default_rng(seed)
        ops = list(circ.ops[:25]) + extra[:2] + list(circ.ops[25:]) + extra[2:]
        circ = I.Circuit(n, ops, np.concatenate([circ.params, rng.uniform(-3, 3, 7)]))
        ham = I.random_hamiltonian(n, 8, seed=seed)
        _say("adjoint general", seed)
        st = sv.State(n, adjoint=True)
        e, g = st.adjoint_grad(circ.ops, circ.params, ham)
        er, gr = O.adjoint_grad(circ, ham)
        assert abs(e - er) <= TOL
        assert np.max(np.abs(g - gr)) <= 1e-11
        st.close()


@pytest.mark.parametrize("kind", ["givens", "dexc"])
def test_adjoint_excitation_gates_closed_form(sv, kind):
    # E = <X0> after H on every qubit and the excitation: cos(t/2) for a
    # Givens rotation, 3/4 + cos(t/2)/4 for a double excitation; the
    # gradient is the derivative of that closed form
    n = 2 if kind == "givens" else 4
    ops = [I.Op("h", (q,)) for q in range(n)] + [I.Op(kind, tuple(range(n)), params=(0,))]
    ham = I.hamiltonian(n, [("X", [0], 1.0)])
    for t in [0.4, 2.3, -1.9]:
        _say("excitation closed form", kind, t)
        st = sv.State(n, adjoint=True)
        e, g = st.adjoint_grad(ops, [t], ham)
        st.close()
        if kind == "givens":
            ew, gw = math.cos(t / 2), -math.sin(t / 2) / 2
        else:
            ew, gw = 0.75 + math.cos(t / 2) / 4, -math.sin(t / 2) / 8
        assert abs(e - ew) <= TOL and abs(g[0] - gw) <= TOL


def test_adjoint_refuses_five_qubit_ops(sv):
    # a controlled double excitation acts on 5 qubits: refused before any
    # device work, state untouched
    n = 6
    st = sv.State(n, adjoint=True)
    before = st.to_numpy()
    with pytest.raises(sv.SvError) as ei:
        st.adjoint_grad([I.Op("dexc", (0, 1, 2, 3), (4,), None, (0,))], [0.3], I.tfim(n))
    assert ei.value.status == -5
    assert np.array_equal(before, st.to_numpy())
    st.close()


def test_adjoint_config3_zero_angle_closed_form(sv):
    # 20-qubit HEA, 10 layers, 400 parameters, TFIM h = 0.7: at all-zero angles
    # E = n - 1, dE/dtheta(RY) = 0.7, dE/dphi(RZ) = 0.
    n, L = 20, 10
    circ = I.hea(n, L)
    p = np.zeros(circ.n_params)
    _say("cfg3 zero angles")
    st = sv.State(n, adjoint=True)
    e, g = st.adjoint_grad(circ.ops, p, I.tfim(n))
    assert abs(e - 19.0) <= TOL
    assert np.max(np.abs(g[0::2] - 0.7)) <= TOL
    assert np.max(np.abs(g[1::2])) <= TOL
    st.close()


def test_adjoint_config3_vs_oracle(sv):
    n, L = 20, 10
    circ = I.hea(n, L, seed=0)
    ham = I.tfim(n)
    _say("cfg3 random angles")
    st = sv.State(n, adjoint=True)
    e, g = st.adjoint_grad(circ.ops, circ.params, ham)
    er, gr = O.adjoint_grad(circ, ham)
    assert abs(e - er) <= TOL
    assert np.max(np.abs(g - gr)) <= TOL
    st.close()


@pytest.mark.parametrize("n", [3, 9, 12, 16, 22])
def test_sampling_bit_exact(sv, n):
    circ = I.layered(n, 3, seed=n)
    _say("sample", n)
    st = sv.State(n)
    st.apply(circ.ops, circ.params, fuse=-1)
    qubits = list(range(n))[::-1]
    got = st.sample(seed=12345, shots=10000, qubits=qubits)
    # contract A: the specification applied to the GPU's own state
    psi_gpu = st.to_numpy()
    a = O.sample(n, psi_gpu, 12345, 10000, qubits)
    assert np.array_equal(got, a)
    # contract B: the oracle's state gives the same draws on this seed
    b = O.sample(n, O.run_circuit(circ), 12345, 10000, qubits)
    assert np.array_equal(got, b)
    # fewer shots take the per-lane draw kernel instead of the cooperative one
    few = st.sample(seed=99, shots=1000, qubits=qubits)
    assert np.array_equal(few, O.sample(n, psi_gpu, 99, 1000, qubits))
    st.close()


def _dyadic_state(n, seed):
    # one power-of-two amplitude per chunk of 1024: exact partial sums
    K = 1 << (n - 10)
    rng = np.random.default_rng(seed)
    psi = np.zeros(1 << n, dtype=complex)
    pos = np.arange(K) * 1024 + rng.integers(0, 1024, size=K)
    psi[pos] = 2.0 ** -rng.integers(11, 14, size=K).astype(float)
    return psi


def _rounding_state(n):
    # chunk sum 1 first, 2^-53 for every other chunk: the blocked prefix
    # total is 1 + 2^-43 only when the blocks are summed as specified
    psi = np.zeros(1 << n, dtype=complex)
    psi[0] = 1.0
    psi[1024::1024] = 2.0 ** -27 * (1 + 1j)
    return psi


@pytest.mark.parametrize("case", ["dyadic22", "rounding21", "layered23"])
def test_sampling_blocked_prefix_states(sv, case):
    # several prefix blocks (K > 1024 chunks): GPU draws equal the
    # specification's on the same state, bit for bit
    _say("sample blocked", case)
    if case == "dyadic22":
        n, psi = 22, _dyadic_state(22, 9)
    elif case == "rounding21":
        n, psi = 21, _rounding_state(21)
    else:
        n = 23
        psi = None
    st = sv.State(n)
    if psi is None:
        circ = I.layered(n, 2, seed=3)
        st.apply(circ.ops, circ.params, fuse=-1)
        psi = st.to_numpy()
    else:
        st.set_planes(psi.real.copy(), psi.imag.copy())
    qubits = list(range(n))
    got = st.sample(seed=777, shots=20000, qubits=qubits)
    want = O.sample(n, psi, 777, 20000, qubits)
    assert np.array_equal(got, want)
    if case == "rounding21":
        # the heavy amplitude takes every draw below 1 / (1 + 2^-43)
        assert np.count_nonzero(got == 0) >= 19990
    st.close()


@pytest.mark.parametrize("n", [4, 12, 17])
def test_complex64_forward(sv, n):
    circ = I.layered(n, 6, seed=n)
    _say("c64", n)
    psi = _forward(sv, circ, -1, dtype="c64")
    ref = O.run_circuit(circ)
    err = float(np.max(np.abs(psi - ref)))
    print(f"complex64 n={n}: max|err| = {err:.3e}", flush=True)
    assert err <= TOL32


def test_complex64_adjoint(sv):
    n = 10
    circ = I.hea(n, 3, seed=4)
    ham = I.tfim(n)
    _say("c64 adjoint")
    st = sv.State(n, "c64", adjoint=True)
    e, g = st.adjoint_grad(circ.ops, circ.params, ham)
    er, gr = O.adjoint_grad(circ, ham)
    assert abs(e - er) <= 1e-4 and np.max(np.abs(g - gr)) <= 1e-4
    st.close()


def test_determinism_bitwise(sv):
    circ = I.hea(16, 3, seed=9)
    ham = I.tfim(16)
    _say("determinism")
    outs = []
    for _ in range(2):
        st = sv.State(16, adjoint=True)
        e, g = st.adjoint_grad(circ.ops, circ.params, ham)
        outs.append((e, g.copy(), st.to_numpy()))
        st.close()
    assert outs[0][0] == outs[1][0]
    assert np.array_equal(outs[0][1], outs[1][1])
    assert np.array_equal(outs[0][2], outs[1][2])


def test_errors_rejected_before_device_work(sv):
    st = sv.State(4)
    before = st.to_numpy()
    bad = [I.Op("x", (5,))]
    with pytest.raises(sv.SvError) as ei:
        st.apply(bad, [], fuse=-1)
    assert ei.value.status == -1
    with pytest.raises(sv.SvError) as ei:
        st.apply([I.Op("ry", (0,), params=(3,))], [0.1], fuse=-1)
    assert ei.value.status == -3
    with pytest.raises(sv.SvError) as ei:
        st.apply([I.Op("ry", (0,), params=(0,))], [math.nan], fuse=-1)
    assert ei.value.status == -3
    with pytest.raises(sv.SvError):
        st.apply([I.Op("ry", (0,), params=(0,))], [0.1], fuse=1)
    with pytest.raises(sv.SvError) as ei:
        st.adjoint_grad([I.Op("ry", (0,), params=(0,))], [0.1], I.tfim(4))
    assert ei.value.status == -4   # workspace without adjoint room
    assert np.array_equal(before, st.to_numpy())
    st.close()


def test_reset_is_lazy_and_exact(sv):
    # sv_reset defers |0..0>: the next sweep synthesises it, other readers write it
    n = 14
    circ = I.layered(n, 2, seed=5)
    st = sv.State(n)
    st.apply(circ.ops, circ.params, fuse=-1)
    st.reset()
    psi0 = st.to_numpy()
    assert psi0[0] == 1 and np.count_nonzero(psi0) == 1
    st.apply(circ.ops, circ.params, fuse=-1)
    st.reset()
    z, _ = st.expect(I.hamiltonian(n, [("Z", [q], 1.0) for q in range(n)]))
    assert np.all(z == 1.0)
    st.reset()
    st.apply(circ.ops, circ.params, fuse=-1)
    assert np.max(np.abs(st.to_numpy() - O.run_circuit(circ))) <= TOL
    st.reset()
    st.apply(circ.ops, circ.params, fuse=0)     # first step is a gate kernel: materialised
    assert np.max(np.abs(st.to_numpy() - O.run_circuit(circ))) <= TOL
    st.close()


def test_expectation_z_terms_and_lambda_large(sv):
    # many Z-only terms (thread/row parity split) and X/Y terms in one pass
    n = 17
    circ = I.random_circuit(n, 60, seed=71)
    ham = I.random_hamiltonian(n, 40, seed=9)
    zham = I.hamiltonian(n, [("Z" * (q % 5 + 1), list(range(q, q + q % 5 + 1)), 0.1 * q)
                             for q in range(n - 5)])
    st = sv.State(n, adjoint=True)
    st.apply(circ.ops, circ.params, fuse=-1)
    ref = O.run_circuit(circ)
    for h in (ham, zham):
        t, e = st.expect(h)
        tr, er, _ = O.expect(n, ref, h)
        assert np.max(np.abs(t - tr)) <= TOL and abs(e - er) <= TOL
    st.close()


@pytest.mark.parametrize("n,dtype", [(14, "c128"), (19, "c128"), (18, "c64")])
def test_expectation_diagonal_stream(sv, n, dtype):
    # more Z-only terms than one streamed read holds (two groups), strings on
    # the lowest, middle and highest qubits, the identity term, and X/Y terms
    # in the same call
    circ = I.random_circuit(n, 50, seed=300 + n)
    rng = np.random.default_rng(n)
    spec = [("Z", [q], 0.5) for q in range(n)]
    spec += [("ZZ", [q, (q + 7) % n], -0.25) for q in range(n)]
    spec += [("ZZZ", [0, n // 2, n - 1], 1.5), ("I", [0], 2.0), ("XZ", [1, n - 1], 0.7)]
    spec += [("".join(rng.choice(list("IZ"), n)), list(range(n)), float(rng.normal()))
             for _ in range(6)]
    ham = I.hamiltonian(n, spec)
    assert sum(1 for x in ham.x if int(x) == 0) > 32
    _say("expect diag", n, dtype, len(ham))
    st = sv.State(n, dtype)
    st.apply(circ.ops, circ.params, fuse=-1)
    t, e = st.expect(ham)
    st.close()
    ref = O.run_circuit(circ)
    tr, er, _ = O.expect(n, ref, ham)
    tol = TOL if dtype == "c128" else 4 * TOL32
    assert np.max(np.abs(t - tr)) <= tol and abs(e - er) <= tol * np.sum(np.abs(ham.c))


@pytest.mark.parametrize("tiling", [(13, 3, 4), (12, 3, 3), (13, 3, 5), (12, 4, 4)])
def test_remapped_layout_plans(sv, tiling):
    # tilings whose AUTO plans permute qubits among tile positions between
    # sweeps and restore the layout at the end
    n = 20
    circ = I.layered(n, 8, seed=11)
    _say("remap", tiling)
    psi = _forward(sv, circ, -1, tiling=tiling)
    ref = O.run_circuit(circ)
    assert np.max(np.abs(psi - ref)) <= TOL
    circ2 = I.random_circuit(18, 120, seed=12, max_qubits=3)
    psi2 = _forward(sv, circ2, -1, tiling=tiling)
    assert np.max(np.abs(psi2 - O.run_circuit(circ2))) <= TOL
