"""Pins for the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test checks it against an
independent construction (dense Kronecker products and matrix exponentials for
n <= 6), a closed form, an invariant or a number printed in the paper.
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_09733_amd import inputs as I
from tests import bruteforce as BF

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(v) for v in line.split()])
    return rows


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(O.LIB_PATH):
        from oracle import build
        build.build()


# ------------------------------------------------------------------ gates

@pytest.mark.parametrize("kind", [k for k in I.GATES if k != "unitary"])
def test_gate_matrix_matches_generator_exponential(kind):
    nt, npar = I.GATES[kind]
    rng = np.random.default_rng(hash(kind) % 1000)
    params = rng.uniform(-7, 7, npar)
    op = I.Op(kind, tuple(range(nt)), params=tuple(range(npar)))
    m = O.gate_matrix(op, params)
    ref = BF.local_matrix(kind, list(params))
    assert np.max(np.abs(m - ref)) < 1e-13
    assert np.max(np.abs(m.conj().T @ m - np.eye(m.shape[0]))) < 1e-13


@pytest.mark.parametrize("kind", ["rx", "ry", "rz", "p", "u2", "u3", "rxx", "ryy", "rzz",
                                  "givens", "dexc"])
def test_gate_derivative_matches_central_difference(kind):
    nt, npar = I.GATES[kind]
    rng = np.random.default_rng(7)
    params = rng.uniform(-3, 3, npar)
    op = I.Op(kind, tuple(range(nt)), params=tuple(range(npar)))
    h = 1e-5
    for w in range(npar):
        pp = params.copy()
        pp[w] += h
        mp = BF.local_matrix(kind, list(pp))
        pp[w] -= 2 * h
        mm = BF.local_matrix(kind, list(pp))
        num = (mp - mm) / (2 * h)
        assert np.max(np.abs(O.gate_dmatrix(op, params, w) - num)) < 1e-9


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_random_circuits_match_bruteforce(n, seed):
    circ = I.random_circuit(n, 30, seed=seed * 10 + n, max_controls=min(2, n - 1))
    psi = O.run_circuit(circ)
    ref = BF.run(n, circ.ops, circ.params)
    assert np.max(np.abs(psi - ref)) < 1e-12


def test_arbitrary_initial_state_matches_bruteforce():
    n = 5
    circ = I.random_circuit(n, 25, seed=99)
    re, im = I.random_state(n, seed=3)
    psi0 = re + 1j * im
    out = O.run(n, circ.ops, circ.params, psi0)
    ref = BF.circuit_unitary(n, circ.ops, circ.params) @ psi0
    assert np.max(np.abs(out - ref)) < 1e-12


def test_layered_endianness_sensitive():
    # The layered family is not invariant under bit reversal (paper Section 9.1
    # meta-test), so a flipped convention would fail this comparison.
    circ = I.layered(5, 3, seed=1)
    psi = O.run_circuit(circ)
    ref = BF.run(5, circ.ops, circ.params)
    assert np.max(np.abs(psi - ref)) < 1e-12
    rev = np.array([int(format(b, "05b")[::-1], 2) for b in range(32)])
    assert np.max(np.abs(psi - psi[rev])) > 1e-3


# ------------------------------------------------------- fixed points

@pytest.mark.parametrize("n", [2, 3, 8, 12])
def test_ghz_amplitudes(n):
    psi = O.run_circuit(I.ghz(n))
    ref = np.zeros(1 << n, dtype=complex)
    ref[0] = ref[-1] = 1 / math.sqrt(2)
    assert np.max(np.abs(psi - ref)) < 1e-15


def _rev(v, n):
    return int(format(v, f"0{n}b")[::-1], 2)


@pytest.mark.parametrize("n", [1, 3, 5, 6])
def test_qft_closed_form_every_basis_state(n):
    circ = I.qft(n)
    N = 1 << n
    for x in range(N):
        psi0 = np.zeros(N, dtype=complex)
        psi0[x] = 1
        out = O.run(n, circ.ops, circ.params, psi0)
        y = np.arange(N)
        ry = np.array([_rev(v, n) for v in y])
        ref = np.exp(2j * math.pi * x * ry / N) / math.sqrt(N)
        assert np.max(np.abs(out - ref)) < 1e-13
        # the same map through numpy's inverse FFT (unnormalised DFT with e^{+i})
        fft = np.fft.ifft(psi0) * math.sqrt(N)
        assert np.max(np.abs(out - fft[ry])) < 1e-13


def test_qft_gate_count_matches_paper():
    for n, gates in _load_golden("qft_gate_count.txt"):
        assert I.qft(n).gate_count() == gates


def test_norm_preserved_on_layered_circuit():
    circ = I.layered(14, 20, seed=0)
    psi = O.run_circuit(circ)
    assert abs(np.vdot(psi, psi).real - 1) < 1e-13


def test_config1_shape():
    circ = I.layered(12, 20, seed=0)
    assert circ.gate_count() == 700 and circ.n_params == 480


# -------------------------------------------------------- observables

@pytest.mark.parametrize("n", [1, 2, 4, 6])
def test_expectation_matches_dense_pauli(n):
    circ = I.random_circuit(n, 20, seed=n)
    psi = O.run_circuit(circ)
    ham = I.random_hamiltonian(n, 12, seed=n)
    terms, tot, ims = O.expect(n, psi, ham)
    for j in range(len(ham)):
        P = BF.pauli_dense(n, int(ham.x[j]), int(ham.z[j]))
        ref = np.vdot(psi, P @ psi)
        assert abs(terms[j] - ref.real) < 1e-13
        assert abs(ims[j]) < 1e-13  # Hermitian: imaginary part vanishes
    H = BF.ham_dense(n, ham)
    assert abs(tot - np.vdot(psi, H @ psi).real) < 1e-12


def test_y_string_expectation():
    # A pure Y-string term, the case the paper validates separately (Section 9.3).
    n = 4
    circ = I.random_circuit(n, 25, seed=4)
    psi = O.run_circuit(circ)
    ham = I.hamiltonian(n, [("YYYY", [0, 1, 2, 3], 1.0), ("YXZY", [0, 1, 2, 3], -0.5)])
    terms, _, _ = O.expect(n, psi, ham)
    for j in range(2):
        P = BF.pauli_dense(n, int(ham.x[j]), int(ham.z[j]))
        assert abs(terms[j] - np.vdot(psi, P @ psi).real) < 1e-13


def test_single_ry_layer_z_expectation_is_cos():
    n = 6
    rng = np.random.default_rng(5)
    th = rng.uniform(0, 2 * math.pi, n)
    ops = [I.Op("ry", (q,), params=(q,)) for q in range(n)]
    psi = O.run(n, ops, th)
    ham = I.hamiltonian(n, [("Z", [q], 1.0) for q in range(n)])
    terms, _, _ = O.expect(n, psi, ham)
    assert np.max(np.abs(terms - np.cos(th))) < 1e-14


def test_zero_angles_give_unit_z():
    circ = I.layered(8, 3, seed=0)
    psi = O.run(8, circ.ops, np.zeros(circ.n_params))
    ham = I.hamiltonian(8, [("Z", [q], 1.0) for q in range(8)])
    terms, _, _ = O.expect(8, psi, ham)
    assert np.all(terms == 1.0)


@pytest.mark.parametrize("n", [3, 5])
def test_apply_pauli_sum_matches_dense(n):
    circ = I.random_circuit(n, 20, seed=11 + n)
    psi = O.run_circuit(circ)
    ham = I.random_hamiltonian(n, 9, seed=n)
    lam = O.apply_pauli_sum(n, psi, ham)
    assert np.max(np.abs(lam - BF.ham_dense(n, ham) @ psi)) < 1e-13


# ----------------------------------------------------------- gradients

def test_adjoint_single_qubit_closed_form():
    # RY(t)|0> with H = X: E = sin t, dE/dt = cos t.
    for t in [0.0, 0.3, 1.7, -2.5, 4.0]:
        circ = I.Circuit(1, [I.Op("ry", (0,), params=(0,))], np.array([t]))
        e, g = O.adjoint_grad(circ, I.hamiltonian(1, [("X", [0], 1.0)]))
        assert abs(e - math.sin(t)) < 1e-15
        assert abs(g[0] - math.cos(t)) < 1e-15


@pytest.mark.parametrize("n,L", [(3, 2), (4, 3), (6, 2)])
def test_hea_zero_angle_closed_form(n, L):
    # All angles zero: psi = |0..0>, so E = n-1 (every ZZ is +1, every X is 0);
    # dE/dtheta = 0.7 for every RY parameter and 0 for every RZ parameter.
    circ = I.hea(n, L)
    circ.params[:] = 0.0
    e, g = O.adjoint_grad(circ, I.tfim(n))
    assert abs(e - (n - 1)) < 1e-13
    assert np.max(np.abs(g[0::2] - 0.7)) < 1e-13
    assert np.max(np.abs(g[1::2])) < 1e-13
    # dense brute-force check of the same closed form (parameter shift by hand)
    H = BF.ham_dense(n, I.tfim(n))
    for i in [0, 1, 2 * n - 2]:
        p = circ.params.copy()
        p[i] = math.pi / 2
        ep = np.vdot(BF.run(n, circ.ops, p), H @ BF.run(n, circ.ops, p)).real
        p[i] = -math.pi / 2
        em = np.vdot(BF.run(n, circ.ops, p), H @ BF.run(n, circ.ops, p)).real
        assert abs(0.5 * (ep - em) - g[i]) < 1e-12


@pytest.mark.parametrize("seed", [0, 1])
def test_adjoint_matches_parameter_shift_and_fd(seed):
    circ = I.hea(6, 3, seed=seed)
    ham = I.tfim(6)
    e, g = O.adjoint_grad(circ, ham)
    idx = list(range(0, circ.n_params, 3))
    ps = O.param_shift_grad(circ, ham, idx)
    fd = O.finite_diff_grad(circ, ham, idx, h=1e-6)
    assert np.max(np.abs(g[idx] - ps)) < 1e-12
    assert np.max(np.abs(g[idx] - fd)) < 1e-7
    psi = BF.run(6, circ.ops, circ.params)
    assert abs(e - np.vdot(psi, BF.ham_dense(6, ham) @ psi).real) < 1e-12


def test_adjoint_general_gates_vs_dense_fd():
    # Every parameterised kind, controls, multi-parameter U3 and shared
    # parameters: adjoint vs a dense-matrix central difference.
    n = 4
    circ = I.random_circuit(n, 25, seed=21, allow_unitary=True)
    # share one parameter between two gates
    ops = list(circ.ops)
    pidx = [op for op in ops if op.params]
    if len(pidx) >= 2:
        a = pidx[0]
        b = pidx[1]
        ops[ops.index(b)] = I.Op(b.kind, b.targets, b.controls, b.cstate,
                                 (a.params[0],) + tuple(b.params[1:]), b.matrix)
    circ = I.Circuit(n, ops, circ.params)
    ham = I.random_hamiltonian(n, 6, seed=2)
    _, g = O.adjoint_grad(circ, ham)
    H = BF.ham_dense(n, ham)
    h = 1e-6
    for i in range(circ.n_params):
        p = circ.params.copy()
        p[i] += h
        ep = np.vdot(BF.run(n, ops, p), H @ BF.run(n, ops, p)).real
        p[i] -= 2 * h
        em = np.vdot(BF.run(n, ops, p), H @ BF.run(n, ops, p)).real
        assert abs((ep - em) / (2 * h) - g[i]) < 1e-7


def _two_term(circ, ham, i):
    p = np.array(circ.params, dtype=np.float64)
    p[i] += math.pi / 2
    ep = O.energy(circ, ham, p)
    p[i] -= math.pi
    return 0.5 * (ep - O.energy(circ, ham, p))


@pytest.mark.parametrize("case", ["givens", "dexc", "cry"])
def test_four_term_shift_rule_closed_forms(case):
    # Generators with the eigenvalues {-1, 0, 1} (Section 4.2: excitation
    # gates take a four-term rule).  Each state below has weight on both the
    # zero and the +-1 eigenspaces, so E carries the half frequency:
    #   givens: H0 H1, G(t) on (0, 1), <X0>        = cos(t/2)
    #   dexc:   H0..H3, D(t) on (0, 1, 2, 3), <X0> = 3/4 + cos(t/2)/4
    #   cry:    H0, RY(t) on 1 controlled by 0, <X0> = cos(t/2)
    if case == "givens":
        ops = [I.Op("h", (0,)), I.Op("h", (1,)), I.Op("givens", (0, 1), params=(0,))]
        e = lambda t: math.cos(t / 2)
        de = lambda t: -math.sin(t / 2) / 2
        n = 2
    elif case == "dexc":
        ops = [I.Op("h", (q,)) for q in range(4)] + [I.Op("dexc", (0, 1, 2, 3), params=(0,))]
        e = lambda t: 0.75 + math.cos(t / 2) / 4
        de = lambda t: -math.sin(t / 2) / 8
        n = 4
    else:
        ops = [I.Op("h", (0,)), I.Op("ry", (1,), (0,), params=(0,))]
        e = lambda t: math.cos(t / 2)
        de = lambda t: -math.sin(t / 2) / 2
        n = 2
    ham = I.hamiltonian(n, [("X", [0], 1.0)])
    worst_two = 0.0
    for t in [0.3, 1.1, 2.0, -2.7, 4.4]:
        circ = I.Circuit(n, ops, np.array([t]))
        assert abs(O.energy(circ, ham) - e(t)) < 1e-15
        g = O.param_shift_grad(circ, ham, [0])[0]
        assert abs(g - de(t)) < 1e-15
        _, ga = O.adjoint_grad(circ, ham)
        assert abs(ga[0] - de(t)) < 1e-15
        worst_two = max(worst_two, abs(_two_term(circ, ham, 0) - de(t)))
    # the two-term rule misses the half frequency here
    assert worst_two > 1e-2


def test_shift_rules_match_adjoint_on_every_parameterised_kind():
    # every parameterised kind, with and without controls (control states
    # included), one parameter shared by two gates: shift rules = adjoint
    n = 5
    kinds = ["rx", "ry", "rz", "p", "u2", "u3", "rxx", "ryy", "rzz", "givens", "dexc", "h", "x"]
    for seed in range(3):
        circ = I.random_circuit(n, 30, seed=40 + seed, kinds=kinds, max_controls=1)
        ops = list(circ.ops)
        par = [k for k, o in enumerate(ops) if o.params]
        a, b = par[0], par[1]
        ops[b] = I.Op(ops[b].kind, ops[b].targets, ops[b].controls, ops[b].cstate,
                      (ops[a].params[0],) + tuple(ops[b].params[1:]))
        circ = I.Circuit(n, ops, circ.params)
        ham = I.random_hamiltonian(n, 6, seed=seed)
        _, ga = O.adjoint_grad(circ, ham)
        idx = list(range(circ.n_params))
        assert np.max(np.abs(O.param_shift_grad(circ, ham, idx) - ga)) < 1e-12


# ------------------------------------------------------------- sampling

def test_splitmix64_reference_values():
    # SplitMix64 (Steele, Lea, Flood 2014) with state 0: the first outputs of
    # the published generator.
    assert O.splitmix64(0, 0) == 0xE220A8397B1DCDAF
    assert O.splitmix64(0, 1) == 0x6E789E6AA1B965F4
    assert O.splitmix64(0, 2) == 0x06C45D188009454F


def test_sampling_basis_state_is_deterministic():
    n = 7
    psi = np.zeros(1 << n, dtype=complex)
    psi[0b1011001] = 1.0
    out = O.sample(n, psi, seed=3, shots=200, qubits=list(range(n)))
    assert np.all(out == 0b1011001)
    sub = O.sample(n, psi, seed=3, shots=10, qubits=[6, 0, 3])
    assert np.all(sub == 0b111)  # bits 6,0,3 of 1011001 are 1,1,1


def test_sampling_two_point_distribution():
    # |psi> = sqrt(1/4)|0> + sqrt(3/4)|5>: exact binary probabilities, so a
    # draw u < 1/4 must give 0 and u >= 1/4 must give 5.
    n = 3
    psi = np.zeros(8, dtype=complex)
    psi[0] = 0.5
    psi[5] = math.sqrt(3) / 2 * 1j
    shots = 2000
    out = O.sample(n, psi, seed=11, shots=shots, qubits=[0, 1, 2])
    S, P = O.sample_prefix(n, psi)
    T = P[-1]
    for s in range(shots):
        u = (O.splitmix64(11, s) >> 11) * 2.0 ** -53
        expect = 0 if u * T < 0.25 else 5
        assert out[s] == expect


def test_sampling_chi_square():
    n = 6
    circ = I.random_circuit(n, 30, seed=5)
    psi = O.run_circuit(circ)
    p = np.abs(psi) ** 2
    shots = 200000
    out = O.sample(n, psi, seed=1234, shots=shots, qubits=list(range(n)))
    counts = np.bincount(out.astype(np.int64), minlength=1 << n)
    mask = p * shots > 5
    chi2 = np.sum((counts[mask] - p[mask] * shots) ** 2 / (p[mask] * shots))
    dof = int(mask.sum()) - 1
    # 6-sigma band of the chi-square distribution
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    assert np.all(counts[p == 0] == 0)


def test_sampling_same_seed_same_bits():
    n = 9
    psi = O.run_circuit(I.layered(n, 3, seed=2))
    a = O.sample(n, psi, 77, 500, list(range(n)))
    b = O.sample(n, psi, 77, 500, list(range(n)))
    c = O.sample(n, psi, 78, 500, list(range(n)))
    assert np.array_equal(a, b) and not np.array_equal(a, c)


def test_sampling_prefix_total_is_norm():
    n = 13
    psi = O.run_circuit(I.layered(n, 2, seed=4))
    S, P = O.sample_prefix(n, psi)
    assert len(S) == 8 and abs(P[-1] - 1) < 1e-13
    assert np.all(np.diff(P) >= 0)


def test_sampling_blocked_prefix_exact_dyadic():
    # n = 22: K = 4096 chunks in 4 blocks of 1024.  One amplitude per chunk,
    # a power of two, so every probability and every partial sum is an exact
    # binary fraction and the prefix must equal the exact cumulative sum
    # whatever the order: this pins the block and chunk indexing.
    n = 22
    K = 1 << (n - 10)
    rng = np.random.default_rng(9)
    e = rng.integers(11, 14, size=K)            # amplitude 2^-e, p = 2^-2e
    psi = np.zeros(1 << n, dtype=complex)
    pos = np.arange(K) * 1024 + rng.integers(0, 1024, size=K)
    psi[pos] = 2.0 ** -e.astype(float)
    S, P = O.sample_prefix(n, psi)
    units = [1 << (2 * (13 - int(x))) for x in e]   # p in units of 2^-26
    exact = np.concatenate([[0], np.cumsum(units)]).astype(np.float64) * 2.0 ** -26
    assert np.array_equal(S, np.array(units, dtype=np.float64) * 2.0 ** -26)
    assert np.array_equal(P, exact)


def test_sampling_blocked_prefix_rounding_order():
    # n = 21: two blocks of 1024 chunks.  S_0 = 1 and every other chunk sum is
    # 2^-53 (x = y = 2^-27).  Inside block 0 each 1 + 2^-53 rounds back to 1
    # (ties to even), so P_1024 = 1; block 1 sums its 1024 chunks exactly to
    # 2^-43 before the block offset is added, so T = 1 + 2^-43 and
    # P_1026 = 1 + 2^-52.  A single left-to-right prefix would give T = 1.
    n = 21
    psi = np.zeros(1 << n, dtype=complex)
    psi[0] = 1.0
    psi[1024::1024] = 2.0 ** -27 * (1 + 1j)
    S, P = O.sample_prefix(n, psi)
    assert S[0] == 1.0 and np.all(S[1:] == 2.0 ** -53)
    assert np.all(P[1:1025] == 1.0)
    assert P[1026] == 1.0 + 2.0 ** -52
    assert P[2048] == 1.0 + 2.0 ** -43


def _u(seed, s):
    return (O.splitmix64(seed, s) >> 11) * 2.0 ** -53


def _points(n, pts):
    psi = np.zeros(1 << n, dtype=complex)
    for b, a in pts.items():
        psi[b] = a
    return psi


@pytest.mark.parametrize("n,b", [(12, 2 * 1024 + 517), (12, 3 * 1024 + 1023), (12, 1024),
                                 (21, 1500 * 1024 + 3), (21, 1023 * 1024 + 9),
                                 (21, 2047 * 1024 + 1000)])
def test_sampling_basis_state_in_a_late_chunk(n, b):
    # Several chunks of 1024 indices (n = 21: two prefix blocks of 1024
    # chunks).  All the mass on one index, so every draw must return it: the
    # chunk search and the in-chunk search must both land on that index.
    psi = _points(n, {b: 1j})
    out = O.sample(n, psi, seed=5, shots=300, qubits=list(range(n)))
    assert np.all(out == b)


@pytest.mark.parametrize("n,pts", [
    # n = 12: four chunks; two empty chunks between the points
    (12, {1024 + 100: 0.5, 3 * 1024 + 10: 0.5j, 3 * 1024 + 900: 0.5 + 0.5j}),
    # n = 21: two prefix blocks; points in block 0, in block 1 and in the last chunk
    (21, {3 * 1024 + 1: 0.5, (1024 + 77) * 1024 + 512: -0.5j, 2047 * 1024 + 1023: 0.5 - 0.5j}),
])
def test_sampling_points_across_chunks_exact(n, pts):
    # Probabilities 1/4, 1/4, 1/2 (exact binary fractions, T = 1): a draw
    # with t = u * T must give the first point for t < 1/4, the second for
    # 1/4 <= t < 1/2 and the third for t >= 1/2, draw by draw.
    psi = _points(n, pts)
    b = sorted(pts)
    S, P = O.sample_prefix(n, psi)
    assert P[-1] == 1.0
    shots = 3000
    out = O.sample(n, psi, seed=13, shots=shots, qubits=list(range(n)))
    for s in range(shots):
        t = _u(13, s) * 1.0
        want = b[0] if t < 0.25 else b[1] if t < 0.5 else b[2]
        assert out[s] == want
    # every point is drawn (about 750 / 750 / 1500 times)
    assert all(np.count_nonzero(out == x) > 500 for x in b)


def test_sampling_search_boundaries_and_fallbacks():
    # n = 12, chunk masses S = (1/8, 0, 3/8, 1/2), prefix P = (0, 1/8, 1/8, 1/2, 1).
    # The chunk is the first k with P[k+1] > t (strict), the index the first
    # b in the chunk whose running sum exceeds r = t - P[k] (strict); t >= T
    # takes the last chunk with mass and, there, the last index with mass.
    n = 12
    psi = _points(n, {10: 0.25 + 0.25j, 2048 + 5: 0.5, 2048 + 700: 0.25 - 0.25j,
                      3072: 0.5j, 3500: -0.5})
    S, P = O.sample_prefix(n, psi)
    assert list(S) == [0.125, 0.0, 0.375, 0.5]
    assert list(P) == [0.0, 0.125, 0.125, 0.5, 1.0]
    below = lambda t: float(np.nextafter(t, 0.0))   # the largest double under t
    probes = [(0.0, 10), (below(0.125), 10), (0.125, 2053), (below(0.375), 2053),
              (0.375, 2748), (below(0.5), 2748), (0.5, 3072), (below(0.75), 3072),
              (0.75, 3500), (below(1.0), 3500), (1.0, 3500), (7.0, 3500)]
    got = O.sample_at(n, psi, [t for t, _ in probes])
    assert [int(g) for g in got] == [b for _, b in probes]
    # the last chunk with mass is chunk 2 once chunk 3 is emptied: t >= T falls
    # back there and takes its last index with mass
    psi2 = psi.copy()
    psi2[3072] = psi2[3500] = 0
    assert [int(g) for g in O.sample_at(n, psi2, [0.5, 9.0, 0.499])] == [2748, 2748, 2748]
    # one-chunk state whose running sum never reaches its pairwise-tree total:
    # p_0 = 1 and 1023 entries of 2^-54, each lost when added to 1 left to
    # right; for 1 <= t < T the in-chunk search falls back to the last index
    # with mass
    n = 10
    psi3 = np.full(1 << n, 2.0 ** -27, dtype=complex)
    psi3[0] = 1.0
    S3, P3 = O.sample_prefix(n, psi3)
    assert P3[-1] > 1.0
    assert [int(g) for g in O.sample_at(n, psi3, [0.0, 0.999, 1.0, P3[-1] * (1 - 2.0 ** -53)])] == \
        [0, 0, 1023, 1023]


def test_sampling_at_matches_sampler():
    # The sampler draws t = u_s * T and takes the same search.
    n = 13
    psi = O.run_circuit(I.layered(n, 2, seed=6))
    S, P = O.sample_prefix(n, psi)
    shots = 400
    t = np.array([_u(99, s) * P[-1] for s in range(shots)])
    assert np.array_equal(O.sample(n, psi, 99, shots, list(range(n))), O.sample_at(n, psi, t))


def test_sampling_chi_square_several_chunks():
    n = 12
    psi = O.run_circuit(I.random_circuit(n, 60, seed=12))
    p = np.abs(psi) ** 2
    shots = 400000
    out = O.sample(n, psi, seed=4321, shots=shots, qubits=list(range(n)))
    counts = np.bincount(out.astype(np.int64), minlength=1 << n)
    # per chunk of 1024 indices, then per index
    cp = p.reshape(4, 1024).sum(axis=1) * shots
    cc = counts.reshape(4, 1024).sum(axis=1)
    assert np.all(np.abs(cc - cp) < 6 * np.sqrt(cp) + 1)
    mask = p * shots > 5
    chi2 = np.sum((counts[mask] - p[mask] * shots) ** 2 / (p[mask] * shots))
    dof = int(mask.sum()) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)


# ---------------------------------------------------------- shot readout

def test_qwc_grouping():
    assert [ids for ids, _ in O.qwc_groups(I.tfim(6))] == [[0, 1, 2, 3, 4], [5, 6, 7, 8, 9, 10]]
    # X0 opens g0; Z0 clashes on qubit 0 and opens g1; X0X1 joins g0; Y1
    # clashes with g0 on qubit 1 and joins g1; the identity term is in none
    h = I.hamiltonian(3, [("X", [0], 1.0), ("Z", [0], 1.0), ("XX", [0, 1], 1.0),
                          ("Y", [1], 1.0), ("I", [2], 2.0)])
    groups = O.qwc_groups(h)
    assert [ids for ids, _ in groups] == [[0, 2], [1, 3]]
    assert groups[0][1] == {0: "X", 1: "X"} and groups[1][1] == {0: "Z", 1: "Y"}


def test_shot_estimate_eigenstates_exact():
    # RX(-pi/2)|0> is the +1 eigenstate of Y; H|0> of X; X|0> the -1 one of Z
    n = 3
    ops = [I.Op("rx", (0,), params=(0,)), I.Op("h", (1,)), I.Op("x", (2,))]
    psi = O.run(n, ops, [-math.pi / 2])
    h = I.hamiltonian(n, [("Y", [0], 0.5), ("X", [1], 2.0), ("Z", [2], 1.0),
                          ("YXZ", [0, 1, 2], -1.5), ("I", [0], 3.0)])
    vals, e, var, G = O.shot_estimate(n, psi, 5, 999, h)
    assert G == 1
    assert list(vals) == [1.0, 1.0, -1.0, -1.0, 1.0]
    assert e == 0.5 + 2.0 - 1.0 + 1.5 + 3.0 and var == 0.0


def test_shot_estimate_single_term_variance_closed_form():
    # one Z term on |+>: per-shot +-1, so Var(y) = 1 - v^2 and the reported
    # variance of the mean is (1 - v^2) / N
    psi = O.run(1, [I.Op("h", (0,))], [])
    h = I.hamiltonian(1, [("Z", [0], 1.0)])
    N = 4001
    vals, e, var, _ = O.shot_estimate(1, psi, 17, N, h)
    assert abs(var - (1 - vals[0] ** 2) / N) < 1e-15
    assert abs(vals[0]) < 6 / math.sqrt(N) and e == vals[0]


def test_shot_counts_basis_state():
    n = 6
    psi = np.zeros(1 << n, dtype=complex)
    psi[0b101100] = 1j
    counts = O.shot_counts(n, psi, 3, 500, [2, 5, 0])
    want = np.zeros(8, dtype=np.uint64)
    want[0b011] = 500          # bits of qubits 2, 5, 0 are 1, 1, 0
    assert np.array_equal(counts, want)


def test_shot_estimate_unbiased():
    n = 6
    psi = O.run_circuit(I.random_circuit(n, 40, seed=8))
    h = I.hamiltonian(n, [("Y", [0], 1.0), ("XY", [1, 2], -0.7), ("ZZ", [3, 4], 0.4),
                          ("X", [5], 1.1), ("YZ", [0, 3], 0.3)])
    shots = 60000
    vals, e, var, G = O.shot_estimate(n, psi, 21, shots, h)
    exact, ee, _ = O.expect(n, psi, h)
    per = shots // G
    for j in range(len(h)):
        assert abs(vals[j] - exact[j]) < 5 * math.sqrt(max(1 - exact[j] ** 2, 1e-4) / per)
    assert abs(e - ee) < 5 * math.sqrt(var) + 1e-12


# ----------------------------------------------------------- density matrix

def _depolarizing(p):
    s = math.sqrt(p / 3)
    return [math.sqrt(1 - p) * np.eye(2), s * np.array([[0, 1], [1, 0]]),
            s * np.array([[0, -1j], [1j, 0]]), s * np.diag([1.0, -1.0])]


def test_dm_pure_evolution_is_outer_product():
    n = 4
    circ = I.random_circuit(n, 25, seed=4, allow_unitary=True)
    rho = O.dm_run(n, circ.ops, circ.params)
    psi = O.run_circuit(circ)
    assert np.max(np.abs(rho - np.outer(psi, psi.conj()))) < 1e-13
    h = I.random_hamiltonian(n, 8, seed=2)
    vals, e = O.dm_expect(n, rho, h)
    ev, ee, _ = O.expect(n, psi, h)
    assert np.max(np.abs(vals - ev)) < 1e-13 and abs(e - ee) < 1e-12


def test_dm_depolarizing_closed_form():
    # (1-p) rho + p/3 (X rho X + Y rho Y + Z rho Z) on |0><0| gives <Z> = 1 - 4p/3
    rho = O.dm_run(1, [], [])
    p = 0.3
    r = O.dm_kraus(1, rho, 0, _depolarizing(p))
    vals, _ = O.dm_expect(1, r, I.hamiltonian(1, [("Z", [0], 1.0), ("X", [0], 1.0), ("I", [0], 1.0)]))
    assert abs(vals[0] - (1 - 4 * p / 3)) < 1e-15 and abs(vals[1]) < 1e-15 and abs(vals[2] - 1) < 1e-15


def test_dm_amplitude_damping_closed_form():
    # |1><1| under amplitude damping gamma: <Z> = -1 + 2 gamma, <X> stays 0
    n, q, g = 3, 1, 0.35
    rho = O.dm_run(n, [I.Op("x", (q,))], [])
    K = [np.array([[1, 0], [0, math.sqrt(1 - g)]]), np.array([[0, math.sqrt(g)], [0, 0]])]
    r = O.dm_kraus(n, rho, q, K)
    vals, _ = O.dm_expect(n, r, I.hamiltonian(n, [("Z", [q], 1.0), ("X", [q], 1.0), ("Z", [0], 1.0)]))
    assert abs(vals[0] - (-1 + 2 * g)) < 1e-15 and abs(vals[1]) < 1e-15 and abs(vals[2] - 1) < 1e-15
    assert abs(np.trace(r).real - 1) < 1e-15


def test_dm_two_qubit_depolarizing_closed_form():
    # two-qubit depolarizing: (1-p) rho + p/15 sum over the 15 non-identity
    # Pauli pairs; on |00><00| it leaves <Z0> = <Z1> = <Z0 Z1> = 1 - 16p/15
    P = [np.eye(2), np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.diag([1.0, -1.0])]
    p = 0.27
    K = [math.sqrt(1 - p) * np.eye(4)]
    for a in range(4):
        for b in range(4):
            if a or b:
                K.append(math.sqrt(p / 15) * np.kron(P[b], P[a]))   # local index bit(q0) + 2 bit(q1)
    n = 3
    rho = O.dm_run(n, [], [])
    r = O.dm_kraus2(n, rho, 2, 0, K)
    h = I.hamiltonian(n, [("Z", [2], 1.0), ("Z", [0], 1.0), ("ZZ", [0, 2], 1.0), ("X", [2], 1.0),
                          ("Z", [1], 1.0)])
    vals, _ = O.dm_expect(n, r, h)
    want = [1 - 16 * p / 15] * 3 + [0.0, 1.0]
    assert np.max(np.abs(vals - want)) < 1e-14
    assert abs(np.trace(r).real - 1) < 1e-14


# --------------------------------------------------------------- fusion

def test_fusion_counts_match_paper_table():
    for n, gates, blocks in _load_golden("fusion_counts.txt"):
        ops = I.layered_structure(n, 4)
        assert len(ops) == gates
        nb, _ = O.fuse_greedy(4, ops)
        assert nb == blocks


def test_fused_block_product_equals_circuit():
    # Multiplying each greedy block's gates and applying the blocks reproduces
    # the unfused state (the paper's unitary check before fused timings).
    n = 6
    circ = I.layered(n, 3, seed=9)
    nb, blk = O.fuse_greedy(4, circ.ops)
    psi = np.zeros(1 << n, dtype=complex)
    psi[0] = 1
    for b in range(nb):
        U = np.eye(1 << n, dtype=complex)
        for op, bo in zip(circ.ops, blk):
            if bo == b:
                U = BF.full_matrix(n, op, circ.params) @ U
        psi = U @ psi
    assert np.max(np.abs(psi - O.run_circuit(circ))) < 1e-12
