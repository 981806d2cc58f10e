"""GPU density matrices (rho of n qubits as a 2n-qubit vector) against the
dense oracle: the vectorised rho element by element and Tr(rho P) at 1e-12,
through gates of every kind, one-qubit Kraus channels and a second circuit."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_09733_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def sv():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2608_09733_amd import sv as _sv
    _sv.lib()
    return _sv


def _say(*a):
    print("[case]", *a, flush=True)


def _depolarizing(p):
    s = math.sqrt(p / 3)
    return [math.sqrt(1 - p) * np.eye(2), s * np.array([[0, 1], [1, 0]]),
            s * np.array([[0, -1j], [1j, 0]]), s * np.diag([1.0, -1.0])]


def _damping(g):
    return [np.array([[1, 0], [0, math.sqrt(1 - g)]]), np.array([[0, math.sqrt(g)], [0, 0]])]


def _mixed_unitaries(seed):
    # complex two-qubit Kraus set: sqrt(0.7) U, sqrt(0.3) V for random unitaries
    rng = np.random.default_rng(seed)
    out = []
    for w in (0.7, 0.3):
        a = rng.normal(size=(4, 4)) + 1j * rng.normal(size=(4, 4))
        q, _ = np.linalg.qr(a)
        out.append(math.sqrt(w) * q)
    return out


@pytest.mark.parametrize("n", [3, 6, 7])
def test_dm_vs_oracle(sv, n):
    _say("density matrix", n)
    c1 = I.random_circuit(n, 30, seed=10 + n, max_qubits=3)
    c2 = I.layered(n, 2, seed=n)
    h = I.random_hamiltonian(n, 10, seed=n)
    st = sv.State(2 * n)
    st.reset()
    st.dm_apply(c1.ops, c1.params)
    st.dm_apply_kraus(0, _depolarizing(0.2))
    st.dm_apply_kraus(n - 1, _damping(0.3))
    st.dm_apply(c2.ops, c2.params)
    st.dm_apply_kraus(list(range(n)), _depolarizing(0.05))
    K2 = _mixed_unitaries(n)
    st.dm_apply_kraus2(n - 1, 0, K2)
    got = st.to_numpy()
    rho = O.dm_run(n, c1.ops, c1.params)
    rho = O.dm_kraus(n, rho, 0, _depolarizing(0.2))
    rho = O.dm_kraus(n, rho, n - 1, _damping(0.3))
    rho = O.dm_run(n, c2.ops, c2.params, rho)
    for q in range(n):
        rho = O.dm_kraus(n, rho, q, _depolarizing(0.05))
    rho = O.dm_kraus2(n, rho, n - 1, 0, K2)
    assert np.max(np.abs(got - rho.reshape(-1))) <= TOL
    vals, e = st.dm_expect(h)
    ov, oe = O.dm_expect(n, rho, h)
    assert np.max(np.abs(vals - ov)) <= TOL and abs(e - oe) <= TOL
    st.close()


def test_dm_handle_size_checked(sv):
    _say("density matrix handle check")
    st = sv.State(5)
    with pytest.raises(sv.SvError):
        st.dm_apply_kraus(0, _damping(0.1))
    st.close()
