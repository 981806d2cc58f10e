"""Element-wise oracle parity where the tile sweep reaches its steady state.

With the default FP64 tiling (13-qubit tiles) a launch has one workgroup per
compute unit, so every workgroup holds exactly one tile up to 21 qubits; from
22 qubits on each workgroup walks several tiles through the sweep's
prefetch / store pipeline and XCD-ordered tile rounds (2 tiles each at 22
qubits and 8 at 24 on 256 compute units).  These cases compare every
amplitude, expectation value and gradient with the CPU oracle there, in the
default plan and tiling, at 1e-12 (FP64) and 1e-5 (complex64).
"""
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


@pytest.fixture(scope="module")
def cus():
    import torch
    return torch.cuda.get_device_properties(0).multi_processor_count


def _say(*a):
    print("[case]", *a, flush=True)


def _tiles_per_workgroup(sv, n, cus):
    M, c, R = sv.default_tiling(n)
    return (1 << (n - M)) / cus


@pytest.mark.parametrize("n,L", [(22, 3), (24, 2)])
def test_layered_steady_state(sv, cus, n, L):
    assert _tiles_per_workgroup(sv, n, cus) >= 2
    circ = I.layered(n, L, seed=n)
    _say("steady state layered", n, L)
    st = sv.State(n)
    st.apply(circ.ops, circ.params, fuse=-1)
    psi = st.to_numpy()
    ref = O.run_circuit(circ)
    assert np.max(np.abs(psi - ref)) <= TOL
    ham = I.hamiltonian(n, [("Z", [q], 1.0) for q in range(n)])
    z, _ = st.expect(ham)
    zr, _, _ = O.expect(n, ref, ham)
    assert np.max(np.abs(z - zr)) <= TOL
    h = I.tfim(n)
    t, e = st.expect(h)
    tr, er, _ = O.expect(n, ref, h)
    assert np.max(np.abs(t - tr)) <= TOL and abs(e - er) <= TOL
    st.close()


def test_random_all_kinds_steady_state(sv, cus):
    n = 22
    assert _tiles_per_workgroup(sv, n, cus) >= 2
    circ = I.random_circuit(n, 80, seed=2222, max_controls=2)
    ham = I.random_hamiltonian(n, 24, seed=22)
    _say("steady state random", n)
    st = sv.State(n)
    st.apply(circ.ops, circ.params, fuse=-1)
    psi = st.to_numpy()
    ref = O.run_circuit(circ)
    assert np.max(np.abs(psi - ref)) <= TOL
    t, e = st.expect(ham)
    tr, er, _ = O.expect(n, ref, ham)
    assert np.max(np.abs(t - tr)) <= TOL and abs(e - er) <= TOL
    st.close()


def test_adjoint_steady_state(sv):
    n = 22
    circ = I.hea(n, 2, seed=22)
    ham = I.tfim(n)
    _say("steady state adjoint", n)
    st = sv.State(n, adjoint=True)
    e, g = st.adjoint_grad(circ.ops, circ.params, ham)
    er, gr = O.adjoint_grad(circ, ham)
    assert abs(e - er) <= TOL
    assert np.max(np.abs(g - gr)) <= TOL
    assert np.max(np.abs(st.to_numpy() - O.run_circuit(circ))) <= TOL
    st.close()


@pytest.mark.parametrize("n", [22, 24])
def test_complex64_steady_state(sv, n):
    circ = I.layered(n, 3, seed=n + 1)
    _say("steady state complex64", n)
    st = sv.State(n, "c64")
    st.apply(circ.ops, circ.params, fuse=-1)
    psi = st.to_numpy()
    st.close()
    ref = O.run_circuit(circ)
    err = float(np.max(np.abs(psi - ref)))
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    print(f"complex64 n={n}: max|err| = {err:.3e} = {err / rms:.3e} x rms amplitude", flush=True)
    assert err <= TOL32


@pytest.mark.parametrize("n,dtype", [(20, "c128"), (24, "c128"), (22, "c64")])
def test_sweeps_from_zero_equal_every_tile(sv, n, dtype):
    """A circuit run from the handle's pending |0..0> takes the support-
    restricted sweeps (the first sweep runs only tile 0, the next ones only
    the tiles on the qubits swept so far); the same circuit from an uploaded
    |0..0> runs every tile of every sweep.  The results are equal exactly."""
    _say("support-restricted sweeps vs every tile", n, dtype)
    c = I.layered(n, 6, seed=11)
    oa = sv.OpArray(c.ops)
    a = sv.State(n, dtype)
    b = sv.State(n, dtype)
    try:
        a.reset()
        a.apply(None, c.params, op_array=oa)
        re = np.zeros(1 << n)
        re[0] = 1.0
        b.set_planes(re, np.zeros(1 << n))
        b.apply(None, c.params, op_array=oa)
        assert np.array_equal(a.to_numpy(), b.to_numpy())
    finally:
        a.close()
        b.close()
