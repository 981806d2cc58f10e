"""The allocation-free entry point sv_expect_pauli_noalloc (fixed device
scratch) against sv_expect_pauli, through the C ABI: same values on two
calls in a row, the second on a smaller state with fewer terms; no device
memory taken; a request beyond the fixed scratch refused before device work."""
import numpy as np
import pytest

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


def _prepared(sv, n, seed):
    circ = I.random_circuit(n, 40, seed=seed, max_controls=2)
    st = sv.State(n)
    st.apply(circ.ops, circ.params, fuse=-1)
    return st


def test_noalloc_matches_allocating_call(sv):
    import torch
    # code object and symbol set-up on this GPU happen on a first call
    warm = _prepared(sv, 10, 1)
    warm.expect_noalloc(I.tfim(10))
    cases = [(18, I.random_hamiltonian(18, 40, seed=3)), (12, I.tfim(12, 0.3))]
    states = [_prepared(sv, n, 10 + n) for n, _ in cases]
    torch.cuda.synchronize()
    for (n, ham), st in zip(cases, states):
        _say("noalloc", n, len(ham))
        free0 = torch.cuda.mem_get_info()[0]
        t0, e0 = st.expect_noalloc(ham)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0        # no device memory taken
        t1, e1 = st.expect(ham)                             # the allocating entry point
        assert np.max(np.abs(t0 - t1)) <= TOL and abs(e0 - e1) <= TOL
        # and again after the allocating call ran on the same state
        t2, e2 = st.expect_noalloc(ham)
        assert np.max(np.abs(t2 - t1)) <= TOL and abs(e2 - e1) <= TOL
    for st in states + [warm]:
        st.close()


def test_noalloc_refuses_oversized_request(sv):
    n = 14
    st = _prepared(sv, n, 5)
    before = st.to_numpy()
    big = I.random_hamiltonian(n, 4096, seed=1)       # X/Y terms: partial sums per workgroup
    _say("noalloc oversize", len(big))
    with pytest.raises(sv.SvError) as ei:
        st.expect_noalloc(big)
    assert ei.value.status == -4
    assert np.array_equal(before, st.to_numpy())
    t, e = st.expect(big)                               # the allocating call takes it
    assert np.all(np.isfinite(t))
    st.close()
