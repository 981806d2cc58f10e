"""GPU parity of the ragged batch (one persistent launch over a work queue)
against the CPU oracle, plus the batch's own contracts: a circuit's result is
the same alone and inside a mix (bit for bit), graph replays equal eager runs,
and the bounded dependency wait reports expiry instead of hanging.
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


def _say(*a):
    print("[case]", *a, flush=True)


def _mixed(seed=0, max_qubits=5):
    """Ragged mix: every gate kind, 1..16 qubits (one- and multi-tile circuits,
    an empty circuit), random observables with X/Y/Z strings."""
    circs, hams = [], []
    for k, n in enumerate([1, 2, 3, 5, 8, 12, 13, 14, 16, 9, 4, 15]):
        depth = 0 if k == 9 else 30 + 5 * (k % 4)
        c = I.random_circuit(n, depth, seed=seed * 100 + k, max_controls=min(2, n - 1),
                             max_qubits=max_qubits)
        circs.append(c)
        hams.append(I.random_hamiltonian(n, 1 + k % 5, seed=seed * 100 + k + 50))
    return circs, hams


@pytest.mark.parametrize("group_bits", [3, 5])
def test_batch_mixed_vs_oracle(sv, group_bits):
    # 3-qubit register groups hold ops on at most 3 qubits
    circs, hams = _mixed(max_qubits=group_bits)
    _say("batch mixed", group_bits)
    b = sv.Batch(circs, hams, group_bits=group_bits)
    b.run()
    res = b.results()
    for k, (c, h) in enumerate(zip(circs, hams)):
        ref = O.run_circuit(c)
        psi = b.state(k)
        assert np.max(np.abs(psi - ref)) <= TOL, (k, c.n)
        e_ref = O.expect(c.n, ref, h)[1]
        assert abs(res[k] - e_ref) <= TOL * max(1.0, np.sum(np.abs(h.c))), (k, res[k], e_ref)
    b.close()


@pytest.mark.parametrize("low_bits", [1, 3, 4])
def test_batch_low_bits(sv, low_bits):
    circs, hams = _mixed(seed=1)
    _say("batch low_bits", low_bits)
    b = sv.Batch(circs, hams, low_bits=low_bits)
    b.run()
    res = b.results()
    for k, (c, h) in enumerate(zip(circs, hams)):
        ref = O.run_circuit(c)
        assert np.max(np.abs(b.state(k) - ref)) <= TOL, (k, c.n)
        assert abs(res[k] - O.expect(c.n, ref, h)[1]) <= TOL * max(1.0, np.sum(np.abs(h.c)))
    b.close()


def test_batch_layered_ragged_vs_oracle(sv):
    # the ragged layered family (RY/RZ + CNOT ladder, <Z0 Z1>) at sizes the
    # oracle finishes quickly: 48 circuits, n in 8..16, L in 10..40
    circs = I.batch_circuits(48, seed=3, n_lo=8, n_hi=16)
    hams = [I.z0z1(c.n) for c in circs]
    _say("batch layered 48")
    b = sv.Batch(circs, hams)
    b.run()
    res = b.results()
    for k, (c, h) in enumerate(zip(circs, hams)):
        ref = O.run_circuit(c)
        assert abs(res[k] - O.expect(c.n, ref, h)[1]) <= TOL, k
        if k % 8 == 0:
            assert np.max(np.abs(b.state(k) - ref)) <= TOL, k
    b.close()


def test_batch_full_config_sampled(sv):
    # 512 circuits, n in 8..22, L in 10..40, <Z0 Z1> each; the oracle checks
    # a sample (every circuit up to 12 qubits and the first three larger ones,
    # including one at the top of the range); every circuit is also checked
    # against the plain per-circuit path on the GPU
    circs = I.batch_circuits(512, seed=0)
    hams = [I.z0z1(c.n) for c in circs]
    _say("batch 512 plan")
    b = sv.Batch(circs, hams)
    _say("batch 512 run")
    b.run(graph=True)
    res = b.results()
    big = [k for k, c in enumerate(circs) if c.n > 12]
    top = [k for k in big if circs[k].n >= 21][:1]
    sample = [k for k, c in enumerate(circs) if c.n <= 12] + big[:2] + top
    for k in sample:
        c = circs[k]
        _say("oracle", k, c.n, len(c.ops))
        ref = O.run_circuit(c)
        assert abs(res[k] - O.expect(c.n, ref, hams[k])[1]) <= TOL, (k, c.n)
    _say("plain path 512")
    for k, c in enumerate(circs):
        st = sv.State(c.n)
        st.apply(c.ops, c.params)
        _, e = st.expect(hams[k])
        st.close()
        assert abs(res[k] - e) <= TOL, (k, c.n)
    b.close()


def test_batch_alone_equals_mix_bitwise(sv):
    # same kernel (register-group width) for the mix and the singles
    circs, hams = _mixed(seed=2)
    _say("batch alone vs mix")
    b = sv.Batch(circs, hams, group_bits=5)
    b.run()
    mix = b.results()
    states = [b.state(k) for k in range(len(circs))]
    b.close()
    for k in (0, 4, 7, 8, 11):
        one = sv.Batch([circs[k]], [hams[k]], group_bits=5)
        one.run()
        r = one.results()
        assert r[0] == mix[k], (k, r[0], mix[k])
        assert np.array_equal(one.state(0), states[k]), k
        one.close()


def test_batch_graph_replays_with_new_params(sv):
    import torch
    circs = I.batch_circuits(24, seed=5, n_lo=6, n_hi=15)
    hams = [I.z0z1(c.n) for c in circs]
    _say("batch graph replays")
    b = sv.Batch(circs, hams)
    rng = np.random.default_rng(7)
    for rep in range(4):
        new = [rng.uniform(0, 2 * np.pi, len(c.params)) for c in circs]
        b.set_params(new)
        b.run()
        eager = b.results()
        # unrelated eager work on the device between the runs
        x = torch.ones(1 << 20, device="cuda", dtype=torch.float64)
        float(x.sum())
        b.run(graph=True)
        replay = b.results()
        assert np.array_equal(eager, replay), rep
        for k in (0, 5, 11):
            c = circs[k]
            ref = O.run(c.n, c.ops, new[k])
            assert abs(replay[k] - O.expect(c.n, ref, hams[k])[1]) <= TOL, (rep, k)
    b.close()


def test_batch_complex64(sv):
    circs, hams = _mixed(seed=4)
    _say("batch c64")
    b = sv.Batch(circs, hams, dtype="c64")
    b.run()
    res = b.results()
    for k, (c, h) in enumerate(zip(circs, hams)):
        ref = O.run_circuit(c)
        assert np.max(np.abs(b.state(k) - ref)) <= TOL32, k
        assert abs(res[k] - O.expect(c.n, ref, h)[1]) <= TOL32 * max(1.0, np.sum(np.abs(h.c))) * 4
    b.close()


def test_batch_expired_wait_is_reported(sv):
    # forced from the host: a negative spin limit makes every dependency wait
    # expire at once, so the kernel still exits normally and the check reports it
    circs = I.batch_circuits(4, seed=9, n_lo=15, n_hi=16)
    hams = [I.z0z1(c.n) for c in circs]
    _say("batch expired wait")
    b = sv.Batch(circs, hams)
    b.set_spin_limit(-1)
    b.run()
    with pytest.raises(sv.SvError, match="dependency wait expired"):
        b.check()
    b.set_spin_limit(1 << 22)
    b.run()
    res = b.results()
    for k, c in enumerate(circs):
        ref = O.run_circuit(c)
        assert abs(res[k] - O.expect(c.n, ref, hams[k])[1]) <= TOL
    b.close()
