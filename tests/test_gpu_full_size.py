"""Full-size checks: the 30-qubit layered workload (16 GiB of FP64 planes) in
the launch configuration the benchmark times (default plan and tiling),
through the C ABI.

The oracle's own run of this workload (tests/golden/layered30_seed0.npz,
written once by oracle/make_golden_layered30.py) pins amplitudes at 65536
seeded indices, every <Z_q>, the norm and 1000 draws.  The oracle cannot
simulate 30 qubits in seconds, so the other cases use facts that hold at
any size:
* with every RY angle in {0, pi} the layered circuit maps |0...0> to a single
  basis state; its index and phase follow gate by gate from the gate
  definitions (RY(pi) flips the bit, with a sign when the bit was 1; RZ(phi)
  multiplies by exp(-+i phi/2); CNOT flips the target when the control is 1);
* the circuit followed by its inverse returns |0...0>;
* two unrelated plans (LDS tile clusters with Kronecker stages, and the
  paper's in-order blocks of up to 5 qubits as dense block sweeps) give the
  same amplitudes and <Z_i>;
* terminal draws of a basis state all return it, and a grouped shot estimate
  lands within 6 standard deviations of the exact <H>.
"""
import math
import os

import numpy as np
import pytest

from paper_2608_09733_amd import inputs as I

pytestmark = pytest.mark.gpu

N = 30
L = 20
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


def _zs(n):
    return I.hamiltonian(n, [("Z", [q], 1.0) for q in range(n)] + [("I", [0], 1.0)])


def _track_basis_state(circ):
    """Index and amplitude of the single basis state reached from |0...0>
    when every RY angle is 0 or pi."""
    b, amp = 0, 1.0 + 0.0j
    for op in circ.ops:
        if op.kind == "ry":
            th = circ.params[op.params[0]]
            if th == 0.0:
                continue
            assert th == math.pi
            q = op.targets[0]
            s = math.sin(th / 2)
            if (b >> q) & 1:
                amp *= -s
            else:
                amp *= s
            b ^= 1 << q
        elif op.kind == "rz":
            phi = circ.params[op.params[0]]
            sign = -1.0 if ((b >> op.targets[0]) & 1) == 0 else 1.0
            amp *= complex(math.cos(phi / 2), sign * math.sin(phi / 2))
        elif op.kind == "x":
            if all((b >> c) & 1 for c in op.controls):
                b ^= 1 << op.targets[0]
        else:
            raise AssertionError(op.kind)
    return b, amp


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "layered30_seed0.npz")


def test_full_size_oracle_golden(sv):
    # The CPU oracle's own run of this exact workload (written by
    # oracle/make_golden_layered30.py, 46 min on 6 host threads): amplitudes
    # at 65536 seeded indices, every <Z_q>, the norm and 1000 terminal draws.
    g = np.load(GOLDEN, allow_pickle=False)
    assert tuple(g["meta"][:3]) == (N, L, 0)
    circ = I.layered(N, L, seed=0)
    oa = sv.OpArray(circ.ops)
    _say("full size: FP64 against the oracle golden", N, L)
    st = sv.State(N)
    st.apply(None, circ.params, op_array=oa)
    amp = st.gather(g["idx"])
    err = float(np.max(np.abs(amp - g["amp"])))
    print(f"fp64 30q: max|err| over {len(amp)} amplitudes = {err:.3e}", flush=True)
    assert err <= TOL
    vals, _ = st.expect(_zs(N))
    assert np.max(np.abs(vals[:N] - g["zexp"])) <= TOL
    assert abs(vals[N] - g["norm"][0]) <= TOL
    # terminal draws: the same draws as the oracle's on its own state
    draws = st.sample(0, len(g["samples"]), list(range(N)))
    assert np.array_equal(draws, g["samples"]), int(np.count_nonzero(draws != g["samples"]))
    st.close()
    _say("full size: complex64 against the oracle golden", N, L)
    s32 = sv.State(N, "c64")
    s32.apply(None, circ.params, op_array=oa)
    a32 = s32.gather(g["idx"])
    s32.close()
    err32 = float(np.max(np.abs(a32 - g["amp"])))
    rms = math.sqrt(2.0 ** -N)
    print(f"complex64 30q: max|err| = {err32:.3e} = {err32 / rms:.3e} x rms amplitude", flush=True)
    assert err32 <= 1e-5


def test_full_size_basis_state_tracking(sv):
    _say("full size: RY in {0, pi}", N, L)
    circ = I.layered(N, L, seed=0)
    rng = np.random.default_rng(5)
    p = circ.params.copy().reshape(L, N, 2)
    p[:, :, 0] = np.where(rng.random((L, N)) < 0.5, 0.0, math.pi)
    circ = I.Circuit(N, circ.ops, p.reshape(-1))
    b, amp = _track_basis_state(circ)
    st = sv.State(N)
    st.apply(None, circ.params, op_array=sv.OpArray(circ.ops))
    re, im = st.planes(b, 1)
    got = complex(re[0], im[0])
    assert abs(got - amp) <= TOL, (b, got, amp)
    vals, _ = st.expect(_zs(N))
    want = np.array([-1.0 if (b >> q) & 1 else 1.0 for q in range(N)] + [1.0])
    assert np.max(np.abs(vals - want)) <= TOL
    # every terminal draw is that basis state (the leaked amplitudes of
    # RY(pi) are ~1e-16, probabilities ~1e-32)
    draws = st.sample(3, 4096, list(range(N)))
    assert np.all(draws == b)
    qs = [29, 0, 17, 4]
    counts = st.sample_counts(3, 4096, qs)
    packed = sum(((b >> q) & 1) << i for i, q in enumerate(qs))
    assert int(counts[packed]) == 4096 and int(counts.sum()) == 4096
    st.close()


def test_full_size_shot_estimate(sv):
    _say("full size: grouped shot estimate of TFIM", N, L)
    circ = I.layered(N, L, seed=0)
    h = I.tfim(N, 0.7)
    st = sv.State(N)
    st.apply(None, circ.params, op_array=sv.OpArray(circ.ops))
    _, exact = st.expect(h)
    vals, e, var, G = st.shot_estimate(5, 1 << 18, h)
    assert G == 2 and var > 0
    assert abs(e - exact) <= 6 * math.sqrt(var)
    st.close()


def test_full_size_round_trip(sv):
    _say("full size: circuit then inverse", N, L)
    circ = I.layered(N, L, seed=0)
    P = circ.n_params
    inv = []
    for op in reversed(circ.ops):
        if op.params:
            inv.append(I.Op(op.kind, op.targets, op.controls, op.cstate,
                            tuple(k + P for k in op.params)))
        else:
            inv.append(op)
    params = np.concatenate([circ.params, -circ.params])
    ops = list(circ.ops) + inv
    st = sv.State(N)
    st.apply(None, params, op_array=sv.OpArray(ops))
    re, im = st.planes(0, 1 << 12)
    assert abs(complex(re[0], im[0]) - 1.0) <= TOL
    assert np.max(np.abs(re[1:])) <= TOL and np.max(np.abs(im[1:])) <= TOL
    vals, _ = st.expect(_zs(N))
    assert np.max(np.abs(vals - 1.0)) <= TOL
    st.close()


def test_full_size_two_plans_agree(sv):
    _say("full size: tile clusters vs width-5 blocks", N, L)
    circ = I.layered(N, L, seed=0)
    oa = sv.OpArray(circ.ops)
    a = sv.State(N)
    a.apply(None, circ.params, op_array=oa)
    b = sv.State(N)
    b.apply(None, circ.params, fuse=5, op_array=oa)
    za, _ = a.expect(_zs(N))
    zb, _ = b.expect(_zs(N))
    assert np.max(np.abs(za - zb)) <= TOL
    assert abs(za[-1] - 1.0) <= TOL          # <I> = norm^2
    rng = np.random.default_rng(11)
    offsets = [0, (1 << N) - 4096] + [int(x) * 4096 for x in rng.integers(0, (1 << N) // 4096, 6)]
    for off in offsets:
        ra, ia = a.planes(off, 4096)
        rb, ib = b.planes(off, 4096)
        assert np.max(np.abs(ra - rb)) <= TOL and np.max(np.abs(ia - ib)) <= TOL, off
    a.close()
    b.close()


def test_adjoint_26q_matches_parameter_shift(sv):
    # the adjoint extra's workload (26-qubit HEA, 10 layers, TFIM): sampled
    # gradient components against the parameter-shift rule
    # dE/dtheta_j = (E(theta_j + pi/2) - E(theta_j - pi/2)) / 2, each energy a
    # forward pass and <H> on the same handle
    n = 26
    _say("full size: 26-qubit adjoint vs parameter shift")
    circ = I.hea(n, 10, seed=0)
    h = I.tfim(n, 0.7)
    oa = sv.OpArray(circ.ops)
    st = sv.State(n, adjoint=True)
    st.reset()
    e, g = st.adjoint_grad(None, circ.params, h, op_array=oa)
    for j in (0, 1, 2 * n + 7, len(circ.params) // 2 + 3, len(circ.params) - 1):
        es = []
        for sgn in (1.0, -1.0):
            p = circ.params.copy()
            p[j] += sgn * math.pi / 2
            st.reset()
            st.apply(None, p, op_array=oa)
            es.append(st.expect(h)[1])
        assert abs((es[0] - es[1]) / 2 - g[j]) <= 1e-10, (j, g[j], es)
    st.reset()
    st.apply(None, circ.params, op_array=oa)
    assert abs(st.expect(h)[1] - e) <= 1e-10
    st.close()
