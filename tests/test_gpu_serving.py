"""The serving loop on the GPU: every served (E, grad) -- from the batch path
(n <= 13) and from the stream lanes alike -- equals the oracle's adjoint at
1e-12, and equals the same request run alone bit for bit."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_09733_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


def test_served_results_match_oracle_and_alone():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_09733_amd import serving as S
    trace = I.serving_trace(400.0, 24, seed=3, n_lo=10, n_hi=16, l_lo=2, l_hi=8)
    print("[case] serving 24 requests, 3 lanes", flush=True)
    ex = S.GpuExecutor(3)
    try:
        rep = S.Server(ex, 3).serve(trace)
    finally:
        ex.close()
    assert len(rep.outcomes) == len(trace)
    assert any(o.lane < 0 for o in rep.outcomes) and any(o.lane >= 0 for o in rep.outcomes)
    by_id = {r.rid: r for r in trace}
    for o in rep.outcomes:
        r = by_id[o.rid]
        e_ref, g_ref = O.adjoint_grad(r.circuit, r.ham)
        assert abs(o.energy - e_ref) <= TOL * max(1.0, abs(e_ref)), o.rid
        assert np.max(np.abs(o.grad - g_ref)) <= TOL, o.rid
    print("[case] serving alone vs mix", flush=True)
    assert S.alone_vs_mix(rep, trace) == 0
