"""torch.autograd over the adjoint path: gradients equal the oracle's adjoint
gradient (1e-12), pass torch's finite-difference gradcheck, and compose with
the chain rule."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2608_09733_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch
    assert torch.cuda.is_available()
    from paper_2608_09733_amd import autograd as A
    from paper_2608_09733_amd import sv
    return torch, A, sv


def test_energy_and_grad_match_oracle(mods):
    torch, A, sv = mods
    circ = I.hea(10, 3, seed=4)
    ham = I.tfim(10)
    print("[case] autograd hea 10q", flush=True)
    st = sv.State(10, adjoint=True)
    theta = torch.tensor(circ.params, dtype=torch.float64, device="cuda", requires_grad=True)
    e = A.energy(theta, circ.ops, ham, st)
    e.backward()
    e_ref, g_ref = O.adjoint_grad(circ, ham)
    assert abs(e.detach().item() - e_ref) <= 1e-12
    assert np.max(np.abs(theta.grad.cpu().numpy() - g_ref)) <= 1e-12
    st.close()


def test_gradcheck_finite_differences(mods):
    torch, A, sv = mods
    circ = I.hea(5, 2, seed=5)
    ham = I.tfim(5)
    print("[case] autograd gradcheck", flush=True)
    st = sv.State(5, adjoint=True)
    theta = torch.tensor(circ.params, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda p: A.energy(p, circ.ops, ham, st), (theta,),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)
    st.close()


def test_chain_rule(mods):
    torch, A, sv = mods
    circ = I.layered(8, 3, seed=6)
    ham = I.tfim(8)
    print("[case] autograd chain rule", flush=True)
    st = sv.State(8, adjoint=True)
    theta = torch.tensor(circ.params, dtype=torch.float64, device="cuda", requires_grad=True)
    e = A.energy(theta, circ.ops, ham, st)
    (3.0 * e * e).backward()
    e_ref, g_ref = O.adjoint_grad(circ, ham)
    assert np.max(np.abs(theta.grad.cpu().numpy() - 6.0 * e_ref * g_ref)) <= 1e-11
    st.close()
