"""The differentiation hook: torch.autograd.Function with the exact gradient as backward,
checked by gradcheck (FP64), against the oracle gradient and against the patch
central-difference gradient, including a scaled incoming gradient and the case where the
gradient kept by the forward pass was overwritten before backward."""

import numpy as np
import pytest
import torch

import p1e_synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_01158_amd as P
    return P


def _mesh(P, prob, modes=None):
    modes = modes or (P.P1E_FP64 | P.P1E_MIXED | P.P1E_FD)
    return P.Mesh.from_problem(prob, modes=modes)


@pytest.mark.parametrize("which", ["nh3d", "plap2d"])
def test_gradcheck_fp64(P, which):
    prob = (S.neohooke_box_3d(3, 2, 2, 1.0, 0.7, 0.6, amp=0.02, seed=1) if which == "nh3d"
            else S.plaplace_square(n=5, p=3.0, seed=2))
    mesh = _mesh(P, prob)
    v = torch.tensor(prob.vhat(), device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: P.p1_energy(x, mesh, "fp64"), (v,),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-4)])
def test_backward_matches_oracle_and_patch_fd(P, oracle_mod, prec, tol):
    prob = S.neohooke_box_3d(17, 6, 5, 1.0, 6 / 17, 5 / 17, seed=4)
    O = oracle_mod.Oracle(prob)
    gref = O.grad_exact(prob.v)
    mesh = _mesh(P, prob)
    v = torch.tensor(prob.vhat(), device="cuda", requires_grad=True)
    J = P.p1_energy(v, mesh, prec)
    J.backward()
    g = v.grad.cpu().numpy()
    assert abs(J.item() - O.energy(prob.v)["J"]) <= (1e-12 if prec == "fp64" else 1e-5) * abs(J.item())
    assert np.linalg.norm(g - gref) / np.linalg.norm(gref) <= tol
    gfd, _ = mesh.grad_patch_fd(v.detach(), 1e-6)
    gfd = gfd.cpu().numpy()
    assert np.linalg.norm(g - gfd) / np.linalg.norm(gfd) <= max(tol, 1e-7)


def test_scaled_incoming_gradient_and_stale_forces(P, oracle_mod):
    prob = S.neohooke_beam_2d(30, 6, 2.0, 0.4, seed=5)
    O = oracle_mod.Oracle(prob)
    mesh = _mesh(P, prob)
    v1 = torch.tensor(prob.vhat(), device="cuda", requires_grad=True)
    (3.0 * P.p1_energy(v1, mesh, "fp64")).backward()
    g1 = O.grad_exact(prob.v)
    assert np.allclose(v1.grad.cpu().numpy(), 3.0 * g1, rtol=1e-12, atol=1e-12 * np.abs(g1).max())
    # two forwards, then the first backward: its kept gradient was overwritten -> recomputed
    v2 = v1.detach().clone().requires_grad_(True)
    v3 = (v1.detach() * 1.0001).requires_grad_(True)
    J2 = P.p1_energy(v2, mesh, "fp64")
    J3 = P.p1_energy(v3, mesh, "fp64")
    J2.backward()
    J3.backward()
    g3 = O.grad_exact(O.expand(v3.detach().cpu().numpy()))
    assert np.allclose(v2.grad.cpu().numpy(), g1, rtol=1e-12, atol=1e-12 * np.abs(g1).max())
    assert np.allclose(v3.grad.cpu().numpy(), g3, rtol=1e-12, atol=1e-12 * np.abs(g3).max())


def test_grad_gather_requires_forces(P):
    prob = S.plaplace_square(n=6)
    mesh = _mesh(P, prob)
    v = torch.tensor(prob.vhat(), device="cuda")
    mesh.grad_patch_fd(v, 1e-6)
    with pytest.raises(P.P1EError) as ei:
        mesh.grad_gather("fp64")
    assert ei.value.status == -7
    mesh.energy_forces(v, "mixed")
    with pytest.raises(P.P1EError):
        mesh.grad_gather("fp64")
    g = mesh.grad_gather("mixed")
    g2, _, _ = mesh.grad_exact(v, "mixed")
    assert torch.equal(g, g2)
