"""The differentiation hook: torch.autograd.Function with the exact gradient as backward,
checked by gradcheck (FP64), against the oracle gradient and against the patch
central-difference gradient, including a scaled incoming gradient, interleaved forwards and
backwards, a second backward through a retained graph, and the in-place scaling call."""

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
    # two forwards, then their backwards: each keeps its own gradient
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


def test_retained_graph_second_backward(P, oracle_mod):
    prob = S.neohooke_beam_2d(20, 5, 2.0, 0.4, seed=6)
    O = oracle_mod.Oracle(prob)
    g1 = O.grad_exact(prob.v)
    mesh = _mesh(P, prob)
    v = torch.tensor(prob.vhat(), device="cuda", requires_grad=True)
    J = P.p1_energy(v, mesh, "fp64")
    J.backward(retain_graph=True)
    first = v.grad.clone()
    (2.0 * J).backward()  # recomputed at the saved input, scaled by 2, accumulated
    tol = 1e-12 * np.abs(g1).max()
    assert np.allclose(first.cpu().numpy(), g1, rtol=1e-12, atol=tol)
    assert np.allclose(v.grad.cpu().numpy(), 3.0 * g1, rtol=1e-12, atol=3 * tol)


def test_grad_scale_in_place(P):
    prob = S.plaplace_square(n=10, p=3.0, seed=3)  # 81 free DOFs
    mesh = _mesh(P, prob)
    v = torch.tensor(prob.vhat(), device="cuda")
    g, _, _ = mesh.grad_exact(v, "fp64")
    ref = g.clone()
    one = torch.ones(1, dtype=torch.float64, device="cuda")
    mesh.grad_scale(g, one)
    assert torch.equal(g, ref)  # scale 1: untouched, bitwise
    s = torch.full((1,), -2.5, dtype=torch.float64, device="cuda")
    mesh.grad_scale(g, s)
    assert torch.equal(g, ref * -2.5)  # one IEEE product per entry
    # an odd length and a buffer 8 bytes off a 16-byte boundary take the scalar path
    buf = torch.empty(mesh.n_free_dofs + 1, dtype=torch.float64, device="cuda")
    h = buf[1:]
    h.copy_(ref)
    mesh.grad_scale(h, s)
    assert torch.equal(h, ref * -2.5)


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_graph_replays_match_eager_steps(P, prec):
    """The autograd step captured in a HIP graph (GraphedStep) after eager backward passes on
    the same vhat: every replay, with eager steps, synchronisations and an in-place change of
    vhat between the replays, gives J and the gradient of an eager step at the same vhat,
    bitwise."""
    prob = S.neohooke_box_3d(17, 6, 5, 1.0, 6 / 17, 5 / 17, seed=4)
    mesh = _mesh(P, prob)
    v = torch.tensor(prob.vhat(), device="cuda", requires_grad=True)
    for _ in range(2):
        v.grad = None
        P.p1_energy(v, mesh, prec).backward()
    gs = P.GraphedStep(v, mesh, prec)
    rng = np.random.default_rng(7)
    for k in range(5):
        if k:
            dv = torch.tensor(1e-4 * rng.standard_normal(v.numel()), device="cuda")
            v.data.add_(dv)
        ve = v.detach().clone().requires_grad_(True)
        Je = P.p1_energy(ve, mesh, prec)
        Je.backward()
        torch.cuda.synchronize()
        J, g = gs.replay()
        torch.cuda.synchronize()
        assert g is gs.grad
        assert J.item() == Je.item()
        assert torch.equal(g, ve.grad)
