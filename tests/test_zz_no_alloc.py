"""The allocation-free exact gradient p1e_grad_exact_static (scratch in the library's static
per-device array) against p1e_grad_exact (scratch in the mesh's bound buffer), through the C
ABI: the same kernels on the same inputs, so the results must agree bitwise; both are also
held to the FP64 oracle's bars (FP64 1e-12, mixed 1e-5 energy / 1e-4 gradient, relative).
Two calls in a row, the second on a smaller mesh, so that the second call finds the first
call's values in the shared array."""

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


def _call(P, fn, mesh, vhat, prec):
    dev = mesh.device
    g = torch.full((mesh.n_free_dofs,), float("nan"), dtype=torch.float64, device=dev)
    out3 = torch.full((3,), float("nan"), dtype=torch.float64, device=dev)
    flag = torch.full((1,), -1, dtype=torch.int32, device=dev)
    fn(mesh.handle, vhat, prec, g, out3, flag)
    torch.cuda.synchronize()
    return g.cpu().numpy(), out3.cpu().numpy(), int(flag.item())


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_static_scratch_matches_grad_exact(P, oracle_mod, prec):
    from paper_2109_01158_amd import api
    dev = torch.device("cuda:0")
    # a 3D box of several tiles with halo rows, then a smaller 2D beam
    probs = [S.neohooke_box_3d(48, 12, 12, 1.0, 0.25, 0.25, seed=21),
             S.neohooke_beam_2d(60, 13, 2.0, 13 * 2.0 / 60, seed=22)]
    for prob in probs:
        print(f"static scratch: {prob.name} ne={prob.ne} {prec}", flush=True)
        mesh = P.Mesh.from_problem(prob, modes=P.P1E_FP64 | P.P1E_MIXED, device=dev)
        info = mesh.info
        need = (-(-32 * max(info["n_tiles"], 1) // 256) * 256 + -(-4 * max(info["n_tiles"], 1) // 256) * 256
                + 8 * info["n_halo_slots"] * info["ncomp"])
        assert need <= P.P1E_STATIC_SCRATCH_BYTES
        vhat = torch.tensor(prob.vhat(), device=dev)
        gs, os_, fs = _call(P, api.grad_exact_static, mesh, vhat, prec)
        gr, or_, fr = _call(P, api.grad_exact, mesh, vhat, prec)
        assert fs == 0 and fr == 0
        assert np.array_equal(gs, gr), "gradient differs from p1e_grad_exact"
        assert np.array_equal(os_, or_), "energy differs from p1e_grad_exact"
        O = oracle_mod.Oracle(prob)
        ref = O.energy(prob.v)
        gref = O.grad_exact(prob.v)
        ej = abs(os_[0] - ref["J"]) / abs(ref["J"])
        eg = np.linalg.norm(gs - gref) / np.linalg.norm(gref)
        tj, tg = (1e-12, 1e-12) if prec == "fp64" else (1e-5, 1e-4)
        print(f"  J rel err {ej:.2e}  grad rel err {eg:.2e}", flush=True)
        assert ej <= tj and eg <= tg
        mesh.close()
