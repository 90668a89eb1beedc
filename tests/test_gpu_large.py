"""Parity at the full workload sizes, in the launch configuration the benchmark times.

* 2D Neo-Hookean beam, 1,003,520 triangles: FP64 and mixed J and exact gradient vs the
  oracle (all DOFs).
* 3D Neo-Hookean box, 5,840,160 tets: the same, plus patch central differences (eps = 1e-6)
  on 3000 sampled DOFs against the oracle.
* 3D Neo-Hookean box, 48,261,420 tets: FP64 exact gradient vs FP64 patch central differences
  (eps = 1e-8) over all 24,652,440 DOFs on the GPU, and both against the oracle on sampled
  DOFs (the oracle evaluates the energy and the exact gradient of the whole mesh).

Tolerances as in test_gpu_parity.py.
"""

import numpy as np
import pytest
import torch

import p1e_synth as S

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_01158_amd as P
    return P


def _note(msg):
    print(msg, flush=True)


def _rel2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _fd_tol(v, gref, cond, gabs, eps):
    return 32 * U * cond / (2 * eps) + 4 * U * (np.abs(v) + eps) / eps * gabs + 1e-12 * np.abs(gref)


@pytest.mark.timeout(300)
@pytest.mark.parametrize("name", ["nh2d_beam_1M", "nh3d_box_6M"])
def test_full_size_energy_gradient(P, oracle_mod, name):
    _note(f"[large] {name}: building inputs")
    prob = S.config_problem(name)
    O = oracle_mod.Oracle(prob)
    ref = O.energy(prob.v)
    gref = O.grad_exact(prob.v)
    _note(f"[large] {name}: oracle done, ne={prob.ne}")
    mesh = P.Mesh.from_problem(prob, modes=P.P1E_FP64 | P.P1E_MIXED | P.P1E_FD)
    v = torch.tensor(prob.vhat(), device="cuda")
    for prec, tj, tg in (("fp64", 1e-12, 1e-12), ("mixed", 1e-5, 1e-4)):
        g, out3, flag = mesh.grad_exact(v, prec)
        torch.cuda.synchronize()
        assert int(flag.item()) == 0
        J = out3.cpu().numpy()
        ej = abs(J[0] - ref["J"]) / abs(ref["J"])
        eg = _rel2(g.cpu().numpy(), gref)
        _note(f"[large] {name} {prec}: J rel err {ej:.2e}, grad rel err {eg:.2e}")
        assert ej <= tj and eg <= tg
    if name == "nh3d_box_6M":
        rng = np.random.default_rng(5)
        pos = np.sort(rng.choice(O.free_dofs.size, 3000, replace=False))
        gfr, cond, gabs = O.grad_patch_fd(prob.v, prob.eps, sample=pos, with_cond=True)
        gf, flag = mesh.grad_patch_fd(v, prob.eps)
        gf = gf.cpu().numpy()[pos]
        tol = _fd_tol(prob.vhat()[pos], gfr, cond, gabs, prob.eps)
        assert np.all(np.abs(gf - gfr) <= tol)


@pytest.mark.timeout(600)
def test_48M_exact_vs_patch_fd(P, oracle_mod):
    _note("[large] nh3d_box_48M: building inputs")
    prob = S.config_problem("nh3d_box_48M")
    assert prob.ne == 48261420 and prob.n_free_dofs == 24652440
    mesh = P.Mesh.from_problem(prob, modes=P.P1E_FP64 | P.P1E_FD)
    info = mesh.info
    # 4 incidences per tet minus the 12 per cube of the clamped face x = 0
    assert info["nnz"] == 4 * prob.ne - 12 * 93 * 93 and info["max_valence"] == 24
    _note("[large] nh3d_box_48M: mesh bound")
    v = torch.tensor(prob.vhat(), device="cuda")
    ge, out3, flag = mesh.grad_exact(v, "fp64")
    gf, flag2 = mesh.grad_patch_fd(v, prob.eps)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0 and int(flag2.item()) == 0
    ge = ge.cpu().numpy()
    gf = gf.cpu().numpy()
    d = _rel2(gf, ge)
    _note(f"[large] 48M: ||g_fd - g_exact|| / ||g_exact|| = {d:.2e}")
    assert d <= 1e-6
    J = out3.cpu().numpy()
    del mesh
    torch.cuda.empty_cache()
    O = oracle_mod.Oracle(prob)
    ref = O.energy(prob.v)
    assert abs(J[0] - ref["J"]) <= 1e-12 * abs(ref["J"])
    gref = O.grad_exact(prob.v)
    eg = _rel2(ge, gref)
    _note(f"[large] 48M: exact gradient rel err vs oracle {eg:.2e}")
    assert eg <= 1e-12
    rng = np.random.default_rng(7)
    pos = np.sort(rng.choice(O.free_dofs.size, 1000, replace=False))
    gfr, cond, gabs = O.grad_patch_fd(prob.v, prob.eps, sample=pos, with_cond=True)
    tol = _fd_tol(prob.vhat()[pos], gfr, cond, gabs, prob.eps)
    assert np.all(np.abs(gf[pos] - gfr) <= tol)
