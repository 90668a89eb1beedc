"""Benchmark 4 of the paper (time-dependent twist of the Kuhn bar) with the library's
minimizer: the sequence of 24 minimizations of J (Neo-Hookean, f = 0) with the right wall
rotated by alpha(t) = 8 pi t / 24, each started from the previous minimizer, on the level-1,
-2 and -3 meshes (2133, 11925 and 77517 free DOFs). The minimal energies J_grad at
t = 3, 6, ..., 24 are compared with the values printed in Table 4
(tests/golden/table4_benchmark4.json).

The paper minimizes with a trust-region method and patch-difference gradients and stops at its
own tolerance; here L-BFGS(5) runs a fixed 2000, 4000 and 8000 iterations per step (the
conditioning grows about fourfold per level). Levels 1 and 2 reach the printed minima to
1.3e-4 and 8.9e-5, and the bar is 5e-4 relative. At level 3 the library's minima agree to
6e-5 up to t = 12, and from t = 15 on they lie below the printed energies by up to 8.8e-4
(t = 18); doubling the iterations moves them by at most 7e-5, so there the printed values are
not the converged minimum (or the trust-region path ended in another local minimum). Level 3
is therefore held to 1e-3, and at every level J_grad may exceed the printed value by at
most 5e-4 relative: the library never stops above the paper's minima.
"""

import json
import os

import numpy as np
import pytest
import torch

import p1e_synth as S

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2109_01158_amd as P
    return P


@pytest.mark.timeout(240)
@pytest.mark.parametrize("level,iters,bar", [(1, 2000, 5e-4), (2, 4000, 5e-4), (3, 8000, 1e-3)])
def test_benchmark4_twist_sequence(P, level, iters, bar):
    with open(os.path.join(HERE, "golden", "table4_benchmark4.json")) as f:
        gold = json.load(f)
    table = dict(zip(gold["steps"], gold["jgrad_printed"][str(level)]))
    T, amax = 24, 8.0 * np.pi
    vprev, worst = None, 0.0
    for t in range(1, T + 1):
        prob = S.twisted_bar(level, alpha=amax * t / T)
        mesh = P.Mesh.from_problem(prob, modes=P.P1E_FP64)
        assert mesh.info["n_free_dofs"] == gold["free_dofs"][str(level)]
        if vprev is None:  # t = 1: from the undeformed state v = x
            prob.v = np.where(prob.dirichlet == 1, prob.dirichlet_values, prob.coords)
            vprev = prob.vhat()
        v = torch.tensor(vprev, device="cuda")
        rep = P.mesh_minimize(mesh, v, history=5, max_iters=iters, prec="fp64")
        assert rep["status"] in (0, 2), rep
        vprev = v.cpu().numpy()
        if t in table:
            rel = (rep["J_grad"] - table[t]) / table[t]
            worst = max(worst, abs(rel))
            print(f"[benchmark 4] level {level} t={t:2d} J_grad {rep['J_grad']:.4f} "
                  f"table {table[t]:.4f} rel {rel:+.1e}", flush=True)
            assert abs(rel) <= bar and rel <= 5e-4, (t, rep["J_grad"], table[t])
        mesh.close()
    print(f"[benchmark 4] level {level}: worst relative difference {worst:.1e}", flush=True)
