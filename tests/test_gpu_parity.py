"""GPU parity: libp1e (through its C ABI) against the FP64 oracle on the same seeded inputs.

Tolerances (stated, not tuned):
* FP64 mode: relative 1e-12 for J and for ||g - g_ref||_2 / ||g_ref||_2 (exact gradient).
* Mixed mode: relative 1e-5 for J, 1e-4 for the exact gradient in the 2-norm.
* Patch central differences (FP64): per DOF
      |g - g_ref| <= 32 u cond_n / (2 eps) + 4 u (|v_n| + eps) / eps * gabs_n + 1e-12 |g_ref|
  with u = 2^-53, cond_n = sum_T |T| (|W+|_abs + |W-|_abs) (rounding of the summed
  densities) and gabs_n = sum_T |T| |W+ - W-| / (2 eps) (rounding of the perturbed value
  v_n +- eps in the oracle); both scales come from the oracle.
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


def _cases():
    return {
        # the small configuration: p = 3 on the 33x33 unit-square grid, eps = 1e-6
        "plap_square_33": lambda: S.config_problem("plap_square_33"),
        "plap_p1.5_45": lambda: S.plaplace_square(n=45, p=1.5, seed=3),
        "plap_p5_37": lambda: S.plaplace_square(n=37, p=5.0, seed=4),
        # p = 4.5 and 2.7: the quarter-root branch and the general power of |g|^p
        "plap_p4.5_19": lambda: S.plaplace_square(n=19, p=4.5, seed=10),
        "plap_p2.7_23": lambda: S.plaplace_square(n=23, p=2.7, seed=11),
        "plap_lshape_16": lambda: S.plaplace_lshape(16, p=3.0, seed=5),
        "nh2d_beam_60x13": lambda: S.neohooke_beam_2d(60, 13, 2.0, 13 * 2.0 / 60, seed=6),
        "nh3d_box_13x7x5": lambda: S.neohooke_box_3d(13, 7, 5, 1.0, 7 / 13, 5 / 13, seed=7),
        # St. Venant-Kirchhoff (the extension named after eq. neoHook): energy, exact
        # gradient and patch differences through the same tiles
        "svk2d_beam_60x13": lambda: S.svk_beam_2d(60, 13, 2.0, 13 * 2.0 / 60, seed=12),
        "svk3d_box_13x7x5": lambda: S.svk_box_3d(13, 7, 5, 1.0, 7 / 13, 5 / 13, seed=13),
        "twisted_bar_L1": lambda: S.twisted_bar(1),
        "twisted_bar_L2": lambda: S.twisted_bar(2),
        # non-constant nodal loads (b = M f with the full consistent mass matrix): a linear
        # load on the structured box (geometry classes) ...
        "nh3d_box_13x7x5_linload": lambda: S.with_load(
            S.neohooke_box_3d(13, 7, 5, 1.0, 7 / 13, 5 / 13, seed=18), "linear"),
        # ... and jittered meshes (interior nodes moved by up to 0.2 h per coordinate: every
        # element has its own shape, so the per-element geometry path runs and the Morton
        # order sees irregular centroids) with random and linear loads
        "nh3d_box_jit_randload": lambda: S.with_load(
            S.neohooke_box_3d(13, 7, 5, 1.0, 7 / 13, 5 / 13, seed=14, jitter=0.2), "random",
            seed=1),
        "nh2d_beam_jit_linload": lambda: S.with_load(
            S.neohooke_beam_2d(60, 13, 2.0, 13 * 2.0 / 60, seed=15, jitter=0.2), "linear"),
        "plap_square_jit_randload": lambda: S.with_load(
            S.plaplace_square(n=29, p=3.0, seed=16, jitter=0.2), "random", seed=2),
        "svk3d_box_jit_linload": lambda: S.with_load(
            S.svk_box_3d(13, 7, 5, 1.0, 7 / 13, 5 / 13, seed=17, jitter=0.2), "linear"),
        # p = 1.5 with v = 0 on a sub-region: elements with grad v = 0 (gradient 0 there)
        "plap_p1.5_flat": lambda: _flat(S.plaplace_square(n=31, p=1.5, seed=19)),
        # Ginzburg-Landau (the scalar example of Section 7): a diffuse interface across a
        # strip and a slab, u = -1 / +1 prescribed at the two ends; the slab jittered with a
        # random load
        # the p-Laplacian with the component-wise norm (the density of Table 6)
        "plapo_lshape_16": lambda: S.plaplace_lshape(16, p=3.0, seed=22, kind="plaplace_ortho"),
        "plapo_square_jit_p1.5": lambda: S.plaplace_square(n=27, p=1.5, seed=23, jitter=0.2,
                                                           kind="plaplace_ortho"),
        "gl2d_strip_64": lambda: S.gl_domain(dim=2, n=64, width=0.5, eps_gl=0.01, seed=20),
        "gl3d_slab_jit_randload": lambda: S.with_load(
            S.gl_domain(dim=3, n=24, width=0.5, eps_gl=0.02, seed=21, jitter=0.2), "random",
            seed=3, scale=0.5),
    }


def _flat(prob, x_cut=0.4):
    """v = 0 on the nodes with x < x_cut: the elements there have a zero gradient."""
    prob.v[prob.coords[:, 0] < x_cut] = 0.0
    return prob


CASES = list(_cases().keys())


def _plap3d():
    """scalar p-Laplacian on a 3D Kuhn box (dim 3, d = 1), zero Dirichlet on the boundary"""
    coords, conn = S.kuhn_box_mesh(9, 6, 7, 0, 1, 0, 0.7, 0, 0.8)
    X = coords
    on = np.any((X < 1e-9) | (X > np.array([1, 0.7, 0.8]) - 1e-9), axis=1)
    rng = np.random.default_rng(9)
    v = rng.uniform(-1, 1, size=(X.shape[0], 1))
    v[on] = 0.0
    return S.Problem(name="plap3d", dim=3, ncomp=1, kind="plaplace", coords=coords, conn=conn,
                     dirichlet=on.astype(np.uint8)[:, None],
                     dirichlet_values=np.zeros((X.shape[0], 1)),
                     load=np.full((X.shape[0], 1), 2.0), v=v, p=3.0, eps=1e-6, h=1 / 9)


def _get(name):
    if name == "plap3d_box":
        return _plap3d()
    return _cases()[name]()


ALL = CASES + ["plap3d_box"]


def _setup(P, prob, modes):
    mesh = P.Mesh.from_problem(prob, modes=modes)
    vhat = torch.tensor(prob.vhat(), dtype=torch.float64, device="cuda")
    return mesh, vhat


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _rel2(g, gref):
    return np.linalg.norm(g - gref) / np.linalg.norm(gref)


@pytest.mark.parametrize("name", ALL)
def test_energy_and_exact_gradient_fp64(P, oracle_mod, name):
    _note(f"[parity fp64] {name}")
    prob = _get(name)
    O = oracle_mod.Oracle(prob)
    ref = O.energy(prob.v)
    gref = O.grad_exact(prob.v)
    mesh, vhat = _setup(P, prob, P.P1E_FP64)
    out3, flag = mesh.energy(vhat, "fp64")
    g, out3g, flag2 = mesh.grad_exact(vhat, "fp64")
    torch.cuda.synchronize()
    J, Jg, bv = out3.cpu().numpy()
    assert int(flag.item()) == 0 and int(flag2.item()) == 0
    assert _rel(J, ref["J"]) <= 1e-12
    assert _rel(Jg, ref["Jgrad"]) <= 1e-12
    assert abs(bv - ref["bv"]) <= 1e-12 * max(abs(ref["bv"]), abs(ref["Jgrad"]))
    assert np.array_equal(out3.cpu().numpy(), out3g.cpu().numpy())
    g = g.cpu().numpy()
    assert _rel2(g, gref) <= 1e-12
    # entrywise: the element forces summed per node are larger than the node's gradient
    # (they cancel), so the max-norm deviation is bounded looser than the 2-norm one
    assert np.abs(g - gref).max() <= 1e-11 * np.abs(gref).max()


@pytest.mark.parametrize("name", ALL)
def test_energy_and_exact_gradient_mixed(P, oracle_mod, name):
    _note(f"[parity mixed] {name}")
    prob = _get(name)
    O = oracle_mod.Oracle(prob)
    ref = O.energy(prob.v)
    gref = O.grad_exact(prob.v)
    mesh, vhat = _setup(P, prob, P.P1E_MIXED)
    g, out3, flag = mesh.grad_exact(vhat, "mixed")
    out3e, flage = mesh.energy(vhat, "mixed")
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    J = out3.cpu().numpy()
    assert _rel(J[0], ref["J"]) <= 1e-5
    assert _rel(J[1], ref["Jgrad"]) <= 1e-5
    assert np.array_equal(out3e.cpu().numpy(), J)
    assert _rel2(g.cpu().numpy(), gref) <= 1e-4


def _fd_tol(prob, gref, cond, gabs, eps):
    v = prob.vhat()
    return 32 * U * cond / (2 * eps) + 4 * U * (np.abs(v) + eps) / eps * gabs + 1e-12 * np.abs(gref)


@pytest.mark.parametrize("name", ALL)
def test_patch_fd_gradient(P, oracle_mod, name):
    _note(f"[parity fd] {name}")
    prob = _get(name)
    eps = prob.eps
    O = oracle_mod.Oracle(prob)
    gref, cond, gabs = O.grad_patch_fd(prob.v, eps, with_cond=True)
    mesh, vhat = _setup(P, prob, P.P1E_FD)
    g, flag = mesh.grad_patch_fd(vhat, eps)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    g = g.cpu().numpy()
    tol = _fd_tol(prob, gref, cond, gabs, eps)
    _note(f"[parity fd] {name}: worst |g - g_ref| / tol = {np.max(np.abs(g - gref) / tol):.3g}")
    bad = np.flatnonzero(np.abs(g - gref) > tol)
    assert bad.size == 0, (bad[:5], g[bad[:5]], gref[bad[:5]], tol[bad[:5]])
    # and the patch differences approximate the exact gradient to O(eps^2)
    gex = O.grad_exact(prob.v)
    assert _rel2(g, gex) <= 1e-6


FD4_CASES = ["plap_p1.5_45", "plap_p5_37", "nh2d_beam_60x13", "nh3d_box_13x7x5",
             "svk2d_beam_60x13", "svk3d_box_13x7x5", "gl2d_strip_64", "gl3d_slab_jit_randload"]


@pytest.mark.parametrize("name", FD4_CASES)
def test_fourth_order_patch_fd_gradient(P, oracle_mod, name):
    """The fourth-order scheme against the oracle's, per DOF, with its rounding scales (the
    oracle's cond and gabs for this scheme), and (deformations, whose second-order error is
    truncation at this step) closer to the exact gradient than the second-order scheme."""
    _note(f"[parity fd4] {name}")
    prob = _get(name)
    eps = prob.eps
    O = oracle_mod.Oracle(prob)
    gref, cond, gabs = O.grad_patch_fd(prob.v, eps, with_cond=True, order=4)
    mesh, vhat = _setup(P, prob, P.P1E_FD)
    g, flag = mesh.grad_patch_fd4(vhat, eps)
    g2, _ = mesh.grad_patch_fd(vhat, eps)
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    g, g2 = g.cpu().numpy(), g2.cpu().numpy()
    v = prob.vhat()
    tol = 32 * U * cond / (2 * eps) + 4 * U * (np.abs(v) + 2 * eps) / eps * gabs + 1e-12 * np.abs(gref)
    _note(f"[parity fd4] {name}: worst |g - g_ref| / tol = {np.max(np.abs(g - gref) / tol):.3g}")
    bad = np.flatnonzero(np.abs(g - gref) > tol)
    assert bad.size == 0, (bad[:5], g[bad[:5]], gref[bad[:5]], tol[bad[:5]])
    gex = O.grad_exact(prob.v)
    if prob.kind == "gl":  # a quartic in every nodal value: the scheme is exact up to rounding
        assert _rel2(g, gex) <= 1e-8
    elif prob.kind != "plaplace":  # (the p-Laplacian differences are rounding-limited here)
        assert _rel2(g, gex) <= _rel2(g2, gex)


def test_determinism_bitwise(P):
    prob = S.neohooke_box_3d(11, 9, 6, seed=2)
    mesh, vhat = _setup(P, prob, P.P1E_FP64 | P.P1E_MIXED | P.P1E_FD)
    for prec in ("fp64", "mixed"):
        a = [t.clone() for t in mesh.grad_exact(vhat, prec)]
        b = [t.clone() for t in mesh.grad_exact(vhat, prec)]
        for x, y in zip(a, b):
            assert torch.equal(x, y)
    f1, _ = mesh.grad_patch_fd(vhat, 1e-6)
    f1 = f1.clone()
    f2, _ = mesh.grad_patch_fd(vhat, 1e-6)
    assert torch.equal(f1, f2)


def test_bad_elements_are_flagged(P, oracle_mod):
    """det F <= 0 -> J = +Inf and the number of bad elements (oracle's count)."""
    prob = S.neohooke_box_3d(6, 5, 4, seed=3)
    rng = np.random.default_rng(0)
    v = prob.v.copy()
    free_nodes = np.flatnonzero(prob.dirichlet.max(axis=1) == 0)
    pick = rng.choice(free_nodes, 5, replace=False)
    v[pick] += 0.5 * rng.standard_normal((5, 3))  # large jumps invert some elements
    ref = oracle_mod.Oracle(prob).energy(v)
    assert ref["nbad"] > 0
    mesh = P.Mesh.from_problem(prob, modes=P.P1E_FP64 | P.P1E_MIXED | P.P1E_FD)
    vhat = torch.tensor(v.reshape(-1)[prob.free_mask], device="cuda")
    for prec in ("fp64", "mixed"):
        out3, flag = mesh.energy(vhat, prec)
        torch.cuda.synchronize()
        assert int(flag.item()) == ref["nbad"]
        assert np.isinf(out3[0].item()) and out3[0].item() > 0
    _, flag = mesh.grad_patch_fd(vhat, 1e-6)
    assert int(flag.item()) >= ref["nbad"]
    vnan = vhat.clone()
    vnan[7] = float("nan")
    out3, flag = mesh.energy(vnan, "fp64")
    assert int(flag.item()) > 0 and np.isinf(out3[0].item())


def test_empty_and_all_prescribed(P):
    """No elements: J = -b.v = 0 (b = 0), g = 0. No free DOFs: J from Dirichlet data only."""
    coords = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    conn = np.array([[0, 1, 2], [1, 3, 2]], dtype=np.int32)
    m = P.Mesh(2, "plaplace", conn[:0], coords, p=3.0, modes=P.P1E_FP64 | P.P1E_FD)
    vh = torch.ones(4, dtype=torch.float64, device="cuda")
    out3, flag = m.energy(vh, "fp64")
    g, _, _ = m.grad_exact(vh, "fp64")
    gf, _ = m.grad_patch_fd(vh, 1e-6)
    torch.cuda.synchronize()
    assert out3.cpu().tolist() == [0.0, 0.0, 0.0] and int(flag.item()) == 0
    assert torch.count_nonzero(g).item() == 0 and torch.count_nonzero(gf).item() == 0
    vals = np.array([[0.0], [1.0], [2.0], [3.0]])
    m2 = P.Mesh(2, "plaplace", conn, coords, dirichlet=np.ones((4, 1), np.uint8),
                dirichlet_values=vals, load=np.ones((4, 1)), p=2.0, modes=P.P1E_FP64)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    out3, flag = m2.energy(e, "fp64")
    g, _, _ = m2.grad_exact(e, "fp64")
    torch.cuda.synchronize()
    # grad v = (1, 2) on both triangles: J_grad = 1/2 * |(1,2)|^2 * 1 = 2.5;
    # b = M 1 = row sums of M: patch areas / 3; b.v = integral of v = 1.5
    J, Jg, bv = out3.cpu().tolist()
    assert Jg == pytest.approx(2.5, rel=1e-14) and bv == pytest.approx(1.5, rel=1e-14)
    assert J == pytest.approx(1.0, rel=1e-14)


def test_svk_is_finite_for_inverted_elements(P, oracle_mod):
    """St. Venant-Kirchhoff has no barrier at det F = 0: a reflected box (det F = -1 in every
    element) gives a finite energy and gradient equal to the oracle's, with no bad elements;
    a NaN in vhat is still flagged."""
    prob = S.svk_box_3d(5, 4, 3, 1.0, 0.8, 0.6, seed=3)
    v = prob.v.copy()
    v[:, 0] *= -1.0
    vh = torch.tensor(v.reshape(-1)[prob.free_mask], device="cuda")
    O = oracle_mod.Oracle(prob)
    ref = O.energy(v)
    assert ref["nbad"] == 0 and np.isfinite(ref["J"])
    mesh = P.Mesh.from_problem(prob, modes=P.P1E_FP64 | P.P1E_FD)
    g, out3, flag = mesh.grad_exact(vh, "fp64")
    torch.cuda.synchronize()
    assert int(flag.item()) == 0
    assert _rel(out3[0].item(), ref["J"]) <= 1e-12
    assert _rel2(g.cpu().numpy(), O.grad_exact(v)) <= 1e-12
    vnan = vh.clone()
    vnan[3] = float("nan")
    out3, flag = mesh.energy(vnan, "fp64")
    assert int(flag.item()) > 0 and np.isinf(out3[0].item())


def test_abi_errors_on_device(P):
    prob = S.plaplace_square(n=4)
    mesh, vhat = _setup(P, prob, P.P1E_FP64)
    with pytest.raises(P.P1EError) as ei:
        mesh.energy(vhat, "mixed")  # not bound for mixed
    assert ei.value.status == -7
    with pytest.raises(P.P1EError) as ei:
        mesh.grad_patch_fd4(vhat, 1e-6)  # not bound for the differences
    assert ei.value.status == -7
    m2, _ = _setup(P, prob, P.P1E_FD)
    for fd in (m2.grad_patch_fd, m2.grad_patch_fd4):
        for eps in (0.0, -1e-6, float("nan")):
            with pytest.raises(P.P1EError) as ei:
                fd(vhat, eps)
            assert ei.value.status == -1
    buf = torch.empty(64, dtype=torch.uint8, device="cuda")
    h = P.mesh_create(2, "plaplace", prob.conn, prob.coords, prob.dirichlet, p=3.0)
    try:
        with pytest.raises(P.P1EError) as ei:
            P.mesh_bind(h, buf, 64, P.P1E_FP64)
        assert ei.value.status in (-3, -1)
    finally:
        P.mesh_destroy(h)


def test_internal_order_does_not_change_results(P, oracle_mod):
    """The locality renumbering changes only the order of sums."""
    prob = S.neohooke_box_3d(14, 6, 5, 1.0, 6 / 14, 5 / 14, seed=11)
    v = torch.tensor(prob.vhat(), device="cuda")
    outs = []
    for flags in (0, P.P1E_INPUT_ORDER):
        m = P.Mesh.from_problem(prob, modes=P.P1E_FP64 | P.P1E_FD, flags=flags)
        g, o, _ = m.grad_exact(v, "fp64")
        f, _ = m.grad_patch_fd(v, 1e-6)
        outs.append((g.cpu().numpy(), o.cpu().numpy(), f.cpu().numpy()))
    (g0, o0, f0), (g1, o1, f1) = outs
    assert np.abs(o0 - o1).max() <= 1e-13 * np.abs(o0).max()
    assert np.linalg.norm(g0 - g1) <= 1e-13 * np.linalg.norm(g0)
    assert np.linalg.norm(f0 - f1) <= 1e-9 * np.linalg.norm(f0)


@pytest.mark.parametrize("name", ["nh3d_box_13x7x5", "plap_square_33", "nh2d_beam_60x13",
                                  "plap3d_box"])
def test_lds_slot_colouring_changes_nothing(P, name):
    """Binding for mixed precision recolours where each tile keeps its nodal values in LDS;
    FP64 results must be bitwise those of the same mesh bound without it (identity slots)."""
    prob = _plap3d() if name == "plap3d_box" else _cases()[name]()
    v = torch.tensor(prob.vhat(), device="cuda")
    outs = []
    for modes in (P.P1E_FP64 | P.P1E_FD, P.P1E_FP64 | P.P1E_FD | P.P1E_MIXED):
        m = P.Mesh.from_problem(prob, modes=modes)
        g, o, _ = m.grad_exact(v, "fp64")
        f, _ = m.grad_patch_fd(v, 1e-6)
        outs.append((g.clone(), o.clone(), f.clone()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("name", ["nh3d_box_13x7x5", "plap_square_33", "nh2d_beam_60x13"])
def test_geometry_classes_match_per_element_geometry(P, name):
    """Classed geometry (one record per class of elements whose records agree to 2^-40)
    changes results only at the level of coordinate rounding."""
    prob = _get(name)
    v = torch.tensor(prob.vhat(), device="cuda")
    outs = []
    for flags in (0, P.P1E_FULL_GEOMETRY):
        m = P.Mesh.from_problem(prob, modes=P.P1E_FP64 | P.P1E_MIXED | P.P1E_FD, flags=flags)
        assert (m.info["geometry_classes"] > 0) == (flags == 0)
        res = []
        for prec in ("fp64", "mixed"):
            g, o, _ = m.grad_exact(v, prec)
            e, _ = m.energy(v, prec)
            res += [g.cpu().numpy(), o.cpu().numpy(), e.cpu().numpy()]
        f, _ = m.grad_patch_fd(v, prob.eps)
        res.append(f.cpu().numpy())
        outs.append(res)
    tols = [1e-13, 1e-14, 1e-14, 1e-6, 1e-6, 1e-6, 1e-9]
    for a, b, t in zip(*outs, tols):
        assert np.linalg.norm(a - b) <= t * np.linalg.norm(b)


@pytest.mark.parametrize("name", ["nh3d_box_jit_randload", "nh2d_beam_jit_linload",
                                  "plap_square_jit_randload", "svk3d_box_jit_linload",
                                  "gl3d_slab_jit_randload"])
def test_geometry_on_the_fly_matches_stored_geometry(P, oracle_mod, name):
    """Jittered meshes have no geometry classes: by default the element pass forms B^-1 and
    |T| from the vertices' coordinate offsets (FP32 in mixed mode, FP64 otherwise);
    P1E_FULL_GEOMETRY stores them per element instead. Both against the oracle at the parity
    bars (FP64 1e-12; mixed 1e-5 energy, 1e-4 gradient), and FP64 against each other."""
    prob = _get(name)
    O = oracle_mod.Oracle(prob)
    ref = O.energy(prob.v)
    gref = O.grad_exact(prob.v)
    v = torch.tensor(prob.vhat(), device="cuda")
    g64 = {}
    for flags, mode in ((0, 2), (P.P1E_FULL_GEOMETRY, 0)):
        m = P.Mesh.from_problem(prob, modes=P.P1E_FP64 | P.P1E_MIXED, flags=flags)
        assert m.info["geometry_mode"] == mode
        for prec, tj, tg in (("fp64", 1e-12, 1e-12), ("mixed", 1e-5, 1e-4)):
            g, o, f = m.grad_exact(v, prec)
            torch.cuda.synchronize()
            assert int(f.item()) == 0
            ej = _rel(o[0].item(), ref["J"])
            eg = _rel2(g.cpu().numpy(), gref)
            _note(f"[geometry mode {mode}] {name} {prec}: J rel err {ej:.2e}, grad {eg:.2e}")
            assert ej <= tj and eg <= tg
            if prec == "fp64":
                g64[mode] = g.cpu().numpy()
        m.close()
    assert _rel2(g64[2], g64[0]) <= 1e-13


DELTAS = [-0.999, -0.9, -0.5, -0.3, -0.2929, -0.2928, -0.1, -1e-3, -1e-7, -1e-12, 0.0, 1e-12,
          1e-7, 1e-3, 0.2, 0.4142, 0.4143, 0.9, 1.5, 3.0, 20.0, 1e3]


def _w_exact(G, C1, D1):
    """W of eq. (neoHook) at F = I + G in 80-digit arithmetic (G's binary values taken exactly)."""
    import mpmath
    with mpmath.workdps(80):
        dim = G.shape[0]
        F = mpmath.matrix([[mpmath.mpf(float(G[i, j])) + (1 if i == j else 0) for j in range(dim)]
                           for i in range(dim)])
        detF = mpmath.det(F)
        I1 = sum(F[i, j] ** 2 for i in range(dim) for j in range(dim))
        return float(C1 * (I1 - dim - 2 * mpmath.log(detF)) + D1 * (detF - 1) ** 2)


@pytest.mark.parametrize("dim", [2, 3])
def test_neohooke_log_term_over_wide_det_range(P, dim):
    """One reference simplex (B^-1 = I, |T| = 1/dim!) under F = I + G with det F - 1 from
    -0.999 to 1e3 and down to 1e-12: J = |T| W against W evaluated in 80-digit arithmetic at
    the G the kernels see. Covers both branches of the log term (1 + d inside and outside
    [1/sqrt 2, sqrt 2)) and the cancellation near det F = 1."""
    C1, D1 = 0.7, 1.9
    x = np.vstack([np.zeros(dim), np.eye(dim)])
    conn = np.arange(dim + 1, dtype=np.int32)[None, :]
    mesh = P.Mesh(dim, "neohooke", conn, x, C1=C1, D1=D1, modes=P.P1E_FP64 | P.P1E_MIXED)
    vol = 1.0 / (2.0 if dim == 2 else 6.0)
    worst = {"fp64": 0.0, "mixed": 0.0}
    for d in DELTAS:
        for shear in (0.0, 0.3):
            G = np.zeros((dim, dim))
            G[0, 0] = d
            G[0, 1] = shear
            v = x + x @ G.T  # v_l = x_l + G x_l
            Geff = (v - x)[1:].T  # the displacement gradient the kernels form (B^-1 = I)
            vhat = torch.tensor(v.ravel(), device="cuda")
            for prec in ("fp64", "mixed"):
                Gk = Geff if prec == "fp64" else Geff.astype(np.float32).astype(np.float64)
                want = vol * _w_exact(Gk, C1, D1)
                out3, flag = mesh.energy(vhat, prec)
                J = float(out3[0].item())
                assert int(flag.item()) == 0
                if want == 0.0:
                    assert abs(J) <= 1e-300
                    continue
                worst[prec] = max(worst[prec], abs(J - want) / want)
    _note(f"[log term dim {dim}] worst relative error {worst}")
    assert worst["fp64"] <= 1e-13
    assert worst["mixed"] <= 1e-5


def test_binding_rejects_bad_buffers(P):
    """The binding validates every buffer whose raw pointer it hands to the library (dtype,
    device, contiguity, length) and raises ValueError before any kernel is launched."""
    prob = S.plaplace_square(n=6, p=3.0, seed=1)
    mesh, vhat = _setup(P, prob, P.P1E_FP64)
    n = mesh.n_free_dofs
    dev = vhat.device
    bad_vhats = [vhat.float(), vhat[:-1], vhat.cpu(), torch.zeros(2 * n, dtype=torch.float64,
                                                                  device=dev)[::2]]
    for bv in bad_vhats:
        for call in (lambda: mesh.energy(bv, "fp64"), lambda: mesh.grad_exact(bv, "fp64"),
                     lambda: P.mesh_minimize(mesh, bv, history=3, max_iters=2, prec="fp64")):
            with pytest.raises(ValueError):
                call()
    g_bad = [torch.empty(n, dtype=torch.float32, device=dev),
             torch.empty(n - 1, dtype=torch.float64, device=dev),
             torch.empty(n, dtype=torch.float64)]
    for gb in g_bad:
        with pytest.raises(ValueError):
            mesh.grad_exact(vhat, "fp64", g=gb)
        with pytest.raises(ValueError):
            mesh.grad_gather("fp64", g=gb)
    with pytest.raises(ValueError):
        mesh.grad_exact(vhat, "fp64", out3=torch.empty(2, dtype=torch.float64, device=dev))
    with pytest.raises(ValueError):
        mesh.grad_exact(vhat, "fp64", flag=torch.empty(1, dtype=torch.int64, device=dev))
    with pytest.raises(ValueError):
        mesh.energy_forces(vhat, "fp64", out3=torch.empty(3, dtype=torch.float32, device=dev))
    with pytest.raises(ValueError):
        mesh.grad_scale(torch.empty(n, dtype=torch.float64, device=dev),
                        torch.ones(2, dtype=torch.float64, device=dev))
    ws = torch.empty(64, dtype=torch.uint8, device=dev)
    with pytest.raises(ValueError):
        P.minimize(mesh.handle, vhat[:-1], 3, 2, "fp64", ws)
    with pytest.raises(ValueError):
        P.minimize(mesh.handle, vhat, 3, 2, "fp64", ws.cpu())
    # the mesh is untouched: a valid call still matches a fresh one bitwise
    g1, o1, _ = mesh.grad_exact(vhat, "fp64")
    g2, o2, _ = mesh.grad_exact(vhat, "fp64")
    assert torch.equal(g1, g2) and torch.equal(o1, o2)
