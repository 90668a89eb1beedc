"""Seeded problem instances shaped like the paper's workloads.

A :class:`Problem` carries everything both sides consume: mesh, Dirichlet mask and values
per DOF, nodal load f (its P1 interpolant is the loading functional), material data and a
full nodal trial field ``v`` (the deformation for Neo-Hookean, the scalar field for the
p-Laplacian). Free DOFs are the DOFs with ``dirichlet == 0``, numbered in ascending global
DOF order n = d*i + j (node-major, interleaved components).

Amplitude rule for random displacements: the literal amplitude 1e-3 inverts elements on the
fine meshes, so the displacement amplitude is ``min(1e-3, 0.15*h)`` with h the cell edge.
For axis-aligned right triangles and Kuhn tetrahedra every displacement-gradient entry is a
difference of two nodal values over h, hence bounded by 0.3, which keeps det F > 0.
"""

from dataclasses import dataclass, field, replace

import numpy as np

from .meshes import (jitter_interior, kuhn_bar_level, kuhn_box_mesh, lshape_tri_mesh,
                     rect_tri_mesh)


@dataclass
class Problem:
    name: str
    dim: int
    ncomp: int
    kind: str                 # "plaplace", "plaplace_ortho" (component-wise norm), "neohooke",
                              # "svk" (St. Venant-Kirchhoff) or "gl" (Ginzburg-Landau)
    coords: np.ndarray        # f64 [nn, dim]
    conn: np.ndarray          # i32 [ne, dim+1]
    dirichlet: np.ndarray     # u8  [nn, ncomp], 1 = prescribed
    dirichlet_values: np.ndarray  # f64 [nn, ncomp]
    load: np.ndarray          # f64 [nn, ncomp], nodal values of f
    v: np.ndarray             # f64 [nn, ncomp], trial field (full, Dirichlet values included)
    p: float = 2.0
    E: float = 0.0
    nu: float = 0.0
    eps: float = 1e-6         # central-difference step
    h: float = 0.0
    amp: float = 0.0
    C1: float = 0.0           # Ginzburg-Landau coefficients (the other kinds derive theirs
    D1: float = 0.0           # from p or from E, nu)
    meta: dict = field(default_factory=dict)

    @property
    def nn(self):
        return self.coords.shape[0]

    @property
    def ne(self):
        return self.conn.shape[0]

    @property
    def free_mask(self):
        """Boolean mask over the flattened DOF vector (ascending DOF order)."""
        return self.dirichlet.reshape(-1) == 0

    @property
    def n_free_dofs(self):
        return int(self.free_mask.sum())

    def vhat(self, v=None):
        """Restriction of a full nodal field to the free DOFs, ascending DOF order."""
        v = self.v if v is None else v
        return np.ascontiguousarray(v.reshape(-1)[self.free_mask], dtype=np.float64)


def _dirichlet_on(coords, ncomp, pred):
    on = pred(coords)
    mask = np.zeros((coords.shape[0], ncomp), dtype=np.uint8)
    mask[on, :] = 1
    return mask


def plaplace_square(n=32, p=3.0, f=-10.0, seed=0, eps=1e-6, amp=1.0, jitter=0.0,
                    kind="plaplace"):
    """Unit square, (n+1)^2 nodes, 2n^2 right triangles, zero Dirichlet boundary,
    interior v ~ amp*U[-1,1]. jitter > 0: interior nodes moved by up to jitter/n per
    coordinate (jitter_interior, seed + 1000). kind: "plaplace" or "plaplace_ortho"."""
    coords, conn = rect_tri_mesh(n, n)
    if jitter > 0.0:
        coords = jitter_interior(coords, 1.0 / n, jitter, seed + 1000)
    tol = 0.5 / n
    dmask = _dirichlet_on(
        coords, 1,
        lambda X: (X[:, 0] < tol) | (X[:, 0] > 1 - tol) | (X[:, 1] < tol) | (X[:, 1] > 1 - tol))
    rng = np.random.default_rng(seed)
    v = amp * rng.uniform(-1.0, 1.0, size=(coords.shape[0], 1))
    v[dmask == 1] = 0.0
    return Problem(
        name=f"{kind}_square_n{n}_p{p:g}", dim=2, ncomp=1, kind=kind,
        coords=coords, conn=conn, dirichlet=dmask,
        dirichlet_values=np.zeros((coords.shape[0], 1)),
        load=np.full((coords.shape[0], 1), float(f)), v=v, p=float(p), eps=eps, h=1.0 / n,
        amp=amp)


def _neohooke_random(coords, conn, dim, dmask, load_vec, seed, h, eps, name, amp=None):
    if amp is None:
        amp = min(1e-3, 0.15 * h)
    rng = np.random.default_rng(seed)
    u = amp * rng.uniform(-1.0, 1.0, size=(coords.shape[0], dim))
    u[dmask == 1] = 0.0
    v = coords + u
    load = np.tile(np.asarray(load_vec, dtype=np.float64), (coords.shape[0], 1))
    return Problem(
        name=name, dim=dim, ncomp=dim, kind="neohooke", coords=coords, conn=conn,
        dirichlet=dmask, dirichlet_values=np.where(dmask == 1, coords, 0.0), load=load, v=v,
        E=2e8, nu=0.3, eps=eps, h=h, amp=amp)


def neohooke_beam_2d(nx=2240, ny=224, lx=2.0, ly=0.2, seed=0, eps=1e-6, amp=None, jitter=0.0):
    """Beam [0,lx]x[0,ly], left edge clamped (v = x), f = (0, -3.5e7). jitter > 0: interior
    nodes moved by up to jitter*h per coordinate (jitter_interior, seed + 1000)."""
    coords, conn = rect_tri_mesh(nx, ny, 0.0, lx, 0.0, ly)
    h = lx / nx
    if jitter > 0.0:
        coords = jitter_interior(coords, min(h, ly / ny), jitter, seed + 1000)
    dmask = _dirichlet_on(coords, 2, lambda X: X[:, 0] < 0.5 * h)
    return _neohooke_random(coords, conn, 2, dmask, (0.0, -3.5e7), seed, h, eps,
                            f"neohooke_beam_{nx}x{ny}", amp)


def neohooke_box_3d(nx=460, ny=46, nz=46, lx=1.0, ly=0.1, lz=0.1, seed=0, eps=1e-6, amp=None,
                    jitter=0.0):
    """Box [0,lx]x[0,ly]x[0,lz], Kuhn tets, face x = 0 clamped (v = x), f = (0,-3.5e7,0).
    jitter > 0: interior nodes moved by up to jitter*h per coordinate (jitter_interior,
    seed + 1000)."""
    coords, conn = kuhn_box_mesh(nx, ny, nz, 0.0, lx, 0.0, ly, 0.0, lz)
    h = lx / nx
    if jitter > 0.0:
        coords = jitter_interior(coords, min(h, ly / ny, lz / nz), jitter, seed + 1000)
    dmask = _dirichlet_on(coords, 3, lambda X: X[:, 0] < 0.5 * h)
    return _neohooke_random(coords, conn, 3, dmask, (0.0, -3.5e7, 0.0), seed, h, eps,
                            f"neohooke_box_{nx}x{ny}x{nz}", amp)


def svk_beam_2d(nx=60, ny=13, lx=2.0, ly=0.4, seed=0, eps=1e-6, amp=None, jitter=0.0):
    """The beam of neohooke_beam_2d (same mesh, clamp, load, E, nu and displacement draw)
    with the St. Venant-Kirchhoff density."""
    pb = neohooke_beam_2d(nx, ny, lx, ly, seed, eps, amp, jitter)
    return replace(pb, kind="svk", name=f"svk_beam_{nx}x{ny}")


def svk_box_3d(nx=13, ny=7, nz=5, lx=1.0, ly=0.5, lz=0.4, seed=0, eps=1e-6, amp=None,
               jitter=0.0):
    """The box of neohooke_box_3d with the St. Venant-Kirchhoff density."""
    pb = neohooke_box_3d(nx, ny, nz, lx, ly, lz, seed, eps, amp, jitter)
    return replace(pb, kind="svk", name=f"svk_box_{nx}x{ny}x{nz}")


def gl_domain(dim=2, n=64, width=0.25, eps_gl=0.01, seed=0, eps=1e-6, amp=0.1, jitter=0.0,
              f=0.0):
    """Ginzburg-Landau (scalar, W = C1 |grad u|^2 + D1 (u^2 - 1)^2 with C1 = eps_gl / 2,
    D1 = 1/4): the strip [-1,1] x [0,width] (2D, right triangles) or the box
    [-1,1] x [0,width]^2 (3D, Kuhn tets) with n cells along x; u = -1 prescribed at x = -1 and
    u = +1 at x = +1; trial field the interface profile tanh(x / sqrt(2 eps_gl)) plus
    amp * U[-1,1] on the free nodes; constant load f."""
    m = max(1, int(round(n * width / 2.0)))
    if dim == 2:
        coords, conn = rect_tri_mesh(n, m, -1.0, 1.0, 0.0, width)
    else:
        coords, conn = kuhn_box_mesh(n, m, m, -1.0, 1.0, 0.0, width, 0.0, width)
    h = 2.0 / n
    if jitter > 0.0:
        coords = jitter_interior(coords, min(h, width / m), jitter, seed + 1000)
    x = coords[:, 0]
    dmask = _dirichlet_on(coords, 1, lambda X: (X[:, 0] < -1 + 0.5 * h) | (X[:, 0] > 1 - 0.5 * h))
    dval = np.where(x > 0, 1.0, -1.0)[:, None] * dmask
    rng = np.random.default_rng(seed)
    v = np.tanh(x / np.sqrt(2.0 * eps_gl))[:, None] + amp * rng.uniform(-1.0, 1.0, (len(x), 1))
    v = np.where(dmask == 1, dval, v)
    return Problem(
        name=f"gl{dim}d_n{n}", dim=dim, ncomp=1, kind="gl", coords=coords, conn=conn,
        dirichlet=dmask, dirichlet_values=dval.astype(np.float64),
        load=np.full((len(x), 1), float(f)), v=v, eps=eps, h=h, amp=amp,
        C1=0.5 * eps_gl, D1=0.25, meta={"eps_gl": eps_gl, "width": width})


def twisted_bar(level, alpha=2.0 * np.pi, lx=0.4, ly=0.01, lz=0.01):
    """Benchmark-2 workload: Kuhn bar at ``level``, both end walls prescribed, and the
    twist deformation (x, R(alpha x / lx) (y, z)) at every node, no load."""
    coords, conn = kuhn_bar_level(level, lx, ly, lz)
    h = lx / (80 * 2 ** (level - 1))
    dmask = _dirichlet_on(coords, 3, lambda X: (X[:, 0] < 0.5 * h) | (X[:, 0] > lx - 0.5 * h))
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    th = alpha * x / lx
    v = np.stack([x, np.cos(th) * y + np.sin(th) * z, -np.sin(th) * y + np.cos(th) * z], axis=1)
    return Problem(
        name=f"twisted_bar_L{level}", dim=3, ncomp=3, kind="neohooke", coords=coords,
        conn=conn, dirichlet=dmask, dirichlet_values=np.where(dmask == 1, v, 0.0),
        load=np.zeros_like(coords), v=v, E=2e8, nu=0.3, eps=1e-8, h=h, amp=0.0,
        meta={"alpha": alpha, "lx": lx, "ly": ly, "lz": lz})


def plaplace_lshape(n, p=3.0, f=-10.0, seed=0, amp=1.0, eps=1e-5, kind="plaplace"):
    """L-shape of three unit squares, n cells per unit length, zero Dirichlet boundary.
    kind: "plaplace" (|grad v|^p / p) or "plaplace_ortho" (sum_m |d_m v|^p / p)."""
    coords, conn = lshape_tri_mesh(n)
    # boundary nodes: on the outer square boundary or on the two re-entrant edges
    X = coords
    t = 0.5 / n
    on = ((np.abs(X[:, 0]) > 1 - t) | (np.abs(X[:, 1]) > 1 - t)
          | ((X[:, 0] > -t) & (np.abs(X[:, 1]) < t))
          | ((np.abs(X[:, 0]) < t) & (X[:, 1] < t)))
    dmask = on.astype(np.uint8)[:, None]
    rng = np.random.default_rng(seed)
    v = amp * rng.uniform(-1.0, 1.0, size=(coords.shape[0], 1))
    v[dmask == 1] = 0.0
    return Problem(
        name=f"{kind}_lshape_n{n}", dim=2, ncomp=1, kind=kind, coords=coords,
        conn=conn, dirichlet=dmask, dirichlet_values=np.zeros((coords.shape[0], 1)),
        load=np.full((coords.shape[0], 1), float(f)), v=v, p=float(p), eps=eps, h=1.0 / n,
        amp=amp)


def with_load(prob, kind, seed=0, scale=None):
    """A copy of ``prob`` with another nodal load f (its P1 interpolant is the load):
    "linear": f_j(x) = scale_j (1 + sum_m c_jm x_m / L) with fixed coefficients c in
    [-1, 1] (L = the domain's largest extent); "random": f_j = scale_j * U[-1, 1] per node
    (seeded). scale defaults to the magnitude of the problem's own constant load (per
    component, 1 where it is zero)."""
    X = prob.coords
    d = prob.ncomp
    if scale is None:
        base = np.abs(prob.load).max(axis=0)
        scale = np.where(base > 0, base, 1.0)
    scale = np.broadcast_to(np.asarray(scale, dtype=np.float64), (d,))
    if kind == "linear":
        L = float((X.max(axis=0) - X.min(axis=0)).max())
        c = np.array([[0.5, -0.75, 0.25], [-0.25, 1.0, -0.5], [0.75, 0.5, -1.0]])[:d, :prob.dim]
        f = scale[None, :] * (1.0 + X @ c.T / L)
    elif kind == "random":
        rng = np.random.default_rng(seed)
        f = scale[None, :] * rng.uniform(-1.0, 1.0, size=(prob.nn, d))
    else:
        raise ValueError(kind)
    return replace(prob, load=np.ascontiguousarray(f), name=f"{prob.name}_{kind}load")


# The five workloads: small p-Laplacian, 2D beam, 3D box (the headline), the serving mix
# (built by the serving driver, not here) and the large 3D box for exact vs FD.
CONFIGS = {
    "plap_square_33": dict(fn=plaplace_square, kw=dict(n=32, p=3.0, f=-10.0, seed=0, eps=1e-6)),
    "nh2d_beam_1M": dict(fn=neohooke_beam_2d, kw=dict(nx=2240, ny=224, seed=0, eps=1e-6)),
    "nh3d_box_6M": dict(fn=neohooke_box_3d, kw=dict(nx=460, ny=46, nz=46, seed=0, eps=1e-6)),
    "nh3d_box_48M": dict(fn=neohooke_box_3d, kw=dict(nx=930, ny=93, nz=93, seed=0, eps=1e-8)),
}


def config_problem(name, **override):
    c = CONFIGS[name]
    kw = dict(c["kw"])
    kw.update(override)
    return c["fn"](**kw)
