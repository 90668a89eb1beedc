"""Structured triangle and tetrahedron meshes (pure index/coordinate generation).

Node numbering is lexicographic with x fastest. Element connectivity is 0-based int32.

* 2D: every grid cell (i, j) is split along its SW-NE diagonal into the triangles
  (i,j),(i+1,j),(i+1,j+1) and (i,j),(i+1,j+1),(i,j+1).
* 3D: every cube is split into the six Kuhn tetrahedra that share the cube diagonal from
  corner (0,0,0) to corner (1,1,1): {c000, c000+e_a, c000+e_a+e_b, c111} for the six
  permutations (a, b, c) of the axes. Uniform refinement of this split by halving the
  cell size gives the bar meshes of the paper's 3D benchmarks (Section 4.2, Table 1).
"""

import itertools

import numpy as np


def rect_tri_mesh(nx, ny, x0=0.0, x1=1.0, y0=0.0, y1=1.0):
    """Right-triangle mesh of [x0,x1]x[y0,y1] with nx*ny cells -> (coords[nn,2], conn[ne,3])."""
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")  # shape (ny+1, nx+1), x fastest when raveled
    coords = np.stack([X.ravel(), Y.ravel()], axis=1).astype(np.float64)
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    n00 = i + (nx + 1) * j
    n10 = n00 + 1
    n01 = n00 + (nx + 1)
    n11 = n01 + 1
    t1 = np.stack([n00, n10, n11], axis=1)
    t2 = np.stack([n00, n11, n01], axis=1)
    conn = np.stack([t1, t2], axis=1).reshape(-1, 3).astype(np.int32)
    return coords, conn


def kuhn_box_mesh(nx, ny, nz, x0=0.0, x1=1.0, y0=0.0, y1=1.0, z0=0.0, z1=1.0):
    """Kuhn 6-tet mesh of a box with nx*ny*nz cubes -> (coords[nn,3], conn[ne,4])."""
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    zs = np.linspace(z0, z1, nz + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")  # x fastest when raveled
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1).astype(np.float64)
    sx, sy, sz = 1, nx + 1, (nx + 1) * (ny + 1)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    base = (i * sx + j * sy + k * sz).ravel().astype(np.int64)
    step = (sx, sy, sz)
    tets = []
    for perm in itertools.permutations(range(3)):
        a, b, _ = perm
        v0 = base
        v1 = base + step[a]
        v2 = base + step[a] + step[b]
        v3 = base + sx + sy + sz
        tets.append(np.stack([v0, v1, v2, v3], axis=1))
    conn = np.stack(tets, axis=1).reshape(-1, 4).astype(np.int32)
    return coords, conn


def kuhn_bar_level(level, lx=0.4, ly=0.01, lz=0.01):
    """The 3D bar (0,lx) x (-ly/2,ly/2) x (-lz/2,lz/2) at refinement ``level`` (1-based).

    Level L has (80*2^(L-1)) x (2*2^(L-1))^2 cubes of side lx/(80*2^(L-1)), i.e. the node,
    element and free-DOF counts printed in Table 1 of the paper.
    """
    r = 2 ** (level - 1)
    return kuhn_box_mesh(80 * r, 2 * r, 2 * r, 0.0, lx, -ly / 2, ly / 2, -lz / 2, lz / 2)


def jitter_interior(coords, h, frac=0.2, seed=0):
    """A copy of ``coords`` whose nodes strictly inside the bounding box are moved by
    independent offsets drawn from U[-frac h, frac h] per coordinate (seeded); nodes on the
    bounding box stay, so the domain, its boundary faces and the clamped faces are unchanged.

    On the right-triangle and Kuhn meshes above every element height is at least h / sqrt(2)
    and a vertex moves by at most frac h sqrt(2) along any face normal of the form
    (e_a - e_b) / sqrt(2) or e_a, so no element degenerates or flips for frac < 0.25. The moved
    meshes have as many element shapes as elements (an unstructured mesh for the kernels).
    """
    coords = np.array(coords, dtype=np.float64, copy=True)
    lo, hi = coords.min(axis=0), coords.max(axis=0)
    tol = 1e-9 * max(1.0, float(np.abs(coords).max()))
    inside = np.all((coords > lo + tol) & (coords < hi - tol), axis=1)
    rng = np.random.default_rng(seed)
    off = rng.uniform(-frac * h, frac * h, size=coords.shape)
    coords[inside] += off[inside]
    return coords


def lshape_tri_mesh(n):
    """L-shaped domain [-1,1]^2 minus (0,1]x[-1,0) as three unit squares, n cells per unit.

    Built from the right-triangle grid of [-1,1]^2 with the cells of the removed quadrant
    dropped and unused nodes compacted away.
    """
    coords, conn = rect_tri_mesh(2 * n, 2 * n, -1.0, 1.0, -1.0, 1.0)
    cent = coords[conn].mean(axis=1)
    keep = ~((cent[:, 0] > 0.0) & (cent[:, 1] < 0.0))
    conn = conn[keep]
    used = np.unique(conn)
    remap = -np.ones(coords.shape[0], dtype=np.int64)
    remap[used] = np.arange(used.size)
    return coords[used].copy(), remap[conn].astype(np.int32)
