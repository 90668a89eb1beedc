"""FP64 CPU oracle for P1 energies and gradients (arXiv 2109.01158).

TEST INFRASTRUCTURE ONLY: the test suite, the package smoke check and the CPU-baseline leg
of the benchmark are the only users. The product path never imports this package, and this
package never imports the product.

The arithmetic lives in ``p1e_oracle.c`` (plain element loops, FP64, single-threaded); this
module marshals numpy arrays into it and adds the free-DOF bookkeeping:

* DOF n = d*i + j of node i, component j (Section 5, eq. bvvectors); free DOFs are the ones
  without a Dirichlet value, in ascending n (the vector hat v).
* J(v) = J_grad(v) - b.v with b = M f over all DOFs (reading of Sections 1 and 3.2: the
  linear part of the energy is minus the load work).
* Gradients are restricted to free DOFs (Remark 1) and include -b.

Parity status of every function is listed in the module's tests; none is unpinned.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "p1e_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PLAPLACE, NEOHOOKE, SVK, GL, PLAPLACE_ORTHO = 1, 2, 3, 4, 5
_KINDS = {"plaplace": PLAPLACE, "neohooke": NEOHOOKE, "svk": SVK, "gl": GL,
          "plaplace_ortho": PLAPLACE_ORTHO}


def build(force=True):
    """Compile the C oracle with gcc (-O2, no FMA contraction, single-threaded)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-std=c99",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("ncomp", ctypes.c_int32), ("kind", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("nn", ctypes.c_int64), ("ne", ctypes.c_int64),
                ("conn", ctypes.c_void_p), ("coords", ctypes.c_void_p),
                ("p", ctypes.c_double), ("C1", ctypes.c_double), ("D1", ctypes.c_double)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Problem)
        vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        lib.orc_geometry.argtypes = [P, vp, vp]
        lib.orc_geometry.restype = i64
        lib.orc_energy.argtypes = [P, vp, vp, vp, vp]
        lib.orc_energy.restype = i64
        lib.orc_densities.argtypes = [P, vp, vp, vp]
        lib.orc_densities.restype = None
        lib.orc_load_vector.argtypes = [P, vp, vp, vp]
        lib.orc_load_vector.restype = None
        lib.orc_dot.argtypes = [i64, vp, vp]
        lib.orc_dot.restype = dbl
        lib.orc_grad_exact.argtypes = [P, vp, vp, vp, vp]
        lib.orc_grad_exact.restype = i64
        lib.orc_patches.argtypes = [P, vp, vp]
        lib.orc_patches.restype = None
        lib.orc_grad_patch_fd.argtypes = [P, vp, vp, vp, vp, vp, dbl, i64, vp, vp, vp, vp]
        lib.orc_grad_patch_fd.restype = i64
        lib.orc_grad_patch_fd4.argtypes = [P, vp, vp, vp, vp, vp, dbl, i64, vp, vp, vp, vp]
        lib.orc_grad_patch_fd4.restype = i64
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def neohooke_constants(E, nu):
    """C1 = mu/2, D1 = K/2 with mu = E/(2(1+nu)), K = E/(3(1-2nu)) (Benchmark 2)."""
    mu = E / (2.0 * (1.0 + nu))
    K = E / (3.0 * (1.0 - 2.0 * nu))
    return mu / 2.0, K / 2.0


def svk_constants(E, nu):
    """St. Venant-Kirchhoff W = C1 |E|^2 + D1 (tr E)^2: C1 = mu, D1 = lambda/2 with the Lame
    constants mu = E/(2(1+nu)), lambda = E nu/((1+nu)(1-2nu))."""
    mu = E / (2.0 * (1.0 + nu))
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    return mu, lam / 2.0


class Oracle:
    """Oracle bound to one mesh/problem. ``prob`` needs the attributes of
    ``p1e_synth.Problem`` (dim, ncomp, kind, coords, conn, dirichlet, dirichlet_values,
    load, p, E, nu)."""

    def __init__(self, prob, C1=None, D1=None):
        self.lib = _load()
        self.dim = int(prob.dim)
        self.d = int(prob.ncomp)
        self.kind = prob.kind
        self.coords = np.ascontiguousarray(prob.coords, dtype=np.float64)
        self.conn = np.ascontiguousarray(prob.conn, dtype=np.int32)
        self.nn = self.coords.shape[0]
        self.ne = self.conn.shape[0]
        self.free = np.ascontiguousarray(prob.dirichlet.reshape(-1) == 0)
        self.free_dofs = np.flatnonzero(self.free).astype(np.int64)
        self.vD = np.ascontiguousarray(prob.dirichlet_values, dtype=np.float64).reshape(-1)
        if self.kind in ("neohooke", "svk"):
            c1, d1 = (neohooke_constants if self.kind == "neohooke" else svk_constants)(
                prob.E, prob.nu)
            self.C1 = c1 if C1 is None else C1
            self.D1 = d1 if D1 is None else D1
            self.p = 0.0
        elif self.kind == "gl":  # Ginzburg-Landau: the coefficients are the problem's own
            self.C1 = float(prob.C1) if C1 is None else C1
            self.D1 = float(prob.D1) if D1 is None else D1
            self.p = 0.0
        else:
            self.C1 = self.D1 = 0.0
            self.p = float(prob.p)
        self._P = _Problem(self.dim, self.d, _KINDS[self.kind], 0,
                           self.nn, self.ne, _ptr(self.conn).value, _ptr(self.coords).value,
                           self.p, self.C1, self.D1)
        k = self.dim + 1
        self.vol = np.zeros(self.ne)
        self.dphi = np.zeros((self.ne, k, self.dim))
        self.ndegen = self.lib.orc_geometry(ctypes.byref(self._P), _ptr(self.vol), _ptr(self.dphi))
        f = np.ascontiguousarray(prob.load, dtype=np.float64).reshape(-1)
        self.b = np.zeros(self.nn * self.d)
        self.lib.orc_load_vector(ctypes.byref(self._P), _ptr(self.vol), _ptr(f), _ptr(self.b))
        self._patch = None

    # --------------------------------------------------------------- DOF bookkeeping
    def expand(self, vhat):
        """Full nodal field [nn, d] from free-DOF values (Dirichlet values elsewhere)."""
        v = self.vD.copy()
        v[self.free] = np.asarray(vhat, dtype=np.float64)
        return v.reshape(self.nn, self.d)

    def _full(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        if v.size == self.free_dofs.size and v.size != self.nn * self.d:
            v = self.expand(v).reshape(-1)
        return v

    # --------------------------------------------------------------- energy
    def energy(self, v):
        """Returns dict(J, Jgrad, bv, nbad); v is full nodal or free-DOF."""
        v = self._full(v)
        jg = ctypes.c_double(0.0)
        nbad = self.lib.orc_energy(ctypes.byref(self._P), _ptr(v), _ptr(self.vol),
                                   _ptr(self.dphi), ctypes.byref(jg))
        bv = self.lib.orc_dot(v.size, _ptr(self.b), _ptr(v))
        J = jg.value - bv if nbad == 0 else np.inf
        return dict(J=J, Jgrad=jg.value, bv=bv, nbad=int(nbad))

    def densities(self, v):
        v = self._full(v)
        W = np.zeros(self.ne)
        self.lib.orc_densities(ctypes.byref(self._P), _ptr(v), _ptr(self.dphi), _ptr(W))
        return W

    # --------------------------------------------------------------- gradients
    def grad_exact_full(self, v):
        """dJ_grad/dv over all DOFs (no load term); returns (g_full, nbad)."""
        v = self._full(v)
        g = np.zeros(self.nn * self.d)
        nbad = self.lib.orc_grad_exact(ctypes.byref(self._P), _ptr(v), _ptr(self.vol),
                                       _ptr(self.dphi), _ptr(g))
        return g, int(nbad)

    def grad_exact(self, v):
        """dJ/dv on the free DOFs (ascending): exact J_grad gradient minus b."""
        g, _ = self.grad_exact_full(v)
        return (g - self.b)[self.free]

    def patches(self):
        if self._patch is None:
            ptr = np.zeros(self.nn + 1, dtype=np.int64)
            ent = np.zeros((self.dim + 1) * self.ne, dtype=np.int64)
            self.lib.orc_patches(ctypes.byref(self._P), _ptr(ptr), _ptr(ent))
            self._patch = (ptr, ent)
        return self._patch

    def grad_patch_fd(self, v, eps, sample=None, with_cond=False, order=2):
        """Patch central differences on free DOFs (or on free-DOF positions ``sample``),
        minus b; order 2 (+-eps) or 4 (+-eps, +-2 eps). With ``with_cond`` also returns the
        per-DOF rounding scales (order 2: cond = sum |T|(|W+|_abs + |W-|_abs),
        gabs = sum |T||W+ - W-|/(2 eps); order 4: see orc_grad_patch_fd4)."""
        v = self._full(v).copy()
        ptr, ent = self.patches()
        pos = np.arange(self.free_dofs.size) if sample is None else np.asarray(sample, np.int64)
        dofs = np.ascontiguousarray(self.free_dofs[pos])
        g = np.zeros(dofs.size)
        cond = np.zeros(dofs.size)
        gabs = np.zeros(dofs.size)
        fn = self.lib.orc_grad_patch_fd if order == 2 else self.lib.orc_grad_patch_fd4
        fn(ctypes.byref(self._P), _ptr(v), _ptr(self.vol), _ptr(self.dphi), _ptr(ptr),
           _ptr(ent), float(eps), dofs.size, _ptr(dofs), _ptr(g), _ptr(cond), _ptr(gabs))
        g = g - self.b[dofs]
        return (g, cond, gabs) if with_cond else g

    def grad_brute_fd(self, v, eps, order=2):
        """Central differences of the full energy J (all elements re-evaluated), order 2 or
        4: tiny meshes only."""
        v = self._full(v).copy()
        g = np.zeros(self.free_dofs.size)

        def J_at(n, v0, h):
            v[n] = v0 + h
            return self.energy(v)["J"]

        for q, n in enumerate(self.free_dofs):
            v0 = v[n]
            if order == 2:
                g[q] = (J_at(n, v0, eps) - J_at(n, v0, -eps)) / (2.0 * eps)
            else:
                d1 = J_at(n, v0, eps) - J_at(n, v0, -eps)
                d2 = J_at(n, v0, 2 * eps) - J_at(n, v0, -2 * eps)
                g[q] = (8.0 * d1 - d2) / (12.0 * eps)
            v[n] = v0
        return g
