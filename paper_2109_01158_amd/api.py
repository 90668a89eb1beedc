"""Python binding of libp1e: argument marshalling only.

The functions ``mesh_create``, ``mesh_get_info``, ``workspace_bytes``, ``mesh_bind``,
``energy``, ``grad_exact`` and ``grad_patch_fd`` mirror the C entry points ``p1e_*`` one to
one. :class:`Mesh` bundles a handle with its torch-owned device buffer. Every step of the
computation runs in libp1e's HIP kernels; torch only provides device memory and streams.
"""

import ctypes
import time

import numpy as np
import torch

from . import _lib as L
from ._lib import (P1E_FD, P1E_FP64, P1E_GINZBURG_LANDAU, P1E_MIXED, P1E_NEOHOOKE, P1E_PLAPLACE,
                   P1E_PLAPLACE_ORTHO, P1E_SVK, check)

_KINDS = {"plaplace": P1E_PLAPLACE, "plaplace_ortho": P1E_PLAPLACE_ORTHO, "neohooke": P1E_NEOHOOKE,
          "svk": P1E_SVK, "gl": P1E_GINZBURG_LANDAU, P1E_PLAPLACE: P1E_PLAPLACE,
          P1E_PLAPLACE_ORTHO: P1E_PLAPLACE_ORTHO, P1E_NEOHOOKE: P1E_NEOHOOKE, P1E_SVK: P1E_SVK,
          P1E_GINZBURG_LANDAU: P1E_GINZBURG_LANDAU}
_SCALAR = (P1E_PLAPLACE, P1E_PLAPLACE_ORTHO, P1E_GINZBURG_LANDAU)

PREC = {"fp64": P1E_FP64, "mixed": P1E_MIXED, P1E_FP64: P1E_FP64, P1E_MIXED: P1E_MIXED}


def _ptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if (t is not None and t.numel() > 0) else None


def _check_buf(t, dtype, n, device, name):
    """Raise ValueError unless t is a contiguous tensor of dtype with n entries on device: the
    library reads and writes exactly that many entries through the raw pointer."""
    if (not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device
            or not t.is_contiguous() or t.numel() != n):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of {n} entries on {device}")


def _stream_ptr(stream, device):
    s = torch.cuda.current_stream(device) if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def material_constants(kind, E, nu):
    """p1e_material_constants: (C1, D1) of kind "neohooke" or "svk" from (E, nu)."""
    c1, d1 = ctypes.c_double(), ctypes.c_double()
    check(L.lib().p1e_material_constants(_KINDS[kind], float(E), float(nu), ctypes.byref(c1),
                                         ctypes.byref(d1)))
    return c1.value, d1.value


def neohooke_constants(E, nu):
    """Benchmark 2's C1 = mu/2, D1 = K/2 (computed by the library)."""
    return material_constants("neohooke", E, nu)


def svk_constants(E, nu):
    """St. Venant-Kirchhoff C1 = mu, D1 = lambda/2 (computed by the library)."""
    return material_constants("svk", E, nu)


# ------------------------------------------------------------------ 1:1 entry points
def mesh_create(dim, kind, conn, coords, dirichlet=None, dirichlet_values=None, load=None,
                p=2.0, C1=0.0, D1=0.0, flags=0):
    """p1e_mesh_create. kind: "plaplace" | "plaplace_ortho" | "neohooke" | "svk" | "gl". Arrays
    are host numpy;
    returns an opaque handle (int). flags: 0 or P1E_INPUT_ORDER | P1E_FULL_GEOMETRY."""
    k = _KINDS[kind]
    ncomp = 1 if k in _SCALAR else dim
    conn = np.ascontiguousarray(conn, dtype=np.int32)
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    dmask = None if dirichlet is None else np.ascontiguousarray(dirichlet, dtype=np.uint8)
    dval = None if dirichlet_values is None else np.ascontiguousarray(dirichlet_values,
                                                                     dtype=np.float64)
    f = None if load is None else np.ascontiguousarray(load, dtype=np.float64)
    desc = L.MeshDesc(dim, ncomp, k, int(flags), coords.shape[0] if coords.ndim else 0,
                      conn.shape[0] if conn.size else 0,
                      _ptr(conn) if conn.size else None, _ptr(coords), _ptr(dmask), _ptr(dval),
                      _ptr(f), float(p), float(C1), float(D1))
    h = ctypes.c_void_p()
    check(L.lib().p1e_mesh_create(ctypes.byref(desc), ctypes.byref(h)))
    return h.value


def mesh_destroy(handle):
    L.lib().p1e_mesh_destroy(ctypes.c_void_p(handle))


def mesh_get_info(handle):
    info = L.MeshInfo()
    check(L.lib().p1e_mesh_get_info(ctypes.c_void_p(handle), ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in L.MeshInfo._fields_}


def workspace_bytes(handle, mode_mask):
    return int(L.lib().p1e_workspace_bytes(ctypes.c_void_p(handle), int(mode_mask)))


def mesh_bind(handle, buf, nbytes, mode_mask, stream=None):
    """p1e_mesh_bind on a device buffer given as a torch uint8 tensor (or raw pointer)."""
    ptr = buf.data_ptr() if isinstance(buf, torch.Tensor) else int(buf)
    dev = buf.device if isinstance(buf, torch.Tensor) else None
    check(L.lib().p1e_mesh_bind(ctypes.c_void_p(handle), ctypes.c_void_p(ptr), int(nbytes),
                                int(mode_mask), _stream_ptr(stream, dev)))


def energy(handle, vhat, prec, out3, flag, stream=None):
    """p1e_energy on device tensors: vhat f64[n_free_dofs], out3 f64[3], flag i32[1]."""
    check(L.lib().p1e_energy(ctypes.c_void_p(handle), _dptr(vhat), PREC[prec], _dptr(out3),
                             _dptr(flag), _stream_ptr(stream, out3.device)))


def grad_exact(handle, vhat, prec, g, out3, flag, stream=None):
    """p1e_grad_exact on device tensors; out3 may be None."""
    check(L.lib().p1e_grad_exact(ctypes.c_void_p(handle), _dptr(vhat), PREC[prec], _dptr(g),
                                 _dptr(out3), _dptr(flag), _stream_ptr(stream, flag.device)))


def grad_exact_static(handle, vhat, prec, g, out3, flag, stream=None):
    """p1e_grad_exact_static: p1e_grad_exact with the library's static scratch (allocates
    nothing); out3 may be None."""
    check(L.lib().p1e_grad_exact_static(ctypes.c_void_p(handle), _dptr(vhat), PREC[prec],
                                        _dptr(g), _dptr(out3), _dptr(flag),
                                        _stream_ptr(stream, flag.device)))


def energy_forces(handle, vhat, prec, out3, flag, stream=None):
    """p1e_energy_forces: energy, and the exact gradient kept for grad_gather."""
    check(L.lib().p1e_energy_forces(ctypes.c_void_p(handle), _dptr(vhat), PREC[prec],
                                    _dptr(out3), _dptr(flag), _stream_ptr(stream, flag.device)))


def grad_gather(handle, prec, scale, g, stream=None):
    """p1e_grad_gather: g = scale * (kept gradient); scale is a device 0-d/1-element f64
    tensor or None."""
    check(L.lib().p1e_grad_gather(ctypes.c_void_p(handle), PREC[prec], _dptr(scale), _dptr(g),
                                  _stream_ptr(stream, g.device)))


def grad_patch_fd4(handle, vhat, eps, g, flag, stream=None):
    """p1e_grad_patch_fd4 (fourth-order scheme) on device tensors."""
    check(L.lib().p1e_grad_patch_fd4(ctypes.c_void_p(handle), _dptr(vhat), float(eps),
                                     _dptr(g), _dptr(flag), _stream_ptr(stream, flag.device)))


def grad_scale(handle, scale, g, stream=None):
    """p1e_grad_scale: g *= scale in place (a device 1-element f64 tensor); no write when the
    scale is 1."""
    check(L.lib().p1e_grad_scale(ctypes.c_void_p(handle), _dptr(scale), _dptr(g),
                                 _stream_ptr(stream, g.device)))


def grad_patch_fd(handle, vhat, eps, g, flag, stream=None):
    """p1e_grad_patch_fd on device tensors."""
    check(L.lib().p1e_grad_patch_fd(ctypes.c_void_p(handle), _dptr(vhat), float(eps), _dptr(g),
                                    _dptr(flag), _stream_ptr(stream, flag.device)))


# ------------------------------------------------------------------ kernel timing
def prof_enable(on=True):
    check(L.lib().p1e_prof_enable(1 if on else 0))


def prof_reset():
    check(L.lib().p1e_prof_reset())


def prof_collect():
    """{kernel name: (launches, total ms)} for the launches recorded while enabled."""
    cap = 64
    names = ctypes.create_string_buffer(8192)
    counts = (ctypes.c_int64 * cap)()
    ms = (ctypes.c_double * cap)()
    n = ctypes.c_int32(0)
    check(L.lib().p1e_prof_collect(names, 8192, counts, ms, cap, ctypes.byref(n)))
    keys = names.value.decode().split("\n")[: n.value]
    return {k: (counts[i], ms[i]) for i, k in enumerate(keys)}


# ------------------------------------------------------------------ convenience wrapper
class Mesh:
    """A mesh handle bound to a torch-owned device buffer.

    ``modes`` is a mask of P1E_FP64 | P1E_MIXED | P1E_FD: which precisions the buffer holds
    arrays for.
    """

    def __init__(self, dim, kind, conn, coords, dirichlet=None, dirichlet_values=None,
                 load=None, p=2.0, C1=0.0, D1=0.0, modes=P1E_FP64 | P1E_MIXED,
                 device="cuda", stream=None, flags=0):
        t0 = time.perf_counter()
        self.handle = mesh_create(dim, kind, conn, coords, dirichlet, dirichlet_values, load,
                                  p, C1, D1, flags)
        self.create_s = time.perf_counter() - t0  # host setup time (p1e_mesh_create)
        self.info = mesh_get_info(self.handle)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.modes = modes
        self.nbytes = workspace_bytes(self.handle, modes)
        align = int(self.info["alignment"])
        self._buf = torch.empty(self.nbytes + align, dtype=torch.uint8, device=self.device)
        off = (-self._buf.data_ptr()) % align
        self.buf = self._buf[off: off + self.nbytes]
        t0 = time.perf_counter()
        with torch.cuda.device(self.device):
            mesh_bind(self.handle, self.buf, self.nbytes, modes, stream)
        self.bind_s = time.perf_counter() - t0  # upload (p1e_mesh_bind synchronises)
        self.n_free_dofs = int(self.info["n_free_dofs"])
        # bumped by every call that rewrites the kept gradient (energy_forces, minimize); lets
        # a differentiation hook know whether the gradient of its forward pass is still there
        self.forces_gen = 0

    @classmethod
    def from_problem(cls, prob, modes=P1E_FP64 | P1E_MIXED, device="cuda", stream=None,
                     flags=0):
        """Build from an object with the fields of ``p1e_synth.Problem``."""
        if prob.kind in ("neohooke", "svk"):
            C1, D1 = (neohooke_constants if prob.kind == "neohooke" else svk_constants)(
                prob.E, prob.nu)
            p = 2.0
        elif prob.kind == "gl":  # Ginzburg-Landau: the problem's own coefficients
            C1, D1, p = prob.C1, prob.D1, 2.0
        else:
            C1 = D1 = 0.0
            p = prob.p
        return cls(prob.dim, prob.kind, prob.conn, prob.coords, prob.dirichlet,
                   prob.dirichlet_values, prob.load, p=p, C1=C1, D1=D1, modes=modes,
                   device=device, stream=stream, flags=flags)

    def close(self):
        if getattr(self, "handle", None):
            mesh_destroy(self.handle)
            self.handle = None
            self._buf = self.buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_vhat(self, vhat):
        _check_buf(vhat, torch.float64, self.n_free_dofs, self.device, "vhat")

    def _out(self, t, dtype, n, name):
        """A caller-supplied output buffer after the same checks as vhat, or a new one."""
        if t is None:
            return torch.empty(n, dtype=dtype, device=self.device)
        _check_buf(t, dtype, n, self.device, name)
        return t

    def energy(self, vhat, prec="mixed", stream=None):
        """Returns (out3 = [J, J_grad, b.v] f64 tensor, flag i32[1]) -- asynchronous."""
        self._check_vhat(vhat)
        out3 = torch.empty(3, dtype=torch.float64, device=self.device)
        flag = torch.empty(1, dtype=torch.int32, device=self.device)
        energy(self.handle, vhat, prec, out3, flag, stream)
        return out3, flag

    def grad_exact(self, vhat, prec="mixed", stream=None, g=None, out3=None, flag=None):
        """Returns (g, out3, flag): exact dJ/dvhat, the energy of the same call, bad count."""
        self._check_vhat(vhat)
        g = self._out(g, torch.float64, self.n_free_dofs, "g")
        out3 = self._out(out3, torch.float64, 3, "out3")
        flag = self._out(flag, torch.int32, 1, "flag")
        grad_exact(self.handle, vhat, prec, g, out3, flag, stream)
        return g, out3, flag

    def energy_forces(self, vhat, prec="mixed", stream=None, out3=None, flag=None):
        """Energy plus the exact gradient kept for grad_gather; returns (out3, flag,
        generation)."""
        self._check_vhat(vhat)
        out3 = self._out(out3, torch.float64, 3, "out3")
        flag = self._out(flag, torch.int32, 1, "flag")
        energy_forces(self.handle, vhat, prec, out3, flag, stream)
        self.forces_gen += 1
        return out3, flag, self.forces_gen

    def grad_gather(self, prec="mixed", scale=None, stream=None, g=None):
        """g = scale * (the gradient kept by the last energy_forces call)."""
        g = self._out(g, torch.float64, self.n_free_dofs, "g")
        if scale is not None:
            _check_buf(scale, torch.float64, 1, self.device, "scale")
        grad_gather(self.handle, prec, scale, g, stream)
        return g

    def grad_patch_fd4(self, vhat, eps, stream=None):
        """Returns (g, flag): fourth-order patch central-difference gradient (FP64)."""
        self._check_vhat(vhat)
        g = torch.empty(self.n_free_dofs, dtype=torch.float64, device=self.device)
        flag = torch.empty(1, dtype=torch.int32, device=self.device)
        grad_patch_fd4(self.handle, vhat, eps, g, flag, stream)
        return g, flag

    def grad_scale(self, g, scale, stream=None):
        """g *= scale in place (scale: device f64 tensor of one element); returns g."""
        _check_buf(g, torch.float64, self.n_free_dofs, self.device, "g")
        _check_buf(scale, torch.float64, 1, self.device, "scale")
        grad_scale(self.handle, scale, g, stream)
        return g

    def grad_patch_fd(self, vhat, eps, stream=None):
        """Returns (g, flag): patch central-difference gradient (FP64)."""
        self._check_vhat(vhat)
        g = torch.empty(self.n_free_dofs, dtype=torch.float64, device=self.device)
        flag = torch.empty(1, dtype=torch.int32, device=self.device)
        grad_patch_fd(self.handle, vhat, eps, g, flag, stream)
        return g, flag


# ------------------------------------------------------------------ minimization
def minimize_workspace_bytes(handle, history=5, max_iters=200, prec="fp64"):
    o = L.LbfgsOpts(int(history), int(max_iters), PREC[prec], 0)
    return int(L.lib().p1e_minimize_workspace_bytes(ctypes.c_void_p(handle), ctypes.byref(o)))


def minimize(handle, vhat, history, max_iters, prec, ws, stream=None):
    """p1e_minimize: vhat (device f64, in/out, n_free_dofs entries), ws a device uint8 tensor
    (256-byte aligned, at least minimize_workspace_bytes). Returns the report as a dict."""
    n = int(mesh_get_info(handle)["n_free_dofs"])
    if not isinstance(ws, torch.Tensor) or ws.device.type != "cuda":
        raise ValueError("ws must be a device tensor")
    _check_buf(vhat, torch.float64, n, ws.device, "vhat")
    if ws.dtype != torch.uint8 or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous uint8 tensor")
    o = L.LbfgsOpts(int(history), int(max_iters), PREC[prec], 0)
    rep = L.MinReport()
    check(L.lib().p1e_minimize(ctypes.c_void_p(handle), _dptr(vhat), ctypes.byref(o),
                               ctypes.c_void_p(ws.data_ptr()), int(ws.numel()), ctypes.byref(rep),
                               _stream_ptr(stream, ws.device)))
    return {name: getattr(rep, name) for name, _ in L.MinReport._fields_ if name != "reserved"}


def _aligned_buffer(nbytes, device, align=256):
    raw = torch.empty(nbytes + align, dtype=torch.uint8, device=device)
    off = (-raw.data_ptr()) % align
    return raw, raw[off: off + nbytes]


def mesh_minimize(mesh, vhat, history=5, max_iters=200, prec="fp64", stream=None):
    """Minimize in place from vhat on a bound Mesh (allocates the workspace with torch)."""
    mesh._check_vhat(vhat)
    nb = minimize_workspace_bytes(mesh.handle, history, max_iters, prec)
    raw, ws = _aligned_buffer(nb, mesh.device)
    rep = minimize(mesh.handle, vhat, history, max_iters, prec, ws, stream)
    mesh.forces_gen += 1
    del raw
    return rep


# ------------------------------------------------------------------ serving
def _desc_of(prob, flags=0):
    """A MeshDesc for a p1e_synth.Problem-like object; returns (desc, arrays kept alive)."""
    k = _KINDS[prob.kind]
    if k == P1E_GINZBURG_LANDAU:
        C1, D1, p = prob.C1, prob.D1, 2.0
    elif k not in (P1E_PLAPLACE, P1E_PLAPLACE_ORTHO):
        C1, D1 = (neohooke_constants if k == P1E_NEOHOOKE else svk_constants)(prob.E, prob.nu)
        p = 2.0
    else:
        C1 = D1 = 0.0
        p = prob.p
    conn = np.ascontiguousarray(prob.conn, dtype=np.int32)
    coords = np.ascontiguousarray(prob.coords, dtype=np.float64)
    dm = np.ascontiguousarray(prob.dirichlet, dtype=np.uint8)
    dv = np.ascontiguousarray(prob.dirichlet_values, dtype=np.float64)
    f = np.ascontiguousarray(prob.load, dtype=np.float64)
    desc = L.MeshDesc(prob.dim, prob.ncomp, k, int(flags), coords.shape[0], conn.shape[0],
                      _ptr(conn), _ptr(coords), _ptr(dm), _ptr(dv), _ptr(f), float(p), float(C1),
                      float(D1))
    return desc, (conn, coords, dm, dv, f)


class Server:
    """Continuous-batching minimization server on one GPU (p1e_server_*).

    The pool is a torch-owned device buffer; all work runs on a dedicated torch stream (default
    priority). Drive it from one thread: submit(), step() until idle, poll()."""

    def __init__(self, pool_bytes, max_slots=256, history=5, max_iters=200, prec="fp64",
                 use_graph=True, setup_threads=8, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self._raw, self.pool = _aligned_buffer(int(pool_bytes), self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        o = L.ServerOpts(int(max_slots), int(history), int(max_iters), PREC[prec],
                         1 if use_graph else 0, int(setup_threads), int(pool_bytes),
                         ctypes.c_void_p(self.pool.data_ptr()),
                         ctypes.c_void_p(self.stream.cuda_stream))
        h = ctypes.c_void_p()
        torch.cuda.synchronize(self.device)
        with torch.cuda.device(self.device):
            check(L.lib().p1e_server_create(ctypes.byref(o), ctypes.byref(h)))
        self.handle = h.value

    def close(self):
        if getattr(self, "handle", None):
            with torch.cuda.device(self.device):
                L.lib().p1e_server_destroy(ctypes.c_void_p(self.handle))
            self.handle = None
            torch.cuda.synchronize(self.device)
            self._raw = self.pool = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def clock(self):
        return float(L.lib().p1e_server_clock(ctypes.c_void_p(self.handle)))

    def submit(self, prob, vhat0=None, flags=0):
        desc, keep = _desc_of(prob, flags)
        rid = ctypes.c_int64()
        v0 = None if vhat0 is None else np.ascontiguousarray(vhat0, dtype=np.float64)
        check(L.lib().p1e_server_submit(ctypes.c_void_p(self.handle), ctypes.byref(desc),
                                        _ptr(v0), 0 if v0 is None else v0.size,
                                        ctypes.byref(rid)))
        del keep
        return rid.value

    def submit_at(self, prob, t_arrival, vhat0=None, flags=0):
        """Submit a request that arrives at t_arrival (server clock seconds)."""
        desc, keep = _desc_of(prob, flags)
        rid = ctypes.c_int64()
        v0 = None if vhat0 is None else np.ascontiguousarray(vhat0, dtype=np.float64)
        check(L.lib().p1e_server_submit_at(ctypes.c_void_p(self.handle), ctypes.byref(desc),
                                           _ptr(v0), 0 if v0 is None else v0.size,
                                           float(t_arrival), ctypes.byref(rid)))
        del keep
        return rid.value

    def run(self, max_steps=0, max_seconds=0.0):
        """Step until idle (or a limit); returns (active, waiting)."""
        a, w = ctypes.c_int32(), ctypes.c_int32()
        with torch.cuda.device(self.device):
            check(L.lib().p1e_server_run(ctypes.c_void_p(self.handle), int(max_steps),
                                         float(max_seconds), ctypes.byref(a), ctypes.byref(w)))
        return a.value, w.value

    def step(self):
        a, w = ctypes.c_int32(), ctypes.c_int32()
        with torch.cuda.device(self.device):
            check(L.lib().p1e_server_step(ctypes.c_void_p(self.handle), ctypes.byref(a),
                                          ctypes.byref(w)))
        return a.value, w.value

    def poll(self, cap=1024):
        buf = (L.RequestInfo * cap)()
        n = ctypes.c_int32()
        check(L.lib().p1e_server_poll(ctypes.c_void_p(self.handle), buf, cap, ctypes.byref(n)))
        return [{name: getattr(buf[i], name) for name, _ in L.RequestInfo._fields_}
                for i in range(n.value)]

    def result_vhat(self, rid, n):
        out = np.zeros(int(n))
        check(L.lib().p1e_server_result_vhat(ctypes.c_void_p(self.handle), int(rid),
                                             _ptr(out), int(n)))
        return out

    def release(self, rid):
        check(L.lib().p1e_server_release(ctypes.c_void_p(self.handle), int(rid)))
