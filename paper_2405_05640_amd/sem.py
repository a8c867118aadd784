"""Python binding of libsem (ctypes): argument marshalling only.

Every computation runs in the HIP library; this module checks shapes, dtypes
and devices on the host (so no kernel is launched on a buffer that does not
match the mesh), passes raw device pointers and torch's current stream, and
turns status codes into exceptions.  There is no fallback: if libsem.so is
missing, loading fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsem.so")

SEM_OK, SEM_ERR_INVALID_ARG, SEM_ERR_OUT_OF_MEMORY, SEM_ERR_HIP, SEM_ERR_NOT_CONVERGED, \
    SEM_ERR_BREAKDOWN, SEM_ERR_UNSUPPORTED = range(7)
SEM_F64, SEM_F32, SEM_BF16, SEM_BF16_SPLIT = 0, 1, 2, 3
SEM_PREP_F32, SEM_PREP_BF16, SEM_PREP_HSMG = 1, 2, 4
FIELD_GLO_NUM, FIELD_MULT, FIELD_MASK, FIELD_G, FIELD_B, FIELD_XYZ, FIELD_GLL, FIELD_DERIV = range(8)
(FORM_JACOBI_PCG, FORM_DC_FP32, FORM_DC_BF16, FORM_FCG_LEARNED, FORM_FCG_INNER_FP32, FORM_FCG_INNER_BF16,
 FORM_RELIABLE_FP32, FORM_RELIABLE_BF16, FORM_PCG_1RED, FORM_GMRES_HSMG, FORM_PCG_BLOCK_JACOBI,
 FORM_PCG_HSMG, FORM_GMRES_LEARNED_MG, FORM_FCG_LEARNED_MG) = range(14)
PRECOND_HSMG, PRECOND_SCHWARZ, PRECOND_BLOCK_JACOBI, PRECOND_HSMG_SYM = 0, 1, 2, 3
SMOOTHER_PARAMS = 8208
NOALLOC_SCRATCH_BYTES = 32 << 20    # SEM_NOALLOC_SCRATCH_BYTES

EXPORTED_SYMBOLS = [
    "sem_mesh_create", "sem_mesh_destroy", "sem_mesh_query", "sem_mesh_export", "sem_ax",
    "sem_dssum", "sem_rhs", "sem_jacobi", "sem_dot", "sem_solve_workspace_bytes",
    "sem_pcg_solve", "sem_last_error", "sem_version", "sem_smoother_create", "sem_smoother_destroy",
    "sem_smoother_set_weights", "sem_smoother_get_weights", "sem_smoother_apply", "sem_smoother_loss_grad",
    "sem_smoother_train_step", "sem_pcg_snapshots", "sem_pcg_solve_batched", "sem_solve_workspace_bytes_batched",
    "sem_smoother_get_state", "sem_smoother_set_state", "sem_pcg_solve_noalloc", "sem_precond_workspace_bytes",
    "sem_precond_apply", "sem_smoother_mg_apply",
]


class SemError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libsem status %d: %s" % (status, msg))
        self.status = status


class MeshDesc(ctypes.Structure):
    _fields_ = [("nelx", ctypes.c_int32), ("nely", ctypes.c_int32), ("nelz", ctypes.c_int32),
                ("order", ctypes.c_int32), ("vertices", ctypes.POINTER(ctypes.c_double)),
                ("periodic", ctypes.c_uint8 * 3), ("dirichlet_faces", ctypes.c_uint8),
                ("prepare", ctypes.c_uint8)]


class MeshInfo(ctypes.Structure):
    _fields_ = [("nelem", ctypes.c_int64), ("n_local", ctypes.c_int64), ("n_global", ctypes.c_int64),
                ("n_shared_global", ctypes.c_int64), ("n_shared_local", ctypes.c_int64),
                ("n_masked_global", ctypes.c_int64), ("order", ctypes.c_int32),
                ("npts_elem", ctypes.c_int32), ("device_bytes", ctypes.c_size_t)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("h1", ctypes.c_double), ("h2", ctypes.c_double), ("rel_tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("form", ctypes.c_int32), ("max_outer", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("smoother", ctypes.c_void_p),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_len", ctypes.c_int32),
                ("inner_iters", ctypes.c_int32), ("restart", ctypes.c_int32)]


class SmootherDesc(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("stall_window", ctypes.c_int32),
                ("stall_rate", ctypes.c_double), ("mg_context", ctypes.c_int32)]


class SolveReport(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("outer_iterations", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("fallback_used", ctypes.c_int32), ("history_written", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("true_rel_res", ctypes.c_double),
                ("elapsed_ms", ctypes.c_double)]


_lib = None


def lib():
    """Load libsem.so (built by ``paper_2405_05640_amd.build``)."""
    global _lib
    if _lib is None:
        # torch ships its own HIP runtime with the same soname as the one
        # libsem links; importing torch first makes the dynamic loader bind
        # libsem to that single runtime instance (device memory and streams
        # then come from, and are used by, one runtime).
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsem.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2405_05640_amd.build); there is no fallback")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        sig = {
            "sem_mesh_create": [ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)],
            "sem_mesh_destroy": [vp],
            "sem_mesh_query": [vp, ctypes.POINTER(MeshInfo)],
            "sem_mesh_export": [vp, ctypes.c_int, vp, ctypes.c_size_t],
            "sem_ax": [vp, dbl, dbl, ctypes.c_int, vp, vp, vp],
            "sem_dssum": [vp, ctypes.c_int, vp, ctypes.c_int, vp],
            "sem_rhs": [vp, vp, vp, vp],
            "sem_jacobi": [vp, dbl, dbl, vp, vp],
            "sem_dot": [vp, vp, vp, vp, vp],
            "sem_solve_workspace_bytes": [vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(ctypes.c_size_t)],
            "sem_pcg_solve": [vp, ctypes.POINTER(SolveOpts), vp, vp, vp, ctypes.c_size_t,
                              ctypes.POINTER(SolveReport), vp],
            "sem_pcg_solve_noalloc": [vp, ctypes.POINTER(SolveOpts), vp, vp, ctypes.POINTER(SolveReport), vp],
            "sem_precond_workspace_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
            "sem_precond_apply": [vp, ctypes.c_int, dbl, dbl, vp, vp, vp, ctypes.c_size_t, vp],
            "sem_smoother_create": [vp, ctypes.POINTER(SmootherDesc), ctypes.POINTER(vp)],
            "sem_smoother_destroy": [vp],
            "sem_smoother_set_weights": [vp, vp, ctypes.c_size_t],
            "sem_smoother_get_weights": [vp, vp, ctypes.c_size_t],
            "sem_smoother_get_state": [vp, vp, vp, vp, ctypes.c_size_t, ctypes.POINTER(i32)],
            "sem_smoother_set_state": [vp, vp, vp, vp, ctypes.c_size_t, i32],
            "sem_smoother_apply": [vp, vp, dbl, dbl, ctypes.c_int, vp, vp, vp],
            "sem_smoother_mg_apply": [vp, vp, dbl, dbl, ctypes.c_int, vp, vp, vp, ctypes.c_size_t, vp],
            "sem_smoother_loss_grad": [vp, vp, dbl, dbl, vp, ctypes.POINTER(dbl), vp, vp],
            "sem_smoother_train_step": [vp, vp, dbl, dbl, vp, vp, vp],
            "sem_pcg_snapshots": [vp, ctypes.POINTER(SolveOpts), vp, vp, ctypes.c_int32, vp, vp, ctypes.c_size_t,
                                  ctypes.POINTER(SolveReport), vp],
            "sem_pcg_solve_batched": [vp, ctypes.POINTER(SolveOpts), ctypes.c_int32, vp, vp, vp, ctypes.c_size_t,
                                      ctypes.POINTER(SolveReport), vp],
            "sem_solve_workspace_bytes_batched": [vp, ctypes.POINTER(SolveOpts), ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_size_t)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.sem_last_error.restype = ctypes.c_char_p
        L.sem_last_error.argtypes = []
        L.sem_version.restype = ctypes.c_char_p
        L.sem_version.argtypes = []
        _check_single_hip_runtime()
        _lib = L
    return _lib


def _check_single_hip_runtime():
    """Fail loudly if two HIP runtimes ended up in this process."""
    try:
        maps = open("/proc/self/maps").read().split("\n")
    except OSError:
        return
    paths = {ln.split()[-1] for ln in maps if "libamdhip64" in ln and "/" in ln}
    real = {os.path.realpath(p) for p in paths}
    if len(real) > 1:
        raise RuntimeError("two HIP runtimes loaded in one process: %s" % sorted(real))


def _check(st):
    if st != SEM_OK:
        raise SemError(st, lib().sem_last_error().decode())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


_TORCH_DT = {}


def _want(t, dtype_name, numel, what):
    import torch
    dt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
          "u16": torch.int16}[dtype_name]
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % what)
    if not t.is_cuda:
        raise ValueError("%s must be on a HIP device" % what)
    if t.dtype != dt and not (dtype_name == "bf16" and t.dtype in (torch.int16, torch.uint16)):
        raise ValueError("%s must have dtype %s, got %s" % (what, dt, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.numel() != numel:
        raise ValueError("%s has %d elements, mesh needs %d" % (what, t.numel(), numel))
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class Report:
    status: int
    iterations: int
    outer_iterations: int
    restarts: int
    fallback_used: int
    rel_res: float
    true_rel_res: float
    elapsed_ms: float
    history: np.ndarray | None = None


class Mesh:
    """A device-resident spectral-element mesh (``sem_mesh``)."""

    def __init__(self, nelx, nely, nelz, order, vertices, periodic=(0, 0, 0), dirichlet=0x3F,
                 prepare=0):
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        if v.shape != (nelz + 1, nely + 1, nelx + 1, 3):
            raise ValueError("vertices must have shape (nelz+1, nely+1, nelx+1, 3)")
        self._vert = v
        d = MeshDesc(nelx, nely, nelz, order, v.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                     (ctypes.c_uint8 * 3)(*[1 if p else 0 for p in periodic]), dirichlet, prepare)
        h = ctypes.c_void_p()
        _check(lib().sem_mesh_create(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        info = MeshInfo()
        _check(lib().sem_mesh_query(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in MeshInfo._fields_}
        self.nelx, self.nely, self.nelz, self.order = nelx, nely, nelz, order
        self.E = info.nelem
        self.n_local = info.n_local
        self.n_global = info.n_global
        self.shape = (self.E, order + 1, order + 1, order + 1)

    @classmethod
    def from_spec(cls, spec, prepare=0):
        return cls(spec.nelx, spec.nely, spec.nelz, spec.order, spec.vertices, spec.periodic,
                   spec.dirichlet, prepare)

    def close(self):
        if getattr(self, "_h", None):
            lib().sem_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ export
    def export(self, field):
        n, nl = self.order + 1, self.n_local
        spec = {FIELD_GLO_NUM: (np.int64, (self.E, n, n, n)), FIELD_MULT: (np.int32, (self.E, n, n, n)),
                FIELD_MASK: (np.uint8, (self.E, n, n, n)), FIELD_G: (np.float64, (6, self.E, n, n, n)),
                FIELD_B: (np.float64, (self.E, n, n, n)), FIELD_XYZ: (np.float64, (3, self.E, n, n, n)),
                FIELD_GLL: (np.float64, (2, n)), FIELD_DERIV: (np.float64, (n, n))}[field]
        out = np.zeros(spec[1], dtype=spec[0])
        _check(lib().sem_mesh_export(self._h, field, out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    # ------------------------------------------------------------ ops
    def ax(self, u, w, h1=1.0, h2=0.0, dtype=SEM_F64):
        name = {SEM_F64: ("f64", "f64"), SEM_F32: ("f32", "f32"), SEM_BF16: ("bf16", "f32"),
                SEM_BF16_SPLIT: ("f32", "f32")}[dtype]
        pu = _want(u, name[0], self.n_local, "u")
        pw = _want(w, name[1], self.n_local, "w")
        _check(lib().sem_ax(self._h, float(h1), float(h2), dtype, pu, pw, _stream()))
        return w

    def dssum(self, u, mask=False, dtype=SEM_F64):
        pu = _want(u, "f64" if dtype == SEM_F64 else "f32", self.n_local, "u")
        _check(lib().sem_dssum(self._h, dtype, pu, 1 if mask else 0, _stream()))
        return u

    def rhs(self, f, b):
        _check(lib().sem_rhs(self._h, _want(f, "f64", self.n_local, "f"),
                             _want(b, "f64", self.n_local, "b"), _stream()))
        return b

    def jacobi(self, dinv, h1=1.0, h2=0.0):
        _check(lib().sem_jacobi(self._h, float(h1), float(h2), _want(dinv, "f64", self.n_local, "dinv"),
                                _stream()))
        return dinv

    def dot(self, u, v, out):
        _check(lib().sem_dot(self._h, _want(u, "f64", self.n_local, "u"), _want(v, "f64", self.n_local, "v"),
                             _want(out, "f64", 1, "out"), _stream()))
        return out

    def precond(self, r, z, kind=PRECOND_HSMG, h1=1.0, h2=0.0, workspace=None):
        """z = M r for a continuous, masked local r (sem_precond_apply)."""
        import torch
        n = ctypes.c_size_t()
        _check(lib().sem_precond_workspace_bytes(self._h, ctypes.byref(n)))
        if workspace is None:
            workspace = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        if workspace.numel() * workspace.element_size() < n.value:
            raise ValueError("workspace too small")
        _check(lib().sem_precond_apply(self._h, int(kind), float(h1), float(h2), _want(r, "f64", self.n_local, "r"),
                                       _want(z, "f64", self.n_local, "z"), ctypes.c_void_p(workspace.data_ptr()),
                                       workspace.numel() * workspace.element_size(), _stream()))
        return z

    def solve_opts(self, h1=1.0, h2=0.0, rel_tol=1e-10, max_iter=20000, check_every=16,
                   form=FORM_JACOBI_PCG, max_outer=30, inner_tol=1e-4, smoother=None, history=None,
                   inner_iters=8, restart=0):
        o = SolveOpts()
        o.h1, o.h2, o.rel_tol, o.max_iter, o.check_every = h1, h2, rel_tol, max_iter, check_every
        o.form, o.max_outer, o.inner_tol, o.inner_iters, o.restart = form, max_outer, inner_tol, inner_iters, restart
        o.smoother = smoother._h.value if smoother is not None else None
        if history is not None:
            o.history = history.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            o.history_len = len(history)
        return o

    def workspace_bytes(self, opts):
        n = ctypes.c_size_t()
        _check(lib().sem_solve_workspace_bytes(self._h, ctypes.byref(opts), ctypes.byref(n)))
        return n.value

    def workspace(self, opts):
        import torch
        nb = self.workspace_bytes(opts)
        return torch.empty(nb, dtype=torch.uint8, device="cuda")

    def pcg_solve(self, b, x, workspace=None, raise_on_error=True, history=False, **kw):
        import torch
        hist = np.zeros(kw.get("max_iter", 20000) + 1) if history else None
        opts = self.solve_opts(history=hist, **kw)
        if workspace is None:
            workspace = self.workspace(opts)
        need = self.workspace_bytes(opts)
        if not (isinstance(workspace, torch.Tensor) and workspace.is_cuda and workspace.is_contiguous()):
            raise ValueError("workspace must be a contiguous device tensor")
        if workspace.numel() * workspace.element_size() < need:
            raise ValueError("workspace too small")
        rep = SolveReport()
        st = lib().sem_pcg_solve(self._h, ctypes.byref(opts), _want(b, "f64", self.n_local, "b"),
                                 _want(x, "f64", self.n_local, "x"), ctypes.c_void_p(workspace.data_ptr()),
                                 workspace.numel() * workspace.element_size(), ctypes.byref(rep), _stream())
        r = Report(rep.status, rep.iterations, rep.outer_iterations, rep.restarts, rep.fallback_used,
                   rep.rel_res, rep.true_rel_res, rep.elapsed_ms,
                   hist[: rep.history_written].copy() if hist is not None else None)
        if st != SEM_OK and raise_on_error:
            raise SemError(st, lib().sem_last_error().decode())
        return r


    def pcg_solve_noalloc(self, b, x, raise_on_error=True, **kw):
        """sem_pcg_solve_noalloc: the solve with its workspace in the
        library's static device scratch (no allocation)."""
        opts = self.solve_opts(**kw)
        rep = SolveReport()
        st = lib().sem_pcg_solve_noalloc(self._h, ctypes.byref(opts), _want(b, "f64", self.n_local, "b"),
                                         _want(x, "f64", self.n_local, "x"), ctypes.byref(rep), _stream())
        r = Report(rep.status, rep.iterations, rep.outer_iterations, rep.restarts, rep.fallback_used,
                   rep.rel_res, rep.true_rel_res, rep.elapsed_ms, None)
        if st != SEM_OK and raise_on_error:
            raise SemError(st, lib().sem_last_error().decode())
        return r


class Smoother:
    """Learned per-element smoother (``sem_smoother``) bound to one N = 7 mesh."""

    def __init__(self, mesh, seed=0, lr=1e-3, stall_window=25, stall_rate=0.0, beta1=0.9, beta2=0.999, eps=1e-8,
                 mg_context=False):
        d = SmootherDesc(seed, lr, beta1, beta2, eps, stall_window, stall_rate, 1 if mg_context else 0)
        h = ctypes.c_void_p()
        _check(lib().sem_smoother_create(mesh._h, ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self.mesh = mesh

    def close(self):
        if getattr(self, "_h", None):
            lib().sem_smoother_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32).ravel()
        if w.size != SMOOTHER_PARAMS:
            raise ValueError("expected %d weights" % SMOOTHER_PARAMS)
        _check(lib().sem_smoother_set_weights(self._h, w.ctypes.data_as(ctypes.c_void_p), w.size))

    def get_weights(self):
        w = np.zeros(SMOOTHER_PARAMS, dtype=np.float32)
        _check(lib().sem_smoother_get_weights(self._h, w.ctypes.data_as(ctypes.c_void_p), w.size))
        return w

    def get_state(self):
        """(weights, adam_m, adam_v, step): the training checkpoint."""
        w, m, v = (np.zeros(SMOOTHER_PARAMS, dtype=np.float32) for _ in range(3))
        step = ctypes.c_int32()
        _check(lib().sem_smoother_get_state(self._h, w.ctypes.data_as(ctypes.c_void_p),
                                            m.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p),
                                            SMOOTHER_PARAMS, ctypes.byref(step)))
        return w, m, v, int(step.value)

    def set_state(self, w, m, v, step):
        arrs = [np.ascontiguousarray(a, dtype=np.float32).ravel() for a in (w, m, v)]
        if any(a.size != SMOOTHER_PARAMS for a in arrs):
            raise ValueError("expected %d values per array" % SMOOTHER_PARAMS)
        _check(lib().sem_smoother_set_state(self._h, *(a.ctypes.data_as(ctypes.c_void_p) for a in arrs),
                                            SMOOTHER_PARAMS, int(step)))

    def apply(self, r, z, h1=1.0, h2=0.0, fp32=False):
        m = self.mesh
        _check(lib().sem_smoother_apply(self._h, m._h, float(h1), float(h2), 1 if fp32 else 0,
                                        _want(r, "f64", m.n_local, "r"), _want(z, "f64", m.n_local, "z"), _stream()))
        return z

    def mg_apply(self, r, z, h1=1.0, h2=0.0, fp32=False, workspace=None):
        """z = the learned multigrid applied to r (sem_smoother_mg_apply)."""
        import torch
        m = self.mesh
        n = ctypes.c_size_t()
        _check(lib().sem_precond_workspace_bytes(m._h, ctypes.byref(n)))
        if workspace is None:
            workspace = torch.empty(n.value, dtype=torch.uint8, device="cuda")
        if workspace.numel() * workspace.element_size() < n.value:
            raise ValueError("workspace too small")
        _check(lib().sem_smoother_mg_apply(self._h, m._h, float(h1), float(h2), 1 if fp32 else 0,
                                           _want(r, "f64", m.n_local, "r"), _want(z, "f64", m.n_local, "z"),
                                           ctypes.c_void_p(workspace.data_ptr()),
                                           workspace.numel() * workspace.element_size(), _stream()))
        return z

    def loss_grad(self, e, h1=1.0, h2=0.0, mesh=None):
        m = self.mesh if mesh is None else mesh
        loss = ctypes.c_double()
        g = np.zeros(SMOOTHER_PARAMS, dtype=np.float32)
        _check(lib().sem_smoother_loss_grad(self._h, m._h, float(h1), float(h2), _want(e, "f64", m.n_local, "e"),
                                            ctypes.byref(loss), g.ctypes.data_as(ctypes.c_void_p), _stream()))
        return loss.value, g

    def train_step(self, e_global, loss_out=None, h1=1.0, h2=0.0, mesh=None):
        m = self.mesh if mesh is None else mesh
        _check(lib().sem_smoother_train_step(self._h, m._h, float(h1), float(h2),
                                             _want(e_global, "f32", m.n_global, "e_global"),
                                             _want(loss_out, "f64", 1, "loss_out") if loss_out is not None else None,
                                             _stream()))


def pcg_snapshots(mesh, b, iters, e_out, workspace=None, **kw):
    """Errors x* - x_k of Jacobi-PCG iterates (assembled, lexicographic) into e_out[len(iters), n_global]."""
    import torch
    it = np.ascontiguousarray(iters, dtype=np.int32)
    opts = mesh.solve_opts(**kw)
    if workspace is None:
        workspace = mesh.workspace(opts)
    need = mesh.workspace_bytes(opts)
    if workspace.numel() * workspace.element_size() < need:
        raise ValueError("workspace too small")
    if not (isinstance(e_out, torch.Tensor) and e_out.is_cuda and e_out.dtype == torch.float64 and
            e_out.is_contiguous() and e_out.numel() == len(it) * mesh.n_global):
        raise ValueError("e_out must be a contiguous device float64 tensor of len(iters) * n_global")
    rep = SolveReport()
    _check(lib().sem_pcg_snapshots(mesh._h, ctypes.byref(opts), _want(b, "f64", mesh.n_local, "b"),
                                   it.ctypes.data_as(ctypes.c_void_p), len(it), ctypes.c_void_p(e_out.data_ptr()),
                                   ctypes.c_void_p(workspace.data_ptr()),
                                   workspace.numel() * workspace.element_size(), ctypes.byref(rep), _stream()))
    return Report(rep.status, rep.iterations, rep.outer_iterations, rep.restarts, rep.fallback_used, rep.rel_res,
                  rep.true_rel_res, rep.elapsed_ms)


def pcg_solve_batched(mesh, b, x, workspace=None, raise_on_error=True, **kw):
    """Jacobi-PCG (form=FORM_JACOBI_PCG, the default) or block-Jacobi CG
    (form=FORM_PCG_BLOCK_JACOBI, a mesh prepared with SEM_PREP_HSMG) for
    nrhs = b.shape[0] fields sharing the operator (one pass over the
    geometric factors per iteration).  b, x: (nrhs, E, n, n, n)."""
    import torch
    nrhs = b.shape[0]
    if b.shape != x.shape or nrhs < 1 or nrhs > 4:
        raise ValueError("b and x must both be (nrhs, E, n, n, n) with 1 <= nrhs <= 4")
    opts = mesh.solve_opts(**kw)
    need = ctypes.c_size_t()
    _check(lib().sem_solve_workspace_bytes_batched(mesh._h, ctypes.byref(opts), nrhs, ctypes.byref(need)))
    if workspace is None:
        workspace = torch.empty(need.value, dtype=torch.uint8, device="cuda")
    if workspace.numel() * workspace.element_size() < need.value:
        raise ValueError("workspace too small")
    reps = (SolveReport * nrhs)()
    st = lib().sem_pcg_solve_batched(mesh._h, ctypes.byref(opts), nrhs, _want(b, "f64", nrhs * mesh.n_local, "b"),
                                     _want(x, "f64", nrhs * mesh.n_local, "x"), ctypes.c_void_p(workspace.data_ptr()),
                                     workspace.numel() * workspace.element_size(), reps, _stream())
    out = [Report(r.status, r.iterations, r.outer_iterations, r.restarts, r.fallback_used, r.rel_res,
                  r.true_rel_res, r.elapsed_ms) for r in reps]
    if st != SEM_OK and raise_on_error:
        raise SemError(st, lib().sem_last_error().decode())
    return out


def version():
    return lib().sem_version().decode()
