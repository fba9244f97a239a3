"""Python binding of libtetmf (argument marshalling only).

Every step of the operator runs in the HIP kernels of ``libtetmf.so``; this
module converts torch tensors to device pointers and the current torch stream
to a HIP stream, and turns status codes into exceptions.  PyTorch provides
device memory and streams only.  There is no CPU fallback: if the shared
library is missing, every entry point raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtetmf.so")
_LIB = None

CG, DG = 0, 1
NEUMANN, DIRICHLET = 0, 1
F64, F32, BF16IN = 0, 1, 2
ORDER_LOCALITY, ORDER_AS_GIVEN = 0, 1

_PREC = {"f64": F64, "f32": F32, "bf16in": BF16IN}
_KIND = {"cg": CG, "dg": DG}
_BC = {"neumann": NEUMANN, "dirichlet": DIRICHLET}
_ORDER = {"locality": ORDER_LOCALITY, "as_given": ORDER_AS_GIVEN}


class TetmfError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tetmf status {status}: {msg}")
        self.status = status


class OpDesc(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32), ("degree", ctypes.c_int32), ("bc", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("ordering", ctypes.c_int32),
        ("n_q", ctypes.c_int32), ("q_points", ctypes.c_void_p), ("q_weights", ctypes.c_void_p),
        ("n_qf", ctypes.c_int32), ("qf_points", ctypes.c_void_p), ("qf_weights", ctypes.c_void_p),
        ("sigma", ctypes.c_double), ("eta", ctypes.c_double), ("device", ctypes.c_int32),
        ("q_jacobians", ctypes.c_void_p), ("n_components", ctypes.c_int32),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("n_dofs", ctypes.c_int64), ("n_free", ctypes.c_int64), ("n_cell", ctypes.c_int64),
        ("n_face", ctypes.c_int64), ("n_interior_face", ctypes.c_int64),
        ("n_q", ctypes.c_int32), ("n_qf", ctypes.c_int32), ("n_dof_cell", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("n_blocks", ctypes.c_int64), ("n_shared", ctypes.c_int64), ("n_partials", ctypes.c_int64),
        ("flops_per_apply", ctypes.c_double), ("bytes_per_apply", ctypes.c_double),
        ("device_bytes", ctypes.c_int64), ("n_components", ctypes.c_int32),
        ("flops_per_backward", ctypes.c_double), ("bytes_per_backward", ctypes.c_double),
        ("n_cell_data", ctypes.c_int64),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("max_inner", ctypes.c_int32), ("precond", ctypes.c_int32), ("method", ctypes.c_int32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("outer_its", ctypes.c_int32), ("inner_its", ctypes.c_int32),
                ("final_relres", ctypes.c_double), ("seconds", ctypes.c_double)]


# exported C symbols and their signatures
_SIGS = {
    "tetmf_mesh_create": (ctypes.c_int, [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_void_p)]),
    "tetmf_mesh_destroy": (None, [ctypes.c_void_p]),
    "tetmf_mesh_faces": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                        ctypes.POINTER(ctypes.c_int64)]),
    "tetmf_op_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(OpDesc), ctypes.POINTER(ctypes.c_void_p)]),
    "tetmf_op_destroy": (None, [ctypes.c_void_p]),
    "tetmf_op_info": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "tetmf_op_check": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(OpDesc), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64)]),
    "tetmf_op_numbering": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "tetmf_cell_data_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                              ctypes.c_void_p]),
    "tetmf_apply": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 5),
    "tetmf_apply_noalloc": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 5),
    "tetmf_apply_backward": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 8),
    "tetmf_diagonal": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 4),
    "tetmf_load_vector": (ctypes.c_int, [ctypes.c_void_p] + [ctypes.c_void_p] * 3),
    "tetmf_solve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(SolveOpts),
                                   ctypes.POINTER(SolveStats), ctypes.c_void_p]),
    "tetmf_chebyshev": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                       ctypes.c_void_p]),
    "tetmf_estimate_lambda_max": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                                 ctypes.POINTER(ctypes.c_double), ctypes.c_void_p]),
    "tetmf_op_profile": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "tetmf_op_profile_read": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                             ctypes.POINTER(ctypes.c_int64)]),
    "tetmf_op_profile_times": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                              ctypes.POINTER(ctypes.c_int64)]),
    "tetmf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "tetmf_last_error": (ctypes.c_char_p, []),
}


def lib():
    """Load libtetmf.so (built in-tree by ``_build.py``); raise if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run python paper_2509_10226_amd/_build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _check(status):
    if status < 0:
        L = lib()
        raise TetmfError(status, L.tetmf_last_error().decode())
    return status


def _torch():
    import torch
    return torch


def _stream(device=None):
    """The current torch stream of ``device`` (default: the current device)."""
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t, dtype=None, numel=None, name="tensor", device=None):
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if device is not None and t.device.index != device:
        raise ValueError(f"{name} is on {t.device}, the operator on cuda:{device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} entries, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Mesh:
    """Host-side tetrahedral mesh (vertex coordinates and cell vertex lists)."""

    def __init__(self, xyz, tets):
        L = lib()
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        self.tets = np.ascontiguousarray(tets, dtype=np.int32)
        if self.xyz.ndim != 2 or self.xyz.shape[1] != 3 or self.tets.ndim != 2 or self.tets.shape[1] != 4:
            raise ValueError("xyz must be [n_vert, 3] and tets [n_cell, 4]")
        h = ctypes.c_void_p()
        _check(L.tetmf_mesh_create(self.xyz.shape[0], self.xyz.ctypes.data, self.tets.shape[0],
                                   self.tets.ctypes.data, ctypes.byref(h)))
        self._h = h
        nf, ni = ctypes.c_int64(), ctypes.c_int64()
        _check(L.tetmf_mesh_faces(h, ctypes.byref(nf), ctypes.byref(ni)))
        self.n_face, self.n_interior_face = nf.value, ni.value

    @property
    def n_cell(self):
        return self.tets.shape[0]

    def __del__(self):
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.tetmf_mesh_destroy(self._h)
            self._h = None


def _make_desc(degree, qrule, kind, frule, precision, bc, sigma, eta, ordering, device, mesh=None,
               q_jacobians=None, n_components=1):
    qp, qw = (np.ascontiguousarray(a, dtype=np.float64) for a in qrule)
    d = OpDesc()
    d.kind = _KIND[kind]
    d.degree = int(degree)
    d.bc = _BC[bc]
    d.precision = _PREC[precision]
    d.ordering = _ORDER[ordering]
    d.n_q = qw.size
    d.q_points = qp.ctypes.data
    d.q_weights = qw.ctypes.data
    keep = [qp, qw]
    if frule is not None:
        fp, fw = (np.ascontiguousarray(a, dtype=np.float64) for a in frule)
        d.n_qf = fw.size
        d.qf_points = fp.ctypes.data
        d.qf_weights = fw.ctypes.data
        keep += [fp, fw]
    d.sigma = float(sigma)
    d.eta = float(eta)
    d.device = int(device)
    d.n_components = int(n_components)
    if q_jacobians is not None:
        jac = np.ascontiguousarray(q_jacobians, dtype=np.float64)
        if jac.shape != (mesh.tets.shape[0], qw.size, 3, 3):
            raise ValueError(f"q_jacobians must have shape [{mesh.tets.shape[0]}, {qw.size}, 3, 3]")
        d.q_jacobians = jac.ctypes.data
        keep.append(jac)
    return d, keep


def check_setup(mesh, degree, qrule, kind="cg", frule=None, precision="f64", bc="neumann", sigma=0.0, eta=1.0,
                ordering="locality", q_jacobians=None, n_components=1):
    """Host-only run of the operator set-up with its invariant checks (no GPU
    needed); returns (n_dofs, n_free) or raises TetmfError."""
    d, keep = _make_desc(degree, qrule, kind, frule, precision, bc, sigma, eta, ordering, 0, mesh, q_jacobians,
                         n_components)
    nd, nf = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().tetmf_op_check(mesh._h, ctypes.byref(d), ctypes.byref(nd), ctypes.byref(nf)))
    del keep
    return nd.value, nf.value


class Operator:
    """Matrix-free operator A(kappa) on a mesh (see include/tetmf.h)."""

    def __init__(self, mesh, degree, qrule, kind="cg", frule=None, precision="f64", bc="neumann",
                 sigma=0.0, eta=1.0, ordering="locality", device=0, q_jacobians=None, n_components=1):
        """q_jacobians: None (straight-sided cells) or [n_cell, n_q, 3, 3]
        Jacobians of curved cells at the rule points; n_components: 1, or 3
        for a vector field whose vectors hold the components one after
        another (tetmf_op_desc)."""
        L = lib()
        d, keep = _make_desc(degree, qrule, kind, frule, precision, bc, sigma, eta, ordering, device, mesh,
                             q_jacobians, n_components)
        h = ctypes.c_void_p()
        _check(L.tetmf_op_create(mesh._h, ctypes.byref(d), ctypes.byref(h)))
        del keep
        self._h = h
        self.kind, self.precision, self.degree = kind, precision, degree
        self.device = int(device)
        info = Info()
        _check(L.tetmf_op_info(h, ctypes.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in Info._fields_}
        self.n_dofs = self.info["n_dofs"]
        self.n_components = max(1, self.info["n_components"])
        self.n_vec = self.n_dofs * self.n_components  # length of the operator's vectors
        self.n_free = self.info["n_free"]
        self.n_cell = self.info["n_cell"]
        self.n_face = self.info["n_face"]
        self.n_q = self.info["n_q"]
        self.n_qf = self.info["n_qf"]
        # entries of per-point cell data in library layout (16-cell tiles)
        self.n_cell_data = self.info["n_cell_data"]

    def __del__(self):
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.tetmf_op_destroy(self._h)
            self._h = None

    @property
    def dtype(self):
        torch = _torch()
        return torch.float64 if self.precision == "f64" else torch.float32

    def numbering(self):
        """(cell_perm [n_cell], dof_xyz [n_dofs, 3], dof_cell [n_dofs]) host arrays."""
        cp = np.empty(self.n_cell, dtype=np.int32)
        xyz = np.empty((self.n_dofs, 3), dtype=np.float64)
        dc = np.empty(self.n_dofs, dtype=np.int32)
        _check(lib().tetmf_op_numbering(self._h, cp.ctypes.data, xyz.ctypes.data, dc.ctypes.data))
        return cp, xyz, dc

    def _p(self, t, dtype=None, numel=None, name="tensor"):
        """Device pointer of a tensor on the operator's device."""
        return _ptr(t, dtype, numel, name, self.device)

    def _device(self):
        torch = _torch()
        return torch.device("cuda", self.device)

    def cell_data_index(self, q, cell):
        """Index of point q of library cell ``cell`` in library-layout cell
        data: tiles of 16 cells, [ceil(n_cell / 16)][n_q][16]."""
        return ((cell >> 4) * self.n_q + q) * 16 + (cell & 15)

    def cell_data_to_library(self, data_user):
        """[n_cell, n_q] FP64 (user order) -> library layout (n_cell_data
        entries, op dtype, library cell order), on the GPU."""
        torch = _torch()
        src = data_user.to(device=self._device(), dtype=torch.float64).contiguous()
        if src.shape != (self.n_cell, self.n_q):
            raise ValueError(f"expected [{self.n_cell}, {self.n_q}]")
        dst = torch.empty(self.n_cell_data, dtype=self.dtype, device=self._device())
        _check(lib().tetmf_cell_data_layout(self._h, self._p(src), self._p(dst), 0, _stream(self.device)))
        return dst

    def cell_data_to_user(self, data_lib):
        torch = _torch()
        dst = torch.empty((self.n_cell, self.n_q), dtype=torch.float64, device=self._device())
        _check(lib().tetmf_cell_data_layout(self._h, self._p(data_lib, self.dtype, self.n_cell_data),
                                            self._p(dst), 1, _stream(self.device)))
        return dst

    def apply(self, u, kappa_cell=None, kappa_face=None, out=None):
        torch = _torch()
        if out is None:
            out = torch.empty(self.n_vec, dtype=self.dtype, device=self._device())
        _check(lib().tetmf_apply(self._h, self._p(u, self.dtype, self.n_vec, "u"),
                                 self._p(kappa_cell, self.dtype, self.n_cell_data, "kappa_cell"),
                                 self._p(kappa_face, self.dtype, self.n_qf * self.n_face, "kappa_face"),
                                 self._p(out, self.dtype, self.n_vec, "v"), _stream(self.device)))
        return out

    def apply_noalloc(self, u, out, kappa_cell=None, kappa_face=None):
        """v = A(kappa) u into the caller's ``out`` with the library's fixed
        scratch (tetmf_apply_noalloc): nothing is allocated."""
        _check(lib().tetmf_apply_noalloc(self._h, self._p(u, self.dtype, self.n_vec, "u"),
                                         self._p(kappa_cell, self.dtype, self.n_cell_data, "kappa_cell"),
                                         self._p(kappa_face, self.dtype, self.n_qf * self.n_face, "kappa_face"),
                                         self._p(out, self.dtype, self.n_vec, "v"), _stream(self.device)))
        return out

    def backward(self, u, g, kappa_cell=None, need_du=True, need_dkappa=True, kappa_face=None,
                 need_dkappa_face=False):
        """du = A g and dkappa_cell = d(g^T A u)/dkappa_cell (see
        tetmf_apply_backward).  Returns (du, dkappa_cell), or, for a DG
        operator with need_dkappa_face, (du, dkappa_cell, dkappa_face)."""
        torch = _torch()
        dev = self._device()
        du = torch.empty(self.n_vec, dtype=self.dtype, device=dev) if need_du else None
        dk = torch.empty(self.n_cell_data, dtype=self.dtype, device=dev) if need_dkappa else None
        dkf = torch.empty((self.n_qf, self.n_face), dtype=self.dtype, device=dev) if need_dkappa_face else None
        _check(lib().tetmf_apply_backward(self._h, self._p(u, self.dtype, self.n_vec, "u"),
                                          self._p(g, self.dtype, self.n_vec, "g"),
                                          self._p(kappa_cell, self.dtype, self.n_cell_data, "kappa_cell"),
                                          self._p(kappa_face, self.dtype, self.n_qf * self.n_face, "kappa_face"),
                                          self._p(du), self._p(dk), self._p(dkf), _stream(self.device)))
        return (du, dk, dkf) if need_dkappa_face else (du, dk)

    def diagonal(self, kappa_cell=None):
        torch = _torch()
        d = torch.empty(self.n_vec, dtype=self.dtype, device=self._device())
        _check(lib().tetmf_diagonal(self._h, self._p(kappa_cell, self.dtype, self.n_cell_data, "kappa_cell"),
                                    None, self._p(d), _stream(self.device)))
        return d

    def load_vector(self, f=None):
        torch = _torch()
        b = torch.empty(self.n_dofs, dtype=self.dtype, device=self._device())
        _check(lib().tetmf_load_vector(self._h, self._p(f, self.dtype, self.n_cell_data, "f"), self._p(b),
                                       _stream(self.device)))
        return b

    def solve(self, b, x0=None, kappa=None, inner=None, kappa_inner=None, rtol=1e-10, inner_rtol=1e-4,
              max_outer=50, max_inner=5000, precond="jacobi", method="refinement"):
        """Solve A x = b (see tetmf_solve; method "refinement" or "reliable"
        with an inner operator).  Returns (x, stats dict, converged)."""
        torch = _torch()
        x = torch.zeros(self.n_vec, dtype=torch.float64, device=self._device()) if x0 is None else x0.clone()
        if method not in ("refinement", "reliable"):
            raise ValueError(f"unknown solve method {method!r}")
        o = SolveOpts(rtol, inner_rtol, max_outer, max_inner, 1 if precond == "jacobi" else 0,
                      1 if method == "reliable" else 0)
        st = SolveStats()
        status = _check(lib().tetmf_solve(
            self._h, self._p(kappa, torch.float64, self.n_cell_data, "kappa"),
            inner._h if inner is not None else None,
            self._p(kappa_inner, inner.dtype if inner is not None else None, None, "kappa_inner"),
            self._p(b, torch.float64, self.n_vec, "b"), self._p(x, torch.float64, self.n_vec, "x"),
            ctypes.byref(o), ctypes.byref(st), _stream(self.device)))
        stats = {k: getattr(st, k) for k, _ in SolveStats._fields_}
        return x, stats, status == 0

    def chebyshev(self, b, inv_diag, degree, lambda_min, lambda_max, x=None, kappa=None):
        """Jacobi-preconditioned Chebyshev smoothing of A x = b (see
        tetmf_chebyshev); x None starts from zero.  Returns x (updated in place
        when given)."""
        torch = _torch()
        zero = x is None
        if zero:
            x = torch.empty(self.n_vec, dtype=self.dtype, device=self._device())
        _check(lib().tetmf_chebyshev(self._h, self._p(kappa, self.dtype, self.n_cell_data, "kappa"),
                                     self._p(inv_diag, self.dtype, self.n_vec, "inv_diag"),
                                     self._p(b, self.dtype, self.n_vec, "b"), self._p(x, self.dtype, self.n_vec, "x"),
                                     int(degree), float(lambda_min), float(lambda_max), 1 if zero else 0, _stream(self.device)))
        return x

    def estimate_lambda_max(self, inv_diag, n_iter=20, kappa=None):
        """Lanczos estimate of the largest eigenvalue of D^-1 A (see
        tetmf_estimate_lambda_max)."""
        lam = ctypes.c_double()
        _check(lib().tetmf_estimate_lambda_max(self._h, self._p(kappa, self.dtype, self.n_cell_data, "kappa"),
                                               self._p(inv_diag, self.dtype, self.n_vec, "inv_diag"), int(n_iter),
                                               ctypes.byref(lam), _stream(self.device)))
        return lam.value


def _profile_methods():
    def profile(self, enable=True):
        """Start (or stop) recording HIP events around the op's main kernel."""
        _check(lib().tetmf_op_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """(summed main-kernel milliseconds, launches) since profiling started."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().tetmf_op_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value
    def profile_times(self, capacity=4096):
        """Milliseconds of each recorded main-kernel launch (numpy array)."""
        ms = np.empty(capacity, dtype=np.float64)
        n = ctypes.c_int64()
        _check(lib().tetmf_op_profile_times(self._h, ms.ctypes.data, capacity, ctypes.byref(n)))
        return ms[:min(n.value, capacity)].copy()
    Operator.profile = profile
    Operator.profile_read = profile_read
    Operator.profile_times = profile_times


_profile_methods()


def _autograd():
    torch = _torch()

    class ApplyFunction(torch.autograd.Function):
        """v = A(kappa) u with hand-written backward kernels:
        dL/du = A^T dL/dv, dL/dkappa_cell = w_q |det J| grad u . grad (dL/dv)
        and, for DG, dL/dkappa_face from the face terms (tetmf_apply_backward)."""

        @staticmethod
        def forward(ctx, u, kappa, kappa_face, op):
            # the contiguous tensors the apply reads are the ones the backward
            # reads again
            u, kappa = u.contiguous(), kappa.contiguous()
            kappa_face = kappa_face.contiguous() if kappa_face is not None else None
            ctx.op = op
            ctx.has_face = kappa_face is not None
            ctx.save_for_backward(u, kappa, kappa_face)
            return op.apply(u, kappa, kappa_face)

        @staticmethod
        def backward(ctx, gv):
            u, kappa, kappa_face = ctx.saved_tensors
            need_face = ctx.has_face and ctx.needs_input_grad[2]
            out = ctx.op.backward(u, gv.contiguous(), kappa, need_du=ctx.needs_input_grad[0],
                                  need_dkappa=ctx.needs_input_grad[1], kappa_face=kappa_face,
                                  need_dkappa_face=need_face)
            return out[0], out[1], out[2] if need_face else None, None

    return ApplyFunction


_APPLY_FN = None


def apply_autograd(op, u, kappa, kappa_face=None):
    """Differentiable v = A(kappa) u (kappa in library layout, op.n_cell_data entries;
    kappa_face, DG only, [n_qf, n_face])."""
    global _APPLY_FN
    if _APPLY_FN is None:
        _APPLY_FN = _autograd()
    return _APPLY_FN.apply(u, kappa, kappa_face, op)
