"""Thin ctypes binding of libmfh.so (include/mfh.h).

Argument marshalling only: torch tensors supply device memory and the current
HIP stream; every step of the computation runs in the library's kernels.  The
binding refuses to run when the library is missing.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfh.so")

MFH_OK = 0
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "HIP", -3: "WORKSPACE", -4: "INVERTED",
          -5: "NOT_CONVERGED", -6: "BREAKDOWN", -7: "NOT_SPD"}
F64, F32 = 0, 1
QP_RECOMPUTE, QP_CACHE_F, QP_CACHE_T2, QP_CACHE_T4 = 0, 1, 2, 3
LAW_NEO_HOOKE, LAW_MOONEY_RIVLIN = 0, 1
SCATTER_AUTO, SCATTER_ATOMIC, SCATTER_COLOR, SCATTER_TILE, SCATTER_ELEMENT = -1, 0, 1, 2, 3
SCATTER_NAMES = {0: "atomic", 1: "color", 2: "tile", 3: "element"}
LEVEL_FIELD_NODAL, LEVEL_FIELD_VERTEX = 0, 1
COARSE_DIRECT, COARSE_CHEBYSHEV = 0, 1
BATCH_LAUNCH_AUTO, BATCH_LAUNCH_PER_DEGREE, BATCH_LAUNCH_FUSED = -1, 0, 1


class MfhError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"mfh {STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("n_cells", ctypes.c_int), ("degree", ctypes.c_int),
        ("n_levels", ctypes.c_int), ("n_materials", ctypes.c_int),
        ("mu", ctypes.POINTER(ctypes.c_double)), ("lambda_", ctypes.POINTER(ctypes.c_double)),
        ("n_inclusions", ctypes.c_int), ("inclusions", ctypes.POINTER(ctypes.c_double)),
        ("dirichlet_mask", ctypes.c_uint), ("qp_policy", ctypes.c_int), ("scatter", ctypes.c_int),
        ("vcycle_dtype", ctypes.c_int), ("cheb_degree", ctypes.c_int), ("n_smooth", ctypes.c_int),
        ("eig_iters", ctypes.c_int), ("cheb_lo", ctypes.c_double), ("cheb_hi", ctypes.c_double),
        ("level_field", ctypes.c_int), ("coarse_solver", ctypes.c_int), ("eig_refresh", ctypes.c_int),
        ("law", ctypes.c_int), ("mu2", ctypes.POINTER(ctypes.c_double)), ("tile_shape", ctypes.c_int),
        ("cell_block", ctypes.c_int),
    ]


class NewtonRecord(ctypes.Structure):
    _fields_ = [
        ("load_step", ctypes.c_int), ("newton_iter", ctypes.c_int), ("cg_iters", ctypes.c_int),
        ("residual_norm", ctypes.c_double), ("residual_after", ctypes.c_double),
        ("du_norm", ctypes.c_double), ("cg_relres", ctypes.c_double), ("min_J", ctypes.c_double),
        ("setup_ms", ctypes.c_double), ("residual_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
        ("coarse_negative", ctypes.c_int), ("load_fraction", ctypes.c_double), ("cutbacks", ctypes.c_int),
        ("step_length", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    """Loads libmfh.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1904_13131_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    sig = {
        "mfh_desc_defaults": (None, [ctypes.POINTER(Desc)]),
        "mfh_workspace_size": (st, [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_size_t)]),
        "mfh_create": (st, [ctypes.POINTER(Desc), _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)]),
        "mfh_destroy": (st, [_P]),
        "mfh_n_dofs": (st, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]),
        "mfh_set_deformation": (st, [_P, _P, _D]),
        "mfh_tangent_vmult": (st, [_P, ctypes.c_int, ctypes.c_int, _P, _P]),
        "mfh_residual": (st, [_P, _P, _P]),
        "mfh_gmg_vcycle": (st, [_P, _P, _P]),
        "mfh_cg_solve": (st, [_P, _P, _P, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _D]),
        "mfh_last_error": (ctypes.c_char_p, [_P]),
        "mfh_apply_dirichlet": (st, [_P, _P, _D, ctypes.c_double]),
        "mfh_newton_solve": (st, [_P, _P, _D, _D, ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.POINTER(NewtonRecord),
                                  ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "mfh_external_force": (st, [_P, _D, _P]),
        "mfh_level_displacement": (st, [_P, ctypes.c_int, _P]),
        "mfh_level_diagonal": (st, [_P, ctypes.c_int, _P]),
        "mfh_level_lambda_max": (st, [_P, ctypes.c_int, _D]),
        "mfh_set_level_eigenvalues": (st, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double]),
        "mfh_prolongate": (st, [_P, ctypes.c_int, ctypes.c_int, _P, _P]),
        "mfh_restrict": (st, [_P, ctypes.c_int, ctypes.c_int, _P, _P]),
        "mfh_chebyshev": (st, [_P, ctypes.c_int, _P, _P]),
        "mfh_coarse_inertia": (st, [_P, ctypes.POINTER(ctypes.c_int)]),
        "mfh_dense_inverse_workspace": (st, [ctypes.c_longlong, ctypes.POINTER(ctypes.c_size_t)]),
        "mfh_dense_inverse": (st, [_P, _P, ctypes.c_longlong, _P, ctypes.c_size_t, _P, ctypes.POINTER(ctypes.c_int)]),
        "mfh_dense_inverse_static": (st, [_P, _P, ctypes.c_longlong, _P, ctypes.POINTER(ctypes.c_int)]),
        "mfh_enable_graphs": (st, [_P, ctypes.c_int]),
        "mfh_batch_workspace_size": (st, [ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_size_t)]),
        "mfh_batch_create": (st, [ctypes.c_int, ctypes.POINTER(_P), _P, ctypes.c_size_t, _P,
                                  ctypes.POINTER(_P)]),
        "mfh_batch_destroy": (st, [_P]),
        "mfh_batch_last_error": (ctypes.c_char_p, [_P]),
        "mfh_batch_set_deformation": (st, [_P, ctypes.POINTER(_P), _D]),
        "mfh_batch_tangent_vmult": (st, [_P, ctypes.c_int, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
        "mfh_batch_set_launch": (st, [_P, ctypes.c_int]),
        "mfh_contraction_stage": (st, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P, _P]),
        "mfh_batch_cg_solve": (st, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P), ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), _D, _D]),
        "mfh_node_coords_1d": (st, [_P, ctypes.c_int, _D]),
        "mfh_scatter_mode": (st, [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "mfh_tile_shape": (st, [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]),
        "mfh_cell_block": (st, [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]),
        "mfh_timer_enable": (st, [_P, ctypes.c_int]),
        "mfh_timer_read": (st, [_P, _D, ctypes.POINTER(ctypes.c_longlong)]),
        "mfh_csr_size": (st, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)]),
        "mfh_csr_assemble": (st, [_P, ctypes.c_int, _P, _P, _P]),
        "mfh_csr_spmv": (st, [_P, ctypes.c_int, _P, _P, _P, _P, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(st, handle=None):
    if st != MFH_OK:
        msg = lib().mfh_last_error(handle)
        raise MfhError(st, msg.decode() if msg else "")


def _darr(vals):
    vals = [float(v) for v in vals]
    return (ctypes.c_double * max(1, len(vals)))(*vals)


def make_desc(dim, n_cells, degree, n_levels=1, mu=(1.0,), lam=(1.5,), inclusions=(), dirichlet_mask=0,
              qp_policy=QP_RECOMPUTE, scatter=SCATTER_AUTO, vcycle_dtype=F32, cheb_degree=4, n_smooth=2,
              eig_iters=30, cheb_lo=0.6, cheb_hi=1.2, level_field=0, coarse_solver=0, eig_refresh=1,
              law=LAW_NEO_HOOKE, mu2=None, tile_shape=-1, cell_block=-1):
    """Builds an mfh_desc; the returned tuple keeps the host arrays alive."""
    d = Desc()
    lib().mfh_desc_defaults(ctypes.byref(d))
    mu_a, lam_a = _darr(mu), _darr(lam)
    rows = []
    for c, r, m in inclusions:
        rows += list(c)[:dim] + [r, m]
    inc_a = _darr(rows)
    d.dim, d.n_cells, d.degree, d.n_levels = dim, n_cells, degree, n_levels
    d.n_materials = len(mu)
    d.mu = ctypes.cast(mu_a, _D)
    d.lambda_ = ctypes.cast(lam_a, _D)
    d.n_inclusions = len(inclusions)
    d.inclusions = ctypes.cast(inc_a, _D)
    d.dirichlet_mask = dirichlet_mask
    d.qp_policy, d.scatter, d.vcycle_dtype = qp_policy, scatter, vcycle_dtype
    d.cheb_degree, d.n_smooth, d.eig_iters = cheb_degree, n_smooth, eig_iters
    d.cheb_lo, d.cheb_hi = cheb_lo, cheb_hi
    d.level_field = level_field
    d.coarse_solver, d.eig_refresh = coarse_solver, eig_refresh
    d.law = law
    d.tile_shape = tile_shape
    d.cell_block = cell_block
    mu2_a = _darr(mu2 if mu2 is not None else [0.0] * len(mu))
    d.mu2 = ctypes.cast(mu2_a, _D)
    return d, (mu_a, lam_a, inc_a, mu2_a)


def workspace_size(desc):
    n = ctypes.c_size_t()
    _check(lib().mfh_workspace_size(ctypes.byref(desc), ctypes.byref(n)))
    return n.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


_DTYPES = {torch.float64: F64, torch.float32: F32}


def _arg(t, name, device, n, dtypes=(torch.float64,)):
    """Checks one vector argument before its pointer crosses the C ABI: a torch
    tensor on the problem's device, of an accepted dtype, contiguous, with
    exactly n entries.  Raises ValueError (never stripped, unlike assert)."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.device != device:
        raise ValueError(f"{name}: tensor on device {t.device}, the problem lives on device {device}")
    if t.dtype not in dtypes:
        raise ValueError(f"{name}: dtype {t.dtype}, expected one of {[str(d) for d in dtypes]}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor is not contiguous")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} entries, expected {n}")
    return t


class Problem:
    """One mfh_problem with its workspace (a torch uint8 device tensor)."""

    def __init__(self, dim, n_cells, degree, device="cuda", stream=None, **kw):
        self.desc, self._keep = make_desc(dim, n_cells, degree, **kw)
        self.device = torch.device(device)
        if self.device.type == "cuda" and self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.dim = dim
        size = workspace_size(self.desc)
        self.workspace = torch.empty(size + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        base = self.workspace.data_ptr() + off
        self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
        h = ctypes.c_void_p()
        _check(lib().mfh_create(ctypes.byref(self.desc), ctypes.c_void_p(base), size,
                                ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.handle = h
        self.n_levels = self.desc.n_levels

    def close(self):
        if getattr(self, "handle", None):
            lib().mfh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n_dofs(self, level=-1):
        level = level % self.n_levels
        n = ctypes.c_longlong()
        _check(lib().mfh_n_dofs(self.handle, level, ctypes.byref(n)), self.handle)
        return n.value

    def _vec(self, level, dtype):
        return torch.empty(self.n_dofs(level), dtype=dtype, device=self.device)

    def _out(self, t, name, level, dtype):
        if t is None:
            return self._vec(level, dtype)
        return _arg(t, name, self.device, self.n_dofs(level), (dtype,))

    def set_deformation(self, u):
        _arg(u, "u", self.device, self.n_dofs())
        mj = ctypes.c_double()
        _check(lib().mfh_set_deformation(self.handle, _ptr(u), ctypes.byref(mj)), self.handle)
        return mj.value

    def tangent_vmult(self, x, y=None, level=-1):
        level = level % self.n_levels
        _arg(x, "x", self.device, self.n_dofs(level), (torch.float64, torch.float32))
        dt = _DTYPES[x.dtype]
        y = self._out(y, "y", level, x.dtype)
        _check(lib().mfh_tangent_vmult(self.handle, level, dt, _ptr(x), _ptr(y)), self.handle)
        return y

    def residual(self, u, r=None):
        _arg(u, "u", self.device, self.n_dofs())
        r = self._out(r, "r", -1, torch.float64)
        _check(lib().mfh_residual(self.handle, _ptr(u), _ptr(r)), self.handle)
        return r

    def gmg_vcycle(self, r, z=None):
        _arg(r, "r", self.device, self.n_dofs())
        z = self._out(z, "z", -1, torch.float64)
        _check(lib().mfh_gmg_vcycle(self.handle, _ptr(r), _ptr(z)), self.handle)
        return z

    def cg_solve(self, b, x=None, rtol=1e-8, max_it=200, raise_on_error=True):
        _arg(b, "b", self.device, self.n_dofs())
        x = self._out(x, "x", -1, torch.float64)
        it = ctypes.c_int()
        rel = ctypes.c_double()
        st = lib().mfh_cg_solve(self.handle, _ptr(b), _ptr(x), rtol, max_it, ctypes.byref(it), ctypes.byref(rel))
        if raise_on_error:
            _check(st, self.handle)
        return x, it.value, rel.value, st

    def _faces(self, rows, name):
        rows = [list(r) for r in rows]
        if len(rows) != 2 * self.dim or any(len(r) != self.dim for r in rows):
            raise ValueError(f"{name}: expected {2 * self.dim} faces x {self.dim} components")
        return rows

    def apply_dirichlet(self, u, face_values, scale=1.0):
        _arg(u, "u", self.device, self.n_dofs())
        face_values = self._faces(face_values, "face_values")
        fv = _darr([v for row in face_values for v in row])
        _check(lib().mfh_apply_dirichlet(self.handle, _ptr(u), fv, scale), self.handle)

    def newton_solve(self, u, face_values, n_steps, cg_rtol=1e-8, cg_max_it=200, du_tol=1e-5, r_tol=1e-8,
                     max_newton=20, max_records=512, raise_on_error=True, face_traction=None, max_seconds=0.0):
        _arg(u, "u", self.device, self.n_dofs())
        face_values = self._faces(face_values, "face_values")
        if face_traction is not None:
            face_traction = self._faces(face_traction, "face_traction")
        fv = _darr([v for row in face_values for v in row])
        ft = _darr([v for row in face_traction for v in row]) if face_traction is not None else None
        recs = (NewtonRecord * max_records)()
        n = ctypes.c_int()
        st = lib().mfh_newton_solve(self.handle, _ptr(u), fv, ft, n_steps, cg_rtol, cg_max_it, du_tol, r_tol,
                                    max_newton, float(max_seconds), recs, max_records, ctypes.byref(n))
        out = [recs[i].as_dict() for i in range(min(n.value, max_records))]
        if raise_on_error:
            _check(st, self.handle)
        return out, st

    def external_force(self, face_traction, f=None):
        ft = _darr([v for row in self._faces(face_traction, "face_traction") for v in row])
        f = self._out(f, "f", -1, torch.float64)
        _check(lib().mfh_external_force(self.handle, ft, _ptr(f)), self.handle)
        return f

    def csr_size(self, level=-1):
        """(n_rows, nnz) of the CSR form of K_c on a level."""
        n, z = ctypes.c_longlong(), ctypes.c_longlong()
        _check(lib().mfh_csr_size(self.handle, level % self.n_levels, ctypes.byref(n), ctypes.byref(z)), self.handle)
        return n.value, z.value

    def csr_assemble(self, level=-1):
        """K_c of a level at the linearisation point as device CSR arrays
        (row_ptr int64, col int32, val float64)."""
        level = level % self.n_levels
        n, nnz = self.csr_size(level)
        rp = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(nnz, dtype=torch.int32, device=self.device)
        val = torch.empty(nnz, dtype=torch.float64, device=self.device)
        _check(lib().mfh_csr_assemble(self.handle, level, _ptr(rp), _ptr(col), _ptr(val)), self.handle)
        return rp, col, val

    def csr_spmv(self, csr, x, y=None, level=-1):
        """y = A x for the arrays of csr_assemble (FP64)."""
        level = level % self.n_levels
        rp, col, val = csr
        n, nnz = self.csr_size(level)
        _arg(rp, "row_ptr", self.device, n + 1, (torch.int64,))
        _arg(col, "col", self.device, nnz, (torch.int32,))
        _arg(val, "val", self.device, nnz)
        _arg(x, "x", self.device, self.n_dofs(level))
        y = self._out(y, "y", level, torch.float64)
        _check(lib().mfh_csr_spmv(self.handle, level, _ptr(rp), _ptr(col), _ptr(val), _ptr(x), _ptr(y)),
               self.handle)
        return y

    def scatter_mode(self, level=-1, dtype=F64):
        """Scatter mode the vmult uses on a level (resolved when the descriptor says AUTO)."""
        m = ctypes.c_int()
        _check(lib().mfh_scatter_mode(self.handle, level % self.n_levels, dtype, ctypes.byref(m)), self.handle)
        return m.value

    def tile_shape(self, level=-1, dtype=F64):
        """Tile shape of the TILE scatter on a level: (shape 0 or 1, (cells x, y, z))."""
        shape = ctypes.c_int()
        cells = (ctypes.c_int * 3)()
        _check(lib().mfh_tile_shape(self.handle, level % self.n_levels, dtype, ctypes.byref(shape), cells),
               self.handle)
        return shape.value, tuple(cells)

    def cell_block(self, level=-1, dtype=F64):
        """Cell-block variant of the tangent vmult's pencil kernels on a level: (variant, cells per workgroup)."""
        v, cells = ctypes.c_int(), ctypes.c_int()
        _check(lib().mfh_cell_block(self.handle, level % self.n_levels, dtype, ctypes.byref(v), ctypes.byref(cells)),
               self.handle)
        return v.value, cells.value

    def node_coords_1d(self, level=-1):
        """Support-point coordinates along one axis (numpy array of L values)."""
        import numpy as np
        level = level % self.n_levels
        L = self.desc.degree * (self.desc.n_cells >> (self.n_levels - 1 - level)) + 1
        x = (ctypes.c_double * L)()
        _check(lib().mfh_node_coords_1d(self.handle, level, x), self.handle)
        return np.array(x[:])

    def level_displacement(self, level):
        u = self._vec(level, torch.float64)
        _check(lib().mfh_level_displacement(self.handle, level % self.n_levels, _ptr(u)), self.handle)
        return u

    def level_diagonal(self, level):
        d = self._vec(level, torch.float64)
        _check(lib().mfh_level_diagonal(self.handle, level % self.n_levels, _ptr(d)), self.handle)
        return d

    def level_lambda_max(self, level):
        v = ctypes.c_double()
        _check(lib().mfh_level_lambda_max(self.handle, level % self.n_levels, ctypes.byref(v)), self.handle)
        return v.value

    def _transfer_level(self, level):
        if not 1 <= level < self.n_levels:
            raise ValueError(f"level {level}: transfers connect levels 1..{self.n_levels - 1} to the next coarser")
        return level

    def set_level_eigenvalues(self, level, lam_max, lam_min=0.0):
        """Fixes the eigenvalue estimates a level's smoother (or, on level 0, the
        Chebyshev coarse solver) is built from; lam_max = 0 clears the override."""
        _check(lib().mfh_set_level_eigenvalues(self.handle, level % self.n_levels, float(lam_min),
                                               float(lam_max)), self.handle)

    def prolongate(self, level, x, y=None):
        self._transfer_level(level)
        _arg(x, "x", self.device, self.n_dofs(level - 1), (torch.float64, torch.float32))
        dt = _DTYPES[x.dtype]
        y = self._out(y, "y", level, x.dtype)
        _check(lib().mfh_prolongate(self.handle, level, dt, _ptr(x), _ptr(y)), self.handle)
        return y

    def restrict(self, level, x, y=None):
        self._transfer_level(level)
        _arg(x, "x", self.device, self.n_dofs(level), (torch.float64, torch.float32))
        dt = _DTYPES[x.dtype]
        y = self._out(y, "y", level - 1, x.dtype)
        _check(lib().mfh_restrict(self.handle, level, dt, _ptr(x), _ptr(y)), self.handle)
        return y

    def enable_graphs(self, enable=True):
        _check(lib().mfh_enable_graphs(self.handle, 1 if enable else 0), self.handle)

    def coarse_inertia(self):
        n = ctypes.c_int()
        _check(lib().mfh_coarse_inertia(self.handle, ctypes.byref(n)), self.handle)
        return n.value

    def timer_enable(self, enable=True):
        _check(lib().mfh_timer_enable(self.handle, 1 if enable else 0), self.handle)

    def timer_read(self):
        ms = ctypes.c_double()
        n = ctypes.c_longlong()
        _check(lib().mfh_timer_read(self.handle, ctypes.byref(ms), ctypes.byref(n)), self.handle)
        return ms.value, n.value

    def chebyshev(self, level, f, x):
        level = level % self.n_levels
        dt = torch.float32 if self.desc.vcycle_dtype == F32 else torch.float64
        _arg(f, "f", self.device, self.n_dofs(level), (dt,))
        _arg(x, "x", self.device, self.n_dofs(level), (dt,))
        _check(lib().mfh_chebyshev(self.handle, level, _ptr(f), _ptr(x)), self.handle)
        return x


def dense_inverse(a, stream=None, static=False):
    """The coarse level's pivoted dense inverse on a symmetric FP64 device
    matrix: returns (A^-1, number of negative eigenvalues); `a` is left
    unchanged (the library works on a copy).  static=True calls the
    allocation-free entry point (n <= 2048, work arrays in the library's
    static device array)."""
    if not isinstance(a, torch.Tensor) or a.dim() != 2 or a.shape[0] != a.shape[1]:
        raise ValueError("a: expected a square 2-D torch tensor")
    n = a.shape[0]
    _arg(a.reshape(-1), "a", a.device, n * n)
    if a.device.type != "cuda":
        raise ValueError("a: expected a device tensor")
    work_a = a.clone()
    inv = torch.empty_like(a)
    stream = torch.cuda.current_stream(a.device) if stream is None else stream
    neg = ctypes.c_int()
    if static:
        with torch.cuda.device(a.device):
            _check(lib().mfh_dense_inverse_static(_ptr(work_a), _ptr(inv), n, ctypes.c_void_p(stream.cuda_stream),
                                                  ctypes.byref(neg)))
        return inv, neg.value
    size = ctypes.c_size_t()
    _check(lib().mfh_dense_inverse_workspace(n, ctypes.byref(size)))
    ws = torch.empty(size.value + 256, dtype=torch.uint8, device=a.device)
    base = ws.data_ptr() + (-ws.data_ptr()) % 256
    _check(lib().mfh_dense_inverse(_ptr(work_a), _ptr(inv), n, ctypes.c_void_p(base), size.value,
                                   ctypes.c_void_p(stream.cuda_stream), ctypes.byref(neg)))
    return inv, neg.value


def contraction_stage(degree, mfma, sweeps, blocks, out, stream=None):
    """The sum factorisation's contraction stage alone (autotuner measurement);
    out: float32 device tensor of blocks * (degree + 1) * 256 entries."""
    _arg(out, "out", out.device, blocks * (degree + 1) * 256, (torch.float32,))
    stream = torch.cuda.current_stream(out.device) if stream is None else stream
    _check(lib().mfh_contraction_stage(int(degree), int(mfma), int(sweeps), int(blocks), _ptr(out),
                                       ctypes.c_void_p(stream.cuda_stream)))
    return out


def _check_batch(st, handle):
    if st != MFH_OK:
        msg = lib().mfh_batch_last_error(handle)
        raise MfhError(st, msg.decode() if msg else "")


def _parr(tensors):
    return (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])


class Batch:
    """An mfh_batch over existing Problems (kept alive by the batch)."""

    def __init__(self, problems, stream=None):
        self.problems = list(problems)
        n = len(self.problems)
        handles = (ctypes.c_void_p * n)(*[p.handle.value for p in self.problems])
        self._handles = handles
        size = ctypes.c_size_t()
        _check_batch(lib().mfh_batch_workspace_size(n, handles, ctypes.byref(size)), None)
        dev = self.problems[0].device
        self.workspace = torch.empty(size.value + 256, dtype=torch.uint8, device=dev)
        base = self.workspace.data_ptr() + (-self.workspace.data_ptr()) % 256
        self.stream = torch.cuda.current_stream(dev) if stream is None else stream
        h = ctypes.c_void_p()
        _check_batch(lib().mfh_batch_create(n, handles, ctypes.c_void_p(base), size.value,
                                            ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), None)
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().mfh_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _vectors(self, ts, name, dtypes=(torch.float64,)):
        ts = list(ts)
        if len(ts) != len(self.problems):
            raise ValueError(f"{name}: {len(ts)} vectors for {len(self.problems)} problems")
        for i, (t, p) in enumerate(zip(ts, self.problems)):
            _arg(t, f"{name}[{i}]", p.device, p.n_dofs(), dtypes)
        if len({t.dtype for t in ts}) > 1:
            raise ValueError(f"{name}: mixed dtypes")
        return ts

    def set_deformation(self, us):
        us = self._vectors(us, "us")
        mj = (ctypes.c_double * len(us))()
        _check_batch(lib().mfh_batch_set_deformation(self.handle, _parr(us), mj), self.handle)
        return list(mj)

    def set_launch(self, mode):
        """Batched vmult launch form: BATCH_LAUNCH_AUTO (tuned), _PER_DEGREE or _FUSED."""
        _check_batch(lib().mfh_batch_set_launch(self.handle, int(mode)), self.handle)

    def tangent_vmult(self, xs, ys):
        xs = self._vectors(xs, "xs", (torch.float64, torch.float32))
        ys = self._vectors(ys, "ys", (xs[0].dtype,))
        dt = _DTYPES[xs[0].dtype]
        _check_batch(lib().mfh_batch_tangent_vmult(self.handle, dt, _parr(xs), _parr(ys)), self.handle)
        return ys

    def cg_solve(self, bs, xs, rtol=1e-8, max_it=200):
        bs, xs = self._vectors(bs, "bs"), self._vectors(xs, "xs")
        n = len(bs)
        it = (ctypes.c_int * n)()
        rel = (ctypes.c_double * n)()
        ms = (ctypes.c_double * n)()
        _check_batch(lib().mfh_batch_cg_solve(self.handle, _parr(bs), _parr(xs), rtol, max_it, it, rel, ms),
                     self.handle)
        return list(it), list(rel), list(ms)
