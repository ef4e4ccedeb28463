"""Python binding of libmgr355 (ctypes): argument marshalling only.

Every step of setup, preconditioner application and FGMRES runs in the HIP library; this
module passes device pointers of torch tensors and the current HIP stream across the C ABI
declared in include/mgr355.h.  It fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmgr355.so")

MGR_OK, MGR_ERR_ARG, MGR_ERR_ALLOC, MGR_ERR_HIP, MGR_ERR_ZERO_PIVOT = 0, 1, 2, 3, 4
MGR_ERR_NOT_CONVERGED, MGR_ERR_PATTERN, MGR_ERR_UNSUPPORTED = 5, 6, 7
STATUS_NAMES = {0: "OK", 1: "ARG", 2: "ALLOC", 3: "HIP", 4: "ZERO_PIVOT", 5: "NOT_CONVERGED",
                6: "PATTERN", 7: "UNSUPPORTED"}

INTERP = {"jacobi": 0, "zero": 1}
FRELAX = {"jacobi": 0, "amg": 1, "dense": 2}
GSMOOTH = {"none": 0, "block_jacobi": 1, "block_gs": 2, "ilu": 3}
COARSE = {"amg": 0, "dense": 1}
PREC = {"fp64": 0, "fp32": 1}
COUPLING = {"full": 0, "quasi_impes": 1}

X_LEVEL_A, X_F, X_C, X_WP, X_ACOR, X_G, X_COARSE, X_AMG_A, X_AMG_P, X_AMG_AGG, X_AMG_NLEV = range(11)
X_GS_COLOR = 11
X_ILU = 12
X_WR = 13
MAX_LEVELS = 8


class MgrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class mgr_csr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("val", C.c_void_p), ("block", C.c_int32),
                ("reserved", C.c_int32)]


class mgr_amg_opts(C.Structure):
    _fields_ = [("theta0", C.c_double), ("max_levels", C.c_int32), ("coarse_size", C.c_int32)]


class mgr_level_opts(C.Structure):
    _fields_ = [("f_label_mask", C.c_uint32), ("interp", C.c_int32), ("nmax_drop", C.c_int32),
                ("frelax", C.c_int32), ("frelax_sweeps", C.c_int32), ("frelax_omega", C.c_double),
                ("frelax_block", C.c_int32), ("global_smoother", C.c_int32),
                ("global_sweeps", C.c_int32), ("coupling", C.c_int32),
                ("global_omega", C.c_double), ("drop_tol", C.c_double),
                ("ilu_level", C.c_int32), ("ilu_sweeps", C.c_int32),
                ("ilu_tri_sweeps", C.c_int32), ("restrict_", C.c_int32),
                ("dff_block", C.c_int32), ("reserved1", C.c_int32)]


class mgr_opts(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("level", mgr_level_opts * MAX_LEVELS),
                ("coarse", C.c_int32), ("amg_frelax", mgr_amg_opts), ("amg_coarse", mgr_amg_opts),
                ("precision", C.c_int32), ("use_graph", C.c_int32), ("keep_setup", C.c_int32)]


class fgmres_opts(C.Structure):
    _fields_ = [("restart", C.c_int32), ("maxit", C.c_int32), ("rtol", C.c_double)]


class fgmres_result(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("true_relres", C.c_double), ("est_relres", C.c_double),
                ("history", C.POINTER(C.c_double)), ("history_cap", C.c_int32),
                ("history_len", C.c_int32)]


class mgr_server_config(C.Structure):
    _fields_ = [("budget_bytes", C.c_size_t), ("slots", C.c_int32), ("opts", mgr_opts),
                ("fopts", fgmres_opts), ("cache_setups", C.c_int32), ("batch_rows", C.c_int32),
                ("batch_max", C.c_int32)]


class mgr_request(C.Structure):
    _fields_ = [("A", C.POINTER(mgr_csr)), ("nnz", C.c_int64), ("labels", C.c_void_p),
                ("b", C.c_void_p), ("x", C.c_void_p), ("key", C.c_uint64),
                ("refresh_setup", C.c_int32), ("last_use", C.c_int32)]


class mgr_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("setup_reused", C.c_int32),
                ("slot", C.c_int32), ("true_relres", C.c_double), ("t_submit_ms", C.c_double),
                ("t_admit_ms", C.c_double), ("t_start_ms", C.c_double), ("t_end_ms", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double), ("footprint", C.c_size_t),
                ("batch", C.c_int32)]


class mgr_server_stats_t(C.Structure):
    _fields_ = [("completed", C.c_int64), ("queued", C.c_int64), ("cache_hits", C.c_int64),
                ("cache_misses", C.c_int64), ("evictions", C.c_int64),
                ("cached_setups", C.c_int64), ("reserved_bytes", C.c_size_t),
                ("peak_reserved_bytes", C.c_size_t)]


class mgr_poro_params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("reserved", C.c_int32),
                ("nu", C.c_double), ("phi0", C.c_double), ("biot", C.c_double),
                ("grav", C.c_double), ("p_ref", C.c_double), ("rho_solid", C.c_double),
                ("rho0", C.c_double * 2), ("comp", C.c_double * 2), ("visc", C.c_double * 2),
                ("dt", C.c_double)]


NEWTON_MAX_RECORD = 32


class mgr_newton_opts(C.Structure):
    _fields_ = [("max_newton", C.c_int32), ("max_backtracks", C.c_int32),
                ("tol_flow", C.c_double), ("tol_mech", C.c_double), ("max_ds", C.c_double),
                ("armijo", C.c_double)]


class mgr_newton_stats(C.Structure):
    _fields_ = [("newton_iters", C.c_int32), ("linear_iters", C.c_int32),
                ("backtracks", C.c_int32), ("converged", C.c_int32), ("setups", C.c_int32),
                ("linear_failures", C.c_int32), ("lin_iters", C.c_int32 * NEWTON_MAX_RECORD),
                ("merit", C.c_double * (NEWTON_MAX_RECORD + 1)),
                ("lambda_", C.c_double * NEWTON_MAX_RECORD), ("assemble_ms", C.c_double),
                ("setup_ms", C.c_double), ("solve_ms", C.c_double)]


_lib = None


def lib():
    """Load libmgr355.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1904_05960_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, st = C.c_void_p, C.c_int
    sig = {
        "mgr_default_opts": (None, [C.POINTER(mgr_opts)]),
        "mgr_setup": (st, [C.POINTER(mgr_csr), vp, C.POINTER(mgr_opts), vp, C.POINTER(vp)]),
        "mgr_setup_numeric": (st, [vp, C.POINTER(mgr_csr), vp]),
        "mgr_apply": (st, [vp, vp, vp, vp]),
        "fgmres_workspace_bytes": (C.c_size_t, [C.c_int64, C.c_int32]),
        "fgmres_solve": (st, [C.POINTER(mgr_csr), vp, vp, vp, C.POINTER(fgmres_opts), vp,
                              C.c_size_t, C.POINTER(fgmres_result), vp]),
        "fgmres_noalloc_max_bytes": (C.c_size_t, []),
        "fgmres_solve_noalloc": (st, [C.POINTER(mgr_csr), vp, vp, vp, C.POINTER(fgmres_opts),
                                      C.POINTER(fgmres_result), vp]),
        "mgr_batch_solve": (st, [C.c_int32, C.POINTER(mgr_csr), C.POINTER(vp), C.POINTER(vp),
                                 C.POINTER(vp), C.POINTER(mgr_opts), C.POINTER(fgmres_opts),
                                 C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                 C.POINTER(fgmres_result), vp]),
        "mgr_destroy": (None, [vp]),
        "mgr_footprint": (st, [vp, C.POINTER(C.c_size_t)]),
        "mgr_estimate_footprint": (st, [C.c_int64, C.c_int64, C.POINTER(mgr_opts),
                                        C.POINTER(C.c_size_t)]),
        "mgr_set_allocator": (None, [vp, vp, vp]),
        "mgr_last_error": (C.c_char_p, []),
        "mgr_query": (st, [vp, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int64)]),
        "mgr_export": (st, [vp, C.c_int32, C.c_int32, C.c_int32, vp, vp, vp, vp]),
        "mgr_spmv": (st, [C.POINTER(mgr_csr), vp, vp, vp]),
        "mgr_stream_copy": (st, [vp, vp, C.c_int64, vp]),
        "mgr_profile_enable": (st, [C.c_int32, C.c_int32]),
        "mgr_profile_read": (st, [C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]),
        "mgr_spgemm": (st, [C.POINTER(mgr_csr), C.POINTER(mgr_csr), C.POINTER(vp),
                            C.POINTER(C.c_int64), vp]),
        "mgr_spgemm_b3": (st, [C.POINTER(mgr_csr), C.POINTER(mgr_csr), C.c_int32, C.POINTER(vp),
                               C.POINTER(C.c_int64), vp]),
        "mgr_transpose": (st, [C.POINTER(mgr_csr), C.POINTER(vp), C.POINTER(C.c_int64), vp]),
        "mgr_merge_drop": (st, [C.POINTER(mgr_csr), C.POINTER(mgr_csr), vp, C.c_int32, vp,
                                C.POINTER(vp), C.POINTER(C.c_int64), vp]),
        "mgr_dense_inverse": (st, [vp, vp, C.c_int32, vp]),
        "mgr_spgemm_grouped": (st, [C.POINTER(mgr_csr), C.POINTER(mgr_csr), C.c_int32,
                                    C.POINTER(vp), C.POINTER(C.c_int64), vp]),
        "mgr_csr_to_bsr": (st, [C.POINTER(mgr_csr), C.c_int32, C.c_int32, vp, vp, vp,
                                C.c_int64, C.POINTER(C.c_int64), vp]),
        "mgr_ilu": (st, [C.POINTER(mgr_csr), C.c_int32, C.c_int32, C.POINTER(vp),
                         C.POINTER(C.c_int64), vp]),
        "mgr_aggregate": (st, [C.POINTER(mgr_csr), C.c_int32, C.c_double, C.c_int32, vp,
                               C.POINTER(C.c_int64), vp]),
        "mgr_owned_export": (st, [vp, vp, vp, vp, vp]),
        "mgr_owned_free": (None, [vp]),
        "mgr_release_cache": (st, []),
        "mgr_cached_bytes": (C.c_size_t, []),
        "mgr_alloc_stats": (None, [C.POINTER(C.c_size_t), C.POINTER(C.c_size_t), C.c_int32]),
        "mgr_server_default_config": (None, [C.POINTER(mgr_server_config)]),
        "mgr_server_create": (st, [C.POINTER(mgr_server_config), C.POINTER(vp)]),
        "mgr_server_submit": (st, [vp, C.POINTER(mgr_request), C.POINTER(C.c_uint64)]),
        "mgr_server_wait": (st, [vp, C.c_uint64, C.POINTER(mgr_result)]),
        "mgr_server_poll": (C.c_int32, [vp, C.c_uint64]),
        "mgr_server_stats": (st, [vp, C.POINTER(mgr_server_stats_t)]),
        "mgr_server_destroy": (None, [vp]),
        "mgr_poro_default_params": (None, [C.POINTER(mgr_poro_params), C.c_int32, C.c_int32,
                                           C.c_int32]),
        "mgr_newton_default_opts": (None, [C.POINTER(mgr_newton_opts)]),
        "mgr_poro_create": (st, [C.POINTER(mgr_poro_params), vp, vp, vp, vp, vp, vp, vp, vp,
                                 C.POINTER(vp)]),
        "mgr_poro_set_dt": (st, [vp, C.c_double]),
        "mgr_poro_matrix": (st, [vp, C.POINTER(mgr_csr), C.POINTER(vp)]),
        "mgr_poro_sizes": (st, [vp, C.POINTER(C.c_int64)]),
        "mgr_poro_export": (st, [vp, vp, vp, vp, vp, vp]),
        "mgr_poro_assemble": (st, [vp, vp, vp, vp, C.c_int32, C.POINTER(C.c_double), vp]),
        "mgr_poro_newton": (st, [vp, C.POINTER(vp), C.POINTER(mgr_opts), C.POINTER(fgmres_opts),
                                 vp, vp, C.POINTER(mgr_newton_opts),
                                 C.POINTER(mgr_newton_stats), vp]),
        "mgr_poro_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(status):
    if status != MGR_OK:
        raise MgrError(status, lib().mgr_last_error().decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


# ----------------------------------------------------------------------------------------
class Matrix:
    """Device CSR matrix (int64 row pointers, int32 columns, FP64 values) in torch tensors,
    or BSR with block x block row-major blocks (block = 2 or 3: row pointers and columns
    over blocks, values nnzb * block^2).  `nrows` / `ncols` count scalar rows / columns."""

    def __init__(self, row_ptr, col, val, ncols=None, block=1):
        import torch
        assert row_ptr.dtype == torch.int64 and col.dtype == torch.int32
        assert val.dtype == torch.float64 and block in (1, 2, 3)
        self.row_ptr, self.col, self.val, self.block = row_ptr, col, val, block
        nbr = row_ptr.numel() - 1
        self.nrows = nbr * block
        self.ncols = self.nrows if ncols is None else ncols
        self.c = mgr_csr(nbr, self.ncols // block, row_ptr.data_ptr(), col.data_ptr(),
                         val.data_ptr(), block, 0)

    @staticmethod
    def from_host(indptr, indices, data, device="cuda", ncols=None):
        import torch
        return Matrix(torch.as_tensor(np.asarray(indptr, dtype=np.int64)).to(device),
                      torch.as_tensor(np.asarray(indices, dtype=np.int32)).to(device),
                      torch.as_tensor(np.asarray(data, dtype=np.float64)).to(device), ncols)

    @staticmethod
    def bsr_from_host(indptr, indices, blocks, device="cuda"):
        """BSR from host arrays: block row pointers, block columns (sorted within a block
        row), blocks of shape (nnzb, b, b)."""
        import torch
        blocks = np.ascontiguousarray(blocks, dtype=np.float64)
        b = blocks.shape[1]
        nbc = int(np.max(indices)) + 1 if len(indices) else 0
        return Matrix(torch.as_tensor(np.asarray(indptr, dtype=np.int64)).to(device),
                      torch.as_tensor(np.asarray(indices, dtype=np.int32)).to(device),
                      torch.as_tensor(blocks.reshape(-1)).to(device),
                      ncols=(len(indptr) - 1) * b, block=b)

    @property
    def nnz(self):
        """Scalar entries (stored zeros of blocks included)."""
        return int(self.col.numel()) * self.block * self.block

    def spmv(self, x, y=None, stream=None):
        import torch
        if y is None:
            y = torch.empty(self.nrows, dtype=torch.float64, device=x.device)
        _check(lib().mgr_spmv(C.byref(self.c), _ptr(x), _ptr(y), _stream(stream)))
        return y


@dataclass
class Level:
    """One reduction level (Sec. 5.2): F labels and the components of Algorithm 2."""
    f_labels: tuple
    interp: str = "jacobi"
    nmax: int = -1
    frelax: str = "jacobi"
    frelax_sweeps: int = 1
    frelax_omega: float = 1.0
    frelax_block: int = 1
    global_smoother: str = "none"
    global_sweeps: int = 1
    global_omega: float = 1.0
    coupling: str = "full"          # 'full' | 'quasi_impes'
    drop_tol: float = -1.0          # >= 0: tolerance form of G (nmax must be < 0)
    ilu_level: int = 1              # global_smoother 'ilu': ILU(k), k = 0 or 1
    ilu_sweeps: int = 3             # fixed-point sweeps of the factorisation
    ilu_tri_sweeps: int = 3         # Jacobi sweeps per triangular solve
    restrict: str = "injection"     # 'injection' | 'jacobi' (W_r = -A_CF D_FF^{-1})
    dff_block: int = 1              # D_FF pointwise (1) or blocks of 2 / 3 F rows


@dataclass
class AMG:
    theta0: float = 0.08
    max_levels: int = 10
    coarse_size: int = 256


@dataclass
class Options:
    levels: list
    coarse: str = "amg"
    amg_frelax: AMG = field(default_factory=AMG)
    amg_coarse: AMG = field(default_factory=AMG)
    precision: str = "fp64"
    use_graph: bool = True
    keep_setup: bool = False

    def to_c(self) -> mgr_opts:
        o = mgr_opts()
        lib().mgr_default_opts(C.byref(o))
        if len(self.levels) > MAX_LEVELS:
            raise ValueError("too many levels")
        o.nlevels = len(self.levels)
        for i, L in enumerate(self.levels):
            c = o.level[i]
            c.f_label_mask = sum(1 << int(t) for t in L.f_labels)
            c.interp = INTERP[L.interp]
            c.nmax_drop = int(L.nmax)
            c.frelax = FRELAX[L.frelax]
            c.frelax_sweeps = int(L.frelax_sweeps)
            c.frelax_omega = float(L.frelax_omega)
            c.frelax_block = int(L.frelax_block)
            c.global_smoother = GSMOOTH[L.global_smoother]
            c.global_sweeps = int(L.global_sweeps)
            c.global_omega = float(L.global_omega)
            c.coupling = COUPLING[L.coupling]
            c.drop_tol = float(L.drop_tol)
            c.ilu_level = int(L.ilu_level)
            c.ilu_sweeps = int(L.ilu_sweeps)
            c.ilu_tri_sweeps = int(L.ilu_tri_sweeps)
            c.restrict_ = {"injection": 0, "jacobi": 1}[L.restrict]
            c.dff_block = int(L.dff_block)
        o.coarse = COARSE[self.coarse]
        for dst, src in ((o.amg_frelax, self.amg_frelax), (o.amg_coarse, self.amg_coarse)):
            dst.theta0, dst.max_levels, dst.coarse_size = src.theta0, src.max_levels, src.coarse_size
        o.precision = PREC[self.precision]
        o.use_graph = int(self.use_graph)
        o.keep_setup = int(self.keep_setup)
        return o


def paper_plan(model: str, quasi_impes: bool = False, global_sweeps: int = 4,
               sat_nmax: int | None = None, global_smoother: str = "block_jacobi",
               global_omega: float | None = None, **kw) -> Options:
    """Reduction order of Sec. 5.3: displacement first (one nodal AMG V-cycle, N_max = 4),
    then the saturations (Jacobi, Galerkin, with the global block smoother on the levels that
    hold only cell unknowns), pressure last (AMG).  `quasi_impes` uses the quasi-IMPES
    coupling on the saturation levels; `global_smoother` is 'block_jacobi' or 'block_gs'
    (multicolour block Gauss-Seidel); `global_sweeps` sets the block smoother's sweeps
    (four: the block-Jacobi sweeps stand in for the single, stronger ILU(1) step of
    Sec. 6) and `global_omega` the weight of the sweeps after the first (0.9 for block
    Jacobi, 1 otherwise); `sat_nmax` >= 0 applies the dropping operator on the saturation
    levels too.
    By default the two-phase saturation level is Galerkin (eq. coarse_grid_pressure); the
    three-phase model, which the paper does not treat, drops with the paper's N_max = 4 on
    both saturation levels: two Galerkin eliminations in a row leave a pressure grid with
    distance-3 fill that makes the AMG setup several times slower and its V-cycle weaker."""
    if sat_nmax is None:
        sat_nmax = 4 if model == "three" else -1
    if global_omega is None:
        global_omega = 0.9 if global_smoother == "block_jacobi" else 1.0
    sat = dict(nmax=sat_nmax, frelax="jacobi", global_smoother=global_smoother,
               global_sweeps=global_sweeps, global_omega=global_omega,
               coupling="quasi_impes" if quasi_impes else "full")
    if model == "biot1":
        levels = [Level((0,), nmax=4, frelax="amg", frelax_block=3)]
    elif model == "two":
        levels = [Level((0,), nmax=4, frelax="amg", frelax_block=3), Level((1,), **sat)]
    elif model == "three":
        levels = [Level((0,), nmax=4, frelax="amg", frelax_block=3), Level((3,), **sat),
                  Level((1,), **sat)]
    else:
        raise ValueError(model)
    return Options(levels=levels, **kw)


def saturation_first_plan(model: str, **kw) -> Options:
    """Saturations reduced first (Jacobi, Galerkin), then displacement (nodal AMG,
    N_max = 4), pressure last (AMG)."""
    if model == "two":
        levels = [Level((1,), nmax=-1, frelax="jacobi"),
                  Level((0,), nmax=4, frelax="amg", frelax_block=3)]
    elif model == "three":
        levels = [Level((3,), nmax=-1, frelax="jacobi"), Level((1,), nmax=-1, frelax="jacobi"),
                  Level((0,), nmax=4, frelax="amg", frelax_block=3)]
    else:
        raise ValueError(model)
    return Options(levels=levels, **kw)


class Preconditioner:
    """MGR hierarchy owned by the library (mgr_setup / mgr_apply / mgr_destroy)."""

    def __init__(self, A: Matrix, labels, opts: Options, stream=None):
        self.n = A.nrows
        self.opts = opts
        self._copts = opts.to_c()
        h = C.c_void_p()
        _check(lib().mgr_setup(C.byref(A.c), _ptr(labels), C.byref(self._copts), _stream(stream),
                               C.byref(h)))
        self.h = h

    def apply(self, v, z=None, stream=None):
        import torch
        if z is None:
            z = torch.empty_like(v)
        _check(lib().mgr_apply(self.h, _ptr(v), _ptr(z), _stream(stream)))
        return z

    def setup_numeric(self, A: Matrix, stream=None):
        _check(lib().mgr_setup_numeric(self.h, C.byref(A.c), _stream(stream)))

    def footprint(self) -> int:
        b = C.c_size_t()
        _check(lib().mgr_footprint(self.h, C.byref(b)))
        return int(b.value)

    def query(self, what, level=0, sub=0):
        out = (C.c_int64 * 3)()
        _check(lib().mgr_query(self.h, what, level, sub, out))
        return int(out[0]), int(out[1]), int(out[2])

    def export(self, what, level=0, sub=0, stream=None):
        """Copy an object of the hierarchy to the host: (indptr, indices, data) for CSR
        objects, an int array for index lists and aggregates."""
        import torch
        rows, cols, nnz = self.query(what, level, sub)
        dev = torch.device("cuda")
        if what in (X_F, X_C, X_AMG_AGG, X_GS_COLOR):
            col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
            _check(lib().mgr_export(self.h, what, level, sub, None, _ptr(col), None,
                                    _stream(stream)))
            return col[:nnz].cpu().numpy()
        rp = torch.empty(rows + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
        val = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev)
        _check(lib().mgr_export(self.h, what, level, sub, _ptr(rp), _ptr(col), _ptr(val),
                                _stream(stream)))
        return (rp.cpu().numpy(), col[:nnz].cpu().numpy().astype(np.int64),
                val[:nnz].cpu().numpy(), (rows, cols))

    def amg_levels(self, level):
        return self.query(X_AMG_NLEV, level, 0)[0]

    def close(self):
        if getattr(self, "h", None):
            lib().mgr_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def estimate_footprint(n, nnz, opts: Options) -> int:
    b = C.c_size_t()
    o = opts.to_c()
    _check(lib().mgr_estimate_footprint(int(n), int(nnz), C.byref(o), C.byref(b)))
    return int(b.value)


class Workspace:
    """Caller-owned FGMRES workspace (torch allocation, reused across solves)."""

    def __init__(self, n, restart, device="cuda"):
        import torch
        nbytes = int(lib().fgmres_workspace_bytes(int(n), int(restart)))
        self.buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes
        self.n, self.restart = n, restart


def fgmres(A: Matrix, b, x=None, M: Preconditioner | None = None, restart=30, rtol=1e-6,
           maxit=1000, work: Workspace | None = None, history=False, stream=None,
           raise_on_fail=True):
    """Solve A x = b with FGMRES(restart) preconditioned by M (None = identity)."""
    import torch
    if x is None:
        x = torch.zeros_like(b)
    o = fgmres_opts(int(restart), int(maxit), float(rtol))
    r = fgmres_result()
    hist = None
    if history:
        cap = maxit + maxit // max(restart, 1) + 8
        hist = (C.c_double * cap)()
        r.history = C.cast(hist, C.POINTER(C.c_double))
        r.history_cap = cap
    wp, wb = (C.c_void_p(work.buf.data_ptr()), work.nbytes) if work is not None else (None, 0)
    st = lib().fgmres_solve(C.byref(A.c), M.h if M is not None else None, _ptr(b), _ptr(x),
                            C.byref(o), wp, C.c_size_t(wb), C.byref(r), _stream(stream))
    info = dict(iters=r.iters, restarts=r.restarts, converged=bool(r.converged),
                true_relres=r.true_relres, est_relres=r.est_relres, status=st)
    if history:
        info["history"] = [hist[i] for i in range(r.history_len)]
    if st not in (MGR_OK, MGR_ERR_NOT_CONVERGED) or (st != MGR_OK and raise_on_fail):
        raise MgrError(st, lib().mgr_last_error().decode())
    return x, info


def fgmres_noalloc(A: Matrix, b, x=None, M: Preconditioner | None = None, restart=30,
                   rtol=1e-6, maxit=1000, stream=None, raise_on_fail=True):
    """fgmres with the library's static per-device workspace (fgmres_solve_noalloc): no
    allocation inside the call.  M, when given, must have been applied once before."""
    import torch
    if x is None:
        x = torch.zeros_like(b)
    o = fgmres_opts(int(restart), int(maxit), float(rtol))
    r = fgmres_result()
    st = lib().fgmres_solve_noalloc(C.byref(A.c), M.h if M is not None else None, _ptr(b),
                                    _ptr(x), C.byref(o), C.byref(r), _stream(stream))
    info = dict(iters=r.iters, restarts=r.restarts, converged=bool(r.converged),
                true_relres=r.true_relres, est_relres=r.est_relres, status=st)
    if st not in (MGR_OK, MGR_ERR_NOT_CONVERGED) or (st != MGR_OK and raise_on_fail):
        raise MgrError(st, lib().mgr_last_error().decode())
    return x, info


def batch_solve(As, labels, bs, opts: Options, xs=None, restart=30, rtol=1e-6, maxit=1000,
                stream=None, raise_on_fail=True):
    """Solve the independent systems As[i] x_i = bs[i] together (mgr_batch_solve): one
    setup and one FGMRES over their block-diagonal union.  Returns (xs, relres, info)."""
    import torch
    k = len(As)
    if xs is None:
        xs = [torch.zeros_like(b) for b in bs]
    Ac = (mgr_csr * k)(*[A.c for A in As])
    lp = (C.c_void_p * k)(*[_ptr(l) for l in labels])
    bp = (C.c_void_p * k)(*[_ptr(b) for b in bs])
    xp = (C.c_void_p * k)(*[_ptr(x) for x in xs])
    rel = (C.c_double * k)()
    its = (C.c_int32 * k)()
    copts = opts.to_c()
    o = fgmres_opts(int(restart), int(maxit), float(rtol))
    r = fgmres_result()
    st = lib().mgr_batch_solve(k, Ac, lp, bp, xp, C.byref(copts), C.byref(o), rel, its,
                               C.byref(r), _stream(stream))
    info = dict(iters=r.iters, system_iters=[its[i] for i in range(k)],
                converged=bool(r.converged), true_relres=r.true_relres, status=st)
    if st not in (MGR_OK, MGR_ERR_NOT_CONVERGED) or (st != MGR_OK and raise_on_fail):
        raise MgrError(st, lib().mgr_last_error().decode())
    return xs, [rel[i] for i in range(k)], info


def _owned_to_host(h, sizes, stream=None):
    import torch
    rows, cols, nnz = (int(x) for x in sizes)
    rp = torch.empty(rows + 1, dtype=torch.int64, device="cuda")
    ci = torch.empty(max(nnz, 1), dtype=torch.int32, device="cuda")
    v = torch.empty(max(nnz, 1), dtype=torch.float64, device="cuda")
    try:
        _check(lib().mgr_owned_export(h, _ptr(rp), _ptr(ci), _ptr(v), _stream(stream)))
    finally:
        lib().mgr_owned_free(h)
    return (rp.cpu().numpy(), ci[:nnz].cpu().numpy().astype(np.int64), v[:nnz].cpu().numpy(),
            (rows, cols))


def spgemm(A: Matrix, B: Matrix, stream=None):
    """C = A B with the pinned summation order; returns host (indptr, indices, data, shape)."""
    h = C.c_void_p()
    sz = (C.c_int64 * 3)()
    _check(lib().mgr_spgemm(C.byref(A.c), C.byref(B.c), C.byref(h), sz, _stream(stream)))
    return _owned_to_host(h, sz, stream)


def spgemm_grouped(A: Matrix, B: Matrix, group: int, stream=None):
    """C = A B as spgemm, computed `group` rows of A at a time where the rows of a group share
    their columns; returns host (indptr, indices, data, shape)."""
    h = C.c_void_p()
    sz = (C.c_int64 * 3)()
    _check(lib().mgr_spgemm_grouped(C.byref(A.c), C.byref(B.c), int(group), C.byref(h), sz,
                                    _stream(stream)))
    return _owned_to_host(h, sz, stream)


def spgemm_b3(A: Matrix, B: Matrix, diag_b=False, stream=None):
    """C = A B on full 3x3 blocks (with diag_b only the diagonals of B's blocks); returns
    host (indptr, indices, data, shape)."""
    h = C.c_void_p()
    sz = (C.c_int64 * 3)()
    _check(lib().mgr_spgemm_b3(C.byref(A.c), C.byref(B.c), int(bool(diag_b)), C.byref(h), sz,
                               _stream(stream)))
    return _owned_to_host(h, sz, stream)


def transpose(A: Matrix, stream=None):
    h = C.c_void_p()
    sz = (C.c_int64 * 3)()
    _check(lib().mgr_transpose(C.byref(A.c), C.byref(h), sz, _stream(stream)))
    return _owned_to_host(h, sz, stream)


def merge_drop(A: Matrix, B: Matrix, w=None, nmax=-1, labels_c=None, stream=None):
    h = C.c_void_p()
    sz = (C.c_int64 * 3)()
    _check(lib().mgr_merge_drop(C.byref(A.c), C.byref(B.c), _ptr(w), int(nmax), _ptr(labels_c),
                                C.byref(h), sz, _stream(stream)))
    return _owned_to_host(h, sz, stream)


def ilu(A: Matrix, level: int, sweeps: int, stream=None):
    """Incomplete factors of A on its ILU(level) pattern after `sweeps` fixed-point sweeps
    (mgr_ilu): (indptr, indices, data, shape) on the host."""
    h = C.c_void_p()
    sizes = (C.c_int64 * 3)()
    _check(lib().mgr_ilu(C.byref(A.c), int(level), int(sweeps), C.byref(h), sizes,
                         _stream(stream)))
    return _owned_to_host(h, sizes, stream)


def dense_inverse(D, stream=None):
    """Inverse of a dense square FP64 device tensor by the setup's Gauss-Jordan kernels."""
    import torch
    n = int(D.shape[0])
    D = D.contiguous()
    Inv = torch.empty_like(D)
    _check(lib().mgr_dense_inverse(_ptr(D), _ptr(Inv), n, _stream(stream)))
    return Inv


def csr_to_bsr(A: Matrix, br: int, bc: int | None = None, stream=None):
    """The br x bc block CSR of a matrix over cells of br rows and column groups of bc
    (bc = br by default), as the library stores cell-blocked operators: (block row pointer,
    block columns, blocks (nblk, br, bc)) device tensors."""
    import torch
    bc = br if bc is None else bc
    nb = C.c_int64()
    _check(lib().mgr_csr_to_bsr(C.byref(A.c), int(br), int(bc), None, None, None, 0,
                                C.byref(nb), _stream(stream)))
    k = int(nb.value)
    brp = torch.empty(A.nrows // br + 1, dtype=torch.int32, device="cuda")
    bci = torch.empty(max(k, 1), dtype=torch.int32, device="cuda")
    bv = torch.empty(max(k, 1) * br * bc, dtype=torch.float64, device="cuda")
    _check(lib().mgr_csr_to_bsr(C.byref(A.c), int(br), int(bc), _ptr(brp), _ptr(bci),
                                _ptr(bv), k, C.byref(nb), _stream(stream)))
    return brp, bci[:k], bv[:k * br * bc].view(k, br, bc)


def aggregate(A: Matrix, bs: int, theta: float, level: int, stream=None):
    import torch
    agg = torch.empty(max(A.nrows // bs, 1), dtype=torch.int32, device="cuda")
    na = C.c_int64()
    _check(lib().mgr_aggregate(C.byref(A.c), int(bs), float(theta), int(level), _ptr(agg),
                               C.byref(na), _stream(stream)))
    return agg[:A.nrows // bs].cpu().numpy().astype(np.int64), int(na.value)


def stream_copy(src, dst, stream=None):
    _check(lib().mgr_stream_copy(_ptr(src), _ptr(dst), int(src.numel()), _stream(stream)))


def alloc_stats(reset_peak=False):
    """(bytes handed out by the library allocator, peak since the last reset)."""
    live, peak = C.c_size_t(), C.c_size_t()
    lib().mgr_alloc_stats(C.byref(live), C.byref(peak), int(reset_peak))
    return int(live.value), int(peak.value)


def release_cache():
    _check(lib().mgr_release_cache())


def profile_enable(family: int, on: bool = True):
    _check(lib().mgr_profile_enable(family, int(on)))


def profile_read(family: int):
    n = C.c_int64()
    ms = C.c_double()
    by = C.c_double()
    _check(lib().mgr_profile_read(family, C.byref(n), C.byref(ms), C.byref(by)))
    return int(n.value), float(ms.value), float(by.value)
