"""ctypes binding of libmfl.so (include/mfl.h): argument marshalling only.

Every computation runs in the library's HIP kernels; torch supplies device memory and
the current HIP stream.  Loading fails loudly when the library has not been built.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfl.so")

MFL_OK, MFL_EINVAL, MFL_ENOCONV, MFL_EBREAKDOWN, MFL_EHIP, MFL_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
CG, SIPG = 0, 1
CARTESIAN, CURVED = 0, 1
DIRICHLET, NEUMANN, MIXED = 0, 1, 2
DG_JACOBI_GAUSS, DG_JACOBI_GLL = 0, 1
KAPPA_CELLWISE, KAPPA_COSINE = 0, 1
METRIC_AUTO, METRIC_STORED, METRIC_ON_THE_FLY = 0, 1, 2
F64, F32 = 0, 1
_DT = {F64: torch.float64, F32: torch.float32}


class MflError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("mfl error %d: %s" % (code, message))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("degree", ctypes.c_int),
        ("cells_per_dim", ctypes.c_int),
        ("min_level_cells", ctypes.c_int),
        ("disc", ctypes.c_int),
        ("geometry", ctypes.c_int),
        ("curve_amp", ctypes.c_double),
        ("bc", ctypes.c_int),
        ("penalty_factor", ctypes.c_double),
        ("cheb_degree", ctypes.c_int),
        ("cheb_lo", ctypes.c_double),
        ("cheb_hi", ctypes.c_double),
        ("eig_iters", ctypes.c_int),
        ("coarse_tol", ctypes.c_double),
        ("mg_precision", ctypes.c_int),
        ("build_mg", ctypes.c_int),
        ("domain_lo", ctypes.c_double),
        ("domain_len", ctypes.c_double),
        ("dg_jacobi_basis", ctypes.c_int),
        ("use_graphs", ctypes.c_int),
        ("kappa_field", ctypes.c_int),
        ("kappa_field_amp", ctypes.c_double),
        ("metric_mode", ctypes.c_int),
    ]


_lib = None
P = ctypes.c_void_p
I64P = ctypes.POINTER(ctypes.c_int64)
IP = ctypes.POINTER(ctypes.c_int)
DP = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "mfl_default_params": (ctypes.c_int, [ctypes.POINTER(Params)]),
    "mfl_query": (ctypes.c_int, [ctypes.POINTER(Params), I64P, I64P, I64P]),
    "mfl_setup": (ctypes.c_int, [ctypes.POINTER(Params), P, ctypes.c_int64, P, P, ctypes.POINTER(P)]),
    "mfl_set_kappa": (ctypes.c_int, [P, P, P]),
    "mfl_num_levels": (ctypes.c_int, [P]),
    "mfl_level_info": (ctypes.c_int, [P, ctypes.c_int, IP, I64P, DP, DP, DP, IP]),
    "mfl_apply": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, P, P, P]),
    "mfl_diagonal": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, P, P]),
    "mfl_transfer": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]),
    "mfl_vcycle": (ctypes.c_int, [P, P, P, P]),
    "mfl_pcg_solve": (ctypes.c_int, [P, P, P, ctypes.c_double, ctypes.c_int, IP, DP, P]),
    "mfl_rhs_sine": (ctypes.c_int, [P, P, P]),
    "mfl_rhs_gaussians": (ctypes.c_int, [P, P, P]),
    "mfl_adjoint_solve": (ctypes.c_int, [P, P, P, ctypes.c_double, ctypes.c_int, IP, DP, P]),
    "mfl_kappa_gradient": (ctypes.c_int, [P, P, P, P, P]),
    "mfl_profile": (ctypes.c_int, [P, ctypes.c_int, IP, DP]),
    "mfl_apply_noalloc": (ctypes.c_int, [ctypes.POINTER(Params), P, ctypes.c_int, P, P, P]),
    "mfl_destroy": (ctypes.c_int, [P]),
    "mfl_last_error": (ctypes.c_char_p, []),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libmfl.so is not built (run __graft_entry__.build()); "
                              "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc, allow=()):
    if rc != MFL_OK and rc not in allow:
        raise MflError(rc, lib().mfl_last_error().decode())
    return rc


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def make_params(degree, cells_per_dim, disc=CG, geometry=CARTESIAN, curve_amp=0.1, bc=DIRICHLET,
                penalty_factor=1.0, build_mg=False, mg_precision=F64, min_level_cells=2,
                cheb_degree=5, cheb_lo=0.06, cheb_hi=1.2, eig_iters=15, coarse_tol=1e-3,
                domain_lo=0.0, domain_len=1.0, dg_jacobi_basis=DG_JACOBI_GLL, use_graphs=True,
                kappa_field=KAPPA_CELLWISE, kappa_field_amp=1e6, metric_mode=METRIC_AUTO):
    p = Params()
    _check(lib().mfl_default_params(ctypes.byref(p)))
    p.degree, p.cells_per_dim, p.min_level_cells = degree, cells_per_dim, min_level_cells
    p.disc, p.geometry, p.curve_amp, p.bc = disc, geometry, curve_amp, bc
    p.penalty_factor, p.build_mg, p.mg_precision = penalty_factor, int(bool(build_mg)), mg_precision
    p.cheb_degree, p.cheb_lo, p.cheb_hi = cheb_degree, cheb_lo, cheb_hi
    p.eig_iters, p.coarse_tol = eig_iters, coarse_tol
    p.domain_lo, p.domain_len = domain_lo, domain_len
    p.dg_jacobi_basis = dg_jacobi_basis
    p.use_graphs = int(bool(use_graphs))
    p.kappa_field, p.kappa_field_amp = kappa_field, kappa_field_amp
    p.metric_mode = metric_mode
    return p


def check_vector(t, n, dtype, name):
    """Raise ValueError unless t is a contiguous CUDA tensor of `dtype` with n values: the
    library reads or writes n values of that type through the pointer."""
    if not torch.is_tensor(t):
        raise ValueError("%s must be a torch tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must be a CUDA tensor (got device %s)" % (name, t.device))
    if t.dtype != dtype:
        raise ValueError("%s must be %s (got %s)" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() != n:
        raise ValueError("%s must hold %d values (got %d)" % (name, n, t.numel()))
    return t


NOALLOC_SCRATCH_BYTES = 48 << 20


def apply_noalloc(params, src, dst, kappa=None):
    """dst = A src through mfl_apply_noalloc (continuous Q_k, Cartesian cells): no handle,
    no workspace; the library's fixed per-GPU scratch array holds its halo records.  kappa:
    None or a float64 CUDA tensor of n_cells values."""
    n, cells, _ = query(params)
    dtype = F32 if torch.is_tensor(src) and src.dtype == torch.float32 else F64
    check_vector(src, n, _DT[dtype], "src")
    check_vector(dst, n, _DT[dtype], "dst")
    kptr = None
    if kappa is not None:
        check_vector(kappa, cells, torch.float64, "kappa")
        kptr = _ptr(kappa)
    _check(lib().mfl_apply_noalloc(ctypes.byref(params), kptr, dtype, _ptr(src), _ptr(dst), _stream()))
    return dst


def query(params):
    nd, nc, ws = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    _check(lib().mfl_query(ctypes.byref(params), ctypes.byref(nd), ctypes.byref(nc), ctypes.byref(ws)))
    return nd.value, nc.value, ws.value


class Problem:
    """A set-up operator (and optionally its multigrid hierarchy) on the current GPU.

    Owns the device workspace (a torch uint8 tensor) and the library handle.
    """

    def __init__(self, degree, cells_per_dim, kappa=None, device="cuda", **kw):
        self.params = make_params(degree, cells_per_dim, **kw)
        self.n_dofs, self.n_cells, ws = query(self.params)
        self.device = torch.device(device)
        self.workspace = torch.empty(max(ws, 256) + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        self._kappa = None
        h = ctypes.c_void_p()
        kptr = None
        if kappa is not None:
            self._kappa = self._as_f64(kappa, self.n_cells)
            kptr = _ptr(self._kappa)
        _check(lib().mfl_setup(ctypes.byref(self.params), ctypes.c_void_p(self._ws_ptr),
                               ctypes.c_int64(ws), kptr, _stream(), ctypes.byref(h)))
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value and _lib is not None:
            _lib.mfl_destroy(h)
            self.handle = None

    def _as_f64(self, t, n):
        t = torch.as_tensor(t, dtype=torch.float64, device=self.device).contiguous()
        if t.numel() != n:
            raise ValueError("expected %d values, got %d" % (n, t.numel()))
        return t

    @property
    def num_levels(self):
        return _check(lib().mfl_num_levels(self.handle), allow=range(1, 1 << 20))

    def _level_dofs(self, level):
        cache = self.__dict__.setdefault("_dofs_cache", {})
        if level not in cache:
            cache[level] = self.level_info(level)["n_dofs"]
        return cache[level]

    def level_info(self, level=-1):
        c, nd = ctypes.c_int(), ctypes.c_int64()
        lam, lmin, lmax, st = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        _check(lib().mfl_level_info(self.handle, level, ctypes.byref(c), ctypes.byref(nd), ctypes.byref(lam),
                                    ctypes.byref(lmin), ctypes.byref(lmax), ctypes.byref(st)))
        return {"cells_per_dim": c.value, "n_dofs": nd.value, "lambda_max": lam.value,
                "coarse_lmin": lmin.value, "coarse_lmax": lmax.value, "coarse_steps": st.value}

    def profile_start(self):
        """Start timing the operator cell kernels launched by apply() with HIP events."""
        _check(lib().mfl_profile(self.handle, 1, None, None))

    def profile_stop(self):
        """Stop timing; returns (number of timed cell-kernel launches, total ms)."""
        n, ms = ctypes.c_int(), ctypes.c_double()
        _check(lib().mfl_profile(self.handle, 0, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def set_kappa(self, kappa):
        self._kappa = self._as_f64(kappa, self.n_cells)
        _check(lib().mfl_set_kappa(self.handle, _ptr(self._kappa), _stream()))

    def apply(self, src, dst=None, level=-1):
        dtype = F32 if torch.is_tensor(src) and src.dtype == torch.float32 else F64
        n = self._level_dofs(level)
        check_vector(src, n, _DT[dtype], "src")
        dst = torch.empty_like(src) if dst is None else check_vector(dst, n, _DT[dtype], "dst")
        _check(lib().mfl_apply(self.handle, level, dtype, _ptr(src), _ptr(dst), _stream()))
        return dst

    def diagonal(self, level=-1, dtype=torch.float64):
        n = self.level_info(level)["n_dofs"]
        out = torch.empty(n, dtype=dtype, device=self.device)
        _check(lib().mfl_diagonal(self.handle, level, F32 if dtype == torch.float32 else F64, _ptr(out),
                                  _stream()))
        return out

    def transfer(self, level, direction, src, dst):
        """direction 0: dst (level) += P src (level - 1); 1: dst (level - 1) = P^T src (level).
        The fine vector is in the dtype of the call (float32 or float64); the coarse vector in
        the same dtype, except on the coarsest level, which is always float64."""
        nl = self.num_levels
        lev = nl - 1 if level == -1 else level
        if not 1 <= lev < nl:
            raise ValueError("transfer needs a level in 1..%d (got %d)" % (nl - 1, level))
        fine, coarse = (dst, src) if direction == 0 else (src, dst)
        if direction not in (0, 1):
            raise ValueError("direction must be 0 (prolongate) or 1 (restrict)")
        dtype = F32 if torch.is_tensor(fine) and fine.dtype == torch.float32 else F64
        cdt = torch.float64 if lev - 1 == 0 else _DT[dtype]
        check_vector(fine, self._level_dofs(lev), _DT[dtype], "fine vector")
        check_vector(coarse, self._level_dofs(lev - 1), cdt, "coarse vector")
        _check(lib().mfl_transfer(self.handle, lev, direction, dtype, _ptr(src), _ptr(dst), _stream()))
        return dst

    def vcycle(self, r, z=None):
        r = self._as_f64(r, self.n_dofs)
        z = torch.empty_like(r) if z is None else check_vector(z, self.n_dofs, torch.float64, "z")
        _check(lib().mfl_vcycle(self.handle, _ptr(r), _ptr(z), _stream()))
        return z

    def rhs_sine(self):
        b = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        _check(lib().mfl_rhs_sine(self.handle, _ptr(b), _stream()))
        return b

    def rhs_gaussians(self):
        """Right-hand side of the three-Gaussian example (mfl_rhs_gaussians)."""
        b = torch.empty(self.n_dofs, dtype=torch.float64, device=self.device)
        _check(lib().mfl_rhs_gaussians(self.handle, _ptr(b), _stream()))
        return b

    def _solve(self, fn, b, rtol, maxit, x, raise_on_noconv):
        b = self._as_f64(b, self.n_dofs)
        x = torch.empty_like(b) if x is None else check_vector(x, self.n_dofs, torch.float64, "x")
        it, res = ctypes.c_int(), ctypes.c_double()
        rc = fn(self.handle, _ptr(b), _ptr(x), ctypes.c_double(rtol), ctypes.c_int(maxit),
                ctypes.byref(it), ctypes.byref(res), _stream())
        _check(rc, allow=() if raise_on_noconv else (MFL_ENOCONV,))
        return x, it.value, res.value

    def solve(self, b, rtol=1e-10, maxit=100, x=None, raise_on_noconv=True):
        """PCG with one V-cycle per iteration; returns (x, iterations, relative residual)."""
        return self._solve(lib().mfl_pcg_solve, b, rtol, maxit, x, raise_on_noconv)

    def adjoint_solve(self, dJdu, rtol=1e-10, maxit=100, x=None, raise_on_noconv=True):
        return self._solve(lib().mfl_adjoint_solve, dJdu, rtol, maxit, x, raise_on_noconv)

    def kappa_gradient(self, u, lam):
        u = self._as_f64(u, self.n_dofs)
        lam = self._as_f64(lam, self.n_dofs)
        g = torch.empty(self.n_cells, dtype=torch.float64, device=self.device)
        _check(lib().mfl_kappa_gradient(self.handle, _ptr(u), _ptr(lam), _ptr(g), _stream()))
        return g
