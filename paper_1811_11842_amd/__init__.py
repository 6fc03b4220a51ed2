"""MI355X (gfx950) solver for the per-step linear systems of the 2D modified
Cahn-Hilliard / Flory-Huggins biofilm-flow model (arXiv:1811.11842).

Thin ctypes binding of libbiofilm.so (C ABI in include/biofilm.h).  Every
step of the computation runs in the library's HIP kernels; this module only
checks tensors and marshals arguments.  PyTorch supplies device memory and the
stream.  There is no CPU fallback: if the library is not built, every call
raises.

Fields are float64 CUDA tensors of shape (n+1, n) (rows = y nodes 0..n,
columns = x nodes 0..n-1), contiguous.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbiofilm.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "biofilm.h")

# status codes (include/biofilm.h)
OK, NOT_CONVERGED, AT_FLOOR = 0, 1, 2
EINVAL, ENOMEM, EHIP, ENONFINITE, EUNSUPPORTED = -1, -2, -3, -4, -5
OP_LAP, OP_CH, OP_HELM = 0, 1, 2
KSP_CG, KSP_GMRES = 0, 1
PC_NONE, PC_JACOBI, PC_MG = 0, 1, 2
SMOOTH_CHEBYSHEV, SMOOTH_JACOBI = 0, 1
MG_F64, MG_F32 = 0, 1
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "AT_FLOOR", -1: "EINVAL", -2: "ENOMEM",
                -3: "EHIP", -4: "ENONFINITE", -5: "EUNSUPPORTED"}


class GridDesc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("dtype", ctypes.c_int32), ("stream", ctypes.c_void_p)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("ksp", ctypes.c_int32), ("pc", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("restart", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("degree", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("ratio", ctypes.c_double), ("omega", ctypes.c_double),
                ("mg_precision", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def __repr__(self):
        return "SolverOpts(" + ", ".join(f"{k}={getattr(self, k)}" for k, _ in self._fields_) + ")"


class SolveStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("clamped", ctypes.c_int32),
                ("rel_res", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("ms", ctypes.c_double), ("floor_est", ctypes.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS_NAMES.get(self.status, str(self.status))
        return d

    def __repr__(self):
        return f"SolveStats({self.as_dict()})"


class Params(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("dt", "M", "kappa", "Npoly", "chi", "phi_lo",
                                               "phi_hi")]


class BiofilmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None
_P = ctypes.c_void_p


def lib():
    """Load libbiofilm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} not found: build it with "
                               "`python -m paper_1811_11842_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "bf_solver_opts_default": (None, [ctypes.c_int32, ctypes.POINTER(SolverOpts)]),
            "bf_grid_create": (ctypes.c_int, [ctypes.POINTER(GridDesc), ctypes.POINTER(_P)]),
            "bf_grid_destroy": (ctypes.c_int, [_P]),
            "bf_grid_shape": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64),
                                             ctypes.POINTER(ctypes.c_int64)]),
            "bf_apply": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, _P, _P]),
            "bf_solve_ch": (ctypes.c_int, [_P, ctypes.c_double, _P, _P, ctypes.POINTER(SolverOpts),
                                           ctypes.POINTER(SolveStats)]),
            "bf_solve_pressure": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(SolverOpts),
                                                 ctypes.POINTER(SolveStats)]),
            "bf_solve_helmholtz": (ctypes.c_int, [_P, ctypes.c_double, _P, _P,
                                                  ctypes.POINTER(SolverOpts),
                                                  ctypes.POINTER(SolveStats)]),
            "bf_momentum_predict": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_double, ctypes.c_double, _P, _P, _P,
                                                   _P, ctypes.POINTER(SolverOpts),
                                                   ctypes.POINTER(SolveStats)]),
            "bf_apply_mob": (ctypes.c_int, [_P, ctypes.c_double, _P, _P, _P]),
            "bf_solve_ch_mob": (ctypes.c_int, [_P, ctypes.c_double, _P, _P, _P,
                                               ctypes.POINTER(SolverOpts),
                                               ctypes.POINTER(SolveStats)]),
            "bf_step_ch_mob": (ctypes.c_int, [_P, ctypes.POINTER(Params), _P,
                                              ctypes.POINTER(SolverOpts),
                                              ctypes.POINTER(SolveStats)]),
            "bf_ch_rhs": (ctypes.c_int, [_P, ctypes.POINTER(Params), _P, _P, _P]),
            "bf_pressure_rhs": (ctypes.c_int, [_P, ctypes.c_double, _P, _P, _P]),
            "bf_velocity_correct": (ctypes.c_int, [_P, ctypes.c_double, _P, _P, _P, _P, _P]),
            "bf_step": (ctypes.c_int, [_P, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P,
                                       ctypes.POINTER(SolverOpts), ctypes.POINTER(SolverOpts),
                                       ctypes.POINTER(SolveStats)]),
            "bf_step_ch": (ctypes.c_int, [_P, ctypes.POINTER(Params), _P, _P, _P,
                                          ctypes.POINTER(SolverOpts), ctypes.POINTER(SolveStats)]),
            "bf_step_ch_cn": (ctypes.c_int, [_P, ctypes.POINTER(Params), _P, _P, ctypes.c_int32,
                                             ctypes.POINTER(SolverOpts),
                                             ctypes.POINTER(SolveStats)]),
            "bf_adjoint_step": (ctypes.c_int, [_P, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P,
                                               _P, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(SolverOpts),
                                               ctypes.POINTER(SolveStats)]),
            "bf_vcycle": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double,
                                         ctypes.POINTER(SolverOpts), _P, _P]),
            "bf_restrict": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
            "bf_prolong_add": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P]),
            "bf_wdot": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(ctypes.c_double)]),
            "bf_copy": (ctypes.c_int, [_P, _P, _P]),
            "bf_smooth": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, _P, _P, _P, _P,
                                         ctypes.c_double, ctypes.c_double]),
            "bf_residual": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_double, _P, _P, _P,
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                           ctypes.POINTER(ctypes.c_double)]),
            "bf_grid_cg_timing": (ctypes.c_int, [_P, ctypes.c_int32]),
            "bf_grid_rupdate_timing_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                                           ctypes.POINTER(ctypes.c_int64)]),
            "bf_grid_cg_timing_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double),
                                                      ctypes.POINTER(ctypes.c_int64),
                                                      ctypes.POINTER(ctypes.c_int64)]),
            "bf_residual_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                                   _P, _P, _P, _P, _P]),
            "bf_ensemble_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                                  _P, ctypes.POINTER(_P)]),
            "bf_ensemble_destroy": (ctypes.c_int, [_P]),
            "bf_ensemble_layout": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64),
                                                  ctypes.POINTER(ctypes.c_int64)]),
            "bf_ensemble_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                                ctypes.POINTER(ctypes.c_int32),
                                                ctypes.POINTER(ctypes.c_int32),
                                                ctypes.POINTER(ctypes.c_int32)]),
            "bf_ensemble_step": (ctypes.c_int, [_P, ctypes.POINTER(Params), _P, _P, _P, _P, _P, _P,
                                                ctypes.POINTER(SolverOpts),
                                                ctypes.POINTER(SolverOpts),
                                                ctypes.POINTER(SolveStats),
                                                ctypes.POINTER(ctypes.c_double)]),
            "bf_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def declared_symbols():
    """Names of the functions declared in include/biofilm.h."""
    with open(HEADER_PATH) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(bf_\w+)\s*\(", text, re.M)))


def _check(code):
    if code < 0:
        raise BiofilmError(code, lib().bf_last_error().decode())
    return code


def default_opts(op: int, **kw) -> SolverOpts:
    o = SolverOpts()
    lib().bf_solver_opts_default(op, ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def make_params(dt=1e-4, M=1.0, kappa=1e-3, Npoly=100.0, chi=0.6, phi_lo=1e-6,
                phi_hi=1.0 - 1e-6) -> Params:
    return Params(dt, M, kappa, Npoly, chi, phi_lo, phi_hi)


class Grid:
    """Handle of a grid of n intervals per side (bf_grid_create)."""

    def __init__(self, n: int, stream: torch.cuda.Stream | None = None):
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.n = n
        self.stream = stream
        self.device = stream.device
        desc = GridDesc(n, 0, stream.cuda_stream)
        h = _P()
        with torch.cuda.device(self.device):
            _check(L.bf_grid_create(ctypes.byref(desc), ctypes.byref(h)))
        self._h = h

    # ------------------------------------------------------------ plumbing
    def close(self):
        if getattr(self, "_h", None):
            lib().bf_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def shape(self):
        return (self.n + 1, self.n)

    def field(self, fill=None):
        t = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        if fill is not None:
            t.fill_(fill)
        return t

    def _ptr(self, t, name, shape=None):
        if t is None:
            return None
        shape = self.shape if shape is None else shape
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA tensor")
        if t.dtype != torch.float64:
            raise TypeError(f"{name} must be float64, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, grid on {self.device}")
        return _P(t.data_ptr())

    # ------------------------------------------------------------ entry points
    def apply(self, op, c, x, y=None):
        y = self.field() if y is None else y
        _check(lib().bf_apply(self._h, op, c, self._ptr(x, "x"), self._ptr(y, "y")))
        return y

    def solve_ch(self, c, b, x, opts=None) -> SolveStats:
        st = SolveStats()
        _check(lib().bf_solve_ch(self._h, c, self._ptr(b, "b"), self._ptr(x, "x"),
                                 ctypes.byref(opts) if opts is not None else None,
                                 ctypes.byref(st)))
        return st

    def solve_pressure(self, rhs, p, opts=None) -> SolveStats:
        st = SolveStats()
        _check(lib().bf_solve_pressure(self._h, self._ptr(rhs, "rhs"), self._ptr(p, "p"),
                                       ctypes.byref(opts) if opts is not None else None,
                                       ctypes.byref(st)))
        return st

    def solve_helmholtz(self, beta, b, x, opts=None) -> SolveStats:
        """x - beta L_D x = b inside, x = b on the wall rows (Dirichlet data)."""
        st = SolveStats()
        _check(lib().bf_solve_helmholtz(self._h, beta, self._ptr(b, "b"), self._ptr(x, "x"),
                                        ctypes.byref(opts) if opts is not None else None,
                                        ctypes.byref(st)))
        return st

    def apply_mob(self, c, m, x, y=None):
        """y = x + c L_m L x for the node mobilities m."""
        y = self.field() if y is None else y
        _check(lib().bf_apply_mob(self._h, c, self._ptr(m, "m"), self._ptr(x, "x"),
                                  self._ptr(y, "y")))
        return y

    def solve_ch_mob(self, c, m, b, x, opts=None) -> SolveStats:
        st = SolveStats()
        _check(lib().bf_solve_ch_mob(self._h, c, self._ptr(m, "m"), self._ptr(b, "b"),
                                     self._ptr(x, "x"),
                                     ctypes.byref(opts) if opts is not None else None,
                                     ctypes.byref(st)))
        return st

    def step_ch_mob(self, params: Params, phi, opts=None) -> SolveStats:
        """One Cahn-Hilliard step in place with the mobility M clamp(phi)."""
        st = SolveStats()
        _check(lib().bf_step_ch_mob(self._h, ctypes.byref(params), self._ptr(phi, "phi"),
                                    ctypes.byref(opts) if opts is not None else None,
                                    ctypes.byref(st)))
        return st

    def momentum_predict(self, dt, nu, theta, U, u, v, ustar=None, vstar=None, opts=None):
        """(u*, v*, stats) of the momentum predictor; ustar may be u, vstar may be v."""
        ustar = self.field() if ustar is None else ustar
        vstar = self.field() if vstar is None else vstar
        st = (SolveStats * 2)()
        _check(lib().bf_momentum_predict(self._h, dt, nu, theta, U, self._ptr(u, "u"),
                                         self._ptr(v, "v"), self._ptr(ustar, "ustar"),
                                         self._ptr(vstar, "vstar"),
                                         ctypes.byref(opts) if opts is not None else None, st))
        return ustar, vstar, (st[0], st[1])

    def ch_rhs(self, params: Params, phi, b=None, clamped=None):
        b = self.field() if b is None else b
        cp = None
        if clamped is not None:
            if clamped.dtype != torch.int32 or not clamped.is_cuda:
                raise TypeError("clamped must be an int32 CUDA tensor")
            cp = _P(clamped.data_ptr())
        _check(lib().bf_ch_rhs(self._h, ctypes.byref(params), self._ptr(phi, "phi"),
                               self._ptr(b, "b"), cp))
        return b

    def pressure_rhs(self, dt, u, v, rhs=None):
        rhs = self.field() if rhs is None else rhs
        _check(lib().bf_pressure_rhs(self._h, dt, self._ptr(u, "u"), self._ptr(v, "v"),
                                     self._ptr(rhs, "rhs")))
        return rhs

    def velocity_correct(self, dt, p, ustar, vstar, u=None, v=None):
        u = self.field() if u is None else u
        v = self.field() if v is None else v
        _check(lib().bf_velocity_correct(self._h, dt, self._ptr(p, "p"),
                                         self._ptr(ustar, "ustar"), self._ptr(vstar, "vstar"),
                                         self._ptr(u, "u"), self._ptr(v, "v")))
        return u, v

    def step(self, params: Params, phi, ustar, vstar, p, u=None, v=None, ch=None, pr=None):
        st = (SolveStats * 2)()
        _check(lib().bf_step(self._h, ctypes.byref(params), self._ptr(phi, "phi"),
                             self._ptr(ustar, "ustar"), self._ptr(vstar, "vstar"),
                             self._ptr(p, "p"), self._ptr(u, "u"), self._ptr(v, "v"),
                             ctypes.byref(ch) if ch is not None else None,
                             ctypes.byref(pr) if pr is not None else None, st))
        return st[0], st[1]

    def step_ch(self, params: Params, phi, u=None, v=None, opts=None) -> SolveStats:
        """One Cahn-Hilliard step in place, advected by (u, v) if given."""
        st = SolveStats()
        _check(lib().bf_step_ch(self._h, ctypes.byref(params), self._ptr(phi, "phi"),
                                self._ptr(u, "u"), self._ptr(v, "v"),
                                ctypes.byref(opts) if opts is not None else None,
                                ctypes.byref(st)))
        return st

    def step_ch_cn(self, params: Params, phi, phi_prev, first=False, opts=None) -> SolveStats:
        """One Crank-Nicolson step: phi -> phi^{n+1}, phi_prev -> phi^n."""
        st = SolveStats()
        _check(lib().bf_step_ch_cn(self._h, ctypes.byref(params), self._ptr(phi, "phi"),
                                   self._ptr(phi_prev, "phi_prev"), 1 if first else 0,
                                   ctypes.byref(opts) if opts is not None else None,
                                   ctypes.byref(st)))
        return st

    def adjoint_step(self, params: Params, phi_n, lam_in, lam_out=None, u=None, v=None,
                     du=None, dv=None, opts=None):
        """(lam_out, [dJ/dchi, dJ/dU] contributions, stats) of one reverse step."""
        lam_out = self.field() if lam_out is None else lam_out
        g = (ctypes.c_double * 2)(0.0, 0.0)
        st = SolveStats()
        _check(lib().bf_adjoint_step(self._h, ctypes.byref(params), self._ptr(phi_n, "phi_n"),
                                     self._ptr(u, "u"), self._ptr(v, "v"),
                                     self._ptr(du, "du"), self._ptr(dv, "dv"),
                                     self._ptr(lam_in, "lam_in"), self._ptr(lam_out, "lam_out"),
                                     g, ctypes.byref(opts) if opts is not None else None,
                                     ctypes.byref(st)))
        return lam_out, (g[0], g[1]), st

    def vcycle(self, op, c, r, z=None, opts=None):
        z = self.field() if z is None else z
        _check(lib().bf_vcycle(self._h, op, c, ctypes.byref(opts) if opts is not None else None,
                               self._ptr(r, "r"), self._ptr(z, "z")))
        return z

    def restrict(self, nf, fine, coarse=None):
        cs = (nf // 2 + 1, nf // 2)
        coarse = torch.empty(cs, dtype=torch.float64, device=self.device) if coarse is None else coarse
        _check(lib().bf_restrict(self._h, nf, self._ptr(fine, "fine", (nf + 1, nf)),
                                 self._ptr(coarse, "coarse", cs)))
        return coarse

    def prolong_add(self, nf, coarse, fine):
        cs = (nf // 2 + 1, nf // 2)
        _check(lib().bf_prolong_add(self._h, nf, self._ptr(coarse, "coarse", cs),
                                    self._ptr(fine, "fine", (nf + 1, nf))))
        return fine

    def residual(self, op, c, b, x, r=None, accurate=True):
        """(r, ||r||_W/||b||_W, floor estimate) with r = b - A x."""
        r = self.field() if r is None else r
        rel, fl = ctypes.c_double(), ctypes.c_double()
        _check(lib().bf_residual(self._h, op, c, self._ptr(b, "b"), self._ptr(x, "x"),
                                 self._ptr(r, "r"), 1 if accurate else 0, ctypes.byref(rel),
                                 ctypes.byref(fl)))
        return r, rel.value, fl.value

    def smooth(self, op, c, x, b, xout=None, xprev=None, a=1.0, g=0.0):
        xout = self.field() if xout is None else xout
        _check(lib().bf_smooth(self._h, op, c, self._ptr(x, "x"),
                               self._ptr(xprev, "xprev") if xprev is not None else None,
                               self._ptr(b, "b"), self._ptr(xout, "xout"), a, g))
        return xout

    def copy(self, x, y=None):
        y = self.field() if y is None else y
        _check(lib().bf_copy(self._h, self._ptr(x, "x"), self._ptr(y, "y")))
        return y

    def cg_timing(self, every):
        """Start timing every `every`-th launch of the Cahn-Hilliard CG step
        kernel (True: every launch; clears the record), or stop (0 / False)."""
        _check(lib().bf_grid_cg_timing(self._h, int(every)))

    def cg_timing_read(self):
        """(summed ms, launches, first-step launches) since timing started; clears the record."""
        ms, n, nf = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().bf_grid_cg_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n),
                                            ctypes.byref(nf)))
        return ms.value, n.value, nf.value

    def rupdate_timing_read(self):
        """(summed ms, launches) of the residual updates timed with the CG steps; clears it."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().bf_grid_rupdate_timing_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def wdot(self, x, y) -> float:
        out = ctypes.c_double()
        _check(lib().bf_wdot(self._h, self._ptr(x, "x"), self._ptr(y, "y"), ctypes.byref(out)))
        return out.value


def residual_noalloc(op, c, b, x, r, norms, stream: torch.cuda.Stream | None = None):
    """bf_residual_noalloc: r = b - A x (double-double) and norms[0:3] =
    (||r||_W / ||b||_W, float64 floor estimate, ||b||_W), both on the device;
    no grid handle, no allocation, no synchronisation.  b, x, r: float64 CUDA
    tensors of shape (n+1, n); norms: a float64 CUDA tensor of 3 elements."""
    for name, t in (("b", b), ("x", x), ("r", r)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and t.dim() == 2 and t.shape[0] == t.shape[1] + 1):
            raise TypeError(f"{name} must be a contiguous float64 CUDA tensor of shape (n+1, n)")
        if t.shape != b.shape:
            raise TypeError(f"{name} has shape {tuple(t.shape)}, b has {tuple(b.shape)}")
    if not (isinstance(norms, torch.Tensor) and norms.is_cuda and norms.dtype == torch.float64
            and norms.is_contiguous() and norms.numel() >= 3):
        raise TypeError("norms must be a contiguous float64 CUDA tensor of at least 3 elements")
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().bf_residual_noalloc(b.shape[1], op, c, _P(b.data_ptr()), _P(x.data_ptr()),
                                     _P(r.data_ptr()), _P(norms.data_ptr()),
                                     _P(stream.cuda_stream)))
    return r, norms


grid_create = Grid


class Ensemble:
    """Handle of an ensemble of independent grids (bf_ensemble_create).

    Fields are packed: one float64 device tensor of `total` elements per
    quantity, instance i in the (n_i+1) x n_i block at offsets[i] (`view`)."""

    def __init__(self, sizes, stream: torch.cuda.Stream | None = None):
        L = lib()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.sizes = [int(n) for n in sizes]
        self.count = len(self.sizes)
        self.stream = stream
        self.device = stream.device
        arr = (ctypes.c_int32 * self.count)(*self.sizes)
        h = _P()
        with torch.cuda.device(self.device):
            _check(L.bf_ensemble_create(arr, self.count, stream.cuda_stream, ctypes.byref(h)))
        self._h = h
        offs = (ctypes.c_int64 * self.count)()
        tot = ctypes.c_int64()
        _check(L.bf_ensemble_layout(self._h, offs, ctypes.byref(tot)))
        self.offsets = list(offs)
        self.total = tot.value

    def info(self):
        """[(n, instances, tile height)] per size class."""
        nc = ctypes.c_int32()
        cn = (ctypes.c_int32 * self.count)()
        cc = (ctypes.c_int32 * self.count)()
        cr = (ctypes.c_int32 * self.count)()
        _check(lib().bf_ensemble_info(self._h, ctypes.byref(nc), cn, cc, cr))
        return [(cn[k], cc[k], cr[k]) for k in range(nc.value)]

    def field(self, fill=None):
        t = torch.empty(self.total, dtype=torch.float64, device=self.device)
        if fill is not None:
            t.fill_(fill)
        return t

    def view(self, t, i):
        n = self.sizes[i]
        o = self.offsets[i]
        return t[o:o + (n + 1) * n].view(n + 1, n)

    def _ptr(self, t, name):
        if t is None:
            return None
        if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                and t.numel() == self.total):
            raise ValueError(f"{name}: expected a contiguous float64 CUDA tensor of "
                             f"{self.total} elements")
        return ctypes.c_void_p(t.data_ptr())

    def step(self, params, phi, ustar, vstar, p, u=None, v=None, ch=None, pr=None):
        """One step of every instance; params: list of Params (one per instance).
        Returns ([(ch_stats, p_stats)] per instance, device ms of the step)."""
        if len(params) != self.count:
            raise ValueError("one Params per instance")
        prm = (Params * self.count)(*params)
        st = (SolveStats * (2 * self.count))()
        ms = ctypes.c_double()
        _check(lib().bf_ensemble_step(self._h, prm, self._ptr(phi, "phi"),
                                      self._ptr(ustar, "ustar"), self._ptr(vstar, "vstar"),
                                      self._ptr(p, "p"), self._ptr(u, "u"), self._ptr(v, "v"),
                                      ctypes.byref(ch) if ch is not None else None,
                                      ctypes.byref(pr) if pr is not None else None, st,
                                      ctypes.byref(ms)))
        return [(st[2 * i], st[2 * i + 1]) for i in range(self.count)], ms.value

    def close(self):
        if getattr(self, "_h", None):
            lib().bf_ensemble_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
