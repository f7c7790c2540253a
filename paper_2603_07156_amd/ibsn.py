"""ctypes binding of libibsn.so (include/ibsn.h).

Argument marshalling only: every function below checks its torch tensors (device,
dtype, contiguity, length), passes their device pointers and the current HIP stream
to the C ABI, and returns the outputs.  All arithmetic runs in the library's HIP
kernels.  The library must be built (``python -m paper_2603_07156_amd.build``); a
missing library is an error, never a fallback.
"""
from __future__ import annotations

import ctypes as ct
import os
import sys
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libibsn.so")

IBSN_OK = 0
IBSN_WARN_MAXITER = 1
IBSN_COST_F64 = 0
IBSN_COST_F32 = 1
IBSN_COST_POINTS = 2
PREC_F64 = 0    # ibsn_precision
PREC_MIXED = 1
CG_AUTO, CG_LAUNCHES, CG_PERSISTENT, CG_SINGLE, CG_PIPE = 0, 1, 2, 3, 4   # ibsn_set_cg_kernel
CSC_AUTO, CSC_ENTRY, CSC_BLOCK = 0, 1, 2   # ibsn_set_csc_fill
WS_HEAD_FEATURES = 8   # per-target features of the learned warm start's head (fth columns)
MAX_N_F64 = 10240


class IBSNError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libibsn error {code}: {msg}")
        self.code = code


class _Problem(ct.Structure):
    _fields_ = [("m", ct.c_int64), ("n", ct.c_int64), ("cost_kind", ct.c_int32),
                ("precision", ct.c_int32), ("C", ct.c_void_p), ("ldc", ct.c_int64),
                ("a", ct.c_void_p), ("b", ct.c_void_p), ("eta", ct.c_double),
                ("y", ct.c_void_p), ("cost_scale", ct.c_double)]


class _Center(ct.Structure):
    _fields_ = [("k", ct.c_int64), ("r", ct.c_void_p), ("s", ct.c_void_p),
                ("quantum", ct.c_double)]


class Tile(ct.Structure):
    _fields_ = [("nt", ct.c_int32), ("q", ct.c_int32), ("qf", ct.c_int32), ("nt_h", ct.c_int32),
                ("q_h", ct.c_int32), ("qf_h", ct.c_int32), ("grid", ct.c_int32),
                ("reserved", ct.c_int32), ("light_ms", ct.c_double), ("heavy_ms", ct.c_double),
                ("default_light_ms", ct.c_double), ("default_heavy_ms", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class Options(ct.Structure):
    _fields_ = [
        ("sigma_armijo", ct.c_double), ("beta", ct.c_double),
        ("sinkhorn_tol", ct.c_double), ("sinkhorn_maxit", ct.c_int32),
        ("mu0", ct.c_double), ("mu_floor", ct.c_double),
        ("gap_tol", ct.c_double), ("marg_tol", ct.c_double), ("kkt_tol", ct.c_double),
        ("max_outer", ct.c_int32), ("max_newton", ct.c_int32), ("max_backtrack", ct.c_int32),
        ("cg_maxit", ct.c_int32), ("cg_forcing_max", ct.c_double), ("rho_mode", ct.c_int32),
        ("cg_rtol_min", ct.c_double), ("stall_limit", ct.c_int32),
        ("eot", ct.c_int32), ("eot_tol", ct.c_double), ("mixed_switch", ct.c_double),
        ("trace", ct.c_void_p), ("trace_cap", ct.c_int64), ("armijo_warm", ct.c_int32),
    ]


class IterRecord(ct.Structure):
    """ibsn_iter_record: one outer iteration of ibsn_solve."""
    _fields_ = [
        ("k", ct.c_int64), ("newton", ct.c_int64), ("cg", ct.c_int64), ("sinkhorn", ct.c_int64),
        ("backtracks", ct.c_int64), ("stop_tests", ct.c_int64), ("passes", ct.c_int64),
        ("mixed_passes", ct.c_int64),
        ("grad_norm", ct.c_double), ("primal", ct.c_double), ("dual", ct.c_double),
        ("rel_gap", ct.c_double), ("kkt", ct.c_double), ("dphi", ct.c_double),
        ("marg_l1", ct.c_double), ("nnz_mean", ct.c_double),
        ("t_eval", ct.c_double), ("t_sparsify", ct.c_double), ("t_cg", ct.c_double),
        ("t_linesearch", ct.c_double), ("t_stop", ct.c_double), ("t_total", ct.c_double),
        ("inner_stopped", ct.c_int32), ("reserved", ct.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


class Report(ct.Structure):
    _fields_ = [
        ("outer", ct.c_int64), ("newton", ct.c_int64), ("cg", ct.c_int64),
        ("sinkhorn", ct.c_int64), ("backtracks", ct.c_int64), ("stop_tests", ct.c_int64),
        ("passes", ct.c_int64),
        ("grad_norm", ct.c_double), ("primal", ct.c_double), ("dual", ct.c_double),
        ("rel_gap", ct.c_double), ("kkt", ct.c_double), ("dphi", ct.c_double),
        ("marg_l1", ct.c_double),
        ("t_eval", ct.c_double), ("t_sparsify", ct.c_double), ("t_cg", ct.c_double),
        ("t_linesearch", ct.c_double), ("t_stop", ct.c_double), ("t_total", ct.c_double),
        ("nnz_mean", ct.c_double), ("nnz_last", ct.c_double),
        ("mixed_passes", ct.c_int64), ("trace_len", ct.c_int64),
        ("status", ct.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


KT_NAMES = ("eval", "trial", "sparsify", "csc", "stop1", "stop2", "cg", "colreduce",
            "eval_mixed", "trial_mixed", "sparsify_mixed")


class _KernelTimes(ct.Structure):
    _fields_ = [("ms", ct.c_double * len(KT_NAMES)), ("count", ct.c_int64 * len(KT_NAMES))]


_lib = None
EXPORTS = ("ibsn_create", "ibsn_destroy", "ibsn_last_error", "ibsn_num_cus", "ibsn_set_cg_kernel",
           "ibsn_set_row_split", "ibsn_set_csc_fill", "ibsn_autotune",
           "ibsn_center_init", "ibsn_center_quantum", "ibsn_sinkhorn_step", "ibsn_outer_update", "ibsn_subproblem_eval", "ibsn_trial", "ibsn_sparsify", "ibsn_csr_info",
           "ibsn_csr_export", "ibsn_csr_free", "ibsn_hvp", "ibsn_cg", "ibsn_stop",
           "ibsn_default_options", "ibsn_solve", "ibsn_kernel_timing", "ibsn_kernel_times_get",
           "ibsn_solve_batch", "ibsn_hvp_noalloc", "ibsn_ws_param_count", "ibsn_ws_create",
           "ibsn_ws_free", "ibsn_ws_get_params", "ibsn_ws_set_params", "ibsn_ws_features",
           "ibsn_ws_forward", "ibsn_ws_predict", "ibsn_ws_train_step")


def load():
    """Load libibsn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2603_07156_amd.build` (no CPU fallback exists)")
    L = ct.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ct.c_void_p, ct.c_int64, ct.c_int32, ct.c_double
    P, C = ct.POINTER(_Problem), ct.POINTER(_Center)
    L.ibsn_create.argtypes = [ct.POINTER(vp), ct.c_int, vp]
    L.ibsn_destroy.argtypes = [vp]
    L.ibsn_destroy.restype = None
    L.ibsn_last_error.argtypes = [vp]
    L.ibsn_last_error.restype = ct.c_char_p
    L.ibsn_num_cus.argtypes = [vp]
    L.ibsn_set_cg_kernel.argtypes = [vp, ct.c_int, ct.c_int]
    L.ibsn_set_row_split.argtypes = [vp, i64]
    L.ibsn_set_csc_fill.argtypes = [vp, ct.c_int]
    L.ibsn_autotune.argtypes = [vp, ct.c_void_p, ct.POINTER(Tile)]
    L.ibsn_center_init.argtypes = [vp, P, vp, vp]
    L.ibsn_center_quantum.argtypes = [vp, P, C, vp, ct.POINTER(dbl)]
    L.ibsn_subproblem_eval.argtypes = [vp, P, C, vp, vp, vp, vp, vp, vp, ct.POINTER(dbl), vp]
    L.ibsn_trial.argtypes = [vp, P, C, vp, vp, vp, dbl, ct.POINTER(dbl), vp, vp, vp, vp]
    L.ibsn_sparsify.argtypes = [vp, P, C, vp, vp, vp, dbl, i64, ct.POINTER(vp)]
    L.ibsn_sinkhorn_step.argtypes = [vp, P, C, vp, vp, vp, vp, vp]
    L.ibsn_outer_update.argtypes = [vp, P, C, vp, vp, vp, vp, vp]
    L.ibsn_csr_info.argtypes = [vp, vp, ct.POINTER(i64), ct.POINTER(i64)]
    L.ibsn_csr_export.argtypes = [vp, vp, vp, vp, vp, vp]
    L.ibsn_csr_free.argtypes = [vp]
    L.ibsn_csr_free.restype = None
    L.ibsn_hvp.argtypes = [vp, vp, vp, dbl, dbl, vp, vp]
    L.ibsn_hvp_noalloc.argtypes = [vp, vp, vp, dbl, dbl, vp, vp]
    L.ibsn_cg.argtypes = [vp, vp, vp, dbl, dbl, vp, dbl, ct.c_int, vp, ct.POINTER(ct.c_int)]
    L.ibsn_stop.argtypes = [vp, P, C, vp, vp, vp, ct.POINTER(dbl), vp]
    L.ibsn_default_options.argtypes = [ct.POINTER(Options)]
    L.ibsn_default_options.restype = None
    L.ibsn_solve.argtypes = [vp, P, ct.POINTER(Options), vp, vp, vp, ct.POINTER(i64), vp,
                             ct.POINTER(Report)]
    L.ibsn_solve_batch.argtypes = [ct.POINTER(vp), ct.c_int, i64, P, ct.POINTER(Options),
                                   ct.POINTER(vp), ct.POINTER(Report), ct.POINTER(ct.c_int32)]
    fp = ct.POINTER(ct.c_float)
    L.ibsn_ws_param_count.argtypes = []
    L.ibsn_ws_param_count.restype = i64
    L.ibsn_ws_create.argtypes = [vp, ct.c_uint64, ct.POINTER(vp)]
    L.ibsn_ws_free.argtypes = [vp]
    L.ibsn_ws_free.restype = None
    L.ibsn_ws_get_params.argtypes = [vp, vp, fp, i64]
    L.ibsn_ws_set_params.argtypes = [vp, vp, fp, i64]
    L.ibsn_ws_features.argtypes = [vp, P, vp, vp, vp, vp, vp, ct.POINTER(dbl)]
    L.ibsn_ws_forward.argtypes = [vp, vp, i64, i64, i64, vp, vp, vp, vp]
    L.ibsn_ws_predict.argtypes = [vp, vp, i64, i64, vp, vp, vp, dbl, vp]
    L.ibsn_ws_train_step.argtypes = [vp, vp, i64, i64, i64, vp, vp, vp, vp, ct.c_float,
                                     ct.POINTER(ct.c_float), fp]
    L.ibsn_kernel_timing.argtypes = [vp, ct.c_int]
    L.ibsn_kernel_times_get.argtypes = [vp, ct.POINTER(_KernelTimes)]
    for name in EXPORTS:
        if not hasattr(L, name):
            raise ImportError(f"{LIB_PATH} does not export {name}")
    _lib = L
    return L


def _ptr(t, n=None, dtype=torch.float64, name="tensor", device=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (HIP) tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return ct.c_void_p(t.data_ptr())


class Context:
    """An ibsn_ctx bound to a device and to that device's current torch stream."""

    def __init__(self, device: int | torch.device = 0, stream: torch.cuda.Stream | None = None):
        L = load()
        self._lib = L   # handles are released through the library that made them
        self.device = torch.device("cuda", device) if isinstance(device, int) else device
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ct.c_void_p()
        rc = L.ibsn_create(ct.byref(h), self.device.index or 0, ct.c_void_p(self.stream.cuda_stream))
        if rc != 0:
            raise IBSNError(rc, "ibsn_create failed")
        self.h = h

    def check(self, rc):
        if rc < 0:
            raise IBSNError(rc, load().ibsn_last_error(self.h).decode())
        return rc

    @property
    def num_cus(self):
        return load().ibsn_num_cus(self.h)

    def set_cg_kernel(self, mode: int = 0, blocks: int = 0):
        """ibsn_set_cg_kernel: CG_AUTO, CG_LAUNCHES, CG_PERSISTENT, CG_SINGLE or CG_PIPE, and
        the grid of the cooperative forms (0: from the problem size)."""
        self.check(load().ibsn_set_cg_kernel(self.h, int(mode), int(blocks)))

    def set_row_split(self, cols: int = 0):
        """ibsn_set_row_split: rows wider than `cols` columns run as column blocks of at most
        `cols` (0: only rows wider than the register tiles, in blocks of 10240 columns for an
        FP64 or points cost and 12288 for an FP32 cost)."""
        self.check(load().ibsn_set_row_split(self.h, int(cols)))

    def set_csc_fill(self, mode: int = 0):
        """ibsn_set_csc_fill: CSC_AUTO, CSC_ENTRY or CSC_BLOCK (the transpose's fill)."""
        self.check(load().ibsn_set_csc_fill(self.h, int(mode)))

    def autotune(self, prob: "Problem | None"):
        """ibsn_autotune: choose and record the dense-pass tiles for problems of prob's shape
        on this context (None: clear the records); returns the choice and its timings."""
        if prob is None:
            self.check(load().ibsn_autotune(self.h, None, None))
            return None
        t = Tile()
        self.check(load().ibsn_autotune(self.h, ct.byref(prob.raw()), ct.byref(t)))
        return t.as_dict()

    def kernel_timing(self, enable: bool = True):
        """ibsn_kernel_timing: enable (and clear) or disable HIP-event kernel timing."""
        self.check(load().ibsn_kernel_timing(self.h, 1 if enable else 0))

    def kernel_times(self):
        """ibsn_kernel_times_get: {phase: (total ms, launches)}."""
        kt = _KernelTimes()
        self.check(load().ibsn_kernel_times_get(self.h, ct.byref(kt)))
        return {name: (kt.ms[i], kt.count[i]) for i, name in enumerate(KT_NAMES)}

    def close(self):
        if getattr(self, "h", None):
            self._lib.ibsn_destroy(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the HIP runtime may already be gone: leave the memory to
        # the process's end rather than call into it (the module's globals may be gone too,
        # hence the bound default)
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Problem:
    """eq. (1) data on the device: C (m x n, float64 or float32, row-major), a, b, eta;
    precision: PREC_F64 or PREC_MIXED (FP32 exponentials and sparse values, FP64 sums).
    Points cost (no stored matrix): C = x (m x dim, float64), y (n x dim) and cost_scale,
    C_ij = cost_scale * sum_d (x_id - y_jd)^2 (see Problem.from_points)."""

    C: torch.Tensor
    a: torch.Tensor
    b: torch.Tensor
    eta: float
    precision: int = 0
    y: torch.Tensor | None = None
    cost_scale: float = 0.0

    @classmethod
    def from_points(cls, x, y, a, b, eta, cost_scale, precision=0):
        return cls(x, a, b, eta, precision, y, float(cost_scale))

    @property
    def m(self):
        return self.C.shape[0]

    @property
    def n(self):
        return self.C.shape[1] if self.y is None else self.y.shape[0]

    def raw(self):
        if self.C.dim() != 2 or self.C.stride(1) != 1:
            raise ValueError("C must be a row-major 2-D tensor")
        if self.precision not in (PREC_F64, PREC_MIXED):
            raise ValueError("precision must be PREC_F64 or PREC_MIXED")
        if self.y is not None:
            x, y = self.C, self.y
            if (x.dtype != torch.float64 or y.dtype != torch.float64 or not x.is_contiguous()
                    or not y.is_contiguous() or y.dim() != 2 or y.shape[1] != x.shape[1]):
                raise ValueError("points: x (m x d) and y (n x d), contiguous float64")
            dev = x.device
            return _Problem(self.m, self.n, IBSN_COST_POINTS, int(self.precision),
                            ct.c_void_p(x.data_ptr()), x.shape[1],
                            _ptr(self.a, self.m, name="a", device=dev),
                            _ptr(self.b, self.n, name="b", device=dev), float(self.eta),
                            ct.c_void_p(y.data_ptr()), float(self.cost_scale))
        if self.C.dtype == torch.float64:
            kind = IBSN_COST_F64
        elif self.C.dtype == torch.float32:
            kind = IBSN_COST_F32
        else:
            raise TypeError("C must be float64 or float32")
        if not self.C.is_cuda:
            raise ValueError("C must be a device tensor")
        dev = self.C.device
        return _Problem(self.m, self.n, kind, int(self.precision), ct.c_void_p(self.C.data_ptr()),
                        self.C.stride(0),
                        _ptr(self.a, self.m, name="a", device=dev),
                        _ptr(self.b, self.n, name="b", device=dev), float(self.eta))


@dataclass
class Center:
    """Implicit prox centre log X^k = r + s - k C / eta (r may be None if unused), with the
    grid spacing `quantum` of the potentials (a power of two; see include/ibsn.h)."""

    k: int
    r: torch.Tensor | None
    s: torch.Tensor
    quantum: float

    def raw(self, m, n):
        return _Center(int(self.k), _ptr(self.r, m, name="r"), _ptr(self.s, n, name="s"),
                       float(self.quantum))

    @staticmethod
    def initial(ctx: "Context", prob: Problem, gamma: torch.Tensor | None = None) -> "Center":
        """X^0 = a b^T (Algorithm 2 input; r = log a, s = log b from ibsn_center_init), with
        the solver's grid for gamma (0 if None)."""
        r, s = _new(prob, prob.m), _new(prob, prob.n)
        center_init(ctx, prob, r, s)
        c = Center(0, r, s, 1.0)
        g = gamma if gamma is not None else torch.zeros_like(prob.b)
        c.quantum = center_quantum(ctx, prob, c, g)
        return c


def center_init(ctx: "Context", prob: Problem, r, s):
    """ibsn_center_init: r = log a, s = log b (the centre X^0 = a b^T) into r (m), s (n)."""
    ctx.check(load().ibsn_center_init(ctx.h, ct.byref(prob.raw()), _ptr(r, prob.m, name="r"),
                                      _ptr(s, prob.n, name="s")))
    return r, s


def center_quantum(ctx: "Context", prob: Problem, center: Center, gamma) -> float:
    """ibsn_center_quantum: grid spacing for (prob, center.k, center.s, gamma)."""
    q = ct.c_double()
    raw = _Center(int(center.k), None, _ptr(center.s, prob.n, name="s"), 1.0)
    ctx.check(load().ibsn_center_quantum(ctx.h, ct.byref(prob.raw()), ct.byref(raw),
                                         _ptr(gamma, prob.n, name="gamma"), ct.byref(q)))
    return q.value


def _new(prob, count):
    return torch.empty(count, dtype=torch.float64, device=prob.C.device)


def subproblem_eval(ctx: Context, prob: Problem, center: Center, gamma: torch.Tensor,
                    want_obj: bool = True, want_plan: bool = False, want_lse: bool = True):
    """ibsn_subproblem_eval: returns dict(M, S, lse, c, g, L, plan)."""
    m, n = prob.m, prob.n
    M, S, c, g = _new(prob, m), _new(prob, m), _new(prob, n), _new(prob, n)
    lse = _new(prob, m) if want_lse else None
    plan = torch.empty((m, n), dtype=torch.float64, device=prob.C.device) if want_plan else None
    obj = ct.c_double(float("nan"))
    ctx.check(load().ibsn_subproblem_eval(
        ctx.h, ct.byref(prob.raw()), ct.byref(center.raw(m, n)), _ptr(gamma, n, name="gamma"),
        _ptr(M), _ptr(S), _ptr(lse), _ptr(c), _ptr(g), ct.byref(obj) if want_obj else None,
        _ptr(plan)))
    return dict(M=M, S=S, lse=lse, c=c, g=g, L=obj.value if want_obj else None, plan=plan)


def trial(ctx: Context, prob: Problem, center: Center, gamma, M, Delta, t: float):
    """ibsn_trial: Armijo trial at gamma + t Delta.  Returns dict(dL, M, S, c, g)."""
    m, n = prob.m, prob.n
    Mn, Sn, cn, gn = _new(prob, m), _new(prob, m), _new(prob, n), _new(prob, n)
    dL = ct.c_double()
    ctx.check(load().ibsn_trial(ctx.h, ct.byref(prob.raw()), ct.byref(center.raw(m, n)),
                                _ptr(gamma, n, name="gamma"), _ptr(M, m, name="M"),
                                _ptr(Delta, n, name="Delta"), float(t), ct.byref(dL), _ptr(Mn),
                                _ptr(Sn), _ptr(cn), _ptr(gn)))
    return dict(dL=dL.value, M=Mn, S=Sn, c=cn, g=gn)


def sinkhorn_step(ctx: Context, prob: Problem, center: Center, gamma, M, S, c):
    """ibsn_sinkhorn_step: gamma + eta (log b - log c), centred, from the eval at gamma."""
    m, n = prob.m, prob.n
    out = _new(prob, n)
    ctx.check(load().ibsn_sinkhorn_step(ctx.h, ct.byref(prob.raw()), ct.byref(center.raw(m, n)),
                                        _ptr(gamma, n, name="gamma"), _ptr(M, m, name="M"),
                                        _ptr(S, m, name="S"), _ptr(c, n, name="c"), _ptr(out)))
    return out


def outer_update(ctx: Context, prob: Problem, center: Center, gamma, M, S):
    """ibsn_outer_update: the next centre's (r, s) from the row state (M, S) at gamma."""
    m, n = prob.m, prob.n
    r, s = _new(prob, m), _new(prob, n)
    ctx.check(load().ibsn_outer_update(ctx.h, ct.byref(prob.raw()), ct.byref(center.raw(m, n)),
                                       _ptr(gamma, n, name="gamma"), _ptr(M, m, name="M"),
                                       _ptr(S, m, name="S"), _ptr(r), _ptr(s)))
    return r, s


class Csr:
    """Library-owned sparsified factor P_rho (Algorithm 1)."""

    def __init__(self, ctx: Context, h, m, n, device):
        self.ctx, self.h, self.m, self.n, self.device = ctx, h, m, n, device
        nnz, istar = ct.c_int64(), ct.c_int64()
        ctx.check(load().ibsn_csr_info(ctx.h, h, ct.byref(nnz), ct.byref(istar)))
        self.nnz, self.istar = nnz.value, istar.value

    def export(self):
        """Standard CSR copy: (row_ptr int64, col int32, val f64, d f64) device tensors."""
        row_ptr = torch.empty(self.m + 1, dtype=torch.int64, device=self.device)
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        val = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=self.device)
        d = torch.empty(self.n, dtype=torch.float64, device=self.device)
        self.ctx.check(load().ibsn_csr_export(self.ctx.h, self.h, _ptr(row_ptr, dtype=torch.int64),
                                              _ptr(col, dtype=torch.int32), _ptr(val), _ptr(d)))
        return row_ptr, col[: self.nnz], val[: self.nnz], d

    def free(self):
        if self.h:
            self.ctx._lib.ibsn_csr_free(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the HIP runtime may already be gone: leave the memory to
        # the process's end rather than call into it (the module's globals may be gone too,
        # hence the bound default)
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def sparsify(ctx: Context, prob: Problem, center: Center, gamma, M, S, rho: float,
             istar: int = -1) -> Csr:
    """ibsn_sparsify (Algorithm 1) from the row state (M, S)."""
    m, n = prob.m, prob.n
    h = ct.c_void_p()
    ctx.check(load().ibsn_sparsify(ctx.h, ct.byref(prob.raw()), ct.byref(center.raw(m, n)),
                                   _ptr(gamma, n, name="gamma"), _ptr(M, m, name="M"),
                                   _ptr(S, m, name="S"), float(rho), int(istar), ct.byref(h)))
    return Csr(ctx, h, m, n, prob.C.device)


def hvp(ctx: Context, csr: Csr, a, eta: float, shift: float, v):
    """ibsn_hvp: (H_rho + shift I) v."""
    y = torch.empty(csr.n, dtype=torch.float64, device=csr.device)
    ctx.check(load().ibsn_hvp(ctx.h, csr.h, _ptr(a, csr.m, name="a"), float(eta), float(shift),
                              _ptr(v, csr.n, name="v"), _ptr(y)))
    return y


NOALLOC_MAX_M = 1048576


def hvp_noalloc(ctx: Context, csr: Csr, a, eta: float, shift: float, v, y):
    """ibsn_hvp_noalloc: y = (H_rho + shift I) v into the caller's y; the library allocates
    nothing (its intermediate lives in a fixed per-device array; m <= NOALLOC_MAX_M)."""
    ctx.check(load().ibsn_hvp_noalloc(ctx.h, csr.h, _ptr(a, csr.m, name="a"), float(eta),
                                      float(shift), _ptr(v, csr.n, name="v"),
                                      _ptr(y, csr.n, name="y")))
    return y


def cg(ctx: Context, csr: Csr, a, eta: float, shift: float, rhs, tol: float, maxit: int):
    """ibsn_cg: returns (x, iterations)."""
    x = torch.empty(csr.n, dtype=torch.float64, device=csr.device)
    it = ct.c_int()
    ctx.check(load().ibsn_cg(ctx.h, csr.h, _ptr(a, csr.m, name="a"), float(eta), float(shift),
                             _ptr(rhs, csr.n, name="rhs"), float(tol), int(maxit), _ptr(x),
                             ct.byref(it)))
    return x, it.value


STOP_FIELDS = ("dphi", "primal", "dual", "cx", "kkt", "xhat_min", "er1", "xu", "dual_gamma",
               "dual_psi")


def stop(ctx: Context, prob: Problem, center: Center, gamma, M, S, want_xhat: bool = False):
    """ibsn_stop: rounding (Algorithm 3), D_phi and the certificate."""
    m, n = prob.m, prob.n
    out = (ct.c_double * 10)()
    xhat = torch.empty((m, n), dtype=torch.float64, device=prob.C.device) if want_xhat else None
    ctx.check(load().ibsn_stop(ctx.h, ct.byref(prob.raw()), ct.byref(center.raw(m, n)),
                               _ptr(gamma, n, name="gamma"), _ptr(M, m, name="M"),
                               _ptr(S, m, name="S"), out, _ptr(xhat)))
    res = dict(zip(STOP_FIELDS, list(out)))
    if want_xhat:
        res["xhat"] = xhat
    return res


class WarmStart:
    """The learned warm start (ibsn_ws_*): a point-set network predicting the first
    subproblem's dual, with BF16 MFMA kernels.  Features and outputs are device tensors."""

    def __init__(self, ctx: Context, seed: int = 0):
        L = load()
        self.ctx, self._lib = ctx, L
        h = ct.c_void_p()
        ctx.check(L.ibsn_ws_create(ctx.h, ct.c_uint64(seed), ct.byref(h)))
        self.h = h
        self.count = int(L.ibsn_ws_param_count())

    def params(self):
        import numpy as np
        out = np.empty(self.count, dtype=np.float32)
        self.ctx.check(load().ibsn_ws_get_params(
            self.ctx.h, self.h, out.ctypes.data_as(ct.POINTER(ct.c_float)), self.count))
        return out

    def set_params(self, flat):
        import numpy as np
        arr = np.ascontiguousarray(flat, dtype=np.float32)
        if arr.size != self.count:
            raise ValueError(f"expected {self.count} parameters, got {arr.size}")
        self.ctx.check(load().ibsn_ws_set_params(
            self.ctx.h, self.h, arr.ctypes.data_as(ct.POINTER(ct.c_float)), self.count))

    def features(self, prob: "Problem", x, y):
        """ibsn_ws_features: (fs, fte, fth, scale) of one problem with 2-D points x, y."""
        m, n = prob.m, prob.n
        dev = prob.a.device
        fs = torch.empty((m, 4), dtype=torch.float32, device=dev)
        fte = torch.empty((n, 4), dtype=torch.float32, device=dev)
        fth = torch.empty((n, WS_HEAD_FEATURES), dtype=torch.float32, device=dev)
        sc = ct.c_double()
        self.ctx.check(load().ibsn_ws_features(
            self.ctx.h, ct.byref(prob.raw()), _ptr(x, 2 * m, name="x"), _ptr(y, 2 * n, name="y"),
            _ptr(fs, dtype=torch.float32), _ptr(fte, dtype=torch.float32),
            _ptr(fth, dtype=torch.float32), ct.byref(sc)))
        return fs, fte, fth, sc.value

    def forward(self, B, m, n, fs, fte, fth):
        """ibsn_ws_forward: raw outputs (B n) for stacked instances."""
        out = torch.empty(B * n, dtype=torch.float32, device=fs.device)
        f32 = torch.float32
        self.ctx.check(load().ibsn_ws_forward(
            self.ctx.h, self.h, B, m, n, _ptr(fs, B * m * 4, f32, "fs"),
            _ptr(fte, B * n * 4, f32, "fte"), _ptr(fth, B * n * WS_HEAD_FEATURES, f32, "fth"),
            _ptr(out, dtype=f32)))
        return out

    def predict(self, m, n, fs, fte, fth, scale):
        """ibsn_ws_predict: the warm-start dual (n, float64) of one instance."""
        g = torch.empty(n, dtype=torch.float64, device=fs.device)
        f32 = torch.float32
        self.ctx.check(load().ibsn_ws_predict(
            self.ctx.h, self.h, m, n, _ptr(fs, m * 4, f32, "fs"), _ptr(fte, n * 4, f32, "fte"),
            _ptr(fth, n * WS_HEAD_FEATURES, f32, "fth"), float(scale), _ptr(g)))
        return g

    def train_step(self, B, m, n, fs, fte, fth, target, lr, want_grad=False):
        """ibsn_ws_train_step: (loss, gradient or None)."""
        import numpy as np
        loss = ct.c_float()
        grad = np.empty(self.count, dtype=np.float32) if want_grad else None
        f32 = torch.float32
        self.ctx.check(load().ibsn_ws_train_step(
            self.ctx.h, self.h, B, m, n, _ptr(fs, B * m * 4, f32, "fs"),
            _ptr(fte, B * n * 4, f32, "fte"), _ptr(fth, B * n * WS_HEAD_FEATURES, f32, "fth"),
            _ptr(target, B * n, f32, "target"), float(lr), ct.byref(loss),
            grad.ctypes.data_as(ct.POINTER(ct.c_float)) if want_grad else None))
        return loss.value, grad

    def free(self):
        if getattr(self, "h", None):
            self._lib.ibsn_ws_free(self.h)
            self.h = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the HIP runtime may already be gone: leave the memory to
        # the process's end rather than call into it (the module's globals may be gone too,
        # hence the bound default)
        if _finalizing():
            return
        try:
            self.free()
        except Exception:
            pass


def default_options(**kw) -> Options:
    o = Options()
    load().ibsn_default_options(ct.byref(o))
    for key, v in kw.items():
        if not hasattr(o, key):
            raise KeyError(key)
        setattr(o, key, v)
    return o


def solve(ctx: Context, prob: Problem, options: Options | None = None, gamma0=None, state=None,
          want_plan: bool = False, trace_cap: int = 0):
    """ibsn_solve (Algorithm 2).  state = (r, s, k) resumes an outer state.  trace_cap > 0
    returns the first trace_cap per-outer-iteration records (ibsn_iter_record) as dicts.
    Returns dict(status, gamma, r, s, k, plan, report, trace)."""
    m, n = prob.m, prob.n
    gamma = _new(prob, n)
    if gamma0 is not None:
        gamma.copy_(gamma0)
    else:
        gamma.zero_()
    r, s = _new(prob, m), _new(prob, n)
    k = ct.c_int64(0)
    if state is not None:
        r.copy_(state[0])
        s.copy_(state[1])
        k.value = int(state[2])
    plan = torch.empty((m, n), dtype=torch.float64, device=prob.C.device) if want_plan else None
    rep = Report()
    opt = Options()
    ct.pointer(opt)[0] = options if options is not None else default_options()
    recs = (IterRecord * max(int(trace_cap), 1))()
    opt.trace = ct.cast(recs, ct.c_void_p) if trace_cap > 0 else None
    opt.trace_cap = int(trace_cap)
    rc = ctx.check(load().ibsn_solve(ctx.h, ct.byref(prob.raw()), ct.byref(opt), _ptr(gamma),
                                     _ptr(r), _ptr(s), ct.byref(k), _ptr(plan), ct.byref(rep)))
    trace = [recs[i].as_dict() for i in range(rep.trace_len)] if trace_cap > 0 else None
    return dict(status=rc, gamma=gamma, r=r, s=s, k=k.value, plan=plan, report=rep.as_dict(),
                trace=trace)


def solve_batch(ctxs, probs, options: Options | None = None, gamma0=None):
    """ibsn_solve_batch: solve independent problems with one host worker per context (each
    context on its own stream).  gamma0: optional list of warm starts.  Returns a list of
    dict(status, gamma, report), in the order of `probs`."""
    ctxs = list(ctxs)
    if not ctxs:
        raise ValueError("at least one context")
    L = load()
    raws = (_Problem * max(len(probs), 1))(*[p.raw() for p in probs])
    gammas = []
    for i, p in enumerate(probs):
        g = _new(p, p.n)
        if gamma0 is not None and gamma0[i] is not None:
            g.copy_(gamma0[i])
        else:
            g.zero_()
        gammas.append(g)
    gptr = (ct.c_void_p * max(len(probs), 1))(*[ct.c_void_p(g.data_ptr()) for g in gammas])
    reps = (Report * max(len(probs), 1))()
    status = (ct.c_int32 * max(len(probs), 1))()
    handles = (ct.c_void_p * len(ctxs))(*[c.h for c in ctxs])
    opt = options if options is not None else default_options()
    for p in probs:
        if p.C.device != probs[0].C.device:
            raise ValueError("all problems must live on one device")
    torch.cuda.synchronize()   # inputs written on torch's stream are visible to every worker
    ctxs[0].check(L.ibsn_solve_batch(handles, len(ctxs), len(probs), raws, ct.byref(opt), gptr,
                                     reps, status))
    return [dict(status=int(status[i]), gamma=gammas[i], report=reps[i].as_dict())
            for i in range(len(probs))]


# the C-ABI names
ibsn_center_init = center_init
ibsn_center_quantum = center_quantum
ibsn_subproblem_eval = subproblem_eval
ibsn_trial = trial
ibsn_sinkhorn_step = sinkhorn_step
ibsn_outer_update = outer_update
ibsn_sparsify = sparsify
ibsn_hvp = hvp
ibsn_hvp_noalloc = hvp_noalloc
ibsn_cg = cg
ibsn_stop = stop
ibsn_solve = solve
ibsn_solve_batch = solve_batch
