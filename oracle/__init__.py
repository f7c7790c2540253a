"""CPU oracle for the IBSN method (test infrastructure only).

This package wraps ``ibsn_oracle.c``, a plain FP64 implementation of every step of
the Inexact Bregman Sparse Newton method, written from the paper and sharing no
code with the HIP library.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import it; the product path never does.

All arrays are numpy float64 (int64/int32 for CSR indices), C-contiguous.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ibsn_oracle.c")
_LIB = os.path.join(_HERE, "libibsn_oracle.so")

GCC_FLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC"]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no HIP involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ct.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = ct.POINTER(ct.c_double)
_i64p = ct.POINTER(ct.c_int64)
_i32p = ct.POINTER(ct.c_int32)


class Options(ct.Structure):
    _fields_ = [
        ("sigma_armijo", ct.c_double), ("beta", ct.c_double),
        ("sinkhorn_tol", ct.c_double), ("sinkhorn_maxit", ct.c_int),
        ("mu0", ct.c_double), ("mu_floor", ct.c_double),
        ("gap_tol", ct.c_double), ("marg_tol", ct.c_double), ("kkt_tol", ct.c_double),
        ("max_outer", ct.c_int), ("max_newton", ct.c_int), ("max_backtrack", ct.c_int),
        ("cg_maxit", ct.c_int), ("cg_forcing_max", ct.c_double), ("rho_mode", ct.c_int),
        ("cg_rtol_min", ct.c_double), ("stall_limit", ct.c_int),
        ("eot", ct.c_int), ("eot_tol", ct.c_double), ("armijo_warm", ct.c_int),
    ]


class Report(ct.Structure):
    _fields_ = [
        ("outer", ct.c_int64), ("newton", ct.c_int64), ("cg", ct.c_int64),
        ("sinkhorn", ct.c_int64), ("backtracks", ct.c_int64), ("stop_tests", ct.c_int64),
        ("grad_norm", ct.c_double), ("primal", ct.c_double), ("dual", ct.c_double),
        ("rel_gap", ct.c_double), ("kkt", ct.c_double), ("dphi", ct.c_double),
        ("marg_l1", ct.c_double), ("status", ct.c_int),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def _declare(L):
    i64, dbl, vp, i32 = ct.c_int64, ct.c_double, ct.c_void_p, ct.c_int
    L.orc_quantum.restype = dbl
    L.orc_quantum.argtypes = [dbl]
    L.orc_cost_max.restype = dbl
    L.orc_cost_max.argtypes = [i64, i64, vp, i32, i64]
    L.orc_center_quantum.restype = dbl
    L.orc_center_quantum.argtypes = [i64, _dp, _dp, dbl, i64, dbl]
    L.orc_make_w.restype = None
    L.orc_make_w.argtypes = [i64, _dp, _dp, dbl, dbl, _dp, _dp]
    L.orc_eval.restype = ct.c_int
    L.orc_eval.argtypes = [i64, i64, vp, i32, i64, i64, dbl, dbl, _dp, _dp, _dp, _dp, _dp, _dp,
                           _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_trial.restype = ct.c_int
    L.orc_trial.argtypes = [i64, i64, vp, i32, i64, i64, dbl, dbl, _dp, _dp, _dp, _dp, _dp, _dp,
                            dbl, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_sparsify.restype = ct.c_int64
    L.orc_sparsify.argtypes = [i64, i64, vp, i32, i64, i64, dbl, _dp, _dp, _dp, _dp, _dp, dbl,
                               i64, i64, _i64p, _i32p, _dp, _dp]
    L.orc_hvp.restype = None
    L.orc_hvp.argtypes = [i64, i64, _i64p, _i32p, _dp, _dp, _dp, dbl, dbl, _dp, _dp]
    L.orc_cg.restype = ct.c_int
    L.orc_cg.argtypes = [i64, i64, _i64p, _i32p, _dp, _dp, _dp, dbl, dbl, _dp, dbl, i32, _dp]
    L.orc_stop.restype = ct.c_int
    L.orc_stop.argtypes = [i64, i64, vp, i32, i64, i64, dbl, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                           _dp, _dp]
    L.orc_sinkhorn_step.restype = ct.c_int
    L.orc_sinkhorn_step.argtypes = [i64, i64, vp, i32, i64, i64, dbl, dbl, _dp, _dp, _dp, _dp,
                                    _dp, _dp, _dp, _dp]
    L.orc_outer_update.restype = None
    L.orc_outer_update.argtypes = [i64, i64, dbl, dbl, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_default_options.restype = None
    L.orc_default_options.argtypes = [ct.POINTER(Options)]
    L.orc_plain_eval.restype = ct.c_int
    L.orc_plain_eval.argtypes = [i64, i64, vp, i32, i64, i64, dbl, _dp, _dp, _dp, _dp, _dp, _dp,
                                 _dp, _dp, _dp, _dp]
    L.orc_plain_sparsify.restype = ct.c_int64
    L.orc_plain_sparsify.argtypes = [i64, i64, vp, i32, i64, i64, dbl, _dp, _dp, _dp, dbl, i64,
                                     i64, _i64p, _i32p, _dp, _dp]
    L.orc_plain_stop.restype = ct.c_int
    L.orc_plain_stop.argtypes = [i64, i64, vp, i32, i64, i64, dbl, _dp, _dp, _dp, _dp, _dp, _dp,
                                 _dp, _dp, _dp, _dp]
    L.orc_round.restype = None
    L.orc_round.argtypes = [i64, i64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
    L.orc_solve.restype = ct.c_int
    L.orc_solve.argtypes = [i64, i64, vp, i32, i64, _dp, _dp, dbl, ct.POINTER(Options), _dp, _dp,
                            _dp, _i64p, _dp, ct.POINTER(Report), _dp, i64]


def _p(x):
    if x is None:
        return None
    assert x.flags.c_contiguous
    if x.dtype == np.float64:
        return x.ctypes.data_as(_dp)
    if x.dtype == np.int64:
        return x.ctypes.data_as(_i64p)
    if x.dtype == np.int32:
        return x.ctypes.data_as(_i32p)
    raise TypeError(x.dtype)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _cost(C):
    C = np.ascontiguousarray(C)
    if C.dtype == np.float64:
        return C, 0
    if C.dtype == np.float32:
        return C, 1
    raise TypeError(C.dtype)


@dataclass
class EvalResult:
    M: np.ndarray
    S: np.ndarray
    c: np.ndarray
    g: np.ndarray
    L: float
    plan: np.ndarray | None
    q: float
    w: np.ndarray
    wl: np.ndarray | None = None

    @property
    def lse(self):
        return self.M + np.log(self.S)


def default_state(a, b):
    """Prox centre X^0 = a b^T: r = log a, s = log b, k = 0 (Algorithm 2 input)."""
    return np.log(_f64(a)), np.log(_f64(b)), 0


def cost_max(C):
    C, kind = _cost(C)
    return lib().orc_cost_max(C.shape[0], C.shape[1], C.ctypes.data, kind, C.shape[1])


def center_quantum(C, s, gamma, eta, k):
    """Grid spacing of an outer iteration (bound max|s + gamma/eta| + sigma max|C|)."""
    s, gamma = _f64(s), _f64(gamma)
    return lib().orc_center_quantum(len(s), _p(s), _p(gamma), float(eta), int(k), cost_max(C))


def make_w(s, gamma, eta, q, split=True):
    """Two-level potentials (w, wl) with w + wl = s + gamma/eta, w on the grid of spacing q
    (split=False: w = grid(s + gamma/eta) and wl = None)."""
    s, gamma = _f64(s), _f64(gamma)
    w = np.empty(len(s))
    wl = np.empty(len(s)) if split else None
    lib().orc_make_w(len(s), _p(s), _p(gamma), float(eta), float(q), _p(w), _p(wl))
    return w, wl


def _wq(C, b, eta, gamma, s, k, q, split):
    s = np.log(_f64(b)) if s is None else _f64(s)
    gamma = _f64(gamma)
    if q is None:
        q = center_quantum(C, s, gamma, eta, k)
    w, wl = make_w(s, gamma, eta, q, split)
    return s, w, wl, q


def eval_pass(C, a, b, eta, gamma, r=None, s=None, k=0, want_plan=False, q=None,
              split=True) -> EvalResult:
    """Eval at w = s + gamma/eta held as two-level potentials (split=False: on the grid)."""
    C, kind = _cost(C)
    m, n = C.shape
    a, b, gamma = _f64(a), _f64(b), _f64(gamma)
    r = np.log(a) if r is None else _f64(r)
    s, w, wl, q = _wq(C, b, eta, gamma, s, k, q, split)
    M, S, c, g = np.empty(m), np.empty(m), np.empty(n), np.empty(n)
    L = ct.c_double()
    plan = np.empty((m, n)) if want_plan else None
    rc = lib().orc_eval(m, n, C.ctypes.data, kind, n, k, eta, q, _p(w), _p(wl), _p(r), _p(gamma),
                        _p(a), _p(b), _p(M), _p(S), _p(c), _p(g), ct.byref(L), _p(plan))
    assert rc == 0, rc
    return EvalResult(M, S, c, g, L.value, plan, q, w, wl)


def trial_pass(C, a, b, eta, gamma, M, Delta, t, s=None, k=0, q=None, split=True):
    """Armijo trial at w + t*Delta/eta (split=False: the step on the grid) from the row state
    M of w.  Returns (dL, M_new, S_new, c_new, g_new)."""
    C, kind = _cost(C)
    m, n = C.shape
    a, b, M, Delta = map(_f64, (a, b, M, Delta))
    s, w, wl, q = _wq(C, b, eta, gamma, s, k, q, split)
    Mn, Sn, cn, gn = np.empty(m), np.empty(m), np.empty(n), np.empty(n)
    dL = ct.c_double()
    rc = lib().orc_trial(m, n, C.ctypes.data, kind, n, k, eta, q, _p(w), _p(wl), _p(a), _p(b),
                         _p(M), _p(Delta), float(t), ct.byref(dL), None, _p(Mn), _p(Sn), _p(cn),
                         _p(gn))
    assert rc == 0, rc
    return dL.value, Mn, Sn, cn, gn


def sinkhorn_step(C, a, b, eta, gamma, M, S, c, s, k=0, q=None):
    """One Sinkhorn gamma-step (Algorithm 2, steps 3-4) from the eval (M, S, c) at gamma,
    centred; log c in the log domain where a column sum underflows."""
    C, kind = _cost(C)
    m, n = C.shape
    a, b, gamma, M, S, c, s = map(_f64, (a, b, gamma, M, S, c, s))
    if q is None:
        q = center_quantum(C, s, gamma, eta, k)
    out = np.empty(n)
    rc = lib().orc_sinkhorn_step(m, n, C.ctypes.data, kind, n, int(k), float(eta), float(q),
                                 _p(s), _p(gamma), _p(a), _p(b), _p(M), _p(S), _p(c), _p(out))
    assert rc == 0
    return out


def outer_update(a, eta, gamma, M, S, s, q):
    """The next centre (r, s) from the row state (M, S) at gamma (Algorithm 2, step 13)."""
    a, gamma, M, S, s = map(_f64, (a, gamma, M, S, s))
    m, n = len(a), len(s)
    r_out, s_out = np.empty(m), np.empty(n)
    lib().orc_outer_update(m, n, float(eta), float(q), _p(a), _p(M), _p(S), _p(s), _p(gamma),
                           _p(r_out), _p(s_out))
    return r_out, s_out


@dataclass
class CSR:
    m: int
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    d: np.ndarray
    istar: int

    @property
    def nnz(self):
        return int(self.row_ptr[-1])

    def dense(self):
        P = np.zeros((self.m, self.n))
        for i in range(self.m):
            sl = slice(self.row_ptr[i], self.row_ptr[i + 1])
            P[i, self.col[sl]] = self.val[sl]
        return P


def istar_of(a):
    """i* = argmax a, lowest index on ties (Algorithm 1 input)."""
    return int(np.argmax(np.asarray(a)))


def sparsify(C, a, eta, gamma, M, S, rho, s, k=0, istar=None, q=None, split=True) -> CSR:
    """Algorithm 1 from the row state (M, S) at (s, gamma, k)."""
    C, kind = _cost(C)
    m, n = C.shape
    a, M, S = map(_f64, (a, M, S))
    s = _f64(s)
    gamma = _f64(gamma)
    if q is None:
        q = center_quantum(C, s, gamma, eta, k)
    w, wl = make_w(s, gamma, eta, q, split)
    istar = istar_of(a) if istar is None else int(istar)
    row_ptr = np.empty(m + 1, dtype=np.int64)
    need = lib().orc_sparsify(m, n, C.ctypes.data, kind, n, k, eta, _p(w), _p(wl), _p(a), _p(M),
                              _p(S), float(rho), istar, 0, _p(row_ptr), None, None, None)
    nnz = -need - 1
    col = np.empty(max(nnz, 1), dtype=np.int32)
    val = np.empty(max(nnz, 1))
    d = np.empty(n)
    got = lib().orc_sparsify(m, n, C.ctypes.data, kind, n, k, eta, _p(w), _p(wl), _p(a), _p(M),
                             _p(S), float(rho), istar, nnz, _p(row_ptr), _p(col), _p(val), _p(d))
    assert got == nnz
    return CSR(m, n, row_ptr, col[:nnz], val[:nnz], d, istar)


def hvp(csr: CSR, a, eta, shift, v):
    v = _f64(v)
    y = np.empty(csr.n)
    lib().orc_hvp(csr.m, csr.n, _p(csr.row_ptr), _p(np.ascontiguousarray(csr.col)),
                  _p(np.ascontiguousarray(csr.val)), _p(csr.d), _p(_f64(a)), float(eta),
                  float(shift), _p(v), _p(y))
    return y


def cg(csr: CSR, a, eta, shift, rhs, tol, maxit):
    x = np.empty(csr.n)
    it = lib().orc_cg(csr.m, csr.n, _p(csr.row_ptr), _p(np.ascontiguousarray(csr.col)),
                      _p(np.ascontiguousarray(csr.val)), _p(csr.d), _p(_f64(a)), float(eta),
                      float(shift), _p(_f64(rhs)), float(tol), int(maxit), _p(x))
    return x, it


STOP_FIELDS = ("dphi", "primal", "dual", "cx", "kkt", "xhat_min", "er1", "xu", "dual_gamma",
               "dual_psi")


def stop_pass(C, a, b, eta, gamma, M, S, s=None, k=0, want_xhat=False, q=None, split=True):
    """Rounding, D_phi and certificate for the plan of the row state (M, S) at w.
    The certificate's dual is gamma as given."""
    C, kind = _cost(C)
    m, n = C.shape
    a, b, gamma, M, S = map(_f64, (a, b, gamma, M, S))
    s, w, wl, q = _wq(C, b, eta, gamma, s, k, q, split)
    out = np.empty(10)
    xhat = np.empty((m, n)) if want_xhat else None
    rc = lib().orc_stop(m, n, C.ctypes.data, kind, n, k, eta, _p(w), _p(wl), _p(gamma), _p(a),
                        _p(b), _p(M), _p(S), _p(out), _p(xhat))
    assert rc == 0
    res = dict(zip(STOP_FIELDS, out.tolist()))
    if want_xhat:
        res["xhat"] = xhat
    return res


def default_options(**kw) -> Options:
    o = Options()
    lib().orc_default_options(ct.byref(o))
    for key, v in kw.items():
        if not hasattr(o, key):
            raise KeyError(key)
        setattr(o, key, v)
    return o


def solve(C, a, b, eta, gamma0=None, options: Options | None = None, want_plan=False,
          state=None, trace_cap=0):
    """Full IBSN (Algorithm 2).  Returns dict with gamma, report, plan, r, s, k, trace."""
    C, kind = _cost(C)
    m, n = C.shape
    a, b = _f64(a), _f64(b)
    gamma = np.zeros(n) if gamma0 is None else _f64(gamma0).copy()
    if state is not None:
        r, s, k = _f64(state[0]).copy(), _f64(state[1]).copy(), int(state[2])
    else:
        r, s, k = np.empty(m), np.empty(n), 0
    kk = ct.c_int64(k)
    plan = np.empty((m, n)) if want_plan else None
    rep = Report()
    trace = np.zeros((trace_cap, 6)) if trace_cap else None
    opt = options if options is not None else default_options()
    status = lib().orc_solve(m, n, C.ctypes.data, kind, n, _p(a), _p(b), float(eta),
                             ct.byref(opt), _p(gamma), _p(r), _p(s), ct.byref(kk), _p(plan),
                             ct.byref(rep), _p(trace), trace_cap)
    out = dict(status=status, gamma=gamma, report=rep.as_dict(), plan=plan, r=r, s=s, k=kk.value)
    if trace is not None:
        out["trace"] = trace[: min(trace_cap, rep.outer)]
    return out


# ---------------------------------------------------------------------------
# Plain reference passes: the definitions with no potential grid (w = s + gamma/eta,
# theta = fma(-sigma, C, w), M = max theta, S = sum exp(theta - M), P = exp(theta - M)/S).
# ---------------------------------------------------------------------------
@dataclass
class PlainEval:
    lse: np.ndarray
    c: np.ndarray
    g: np.ndarray
    L: float | None
    plan: np.ndarray | None


def plain_eval(C, a, b, eta, gamma, r=None, s=None, k=0, want_plan=False) -> PlainEval:
    """Eqs. (5)-(8) at (k, s, gamma) with the implicit centre; r = log a, s = log b default."""
    C, kind = _cost(C)
    m, n = C.shape
    a, b, gamma = _f64(a), _f64(b), _f64(gamma)
    r = np.log(a) if r is None else _f64(r)
    s = np.log(b) if s is None else _f64(s)
    lse, c, g = np.empty(m), np.empty(n), np.empty(n)
    L = ct.c_double()
    plan = np.empty((m, n)) if want_plan else None
    rc = lib().orc_plain_eval(m, n, C.ctypes.data, kind, n, int(k), float(eta), _p(r), _p(s),
                              _p(gamma), _p(a), _p(b), _p(lse), _p(c), _p(g), ct.byref(L),
                              _p(plan))
    assert rc == 0, rc
    return PlainEval(lse, c, g, L.value, plan)


def plain_sparsify(C, a, eta, gamma, rho, s, k=0, istar=None) -> CSR:
    """Algorithm 1 on the plain P at (k, s, gamma)."""
    C, kind = _cost(C)
    m, n = C.shape
    a, s, gamma = _f64(a), _f64(s), _f64(gamma)
    istar = istar_of(a) if istar is None else int(istar)
    row_ptr = np.empty(m + 1, dtype=np.int64)
    need = lib().orc_plain_sparsify(m, n, C.ctypes.data, kind, n, int(k), float(eta), _p(s),
                                    _p(gamma), _p(a), float(rho), istar, 0, _p(row_ptr), None,
                                    None, None)
    nnz = -need - 1
    col = np.empty(max(nnz, 1), dtype=np.int32)
    val = np.empty(max(nnz, 1))
    d = np.empty(n)
    got = lib().orc_plain_sparsify(m, n, C.ctypes.data, kind, n, int(k), float(eta), _p(s),
                                   _p(gamma), _p(a), float(rho), istar, nnz, _p(row_ptr),
                                   _p(col), _p(val), _p(d))
    assert got == nnz
    return CSR(m, n, row_ptr, col[:nnz], val[:nnz], d, istar)


def plain_stop(C, a, b, eta, gamma, s, k=0, want_xhat=False, want_steps=False):
    """Algorithm 3, D_phi and the certificate for the plain plan at (k, s, gamma).
    want_steps: also return Algorithm 3's z, y, e_r, e_c."""
    C, kind = _cost(C)
    m, n = C.shape
    a, b, gamma, s = map(_f64, (a, b, gamma, s))
    out = np.empty(10)
    xhat = np.empty((m, n)) if want_xhat else None
    z, er = (np.empty(m), np.empty(m)) if want_steps else (None, None)
    y, ec = (np.empty(n), np.empty(n)) if want_steps else (None, None)
    rc = lib().orc_plain_stop(m, n, C.ctypes.data, kind, n, int(k), float(eta), _p(s),
                              _p(gamma), _p(a), _p(b), _p(out), _p(xhat), _p(z), _p(y), _p(er),
                              _p(ec))
    assert rc == 0
    res = dict(zip(STOP_FIELDS, out.tolist()))
    if want_xhat:
        res["xhat"] = xhat
    if want_steps:
        res.update(z=z, y=y, er=er, ec=ec)
    return res


def round_plan(X, a, b):
    """Algorithm 3 on a nonnegative matrix X: returns (xhat, z, y, e_r, e_c)."""
    X, a, b = map(_f64, (X, a, b))
    m, n = X.shape
    xhat, z, y, er, ec = np.empty((m, n)), np.empty(m), np.empty(n), np.empty(m), np.empty(n)
    lib().orc_round(m, n, _p(X), _p(a), _p(b), _p(xhat), _p(z), _p(y), _p(er), _p(ec))
    return xhat, z, y, er, ec
