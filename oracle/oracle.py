"""FP64 CPU oracle for generalized min-marginal averaging -- ctypes front end.

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the GPU
library.  The arithmetic lives in ``dd_oracle.c``; this file only marshals
numpy arrays.  See that file's header for the readings of the paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, E_ARG, E_INFEASIBLE, E_FORCED = 0, -1, -2, -3


class OracleError(RuntimeError):
    pass


def build(force=True):
    """Compile dd_oracle.c with gcc (OpenMP) into oracle/liboracle.so."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unused-function",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = C.CDLL(_LIB)
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def _prob_args(p):
    rp = np.ascontiguousarray(p.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(p.col, dtype=np.int32)
    coef = np.ascontiguousarray(p.coef, dtype=np.int32)
    sense = np.ascontiguousarray(p.sense, dtype=np.int8)
    rhs = np.ascontiguousarray(p.rhs, dtype=np.int64)
    keep = (rp, col, coef, sense, rhs)
    return keep, [_p(rp, C.c_int64), _p(col, C.c_int32), _p(coef, C.c_int32), _p(sense, C.c_int8),
                  _p(rhs, C.c_int64)]


def _check(st, what):
    if st != OK:
        raise OracleError(f"{what}: oracle status {st}")


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None and a.shape != (n,):
        raise ValueError(f"expected shape ({n},), got {a.shape}")
    return a


def softmax_alpha(prob, alpha_hat):
    """alpha_{i.} = softmax over J_i of the logits alpha_hat_{i.} (Alg. 3, transform line)."""
    ah = _f64(alpha_hat, prob.nnz)
    var = prob.col.astype(np.int64)
    mx = np.full(prob.n, -np.inf)
    np.maximum.at(mx, var, ah)
    z = np.exp(ah - mx[var])
    den = np.zeros(prob.n)
    np.add.at(den, var, z)
    return z / den[var]


def softmax_alpha_vjp(prob, alpha, d_alpha):
    """d alpha_hat_e = alpha_e (d alpha_e - sum_{k in J_i} alpha_k d alpha_k)."""
    var = prob.col.astype(np.int64)
    s = np.zeros(prob.n)
    np.add.at(s, var, alpha * d_alpha)
    return alpha * (d_alpha - s[var])


def init_lambda(prob):
    lib = _load()
    lam = np.empty(prob.nnz)
    c = _f64(prob.c, prob.n)
    col = np.ascontiguousarray(prob.col, dtype=np.int32)
    _check(lib.orc_init_lambda(C.c_int(prob.n), _p(c, C.c_double), C.c_int64(prob.nnz), _p(col, C.c_int32),
                               _p(lam, C.c_double)), "init_lambda")
    return lam


def run_pass(prob, omega, alpha, lam, M, direction, literal=False, threads=0):
    """One pass in place (direction 0 forward, 1 backward)."""
    lib = _load()
    keep, pa = _prob_args(prob)
    om, al = _f64(omega, prob.nnz), _f64(alpha, prob.nnz)
    assert lam.dtype == np.float64 and M.dtype == np.float64 and lam.flags.c_contiguous and M.flags.c_contiguous
    _check(lib.orc_pass(C.c_int(prob.n), C.c_int(prob.m), *pa, _p(om, C.c_double), _p(al, C.c_double),
                        C.c_int(direction), C.c_int(int(literal)), _p(lam, C.c_double), _p(M, C.c_double),
                        C.c_int(threads)), "pass")
    return lam, M


def run(prob, omega, alpha, T, lam=None, M=None, literal=False, threads=0):
    """T iterations of Alg. 1 from (lam, M) (default: lambda = c/|J|, M = 0). Returns (lam, M)."""
    lib = _load()
    keep, pa = _prob_args(prob)
    om, al = _f64(omega, prob.nnz), _f64(alpha, prob.nnz)
    lam = init_lambda(prob) if lam is None else np.array(lam, dtype=np.float64)
    M = np.zeros(prob.nnz) if M is None else np.array(M, dtype=np.float64)
    _check(lib.orc_run(C.c_int(prob.n), C.c_int(prob.m), *pa, _p(om, C.c_double), _p(al, C.c_double), C.c_int(T),
                       C.c_int(int(literal)), _p(lam, C.c_double), _p(M, C.c_double), C.c_int(threads)), "run")
    return lam, M


def rows_pass(prob, omega, alpha, S_edge, lam, direction, literal=False, threads=0):
    """One pass over every row of prob with the deferred sums given per edge. Returns (lam_out, M_out)."""
    lib = _load()
    keep, pa = _prob_args(prob)
    om, al, se = _f64(omega, prob.nnz), _f64(alpha, prob.nnz), _f64(S_edge, prob.nnz)
    lam = np.array(lam, dtype=np.float64)
    M = np.zeros(prob.nnz)
    _check(lib.orc_rows_pass(C.c_int(prob.m), *pa, _p(om, C.c_double), _p(al, C.c_double), _p(se, C.c_double),
                             C.c_int(direction), C.c_int(int(literal)), _p(lam, C.c_double), _p(M, C.c_double),
                             C.c_int(threads)), "rows_pass")
    return lam, M


def energies(prob, lam, threads=0):
    lib = _load()
    keep, pa = _prob_args(prob)
    lam = _f64(lam, prob.nnz)
    Ej = np.empty(prob.m)
    _check(lib.orc_energies(C.c_int(prob.m), *pa, _p(lam, C.c_double), _p(Ej, C.c_double), C.c_int(threads)),
           "energies")
    return Ej


def lower_bound(prob, alpha, lam, M, threads=0):
    """Returns (LB at the flushed multipliers, D_L, lambda_bar)."""
    lib = _load()
    keep, pa = _prob_args(prob)
    c = _f64(prob.c, prob.n)
    al, lam, M = _f64(alpha, prob.nnz), _f64(lam, prob.nnz), _f64(M, prob.nnz)
    lb, dl = C.c_double(), C.c_double()
    lbar = np.empty(prob.nnz)
    _check(lib.orc_lower_bound(C.c_int(prob.n), C.c_int(prob.m), *pa, _p(c, C.c_double), _p(al, C.c_double),
                               _p(lam, C.c_double), _p(M, C.c_double), C.byref(lb), C.byref(dl),
                               _p(lbar, C.c_double), C.c_int(threads)), "lower_bound")
    return lb.value, dl.value, lbar


def flushed(prob, alpha, lam, M):
    """lambda_bar = lambda + alpha * S with S_i = sum_{k in J_i} M_ik."""
    S = np.zeros(prob.n)
    np.add.at(S, prob.col.astype(np.int64), M)
    return lam + alpha * S[prob.col]


def min_marginals(prob, lam, threads=0):
    lib = _load()
    keep, pa = _prob_args(prob)
    lam = _f64(lam, prob.nnz)
    m0, m1 = np.empty(prob.nnz), np.empty(prob.nnz)
    _check(lib.orc_min_marginals(C.c_int(prob.m), *pa, _p(lam, C.c_double), _p(m0, C.c_double), _p(m1, C.c_double),
                                 C.c_int(threads)), "min_marginals")
    return m0, m1


def smoothed(prob, lam, tau, threads=0):
    """(E_tau^j [m], p [E]): smoothed energies -tau log sum_{x in X_j} exp(-<lambda, x>/tau) and their
    gradient, the marginals P(x_l = 1) of the Gibbs distribution on each X_j."""
    lib = _load()
    keep, pa = _prob_args(prob)
    lam = _f64(lam, prob.nnz)
    E = np.empty(max(prob.m, 1))
    pm = np.empty(max(prob.nnz, 1))
    _check(lib.orc_smoothed(C.c_int(prob.m), *pa, _p(lam, C.c_double), C.c_double(tau), _p(E, C.c_double),
                            _p(pm, C.c_double), C.c_int(threads)), "smoothed")
    return E[:prob.m], pm[:prob.nnz]


def argmin(prob, lam, threads=0, with_gap=False):
    """Minimizing assignment of every row; with_gap also returns each row's smallest relative
    gap between the two options of a decision (tiny gap: the minimizer is not unique up to rounding)."""
    lib = _load()
    keep, pa = _prob_args(prob)
    lam = _f64(lam, prob.nnz)
    x = np.empty(prob.nnz, dtype=np.int8)
    gap = np.full(max(prob.m, 1), np.inf)
    _check(lib.orc_argmin(C.c_int(prob.m), *pa, _p(lam, C.c_double), _p(x, C.c_int8), _p(gap, C.c_double),
                          C.c_int(threads)), "argmin")
    return (x, gap[:prob.m]) if with_gap else x


def pass_vjp(prob, omega, alpha, direction, lam_in, M_in, dlam_out, dM_out, threads=0, with_gap=False):
    """Alg. 2 over one pass. Returns (dlam_in, dM_in, d_alpha, d_omega) [+ per-row minimizer gap]."""
    lib = _load()
    keep, pa = _prob_args(prob)
    E = prob.nnz
    om, al = _f64(omega, E), _f64(alpha, E)
    li, mi, dlo, dmo = _f64(lam_in, E), _f64(M_in, E), _f64(dlam_out, E), _f64(dM_out, E)
    dli, dmi, da, dw = np.empty(E), np.empty(E), np.zeros(E), np.zeros(E)
    gap = np.full(max(prob.m, 1), np.inf)
    _check(lib.orc_pass_vjp(C.c_int(prob.n), C.c_int(prob.m), *pa, _p(om, C.c_double), _p(al, C.c_double),
                            C.c_int(direction), _p(li, C.c_double), _p(mi, C.c_double), _p(dlo, C.c_double),
                            _p(dmo, C.c_double), _p(dli, C.c_double), _p(dmi, C.c_double), _p(da, C.c_double),
                            _p(dw, C.c_double), _p(gap, C.c_double), C.c_int(threads)), "pass_vjp")
    return (dli, dmi, da, dw, gap[:prob.m]) if with_gap else (dli, dmi, da, dw)


def unrolled_grad(prob, omega, alpha, T, threads=0, with_gap=False, lam0=None, M0=None):
    """LB after T iterations and its gradient w.r.t. (omega, alpha, c) [+ the smallest relative gap
    of any minimizer decision taken on the way].  With lam0/M0 the iterations start from that state
    instead of lambda = c/|J_i|, M = 0, and the third gradient is (d_lam0, d_M0) instead of d_c."""
    lib = _load()
    keep, pa = _prob_args(prob)
    E = prob.nnz
    c = _f64(prob.c, prob.n)
    om, al = _f64(omega, E), _f64(alpha, E)
    lb = C.c_double()
    dw, da, dc = np.empty(E), np.empty(E), np.empty(prob.n)
    gap = C.c_double()
    if lam0 is None:
        _check(lib.orc_unrolled_grad(C.c_int(prob.n), C.c_int(prob.m), *pa, _p(c, C.c_double), _p(om, C.c_double),
                                     _p(al, C.c_double), C.c_int(T), None, None, C.byref(lb), _p(dw, C.c_double),
                                     _p(da, C.c_double), _p(dc, C.c_double), None, None, C.byref(gap),
                                     C.c_int(threads)), "unrolled_grad")
        out = (lb.value, dw, da, dc)
    else:
        l0, m0 = _f64(lam0, E), _f64(M0, E)
        dl0, dm0 = np.empty(E), np.empty(E)
        _check(lib.orc_unrolled_grad(C.c_int(prob.n), C.c_int(prob.m), *pa, _p(c, C.c_double), _p(om, C.c_double),
                                     _p(al, C.c_double), C.c_int(T), _p(l0, C.c_double), _p(m0, C.c_double),
                                     C.byref(lb), _p(dw, C.c_double), _p(da, C.c_double), None,
                                     _p(dl0, C.c_double), _p(dm0, C.c_double), C.byref(gap), C.c_int(threads)),
               "unrolled_grad")
        out = (lb.value, dw, da, (dl0, dm0))
    return out + (gap.value,) if with_gap else out


def center(prob, x):
    """x_e minus the mean of x over the edges of e's variable (the feasibility projection of the
    non-parametric update, eq. 2, and of the theta transform of Alg. 3)."""
    x = _f64(x, prob.nnz)
    var = prob.col.astype(np.int64)
    s = np.zeros(prob.n)
    np.add.at(s, var, x)
    deg = np.bincount(var, minlength=prob.n).astype(np.float64)
    return x - s[var] / deg[var]


def nonparam_update(prob, lam, theta_hat):
    """Eq. 2: lambda_ij + theta_hat_ij - (1/|J_i|) sum_{k in J_i} theta_hat_ik."""
    return _f64(lam, prob.nnz) + center(prob, theta_hat)


def sigmoid(x):
    x = np.asarray(x, dtype=np.float64)
    return 1.0 / (1.0 + np.exp(-x))


def param_transform(prob, omega_hat, alpha_hat, theta_hat):
    """Alg. 3's output transforms: omega = sigmoid, alpha = softmax over J_i, theta centred over J_i."""
    return sigmoid(omega_hat), softmax_alpha(prob, alpha_hat), center(prob, theta_hat)


def param_transform_vjp(prob, omega, alpha, d_omega, d_alpha, d_theta):
    """Adjoints of param_transform's inputs (the centring is symmetric and idempotent)."""
    return (_f64(d_omega) * omega * (1.0 - omega), softmax_alpha_vjp(prob, alpha, _f64(d_alpha)),
            center(prob, d_theta))


def lb_after(prob, omega, alpha, T, c=None, threads=0):
    """LB after T iterations from the default start, optionally with other costs c (for finite differences)."""
    if c is not None:
        import dataclasses
        prob = dataclasses.replace(prob, c=np.asarray(c, dtype=np.float64))
    lam, M = run(prob, omega, alpha, T, threads=threads)
    return lower_bound(prob, alpha, lam, M, threads=threads)[0]


def threads(n=0):
    """Number of OpenMP threads the oracle's loops use (n > 0 sets it)."""
    return int(_load().orc_threads(C.c_int(n)))
