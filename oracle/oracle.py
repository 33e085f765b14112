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
# ORACLE_SANITIZE=1: the AddressSanitizer / UndefinedBehaviorSanitizer build (CPU checks)
_SAN = os.environ.get("ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SAN else "liboracle.so")
_SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
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
                           *(_SAN_FLAGS if _SAN else []), "-o", tmp, _SRC, "-lm"])
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


def _gaps(g, m):
    """Per-row (relative, absolute) smallest decision gaps from the oracle's [2 m] layout."""
    g = g[:2 * m].reshape(m, 2)
    return g[:, 0].copy(), g[:, 1].copy()


def argmin(prob, lam, threads=0, with_gap=False, row_gaps=False):
    """Minimizing assignment of every row.  with_gap also returns each row's smallest relative gap
    between the two options of a decision (tiny gap: the minimizer is not unique up to rounding);
    row_gaps returns (x, relative gaps, absolute gaps) instead."""
    lib = _load()
    keep, pa = _prob_args(prob)
    lam = _f64(lam, prob.nnz)
    x = np.empty(prob.nnz, dtype=np.int8)
    gap = np.full(2 * max(prob.m, 1), np.inf)
    _check(lib.orc_argmin(C.c_int(prob.m), *pa, _p(lam, C.c_double), _p(x, C.c_int8), _p(gap, C.c_double),
                          C.c_int(threads)), "argmin")
    rel, ab = _gaps(gap, prob.m)
    if row_gaps:
        return x, rel, ab
    return (x, rel) if with_gap else x


def _taint_args(E, row_tol, t_dlo, t_dmo, nrow):
    if row_tol is None:
        return None, None, None, None, ()
    tol = _f64(row_tol, nrow)
    keep = []
    ptrs = []
    for t in (t_dlo, t_dmo):
        if t is None:
            ptrs.append(None)
        else:
            a = np.ascontiguousarray(t, dtype=np.float64)
            assert a.shape == (E,)
            keep.append(a)
            ptrs.append(_p(a, C.c_double))
    out = np.zeros(5 * max(E, 1), dtype=np.float64)
    return tol, ptrs[0], ptrs[1], out, keep


def pass_vjp(prob, omega, alpha, direction, lam_in, M_in, dlam_out, dM_out, threads=0, with_gap=False,
             row_gaps=False, row_tol=None, t_dlo=None, t_dmo=None):
    """Alg. 2 over one pass. Returns (dlam_in, dM_in, d_alpha, d_omega) [+ per-row relative gaps with
    with_gap, or + (relative, absolute) per-row gaps with row_gaps].  With row_tol ([m] absolute
    decision tolerance per row; t_dlo / t_dmo optionally bound how far the adjoints of the outputs
    may be off) a last item is appended: the flip bounds of dlam_in, dM_in, d_alpha and d_omega --
    how far flips of near-tie decisions (options within the row's tolerance) can move each entry; 0
    where the entry is determined -- and, as a fifth row, d_omega's rounding scale |Mt| s_j ([5, E])."""
    lib = _load()
    keep, pa = _prob_args(prob)
    E = prob.nnz
    om, al = _f64(omega, E), _f64(alpha, E)
    li, mi, dlo, dmo = _f64(lam_in, E), _f64(M_in, E), _f64(dlam_out, E), _f64(dM_out, E)
    dli, dmi, da, dw = np.empty(E), np.empty(E), np.zeros(E), np.zeros(E)
    gap = np.full(2 * max(prob.m, 1), np.inf)
    tol, pdlo, pdmo, tout, keep_t = _taint_args(E, row_tol, t_dlo, t_dmo, prob.m)
    _check(lib.orc_pass_vjp(C.c_int(prob.n), C.c_int(prob.m), *pa, _p(om, C.c_double), _p(al, C.c_double),
                            C.c_int(direction), _p(li, C.c_double), _p(mi, C.c_double), _p(dlo, C.c_double),
                            _p(dmo, C.c_double), _p(dli, C.c_double), _p(dmi, C.c_double), _p(da, C.c_double),
                            _p(dw, C.c_double), _p(gap, C.c_double), None if tol is None else _p(tol, C.c_double),
                            pdlo, pdmo, None if tout is None else _p(tout, C.c_double), C.c_int(threads)), "pass_vjp")
    rel, ab = _gaps(gap, prob.m)
    out = (dli, dmi, da, dw) + ((rel, ab) if row_gaps else (rel,) if with_gap else ())
    return out + ((tout[:5 * E].reshape(5, E),) if tout is not None else ())


def rows_pass_vjp(prob, omega, alpha, S_edge, direction, lam_in, dlam_out, dM_out, threads=0, row_tol=None,
                  t_dlo=None, t_dmo=None):
    """Alg. 2 over one pass of every row of prob with the deferred sums given per edge (prob may be
    a subset of a larger program's rows: given S they are independent).  Returns (dlam_in, gS,
    d_alpha, d_omega, relative gaps, absolute gaps), gS being each edge's share
    dlambda_new * alpha of dS_i = d M_in_ik; with row_tol (as pass_vjp) the flip bounds of dlam_in,
    gS, d_alpha and d_omega and d_omega's rounding scale ([5, E]) are appended."""
    lib = _load()
    keep, pa = _prob_args(prob)
    E = prob.nnz
    om, al, se = _f64(omega, E), _f64(alpha, E), _f64(S_edge, E)
    li, dlo, dmo = _f64(lam_in, E), _f64(dlam_out, E), _f64(dM_out, E)
    dli, gs, da, dw = np.empty(E), np.empty(E), np.zeros(E), np.zeros(E)
    gap = np.full(2 * max(prob.m, 1), np.inf)
    tol, pdlo, pdmo, tout, keep_t = _taint_args(E, row_tol, t_dlo, t_dmo, prob.m)
    _check(lib.orc_rows_pass_vjp(C.c_int(prob.m), *pa, _p(om, C.c_double), _p(al, C.c_double), _p(se, C.c_double),
                                 C.c_int(direction), _p(li, C.c_double), _p(dlo, C.c_double), _p(dmo, C.c_double),
                                 _p(dli, C.c_double), _p(gs, C.c_double), _p(da, C.c_double), _p(dw, C.c_double),
                                 _p(gap, C.c_double), None if tol is None else _p(tol, C.c_double), pdlo, pdmo,
                                 None if tout is None else _p(tout, C.c_double), C.c_int(threads)), "rows_pass_vjp")
    out = (dli, gs, da, dw) + _gaps(gap, prob.m)
    return out + ((tout[:5 * E].reshape(5, E),) if tout is not None else ())


def unrolled_grad(prob, omega, alpha, T, threads=0, with_gap=False, lam0=None, M0=None, row_gaps=False,
                  pass_tol=None):
    """LB after T iterations and its gradient w.r.t. (omega, alpha, c) [+ the smallest relative gap
    of any minimizer decision taken on the way with with_gap, or + per-row (relative, absolute)
    smallest gaps over the trajectory with row_gaps].  With lam0/M0 the iterations start from that
    state instead of lambda = c/|J_i|, M = 0, and the third gradient is (d_lam0, d_M0) instead of d_c.
    pass_tol ([2T + 1, m]: each row's decision tolerance in pass p = 0 .. 2T-1 and in the seed, row
    2T) appends the flip bounds (how far flips of near-tie decisions can move each entry) of the
    gradients, in their order, and d_omega's rounding scale summed over the passes:
    (t_omega, t_alpha, t_c, w_scale) or (t_omega, t_alpha, (t_lam0, t_M0), w_scale)."""
    lib = _load()
    keep, pa = _prob_args(prob)
    E = prob.nnz
    c = _f64(prob.c, prob.n)
    om, al = _f64(omega, E), _f64(alpha, E)
    lb = C.c_double()
    dw, da, dc = np.empty(E), np.empty(E), np.empty(prob.n)
    gap = np.full(2 * max(prob.m, 1), np.inf)
    if pass_tol is not None:
        ptol = np.ascontiguousarray(pass_tol, dtype=np.float64)
        assert ptol.shape == (2 * T + 1, prob.m)
        taint = np.zeros(5 * E + prob.n + 1)
        tp, tt = _p(ptol, C.c_double), _p(taint, C.c_double)
    else:
        tp = tt = None
    if lam0 is None:
        _check(lib.orc_unrolled_grad(C.c_int(prob.n), C.c_int(prob.m), *pa, _p(c, C.c_double), _p(om, C.c_double),
                                     _p(al, C.c_double), C.c_int(T), None, None, C.byref(lb), _p(dw, C.c_double),
                                     _p(da, C.c_double), _p(dc, C.c_double), None, None, _p(gap, C.c_double), tp, tt,
                                     C.c_int(threads)), "unrolled_grad")
        out = (lb.value, dw, da, dc)
    else:
        l0, m0 = _f64(lam0, E), _f64(M0, E)
        dl0, dm0 = np.empty(E), np.empty(E)
        _check(lib.orc_unrolled_grad(C.c_int(prob.n), C.c_int(prob.m), *pa, _p(c, C.c_double), _p(om, C.c_double),
                                     _p(al, C.c_double), C.c_int(T), _p(l0, C.c_double), _p(m0, C.c_double),
                                     C.byref(lb), _p(dw, C.c_double), _p(da, C.c_double), None,
                                     _p(dl0, C.c_double), _p(dm0, C.c_double), _p(gap, C.c_double), tp, tt, C.c_int(threads)),
               "unrolled_grad")
        out = (lb.value, dw, da, (dl0, dm0))
    rel, ab = _gaps(gap, prob.m)
    if row_gaps:
        out = out + (rel, ab)
    elif with_gap:
        out = out + (float(rel.min()) if prob.m else np.inf,)
    if pass_tol is not None:
        t = taint
        third = t[5 * E:5 * E + prob.n] if lam0 is None else (t[2 * E:3 * E], t[3 * E:4 * E])
        out = out + ((t[:E], t[E:2 * E], third, t[4 * E:5 * E]),)
    return out


def trajectory(prob, omega, alpha, T, round_f32=False, threads=0, lam0=None, M0=None):
    """The 2T + 1 states (lambda, M) before every pass of T iterations from lambda = c/|J_i|, M = 0 (or
    from lam0, M0), and after the last.  round_f32 rounds the state to float32 after every pass (fp64
    arithmetic otherwise): the perturbation that storing the state in float32 alone makes."""
    if lam0 is None:
        lam, M = init_lambda(prob), np.zeros(prob.nnz)
    else:
        lam, M = np.array(lam0, dtype=np.float64), np.array(M0, dtype=np.float64)
    states = [(lam.copy(), M.copy())]
    for q in range(2 * T):
        run_pass(prob, omega, alpha, lam, M, q % 2, threads=threads)
        if round_f32:
            lam[:] = lam.astype(np.float32)
            M[:] = M.astype(np.float32)
        states.append((lam.copy(), M.copy()))
    return states


def unrolled_grad_along(prob, omega, alpha, states, threads=0):
    """(LB, d_omega, d_alpha, d_c) of the lower bound at the last of the given states, differentiated
    along the given trajectory: the seed dLB/dlambda_bar = argmin assignment (Sec. "Loss"), the flush
    lambda_bar = lambda + alpha S, Alg. 2 (pass_vjp) on every pass in reverse from its given start
    state, then lambda_0 = c/|J_i| (uncovered variables: dLB/dc_i = [c_i < 0]).  The steps of
    unrolled_grad, with the passes' start states supplied instead of recomputed."""
    npass = len(states) - 1
    lamT, MT = states[-1]
    lb, _, lbar = lower_bound(prob, alpha, lamT, MT, threads=threads)
    x = argmin(prob, lbar, threads=threads).astype(np.float64)
    var = prob.col.astype(np.int64)
    S = np.zeros(prob.n)
    np.add.at(S, var, MT)
    d_alpha = x * S[var]
    gv = np.zeros(prob.n)
    np.add.at(gv, var, x * alpha)
    dl, dM = x, gv[var]
    d_omega = np.zeros(prob.nnz)
    for q in range(npass - 1, -1, -1):
        li, mi = states[q]
        dl, dM, da, dw = pass_vjp(prob, omega, alpha, q % 2, li, mi, dl, dM, threads=threads)
        d_alpha += da
        d_omega += dw
    deg = np.bincount(var, minlength=prob.n).astype(np.float64)
    d_c = np.where(deg == 0, (np.asarray(prob.c) < 0).astype(np.float64), 0.0)
    np.add.at(d_c, var, dl / deg[var])
    return lb, d_omega, d_alpha, d_c


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
