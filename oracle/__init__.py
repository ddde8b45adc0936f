"""FP64 CPU oracle for the aggregation-shattering hot path -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg
of ``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.  See ``smol_oracle.c`` for what each function follows
in the paper (Sec. 1 Eqs. (2) and (4) for the right-hand side, Sec. 2 Eq. (5)
for the time integration) and how each one is pinned.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "smol_oracle.c")
# ORACLE_LIB names another build of the same source (the sanitizer test's)
_LIB = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, ENOMEM, ESTEPSIZE, EMAXSTEPS, ENONFINITE = 0, -1, -2, -4, -5, -6
BS32, DP54 = 0, 1


def build():
    """Compile the oracle with gcc (OpenMP on) into oracle/liboracle.so."""
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)


class _Opts(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("nthreads", ctypes.c_int32),
                ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("t_end", ctypes.c_double), ("h0", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("safety", ctypes.c_double),
                ("facmin", ctypes.c_double), ("facmax", ctypes.c_double),
                ("h_min", ctypes.c_double), ("source", ctypes.c_void_p)]


class _PaperOpts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("nthreads", ctypes.c_int32), ("tol", ctypes.c_double),
                ("t_end", ctypes.c_double), ("h0", ctypes.c_double), ("s", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("h_min", ctypes.c_double),
                ("source", ctypes.c_void_p)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_rhs", ctypes.c_int64), ("n_accept", ctypes.c_int64),
                ("n_reject", ctypes.c_int64), ("t", ctypes.c_double),
                ("h", ctypes.c_double), ("err", ctypes.c_double),
                ("status", ctypes.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("ORACLE_LIB") and (
                not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        i64, i32, d = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.oracle_rhs.argtypes = [i64, i32, P, P, d, P, P, i32]
        L.oracle_rhs_source.argtypes = [i64, i32, P, P, d, P, P, P, i32]
        L.oracle_rhs_entries.argtypes = [i64, i32, P, P, d, P, ctypes.POINTER(i64), i64, P, i32]
        L.oracle_rhs_kernel.argtypes = [i64, i32, d, d, d, P, P, i32]
        L.oracle_kernel_entries.argtypes = [i32, d, d, ctypes.POINTER(i64), ctypes.POINTER(i64),
                                            i64, P]
        L.oracle_integrate.argtypes = [i64, i32, P, P, d, P, ctypes.POINTER(_Opts), P,
                                       ctypes.POINTER(_Stats), P, i64]
        L.oracle_rk_fixed.argtypes = [i64, i32, P, P, d, P, i32, d, i64, i32, P, i32]
        L.oracle_integrate_paper.argtypes = [i64, i32, P, P, d, P, ctypes.POINTER(_PaperOpts), P,
                                             ctypes.POINTER(_Stats), P, i64]
        L.oracle_paper_attempt.argtypes = [i32, i64, i32, P, P, d, P, d, P, P, i32]
        L.oracle_tableau.argtypes = [i32, P, P, P, ctypes.POINTER(i32)]
        L.oracle_moments.argtypes = [i64, P, P]
        L.oracle_moments.restype = None
        L.oracle_features.argtypes = [i64, P, d, P, i32, P]
        L.oracle_features.restype = None
        L.oracle_proposer_features.argtypes = [P, d, P, i32, P]
        L.oracle_proposer_features.restype = None
        L.oracle_proposer_dataset.argtypes = [P, i64, i32, d, P, P]
        L.oracle_proposer_dataset.restype = i64
        L.oracle_learned_factor.argtypes = [P, P, d, P, i32, d, i32]
        L.oracle_learned_factor.restype = d
        L.oracle_learned_steps.argtypes = [P, P, i64, i32, P]
        L.oracle_learned_steps.restype = None
        L.oracle_mlp_nparams.restype = i32
        L.oracle_mlp_forward.argtypes = [P, i64, P, P]
        L.oracle_mlp_forward.restype = None
        L.oracle_mlp_loss_grad.argtypes = [P, i64, P, P, d, P, P]
        L.oracle_mlp_loss_grad.restype = None
        L.oracle_adam.argtypes = [P, P, P, P, i64, i64, d, d, d, d]
        L.oracle_adam.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _factors(U, V, M=None):
    U, V = _f64(U), _f64(V)
    if U.ndim == 1:
        U = U[None, :]
    if V.ndim == 1:
        V = V[None, :]
    assert U.shape == V.shape, "U and V must both be stored alpha-major as (R, M)"
    if M is not None:
        assert U.shape[1] == M
    return U, V


def rhs(U, V, lam, n, threads=0):
    """S(n) for all sizes by the plain O(M^2 R) double sums."""
    n = _f64(n)
    U, V = _factors(U, V, n.size)
    out = np.empty_like(n)
    rc = lib().oracle_rhs(n.size, U.shape[0], _p(U), _p(V), float(lam), _p(n), _p(out), threads)
    assert rc == OK, rc
    return out


# kernels given by a formula (Sec. 3.1)
K_CONSTANT, K_BROWNIAN, K_FREE_MOLECULAR = 1, 2, 3


def rhs_kernel(formula, lam, n, p0=0.0, p1=0.0, threads=0):
    """S(n) by the direct sums with K_ij evaluated from a formula for every
    pair (K_CONSTANT: p0; K_BROWNIAN: (i/j)^p0 + (j/i)^p0 + p1;
    K_FREE_MOLECULAR: (i^(1/3) + j^(1/3))^2 sqrt(1/i + 1/j))."""
    n = _f64(n)
    out = np.empty_like(n)
    rc = lib().oracle_rhs_kernel(n.size, int(formula), float(p0), float(p1), float(lam), _p(n),
                                 _p(out), threads)
    assert rc == OK, rc
    return out


def kernel_entries(formula, i, j, p0=0.0, p1=0.0):
    """K_ij of a formula kernel at 1-based sizes (arrays of equal length)."""
    i = np.ascontiguousarray(i, dtype=np.int64)
    j = np.ascontiguousarray(j, dtype=np.int64)
    assert i.shape == j.shape
    out = np.empty(i.size)
    P64 = ctypes.POINTER(ctypes.c_int64)
    rc = lib().oracle_kernel_entries(int(formula), float(p0), float(p1), i.ctypes.data_as(P64),
                                     j.ctypes.data_as(P64), i.size, _p(out))
    assert rc == OK, rc
    return out.reshape(i.shape)


def kernel_matrix(formula, M, p0=0.0, p1=0.0):
    """The M x M matrix K_ij (row i-1, column j-1) of a formula kernel."""
    s = np.arange(1, M + 1, dtype=np.int64)
    I, J = np.meshgrid(s, s, indexing="ij")
    return kernel_entries(formula, I.ravel(), J.ravel(), p0, p1).reshape(M, M)


def rhs_entries(U, V, lam, n, idx, threads=0):
    """S(n) at 0-based indices idx (index s-1 holds size s)."""
    n = _f64(n)
    U, V = _factors(U, V, n.size)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty(idx.size)
    rc = lib().oracle_rhs_entries(n.size, U.shape[0], _p(U), _p(V), float(lam), _p(n),
                                  idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  idx.size, _p(out), threads)
    assert rc == OK, rc
    return out


def integrate(U, V, lam, n0, t_end, rtol, atol, method=DP54, h0=0.0, max_steps=0,
              alpha=0.0, beta=0.0, safety=0.0, facmin=0.0, facmax=0.0, threads=0,
              log_cap=0, h_min=0.0, source=None):
    """Adaptive embedded RK integration (optional Eq. (3) sources).  Returns
    (n_out, stats, log) where log rows are (t_start, h, err, accepted,
    t_after) per step attempt.  alpha > 0 sets both PI exponents (beta of
    either sign); otherwise both take their defaults 0.7/k and 0.4/k."""
    n0 = _f64(n0)
    U, V = _factors(U, V, n0.size)
    src = None if source is None else _f64(source)
    o = _Opts(method, threads, rtol, atol, t_end, h0, max_steps, alpha, beta, safety,
              facmin, facmax, h_min, None if src is None else src.ctypes.data)
    st = _Stats()
    out = np.empty_like(n0)
    log = np.zeros((max(log_cap, 1), 5))
    lib().oracle_integrate(n0.size, U.shape[0], _p(U), _p(V), float(lam), _p(n0),
                           ctypes.byref(o), _p(out), ctypes.byref(st),
                           _p(log) if log_cap > 0 else None, log_cap)
    stats = {f: getattr(st, f) for f, _ in _Stats._fields_}
    nlog = min(log_cap, stats["n_accept"] + stats["n_reject"]) if log_cap else 0
    return out, stats, log[:nlog].copy()


# the paper's schemes (Sec. 2) and step-size rules
RKF45, RK2_DBL, RK4_DBL = 2, 3, 4
RULE_EQ6, RULE_HALVE_DOUBLE, RULE_FEHLBERG = 0, 1, 2


def rhs_source(U, V, lam, n, source, threads=0):
    """Eq. (3): S(n) + P (constant sources)."""
    n = _f64(n)
    U, V = _factors(U, V, n.size)
    src = _f64(source)
    out = np.empty_like(n)
    rc = lib().oracle_rhs_source(n.size, U.shape[0], _p(U), _p(V), float(lam), _p(n), _p(src),
                                 _p(out), threads)
    assert rc == OK, rc
    return out


def integrate_paper(U, V, lam, n0, t_end, tol, scheme, rule, h0=0.0, s=0.0, max_steps=0,
                    h_min=0.0, threads=0, log_cap=0, source=None):
    """The paper's adaptive schemes with the Euclidean error norm.  Returns
    (n_out, stats, log) with log rows (t_start, h, err/tol, accepted, t_after)."""
    n0 = _f64(n0)
    U, V = _factors(U, V, n0.size)
    src = None if source is None else _f64(source)
    o = _PaperOpts(scheme, rule, threads, tol, t_end, h0, s, max_steps, h_min,
                   None if src is None else src.ctypes.data)
    st = _Stats()
    out = np.empty_like(n0)
    log = np.zeros((max(log_cap, 1), 5))
    lib().oracle_integrate_paper(n0.size, U.shape[0], _p(U), _p(V), float(lam), _p(n0),
                                 ctypes.byref(o), _p(out), ctypes.byref(st),
                                 _p(log) if log_cap > 0 else None, log_cap)
    stats = {f: getattr(st, f) for f, _ in _Stats._fields_}
    nlog = min(log_cap, stats["n_accept"] + stats["n_reject"]) if log_cap else 0
    return out, stats, log[:nlog].copy()


def paper_attempt(U, V, lam, y, tau, scheme, threads=0):
    """One attempt of a paper scheme from y: (RKF45: fourth- and fifth-order
    solutions; doubling: single step and two half steps)."""
    y = _f64(y)
    U, V = _factors(U, V, y.size)
    a, b = np.empty_like(y), np.empty_like(y)
    rc = lib().oracle_paper_attempt(scheme, y.size, U.shape[0], _p(U), _p(V), float(lam), _p(y),
                                    float(tau), _p(a), _p(b), threads)
    assert rc == OK, rc
    return a, b


def rk_fixed(U, V, lam, n0, method, h, nsteps, embedded=False, threads=0):
    n0 = _f64(n0)
    U, V = _factors(U, V, n0.size)
    out = np.empty_like(n0)
    rc = lib().oracle_rk_fixed(n0.size, U.shape[0], _p(U), _p(V), float(lam), _p(n0),
                               method, h, nsteps, int(embedded), _p(out), threads)
    assert rc == OK, rc
    return out


def tableau(method):
    a = np.zeros(49)
    b = np.zeros(7)
    bh = np.zeros(7)
    s = ctypes.c_int32()
    rc = lib().oracle_tableau(method, _p(a), _p(b), _p(bh), ctypes.byref(s))
    assert rc == OK
    S = s.value
    return a[:S * S].reshape(S, S), b[:S], bh[:S]


def moments(n):
    n = _f64(n)
    m = np.zeros(4)
    lib().oracle_moments(n.size, _p(n), _p(m))
    return m


def features(n, h, err_hist):
    n = _f64(n)
    e = _f64(err_hist) if len(err_hist) else np.zeros(1)
    x = np.zeros(9)
    lib().oracle_features(n.size, _p(n), float(h), _p(e), len(err_hist), _p(x))
    return x


def proposer_features(mom, h, err_hist):
    """Feature vector from the moments M0..M3 of the decision's state."""
    mom = _f64(mom)
    e = _f64(err_hist) if len(err_hist) else np.zeros(1)
    x = np.zeros(9)
    lib().oracle_proposer_features(_p(mom), float(h), _p(e), len(err_hist), _p(x))
    return x


def proposer_dataset(log, k, err_target=0.8):
    """(X, target) training rows from a (rows, 9) run log (t, h, err,
    accepted, t_after, M0..M3); k = embedded order + 1."""
    log = _f64(log)
    rows = log.shape[0]
    X = np.zeros((max(rows, 1), 9))
    tg = np.zeros(max(rows, 1))
    n = lib().oracle_proposer_dataset(_p(log), rows, int(k), float(err_target), _p(X), _p(tg))
    return X[:n].copy(), tg[:n].copy()


def learned_factor(params, mom, h, err_hist, err_prev, k):
    """h_next / h of the learned controller at one decision."""
    params, mom = _f64(params), _f64(mom)
    e = _f64(err_hist)
    return lib().oracle_learned_factor(_p(params), _p(mom), float(h), _p(e), len(err_hist),
                                       float(err_prev), int(k))


def learned_steps(params, log, k):
    """Per log row j: the h_{j+1}/h_j the learned controller takes at
    decision j (NaN where the PI rule decides or there is no successor)."""
    params, log = _f64(params), _f64(log)
    out = np.zeros(log.shape[0])
    lib().oracle_learned_steps(_p(params), _p(log), log.shape[0], int(k), _p(out))
    return out


def mlp_nparams():
    return lib().oracle_mlp_nparams()


def mlp_forward(params, X):
    params, X = _f64(params), _f64(X)
    Y = np.zeros(X.shape[0])
    lib().oracle_mlp_forward(_p(params), X.shape[0], _p(X), _p(Y))
    return Y


def mlp_loss_grad(params, X, target, over_w=4.0):
    params, X, target = _f64(params), _f64(X), _f64(target)
    loss = np.zeros(1)
    grad = np.zeros_like(params)
    lib().oracle_mlp_loss_grad(_p(params), X.shape[0], _p(X), _p(target), float(over_w),
                               _p(loss), _p(grad))
    return float(loss[0]), grad


def adam(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of params, m, v (float64 numpy arrays)."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    grad = _f64(grad)
    lib().oracle_adam(_p(params), _p(grad), _p(m), _p(v), params.size, step, lr, b1, b2, eps)
