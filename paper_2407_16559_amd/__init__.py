"""Python binding of libsmol (argument marshalling only).

Every computation runs in the HIP kernels of ``libsmol.so`` (built in-tree for
gfx950 by ``paper_2407_16559_amd/build.py``).  There is no CPU fallback: if the
library is missing, importing works but every call raises.

Arrays are torch tensors on a ROCm device, float64 and contiguous; the kernel
factors U and V are (R, M) alpha-major.  Calls run on the tensors' device and
torch's current stream there.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsmol.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTEPSIZE, EMAXSTEPS, ENONFINITE, EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
METHODS = {"bs3": 0, "bs32": 0, "dp5": 1, "dp54": 1, "rkf45": 2, "rk2_dbl": 3, "rk4_dbl": 4}
PRECISIONS = {"fp64": 0, "fp32x2": 1}
CONTROLLERS = {"pi": 0, "learned": 1, "fehlberg": 2, "step_doubling": 3, "halve_double": 4}
N_PARAMS = 4865

_lib = None


class SmolError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class _Stats(ctypes.Structure):
    _fields_ = [("n_rhs", ctypes.c_int64), ("n_accept", ctypes.c_int64),
                ("n_reject", ctypes.c_int64), ("t", ctypes.c_double),
                ("h", ctypes.c_double), ("err", ctypes.c_double),
                ("status", ctypes.c_int32), ("n_fallback", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class _State(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("h", ctypes.c_double), ("err", ctypes.c_double),
                ("err_prev", ctypes.c_double), ("err_hist", ctypes.c_double * 4),
                ("n_rhs", ctypes.c_int64), ("n_accept", ctypes.c_int64),
                ("n_reject", ctypes.c_int64), ("n_hist", ctypes.c_int32),
                ("rejected", ctypes.c_int32), ("valid", ctypes.c_int32),
                ("n_fallback", ctypes.c_int32), ("k1", ctypes.c_void_p)]


class State:
    """Checkpoint of a run (smol_state): pass it as `state=` to integrate();
    after the call it holds the run's final checkpoint, and a later call with
    it (and the run's output as n0) continues the run.  k1 is a device tensor
    of M doubles owned by this object."""

    def __init__(self, M, device="cuda:0"):
        self.k1 = torch.zeros(M, dtype=torch.float64, device=device)
        self.c = _State()
        self.c.k1 = self.k1.data_ptr()

    @property
    def valid(self):
        return bool(self.c.valid)

    def as_dict(self):
        d = {f: getattr(self.c, f) for f, _ in _State._fields_ if f != "k1"}
        d["err_hist"] = list(self.c.err_hist)
        return d


class _Options(ctypes.Structure):
    _fields_ = [("h0", ctypes.c_double), ("h_min", ctypes.c_double),
                ("max_steps", ctypes.c_int64), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("controller", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("log", ctypes.c_void_p),
                ("log_cap", ctypes.c_int64), ("safety", ctypes.c_double),
                ("source", ctypes.c_void_p), ("state", ctypes.POINTER(_State))]


class _Instance(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int64), ("R", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("U", ctypes.c_void_p), ("V", ctypes.c_void_p), ("lam", ctypes.c_double),
                ("n0", ctypes.c_void_p), ("n_out", ctypes.c_void_p), ("t_end", ctypes.c_double),
                ("rtol", ctypes.c_double), ("atol", ctypes.c_double),
                ("log", ctypes.c_void_p), ("log_cap", ctypes.c_int64),
                ("source", ctypes.c_void_p)]


def lib():
    """Load libsmol.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        i64, i32, d, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
        L.smol_rhs.argtypes = [i64, i32, vp, vp, d, vp, vp, i32, vp]
        L.smol_rhs_ex.argtypes = [i64, i32, vp, vp, d, vp, vp, vp, i32, vp]
        L.smol_rhs_noalloc.argtypes = [i64, i32, vp, vp, d, vp, vp, vp]
        L.smol_integrate.argtypes = [i64, i32, vp, vp, d, vp, d, d, d, i32, i32, vp,
                                     ctypes.POINTER(_Stats), vp]
        L.smol_integrate_ex.argtypes = [i64, i32, vp, vp, d, vp, d, d, d, i32, i32,
                                        ctypes.POINTER(_Options), vp, ctypes.POINTER(_Stats), vp]
        L.smol_integrate_batch.argtypes = [i32, ctypes.POINTER(_Instance), i32, i32,
                                           ctypes.POINTER(_Options), ctypes.POINTER(_Stats), vp]
        L.smol_proposer_set.argtypes = [vp, i32, vp]
        L.smol_proposer_forward.argtypes = [vp, vp, i64, vp, vp]
        L.smol_proposer_loss_grad.argtypes = [vp, vp, vp, i64, ctypes.c_float, vp, vp, vp]
        L.smol_proposer_dataset.argtypes = [vp, i64, i32, d, vp, vp, ctypes.POINTER(i64), vp]
        L.smol_proposer_train.argtypes = [vp, vp, i64, vp, i32, i32, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_uint64, vp, vp]
        L.smol_profile_rhs.argtypes = [i64, i32, vp, vp, d, vp, vp, i32,
                                       ctypes.POINTER(ctypes.c_float), vp]
        L.smol_profile_step.argtypes = [i64, i32, vp, vp, d, vp, i32, i32,
                                        ctypes.POINTER(ctypes.c_float), vp]
        L.smol_set_schedule.argtypes = [i32, ctypes.POINTER(i32)]
        L.smol_get_schedule.argtypes = [i32, ctypes.POINTER(i32)]
        L.smol_autotune.argtypes = [i64, i32, vp, vp, d, vp, i32, i32, i32, ctypes.POINTER(i32),
                                    ctypes.POINTER(ctypes.c_float), vp]
        L.smol_lowrank.argtypes = [i64, i32, d, d, d, i32, vp, vp, ctypes.POINTER(i32),
                                   ctypes.POINTER(d), vp]
        L.smol_release_plans.argtypes = []
        L.smol_strerror.argtypes = [ctypes.c_int]
        L.smol_strerror.restype = ctypes.c_char_p
        L.smol_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def strerror(code):
    try:
        return lib().smol_strerror(code).decode()
    except Exception:  # library missing
        return "status %d" % code


def version():
    return lib().smol_version().decode()


def _check(t, name, dtype=torch.float64, numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a ROCm device")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return t


def _factors(U, V, M):
    if U.dim() == 1:
        U = U.unsqueeze(0)
    if V.dim() == 1:
        V = V.unsqueeze(0)
    _check(U, "U")
    _check(V, "V")
    if U.shape != V.shape or U.shape[1] != M:
        raise ValueError("U and V must both be (R, M) alpha-major")
    return U, V, U.shape[0]


def _stream(t):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _raise(rc, what):
    if rc != OK:
        raise SmolError(rc, what)


def rhs(U, V, lam, n, out=None, precision="fp64", source=None):
    """dn/dt = S(n) of the truncated aggregation-shattering system, plus the
    constant sources of Eq. (3) when `source` (M doubles) is given."""
    _check(n, "n")
    M = n.numel()
    U, V, R = _factors(U, V, M)
    if out is None:
        out = torch.empty_like(n)
    _check(out, "out", numel=M)
    with torch.cuda.device(n.device):
        if source is None:
            rc = lib().smol_rhs(M, R, U.data_ptr(), V.data_ptr(), float(lam), n.data_ptr(),
                                out.data_ptr(), PRECISIONS[precision], _stream(n))
        else:
            _check(source, "source", numel=M)
            rc = lib().smol_rhs_ex(M, R, U.data_ptr(), V.data_ptr(), float(lam), n.data_ptr(),
                                   source.data_ptr(), out.data_ptr(), PRECISIONS[precision],
                                   _stream(n))
    _raise(rc, "smol_rhs")
    return out


NOALLOC_MAX_M, NOALLOC_MAX_R = 65537, 4


def rhs_noalloc(U, V, lam, n, out):
    """S(n) in FP64 with the library's fixed device workspaces (no device
    allocation inside the call; `out` is required).  M <= 65537, R <= 4."""
    _check(n, "n")
    M = n.numel()
    U, V, R = _factors(U, V, M)
    _check(out, "out", numel=M)
    if M > NOALLOC_MAX_M or R > NOALLOC_MAX_R:
        raise ValueError(f"smol_rhs_noalloc serves M <= {NOALLOC_MAX_M} and R <= "
                         f"{NOALLOC_MAX_R}; got M={M}, R={R}")
    with torch.cuda.device(n.device):
        rc = lib().smol_rhs_noalloc(M, R, U.data_ptr(), V.data_ptr(), float(lam), n.data_ptr(),
                                    out.data_ptr(), _stream(n))
    _raise(rc, "smol_rhs_noalloc")
    return out


def _options(h0=0.0, h_min=0.0, max_steps=0, alpha=None, beta=None, controller="pi",
             log=None, safety=0.0, source=None, state=None):
    o = _Options()
    if state is not None:
        if not isinstance(state, State):
            raise TypeError("state must be a paper_2407_16559_amd.State")
        o.state = ctypes.pointer(state.c)
    o.h0, o.h_min, o.max_steps = float(h0), float(h_min), int(max_steps)
    o.safety = float(safety)
    if source is not None:
        _check(source, "source")
        o.source = source.data_ptr()
    if alpha is not None or beta is not None:
        if alpha is None or beta is None:
            raise ValueError("give both alpha and beta, or neither")
        o.alpha, o.beta = float(alpha), float(beta)
    o.controller = CONTROLLERS[controller]
    if log is not None:
        _check(log, "log")
        if log.dim() != 2 or log.shape[1] != 9:
            raise ValueError("log must be (rows, 9) float64")
        o.log, o.log_cap = log.data_ptr(), log.shape[0]
    return o


def integrate(U, V, lam, n0, t_end, rtol, atol, method="dp5", precision="fp64", out=None,
              raise_on_error=False, **opts):
    """Integrate dn/dt = S(n) from n0 to t_end.  Returns (n_out, stats dict).
    Options: h0, h_min, max_steps, alpha, beta, controller ('pi'|'learned'),
    log (a (rows, 9) float64 device tensor), source, safety, state (a State:
    resume from it when valid; receives the final checkpoint)."""
    if opts.get("state") is not None and opts["state"].k1.numel() != n0.numel():
        raise ValueError("state was made for another M")
    _check(n0, "n0")
    M = n0.numel()
    U, V, R = _factors(U, V, M)
    if out is None:
        out = torch.empty_like(n0)
    _check(out, "out", numel=M)
    o = _options(**opts)
    st = _Stats()
    with torch.cuda.device(n0.device):
        rc = lib().smol_integrate_ex(M, R, U.data_ptr(), V.data_ptr(), float(lam),
                                     n0.data_ptr(), float(t_end), float(rtol), float(atol),
                                     METHODS[method], PRECISIONS[precision], ctypes.byref(o),
                                     out.data_ptr(), ctypes.byref(st), _stream(n0))
    stats = st.as_dict()
    if rc in (EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED) or (raise_on_error and rc != OK):
        raise SmolError(rc, "smol_integrate")
    stats["status"] = rc if rc != OK else stats["status"]
    return out, stats


def integrate_batch(instances, method="bs3", precision="fp64", **opts):
    """instances: list of dicts with U, V, lam, n0, t_end, rtol, atol (and
    optionally out).  Returns (list of outputs, list of stats dicts)."""
    n = len(instances)
    arr = (_Instance * n)()
    outs = []
    dev = None
    for i, d in enumerate(instances):
        n0 = _check(d["n0"], "n0")
        M = n0.numel()
        U, V, R = _factors(d["U"], d["V"], M)
        out = d.get("out")
        if out is None:
            out = torch.empty_like(n0)
        _check(out, "out", numel=M)
        outs.append(out)
        dev = n0.device
        arr[i].M, arr[i].R = M, R
        arr[i].U, arr[i].V = U.data_ptr(), V.data_ptr()
        arr[i].lam = float(d["lam"])
        arr[i].n0, arr[i].n_out = n0.data_ptr(), out.data_ptr()
        arr[i].t_end, arr[i].rtol, arr[i].atol = float(d["t_end"]), float(d["rtol"]), float(d["atol"])
        log = d.get("log")
        if log is not None:
            _check(log, "log")
            if log.dim() != 2 or log.shape[1] != 9:
                raise ValueError("log must be (rows, 9) float64")
            arr[i].log, arr[i].log_cap = log.data_ptr(), log.shape[0]
        src = d.get("source")
        if src is not None:
            _check(src, "source", numel=M)
            arr[i].source = src.data_ptr()
    o = _options(**opts)
    st = (_Stats * max(n, 1))()
    with torch.cuda.device(dev):
        rc = lib().smol_integrate_batch(n, arr, METHODS[method], PRECISIONS[precision],
                                        ctypes.byref(o), st, _stream(outs[0]))
    _raise(rc, "smol_integrate_batch")
    return outs, [st[i].as_dict() for i in range(n)]


def proposer_set(params):
    _check(params, "params", dtype=torch.float32, numel=N_PARAMS)
    with torch.cuda.device(params.device):
        _raise(lib().smol_proposer_set(params.data_ptr(), N_PARAMS, _stream(params)),
               "smol_proposer_set")


def proposer_forward(params, X):
    """Network output for each row of X (float32 (n, 9))."""
    _check(params, "params", dtype=torch.float32, numel=N_PARAMS)
    _check(X, "X", dtype=torch.float32)
    Y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    with torch.cuda.device(X.device):
        _raise(lib().smol_proposer_forward(params.data_ptr(), X.data_ptr(), X.shape[0],
                                           Y.data_ptr(), _stream(X)), "smol_proposer_forward")
    return Y


def proposer_loss_grad(params, X, target, over_weight=4.0):
    """(loss, grad) of the weighted MSE over all rows (float32 device tensors)."""
    _check(params, "params", dtype=torch.float32, numel=N_PARAMS)
    _check(X, "X", dtype=torch.float32)
    _check(target, "target", dtype=torch.float32, numel=X.shape[0])
    loss = torch.zeros(1, dtype=torch.float32, device=X.device)
    grad = torch.empty(N_PARAMS, dtype=torch.float32, device=X.device)
    with torch.cuda.device(X.device):
        _raise(lib().smol_proposer_loss_grad(params.data_ptr(), X.data_ptr(), target.data_ptr(),
                                             X.shape[0], float(over_weight), loss.data_ptr(),
                                             grad.data_ptr(), _stream(X)), "smol_proposer_loss_grad")
    return loss, grad


def proposer_dataset(log, rows, method="dp5", err_target=0.8):
    """(X, target) training rows from the first `rows` rows of a run log."""
    _check(log, "log")
    X = torch.empty((max(rows, 1), 9), dtype=torch.float32, device=log.device)
    tg = torch.empty(max(rows, 1), dtype=torch.float32, device=log.device)
    n = ctypes.c_int64()
    with torch.cuda.device(log.device):
        _raise(lib().smol_proposer_dataset(log.data_ptr(), int(rows), METHODS[method],
                                           float(err_target), X.data_ptr(),
                                           tg.data_ptr(), ctypes.byref(n), _stream(log)),
               "smol_proposer_dataset")
    return X[: n.value].contiguous(), tg[: n.value].contiguous()


def proposer_train(X, target, params, epochs, batch=1024, lr=1e-3, over_weight=4.0, seed=0):
    """Train the step proposer in place on (X, target) with the library's own
    forward / backward / Adam kernels.  Returns the per-epoch mean loss."""
    _check(X, "X", dtype=torch.float32)
    nrows = X.shape[0]
    _check(target, "target", dtype=torch.float32, numel=nrows)
    _check(params, "params", dtype=torch.float32, numel=N_PARAMS)
    loss = torch.zeros(epochs, dtype=torch.float32, device=X.device)
    with torch.cuda.device(X.device):
        rc = lib().smol_proposer_train(X.data_ptr(), target.data_ptr(), nrows, params.data_ptr(),
                                       int(epochs), int(batch), float(lr), float(over_weight),
                                       int(seed), loss.data_ptr(), _stream(X))
    _raise(rc, "smol_proposer_train")
    return loss


def profile_rhs(U, V, lam, n, iters=50, out=None):
    """Mean milliseconds per launch of the three right-hand-side kernels
    (column pass, row-pair pass, inverse column pass + finish) and per whole
    right-hand side, timed with HIP events on the current stream."""
    _check(n, "n")
    M = n.numel()
    U, V, R = _factors(U, V, M)
    if out is None:
        out = torch.empty_like(n)
    ms = (ctypes.c_float * 4)()
    with torch.cuda.device(n.device):
        rc = lib().smol_profile_rhs(M, R, U.data_ptr(), V.data_ptr(), float(lam), n.data_ptr(),
                                    out.data_ptr(), int(iters), ms, _stream(n))
    _raise(rc, "smol_profile_rhs")
    return {"phase_a": ms[0], "phase_b": ms[1], "phase_c": ms[2], "rhs": ms[3]}


def profile_step(U, V, lam, n0, method="dp5", iters=50):
    """Mean milliseconds per launch of the integrator's stage kernels at the
    state n0: column pass of stage 2, row-pair pass, fused finish of stage 3
    (with the next column pass) and the last stage's finish, timed with HIP
    events on the current stream."""
    _check(n0, "n0")
    M = n0.numel()
    U, V, R = _factors(U, V, M)
    ms = (ctypes.c_float * 4)()
    with torch.cuda.device(n0.device):
        rc = lib().smol_profile_step(M, R, U.data_ptr(), V.data_ptr(), float(lam), n0.data_ptr(),
                                     METHODS[method], int(iters), ms, _stream(n0))
    _raise(rc, "smol_profile_step")
    return {"int_a": ms[0], "int_b": ms[1], "int_c_fused": ms[2], "int_c_last": ms[3]}


def set_schedule(logL, variants):
    """Kernel variants (A, B, C) for transforms of length 2^logL (FP64)."""
    v = (ctypes.c_int32 * 3)(*[int(x) for x in variants])
    _raise(lib().smol_set_schedule(int(logL), v), "smol_set_schedule")


def get_schedule(logL):
    v = (ctypes.c_int32 * 3)()
    _raise(lib().smol_get_schedule(int(logL), v), "smol_get_schedule")
    return tuple(v)


def autotune(U, V, lam, n0, method="dp5", attempts=64, reps=3):
    """Tune the schedule of n0's transform length on this instance; returns
    (variants, ms per step attempt before, ms per step attempt after)."""
    _check(n0, "n0")
    M = n0.numel()
    U, V, R = _factors(U, V, M)
    v = (ctypes.c_int32 * 3)()
    ms = (ctypes.c_float * 2)()
    with torch.cuda.device(n0.device):
        _raise(lib().smol_autotune(M, R, U.data_ptr(), V.data_ptr(), float(lam), n0.data_ptr(),
                                   METHODS[method], int(attempts), int(reps), v, ms,
                                   _stream(n0)), "smol_autotune")
    return tuple(v), ms[0], ms[1]


KERNELS = {"constant": 1, "brownian": 2, "free_molecular": 3}
MAX_RANK = 32


def lowrank(M, kernel="free_molecular", p0=0.0, p1=0.0, tol=1e-10, max_rank=MAX_RANK,
            device="cuda:0"):
    """Low-rank factors (U, V) of shape (rank, M), float64 on `device`, of a
    kernel given by a formula (adaptive cross approximation on the GPU), and
    the last term's relative Frobenius norm."""
    U = torch.empty((max_rank, M), dtype=torch.float64, device=device)
    V = torch.empty_like(U)
    r = ctypes.c_int32()
    e = ctypes.c_double()
    with torch.cuda.device(U.device):
        _raise(lib().smol_lowrank(int(M), KERNELS[kernel], float(p0), float(p1), float(tol),
                                  int(max_rank), U.data_ptr(), V.data_ptr(), ctypes.byref(r),
                                  ctypes.byref(e), _stream(U)), "smol_lowrank")
    k = r.value
    return U[:k].contiguous(), V[:k].contiguous(), e.value


def release_plans():
    _raise(lib().smol_release_plans(), "smol_release_plans")
