"""Thin Python binding of the C ABI in include/raspen.h (argument marshalling only).

Every function has the name of the C entry point it calls.  Device arrays are
torch tensors (float64, contiguous, on the context's CUDA/HIP device); torch
provides memory and streams, every step of the method runs in libraspen.so.
Importing this module fails loudly if the library has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libraspen.so")

RSP_OK, RSP_NOT_CONVERGED, RSP_LINESEARCH_FAIL, RSP_GMRES_STAGNATION, RSP_REFINE_FALLBACK = 0, 1, 2, 3, 4
RSP_EINVAL, RSP_ENOMEM, RSP_EHIP, RSP_ENUMERIC, RSP_EAGAIN = -1, -2, -3, -4, -5
RSP_TICKET_QUEUED, RSP_TICKET_RUNNING, RSP_TICKET_DONE = 0, 1, 2
RSP_FP64, RSP_FP32_REFINED = 0, 1
RSP_CONT_FIRST, RSP_CONT_NONE, RSP_CONT_EVERY = 0, 1, 2
RSP_HIST_MAX = 64
RSP_TUNE_PARTITION, RSP_TUNE_BATCH = 1, 2


class RaspenError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("raspen error %d: %s" % (code, msg))
        self.code = code


class rsp_problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("phi_kind", ctypes.c_int32),
                ("kappa", ctypes.c_double), ("nu", ctypes.c_double), ("mu", ctypes.c_double),
                ("eps0", ctypes.c_double), ("eps_min", ctypes.c_double), ("gamma", ctypes.c_double),
                ("sx", ctypes.c_int32), ("sy", ctypes.c_int32), ("overlap", ctypes.c_int32),
                ("coef", ctypes.c_void_p)]


class rsp_options(ctypes.Structure):
    _fields_ = [("tol_outer", ctypes.c_double), ("tol_inner", ctypes.c_double),
                ("gmres_rtol", ctypes.c_double), ("sigma", ctypes.c_double),
                ("alpha_min", ctypes.c_double), ("gmres_restart", ctypes.c_int32),
                ("max_outer", ctypes.c_int32), ("max_inner", ctypes.c_int32),
                ("max_gmres", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("continuation", ctypes.c_int32),
                ("record_eps_snapshots", ctypes.c_int32), ("tol_inner_rel", ctypes.c_double),
                ("fallback_rho", ctypes.c_double), ("eps_snapshots", ctypes.c_void_p),
                ("coarse", ctypes.c_int32)]


_H = RSP_HIST_MAX + 1


class rsp_history(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("outer", ctypes.c_int32),
                ("norm", ctypes.c_double * _H), ("gmres_its", ctypes.c_int32 * _H),
                ("gmres_rel", ctypes.c_double * _H), ("inner_min", ctypes.c_int32 * _H),
                ("inner_max", ctypes.c_int32 * _H), ("inner_avg", ctypes.c_double * _H),
                ("backtracks", ctypes.c_int32 * _H), ("subdomains", ctypes.c_int32),
                ("factorizations", ctypes.c_int64), ("local_solves", ctypes.c_int64),
                ("gmres_total", ctypes.c_int64), ("newton_iterations", ctypes.c_int64),
                ("jac_applies", ctypes.c_int64), ("residual_final", ctypes.c_double),
                ("flops", ctypes.c_double), ("ms_eval", ctypes.c_double),
                ("ms_gmres", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("fallback_outer", ctypes.c_int32), ("snapshots", ctypes.c_int32),
                ("snapshot_eps", ctypes.c_double * _H)]

    def as_dict(self):
        k = min(self.outer, RSP_HIST_MAX)
        return dict(status=self.status, outer=self.outer, norm=list(self.norm[:k + 1]),
                    gmres_its=list(self.gmres_its[1:k + 1]), gmres_rel=list(self.gmres_rel[1:k + 1]),
                    inner_min=list(self.inner_min[:k + 1]), inner_max=list(self.inner_max[:k + 1]),
                    inner_avg=list(self.inner_avg[:k + 1]), backtracks=list(self.backtracks[:k + 1]),
                    subdomains=self.subdomains, factorizations=self.factorizations,
                    local_solves=self.local_solves, gmres_total=self.gmres_total,
                    newton_iterations=self.newton_iterations, jac_applies=self.jac_applies,
                    residual_final=self.residual_final, flops=self.flops, ms_eval=self.ms_eval,
                    ms_gmres=self.ms_gmres, ms_total=self.ms_total, fallback_outer=self.fallback_outer,
                    snapshots=self.snapshots, snapshot_eps=list(self.snapshot_eps[:self.snapshots]))


class rsp_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


class rsp_tuning(ctypes.Structure):
    _fields_ = [("graphs", ctypes.c_int32), ("gm_chunk", ctypes.c_int32), ("sx", ctypes.c_int32),
                ("sy", ctypes.c_int32), ("max_batch", ctypes.c_int32), ("solves_per_s", ctypes.c_double),
                ("jac_form", ctypes.c_int32)]


class rsp_server_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("hbm_budget", ctypes.c_size_t), ("opts", rsp_options), ("tune", rsp_tuning),
                ("profile_every", ctypes.c_int32)]


class rsp_server_report(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("failed", ctypes.c_int64), ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("mean_batch", ctypes.c_double),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double),
                ("mean_ms", ctypes.c_double), ("solves_per_s", ctypes.c_double)]


# (name, restype, argtypes) of every exported entry point, in header order
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_PROB = ctypes.POINTER(rsp_problem)
_OPTS = ctypes.POINTER(rsp_options)
_I32P = ctypes.POINTER(ctypes.c_int32)
SIGNATURES = [
    ("rsp_version", _I, []),
    ("rsp_last_error", ctypes.c_char_p, []),
    ("rsp_partition", _I, [_PROB, _I32P, _I32P, _I32P, _I32P]),
    ("rsp_workspace_bytes", ctypes.c_size_t, [_PROB, _OPTS]),
    ("rsp_context_create", _I, [ctypes.POINTER(_P), _I, ctypes.c_size_t]),
    ("rsp_context_destroy", _I, [_P]),
    ("rsp_setup", _I, [_P, _PROB, _OPTS, _P, _P, _P]),
    ("rsp_residual", _I, [_P, _P, _D, _P, _P]),
    ("rsp_control", _I, [_P, _P, _D, _P, _P]),
    ("rsp_restrict", _I, [_P, _P, _P, _P]),
    ("rsp_prolong", _I, [_P, _P, _P, _P]),
    ("rsp_local_residual", _I, [_P, _P, _P, _D, _P, _P, _P]),
    ("rsp_local_residual_noalloc", _I, [_PROB, _P, _P, _P, _P, _D, _P, _P, _P]),
    ("rsp_local_solve", _I, [_P, _P, _P, _D, _P, _P, _P]),
    ("rsp_eval", _I, [_P, _P, _I, _P, ctypes.POINTER(_D), _P]),
    ("rsp_jac_apply", _I, [_P, _P, _P, _P]),
    ("rsp_coarse_jac_apply", _I, [_P, _P, _P, _P, _P]),
    ("rsp_solve", _I, [_P, _PROB, _OPTS, _P, _P, _P, _P, _P, _P, _P,
                       ctypes.POINTER(rsp_history), _P]),
    ("rsp_solve_newton_ras", _I, [_P, _PROB, _OPTS, _P, _P, _P, _P, _P, _P, _P,
                                  ctypes.POINTER(rsp_history), _P]),
    ("rsp_solve_newton", _I, [_P, _PROB, _OPTS, _P, _P, _P, _P, _P, _P, _P,
                              ctypes.POINTER(rsp_history), _P]),
    ("rsp_solve_batch", _I, [_P, _I, _PROB, _OPTS, _P, _P, _P, _P, _P, _P, _P,
                             ctypes.POINTER(rsp_history), _P]),
    ("rsp_batch_workspace_bytes", ctypes.c_size_t, [_I, _PROB, _OPTS]),
    ("rsp_get_tuning", _I, [_P, ctypes.POINTER(rsp_tuning)]),
    ("rsp_set_tuning", _I, [_P, ctypes.POINTER(rsp_tuning)]),
    ("rsp_autotune", _I, [_P, _PROB, _OPTS, _P, _P, _I, ctypes.POINTER(rsp_tuning), _P]),
    ("rsp_server_create", _I, [ctypes.POINTER(_P), ctypes.POINTER(rsp_server_options)]),
    ("rsp_server_submit", _I, [_P, _PROB, _P, _P, _P, _P, _P, ctypes.POINTER(ctypes.c_uint64)]),
    ("rsp_server_poll", _I, [_P, ctypes.c_uint64, _I32P]),
    ("rsp_server_wait", _I, [_P, ctypes.c_uint64, _D, ctypes.POINTER(rsp_history)]),
    ("rsp_server_stats", _I, [_P, ctypes.POINTER(rsp_server_report)]),
    ("rsp_server_kernel_stats", _I, [_P, ctypes.POINTER(rsp_kernel_stat), _I, _I32P]),
    ("rsp_server_destroy", _I, [_P]),
    ("rsp_set_profiling", _I, [_P, _I]),
    ("rsp_set_profiling_filter", _I, [_P, ctypes.c_char_p]),
    ("rsp_set_profiling_sample", _I, [_P, ctypes.c_int]),
    ("rsp_reset_kernel_stats", _I, [_P]),
    ("rsp_kernel_stats", _I, [_P, ctypes.POINTER(rsp_kernel_stat), _I, _I32P]),
]

_lib = None


def load():
    """Load libraspen.so (raises if it is missing: there is no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libraspen.so is not built; run paper_2411_00546_amd.build.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(code, allow_positive=True):
    if code < 0 or (code > 0 and not allow_positive):
        raise RaspenError(code, load().rsp_last_error().decode())
    return code


def _ptr(t, allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError("array argument is required")
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("device arrays must be torch tensors")
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("arrays must be contiguous float64 device tensors")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_problem(p, coef=None):
    """rsp_problem from a synth.Problem-like object.  coef: device tensor (float64) with
    the coefficients of A in the layout of rsp_problem.coef (a1 [ny][nx+1], a2 [ny+1][nx],
    a0 [ny][nx]); required when p.coef is set, and kept alive by the caller."""
    ptr = None
    if coef is not None:
        want = (p.nx + 1) * p.ny + p.nx * (p.ny + 1) + p.nx * p.ny
        if coef.numel() != want or not coef.is_contiguous():
            raise ValueError("coef must be a contiguous tensor of %d doubles" % want)
        ptr = _ptr(coef)
    elif getattr(p, "coef", 0):
        raise ValueError("the problem has variable coefficients: pass them as coef")
    return rsp_problem(p.nx, p.ny, p.phi, p.kappa, p.nu, p.mu, p.eps0, p.eps_min, p.gamma,
                       p.sx, p.sy, p.overlap, ptr)


def make_options(o, eps_snapshots=None):
    """rsp_options from a synth.Options-like object; eps_snapshots: device tensor
    [K][2][ny][nx] that receives up to K = o.record_eps_snapshots snapshots (rsp_solve)."""
    k = int(getattr(o, "record_eps_snapshots", 0))
    if k and eps_snapshots is None:
        raise ValueError("record_eps_snapshots needs an eps_snapshots tensor")
    if k and (eps_snapshots.dim() != 4 or eps_snapshots.shape[0] < k or eps_snapshots.shape[1] != 2):
        raise ValueError("eps_snapshots must be [K >= record_eps_snapshots][2][ny][nx]")
    return rsp_options(o.tol_outer, o.tol_inner, o.gmres_rtol, o.sigma, o.alpha_min,
                       o.gmres_restart, o.max_outer, o.max_inner, o.max_gmres, o.precision,
                       o.max_refine, o.continuation, k, getattr(o, "tol_inner_rel", -1.0),
                       getattr(o, "fallback_rho", 1.0),
                       None if eps_snapshots is None else _ptr(eps_snapshots), int(getattr(o, "coarse", 0)))


# ---------------------------------------------------------------- entry points
def rsp_version():
    return load().rsp_version()


def rsp_last_error():
    return load().rsp_last_error().decode()


def rsp_partition(prob):
    """Returns (S, txm, tym, boxes[S][8]) (host)."""
    lib = load()
    S, tx, ty = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib.rsp_partition(ctypes.byref(prob), ctypes.byref(S), ctypes.byref(tx),
                             ctypes.byref(ty), None))
    boxes = (ctypes.c_int32 * (8 * S.value))()
    _check(lib.rsp_partition(ctypes.byref(prob), None, None, None, boxes))
    b = [list(boxes[8 * i:8 * i + 8]) for i in range(S.value)]
    return S.value, tx.value, ty.value, b


def rsp_workspace_bytes(prob, opts):
    return load().rsp_workspace_bytes(ctypes.byref(prob), ctypes.byref(opts))


def rsp_context_create(device=0, hbm_budget=0):
    h = ctypes.c_void_p()
    _check(load().rsp_context_create(ctypes.byref(h), device, hbm_budget))
    return h


def rsp_context_destroy(ctx):
    return _check(load().rsp_context_destroy(ctx))


def rsp_setup(ctx, prob, opts, yd, f=None, stream=None):
    return _check(load().rsp_setup(ctx, ctypes.byref(prob), ctypes.byref(opts), _ptr(yd),
                                   _ptr(f, True), _stream(stream)))


def rsp_residual(ctx, x, eps, out, stream=None):
    return _check(load().rsp_residual(ctx, _ptr(x), eps, _ptr(out), _stream(stream)))


def rsp_control(ctx, p, eps, u, stream=None):
    return _check(load().rsp_control(ctx, _ptr(p), eps, _ptr(u), _stream(stream)))


def rsp_restrict(ctx, x, tiles, stream=None):
    return _check(load().rsp_restrict(ctx, _ptr(x), _ptr(tiles), _stream(stream)))


def rsp_prolong(ctx, tiles, out, stream=None):
    return _check(load().rsp_prolong(ctx, _ptr(tiles), _ptr(out), _stream(stream)))


def rsp_local_residual(ctx, x, c, eps, out, norms, stream=None):
    return _check(load().rsp_local_residual(ctx, _ptr(x), _ptr(c), eps, _ptr(out), _ptr(norms),
                                            _stream(stream)))


def rsp_local_residual_noalloc(prob, yd, f, x, c, eps, out, norms, stream=None):
    """rsp_local_residual without a context and without device allocation."""
    return _check(load().rsp_local_residual_noalloc(ctypes.byref(prob), _ptr(yd), _ptr(f, True), _ptr(x),
                                                    _ptr(c), eps, _ptr(out), _ptr(norms), _stream(stream)))


def rsp_local_solve(ctx, x, c, eps, rhs, z, stream=None):
    return _check(load().rsp_local_solve(ctx, _ptr(x), _ptr(c), eps, _ptr(rhs), _ptr(z),
                                         _stream(stream)))


def rsp_eval(ctx, x, continuation, out, stream=None):
    """Algorithm 3.  Returns (status, |out|_2)."""
    nrm = ctypes.c_double()
    st = _check(load().rsp_eval(ctx, _ptr(x), int(continuation), _ptr(out), ctypes.byref(nrm),
                                _stream(stream)))
    return st, nrm.value


def rsp_jac_apply(ctx, d, out, stream=None):
    return _check(load().rsp_jac_apply(ctx, _ptr(d), _ptr(out), _stream(stream)))


def rsp_coarse_jac_apply(ctx, x, d, out, stream=None):
    """The two-level outer Newton operator at x (rsp_coarse_jac_apply)."""
    return _check(load().rsp_coarse_jac_apply(ctx, _ptr(x), _ptr(d), _ptr(out), _stream(stream)))


def rsp_solve(ctx, prob, opts, yd, f, y0, p0, y, p, u, stream=None):
    """Algorithm 2.  Returns (status, history dict)."""
    h = rsp_history()
    st = _check(load().rsp_solve(ctx, ctypes.byref(prob), ctypes.byref(opts), _ptr(yd),
                                 _ptr(f, True), _ptr(y0, True), _ptr(p0, True), _ptr(y), _ptr(p),
                                 _ptr(u), ctypes.byref(h), _stream(stream)))
    return st, h.as_dict()


def rsp_solve_newton_ras(ctx, prob, opts, yd, f, y0, p0, y, p, u, stream=None):
    """Newton_RAS,eps (rsp_solve_newton_ras).  Returns (status, history dict)."""
    h = rsp_history()
    st = _check(load().rsp_solve_newton_ras(ctx, ctypes.byref(prob), ctypes.byref(opts), _ptr(yd),
                                            _ptr(f, True), _ptr(y0, True), _ptr(p0, True), _ptr(y),
                                            _ptr(p), _ptr(u), ctypes.byref(h), _stream(stream)))
    return st, h.as_dict()


def rsp_solve_newton(ctx, prob, opts, yd, f, y0, p0, y, p, u, stream=None):
    """Newton_eps, unpreconditioned GMRES (rsp_solve_newton).  Returns (status, history dict)."""
    h = rsp_history()
    st = _check(load().rsp_solve_newton(ctx, ctypes.byref(prob), ctypes.byref(opts), _ptr(yd),
                                        _ptr(f, True), _ptr(y0, True), _ptr(p0, True), _ptr(y),
                                        _ptr(p), _ptr(u), ctypes.byref(h), _stream(stream)))
    return st, h.as_dict()


def _ptr_array(ts, allow_none=False):
    """Host array of device pointers (NULL array when every entry is None and allowed)."""
    if ts is None or (allow_none and all(t is None for t in ts)):
        if allow_none:
            return None
        raise ValueError("array argument is required")
    arr = (ctypes.c_void_p * len(ts))()
    for i, t in enumerate(ts):
        p = _ptr(t, allow_none)
        arr[i] = p.value if p is not None else None
    return arr


def rsp_solve_batch(ctx, probs, opts, yd, f, y0, p0, y, p, u, stream=None):
    """Algorithm 2 for a batch.  probs: list of rsp_problem; yd .. u: lists of tensors
    (f, y0, p0 may be None or hold None).  Returns (status, [history dicts]); the
    status is RSP_ENUMERIC when an instance ended with it (the others' results and
    histories are complete), other hard errors raise."""
    n = len(probs)
    parr = (rsp_problem * n)(*probs)
    hist = (rsp_history * n)()
    none = [None] * n
    st = load().rsp_solve_batch(ctx, n, parr, ctypes.byref(opts), _ptr_array(yd),
                                _ptr_array(f if f is not None else none, True),
                                _ptr_array(y0 if y0 is not None else none, True),
                                _ptr_array(p0 if p0 is not None else none, True),
                                _ptr_array(y), _ptr_array(p), _ptr_array(u), hist, _stream(stream))
    if st != RSP_ENUMERIC:
        _check(st)
    return st, [h.as_dict() for h in hist]


def rsp_batch_workspace_bytes(probs, opts):
    n = len(probs)
    parr = (rsp_problem * n)(*probs)
    return load().rsp_batch_workspace_bytes(n, parr, ctypes.byref(opts))


def rsp_server_create(opts, device=0, max_batch=0, hbm_budget=0, tune=None, profile_every=0):
    """Start a server; opts: rsp_options of every request; tune: rsp_tuning or None."""
    h = ctypes.c_void_p()
    so = rsp_server_options(device, max_batch, hbm_budget, opts, tune if tune is not None else rsp_tuning(),
                            profile_every)
    _check(load().rsp_server_create(ctypes.byref(h), ctypes.byref(so)))
    return h


def rsp_server_submit(srv, prob, yd, f, y, p, u):
    """Queue a solve; the tensors must stay alive until the ticket is done.  Returns the ticket."""
    t = ctypes.c_uint64()
    _check(load().rsp_server_submit(srv, ctypes.byref(prob), _ptr(yd), _ptr(f, True), _ptr(y), _ptr(p),
                                    _ptr(u), ctypes.byref(t)))
    return t.value


def rsp_server_poll(srv, ticket):
    st = ctypes.c_int32()
    _check(load().rsp_server_poll(srv, ticket, ctypes.byref(st)))
    return st.value


def rsp_server_wait(srv, ticket, timeout_ms=-1.0):
    """Returns (status, history dict); raises RaspenError on a hard error or RSP_EAGAIN."""
    h = rsp_history()
    st = _check(load().rsp_server_wait(srv, ticket, float(timeout_ms), ctypes.byref(h)))
    return st, h.as_dict()


def rsp_server_stats(srv):
    r = rsp_server_report()
    _check(load().rsp_server_stats(srv, ctypes.byref(r)))
    return {k: getattr(r, k) for k, _ in rsp_server_report._fields_}


def rsp_server_kernel_stats(srv):
    """Returns {name: dict(launches, ms, flops, bytes)} of the server's main batch."""
    lib = load()
    n = ctypes.c_int32()
    _check(lib.rsp_server_kernel_stats(srv, None, 0, ctypes.byref(n)))
    arr = (rsp_kernel_stat * max(1, n.value))()
    _check(lib.rsp_server_kernel_stats(srv, arr, n.value, ctypes.byref(n)))
    return {a.name.decode(): dict(launches=a.launches, ms=a.ms, flops=a.flops, bytes=a.bytes)
            for a in arr[:n.value]}


def rsp_server_destroy(srv):
    return _check(load().rsp_server_destroy(srv))


def rsp_set_profiling(ctx, on=True):
    return _check(load().rsp_set_profiling(ctx, int(on)))


def rsp_get_tuning(ctx):
    t = rsp_tuning()
    _check(load().rsp_get_tuning(ctx, ctypes.byref(t)))
    return t


def rsp_set_tuning(ctx, graphs=None, gm_chunk=None, jac_form=None):
    t = rsp_get_tuning(ctx)
    if graphs is not None:
        t.graphs = int(graphs)
    if gm_chunk is not None:
        t.gm_chunk = int(gm_chunk)
    if jac_form is not None:
        t.jac_form = int(jac_form)
    return _check(load().rsp_set_tuning(ctx, ctypes.byref(t)))


def rsp_autotune(ctx, prob, opts, yd, f, flags=0, stream=None):
    t = rsp_tuning()
    _check(load().rsp_autotune(ctx, ctypes.byref(prob), ctypes.byref(opts), _ptr(yd), _ptr(f, True),
                               int(flags), ctypes.byref(t), _stream(stream)))
    return t


def rsp_set_profiling_filter(ctx, name=None):
    return _check(load().rsp_set_profiling_filter(ctx, name.encode() if name else None))


def rsp_set_profiling_sample(ctx, every):
    """Time the launches of one in `every` launch sequences (rsp_set_profiling_sample)."""
    return _check(load().rsp_set_profiling_sample(ctx, int(every)))


def rsp_reset_kernel_stats(ctx):
    return _check(load().rsp_reset_kernel_stats(ctx))


def rsp_kernel_stats(ctx):
    """Returns {name: dict(launches, ms, flops, bytes)}."""
    lib = load()
    n = ctypes.c_int32()
    _check(lib.rsp_kernel_stats(ctx, None, 0, ctypes.byref(n)))
    arr = (rsp_kernel_stat * n.value)()
    _check(lib.rsp_kernel_stats(ctx, arr, n.value, ctypes.byref(n)))
    return {a.name.decode(): dict(launches=a.launches, ms=a.ms, flops=a.flops, bytes=a.bytes)
            for a in arr[:n.value]}
