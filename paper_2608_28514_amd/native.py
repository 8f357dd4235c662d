"""Thin ctypes binding of libns.so (include/ns.h).

Argument marshalling only: every step of the sampler runs in the library's
HIP kernels.  Functions keep the C names (``ns_init``, ``ns_step_batch``,
``ns_logZ`` ...); ``Sampler`` is a small convenience wrapper.  Device buffers
and the stream come from PyTorch (``torch.cuda``); the library is loaded from
this directory and its absence is an error, never a fallback.
"""
import ctypes as C
import os
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libns.so")
_lib = None

NS_OK, NS_DONE = 0, 1
STATUS = {0: "NS_OK", 1: "NS_DONE", -1: "NS_EINVAL", -2: "NS_ENOMEM", -3: "NS_EDEVICE",
          -4: "NS_ESTATE", -5: "NS_ENUMERIC"}
PREC = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}
CORR = {"none": 0, "best_of_worst": 1, "sort": 2, "history": 3}
LIK = {"mixture": 0, "rosenbrock": 1, "shell": 2, "mlp": 3, "callback": 4}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_i64p = C.POINTER(C.c_int64)


# int callback(void* user, const double* theta, int64_t n, int d, double* logL)
LIK_CALLBACK = C.CFUNCTYPE(C.c_int, C.c_void_p, _dp, C.c_int64, C.c_int, _dp)


class NsLikelihood(C.Structure):
    _fields_ = [("kind", C.c_int), ("prec", C.c_int), ("n_comp", C.c_int),
                ("logw", _dp), ("mu", _dp), ("ivar", _dp),
                ("ros_a", C.c_double), ("ros_b", C.c_double),
                ("shell_r0", C.c_double), ("shell_w", C.c_double),
                ("n_layers", C.c_int), ("widths", _ip), ("weights", _dp), ("biases", _dp),
                ("data", _dp), ("sigma", _dp), ("callback", LIK_CALLBACK), ("callback_user", C.c_void_p)]


class NsConfig(C.Structure):
    _fields_ = [("slice_steps_per_dim", C.c_int), ("step_width", C.c_double),
                ("max_stepout", C.c_int), ("max_shrink", C.c_int), ("tree_depth", C.c_int),
                ("split_vol_frac", C.c_double), ("min_cluster_pts", C.c_int),
                ("recluster_every", C.c_int), ("kmeans_iters", C.c_int), ("correction", C.c_int),
                ("history_iters", C.c_int), ("hist_cap", C.c_int), ("state_prec", C.c_int),
                ("stop_frac", C.c_double), ("eig_floor", C.c_double), ("seed", C.c_uint64),
                ("batch_rounds", C.c_int), ("stepout_spec", C.c_int), ("shrink_spec", C.c_int),
                ("fused_chains", C.c_int),
                ("wait_limit", C.c_int)]


class NsStats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("dead", C.c_int64), ("evals", C.c_int64),
                ("oob", C.c_int64), ("stepout_caps", C.c_int64), ("shrink_caps", C.c_int64),
                ("clusterings", C.c_int64), ("nan_logL", C.c_int64), ("done", C.c_int32),
                ("n_clusters", C.c_int32), ("screened", C.c_int64), ("net_rows", C.c_int64)]


class NsSurrogateConfig(C.Structure):
    _fields_ = [("hidden", C.c_int), ("replay_cap", C.c_int), ("batch", C.c_int), ("train_every", C.c_int),
                ("train_iters", C.c_int), ("lr", C.c_float), ("margin", C.c_double),
                ("floor_below", C.c_double), ("audit_period", C.c_int), ("max_fn_rate", C.c_double),
                ("min_pairs", C.c_int), ("prec", C.c_int), ("seed", C.c_uint64)]


class NsSurrogateStats(C.Structure):
    _fields_ = [("pairs", C.c_int64), ("net_rows", C.c_int64), ("screened", C.c_int64),
                ("audited", C.c_int64), ("false_screens", C.c_int64), ("train_calls", C.c_int64),
                ("screening", C.c_int32), ("disabled", C.c_int32), ("last_loss", C.c_double)]


class NsMlpDesc(C.Structure):
    _fields_ = [("n_layers", C.c_int), ("widths", C.c_int * 9), ("act", C.c_int),
                ("W", C.c_void_p * 8), ("b", C.c_void_p * 8)]


ACT = {"tanh": 1, "silu": 2}


class NsError(RuntimeError):
    pass


def lib():
    """Load libns.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NsError("libns.so is not built: run __graft_entry__.build() "
                          "(there is no CPU fallback)")
        # PyTorch first: the library then binds to the HIP runtime torch has
        # loaded (same soname), so device memory, streams and kernels share
        # one runtime in the process
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        sigs = {
            "ns_config_default": [C.POINTER(NsConfig)],
            "ns_init": [C.POINTER(vp), _dp, _dp, C.c_int, C.c_int, C.POINTER(NsConfig),
                        C.POINTER(NsLikelihood), vp],
            "ns_step_batch": [vp, C.c_int],
            "ns_run": [vp, C.c_int, C.c_int64, _i64p],
            "ns_sync": [vp],
            "ns_run_many": [C.POINTER(vp), C.c_int, C.c_int, C.c_int64, _i64p],
            "ns_logZ": [vp, _dp, _dp, _dp],
            "ns_get_dead": [vp, _i64p, _dp, _dp, _dp, _dp],
            "ns_get_live": [vp, _dp, _dp, _ip],
            "ns_set_live": [vp, _dp, _dp, _ip],
            "ns_get_tree": [vp, _ip, _ip, _ip, _ip, _dp, _dp, _dp],
            "ns_get_last_batch": [vp, _ip, _ip, _dp, _dp, _dp, _i64p, _dp, _dp, _ip],
            "ns_stats": [vp, C.POINTER(NsStats)],
            "ns_loglike_batch": [vp, vp, C.c_int64, vp],
            "ns_select_order": [vp, C.c_int, vp, vp],
            "ns_select_worst_work_bytes": [],
            "ns_select_worst": [vp, C.c_int64, C.c_int, vp, vp, vp, vp],
            "ns_select_worst_noalloc": [vp, C.c_int64, C.c_int, vp, vp, vp],
            "ns_cluster_split_work_bytes": [],
            "ns_cluster_split": [vp, C.c_int64, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp],
            "ns_correct_batch": [C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp,
                                 vp, vp, vp, vp],
            "ns_philox": [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64, vp,
                          vp],
            "ns_set_timing": [vp, C.c_int],
            "ns_surrogate_default": [C.POINTER(NsSurrogateConfig)],
            "ns_surrogate_enable": [vp, C.POINTER(NsSurrogateConfig)],
            "ns_surrogate_stats": [vp, C.POINTER(NsSurrogateStats)],
            "ns_surrogate_predict": [vp, vp, C.c_int64, vp],
            "ns_mlp_forward": [C.POINTER(NsMlpDesc), C.c_int, vp, C.c_int64, vp, vp, vp, vp],
            "ns_mlp_backward": [C.POINTER(NsMlpDesc), C.c_int, vp, C.c_int64, vp, vp, vp,
                                C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), vp, vp, vp],
            "ns_get_timing": [vp, _dp, _i64p],
        }
        for name, args in sigs.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.ns_select_worst_work_bytes.restype = C.c_size_t
        L.ns_cluster_split_work_bytes.restype = C.c_size_t
        L.ns_last_error.argtypes = [vp]
        L.ns_last_error.restype = C.c_char_p
        L.ns_free.argtypes = [vp]
        L.ns_free.restype = None
        _lib = L
    return _lib


def _check(rc, ctx=None, what=""):
    if rc < 0:
        msg = lib().ns_last_error(ctx).decode(errors="replace")
        raise NsError(f"{what}: {STATUS.get(rc, rc)}: {msg}")
    return rc


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


# ------------------------------------------------------------------ C names
def ns_config_default():
    c = NsConfig()
    _check(lib().ns_config_default(C.byref(c)), None, "ns_config_default")
    return c


def make_likelihood(spec, prec="f64"):
    """ns_likelihood from a workload dict; returns (struct, keep-alive list)."""
    L = NsLikelihood()
    keep = []
    L.kind = LIK[spec["kind"]]
    L.prec = PREC[prec]
    if spec["kind"] == "mixture":
        a = [_f64(spec["logw"]), _f64(spec["mu"]), _f64(spec["ivar"])]
        keep += a
        L.n_comp = a[0].size
        L.logw, L.mu, L.ivar = _d(a[0]), _d(a[1]), _d(a[2])
    elif spec["kind"] == "rosenbrock":
        L.ros_a, L.ros_b = spec.get("a", 1.0), spec.get("b", 100.0)
    elif spec["kind"] == "shell":
        L.shell_r0, L.shell_w = spec.get("r0", 5.0), spec.get("w", 1.0)
    elif spec["kind"] == "callback":
        fn = spec["fn"]

        def _call(user, theta, n, d, out):
            # marshalling only: numpy views of the library's host arrays
            try:
                t = np.ctypeslib.as_array(theta, shape=(int(n), int(d)))
                np.ctypeslib.as_array(out, shape=(int(n),))[:] = np.asarray(fn(t), dtype=np.float64)
                return 0
            except Exception:      # reported to the library as a failed call
                return 1

        cb = LIK_CALLBACK(_call)
        keep.append(cb)
        L.callback = cb
    elif spec["kind"] == "mlp":
        widths = np.ascontiguousarray(np.asarray(spec["widths"], dtype=np.int32))
        W = _f64(np.concatenate([np.asarray(w, dtype=np.float64).ravel() for w in spec["weights"]]))
        b = _f64(np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in spec["biases"]]))
        data, sigma = _f64(spec["data"]), _f64(spec["sigma"])
        keep += [widths, W, b, data, sigma]
        L.n_layers = widths.size - 1
        L.widths = widths.ctypes.data_as(_ip)
        L.weights, L.biases, L.data, L.sigma = _d(W), _d(b), _d(data), _d(sigma)
    return L, keep


def ns_init(spec, n_live, cfg, prec="f64", stream=None, keep=None):
    """keep (list, optional): receives the objects a callback likelihood needs
    for the life of the context."""
    L, kp = make_likelihood(spec, prec)
    if keep is not None:
        keep.extend(kp)
    lo, hi = _f64(spec["lo"]), _f64(spec["hi"])
    ctx = C.c_void_p()
    rc = lib().ns_init(C.byref(ctx), _d(lo), _d(hi), int(spec["d"]), int(n_live), C.byref(cfg),
                       C.byref(L), _stream(stream))
    _check(rc, None, "ns_init")
    return ctx


def ns_step_batch(ctx, m):
    return _check(lib().ns_step_batch(ctx, int(m)), ctx, "ns_step_batch")


def ns_run(ctx, m, max_steps=2 ** 62):
    n = C.c_int64()
    rc = _check(lib().ns_run(ctx, int(m), int(max_steps), C.byref(n)), ctx, "ns_run")
    return rc, n.value


def ns_run_many(ctxs, m, max_steps=2 ** 62):
    """Run the contexts ctxs (a list of ns_ctx handles) to their stopping rule
    at once; returns (status, steps per context)."""
    R = len(ctxs)
    arr = (C.c_void_p * R)(*[c.value if isinstance(c, C.c_void_p) else c for c in ctxs])
    st = np.zeros(R, dtype=np.int64)
    rc = lib().ns_run_many(arr, R, int(m), int(max_steps), st.ctypes.data_as(_i64p))
    if rc < 0:
        for c in ctxs:
            msg = lib().ns_last_error(c).decode(errors="replace")
            if msg:
                raise NsError(f"ns_run_many: {STATUS.get(rc, rc)}: {msg}")
        raise NsError(f"ns_run_many: {STATUS.get(rc, rc)}: {lib().ns_last_error(None).decode(errors='replace')}")
    return rc, st


def run_many(samplers, m, max_steps=2 ** 62):
    """ns_run_many over Sampler objects."""
    return ns_run_many([s.ctx for s in samplers], m, max_steps)


def ns_sync(ctx):
    _check(lib().ns_sync(ctx), ctx, "ns_sync")


def ns_logZ(ctx):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    _check(lib().ns_logZ(ctx, C.byref(a), C.byref(b), C.byref(c)), ctx, "ns_logZ")
    return a.value, b.value, c.value


def ns_get_dead(ctx, d):
    n = C.c_int64()
    _check(lib().ns_get_dead(ctx, C.byref(n), None, None, None, None), ctx, "ns_get_dead")
    n = n.value
    u, l, x, w = np.zeros((n, d)), np.zeros(n), np.zeros(n), np.zeros(n)
    nn = C.c_int64()
    if n:
        _check(lib().ns_get_dead(ctx, C.byref(nn), _d(u), _d(l), _d(x), _d(w)), ctx, "ns_get_dead")
    return {"u": u, "logL": l, "logX": x, "logw": w}


def ns_get_live(ctx, N, d):
    u, l, lab = np.zeros((N, d)), np.zeros(N), np.zeros(N, dtype=np.int32)
    _check(lib().ns_get_live(ctx, _d(u), _d(l), lab.ctypes.data_as(_ip)), ctx, "ns_get_live")
    return {"u": u, "logL": l, "label": lab}


def ns_set_live(ctx, u=None, logL=None, label=None):
    u = None if u is None else _f64(u)
    logL = None if logL is None else _f64(logL)
    lab = None if label is None else np.ascontiguousarray(np.asarray(label, dtype=np.int32))
    _check(lib().ns_set_live(ctx, _d(u) if u is not None else None,
                             _d(logL) if logL is not None else None,
                             lab.ctypes.data_as(_ip) if lab is not None else None), ctx, "ns_set_live")


def ns_get_tree(ctx, d, depth):
    nodes = (1 << (depth + 1)) - 1
    n = C.c_int()
    cnt, acc, sok = (np.zeros(nodes, dtype=np.int32) for _ in range(3))
    logV, cen, chol = np.zeros(nodes), np.zeros((nodes, d)), np.zeros((nodes, d, d))
    ip = lambda a: a.ctypes.data_as(_ip)
    _check(lib().ns_get_tree(ctx, C.byref(n), ip(cnt), ip(acc), ip(sok), _d(logV), _d(cen), _d(chol)),
           ctx, "ns_get_tree")
    return {"n_nodes": n.value, "count": cnt, "accepted": acc, "split_ok": sok, "logV": logV,
            "centre": cen, "chol": chol}


def ns_get_last_batch(ctx, d, T, m_max=1024):
    m = C.c_int()
    _check(lib().ns_get_last_batch(ctx, C.byref(m), None, None, None, None, None, None, None, None),
           ctx, "ns_get_last_batch")
    m = m.value
    out = {"seeds": np.zeros(m, dtype=np.int32), "tau": np.zeros(m), "new_u": np.zeros((m, d)),
           "new_logL": np.zeros(m), "chain_evals": np.zeros(m, dtype=np.int64),
           "hist_logL": np.zeros((T, m)), "hist_u": np.zeros((m, T, d)),
           "hist_n": np.zeros(m, dtype=np.int32)}
    mm = C.c_int()
    _check(lib().ns_get_last_batch(ctx, C.byref(mm), out["seeds"].ctypes.data_as(_ip), _d(out["tau"]),
                                   _d(out["new_u"]), _d(out["new_logL"]),
                                   out["chain_evals"].ctypes.data_as(_i64p), _d(out["hist_logL"]),
                                   _d(out["hist_u"]), out["hist_n"].ctypes.data_as(_ip)),
           ctx, "ns_get_last_batch")
    return out


def ns_stats(ctx):
    s = NsStats()
    _check(lib().ns_stats(ctx, C.byref(s)), ctx, "ns_stats")
    return {k: getattr(s, k) for k, _ in NsStats._fields_}


def ns_loglike_batch(ctx, d_u, d_out):
    """d_u: torch float64 (n, d) on the device; d_out: torch float64 (n,)."""
    _check(lib().ns_loglike_batch(ctx, _ptr(d_u), int(d_out.numel()), _ptr(d_out)), ctx,
           "ns_loglike_batch")


def ns_select_worst(d_logL, m, d_slots, d_work, d_passes=None, stream=None):
    """The m worst entries of d_logL (torch float64, device) into d_slots
    (torch int32, device), ascending; d_work: a device buffer of at least
    ns_select_worst_work_bytes() bytes; d_passes: optional int32 device tensor."""
    _check(lib().ns_select_worst(_ptr(d_logL), int(d_logL.numel()), int(m), _ptr(d_slots), _ptr(d_work),
                                 _ptr(d_passes) if d_passes is not None else None, _stream(stream)),
           None, "ns_select_worst")


def ns_select_worst_noalloc(d_logL, m, d_slots, d_passes=None, stream=None):
    """ns_select_worst without a workspace argument (the library's static
    per-device workspace; nothing is allocated)."""
    _check(lib().ns_select_worst_noalloc(_ptr(d_logL), int(d_logL.numel()), int(m), _ptr(d_slots),
                                         _ptr(d_passes) if d_passes is not None else None, _stream(stream)),
           None, "ns_select_worst_noalloc")


def ns_select_worst_work_bytes():
    return int(lib().ns_select_worst_work_bytes())


def ns_cluster_split(d_u, iters, d_mean, d_cov, d_centres, d_side, d_work, d_passes=None, stream=None):
    """One cluster-tree node of the points d_u (torch float32 (N, d), device):
    mean (d), covariance (d, d), centres (2, 32) and side (N, uint8)."""
    N, d = d_u.shape
    _check(lib().ns_cluster_split(_ptr(d_u), int(N), int(d), int(iters), _ptr(d_mean), _ptr(d_cov),
                                  _ptr(d_centres), _ptr(d_side), _ptr(d_work),
                                  _ptr(d_passes) if d_passes is not None else None, _stream(stream)),
           None, "ns_cluster_split")


def ns_cluster_split_work_bytes():
    return int(lib().ns_cluster_split_work_bytes())


def ns_select_order(d_logL, d_order, stream=None):
    _check(lib().ns_select_order(_ptr(d_logL), int(d_logL.numel()), _ptr(d_order), _stream(stream)),
           None, "ns_select_order")


def ns_correct_batch(m, corr, K, T, d_wlogL, d_nlogL, d_P, d_hist, d_hist_n, outs, stream=None):
    """outs: dict of device tensors acc_code, acc_hslot, acc_logL, rej_code, rej_hslot, rej_logL."""
    c = CORR[corr] if isinstance(corr, str) else int(corr)
    _check(lib().ns_correct_batch(int(m), c, int(K), int(T), _ptr(d_wlogL), _ptr(d_nlogL), _ptr(d_P),
                                  _ptr(d_hist), _ptr(d_hist_n), _ptr(outs["acc_code"]),
                                  _ptr(outs["acc_hslot"]), _ptr(outs["acc_logL"]),
                                  _ptr(outs["rej_code"]), _ptr(outs["rej_hslot"]),
                                  _ptr(outs["rej_logL"]), _stream(stream)), None, "ns_correct_batch")


def ns_philox(seed, c0, c1, c2, c3, n, d_out, stream=None):
    _check(lib().ns_philox(int(seed), c0, c1, c2, c3, int(n), _ptr(d_out), _stream(stream)), None,
           "ns_philox")


TIMING_CLASSES = ("select", "slice", "correct", "cluster", "lik", "draws")


TIMING_ALL = 0x3F


def ns_set_timing(ctx, on=True):
    """on: True (every class), False (none), or a bitmask of 1 << class index."""
    mask = TIMING_ALL if on is True else (0 if on is False else int(on))
    _check(lib().ns_set_timing(ctx, mask), ctx, "ns_set_timing")


def ns_get_timing(ctx):
    ms = np.zeros(len(TIMING_CLASSES))
    n = np.zeros(len(TIMING_CLASSES), dtype=np.int64)
    _check(lib().ns_get_timing(ctx, _d(ms), n.ctypes.data_as(_i64p)), ctx, "ns_get_timing")
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(TIMING_CLASSES)}


def mlp_desc(Ws, bs, act):
    """ns_mlp_desc over device tensors Ws[l] (widths[l] x widths[l+1], float32) and bs[l]."""
    d = NsMlpDesc()
    d.n_layers = len(Ws)
    widths = [int(Ws[0].shape[0])] + [int(w.shape[1]) for w in Ws]
    for i, w in enumerate(widths):
        d.widths[i] = w
    d.act = ACT[act] if isinstance(act, str) else int(act)
    for l, (w, b) in enumerate(zip(Ws, bs)):
        d.W[l] = w.data_ptr()
        d.b[l] = b.data_ptr()
    return d


def ns_mlp_forward(desc, prec, X, Y, Z=None, H=None, stream=None):
    _check(lib().ns_mlp_forward(C.byref(desc), PREC[prec], _ptr(X), int(X.shape[0]), _ptr(Y),
                                _ptr(Z) if Z is not None else None, _ptr(H) if H is not None else None,
                                _stream(stream)), None, "ns_mlp_forward")


def ns_mlp_backward(desc, prec, X, Z, H, dY, dWs, dbs, dX, work, stream=None):
    L = desc.n_layers
    dW = (C.c_void_p * 8)(*[t.data_ptr() for t in dWs] + [0] * (8 - L))
    db = (C.c_void_p * 8)(*[t.data_ptr() for t in dbs] + [0] * (8 - L))
    _check(lib().ns_mlp_backward(C.byref(desc), PREC[prec], _ptr(X), int(X.shape[0]), _ptr(Z),
                                 _ptr(H) if H is not None else None, _ptr(dY), dW, db,
                                 _ptr(dX) if dX is not None else None, _ptr(work), _stream(stream)),
           None, "ns_mlp_backward")


def ns_surrogate_default():
    c = NsSurrogateConfig()
    _check(lib().ns_surrogate_default(C.byref(c)), None, "ns_surrogate_default")
    return c


def ns_surrogate_enable(ctx, **kw):
    c = ns_surrogate_default()
    for k, v in kw.items():
        if k == "prec" and isinstance(v, str):
            v = PREC[v]
        setattr(c, k, v)
    _check(lib().ns_surrogate_enable(ctx, C.byref(c)), ctx, "ns_surrogate_enable")
    return c


def ns_surrogate_stats(ctx):
    s = NsSurrogateStats()
    _check(lib().ns_surrogate_stats(ctx, C.byref(s)), ctx, "ns_surrogate_stats")
    return {k: getattr(s, k) for k, _ in NsSurrogateStats._fields_}


def ns_surrogate_predict(ctx, d_u, d_out):
    _check(lib().ns_surrogate_predict(ctx, _ptr(d_u), int(d_out.numel()), _ptr(d_out)), ctx,
           "ns_surrogate_predict")


def ns_free(ctx):
    if ctx:
        lib().ns_free(ctx)


# ------------------------------------------------------------------ convenience
class Sampler:
    """``Sampler(spec, n_live, m=..., **config)`` over one ns_ctx."""

    def __init__(self, spec, n_live, prec="f64", state="f64", stream=None, **cfg):
        self.spec = spec
        self.d = int(spec["d"])
        self.N = int(n_live)
        c = ns_config_default()
        c.state_prec = PREC[state]
        for k, v in cfg.items():
            if k == "correction" and isinstance(v, str):
                v = CORR[v]
            setattr(c, k, v)
        self.cfg = c
        self.T = c.hist_cap
        self._keep = [stream]
        self.ctx = ns_init(spec, n_live, c, prec=prec, stream=stream, keep=self._keep)

    def step(self, m):
        return ns_step_batch(self.ctx, m)

    def run(self, m, max_steps=2 ** 62):
        return ns_run(self.ctx, m, max_steps)

    def logZ(self):
        return ns_logZ(self.ctx)

    def dead(self):
        return ns_get_dead(self.ctx, self.d)

    def live(self):
        return ns_get_live(self.ctx, self.N, self.d)

    def set_live(self, **kw):
        ns_set_live(self.ctx, **kw)

    def tree(self):
        return ns_get_tree(self.ctx, self.d, self.cfg.tree_depth)

    def last_batch(self):
        return ns_get_last_batch(self.ctx, self.d, self.T)

    def stats(self):
        return ns_stats(self.ctx)

    def enable_surrogate(self, **kw):
        return ns_surrogate_enable(self.ctx, **kw)

    def surrogate_stats(self):
        return ns_surrogate_stats(self.ctx)

    def timing(self, on=None):
        if on is not None:
            ns_set_timing(self.ctx, on)
        return ns_get_timing(self.ctx)

    def close(self):
        if getattr(self, "ctx", None):
            ns_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
