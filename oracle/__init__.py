"""ctypes wrapper of the FP64 CPU oracle (oracle/liboracle.so).

TEST INFRASTRUCTURE.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It never imports the
GPU package and the GPU package never imports it; both take their inputs from
``paper_2608_28514_amd.workloads`` (seeded input construction only).

Likelihood specifications are plain dicts (see ``workloads.py``):
``{"kind": "mixture"|"rosenbrock"|"shell"|"mlp", "d", "lo", "hi", ...}``.
"""
import ctypes as C
import os
import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MAXD = 32
STREAM_INIT, STREAM_SEED, STREAM_SLICE = 1, 2, 3
SLOT_DIR0, SLOT_STEPOUT, SLOT_SHRINK0 = 0, 16, 32
LIK = {"mixture": 0, "rosenbrock": 1, "shell": 2, "mlp": 3}
CORR = {"none": 0, "best_of_worst": 1, "sort": 2, "history": 3}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_lp = C.POINTER(C.c_long)


class OrcLik(C.Structure):
    _fields_ = [("kind", C.c_int), ("d", C.c_int), ("n_comp", C.c_int),
                ("logw", _dp), ("mu", _dp), ("ivar", _dp),
                ("ros_a", C.c_double), ("ros_b", C.c_double),
                ("shell_r0", C.c_double), ("shell_w", C.c_double),
                ("n_layers", C.c_int), ("widths", _ip), ("weights", _dp), ("biases", _dp),
                ("data", _dp), ("sigma", _dp)]


class OrcConfig(C.Structure):
    _fields_ = [("slice_steps_per_dim", C.c_int), ("step_width", C.c_double),
                ("max_stepout", C.c_int), ("max_shrink", C.c_int), ("tree_depth", C.c_int),
                ("split_vol_frac", C.c_double), ("min_cluster_pts", C.c_int),
                ("recluster_every", C.c_int), ("kmeans_iters", C.c_int), ("correction", C.c_int),
                ("history_iters", C.c_int), ("hist_cap", C.c_int), ("stop_frac", C.c_double),
                ("eig_floor", C.c_double), ("seed", C.c_uint64)]


class OrcTree(C.Structure):
    _fields_ = [("depth", C.c_int), ("d", C.c_int), ("n_nodes", C.c_int),
                ("count", C.c_int * 127), ("split_ok", C.c_int * 127), ("accepted", C.c_int * 127),
                ("logV", C.c_double * 127), ("logV_eff", C.c_double * 127),
                ("centre", C.c_double * (127 * MAXD)),
                ("chol", C.c_double * (127 * MAXD * MAXD))]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError("oracle/liboracle.so is not built (run __graft_entry__.build())")
        L = C.CDLL(_LIB_PATH)
        L.orc_philox4x32_10.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_uniform2.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _dp]
        L.orc_loglike.argtypes = [C.POINTER(OrcLik), _dp, _dp, _dp, C.c_long, _dp]
        L.orc_select.argtypes = [_dp, C.c_int, _ip]
        L.orc_jacobi_eig.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_cholesky.argtypes = [C.c_int, _dp, _dp]
        L.orc_cholesky.restype = C.c_int
        L.orc_regularise.argtypes = [C.c_int, _dp, C.c_double, _dp, _ip]
        L.orc_regularise.restype = C.c_double
        L.orc_cluster.argtypes = [_dp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                  C.c_double, C.POINTER(OrcTree), _ip]
        L.orc_nearest_centre.argtypes = [C.POINTER(OrcTree), _dp]
        L.orc_two_means.argtypes = [_dp, C.c_int, C.c_int, C.c_int, _dp, _dp, _ip]
        L.orc_two_means.restype = None
        L.orc_correct.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _ip,
                                  _ip, _ip, _dp, _ip, _ip, _dp]
        L.orc_config_default.argtypes = [C.POINTER(OrcConfig)]
        L.orc_create.argtypes = [_dp, _dp, C.c_int, C.c_int, C.POINTER(OrcConfig), C.POINTER(OrcLik)]
        L.orc_create.restype = C.c_void_p
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_step.argtypes = [C.c_void_p, C.c_int]
        L.orc_run.argtypes = [C.c_void_p, C.c_int, C.c_long]
        L.orc_run.restype = C.c_long
        L.orc_logZ.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_n_dead.argtypes = [C.c_void_p]
        L.orc_n_dead.restype = C.c_long
        L.orc_get_dead.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.orc_get_live.argtypes = [C.c_void_p, _dp, _dp, _ip]
        L.orc_set_live.argtypes = [C.c_void_p, _dp, _dp, _ip]
        L.orc_get_tree.argtypes = [C.c_void_p, C.POINTER(OrcTree)]
        L.orc_set_tree.argtypes = [C.c_void_p, C.POINTER(OrcTree)]
        L.orc_get_counters.argtypes = [C.c_void_p, _lp]
        L.orc_get_state.argtypes = [C.c_void_p, _dp, _dp, _lp, _ip]
        L.orc_get_last_batch.argtypes = [C.c_void_p, _ip, _dp, _dp, _dp, _lp, _dp, _dp, _ip]
        L.orc_get_last_brackets.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _ip, _ip]
        L.orc_get_last_brackets.restype = None
        L.orc_slice_direction.argtypes = [C.c_uint64, C.c_int, C.c_uint32, C.c_int, _dp, C.c_int, _dp]
        L.orc_slice_direction.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_get_threads.restype = C.c_int
        L.orc_mlp_forward.argtypes = [C.c_int, _ip, _dp, _dp, C.c_int, _dp, C.c_long, _dp, _dp]
        L.orc_mlp_backward.argtypes = [C.c_int, _ip, _dp, _dp, C.c_int, _dp, C.c_long, _dp, _dp,
                                       _dp, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- random numbers
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xffffffff for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xffffffff for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def uniform2(seed, c0, c1, c2, c3):
    o = np.zeros(2)
    lib().orc_uniform2(seed, c0, c1, c2, c3, _d(o))
    return o


# ---------------------------------------------------------------- likelihoods
class _LikHolder:
    """Keeps the numpy buffers referenced by an OrcLik alive."""

    def __init__(self, spec):
        self.keep = []
        L = OrcLik()
        L.kind = LIK[spec["kind"]]
        L.d = int(spec["d"])
        if spec["kind"] == "mixture":
            logw, mu, ivar = (_f64(spec["logw"]), _f64(spec["mu"]), _f64(spec["ivar"]))
            self.keep += [logw, mu, ivar]
            L.n_comp = logw.size
            L.logw, L.mu, L.ivar = _d(logw), _d(mu), _d(ivar)
        elif spec["kind"] == "rosenbrock":
            L.ros_a, L.ros_b = spec.get("a", 1.0), spec.get("b", 100.0)
        elif spec["kind"] == "shell":
            L.shell_r0, L.shell_w = spec.get("r0", 5.0), spec.get("w", 1.0)
        elif spec["kind"] == "mlp":
            widths = np.ascontiguousarray(np.asarray(spec["widths"], dtype=np.int32))
            W = _f64(np.concatenate([np.asarray(w, dtype=np.float64).ravel() for w in spec["weights"]]))
            b = _f64(np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in spec["biases"]]))
            data, sigma = _f64(spec["data"]), _f64(spec["sigma"])
            self.keep += [widths, W, b, data, sigma]
            L.n_layers = widths.size - 1
            L.widths, L.weights, L.biases = _i(widths), _d(W), _d(b)
            L.data, L.sigma = _d(data), _d(sigma)
        else:
            raise ValueError(spec["kind"])
        self.lik = L
        self.lo = _f64(spec["lo"])
        self.hi = _f64(spec["hi"])


def loglike(spec, u):
    """FP64 logL of unit-cube points u (n x d)."""
    h = _LikHolder(spec)
    u = _f64(u).reshape(-1, int(spec["d"]))
    out = np.zeros(u.shape[0])
    lib().orc_loglike(C.byref(h.lik), _d(h.lo), _d(h.hi), _d(u), u.shape[0], _d(out))
    return out


# ---------------------------------------------------------------- selection / clustering
def select(logL):
    x = _f64(logL)
    order = np.zeros(x.size, dtype=np.int32)
    lib().orc_select(_d(x), x.size, _i(order))
    return order


def jacobi_eig(A):
    A = _f64(A)
    d = A.shape[0]
    ev = np.zeros(d)
    Q = np.zeros((d, d))
    lib().orc_jacobi_eig(d, _d(A), _d(ev), _d(Q))
    return ev, Q


def cholesky(A):
    A = _f64(A)
    d = A.shape[0]
    L = np.zeros((d, d))
    rc = lib().orc_cholesky(d, _d(A), _d(L))
    return rc, L


def regularise(cov, eps=1e-8):
    cov = _f64(cov)
    d = cov.shape[0]
    L = np.zeros((d, d))
    clipped = np.zeros(1, dtype=np.int32)
    logV = lib().orc_regularise(d, _d(cov), eps, _d(L), _i(clipped))
    return logV, L, bool(clipped[0])


def tree_to_dict(t):
    n = t.n_nodes
    d = t.d
    cen = np.ctypeslib.as_array(t.centre).reshape(127, MAXD)[:n, :d].copy()
    chol = np.ctypeslib.as_array(t.chol).reshape(127, MAXD, MAXD)[:n, :d, :d].copy()
    return {"n_nodes": n, "count": np.array(t.count[:n]), "split_ok": np.array(t.split_ok[:n]),
            "accepted": np.array(t.accepted[:n]), "logV": np.array(t.logV[:n]),
            "logV_eff": np.array(t.logV_eff[:n]), "centre": cen, "chol": chol}


def cluster(u, depth, p=0.3, nmin=None, iters=20, eps=1e-8):
    u = _f64(u)
    N, d = u.shape
    if nmin is None:
        nmin = 2 * (d + 1)
    t = OrcTree()
    labels = np.zeros(N, dtype=np.int32)
    lib().orc_cluster(_d(u), N, d, depth, p, nmin, iters, eps, C.byref(t), _i(labels))
    return tree_to_dict(t), labels


def make_tree(d, depth, accepted, centre):
    """A hand-built cluster tree (heap indexed, 2^(depth+1) - 1 nodes) with the
    given accepted flags and centres (n_nodes x d), for orc_nearest_centre."""
    t = OrcTree()
    t.depth, t.d = int(depth), int(d)
    t.n_nodes = (1 << (depth + 1)) - 1
    cen = np.asarray(centre, dtype=np.float64)
    for n in range(t.n_nodes):
        t.accepted[n] = int(accepted[n])
        for i in range(d):
            t.centre[n * MAXD + i] = float(cen[n, i])
    return t


def nearest_centre(tree, x):
    """Accepted node whose centre is nearest to x (Sec. 2.1, last paragraph)."""
    return int(lib().orc_nearest_centre(C.byref(tree), _d(_f64(x))))


def two_means(u, iters=20):
    """k-means split (k = 2) of all points u (n x d) as one tree node: (ca, cb, side)."""
    u = _f64(u)
    n, d = u.shape
    ca, cb = np.zeros(d), np.zeros(d)
    side = np.zeros(n, dtype=np.int32)
    lib().orc_two_means(_d(u), n, d, iters, _d(ca), _d(cb), _i(side))
    return ca, cb, side


def correct(m, corr, K, T, wlogL, nlogL, P, hist, hist_n):
    """Algorithms 1/2 on explicit arrays.  hist: T x m (column = chain)."""
    wl, nl, Pp, H = _f64(wlogL), _f64(nlogL), _f64(P), _f64(hist).reshape(T, m)
    hn = np.ascontiguousarray(np.asarray(hist_n, dtype=np.int32))
    out = [np.zeros(m, dtype=np.int32), np.zeros(m, dtype=np.int32), np.zeros(m),
           np.zeros(m, dtype=np.int32), np.zeros(m, dtype=np.int32), np.zeros(m)]
    lib().orc_correct(m, CORR[corr] if isinstance(corr, str) else corr, K, T, _d(wl), _d(nl), _d(Pp),
                      _d(H), _i(hn), _i(out[0]), _i(out[1]), _d(out[2]), _i(out[3]), _i(out[4]),
                      _d(out[5]))
    keys = ["acc_code", "acc_hslot", "acc_logL", "rej_code", "rej_hslot", "rej_logL"]
    return dict(zip(keys, out))


# ---------------------------------------------------------------- sampler
def default_config():
    c = OrcConfig()
    lib().orc_config_default(C.byref(c))
    return c


class Oracle:
    """The batched nested sampler, FP64, step by step."""

    def __init__(self, spec, n_live, **cfg):
        self.spec = spec
        self._h = _LikHolder(spec)
        self.d = int(spec["d"])
        self.N = int(n_live)
        c = default_config()
        for k, v in cfg.items():
            if k == "correction" and isinstance(v, str):
                v = CORR[v]
            setattr(c, k, v)
        self.cfg = c
        self.T = c.hist_cap
        self.ctx = lib().orc_create(_d(self._h.lo), _d(self._h.hi), self.d, self.N, C.byref(c),
                                    C.byref(self._h.lik))
        if not self.ctx:
            raise ValueError("orc_create rejected the arguments")

    def __del__(self):
        try:
            if self.ctx:
                lib().orc_free(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def step(self, m):
        return lib().orc_step(self.ctx, int(m))

    def run(self, m, max_steps=10 ** 9):
        return lib().orc_run(self.ctx, int(m), int(max_steps))

    def logZ(self):
        a, b, c = C.c_double(), C.c_double(), C.c_double()
        lib().orc_logZ(self.ctx, C.byref(a), C.byref(b), C.byref(c))
        return a.value, b.value, c.value

    def n_dead(self):
        return lib().orc_n_dead(self.ctx)

    def dead(self):
        n = self.n_dead()
        u = np.zeros((n, self.d)); l = np.zeros(n); x = np.zeros(n); w = np.zeros(n)
        if n:
            lib().orc_get_dead(self.ctx, _d(u), _d(l), _d(x), _d(w))
        return {"u": u, "logL": l, "logX": x, "logw": w}

    def live(self):
        u = np.zeros((self.N, self.d)); l = np.zeros(self.N); lab = np.zeros(self.N, dtype=np.int32)
        lib().orc_get_live(self.ctx, _d(u), _d(l), _i(lab))
        return {"u": u, "logL": l, "label": lab}

    def set_live(self, u=None, logL=None, label=None):
        u = None if u is None else _f64(u)
        logL = None if logL is None else _f64(logL)
        label = None if label is None else np.ascontiguousarray(np.asarray(label, dtype=np.int32))
        lib().orc_set_live(self.ctx, _d(u) if u is not None else None,
                           _d(logL) if logL is not None else None,
                           _i(label) if label is not None else None)

    def tree(self):
        t = OrcTree()
        lib().orc_get_tree(self.ctx, C.byref(t))
        return tree_to_dict(t)

    def counters(self):
        o = np.zeros(8, dtype=np.int64)
        lib().orc_get_counters(self.ctx, o.ctypes.data_as(_lp))
        keys = ["evals", "oob", "stepout_caps", "shrink_caps", "steps", "dead", "nan", "clusterings"]
        return dict(zip(keys, [int(x) for x in o]))

    def state(self):
        a, b, s, dn = C.c_double(), C.c_double(), C.c_long(), C.c_int()
        lib().orc_get_state(self.ctx, C.byref(a), C.byref(b), C.byref(s), C.byref(dn))
        return {"logZ_run": a.value, "A_run": b.value, "step": s.value, "done": bool(dn.value)}

    def last_brackets(self, m):
        """Per chain of the last step: start point x0 and direction v of the
        last slice iteration, its stepped-out bracket [a, b] and the steps ka,
        kb taken on each side (before shrinking)."""
        d = self.d
        out = {"x0": np.zeros((m, d)), "v": np.zeros((m, d)), "a": np.zeros(m), "b": np.zeros(m),
               "ka": np.zeros(m, dtype=np.int32), "kb": np.zeros(m, dtype=np.int32)}
        lib().orc_get_last_brackets(self.ctx, _d(out["x0"]), _d(out["v"]), _d(out["a"]), _d(out["b"]),
                                    _i(out["ka"]), _i(out["kb"]))
        return out

    def last_batch(self, m):
        T, d = self.T, self.d
        out = {"seeds": np.zeros(m, dtype=np.int32), "tau": np.zeros(m), "new_u": np.zeros((m, d)),
               "new_logL": np.zeros(m), "chain_evals": np.zeros(m, dtype=np.int64),
               "hist_logL": np.zeros((T, m)), "hist_u": np.zeros((m, T, d)),
               "hist_n": np.zeros(m, dtype=np.int32)}
        lib().orc_get_last_batch(self.ctx, _i(out["seeds"]), _d(out["tau"]), _d(out["new_u"]),
                                 _d(out["new_logL"]), out["chain_evals"].ctypes.data_as(_lp),
                                 _d(out["hist_logL"]), _d(out["hist_u"]), _i(out["hist_n"]))
        return out


def slice_direction(seed, chain, step, it, L):
    """Direction v = L zhat of slice iteration `it` of a chain (Sec. 2.2); L is
    a lower-triangular d x d Cholesky factor."""
    L = _f64(L)
    d = L.shape[0]
    Lp = np.zeros((MAXD, MAXD))
    Lp[:d, :d] = L
    v = np.zeros(d)
    lib().orc_slice_direction(int(seed), int(chain), int(step), int(it), _d(Lp), d, _d(v))
    return v


def set_threads(n):
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------------- MLP
def mlp_forward(widths, Ws, bs, act, X):
    widths = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
    W = _f64(np.concatenate([np.asarray(w, dtype=np.float64).ravel() for w in Ws]))
    b = _f64(np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in bs]))
    X = _f64(X).reshape(-1, widths[0])
    B = X.shape[0]
    Y = np.zeros((B, widths[-1]))
    acts = np.zeros(B * int(widths[1:].sum()))
    lib().orc_mlp_forward(widths.size - 1, _i(widths), _d(W), _d(b), int(act), _d(X), B, _d(Y), _d(acts))
    return Y, acts


def mlp_backward(widths, Ws, bs, act, X, acts, dY):
    widths = np.ascontiguousarray(np.asarray(widths, dtype=np.int32))
    W = _f64(np.concatenate([np.asarray(w, dtype=np.float64).ravel() for w in Ws]))
    b = _f64(np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in bs]))
    X = _f64(X).reshape(-1, widths[0])
    B = X.shape[0]
    dY = _f64(dY).reshape(B, widths[-1])
    acts = _f64(acts)
    dW = np.zeros(W.size); db = np.zeros(b.size); dX = np.zeros(X.shape)
    lib().orc_mlp_backward(widths.size - 1, _i(widths), _d(W), _d(b), int(act), _d(X), B, _d(acts),
                           _d(dY), _d(dW), _d(db), _d(dX))
    # split back per layer
    dWs, dbs, o, ob = [], [], 0, 0
    for l in range(widths.size - 1):
        n = int(widths[l]) * int(widths[l + 1])
        dWs.append(dW[o:o + n].reshape(int(widths[l]), int(widths[l + 1])))
        dbs.append(db[ob:ob + int(widths[l + 1])])
        o += n
        ob += int(widths[l + 1])
    return dWs, dbs, dX
