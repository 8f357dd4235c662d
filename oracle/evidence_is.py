"""Evidence integrals by importance sampling, FP64.  TEST INFRASTRUCTURE
(oracle): only tests, the smoke check, the benchmark's CPU-baseline leg and
the scripts that write stored reference values use it.

The evidence of Eq. (1) under a uniform prior on a box is, in unit-cube
coordinates u, Z = int_[0,1]^d L(theta(u)) du.  Nested sampling estimates it;
this module computes the same integral independently, for likelihoods whose
posterior is a single peak (the 27-d emulator of Sec. 5's stand-in):

    Z = E_q[ L(u) 1[u in box] / q(u) ],   u ~ q,

with q a multivariate Student-t centred on the posterior mode, with scale
matrix from the curvature there (Laplace's approximation, widened).  The
estimate is unbiased for any q that covers the posterior; its standard error
follows from the sample variance of the weights.  Likelihood values come from
the oracle's own FP64 likelihood (oracle.loglike).

For the emulator (tanh network, linear output, diagonal chi^2) the mode is
found by Gauss-Newton on the scaled residuals r = (y(u) - D)/sigma, with the
network Jacobian from the chain rule, and the curvature is the Hessian of
-log L by central differences of its analytic gradient J_r^T r.
"""
import math

import numpy as np
from scipy.special import gammaln

from . import loglike


# ---------------------------------------------------------------- the emulator network (FP64)
def _forward_jac(spec, u):
    """y(theta) and dy/du of the emulator network at one unit-cube point u."""
    lo, hi = np.asarray(spec["lo"], float), np.asarray(spec["hi"], float)
    h = lo + (hi - lo) * np.asarray(u, float)
    J = np.diag(hi - lo)                               # d theta / d u
    Ws, bs = spec["weights"], spec["biases"]
    for l, (Wl, bl) in enumerate(zip(Ws, bs)):
        Wl = np.asarray(Wl, float)
        z = h @ Wl + np.asarray(bl, float)
        J = Wl.T @ J
        if l + 1 < len(Ws):
            h = np.tanh(z)
            J = (1.0 - h * h)[:, None] * J
        else:
            h = z
    return h, J


def emulator_residual(spec, u):
    """Scaled residuals r = (y(u) - D) / sigma and their Jacobian dr/du."""
    y, J = _forward_jac(spec, u)
    isig = 1.0 / np.asarray(spec["sigma"], float)
    return (y - np.asarray(spec["data"], float)) * isig, J * isig[:, None]


def emulator_mode(spec, u0, iters=100, tol=1e-15):
    """Posterior mode of the emulator likelihood (uniform prior, mode inside
    the box): Gauss-Newton on |r|^2 with step halving, from u0."""
    u = np.asarray(u0, float).copy()
    r, J = emulator_residual(spec, u)
    f = float(r @ r)
    for _ in range(iters):
        step = np.linalg.lstsq(J, -r, rcond=None)[0]
        t = 1.0
        while t > 1e-6:
            un = u + t * step
            rn, Jn = emulator_residual(spec, un)
            fn = float(rn @ rn)
            if fn <= f:
                break
            t *= 0.5
        if fn > f:
            break
        done = np.max(np.abs(un - u)) <= tol * max(1.0, np.max(np.abs(u)))
        u, r, J, f = un, rn, Jn, fn
        if done:
            break
    return u


def emulator_hessian(spec, u, rel_step=1e-4):
    """Hessian of -log L = |r|^2 / 2 at u: central differences of the analytic
    gradient J_r^T r, with per-coordinate steps of rel_step times the
    Gauss-Newton posterior width; symmetrised."""
    r, J = emulator_residual(spec, u)
    Hgn = J.T @ J
    width = np.sqrt(np.diag(np.linalg.inv(Hgn)))
    d = u.size
    H = np.empty((d, d))
    for k in range(d):
        e = np.zeros(d)
        e[k] = rel_step * width[k]
        rp, Jp = emulator_residual(spec, u + e)
        rm, Jm = emulator_residual(spec, u - e)
        H[:, k] = (Jp.T @ rp - Jm.T @ rm) / (2.0 * e[k])
    return 0.5 * (H + H.T), Hgn


# ---------------------------------------------------------------- importance sampling
def student_t_logpdf(x, mu, L, nu):
    """log density of the multivariate t with location mu, scale L L^T
    (L lower triangular) and nu degrees of freedom, at the rows of x."""
    d = mu.size
    z = np.linalg.solve(L, (x - mu).T).T if x.ndim == 2 else np.linalg.solve(L, x - mu)
    q = np.sum(z * z, axis=-1)
    return (gammaln(0.5 * (nu + d)) - gammaln(0.5 * nu) - 0.5 * d * math.log(nu * math.pi)
            - np.sum(np.log(np.diag(L))) - 0.5 * (nu + d) * np.log1p(q / nu))


def importance_logZ(spec, mode, cov, n, seed, nu=10.0, scale=1.2, chunk=20000):
    """log Z of spec over its unit-cube prior by importance sampling from a
    Student-t (nu degrees of freedom) at `mode` with scale matrix
    scale^2 * cov.  Returns a dict: logZ, its standard error, the information
    H = E_post[log L] - log Z, the effective sample size and the weights' log
    maximum share."""
    mode = np.asarray(mode, float)
    d = mode.size
    L = np.linalg.cholesky(np.asarray(cov, float)) * scale
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x15]))
    logw, logl = [], []
    left = int(n)
    while left > 0:
        k = min(chunk, left)
        z = rng.standard_normal((k, d))
        g = rng.chisquare(nu, size=k)
        x = mode + (z @ L.T) / np.sqrt(g / nu)[:, None]
        lq = student_t_logpdf(x, mode, L, nu)
        ll = loglike(spec, x)                    # -inf outside the box (zero prior mass)
        logw.append(ll - lq)
        logl.append(ll)
        left -= k
    logw = np.concatenate(logw)
    logl = np.concatenate(logl)
    mx = np.max(logw)
    w = np.exp(logw - mx)
    s1 = w.sum()
    logZ = mx + math.log(s1 / w.size)
    # relative standard error of the mean weight -> standard error of log Z
    rel = math.sqrt(np.var(w, ddof=1) / w.size) / (s1 / w.size)
    p = w / s1
    fin = np.isfinite(logl)
    H = float(np.sum(p[fin] * logl[fin])) - logZ
    return {"logZ": logZ, "se": rel, "H": H, "ess": float(1.0 / np.sum(p * p)), "n": int(w.size),
            "max_weight_share": float(p.max()), "nu": nu, "scale": scale}


def laplace_logZ(logL_mode, hessian):
    """Laplace's approximation: log L(mode) + (d/2) log 2 pi - (1/2) log det H."""
    d = hessian.shape[0]
    sign, logdet = np.linalg.slogdet(hessian)
    if sign <= 0:
        return float("nan")
    return float(logL_mode + 0.5 * d * math.log(2.0 * math.pi) - 0.5 * logdet)


def emulator_evidence(spec, n=100_000, seed=0, nu=10.0, scale=1.2):
    """Mode, curvature, Laplace estimate and importance-sampling evidence of
    the emulator likelihood `spec` (the data were drawn at spec["theta0"])."""
    lo, hi = np.asarray(spec["lo"], float), np.asarray(spec["hi"], float)
    u0 = (np.asarray(spec["theta0"], float) - lo) / (hi - lo)
    mode = emulator_mode(spec, u0)
    H, Hgn = emulator_hessian(spec, mode)
    cov = np.linalg.inv(H)
    cov = 0.5 * (cov + cov.T)
    lmode = float(loglike(spec, mode[None, :])[0])
    res = importance_logZ(spec, mode, cov, n, seed, nu=nu, scale=scale)
    res.update({"mode": mode, "cov": cov, "logL_mode": lmode, "laplace_logZ": laplace_logZ(lmode, H),
                "laplace_gn_logZ": laplace_logZ(lmode, Hgn),
                "posterior_sd": np.sqrt(np.diag(cov)),
                "mode_to_box_edge_in_sd": float(np.min(np.minimum(mode, 1.0 - mode) / np.sqrt(np.diag(cov))))})
    return res
