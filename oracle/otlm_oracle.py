"""FP64 reference ("oracle") for the OTLM scaling algorithm.  TEST INFRASTRUCTURE.

This module is the correctness reference for the GPU library and nothing else:
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  The GPU path never calls it and shares no code with it.

Everything here is plain NumPy in float64, written from the paper
(Kacprzak et al., "Scalable Approximate Algorithms for Optimal Transport Linear
Models"):

* the Gibbs kernel and the scaling loop of Algorithm 1 (section "Scaling
  Algorithm Framework for OTLM", Algorithm 1 "Scaling Algorithm for OTLM");
* the datafit proximal operators of Table 1, with the squared-error row derived
  in Appendix B;
* the single majorisation-minimisation weight step of Table 2 and Appendix A
  (section "MM for Penalized Column Span Projection with KL Divergence");
* the exact weight proximal step (ProxP in section "Scaling Algorithm Framework
  for OTLM"), which the paper allows in place of the single MM step (subsection
  "Iterative Algorithm for OTLM"); its minimiser is computed here by an
  active-set Newton method on the same objective V(w);
* the objective of the OTLM problem (eq. OTLM, in the scaling-algorithm form
  eps KL(Q|K) + F1(Q1) + F2(Q^T 1)), its Fenchel dual and KKT residuals.

Naming: the paper's X (dictionary, N x M) is ``D`` (n x k); the paper's u_1
(target-side scaling) is ``v`` and u_2 (source-side scaling) is ``u``; the plan
is Q = diag(u) K diag(v), i.e. Q_ij = u_i K_ij v_j with rows indexing source
bins.  Batched arrays are [B, n] with one spectrum per row.

Readings of the paper where it is silent or garbled (all listed in the design
notes):
* the l1 row of Table 2 is applied as exp(nu_j - alpha/(eps x_j)) (Appendix A's
  stationarity), which equals the table for unit-mass columns;
* the squared-l2 and elastic-net rows are taken from Appendix A
  (ln w_j + gamma_j w_j = nu_j, solved with Lambert W), not from the garbled
  table entries;
* the penalty is alpha R(w) with R = ||w||_1 (l1), R = ||w||^2 / 2 (squared l2),
  R = ||w||_1 + (beta/alpha) ||w||^2 / 2 (elastic net, i.e. alpha l1 + beta/2 l2^2);
* the sum datafit lam L2 + lam2 TV uses prox_L2 o prox_TV (not in the paper);
* the Poisson row's "W^{-1}_0" is read as the reciprocal 1/W_0 (Appendix B);
* terms with D_ij = 0 are dropped (0 log 0 = 0, section "Optimal Transport"),
  u_i = 0 where (Dw)_i = 0;
* the initial weights are mass matched, w0_j = sum(y) / (k x_j), v0 = 1;
* "while not converged" stops when both the relative weight change
  max|w - w_prev| / max|w| and the source-marginal violation
  sum|u * (K v) - D w| / sum(D w) fall to ``tol``.
"""
from __future__ import annotations

import numpy as np
from scipy.special import wrightomega as _scipy_wrightomega

FITS = ("balanced", "kl", "tv", "l2", "l2tv", "poisson")
PENS = ("none", "l1", "l2sq", "en")


# --------------------------------------------------------------------------
# special functions
# --------------------------------------------------------------------------
def omega(z):
    """Wright omega, omega(z) = W_0(exp(z)), real argument, FP64.

    Table 1 (L2 row), Table 2 and Appendix A use W_0(c e^z); writing it as
    omega(z + log c) avoids overflow of the exponential.  The library routine
    is SciPy's complex Wright omega evaluated on the real axis.
    """
    z = np.asarray(z, dtype=np.float64)
    return np.real(_scipy_wrightomega(z.astype(np.complex128)))


# --------------------------------------------------------------------------
# Gibbs kernel  (Algorithm 1, initialisation:  K = exp(-C / eps))
# --------------------------------------------------------------------------
def gibbs_kernel(C: np.ndarray, eps: float) -> np.ndarray:
    return np.exp(-np.asarray(C, dtype=np.float64) / eps)


# --------------------------------------------------------------------------
# Table 1: prox^KL_L(s | y) = argmin_p  L(p | y) + eps KL(p || s)
# --------------------------------------------------------------------------
def prox_datafit(t, y, fit: str, eps: float, lam: float, lam2: float = 0.0):
    """Target-side proximal operator, elementwise (Table 1).

    ``t`` is the argument K^T u (the paper's K^T u_2), ``y`` the target.
    """
    t = np.asarray(t, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    if fit == "balanced":                    # iota_{=}(s|y): prox = y
        return np.broadcast_to(y, t.shape).copy()
    if fit == "kl":                          # lam KL(s|y): s^{eps/(eps+lam)} y^{lam/(eps+lam)}
        return t ** (eps / (eps + lam)) * y ** (lam / (eps + lam))
    if fit == "tv":                          # lam TV(s|y): min(s e^{lam/eps}, max(s e^{-lam/eps}, y))
        return np.minimum(t * np.exp(lam / eps), np.maximum(t * np.exp(-lam / eps), y))
    if fit == "l2":                          # lam L2: (eps/lam) W0((lam/eps) s exp(lam y / eps))
        with np.errstate(divide="ignore"):
            z = np.log(lam / eps) + np.log(t) + lam * y / eps
        return (eps / lam) * omega(z)
    if fit == "l2tv":                        # lam L2 + lam2 TV: prox_L2 o prox_TV (reading)
        tau = prox_datafit(t, y, "tv", eps, lam2)
        return prox_datafit(tau, y, "l2", eps, lam)
    if fit == "poisson":                     # (lam/eps) y / W0((lam/eps)(y/s) e^{lam/eps})
        with np.errstate(divide="ignore"):
            z = np.log(lam / eps) + np.log(y) - np.log(t) + lam / eps
        p = (lam / eps) * y / omega(z)
        return np.where(y > 0, p, 0.0)
    raise ValueError(f"unknown datafit {fit!r}")


# --------------------------------------------------------------------------
# Table 2 / Appendix A: one MM step of the weight proximal problem
# --------------------------------------------------------------------------
def _log_ratio(S, A, D):
    """r_i = log(s_i / a_i) for bins covered by the dictionary, 0 elsewhere.

    Bins where (Dw)_i = 0 have D_ij w_j = 0 for all j; their Z_ij are zero and
    their terms drop (0 log 0 = 0).
    """
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.log(S / A)
    return np.where(A > 0, r, 0.0)


def mm_step(W, S, D, pen: str, eps: float, alpha: float, beta: float = 0.0):
    """w <- wMMstep(s, Z | D)  (Table 2, derivation in Appendix A).

    With Z_ij = D_ij w'_j / (D w')_i (Table 2 caption) and s = K v the kernel
    product (the argument named y in Table 2),

        (1/x_j) sum_i D_ij log(Z_ij s_i / D_ij) = log w'_j + (1/x_j) sum_i D_ij log(s_i / (D w')_i),

    so nu_j = log w'_j + g_j with g = D^T r / x, r = log(s / (D w')).  The
    stationarity condition of the majorised objective G(w, w') (Appendix A)
    is then

        log w_j + alpha R'(w_j) / (eps x_j) = nu_j .
    """
    W = np.asarray(W, dtype=np.float64)
    x = D.sum(axis=0)
    A = W @ D.T
    r = _log_ratio(S, A, D)
    with np.errstate(divide="ignore"):
        nu = np.log(W) + (r @ D) / x
    if pen == "none":
        return np.exp(nu)
    if pen == "l1":
        return np.exp(nu - alpha / (eps * x))
    if pen == "l2sq":
        gam = alpha / (eps * x)
        return omega(nu + np.log(gam)) / gam
    if pen == "en":
        gam = beta / (eps * x)
        return omega(nu - alpha / (eps * x) + np.log(gam)) / gam
    raise ValueError(f"unknown penalty {pen!r}")


def penalty_value(W, pen: str, alpha: float, beta: float = 0.0):
    """alpha R(w) per spectrum."""
    W = np.atleast_2d(W)
    if pen == "none":
        return np.zeros(W.shape[0])
    if pen == "l1":
        return alpha * W.sum(axis=1)
    if pen == "l2sq":
        return 0.5 * alpha * (W * W).sum(axis=1)
    if pen == "en":
        return alpha * W.sum(axis=1) + 0.5 * beta * (W * W).sum(axis=1)
    raise ValueError(pen)


def penalty_grad(W, pen: str, alpha: float, beta: float = 0.0):
    """alpha R'(w), elementwise (Appendix A: [0, alpha, alpha w, alpha + beta w])."""
    if pen == "none":
        return np.zeros_like(W)
    if pen == "l1":
        return np.full_like(W, alpha)
    if pen == "l2sq":
        return alpha * W
    if pen == "en":
        return alpha + beta * W
    raise ValueError(pen)


def _kl_vec(a, s):
    """sum_i a_i log(a_i/s_i) - a_i + s_i with 0 log 0 = 0 (generalised KL)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(a > 0, a * np.log(a / s), 0.0)
    return np.sum(t - a + s, axis=-1)


def prox_objective(w, s, D, pen, eps, alpha, beta=0.0):
    """V(w) = alpha R(w) + eps KL(Dw || s)  (objective of ProxP)."""
    return penalty_value(w[None], pen, alpha, beta)[0] + eps * _kl_vec(D @ w, s)


def prox_P_exact(s, D, w0, pen: str, eps: float, alpha: float, beta: float = 0.0,
                 max_newton: int = 500, gtol: float = 1e-13):
    """Exact weight prox: argmin_{w >= 0} alpha R(w) + eps KL(Dw || s)  (ProxP).

    Active-set Newton method on the smooth convex objective V(w), gradient
    alpha R'(w) + eps D^T log(Dw / s), Hessian alpha R'' + eps D^T diag(1/Dw) D:
    Newton steps on the free weights with a ratio test that stops at the first
    weight reaching 0 (which then joins the active set) and Armijo backtracking;
    the active weight with the most negative gradient is released once the free
    gradient is small next to it (or no descent is left on the free set).  Ends
    when the free gradient is below ``gtol`` (scaled) and no active weight has a
    negative gradient.  One spectrum at a time.
    """
    w = np.maximum(np.array(w0, dtype=np.float64), 0.0)
    cover = D.sum(axis=1) > 0                # bins in the support of the dictionary
    Dc, sc = D[cover], s[cover]
    hess_pen = {"none": 0.0, "l1": 0.0, "l2sq": alpha, "en": beta}[pen]
    tiny = 1e-300
    gscale = max(alpha, eps, 1e-300)

    def V(ww):
        return prox_objective(ww, sc, Dc, pen, eps, alpha, beta)

    act = w <= 0.0
    f = V(w)
    for _ in range(max_newton):
        a = np.maximum(Dc @ w, tiny)
        g = penalty_grad(w, pen, alpha, beta) + eps * (Dc.T @ np.log(a / sc))
        free = ~act
        kkt = np.max(np.abs(g[free])) if free.any() else 0.0
        cand = np.flatnonzero(act & (g < -gtol * gscale))
        jmin = cand[np.argmin(g[cand])] if cand.size else -1
        if kkt <= gtol * gscale and jmin < 0:
            break                              # optimal
        released = -1
        if jmin >= 0 and kkt <= max(gtol * gscale, 0.1 * abs(g[jmin])):
            act[jmin] = False                  # free problem solved well enough: release
            free = ~act
            released, jmin = jmin, -1
        F = np.flatnonzero(free)
        Df = Dc[:, F]
        H = eps * (Df.T * (1.0 / a)) @ Df + hess_pen * np.eye(F.size)
        try:
            d = -np.linalg.solve(H, g[F])
        except np.linalg.LinAlgError:
            d = -np.linalg.lstsq(H, g[F], rcond=None)[0]
        d[(w[F] <= 0.0) & (d < 0.0)] = 0.0     # weights at 0 cannot decrease
        if released >= 0:
            r = int(np.flatnonzero(F == released)[0])
            if d[r] <= 0.0:                    # coupling swamped the released weight:
                d[:] = 0.0                     # take its own Newton coordinate step
                d[r] = -g[released] / H[r, r]
        neg = d < 0
        tmax = float(np.min(-w[F][neg] / d[neg])) if neg.any() else np.inf
        t = min(1.0, tmax)
        slope = float(g[F] @ d)
        accepted = False
        if slope < 0 and -slope <= 1e-14 * abs(f):
            # predicted decrease below the FP64 resolution of V: take the step untested
            wn = w.copy()
            wn[F] = np.maximum(w[F] + t * d, 0.0)
            accepted = True
        elif slope < 0:
            for _ in range(30):
                wn = w.copy()
                wn[F] = np.maximum(w[F] + t * d, 0.0)
                fn = V(wn)
                if fn <= f + 1e-4 * t * slope:
                    accepted = True
                    break
                t *= 0.5
        if not accepted:                       # no descent left on this free set
            if jmin >= 0:
                act[jmin] = False
                continue
            break
        if t == tmax:                          # the blocking weights join the active set
            blk = neg & (-w[F] / np.where(neg, d, -1.0) <= tmax * (1.0 + 1e-12))
            z = F[blk]
            act[z] = True
            wn[z] = 0.0
        w, f = wn, V(wn)
    return w


# --------------------------------------------------------------------------
# Algorithm 1: scaling algorithm for OTLM
# --------------------------------------------------------------------------
def initial_weights(Y, D):
    """Mass-matched start w0_j = sum(y) / (k x_j) (Algorithm 1 requires a start)."""
    x = D.sum(axis=0)
    return (np.asarray(Y).sum(axis=1, keepdims=True) / D.shape[1]) / x[None, :]


def solve(K, D, Y, *, fit="kl", pen="l1", eps=0.01, lam=1.0, alpha=0.0, lam2=0.0,
          beta=0.0, max_iter=1000, tol=0.0, mode="single", W0=None, V0=None,
          trace=None, mm_warmup=3):
    """Algorithm 1 on a batch of targets Y [B, n] sharing K and D.

    Per iteration (Algorithm 1, in order):
      s = K v;  w = wMMstep(s, Z | D) (mode "single") or ProxP(s) (mode "exact");
      u = D w / s;  t = K^T u;  p = prox_L(t | y);  v = p / t.
    Each spectrum stops on its own (and is frozen) once both the weight change
    and the source-marginal violation are <= tol; ``tol = 0`` runs max_iter.
    In mode "exact" the first ``mm_warmup`` iterations still take the single MM
    step: from a cold start s = K 1 carries far more mass than y, and an exact
    prox there drives weights to scales from which Newton recovers slowly.

    Returns a dict with W [B,k], logU [B,n], logV [B,n], iters [B] and
    converged [B].
    """
    K = np.asarray(K, dtype=np.float64)
    D = np.asarray(D, dtype=np.float64)
    Y = np.atleast_2d(np.asarray(Y, dtype=np.float64))
    B, n = Y.shape
    W = initial_weights(Y, D) if W0 is None else np.array(W0, dtype=np.float64, ndmin=2)
    V = np.ones((B, n)) if V0 is None else np.array(V0, dtype=np.float64, ndmin=2)
    KT = K.T
    A = W @ D.T
    U = np.zeros((B, n))
    iters = np.full(B, max_iter, dtype=np.int64)
    done = np.zeros(B, dtype=bool)
    for it in range(1, max_iter + 1):
        act = ~done
        if not act.any():
            break
        Va, Wa, Aa = V[act], W[act], A[act]
        S = Va @ KT                                   # s = K v
        with np.errstate(invalid="ignore", divide="ignore"):
            e_src = (np.abs(U[act] * S - Aa).sum(axis=1) / Aa.sum(axis=1)
                     if it > 1 else np.full(Va.shape[0], np.inf))
        if mode == "single" or (mode == "exact" and it <= mm_warmup):
            Wn = mm_step(Wa, S, D, pen, eps, alpha, beta)
        elif mode == "exact":
            Wn = np.stack([prox_P_exact(S[b], D, Wa[b], pen, eps, alpha, beta)
                           for b in range(S.shape[0])])
        else:
            raise ValueError(mode)
        An = Wn @ D.T                                 # D w
        with np.errstate(invalid="ignore", divide="ignore"):
            Un = np.where(An > 0, An / S, 0.0)        # u = D w / K v
        T = Un @ K                                    # t = K^T u
        P = prox_datafit(T, Y[act], fit, eps, lam, lam2)
        with np.errstate(invalid="ignore", divide="ignore"):
            Vn = np.where(T > 0, P / T, 1.0)          # v = prox / K^T u
        e_w = np.max(np.abs(Wn - Wa), axis=1) / np.max(np.abs(Wn), axis=1)
        W[act], A[act], U[act], V[act] = Wn, An, Un, Vn
        if trace is not None:
            trace.append((it, W.copy()))
        if tol > 0:
            newly = (e_w <= tol) & (e_src <= tol)
            idx = np.flatnonzero(act)[newly]
            done[idx] = True
            iters[idx] = it
    with np.errstate(divide="ignore"):
        logU, logV = np.log(U), np.log(V)
    return {"W": W, "logU": logU, "logV": logV, "iters": iters, "converged": done}


# --------------------------------------------------------------------------
# objective, dual and KKT residuals
# --------------------------------------------------------------------------
def _datafit_value(m, y, fit, lam, lam2):
    """lam L(m | y) per spectrum (eq. OTLM target term; Notation for L2 and TV)."""
    if fit == "kl":
        return lam * _kl_vec(m, y)
    if fit == "tv":
        return lam * np.abs(m - y).sum(axis=-1)
    if fit == "l2":
        return 0.5 * lam * ((m - y) ** 2).sum(axis=-1)
    if fit == "l2tv":
        return 0.5 * lam * ((m - y) ** 2).sum(axis=-1) + lam2 * np.abs(m - y).sum(axis=-1)
    if fit == "balanced":
        return np.where(np.abs(m - y).max(axis=-1) <= 1e-9 * np.abs(y).max(axis=-1), 0.0, np.inf)
    if fit == "poisson":
        with np.errstate(divide="ignore", invalid="ignore"):
            return -lam * (np.where(y > 0, y * np.log(m), 0.0) - m).sum(axis=-1)
    raise ValueError(fit)


def _datafit_conj_neg(g, y, fit, lam, lam2):
    """F2*(-g) summed per spectrum, F2 = lam L(.|y) on m >= 0."""
    z = -g
    if fit == "kl":
        return lam * (y * (np.exp(z / lam) - 1.0)).sum(axis=-1)
    if fit == "l2":
        m = y + z / lam
        val = np.where(m >= 0, z * y + z * z / (2 * lam), -0.5 * lam * y * y)
        return val.sum(axis=-1)
    if fit == "tv":
        val = np.where(z <= lam, np.maximum(z * y, -lam * y), np.inf)
        return val.sum(axis=-1)
    if fit == "l2tv":
        # sup_{m>=0} z m - lam/2 (m-y)^2 - lam2 |m-y|
        m = np.where(z > lam2, y + (z - lam2) / lam, np.where(z < -lam2, y + (z + lam2) / lam, y))
        m = np.maximum(m, 0.0)
        val = z * m - 0.5 * lam * (m - y) ** 2 - lam2 * np.abs(m - y)
        return val.sum(axis=-1)
    return np.full(z.shape[:-1], np.nan)


def _pen_conj_neg(Df, pen, alpha, beta):
    """F1*(-f) where F1 = alpha P_R(.|D); argument Dt = D^T f (per spectrum)."""
    if pen == "l2sq":
        return (np.maximum(0.0, -Df) ** 2).sum(axis=-1) / (2 * alpha)
    if pen == "en":
        return (np.maximum(0.0, -Df - alpha) ** 2).sum(axis=-1) / (2 * beta)
    if pen in ("l1", "none"):
        # F1* is the indicator of D^T f >= -alpha (l1) or >= 0 (none); its finite
        # part is 0 and the constraint is reported by the weight KKT residual.
        return np.zeros(Df.shape[:-1])
    raise ValueError(pen)


def objective(K, C, D, Y, W, logU, logV, *, fit="kl", pen="l1", eps=0.01, lam=1.0,
              alpha=0.0, lam2=0.0, beta=0.0):
    """Per-spectrum [primal, dual, <C,Q>, src_err, tgt_kkt, w_kkt], FP64.

    primal  J = eps KL(Q||K) + lam L(Q^T 1 | y) + alpha R(w), Q = diag(u) K diag(v)
              = eps(<a, log u> + <m, log v> - sum a + sum K) + ...   (a = Q1, m = Q^T 1)
    dual    = -F1*(-f) - F2*(-g) - eps sum_ij K_ij (exp((f_i + g_j)/eps) - 1),
              f = eps log u, g = eps log v (Fenchel dual of the scaling form);
              for l1 / no penalty F1* is an indicator: its finite part (0) is
              used and feasibility D^T f >= -alpha shows in w_kkt
    <C,Q>   = u^T (C o K) v
    src_err = ||Q1 - Dw||_1 / ||Dw||_1
    tgt_kkt = max_j dist(-g_j, d F2(m_j)) / lam
    w_kkt   = max_j |min(w_j, alpha R'(w_j) + eps (D^T log u)_j)|
    """
    K = np.asarray(K, dtype=np.float64)
    Y = np.atleast_2d(Y)
    W, logU, logV = np.atleast_2d(W), np.atleast_2d(logU), np.atleast_2d(logV)
    U, V = np.exp(logU), np.exp(logV)
    S = V @ K.T                       # K v
    T = U @ K                         # K^T u
    a, m = U * S, V * T
    sumK = K.sum()
    with np.errstate(invalid="ignore"):
        la = np.where(a > 0, a * logU, 0.0).sum(axis=1)
        lm = np.where(m > 0, m * logV, 0.0).sum(axis=1)
    klq = la + lm - a.sum(axis=1) + sumK
    J = eps * klq + _datafit_value(m, Y, fit, lam, lam2) + penalty_value(W, pen, alpha, beta)
    f, g = eps * logU, eps * logV
    with np.errstate(invalid="ignore"):
        Df = np.where(np.isfinite(f), f, 0.0) @ D        # D^T f (D_ij = 0 where u_i = 0)
    dual = (-_pen_conj_neg(Df, pen, alpha, beta) - _datafit_conj_neg(g, Y, fit, lam, lam2)
            - eps * ((U * S).sum(axis=1) - sumK))
    CQ = ((U @ (C * K)) * V).sum(axis=1)
    Dw = W @ D.T
    src = np.abs(a - Dw).sum(axis=1) / Dw.sum(axis=1)
    # target stationarity: -g in d F2(m)
    if fit == "kl":
        with np.errstate(divide="ignore", invalid="ignore"):
            res = np.abs(-g - lam * np.log(m / Y))
    elif fit == "l2":
        res = np.abs(-g - lam * (m - Y))
    elif fit in ("tv", "l2tv"):
        lt = lam if fit == "tv" else lam2
        base = 0.0 if fit == "tv" else lam * (m - Y)
        zz = -g - base
        on = np.abs(m - Y) <= 1e-12 * np.maximum(np.abs(Y), 1e-300)
        res = np.where(on, np.maximum(np.abs(zz) - lt, 0.0), np.abs(zz - lt * np.sign(m - Y)))
    else:
        res = np.zeros_like(m)
    tgt = np.max(res, axis=1) / max(lam, 1e-300)
    grad = penalty_grad(W, pen, alpha, beta) + Df      # alpha R'(w) + eps D^T log u
    wk = np.max(np.abs(np.minimum(W, grad)), axis=1)
    return np.stack([J, dual, CQ, src, tgt, wk], axis=1)
