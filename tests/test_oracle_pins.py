"""Pins for the FP64 oracle: checks against facts fixed by the paper and by
mathematics, not against the oracle's own formulas.

* prox operators (Table 1): scalar bisection of each 1-D convex problem's
  (sub)gradient condition;
* Wright omega: its defining identity, known values and SciPy's Lambert W;
* the MM step (Table 2 / Appendix A): majorisation G(w,w') >= V(w) with equality
  at w = w', monotone decrease of V, and the stationarity of G written in the
  paper's Z notation;
* Algorithm 1's fixed point: KKT conditions and a zero duality gap; agreement of
  the single-step and exact-prox variants; independence of the start;
* brute force on tiny problems: a generic optimiser on the Fenchel dual;
* special cases: D = I (closed form after one iteration), the balanced k = 1 case
  against a textbook Sinkhorn plan, lam = 0 (one ProxP at s = K 1);
* the eps -> 0 limit against an LP.
"""
import numpy as np
import pytest
from scipy.optimize import brentq, linprog, minimize
from scipy.special import lambertw

import oracle as orc
from paper_2504_04609_amd import synth


def _kl_scalar(p, s):
    return p * np.log(p / s) - p + s


# ---------------------------------------------------------------- omega
def test_omega_identity_and_known_values():
    z = np.concatenate([np.linspace(-60, 60, 2001), [100.0, 300.0, 700.0]])
    w = orc.omega(z)
    assert np.all(w > 0)
    np.testing.assert_allclose(w + np.log(w), z, rtol=1e-14, atol=1e-13)
    assert orc.omega(1.0) == pytest.approx(1.0, rel=1e-15)            # 1 + log 1 = 1
    assert orc.omega(0.0) == pytest.approx(0.5671432904097838, rel=1e-15)  # omega constant
    zz = np.linspace(-20, 20, 101)
    np.testing.assert_allclose(orc.omega(zz), np.real(lambertw(np.exp(zz))), rtol=1e-13)


# ---------------------------------------------------------------- Table 1
def _bisect_prox(h, t, y):
    """Root of a strictly increasing h(p) over p in (0, inf) via log-space bisection."""
    lo, hi = -200.0, 200.0
    return np.exp(brentq(lambda q: h(np.exp(q)), lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500))


@pytest.mark.parametrize("fit", ["kl", "tv", "l2", "l2tv", "poisson", "balanced"])
def test_prox_table1_against_scalar_bisection(fit):
    rng = np.random.default_rng(11)
    for _ in range(40):
        eps = 10 ** rng.uniform(-3, 0)
        lam = 10 ** rng.uniform(-2, 1)
        lam2 = 10 ** rng.uniform(-3, -1)
        t = 10 ** rng.uniform(-3, 1)
        y = 10 ** rng.uniform(-3, 1)
        p = float(orc.prox_datafit(np.array([t]), np.array([y]), fit, eps, lam, lam2)[0])
        if fit == "balanced":
            assert p == y
            continue
        # derivative of F(p) + eps KL(p | t); subgradient sets for |p - y|
        if fit == "kl":
            dF = lambda q: lam * np.log(q / y)
        elif fit == "l2":
            dF = lambda q: lam * (q - y)
        elif fit == "poisson":
            dF = lambda q: -lam * (y / q - 1.0)
        elif fit == "tv":
            dF = lambda q: lam * np.sign(q - y)
        else:
            dF = lambda q: lam * (q - y) + lam2 * np.sign(q - y)
        h = lambda q: dF(q) + eps * np.log(q / t)
        if fit in ("tv", "l2tv"):
            lo = -lam2 if fit == "l2tv" else -lam
            hi = -lo
            g_at_y = eps * np.log(y / t)
            if lo + g_at_y <= 0 <= hi + g_at_y:      # 0 in subdifferential at p = y
                assert p == pytest.approx(y, rel=1e-13)
                continue
        ref = _bisect_prox(h, t, y)
        assert p == pytest.approx(ref, rel=1e-11), (fit, eps, lam, t, y)


# ---------------------------------------------------------------- Table 2 / App. A
def _G_paper(w, wp, s, X, pen, eps, alpha, beta=0.0):
    """Majorised objective G(w, w') written in Z notation (MM subsection)."""
    Z = X * wp[None, :] / (X @ wp)[:, None]
    m = X > 0
    val = 0.0
    for i in range(X.shape[0]):
        for j in range(X.shape[1]):
            if not m[i, j]:
                continue
            q = X[i, j] * w[j] / Z[i, j]
            val += Z[i, j] * (q * np.log(q / s[i]) - q + s[i])
    # the paper's G carries the y_i (here s_i) term once per (i, j) pair weighted by Z,
    # and sum_j Z_ij = 1, so the constant reduces to sum_i s_i as in V.
    return eps * val + float(orc.penalty_value(w[None], pen, alpha, beta)[0])


def _V(w, s, X, pen, eps, alpha, beta=0.0):
    a = X @ w
    return eps * np.sum(a * np.log(a / s) - a + s) + float(orc.penalty_value(w[None], pen, alpha, beta)[0])


@pytest.mark.parametrize("pen", ["none", "l1", "l2sq", "en"])
def test_mm_step_majorises_and_decreases(pen):
    rng = np.random.default_rng(5)
    for _ in range(10):
        n, k = 9, 4
        X = rng.uniform(0.0, 1.0, (n, k)) * (rng.uniform(size=(n, k)) > 0.2)
        X[X.sum(1) == 0, 0] = 0.3                 # every bin covered by some column
        X[:, X.sum(0) == 0] = 0.5
        s = rng.uniform(0.2, 2.0, n)
        wp = rng.uniform(0.1, 2.0, k)
        eps, alpha, beta = 0.05, 0.01, 0.02
        wn = orc.mm_step(wp[None], s[None], X, pen, eps, alpha, beta)[0]
        assert np.all(wn > 0)
        # G(w', w') = V(w') and G(w, w') >= V(w)
        assert _G_paper(wp, wp, s, X, pen, eps, alpha, beta) == pytest.approx(_V(wp, s, X, pen, eps, alpha, beta), rel=1e-12)
        for _ in range(5):
            w = rng.uniform(0.05, 3.0, k)
            assert _G_paper(w, wp, s, X, pen, eps, alpha, beta) >= _V(w, s, X, pen, eps, alpha, beta) - 1e-12
        # wn minimises G(., w'): gradient from Appendix A vanishes
        Z = X * wp[None, :] / (X @ wp)[:, None]
        m = X > 0
        for j in range(k):
            gj = eps * np.sum(X[m[:, j], j] * np.log(X[m[:, j], j] * wn[j] / (Z[m[:, j], j] * s[m[:, j]])))
            gj += float(orc.penalty_grad(wn[j:j + 1], pen, alpha, beta)[0])
            assert abs(gj) < 1e-11
        # one step decreases V
        assert _V(wn, s, X, pen, eps, alpha, beta) <= _V(wp, s, X, pen, eps, alpha, beta) + 1e-14


@pytest.mark.parametrize("pen", ["none", "l1", "l2sq"])
def test_exact_prox_kkt(pen):
    """ProxP minimiser: natural residual min(w, grad V) = 0 (complementarity)."""
    rng = np.random.default_rng(7)
    dic = synth.make_dictionary(64, 8, 3)
    s = dic.D @ rng.exponential(1.0, 8) + 0.01
    w0 = np.full(8, 0.5)
    eps, alpha = 0.01, 0.002
    w = orc.prox_P_exact(s, dic.D, w0, pen, eps, alpha)
    cover = dic.D.sum(1) > 0
    a = dic.D[cover] @ w
    grad = orc.penalty_grad(w, pen, alpha) + eps * dic.D[cover].T @ np.log(a / s[cover])
    assert np.max(np.abs(np.minimum(w, grad))) < 1e-11


# ---------------------------------------------------------------- Algorithm 1
def _small_problem(n=48, k=5, seed=3, eps=0.01):
    dic = synth.make_dictionary(n, k, seed)
    y, *_ = synth.make_target(dic, seed, 0, 0.02, (0.9, 1.1))
    C = synth.sq_cost(dic.x, dic.x)
    return dic, y, C, orc.gibbs_kernel(C, eps)


@pytest.mark.parametrize("fit,pen", [("kl", "l2sq"), ("l2", "l2sq"), ("tv", "l2sq"),
                                     ("kl", "en"), ("l2tv", "l2sq")])
def test_fixed_point_kkt_and_duality(fit, pen):
    eps, lam, alpha, lam2, beta = 0.01, 1.0, 1e-3, 0.1, 2e-3
    dic, y, C, K = _small_problem(eps=eps)
    kw = dict(fit=fit, pen=pen, eps=eps, lam=lam, alpha=alpha, lam2=lam2, beta=beta)
    out = orc.solve(K, dic.D, y[None], max_iter=20000, tol=1e-14, **kw)
    assert out["converged"][0] or out["iters"][0] == 20000
    obj = orc.objective(K, C, dic.D, y[None], out["W"], out["logU"], out["logV"], **kw)[0]
    J, dual, CQ, src, tgt, wk = obj
    assert src < 1e-10
    assert tgt < 1e-8
    assert wk < 1e-9
    assert abs(J - dual) <= 1e-9 * abs(J)
    assert CQ > 0


def test_single_and_exact_modes_share_fixed_point():
    eps = 0.01
    dic, y, C, K = _small_problem(eps=eps)
    kw = dict(fit="kl", pen="l2sq", eps=eps, lam=1.0, alpha=1e-3)
    a = orc.solve(K, dic.D, y[None], max_iter=20000, tol=1e-14, mode="single", **kw)
    b = orc.solve(K, dic.D, y[None], max_iter=2000, tol=1e-13, mode="exact", **kw)
    np.testing.assert_allclose(a["W"], b["W"], rtol=1e-9)


def test_fixed_point_independent_of_start():
    eps = 0.01
    dic, y, C, K = _small_problem(eps=eps)
    kw = dict(fit="kl", pen="l2sq", eps=eps, lam=1.0, alpha=1e-3)
    rng = np.random.default_rng(1)
    ws = []
    for _ in range(3):
        w0 = rng.uniform(0.1, 5.0, (1, dic.D.shape[1]))
        v0 = rng.uniform(0.5, 2.0, (1, dic.D.shape[0]))
        ws.append(orc.solve(K, dic.D, y[None], max_iter=20000, tol=1e-14, W0=w0, V0=v0, **kw)["W"])
    np.testing.assert_allclose(ws[0], ws[1], rtol=1e-10)
    np.testing.assert_allclose(ws[0], ws[2], rtol=1e-10)


def _dual_neg(z, K, D, y, eps, lam, alpha, n):
    f, g = z[:n], z[n:]
    Df = D.T @ f
    F1 = np.sum(np.maximum(0.0, -Df) ** 2) / (2 * alpha)
    F2 = lam * np.sum(y * (np.exp(-g / lam) - 1.0))
    E = np.exp((f[:, None] + g[None, :]) / eps) * K
    val = -F1 - F2 - eps * np.sum(E - K)
    gf = -(D @ (-np.maximum(0.0, -Df) / alpha)) - E.sum(1)
    gg = y * np.exp(-g / lam) - E.sum(0)
    return -val, -np.concatenate([gf, gg])


def test_brute_force_dual_tiny_ridge_kl():
    """Generic optimiser on the smooth Fenchel dual (ridge + KL), n = 8, k = 3.
    The cost is asymmetric so that a transposed kernel product cannot pass."""
    rng = np.random.default_rng(2)
    n, k, eps, lam, alpha = 8, 3, 0.05, 1.0, 0.05
    x = synth.grid(n)
    D = synth.gaussian_peaks(x, np.array([0.2, 0.5, 0.8]), np.array([0.1, 0.12, 0.15]))
    y = D @ np.array([1.0, 0.5, 2.0]) + rng.uniform(0.01, 0.1, n)
    C = synth.sq_cost(x, x) + 0.1 * x[:, None] * (1.0 - x[None, :])
    K = np.exp(-C / eps)
    res = minimize(_dual_neg, np.zeros(2 * n), args=(K, D, y, eps, lam, alpha, n), jac=True,
                   method="BFGS", options={"gtol": 1e-13, "maxiter": 20000})
    f = res.x[:n]
    w_bf = np.maximum(0.0, -(D.T @ f)) / alpha
    out = orc.solve(K, D, y[None], fit="kl", pen="l2sq", eps=eps, lam=lam, alpha=alpha,
                    max_iter=50000, tol=1e-14)
    np.testing.assert_allclose(out["W"][0], w_bf, rtol=1e-7)


def test_brute_force_dual_tiny_l1_kl():
    """l1 + KL: dual with the linear constraint D^T f >= -alpha (SLSQP); weights from
    the plan's source marginal a = u * K v = D w (D has full column rank)."""
    rng = np.random.default_rng(4)
    n, k, eps, lam, alpha = 7, 2, 0.05, 1.0, 0.02
    x = synth.grid(n)
    D = synth.gaussian_peaks(x, np.array([0.3, 0.7]), np.array([0.12, 0.1]))
    y = D @ np.array([1.0, 0.7]) + rng.uniform(0.01, 0.05, n)
    K = np.exp(-synth.sq_cost(x, x) / eps)

    def neg(z):
        f, g = z[:n], z[n:]
        F2 = lam * np.sum(y * (np.exp(-g / lam) - 1.0))
        E = np.exp((f[:, None] + g[None, :]) / eps) * K
        return F2 + eps * np.sum(E - K)

    def grad(z):
        f, g = z[:n], z[n:]
        E = np.exp((f[:, None] + g[None, :]) / eps) * K
        return np.concatenate([E.sum(1), -y * np.exp(-g / lam) + E.sum(0)])

    cons = {"type": "ineq", "fun": lambda z: D.T @ z[:n] + alpha,
            "jac": lambda z: np.hstack([D.T, np.zeros((k, n))])}
    res = minimize(neg, np.zeros(2 * n), jac=grad, constraints=[cons], method="SLSQP",
                   options={"ftol": 1e-16, "maxiter": 5000})
    f, g = res.x[:n], res.x[n:]
    a = (np.exp((f[:, None] + g[None, :]) / eps) * K).sum(1)
    w_bf = np.linalg.lstsq(D, a, rcond=None)[0]
    out = orc.solve(K, D, y[None], fit="kl", pen="l1", eps=eps, lam=lam, alpha=alpha,
                    max_iter=300, tol=1e-13, mode="exact")
    np.testing.assert_allclose(out["W"][0], w_bf, rtol=2e-6)


def test_identity_dictionary_closed_form():
    """D = I, no penalty: after one iteration u = 1 and v = (y / K^T 1)^{lam/(lam+eps)}."""
    n, eps, lam = 30, 0.02, 0.7
    x = synth.grid(n)
    K = np.exp(-synth.sq_cost(x, x) / eps)
    y = np.random.default_rng(0).uniform(0.1, 1.0, n)
    out = orc.solve(K, np.eye(n), y[None], fit="kl", pen="none", eps=eps, lam=lam, max_iter=1)
    np.testing.assert_allclose(out["logU"][0], 0.0, atol=1e-14)
    np.testing.assert_allclose(np.exp(out["logV"][0]), (y / K.sum(0)) ** (lam / (lam + eps)), rtol=1e-13)
    np.testing.assert_allclose(out["W"][0], K.sum(1), rtol=1e-13)


def test_balanced_single_column_matches_textbook_sinkhorn():
    """Balanced datafit, k = 1: w = sum(y)/x_1 and Q is the Sinkhorn plan between
    D[:,0] w and y (scaling-algorithm section, balanced case)."""
    n, eps = 40, 0.02
    x = synth.grid(n)
    D = synth.gaussian_peaks(x, np.array([0.45]), np.array([0.1]))
    y = synth.gaussian_peaks(x, np.array([0.55]), np.array([0.08]))[:, 0] * 2.5
    K = np.exp(-synth.sq_cost(x, x) / eps)
    out = orc.solve(K, D, y[None], fit="balanced", pen="none", eps=eps, max_iter=20000, tol=1e-14)
    w = out["W"][0, 0]
    assert w == pytest.approx(y.sum() / D[:, 0].sum(), rel=1e-11)
    a, b = D[:, 0] * w, y
    u, v = np.ones(n), np.ones(n)
    for _ in range(20000):                       # textbook Sinkhorn
        u = a / (K @ v)
        v = b / (K.T @ u)
    Q_ref = u[:, None] * K * v[None, :]
    Q = np.exp(out["logU"][0])[:, None] * K * np.exp(out["logV"][0])[None, :]
    np.testing.assert_allclose(Q, Q_ref, rtol=1e-8, atol=1e-14 * Q_ref.max())


def test_lambda_zero_reduces_to_one_prox():
    """lam = 0 (KL datafit): v stays 1, so the loop is MM on ProxP at s = K 1."""
    eps = 0.02
    dic, y, C, K = _small_problem(n=40, k=4, eps=eps)
    out = orc.solve(K, dic.D, y[None], fit="kl", pen="l2sq", eps=eps, lam=0.0, alpha=1e-3,
                    max_iter=50000, tol=1e-14)
    np.testing.assert_allclose(out["logV"][0], 0.0, atol=1e-15)
    cov = dic.D.sum(1) > 0
    s = K.sum(1)[cov]
    a = dic.D[cov] @ out["W"][0]
    grad = 1e-3 * out["W"][0] + eps * dic.D[cov].T @ np.log(a / s)
    assert np.max(np.abs(grad)) < 1e-10


def test_eps_to_zero_approaches_lp():
    """OT-TV + l1 with linear cost (scaling-test problem ii): the entropic weights
    approach the LP weights as eps decreases."""
    n, k, lam, alpha = 12, 3, 1.0, 0.01
    x = synth.grid(n)
    D = synth.gaussian_peaks(x, np.array([0.25, 0.5, 0.75]), np.array([0.08, 0.08, 0.08]))
    y = synth.gaussian_peaks(x, np.array([0.3, 0.5, 0.7]), np.array([0.09, 0.07, 0.08])) @ np.array([1.0, 0.6, 1.4])
    C = 0.5 * np.abs(x[:, None] - x[None, :])
    # LP: variables Q (n*n), w (k), r+ (n), r- (n):  min <C,Q> + lam sum(r+ + r-) + alpha sum w
    nq = n * n
    c = np.concatenate([C.ravel(), alpha * np.ones(k), lam * np.ones(2 * n)])
    Aeq = np.zeros((2 * n, nq + k + 2 * n))
    beq = np.zeros(2 * n)
    for i in range(n):
        Aeq[i, i * n:(i + 1) * n] = 1.0           # Q1 - Dw = 0
        Aeq[i, nq:nq + k] = -D[i]
    for j in range(n):
        Aeq[n + j, j:nq:n] = 1.0                   # Q^T 1 - r+ + r- = y
        Aeq[n + j, nq + k + j] = -1.0
        Aeq[n + j, nq + k + n + j] = 1.0
        beq[n + j] = y[j]
    lp = linprog(c, A_eq=Aeq, b_eq=beq, bounds=(0, None), method="highs")
    w_lp = lp.x[nq:nq + k]
    errs = []
    for eps in (0.1, 0.03, 0.01):
        K = np.exp(-C / eps)
        out = orc.solve(K, D, y[None], fit="tv", pen="l1", eps=eps, lam=lam, alpha=alpha,
                        max_iter=3000, tol=1e-12, mode="exact")
        errs.append(np.sqrt(np.mean((out["W"][0] - w_lp) ** 2)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 0.05 * np.linalg.norm(w_lp)


def test_config1_converges_with_kkt():
    """Single-target workload (n = 200, k = 10, eps = 0.01, KL, ridge 1e-3)."""
    wl = synth.CONFIG1
    dic = wl.dictionary()
    Y = wl.targets(dic=dic)
    C = wl.cost()
    K = orc.gibbs_kernel(C, wl.eps)
    kw = dict(fit=wl.fit, pen=wl.pen, eps=wl.eps, lam=wl.lam, alpha=wl.alpha)
    out = orc.solve(K, dic.D, Y, max_iter=2000, tol=1e-12, **kw)
    assert out["converged"][0]
    obj = orc.objective(K, C, dic.D, Y, out["W"], out["logU"], out["logV"], **kw)[0]
    assert obj[3] < 1e-11 and obj[4] < 1e-9 and obj[5] < 1e-9
    assert abs(obj[0] - obj[1]) < 1e-6 * abs(obj[0])
