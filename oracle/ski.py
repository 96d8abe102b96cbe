"""m-space algebra of the oracle (test infrastructure only), FP64 NumPy/SciPy.

Each function states the passage of the paper it follows.  Dense n-space
routines exist only as references for small problems.
"""
import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla

from . import native

__all__ = [
    "make_grid", "grid_size", "toeplitz_column", "toeplitz_column_dlog_ell",
    "kg_dense", "kg_matvec", "dkg_matvec", "dense_w", "wtw_dense_from_dia",
    "B_apply", "solve_mean", "solve_grid_rhs", "fcg_probe", "lanczos_from_cg",
    "logm_e1", "mll_and_grad", "ski_dense_mean", "exact_gp_mean",
    "ski_dense_mll", "ski_dense_grad", "gsgp_mll_fact2", "lanczos_dense",
    "se_kernel", "kernel_1d", "kernel_1d_dlog_ell", "ski_dense_cov", "efla", "love_cov",
    "logm_e1_grad", "slq_logdet_grad_dense", "slq_logdet_grad",
]


# ---------------------------------------------------------------------------
# Grid and kernel (Sec. 2.3: K_G is the kernel on an equispaced grid, which is
# multilevel Toeplitz for a product stationary kernel; Sec. 5 uses a squared
# exponential inside a scale kernel; the Matern kernels are the other
# product stationary kernels offered).
# ---------------------------------------------------------------------------
def make_grid(m, lo=None, hi=None, origin=None, spacing=None):
    """Grid of prod(m) nodes.  Either explicit origin/spacing, or the padding
    rule h = (hi - lo)/(m - 3), origin = lo - h (one node of padding on each
    side so every point of [lo, hi] has a full cubic stencil)."""
    m = [int(v) for v in m]
    d = len(m)
    if origin is None:
        lo = np.broadcast_to(np.asarray(lo, float), (d,))
        hi = np.broadcast_to(np.asarray(hi, float), (d,))
        spacing = [(hi[k] - lo[k]) / (m[k] - 3) for k in range(d)]
        origin = [lo[k] - spacing[k] for k in range(d)]
    return {"d": d, "m": m, "origin": [float(v) for v in origin],
            "spacing": [float(v) for v in spacing]}


def grid_size(grid):
    return int(np.prod(grid["m"]))


def se_kernel(xa, xb, ell, s):
    """k(x, x') = s * exp(-1/2 sum_d (x_d - x'_d)^2 / l_d^2); xa [na, d]."""
    xa = np.atleast_2d(xa)
    xb = np.atleast_2d(xb)
    ell = np.asarray(ell, float)
    d2 = (((xa[:, None, :] - xb[None, :, :]) / ell) ** 2).sum(-1)
    return s * np.exp(-0.5 * d2)


def kernel_1d(r, kind="se"):
    """One-dimensional stationary kernel at scaled distance r = |x - x'| / l
    (K_G is multilevel Toeplitz for a product of such kernels, Sec. 2.3):
    squared exponential exp(-r^2/2) (Sec. 5), or the Matern kernels of
    smoothness 1/2, 3/2, 5/2 in their closed forms."""
    r = np.abs(np.asarray(r, np.float64))
    if kind == "se":
        return np.exp(-0.5 * r * r)
    if kind == "matern12":
        return np.exp(-r)
    if kind == "matern32":
        a = np.sqrt(3.0) * r
        return (1.0 + a) * np.exp(-a)
    if kind == "matern52":
        a = np.sqrt(5.0) * r
        return (1.0 + a + a * a / 3.0) * np.exp(-a)
    raise ValueError(kind)


def kernel_1d_dlog_ell(r, kind="se"):
    """d/d(log l) of kernel_1d(|x - x'| / l): since dr/dlog l = -r, it is
    -r k'(r): r^2 exp(-r^2/2); r exp(-r); 3 r^2 exp(-sqrt3 r);
    (5/3) r^2 (1 + sqrt5 r) exp(-sqrt5 r)."""
    r = np.abs(np.asarray(r, np.float64))
    if kind == "se":
        return r * r * np.exp(-0.5 * r * r)
    if kind == "matern12":
        return r * np.exp(-r)
    if kind == "matern32":
        return 3.0 * r * r * np.exp(-np.sqrt(3.0) * r)
    if kind == "matern52":
        a = np.sqrt(5.0) * r
        return (5.0 / 3.0) * r * r * (1.0 + a) * np.exp(-a)
    raise ValueError(kind)


def toeplitz_column(m, h, ell, kind="se"):
    """First column of the per-dimension Toeplitz factor: k1(j h / l)."""
    j = np.arange(m, dtype=np.float64)
    return kernel_1d(j * h / ell, kind)


def toeplitz_column_dlog_ell(m, h, ell, kind="se"):
    """d/d(log l) of the column."""
    j = np.arange(m, dtype=np.float64)
    return kernel_1d_dlog_ell(j * h / ell, kind)


def _hyp(hypers, d):
    ell = np.broadcast_to(np.asarray(hypers["lengthscale"], float), (d,))
    return ell, float(hypers["outputscale"]), float(hypers["noise"])


def _kind(hypers):
    return hypers.get("kernel", "se")


def kg_dense(grid, hypers):
    """Dense K_G = s * T_0 (x) ... (x) T_{d-1} (C-order flattening)."""
    d = grid["d"]
    ell, s, _ = _hyp(hypers, d)
    K = np.ones((1, 1))
    for k in range(d):
        T = sla.toeplitz(toeplitz_column(grid["m"][k], grid["spacing"][k], ell[k],
                                         _kind(hypers)))
        K = np.kron(K, T)
    return s * K


def _toeplitz_apply_axis(V, col, axis, workers=1):
    """Symmetric Toeplitz (first column col) applied along `axis` of V through a
    circulant embedding of length 2m (exact up to rounding)."""
    m = col.shape[0]
    L = 2 * m
    emb = np.zeros(L)
    emb[:m] = col
    emb[L - m + 1:] = col[1:][::-1]
    lam = sfft.rfft(emb)
    F = sfft.rfft(V, n=L, axis=axis, workers=workers)
    shape = [1] * V.ndim
    shape[axis] = lam.shape[0]
    out = sfft.irfft(F * lam.reshape(shape), n=L, axis=axis, workers=workers)
    return np.take(out, np.arange(m), axis=axis)


def _kron_apply(grid, cols, v, scale, workers=1):
    d = grid["d"]
    V = np.asarray(v, np.float64)
    lead = V.shape[:-1]
    V = V.reshape(lead + tuple(grid["m"]))
    base = len(lead)
    for k in range(d):
        V = _toeplitz_apply_axis(V, cols[k], base + k, workers)
    return scale * V.reshape(lead + (-1,))


def kg_matvec(grid, hypers, v, workers=1):
    """K_G v (v: [..., M]) via per-dimension circulant embeddings (`workers`:
    threads of the FFTs)."""
    d = grid["d"]
    ell, s, _ = _hyp(hypers, d)
    cols = [toeplitz_column(grid["m"][k], grid["spacing"][k], ell[k], _kind(hypers))
            for k in range(d)]
    return _kron_apply(grid, cols, v, s, workers)


def dkg_matvec(grid, hypers, v, which):
    """(dK_G/d theta) v for theta = log l_which (0 <= which < d) or log s
    (which == d; dK_G/dlog s = K_G)."""
    d = grid["d"]
    ell, s, _ = _hyp(hypers, d)
    cols = []
    for k in range(d):
        if k == which:
            cols.append(toeplitz_column_dlog_ell(grid["m"][k], grid["spacing"][k], ell[k],
                                                 _kind(hypers)))
        else:
            cols.append(toeplitz_column(grid["m"][k], grid["spacing"][k], ell[k],
                                        _kind(hypers)))
    return _kron_apply(grid, cols, v, s)


# ---------------------------------------------------------------------------
# Interpolation matrix and W^T W (Sec. 2.3; Claim 2).
# ---------------------------------------------------------------------------
def dense_w(grid, x):
    """Explicit dense W (n x M) from the per-point stencils (small n, M only)."""
    nodes, w, _ = native.stencils(grid, x)
    n = nodes.shape[0]
    W = np.zeros((n, grid_size(grid)))
    for i in range(n):
        for a in range(nodes.shape[1]):
            W[i, nodes[i, a]] += w[i, a]
    return W


def wtw_dense_from_dia(grid, wtw):
    """Dense M x M matrix from the [M, 7^d] stencil-diagonal layout."""
    d = grid["d"]
    m = grid["m"]
    M = grid_size(grid)
    A = np.zeros((M, M))
    offs = np.array(np.unravel_index(np.arange(7 ** d), (7,) * d)).T - 3
    for j in range(M):
        c = np.array(np.unravel_index(j, m))
        for oi, o in enumerate(offs):
            cc = c + o
            if np.all(cc >= 0) and np.all(cc < np.asarray(m)):
                A[j, np.ravel_multi_index(tuple(cc), m)] = wtw[j, oi]
    return A


# ---------------------------------------------------------------------------
# The GSGP operator B(x) = ((K_G W^T W + sigma^2 I) x, W^T W x)  (App. B,
# efficient factorized CG), with W^T W in stencil-diagonal form.
# ---------------------------------------------------------------------------
def B_apply(grid, hypers, wtw, x, threads=1):
    _, _, sig = _hyp(hypers, grid["d"])
    u = native.wtw_matvec(grid, wtw, x, threads)
    v = kg_matvec(grid, hypers, u, threads) + sig * sig * np.asarray(x, np.float64)
    return v, u


def solve_mean(grid, hypers, wtw, wty, yty, tol=1e-8, maxiter=10000, history=False):
    """Posterior mean on the grid through the simplified efficiently-factorized
    CG of the appendix (initial residual in the span of W), started at
    x_0 = y / sigma^2 so that r_0 = -W K_G W^T y / sigma^2.

    Loop index starts at 0; stop when ||r_k|| <= tol ||y||, where
    ||r_k||^2 = u_k^T r_k (r = W r_hat).  Returns (mu_G, W^T z~, info) with
    z~ = (W K_G W^T + sigma^2 I)^{-1} y and mu_G = K_G W^T z~ (Fact 2 mean
    weights; Claim 5 equates them with the SKI mean weights of Def. 2).
    """
    _, _, sig = _hyp(hypers, grid["d"])
    s2 = sig * sig
    r = -kg_matvec(grid, hypers, wty) / s2
    xd, it, hist, rho_hist = _efcg_core(grid, hypers, wtw, r, tol * tol * yty, maxiter, history)
    wtz = xd + wty / s2
    mu = kg_matvec(grid, hypers, wtz)
    info = {"iterations": it, "rho": rho_hist}
    if history:
        info["wtx_history"] = [h + wty / s2 for h in hist]
    return mu, wtz, info


def solve_grid_rhs(grid, hypers, wtw, yhat, tol=1e-10, maxiter=10000):
    """Second use of the simplified factorized CG: right-hand side b = W yhat,
    x_0 = 0, r_hat_0 = yhat; returns W^T (W K_G W^T + sigma^2 I)^{-1} W yhat."""
    yhat = np.asarray(yhat, np.float64)
    bnorm2 = float(yhat @ native.wtw_matvec(grid, wtw, yhat))
    xd, it, _, _ = _efcg_core(grid, hypers, wtw, yhat.copy(), tol * tol * bnorm2, maxiter, False)
    return xd, {"iterations": it}


def _efcg_core(grid, hypers, wtw, r, eps, maxiter, history):
    v, u = B_apply(grid, hypers, wtw, r)
    s = u.copy()
    z = v.copy()
    xd = np.zeros_like(r)
    rho = float(u @ r)
    hist = [xd.copy()] if history else []
    rhos = [rho]
    it = 0
    if rho <= eps:
        return xd, it, hist, rhos
    for k in range(maxiter):
        alpha = rho / float(s @ z)
        xd = xd + alpha * s
        r = r - alpha * z
        v, u = B_apply(grid, hypers, wtw, r)
        rho_new = float(u @ r)
        it = k + 1
        rhos.append(rho_new)
        if history:
            hist.append(xd.copy())
        if rho_new <= eps:
            break
        beta = rho_new / rho
        s = u + beta * s
        z = v + beta * z
        rho = rho_new
    return xd, it, hist, rhos


def fcg_probe(grid, hypers, wtw, bhat, bnorm2, tol=1e-8, maxiter=1000, history=False,
              residuals=0):
    """Factorized CG from x_0 = 0 for an n-space right-hand side b that is not
    in the span of W (Claims 3 and 4, efficient variant with one B per
    iteration).  Iterates: r = W r_hat + c_r b, p = W p_hat + c_p b,
    x = W x_hat + c_x b.  Needs only bhat = W^T b and ||b||^2.

    Returns (W^T x, info) with the CG coefficients alpha, beta (for the
    Lanczos tridiagonal) and, on request, the W^T x_k history and the first
    `residuals` residuals r_k = W r_hat_k + c_r,k b (k = 0, 1, ...) as
    (r_hat_k, c_r,k, ||r_k||^2)."""
    _, _, sig = _hyp(hypers, grid["d"])
    s2 = sig * sig
    kb = kg_matvec(grid, hypers, bhat)
    M = bhat.shape[0]
    rh = np.zeros(M); cr = 1.0
    ph = np.zeros(M); cp = 1.0
    ux = np.zeros(M); cx = 0.0          # u_x = W^T W x_hat
    ur = np.zeros(M); vr = np.zeros(M)  # B(r_hat)
    sp = np.zeros(M); zp = np.zeros(M)  # W^T W p_hat, (K_G W^T W + s2) p_hat
    rho = float(rh @ ur) + 2 * cr * float(rh @ bhat) + cr * cr * bnorm2
    eps = tol * tol * bnorm2
    alphas, betas, hist = [], [], []
    res = [(rh.copy(), cr, rho)] if residuals > 0 else []
    it = 0
    for k in range(maxiter):
        ap = zp + cp * kb               # compressed A p (Claim 3)
        apc = s2 * cp
        pap = float(sp @ ap) + apc * float(ph @ bhat) + cp * float(ap @ bhat) + cp * apc * bnorm2
        alpha = rho / pap
        ux = ux + alpha * sp
        cx = cx + alpha * cp
        rh = rh - alpha * ap
        cr = cr - alpha * apc
        vr, ur = B_apply(grid, hypers, wtw, rh)
        rho_new = float(rh @ ur) + 2 * cr * float(rh @ bhat) + cr * cr * bnorm2
        alphas.append(alpha)
        it = k + 1
        if history:
            hist.append(ux + cx * bhat)
        if len(res) < residuals:
            res.append((rh.copy(), cr, rho_new))
        if rho_new <= eps:
            break
        beta = rho_new / rho
        betas.append(beta)
        ph = rh + beta * ph
        cp = cr + beta * cp
        sp = ur + beta * sp
        zp = vr + beta * zp
        rho = rho_new
    info = {"iterations": it, "alpha": np.array(alphas), "beta": np.array(betas)}
    if history:
        info["wtx_history"] = hist
    if residuals:
        info["residuals"] = res
    return ux + cx * bhat, info


def lanczos_from_cg(alpha, beta, k=None):
    """Lanczos tridiagonal from CG coefficients (the mBCG relation):
    T_ii = 1/alpha_i + beta_{i-1}/alpha_{i-1}, T_{i,i+1} = sqrt(beta_i)/alpha_i."""
    n = len(alpha) if k is None else min(k, len(alpha))
    T = np.zeros((n, n))
    for i in range(n):
        T[i, i] = 1.0 / alpha[i] + (beta[i - 1] / alpha[i - 1] if i > 0 else 0.0)
        if i + 1 < n:
            T[i, i + 1] = T[i + 1, i] = np.sqrt(beta[i]) / alpha[i]
    return T


def logm_e1(T):
    """e_1^T log(T) e_1 from the eigendecomposition of the symmetric T
    (Gauss quadrature of log at the Ritz values)."""
    ev, V = np.linalg.eigh(T)
    return float(np.sum(V[0, :] ** 2 * np.log(ev)))


def logm_e1_grad(T):
    """Gradient of e_1^T log(T) e_1 with respect to the entries of the
    symmetric T = V diag(lam) V^T (the derivative of a matrix function):
    V (F o (v v^T)) V^T with v = V^T e_1, F_ll = 1/lam_l and
    F_lm = (log lam_l - log lam_m)/(lam_l - lam_m) (l != m).  Returns
    (d/d diag [k], d/d off-diagonal [k-1]): a change of an off-diagonal
    entry moves both T_{i,i+1} and T_{i+1,i}."""
    lam, V = np.linalg.eigh(T)
    k = lam.shape[0]
    L = np.log(lam)
    F = np.empty((k, k))
    for a in range(k):
        for b in range(k):
            gap = lam[a] - lam[b]
            F[a, b] = (L[a] - L[b]) / gap if abs(gap) > 1e-13 * abs(lam[a]) else 1.0 / lam[a]
    v = V[0, :]
    G = V @ (F * np.outer(v, v)) @ V.T
    return np.diag(G).copy(), 2.0 * np.diag(G, 1).copy()


def slq_logdet_grad_dense(A, dA, z, k):
    """Reverse-mode derivative of ||z||^2 e_1^T log(T_k) e_1, T_k the k-step
    Lanczos tridiagonal of the dense symmetric A from z / ||z|| (plain
    Lanczos, as the CG coefficients give it), with respect to the
    parameters whose matrices dA[t] = dA/dtheta_t are given.  Forward:
    u_i = A q_i, alpha_i = q_i^T u_i, r_i = u_i - alpha_i q_i - beta_{i-1}
    q_{i-1}, beta_i = ||r_i||, q_{i+1} = r_i / beta_i; the reverse sweep runs
    these statements backwards with adjoints (checkpointed q_i, u_i) and
    collects d/dtheta_t = sum_i ubar_i^T dA[t] q_i.
    Returns (value, gradient [len(dA)])."""
    zz = float(z @ z)
    Q = [z / np.sqrt(zz)]
    U, al, be = [], [], []
    for i in range(k):
        u = A @ Q[i]
        a = float(Q[i] @ u)
        r = u - a * Q[i] - (be[i - 1] * Q[i - 1] if i > 0 else 0.0)
        U.append(u)
        al.append(a)
        if i == k - 1:
            break
        b = float(np.linalg.norm(r))
        be.append(b)
        Q.append(r / b)
    T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    abar, bbar = logm_e1_grad(T)
    qbar = [np.zeros_like(z) for _ in range(k)]
    g = np.zeros(len(dA))
    for i in range(k - 1, -1, -1):
        rbar = np.zeros_like(z)
        if i < k - 1:
            rbar = qbar[i + 1] / be[i]
            bbar[i] -= float(qbar[i + 1] @ Q[i + 1]) / be[i]
            rbar = rbar + bbar[i] * Q[i + 1]
        ubar = rbar.copy()
        abar[i] -= float(rbar @ Q[i])
        qbar[i] = qbar[i] - al[i] * rbar
        if i > 0:
            bbar[i - 1] -= float(rbar @ Q[i - 1])
            qbar[i - 1] = qbar[i - 1] - be[i - 1] * rbar
        qbar[i] = qbar[i] + abar[i] * U[i]
        ubar = ubar + abar[i] * Q[i]
        for t in range(len(dA)):
            g[t] += float(ubar @ (dA[t] @ Q[i]))
        qbar[i] = qbar[i] + A @ ubar
    return zz * logm_e1(T), zz * g


def slq_logdet_grad(grid, hypers, wtw, bhat, n, k, tol=1e-10, maxiter=2000):
    """The same derivative for one probe z (||z||^2 = n, W^T z = bhat) in
    m-space, as the factorized method forms it: T from the first k CG
    coefficients of the factorized CG from x_0 = 0 (Claims 3 and 4), the
    Lanczos vectors from its residuals, q_{i+1} = (-1)^i r_i / ||r_i||, all
    n-vectors kept as pairs (a, c) for W a + c z.  Then
        A (a, c) = (K_G (W^T W a + c bhat) + s2 a, s2 c),
        <(a, c), (e, f)> = (W^T W a).e + c bhat.e + f bhat.a + c f n,
    and for theta = log l_d, log s (dA = W dK_G W^T):
        ubar^T dA q = (W^T ubar)^T dK_G (W^T q),  W^T (a, c) = W^T W a + c bhat,
    for log sigma (dA = 2 s2 I): 2 s2 <ubar, q>.
    Returns (value ||z||^2 e_1^T log T e_1, gradient [d + 2])."""
    d = grid["d"]
    _, _, sig = _hyp(hypers, d)
    s2 = sig * sig
    bhat = np.asarray(bhat, np.float64)
    _, info = fcg_probe(grid, hypers, wtw, bhat, float(n), tol=tol, maxiter=maxiter,
                        residuals=k)
    kk = min(k, len(info["alpha"]))
    T = lanczos_from_cg(info["alpha"], info["beta"], kk)
    kb = kg_matvec(grid, hypers, bhat)

    def wtw_of(a):
        return native.wtw_matvec(grid, wtw, a)

    def inner(a, ca, e, ce):
        return float(wtw_of(a) @ e + ca * (bhat @ e) + ce * (bhat @ a) + ca * ce * n)

    def apply_A(a, ca):
        return kg_matvec(grid, hypers, wtw_of(a) + ca * bhat) + s2 * a, s2 * ca

    def wt(a, ca):
        return wtw_of(a) + ca * bhat

    Qa, Qc = [], []
    for i in range(kk):
        rh, cr, rho = info["residuals"][i]
        sgn = 1.0 if i % 2 == 0 else -1.0
        Qa.append(sgn * rh / np.sqrt(rho))
        Qc.append(sgn * cr / np.sqrt(rho))
    Ua, Uc = zip(*[apply_A(Qa[i], Qc[i]) for i in range(kk)])
    al = np.diag(T).copy()
    be = np.diag(T, 1).copy()
    abar, bbar = logm_e1_grad(T)
    qa = [np.zeros_like(bhat) for _ in range(kk)]
    qc = [0.0] * kk
    g = np.zeros(d + 2)
    for i in range(kk - 1, -1, -1):
        ra, rc = np.zeros_like(bhat), 0.0
        if i < kk - 1:
            ra, rc = qa[i + 1] / be[i], qc[i + 1] / be[i]
            bbar[i] -= inner(qa[i + 1], qc[i + 1], Qa[i + 1], Qc[i + 1]) / be[i]
            ra, rc = ra + bbar[i] * Qa[i + 1], rc + bbar[i] * Qc[i + 1]
        ua, uc = ra.copy(), rc
        abar[i] -= inner(ra, rc, Qa[i], Qc[i])
        qa[i], qc[i] = qa[i] - al[i] * ra, qc[i] - al[i] * rc
        if i > 0:
            bbar[i - 1] -= inner(ra, rc, Qa[i - 1], Qc[i - 1])
            qa[i - 1], qc[i - 1] = qa[i - 1] - be[i - 1] * ra, qc[i - 1] - be[i - 1] * rc
        qa[i], qc[i] = qa[i] + abar[i] * Ua[i], qc[i] + abar[i] * Uc[i]
        ua, uc = ua + abar[i] * Qa[i], uc + abar[i] * Qc[i]
        wu, wq = wt(ua, uc), wt(Qa[i], Qc[i])
        for th in range(d + 1):
            g[th] += float(wu @ dkg_matvec(grid, hypers, wq, th))
        g[d + 1] += 2.0 * s2 * inner(ua, uc, Qa[i], Qc[i])
        Aa, Ac = apply_A(ua, uc)
        qa[i], qc[i] = qa[i] + Aa, qc[i] + Ac
    return n * logm_e1(T), n * g


def lanczos_dense(A, b, k):
    """Plain Lanczos with full reorthogonalisation on a dense SPD A, started at
    b/||b|| (Alg. 5 of the appendix with its index slips corrected: the new
    vector subtracts alpha_i q_i, and T is symmetric)."""
    n = A.shape[0]
    Q = np.zeros((n, k))
    q = b / np.linalg.norm(b)
    Q[:, 0] = q
    al = np.zeros(k)
    be = np.zeros(k)
    qprev = np.zeros(n)
    bprev = 0.0
    kk = k
    for i in range(k):
        w = A @ Q[:, i] - bprev * qprev
        al[i] = Q[:, i] @ w
        if i == k - 1:
            break
        w = w - al[i] * Q[:, i]
        w = w - Q[:, :i + 1] @ (Q[:, :i + 1].T @ w)
        bprev = np.linalg.norm(w)
        be[i] = bprev
        if bprev < 1e-14:
            kk = i + 1
            break
        qprev = Q[:, i]
        Q[:, i + 1] = w / bprev
    T = np.diag(al[:kk]) + np.diag(be[:kk - 1], 1) + np.diag(be[:kk - 1], -1)
    return T, Q[:, :kk]


# ---------------------------------------------------------------------------
# Marginal log-likelihood and gradient (Fact 2; the gradient trace term of
# Sec. 2.2; stochastic Lanczos quadrature as used in Sec. 5).
# ---------------------------------------------------------------------------
def mll_and_grad(grid, hypers, wtw, wty, yty, n, sketches, lanczos_steps=30,
                 tol=1e-10, maxiter=2000, exact_trace=False, x=None, slq_grad=False):
    """MLL = -1/2 [ logdet(A) + y^T A^{-1} y + n log 2 pi ],
    A = W K_G W^T + sigma^2 I.

    logdet(A) ~ (1/N) sum_j ||z_j||^2 e_1^T log(T_j) e_1 with T_j from the
    factorized CG on each probe z_j (||z_j||^2 = n for Rademacher probes).
    y^T A^{-1} y = (y^T y - (W^T y)^T mu_G)/sigma^2.

    Gradient w.r.t. (log l_0..log l_{d-1}, log s, log sigma):
      g = 1/2 [ x_y^T dA x_y - tr(A^{-1} dA) ],
    with tr(A^{-1} dA) ~ (1/N) sum_j x_j^T dA z_j (x_j = A^{-1} z_j), or, with
    exact_trace, the exact trace through S = W^T A^{-1} W (small M only), or,
    with slq_grad, the exact derivative of the log-determinant estimate
    itself (reverse mode through each probe's Lanczos steps,
    slq_logdet_grad), so that the gradient is that of the returned MLL.
    Returns (mll, grad, info)."""
    d = grid["d"]
    ell, s, sig = _hyp(hypers, d)
    s2 = sig * sig
    M = grid_size(grid)
    mu, wtz, info_y = solve_mean(grid, hypers, wtw, wty, yty, tol=tol, maxiter=maxiter)
    q = (yty - float(wty @ mu)) / s2
    N = sketches.shape[0]
    logdets = []
    wtx = []
    for j in range(N):
        bj = sketches[j]
        wx, inf = fcg_probe(grid, hypers, wtw, bj, float(n), tol=tol, maxiter=maxiter)
        T = lanczos_from_cg(inf["alpha"], inf["beta"], lanczos_steps)
        logdets.append(n * logm_e1(T))
        wtx.append(wx)
    logdet = float(np.mean(logdets)) if N else float("nan")
    mll = -0.5 * (logdet + q + n * np.log(2 * np.pi))

    # quadratic-term pieces: x_y = z~, W^T x_y = wtz
    grad = np.zeros(d + 2)
    # ||z~||^2 = (y^T y - 2 (W^T y)^T mu + mu^T W^T W mu) / sigma^4
    zz = (yty - 2 * float(wty @ mu) + float(mu @ native.wtw_matvec(grid, wtw, mu))) / (s2 * s2)
    if slq_grad:
        dld = np.mean([slq_logdet_grad(grid, hypers, wtw, sketches[j], n, lanczos_steps,
                                       tol=tol, maxiter=maxiter)[1] for j in range(N)], axis=0)
    for th in range(d + 1):
        quad = float(wtz @ dkg_matvec(grid, hypers, wtz, th))
        if slq_grad:
            tr = dld[th]
        elif exact_trace:
            tr = _exact_trace(grid, hypers, wtw, th, n)
        else:
            tr = float(np.mean([wtx[j] @ dkg_matvec(grid, hypers, sketches[j], th)
                                for j in range(N)]))
        grad[th] = 0.5 * (quad - tr)
    # sigma: dA/dlog sigma = 2 sigma^2 I
    quad = 2 * s2 * zz
    if slq_grad:
        tr = dld[d + 1]
    elif exact_trace:
        tr = 2 * s2 * _exact_trace(grid, hypers, wtw, "inv", n)
    else:
        # z^T A^{-1} z = (n - (W^T z)^T K_G (W^T A^{-1} z)) / sigma^2
        vals = [(n - float(sketches[j] @ kg_matvec(grid, hypers, wtx[j]))) / s2 for j in range(N)]
        tr = 2 * s2 * float(np.mean(vals))
    grad[d + 1] = 0.5 * (quad - tr)
    info = {"q": q, "logdet": logdet, "logdet_samples": np.array(logdets),
            "iterations_y": info_y["iterations"], "mu": mu, "wtz": wtz}
    return mll, grad, info


def _exact_trace(grid, hypers, wtw, which, n):
    """Exact traces through S = W^T A^{-1} W (M grid-RHS solves):
    tr(A^{-1} W dK W^T) = tr(S dK);  tr(A^{-1}) = (n - tr(K_G S)) / sigma^2."""
    M = grid_size(grid)
    _, _, sig = _hyp(hypers, grid["d"])
    S = np.zeros((M, M))
    for j in range(M):
        e = np.zeros(M)
        e[j] = 1.0
        S[:, j], _ = solve_grid_rhs(grid, hypers, wtw, e, tol=1e-13)
    if which == "inv":
        KS = kg_matvec(grid, hypers, S.T)  # rows: K_G S[:, j]
        return (n - float(np.trace(KS.T))) / (sig * sig)
    dKS = dkg_matvec(grid, hypers, S.T, which)
    return float(np.trace(dKS.T))


# ---------------------------------------------------------------------------
# Dense n-space references (small n only).
# ---------------------------------------------------------------------------
def ski_dense_mean(grid, hypers, x, y):
    """Def. 2 directly: z~ = (W K_G W^T + sigma^2 I)^{-1} y by Cholesky;
    returns (mu_G = K_G W^T z~, z~, W)."""
    _, _, sig = _hyp(hypers, grid["d"])
    W = dense_w(grid, x)
    KG = kg_dense(grid, hypers)
    A = W @ KG @ W.T + sig * sig * np.eye(W.shape[0])
    z = sla.cho_solve(sla.cho_factor(A), np.asarray(y, float))
    return KG @ (W.T @ z), z, W


def ski_dense_cov(grid, hypers, x, xq):
    """Posterior covariance of the SKI model (Def. 2) between query points
    xq [d, nq], covariance form: Wq K_G Wq^T - Wq K_G W^T A^{-1} W K_G Wq^T
    with A = W K_G W^T + sigma^2 I (dense, small n)."""
    _, _, sig = _hyp(hypers, grid["d"])
    W = dense_w(grid, x)
    Wq = dense_w(grid, xq)
    KG = kg_dense(grid, hypers)
    A = W @ KG @ W.T + sig * sig * np.eye(W.shape[0])
    B = W @ KG @ Wq.T
    return Wq @ KG @ Wq.T - B.T @ sla.cho_solve(sla.cho_factor(A), B)


def efla(grid, hypers, wtw, bhat, bb, k, reorth=2, tol_break=1e-10):
    """Lanczos with full reorthogonalisation on A = W K_G W^T + sigma^2 I from
    b / ||b||, in the factorized form of the appendix (FLA and EFLA, Algs. 6
    and 7): the i-th Lanczos vector is Q_i = W qh_i + d_i b, kept as the pair
    (qh_i, d_i) together with p_i = W^T W qh_i and s_i = (K_G W^T W +
    sigma^2 I) qh_i.  Then A Q_i = W (s_i + d_i K_G bhat) + sigma^2 d_i b, and
    the n-space inner product of two pairs needs only p, bhat = W^T b and
    ||b||^2 = bb:
        <(a, ca), (e, ce)> = p_a . e + ca (bhat . e) + ce (bhat . a) + ca ce bb.
    One operator B per step, applied to the new vector after it has been
    orthogonalised (`reorth` classical Gram-Schmidt passes against all earlier
    vectors).  Stops early when beta_{i+1} <= tol_break * max |alpha| (the
    Krylov space is exhausted).
    Returns (alpha [kk], beta [kk-1], Qh [kk, M], P [kk, M], d [kk])."""
    _, _, sig = _hyp(hypers, grid["d"])
    s2 = sig * sig
    bhat = np.asarray(bhat, np.float64)
    M = bhat.shape[0]
    kb = kg_matvec(grid, hypers, bhat)
    Qh = np.zeros((k, M))
    P = np.zeros((k, M))
    d = np.zeros(k)
    d[0] = 1.0 / np.sqrt(bb)
    s_cur = np.zeros(M)
    al = np.zeros(k)
    be = np.zeros(k)
    kk = k

    def inner(a, ca, pa, e, ce):
        return float(pa @ e + ca * (bhat @ e) + ce * (bhat @ a) + ca * ce * bb)

    for i in range(k):
        # w = A Q_i - beta_i Q_{i-1}
        wq = s_cur + d[i] * kb
        wc = s2 * d[i]
        if i > 0:
            wq = wq - be[i - 1] * Qh[i - 1]
            wc -= be[i - 1] * d[i - 1]
        al[i] = inner(Qh[i], d[i], P[i], wq, wc)
        if i == k - 1:
            break
        wq = wq - al[i] * Qh[i]
        wc -= al[i] * d[i]
        for _ in range(reorth):
            lam = (P[:i + 1] @ wq + d[:i + 1] * (bhat @ wq) + wc * (Qh[:i + 1] @ bhat)
                   + d[:i + 1] * wc * bb)
            wq = wq - lam @ Qh[:i + 1]
            wc -= float(lam @ d[:i + 1])
        v, u = B_apply(grid, hypers, wtw, wq)
        b2 = float(u @ wq + 2.0 * wc * (bhat @ wq) + wc * wc * bb)
        beta = np.sqrt(max(b2, 0.0))
        if beta <= tol_break * np.max(np.abs(al[:i + 1])):
            kk = i + 1
            break
        be[i] = beta
        Qh[i + 1] = wq / beta
        d[i + 1] = wc / beta
        P[i + 1] = u / beta
        s_cur = v / beta
    return al[:kk], be[:kk - 1], Qh[:kk], P[:kk], d[:kk]


def love_cov(grid, hypers, wtw, wty, yty, xq, k):
    """Rank-k posterior covariance between query points xq [d, nq] from the
    factorized Lanczos decomposition A ~ Q T Q^T started at y (the low-rank
    covariance of Sec. 5): with u_j(x) = <Q_j, W K_G w_x> = (p_j + d_j W^T y)
    . (K_G w_x),
        cov(x, x') ~ w_x^T K_G w_x' - u(x)^T T^{-1} u(x').
    Exact when the Krylov space holds every W K_G w_x (k large enough)."""
    al, be, Qh, P, d = efla(grid, hypers, wtw, wty, yty, k)
    T = np.diag(al) + np.diag(be, 1) + np.diag(be, -1)
    Wq = dense_w(grid, xq)
    V = np.column_stack([kg_matvec(grid, hypers, w) for w in Wq])
    U = (P + np.outer(d, np.asarray(wty, np.float64))) @ V
    return Wq @ V - U.T @ np.linalg.solve(T, U)


def ski_dense_mll(grid, hypers, x, y):
    """Def. 2 log likelihood by Cholesky of W K_G W^T + sigma^2 I."""
    _, _, sig = _hyp(hypers, grid["d"])
    W = dense_w(grid, x)
    KG = kg_dense(grid, hypers)
    n = W.shape[0]
    A = W @ KG @ W.T + sig * sig * np.eye(n)
    c = sla.cho_factor(A)
    z = sla.cho_solve(c, np.asarray(y, float))
    logdet = 2 * np.sum(np.log(np.diag(c[0])))
    return -0.5 * (logdet + float(y @ z) + n * np.log(2 * np.pi))


def ski_dense_grad(grid, hypers, x, y):
    """Textbook gradient 1/2 tr((a a^T - A^{-1}) dA), a = A^{-1} y, w.r.t.
    (log l_k, log s, log sigma), all dense."""
    d = grid["d"]
    ell, s, sig = _hyp(hypers, d)
    W = dense_w(grid, x)
    n = W.shape[0]
    M = W.shape[1]
    KG = kg_dense(grid, hypers)
    A = W @ KG @ W.T + sig * sig * np.eye(n)
    Ai = np.linalg.inv(A)
    a = Ai @ y
    g = np.zeros(d + 2)
    for th in range(d + 1):
        dK = np.column_stack([dkg_matvec(grid, hypers, e, th) for e in np.eye(M)])
        dA = W @ dK @ W.T
        g[th] = 0.5 * (a @ dA @ a - np.trace(Ai @ dA))
    dA = 2 * sig * sig * np.eye(n)
    g[d + 1] = 0.5 * (a @ dA @ a - np.trace(Ai @ dA))
    return g


def gsgp_mll_fact2(grid, hypers, wtw, wty, yty, n):
    """Fact 2 log likelihood in m-space (dense, small M):
    -1/2 [ logdet(K_G W^T W + s2 I) + y^T (y - W zbar)/s2 + n log 2pi + (n - M) log s2 ]."""
    _, _, sig = _hyp(hypers, grid["d"])
    s2 = sig * sig
    M = grid_size(grid)
    KG = kg_dense(grid, hypers)
    A = wtw_dense_from_dia(grid, wtw)
    G = KG @ A + s2 * np.eye(M)
    zbar = np.linalg.solve(G, KG @ wty)
    sign, ld = np.linalg.slogdet(G)
    assert sign > 0
    return -0.5 * (ld + (yty - float(wty @ zbar)) / s2 + n * np.log(2 * np.pi) + (n - M) * np.log(s2))


def exact_gp_mean(xtr, y, xq, ell, s, sig):
    """Fact 1 posterior mean with the exact SE kernel (dense, small n)."""
    K = se_kernel(xtr, xtr, ell, s) + sig * sig * np.eye(xtr.shape[0])
    z = sla.cho_solve(sla.cho_factor(K), y)
    return se_kernel(xq, xtr, ell, s) @ z
