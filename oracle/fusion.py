"""Optimisation (Sec. II-C): fuse semi-dense and network terms into log-depth x and scale.

Cost (Sec. II-C, total cost and the three term equations), with x_i = ln d_i and
tau = ln s (readings R16, R12):

    c(x, tau) = sum_i       H((x_i - mu_i) / sigma_net,i)
              + sum_{i in S} H((x_i - tau - z_i) / sqrt(R_i))
              + sum_{u<W-1} H((x_{i+1} - x_i - g_x,i) / sigma_gx,i)
              + sum_{v<H-1} H((x_{i+W} - x_i - g_y,i) / sigma_gy,i)

H(r) = r^2 for |r| <= delta, 2 delta |r| - delta^2 beyond (Huber, equal to the
paper's r^T R^-1 r inside the quadratic zone). Tukey's biweight, which the paper
names as the alternative to try (Sec. V), is the other robust cost available
(``SolverParams.robust``, reading R26): T(r) = (c^2/3) (1 - (1 - (r/c)^2)^3) for
|r| <= c and c^2/3 beyond, normalised like H so that T(r) ~ r^2 for small r; its
IRLS weight T'(r) / (2 r) = (1 - (r/c)^2)^2 inside and 0 beyond. T is not convex:
the uniqueness statements below are Huber's. Every residual is affine in
(x, tau), so c is convex, and strictly convex in x because every pixel has a
network term.

Solvers:
* ``gauss_newton``: the paper's scheme (Sec. II-C, last paragraph): n_gn
  iterations, each fixing IRLS weights, solving for x with tau fixed, then
  updating tau in closed form (reading R13). The x-solve is a direct sparse
  solve or Jacobi PCG with a given iteration count / tolerance (reading R14).
* ``minimiser``: the unique minimiser (x*, tau*) by IRLS on the joint system
  (x and tau together) until the update stops, then exact Newton polishing.

The two ablations of Sec. III are variants of ``gauss_newton``
(``SolverParams.variant``):
* "no_pairwise" (Table III): the cost without c_grad. A is then diagonal and
  each Gauss-Newton x-step is the per-pixel weighted mean of the network and
  semi-dense log-depths, (w_n mu + w_s (tau + z)) / (w_n + w_s).
* "scale_postfit" (Table II): a scale-ambiguous log-depth y minimising
  c_semi + c_grad with tau held at 0 (the semi-dense depths' own scale), then
  the least-squares fit of the scale to the network's log-depth,
  tau = mean_i (mu_i - y_i) over all pixels, unweighted (reading R22), and
  x = y + tau.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class PriorMaps:
    """Network predictions and their variances (Sec. II-A): all H x W float64."""
    mu: np.ndarray        # ln d_net
    var_n: np.ndarray     # sigma_theta,depth^2
    gx: np.ndarray        # g_x (last column unused, R10)
    var_gx: np.ndarray
    gy: np.ndarray        # g_y (last row unused, R10)
    var_gy: np.ndarray


@dataclass
class SemiMeasurements:
    """Semi-dense log-depth measurements (Sec. II-B last step): z = ln d_semi, R = sigma^2."""
    z: np.ndarray
    R: np.ndarray
    valid: np.ndarray     # the set S


@dataclass
class SolverParams:
    n_gn: int = 10
    n_cg: int = 20            # PCG iterations per Gauss-Newton iteration (fixed-count mode)
    cg_rtol: float = 0.0      # > 0: iterate until ||r|| <= rtol ||b|| (cap cg_max)
    cg_max: int = 4000
    huber_delta: float = 1.345
    linear_solver: str = "pcg"   # "pcg" or "direct"
    variant: str = "full"        # "full" (Sec. II-C), "no_pairwise" (Table III), "scale_postfit" (Table II)
    robust: str = "huber"        # "huber" (Sec. II-C) or "tukey" (Sec. V); threshold huber_delta either way


# ---------------------------------------------------------------- Huber

def huber(r, delta):
    a = np.abs(r)
    if np.isinf(delta):
        return r * r
    return np.where(a <= delta, r * r, 2.0 * delta * a - delta * delta)


def huber_derivative(r, delta):
    if np.isinf(delta):
        return 2.0 * r
    return np.where(np.abs(r) <= delta, 2.0 * r, 2.0 * delta * np.sign(r))


def huber_weight(r, delta):
    """IRLS weight H'(r) / (2 r) = min(1, delta / |r|)."""
    if np.isinf(delta):
        return np.ones_like(r)
    a = np.abs(r)
    with np.errstate(divide="ignore"):
        return np.where(a <= delta, 1.0, delta / a)


def tukey(r, c):
    """Tukey's biweight, normalised to r^2 near zero: (c^2/3)(1 - (1 - (r/c)^2)^3), c^2/3 beyond c."""
    t2 = (np.asarray(r) / c) ** 2
    return np.where(t2 <= 1.0, (c * c / 3.0) * (1.0 - (1.0 - t2) ** 3), c * c / 3.0)


def tukey_derivative(r, c):
    r = np.asarray(r)
    t2 = (r / c) ** 2
    return np.where(t2 <= 1.0, 2.0 * r * (1.0 - t2) ** 2, 0.0)


def tukey_weight(r, c):
    """IRLS weight T'(r) / (2 r) = (1 - (r/c)^2)^2 inside c, 0 beyond."""
    t2 = (np.asarray(r) / c) ** 2
    return np.where(t2 <= 1.0, (1.0 - t2) ** 2, 0.0)


def robust_cost(r, delta, robust="huber"):
    return huber(r, delta) if robust == "huber" else tukey(r, delta)


def robust_derivative(r, delta, robust="huber"):
    return huber_derivative(r, delta) if robust == "huber" else tukey_derivative(r, delta)


def robust_weight(r, delta, robust="huber"):
    return huber_weight(r, delta) if robust == "huber" else tukey_weight(r, delta)


# ---------------------------------------------------------------- residuals, cost

def residuals(x, tau, prior: PriorMaps, semi: SemiMeasurements):
    """The four residual families of Sec. II-C (unwhitened)."""
    r_net = x - prior.mu
    r_semi = np.where(semi.valid, x - tau - semi.z, 0.0)
    r_gx = x[:, 1:] - x[:, :-1] - prior.gx[:, :-1]
    r_gy = x[1:, :] - x[:-1, :] - prior.gy[:-1, :]
    return r_net, r_semi, r_gx, r_gy


def _sd(var):
    return np.sqrt(var)


def cost(x, tau, prior: PriorMaps, semi: SemiMeasurements, delta, robust="huber") -> float:
    r_net, r_semi, r_gx, r_gy = residuals(x, tau, prior, semi)
    S = semi.valid
    c = np.sum(robust_cost(r_net / _sd(prior.var_n), delta, robust))
    if np.any(S):
        c += np.sum(robust_cost(r_semi[S] / _sd(semi.R[S]), delta, robust))
    c += np.sum(robust_cost(r_gx / _sd(prior.var_gx[:, :-1]), delta, robust))
    c += np.sum(robust_cost(r_gy / _sd(prior.var_gy[:-1, :]), delta, robust))
    return float(c)


def cost_gradient(x, tau, prior: PriorMaps, semi: SemiMeasurements, delta, robust="huber"):
    """(dc/dx, dc/dtau), by differentiating each term directly (no normal equations)."""
    huber_derivative = lambda r, d: robust_derivative(r, d, robust)   # noqa: E731
    r_net, r_semi, r_gx, r_gy = residuals(x, tau, prior, semi)
    S = semi.valid
    sn = _sd(prior.var_n)
    g = huber_derivative(r_net / sn, delta) / sn
    gt = 0.0
    if np.any(S):
        ss = np.where(S, _sd(np.where(S, semi.R, 1.0)), 1.0)
        ds = np.where(S, huber_derivative(r_semi / ss, delta) / ss, 0.0)
        g = g + ds
        gt = -float(np.sum(ds))
    sx = _sd(prior.var_gx[:, :-1])
    dx = huber_derivative(r_gx / sx, delta) / sx
    g[:, 1:] += dx
    g[:, :-1] -= dx
    sy = _sd(prior.var_gy[:-1, :])
    dy = huber_derivative(r_gy / sy, delta) / sy
    g[1:, :] += dy
    g[:-1, :] -= dy
    return g, gt


# ---------------------------------------------------------------- normal equations

def irls_weights(x, tau, prior: PriorMaps, semi: SemiMeasurements, delta, robust="huber"):
    """Per-term weights h(r/sigma)/sigma^2 at (x, tau) (readings R12, R26)."""
    huber_weight = lambda r, d: robust_weight(r, d, robust)   # noqa: E731
    r_net, r_semi, r_gx, r_gy = residuals(x, tau, prior, semi)
    w_n = huber_weight(r_net / _sd(prior.var_n), delta) / prior.var_n
    S = semi.valid
    Rs = np.where(S, semi.R, 1.0)
    w_s = np.where(S, huber_weight(r_semi / _sd(Rs), delta) / Rs, 0.0)
    vx = prior.var_gx[:, :-1]
    c_x = huber_weight(r_gx / _sd(vx), delta) / vx
    vy = prior.var_gy[:-1, :]
    c_y = huber_weight(r_gy / _sd(vy), delta) / vy
    return w_n, w_s, c_x, c_y


def normal_equations(w_n, w_s, c_x, c_y, tau, prior: PriorMaps, semi: SemiMeasurements):
    """A x = b of the weighted least-squares problem in x with tau fixed.

    A_ii = w_n + w_s + (weights of the up to four edges at i); A_{i,i+1} = -c_x,i;
    A_{i,i+W} = -c_y,i; b_i = w_n mu_i + w_s (tau + z_i) - c_x,i g_x,i + c_x,i-1 g_x,i-1
    - c_y,i g_y,i + c_y,i-W g_y,i-W.
    """
    H, W = prior.mu.shape
    N = H * W
    diag = w_n + w_s
    diag = diag.copy()
    diag[:, :-1] += c_x
    diag[:, 1:] += c_x
    diag[:-1, :] += c_y
    diag[1:, :] += c_y
    z = np.where(semi.valid, semi.z, 0.0)
    b = w_n * prior.mu + w_s * (tau + z)
    gx = prior.gx[:, :-1]
    gy = prior.gy[:-1, :]
    b[:, :-1] -= c_x * gx
    b[:, 1:] += c_x * gx
    b[:-1, :] -= c_y * gy
    b[1:, :] += c_y * gy
    idx = np.arange(N).reshape(H, W)
    rows = [idx.ravel()]
    cols = [idx.ravel()]
    vals = [diag.ravel()]
    ia, ib = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    rows += [ia, ib]
    cols += [ib, ia]
    vals += [-c_x.ravel(), -c_x.ravel()]
    ja, jb = idx[:-1, :].ravel(), idx[1:, :].ravel()
    rows += [ja, jb]
    cols += [jb, ja]
    vals += [-c_y.ravel(), -c_y.ravel()]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    return A, b.ravel()


# ---------------------------------------------------------------- linear solvers

def solve_direct(A, b):
    """Sparse LU (SuperLU) solve."""
    return spla.splu(A.tocsc()).solve(b)


def pcg(A, b, x0, n_iter: int, rtol: float = 0.0, max_iter: int = 4000):
    """Jacobi-preconditioned conjugate gradients, textbook form.

    Fixed-count mode (rtol == 0): exactly n_iter iterations. Tolerance mode:
    stop once ||r|| <= rtol ||b|| (tested before the first iteration and after
    each), at most max_iter iterations. Stops early if r^T z reaches zero.
    Returns (x, iterations done).
    """
    d = A.diagonal()
    # a row whose every term has zero weight (possible with Tukey's cost) keeps
    # its value: its preconditioned residual is taken as 0
    dinv = np.divide(1.0, d, out=np.zeros_like(d), where=d > 0)
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - A @ x
    z = r * dinv
    p = z.copy()
    rz = float(r @ z)
    bnorm = float(np.sqrt(b @ b))
    limit = max_iter if rtol > 0 else n_iter
    if rtol > 0 and np.sqrt(r @ r) <= rtol * bnorm:
        return x, 0
    it = 0
    while it < limit:
        if rz == 0.0:
            break
        q = A @ p
        alpha = rz / float(p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        z = r * dinv
        rz_new = float(r @ z)
        if rtol > 0 and np.sqrt(r @ r) <= rtol * bnorm:
            break
        if it == limit:
            break
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, it


# ---------------------------------------------------------------- Gauss-Newton

def scale_step(x, tau, semi: SemiMeasurements, delta, robust="huber"):
    """Closed-form tau with the semi weights at (x, tau): sum w (x - z) / sum w (R13);
    unchanged when no semi-dense term has weight."""
    S = semi.valid
    if not np.any(S):
        return tau
    r = (x[S] - tau - semi.z[S]) / np.sqrt(semi.R[S])
    w = robust_weight(r, delta, robust) / semi.R[S]
    if not np.sum(w) > 0.0:
        return tau
    return float(np.sum(w * (x[S] - semi.z[S])) / np.sum(w))


@dataclass
class GNInfo:
    cg_iterations: List[int] = field(default_factory=list)
    costs: List[float] = field(default_factory=list)


def gauss_newton(x0, tau0, prior: PriorMaps, semi: SemiMeasurements, params: SolverParams):
    """The paper's alternating Gauss-Newton scheme (Sec. II-C; readings R13, R14),
    or one of its two ablations (Sec. III, Tables II and III)."""
    if params.variant == "scale_postfit":
        return scale_postfit(x0, tau0, prior, semi, params)
    if params.variant not in ("full", "no_pairwise"):
        raise ValueError(params.variant)
    delta = params.huber_delta
    H, W = prior.mu.shape
    x = np.array(x0, dtype=np.float64, copy=True)
    tau = float(tau0)
    info = GNInfo()
    rb = params.robust
    for _ in range(params.n_gn):
        w_n, w_s, c_x, c_y = irls_weights(x, tau, prior, semi, delta, rb)
        if params.variant == "no_pairwise":
            # Table III: no gradient terms, so A is diagonal and the x-step is
            # the per-pixel weighted mean of the two log-depth estimates
            z = np.where(semi.valid, semi.z, 0.0)
            wsum = w_n + w_s
            x = np.where(wsum > 0, (w_n * prior.mu + w_s * (tau + z)) / np.where(wsum > 0, wsum, 1.0), x)
            its = 0
        else:
            A, b = normal_equations(w_n, w_s, c_x, c_y, tau, prior, semi)
            if params.linear_solver == "direct":
                xv = solve_direct(A, b)
                its = -1
            else:
                xv, its = pcg(A, b, x.ravel(), params.n_cg, params.cg_rtol, params.cg_max)
            x = xv.reshape(H, W)
        tau = scale_step(x, tau, semi, delta, rb)
        info.cg_iterations.append(its)
        info.costs.append(cost(x, tau, prior, semi, delta, rb))
    return x, tau, info


def scale_postfit(x0, tau0, prior: PriorMaps, semi: SemiMeasurements, params: SolverParams):
    """Table II's alternative to solving for the scale: n_gn IRLS Gauss-Newton
    iterations on c_semi + c_grad alone with tau = 0, which gives a log-depth y
    in the semi-dense depths' scale (warm start y = x0 - tau0), then the
    least-squares fit of a global log-scale offset to the network log-depth,
    tau = mean(mu - y) (reading R22). Returns (y + tau, tau, info)."""
    delta = params.huber_delta
    H, W = prior.mu.shape
    y = np.array(x0, dtype=np.float64, copy=True) - float(tau0)
    info = GNInfo()
    zeros = np.zeros((H, W))
    for _ in range(params.n_gn):
        _, w_s, c_x, c_y = irls_weights(y, 0.0, prior, semi, delta, params.robust)
        A, b = normal_equations(zeros, w_s, c_x, c_y, 0.0, prior, semi)   # no network term
        if params.linear_solver == "direct":
            yv = solve_direct(A, b)
            its = -1
        else:
            yv, its = pcg(A, b, y.ravel(), params.n_cg, params.cg_rtol, params.cg_max)
        y = yv.reshape(H, W)
        info.cg_iterations.append(its)
    tau = float(np.mean(prior.mu - y))
    return y + tau, tau, info


def minimiser(prior: PriorMaps, semi: SemiMeasurements, delta, x0=None, tau0: float = 0.0,
              tol: float = 1e-13, max_iter: int = 5000):
    """The unique minimiser (x*, tau*) of c (tau held at tau0 when S is empty).

    IRLS on the joint (x, tau) system until the step falls below ``tol``, then
    Newton steps on the piecewise-quadratic cost with the active set of the
    current point (accepted only if they lower the gradient norm).
    """
    H, W = prior.mu.shape
    N = H * W
    x = np.array(prior.mu if x0 is None else x0, dtype=np.float64, copy=True)
    tau = float(tau0)
    S = semi.valid
    has_s = bool(np.any(S))
    zs = np.where(S, semi.z, 0.0).ravel()

    def joint_solve(w_n, w_s, c_x, c_y):
        A, b = normal_equations(w_n, w_s, c_x, c_y, 0.0, prior, semi)
        if not has_s:
            A2, b2 = normal_equations(w_n, w_s, c_x, c_y, tau, prior, semi)
            return solve_direct(A2, b2).reshape(H, W), tau
        ws = w_s.ravel()
        col = sp.csr_matrix(-ws[:, None])
        M = sp.bmat([[A, col], [col.T, sp.csr_matrix([[ws.sum()]])]], format="csc")
        rhs = np.concatenate([b, [-(ws * zs).sum()]])
        sol = spla.splu(M).solve(rhs)
        return sol[:N].reshape(H, W), float(sol[N])

    for _ in range(max_iter):
        w = irls_weights(x, tau, prior, semi, delta)
        xn, tn = joint_solve(*w)
        step = max(float(np.max(np.abs(xn - x))), abs(tn - tau))
        x, tau = xn, tn
        if step < tol:
            break
    # Newton polish: weights 1 inside the quadratic zone, 0 outside, with the
    # outside residuals' constant slopes moved to the right-hand side. This is
    # one exact Newton step on the piecewise-quadratic cost.
    if not np.isinf(delta):
        for _ in range(5):
            g, gt = cost_gradient(x, tau, prior, semi, delta)
            gnorm = np.sqrt(np.sum(g * g) + gt * gt)
            if gnorm == 0.0:
                break
            xs, ts = _newton_step(x, tau, prior, semi, delta, has_s)
            if xs is None:
                break
            g2, gt2 = cost_gradient(xs, ts, prior, semi, delta)
            if np.sqrt(np.sum(g2 * g2) + gt2 * gt2) < gnorm:
                x, tau = xs, ts
            else:
                break
    return x, tau


def _newton_step(x, tau, prior, semi, delta, has_s):
    """Exact Newton step of the Huber cost at (x, tau) (generalised Hessian)."""
    H, W = prior.mu.shape
    N = H * W
    r_net, r_semi, r_gx, r_gy = residuals(x, tau, prior, semi)
    S = semi.valid
    # Hessian weights: 1/sigma^2 for quadratic-zone terms, 0 otherwise
    def hw(r, var):
        return np.where(np.abs(r / np.sqrt(var)) <= delta, 1.0 / var, 0.0)
    Rs = np.where(S, semi.R, 1.0)
    w_n = hw(r_net, prior.var_n)
    w_s = np.where(S, hw(r_semi, Rs), 0.0)
    c_x = hw(r_gx, prior.var_gx[:, :-1])
    c_y = hw(r_gy, prior.var_gy[:-1, :])
    A, _ = normal_equations(w_n, w_s, c_x, c_y, 0.0, prior, semi)
    g, gt = cost_gradient(x, tau, prior, semi, delta)
    grad = np.concatenate([g.ravel(), [gt]]) / 2.0   # cost is sum H, Hessian of H/2 is w
    if has_s:
        ws = w_s.ravel()
        col = sp.csr_matrix(-ws[:, None])
        M = sp.bmat([[A, col], [col.T, sp.csr_matrix([[ws.sum()]])]], format="csc")
    else:
        M = A.tocsc()
        grad = grad[:N]
    try:
        step = spla.splu(M).solve(-grad)
    except RuntimeError:
        return None, None
    if not np.all(np.isfinite(step)):
        return None, None
    xs = x + step[:N].reshape(H, W)
    ts = tau + (float(step[N]) if has_s else 0.0)
    return xs, ts
