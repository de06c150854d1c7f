"""Pins of the fusion oracle (Sec. II-C): invariants, closed forms, independent solvers."""

import numpy as np
import pytest
import scipy.linalg
import scipy.optimize
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fusion
from oracle.fusion import PriorMaps, SemiMeasurements, SolverParams

DELTA = 1.345


def _problem(H, W, seed=0, semi_frac=0.4, outliers=0.05, noiseless=False, tau_true=0.3):
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:H, 0:W]
    xt = 0.6 + 0.02 * xx - 0.015 * yy + 0.1 * np.sin(0.3 * xx) * np.cos(0.2 * yy)
    vn = np.exp(rng.uniform(np.log(0.02), np.log(0.3), (H, W))) ** 2
    vgx = np.exp(rng.uniform(np.log(0.01), np.log(0.2), (H, W))) ** 2
    vgy = np.exp(rng.uniform(np.log(0.01), np.log(0.2), (H, W))) ** 2
    gx = np.zeros((H, W))
    gx[:, :-1] = xt[:, 1:] - xt[:, :-1]
    gy = np.zeros((H, W))
    gy[:-1, :] = xt[1:, :] - xt[:-1, :]
    S = rng.random((H, W)) < semi_frac
    R = np.exp(rng.uniform(np.log(1e-4), np.log(1e-2), (H, W)))
    z = xt - tau_true
    mu = xt.copy()
    if not noiseless:
        mu = mu + np.sqrt(vn) * rng.standard_normal((H, W))
        gx = gx + np.sqrt(vgx) * rng.standard_normal((H, W))
        gy = gy + np.sqrt(vgy) * rng.standard_normal((H, W))
        z = z + np.sqrt(R) * rng.standard_normal((H, W))
        out = rng.random((H, W)) < outliers
        z = np.where(out, z + rng.normal(0, 0.5, (H, W)), z)
    prior = PriorMaps(mu, vn, gx, vgx, gy, vgy)
    semi = SemiMeasurements(np.where(S, z, 0.0), np.where(S, R, np.inf), S)
    return prior, semi, xt


def _stacked_system(prior, semi, w_n, w_s, c_x, c_y, tau):
    """Whitened residual rows sqrt(w) (J x - y), built term by term (no normal equations)."""
    H, W = prior.mu.shape
    N = H * W
    idx = np.arange(N).reshape(H, W)
    rows, cols, vals, rhs = [], [], [], []
    r = 0
    for i in range(N):
        rows.append(r); cols.append(i); vals.append(np.sqrt(w_n.ravel()[i]))
        rhs.append(np.sqrt(w_n.ravel()[i]) * prior.mu.ravel()[i]); r += 1
    for i in np.flatnonzero(semi.valid.ravel()):
        s = np.sqrt(w_s.ravel()[i])
        rows.append(r); cols.append(i); vals.append(s)
        rhs.append(s * (tau + semi.z.ravel()[i])); r += 1
    for v in range(H):
        for u in range(W - 1):
            s = np.sqrt(c_x[v, u])
            rows += [r, r]; cols += [idx[v, u + 1], idx[v, u]]; vals += [s, -s]
            rhs.append(s * prior.gx[v, u]); r += 1
    for v in range(H - 1):
        for u in range(W):
            s = np.sqrt(c_y[v, u])
            rows += [r, r]; cols += [idx[v + 1, u], idx[v, u]]; vals += [s, -s]
            rhs.append(s * prior.gy[v, u]); r += 1
    J = np.zeros((r, N))
    J[rows, cols] = vals
    return J, np.array(rhs)


def test_normal_equations_match_stacked_least_squares():
    """P12/P4: A, b equal J^T J, J^T y of the term-by-term residual rows; lstsq agrees."""
    prior, semi, _ = _problem(5, 7, seed=1)
    x = prior.mu + 0.05
    tau = 0.1
    w = fusion.irls_weights(x, tau, prior, semi, DELTA)
    A, b = fusion.normal_equations(*w, tau, prior, semi)
    J, y = _stacked_system(prior, semi, *w, tau)
    assert np.allclose(A.toarray(), J.T @ J, rtol=1e-12, atol=1e-9)
    assert np.allclose(b, J.T @ y, rtol=1e-12, atol=1e-9)
    xs = fusion.solve_direct(A, b)
    xl = np.linalg.lstsq(J, y, rcond=None)[0]
    assert np.allclose(xs, xl, rtol=0, atol=1e-10)
    Ad = A.toarray()
    assert np.allclose(Ad, Ad.T)
    off = np.sum(np.abs(Ad), axis=1) - np.abs(np.diag(Ad))
    assert np.all(np.diag(Ad) > off)                     # strictly diagonally dominant -> SPD
    assert np.linalg.norm(A @ xs - b) / np.linalg.norm(b) < 1e-12


def test_prior_only_returns_prior():
    """P1: no semi-dense measurement and g = forward difference of mu -> x = mu, tau = 0."""
    prior, semi, _ = _problem(12, 16, seed=2, semi_frac=0.0)
    mu = prior.mu
    prior.gx[:, :-1] = mu[:, 1:] - mu[:, :-1]
    prior.gy[:-1, :] = mu[1:, :] - mu[:-1, :]
    for solver in ("direct", "pcg"):
        x, tau, _ = fusion.gauss_newton(mu, 0.0, prior, semi,
                                        SolverParams(n_gn=10, n_cg=20, linear_solver=solver))
        assert np.max(np.abs(x - mu)) <= 1e-12
        assert tau == 0.0
    xm, tm = fusion.minimiser(prior, semi, DELTA)
    assert np.max(np.abs(xm - mu)) <= 1e-12 and tm == 0.0


def test_noiseless_consistent_input_recovers_truth():
    """P2: mu = x_true, g = D x_true, z = x_true - tau_true -> unique minimiser (x_true, tau_true)."""
    prior, semi, xt = _problem(10, 14, seed=3, noiseless=True, tau_true=0.3)
    xm, tm = fusion.minimiser(prior, semi, DELTA)
    assert np.max(np.abs(xm - xt)) < 1e-10
    assert abs(tm - 0.3) < 1e-10
    # the paper's 10-iteration alternating scheme moves toward it from (mu, 0) ... here mu = x_true
    x, tau, info = fusion.gauss_newton(prior.mu, 0.0, prior, semi, SolverParams(n_gn=10, linear_solver="direct"))
    assert info.costs[-1] <= info.costs[0]
    assert abs(tau - 0.3) < abs(0.0 - 0.3)


@pytest.mark.parametrize("delta", [DELTA, np.inf])
def test_kkt_at_minimiser(delta):
    """P3: the gradient of c (differentiated term by term) vanishes at the minimiser."""
    prior, semi, _ = _problem(9, 11, seed=4)
    g0, gt0 = fusion.cost_gradient(prior.mu, 0.0, prior, semi, delta)
    xm, tm = fusion.minimiser(prior, semi, delta)
    g, gt = fusion.cost_gradient(xm, tm, prior, semi, delta)
    scale = np.sqrt(np.sum(g0 * g0) + gt0 * gt0)
    assert np.sqrt(np.sum(g * g) + gt * gt) <= 1e-9 * scale


def test_cost_gradient_matches_finite_differences():
    prior, semi, _ = _problem(4, 5, seed=5)
    rng = np.random.default_rng(0)
    x = prior.mu + 0.1 * rng.standard_normal(prior.mu.shape)
    tau = 0.2
    g, gt = fusion.cost_gradient(x, tau, prior, semi, DELTA)
    h = 1e-6
    for i in range(x.size):
        e = np.zeros(x.size)
        e[i] = h
        e = e.reshape(x.shape)
        fd = (fusion.cost(x + e, tau, prior, semi, DELTA) - fusion.cost(x - e, tau, prior, semi, DELTA)) / (2 * h)
        assert abs(fd - g.ravel()[i]) <= 1e-5 * max(1.0, abs(fd))
    fd = (fusion.cost(x, tau + h, prior, semi, DELTA) - fusion.cost(x, tau - h, prior, semi, DELTA)) / (2 * h)
    assert abs(fd - gt) <= 1e-5 * max(1.0, abs(fd))


def test_huber_weight_is_derivative_ratio():
    r = np.linspace(-5, 5, 1001)
    w = fusion.huber_weight(r, DELTA)
    dH = fusion.huber_derivative(r, DELTA)
    nz = r != 0
    assert np.allclose(w[nz], dH[nz] / (2 * r[nz]))
    # H is C^1 at |r| = delta and equals r^2 inside
    assert np.allclose(fusion.huber(np.array([0.5, -1.0]), DELTA), [0.25, 1.0])
    eps = 1e-9
    assert abs(fusion.huber(np.array([DELTA + eps]), DELTA)[0] - fusion.huber(np.array([DELTA - eps]), DELTA)[0]) < 1e-8


def test_independent_minimiser_scipy_least_squares():
    """P15: scipy's robust least squares (loss='huber', f_scale=delta) finds the same point.

    scipy minimises 0.5 sum f_scale^2 rho((f/f_scale)^2) with rho(z) = z (z <= 1),
    2 sqrt(z) - 1 otherwise, which is half of sum H(f) for the whitened residuals f.
    """
    prior, semi, _ = _problem(6, 8, seed=6, outliers=0.15)
    H, W = prior.mu.shape
    S = semi.valid

    def fun(p):
        x = p[:-1].reshape(H, W)
        tau = p[-1]
        rn, rs, rgx, rgy = fusion.residuals(x, tau, prior, semi)
        return np.concatenate([
            (rn / np.sqrt(prior.var_n)).ravel(),
            (rs[S] / np.sqrt(semi.R[S])).ravel(),
            (rgx / np.sqrt(prior.var_gx[:, :-1])).ravel(),
            (rgy / np.sqrt(prior.var_gy[:-1, :])).ravel(),
        ])

    p0 = np.concatenate([prior.mu.ravel(), [0.0]])
    sol = scipy.optimize.least_squares(fun, p0, loss="huber", f_scale=DELTA, xtol=1e-15, ftol=1e-15,
                                       gtol=1e-15, max_nfev=20000, method="trf")
    xm, tm = fusion.minimiser(prior, semi, DELTA)
    assert np.max(np.abs(sol.x[:-1] - xm.ravel())) < 1e-8
    assert abs(sol.x[-1] - tm) < 1e-8


def test_no_gradient_terms_closed_form():
    """P5 (the paper's no-pairwise variant): each pixel is a weighted mean of its unaries."""
    prior, semi, _ = _problem(7, 9, seed=7)
    prior.var_gx[:] = np.inf
    prior.var_gy[:] = np.inf
    x0 = prior.mu + 0.01
    tau = 0.15
    w_n, w_s, c_x, c_y = fusion.irls_weights(x0, tau, prior, semi, DELTA)
    assert np.all(c_x == 0) and np.all(c_y == 0)
    A, b = fusion.normal_equations(w_n, w_s, c_x, c_y, tau, prior, semi)
    x = fusion.solve_direct(A, b).reshape(prior.mu.shape)
    z = np.where(semi.valid, semi.z, 0.0)
    expect = (w_n * prior.mu + w_s * (tau + z)) / (w_n + w_s)
    assert np.allclose(x, expect, rtol=1e-13, atol=1e-14)


def test_single_row_is_tridiagonal():
    """P6: H = 1 gives a tridiagonal system; banded and dense solvers agree with SuperLU."""
    prior, semi, _ = _problem(1, 40, seed=8)
    w = fusion.irls_weights(prior.mu, 0.0, prior, semi, DELTA)
    A, b = fusion.normal_equations(*w, 0.0, prior, semi)
    Ad = A.toarray()
    assert np.count_nonzero(np.triu(Ad, 2)) == 0 and np.count_nonzero(np.tril(Ad, -2)) == 0
    ab = np.zeros((3, 40))
    ab[0, 1:] = np.diag(Ad, 1)
    ab[1] = np.diag(Ad)
    ab[2, :-1] = np.diag(Ad, -1)
    xb = scipy.linalg.solve_banded((1, 1), ab, b)
    assert np.allclose(fusion.solve_direct(A, b), xb, rtol=1e-13, atol=1e-13)
    assert np.allclose(np.linalg.solve(Ad, b), xb, rtol=1e-12, atol=1e-13)


def test_shift_invariance():
    """P13: mu + c and z + c (gradients unchanged) shift x by c and leave tau unchanged."""
    prior, semi, _ = _problem(8, 10, seed=9)
    c = 0.37
    x1, t1, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi, SolverParams(n_gn=4, linear_solver="direct"))
    p2 = PriorMaps(prior.mu + c, prior.var_n, prior.gx, prior.var_gx, prior.gy, prior.var_gy)
    s2 = SemiMeasurements(np.where(semi.valid, semi.z + c, 0.0), semi.R, semi.valid)
    x2, t2, _ = fusion.gauss_newton(p2.mu, 0.0, p2, s2, SolverParams(n_gn=4, linear_solver="direct"))
    assert np.allclose(x2, x1 + c, atol=1e-11)
    assert abs(t2 - t1) < 1e-11


def test_scale_shift_metamorphic():
    """P7 (solver side): z - c (a pose source at another scale) moves tau by +c, x unchanged."""
    prior, semi, _ = _problem(8, 10, seed=10)
    c = 0.25
    xm, tm = fusion.minimiser(prior, semi, DELTA)
    s2 = SemiMeasurements(np.where(semi.valid, semi.z - c, 0.0), semi.R, semi.valid)
    xm2, tm2 = fusion.minimiser(prior, s2, DELTA, tau0=c)
    assert np.max(np.abs(xm2 - xm)) < 1e-10
    assert abs(tm2 - (tm + c)) < 1e-10


def test_transpose_invariance():
    """P14: transposing every map and swapping the x/y gradient predictions transposes x."""
    prior, semi, _ = _problem(6, 9, seed=11)
    pt = PriorMaps(prior.mu.T.copy(), prior.var_n.T.copy(), prior.gy.T.copy(), prior.var_gy.T.copy(),
                   prior.gx.T.copy(), prior.var_gx.T.copy())
    st = SemiMeasurements(semi.z.T.copy(), semi.R.T.copy(), semi.valid.T.copy())
    prm = SolverParams(n_gn=3, linear_solver="direct")
    x1, t1, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi, prm)
    x2, t2, _ = fusion.gauss_newton(pt.mu, 0.0, pt, st, prm)
    assert np.allclose(x2, x1.T, atol=1e-12)
    assert abs(t1 - t2) < 1e-12


def test_pcg_matches_scipy_cg_iterates():
    """The textbook Jacobi PCG equals scipy's CG with the Jacobi preconditioner, iterate by iterate."""
    prior, semi, _ = _problem(12, 15, seed=12)
    w = fusion.irls_weights(prior.mu, 0.0, prior, semi, DELTA)
    A, b = fusion.normal_equations(*w, 0.0, prior, semi)
    d = A.diagonal()
    M = spla.LinearOperator(A.shape, matvec=lambda v: v / d)
    x0 = prior.mu.ravel() + 0.01
    for k in (1, 3, 7, 20):
        xo, its = fusion.pcg(A, b, x0, k)
        assert its == k
        xs, _ = spla.cg(A, b, x0=x0, rtol=0.0, atol=0.0, maxiter=k, M=M)
        assert np.allclose(xo, xs, rtol=1e-10, atol=1e-12)
    xr, its = fusion.pcg(A, b, x0, 0, rtol=1e-12, max_iter=4000)
    assert np.linalg.norm(A @ xr - b) <= 1e-12 * np.linalg.norm(b) * 1.01
    assert np.allclose(xr, fusion.solve_direct(A, b), atol=1e-9)


def test_scale_step_zeroes_tau_gradient():
    """R13: after the closed-form step, dc/dtau = 0 for plain least squares (delta = inf)."""
    prior, semi, _ = _problem(8, 8, seed=13)
    x = prior.mu
    tau = fusion.scale_step(x, 0.0, semi, np.inf)
    _, gt = fusion.cost_gradient(x, tau, prior, semi, np.inf)
    assert abs(gt) < 1e-8
    # empty S leaves tau unchanged
    empty = SemiMeasurements(semi.z, semi.R, np.zeros_like(semi.valid))
    assert fusion.scale_step(x, 0.42, empty, DELTA) == 0.42


def test_alternating_scheme_converges_to_minimiser():
    """Many alternating iterations (R13) reach the joint minimiser of c."""
    prior, semi, _ = _problem(6, 7, seed=14)
    xm, tm = fusion.minimiser(prior, semi, DELTA)
    x, tau, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi, SolverParams(n_gn=3000, linear_solver="direct"))
    assert np.max(np.abs(x - xm)) < 1e-8 and abs(tau - tm) < 1e-8


def test_gauss_newton_cost_decreases():
    prior, semi, _ = _problem(20, 24, seed=15)
    c0 = fusion.cost(prior.mu, 0.0, prior, semi, DELTA)
    x, tau, info = fusion.gauss_newton(prior.mu, 0.0, prior, semi, SolverParams(n_gn=10, linear_solver="direct"))
    costs = [c0] + info.costs
    assert all(b <= a * (1 + 1e-12) for a, b in zip(costs, costs[1:]))


# ------------------------------------------------------------------ ablation variants (Sec. III)

def _no_grad(prior):
    return PriorMaps(prior.mu, prior.var_n, prior.gx, np.full_like(prior.var_gx, np.inf), prior.gy,
                     np.full_like(prior.var_gy, np.inf))


def _no_net(prior):
    return PriorMaps(prior.mu, np.full_like(prior.var_n, np.inf), prior.gx, prior.var_gx, prior.gy, prior.var_gy)


@pytest.mark.parametrize("delta", [DELTA, np.inf])
def test_no_pairwise_variant_equals_full_scheme_without_gradient_terms(delta):
    """Table III variant: its closed-form x-steps equal the full scheme's sparse
    solves on the same problem with the gradient terms removed (infinite gradient
    variances: zero edge weights), iteration by iteration. A gradient term left in
    the variant, or a wrong weight in its weighted mean, fails."""
    prior, semi, _ = _problem(8, 11, seed=21)
    x0 = prior.mu + 0.02
    a = fusion.gauss_newton(x0, 0.1, prior, semi, SolverParams(n_gn=6, huber_delta=delta, variant="no_pairwise"))
    b = fusion.gauss_newton(x0, 0.1, _no_grad(prior), semi, SolverParams(n_gn=6, huber_delta=delta,
                                                                          linear_solver="direct"))
    assert np.max(np.abs(a[0] - b[0])) <= 1e-12 and abs(a[1] - b[1]) <= 1e-12


def test_no_pairwise_variant_converges_to_the_minimiser_without_gradient_terms():
    """Iterated to convergence the variant reaches the unique minimiser of
    c_net + c_semi (joint IRLS + Newton polish, an independent solver)."""
    prior, semi, _ = _problem(7, 9, seed=22)
    xm, tm = fusion.minimiser(_no_grad(prior), semi, DELTA)
    x, tau, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi, SolverParams(n_gn=400, variant="no_pairwise"))
    assert np.max(np.abs(x - xm)) <= 1e-9 and abs(tau - tm) <= 1e-9


@pytest.mark.parametrize("delta", [DELTA, np.inf])
def test_scale_postfit_noiseless_recovers_truth(delta):
    """Table II variant on noiseless consistent input (mu = x_true, g = D x_true,
    z = x_true - tau_true): the scale-ambiguous solve gives y = x_true - tau_true
    and the least-squares fit tau = tau_true, so x = x_true."""
    prior, semi, xt = _problem(9, 12, seed=23, noiseless=True, tau_true=0.4)
    x, tau, _ = fusion.gauss_newton(prior.mu + 0.05, 0.0, prior, semi,
                                    SolverParams(n_gn=3, huber_delta=delta, linear_solver="direct",
                                                 variant="scale_postfit"))
    assert np.max(np.abs(x - xt)) <= 1e-10 and abs(tau - 0.4) <= 1e-10


def test_scale_postfit_ignores_the_network_depth_until_the_fit():
    """The scale-ambiguous log-depth y = x - tau does not depend on the network's
    log-depth at all; replacing mu moves only tau, by the mean of the change.
    A network term left in the scale-ambiguous solve fails."""
    prior, semi, _ = _problem(8, 10, seed=24)
    prm = SolverParams(n_gn=5, linear_solver="direct", variant="scale_postfit")
    x1, t1, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi, prm)
    rng = np.random.default_rng(5)
    dmu = rng.normal(0.0, 0.3, prior.mu.shape)
    p2 = PriorMaps(prior.mu + dmu, prior.var_n, prior.gx, prior.var_gx, prior.gy, prior.var_gy)
    x2, t2, _ = fusion.gauss_newton(prior.mu, 0.0, p2, semi, prm)
    assert np.max(np.abs((x2 - t2) - (x1 - t1))) <= 1e-12
    assert abs((t2 - t1) - float(np.mean(dmu))) <= 1e-12


def test_scale_postfit_solve_is_stationary_for_semi_and_gradient_terms():
    """Iterated to convergence, y zeroes the gradient of c_semi + c_grad at tau = 0
    (differentiated term by term, the network term removed)."""
    prior, semi, _ = _problem(7, 9, seed=25)
    x, tau, _ = fusion.gauss_newton(prior.mu, 0.0, prior, semi,
                                    SolverParams(n_gn=300, linear_solver="direct", variant="scale_postfit"))
    y = x - tau
    g0, _ = fusion.cost_gradient(prior.mu, 0.0, _no_net(prior), semi, DELTA)
    g, _ = fusion.cost_gradient(y, 0.0, _no_net(prior), semi, DELTA)
    assert np.sqrt(np.sum(g * g)) <= 1e-9 * np.sqrt(np.sum(g0 * g0))


# ------------------------------------------------------------------ Tukey's biweight (Sec. V)

def test_tukey_weight_is_derivative_ratio_and_cost_matches_finite_differences():
    """R26: T'(r) / (2 r) is the IRLS weight; T' agrees with central differences
    of T; T ~ r^2 for small r and is flat (c^2/3) beyond c."""
    c = 4.685
    r = np.linspace(-9.0, 9.0, 1001)
    r = r[np.abs(np.abs(r) - c) > 1e-3]
    h = 1e-6
    fd = (fusion.tukey(r + h, c) - fusion.tukey(r - h, c)) / (2 * h)
    assert np.allclose(fusion.tukey_derivative(r, c), fd, atol=1e-6)
    nz = np.abs(r) > 1e-3
    assert np.allclose(fusion.tukey_weight(r[nz], c), fusion.tukey_derivative(r[nz], c) / (2 * r[nz]), atol=1e-12)
    assert np.allclose(fusion.tukey(np.array([1e-4]), c), 1e-8, rtol=1e-6)
    assert np.all(fusion.tukey(np.array([c, 2 * c, 50.0]), c) == c * c / 3.0)
    assert np.all(fusion.tukey_weight(np.array([c * 1.0001, 10 * c]), c) == 0.0)


def test_tukey_with_a_huge_threshold_is_least_squares():
    """c -> infinity: every weight -> 1, so Tukey's scheme equals plain least squares."""
    prior, semi, _ = _problem(8, 9, seed=31)
    a = fusion.gauss_newton(prior.mu, 0.0, prior, semi, SolverParams(n_gn=4, huber_delta=1e7, robust="tukey",
                                                                      linear_solver="direct"))
    b = fusion.gauss_newton(prior.mu, 0.0, prior, semi, SolverParams(n_gn=4, huber_delta=np.inf,
                                                                      linear_solver="direct"))
    assert np.max(np.abs(a[0] - b[0])) <= 1e-9 and abs(a[1] - b[1]) <= 1e-9


def test_tukey_rejects_a_gross_outlier_exactly():
    """A semi-dense measurement whose whitened residual stays beyond c at every
    iterate gets weight 0: the result equals the problem without it (Huber would
    still pull on it)."""
    prior, semi, _ = _problem(8, 10, seed=32, outliers=0.0)
    S = np.argwhere(semi.valid)
    v, u = S[len(S) // 2]
    z2 = semi.z.copy()
    z2[v, u] += 3.0                                       # whitened residual ~ 3 / 0.1 = 30 >> c
    bad = SemiMeasurements(z2, semi.R, semi.valid)
    keep = semi.valid.copy()
    keep[v, u] = False
    drop = SemiMeasurements(np.where(keep, semi.z, 0.0), np.where(keep, semi.R, np.inf), keep)
    prm = SolverParams(n_gn=6, huber_delta=4.685, robust="tukey", linear_solver="direct")
    a = fusion.gauss_newton(prior.mu, 0.0, prior, bad, prm)
    b = fusion.gauss_newton(prior.mu, 0.0, prior, drop, prm)
    assert np.max(np.abs(a[0] - b[0])) <= 1e-12 and abs(a[1] - b[1]) <= 1e-12
    hub = fusion.gauss_newton(prior.mu, 0.0, prior, bad, SolverParams(n_gn=6, huber_delta=4.685,
                                                                       linear_solver="direct"))
    hub0 = fusion.gauss_newton(prior.mu, 0.0, prior, drop, SolverParams(n_gn=6, huber_delta=4.685,
                                                                         linear_solver="direct"))
    assert np.max(np.abs(hub[0] - hub0[0])) > 1e-6


def test_tukey_irls_does_not_increase_the_cost():
    """IRLS with exact solves is a majorise-minimise scheme for Tukey's cost: each
    weighted least-squares step and each closed-form scale step lowers (or keeps)
    the Tukey cost."""
    prior, semi, _ = _problem(9, 11, seed=33, outliers=0.15)
    prm = SolverParams(n_gn=12, huber_delta=4.685, robust="tukey", linear_solver="direct")
    c0 = fusion.cost(prior.mu, 0.0, prior, semi, 4.685, "tukey")
    _, _, info = fusion.gauss_newton(prior.mu, 0.0, prior, semi, prm)
    costs = [c0] + info.costs
    assert all(b <= a * (1 + 1e-12) for a, b in zip(costs, costs[1:]))
