"""Pins of the CPU oracle's building blocks against what the paper and the
mathematics fix (no GPU).  Each test names the passage it checks."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GAMMA = 1.4
RNG = np.random.default_rng(20140222)


# ------------------------------------------------------------------ helpers
def poly_avgs(coef, edges):
    """Exact averages of sum coef[k] x^k over [edges[i], edges[i+1]]."""
    anti = np.polynomial.polynomial.polyint(coef)
    Q = np.polynomial.polynomial.polyval(edges, anti)
    return (Q[1:] - Q[:-1]) / np.diff(edges)


def euler_flux(U, nrm=1):
    ncomp = len(U)
    rho, E = U[0], U[-1]
    u = U[nrm] / rho
    m2 = sum(U[k] ** 2 for k in range(1, ncomp - 1))
    p = (GAMMA - 1) * (E - 0.5 * m2 / rho)
    F = np.array([U[k] * u for k in range(ncomp)], dtype=float)
    F[nrm] += p
    F[-1] = u * (E + p)
    return F


def rand_state(ncomp=3, rho=(0.1, 10), u=(-3, 3), p=(0.01, 10)):
    r = 10 ** RNG.uniform(math.log10(rho[0]), math.log10(rho[1]))
    vel = RNG.uniform(u[0], u[1], size=ncomp - 2)
    pr = 10 ** RNG.uniform(math.log10(p[0]), math.log10(p[1]))
    return np.array([r, *(r * vel), pr / (GAMMA - 1) + 0.5 * r * (vel ** 2).sum()])


def spec_e(U):
    m2 = sum(U[k] ** 2 for k in range(1, len(U) - 1))
    return U[-1] / U[0] - 0.5 * m2 / U[0] ** 2


# ------------------------------------------------------------ Sec 2.2 rows
def test_linear_rows_are_the_printed_fifth_order_schemes():
    """With omega = c, eq. (CWENO-FV) and its mirror must be eqs. (5th-order1)
    and (5th-order2): check the solved nodal values satisfy the printed rows."""
    n = 24
    u = RNG.normal(size=n)
    ue = np.concatenate([u[-3:], u, u[:3]])
    um, up = oracle.recon_scalar(ue, True, oracle.params(linear=True))
    im, ip = np.roll(np.arange(n), 1), np.roll(np.arange(n), -1)
    lhs = 3 / 10 * um[im] + 6 / 10 * um + 1 / 10 * um[ip]
    rhs = 1 / 30 * u[im] + 19 / 30 * u + 10 / 30 * u[ip]
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-14)
    # eq. (5th-order2) at node i-1/2 (up[i] is u+ at node i-1/2)
    lhs = 1 / 10 * up[im] + 6 / 10 * up + 3 / 10 * up[ip]
    rhs = 10 / 30 * u[im] + 19 / 30 * u + 1 / 30 * u[ip]
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_linear_reconstruction_exact_for_quartics(seed):
    """Sec 2.2: the linear compact schemes match Taylor terms up to K = 5, so
    they are exact for polynomials of degree <= 4; so is the explicit
    fifth-order closure with linear weights (non-periodic line)."""
    rng = np.random.default_rng(seed)
    coef = rng.normal(size=5)
    n, h = 17, 1.0 / 17
    edges = (np.arange(-3, n + 4)) * h
    ue = poly_avgs(coef, edges)
    um, up = oracle.recon_scalar(ue, False, oracle.params(linear=True))
    xr = (np.arange(n) + 1) * h
    xl = np.arange(n) * h
    scale = np.abs(ue).max()
    np.testing.assert_allclose(um, np.polynomial.polynomial.polyval(xr, coef), atol=1e-12 * scale)
    np.testing.assert_allclose(up, np.polynomial.polynomial.polyval(xl, coef), atol=1e-12 * scale)


@pytest.mark.parametrize("seed", range(5))
def test_nonlinear_reconstruction_exact_for_quadratics(seed):
    """Each candidate of eq. (candidates) is third order, so any convex
    combination (any omega) is exact for quadratics: the nonlinear rows,
    the closure and the solve must reproduce quadratic nodal values."""
    rng = np.random.default_rng(100 + seed)
    coef = rng.normal(size=3) * np.array([1.0, 5.0, 30.0])
    n, h = 23, 0.37
    edges = (np.arange(-3, n + 4)) * h - 2.0
    ue = poly_avgs(coef, edges)
    um, up = oracle.recon_scalar(ue, False, oracle.params())
    xr, xl = edges[4:n + 4], edges[3:n + 3]
    scale = np.abs(ue).max()
    np.testing.assert_allclose(um, np.polynomial.polynomial.polyval(xr, coef), atol=1e-12 * scale)
    np.testing.assert_allclose(up, np.polynomial.polynomial.polyval(xl, coef), atol=1e-12 * scale)


# ----------------------------------------------------------- eq. (weight)
def test_weights_uniform_data_are_linear_weights():
    wm, wp = oracle.weights(np.full(6, 3.7))
    assert list(wm) == [0.2, 0.5, 0.3] and list(wp) == [0.2, 0.5, 0.3]


def test_weights_pick_the_smooth_stencil_at_a_jump():
    """Near a discontinuity the weight of every stencil crossing it tends to
    0 (Sec 2.2, last paragraph): the system becomes bidiagonal there."""
    wm, wp = oracle.weights([0, 0, 0, 1, 1, 1])   # jump between cells j and j+1
    assert wm[0] > 1 - 1e-12 and wp[0] > 1 - 1e-12
    wm, _ = oracle.weights([0, 0, 1, 1, 1, 1])    # jump between cells j-1 and j
    assert wm[2] > 1 - 1e-12
    _, wp = oracle.weights([0, 0, 0, 0, 1, 1])    # jump between cells j+1 and j+2
    assert wp[2] > 1 - 1e-12


def test_weights_converge_to_linear_weights_fast():
    """WENO-Z with tau5 = O(h^5), beta = O(h^2) and power 2: omega - c is
    O(h^6) or smaller at smooth points (power 1 would only give O(h^3))."""
    x0, devs = 0.3, []
    for h in (0.1, 0.05):
        j = np.arange(-2, 4)
        v = (np.cos(x0 + j * h - h / 2) - np.cos(x0 + j * h + h / 2)) / h
        wm, wp = oracle.weights(v)
        devs.append((np.abs(wm - [0.2, 0.5, 0.3]).max(), np.abs(wp - [0.2, 0.5, 0.3]).max()))
    for side in (0, 1):
        assert math.log2(devs[0][side] / devs[1][side]) > 5.5


def test_weights_scale_invariant():
    v = RNG.normal(size=6)
    w1 = np.concatenate(oracle.weights(v))
    w2 = np.concatenate(oracle.weights(7.5 * v + 3.0))
    np.testing.assert_allclose(w1, w2, rtol=1e-10)


# ------------------------------------------------------- tridiagonal solves
def weno_rows(u, side):
    """Rows of eq. (CWENO-FV) built from oracle weights on periodic data."""
    n = len(u)
    a, b, c, r = (np.empty(n) for _ in range(4))
    for i in range(n):
        v = u[[(i + k) % n for k in range(-2, 4)]]
        wm, wp = oracle.weights(v)
        if side == "-":
            w = wm
            a[i], b[i], c[i] = (2 * w[0] + w[1]) / 3, (w[0] + 2 * (w[1] + w[2])) / 3, w[2] / 3
        else:
            w = wp
            a[i], b[i], c[i] = w[2] / 3, (w[0] + 2 * (w[1] + w[2])) / 3, (2 * w[0] + w[1]) / 3
        r[i] = RNG.normal()
    return a, b, c, r


def dense(a, b, c, cyclic):
    n = len(b)
    A = np.diag(b)
    for i in range(n):
        if i > 0 or cyclic:
            A[i, (i - 1) % n] += a[i]
        if i < n - 1 or cyclic:
            A[i, (i + 1) % n] += c[i]
    return A


@pytest.mark.parametrize("n", [3, 4, 5, 7, 8, 11, 16])
@pytest.mark.parametrize("kind", ["dominant", "weno-", "jumps-"])
def test_chasing_solves_match_pivoted_dense_lu(n, kind):
    """The paper's chasing method (Thomas, no pivoting; P. 2.3) and the cyclic
    variant agree with Gaussian elimination with partial pivoting, also on
    rows that are not diagonally dominant (omega0 > 1/2 next to jumps)."""
    if kind == "dominant":
        a, c = RNG.uniform(0, 1, n), RNG.uniform(0, 1, n)
        b = a + c + RNG.uniform(0.1, 1, n)
        r = RNG.normal(size=n)
    elif kind == "weno-":
        a, b, c, r = weno_rows(RNG.normal(size=n), "-")
    else:
        u = np.where(np.arange(n) < n // 2, 0.0, 1.0) + 1e-3 * RNG.normal(size=n)
        a, b, c, r = weno_rows(u, "-")
        assert np.any(b - a - c < 0) or n < 5
    x = oracle.thomas(a, b, c, r)
    xd = oracle.dense_solve(dense(a, b, c, False), r)
    np.testing.assert_allclose(x, xd, rtol=1e-12, atol=1e-12 * np.abs(xd).max())
    if n >= 3:
        x = oracle.cyclic(a, b, c, r)
        xd = oracle.dense_solve(dense(a, b, c, True), r)
        np.testing.assert_allclose(x, xd, rtol=1e-11, atol=1e-12 * np.abs(xd).max())


# -------------------------------------------------------------- HLLC flux
@pytest.mark.parametrize("ncomp,nrm", [(3, 1), (4, 1), (4, 2)])
def test_hllc_consistency(ncomp, nrm):
    """F(U, U) = f(U): the four branches of eq. (HLLC) all reduce to the
    physical flux of Sec. 1 for equal states."""
    for _ in range(50):
        U = rand_state(ncomp)
        np.testing.assert_allclose(oracle.hllc(U, U, nrm=nrm), euler_flux(U, nrm),
                                   rtol=1e-13, atol=1e-13 * np.abs(U).max())


def test_hllc_resolves_isolated_contacts_exactly():
    """Sec 2.4: the HLLC solver with these wave speeds resolves isolated
    contact waves exactly.  (With the printed rho_l in the right term of
    eq. (contact-v) a moving contact would not be exact.)"""
    for u0 in (0.0, 0.3, -0.7):
        for _ in range(10):
            rl, rr, p = 10 ** RNG.uniform(-2, 1, 2).tolist()[0], 10 ** RNG.uniform(-2, 1), 1.3
            Ul = np.array([rl, rl * u0, p / (GAMMA - 1) + 0.5 * rl * u0 ** 2])
            Ur = np.array([rr, rr * u0, p / (GAMMA - 1) + 0.5 * rr * u0 ** 2])
            F = oracle.hllc(Ul, Ur)
            if u0 == 0.0:
                np.testing.assert_allclose(F, [0.0, p, 0.0], atol=1e-14 * p)
            else:
                up = Ul if u0 > 0 else Ur
                np.testing.assert_allclose(F, euler_flux(up), rtol=1e-13, atol=1e-14)
            S = oracle.hllc_speeds(Ul, Ur)
            assert abs(S[1] - u0) < 1e-13


def test_hllc_supersonic_branches():
    Ul = np.array([1.0, 6.0, 1.0 / 0.4 + 18.0])
    Ur = np.array([0.5, 4.0, 0.7 / 0.4 + 16.0])
    assert np.array_equal(oracle.hllc(Ul, Ur), euler_flux(Ul))
    M = np.array([1.0, -1.0, 1.0])
    assert np.array_equal(oracle.hllc(Ur * M, Ul * M), euler_flux(Ul * M))


def test_hllc_mirror_covariance():
    M = np.array([1.0, -1.0, 1.0])
    for _ in range(50):
        Ul, Ur = rand_state(), rand_state()
        F = oracle.hllc(Ul, Ur)
        Fm = oracle.hllc(Ur * M, Ul * M)
        np.testing.assert_allclose(Fm, F * np.array([-1.0, 1.0, -1.0]), rtol=1e-12,
                                   atol=1e-12 * np.abs(F).max())


def test_hllc_wave_speeds_give_positive_star_states():
    """Eq. (inequ-v): S_L < S_M, S_L < u_l and the stronger bound
    S_L < u_l - sqrt((g-1)/(2g)) a_l derived for E*_l - rho* u*^2/2 > 0; the
    mirror statements hold on the right.  S_R is the max of its two
    candidates (the printed min would violate S_R > u_r)."""
    k = math.sqrt((GAMMA - 1) / (2 * GAMMA))
    for _ in range(300):
        Ul, Ur = rand_state(rho=(1e-4, 10), p=(1e-6, 10)), rand_state(rho=(1e-4, 10), p=(1e-6, 10))
        SL, SM, SR = oracle.hllc_speeds(Ul, Ur)
        ul, ur = Ul[1] / Ul[0], Ur[1] / Ur[0]
        al = math.sqrt(GAMMA * (GAMMA - 1) * (Ul[2] / Ul[0] - 0.5 * ul * ul))
        ar = math.sqrt(GAMMA * (GAMMA - 1) * (Ur[2] / Ur[0] - 0.5 * ur * ur))
        assert SL < SM < SR
        assert SL < ul - k * al and SR > ur + k * ar
        assert SR >= ur + ar - 1e-13 * (abs(ur) + ar)


# ------------------------------------------------ Lax-Friedrichs flux
@pytest.mark.parametrize("ncomp,nrm", [(3, 1), (4, 1), (4, 2)])
def test_lf_consistency(ncomp, nrm):
    """F(U, U) = f(U): the dissipation term vanishes for equal states."""
    for _ in range(50):
        U = rand_state(ncomp)
        np.testing.assert_allclose(oracle.lf(U, U, nrm=nrm), euler_flux(U, nrm),
                                   rtol=1e-13, atol=1e-13 * np.abs(U).max())


def test_lf_mirror_covariance_and_dissipation():
    """Mirror covariance as for HLLC; and the flux is more dissipative than
    HLLC: across an isolated stationary contact HLLC carries no mass, while
    Lax-Friedrichs carries -alpha (rho_r - rho_l) / 2 with alpha the larger
    sound speed of the two sides."""
    M = np.array([1.0, -1.0, 1.0])
    for _ in range(50):
        Ul, Ur = rand_state(), rand_state()
        F = oracle.lf(Ul, Ur)
        Fm = oracle.lf(Ur * M, Ul * M)
        np.testing.assert_allclose(Fm, F * np.array([-1.0, 1.0, -1.0]), rtol=1e-12,
                                   atol=1e-12 * np.abs(F).max())
    p = 1.3
    for rl, rr in ((1.0, 0.125), (0.2, 3.0)):
        Ul = np.array([rl, 0.0, p / (GAMMA - 1)])
        Ur = np.array([rr, 0.0, p / (GAMMA - 1)])
        alpha = max(math.sqrt(GAMMA * p / rl), math.sqrt(GAMMA * p / rr))
        F = oracle.lf(Ul, Ur)
        np.testing.assert_allclose(F, [-0.5 * alpha * (rr - rl), p, 0.0], rtol=1e-13, atol=1e-15)
        assert abs(oracle.hllc(Ul, Ur)[0]) < 1e-14


@pytest.mark.parametrize("seed", range(3))
def test_first_order_lf_scheme_preserves_positivity(seed):
    """The first-order scheme with the local Lax-Friedrichs flux keeps states
    in G at CFL 1/2 on random near-vacuum data (the flux is positivity
    preserving for lambda alpha <= 1)."""
    rng = np.random.default_rng(100 + seed)
    n = 200
    rho = 10 ** rng.uniform(-6, 0, n)
    u = rng.uniform(-5, 5, n)
    p = 10 ** rng.uniform(-10, 0, n)
    U = W.prim_to_cons_1d(rho, u, p, GAMMA)
    h = 1.0 / n
    dt = 0.5 * h / oracle.max_speed_1d(U)
    P = oracle.params(first_order=True, limiter=False, flux=1)
    for bc in ((0, 0), (1, 1), (2, 2)):
        U1 = oracle.stage_1d(U, U, 1, dt, bc, h, P)
        assert np.all(U1[0] > 0)
        assert np.all(W.specific_internal_energy(U1) > 0)


def test_lf_scheme_fifth_order_on_smooth_data():
    """With either flux the scheme stays fifth order on the smooth wave
    (Example 3.1, dt = w1 h^(5/3) / max(|u|+a)): the flux only sees the
    O(h^5) jump of the reconstructed interface values."""
    errs = []
    for n in (20, 40):
        U, info = oracle.run_1d(W.density_wave_1d(n), (0, 0), 2.0 / n, 2.0, rule=1,
                                p=oracle.params(flux=1))
        ex = W.density_wave_1d(n, t=info["t"])
        errs.append(W.error_norms(U[0], ex[0], 2.0 / n)[0])
    order = math.log2(errs[0] / errs[1])
    assert 4.5 < order < 6.5, (errs, order)


@pytest.mark.parametrize("seed", range(3))
def test_first_order_scheme_preserves_positivity(seed):
    """Special case U+- = cell averages: scheme (1DEulerFV-First) with HLLC
    keeps states in G at CFL 1/2 on random near-vacuum data."""
    rng = np.random.default_rng(seed)
    n = 200
    rho = 10 ** rng.uniform(-6, 0, n)
    u = rng.uniform(-5, 5, n)
    p = 10 ** rng.uniform(-10, 0, n)
    U = W.prim_to_cons_1d(rho, u, p, GAMMA)
    h = 1.0 / n
    dt = 0.5 * h / oracle.max_speed_1d(U)
    P = oracle.params(first_order=True, limiter=False)
    for bc in ((0, 0), (1, 1), (2, 2)):
        U1 = oracle.stage_1d(U, U, 1, dt, bc, h, P)
        assert np.all(U1[0] > 0)
        assert np.all(W.specific_internal_energy(U1) > 0)


# --------------------------------------------------------------- limiter
def test_limiter_bounds_and_structure():
    """Sec 2.4 limiter: after limiting rho >= eps at W1..W3 and e >= eps_e,
    density is scaled by theta1*theta2 and the other components by theta2
    toward the cell average."""
    w1 = 1.0 / 12.0
    er, ee = 1e-13, 1e-13
    n_active = 0
    for _ in range(400):
        Ub = rand_state(rho=(1e-3, 10), p=(1e-5, 10))
        Um = Ub + RNG.normal(size=3) * np.abs(Ub) * RNG.uniform(0, 3)
        Up = Ub + RNG.normal(size=3) * np.abs(Ub) * RNG.uniform(0, 3)
        Lm, Lp, act = oracle.limit_cell(Ub, Um, Up, er, ee, w1)
        n_active += act
        W3 = (Ub - w1 * Lp - w1 * Lm) / (1 - 2 * w1)
        for Wa in (Lm, Lp, W3):
            assert Wa[0] >= er * (1 - 1e-9) - 1e-15 * Ub[0]
            assert Wa[0] * Wa[2] - 0.5 * Wa[1] ** 2 - ee * Wa[0] ** 2 >= -1e-12 * Ub[0] * Ub[2]
        dm, dp = Um - Ub, Up - Ub
        th = [(Lm[k] - Ub[k]) / dm[k] for k in (1, 2) if abs(dm[k]) > 1e-8 * abs(Ub[k]) + 1e-300]
        if len(th) == 2:
            assert abs(th[0] - th[1]) < 1e-8
            thp = [(Lp[k] - Ub[k]) / dp[k] for k in (1, 2) if abs(dp[k]) > 1e-8 * abs(Ub[k])]
            if thp:
                assert abs(thp[0] - th[0]) < 1e-8
    assert n_active > 50


def _bisect_largest(ok, iters=200):
    """Largest t in [0, 1] with ok(t), for a predicate true at 0 that stays
    false once it turns false (bisection; no formula of the limiter used)."""
    if ok(1.0):
        return 1.0
    lo, hi = 0.0, 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if ok(mid):
            lo = mid
        else:
            hi = mid
    return lo


@pytest.mark.parametrize("seed", range(4))
def test_limiter_thetas_are_the_binding_scalings(seed):
    """Sec 2.4, steps 2 and 4, pinned by what theta1 and theta2 ARE rather
    than by their formulas: theta1 is the largest scaling toward the cell
    average that keeps the three Gauss-Lobatto densities (the two interface
    values and the interior value fixed by the quadrature mean) at or above
    eps; theta2 is the smallest over the three points of the largest t with
    e((1-t) Ubar + t W) >= eps_e, found here by bisection on e itself.  Also
    checks that when a theta is below 1 its constraint binds: the limited
    minimum density equals eps, the limited minimum e equals eps_e."""
    rng = np.random.default_rng(100 + seed)
    w1 = 1.0 / 12.0
    n_th1 = n_th2 = 0
    for _ in range(300):
        ncomp = 3 if rng.uniform() < 0.5 else 4
        r = 10 ** rng.uniform(-1, 1)
        vel = rng.uniform(-2, 2, size=ncomp - 2)
        pr = 10 ** rng.uniform(-1, 1)
        Ub = np.array([r, *(r * vel), pr / (GAMMA - 1) + 0.5 * r * (vel ** 2).sum()])
        # thresholds far above roundoff so "equals eps" is checkable
        er = Ub[0] * rng.uniform(0.05, 0.6)
        ee = spec_e(Ub) * rng.uniform(0.05, 0.6)
        scale = np.abs(Ub) + 0.3 * Ub[-1]
        Um = Ub + rng.normal(size=ncomp) * scale * rng.uniform(0.2, 1.5)
        Up = Ub + rng.normal(size=ncomp) * scale * rng.uniform(0.2, 1.5)
        Lm, Lp, _ = oracle.limit_cell(Ub, Um, Up, er, ee, w1)

        # --- independent reference
        def gl_mid(a, b):   # interior value fixed by the Gauss-Lobatto mean
            return (Ub - w1 * b - w1 * a) / (1 - 2 * w1)

        rho3 = np.array([Um[0], Up[0], gl_mid(Um, Up)[0]])
        th1 = _bisect_largest(lambda t: np.all(Ub[0] + t * (rho3 - Ub[0]) >= er))
        Hm, Hp = Um.copy(), Up.copy()
        Hm[0] = Ub[0] + th1 * (Um[0] - Ub[0])
        Hp[0] = Ub[0] + th1 * (Up[0] - Ub[0])
        ts = []
        for Wa in (Hm, Hp, gl_mid(Hm, Hp)):
            ts.append(_bisect_largest(lambda t: spec_e(Ub + t * (Wa - Ub)) >= ee))
        th2 = min(ts)
        Rm = Ub + th2 * (Hm - Ub)
        Rp = Ub + th2 * (Hp - Ub)
        tol = 1e-9 * (np.abs(Ub) + np.abs(Um) + np.abs(Up))
        assert np.all(np.abs(Lm - Rm) <= tol), (Lm, Rm, th1, th2)
        assert np.all(np.abs(Lp - Rp) <= tol), (Lp, Rp, th1, th2)
        # --- the constraint binds where a theta is below 1
        if th1 < 1.0 and th2 == 1.0:
            n_th1 += 1
            rmin = min(Lm[0], Lp[0], gl_mid(Lm, Lp)[0])
            assert abs(rmin - er) <= 1e-10 * Ub[0], (rmin, er)
        if th2 < 1.0:
            n_th2 += 1
            emin = min(spec_e(Lm), spec_e(Lp), spec_e(gl_mid(Lm, Lp)))
            assert abs(emin - ee) <= 1e-8 * spec_e(Ub), (emin, ee)
    assert n_th1 > 10 and n_th2 > 30, (n_th1, n_th2)


def test_limiter_is_exact_noop_on_positive_states():
    w1 = 1.0 / 12.0
    for _ in range(100):
        Ub = rand_state()
        # rescaling a state leaves e unchanged, so these stay well inside G
        Um = Ub * (1 + 0.05 * RNG.normal())
        Up = Ub * (1 + 0.05 * RNG.normal())
        Lm, Lp, act = oracle.limit_cell(Ub, Um, Up, 1e-13, 1e-13, w1)
        assert not act and np.array_equal(Lm, Um) and np.array_equal(Lp, Up)


# ------------------------------------------------------------ eq. (RK3)
def test_rk3_stability_polynomial():
    """On L(U) = lam U one step of eq. (RK3) multiplies by 1 + z + z^2/2 + z^3/6."""
    for z in (-0.3, 0.1, -1.7, 0.9):
        lam, dt = z, 1.0
        U0 = np.array([1.0])
        U1 = oracle.rk3_combine(1, dt, U0, U0, lam * U0)
        U2 = oracle.rk3_combine(2, dt, U0, U1, lam * U1)
        U3 = oracle.rk3_combine(3, dt, U0, U2, lam * U2)
        assert abs(U3[0] - (1 + z + z * z / 2 + z ** 3 / 6)) < 1e-15


# ---------------------------------------------------------- whole operator
@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (2, 2), (1, 2)])
def test_free_stream_preserved(bc):
    u = 0.0 if 2 in bc else 0.4
    n = 40
    U = W.prim_to_cons_1d(np.full(n, 1.3), np.full(n, u), np.full(n, 2.0), GAMMA)
    L = oracle.rhs_1d(U, bc, h=0.01)
    F = euler_flux(U[:, 0])
    assert np.abs(L).max() * 0.01 <= 1e-14 * np.abs(F).max()


def test_periodic_conservation():
    """Eq. (1DEulerFV-b) telescopes: with periodic boundaries the totals of
    all conserved variables are constant to roundoff."""
    n = 64
    x = W.cell_centres(0, 1, n)
    rho = np.where((x > 0.3) & (x < 0.6), 1.0, 0.125) + 0.1 * np.sin(6 * np.pi * x)
    U = W.prim_to_cons_1d(rho, 0.5 + 0.3 * np.cos(2 * np.pi * x), np.where(x < 0.5, 1.0, 0.1), GAMMA)
    U2, info = oracle.run_1d(U, (0, 0), 1.0 / n, 10.0, max_steps=40)
    assert info["steps"] == 40
    np.testing.assert_allclose(U2.sum(axis=1), U.sum(axis=1), rtol=1e-13)


@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (2, 2), (1, 2)])
def test_mirror_symmetry_of_a_reversed_line(bc):
    """The "+" side is the mirror of the "-" side: reversing a line (and
    the sign of its momentum and of its boundary roles) mirrors L."""
    n = 50
    x = W.cell_centres(0, 1, n)
    rho = 1 + 0.5 * (x > 0.4) + 0.2 * np.sin(5 * x)
    U = W.prim_to_cons_1d(rho, np.sin(3 * x), 1 + (x < 0.7), GAMMA)
    M = np.array([1.0, -1.0, 1.0])[:, None]
    L = oracle.rhs_1d(U, bc, h=1.0 / n)
    Lr = oracle.rhs_1d(U[:, ::-1] * M, bc[::-1], h=1.0 / n)
    np.testing.assert_allclose(Lr[:, ::-1] * M, L, atol=1e-12 * np.abs(L).max())


# ------------------------------------------------- suite input generators
def test_suite_generators_integrate_the_printed_data():
    """Exact cell averages: the totals equal the integrals of the paper's
    piecewise data (Examples 3.2-3.10), so the inputs carry no quadrature
    error into the GPU suite runs."""
    import math
    g = 1.4
    # Lax on [-5, 5]
    U = W.lax_1d(200)
    h = 10.0 / 200
    assert abs(U[0].sum() * h - (0.445 * 5 + 0.5 * 5)) < 1e-12
    assert abs(U[1].sum() * h - 0.445 * 0.698 * 5) < 1e-12
    # Sod (classical data, see the generator's note)
    U = W.sod_1d(100)
    assert abs(U[2].sum() * 0.1 - (1.0 / (g - 1) * 5 + 0.1 / (g - 1) * 5)) < 1e-12
    # Shu-Osher: the sine integrates in closed form
    U = W.shu_osher_1d(200)
    h = 10.0 / 200
    mass = 3.857143 * 1.0 + 9.0 + 0.2 * (math.cos(-20.0) - math.cos(25.0)) / 5.0
    assert abs(U[0].sum() * h - mass) < 1e-12
    # a cell that straddles x = -4 (n = 190: edges at -5 + k/19) mixes both pieces
    U = W.shu_osher_1d(190)
    assert np.all(np.isfinite(U)) and U[1].max() <= 3.857143 * 2.629369 + 1e-12
    # LeBlanc: p = (gamma - 1) rho e with gamma = 5/3
    U = W.leblanc_1d(400)
    assert abs(U[2][0] - (1.0 * 0.1)) < 1e-15 and abs(U[2][-1] - 1e-3 * 1e-7) < 1e-22
    # Woodward-Colella: total energy of the three pressure slabs
    U = W.woodward_colella_1d(200)
    assert abs(U[2].sum() / 200 - (1000 * 0.1 + 0.01 * 0.8 + 100 * 0.1) / (g - 1)) < 1e-9


# --------------------------------------- explicit WENO-JS / WENO-Z (Sec. 3)
def _explicit_avgs(n, antideriv, a=0.0, b=2.0):
    """Exact averages of cells -3..n+2 from an antiderivative."""
    h = (b - a) / n
    e = a + np.arange(-3, n + 4) * h
    F = antideriv(e)
    return (F[1:] - F[:-1]) / h, h, e


@pytest.mark.parametrize("kind", [1, 2])
def test_explicit_weno_reproduces_quadratics(kind):
    """Each candidate of the explicit reconstruction is exact for quadratics,
    so any convex weighting is: face values of 1 + 2x - 3x^2 from its exact
    averages, both sides, to rounding."""
    n = 12
    ue, h, e = _explicit_avgs(n, lambda x: x + x ** 2 - x ** 3)
    um, up = oracle.recon_scalar(ue, False, oracle.params(recon=kind))
    q = lambda x: 1 + 2 * x - 3 * x ** 2
    np.testing.assert_allclose(um, q(e[4:4 + n]), rtol=0, atol=1e-12)
    np.testing.assert_allclose(up, q(e[3:3 + n]), rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind,linear", [(1, True), (1, False), (2, False)])
def test_explicit_weno_fifth_order(kind, linear):
    """Face values of sin(pi x) from exact averages converge at fifth order
    (measured orders 4.97-5.00 for N = 20..160), with the linear weights
    (0.1, 0.6, 0.3) and with either nonlinear weight rule."""
    errs = []
    for n in (20, 40, 80):
        ue, h, e = _explicit_avgs(n, lambda x: -np.cos(np.pi * x) / np.pi)
        um, up = oracle.recon_scalar(ue, False, oracle.params(recon=kind, linear=linear))
        errs.append(max(np.abs(um - np.sin(np.pi * e[4:4 + n])).max(),
                        np.abs(up - np.sin(np.pi * e[3:3 + n])).max()))
    for a, b in zip(errs[:-1], errs[1:]):
        assert 4.8 < np.log2(a / b) < 5.2, errs


@pytest.mark.parametrize("kind,tol", [(1, 1e-10), (2, 1e-20)])
def test_explicit_weno_is_essentially_non_oscillatory(kind, tol):
    """At a unit step the nonlinear weights pick the candidate that does not
    cross it: the face of the jump sees 0 from the left and 1 from the right
    (the linear weights give 0.4 there instead, a mistake in the weights
    fails this)."""
    n = 20
    ue = np.zeros(n + 6)
    ue[3 + 10:] = 1.0
    um, up = oracle.recon_scalar(ue, False, oracle.params(recon=kind))
    assert abs(um[9]) < tol and abs(up[10] - 1.0) < tol
    lm, _ = oracle.recon_scalar(ue, False, oracle.params(recon=kind, linear=True))
    assert abs(lm[9] - 0.4) < 1e-14


def test_explicit_weno_js_matches_table2_column():
    """Table 2's WENO-JS columns (Example 3.1, lambda max(|u|+a) = 0.16,
    t = 2), run by the oracle's explicit WENO-JS scheme with the same HLLC
    flux and SSP-RK3: L1 and Linf within 2 % of the printed values at
    N = 15, 30, 60 (measured 1.000-1.010; at N = 120 the time error adds 4 %)."""
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "table2_wenojs_conservative.json")) as f:
        rows = {r[0]: r for r in json.load(f)["rows"]}
    for n in (15, 30, 60):
        U0 = W.density_wave_1d(n)
        U, info = oracle.run_1d(U0, (0, 0), 2.0 / n, 2.0, cfl=0.16, rule=0,
                                p=oracle.params(recon=1))
        assert abs(info["t"] - 2.0) < 1e-12
        l1, l2, linf = W.error_norms(U[0], W.density_wave_1d(n, t=info["t"])[0], 2.0 / n)
        assert abs(l1 / rows[n][1] - 1) < 0.02, (n, l1, rows[n][1])
        assert abs(linf / rows[n][2] - 1) < 0.02, (n, linf, rows[n][2])


# ------------------------------------------- Sec 2.3: characteristic fields
def _jacobian_printed(u, e_rho, g=GAMMA):
    """The Jacobian A(U) of Sec. 2.3, in terms of u2/u1 = u and u3/u1 = E/rho.
    The printed (2,1) entry reads -(gamma-3)/2 u^2; the derivative of
    rho u^2 + p with respect to rho is +(gamma-3)/2 u^2, and only that sign
    gives the eigenvalues u - a, u, u + a the text states (reading R28)."""
    return np.array([
        [0.0, 1.0, 0.0],
        [0.5 * (g - 3) * u * u, (3 - g) * u, g - 1],
        [-g * u * e_rho + (g - 1) * u ** 3, g * e_rho - 1.5 * (g - 1) * u * u, g * u],
    ])


@pytest.mark.parametrize("seed", range(3))
def test_char_eigenvectors_diagonalise_the_jacobian(seed):
    """L R = I; L A R = diag(u - a, u, u + a) with A the Jacobian of Sec. 2.3
    at the Roe state (its printed (2,1) sign corrected); and Roe's defining
    property R Lambda L (Ub - Ua) = F(Ub) - F(Ua), which fixes the averaged
    state itself."""
    for _ in range(50 + seed):
        Ua = rand_state()
        Ub = rand_state()
        L, R, lam = oracle.char_eigen(Ua, Ub)
        np.testing.assert_allclose(L @ R, np.eye(3), atol=1e-12)
        u = lam[1]
        a = 0.5 * (lam[2] - lam[0])
        H = R[2, 2] - u * a          # r^(3) = (1, u + a, H + u a)
        e_rho = (H + 0.5 * (GAMMA - 1) * u * u) / GAMMA   # E/rho of the state with (u, H)
        A = _jacobian_printed(u, e_rho)
        D = L @ A @ R
        scale = np.abs(lam).max()
        np.testing.assert_allclose(D, np.diag([u - a, u, u + a]), atol=1e-12 * scale)
        dF = euler_flux(Ub) - euler_flux(Ua)
        np.testing.assert_allclose(R @ np.diag(lam) @ L @ (Ub - Ua), dF,
                                   atol=1e-11 * np.abs(dF).max() + 1e-14)


@pytest.mark.parametrize("n,cyclic", [(1, False), (2, False), (3, False), (7, False), (12, False),
                                      (3, True), (4, True), (9, True)])
def test_block_chasing_matches_dense_solve(n, cyclic):
    """The block chasing of (1DEuler-FVC) (and its cyclic form) against a
    dense solve of the assembled 3n x 3n system."""
    rng = np.random.default_rng(n + 10 * cyclic)
    A = rng.normal(size=(n, 3, 3))
    C = rng.normal(size=(n, 3, 3))
    B = rng.normal(size=(n, 3, 3)) + 8 * np.eye(3)
    Y = rng.normal(size=(n, 3))
    X = oracle.block_solve(A, B, C, Y, cyclic)
    M = np.zeros((3 * n, 3 * n))
    for i in range(n):
        M[3 * i:3 * i + 3, 3 * i:3 * i + 3] += B[i]
        for blk, j in ((A[i], i - 1), (C[i], i + 1)):
            if cyclic:
                j %= n
            elif not 0 <= j < n:
                continue
            M[3 * i:3 * i + 3, 3 * j:3 * j + 3] += blk
    ref = oracle.dense_solve(M, Y.reshape(-1)).reshape(n, 3)
    np.testing.assert_allclose(X, ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("seed", range(3))
def test_char_reconstruction_exact_for_quadratics(seed):
    """Every row of (1DEuler-FVC) is a characteristic combination of the
    scalar rows of eq. (CWENO-FV), each exact for quadratics with any
    weights, so the exact nodal values of quadratic conserved variables
    solve the block system: the characteristic reconstruction (nonlinear
    weights, node-dependent eigenvectors) reproduces them."""
    rng = np.random.default_rng(400 + seed)
    n, h = 23, 0.05
    edges = (np.arange(-3, n + 4)) * h
    coef = [np.array([1.0, 0.3, 0.5]) * rng.uniform(0.5, 1.5, 3),      # rho > 0
            rng.normal(size=3) * 0.3,                                  # rho u
            np.array([4.0, 0.5, 1.0]) * rng.uniform(0.5, 1.5, 3)]      # E: p > 0
    ue = np.array([poly_avgs(c, edges) for c in coef])
    um, up = oracle.recon_char(ue, False)
    xr, xl = edges[4:n + 4], edges[3:n + 3]
    for c in range(3):
        scale = np.abs(ue[c]).max()
        np.testing.assert_allclose(um[c], np.polynomial.polynomial.polyval(xr, coef[c]),
                                   atol=1e-11 * scale)
        np.testing.assert_allclose(up[c], np.polynomial.polynomial.polyval(xl, coef[c]),
                                   atol=1e-11 * scale)


def test_char_reconstruction_of_the_density_wave_equals_componentwise():
    """Table 3 prints the same FVCW errors as Table 2: for the density wave
    (u, p constant) the conserved variables are affine in rho, two
    characteristic fields are constant and the component-wise nodal values
    solve the block system, so the two reconstructions agree to roundoff."""
    n = 40
    U = W.density_wave_1d(n)
    ue = np.concatenate([U[:, -3:], U, U[:, :3]], axis=1)
    um_c, up_c = oracle.recon_char(ue, True)
    for c in range(3):
        um, up = oracle.recon_scalar(ue[c], True)
        np.testing.assert_allclose(um_c[c], um, rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(up_c[c], up, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("cyclic", [True, False])
def test_char_reconstruction_mirror_symmetry(cyclic):
    """Reversing a line and negating its momentum mirrors it: the "-" values
    of the mirrored line are the mirrored "+" values of the line.  Ties the
    "-" rows (node i+1/2, Roe average of cells i, i+1) to the "+" rows (node
    i-1/2, Roe average of cells i-1, i)."""
    n = 30
    x = W.cell_centres(0.0, 1.0, n)
    U = W.prim_to_cons_1d(1 + 0.4 * (x > 0.4) + 0.1 * np.sin(5 * x), 0.3 * np.cos(3 * x),
                          1 + 0.6 * (x < 0.7), GAMMA)
    ue = np.concatenate([U[:, -3:], U, U[:, :3]], axis=1) if cyclic else \
        np.concatenate([np.repeat(U[:, :1], 3, 1), U, np.repeat(U[:, -1:], 3, 1)], axis=1)
    um, up = oracle.recon_char(ue, cyclic)
    flip = np.array([1.0, -1.0, 1.0])[:, None]
    um_r, up_r = oracle.recon_char(flip * ue[:, ::-1], cyclic)
    scale = np.abs(U).max()
    np.testing.assert_allclose(flip * um_r[:, ::-1], up, atol=1e-12 * scale)
    np.testing.assert_allclose(flip * up_r[:, ::-1], um, atol=1e-12 * scale)
