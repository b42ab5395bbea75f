"""Whole-scheme pins of the CPU oracle: convergence against Tables 1-2,
conservation, positivity on the paper's near-vacuum suite, and the 2D
dimension-by-dimension extension (no GPU)."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def golden(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def density_wave_errors(n, cfl, rule, p=None):
    U0 = W.density_wave_1d(n)
    U, info = oracle.run_1d(U0, (0, 0), 2.0 / n, 2.0, cfl=cfl, rule=rule, p=p)
    assert abs(info["t"] - 2.0) < 1e-12 and info["limited"] == 0
    ex = W.density_wave_1d(n, t=info["t"])
    return W.error_norms(U[0], ex[0], 2.0 / n)


# ---------------------------------------------------------- Table 1 / Table 2
def _table1(ns):
    rows = {r[0]: r for r in golden("table1_density_wave.json")["rows"]}
    errs = {n: density_wave_errors(n, 1.0 / 12.0, 1) for n in ns}
    for a, b in zip(ns[:-1], ns[1:]):
        order = math.log2(errs[a][0] / errs[b][0])
        assert 4.5 < order < 6.2, (a, b, order)
    for n in ns:
        l1, l2 = errs[n][0], errs[n][1]
        # magnitudes: within the band the reproduction reaches (0.5x-0.9x of
        # the printed values; see the design notes on Table 1)
        assert 0.4 < l1 / rows[n][1] < 2.5, (n, l1, rows[n][1])
        assert 0.4 < l2 / rows[n][5] < 2.5, (n, l2, rows[n][5])


def test_table1_fifth_order_convergence():
    """Table 1: dt = w1 h^(5/3) / max(|u|+a), t = 2; L1 orders near 5 and
    magnitudes in the printed range.  (Its Linf column is unpinned.)"""
    _table1([10, 20, 40, 80])


@pytest.mark.slow
def test_table1_fine_grids():
    _table1([80, 160, 320])


def _table2(ns, band, band_inf=None):
    rows = {r[0]: r for r in golden("table2_fvcw_conservative.json")["rows"]}
    band_inf = band_inf or band
    for n in ns:
        l1, l2, linf = density_wave_errors(n, 0.16, 0)
        assert band[0] < l1 / rows[n][1] < band[1], (n, l1, rows[n][1])
        assert band[0] < l2 / rows[n][3] < band[1], (n, l2, rows[n][3])
        assert band_inf[0] < linf / rows[n][2] < band_inf[1], (n, linf, rows[n][2])


def test_table2_coarse_grids():
    """Table 2 (conservative-variable FVCW, lambda max(|u|+a) = 0.16) at
    N = 7, 14, 28.  No reading of the scheme reproduces the printed errors
    to 10 %: the scheme as printed, with the time error removed (a 10x
    smaller dt), gives 0.69, 0.68, 0.74 of them, and the candidate readings
    studied (weight exponent 1, Jiang-Shu weights, swapped indicators,
    point-value data, epsilon 1e-6, mean-|e| norm) do not close the gap at
    every N.  The band is that finding, not a fit: 0.6x-0.9x for L1 and L2;
    Linf, one cell's error on these grids, 0.5x-1.0x."""
    _table2([7, 14, 28], (0.6, 0.9), (0.5, 1.0))


def test_table2_coarse_grid_error_reduction_factor():
    """The factor by which L1 drops from N = 7 to N = 14 in Table 2 (48.3)
    is insensitive to an overall error constant and sensitive to the
    nonlinear weights: the WENO-Z weights of eq. (weight) with exponent 2
    reproduce it within 3 %, linear weights miss it by a third."""
    rows = {r[0]: r for r in golden("table2_fvcw_conservative.json")["rows"]}
    printed = rows[7][1] / rows[14][1]
    got = density_wave_errors(7, 0.16, 0)[0] / density_wave_errors(14, 0.16, 0)[0]
    assert abs(got / printed - 1) < 0.03, (got, printed)
    lin = oracle.params(linear=True)
    got_lin = density_wave_errors(7, 0.16, 0, lin)[0] / density_wave_errors(14, 0.16, 0, lin)[0]
    assert got_lin / printed < 0.8, (got_lin, printed)


@pytest.mark.slow
def test_table2_fine_grids_time_error():
    """At N >= 56 the RK3 error at CFL 0.16 exceeds the printed spatial
    error (ratio 1.3 at N = 56, 2.7 at N = 112): recorded, loosely bounded.
    With the time error removed the ratio stays at 0.76-0.81."""
    _table2([56, 112, 224], (0.5, 6.0))


# -------------------------------------------------------------- positivity
def run_case(U, bc, h, T, gamma=1.4, max_steps=1 << 40):
    Uf, info = oracle.run_1d(U, bc, h, T, p=oracle.params(gamma=gamma), max_steps=max_steps)
    assert np.all(np.isfinite(Uf))
    return Uf, info


def test_double_rarefaction_stays_positive():
    """Example 3.8 (h = 0.005): density and pressure stay positive after
    every step; printed minima are soft references only (characteristic
    reconstruction in the paper)."""
    Uf, info = run_case(W.double_rarefaction_1d(400), (1, 1), 0.005, 0.6)
    assert info["min_rho"] > 0 and info["min_p"] > 0 and info["limited"] > 0
    g = golden("positivity_minima.json")["cases"]["double_rarefaction"]
    assert 1e-3 < Uf[0].min() / g["min_rho"] < 1e3


def test_strong_shock_minima():
    """Example 3.7: printed min rho 1.250E-01 and min e 2.000E+00."""
    U = W.riemann_1d(0.0, 1.0, 200, 0.5, (1.0, 0.0, 1e10), (0.125, 0.0, 0.1))
    Uf, info = run_case(U, (1, 1), 1.0 / 200, 2.5e-6)
    g = golden("positivity_minima.json")["cases"]["strong_shock"]
    assert abs(Uf[0].min() / g["min_rho"] - 1) < 0.02
    assert abs(W.specific_internal_energy(Uf).min() / g["min_e"] - 1) < 0.02


def test_low_density_123_problem():
    """Example 3.6 (h = 0.0025): positive, minima near the printed ones."""
    U = W.riemann_1d(0.0, 1.0, 400, 0.5, (1.0, -2.0, 0.4), (1.0, 2.0, 0.4))
    Uf, info = run_case(U, (1, 1), 1.0 / 400, 0.1)
    assert info["min_rho"] > 0 and info["min_p"] > 0
    g = golden("positivity_minima.json")["cases"]["low_density_123"]
    assert 0.5 < Uf[0].min() / g["min_rho"] < 2.0
    assert 0.5 < W.specific_internal_energy(Uf).min() / g["min_e"] < 2.0


def test_leblanc_minima():
    """Example 3.10 (gamma = 5/3, N = 400, t = 6): printed minima 1.000E-03
    and 1.000E-07 are the right state's density and specific internal energy."""
    g = 5.0 / 3.0
    U = W.piecewise_1d(0.0, 9.0, 400, [(0, 3, 1.0, 0.0, (g - 1) * 1.0 * 0.1),
                                       (3, 9, 1e-3, 0.0, (g - 1) * 1e-3 * 1e-7)], g)
    Uf, info = run_case(U, (1, 1), 9.0 / 400, 6.0, gamma=g)
    gold = golden("positivity_minima.json")["cases"]["leblanc"]
    assert abs(Uf[0].min() / gold["min_rho"] - 1) < 0.01
    assert abs(W.specific_internal_energy(Uf).min() / gold["min_p"] - 1) < 0.01


def test_woodward_colella_reflective_walls():
    """Example 3.5: reflective walls carry no mass or energy flux (S_M = 0 by
    symmetry), so total mass and energy are conserved up to accumulated
    roundoff over ~3700 steps."""
    U = W.piecewise_1d(0.0, 1.0, 200, [(0, 0.1, 1, 0, 1000), (0.1, 0.9, 1, 0, 0.01),
                                       (0.9, 1.0, 1, 0, 100)])
    Uf, info = run_case(U, (2, 2), 0.005, 0.038)
    assert info["min_rho"] > 0 and info["min_p"] > 0
    np.testing.assert_allclose(Uf[0].sum(), U[0].sum(), rtol=1e-12)
    np.testing.assert_allclose(Uf[2].sum(), U[2].sum(), rtol=1e-12)


def test_vacuum_blast_early_steps_positive():
    """Near-vacuum blast (p = 1e-10 background, 4e3 in the two centre
    cells): the first 30 steps keep rho and p positive with the limiter
    active."""
    Uf, info = run_case(W.vacuum_blast_1d(4000), (1, 1), 2.0 / 4000, 1e-3, max_steps=30)
    assert info["min_rho"] > 0 and info["min_p"] > 0 and info["limited"] > 0


@pytest.mark.slow
def test_vacuum_blast_full_run():
    """Whole run to t = 1e-3: finite, final density positive and the
    background internal energy kept (transient negative pressures in a few
    steps near the evacuated centre are a known property of the
    component-wise form; see the design notes)."""
    Uf, info = run_case(W.vacuum_blast_1d(4000), (1, 1), 2.0 / 4000, 1e-3)
    assert abs(info["t"] - 1e-3) < 1e-15 and Uf[0].min() > 0
    assert W.specific_internal_energy(Uf).min() > 0.99 * 2.5e-10


def _speed(U, gamma=1.4):
    """|u| + a of each column of a [3][n] array (pressure floored at 0)."""
    r, u = U[0], U[1] / U[0]
    p = (gamma - 1) * (U[2] - 0.5 * r * u * u)
    return np.abs(u) + np.sqrt(gamma * np.maximum(p, 0.0) / r)


def test_interface_state_speed_bound():
    """The norm of condition (CFL-CD) under the interface-state rule is the
    largest |u|+a over the cell averages and the limited interface states
    the operator passes to the flux, recomputed here from the line's
    intermediate arrays."""
    U, _ = oracle.run_1d(W.vacuum_blast_1d(400), (1, 1), 2.0 / 400, 1.0, max_steps=8)
    L, dbg = oracle.line_op(U, 1, 1, 2.0 / 400, debug=True)
    ref = max(_speed(U).max(), _speed(dbg["um_l"]).max(), _speed(dbg["up_l"]).max())
    _, s = oracle.rhs_speed_1d(U, (1, 1), 2.0 / 400)
    assert s == pytest.approx(ref, rel=1e-15) and s == dbg["smax"]
    assert s > _speed(U).max()   # the limited states are faster than the averages here


def test_interface_state_rule_first_step_and_positivity():
    """Rule DT_PP: the first step is cfl h / S with S the bound above; the
    blast keeps every step in G for 200 steps, and later stages whose input
    breaks the bound are counted."""
    n, h = 4000, 2.0 / 4000
    U0 = W.vacuum_blast_1d(n)
    _, s = oracle.rhs_speed_1d(U0, (1, 1), h)
    _, one = oracle.run_1d(U0, (1, 1), h, 1.0, rule=oracle.DT_PP, max_steps=1)
    assert one["t"] == (1.0 / 12.0) * h / s
    _, info = oracle.run_1d(U0, (1, 1), h, 1.0, rule=oracle.DT_PP, max_steps=200)
    assert info["min_rho"] > 0 and info["min_p"] > 0 and info["viol"] > 0
    assert info["out_of_G"] == 0


def test_restart_rule_redoes_a_step_at_half_dt():
    """Rule DT_RESTART: a step that was redone k times equals one step of
    the averages' rule at cfl / 2^k (halving is exact), whose stage outputs
    all lie in G, while the step at cfl / 2^(k-1) has a stage output outside
    G.  On the blast the rule keeps every step in G where the averages' rule
    leaves it."""
    n, h = 4000, 2.0 / 4000
    U, t = W.vacuum_blast_1d(n), 0.0
    found = False
    for _ in range(200):
        Un, info = oracle.run_1d(U, (1, 1), h, 1.0, rule=oracle.DT_RESTART, max_steps=1)
        k = info["restarts"]
        if k > 0:
            cfl = (1.0 / 12.0) / 2 ** k
            ref, i0 = oracle.run_1d(U, (1, 1), h, 1.0, cfl=cfl, rule=oracle.DT_CFL, max_steps=1)
            assert np.array_equal(ref, Un) and i0["t"] == info["t"] and i0["out_of_G"] == 0
            _, i1 = oracle.run_1d(U, (1, 1), h, 1.0, cfl=2 * cfl, rule=oracle.DT_CFL, max_steps=1)
            assert i1["out_of_G"] > 0
            found = True
            break
        U = Un
    assert found
    _, r0 = oracle.run_1d(W.vacuum_blast_1d(n), (1, 1), h, 1.0, max_steps=60)
    _, r3 = oracle.run_1d(W.vacuum_blast_1d(n), (1, 1), h, 1.0, rule=oracle.DT_RESTART,
                          max_steps=60)
    assert r0["out_of_G"] > 0 and r0["min_p"] < 0
    assert r3["out_of_G"] == 0 and r3["min_p"] > 0 and r3["restarts"] > 0


@pytest.mark.slow
def test_restart_rule_blast_full_run():
    """The blast to t = 1e-3 under DT_RESTART: t_end reached, every stage
    output kept in G (2208 steps, 1018 redone)."""
    Uf, info = oracle.run_1d(W.vacuum_blast_1d(4000), (1, 1), 2.0 / 4000, 1e-3,
                             rule=oracle.DT_RESTART)
    assert info["t"] == 1e-3 and info["out_of_G"] == 0 and info["min_p"] > 0


@pytest.mark.slow
def test_planar_sedov_final_minima():
    """Example 3.9 (h = 0.005, t = 0.001): printed minima 4.731E-03 (rho) and
    1.000E-12 (e)."""
    Uf, info = run_case(W.sedov_planar_1d(0.005), (1, 1), 0.005, 1e-3)
    g = golden("positivity_minima.json")["cases"]["planar_sedov"]
    assert 0.5 < Uf[0].min() / g["min_rho"] < 2.0
    assert abs(W.specific_internal_energy(Uf).min() / g["min_e"] - 1) < 0.01


@pytest.mark.slow
def test_double_rarefaction_n4000():
    Uf, info = run_case(W.double_rarefaction_1d(4000), (1, 1), 2.0 / 4000, 0.6)
    assert info["min_rho"] > 0 and info["min_p"] > 0


# ---------------------------------------------------------------------- 2D
def test_2d_x_only_data_reduces_to_1d():
    """Dimension-by-dimension: data that vary only in x give the 1D
    operator on (rho, rho u, E) and no change of rho v."""
    nx, ny = 40, 5
    x = W.cell_centres(0, 1, nx)
    U1 = W.prim_to_cons_1d(1 + 0.5 * (x > 0.5), 0.3 * np.sin(2 * np.pi * x), 1 + 0.5 * np.cos(3 * x),
                           1.4)
    U2 = np.zeros((4, ny, nx))
    U2[0], U2[1], U2[3] = U1[0], U1[1], U1[2]
    for bc in ((0, 0, 0, 0), (1, 2, 0, 0), (2, 1, 1, 1)):
        L2 = oracle.rhs_2d(U2, bc, dx=1.0 / nx, dy=0.1)
        L1 = oracle.line_op(U1, bc[0], bc[1], 1.0 / nx, eps_rho=1e-13, eps_e=1e-13)
        for k2, k1 in ((0, 0), (1, 1), (3, 2)):
            np.testing.assert_allclose(L2[k2], np.broadcast_to(L1[k1], (ny, nx)),
                                       atol=1e-11 * np.abs(L1[k1]).max())
        assert np.abs(L2[2]).max() <= 1e-11 * np.abs(L1).max()


def test_2d_interface_state_rule_reduces_to_1d():
    """The 2D interface-state rule on data varying only in x takes the 1D
    rule's steps (the y-lines are uniform, so S_y is the averages' sound
    speed and the x-term is the 1D bound)."""
    nx, ny = 64, 4
    x = W.cell_centres(0, 1, nx)
    U1 = W.prim_to_cons_1d(1 + 0.5 * (x > 0.5), 0.2 * np.ones(nx), 1 + 0.5 * (x < 0.3), 1.4)
    U2 = np.zeros((4, ny, nx))
    U2[0], U2[1], U2[3] = U1[0], U1[1], U1[2]
    dx, dy = 1.0 / nx, 1e14   # dy large: the y-term of the step bound is negligible
    _, s2 = oracle.rhs_speed_2d(U2, (1, 1, 0, 0), dx, dy)
    _, s1 = oracle.rhs_speed_1d(U1, (1, 1), dx)
    assert s2[0] == pytest.approx(s1, rel=1e-14)
    R2, i2 = oracle.run_2d(U2, (1, 1, 0, 0), dx, dy, 1.0, max_steps=5, rule=oracle.DT_PP)
    R1, i1 = oracle.run_1d(U1, (1, 1), dx, 1.0, rule=oracle.DT_PP, max_steps=5)
    assert i2["t"] == pytest.approx(i1["t"], rel=1e-12)
    np.testing.assert_allclose(R2[0], np.broadcast_to(R1[0], (ny, nx)), rtol=1e-11)


def test_2d_sedov_is_symmetric_and_positive():
    """Quarter-plane blast with reflective x=0, y=0 walls: the solution is
    symmetric under x <-> y (with rho u <-> rho v) and stays positive."""
    n = 24
    U0 = W.sedov_corner_2d(n)
    dx = 1.1 / n
    U, info = oracle.run_2d(U0, (2, 1, 2, 1), dx, dx, 1.0, max_steps=12)
    assert info["min_rho"] > 0 and info["min_p"] > 0
    np.testing.assert_allclose(U[0], U[0].T, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(U[1], U[2].T, rtol=1e-12, atol=1e-12 * np.abs(U[1]).max())
    np.testing.assert_allclose(U[3], U[3].T, rtol=1e-12, atol=1e-14)


def test_2d_density_wave_convergence_and_conservation():
    errs = []
    for n in (16, 32):
        U0 = W.density_wave_2d(n, n)
        U, info = oracle.run_2d(U0, (0, 0, 0, 0), 2.0 / n, 2.0 / n, 0.25, cfl=0.5 / 12)
        np.testing.assert_allclose(U.sum(axis=(1, 2)), U0.sum(axis=(1, 2)), rtol=1e-13)
        ex = W.density_wave_2d(n, n, t=info["t"])
        errs.append(W.error_norms(U[0], ex[0], (2.0 / n) ** 2)[0])
    assert math.log2(errs[0] / errs[1]) > 4.3, errs


def test_batched_runs_match_single_runs():
    ens = W.ensemble_subset(W.riemann_ensemble(nprob=16, n_lo=24, n_hi=48), [0, 3, 7])
    Ub, steps = oracle.run_batch(ens, t_end=0.02)
    for i in range(3):
        sl = slice(ens.offsets[i], ens.offsets[i + 1])
        Ui, info = oracle.run_1d(ens.U[:, sl], (1, 1), ens.dx[i], 0.02)
        np.testing.assert_array_equal(Ub[:, sl], Ui)
        assert steps[i] == info["steps"]
        assert np.all(Ui[0] > 0) and np.all(W.pressure(Ui) > 0)
