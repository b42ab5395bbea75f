"""Pins of the oracle's restart rule in 2D (rule 3; the reading that a step
with a stage output outside G is redone from U^n with half the dt): it is
the CFL rule where no step leaves G, it keeps a near-vacuum blast in G
where the CFL rule leaves it, and each step it keeps is the plain SSP-RK3
step at the CFL dt halved as often as the rule says, the attempt before
it having left G.  CPU only."""
import numpy as np

import oracle
import workloads as W

GAMMA = 1.4


def in_G(U):
    rho = U[0]
    p = (GAMMA - 1) * (U[3] - 0.5 * (U[1] ** 2 + U[2] ** 2) / rho)
    return bool(np.all(np.isfinite(U)) and np.all(rho > 0) and np.all(p > 0))


def planar_blast_2d(nx=200, ny=5):
    """The near-vacuum blast along x ([-1, 1], p = 4e3 in the two centre
    cells, 1e-10 elsewhere) on ny rows, with a 1 % density ripple along y
    so that the y-sweeps act."""
    U1 = W.vacuum_blast_1d(nx)
    y = (np.arange(ny) + 0.5) / ny
    rip = 1.0 + 0.01 * np.sin(2 * np.pi * y)[:, None]
    U = np.zeros((4, ny, nx))
    U[0] = U1[0][None, :] * rip
    U[1] = U1[1][None, :] * rip
    U[3] = U1[2][None, :]
    return U


def hot_spot_2d(n=32):
    x = W.cell_centres(-1, 1, n)[None, :]
    y = W.cell_centres(-1, 1, n)[:, None]
    hot = (np.abs(x) < 2.0 / n) & (np.abs(y) < 2.0 / n)
    rho = np.ones((n, n))
    return np.stack([rho, 0 * rho, 0 * rho, np.where(hot, 4e3, 1e-10) / (GAMMA - 1)])


def test_restart_equals_cfl_rule_without_violations():
    """A hot spot in a 1e-10 background whose 60 CFL steps stay in G: the
    restart rule redoes nothing and its run is the CFL rule's, bitwise."""
    U0 = hot_spot_2d()
    h = 2.0 / 32
    a, ia = oracle.run_2d(U0, (1, 1, 1, 1), h, h, 1.0, max_steps=60, rule=oracle.DT_CFL)
    b, ib = oracle.run_2d(U0, (1, 1, 1, 1), h, h, 1.0, max_steps=60, rule=oracle.DT_RESTART)
    assert ia["out_of_G"] == 0 and ib["restarts"] == 0
    assert np.array_equal(a, b) and ia["t"] == ib["t"]


def test_restart_keeps_the_planar_blast_in_G():
    """The planar near-vacuum blast: 80 CFL steps leave G, the restart rule's
    80 steps redo some and keep every stage output in G."""
    U0 = planar_blast_2d()
    h = 2.0 / 200
    bc = (1, 1, 0, 0)
    try:
        _, ia = oracle.run_2d(U0, bc, h, h, 1.0, max_steps=80, rule=oracle.DT_CFL)
        left = ia["out_of_G"] > 0
    except RuntimeError:
        left = True   # a stage went non-finite
    assert left
    U, ib = oracle.run_2d(U0, bc, h, h, 1.0, max_steps=80, rule=oracle.DT_RESTART)
    assert ib["steps"] == 80 and ib["restarts"] > 0 and ib["out_of_G"] == 0
    assert in_G(U)


def _three_stages(U, dt, bc, h):
    U1 = oracle.stage_2d(U, U, 1, dt, bc, h, h)
    U2 = oracle.stage_2d(U, U1, 2, dt, bc, h, h)
    U3 = oracle.stage_2d(U, U2, 3, dt, bc, h, h)
    return U1, U2, U3


def test_restart_step_is_the_halved_cfl_step():
    """From the state before the first steps the rule redoes: the step kept
    equals three plain stages at the CFL dt / 2^k (k the halvings it
    reports), all of whose outputs are in G, while the attempt at twice that
    dt had a stage output outside G."""
    U = planar_blast_2d()
    h = 2.0 / 200
    bc = (1, 1, 0, 0)
    found = 0
    for _ in range(80):
        Un, info = oracle.run_2d(U, bc, h, h, 1.0, max_steps=1, rule=oracle.DT_RESTART)
        if info["restarts"] > 0:
            s_x, s_y = oracle.max_speed_2d(U)
            dt0 = (1.0 / 12.0) / (s_x / h + s_y / h)
            k = info["restarts"]
            assert info["t"] == dt0 / 2 ** k
            stages = _three_stages(U, info["t"], bc, h)
            assert np.array_equal(stages[2], Un) and all(in_G(V) for V in stages)
            before = _three_stages(U, 2.0 * info["t"], bc, h)
            assert not all(in_G(V) for V in before)
            found += 1
            if found == 3:
                break
        U = Un
    assert found == 3
