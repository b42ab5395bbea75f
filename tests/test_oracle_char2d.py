"""Pins of the oracle's characteristic-wise reconstruction on the lines of
the 2D operator (Sec. 2.3 applied dimension by dimension): 4x4 eigenvector
blocks of the flux Jacobian along the line, the 4x4 block chasing, and the
reconstruction itself.  CPU only."""
import math

import numpy as np
import pytest

import oracle
import workloads as W

GAMMA = 1.4
RNG = np.random.default_rng(2024)


def rand_state2(rho=(0.1, 10), vel=(-3, 3), p=(0.01, 10)):
    r = 10 ** RNG.uniform(math.log10(rho[0]), math.log10(rho[1]))
    u, v = RNG.uniform(vel[0], vel[1], size=2)
    pr = 10 ** RNG.uniform(math.log10(p[0]), math.log10(p[1]))
    return np.array([r, r * u, r * v, pr / (GAMMA - 1) + 0.5 * r * (u * u + v * v)])


def flux2(U, nrm):
    """Euler flux of (rho, rho u, rho v, E) along momentum component nrm;
    works on complex arrays (for the complex-step derivative)."""
    rho, E = U[0], U[3]
    un = U[nrm] / rho
    p = (GAMMA - 1) * (E - 0.5 * (U[1] * U[1] + U[2] * U[2]) / rho)
    F = [U[0] * un, U[1] * un, U[2] * un, (E + p) * un]
    F[nrm] = F[nrm] + p
    return np.array(F)


def jacobian(U, nrm):
    """dF/dU by complex-step differentiation (exact to roundoff; no formula
    of the eigen-decomposition used)."""
    J = np.empty((4, 4))
    h = 1e-30
    for j in range(4):
        Uc = U.astype(complex)
        Uc[j] += 1j * h
        J[:, j] = flux2(Uc, nrm).imag / h
    return J


@pytest.mark.parametrize("nrm", [1, 2])
def test_eigenvectors_diagonalise_the_2d_jacobian(nrm):
    """L R = I; L A R = diag(u_n - a, u_n, u_n, u_n + a) with A the flux
    Jacobian along the line at the Roe state (built from the velocities and
    enthalpy that R carries); and Roe's property R Lambda L (Ub - Ua) =
    F(Ub) - F(Ua), which fixes the averages of both velocity components and
    of the enthalpy."""
    t = 3 - nrm
    for _ in range(60):
        Ua, Ub = rand_state2(), rand_state2()
        L, R, lam = oracle.char_eigen2(Ua, Ub, nrm)
        np.testing.assert_allclose(L @ R, np.eye(4), atol=1e-12)
        un, ut = R[nrm, 1], R[t, 1]
        a = 0.5 * (lam[3] - lam[0])
        H = R[3, 3] - un * a
        assert abs(R[3, 1] - 0.5 * (un * un + ut * ut)) < 1e-12 * (1 + H)
        # a state with these (u, v, H); the Jacobian depends on nothing else
        q2 = un * un + ut * ut
        Us = np.zeros(4)
        Us[0] = 1.0
        Us[nrm], Us[t] = un, ut
        Us[3] = (H + 0.5 * (GAMMA - 1) * q2) / GAMMA
        A = jacobian(Us, nrm)
        D = L @ A @ R
        scale = np.abs(lam).max()
        np.testing.assert_allclose(D, np.diag([un - a, un, un, un + a]), atol=1e-11 * scale)
        dF = flux2(Ub, nrm) - flux2(Ua, nrm)
        np.testing.assert_allclose(R @ np.diag(lam) @ L @ (Ub - Ua), dF,
                                   atol=1e-11 * np.abs(dF).max() + 1e-14)


def test_eigen_degenerate_sound_speed_is_componentwise():
    """Two pressureless states moving together have Roe sound speed 0: the
    node falls back to the identity (the 1D reading, extended)."""
    Ua = np.array([1.0, 0.5, -0.25, 0.5 * (0.25 + 0.0625)])
    Ub = np.array([2.0, 1.0, -0.5, 0.5 * 2.0 * (0.25 + 0.0625)])
    for nrm in (1, 2):
        L, R, lam = oracle.char_eigen2(Ua, Ub, nrm)
        np.testing.assert_array_equal(L, np.eye(4))
        np.testing.assert_array_equal(R, np.eye(4))


def test_eigen_reduces_to_1d_without_tangential_velocity():
    """With u_t = 0 the acoustic and entropy rows act on (rho, m_n, E) as the
    1D eigenvectors do and the shear row picks the tangential momentum."""
    for _ in range(20):
        a3, b3 = RNG.uniform(0.5, 2, 3), RNG.uniform(0.5, 2, 3)
        for v in (a3, b3):
            v[2] = 2.0 + v[1] ** 2 / (2 * v[0])
        L3, R3, lam3 = oracle.char_eigen(a3, b3)
        for nrm in (1, 2):
            t = 3 - nrm
            Ua, Ub = np.zeros(4), np.zeros(4)
            for U, s in ((Ua, a3), (Ub, b3)):
                U[0], U[nrm], U[3] = s
            L, R, lam = oracle.char_eigen2(Ua, Ub, nrm)
            idx = [0, nrm, 3]
            np.testing.assert_allclose(L[np.ix_([0, 1, 3], idx)], L3, rtol=1e-13, atol=1e-14)
            np.testing.assert_allclose(R[np.ix_(idx, [0, 1, 3])], R3, rtol=1e-13, atol=1e-14)
            np.testing.assert_allclose(lam[[0, 1, 3]], lam3, rtol=1e-13, atol=1e-14)
            e = np.zeros(4)
            e[t] = 1.0
            np.testing.assert_array_equal(L[2], e)
            np.testing.assert_array_equal(L[[0, 1, 3], t], 0.0)


@pytest.mark.parametrize("n,cyclic", [(1, False), (2, False), (3, False), (8, False), (13, False),
                                      (3, True), (4, True), (11, True)])
def test_4x4_block_chasing_matches_dense_solve(n, cyclic):
    """The 4x4 block chasing (and its cyclic form) against a dense solve of
    the assembled 4n x 4n system."""
    rng = np.random.default_rng(70 + n + 10 * cyclic)
    A = rng.normal(size=(n, 4, 4))
    C = rng.normal(size=(n, 4, 4))
    B = rng.normal(size=(n, 4, 4)) + 9 * np.eye(4)
    Y = rng.normal(size=(n, 4))
    X = oracle.block_solve(A, B, C, Y, cyclic)
    M = np.zeros((4 * n, 4 * n))
    for i in range(n):
        M[4 * i:4 * i + 4, 4 * i:4 * i + 4] += B[i]
        for blk, j in ((A[i], i - 1), (C[i], i + 1)):
            if cyclic:
                j %= n
            elif not 0 <= j < n:
                continue
            M[4 * i:4 * i + 4, 4 * j:4 * j + 4] += blk
    ref = np.linalg.solve(M, Y.reshape(-1)).reshape(n, 4)
    np.testing.assert_allclose(X, ref, atol=1e-12 * np.abs(ref).max())


def _poly_avgs(coef, edges):
    anti = np.polynomial.polynomial.polyint(coef)
    Q = np.polynomial.polynomial.polyval(edges, anti)
    return (Q[1:] - Q[:-1]) / np.diff(edges)


@pytest.mark.parametrize("nrm", [1, 2])
@pytest.mark.parametrize("seed", range(2))
def test_char2_exact_for_quadratics(nrm, seed):
    """Each block row is a combination of scalar rows of eq. (CWENO-FV),
    each exact for quadratics, so quadratic conserved variables are
    reconstructed exactly (nonlinear weights, node-dependent 4x4 blocks)."""
    rng = np.random.default_rng(500 + seed + 7 * nrm)
    n, h = 21, 0.05
    edges = (np.arange(-3, n + 4)) * h
    coef = [np.array([1.0, 0.3, 0.5]) * rng.uniform(0.5, 1.5, 3),
            rng.normal(size=3) * 0.3, rng.normal(size=3) * 0.3,
            np.array([4.0, 0.5, 1.0]) * rng.uniform(0.5, 1.5, 3)]
    ue = np.array([_poly_avgs(c, edges) for c in coef])
    um, up = oracle.recon_char2(ue, False, nrm)
    xr, xl = edges[4:n + 4], edges[3:n + 3]
    for c in range(4):
        scale = np.abs(ue[c]).max()
        np.testing.assert_allclose(um[c], np.polynomial.polynomial.polyval(xr, coef[c]),
                                   atol=1e-11 * scale)
        np.testing.assert_allclose(up[c], np.polynomial.polynomial.polyval(xl, coef[c]),
                                   atol=1e-11 * scale)


def _riemann_line(n, nrm, vt=0.0):
    x = W.cell_centres(0.0, 1.0, n)
    rho = 1 + 0.4 * (x > 0.4) + 0.1 * np.sin(5 * x)
    un = 0.3 * np.cos(3 * x)
    p = 1 + 0.6 * (x < 0.7)
    U = np.zeros((4, n))
    U[0] = rho
    U[nrm] = rho * un
    U[3 - nrm] = rho * vt * (1 + 0.5 * (x > 0.55))
    U[3] = p / (GAMMA - 1) + 0.5 * rho * (un * un + (U[3 - nrm] / rho) ** 2)
    return U


def _ghosts(U, cyclic):
    if cyclic:
        return np.concatenate([U[:, -3:], U, U[:, :3]], axis=1)
    return np.concatenate([np.repeat(U[:, :1], 3, 1), U, np.repeat(U[:, -1:], 3, 1)], axis=1)


@pytest.mark.parametrize("cyclic", [True, False])
@pytest.mark.parametrize("nrm", [1, 2])
def test_char2_reduces_to_1d_without_tangential_momentum(cyclic, nrm):
    """A line with zero tangential momentum: the 4x4 system splits into the
    1D 3x3 system on (rho, m_n, E) and a zero tangential field."""
    n = 37
    U = _riemann_line(n, nrm)
    um, up = oracle.recon_char2(_ghosts(U, cyclic), cyclic, nrm)
    U3 = U[[0, nrm, 3]]
    um3, up3 = oracle.recon_char(_ghosts(U3, cyclic), cyclic)
    scale = np.abs(U).max()
    np.testing.assert_allclose(um[[0, nrm, 3]], um3, atol=1e-13 * scale)
    np.testing.assert_allclose(up[[0, nrm, 3]], up3, atol=1e-13 * scale)
    assert np.abs(um[3 - nrm]).max() == 0.0 and np.abs(up[3 - nrm]).max() == 0.0


@pytest.mark.parametrize("cyclic", [True, False])
def test_char2_direction_symmetry(cyclic):
    """A y line is an x line with the momentum components exchanged."""
    n = 29
    U = _riemann_line(n, 1, vt=0.4)
    sw = [0, 2, 1, 3]
    um1, up1 = oracle.recon_char2(_ghosts(U, cyclic), cyclic, 1)
    um2, up2 = oracle.recon_char2(_ghosts(U[sw], cyclic), cyclic, 2)
    scale = np.abs(U).max()
    np.testing.assert_allclose(um2[sw], um1, atol=1e-13 * scale)
    np.testing.assert_allclose(up2[sw], up1, atol=1e-13 * scale)


@pytest.mark.parametrize("cyclic", [True, False])
def test_char2_mirror_symmetry(cyclic):
    """Reversing a line and negating its normal momentum mirrors it: the "-"
    values of the mirrored line are the mirrored "+" values (ties the "-"
    rows and their Roe pairs to the "+" rows)."""
    n = 30
    U = _riemann_line(n, 1, vt=0.3)
    um, up = oracle.recon_char2(_ghosts(U, cyclic), cyclic, 1)
    flip = np.array([1.0, -1.0, 1.0, 1.0])[:, None]
    Ur = flip * U[:, ::-1]
    um_r, up_r = oracle.recon_char2(_ghosts(Ur, cyclic), cyclic, 1)
    scale = np.abs(U).max()
    np.testing.assert_allclose(flip * um_r[:, ::-1], up, atol=1e-12 * scale)
    np.testing.assert_allclose(flip * up_r[:, ::-1], um, atol=1e-12 * scale)


def test_char2_density_wave_line_equals_componentwise():
    """Along a line of the 2D density wave (u, v, p constant) the conserved
    variables are affine in rho along r1, three fields are constant and the
    component-wise nodal values solve the block system (Table 3 repeats
    Table 2's errors in 1D for the same reason)."""
    U2 = W.density_wave_2d(40, 8)
    for nrm, line in ((1, U2[:, 3, :]), (2, U2[:, :, 5])):
        line = np.ascontiguousarray(line)
        ue = _ghosts(line, True)
        um_c, up_c = oracle.recon_char2(ue, True, nrm)
        for c in range(4):
            um, up = oracle.recon_scalar(np.ascontiguousarray(ue[c]), True)
            np.testing.assert_allclose(um_c[c], um, rtol=1e-13, atol=1e-13)
            np.testing.assert_allclose(up_c[c], up, rtol=1e-13, atol=1e-13)


def _blast_2d(nx, ny):
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)
    r2 = (X - 0.45) ** 2 + (Y - 0.55) ** 2
    rho = 1.0 + 0.5 * (r2 < 0.06)
    u = 0.3 * np.sin(2 * np.pi * Y)
    v = -0.2 * np.cos(2 * np.pi * X)
    p = 0.4 + 2.0 * (r2 < 0.04)
    return np.stack([rho, rho * u, rho * v, p / (GAMMA - 1) + 0.5 * rho * (u * u + v * v)])


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 2, 2)])
def test_rhs_2d_char_transposition(bc):
    """The 2D operator with characteristic lines commutes with transposing
    the grid and exchanging the momentum components."""
    U = _blast_2d(24, 20)
    p = oracle.params(recon=3)
    L = oracle.rhs_2d(U, bc, 1 / 24, 1 / 20, p)
    sw = [0, 2, 1, 3]
    Ut = np.ascontiguousarray(U[sw].transpose(0, 2, 1))
    bct = (bc[2], bc[3], bc[0], bc[1])
    Lt = oracle.rhs_2d(Ut, bct, 1 / 20, 1 / 24, p)
    scale = np.abs(L).max()
    np.testing.assert_allclose(Lt[sw].transpose(0, 2, 1), L, atol=1e-12 * scale)


def test_rhs_2d_char_one_axis_equals_1d():
    """Data constant in y with v = 0: the x lines are 1D characteristic lines
    and the y lines carry no flux difference, so the 2D operator equals the
    1D one on (rho, rho u, E) and zero in rho v up to the roundoff of the
    y lines' block solves of constant data."""
    n, ny = 40, 6
    x = W.cell_centres(0.0, 1.0, n)
    U1 = W.prim_to_cons_1d(1 + 0.5 * (x > 0.5), 0.2 * np.ones(n), 1 + 1.5 * (x < 0.3), GAMMA)
    U = np.zeros((4, ny, n))
    U[0], U[1], U[3] = U1[0], U1[1], U1[2]
    p = oracle.params(recon=3)
    L2 = oracle.rhs_2d(U, (1, 1, 0, 0), 1 / n, 1 / ny, p)
    L1 = oracle.rhs_1d(U1, (1, 1), 1 / n, p)
    scale = np.abs(L1).max()
    for j in range(ny):
        np.testing.assert_allclose(L2[[0, 1, 3], j], L1, atol=1e-12 * scale)
    assert np.abs(L2[2]).max() < 1e-13 * scale


def test_rhs_2d_char_conserves_on_periodic_grids():
    """The characteristic lines change the face values, not the flux form:
    on a periodic grid the flux differences telescope, so the sum of L over
    the cells vanishes to roundoff in every component."""
    U = _blast_2d(24, 20)
    L = oracle.rhs_2d(U, (0, 0, 0, 0), 1 / 24, 1 / 20, oracle.params(recon=3))
    for k in range(4):
        assert abs(L[k].sum()) <= 1e-12 * np.abs(L[k]).sum(), k
