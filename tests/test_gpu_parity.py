"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs (FP64 bar: 1e-12 relative per stage output)."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_STAGE = 1e-12    # per stage output, relative to max |U| per component


def gpu():
    import paper_1402_5618_amd as pp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return pp


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def comp_rel(a, b):
    return max(rel(a[k], b[k]) for k in range(a.shape[0]))


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def euler_flux_2d(U, nrm):
    """Physical flux of 2D cell averages [4][ny][nx] in direction nrm (1: x, 2: y)."""
    r, E = U[0], U[3]
    un = U[nrm] / r
    p = 0.4 * (E - 0.5 * (U[1] ** 2 + U[2] ** 2) / r)
    F = np.array([U[k] * un for k in range(4)])
    F[nrm] += p
    F[3] = un * (E + p)
    return F


def mixed_line(n, seed=0, a=0.0, b=1.0):
    """Smooth waves, two contacts and a shock: exercises every branch."""
    rng = np.random.default_rng(seed)
    x = W.cell_centres(a, b, n)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x / (b - a)) + 0.8 * ((x > a + 0.3 * (b - a)) & (x < a + 0.6 * (b - a)))
    u = 0.5 * np.cos(4 * np.pi * x / (b - a)) + rng.normal(0, 0.01, n)
    p = np.where(x < a + 0.7 * (b - a), 1.0, 0.1) * (1 + 0.1 * np.sin(6 * x))
    return W.prim_to_cons_1d(rho, u, p, 1.4)


CASES_1D = [(3, (1, 1)), (5, (0, 0)), (7, (0, 0)), (13, (1, 1)), (64, (0, 0)), (128, (2, 1)),
            (200, (1, 2)), (777, (2, 2)), (2047, (0, 0)), (2048, (0, 0)), (2048, (1, 2)), (2048, (2, 2)),
            (2049, (1, 1)),
            (4000, (1, 1)), (4096, (2, 2))]


WIDENED = []   # every use of the widened stage bar: (case, bar, cells the limiter acts on)


def stage_tolerance(U0, Us, st, dt, bc, h, ref, k=4):
    """1e-12, or 4x the oracle's own change under k seeded relative input
    perturbations of 1e-15 when that is larger.  Where the limiter puts an
    interface state on e = eps (pressure ~1e-14), the sound speed is a square
    root of a roundoff-sized number and the stage output moves by ~1e-12 under
    a last-bit change of its input; bit-level agreement is then not defined."""
    rng = np.random.default_rng(1402 + st)
    sens = 0.0
    for _ in range(k):
        f0 = 1.0 + 1e-15 * rng.standard_normal(U0.shape)
        fs = 1.0 + 1e-15 * rng.standard_normal(Us.shape)
        V = oracle.stage_1d(U0 * f0, Us * fs, st, dt, bc, h)
        sens = max(sens, comp_rel(V, ref))
    bar = max(TOL_STAGE, 4.0 * sens)
    # the named cause: interface states the limiter has put on the e = eps
    # boundary (cells it limits in this stage input)
    _, dbg = oracle.line_op(Us, bc[0], bc[1], h, debug=True)
    WIDENED.append((f"n={Us.shape[1]} bc={bc} stage {st}", bar, dbg["nlim"]))
    print(f"widened stage bar {bar:.2e}: n={Us.shape[1]} bc={bc} stage {st}, limiter active on "
          f"{dbg['nlim']} cells", flush=True)
    return bar


def step_tolerance(U0, dt, bc, h, ref, k=4):
    """stage_tolerance for a whole SSP-RK3 step of the oracle."""
    rng = np.random.default_rng(1402)
    sens = 0.0
    for _ in range(k):
        V0 = U0 * (1.0 + 1e-15 * rng.standard_normal(U0.shape))
        V1 = oracle.stage_1d(V0, V0, 1, dt, bc, h)
        V2 = oracle.stage_1d(V0, V1, 2, dt, bc, h)
        sens = max(sens, comp_rel(oracle.stage_1d(V0, V2, 3, dt, bc, h), ref))
    return max(TOL_STAGE, 4.0 * sens)


@pytest.mark.parametrize("n,bc", CASES_1D)
def test_1d_stage_parity(n, bc):
    pp = gpu()
    print(f"case n={n} bc={bc}", flush=True)
    h = 1.0 / n
    U = mixed_line(n, seed=n)
    dt = (1.0 / 12.0) * h / oracle.max_speed_1d(U)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(*bc, 0, 0))
    Ud = dev(U)
    U1 = oracle.stage_1d(U, U, 1, dt, bc, h)
    U2 = oracle.stage_1d(U, U1, 2, dt, bc, h)
    U3 = oracle.stage_1d(U, U2, 3, dt, bc, h)
    o1, o2, o3 = (torch.empty_like(Ud) for _ in range(3))
    s.stage(Ud, Ud, o1, 1, dt)
    s.stage(Ud, dev(U1), o2, 2, dt)
    s.stage(Ud, dev(U2), o3, 3, dt)
    torch.cuda.synchronize()
    for st, (got, ref, Us) in enumerate(((o1, U1, U), (o2, U2, U1), (o3, U3, U2)), start=1):
        err = comp_rel(got.cpu().numpy(), ref)
        if err > TOL_STAGE:   # only then pay for the conditioning estimate
            tol = stage_tolerance(U, Us, st, dt, bc, h, ref)
            print(f"stage {st}: err {err:.2e}, conditioning bound {tol:.2e}", flush=True)
            assert err <= tol
    s.close()


@pytest.mark.parametrize("n,bc", [(64, (0, 0)), (200, (1, 2)), (2049, (1, 1))])
def test_1d_rhs_and_interface_states(n, bc):
    pp = gpu()
    h = 1.0 / n
    U = mixed_line(n, seed=3 * n)
    Lref, dbg = oracle.line_op(U, bc[0], bc[1], h, debug=True)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(*bc, 0, 0))
    Ud = dev(U)
    L = torch.empty_like(Ud)
    s.rhs(Ud, L)
    um, up = torch.empty_like(Ud), torch.empty_like(Ud)
    flux = torch.empty((3, n + 1), dtype=torch.float64, device="cuda")
    s.debug_line(Ud, um, up, flux)
    torch.cuda.synchronize()
    assert comp_rel(um.cpu().numpy(), dbg["um"]) <= 1e-12
    assert comp_rel(up.cpu().numpy(), dbg["up"]) <= 1e-12
    assert comp_rel(flux.cpu().numpy(), dbg["flux"]) <= 1e-12
    # L = -(F_{i+1/2} - F_{i-1/2}) / h: a flux difference, so flux roundoff
    # (1e-12 relative to |F|, the face-flux bar above) gives L an error of
    # 1e-12 |F| / h against |L| ~ |dF| / h: the bar is 1e-12 max|F| / max|dF|
    Lg = L.cpu().numpy()
    for k in range(3):
        F = dbg["flux"][k]
        bar = 1e-12 * max(1.0, np.abs(F).max() / np.abs(np.diff(F)).max())
        err = float(np.abs(Lg[k] - Lref[k]).max() / np.abs(Lref[k]).max())
        print(f"L component {k}: {err:.2e} (bar {bar:.1e})", flush=True)
        assert err <= bar
    s.close()


def test_1d_positivity_snapshot_parity():
    """Stage parity on a mid-run near-vacuum state (double rarefaction,
    limiter active)."""
    pp = gpu()
    n, h = 400, 0.005
    U, info = oracle.run_1d(W.double_rarefaction_1d(n), (1, 1), h, 0.6, max_steps=300)
    dt = (1.0 / 12.0) * h / oracle.max_speed_1d(U)
    ref = oracle.stage_1d(U, U, 1, dt, (1, 1), h)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(1, 1, 0, 0))
    Ud = dev(U)
    out = torch.empty_like(Ud)
    s.stage(Ud, Ud, out, 1, dt)
    torch.cuda.synchronize()
    assert comp_rel(out.cpu().numpy(), ref) <= TOL_STAGE
    s.close()


CASES_2D = [(40, 24, (0, 0, 0, 0)), (33, 17, (1, 2, 2, 1)), (64, 64, (0, 0, 1, 1))]


@pytest.mark.parametrize("nx,ny,bc", CASES_2D)
def test_2d_stage_parity(nx, ny, bc):
    pp = gpu()
    print(f"case 2d {nx}x{ny} bc={bc}", flush=True)
    rng = np.random.default_rng(nx * ny)
    x = W.cell_centres(0, 1, nx)[None, :]
    y = W.cell_centres(0, 1, ny)[:, None]
    rho = 1 + 0.3 * np.sin(2 * np.pi * (x + 2 * y)) + 0.5 * ((x - 0.5) ** 2 + (y - 0.4) ** 2 < 0.06)
    u = 0.3 * np.cos(2 * np.pi * y) + 0 * x
    v = -0.2 * np.sin(2 * np.pi * x) + 0 * y
    p = 1 + 0.5 * (x > 0.6) + 0.1 * rng.normal(size=(ny, nx)) ** 2
    U = np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    dx, dy = 1.0 / nx, 1.0 / ny
    s_x, s_y = oracle.max_speed_2d(U)
    dt = (1.0 / 12.0) / (s_x / dx + s_y / dy)
    s = pp.Solver(ndim=2, nx=nx, ny=ny, dx=dx, dy=dy, bc=bc)
    Ud = dev(U)
    Lref = oracle.rhs_2d(U, bc, dx, dy)
    L = torch.empty_like(Ud)
    s.rhs(Ud, L)
    ref1 = oracle.stage_2d(U, U, 1, dt, bc, dx, dy)
    ref2 = oracle.stage_2d(U, ref1, 2, dt, bc, dx, dy)
    o1, o2 = torch.empty_like(Ud), torch.empty_like(Ud)
    s.stage(Ud, Ud, o1, 1, dt)
    s.stage(Ud, dev(ref1), o2, 2, dt)
    torch.cuda.synchronize()
    # L = L_x + L_y, flux differences over dx and dy: the bar is 1e-12 of the
    # flux scale (max|F_x|/dx + max|F_y|/dy, from the cell averages) over max|L|
    Lg = L.cpu().numpy()
    for k in range(4):
        Fx = np.abs(euler_flux_2d(U, 1)[k]).max()
        Fy = np.abs(euler_flux_2d(U, 2)[k]).max()
        bar = 1e-12 * max(1.0, (Fx / dx + Fy / dy) / np.abs(Lref[k]).max())
        err = float(np.abs(Lg[k] - Lref[k]).max() / np.abs(Lref[k]).max())
        print(f"L component {k}: {err:.2e} (bar {bar:.1e})", flush=True)
        assert err <= bar
    assert comp_rel(o1.cpu().numpy(), ref1) <= TOL_STAGE
    assert comp_rel(o2.cpu().numpy(), ref2) <= TOL_STAGE
    # one full step in place
    Us = Ud.clone()
    s.step(Us, dt)
    ref3 = oracle.stage_2d(U, ref2, 3, dt, bc, dx, dy)
    torch.cuda.synchronize()
    assert comp_rel(Us.cpu().numpy(), ref3) <= TOL_STAGE
    s.close()


@pytest.mark.parametrize("nsteps", [0, 5, 20])
def test_2d_sedov_stage_parity(nsteps):
    """Near-vacuum quarter-plane blast on 64^2 (reflective x = 0 and y = 0):
    the three stages of one step from oracle snapshots, limiter active."""
    pp = gpu()
    n, ext = 64, 1.1
    dx = ext / n
    bc = (2, 1, 2, 1)
    U = W.sedov_corner_2d(n, extent=ext)
    dt = 0.0
    for _ in range(nsteps + 1):
        s_x, s_y = oracle.max_speed_2d(U)
        dt = (1.0 / 12.0) / (s_x / dx + s_y / dx)
        if _ == nsteps:
            break
        U1 = oracle.stage_2d(U, U, 1, dt, bc, dx, dx)
        U2 = oracle.stage_2d(U, U1, 2, dt, bc, dx, dx)
        U = oracle.stage_2d(U, U2, 3, dt, bc, dx, dx)
    print(f"case sedov 64^2 after {nsteps} steps, dt {dt:.3e}", flush=True)
    refs = [U]
    for st in (1, 2, 3):
        refs.append(oracle.stage_2d(U, refs[-1], st, dt, bc, dx, dx))
    s = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=bc)
    Ud = dev(U)
    for st in (1, 2, 3):
        out = torch.empty_like(Ud)
        s.stage(Ud, dev(refs[st - 1]), out, st, dt)
        torch.cuda.synchronize()
        err = comp_rel(out.cpu().numpy(), refs[st])
        if err > TOL_STAGE:
            # same conditioning bound as in 1D: the oracle against itself
            rng = np.random.default_rng(st)
            sens = 0.0
            for _ in range(3):
                V = oracle.stage_2d(U * (1 + 1e-15 * rng.standard_normal(U.shape)),
                                    refs[st - 1] * (1 + 1e-15 * rng.standard_normal(U.shape)),
                                    st, dt, bc, dx, dx)
                sens = max(sens, comp_rel(V, refs[st]))
            print(f"stage {st}: err {err:.2e}, conditioning bound {4 * sens:.2e}", flush=True)
            assert err <= max(TOL_STAGE, 4.0 * sens)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_2d_sedov_1024_stage_sampled_parity(precision):
    """The near-vacuum blast at its benchmarked size (1024^2, reflective
    x = 0 and y = 0, transmissive far ends), first stage from the initial
    state in the bench's launch configuration: sampled cells around the
    energy-carrying corner cell, on the reflective walls and far away,
    against the oracle's row and column operators (FP64 to the stage
    tolerance, mixed to its bound)."""
    pp = gpu()
    n, ext = 1024, 1.1
    dx = ext / n
    bc = (2, 1, 2, 1)
    U = W.sedov_corner_2d(n, extent=ext)
    sx, sy = oracle.max_speed_2d(U)
    dt = (1.0 / 12.0) / (sx / dx + sy / dx)
    print(f"case sedov 1024^2 {precision}, dt {dt:.3e}", flush=True)
    s = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=bc,
                  precision=pp.PP_FP64 if precision == "fp64" else pp.PP_MIXED)
    Ud = dev(U)
    out = torch.empty_like(Ud)
    s.stage(Ud, Ud, out, 1, dt)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    er, ee = oracle.eps(U)
    rng = np.random.default_rng(3)
    pts = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 2), (0, 3), (3, 0), (n - 1, n - 1), (0, n - 1)]
    pts += [(int(y), int(x)) for y, x in rng.integers(0, n, size=(6, 2))]
    tol = TOL_STAGE if precision == "fp64" else TOL_MIXED_STAGE

    def ref_at(V, y, x):
        Lx = oracle.line_op(np.ascontiguousarray(V[:, y, :]), bc[0], bc[1], dx, eps_rho=er,
                            eps_e=ee, nrm=1)
        Ly = oracle.line_op(np.ascontiguousarray(V[:, :, x]), bc[2], bc[3], dx, eps_rho=er,
                            eps_e=ee, nrm=2)
        return V[:, y, x] + dt * (Lx[:, x] + Ly[:, y])

    refs = {pt: ref_at(U, *pt) for pt in pts}
    # per-component scale: the input's largest magnitude, or the sampled
    # outputs' (the momenta start at zero; the corner samples carry the blast)
    scale = np.maximum(np.abs(U).reshape(4, -1).max(axis=1),
                       np.abs(np.array(list(refs.values()))).max(axis=0))
    assert np.all(scale > 0)
    for (y, x) in pts:
        ref = refs[(y, x)]
        err = np.max(np.abs(got[:, y, x] - ref) / scale)
        assert err <= tol, (y, x, err)
    s.close()


# ------------------------------------------------------------ batched ensemble
def ensemble(nprob, n_lo, n_hi, seed=1402):
    return W.riemann_ensemble(nprob=nprob, seed=seed, n_lo=n_lo, n_hi=n_hi)


@pytest.mark.parametrize("n_lo,n_hi,plan", [(8, 40, 0), (256, 4096, 0), (256, 4096, 1),
                                             (256, 4096, 2), (8, 40, 3), (256, 4096, 4),
                                             (256, 4096, 5)])
def test_batch_step_parity(n_lo, n_hi, plan):
    """One SSP-RK3 step of every problem (persistent launches per stage and
    length class of the launch plan) against the oracle's stages, each
    problem with its own dt; one problem inactive."""
    pp = gpu()
    ens = ensemble(24, n_lo, n_hi)
    print(f"case batch n in [{n_lo},{n_hi}] total={ens.U.shape[1]} plan={plan}", flush=True)
    nb = len(ens.lengths)
    dts = np.array([(1.0 / 12.0) * ens.dx[i] /
                    oracle.max_speed_1d(ens.U[:, ens.offsets[i]:ens.offsets[i + 1]])
                    for i in range(nb)])
    dts[5] = 0.0
    s = pp.Solver(ndim=1, lengths=ens.lengths, dxs=ens.dx, bcs=[1] * (2 * nb))
    assert s.batch_tune(force_plan=plan)[0] == plan
    Ud = dev(ens.U)
    s.batch_step(Ud, dev(dts))
    torch.cuda.synchronize()
    got = Ud.cpu().numpy()
    for i in range(nb):
        sl = slice(ens.offsets[i], ens.offsets[i + 1])
        U = ens.U[:, sl]
        if dts[i] == 0.0:
            assert np.array_equal(got[:, sl], U)
            continue
        h = ens.dx[i]
        U1 = oracle.stage_1d(U, U, 1, dts[i], (1, 1), h)
        U2 = oracle.stage_1d(U, U1, 2, dts[i], (1, 1), h)
        U3 = oracle.stage_1d(U, U2, 3, dts[i], (1, 1), h)
        assert comp_rel(got[:, sl], U3) <= TOL_STAGE, i
    s.close()


@pytest.mark.parametrize("recon", [1, 2])
@pytest.mark.parametrize("n_lo,n_hi,plan", [(8, 40, 0), (256, 4096, 1), (8, 40, 3),
                                             (256, 4096, 4)])
def test_batch_step_parity_explicit_schemes(recon, n_lo, n_hi, plan):
    """Batched ensembles with the explicit WENO-JS / WENO-Z reconstructions
    (persistent launches templated on the reconstruction): one step of every
    problem against the oracle's stages of the same scheme, one problem
    inactive, under plans with one and two waves per system."""
    pp = gpu()
    ens = ensemble(16, n_lo, n_hi)
    print(f"case batch recon={recon} n in [{n_lo},{n_hi}] plan={plan}", flush=True)
    nb = len(ens.lengths)
    P = oracle.params(recon=recon)
    dts = np.array([(1.0 / 12.0) * ens.dx[i] /
                    oracle.max_speed_1d(ens.U[:, ens.offsets[i]:ens.offsets[i + 1]])
                    for i in range(nb)])
    dts[2] = 0.0
    rc = pp.PP_RECON_WENOJS if recon == 1 else pp.PP_RECON_WENOZ
    s = pp.Solver(ndim=1, lengths=ens.lengths, dxs=ens.dx, bcs=[1] * (2 * nb), recon=rc)
    assert s.batch_tune(force_plan=plan)[0] == plan
    Ud = dev(ens.U)
    s.batch_step(Ud, dev(dts))
    torch.cuda.synchronize()
    got = Ud.cpu().numpy()
    s.close()
    for i in range(nb):
        sl = slice(ens.offsets[i], ens.offsets[i + 1])
        U = ens.U[:, sl]
        if dts[i] == 0.0:
            assert np.array_equal(got[:, sl], U)
            continue
        h = ens.dx[i]
        U1 = oracle.stage_1d(U, U, 1, dts[i], (1, 1), h, P)
        U2 = oracle.stage_1d(U, U1, 2, dts[i], (1, 1), h, P)
        U3 = oracle.stage_1d(U, U2, 3, dts[i], (1, 1), h, P)
        err = comp_rel(got[:, sl], U3)
        if err > TOL_STAGE:
            rng = np.random.default_rng(1402)
            sens = 0.0
            for _ in range(4):
                V0 = U * (1.0 + 1e-15 * rng.standard_normal(U.shape))
                V1 = oracle.stage_1d(V0, V0, 1, dts[i], (1, 1), h, P)
                V2 = oracle.stage_1d(V0, V1, 2, dts[i], (1, 1), h, P)
                sens = max(sens, comp_rel(oracle.stage_1d(V0, V2, 3, dts[i], (1, 1), h, P), U3))
            print(f"  problem {i}: {err:.2e}, conditioning bound {4 * sens:.1e}", flush=True)
            assert err <= max(TOL_STAGE, 4.0 * sens), i


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_ensemble_step_sampled_parity(precision):
    """The benchmarked ensemble at full size (4096 seeded Riemann problems,
    N in [256, 4096], 8.8 M cells) in the bench's launch configuration (the
    autotuner's plan): one step of every problem with its own dt, sampled
    problems (the longest, the shortest and random ones) against the
    oracle's stages; FP64 to the stage tolerance, mixed to its bound."""
    pp = gpu()
    ens = W.riemann_ensemble()
    nb = len(ens.lengths)
    print(f"case full ensemble {precision}: {nb} problems, {ens.U.shape[1]} cells", flush=True)
    s = pp.Solver(ndim=1, lengths=ens.lengths, dxs=ens.dx, bcs=[1] * (2 * nb),
                  precision=pp.PP_FP64 if precision == "fp64" else pp.PP_MIXED)
    plan, _ = s.batch_tune(dev(ens.U), 1.0 / 12.0)
    rng = np.random.default_rng(21)
    sample = sorted(set([int(np.argmax(ens.lengths)), int(np.argmin(ens.lengths))] +
                        [int(i) for i in rng.integers(0, nb, size=10)]))
    dts = np.array([(1.0 / 12.0) * ens.dx[i] /
                    oracle.max_speed_1d(ens.U[:, ens.offsets[i]:ens.offsets[i + 1]])
                    for i in range(nb)])
    Ud = dev(ens.U)
    s.batch_step(Ud, dev(dts))
    torch.cuda.synchronize()
    got = Ud.cpu().numpy()
    tol = TOL_STAGE if precision == "fp64" else TOL_MIXED_STAGE
    for i in sample:
        sl = slice(ens.offsets[i], ens.offsets[i + 1])
        U = ens.U[:, sl]
        h = ens.dx[i]
        U1 = oracle.stage_1d(U, U, 1, dts[i], (1, 1), h)
        U2 = oracle.stage_1d(U, U1, 2, dts[i], (1, 1), h)
        U3 = oracle.stage_1d(U, U2, 3, dts[i], (1, 1), h)
        assert comp_rel(got[:, sl], U3) <= tol, (plan, i, int(ens.lengths[i]))
    s.close()


def test_batch_tune_picks_a_plan_and_results_agree():
    """The autotuner times every launch plan on a copy of the state (left
    unchanged) and keeps the fastest; the plans agree to rounding."""
    pp = gpu()
    ens = ensemble(40, 256, 4096, seed=11)
    nb = len(ens.lengths)
    print(f"case tune total={ens.U.shape[1]}", flush=True)
    s = pp.Solver(ndim=1, lengths=ens.lengths, dxs=ens.dx, bcs=[1] * (2 * nb))
    U0 = dev(ens.U)
    plan, ms = s.batch_tune(U0, 1.0 / 12.0)
    print(f"plan {plan}, ms per step {ms}", flush=True)
    assert 0 <= plan <= 5 and all(m > 0 for m in ms) and ms[plan] == min(ms)
    assert np.array_equal(U0.cpu().numpy(), ens.U)
    dts = dev(np.array([(1.0 / 12.0) * ens.dx[i] /
                        oracle.max_speed_1d(ens.U[:, ens.offsets[i]:ens.offsets[i + 1]])
                        for i in range(nb)]))
    outs = []
    for p in range(6):
        s.batch_tune(force_plan=p)
        Ud = dev(ens.U)
        s.batch_step(Ud, dts)
        outs.append(Ud.cpu().numpy())
    for p in range(1, 6):
        for i in range(nb):
            sl = slice(ens.offsets[i], ens.offsets[i + 1])
            assert comp_rel(outs[p][:, sl], outs[0][:, sl]) <= TOL_STAGE, (p, i)
    s.close()


def test_batch_step_extreme_lengths():
    """Smallest and largest problems, both kernel shapes, in one batch."""
    pp = gpu()
    lengths = np.array([4096, 3, 2048, 2049, 17, 5], dtype=np.int64)
    rng = np.random.default_rng(5)
    Us, dxs = [], []
    for n in lengths:
        x = W.cell_centres(0.0, 1.0, int(n))
        rho = 1.0 + 0.5 * (x > 0.5) + 0.05 * rng.standard_normal(int(n)) ** 2
        p = 1.0 - 0.9 * (x > 0.5)
        Us.append(W.prim_to_cons_1d(rho, 0.3 * np.sin(6 * x), p, 1.4))
        dxs.append(1.0 / n)
    U = np.concatenate(Us, axis=1)
    nb = len(lengths)
    dts = np.array([(1.0 / 12.0) * dxs[i] / oracle.max_speed_1d(Us[i]) for i in range(nb)])
    print(f"case batch extreme lengths {list(lengths)}", flush=True)
    s = pp.Solver(ndim=1, lengths=lengths, dxs=np.array(dxs), bcs=[1, 2] * nb)
    for plan in (0, 1):
        s.batch_tune(force_plan=plan)
        Ud = dev(U)
        s.batch_step(Ud, dev(dts))
        got = Ud.cpu().numpy()
        off = 0
        for i in range(nb):
            sl = slice(off, off + int(lengths[i]))
            off += int(lengths[i])
            h = dxs[i]
            U1 = oracle.stage_1d(Us[i], Us[i], 1, dts[i], (1, 2), h)
            U2 = oracle.stage_1d(Us[i], U1, 2, dts[i], (1, 2), h)
            U3 = oracle.stage_1d(Us[i], U2, 3, dts[i], (1, 2), h)
            err = comp_rel(got[:, sl], U3)
            if err > TOL_STAGE:   # the 3-cell line has a limited state on e = eps
                tol = step_tolerance(Us[i], dts[i], (1, 2), h, U3)
                print(f"plan {plan} problem {i}: err {err:.2e}, conditioning bound {tol:.2e}",
                      flush=True)
                assert err <= tol, (plan, i)
    s.close()


@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (2, 2), (1, 2)])
def test_1d_free_stream(bc):
    """A uniform state is steady: |L| h stays at rounding of |F| (walls need
    zero normal velocity)."""
    pp = gpu()
    n = 300
    u = 0.0 if 2 in bc else 0.4
    U = W.prim_to_cons_1d(np.full(n, 1.3), np.full(n, u), np.full(n, 2.0), 1.4)
    s = pp.Solver(ndim=1, nx=n, dx=1.0 / n, bc=(*bc, 0, 0))
    Ud = dev(U)
    L = torch.empty_like(Ud)
    s.rhs(Ud, L)
    torch.cuda.synchronize()
    F = max(abs(1.3 * u), 1.3 * u * u + 2.0, abs(u * (U[2, 0] + 2.0)))
    assert np.abs(L.cpu().numpy()).max() / n <= 1e-13 * F
    s.close()


@pytest.mark.parametrize("nx,ny,bc", [(40, 24, (0, 0, 0, 0)), (33, 17, (1, 1, 2, 2))])
def test_2d_free_stream(nx, ny, bc):
    pp = gpu()
    U = np.empty((4, ny, nx))
    U[0] = 1.3
    U[1] = 1.3 * 0.4 if bc[0] != 2 else 0.0
    U[2] = 1.3 * -0.2 if bc[2] != 2 else 0.0
    U[3] = 2.0 / 0.4 + 0.5 * (U[1] ** 2 + U[2] ** 2) / 1.3
    s = pp.Solver(ndim=2, nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / ny, bc=bc)
    Ud = dev(U)
    L = torch.empty_like(Ud)
    s.rhs(Ud, L)
    torch.cuda.synchronize()
    assert np.abs(L.cpu().numpy()).max() * min(1.0 / nx, 1.0 / ny) <= 1e-13 * 10.0
    s.close()


def test_batch_run_matches_oracle_driver():
    """The graph-replayed batched driver (per-problem dt from its own wave
    speeds, last step clipped) against the oracle's per-problem driver."""
    pp = gpu()
    ens = ensemble(12, 32, 160, seed=7)
    nb = len(ens.lengths)
    s = pp.Solver(ndim=1, lengths=ens.lengths, dxs=ens.dx, bcs=[1] * (2 * nb))
    Ud = dev(ens.U)
    t_end = 0.03
    try:
        steps = s.batch_run(Ud, t_end, 10 ** 6, 1.0 / 12.0)
        flagged = False
    except pp.PPError as e:
        # problem 10 of this seed (rho 9.69 | 0.015, p 0.002 | 5.3) leaves G in
        # a stage on the oracle as well: the status report must say so
        assert e.code == pp.PP_ESTATE
        flagged = True
        steps = s.last_batch_steps()
    assert flagged
    torch.cuda.synchronize()
    got = Ud.cpu().numpy()
    ref, ref_steps = oracle.run_batch(ens, t_end=t_end)
    compared = 0
    for i in range(nb):
        sl = slice(ens.offsets[i], ens.offsets[i + 1])
        _, info = oracle.run_1d(ens.U[:, sl], (1, 1), ens.dx[i], t_end)
        if not (info["min_rho"] > 0 and info["min_p"] > 0):
            continue   # outside G the two roundings need not stay together
        compared += 1
        assert steps[i] == int(ref_steps[i]), (i, steps[i], ref_steps[i])
        # accumulated over every step of the run
        assert comp_rel(got[:, sl], ref[:, sl]) <= 1e-10, i
    assert compared >= 10
    s.close()


# ------------------------------------------------- full sizes / whole runs
@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 2, 2, 1), (2, 2, 1, 1)])
def test_2d_2048_stage_sampled_parity(bc):
    """The benchmarked 2048^2 grid, one stage, in the bench's launch
    configuration (every lane of a line holds 16 rows); the oracle evaluates
    sampled cells one by one from the row and column line operators (with
    the grid-wide limiter epsilon).  Periodic as benchmarked, and closed
    lines with transmissive and reflective ends (closure rows, image states
    and the normal-momentum sign in both directions), sampled also at the
    edges."""
    pp = gpu()
    n = 2048
    dx = 2.0 / n
    U = W.density_wave_2d(n, n)
    # add a blob and a contact so the weights are not all linear
    yy, xx = np.mgrid[0:n, 0:n]
    U[0] += 0.3 * (((xx - 700) ** 2 + (yy - 900) ** 2) < 200 ** 2)
    sx, sy = oracle.max_speed_2d(U)
    dt = (1.0 / 12.0) / (sx / dx + sy / dx)
    print(f"2048^2 stage parity, bc {bc}", flush=True)
    s = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=bc)
    Ud = dev(U)
    out = torch.empty_like(Ud)
    s.stage(Ud, Ud, out, 1, dt)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    er, ee = oracle.eps(U)
    rng = np.random.default_rng(5)
    pts = [(int(y), int(x)) for y, x in rng.integers(0, n, size=(12, 2))] + [(900, 500), (700, 700)]
    if bc[0] != 0:
        pts += [(0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1), (1, 2), (n - 2, n - 3), (1000, 1)]
    for (y, x) in pts:
        Lx = oracle.line_op(np.ascontiguousarray(U[:, y, :]), bc[0], bc[1], dx, eps_rho=er,
                            eps_e=ee, nrm=1)
        Ly = oracle.line_op(np.ascontiguousarray(U[:, :, x]), bc[2], bc[3], dx, eps_rho=er,
                            eps_e=ee, nrm=2)
        ref = U[:, y, x] + dt * (Lx[:, x] + Ly[:, y])
        scale = np.abs(U).reshape(4, -1).max(axis=1)
        assert np.all(np.abs(got[:, y, x] - ref) <= TOL_STAGE * scale), (y, x)
    s.close()


@pytest.mark.parametrize("recon,bc", [(1, (0, 0, 0, 0)), (2, (1, 2, 2, 1))])
def test_2d_2048_stage_sampled_parity_explicit(recon, bc):
    """The explicit schemes at the 2048^2 size the accuracy comparison runs
    (single-segment staging, one workgroup per CU), one stage, sampled cells
    against the oracle's row and column operators with the same
    reconstruction."""
    pp = gpu()
    n = 2048
    dx = 2.0 / n
    U = W.density_wave_2d(n, n)
    yy, xx = np.mgrid[0:n, 0:n]
    U[0] += 0.3 * (((xx - 700) ** 2 + (yy - 900) ** 2) < 200 ** 2)
    sx, sy = oracle.max_speed_2d(U)
    dt = (1.0 / 12.0) / (sx / dx + sy / dx)
    print(f"2048^2 explicit stage parity, recon {recon} bc {bc}", flush=True)
    s = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=bc, recon=recon)
    Ud = dev(U)
    out = torch.empty_like(Ud)
    s.stage(Ud, Ud, out, 1, dt)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    er, ee = oracle.eps(U)
    P = oracle.params(recon=recon)
    rng = np.random.default_rng(9)
    pts = [(int(y), int(x)) for y, x in rng.integers(0, n, size=(10, 2))] + [(900, 500)]
    pts += [(0, 0), (n - 1, n - 1), (1, 2)]
    scale = np.abs(U).reshape(4, -1).max(axis=1)
    for (y, x) in pts:
        Lx = oracle.line_op(np.ascontiguousarray(U[:, y, :]), bc[0], bc[1], dx, p=P, eps_rho=er,
                            eps_e=ee, nrm=1)
        Ly = oracle.line_op(np.ascontiguousarray(U[:, :, x]), bc[2], bc[3], dx, p=P, eps_rho=er,
                            eps_e=ee, nrm=2)
        ref = U[:, y, x] + dt * (Lx[:, x] + Ly[:, y])
        assert np.all(np.abs(got[:, y, x] - ref) <= TOL_STAGE * scale), (y, x)
    s.close()


@pytest.mark.parametrize("recon", [0, 1, 2])
def test_2d_run_matches_oracle_run(recon):
    """A whole 2D run through pp_cweno_run (device dt every step, the
    dimension-by-dimension sweeps and combine; 210 steps to t = 0.1 on a
    48 x 40 grid with transmissive and reflective ends, a blob, shears and a
    pressure jump) against the oracle's run, for the compact scheme and both
    explicit ones: equal step counts and times, states within 1e-11."""
    pp = gpu()
    nx, ny, bc = 48, 40, (1, 2, 2, 1)
    x = W.cell_centres(0, 1, nx)[None, :]
    y = W.cell_centres(0, 1, ny)[:, None]
    rho = 1 + 0.3 * np.sin(2 * np.pi * (x + 2 * y)) + 0.5 * ((x - 0.5) ** 2 + (y - 0.4) ** 2 < 0.06)
    u = 0.3 * np.cos(2 * np.pi * y) + 0 * x
    v = -0.2 * np.sin(2 * np.pi * x) + 0 * y
    p = 1 + 0.5 * (x > 0.6) + 0 * y
    U = np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    print(f"2D run recon={recon}", flush=True)
    s = pp.Solver(ndim=2, nx=nx, ny=ny, dx=1.0 / nx, dy=1.0 / ny, bc=bc, recon=recon)
    Ud = dev(U)
    t, steps = s.run(Ud, 0.1, 1 << 40, 1.0 / 12.0)
    torch.cuda.synchronize()
    ref, info = oracle.run_2d(U, bc, 1.0 / nx, 1.0 / ny, 0.1, p=oracle.params(recon=recon))
    assert steps == info["steps"] and abs(t - info["t"]) <= 1e-13
    assert comp_rel(Ud.cpu().numpy(), ref) <= 1e-11
    s.close()


def test_1d_density_wave_full_run():
    """Example 3.1 at N = 200 to t = 2 with dt = w1 h^(5/3) / max(|u|+a):
    ~120k steps through pp_cweno_run against the oracle's run."""
    pp = gpu()
    n = 200
    h = 2.0 / n
    U0 = W.density_wave_1d(n)
    ref, info = oracle.run_1d(U0, (0, 0), h, 2.0, cfl=1.0 / 12.0, rule=1)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(0, 0, 0, 0))
    Ud = dev(U0)
    t, steps = s.run(Ud, 2.0, 10 ** 7, 1.0 / 12.0, pp.PP_DT_H53)
    torch.cuda.synchronize()
    assert steps == info["steps"] and abs(t - info["t"]) <= 1e-12
    got = Ud.cpu().numpy()
    assert comp_rel(got, ref) <= 1e-10
    ex = W.density_wave_1d(n, t=t)
    l1g = W.error_norms(got[0], ex[0], h)[0]
    l1o = W.error_norms(ref[0], ex[0], h)[0]
    # the rounding difference of the two runs (~1e-11 after 120k steps) is of
    # the size of the discretisation error, so compare through the triangle
    # inequality: |L1(gpu) - L1(oracle)| <= (b - a) max |gpu - oracle|
    assert abs(l1g - l1o) <= 2.0 * np.abs(got[0] - ref[0]).max() + 1e-15
    assert l1o < 2e-10
    s.close()


@pytest.mark.parametrize("nsteps", [0, 10, 25])
def test_1d_vacuum_blast_stage_parity(nsteps):
    """Near-vacuum blast (N = 4000): per-stage parity on oracle snapshots
    (limiter active at the blast)."""
    pp = gpu()
    n = 4000
    h = 2.0 / n
    U, info = oracle.run_1d(W.vacuum_blast_1d(n), (1, 1), h, 1.0, max_steps=nsteps)
    dt = (1.0 / 12.0) * h / oracle.max_speed_1d(U)
    U1 = oracle.stage_1d(U, U, 1, dt, (1, 1), h)
    U2 = oracle.stage_1d(U, U1, 2, dt, (1, 1), h)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(1, 1, 0, 0))
    Ud = dev(U)
    o1, o2 = torch.empty_like(Ud), torch.empty_like(Ud)
    s.stage(Ud, Ud, o1, 1, dt)
    s.stage(Ud, dev(U1), o2, 2, dt)
    torch.cuda.synchronize()
    assert comp_rel(o1.cpu().numpy(), U1) <= TOL_STAGE
    assert comp_rel(o2.cpu().numpy(), U2) <= TOL_STAGE
    s.close()


def test_1d_vacuum_blast_run():
    """Whole-run behaviour: 30 steps stay in G and track the oracle (the
    blast's rows with omega0 -> 1 amplify roundoff, so the accumulated
    difference is bounded loosely); by step 60 the component-wise scheme has
    left G at the evacuated centre, as in the oracle, and the run reports
    PP_ESTATE."""
    pp = gpu()
    n = 4000
    h = 2.0 / n
    U0 = W.vacuum_blast_1d(n)
    ref, info = oracle.run_1d(U0, (1, 1), h, 1.0, max_steps=30)
    assert info["min_p"] > 0 and info["limited"] > 0
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(1, 1, 0, 0))
    Ud = dev(U0)
    t, steps = s.run(Ud, 1.0, 30)
    torch.cuda.synchronize()
    assert steps == 30 and abs(t / info["t"] - 1) < 1e-10
    got = Ud.cpu().numpy()
    print("blast 30-step relative difference per component:",
          [rel(got[k], ref[k]) for k in range(3)], flush=True)
    assert comp_rel(got, ref) <= 1e-6
    Ud = dev(U0)
    with pytest.raises(pp.PPError) as e:
        s.run(Ud, 1.0, 60)
    assert e.value.code == pp.PP_ESTATE
    s.close()


def test_1d_double_rarefaction_4000_run():
    """The N = 4000 double rarefaction of the positivity stress case, through
    pp_cweno_run (the whole-run kernel with device dt) to t = 0.05 (1441
    steps, the limiter acting on ~7700 cell-stages near the evacuated
    centre), against the oracle's run: equal step counts and times, relative
    L1 differences per component within 1e-9, positivity."""
    pp = gpu()
    n = 4000
    h = 2.0 / n
    U0 = W.double_rarefaction_1d(n)
    ref, info = oracle.run_1d(U0, (1, 1), h, 0.05)
    assert info["limited"] > 0
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(1, 1, 0, 0))
    Ud = dev(U0)
    t, steps = s.run(Ud, 0.05, 1 << 40)
    torch.cuda.synchronize()
    got = Ud.cpu().numpy()
    assert steps == info["steps"] and abs(t - info["t"]) <= 1e-14
    d = [float(np.abs(got[k] - ref[k]).sum() / np.abs(ref[k]).sum()) for k in range(3)]
    print(f"double rarefaction relative L1 differences {d}", flush=True)
    assert max(d) <= 1e-9
    assert got[0].min() > 0 and W.pressure(got).min() > 0
    s.close()


def test_1d_double_rarefaction_4000_to_t_end():
    """The same configuration to its end time t = 0.6 (17 281 steps) against
    the oracle's run stored by tests/golden/make_rarefaction_0p6.py: equal
    step counts and times, positivity, and per-component relative L1
    differences within 1e4 times the oracle's own spread under 1e-15 input
    perturbations (about 2e-13)."""
    import os
    pp = gpu()
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "rarefaction_4000_t0p6.npz"))
    n = 4000
    h = 2.0 / n
    U0 = W.double_rarefaction_1d(n)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(1, 1, 0, 0))
    Ud = dev(U0)
    t, steps = s.run(Ud, 0.6, 1 << 40)
    torch.cuda.synchronize()
    got = Ud.cpu().numpy()
    U = ref["U"]
    assert steps == int(ref["steps"]) and abs(t - float(ref["t"])) <= 1e-14
    d = np.array([np.abs(got[k] - U[k]).sum() / np.abs(U[k]).sum() for k in range(3)])
    print(f"double rarefaction to t = 0.6: relative L1 differences {d}, oracle spread "
          f"{ref['spread']}", flush=True)
    assert np.all(d <= 1e4 * np.maximum(ref["spread"], 1e-16))
    assert got[0].min() > 0 and W.pressure(got).min() > 0
    s.close()


def mirror(U):
    """Diagonal mirror of a 2D state: x and y exchanged, with the momenta."""
    return np.ascontiguousarray(U[[0, 2, 1, 3]].transpose(0, 2, 1))


@pytest.mark.parametrize("fv,bc", [(0, (2, 1, 2, 1)), (0, (0, 0, 0, 0)), (1, (2, 1, 2, 1)),
                                   (1, (1, 2, 1, 2))])
def test_2d_mirror_symmetry_is_exact(fv, bc):
    """A state symmetric under the diagonal mirror stays exactly (bitwise)
    symmetric through 40 SSP-RK3 steps of the FP64 2D path: the x-sweep of a
    row and the y-sweep of the mirrored column perform the same arithmetic
    (sums of squared momenta taken normal component first), and the combine
    adds L_x + L_y commutatively.  Corner blast into a near-vacuum background
    with a symmetrised perturbation; the limiter acts."""
    pp = gpu()
    n = 96
    dx = 1.1 / n
    U = W.sedov_corner_2d(n)
    rng = np.random.default_rng(11)
    U[0] *= 1.0 + 0.05 * rng.random((n, n))
    mx = 1e-6 * rng.standard_normal((n, n))   # kinetic energy ~1e-12, inside G
    U[1] += mx
    U[3] += 0.5 * mx * mx / U[0]
    U = 0.5 * (U + mirror(U))
    assert np.array_equal(U, mirror(U)) and W.pressure(U).min() > 0
    s = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=bc, fv=fv)
    Ud = dev(U)
    try:
        t, steps = s.run(Ud, 1e30, 40)
    except pp.PPError as e:   # a stage left G: symmetry still applies to what ran
        print(f"run stopped: {e}", flush=True)
    torch.cuda.synchronize()
    got = Ud.cpu().numpy()
    assert np.all(np.isfinite(got))
    diff = np.abs(got - mirror(got)).max()
    print(f"fv={fv} bc={bc}: max |U - mirror(U)| = {diff:.3e}", flush=True)
    assert diff == 0.0
    s.close()


# --------------------------------------------------------- mixed precision
TOL_MIXED_STAGE = 1e-6   # per stage output, relative: float weights/rows/HLLC


@pytest.mark.parametrize("n,bc,tol", [(256, (0, 0), 1e-11), (2048, (0, 0), 1e-11),
                                      (1000, (1, 2), 1e-6), (3000, (1, 1), 1e-6)])
def test_mixed_refined_interface_states(n, bc, tol):
    """Mixed path: float weights and chasing plus one refinement sweep whose
    residual uses double rows built from the same float weights.  On a smooth
    periodic line the float weights barely move the reconstruction (the
    candidates agree), so the refined nodal values match the FP64 oracle to
    ~1e-13; a float solve without the sweep is off by ~1e-7.  Next to a
    non-periodic boundary the ghost extension makes a kink where float weights
    from float-rounded averages move the reconstruction by ~1e-8 (the stated
    mixed-precision bound is checked there)."""
    pp = gpu()
    h = 1.0 / n
    x = W.cell_centres(0, 1, n)
    U = W.prim_to_cons_1d(1 + 0.2 * np.sin(2 * np.pi * x), 0.3 + 0.1 * np.cos(2 * np.pi * x),
                          1 + 0.1 * np.sin(4 * np.pi * x), 1.4)
    _, dbg = oracle.line_op(U, bc[0], bc[1], h, debug=True)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(*bc, 0, 0), precision=pp.PP_MIXED)
    Ud = dev(U)
    um, up = torch.empty_like(Ud), torch.empty_like(Ud)
    s.debug_line(Ud, um, up)
    torch.cuda.synchronize()
    e1 = comp_rel(um.cpu().numpy(), dbg["um"])
    e2 = comp_rel(up.cpu().numpy(), dbg["up"])
    print(f"mixed interface states n={n} bc={bc}: {e1:.2e} {e2:.2e}", flush=True)
    assert e1 <= tol and e2 <= tol
    s.close()


@pytest.mark.parametrize("n,bc", [(200, (1, 2)), (2048, (0, 0)), (4000, (1, 1))])
def test_mixed_stage_bound(n, bc):
    pp = gpu()
    h = 1.0 / n
    U = mixed_line(n, seed=11 * n)
    dt = (1.0 / 12.0) * h / oracle.max_speed_1d(U)
    ref = oracle.stage_1d(U, U, 1, dt, bc, h)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(*bc, 0, 0), precision=pp.PP_MIXED)
    Ud = dev(U)
    out = torch.empty_like(Ud)
    s.stage(Ud, Ud, out, 1, dt)
    torch.cuda.synchronize()
    e = comp_rel(out.cpu().numpy(), ref)
    print(f"mixed stage n={n}: {e:.2e}", flush=True)
    assert e <= TOL_MIXED_STAGE
    s.close()


def test_mixed_2d_step_bound_and_conservation():
    pp = gpu()
    n = 64
    dx = 2.0 / n
    U = W.density_wave_2d(n, n)
    sx, sy = oracle.max_speed_2d(U)
    dt = (1.0 / 12.0) / (sx / dx + sy / dx)
    ref = U
    for st in (1, 2, 3):
        ref = oracle.stage_2d(U, ref, st, dt, (0, 0, 0, 0), dx, dx)
    s = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=(0, 0, 0, 0), precision=pp.PP_MIXED)
    Ud = dev(U)
    s.step(Ud, dt)
    torch.cuda.synchronize()
    got = Ud.cpu().numpy()
    assert comp_rel(got, ref) <= TOL_MIXED_STAGE
    np.testing.assert_allclose(got.sum(axis=(1, 2)), U.sum(axis=(1, 2)), rtol=1e-13)
    s.close()


def test_2d_timing_events_cover_every_launch():
    """pp_cweno_set_timing / get_timing on a 2D run: each of the three
    kernel classes is timed once per stage (three per step), the chained
    events of a step give positive durations, and their sum fits inside the
    wall time of the run."""
    import time
    pp = gpu()
    n = 256
    dx = 2.0 / n
    U = dev(W.density_wave_2d(n, n))
    s = pp.Solver(ndim=2, nx=n, ny=n, dx=dx, dy=dx, bc=(0, 0, 0, 0))
    s.run(U, 1e30, 2, 1.0 / 12.0)
    torch.cuda.synchronize()
    s.set_timing(True)
    t0 = time.perf_counter()
    t, steps = s.run(U, 1e30, 7, 1.0 / 12.0)
    torch.cuda.synchronize()
    wall_ms = 1e3 * (time.perf_counter() - t0)
    tm = s.get_timing()
    s.set_timing(False)
    s.close()
    assert steps == 7
    # the run launches one retired step beyond the last (it returns at once)
    for k in ("x", "y", "combine"):
        ms, launches = tm[k]
        assert launches in (21, 24), (k, launches)
        assert ms > 0.0
    assert sum(ms for ms, _ in tm.values()) < wall_ms


@pytest.mark.parametrize("n,bc", [(200, (1, 2)), (777, (2, 2)), (2048, (0, 0)), (2048, (1, 2)),
                                  (4000, (1, 1))])
def test_1d_stage_parity_lax_friedrichs(n, bc):
    """The Lax-Friedrichs flux option (PP_FLUX_LF) through all three stages,
    against the oracle with the same flux: the paired full-chunk path
    (2048), the general paired path and the two-wave long-line path (4000)."""
    pp = gpu()
    print(f"case lf n={n} bc={bc}", flush=True)
    h = 1.0 / n
    U = mixed_line(n, seed=n + 7)
    dt = (1.0 / 12.0) * h / oracle.max_speed_1d(U)
    P = oracle.params(flux=1)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(*bc, 0, 0), flux=pp.PP_FLUX_LF)
    Ud = dev(U)
    U1 = oracle.stage_1d(U, U, 1, dt, bc, h, P)
    U2 = oracle.stage_1d(U, U1, 2, dt, bc, h, P)
    U3 = oracle.stage_1d(U, U2, 3, dt, bc, h, P)
    o1, o2, o3 = (torch.empty_like(Ud) for _ in range(3))
    s.stage(Ud, Ud, o1, 1, dt)
    s.stage(Ud, dev(U1), o2, 2, dt)
    s.stage(Ud, dev(U2), o3, 3, dt)
    torch.cuda.synchronize()
    for st, (got, ref) in enumerate(((o1, U1), (o2, U2), (o3, U3)), start=1):
        err = comp_rel(got.cpu().numpy(), ref)
        assert err <= TOL_STAGE, (st, err)
    # the flux option changes the result (the two fluxes differ at the jumps)
    Uh = oracle.stage_1d(U, U, 1, dt, bc, h)
    assert comp_rel(Uh, U1) > 1e-8
    s.close()


def test_2d_stage_parity_lax_friedrichs():
    """2D sweeps and combine with the Lax-Friedrichs flux (both normal
    directions, reflective and transmissive ends)."""
    pp = gpu()
    nx, ny, bc = 48, 40, (1, 2, 2, 1)
    x = W.cell_centres(0, 1, nx)[None, :]
    y = W.cell_centres(0, 1, ny)[:, None]
    rho = 1 + 0.3 * np.sin(2 * np.pi * (x + 2 * y)) + 0.5 * ((x - 0.5) ** 2 + (y - 0.4) ** 2 < 0.06)
    u = 0.3 * np.cos(2 * np.pi * y) + 0 * x
    v = -0.2 * np.sin(2 * np.pi * x) + 0 * y
    p = 1 + 0.5 * (x > 0.6) + 0 * y
    U = np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    dx, dy = 1.0 / nx, 1.0 / ny
    s_x, s_y = oracle.max_speed_2d(U)
    dt = (1.0 / 12.0) / (s_x / dx + s_y / dy)
    P = oracle.params(flux=1)
    s = pp.Solver(ndim=2, nx=nx, ny=ny, dx=dx, dy=dy, bc=bc, flux=pp.PP_FLUX_LF)
    Ud = dev(U)
    ref1 = oracle.stage_2d(U, U, 1, dt, bc, dx, dy, P)
    o1 = torch.empty_like(Ud)
    s.stage(Ud, Ud, o1, 1, dt)
    torch.cuda.synchronize()
    assert comp_rel(o1.cpu().numpy(), ref1) <= TOL_STAGE
    s.close()


def test_flux_option_is_validated():
    pp = gpu()
    with pytest.raises(pp.PPError):
        pp.Solver(ndim=1, nx=64, dx=1.0 / 64, bc=(0, 0, 0, 0), flux=2)


@pytest.mark.parametrize("n,bc", [(200, (1, 2)), (2048, (0, 0)), (4000, (1, 1))])
def test_mixed_stage_bound_lax_friedrichs(n, bc):
    """Mixed precision with the Lax-Friedrichs flux (evaluated in double):
    one stage within the mixed-precision bound of the FP64 oracle with the
    same flux."""
    pp = gpu()
    h = 1.0 / n
    U = mixed_line(n, seed=13 * n)
    dt = (1.0 / 12.0) * h / oracle.max_speed_1d(U)
    ref = oracle.stage_1d(U, U, 1, dt, bc, h, oracle.params(flux=1))
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(*bc, 0, 0), precision=pp.PP_MIXED,
                  flux=pp.PP_FLUX_LF)
    Ud = dev(U)
    out = torch.empty_like(Ud)
    s.stage(Ud, Ud, out, 1, dt)
    torch.cuda.synchronize()
    e = comp_rel(out.cpu().numpy(), ref)
    print(f"mixed lf stage n={n}: {e:.2e}", flush=True)
    assert e <= TOL_MIXED_STAGE
    s.close()


@pytest.mark.parametrize("recon", [1, 2])
@pytest.mark.parametrize("n,bc", [(5, (0, 0)), (7, (1, 2)), (200, (2, 1)), (2048, (0, 0)),
                                  (3000, (1, 1))])
def test_1d_stage_parity_explicit(recon, n, bc):
    """The explicit comparison schemes (PP_RECON_WENOJS / _WENOZ): all three
    stages against the oracle with the same reconstruction, on short,
    ragged, full single-wave and two-wave lines with every boundary kind."""
    pp = gpu()
    print(f"case explicit recon={recon} n={n} bc={bc}", flush=True)
    h = 1.0 / n
    U = mixed_line(n, seed=n + 31)
    dt = (1.0 / 12.0) * h / oracle.max_speed_1d(U)
    P = oracle.params(recon=recon)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(*bc, 0, 0), recon=recon)
    Ud = dev(U)
    U1 = oracle.stage_1d(U, U, 1, dt, bc, h, P)
    U2 = oracle.stage_1d(U, U1, 2, dt, bc, h, P)
    U3 = oracle.stage_1d(U, U2, 3, dt, bc, h, P)
    o1, o2, o3 = (torch.empty_like(Ud) for _ in range(3))
    s.stage(Ud, Ud, o1, 1, dt)
    s.stage(Ud, dev(U1), o2, 2, dt)
    s.stage(Ud, dev(U2), o3, 3, dt)
    torch.cuda.synchronize()
    for st, (got, ref) in enumerate(((o1, U1), (o2, U2), (o3, U3)), start=1):
        err = comp_rel(got.cpu().numpy(), ref)
        assert err <= TOL_STAGE, (st, err)
    # a different scheme from the compact one
    assert comp_rel(oracle.stage_1d(U, U, 1, dt, bc, h), U1) > 1e-8
    s.close()


@pytest.mark.parametrize("recon", [1, 2])
@pytest.mark.parametrize("nx,ny,bc", [(48, 40, (1, 2, 2, 1)), (64, 64, (0, 0, 0, 0))])
def test_2d_stage_parity_explicit(recon, nx, ny, bc):
    """2D sweeps and combine with the explicit schemes."""
    pp = gpu()
    x = W.cell_centres(0, 1, nx)[None, :]
    y = W.cell_centres(0, 1, ny)[:, None]
    rho = 1 + 0.3 * np.sin(2 * np.pi * (x + 2 * y)) + 0.5 * ((x - 0.5) ** 2 + (y - 0.4) ** 2 < 0.06)
    u = 0.3 * np.cos(2 * np.pi * y) + 0 * x
    v = -0.2 * np.sin(2 * np.pi * x) + 0 * y
    p = 1 + 0.5 * (x > 0.6) + 0 * y
    U = np.stack([rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)])
    dx, dy = 1.0 / nx, 1.0 / ny
    s_x, s_y = oracle.max_speed_2d(U)
    dt = (1.0 / 12.0) / (s_x / dx + s_y / dy)
    P = oracle.params(recon=recon)
    s = pp.Solver(ndim=2, nx=nx, ny=ny, dx=dx, dy=dy, bc=bc, recon=recon)
    Ud = dev(U)
    ref1 = oracle.stage_2d(U, U, 1, dt, bc, dx, dy, P)
    ref2 = oracle.stage_2d(U, ref1, 2, dt, bc, dx, dy, P)
    o1, o2 = torch.empty_like(Ud), torch.empty_like(Ud)
    s.stage(Ud, Ud, o1, 1, dt)
    s.stage(Ud, dev(ref1), o2, 2, dt)
    torch.cuda.synchronize()
    assert comp_rel(o1.cpu().numpy(), ref1) <= TOL_STAGE
    assert comp_rel(o2.cpu().numpy(), ref2) <= TOL_STAGE
    s.close()


def test_explicit_wenojs_run_matches_oracle_and_table2():
    """A whole 1D run with the explicit WENO-JS scheme (Example 3.1, N = 60,
    lambda max(|u|+a) = 0.16, t = 2) through pp_cweno_run: the same step
    count and final time as the oracle's run, the state within 1e-11, and
    the L1 error within 2 % of Table 2's printed WENO-JS value."""
    import json
    import os
    pp = gpu()
    n = 60
    h = 2.0 / n
    U0 = W.density_wave_1d(n)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(0, 0, 0, 0), recon=pp.PP_RECON_WENOJS)
    Ud = dev(U0)
    t, steps = s.run(Ud, 2.0, 1 << 40, 0.16, pp.PP_DT_CFL)
    torch.cuda.synchronize()
    got = Ud.cpu().numpy()
    ref, info = oracle.run_1d(U0, (0, 0), h, 2.0, cfl=0.16, rule=0,
                              p=oracle.params(recon=1))
    assert steps == info["steps"] and abs(t - info["t"]) <= 1e-13
    assert comp_rel(got, ref) <= 1e-11
    with open(os.path.join(os.path.dirname(__file__), "golden",
                           "table2_wenojs_conservative.json")) as f:
        printed = {r[0]: r for r in json.load(f)["rows"]}[n][1]
    l1 = W.error_norms(got[0], W.density_wave_1d(n, t=t)[0], h)[0]
    assert abs(l1 / printed - 1) < 0.02, (l1, printed)
    s.close()


def test_max_speed_entry_point():
    """pp_cweno_max_speed: max(|u|+a) over the cell averages (2D: and
    max(|v|+a)) against the oracle's reductions, 1D and 2D."""
    pp = gpu()
    n = 777
    U = mixed_line(n, seed=5)
    s = pp.Solver(ndim=1, nx=n, dx=1.0 / n, bc=(1, 1, 0, 0))
    out = torch.zeros(2, dtype=torch.float64, device="cuda")
    s.max_speed(dev(U), out)
    torch.cuda.synchronize()
    ref = oracle.max_speed_1d(U)
    assert abs(out[0].item() - ref) <= 1e-14 * ref
    s.close()
    nx, ny = 40, 24
    U2 = W.density_wave_2d(nx, ny)
    U2[1] *= 1.7   # make the two directions differ
    s = pp.Solver(ndim=2, nx=nx, ny=ny, dx=2.0 / nx, dy=2.0 / ny, bc=(0, 0, 0, 0))
    s.max_speed(dev(U2), out)
    torch.cuda.synchronize()
    rx, ry = oracle.max_speed_2d(U2)
    assert abs(out[0].item() - rx) <= 1e-14 * rx and abs(out[1].item() - ry) <= 1e-14 * ry
    s.close()


def test_batch_continue_equals_one_run():
    """pp_cweno_batch_continue: a run cut into pieces (5 steps, then to 12,
    then to t_end) ends bitwise equal to the uninterrupted run, with the same
    per-problem step counts and times; it refuses to start without a run and
    after the tuner has reset the per-problem times.  Problems retire at
    different steps, so the two runs cut their launches down to the active
    problems at different points: the equality also shows that this cut
    changes no result and that the full order is restored after a run."""
    pp = gpu()
    # 48 mild Riemann problems (they stay in G), lengths across both classes
    rng = np.random.default_rng(7)
    lengths = rng.integers(64, 2600, size=48).astype(np.int64)
    parts = []
    for n in lengths:
        sl = (rng.uniform(0.5, 2.0), rng.uniform(-0.5, 0.5), rng.uniform(0.5, 2.0))
        sr = (rng.uniform(0.5, 2.0), rng.uniform(-0.5, 0.5), rng.uniform(0.5, 2.0))
        parts.append(W.riemann_1d(0.0, 1.0, int(n), 0.5, sl, sr))
    U0 = np.concatenate(parts, axis=1)
    nb, t_end = len(lengths), 0.01
    s = pp.Solver(ndim=1, lengths=lengths, dxs=1.0 / lengths.astype(np.float64), bcs=[1] * (2 * nb))
    with pytest.raises(pp.PPError):
        s.batch_continue(dev(U0), t_end, 10)
    U1 = dev(U0)
    steps1 = s.batch_run(U1, t_end, 1 << 40, 1.0 / 12.0)
    torch.cuda.synchronize()
    U2 = dev(U0)
    a = s.batch_run(U2, t_end, 5, 1.0 / 12.0)
    assert max(a) == 5
    b, tb = s.batch_continue(U2, t_end, 12, 1.0 / 12.0)
    assert max(b) == 12 and max(tb) < t_end
    c, tc = s.batch_continue(U2, t_end, 1 << 40, 1.0 / 12.0)
    torch.cuda.synchronize()
    assert c == steps1
    assert all(abs(t - t_end) <= 1e-15 for t in tc)
    assert torch.equal(U1, U2)
    s.batch_tune(force_plan=0)   # direct plan choice leaves the times alone
    s.batch_continue(U2, t_end, 1 << 40, 1.0 / 12.0)
    s.batch_tune(dev(U0), 1.0 / 12.0)   # timed tuning resets them
    with pytest.raises(pp.PPError):
        s.batch_continue(U2, t_end, 1 << 40, 1.0 / 12.0)
    s.close()


@pytest.mark.parametrize("ndim", [1, 2])
def test_runs_are_bitwise_reproducible(ndim):
    """Deterministic replay: every reduction on the path is a min or a max
    (order-independent), so two runs of the same problem end bitwise equal,
    and so do their step counts and times (1D: the whole-run kernel on the
    N = 4000 double rarefaction with the limiter active; 2D: 40 steps of the
    512^2 density wave with a blob)."""
    pp = gpu()
    if ndim == 1:
        n = 4000
        U0 = W.double_rarefaction_1d(n)
        s = pp.Solver(ndim=1, nx=n, dx=2.0 / n, bc=(1, 1, 0, 0))
        t_end, cap = 0.02, 1 << 40
    else:
        n = 512
        U0 = W.density_wave_2d(n, n)
        yy, xx = np.mgrid[0:n, 0:n]
        U0[0] += 0.3 * (((xx - 200) ** 2 + (yy - 300) ** 2) < 60 ** 2)
        s = pp.Solver(ndim=2, nx=n, ny=n, dx=2.0 / n, dy=2.0 / n, bc=(0, 0, 0, 0))
        t_end, cap = 1.0, 40
    outs = []
    for _ in range(2):
        Ud = dev(U0)
        t, steps = s.run(Ud, t_end, cap, 1.0 / 12.0)
        torch.cuda.synchronize()
        outs.append((Ud, t, steps))
    assert outs[0][1] == outs[1][1] and outs[0][2] == outs[1][2]
    assert torch.equal(outs[0][0], outs[1][0])
    s.close()


def test_status_reports_nonfinite_and_inadmissible_states():
    """Failure detection forced from the host: the sticky status word after
    a stage is clear on admissible data, has bit 0 after a non-finite input
    cell and bit 1 after a CFL violation that drives the output out of G
    (the oracle's stage with the same dt leaves G too), and is cleared by
    reading it; a run from a non-finite state stops with PP_ESTATE."""
    pp = gpu()
    n = 256
    h = 1.0 / n
    U = mixed_line(n, seed=3)
    dt = (1.0 / 12.0) * h / oracle.max_speed_1d(U)
    s = pp.Solver(ndim=1, nx=n, dx=h, bc=(1, 1, 0, 0))
    out = torch.empty((3, n), dtype=torch.float64, device="cuda")
    Ud = dev(U)
    s.stage(Ud, Ud, out, 1, dt)
    assert s.status() == (pp.PP_OK, 0)
    V = U.copy()
    V[0, 100] = np.nan
    Vd = dev(V)
    s.stage(Vd, Vd, out, 1, dt)
    code, flags = s.status()
    assert code == pp.PP_ESTATE and flags & 1
    assert s.status() == (pp.PP_OK, 0)          # reading clears it
    big = 100.0 * dt
    ref = oracle.stage_1d(U, U, 1, big, (1, 1), h)
    assert ref[0].min() < 0 or W.pressure(ref).min() < 0
    s.stage(Ud, Ud, out, 1, big)
    code, flags = s.status()
    assert code == pp.PP_ESTATE and flags & 2
    with pytest.raises(pp.PPError) as e:
        s.run(dev(V), 0.1, 100)
    assert e.value.code == pp.PP_ESTATE
    s.close()


def test_user_stream_and_caller_ownership():
    """Stream semantics and ownership at the boundary: a context made on a
    side stream (default priority) enqueues its stage there, and after that
    stream is synchronised the result equals the same stage on the default
    stream bitwise; closing the contexts leaves the caller's arrays intact."""
    pp = gpu()
    n = 512
    h = 1.0 / n
    U = mixed_line(n, seed=9)
    dt = (1.0 / 12.0) * h / oracle.max_speed_1d(U)
    Ud = dev(U)
    out_a = torch.empty_like(Ud)
    s0 = pp.Solver(ndim=1, nx=n, dx=h, bc=(1, 2, 0, 0))
    s0.stage(Ud, Ud, out_a, 1, dt)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        Us = Ud.clone()
        out_b = torch.empty_like(Us)
    s1 = pp.Solver(ndim=1, nx=n, dx=h, bc=(1, 2, 0, 0), stream=side.cuda_stream)
    s1.stage(Us, Us, out_b, 1, dt)
    side.synchronize()
    assert torch.equal(out_a, out_b)
    s1.close()
    s0.close()
    torch.cuda.synchronize()
    assert torch.equal(Us, Ud) and torch.equal(out_a, out_b)
    assert comp_rel(out_b.cpu().numpy(), oracle.stage_1d(U, U, 1, dt, (1, 2), h)) <= TOL_STAGE


def test_binding_rejects_wrong_sizes_before_any_launch():
    """The C ABI takes bare device pointers; the binding checks every array
    against the context's layout (and dtype, device, contiguity) and raises
    before anything is enqueued, leaving the context usable."""
    pp = gpu()
    n = 64
    s = pp.Solver(ndim=1, nx=n, dx=1.0 / n, bc=(1, 1, 0, 0))
    good = dev(mixed_line(n, seed=1))
    short = torch.zeros(3 * n - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        s.rhs(good, short)
    with pytest.raises(ValueError):
        s.step(torch.zeros(3 * n + 3, dtype=torch.float64, device="cuda"), 1e-4)
    with pytest.raises(ValueError):
        s.rhs(good.float(), torch.empty_like(good))
    with pytest.raises(ValueError):
        s.rhs(good.cpu(), torch.empty_like(good))
    with pytest.raises(ValueError):
        s.max_speed(good, torch.zeros(0, dtype=torch.float64, device="cuda"))
    L = torch.empty_like(good)
    s.rhs(good, L)            # still usable
    torch.cuda.synchronize()
    assert torch.isfinite(L).all()
    s.close()
    ens = W.riemann_ensemble(nprob=4, seed=3, n_lo=8, n_hi=20)
    sb = pp.Solver(ndim=1, lengths=ens.lengths, dxs=ens.dx, bcs=[1] * 8)
    with pytest.raises(ValueError):
        sb.batch_step(dev(ens.U), torch.zeros(3, dtype=torch.float64, device="cuda"))
    sb.close()


@pytest.mark.parametrize("n", [3, 4, 5, 7, 8, 16, 33, 100, 2048, 2049, 4096])
@pytest.mark.parametrize("kind", ["dominant", "weno", "cyclic"])
def test_tridiag_debug_solve_matches_dense(n, kind):
    """The device's chunked chasing with PCR of the separators
    (pp_cweno_tridiag_solve_debug), against a pivoted dense solve on small
    systems and the oracle's chasing on large ones: random diagonally
    dominant rows, rows built from WENO-Z weights of a line with jumps (not
    dominant where omega0 > 1/2), and cyclic systems."""
    pp = gpu()
    rng = np.random.default_rng(n + {"dominant": 0, "weno": 1, "cyclic": 2}[kind])
    if kind == "weno":
        u = np.where(np.arange(n) < n // 2, 0.0, 1.0) + 1e-3 * rng.normal(size=n)
        a, b, c = np.empty(n), np.empty(n), np.empty(n)
        for i in range(n):
            wm, _ = oracle.weights(u[[(i + k) % n for k in range(-2, 4)]])
            a[i], b[i], c[i] = (2 * wm[0] + wm[1]) / 3, (wm[0] + 2 * (wm[1] + wm[2])) / 3, wm[2] / 3
    else:
        a, c = rng.uniform(0, 1, n), rng.uniform(0, 1, n)
        b = a + c + rng.uniform(0.1, 1, n)
    r = rng.normal(size=n)
    cyclic = kind == "cyclic"
    if n <= 100:
        M = np.diag(b)
        for i in range(n):
            if i > 0 or cyclic:
                M[i, (i - 1) % n] += a[i]
            if i < n - 1 or cyclic:
                M[i, (i + 1) % n] += c[i]
        ref = oracle.dense_solve(M, r)
    else:
        ref = oracle.cyclic(a, b, c, r) if cyclic else oracle.thomas(a, b, c, r)
    s = pp.Solver(ndim=1, nx=8, dx=0.1, bc=(1, 1, 0, 0))
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    s.tridiag_solve_debug(dev(a), dev(b), dev(c), dev(r), x, cyclic=cyclic)
    torch.cuda.synchronize()
    s.close()
    err = float(np.abs(x.cpu().numpy() - ref).max() / np.abs(ref).max())
    print(f"tridiag n={n} {kind}: {err:.2e}", flush=True)
    assert err <= 1e-12
