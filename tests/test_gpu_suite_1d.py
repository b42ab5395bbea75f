"""The paper's 1D discontinuous suite (Examples 3.2-3.10) run to the final
times on the GPU through the C ABI (`pp_cweno_run`, the device-resident 1D
run), against the oracle's run of the same problem with the same time-step
rule (dt = w1 h / max(|u|+a) over the cell averages, w1 = 1/12), and
against the minima the paper prints for its positivity tests.

Trajectory agreement: the GPU reciprocals and square roots agree with the
oracle's divisions to rounding, and the limiter and the HLLC branch
decisions are continuous, so the final states stay close.  Measured
relative L1 differences are 7.8e-14 .. 4.2e-12, and 1.3e-9 on the strong
shock, where the pressures span eleven decades; the bounds below leave about
two decades of margin.  Step counts and final times must be equal.

The printed minima come from the paper's characteristic-variable
reconstruction; this path is component-wise, so they are soft references,
with the same bands as the oracle's own tests.
"""
import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
G53 = 5.0 / 3.0


def printed(case):
    with open(os.path.join(GOLD, "positivity_minima.json")) as f:
        return json.load(f)["cases"][case]


# name: (initial averages, (bc_lo, bc_hi), h, t_end, gamma, relative L1 bound)
CASES = {
    "lax": (lambda: W.lax_1d(200), (1, 1), 10.0 / 200, 1.4, 1.4, 1e-9),
    "sod": (lambda: W.sod_1d(100), (1, 1), 10.0 / 100, 2.0, 1.4, 1e-9),
    "shu_osher": (lambda: W.shu_osher_1d(200), (1, 1), 10.0 / 200, 1.8, 1.4, 1e-9),
    "woodward_colella": (lambda: W.woodward_colella_1d(200), (2, 2), 1.0 / 200, 0.038, 1.4, 1e-9),
    "low_density_123": (lambda: W.low_density_123_1d(400), (1, 1), 1.0 / 400, 0.1, 1.4, 1e-9),
    "strong_shock": (lambda: W.strong_shock_1d(200), (1, 1), 1.0 / 200, 2.5e-6, 1.4, 1e-7),
    "double_rarefaction": (lambda: W.double_rarefaction_1d(400), (1, 1), 0.005, 0.6, 1.4, 1e-9),
    "leblanc": (lambda: W.leblanc_1d(400), (1, 1), 9.0 / 400, 6.0, G53, 1e-9),
}


def gpu_run(U0, bc, h, T, gamma, flux=0, recon=0, rule=0):
    import torch
    import paper_1402_5618_amd as pp

    n = U0.shape[1]
    s = pp.Solver(ndim=1, nx=n, dx=h, gamma=gamma, bc=(bc[0], bc[1], 0, 0), flux=flux,
                  recon=recon)
    U = torch.tensor(U0, device="cuda")
    code = pp.PP_OK
    try:
        t, steps = s.run(U, T, 1 << 40, 1.0 / 12.0, rule)
    except pp.PPError as e:
        t, steps, code = None, None, e.code
    torch.cuda.synchronize()
    s.close()
    return U.cpu().numpy(), t, steps, code


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(CASES))
def test_suite_run_matches_oracle(name):
    make, bc, h, T, gamma, tol = CASES[name]
    U0 = make()
    print(f"case {name}: n={U0.shape[1]} t_end={T}", flush=True)
    Ug, t, steps, code = gpu_run(U0, bc, h, T, gamma)
    Uo, info = oracle.run_1d(U0, bc, h, T, p=oracle.params(gamma=gamma))
    assert code == 0, (name, code)
    assert steps == info["steps"], (steps, info["steps"])
    assert abs(t - info["t"]) <= 1e-12 * T
    assert np.all(np.isfinite(Ug))
    for c in range(3):
        d = np.abs(Ug[c] - Uo[c]).sum() / np.abs(Uo[c]).sum()
        assert d <= tol, (name, c, d)
    assert Ug[0].min() > 0 and W.pressure(Ug, gamma).min() > 0
    # conservation: transmissive ends pass fluxes, reflective ends carry
    # no mass or energy flux
    if bc == (2, 2):
        np.testing.assert_allclose(Ug[0].sum(), U0[0].sum(), rtol=1e-12)
        np.testing.assert_allclose(Ug[2].sum(), U0[2].sum(), rtol=1e-12)


@pytest.mark.gpu
@pytest.mark.parametrize("name,case,bands", [
    ("low_density_123", "low_density_123", {"rho": (0.5, 2.0), "e": (0.5, 2.0)}),
    ("strong_shock", "strong_shock", {"rho": (0.98, 1.02), "e": (0.98, 1.02)}),
    ("double_rarefaction", "double_rarefaction", {"rho": (1e-3, 1e3)}),
    ("leblanc", "leblanc", {"rho": (0.99, 1.01), "p": (0.99, 1.01)}),
])
def test_suite_printed_minima(name, case, bands):
    """Final minima against the printed ones (LeBlanc's second printed value
    is the right state's specific internal energy, as in the oracle test)."""
    make, bc, h, T, gamma, _ = CASES[name]
    Ug, t, steps, code = gpu_run(make(), bc, h, T, gamma)
    assert code == 0
    g = printed(case)
    got = {"rho": Ug[0].min(), "e": W.specific_internal_energy(Ug).min()}
    got["p"] = got["e"]
    for key, (lo, hi) in bands.items():
        ref = g["min_rho"] if key == "rho" else g.get("min_e", g.get("min_p"))
        assert lo < got[key] / ref < hi, (name, key, got[key], ref)


@pytest.mark.gpu
def test_planar_sedov_gpu_minima():
    """Example 3.9 (h = 0.005, t = 0.001), about 45 000 steps on the GPU.
    Under the cell-average time-step rule a few early steps leave G
    transiently (as in the oracle), so the run may report PP_ESTATE; the
    final state must be finite with the printed minima: density within
    0.5x-2x of 4.731e-3 and specific internal energy 1e-12."""
    import paper_1402_5618_amd as pp

    U0 = W.sedov_planar_1d(0.005)
    print(f"case planar_sedov: n={U0.shape[1]}", flush=True)
    Ug, t, steps, code = gpu_run(U0, (1, 1), 0.005, 1e-3, 1.4)
    assert code in (pp.PP_OK, pp.PP_ESTATE)
    assert np.all(np.isfinite(Ug)) and Ug[0].min() > 0
    g = printed("planar_sedov")
    assert 0.5 < Ug[0].min() / g["min_rho"] < 2.0
    assert abs(W.specific_internal_energy(Ug).min() / g["min_e"] - 1) < 0.01


@pytest.mark.gpu
def test_low_density_123_with_lax_friedrichs():
    """Example 3.6 with the Lax-Friedrichs flux, the option the paper names
    for damping oscillations of the HLLC run in the low-density centre: the
    run matches the oracle's run with the same flux and stays positive.
    (The paper omits those results; at N = 400 with component-wise
    reconstruction the oracle shows no reduction of the centre velocity
    variation, 0.543 with LF against 0.526 with HLLC, so none is asserted.)"""
    make, bc, h, T, gamma, tol = CASES["low_density_123"]
    U0 = make()
    Ug, t, steps, code = gpu_run(U0, bc, h, T, gamma, flux=1)
    Uo, info = oracle.run_1d(U0, bc, h, T, p=oracle.params(gamma=gamma, flux=1))
    assert code == 0 and steps == info["steps"]
    for c in range(3):
        d = np.abs(Ug[c] - Uo[c]).sum() / np.abs(Uo[c]).sum()
        assert d <= tol, (c, d)
    assert Ug[0].min() > 0 and W.pressure(Ug, gamma).min() > 0


@pytest.mark.gpu
@pytest.mark.parametrize("recon", [1, 2])
@pytest.mark.parametrize("name", ["sod", "shu_osher", "woodward_colella", "leblanc"])
def test_suite_explicit_schemes_match_oracle(name, recon):
    """The explicit WENO-JS (1) and WENO-Z (2) comparison schemes run to the
    final times of four suite examples (transmissive and reflective ends,
    gamma 1.4 and 5/3) through pp_cweno_run, against the oracle's runs with
    the same reconstruction: equal steps and times, the states within the
    suite's bound, positivity."""
    make, bc, h, T, gamma, tol = CASES[name]
    U0 = make()
    print(f"case {name} recon={recon}", flush=True)
    Ug, t, steps, code = gpu_run(U0, bc, h, T, gamma, recon=recon)
    Uo, info = oracle.run_1d(U0, bc, h, T, p=oracle.params(gamma=gamma, recon=recon))
    assert code == 0 and steps == info["steps"], (code, steps, info["steps"])
    assert abs(t - info["t"]) <= 1e-12 * T
    for c in range(3):
        d = np.abs(Ug[c] - Uo[c]).sum() / np.abs(Uo[c]).sum()
        assert d <= tol, (name, c, d)
    assert Ug[0].min() > 0 and W.pressure(Ug, gamma).min() > 0


ROUNDOFF_DECIDED = {"low_density_123"}


@pytest.mark.gpu
@pytest.mark.parametrize("name", list(CASES))
def test_suite_characteristic_matches_oracle(name):
    """The suite with the characteristic-wise reconstruction (Sec. 2.3), the
    paper's choice for these examples: GPU runs against the oracle's runs of
    the same reconstruction (equal steps and times, relative L1 within the
    case's bound, positivity)."""
    make, bc, h, T, gamma, tol = CASES[name]
    U0 = make()
    # Under the CFL rule the 123 problem's characteristic run leaves G or not
    # by roundoff: the oracle's own runs from initial data perturbed by 1e-15
    # leave it for 2 of 7 seeds.  That case runs the restart rule (both
    # sides), which keeps every run in G; its redone steps are again decided
    # by roundoff, so the step count is compared within 2 %.
    rule = oracle.DT_RESTART if name in ROUNDOFF_DECIDED else oracle.DT_CFL
    print(f"case {name} (characteristic): n={U0.shape[1]} t_end={T} rule={rule}", flush=True)
    Ug, t, steps, code = gpu_run(U0, bc, h, T, gamma, recon=3, rule=rule)
    Uo, info = oracle.run_1d(U0, bc, h, T, p=oracle.params(gamma=gamma, recon=3), rule=rule)
    assert code == 0, (name, code)
    if rule == oracle.DT_CFL:
        assert steps == info["steps"], (steps, info["steps"])
    else:
        assert abs(steps / info["steps"] - 1) <= 0.02, (steps, info["steps"])
    assert abs(t - info["t"]) <= 1e-12 * T
    d = max(float(np.abs(Ug[c] - Uo[c]).sum() / np.abs(Uo[c]).sum()) for c in range(3))
    bar = tol
    if d > tol:
        # near vacuum the characteristic runs are ill-conditioned: the Roe
        # sound speed is small and the eigenvector entries ~1/a^2 amplify
        # roundoff; the oracle's own run moves by ~2e-3 (123 problem, double
        # rarefaction) under a 1e-15 perturbation of its initial data.  The
        # bar is then 4x that sensitivity.
        rng = np.random.default_rng(1402)
        Up, _ = oracle.run_1d(U0 * (1.0 + 1e-15 * rng.standard_normal(U0.shape)), bc, h, T,
                              p=oracle.params(gamma=gamma, recon=3), rule=rule)
        sens = max(float(np.abs(Up[c] - Uo[c]).sum() / np.abs(Uo[c]).sum()) for c in range(3))
        bar = max(tol, 4.0 * sens)
    print(f"  relative L1 difference {d:.2e} (bar {bar:.1e})", flush=True)
    assert d <= bar
    assert Ug[0].min() > 0 and W.pressure(Ug, gamma).min() > 0
