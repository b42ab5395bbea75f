"""The allocation-free entry point pp_cweno_step_static against
pp_cweno_step: two calls in a row on one GPU (the second on a shorter line,
so the shared scratch holds the first call's data), both precisions, each
equal to the context path's step to the FP64 bar (1e-12 relative per
component; the two run the same kernels, so equality is expected bitwise)."""
import ctypes

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def gpu():
    import paper_1402_5618_amd as pp
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return pp


def line(n, seed):
    rng = np.random.default_rng(seed)
    x = W.cell_centres(0.0, 1.0, n)
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x) + 0.8 * ((x > 0.3) & (x < 0.6))
    u = 0.5 * np.cos(4 * np.pi * x) + rng.normal(0, 0.01, n)
    p = np.where(x < 0.7, 1.0, 0.1)
    return W.prim_to_cons_1d(rho, u, p, 1.4)


def rel(a, b):
    return max(float(np.abs(a[k] - b[k]).max() / np.abs(b[k]).max()) for k in range(3))


@pytest.mark.parametrize("precision", [0, 1])
def test_static_step_equals_context_step_twice(precision):
    pp = gpu()
    cases = [(3500, (1, 2), 11), (900, (0, 0), 12)]   # second call: shorter line
    for n, bc, seed in cases:
        U0 = line(n, seed)
        h = 1.0 / n
        dt = 0.5 * (1.0 / 12.0) * h
        print(f"static step: n={n}, bc={bc}, precision={precision}", flush=True)
        Us = torch.tensor(U0, device="cuda")
        pp.step_static(Us, dt, n, h, bc=bc, precision=precision)
        s = pp.Solver(ndim=1, nx=n, dx=h, bc=(bc[0], bc[1], 0, 0), precision=precision)
        Uc = torch.tensor(U0, device="cuda")
        s.step(Uc, dt)
        torch.cuda.synchronize()
        s.close()
        a, b = Us.cpu().numpy(), Uc.cpu().numpy()
        d = rel(a, b)
        print(f"  max relative difference {d:.3e}, bitwise equal: {np.array_equal(a, b)}",
              flush=True)
        assert d <= 1e-12
        assert not np.array_equal(a, U0)   # the step did advance the line


def test_static_step_rejects_before_any_device_work():
    pp = gpu()
    c = pp.default_config()
    c.ndim, c.nx, c.dx = 1, 5000, 1e-3
    U = torch.zeros(3 * 5000, dtype=torch.float64, device="cuda")
    code = pp.lib().pp_cweno_step_static(ctypes.byref(c), ctypes.c_void_p(U.data_ptr()), 1e-4)
    assert code == pp.PP_EUNSUPPORTED and pp.lib().pp_cweno_last_error(None)
    c.nx, c.ndim = 64, 2
    c.ny, c.dy = 64, 1e-3
    code = pp.lib().pp_cweno_step_static(ctypes.byref(c), ctypes.c_void_p(U.data_ptr()), 1e-4)
    assert code == pp.PP_EINVAL
