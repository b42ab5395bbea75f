"""The C-ABI library loads and exports every symbol of include/pp_cweno.h;
argument errors are caught on the host before any device call (no GPU)."""
import ctypes
import os
import re

import pytest

import paper_1402_5618_amd as pp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "pp_cweno.h")).read()
    return sorted(set(re.findall(r"\b(pp_cweno_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert header_symbols() == sorted(pp.EXPORTED)


def test_library_exports_every_symbol():
    L = pp.lib()
    for name in header_symbols():
        assert hasattr(L, name), name


def test_config_defaults():
    c = pp.default_config()
    assert c.ndim == 1 and c.gamma == 1.4 and c.weno_eps == 1e-13 and c.pp_eps_cap == 1e-13
    assert abs(c.gl_w1 - 1.0 / 12.0) < 1e-16 and c.precision == pp.PP_FP64 and c.nbatch == 0
    assert c.flux == pp.PP_FLUX_HLLC and c.recon == pp.PP_RECON_CWENO and c.fv == pp.PP_FV_LINE


def _init(**kw):
    c = pp.default_config()
    c.nx, c.dx = 64, 0.01
    for k, v in kw.items():
        if k == "bc":
            for i, b in enumerate(v):
                c.bc[i] = b
        else:
            setattr(c, k, v)
    ctx = ctypes.c_void_p()
    code = pp.lib().pp_cweno_init(ctypes.byref(c), ctypes.byref(ctx))
    return code, pp.lib().pp_cweno_last_error(None).decode()


@pytest.mark.parametrize("kw,code", [
    (dict(ndim=3), pp.PP_EINVAL),
    (dict(gamma=1.0), pp.PP_EINVAL),
    (dict(gl_w1=0.5), pp.PP_EINVAL),
    (dict(nx=4), pp.PP_EINVAL),                  # periodic needs >= 5 cells
    (dict(nx=2, bc=(1, 1, 0, 0)), pp.PP_EINVAL),
    (dict(dx=0.0), pp.PP_EINVAL),
    (dict(bc=(0, 1, 0, 0)), pp.PP_EINVAL),       # periodic on one end only
    (dict(bc=(7, 7, 0, 0)), pp.PP_EINVAL),
    (dict(precision=9), pp.PP_EINVAL),
    (dict(weno_eps=0.0), pp.PP_EINVAL),
    (dict(flux=2), pp.PP_EINVAL),
    (dict(flux=-1), pp.PP_EINVAL),
    (dict(recon=4), pp.PP_EINVAL),
    (dict(recon=3, precision=1), pp.PP_EUNSUPPORTED),             # characteristic: FP64
    (dict(recon=3, ndim=2, ny=64, dy=0.01, precision=1), pp.PP_EUNSUPPORTED),   # also in 2D
    (dict(recon=3, nbatch=2, precision=1), pp.PP_EUNSUPPORTED),   # batched: FP64 too
    (dict(recon=-1), pp.PP_EINVAL),
    (dict(recon=1, precision=1), pp.PP_EUNSUPPORTED),   # explicit schemes: FP64 only
    (dict(recon=2, nbatch=2, precision=1), pp.PP_EUNSUPPORTED),   # batched: FP64 too
    (dict(nx=5000), pp.PP_EUNSUPPORTED),
    (dict(ndim=2, ny=3000, dy=0.1, nx=64), pp.PP_EUNSUPPORTED),
    (dict(ndim=2, ny=64, dy=0.0), pp.PP_EINVAL),
    (dict(nbatch=-1), pp.PP_EINVAL),
    (dict(nbatch=2), pp.PP_EINVAL),              # batch arrays missing
    (dict(batch_rule=1), pp.PP_EINVAL),          # the h^(5/3) rule is not a batch rule
    (dict(batch_rule=4), pp.PP_EINVAL),
    (dict(fv=2), pp.PP_EINVAL),
    (dict(fv=1), pp.PP_EUNSUPPORTED),                                # Gauss nodes: 2D
    (dict(fv=1, ndim=2, ny=64, dy=0.01, precision=1), pp.PP_EUNSUPPORTED),   # FP64
    (dict(fv=1, ndim=2, ny=64, dy=0.01, recon=1), pp.PP_EUNSUPPORTED),       # compact scheme
    (dict(fv=1, ndim=2, ny=64, dy=0.01, recon=3), pp.PP_EUNSUPPORTED),       # component-wise
])
def test_invalid_configs_rejected_before_device(kw, code):
    got, msg = _init(**kw)
    assert got == code and msg


def test_null_arguments():
    L = pp.lib()
    assert L.pp_cweno_init(None, None) == pp.PP_EINVAL
    assert L.pp_cweno_rhs(None, None, None) == pp.PP_EINVAL
    assert L.pp_cweno_step(None, None, 0.1) == pp.PP_EINVAL
    assert L.pp_cweno_stage(None, None, None, None, 1, 0.1) == pp.PP_EINVAL
    assert L.pp_cweno_status(None, None) == pp.PP_EINVAL
    assert L.pp_cweno_restarts(None, None) == pp.PP_EINVAL
    L.pp_cweno_destroy(None)


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU; --gpus N > 1 exits with a message and does
    not touch a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
