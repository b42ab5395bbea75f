"""MI355X (gfx950) compact-WENO Euler solver: Python binding of the C ABI
declared in ``include/pp_cweno.h``.

This module only marshals arguments: every step of the scheme runs in the
HIP kernels of ``libppcweno.so``.  States are contiguous float64 torch
tensors on the GPU in the layouts of the C ABI ([3][n], [4][ny][nx],
[3][sum n_i]).  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libppcweno.so")

PP_OK, PP_EINVAL, PP_ENOMEM, PP_EDEVICE, PP_ESTATE, PP_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
PP_BC_PERIODIC, PP_BC_TRANSMISSIVE, PP_BC_REFLECTIVE = 0, 1, 2
PP_FP64, PP_MIXED = 0, 1
PP_DT_CFL, PP_DT_H53, PP_DT_PP, PP_DT_RESTART = 0, 1, 2, 3
PP_FLUX_HLLC, PP_FLUX_LF = 0, 1
PP_RECON_CWENO, PP_RECON_WENOJS, PP_RECON_WENOZ, PP_RECON_CHAR = 0, 1, 2, 3
PP_FV_LINE, PP_FV_GAUSS = 0, 1

EXPORTED = [
    "pp_cweno_config_defaults", "pp_cweno_init", "pp_cweno_rhs", "pp_cweno_stage",
    "pp_cweno_step", "pp_cweno_step_static", "pp_cweno_run", "pp_cweno_batch_step", "pp_cweno_batch_tune",
    "pp_cweno_batch_run", "pp_cweno_batch_continue",
    "pp_cweno_restarts", "pp_cweno_max_speed", "pp_cweno_status", "pp_cweno_tridiag_solve_debug", "pp_cweno_debug_line", "pp_cweno_set_timing",
    "pp_cweno_get_timing", "pp_cweno_last_error", "pp_cweno_destroy",
]


class PPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pp_cweno error {code}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("gamma", ctypes.c_double),
        ("bc", ctypes.c_int * 4), ("precision", ctypes.c_int),
        ("weno_eps", ctypes.c_double), ("pp_eps_cap", ctypes.c_double),
        ("gl_w1", ctypes.c_double), ("nbatch", ctypes.c_int64),
        ("lengths", ctypes.POINTER(ctypes.c_int64)), ("dxs", ctypes.POINTER(ctypes.c_double)),
        ("bcs", ctypes.POINTER(ctypes.c_int)), ("stream", ctypes.c_void_p),
        ("flux", ctypes.c_int),
        ("recon", ctypes.c_int),
        ("batch_rule", ctypes.c_int),
        ("fv", ctypes.c_int),
    ]


_lib = None
_VP = ctypes.c_void_p


def lib():
    """Load ``libppcweno.so``; raises if it is missing (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        sig = {
            "pp_cweno_config_defaults": (None, [P(Config)]),
            "pp_cweno_init": (ctypes.c_int, [P(Config), P(_VP)]),
            "pp_cweno_rhs": (ctypes.c_int, [_VP, _VP, _VP]),
            "pp_cweno_stage": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int, ctypes.c_double]),
            "pp_cweno_step": (ctypes.c_int, [_VP, _VP, ctypes.c_double]),
            "pp_cweno_step_static": (ctypes.c_int, [P(Config), _VP, ctypes.c_double]),
            "pp_cweno_run": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_int64,
                                            ctypes.c_double, ctypes.c_int, P(ctypes.c_double),
                                            P(ctypes.c_int64)]),
            "pp_cweno_batch_step": (ctypes.c_int, [_VP, _VP, _VP]),
            "pp_cweno_batch_tune": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_int,
                                                   P(ctypes.c_int), P(ctypes.c_double)]),
            "pp_cweno_batch_run": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_int64,
                                                  ctypes.c_double, P(ctypes.c_int64)]),
            "pp_cweno_batch_continue": (ctypes.c_int, [_VP, _VP, ctypes.c_double, ctypes.c_int64,
                                                       ctypes.c_double, P(ctypes.c_int64),
                                                       P(ctypes.c_double)]),
            "pp_cweno_restarts": (ctypes.c_int, [_VP, P(ctypes.c_int64)]),
            "pp_cweno_max_speed": (ctypes.c_int, [_VP, _VP, _VP]),
            "pp_cweno_status": (ctypes.c_int, [_VP, P(ctypes.c_uint32)]),
            "pp_cweno_debug_line": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP]),
            "pp_cweno_tridiag_solve_debug": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int,
                                                            _VP, _VP, _VP, _VP, _VP]),
            "pp_cweno_set_timing": (ctypes.c_int, [_VP, ctypes.c_int]),
            "pp_cweno_get_timing": (ctypes.c_int, [_VP, P(ctypes.c_double)]),
            "pp_cweno_last_error": (ctypes.c_char_p, [_VP]),
            "pp_cweno_destroy": (None, [_VP]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(t, numel=None, at_least=False):
    """Device address of a contiguous float64 GPU tensor, after checking that
    it holds the `numel` elements the kernels will touch (exactly, or at
    least that many for small result buffers): the C ABI takes bare
    pointers and cannot check sizes itself."""
    if t is None:
        return None
    if not (t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous GPU tensor")
    import torch
    if t.dtype != torch.float64:
        raise ValueError("expected float64")
    if numel is not None and (t.numel() < numel if at_least else t.numel() != numel):
        raise ValueError(f"expected {'at least ' if at_least else ''}{numel} elements, "
                         f"got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def default_config() -> Config:
    c = Config()
    lib().pp_cweno_config_defaults(ctypes.byref(c))
    return c


def step_static(U, dt, nx, dx, bc=(1, 1), gamma=1.4, precision=PP_FP64, weno_eps=1e-13,
                pp_eps_cap=1e-13, gl_w1=1.0 / 12.0, flux=None, stream=None):
    """pp_cweno_step_static: one SSP-RK3 step of a 1D line U ([3][nx]) in
    place, without a context and without device allocation (the library's
    fixed scratch array).  Raises PPError on failure."""
    c = default_config()
    c.ndim, c.nx, c.ny, c.dx, c.gamma = 1, nx, 1, dx, gamma
    c.bc[0], c.bc[1] = int(bc[0]), int(bc[1])
    c.precision, c.weno_eps, c.pp_eps_cap, c.gl_w1 = precision, weno_eps, pp_eps_cap, gl_w1
    if flux is not None:
        c.flux = int(flux)
    if stream is None:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    c.stream = ctypes.c_void_p(stream)
    code = lib().pp_cweno_step_static(ctypes.byref(c), _ptr(U, 3 * int(nx)), float(dt))
    if code != PP_OK:
        msg = lib().pp_cweno_last_error(None)
        raise PPError(code, msg.decode() if msg else "")
    return code


class Solver:
    """One pp_cweno context.  Method names follow the C entry points."""

    def __init__(self, ndim=1, nx=0, ny=1, dx=0.0, dy=0.0, gamma=1.4, bc=(0, 0, 0, 0),
                 precision=PP_FP64, weno_eps=1e-13, pp_eps_cap=1e-13, gl_w1=1.0 / 12.0,
                 lengths=None, dxs=None, bcs=None, stream=None, flux=None, recon=None,
                 batch_rule=None, fv=None):
        c = default_config()
        c.ndim, c.nx, c.ny, c.dx, c.dy, c.gamma = ndim, nx, ny, dx, dy, gamma
        for i in range(4):
            c.bc[i] = int(bc[i]) if i < len(bc) else 0
        c.precision, c.weno_eps, c.pp_eps_cap, c.gl_w1 = precision, weno_eps, pp_eps_cap, gl_w1
        if flux is not None:
            c.flux = int(flux)
        if recon is not None:
            c.recon = int(recon)
        if batch_rule is not None:
            c.batch_rule = int(batch_rule)
        if fv is not None:
            c.fv = int(fv)
        self._keep = []
        if lengths is not None:
            nb = len(lengths)
            la = (ctypes.c_int64 * nb)(*[int(v) for v in lengths])
            da = (ctypes.c_double * nb)(*[float(v) for v in dxs])
            ba = (ctypes.c_int * (2 * nb))(*[int(v) for v in bcs])
            self._keep += [la, da, ba]
            c.nbatch = nb
            c.lengths = ctypes.cast(la, ctypes.POINTER(ctypes.c_int64))
            c.dxs = ctypes.cast(da, ctypes.POINTER(ctypes.c_double))
            c.bcs = ctypes.cast(ba, ctypes.POINTER(ctypes.c_int))
        if stream is None:
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        c.stream = ctypes.c_void_p(stream)
        self.cfg = c
        # elements of a state array in this context's layout
        if lengths is not None:
            self._nstate = 3 * int(sum(int(v) for v in lengths))
        elif ndim == 2:
            self._nstate = 4 * int(nx) * int(ny)
        else:
            self._nstate = 3 * int(nx)
        self._nb = len(lengths) if lengths is not None else 0
        self._ctx = ctypes.c_void_p()
        self._check(lib().pp_cweno_init(ctypes.byref(c), ctypes.byref(self._ctx)), init=True)

    def _check(self, code, init=False):
        if code != PP_OK:
            msg = lib().pp_cweno_last_error(None if init else self._ctx)
            raise PPError(code, msg.decode() if msg else "")
        return code

    def rhs(self, U, L):
        n = self._nstate
        return self._check(lib().pp_cweno_rhs(self._ctx, _ptr(U, n), _ptr(L, n)))

    def stage(self, U0, Us, Uout, stage, dt):
        n = self._nstate
        return self._check(lib().pp_cweno_stage(self._ctx, _ptr(U0, n), _ptr(Us, n),
                                                _ptr(Uout, n), int(stage), float(dt)))

    def step(self, U, dt):
        return self._check(lib().pp_cweno_step(self._ctx, _ptr(U, self._nstate), float(dt)))

    def run(self, U, t_end, nsteps_max=1 << 62, cfl=1.0 / 12.0, rule=PP_DT_CFL):
        """pp_cweno_run: advance U in place; returns (t reached, steps)."""
        t = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(lib().pp_cweno_run(self._ctx, _ptr(U, self._nstate), float(t_end),
                                       int(nsteps_max), float(cfl), int(rule), ctypes.byref(t),
                                       ctypes.byref(n)))
        return t.value, n.value

    def batch_step(self, U, dt_dev):
        return self._check(lib().pp_cweno_batch_step(self._ctx, _ptr(U, self._nstate),
                                                     _ptr(dt_dev, self._nb)))

    def batch_tune(self, U=None, cfl=1.0 / 12.0, force_plan=-1):
        """Pick the batched launch plan: timed over every plan on a copy of U
        (force_plan < 0) or set directly.  Returns (plan, [ms per plan])."""
        plan = ctypes.c_int()
        ms = (ctypes.c_double * 6)(*([-1.0] * 6))
        self._check(lib().pp_cweno_batch_tune(self._ctx, _ptr(U, self._nstate), float(cfl),
                                              int(force_plan), ctypes.byref(plan), ms))
        return plan.value, list(ms)

    def batch_run(self, U, t_end, nsteps_max=1 << 62, cfl=1.0 / 12.0):
        """Per-problem step counts; raises PPError(PP_ESTATE) after the run if
        a stage left the admissible set (counts then via last_batch_steps)."""
        nb = self.cfg.nbatch
        steps = (ctypes.c_int64 * nb)()
        self._last_steps = steps
        self._check(lib().pp_cweno_batch_run(self._ctx, _ptr(U, self._nstate), float(t_end),
                                             int(nsteps_max), float(cfl), steps))
        return list(steps)

    def batch_continue(self, U, t_end, nsteps_max=1 << 62, cfl=1.0 / 12.0):
        """Continue the last batch_run: returns (per-problem steps, per-problem
        t); raises PPError(PP_ESTATE) like batch_run (counts then via
        last_batch_steps)."""
        nb = self.cfg.nbatch
        steps = (ctypes.c_int64 * nb)()
        ts = (ctypes.c_double * nb)()
        self._last_steps, self._last_t = steps, ts
        self._check(lib().pp_cweno_batch_continue(self._ctx, _ptr(U, self._nstate),
                                                  float(t_end), int(nsteps_max), float(cfl),
                                                  steps, ts))
        return list(steps), list(ts)

    def last_batch_times(self):
        return list(self._last_t)

    def last_batch_steps(self):
        return list(self._last_steps)

    def restarts(self):
        """Steps redone with half the dt (PP_DT_RESTART) in the last run."""
        v = ctypes.c_int64()
        self._check(lib().pp_cweno_restarts(self._ctx, ctypes.byref(v)))
        return v.value

    def max_speed(self, U, out):
        return self._check(lib().pp_cweno_max_speed(self._ctx, _ptr(U, self._nstate),
                                                    _ptr(out, self.cfg.ndim, at_least=True)))

    def status(self):
        f = ctypes.c_uint32()
        code = lib().pp_cweno_status(self._ctx, ctypes.byref(f))
        return code, f.value

    def debug_line(self, U, um=None, up=None, flux=None):
        n = self._nstate
        return self._check(lib().pp_cweno_debug_line(self._ctx, _ptr(U, n), _ptr(um, n),
                                                     _ptr(up, n), _ptr(flux, n + 3)))

    def tridiag_solve_debug(self, a, b, c, r, x, cyclic=False):
        """Device chunked chase + PCR of one tridiagonal system (test hook)."""
        n = r.numel()
        return self._check(lib().pp_cweno_tridiag_solve_debug(
            self._ctx, n, int(bool(cyclic)), _ptr(a, n), _ptr(b, n), _ptr(c, n), _ptr(r, n),
            _ptr(x, n)))

    def set_timing(self, on=True):
        return self._check(lib().pp_cweno_set_timing(self._ctx, int(bool(on))))

    def get_timing(self):
        """{class: (total ms, launches)} for 'x', 'y', 'combine'."""
        out = (ctypes.c_double * 6)()
        self._check(lib().pp_cweno_get_timing(self._ctx, out))
        return {"x": (out[0], int(out[1])), "y": (out[2], int(out[3])),
                "combine": (out[4], int(out[5]))}

    def close(self):
        if self._ctx:
            lib().pp_cweno_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
