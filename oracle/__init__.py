"""Python access to the plain FP64 CPU oracle (``oracle/oracle.c``).

TEST INFRASTRUCTURE ONLY: this is the independent checker of the HIP path.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it; the product package never does.

Every function takes and returns float64 numpy arrays in the layouts of
``workloads``: ``[3][n]`` (1D), ``[4][ny][nx]`` (2D), ``[3][sum n]`` (batched).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_PERIODIC, BC_TRANSMISSIVE, BC_REFLECTIVE = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: IEEE double, no FMA contraction, OpenMP."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-fopenmp", _SRC, "-o", _LIB + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [("gamma", ctypes.c_double), ("weno_eps", ctypes.c_double),
                ("eps_cap", ctypes.c_double), ("gl_w1", ctypes.c_double),
                ("linear", ctypes.c_int), ("first_order", ctypes.c_int),
                ("limiter", ctypes.c_int), ("flux", ctypes.c_int), ("recon", ctypes.c_int),
                ("fv", ctypes.c_int)]


class LineDbg(ctypes.Structure):
    _fields_ = [("um", ctypes.c_void_p), ("up", ctypes.c_void_p), ("um_l", ctypes.c_void_p),
                ("up_l", ctypes.c_void_p), ("flux", ctypes.c_void_p)]


def params(gamma=1.4, weno_eps=1e-13, eps_cap=1e-13, gl_w1=1.0 / 12.0, linear=False,
           first_order=False, limiter=True, flux=0, recon=0, fv=0) -> Params:
    """flux: 0 HLLC (eq. (HLLC)), 1 local Lax-Friedrichs (the alternative the
    paper names for Example 3.6).  recon: 0 the compact reconstruction
    (Sec. 2.2), 1 explicit WENO-JS, 2 explicit WENO-Z (the non-compact
    schemes the paper compares against in Sec. 3), 3 the compact
    reconstruction along characteristic fields (Sec. 2.3; in 2D along the
    direction of each line).  fv (2D):
    0 one state pair per face (dimension by dimension), 1 three Gauss nodes
    per face from a transverse reconstruction (a multi-dimensional reading
    beyond the paper, which leaves that to future work in Sec. 4)."""
    return Params(gamma, weno_eps, eps_cap, gl_w1, int(linear), int(first_order), int(limiter),
                  int(flux), int(recon), int(fv))


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.c_int
_L = ctypes.c_long
_DBL = ctypes.c_double
_P = ctypes.POINTER(Params)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        sig = {
            "orc_thomas": (_I, [_I, _D, _D, _D, _D, _D]),
            "orc_cyclic": (_I, [_I, _D, _D, _D, _D, _D]),
            "orc_dense_solve": (_I, [_I, _D, _D, _D]),
            "orc_hllc": (None, [_DBL, _I, _I, _D, _D, _D]),
            "orc_lf": (None, [_DBL, _I, _I, _D, _D, _D]),
            "orc_hllc_speeds": (None, [_DBL, _I, _I, _D, _D, _D]),
            "orc_limit_cell": (_I, [_I, _DBL, _DBL, _DBL, _D, _D, _D]),
            "orc_eps": (None, [_L, _I, _D, _DBL, _D, _D]),
            "orc_line_op": (_L, [_I, _I, _I, _D, _I, _I, _DBL, _P, _DBL, _DBL, _D,
                                 ctypes.POINTER(LineDbg), _D]),
            "orc_rhs_speed_1d": (_L, [_I, _D, _I, _I, _DBL, _P, _D, _D]),
            "orc_rhs_2d_speed": (_L, [_I, _I, _D, ctypes.POINTER(_I), _DBL, _DBL, _P, _D, _D]),
            "orc_recon_scalar": (_I, [_I, _I, _D, _P, _D, _D]),
            "orc_rhs_1d": (_L, [_I, _D, _I, _I, _DBL, _P, _D]),
            "orc_rk3_combine": (None, [_L, _I, _DBL, _D, _D, _D, _D]),
            "orc_stage_1d": (_L, [_I, _D, _D, _D, _I, _DBL, _I, _I, _DBL, _P]),
            "orc_max_speed_1d": (_DBL, [_I, _D, _DBL]),
            "orc_run_1d": (_I, [_I, _D, _I, _I, _DBL, _P, _DBL, _DBL, _I, _L, _D]),
            "orc_rhs_2d": (_L, [_I, _I, _D, ctypes.POINTER(_I), _DBL, _DBL, _P, _D]),
            "orc_stage_2d": (_L, [_I, _I, _D, _D, _D, _I, _DBL, ctypes.POINTER(_I), _DBL,
                                  _DBL, _P]),
            "orc_max_speed_2d": (None, [_I, _I, _D, _DBL, _D]),
            "orc_run_2d": (_I, [_I, _I, _D, ctypes.POINTER(_I), _DBL, _DBL, _P, _DBL, _DBL,
                                _L, _D]),
            "orc_run_2d_rule": (_I, [_I, _I, _D, ctypes.POINTER(_I), _DBL, _DBL, _P, _DBL, _DBL,
                                     _I, _L, _D]),
            "orc_run_batch": (_I, [_I, ctypes.POINTER(_L), _D, ctypes.POINTER(_I), _D, _P,
                                   _DBL, _DBL, _L, _D]),
            "orc_run_batch_rule": (_I, [_I, ctypes.POINTER(_L), _D, ctypes.POINTER(_I), _D, _P,
                                        _DBL, _DBL, _I, _L, _D, _D]),
            "orc_num_threads": (_I, []),
            "orc_set_threads": (None, [_I]),
            "orc_weights": (None, [_D, _DBL, _D]),
            "orc_char_eigen": (None, [_DBL, _D, _D, _D, _D, _D]),
            "orc_block_solve": (_I, [_I, _I, _D, _D, _D, _D, _D]),
            "orc_recon_char": (_I, [_I, _I, _D, _P, _D, _D]),
            "orc_char_eigen2": (None, [_DBL, _I, _D, _D, _D, _D, _D]),
            "orc_block_solve_nb": (_I, [_I, _I, _I, _D, _D, _D, _D, _D]),
            "orc_recon_char2": (_I, [_I, _I, _I, _D, _P, _D, _D]),
            "orc_gauss_nodes": (_I, [_D, _D]),
            "orc_limit_nodes": (_I, [_I, _DBL, _DBL, _DBL, _D, _D, _D]),
            "orc_gauss_dir": (_L, [_I, _I, _D, _I, _I, _I, _I, _I, _I, _DBL, _P, _DBL, _DBL,
                                   _D]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _d(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(code, what):
    if code < 0:
        raise RuntimeError(f"oracle {what} failed with code {code}")
    return code


# ------------------------------------------------------------------ pieces
def thomas(a, b, c, r):
    a, b, c, r = map(_f64, (a, b, c, r))
    x = np.empty_like(r)
    _check(lib().orc_thomas(len(r), _d(a), _d(b), _d(c), _d(r), _d(x)), "thomas")
    return x


def cyclic(a, b, c, r):
    a, b, c, r = map(_f64, (a, b, c, r))
    x = np.empty_like(r)
    _check(lib().orc_cyclic(len(r), _d(a), _d(b), _d(c), _d(r), _d(x)), "cyclic")
    return x


def dense_solve(A, r):
    A, r = _f64(A), _f64(r)
    x = np.empty_like(r)
    _check(lib().orc_dense_solve(len(r), _d(A), _d(r), _d(x)), "dense")
    return x


def hllc(Ul, Ur, gamma=1.4, nrm=1):
    Ul, Ur = _f64(Ul), _f64(Ur)
    F = np.empty_like(Ul)
    lib().orc_hllc(gamma, len(Ul), nrm, _d(Ul), _d(Ur), _d(F))
    return F


def lf(Ul, Ur, gamma=1.4, nrm=1):
    """Local Lax-Friedrichs flux (the reading of the paper's unnamed form)."""
    Ul, Ur = _f64(Ul), _f64(Ur)
    F = np.empty_like(Ul)
    lib().orc_lf(gamma, len(Ul), nrm, _d(Ul), _d(Ur), _d(F))
    return F


def hllc_speeds(Ul, Ur, gamma=1.4, nrm=1):
    Ul, Ur = _f64(Ul), _f64(Ur)
    S = np.empty(3)
    lib().orc_hllc_speeds(gamma, len(Ul), nrm, _d(Ul), _d(Ur), _d(S))
    return S


def limit_cell(Ub, Um, Up, eps_rho, eps_e, w1=1.0 / 12.0):
    Ub, Um, Up = _f64(Ub), _f64(Um).copy(), _f64(Up).copy()
    act = lib().orc_limit_cell(len(Ub), w1, eps_rho, eps_e, _d(Ub), _d(Um), _d(Up))
    return Um, Up, bool(act)


def eps(U, cap=1e-13):
    U = _f64(U)
    ncomp = U.shape[0]
    flat = U.reshape(ncomp, -1)
    er, ee = ctypes.c_double(), ctypes.c_double()
    lib().orc_eps(flat.shape[1], ncomp, _d(np.ascontiguousarray(flat)), cap,
                  ctypes.byref(er), ctypes.byref(ee))
    return er.value, ee.value


def line_op(u, bc_lo, bc_hi, h, p=None, eps_rho=None, eps_e=None, nrm=1, debug=False):
    """Spatial operator of one line ``u`` ([ncomp][n]).  Returns L (and a dict
    of intermediate arrays when ``debug``)."""
    p = p or params()
    u = _f64(u)
    ncomp, n = u.shape
    if eps_rho is None or eps_e is None:
        er, ee = eps(u, p.eps_cap)
        eps_rho = er if eps_rho is None else eps_rho
        eps_e = ee if eps_e is None else eps_e
    L = np.empty_like(u)
    dbg = None
    arrs = {}
    if debug:
        arrs = {k: np.empty_like(u) for k in ("um", "up", "um_l", "up_l")}
        arrs["flux"] = np.empty((ncomp, n + 1))
        dbg = LineDbg(*(arrs[k].ctypes.data for k in ("um", "up", "um_l", "up_l", "flux")))
    smax = np.zeros(1)
    nlim = _check(lib().orc_line_op(n, ncomp, nrm, _d(u), bc_lo, bc_hi, h, ctypes.byref(p),
                                    eps_rho, eps_e, _d(L),
                                    ctypes.byref(dbg) if dbg is not None else None, _d(smax)),
                  "line_op")
    if debug:
        arrs["nlim"] = nlim
        arrs["smax"] = float(smax[0])
        return L, arrs
    return L


def recon_scalar(ue, cyclic_line, p=None):
    """Reconstruct a scalar line from ghost-extended averages ``ue`` (cells
    -3..n+2).  Returns (u-_{i+1/2}, u+_{i-1/2}) for i = 0..n-1."""
    p = p or params()
    ue = _f64(ue)
    n = len(ue) - 6
    um, up = np.empty(n), np.empty(n)
    _check(lib().orc_recon_scalar(n, int(cyclic_line), _d(ue), ctypes.byref(p), _d(um), _d(up)),
           "recon")
    return um, up


def rk3_combine(stage, dt, U0, Us, L):
    U0, Us, L = _f64(U0), _f64(Us), _f64(L)
    Uo = np.empty_like(U0)
    lib().orc_rk3_combine(U0.size, stage, dt, _d(U0), _d(Us), _d(L), _d(Uo))
    return Uo


# ---------------------------------------------------------------------- 1D
def rhs_1d(U, bc=(0, 0), h=None, p=None, a=0.0, b=1.0):
    p = p or params()
    U = _f64(U)
    n = U.shape[1]
    h = (b - a) / n if h is None else h
    L = np.empty_like(U)
    _check(lib().orc_rhs_1d(n, _d(U), bc[0], bc[1], h, ctypes.byref(p), _d(L)), "rhs_1d")
    return L


def stage_1d(U0, Us, stage, dt, bc, h, p=None):
    p = p or params()
    U0, Us = _f64(U0), _f64(Us)
    Uo = np.empty_like(U0)
    _check(lib().orc_stage_1d(U0.shape[1], _d(U0), _d(Us), _d(Uo), stage, dt, bc[0], bc[1], h,
                              ctypes.byref(p)), "stage_1d")
    return Uo


def rhs_speed_1d(U, bc, h, p=None):
    """First-stage operator and the step's wave-speed bound (averages and
    limited interface states)."""
    p = p or params()
    U = _f64(U)
    L = np.empty_like(U)
    s = np.zeros(1)
    _check(lib().orc_rhs_speed_1d(U.shape[1], _d(U), bc[0], bc[1], h, ctypes.byref(p), _d(L),
                                  _d(s)), "rhs_speed_1d")
    return L, float(s[0])


def rhs_speed_2d(U, bc, dx, dy, p=None):
    p = p or params()
    U = _f64(U)
    _, ny, nx = U.shape
    L = np.empty_like(U)
    s = np.zeros(2)
    _check(lib().orc_rhs_2d_speed(nx, ny, _d(U), _bc4(bc), dx, dy, ctypes.byref(p), _d(L), _d(s)),
           "rhs_speed_2d")
    return L, s


def max_speed_1d(U, gamma=1.4):
    U = _f64(U)
    return lib().orc_max_speed_1d(U.shape[1], _d(U), gamma)


DT_CFL, DT_H53, DT_PP, DT_RESTART = 0, 1, 2, 3   # time-step rules (see orc_run_1d)


def run_1d(U, bc, h, t_end, cfl=1.0 / 12.0, rule=0, p=None, max_steps=1 << 40):
    """Advance to ``t_end``; returns (U, info dict).  ``viol``: stages whose
    input broke condition (CFL-CD) under the step's dt (rule DT_PP only);
    ``restarts``: steps redone at half dt (DT_RESTART); ``out_of_G``: stage
    outputs with a cell outside G (of the attempts kept)."""
    p = p or params()
    U = _f64(U).copy()
    out = np.zeros(8)
    _check(lib().orc_run_1d(U.shape[1], _d(U), bc[0], bc[1], h, ctypes.byref(p), t_end, cfl, rule,
                            max_steps, _d(out)), "run_1d")
    return U, dict(t=out[0], steps=int(out[1]), limited=int(out[2]), min_rho=out[3],
                   min_p=out[4], viol=int(out[5]), restarts=int(out[6]),
                   out_of_G=int(out[7]))


# ---------------------------------------------------------------------- 2D
def _bc4(bc):
    arr = (ctypes.c_int * 4)(*bc)
    return arr


def rhs_2d(U, bc=(0, 0, 0, 0), dx=None, dy=None, p=None):
    p = p or params()
    U = _f64(U)
    _, ny, nx = U.shape
    dx = 2.0 / nx if dx is None else dx
    dy = 2.0 / ny if dy is None else dy
    L = np.empty_like(U)
    _check(lib().orc_rhs_2d(nx, ny, _d(U), _bc4(bc), dx, dy, ctypes.byref(p), _d(L)), "rhs_2d")
    return L


def stage_2d(U0, Us, stage, dt, bc, dx, dy, p=None):
    p = p or params()
    U0, Us = _f64(U0), _f64(Us)
    _, ny, nx = U0.shape
    Uo = np.empty_like(U0)
    _check(lib().orc_stage_2d(nx, ny, _d(U0), _d(Us), _d(Uo), stage, dt, _bc4(bc), dx, dy,
                              ctypes.byref(p)), "stage_2d")
    return Uo


def max_speed_2d(U, gamma=1.4):
    U = _f64(U)
    out = np.zeros(2)
    lib().orc_max_speed_2d(U.shape[2], U.shape[1], _d(U), gamma, _d(out))
    return out


def run_2d(U, bc, dx, dy, t_end, cfl=1.0 / 12.0, p=None, max_steps=1 << 40, rule=0):
    p = p or params()
    U = _f64(U).copy()
    out = np.zeros(8)
    _check(lib().orc_run_2d_rule(U.shape[2], U.shape[1], _d(U), _bc4(bc), dx, dy, ctypes.byref(p),
                                 t_end, cfl, rule, max_steps, _d(out)), "run_2d")
    return U, dict(t=out[0], steps=int(out[1]), limited=int(out[2]), min_rho=out[3],
                   min_p=out[4], viol=int(out[5]), restarts=int(out[6]), out_of_G=int(out[7]))


# ----------------------------------------------------------------- batched
def run_batch(ens, t_end=None, cfl=1.0 / 12.0, p=None, rule=0, viol_out=None):
    """Advance every problem of a ``workloads.Ensemble`` (transmissive BCs).
    ``viol_out`` (float64 [nprob], optional) receives each problem's count of
    stages that broke (CFL-CD) (rule DT_PP)."""
    p = p or params()
    U = _f64(ens.U).copy()
    nprob = len(ens.lengths)
    offs = (ctypes.c_long * (nprob + 1))(*[int(v) for v in ens.offsets])
    bcs = (ctypes.c_int * (2 * nprob))(*([1] * (2 * nprob)))
    dxs = _f64(ens.dx)
    steps = np.zeros(nprob)
    viol = np.zeros(nprob) if viol_out is None else viol_out
    _check(lib().orc_run_batch_rule(nprob, offs, _d(U), bcs, _d(dxs), ctypes.byref(p),
                                    ens.t_end if t_end is None else t_end, cfl, rule, U.shape[1],
                                    _d(steps), _d(viol)), "run_batch")
    return U, steps


def gauss_nodes(v5):
    """Values at the three Gauss-Legendre nodes of the middle cell of the
    quartic whose averages over five unit cells are v5 (transverse step of
    the Gauss-node 2D operator)."""
    v = _f64(v5).copy()
    assert v.shape == (5,)
    out = np.empty(3)
    _check(lib().orc_gauss_nodes(_d(v), _d(out)), "gauss_nodes")
    return out


def limit_nodes(Ub, Nm, Np, eps_rho, eps_e, w1=1.0 / 12.0):
    """Node limiter of the Gauss-node 2D operator on one cell: Nm, Np are
    [3][ncomp] (right-face and left-face nodes).  Returns (Nm, Np, active)."""
    Ub = _f64(Ub)
    nc = Ub.shape[0]
    a = np.zeros((3, 4)); b = np.zeros((3, 4))
    a[:, :nc] = Nm; b[:, :nc] = Np
    r = lib().orc_limit_nodes(nc, w1, eps_rho, eps_e, _d(Ub), _d(a), _d(b))
    return a[:, :nc].copy(), b[:, :nc].copy(), r


def gauss_dir_x(U, bc, dx, eps_rho, eps_e, p=None):
    """The x-direction part of the Gauss-node operator for a [4][ny][nx]
    state (x-lines closed by bc[0:2], the set of lines by bc[2:4])."""
    p = p or params(fv=1)
    U = _f64(U)
    _, ny, nx = U.shape
    L = np.empty_like(U)
    _check(lib().orc_gauss_dir(nx, ny, _d(U), 1, 2, bc[0], bc[1], bc[2], bc[3], dx,
                               ctypes.byref(p), eps_rho, eps_e, _d(L)), "gauss_dir")
    return L


def rhs_2d_count(U, bc, dx, dy, p=None):
    """rhs_2d that also returns the number of limited cells."""
    p = p or params()
    U = _f64(U)
    _, ny, nx = U.shape
    L = np.empty_like(U)
    r = _check(lib().orc_rhs_2d(nx, ny, _d(U), _bc4(bc), dx, dy, ctypes.byref(p), _d(L)), "rhs_2d")
    return L, r


def weights(v6, eps=1e-13):
    """WENO-Z weights at node j+1/2 from ubar_{j-2..j+3}: ("-" side, "+" side)."""
    v6 = _f64(v6)
    w = np.empty(6)
    lib().orc_weights(_d(v6), eps, _d(w))
    return w[:3], w[3:]


def char_eigen(Ua, Ub, gamma=1.4):
    """Left eigenvectors L (rows), right eigenvectors R (columns) and
    eigenvalues at the Roe average of Ua and Ub (Sec. 2.3)."""
    Ua, Ub = _f64(Ua), _f64(Ub)
    L, R, lam = np.empty(9), np.empty(9), np.empty(3)
    lib().orc_char_eigen(gamma, _d(Ua), _d(Ub), _d(L), _d(R), _d(lam))
    return L.reshape(3, 3), R.reshape(3, 3), lam


def char_eigen2(Ua, Ub, nrm, gamma=1.4):
    """The 2D form of char_eigen: 4x4 eigenvectors of the flux Jacobian along
    a line whose normal momentum is component ``nrm`` (1: x, 2: y)."""
    Ua, Ub = _f64(Ua), _f64(Ub)
    L, R, lam = np.empty(16), np.empty(16), np.empty(4)
    lib().orc_char_eigen2(gamma, int(nrm), _d(Ua), _d(Ub), _d(L), _d(R), _d(lam))
    return L.reshape(4, 4), R.reshape(4, 4), lam


def block_solve(A, B, C, Y, cyclic=False):
    """Block chasing solve of A_i X_{i-1} + B_i X_i + C_i X_{i+1} = Y_i
    (3x3 or 4x4 blocks; cyclic: indices mod n)."""
    A, B, C, Y = (_f64(v) for v in (A, B, C, Y))
    n, nb = Y.shape
    X = np.empty_like(Y)
    _check(lib().orc_block_solve_nb(nb, n, int(cyclic), _d(A), _d(B), _d(C), _d(Y), _d(X)),
           "block")
    return X


def recon_char(ue, cyclic_line, p=None):
    """Characteristic-wise reconstruction of a 1D line from ghost-extended
    averages ``ue`` ([3][n+6], cells -3..n+2): (U-_{i+1/2}, U+_{i-1/2})."""
    p = p or params()
    ue = _f64(ue)
    n = ue.shape[1] - 6
    um, up = np.empty((3, n)), np.empty((3, n))
    _check(lib().orc_recon_char(n, int(cyclic_line), _d(ue), ctypes.byref(p), _d(um), _d(up)),
           "recon_char")
    return um, up


def recon_char2(ue, cyclic_line, nrm, p=None):
    """The 2D form of recon_char: a line of ``ue`` ([4][n+6]) whose normal
    momentum is component ``nrm`` (1: x line, 2: y line)."""
    p = p or params()
    ue = _f64(ue)
    n = ue.shape[1] - 6
    um, up = np.empty((4, n)), np.empty((4, n))
    _check(lib().orc_recon_char2(int(nrm), n, int(cyclic_line), _d(ue), ctypes.byref(p),
                                 _d(um), _d(up)), "recon_char2")
    return um, up


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's later calls (bench.py's one-thread figure)."""
    lib().orc_set_threads(int(n))


def num_threads() -> int:
    return lib().orc_num_threads()
