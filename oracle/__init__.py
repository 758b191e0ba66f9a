"""Reference oracle (test infrastructure only).

Plain, serial, FP64 CPU implementations of what the hx library computes, used
by tests/, the package smoke check and the CPU-baseline leg of bench.py, and by
nothing else.  The arithmetic lives in ``oracle.c`` (compiled with
``gcc -O2 -ffp-contract=off``); this module only marshals numpy arrays and adds
two tiny exact pure-Python checkers for very small inputs.  It shares no code
with the HIP library and never imports it.

Passages followed (of the paper, arXiv:1810.11482):
  * Sec. V-A.1: the 3-point stencil benchmark kernel; built here in its
    explicit heat-equation form (``heat1d_*``) next to the literal kernel
    (``prk_stencil``).
  * Sec. V-A.2, Algorithm 1: per-partition copy-in / kernel / copy-out; the
    partition kernel itself is ``partition_kernel``.  Partitioning does not
    change the arithmetic, so every partitioned result is checked against the
    whole-array loop.
  * The 2D and variable-coefficient forms, their boundaries and the adjoint are
    readings of the method listed in the design doc (zero-Dirichlet ghosts, face
    conductivity = arithmetic mean, reverse-mode derivation of the explicit
    scheme).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64
_f64 = ctypes.c_double


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _bind(path: str):
    """Open a compiled oracle library and declare its signatures."""
    lib = ctypes.CDLL(path)
    sig = {
        "orc_heat1d_periodic": [_dp, _i64, _f64, _i64, _dp],
        "orc_heat1d_dirichlet": [_dp, _i64, _f64, _i64, _dp],
        "orc_heat1d_open": [_dp, _i64, _f64, _i64, _dp],
        "orc_prk_stencil": [_dp, _i64, _dp],
        "orc_partition_kernel": [_i64, _i64, _dp],
        "orc_heat2d_dirichlet": [_dp, _i64, _i64, _f64, _i64, _dp],
        "orc_heat2d_window": [_dp, _i64, _i64, _i64, _i64, _f64, _i64, _dp],
        "orc_heatvc_step": [_dp, _dp, _i64, _i64, _f64, _dp],
        "orc_heatvc_forward": [_dp, _dp, _i64, _i64, _f64, _i64, _dp],
        "orc_heatvc_step_transpose": [_dp, _dp, _i64, _i64, _f64, _dp],
        "orc_heatvc_grad_kappa_step": [_dp, _dp, _i64, _i64, _f64, _dp],
        "orc_heatvc_grad": [_dp, _dp, _dp, _i64, _i64, _f64, _i64, _i64, _dp, _dp, _dp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name in ("orc_loss", "orc_dot"):
        fn = getattr(lib, name)
        fn.argtypes = [_dp, _dp, _i64]
        fn.restype = ctypes.c_double
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=False)
        _lib = _bind(_LIB)
    return _lib


def _in(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _p(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _check(rc: int, name: str) -> None:
    if rc != 0:
        raise ValueError(f"oracle {name}: bad argument")


# --------------------------------------------------------------------------- 1D
def heat1d_periodic(u0, r: float, steps: int) -> np.ndarray:
    """`steps` explicit heat steps on a periodic vector (Sec. V-A.1 stencil, heat form)."""
    u = _in(u0)
    out = np.empty_like(u)
    _check(_load().orc_heat1d_periodic(_p(u), u.size, r, steps, _p(out)), "heat1d_periodic")
    return out


def heat1d_dirichlet(u0, r: float, steps: int) -> np.ndarray:
    """`steps` explicit heat steps with zero ghosts outside [0, n)."""
    u = _in(u0)
    out = np.empty_like(u)
    _check(_load().orc_heat1d_dirichlet(_p(u), u.size, r, steps, _p(out)), "heat1d_dirichlet")
    return out


def heat1d_open(u, r: float, steps: int) -> np.ndarray:
    """Light cone: returns the len-2*steps interior cells after `steps` steps."""
    w = _in(u)
    out = np.empty(w.size - 2 * steps, dtype=np.float64)
    _check(_load().orc_heat1d_open(_p(w), w.size, r, steps, _p(out)), "heat1d_open")
    return out


def heat1d_periodic_at(u0, r: float, steps: int, idx) -> np.ndarray:
    """Values of heat1d_periodic(u0, r, steps) at the indices `idx`, each from its
    own light cone (cells idx-steps .. idx+steps of u0, periodic)."""
    u = _in(u0)
    n = u.size
    res = np.empty(len(idx), dtype=np.float64)
    for k, i in enumerate(idx):
        win = u[(np.arange(int(i) - steps, int(i) + steps + 1)) % n]
        res[k] = heat1d_open(win, r, steps)[0]
    return res


def prk_stencil(x) -> np.ndarray:
    """The paper's kernel s(x_i) = 0.5 x_{i-1} + x_i + 0.5 x_{i+1} (periodic), once."""
    v = _in(x)
    out = np.empty_like(v)
    _check(_load().orc_prk_stencil(_p(v), v.size, _p(out)), "prk_stencil")
    return out


def partition_kernel(first_index: int, n: int) -> np.ndarray:
    """The partition benchmark's kernel k(x_i) = sqrt(sin^2 i + cos^2 i) (Sec. V-A.2)."""
    out = np.empty(n, dtype=np.float64)
    _check(_load().orc_partition_kernel(first_index, n, _p(out)), "partition_kernel")
    return out


# --------------------------------------------------------------------------- 2D
def heat2d_dirichlet(u0, r: float, steps: int) -> np.ndarray:
    """`steps` five-point heat steps on a grid with zero ghosts outside."""
    u = _in(u0)
    ny, nx = u.shape
    out = np.empty_like(u)
    _check(_load().orc_heat2d_dirichlet(_p(u), ny, nx, r, steps, _p(out)), "heat2d_dirichlet")
    return out


def heat2d_dirichlet_at(u0, r: float, steps: int, points) -> np.ndarray:
    """Values of heat2d_dirichlet(u0, r, steps) at the (i, j) `points`, each from
    its own (2*steps+1)^2 light cone."""
    u0 = np.asarray(u0)
    ny, nx = u0.shape
    m = 2 * steps + 1
    res = np.empty(len(points), dtype=np.float64)
    lib = _load()
    for k, (i, j) in enumerate(points):
        gi0, gj0 = int(i) - steps, int(j) - steps
        w = np.zeros((m, m), dtype=np.float64)
        i_lo, i_hi = max(gi0, 0), min(gi0 + m, ny)
        j_lo, j_hi = max(gj0, 0), min(gj0 + m, nx)
        w[i_lo - gi0:i_hi - gi0, j_lo - gj0:j_hi - gj0] = u0[i_lo:i_hi, j_lo:j_hi]
        c = ctypes.c_double()
        _check(lib.orc_heat2d_window(_p(w), gi0, gj0, ny, nx, r, steps, ctypes.byref(c)),
               "heat2d_window")
        res[k] = c.value
    return res


# ------------------------------------------------------------ variable coefficient
def heatvc_step(u, kappa, dt: float) -> np.ndarray:
    uu, kk = _in(u), _in(kappa)
    ny, nx = uu.shape
    out = np.empty_like(uu)
    _check(_load().orc_heatvc_step(_p(uu), _p(kk), ny, nx, dt, _p(out)), "heatvc_step")
    return out


def heatvc_forward(u0, kappa, dt: float, steps: int) -> np.ndarray:
    uu, kk = _in(u0), _in(kappa)
    ny, nx = uu.shape
    out = np.empty_like(uu)
    _check(_load().orc_heatvc_forward(_p(uu), _p(kk), ny, nx, dt, steps, _p(out)),
           "heatvc_forward")
    return out


def heatvc_step_transpose(lam, kappa, dt: float) -> np.ndarray:
    ll, kk = _in(lam), _in(kappa)
    ny, nx = ll.shape
    out = np.empty_like(ll)
    _check(_load().orc_heatvc_step_transpose(_p(ll), _p(kk), ny, nx, dt, _p(out)),
           "heatvc_step_transpose")
    return out


def heatvc_grad_kappa_step(u_t, lam_next, dt: float, gk=None) -> np.ndarray:
    uu, ll = _in(u_t), _in(lam_next)
    ny, nx = uu.shape
    g = np.zeros_like(uu) if gk is None else np.array(gk, dtype=np.float64, copy=True)
    _check(_load().orc_heatvc_grad_kappa_step(_p(uu), _p(ll), ny, nx, dt, _p(g)),
           "heatvc_grad_kappa_step")
    return g


def heatvc_grad(u0, kappa, target, dt: float, steps: int, ckpt: int = 0):
    """(loss, dL/du0, dL/dkappa) for L = 0.5 ||u_T - y||^2; ckpt = segment length
    of the checkpointed sweep, 0 = keep every state."""
    uu, kk, yy = _in(u0), _in(kappa), _in(target)
    ny, nx = uu.shape
    loss = ctypes.c_double()
    lam0 = np.empty_like(uu)
    gk = np.empty_like(uu)
    _check(_load().orc_heatvc_grad(_p(uu), _p(kk), _p(yy), ny, nx, dt, steps, ckpt,
                                   ctypes.byref(loss), _p(lam0), _p(gk)), "heatvc_grad")
    return loss.value, lam0, gk


def heatvc_grad_window(u0, kappa, target, dt: float, steps: int, y0: int, x0: int, hy: int,
                       hx: int):
    """dL/du0 and dL/dkappa of the whole grid's loss, on the cells of the window
    [y0, y0 + hy) x [x0, x0 + hx) (clipped to the grid) that lie at least
    2 * steps cells inside every side where the window cuts the grid.

    The window is run as a grid of its own (heatvc_grad), whose boundary rule
    is wrong only along those cuts.  One step carries that error one cell
    inward; the forward sweep takes `steps` steps and the adjoint sweep
    `steps` more, and the conductivity gradient of a cell also reads its
    neighbours, so cells 2 * steps or more inside every cut get exactly the
    whole grid's values.  Returns (rows, cols, lam0, gk): the index ranges of
    those cells in the grid and their values."""
    uu, kk, yy = _in(u0), _in(kappa), _in(target)
    ny, nx = uu.shape
    a0, a1 = max(y0, 0), min(y0 + hy, ny)
    b0, b1 = max(x0, 0), min(x0 + hx, nx)
    m = 2 * steps
    r0 = a0 if a0 == 0 else a0 + m
    r1 = a1 if a1 == ny else a1 - m
    c0 = b0 if b0 == 0 else b0 + m
    c1 = b1 if b1 == nx else b1 - m
    if r1 <= r0 or c1 <= c0:
        raise ValueError("the window holds no cell 2 * steps inside its cuts")
    sl = (slice(a0, a1), slice(b0, b1))
    _, lam0, gk = heatvc_grad(uu[sl], kk[sl], yy[sl], dt, steps, 0)
    keep = (slice(r0 - a0, r1 - a0), slice(c0 - b0, c1 - b0))
    return (r0, r1), (c0, c1), lam0[keep], gk[keep]


def loss(u, y) -> float:
    uu, yy = _in(u), _in(y)
    return _load().orc_loss(_p(uu), _p(yy), uu.size)


def dot(a, b) -> float:
    aa, bb = _in(a), _in(b)
    return _load().orc_dot(_p(aa), _p(bb), aa.size)


# ------------------------------------------------------------------ batched (1D)
def heat1d_batched(sizes, rs, u0_packed, steps: int) -> np.ndarray:
    """Independent periodic problems packed back to back: problem j occupies
    cells [sum(sizes[:j]), sum(sizes[:j+1])) and uses its own r_j."""
    u = _in(u0_packed)
    out = np.empty_like(u)
    off = 0
    for n, r in zip(sizes, rs):
        out[off:off + n] = heat1d_periodic(u[off:off + n], float(r), steps)
        off += n
    return out


# ------------------------------------------------------ exact pure-Python checkers
def heat1d_periodic_exact(u0, r, steps: int):
    """Exact rational time stepping (fractions.Fraction), for tiny n only."""
    a = [Fraction(x) for x in u0]
    rr = Fraction(r)
    n = len(a)
    for _ in range(steps):
        a = [a[i] + rr * ((a[i - 1] - 2 * a[i]) + a[(i + 1) % n]) for i in range(n)]
    return a
