"""CPU oracle for the strong-form spectral-element volume term (Sec. 2,
Eq. (volterm) of Klöckner, Wilcox, Warburton, ARRAY'16).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The
product path (the HIP library and its Python binding) never imports, links
or calls anything here, and nothing here imports the product package.

* :func:`volume_rhs` / :func:`volume_rhs_adjoint` call the plain FP64 C
  loops in ``sem_oracle.c`` (built with ``gcc -O2 -ffp-contract=off
  -fopenmp``, no fast-math);
* :func:`surface_rhs` calls the plain FP64 C loops of the surface term
  (strong-form discontinuous Galerkin face term with a local Lax-Friedrichs
  flux, the reading taken for the s of dq/dt = v + s in Sec. 2);
* :func:`ssp_rk3_step` composes any rate function into one step of the
  three-stage strong-stability-preserving Runge-Kutta scheme (Shu-Osher
  form), used for the method-of-lines time step of Sec. 2.

Every function takes plain NumPy arrays in the layouts documented in
``sem_oracle.c``; FP32 inputs are upcast exactly to FP64 first.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sem_oracle.c")
_LIB = os.path.join(_HERE, "libsem_oracle.so")
_lib = None

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc into ``oracle/libsem_oracle.so``."""
    cmd = ["gcc", *CFLAGS, _SRC, "-o", _LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    d = ctypes.c_double
    p = ctypes.c_void_p
    i32 = ctypes.c_int32
    i64 = ctypes.c_int64
    lib.sem_oracle_volume_rhs.argtypes = [i64, i64, i32, p, p, p, p, p, d, d, d, d, p, i32]
    lib.sem_oracle_volume_rhs.restype = None
    lib.sem_oracle_volume_rhs_ext.argtypes = [i64, i64, i32, i32, ctypes.c_uint32, p, p, p, p, p,
                                              d, d, d, d, p, i32]
    lib.sem_oracle_volume_rhs_ext.restype = None
    lib.sem_oracle_volume_rhs_adjoint.argtypes = [i64, i64, i32, p, p, p, d, d, d, d, p, p, i32]
    lib.sem_oracle_volume_rhs_adjoint.restype = None
    lib.sem_oracle_surface_rhs.argtypes = [i64, i64, i64, i32, p, p, p, p, d, d, d, p, i32]
    lib.sem_oracle_surface_rhs.restype = None
    lib.sem_oracle_max_threads.restype = ctypes.c_int
    lib.sem_oracle_set_threads.argtypes = [ctypes.c_int]
    _lib = lib
    return lib


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().sem_oracle_max_threads())


def set_threads(n: int) -> None:
    _load().sem_oracle_set_threads(int(n))


def volume_rhs(D, geo, q, rho_ref=None, theta_ref=None, phys=(1e5, 1.4, 287.0, 9.81),
               out=None, accumulate=False, elements=None):
    """Volume term of Eq. (volterm) plus the gravity source, in FP64.

    ``elements=(e0, e1)`` restricts the evaluation to that element range
    (``out`` is still indexed like ``q``; entries outside the range are
    left untouched, or zero when ``out`` is allocated here).
    """
    lib = _load()
    D, geo, q = _f64(D), _f64(geo), _f64(q)
    rho_ref, theta_ref = _f64(rho_ref), _f64(theta_ref)
    if (rho_ref is None) != (theta_ref is None):
        raise ValueError("rho_ref and theta_ref must both be given or both be None")
    Ne, nf, M = q.shape
    Nq = D.shape[0]
    assert nf == 5 and M == Nq ** 3 and geo.shape == (Ne, 10, M)
    if out is None:
        out = np.zeros_like(q)
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.shape == q.shape
    e0, e1 = (0, Ne) if elements is None else elements
    p0, gamma, R, grav = phys
    lib.sem_oracle_volume_rhs(e0, e1, Nq, _ptr(D), _ptr(geo), _ptr(q), _ptr(rho_ref),
                              _ptr(theta_ref), p0, gamma, R, grav, _ptr(out), int(bool(accumulate)))
    return out


DIR_R, DIR_S, DIR_T = 1, 2, 4


def volume_rhs_ext(D, geo, q, rho_ref=None, theta_ref=None, phys=(1e5, 1.4, 287.0, 9.81),
                   dirs=DIR_R | DIR_S | DIR_T, out=None, accumulate=False, elements=None):
    """Volume term with 5 or 8 fields (``q`` shaped ``[Ne, nf, Nq^3]``; fields 5-7
    are passive tracers) and a subset ``dirs`` of the reference directions
    (bit 0 r, bit 1 s, bit 2 t; the paper's benchmark kernel uses r and s)."""
    lib = _load()
    D, geo, q = _f64(D), _f64(geo), _f64(q)
    rho_ref, theta_ref = _f64(rho_ref), _f64(theta_ref)
    if (rho_ref is None) != (theta_ref is None):
        raise ValueError("rho_ref and theta_ref must both be given or both be None")
    Ne, nf, M = q.shape
    Nq = D.shape[0]
    assert nf in (5, 8) and M == Nq ** 3 and geo.shape == (Ne, 10, M)
    if out is None:
        out = np.zeros_like(q)
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.shape == q.shape
    e0, e1 = (0, Ne) if elements is None else elements
    p0, gamma, R, grav = phys
    lib.sem_oracle_volume_rhs_ext(e0, e1, Nq, nf, int(dirs), _ptr(D), _ptr(geo), _ptr(q),
                                  _ptr(rho_ref), _ptr(theta_ref), p0, gamma, R, grav, _ptr(out),
                                  int(bool(accumulate)))
    return out


def volume_rhs_adjoint(D, geo, q, lam, phys=(1e5, 1.4, 287.0, 9.81), out=None,
                       accumulate=False, elements=None):
    """Vector-Jacobian product ``(dv/dq)^T lam`` of the volume term, in FP64."""
    lib = _load()
    D, geo, q, lam = _f64(D), _f64(geo), _f64(q), _f64(lam)
    Ne, nf, M = q.shape
    Nq = D.shape[0]
    assert nf == 5 and M == Nq ** 3 and geo.shape == (Ne, 10, M) and lam.shape == q.shape
    if out is None:
        out = np.zeros_like(q)
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.shape == q.shape
    e0, e1 = (0, Ne) if elements is None else elements
    p0, gamma, R, grav = phys
    lib.sem_oracle_volume_rhs_adjoint(e0, e1, Nq, _ptr(D), _ptr(geo), _ptr(q), p0, gamma, R,
                                      grav, _ptr(lam), _ptr(out), int(bool(accumulate)))
    return out


def surface_rhs(geo, q, nbr, theta_ref=None, phys=(1e5, 1.4, 287.0, 9.81), out=None,
                accumulate=False, elements=None):
    """Surface term s of ``dq/dt = v + s`` in FP64 (see ``sem_oracle_surface_rhs``
    in ``sem_oracle.c``): ``nbr`` is ``[Ne, 6]`` int32, the element across
    faces r-, r+, s-, s+, t-, t+; an index outside ``[0, Ne)`` is a boundary
    face that adds nothing.  With ``theta_ref`` the pressure in the fluxes is
    each side's perturbation about its own reference value."""
    lib = _load()
    geo, q, theta_ref = _f64(geo), _f64(q), _f64(theta_ref)
    nbr = np.ascontiguousarray(nbr, dtype=np.int32)
    Ne, nf, M = q.shape
    Nq = round(M ** (1.0 / 3.0))
    assert nf == 5 and Nq ** 3 == M and geo.shape == (Ne, 10, M) and nbr.shape == (Ne, 6)
    assert theta_ref is None or theta_ref.shape == (Ne, M)
    if out is None:
        out = np.zeros_like(q)
    assert out.dtype == np.float64 and out.flags.c_contiguous and out.shape == q.shape
    e0, e1 = (0, Ne) if elements is None else elements
    p0, gamma, R, _grav = phys
    lib.sem_oracle_surface_rhs(e0, e1, Ne, Nq, _ptr(nbr), _ptr(geo), _ptr(q), _ptr(theta_ref),
                               p0, gamma, R, _ptr(out), int(bool(accumulate)))
    return out


def stage_update(a, x, b, y, c, z):
    """``a x + b (y + c z)`` in FP64: the stage update of an explicit
    Runge-Kutta method (y the stage state, z its rate, c the time step);
    ``x`` may be None when ``a == 0``."""
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    out = b * (y + c * z)
    if x is not None and a != 0.0:
        out = out + a * np.asarray(x, dtype=np.float64)
    return out


# Shu-Osher coefficients of the three-stage SSP Runge-Kutta scheme:
#   q1 = q + dt L(q)
#   q2 = 3/4 q + 1/4 (q1 + dt L(q1))
#   q' = 1/3 q + 2/3 (q2 + dt L(q2))
SSP_RK3 = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def ssp_rk3_step(rate, q, dt, stage_rates=None):
    """One SSP-RK3 step of ``dq/dt = rate(q)`` (explicit method of lines).
    ``stage_rates``, if a list, receives the rate evaluated at each stage."""
    qn = np.asarray(q, dtype=np.float64)
    qs = qn
    for a, b in SSP_RK3:
        v = rate(qs)
        if stage_rates is not None:
            stage_rates.append(v)
        qs = stage_update(a, qn, b, qs, dt, v)
    return qs
