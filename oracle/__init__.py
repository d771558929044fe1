"""CPU oracle for the periodic Hartree solve, its backward and the Gaussian splat.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
CPU-baseline leg of the benchmark, never by the product path.  It shares no
code with the GPU library; the numerics live in ``hartree_oracle.c`` (plain C,
double precision, OpenMP) and this module only marshals numpy arrays.

What each call follows in the paper (Duy & Ozaki, arXiv:1209.4506):

* ``poisson``      -- Eq. (6), Sec. 2.1: the Hartree potential, obtained by
  solving the Poisson equation with FFTs, read as the periodic potential of a
  neutral cell; E_H is the E_Hartree term of Eq. (7), 1/2 * int n v_H, in both
  its real-space and reciprocal-space forms.
* ``fft1d`` / ``fft3d`` -- the transform behind that solve: recursive
  mixed-radix decimation in time, applied along c, b, then a (the layout
  order of Sec. 3.2.4).
* ``backward``     -- gradient of a loss through V and E_H; not in the paper,
  follows from the symmetry of the Poisson operator.
* ``splat`` / ``splat_points`` / ``splat_adjoint`` -- the synthetic atomic
  density standing in for Eq. (9) and its adjoint (Hartree forces).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hartree_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP, -O2, strict IEEE: no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(build())
    d = ctypes.POINTER(ctypes.c_double)
    i = ctypes.POINTER(ctypes.c_int)
    i64 = ctypes.POINTER(ctypes.c_int64)
    c_int, c_double = ctypes.c_int, ctypes.c_double
    sig = {
        "oracle_fft1d": [c_int, c_int, d, d],
        "oracle_fft3d": [i, c_int, d, d],
        "oracle_kernel": [d, i, d],
        "oracle_poisson": [d, i, d, d, d, d, d],
        "oracle_backward": [d, i, d, c_double, d, d],
        "oracle_splat": [d, i, c_int, d, d, d, c_double, c_int, d],
        "oracle_splat_points": [d, i, c_int, d, d, d, c_double, c_int, c_int, i64, d],
        "oracle_splat_adjoint": [d, i, c_int, d, d, d, c_double, d, c_int, i, d],
        "oracle_set_threads": [c_int],
        "oracle_max_threads": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = None if name == "oracle_set_threads" else c_int
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _ip(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _dims(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32).reshape(3)
    return d


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s rejected its arguments (code %d)" % (what, rc))


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def fft1d(x, sign: int = -1) -> np.ndarray:
    """Unnormalized 1-D DFT, X(m) = sum_n x(n) exp(sign * 2 pi i m n / N)."""
    x = np.ascontiguousarray(x, dtype=np.complex128).reshape(-1)
    out = np.empty_like(x)
    _check(_load().oracle_fft1d(x.size, int(sign), _dp(x.view(np.float64)), _dp(out.view(np.float64))), "fft1d")
    return out


def fft3d(x, sign: int = -1) -> np.ndarray:
    """Unnormalized 3-D DFT of an [Na][Nb][Nc] array (c fastest)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    assert x.ndim == 3
    out = np.empty_like(x)
    dims = _dims(x.shape)
    _check(_load().oracle_fft3d(_ip(dims), int(sign), _dp(x.view(np.float64)), _dp(out.view(np.float64))), "fft3d")
    return out


def kernel(cell, dims) -> np.ndarray:
    """K(m) = 4 pi / |G(m)|^2 on the full index grid, K(0) = 0, Nyquist averaged."""
    cell = _f64(cell).reshape(9)
    dims = _dims(dims)
    out = np.empty(tuple(int(v) for v in dims), dtype=np.float64)
    _check(_load().oracle_kernel(_dp(cell), _ip(dims), _dp(out)), "kernel")
    return out


def poisson(cell, rho):
    """Return (V, E_H real-space form, E_H reciprocal-space form, max |Im V|)."""
    cell = _f64(cell).reshape(9)
    rho = _f64(rho)
    dims = _dims(rho.shape)
    V = np.empty_like(rho)
    er, eg, mi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(_load().oracle_poisson(_dp(cell), _ip(dims), _dp(rho), _dp(V), ctypes.byref(er),
                                  ctypes.byref(eg), ctypes.byref(mi)), "poisson")
    return V, er.value, eg.value, mi.value


def backward(cell, rho, grad_v=None, grad_e: float = 0.0) -> np.ndarray:
    """d L / d rho = P grad_v + grad_e * dV * P rho."""
    cell = _f64(cell).reshape(9)
    rho = _f64(rho)
    dims = _dims(rho.shape)
    gv = None if grad_v is None else _f64(grad_v)
    out = np.empty_like(rho)
    _check(_load().oracle_backward(_dp(cell), _ip(dims), _dp(gv), float(grad_e), _dp(rho), _dp(out)), "backward")
    return out


def splat(cell, dims, pos, Z, sigma, cutoff_sigmas: float = 10.0, subtract_background: bool = True):
    """Grid density of periodic normalized Gaussians (every image within cutoff)."""
    cell = _f64(cell).reshape(9)
    dims = _dims(dims)
    pos = _f64(pos).reshape(-1, 3)
    Z = _f64(Z).reshape(-1)
    sigma = _f64(sigma).reshape(-1)
    out = np.empty(tuple(int(v) for v in dims), dtype=np.float64)
    _check(_load().oracle_splat(_dp(cell), _ip(dims), pos.shape[0], _dp(pos), _dp(Z), _dp(sigma),
                                float(cutoff_sigmas), int(bool(subtract_background)), _dp(out)), "splat")
    return out


def splat_points(cell, dims, pos, Z, sigma, flat_idx, cutoff_sigmas: float = 10.0,
                 subtract_background: bool = True) -> np.ndarray:
    """The splat density at selected flat grid indices, each evaluated on its own."""
    cell = _f64(cell).reshape(9)
    dims = _dims(dims)
    pos = _f64(pos).reshape(-1, 3)
    Z = _f64(Z).reshape(-1)
    sigma = _f64(sigma).reshape(-1)
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64).reshape(-1)
    out = np.empty(idx.size, dtype=np.float64)
    _check(_load().oracle_splat_points(_dp(cell), _ip(dims), pos.shape[0], _dp(pos), _dp(Z), _dp(sigma),
                                       float(cutoff_sigmas), int(bool(subtract_background)), idx.size,
                                       idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _dp(out)),
           "splat_points")
    return out


def splat_adjoint(cell, pos, Z, sigma, grad_rho, sel=None, cutoff_sigmas: float = 10.0) -> np.ndarray:
    """sum_r grad_rho(r) d rho(r)/d R_a for every atom (or the atoms in ``sel``)."""
    cell = _f64(cell).reshape(9)
    grad_rho = _f64(grad_rho)
    dims = _dims(grad_rho.shape)
    pos = _f64(pos).reshape(-1, 3)
    Z = _f64(Z).reshape(-1)
    sigma = _f64(sigma).reshape(-1)
    s = None if sel is None else np.ascontiguousarray(sel, dtype=np.int32).reshape(-1)
    nout = pos.shape[0] if s is None else s.size
    out = np.empty((nout, 3), dtype=np.float64)
    _check(_load().oracle_splat_adjoint(_dp(cell), _ip(dims), pos.shape[0], _dp(pos), _dp(Z), _dp(sigma),
                                        float(cutoff_sigmas), _dp(grad_rho), 0 if s is None else s.size,
                                        _ip(s), _dp(out)), "splat_adjoint")
    return out
