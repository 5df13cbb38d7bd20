"""CPU FP64 oracle of the multiple-tau correlator (test infrastructure only).

The oracle is the plain, slow, obviously-correct reference the GPU library is
checked against: Algorithm 1 (update) and Algorithm 2 (readout) of the paper's
Appendix D, applied per channel in double precision, plus the trapezoid
Green-Kubo integral (Eqs. for viscosity and thermal conductivity, Section
2.3), the direct k-space density sum (Eq. k-density, Section "Currents") and
the partial momentum densities of the mass-flux correction (Section 2.3).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
and the GPU library never calls it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = [os.path.join(_HERE, "corr_oracle.c")]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-Wextra", "-o", _LIB_PATH] + _SRC + ["-lm"]
        subprocess.check_call(cmd)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=True)
        L = ctypes.CDLL(_LIB_PATH)
        i64, i32, dbl, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
        L.oracle_create.restype = vp
        L.oracle_create.argtypes = [i64, i32, i32, i32, i32]
        L.oracle_destroy.argtypes = [vp]
        L.oracle_push.argtypes = [vp, vp, vp]
        L.oracle_push.restype = i32
        L.oracle_n_push.argtypes = [vp]
        L.oracle_n_push.restype = i64
        L.oracle_max_out.argtypes = [vp]
        L.oracle_max_out.restype = i32
        L.oracle_readout.argtypes = [vp, i64, i64, vp, vp, vp, vp]
        L.oracle_readout.restype = i32
        L.oracle_raw.argtypes = [vp, i64, vp, vp, vp]
        L.oracle_raw.restype = i32
        L.oracle_trapezoid.argtypes = [i32, vp, vp, dbl, vp]
        L.oracle_trapezoid.restype = dbl
        L.oracle_rhok.argtypes = [vp, i64, vp, i32, dbl, vp, vp]
        L.oracle_rhok.restype = None
        L.oracle_push_rows.argtypes = [vp, i64, vp, vp]
        L.oracle_push_rows.restype = i32
        L.oracle_push_pair.argtypes = [vp, vp, vp, vp, vp]
        L.oracle_push_pair.restype = i32
        L.oracle_currents.argtypes = [vp, vp, i64, vp, i32, dbl, vp, vp]
        L.oracle_currents.restype = i32
        L.oracle_partial_momentum.argtypes = [vp, vp, i64, vp, i32, dbl, vp]
        L.oracle_partial_momentum.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleCorrelator:
    """n_ch independent FP64 multiple-tau correlators (b levels, p points, m)."""

    def __init__(self, n_ch: int, levels: int, points: int, m: int = 2, complex_: bool = False):
        self._h = lib().oracle_create(int(n_ch), int(levels), int(points), int(m), int(complex_))
        if not self._h:
            raise ValueError("invalid oracle correlator parameters")
        self.n_ch, self.levels, self.points, self.m = int(n_ch), int(levels), int(points), int(m)
        self.complex = bool(complex_)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().oracle_destroy(h)
            self._h = None

    def push(self, x) -> None:
        x = np.asarray(x)
        if self.complex:
            xc = x.astype(np.complex128)
            re = np.ascontiguousarray(xc.real)
            im = np.ascontiguousarray(xc.imag)
        else:
            if np.iscomplexobj(x):
                raise TypeError("complex samples pushed into a real correlator")
            re = np.ascontiguousarray(x, dtype=np.float64)
            im = None
        if re.shape != (self.n_ch,):
            raise ValueError(f"expected {self.n_ch} samples, got {re.shape}")
        if lib().oracle_push(self._h, _ptr(re), _ptr(im)) != 0:
            raise RuntimeError("oracle_push failed")

    def _planes(self, x):
        x = np.asarray(x)
        if self.complex:
            xc = x.astype(np.complex128)
            re, im = np.ascontiguousarray(xc.real), np.ascontiguousarray(xc.imag)
        else:
            if np.iscomplexobj(x):
                raise TypeError("complex samples pushed into a real correlator")
            re, im = np.ascontiguousarray(x, dtype=np.float64), None
        if re.shape != (self.n_ch,):
            raise ValueError(f"expected {self.n_ch} samples, got {re.shape}")
        return re, im

    def push_pair(self, x, y) -> None:
        """Pair form of Algorithm 1: C(L) = <x(s) conj(y(s - L))> per channel."""
        xr, xi = self._planes(x)
        yr, yi = self._planes(y)
        if lib().oracle_push_pair(self._h, _ptr(xr), _ptr(xi), _ptr(yr), _ptr(yi)) != 0:
            raise RuntimeError("oracle_push_pair failed (a record is auto or pair from its first push)")

    def push_series(self, xs) -> None:
        """xs: [S][n_ch] -- push S steps in order (one C call)."""
        xs = np.asarray(xs)
        if xs.ndim != 2 or xs.shape[1] != self.n_ch:
            raise ValueError(f"expected [S][{self.n_ch}] samples, got {xs.shape}")
        if self.complex:
            xc = xs.astype(np.complex128)
            re, im = np.ascontiguousarray(xc.real), np.ascontiguousarray(xc.imag)
        else:
            if np.iscomplexobj(xs):
                raise TypeError("complex samples pushed into a real correlator")
            re, im = np.ascontiguousarray(xs, dtype=np.float64), None
        if lib().oracle_push_rows(self._h, xs.shape[0], _ptr(re), _ptr(im)) != 0:
            raise RuntimeError("oracle_push_rows failed")

    @property
    def n_push(self) -> int:
        return int(lib().oracle_n_push(self._h))

    def readout(self, ch_begin: int = 0, ch_end: int | None = None):
        """Group mean over channels [ch_begin, ch_end): (t_steps, C, count)."""
        if ch_end is None:
            ch_end = self.n_ch
        nmax = int(lib().oracle_max_out(self._h))
        t = np.zeros(nmax)
        cre = np.zeros(nmax)
        cim = np.zeros(nmax)
        cnt = np.zeros(nmax, dtype=np.int64)
        n = lib().oracle_readout(self._h, int(ch_begin), int(ch_end), _ptr(t), _ptr(cre),
                                 _ptr(cim), _ptr(cnt))
        if n < 0:
            raise RuntimeError(f"oracle_readout failed ({n})")
        c = cre[:n] + 1j * cim[:n] if self.complex else cre[:n]
        return t[:n], c, cnt[:n]

    def raw(self, ch: int):
        """Per-(level, lag) sums and counts of one channel, shape [b][p]."""
        n = self.levels * self.points
        sre = np.zeros(n)
        sim = np.zeros(n)
        cnt = np.zeros(n, dtype=np.int64)
        if lib().oracle_raw(self._h, int(ch), _ptr(sre), _ptr(sim), _ptr(cnt)) != 0:
            raise RuntimeError("oracle_raw failed")
        s = sre + 1j * sim if self.complex else sre
        return s.reshape(self.levels, self.points), cnt.reshape(self.levels, self.points)


def trapezoid(t, c, t_cut: float | None = None):
    """Running trapezoid integral from t[0] and its value at t_cut (R14)."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    run = np.zeros_like(t)
    if t_cut is None:
        t_cut = float(t[-1]) if len(t) else 0.0
    at = lib().oracle_trapezoid(len(t), _ptr(t), _ptr(c), float(t_cut), _ptr(run))
    return run, float(at)


def rhok(pos_f32: np.ndarray, kvec: np.ndarray, box: float) -> np.ndarray:
    """n(k) = sum_j exp(i k.r_j) from FP32 positions [3][N], in FP64."""
    pos = np.ascontiguousarray(pos_f32, dtype=np.float32)
    assert pos.ndim == 2 and pos.shape[0] == 3
    kv = np.ascontiguousarray(kvec, dtype=np.int32)
    nk = kv.shape[0]
    re = np.zeros(nk)
    im = np.zeros(nk)
    lib().oracle_rhok(_ptr(pos), int(pos.shape[1]), _ptr(kv), int(nk), float(box), _ptr(re),
                      _ptr(im))
    return re + 1j * im


def currents(pos_f32: np.ndarray, vel_f32: np.ndarray, kvec: np.ndarray, box: float) -> np.ndarray:
    """Longitudinal and transverse currents (Eqs. long-current, trans-current;
    readings R19, R20 of the C source): [n_k][3] complex, column 0 = khat . J,
    columns 1, 2 = e1 . J, e2 . J with J = sum_j v_j exp(i k.r_j), in FP64."""
    pos = np.ascontiguousarray(pos_f32, dtype=np.float32)
    vel = np.ascontiguousarray(vel_f32, dtype=np.float32)
    assert pos.shape == vel.shape and pos.ndim == 2 and pos.shape[0] == 3
    kv = np.ascontiguousarray(kvec, dtype=np.int32)
    nk = kv.shape[0]
    re = np.zeros(3 * nk)
    im = np.zeros(3 * nk)
    rc = lib().oracle_currents(_ptr(pos), _ptr(vel), int(pos.shape[1]), _ptr(kv), int(nk),
                               float(box), _ptr(re), _ptr(im))
    if rc != 0:
        raise ValueError("the zero k-vector has no direction")
    return (re + 1j * im).reshape(nk, 3)


def partial_momentum(vel, species, masses, volume: float) -> np.ndarray:
    """Partial momentum densities j_{I_s} = (1/V) sum_{i in I_s} m_i v_i of the
    mass-flux correction (Section "Viscosity and thermal conductivity"; reading
    R22 of the C source): [n_species * 3], component alpha of species s at
    3 s + alpha, in FP64 from velocities [3][N] (any float dtype)."""
    v = np.ascontiguousarray(vel, dtype=np.float64)
    sp = np.ascontiguousarray(species, dtype=np.int32)
    ms = np.ascontiguousarray(masses, dtype=np.float64)
    assert v.ndim == 2 and v.shape[0] == 3 and sp.shape == (v.shape[1],)
    out = np.zeros(3 * len(ms))
    rc = lib().oracle_partial_momentum(_ptr(v), _ptr(sp), int(v.shape[1]), _ptr(ms), int(len(ms)),
                                       float(volume), _ptr(out))
    if rc != 0:
        raise ValueError("species id out of range")
    return out


def current_basis(n) -> np.ndarray:
    """(khat, e1, e2) rows of reading R20 for one integer k-vector (a plain
    restatement used by the tests to check the basis properties)."""
    n = np.asarray(n, dtype=np.float64)
    khat = n / np.linalg.norm(n)
    a = int(np.argmin(np.abs(khat)))
    e1 = np.eye(3)[a] - khat[a] * khat
    e1 /= np.linalg.norm(e1)
    return np.stack([khat, e1, np.cross(khat, e1)])


def green_kubo_viscosity(t, c_shear_mean, volume, kB, temperature, t_cut=None):
    """Eq. (viscosity): V/(kB T) * integral of the mean off-diagonal stress ACF."""
    run, at = trapezoid(t, c_shear_mean, t_cut)
    f = volume / (kB * temperature)
    return run * f, at * f


def green_kubo_conductivity(t, c_flux_mean, volume, kB, temperature, t_cut=None):
    """Eq. (thermal conductivity): V/(3 kB T^2) * integral of q(t).q(0); the dot
    product of three components equals 3x their mean autocorrelation."""
    run, at = trapezoid(t, c_flux_mean, t_cut)
    f = volume / (3.0 * kB * temperature * temperature) * 3.0
    return run * f, at * f
