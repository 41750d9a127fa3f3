"""ctypes binding of the plain FP64 CPU SPME oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The GPU product path never imports it.

Conventions: grids are numpy arrays of shape (K3, K2, K1) (k1 fastest), box is
a (3, 3) array whose rows are the cell vectors, ev = [E, Pxx, Pyy, Pzz, Pxy,
Pxz, Pyz].  See spme_oracle.c for the equations each call follows.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i, d = ctypes.c_int, ctypes.c_double
    lib.orc_bspline_M.argtypes = [i, d]
    lib.orc_bspline_M.restype = d
    lib.orc_bspline.argtypes = [i, d, _dp, _dp]
    lib.orc_moduli.argtypes = [i, i, _dp]
    lib.orc_fft1d.argtypes = [i, _dp, _dp, i]
    lib.orc_fft3d.argtypes = [i, i, i, _dp, _dp, i]
    lib.orc_spme.argtypes = [_dp, _dp, i, _dp, i, i, i, i, d, d, _dp, _dp, _dp, _dp, _dp]
    lib.orc_mirror_grid.argtypes = [_dp, _dp, i, _dp, i, i, i, i, i, _i64p, _fp]
    lib.orc_mirror_spline.argtypes = [i, ctypes.c_float, _fp, _fp]
    lib.orc_ewald_recip.argtypes = [_dp, _dp, i, _dp, d, d, i, _dp, _dp]
    lib.orc_ewald_real.argtypes = [_dp, _dp, i, _dp, d, d, i, d, _dp, _dp, _dp]
    _ip = ctypes.POINTER(ctypes.c_int)
    lib.orc_ewald_excl.argtypes = [_dp, _dp, i, _dp, d, d, d, _ip, _ip, _dp, _dp]
    lib.orc_ewald_real_atoms.argtypes = [_dp, _dp, i, _dp, d, d, i, d, _ip, i, _dp]
    for name in ("orc_bspline", "orc_moduli", "orc_fft1d", "orc_fft3d", "orc_spme",
                 "orc_mirror_grid", "orc_mirror_spline", "orc_ewald_recip", "orc_ewald_real",
                 "orc_ewald_excl", "orc_ewald_real_atoms"):
        getattr(lib, name).restype = i
    _lib = lib
    return lib


def _ptr(a, ct=_dp):
    if a is None:
        return None
    return a.ctypes.data_as(ct)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _box(box):
    b = np.asarray(box, dtype=np.float64)
    if b.shape == (3,):
        b = np.diag(b)
    return np.ascontiguousarray(b.reshape(3, 3))


def _grid3(K):
    if np.isscalar(K):
        return int(K), int(K), int(K)
    K1, K2, K3 = (int(k) for k in K)
    return K1, K2, K3


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"{what} failed with status {rc}")


def bspline_M(n, x):
    return _load().orc_bspline_M(int(n), float(x))


def bspline(p, w):
    """(theta, dtheta) for offsets j = 0..p-1, i.e. M_p(w+p-1-j) and its derivative."""
    th = np.zeros(p)
    dth = np.zeros(p)
    _check(_load().orc_bspline(int(p), float(w), _ptr(th), _ptr(dth)), "orc_bspline")
    return th, dth


def moduli(p, K):
    out = np.zeros(int(K))
    _check(_load().orc_moduli(int(p), int(K), _ptr(out)), "orc_moduli")
    return out


def fft1d(x, sign):
    x = np.asarray(x, dtype=np.complex128)
    re = np.ascontiguousarray(x.real.copy())
    im = np.ascontiguousarray(x.imag.copy())
    _check(_load().orc_fft1d(len(x), _ptr(re), _ptr(im), int(sign)), "orc_fft1d")
    return re + 1j * im


def fft3d(x, sign):
    x = np.asarray(x, dtype=np.complex128)
    K3, K2, K1 = x.shape
    re = np.ascontiguousarray(x.real.copy())
    im = np.ascontiguousarray(x.imag.copy())
    _check(_load().orc_fft3d(K1, K2, K3, _ptr(re), _ptr(im), int(sign)), "orc_fft3d")
    return re + 1j * im


def spme(pos, q, box, K, p, beta, coulomb=1.0, want_grids=False, want_times=False):
    """FP64 SPME reciprocal step.  Returns dict(forces, ev, [Q, phi], [times])."""
    pos = _f64(pos)
    N = pos.shape[0]
    pos = pos.reshape(N, 3)
    q = _f64(q, (N,))
    b = _box(box)
    K1, K2, K3 = _grid3(K)
    forces = np.zeros((N, 3))
    ev = np.zeros(7)
    Q = np.zeros((K3, K2, K1)) if want_grids else None
    phi = np.zeros((K3, K2, K1)) if want_grids else None
    times = np.zeros(4) if want_times else None
    rc = _load().orc_spme(_ptr(pos), _ptr(q), N, _ptr(b), K1, K2, K3, int(p), float(beta),
                          float(coulomb), _ptr(forces), _ptr(ev), _ptr(Q), _ptr(phi),
                          _ptr(times))
    _check(rc, "orc_spme")
    out = {"forces": forces, "ev": ev, "E": ev[0], "virial": ev[1:].copy()}
    if want_grids:
        out["Q"] = Q
        out["phi"] = phi
    if want_times:
        out["times"] = {"spread": times[0], "fft": times[1], "influence": times[2],
                        "gather": times[3]}
    return out


def mirror_spline(p, w32):
    th = np.zeros(p, dtype=np.float32)
    dth = np.zeros(p, dtype=np.float32)
    _check(_load().orc_mirror_spline(int(p), ctypes.c_float(float(np.float32(w32))),
                                     _ptr(th, _fp), _ptr(dth, _fp)), "orc_mirror_spline")
    return th, dth


def mirror_grid(pos, q, box, K, p, frac_bits=32, allow_nonfinite=False):
    """Quantised fixed-point charge grid: (Q_int int64, Q32 float32), shape (K3,K2,K1)."""
    pos = _f64(pos)
    N = pos.shape[0]
    pos = pos.reshape(N, 3)
    q = _f64(q, (N,))
    b = _box(box)
    K1, K2, K3 = _grid3(K)
    Qi = np.zeros((K3, K2, K1), dtype=np.int64)
    Qf = np.zeros((K3, K2, K1), dtype=np.float32)
    rc = _load().orc_mirror_grid(_ptr(pos), _ptr(q), N, _ptr(b), K1, K2, K3, int(p),
                                 int(frac_bits), _ptr(Qi, _i64p), _ptr(Qf, _fp))
    if rc == -2 and allow_nonfinite:
        return Qi, Qf
    _check(rc, "orc_mirror_grid")
    return Qi, Qf


def ewald_recip(pos, q, box, beta, mmax, coulomb=1.0):
    pos = _f64(pos)
    N = pos.shape[0]
    pos = pos.reshape(N, 3)
    q = _f64(q, (N,))
    b = _box(box)
    forces = np.zeros((N, 3))
    ev = np.zeros(7)
    _check(_load().orc_ewald_recip(_ptr(pos), _ptr(q), N, _ptr(b), float(beta), float(coulomb),
                                   int(mmax), _ptr(forces), _ptr(ev)), "orc_ewald_recip")
    return {"forces": forces, "ev": ev, "E": ev[0], "virial": ev[1:].copy()}


def ewald_real(pos, q, box, beta, nimg=1, rcut=0.0, coulomb=1.0):
    pos = _f64(pos)
    N = pos.shape[0]
    pos = pos.reshape(N, 3)
    q = _f64(q, (N,))
    b = _box(box)
    forces = np.zeros((N, 3))
    er = np.zeros(1)
    es = np.zeros(1)
    _check(_load().orc_ewald_real(_ptr(pos), _ptr(q), N, _ptr(b), float(beta), float(coulomb),
                                  int(nimg), float(rcut), _ptr(forces), _ptr(er), _ptr(es)),
           "orc_ewald_real")
    return {"forces": forces, "E_real": float(er[0]), "E_self": float(es[0])}


def ewald_real_atoms(pos, q, box, beta, atoms, nimg=1, rcut=0.0, coulomb=1.0):
    """Real-space forces on the listed atoms only: rows of ewald_real's forces."""
    pos = _f64(pos)
    N = pos.shape[0]
    pos = pos.reshape(N, 3)
    q = _f64(q, (N,))
    b = _box(box)
    at = np.ascontiguousarray(atoms, dtype=np.int32)
    forces = np.zeros((len(at), 3))
    _check(_load().orc_ewald_real_atoms(_ptr(pos), _ptr(q), N, _ptr(b), float(beta),
                                        float(coulomb), int(nimg), float(rcut),
                                        at.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), len(at),
                                        _ptr(forces)), "orc_ewald_real_atoms")
    return forces


def ewald_excl(pos, q, box, beta, excl_off, excl_idx, rcut=0.0, coulomb=1.0):
    """Exclusion correction for symmetric CSR exclusion lists."""
    pos = _f64(pos)
    N = pos.shape[0]
    pos = pos.reshape(N, 3)
    q = _f64(q, (N,))
    b = _box(box)
    off = np.ascontiguousarray(excl_off, dtype=np.int32)
    idx = np.ascontiguousarray(excl_idx, dtype=np.int32)
    assert off.shape == (N + 1,)
    forces = np.zeros((N, 3))
    ee = np.zeros(1)
    ip = ctypes.POINTER(ctypes.c_int)
    _check(_load().orc_ewald_excl(_ptr(pos), _ptr(q), N, _ptr(b), float(beta), float(coulomb),
                                  float(rcut), off.ctypes.data_as(ip), idx.ctypes.data_as(ip),
                                  _ptr(forces), _ptr(ee)), "orc_ewald_excl")
    return {"forces": forces, "E_excl": float(ee[0])}
