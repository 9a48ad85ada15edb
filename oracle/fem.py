"""ORACLE -- test infrastructure only.

ctypes marshalling for ``oracle/fem.c`` (plain FP64 direct element loops).
``build()`` compiles the C file with gcc; ``lib()`` loads the shared object,
compiling it only when none exists.  Nothing here does arithmetic of the method.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fem.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)


def build():
    """Compile fem.c -> liboracle.so (gcc, FP64, OpenMP over elements)."""
    tmp = _SO + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _SO)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        mesh = [ctypes.c_int] * 5 + [_d, _d, _d, _d]
        L.or_num_nodes.restype = ctypes.c_int64
        L.or_num_nodes.argtypes = [ctypes.c_int] * 4
        L.or_gather_map.restype = None
        L.or_gather_map.argtypes = [ctypes.c_int] * 4 + [_i32]
        L.or_internal_force.restype = ctypes.c_int
        L.or_internal_force.argtypes = mesh + [_d, _d, _d, _d]
        L.or_tangent_apply.restype = ctypes.c_int
        L.or_tangent_apply.argtypes = mesh + [_d, _d, _d, _d, ctypes.c_double, _d]
        L.or_mass_apply.restype = None
        L.or_mass_apply.argtypes = mesh + [ctypes.c_double, _d, _d]
        L.or_tangent_diag.restype = ctypes.c_int
        L.or_tangent_diag.argtypes = mesh + [_d, _d, _d, ctypes.c_double, _d]
        L.or_strain_energy.restype = ctypes.c_double
        L.or_strain_energy.argtypes = mesh + [_d, _d, _d]
        L.or_material_grad.restype = None
        L.or_material_grad.argtypes = mesh + [_d, _d, ctypes.c_double, _d, _d]
        L.or_face_traction.restype = None
        L.or_face_traction.argtypes = mesh + [ctypes.c_int, _d, ctypes.c_int, _d, _d, _d]
        L.or_penalty_plane.restype = ctypes.c_double
        L.or_penalty_plane.argtypes = mesh + [ctypes.c_double] * 3 + [ctypes.c_int, _d, _d, _d, _d]
        _lib = L
    return _lib


def _p(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_d)


class Mesh:
    """Structured box of nx*ny*nz hexahedra with a 1D basis table set."""

    def __init__(self, nx, ny, nz, P, Q, h, B, D, w):
        self.nx, self.ny, self.nz, self.P, self.Q = nx, ny, nz, P, Q
        self.h = np.ascontiguousarray(h, dtype=np.float64)
        self.B = np.ascontiguousarray(B, dtype=np.float64)
        self.D = np.ascontiguousarray(D, dtype=np.float64)
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.E = nx * ny * nz
        self.Nx, self.Ny, self.Nz = nx * P + 1, ny * P + 1, nz * P + 1
        self.Nn = int(lib().or_num_nodes(nx, ny, nz, P))

    def _m(self):
        return (self.nx, self.ny, self.nz, self.P, self.Q, _p(self.h), _p(self.B), _p(self.D),
                _p(self.w))

    def vec(self):
        return np.zeros(3 * self.Nn)

    def gather_map(self):
        out = np.zeros(self.E * (self.P + 1) ** 3, dtype=np.int32)
        lib().or_gather_map(self.nx, self.ny, self.nz, self.P, out.ctypes.data_as(_i32))
        return out.reshape(self.E, -1)

    def internal_force(self, mu, lam, u):
        R = self.vec()
        bad = lib().or_internal_force(*self._m(), _p(mu), _p(lam), _p(u), _p(R))
        if bad:
            raise FloatingPointError("det F <= 0 at %d Gauss points" % bad)
        return R

    def tangent_apply(self, mu, lam, ulin, v, cm=0.0):
        y = self.vec()
        bad = lib().or_tangent_apply(*self._m(), _p(mu), _p(lam), _p(ulin), _p(v), cm, _p(y))
        if bad:
            raise FloatingPointError("det F <= 0 at %d Gauss points" % bad)
        return y

    def mass_apply(self, rho, v):
        y = self.vec()
        lib().or_mass_apply(*self._m(), rho, _p(v), _p(y))
        return y

    def tangent_diag(self, mu, lam, ulin, cm=0.0):
        d = self.vec()
        bad = lib().or_tangent_diag(*self._m(), _p(mu), _p(lam), _p(ulin), cm, _p(d))
        if bad:
            raise FloatingPointError("det F <= 0 at %d Gauss points" % bad)
        return d

    def strain_energy(self, mu, lam, u):
        return float(lib().or_strain_energy(*self._m(), _p(mu), _p(lam), _p(u)))

    def material_grad(self, u, wv, scale, g_mu, g_lam):
        lib().or_material_grad(*self._m(), _p(u), _p(wv), scale, _p(g_mu), _p(g_lam))

    def face_traction(self, face, t, Bf, wf, f):
        t = np.ascontiguousarray(t, dtype=np.float64)
        Bf = np.ascontiguousarray(Bf, dtype=np.float64)
        wf = np.ascontiguousarray(wf, dtype=np.float64)
        lib().or_face_traction(*self._m(), face, _p(t), len(wf), _p(Bf), _p(wf), _p(f))

    def penalty_plane(self, eps, z0, origin_z, Bf, wf, u, f):
        Bf = np.ascontiguousarray(Bf, dtype=np.float64)
        wf = np.ascontiguousarray(wf, dtype=np.float64)
        return float(lib().or_penalty_plane(*self._m(), eps, z0, origin_z, len(wf), _p(Bf),
                                            _p(wf), _p(u), _p(f)))
