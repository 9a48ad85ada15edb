"""Thin ctypes binding of libsdme (include/sdme.h): argument marshalling only.

Device arrays are torch tensors on the HIP device (``tensor.data_ptr()`` is
passed through); host arrays are numpy arrays.  Every entry point has the name
of the C function without the ``sdme_`` prefix.  Errors raise ``SdmeError``
with the library's status string.  The library must be built
(``paper_2104_13466_amd/libsdme.so``); nothing here computes on the CPU.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsdme.so")

FP64, FP32 = 0, 1
NODAL, MODAL, SDME_M, SDME_K, SDME_H = 0, 1, 2, 3, 4
MASK_BC, CHECK_JAC = 1, 2
OP_PCG, OP_NEWTON, OP_NEWMARK, OP_EXPLICIT, OP_ADJOINT = 0, 1, 2, 3, 4
STATUS = {0: "SDME_OK", -1: "SDME_EINVAL", -2: "SDME_ENOMEM", -3: "SDME_EDEVICE", -4: "SDME_EEIG",
          -5: "SDME_EJAC", -6: "SDME_ENOCONV", -7: "SDME_EBREAKDOWN", -8: "SDME_ENAN"}


class SdmeError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = _lib().sdme_status_string(code).decode() if _LIB is not None else str(code)
        super().__init__("%s: %s (%s)" % (where, STATUS.get(code, code), msg))


class MeshDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("P", ctypes.c_int), ("Q", ctypes.c_int), ("basis", ctypes.c_int),
                ("k", ctypes.c_double), ("lambda_h", ctypes.c_double),
                ("h", ctypes.c_double * 3), ("origin", ctypes.c_double * 3),
                ("dirichlet", ctypes.c_uint32), ("mass_rule", ctypes.c_int)]


class Material(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_void_p), ("lam", ctypes.c_void_p), ("rho", ctypes.c_double)]


class Contact(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("z0", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iterations", ctypes.c_int), ("outer", ctypes.c_int),
                ("newton", ctypes.c_int), ("mass_iterations", ctypes.c_int), ("pad", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("newton_rel", ctypes.c_double),
                ("time_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


_LIB = None
_vp, _d, _i, _dp = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
_i64, _sz = ctypes.c_int64, ctypes.c_size_t

# name -> argtypes (restype int unless noted)
SIGNATURES = {
    "sdme_status_string": ([_i], ctypes.c_char_p),
    "sdme_basis_build": ([_i, _i, _i, _d, _d, _dp, _dp, _dp, _dp, _dp, _dp, _dp], _i),
    "sdme_basis_eval": ([_i, _i, _d, _d, _i, _dp, _dp, _dp], _i),
    "sdme_create": ([ctypes.POINTER(MeshDesc), ctypes.POINTER(_vp)], _i),
    "sdme_destroy": ([_vp], _i),
    "sdme_sizes": ([_vp, ctypes.POINTER(_i64)], _i),
    "sdme_gather_indices": ([_vp, ctypes.POINTER(ctypes.c_int32)], _i),
    "sdme_dirichlet_flags": ([_vp, ctypes.POINTER(ctypes.c_uint8)], _i),
    "sdme_affine_field": ([_vp, _dp, _dp, _dp], _i),
    "sdme_internal_force": ([_vp, ctypes.POINTER(Material), _i, _vp, _vp, _vp, _i, _vp], _i),
    "sdme_linearize": ([_vp, ctypes.POINTER(Material), _i, _vp, _vp, _i, _vp], _i),
    "sdme_tangent_apply": ([_vp, ctypes.POINTER(Material), _i, _vp, _vp, _d, _vp, _vp, _i, _vp], _i),
    "sdme_mass_apply": ([_vp, _d, _i, _vp, _vp, _i, _vp], _i),
    "sdme_jacobi_diag": ([_vp, ctypes.POINTER(Material), _i, _vp, _d, _vp, _i, _vp], _i),
    "sdme_strain_energy": ([_vp, ctypes.POINTER(Material), _vp, _dp, _vp], _i),
    "sdme_face_traction": ([_vp, _i, _dp, _d, _vp, _vp], _i),
    "sdme_penalty_plane": ([_vp, ctypes.POINTER(Contact), _vp, _vp, _dp, _vp], _i),
    "sdme_quadrature_points": ([_vp, _i, _dp], _i),
    "sdme_body_load": ([_vp, _vp, _vp, _vp], _i),
    "sdme_face_load": ([_vp, _i, _vp, _vp, _vp], _i),
    "sdme_l2_error": ([_vp, _vp, _vp, _dp, _vp], _i),
    "sdme_material_grad_accumulate": ([_vp, _vp, _vp, _d, _vp, _vp, _vp], _i),
    "sdme_workspace_bytes": ([_vp, _i, _i, ctypes.POINTER(_sz)], _i),
    "sdme_jacobi_pcg": ([_vp, ctypes.POINTER(Material), _i, _vp, _d, _i, _vp, _vp, _d, _i, _d,
                         ctypes.POINTER(Stats), _vp, _sz, _vp], _i),
    "sdme_newton_static": ([_vp, ctypes.POINTER(Material), _i, _vp, _vp, _d, _d, _i, _i,
                            ctypes.POINTER(Stats), _vp, _sz, _vp], _i),
    "sdme_newmark_newton_step": ([_vp, ctypes.POINTER(Material), _i, _vp, _vp, _vp, _vp, _d, _d, _d,
                                  _d, _d, _i, _i, ctypes.POINTER(Stats), _vp, _sz, _vp], _i),
    "sdme_explicit_step": ([_vp, ctypes.POINTER(Material), _i, _vp, _vp, _vp, _vp, _vp, _d,
                            ctypes.POINTER(Contact), _d, ctypes.POINTER(Stats), _vp, _sz, _vp], _i),
    "sdme_energies": ([_vp, ctypes.POINTER(Material), _vp, _vp, _vp, _d, ctypes.POINTER(Contact),
                       _dp, _vp, _sz, _vp], _i),
    "sdme_lambda_max": ([_vp, ctypes.POINTER(Material), _vp, ctypes.POINTER(Contact), _vp, _i, _d,
                         _dp, _vp, _sz, _vp], _i),
    "sdme_explicit_adjoint_step": ([_vp, ctypes.POINTER(Material), _vp, _vp, _vp, _vp, _d, _i, _d,
                                    _vp, _vp, ctypes.POINTER(Stats), _vp, _sz, _vp], _i),
    "sdme_misfit": ([_vp, _vp, _vp, _vp, _dp, _vp], _i),
    "sdme_axpby": ([_vp, _i64, _d, _vp, _d, _vp, _vp], _i),
    "sdme_profile": ([_vp, _i, _dp, ctypes.POINTER(_i64)], _i),
}


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsdme.so is not built (run python -m "
                              "paper_2104_13466_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _LIB = L
    return _LIB


def lib_path():
    return LIB_PATH


def _chk(rc, where):
    if rc != 0:
        raise SdmeError(rc, where)


def _hp(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def basis_build(P, Q, kind, k=0.5, lambda_h=100.0):
    """Host tables: dict with x, w, B, D, M1, K1, lambda_s (numpy)."""
    n = P + 1
    out = dict(x=np.zeros(Q), w=np.zeros(Q), B=np.zeros((Q, n)), D=np.zeros((Q, n)),
               M1=np.zeros((n, n)), K1=np.zeros((n, n)), lambda_s=np.zeros(max(P - 1, 1)))
    _chk(_lib().sdme_basis_build(P, Q, kind, k, lambda_h, _hp(out["x"]), _hp(out["w"]),
                                 _hp(out["B"]), _hp(out["D"]), _hp(out["M1"]), _hp(out["K1"]),
                                 _hp(out["lambda_s"])), "basis_build")
    out["lambda_s"] = out["lambda_s"][:max(P - 1, 0)]
    return out


def basis_eval(P, kind, pts, k=0.5, lambda_h=100.0):
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    V = np.zeros((pts.size, P + 1))
    dV = np.zeros((pts.size, P + 1))
    _chk(_lib().sdme_basis_eval(P, kind, k, lambda_h, pts.size, _hp(pts), _hp(V), _hp(dV)),
         "basis_eval")
    return V, dV


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Context:
    """Structured box mesh + basis (sdme_create / sdme_destroy)."""

    def __init__(self, n, L, P, basis=SDME_H, k=0.5, lambda_h=100.0, dirichlet=0, origin=(0, 0, 0),
                 Q=None, lumped_mass=False):
        self.L = _lib()
        self.P, self.Q = P, (P + 2 if Q is None else Q)
        d = MeshDesc()
        d.nx, d.ny, d.nz = n
        d.P, d.Q, d.basis = P, self.Q, basis
        d.k, d.lambda_h = k, lambda_h
        for i in range(3):
            d.h[i] = L[i] / n[i] if n[i] > 0 else 0.0
            d.origin[i] = origin[i]
        d.dirichlet = dirichlet
        d.mass_rule = 1 if lumped_mass else 0
        self.desc = d
        self.n = tuple(n)
        self.h = [d.h[i] for i in range(3)]
        h = ctypes.c_void_p()
        _chk(self.L.sdme_create(ctypes.byref(d), ctypes.byref(h)), "create")
        self.handle = h
        sz = (ctypes.c_int64 * 4)()
        _chk(self.L.sdme_sizes(h, sz), "sizes")
        self.Nn, self.E, self.nqp, self.state_words = (int(v) for v in sz)
        self._ws = None

    def close(self):
        if getattr(self, "handle", None):
            self.L.sdme_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ host helpers
    def gather_indices(self):
        out = np.zeros(self.E * (self.P + 1) ** 3, dtype=np.int32)
        _chk(self.L.sdme_gather_indices(self.handle, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_int32))), "gather_indices")
        return out.reshape(self.E, -1)

    def dirichlet_flags(self):
        out = np.zeros(3 * self.Nn, dtype=np.uint8)
        _chk(self.L.sdme_dirichlet_flags(self.handle, out.ctypes.data_as(
            ctypes.POINTER(ctypes.c_uint8))), "dirichlet_flags")
        return out

    def affine_field(self, a, G):
        out = np.zeros(3 * self.Nn)
        a = np.ascontiguousarray(a, dtype=np.float64)
        G = np.ascontiguousarray(np.asarray(G, dtype=np.float64).reshape(9))
        _chk(self.L.sdme_affine_field(self.handle, _hp(a), _hp(G), _hp(out)), "affine_field")
        return out

    # ------------------------------------------------------------- workspace
    def workspace_bytes(self, op, prec):
        b = ctypes.c_size_t()
        _chk(self.L.sdme_workspace_bytes(self.handle, op, prec, ctypes.byref(b)), "workspace_bytes")
        return b.value

    def workspace(self, nbytes, device="cuda"):
        import torch
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self._ws

    def _wsargs(self, op, prec):
        nb = self.workspace_bytes(op, prec)
        ws = self.workspace(nb)
        return ctypes.c_void_p(ws.data_ptr()), ctypes.c_size_t(ws.numel())

    @staticmethod
    def material(mu, lam, rho):
        m = Material()
        m.mu = mu.data_ptr()
        m.lam = lam.data_ptr()
        m.rho = rho
        m._keep = (mu, lam)
        return m

    # -------------------------------------------------------------- operators
    def internal_force(self, mat, prec, u, R, state=None, flags=0, stream=None):
        _chk(self.L.sdme_internal_force(self.handle, ctypes.byref(mat), prec, _ptr(u), _ptr(R),
                                        _ptr(state), flags, _stream(stream)), "internal_force")

    def linearize(self, mat, prec, u, state, flags=0, stream=None):
        _chk(self.L.sdme_linearize(self.handle, ctypes.byref(mat), prec, _ptr(u), _ptr(state), flags,
                                   _stream(stream)), "linearize")

    def tangent_apply(self, mat, prec, v, y, u_lin=None, state=None, mass_shift=0.0, flags=0,
                      stream=None):
        _chk(self.L.sdme_tangent_apply(self.handle, ctypes.byref(mat), prec, _ptr(u_lin),
                                       _ptr(state), mass_shift, _ptr(v), _ptr(y), flags,
                                       _stream(stream)), "tangent_apply")

    def mass_apply(self, rho, prec, v, y, flags=0, stream=None):
        _chk(self.L.sdme_mass_apply(self.handle, rho, prec, _ptr(v), _ptr(y), flags,
                                    _stream(stream)), "mass_apply")

    def jacobi_diag(self, mat, prec, state, mass_shift, d, flags=0, stream=None):
        _chk(self.L.sdme_jacobi_diag(self.handle, ctypes.byref(mat), prec, _ptr(state), mass_shift,
                                     _ptr(d), flags, _stream(stream)), "jacobi_diag")

    def strain_energy(self, mat, u, stream=None):
        out = ctypes.c_double()
        _chk(self.L.sdme_strain_energy(self.handle, ctypes.byref(mat), _ptr(u), ctypes.byref(out),
                                       _stream(stream)), "strain_energy")
        return out.value

    def face_traction(self, face, t, f, scale=1.0, stream=None):
        t = np.ascontiguousarray(t, dtype=np.float64)
        _chk(self.L.sdme_face_traction(self.handle, face, _hp(t), scale, _ptr(f), _stream(stream)),
             "face_traction")

    def penalty_plane(self, eps, z0, u, f, energy=False, stream=None):
        c = Contact(eps, z0)
        e = ctypes.c_double()
        _chk(self.L.sdme_penalty_plane(self.handle, ctypes.byref(c), _ptr(u), _ptr(f),
                                       ctypes.byref(e) if energy else None, _stream(stream)),
             "penalty_plane")
        return e.value if energy else None

    # ------------------------------------------ loads at quadrature points
    def face_elements(self, face):
        """Number of element faces on box face `face` (0..5)."""
        d = face // 2
        t1, t2 = (1, 2) if d == 0 else ((0, 2) if d == 1 else (0, 1))
        return self.n[t1] * self.n[t2]

    def quadrature_points(self, face=-1):
        """Coordinates of the volume Gauss points, shape (3, E, Q^3) (face = -1),
        or of the face Gauss points of face 0..5, shape (3, nfe, (P+1)^2)."""
        if face < 0:
            shape = (3, self.E, self.Q ** 3)
        else:
            shape = (3, self.face_elements(face), (self.P + 1) ** 2)
        out = np.zeros(shape)
        _chk(self.L.sdme_quadrature_points(self.handle, face, _hp(out)), "quadrature_points")
        return out

    def body_load(self, b, f, stream=None):
        _chk(self.L.sdme_body_load(self.handle, _ptr(b), _ptr(f), _stream(stream)), "body_load")

    def face_load(self, face, t, f, stream=None):
        _chk(self.L.sdme_face_load(self.handle, face, _ptr(t), _ptr(f), _stream(stream)),
             "face_load")

    def l2_error(self, u, g, stream=None):
        """L2 norms over the box of (u_h - g) per component; g at the volume
        Gauss points (3, E, Q^3)."""
        out = np.zeros(3)
        _chk(self.L.sdme_l2_error(self.handle, _ptr(u), _ptr(g), _hp(out), _stream(stream)),
             "l2_error")
        return out

    def material_grad_accumulate(self, u, w, scale, g_mu, g_lam, stream=None):
        _chk(self.L.sdme_material_grad_accumulate(self.handle, _ptr(u), _ptr(w), scale, _ptr(g_mu),
                                                  _ptr(g_lam), _stream(stream)),
             "material_grad_accumulate")

    def axpby(self, alpha, x, beta, y, stream=None):
        _chk(self.L.sdme_axpby(self.handle, y.numel(), alpha, _ptr(x), beta, _ptr(y),
                               _stream(stream)), "axpby")

    def profile(self, enable):
        """Return {fp64_ms, fp64_count, fp32_ms, fp32_count} accumulated since
        the previous call, then reset and switch PCG-operator timing on/off."""
        ms = (ctypes.c_double * 2)()
        cnt = (ctypes.c_int64 * 2)()
        _chk(self.L.sdme_profile(self.handle, 1 if enable else 0, ms, cnt), "profile")
        return dict(fp64_ms=ms[0], fp64_count=cnt[0], fp32_ms=ms[1], fp32_count=cnt[1])

    def misfit(self, u, target, lam_out, stream=None):
        J = ctypes.c_double()
        _chk(self.L.sdme_misfit(self.handle, _ptr(u), _ptr(target), _ptr(lam_out), ctypes.byref(J),
                                _stream(stream)), "misfit")
        return J.value

    # ---------------------------------------------------------------- solvers
    def jacobi_pcg(self, mat, prec, b, x, u_lin=None, mass_shift=0.0, mass_only=False, rtol=1e-8,
                   maxit=100000, inner_rtol=1e-2, stream=None, check=True):
        st = Stats()
        ws, nb = self._wsargs(OP_PCG, prec)
        rc = self.L.sdme_jacobi_pcg(self.handle, ctypes.byref(mat), prec, _ptr(u_lin), mass_shift,
                                    1 if mass_only else 0, _ptr(b), _ptr(x), rtol, maxit,
                                    inner_rtol, ctypes.byref(st), ws, nb, _stream(stream))
        if check:
            _chk(rc, "jacobi_pcg")
        return st.as_dict()

    def newton_static(self, mat, prec, u, f_ext=None, newton_rtol=1e-8, pcg_rtol=1e-8,
                      max_newton=20, max_pcg=100000, stream=None):
        st = Stats()
        ws, nb = self._wsargs(OP_NEWTON, prec)
        _chk(self.L.sdme_newton_static(self.handle, ctypes.byref(mat), prec, _ptr(u), _ptr(f_ext),
                                       newton_rtol, pcg_rtol, max_newton, max_pcg, ctypes.byref(st),
                                       ws, nb, _stream(stream)), "newton_static")
        return st.as_dict()

    def newmark_newton_step(self, mat, prec, u, v, a, f_next, dt, beta=0.25, gamma=0.5,
                            newton_rtol=1e-8, pcg_rtol=1e-8, max_newton=20, max_pcg=100000,
                            stream=None):
        st = Stats()
        ws, nb = self._wsargs(OP_NEWMARK, prec)
        _chk(self.L.sdme_newmark_newton_step(self.handle, ctypes.byref(mat), prec, _ptr(u), _ptr(v),
                                             _ptr(a), _ptr(f_next), dt, beta, gamma, newton_rtol,
                                             pcg_rtol, max_newton, max_pcg, ctypes.byref(st), ws,
                                             nb, _stream(stream)), "newmark_newton_step")
        return st.as_dict()

    def explicit_step(self, mat, prec_force, u_prev, u_cur, u_next, dt, v0=None, f_ext=None,
                      contact=None, mass_rtol=1e-10, stream=None):
        st = Stats()
        ws, nb = self._wsargs(OP_EXPLICIT, FP64)
        c = None if contact is None else ctypes.byref(Contact(*contact))
        _chk(self.L.sdme_explicit_step(self.handle, ctypes.byref(mat), prec_force, _ptr(u_prev),
                                       _ptr(u_cur), _ptr(u_next), _ptr(v0), _ptr(f_ext), dt, c,
                                       mass_rtol, ctypes.byref(st), ws, nb, _stream(stream)),
             "explicit_step")
        return st.as_dict()

    def energies(self, mat, u_prev, u_cur, u_next, dt, contact=None, stream=None):
        out = (ctypes.c_double * 3)()
        ws, nb = self._wsargs(OP_EXPLICIT, FP64)
        c = None if contact is None else ctypes.byref(Contact(*contact))
        _chk(self.L.sdme_energies(self.handle, ctypes.byref(mat), _ptr(u_prev), _ptr(u_cur),
                                  _ptr(u_next), dt, c, out, ws, nb, _stream(stream)), "energies")
        return tuple(out)

    def lambda_max(self, mat, u_lin, x0, iters=50, contact=None, mass_rtol=1e-10, stream=None):
        lam = ctypes.c_double()
        nb = self.workspace_bytes(OP_EXPLICIT, FP64) + self.nqp * 80 + 4096
        ws = self.workspace(nb)
        c = None if contact is None else ctypes.byref(Contact(*contact))
        _chk(self.L.sdme_lambda_max(self.handle, ctypes.byref(mat), _ptr(u_lin), c, _ptr(x0), iters,
                                    mass_rtol, ctypes.byref(lam), ctypes.c_void_p(ws.data_ptr()),
                                    ctypes.c_size_t(ws.numel()), _stream(stream)), "lambda_max")
        return lam.value

    def explicit_adjoint_step(self, mat, u_n, lam_next, lam_next2, lam_out, dt, first, g_mu, g_lam,
                              mass_rtol=1e-12, stream=None):
        st = Stats()
        ws, nb = self._wsargs(OP_ADJOINT, FP64)
        _chk(self.L.sdme_explicit_adjoint_step(self.handle, ctypes.byref(mat), _ptr(u_n),
                                               _ptr(lam_next), _ptr(lam_next2), _ptr(lam_out), dt,
                                               1 if first else 0, mass_rtol, _ptr(g_mu),
                                               _ptr(g_lam), ctypes.byref(st), ws, nb,
                                               _stream(stream)), "explicit_adjoint_step")
        return st.as_dict()
