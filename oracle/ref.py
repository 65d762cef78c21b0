"""ctypes wrapper of the C oracle (tlb_oracle.c).

TEST INFRASTRUCTURE ONLY: the plain CPU reference that the HIP library is checked against.
Only tests, the smoke check and the benchmark's CPU-baseline leg may import this module.
It imports nothing from the GPU package.

All arrays crossing this boundary are host float64 numpy arrays:
    f   : (16, n_theta, n_phi), population k = 4 i + j (i: v^theta index, j: v^phi index)
    phi, n, u_theta, u_phi, mu : (n_theta, n_phi)
"""
import ctypes
import os

import numpy as np

from . import build as _build

FLAT = 1
CH_NO_ADVECTION = 2
WENO5 = 8
CH4 = 32

_DP = ctypes.POINTER(ctypes.c_double)


class _Params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_double), ("R", ctypes.c_double),
                ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("A", ctypes.c_double), ("kappa", ctypes.c_double), ("M", ctypes.c_double),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


_LIBS = {}


def _lib(bits=64):
    if bits not in _LIBS:
        path = _build.lib_path(bits)
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        lib.tlbref_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(vp)]
        lib.tlbref_create.restype = ctypes.c_int
        lib.tlbref_destroy.argtypes = [vp]
        lib.tlbref_destroy.restype = None
        lib.tlbref_set_state.argtypes = [vp, _DP, _DP, _DP, _DP, _DP]
        lib.tlbref_set_state.restype = ctypes.c_int
        lib.tlbref_get_state.argtypes = [vp, _DP, _DP]
        lib.tlbref_get_state.restype = ctypes.c_int
        lib.tlbref_step_n.argtypes = [vp, ctypes.c_int64]
        lib.tlbref_step_n.restype = ctypes.c_int
        lib.tlbref_get_moments.argtypes = [vp, _DP, _DP, _DP, _DP, _DP]
        lib.tlbref_get_moments.restype = ctypes.c_int
        lib.tlbref_invariants.argtypes = [vp, _DP]
        lib.tlbref_invariants.restype = ctypes.c_int
        lib.tlbref_rhs_terms.argtypes = [vp, _DP, _DP] + [_DP] * 10
        lib.tlbref_rhs_terms.restype = ctypes.c_int
        lib.tlbref_velocity_set.argtypes = [_DP, _DP, _DP, _DP]
        lib.tlbref_velocity_set.restype = None
        lib.tlbref_geometry.argtypes = [vp, _DP, _DP, _DP, _DP]
        lib.tlbref_geometry.restype = ctypes.c_int
        lib.tlbref_steps.argtypes = [vp]
        lib.tlbref_steps.restype = ctypes.c_int64
        lib.tlbref_diagnostics.argtypes = [vp, _DP, _DP, _DP]
        lib.tlbref_diagnostics.restype = ctypes.c_int
        lib.tlbref_uw5_face.argtypes = [_DP]
        lib.tlbref_uw5_face.restype = ctypes.c_double
        lib.tlbref_weno5_face.argtypes = [_DP, ctypes.c_double]
        lib.tlbref_weno5_face.restype = ctypes.c_double
        lib.tlbref_real_bytes.argtypes = []
        lib.tlbref_real_bytes.restype = ctypes.c_int
        _LIBS[bits] = lib
    return _LIBS[bits]


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_DP)


def uw5_face(h):
    """UW5 face value between h[2] and h[3] from h[0..4] (upwind side on the left)."""
    a = np.ascontiguousarray(h, dtype=np.float64)
    return float(_lib().tlbref_uw5_face(_ptr(a)))


def weno5_face(h, eps=1e-6):
    """WENO-5 (Jiang-Shu) face value between h[2] and h[3] from h[0..4]."""
    a = np.ascontiguousarray(h, dtype=np.float64)
    return float(_lib().tlbref_weno5_face(_ptr(a), float(eps)))


def velocity_set():
    """(v[4], w[4], K[4,4], Kt[4,4]) as computed by the oracle from Hermite polynomials."""
    v, w = np.zeros(4), np.zeros(4)
    K, Kt = np.zeros(16), np.zeros(16)
    _lib().tlbref_velocity_set(_ptr(v), _ptr(w), _ptr(K), _ptr(Kt))
    return v, w, K.reshape(4, 4), Kt.reshape(4, 4)


class RefGrid:
    """One torus (or flat, flags=FLAT) grid stepped by the CPU oracle."""

    def __init__(self, r, R, n_theta, n_phi, A, kappa, M, tau, dt, flags=0, bits=64):
        self.lib = _lib(bits)
        self.shape = (int(n_theta), int(n_phi))
        self.params = dict(r=r, R=R, n_theta=n_theta, n_phi=n_phi, A=A, kappa=kappa, M=M,
                           tau=tau, dt=dt, flags=flags)
        p = _Params(r, R, n_theta, n_phi, A, kappa, M, tau, dt, flags)
        h = ctypes.c_void_p()
        rc = self.lib.tlbref_create(ctypes.byref(p), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"tlbref_create failed ({rc}) for {self.params}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.tlbref_destroy(self._h)
            self._h = None

    __del__ = close

    def _scalar(self, a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        assert a.shape == self.shape, (a.shape, self.shape)
        return a

    def set_state(self, phi, n=None, u_theta=None, u_phi=None, f=None):
        phi = self._scalar(phi)
        if f is None:
            n, u_theta, u_phi = (self._scalar(x) for x in (n, u_theta, u_phi))
        else:
            f = np.ascontiguousarray(f, dtype=np.float64)
            assert f.shape == (16,) + self.shape
        rc = self.lib.tlbref_set_state(self._h, _ptr(f), _ptr(phi), _ptr(n), _ptr(u_theta),
                                       _ptr(u_phi))
        if rc != 0:
            raise ValueError(f"tlbref_set_state failed ({rc})")

    def step(self, nsteps):
        rc = self.lib.tlbref_step_n(self._h, int(nsteps))
        if rc != 0:
            raise ValueError(f"tlbref_step_n failed ({rc})")

    @property
    def steps(self):
        return int(self.lib.tlbref_steps(self._h))

    def get_state(self):
        f = np.zeros((16,) + self.shape)
        phi = np.zeros(self.shape)
        self.lib.tlbref_get_state(self._h, _ptr(f), _ptr(phi))
        return f, phi

    def moments(self):
        out = {k: np.zeros(self.shape) for k in ("n", "u_theta", "u_phi", "phi", "mu")}
        self.lib.tlbref_get_moments(self._h, *(_ptr(out[k]) for k in
                                               ("n", "u_theta", "u_phi", "phi", "mu")))
        return out

    def invariants(self):
        out = np.zeros(3)
        self.lib.tlbref_invariants(self._h, _ptr(out))
        return float(out[0]), float(out[1]), int(out[2])

    def rhs_terms(self, f, phi):
        f = np.ascontiguousarray(f, dtype=np.float64)
        phi = self._scalar(phi)
        big = ("Lf", "adv", "frc", "con", "bgk")
        small = ("Lphi", "mu", "lap", "Fth", "Fph")
        out = {k: np.zeros((16,) + self.shape) for k in big}
        out.update({k: np.zeros(self.shape) for k in small})
        rc = self.lib.tlbref_rhs_terms(self._h, _ptr(f), _ptr(phi), _ptr(out["Lf"]),
                                       _ptr(out["Lphi"]), _ptr(out["adv"]), _ptr(out["frc"]),
                                       _ptr(out["con"]), _ptr(out["bgk"]), _ptr(out["mu"]),
                                       _ptr(out["lap"]), _ptr(out["Fth"]), _ptr(out["Fph"]))
        if rc != 0:
            raise ValueError(f"tlbref_rhs_terms failed ({rc})")
        return out

    def diagnostics(self):
        """dict(L_I, A_total, L_d, phi_avg[n_theta], p_avg[n_theta]) of the current state."""
        out = np.zeros(2)
        pa = np.zeros(self.shape[0])
        pp = np.zeros(self.shape[0])
        self.lib.tlbref_diagnostics(self._h, _ptr(out), _ptr(pa), _ptr(pp))
        LI, A = float(out[0]), float(out[1])
        return dict(L_I=LI, A_total=A, L_d=(A / LI if LI > 0 else float("inf")), phi_avg=pa,
                    p_avg=pp)

    def geometry(self):
        nt = self.shape[0]
        J, Jp, Jm, G = (np.zeros(nt) for _ in range(4))
        self.lib.tlbref_geometry(self._h, _ptr(J), _ptr(Jp), _ptr(Jm), _ptr(G))
        return dict(J=J, Jp=Jp, Jm=Jm, G=G)
