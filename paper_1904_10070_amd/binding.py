"""Thin ctypes binding of the C interface in include/tlb.h and include/tlb_learn.h.

Argument marshalling only: PyTorch provides the device buffers and the stream, and every step
of the method runs in the HIP kernels of libtlb.so.  There is no fallback: if the library has
not been built, or no GPU is visible, the calls raise.
"""
import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtlb.so")

TLB_OK = 0
TLB_EINVAL = -1
TLB_ENOMEM = -2
TLB_EHIP = -3
TLB_ENONFINITE = -4
TLB_EUNSTABLE = -5

FLAT = 1
CH_NO_ADVECTION = 2
NO_GRAPH = 4
WENO5 = 8
STRICT_DT = 16
CH4 = 32

EXPORTED = ("tlb_stable_dt", "tlb_create_torus_grid", "tlb_set_state", "tlb_step_n", "tlb_get_moments",
            "tlb_get_state", "tlb_invariants", "tlb_diagnostics", "tlb_destroy",
            "tlb_last_error", "tlb_set_tile_rows", "tlb_autotune", "tlb_create_batch",
            "tlb_batch_step_n", "tlb_batch_autotune", "tlb_destroy_batch", "tlb_structure_length",
            "tlb_structure_length_noalloc",
            "tlb_cnn_create", "tlb_cnn_destroy", "tlb_cnn_set_params", "tlb_cnn_get_params",
            "tlb_cnn_forward", "tlb_cnn_gradient", "tlb_cnn_train_step", "tlb_learn_stats",
            "tlb_restrict", "tlb_learn_pair", "tlb_apply_correction", "tlb_learned_step_n",
            "tlb_hbm_stream")

CNN_PARAMS = 30660


class TlbError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_double), ("R", ctypes.c_double),
                ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("A", ctypes.c_double), ("kappa", ctypes.c_double), ("M", ctypes.c_double),
                ("tau", ctypes.c_double), ("dt", ctypes.c_double),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("check_every", ctypes.c_int32)]


class Buffers(ctypes.Structure):
    _fields_ = [("f", ctypes.c_void_p * 3), ("phi", ctypes.c_void_p * 3)]


class CnnDesc(ctypes.Structure):
    _fields_ = [("r", ctypes.c_double), ("R", ctypes.c_double),
                ("n_theta", ctypes.c_int32), ("n_phi", ctypes.c_int32),
                ("max_batch", ctypes.c_int32), ("apply_mask", ctypes.c_uint32),
                ("in_shift", ctypes.c_float * 4), ("in_scale", ctypes.c_float * 4),
                ("out_scale", ctypes.c_float * 4), ("loss_weight", ctypes.c_float * 4)]


class Adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("step", ctypes.c_int32)]


_LIB = None


def load_library(path=None):
    """Load libtlb.so and declare its signatures; raises if it has not been built.

    TLB_LIBRARY in the environment selects another build of the same source (tuning runs)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or os.environ.get("TLB_LIBRARY") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not found: build it first (python -m paper_1904_10070_amd.build)")
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.tlb_stable_dt.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_double)]
    lib.tlb_stable_dt.restype = i32
    lib.tlb_create_torus_grid.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Buffers), vp,
                                          ctypes.POINTER(vp)]
    lib.tlb_create_torus_grid.restype = i32
    lib.tlb_set_state.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.tlb_set_state.restype = i32
    lib.tlb_step_n.argtypes = [vp, i64]
    lib.tlb_step_n.restype = i32
    lib.tlb_get_moments.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.tlb_get_moments.restype = i32
    lib.tlb_get_state.argtypes = [vp, vp, vp]
    lib.tlb_get_state.restype = i32
    lib.tlb_invariants.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.tlb_invariants.restype = i32
    lib.tlb_diagnostics.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp, vp]
    lib.tlb_diagnostics.restype = i32
    lib.tlb_structure_length.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.tlb_structure_length.restype = i32
    lib.tlb_structure_length_noalloc.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.tlb_structure_length_noalloc.restype = i32
    lib.tlb_set_tile_rows.argtypes = [vp, i32]
    lib.tlb_set_tile_rows.restype = i32
    lib.tlb_autotune.argtypes = [vp, ctypes.POINTER(i32)]
    lib.tlb_autotune.restype = i32
    lib.tlb_create_batch.argtypes = [ctypes.POINTER(vp), i32, vp, ctypes.POINTER(vp)]
    lib.tlb_create_batch.restype = i32
    lib.tlb_batch_step_n.argtypes = [vp, i64]
    lib.tlb_batch_step_n.restype = i32
    lib.tlb_batch_autotune.argtypes = [vp, ctypes.POINTER(i32)]
    lib.tlb_batch_autotune.restype = i32
    lib.tlb_destroy_batch.argtypes = [vp]
    lib.tlb_destroy_batch.restype = None
    lib.tlb_destroy.argtypes = [vp]
    lib.tlb_destroy.restype = None
    lib.tlb_last_error.argtypes = []
    lib.tlb_last_error.restype = ctypes.c_char_p
    dp, fp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_float)
    lib.tlb_cnn_create.argtypes = [ctypes.POINTER(CnnDesc), vp, ctypes.POINTER(vp)]
    lib.tlb_cnn_destroy.argtypes = [vp]
    lib.tlb_cnn_destroy.restype = None
    lib.tlb_cnn_set_params.argtypes = [vp, fp]
    lib.tlb_cnn_get_params.argtypes = [vp, fp]
    lib.tlb_cnn_forward.argtypes = [vp, vp, vp, i32, vp]
    lib.tlb_cnn_gradient.argtypes = [vp, vp, vp, vp, i32, dp, fp]
    lib.tlb_cnn_train_step.argtypes = [vp, vp, vp, vp, i32, ctypes.POINTER(Adam), dp]
    lib.tlb_learn_stats.argtypes = [vp, i64, vp, dp]
    lib.tlb_restrict.argtypes = [vp, vp]
    lib.tlb_learn_pair.argtypes = [vp, vp, vp, vp]
    lib.tlb_apply_correction.argtypes = [vp, vp]
    lib.tlb_learned_step_n.argtypes = [vp, vp, i64]
    lib.tlb_hbm_stream.argtypes = [i32, vp, vp, vp, i64, vp]
    lib.tlb_hbm_stream.restype = i32
    for name in ("tlb_cnn_create", "tlb_cnn_set_params", "tlb_cnn_get_params",
                 "tlb_cnn_forward", "tlb_cnn_gradient", "tlb_cnn_train_step", "tlb_learn_stats",
                 "tlb_restrict", "tlb_learn_pair", "tlb_apply_correction", "tlb_learned_step_n"):
        getattr(lib, name).restype = i32
    _LIB = lib
    return lib


def _check(lib, rc, what):
    if rc != TLB_OK:
        raise TlbError(rc, f"{what}: {lib.tlb_last_error().decode()}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def stable_dt(params, precision=64):
    """Explicit stability bound of the time step (tlb_stable_dt; host only, no GPU needed)."""
    lib = load_library()
    p = Params(params.r, params.R, int(params.n_theta), int(params.n_phi), params.A, params.kappa,
               params.M, params.tau, params.dt, precision, int(getattr(params, "flags", 0)), 0)
    out = ctypes.c_double()
    _check(lib, lib.tlb_stable_dt(ctypes.byref(p), ctypes.byref(out)), "tlb_stable_dt")
    return out.value


class TorusGrid:
    """A torus grid whose state lives in torch-owned device memory and is stepped by libtlb.

    params: an object with the fields of tlb_params (e.g. inputs.TorusParams).
    precision: 32 or 64.  stream: a torch.cuda.Stream (default: the current stream).
    check_every: tlb_params.check_every (0: no non-finite checks in step()).
    buffers: optional (f, phi), two lists of three torch tensors to use as the state copies
    instead of new ones (e.g. those of a grid closed before).
    """

    def __init__(self, params, precision=64, device="cuda", stream=None, check_every=0,
                 buffers=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the torus step runs only in the HIP kernels")
        self.device = torch.device(device)
        self.dtype = torch.float64 if precision == 64 else torch.float32
        self.precision = precision
        self.params = params
        nt, np_ = int(params.n_theta), int(params.n_phi)
        self.shape = (nt, np_)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # state copies: 0 = current state, 1 and 2 = Runge-Kutta stage scratch
        if buffers is not None:
            self.f, self.phi = list(buffers[0]), list(buffers[1])
            for t in self.f + self.phi:
                assert t.dtype == self.dtype and t.is_contiguous() and t.is_cuda
            assert all(tuple(t.shape) == (16, nt, np_) for t in self.f)
            assert all(tuple(t.shape) == (nt, np_) for t in self.phi)
        else:
            self.f = [torch.zeros((16, nt, np_), dtype=self.dtype, device=self.device)
                      for _ in range(3)]
            self.phi = [torch.zeros((nt, np_), dtype=self.dtype, device=self.device)
                        for _ in range(3)]
        p = Params(params.r, params.R, nt, np_, params.A, params.kappa, params.M, params.tau,
                   params.dt, precision, int(getattr(params, "flags", 0)), int(check_every))
        b = Buffers()
        for i in range(3):
            b.f[i] = self.f[i].data_ptr()
            b.phi[i] = self.phi[i].data_ptr()
        h = ctypes.c_void_p()
        torch.cuda.synchronize(self.device)
        _check(self.lib, self.lib.tlb_create_torus_grid(ctypes.byref(p), ctypes.byref(b),
                                                        ctypes.c_void_p(self.stream.cuda_stream),
                                                        ctypes.byref(h)), "tlb_create_torus_grid")
        self._h = h

    # -- helpers ------------------------------------------------------------------------------
    def _dev(self, x, shape):
        t = self.torch.as_tensor(np.asarray(x) if not isinstance(x, self.torch.Tensor) else x)
        t = t.to(device=self.device, dtype=self.dtype).contiguous()
        assert tuple(t.shape) == shape, (tuple(t.shape), shape)
        return t

    def close(self):
        if getattr(self, "_h", None):
            self.lib.tlb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C interface ------------------------------------------------------------------------
    def set_state(self, phi, n=None, u_theta=None, u_phi=None, f=None):
        with self.torch.cuda.stream(self.stream):
            phi_t = self._dev(phi, self.shape)
            if f is not None:
                f_t = self._dev(f, (16,) + self.shape)
                args = (f_t, phi_t, None, None, None)
            else:
                args = (None, phi_t, self._dev(n, self.shape), self._dev(u_theta, self.shape),
                        self._dev(u_phi, self.shape))
            _check(self.lib, self.lib.tlb_set_state(self._h, *(_ptr(a) for a in args)),
                   "tlb_set_state")
            self._keep = args  # keep the inputs alive until the stream has consumed them

    def step(self, nsteps):
        _check(self.lib, self.lib.tlb_step_n(self._h, int(nsteps)), "tlb_step_n")

    def moments(self, with_mu=True):
        out = {k: self.torch.empty(self.shape, dtype=self.dtype, device=self.device)
               for k in ("n", "u_theta", "u_phi", "phi")}
        out["mu"] = (self.torch.empty(self.shape, dtype=self.dtype, device=self.device)
                     if with_mu else None)
        _check(self.lib, self.lib.tlb_get_moments(self._h, *(_ptr(out[k]) for k in
                                                             ("n", "u_theta", "u_phi", "phi", "mu"))),
               "tlb_get_moments")
        return out

    def get_state(self):
        f = self.torch.empty((16,) + self.shape, dtype=self.dtype, device=self.device)
        phi = self.torch.empty(self.shape, dtype=self.dtype, device=self.device)
        _check(self.lib, self.lib.tlb_get_state(self._h, _ptr(f), _ptr(phi)), "tlb_get_state")
        return f, phi

    def invariants(self, check=False):
        out = (ctypes.c_double * 3)()
        rc = self.lib.tlb_invariants(self._h, out)
        if rc not in (TLB_OK, TLB_ENONFINITE) or (check and rc != TLB_OK):
            _check(self.lib, rc, "tlb_invariants")
        return float(out[0]), float(out[1]), int(out[2])

    def diagnostics(self, profiles=True):
        """dict(L_I, A_total, L_d, phi_avg, p_avg): phi_avg / p_avg are float64 device tensors
        of n_theta values (or None with profiles=False)."""
        out = (ctypes.c_double * 2)()
        pa = pp = None
        if profiles:
            pa = self.torch.empty(self.shape[0], dtype=self.torch.float64, device=self.device)
            pp = self.torch.empty(self.shape[0], dtype=self.torch.float64, device=self.device)
        _check(self.lib, self.lib.tlb_diagnostics(self._h, out, _ptr(pa), _ptr(pp)),
               "tlb_diagnostics")
        LI, A = float(out[0]), float(out[1])
        return dict(L_I=LI, A_total=A, L_d=(A / LI if LI > 0 else float("inf")), phi_avg=pa,
                    p_avg=pp)

    def structure_length(self):
        """(L_S, sum S, sum |k| S) of phi: the structure-factor coarsening length."""
        out = (ctypes.c_double * 3)()
        _check(self.lib, self.lib.tlb_structure_length(self._h, out), "tlb_structure_length")
        return float(out[0]), float(out[1]), float(out[2])

    def structure_length_noalloc(self):
        """structure_length() through tlb_structure_length_noalloc (no allocation)."""
        out = (ctypes.c_double * 3)()
        _check(self.lib, self.lib.tlb_structure_length_noalloc(self._h, out),
               "tlb_structure_length_noalloc")
        return float(out[0]), float(out[1]), float(out[2])

    def set_tile_rows(self, rows):
        _check(self.lib, self.lib.tlb_set_tile_rows(self._h, int(rows)), "tlb_set_tile_rows")

    def autotune(self):
        rows = ctypes.c_int32()
        _check(self.lib, self.lib.tlb_autotune(self._h, ctypes.byref(rows)), "tlb_autotune")
        return rows.value


class TorusBatch:
    """An ensemble of TorusGrid objects advanced together by one fused launch per stage."""

    def __init__(self, grids, stream=None):
        import torch
        self.lib = load_library()
        self.grids = list(grids)
        self.stream = stream if stream is not None else self.grids[0].stream
        arr = (ctypes.c_void_p * len(self.grids))(*[g._h.value for g in self.grids])
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(self.lib, self.lib.tlb_create_batch(arr, len(self.grids),
                                                   ctypes.c_void_p(self.stream.cuda_stream),
                                                   ctypes.byref(h)), "tlb_create_batch")
        self._h = h

    def step(self, nsteps):
        _check(self.lib, self.lib.tlb_batch_step_n(self._h, int(nsteps)), "tlb_batch_step_n")

    def autotune(self):
        rows = ctypes.c_int32()
        _check(self.lib, self.lib.tlb_batch_autotune(self._h, ctypes.byref(rows)),
               "tlb_batch_autotune")
        return rows.value

    def close(self):
        if getattr(self, "_h", None):
            self.lib.tlb_destroy_batch(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- the learned coarse-step correction (include/tlb_learn.h) ---------------------------------------

def _f32(t, shape=None):
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), "float32 device tensor"
    if shape is not None:
        assert tuple(t.shape[-len(shape):]) == tuple(shape), (tuple(t.shape), shape)
    return ctypes.c_void_p(t.data_ptr())


def _idx(idx):
    import torch
    if idx is None:
        return None, None
    t = torch.as_tensor(idx, dtype=torch.int32).to("cuda").contiguous()
    return t, ctypes.c_void_p(t.data_ptr())


class CoarseCNN:
    """The periodic five-layer 3x3 network of tlb_learn.h, trained and run by libtlb's kernels.

    r, R, n_theta, n_phi: the torus and grid it runs on; max_batch: largest batch of samples;
    in_shift / in_scale (4 each), out_scale (4), loss_weight (4), apply_mask: as in
    tlb_cnn_desc."""

    def __init__(self, r, R, n_theta, n_phi, max_batch, in_shift, in_scale, out_scale,
                 loss_weight=(1.0, 1.0, 1.0, 1.0), apply_mask=0, stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the network runs only in the HIP kernels")
        self.shape = (int(n_theta), int(n_phi))
        self.max_batch = int(max_batch)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        d = CnnDesc(float(r), float(R), int(n_theta), int(n_phi), int(max_batch), int(apply_mask))
        for name, vals in (("in_shift", in_shift), ("in_scale", in_scale),
                           ("out_scale", out_scale), ("loss_weight", loss_weight)):
            arr = getattr(d, name)
            for c in range(4):
                arr[c] = float(vals[c])
        self.desc = d
        h = ctypes.c_void_p()
        torch.cuda.synchronize()
        _check(self.lib, self.lib.tlb_cnn_create(ctypes.byref(d), ctypes.c_void_p(self.stream.cuda_stream),
                                                 ctypes.byref(h)), "tlb_cnn_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self.lib.tlb_cnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        assert p.shape == (CNN_PARAMS,)
        _check(self.lib, self.lib.tlb_cnn_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "tlb_cnn_set_params")

    def get_params(self):
        p = np.zeros(CNN_PARAMS, dtype=np.float32)
        _check(self.lib, self.lib.tlb_cnn_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "tlb_cnn_get_params")
        return p

    def forward(self, moments, idx=None, n=None):
        """moments: float32 device tensor [*, n_theta, n_phi, 4]; returns corrections [n, ..., 4]."""
        t, ip = _idx(idx)
        n = int(len(idx) if idx is not None else (n if n is not None else moments.shape[0]))
        out = self.torch.empty((n,) + self.shape + (4,), dtype=self.torch.float32, device="cuda")
        _check(self.lib, self.lib.tlb_cnn_forward(self._h, _f32(moments, self.shape + (4,)), ip, n,
                                                  _f32(out)), "tlb_cnn_forward")
        self._keep = t
        return out

    def gradient(self, moments, targets, idx=None, n=None):
        """(loss, gradient as float32 numpy array) on a batch; weights unchanged."""
        t, ip = _idx(idx)
        n = int(len(idx) if idx is not None else (n if n is not None else moments.shape[0]))
        loss = ctypes.c_double()
        g = np.zeros(CNN_PARAMS, dtype=np.float32)
        _check(self.lib, self.lib.tlb_cnn_gradient(self._h, _f32(moments, self.shape + (4,)),
                                                   _f32(targets, self.shape + (4,)), ip, n,
                                                   ctypes.byref(loss),
                                                   g.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "tlb_cnn_gradient")
        return loss.value, g

    def train_step(self, moments, targets, idx, step, lr, beta1=0.9, beta2=0.999, eps=1e-8,
                   want_loss=False):
        t, ip = _idx(idx)
        adam = Adam(float(lr), float(beta1), float(beta2), float(eps), int(step))
        loss = ctypes.c_double()
        _check(self.lib, self.lib.tlb_cnn_train_step(self._h, _f32(moments, self.shape + (4,)),
                                                     _f32(targets, self.shape + (4,)), ip, len(idx),
                                                     ctypes.byref(adam),
                                                     ctypes.byref(loss) if want_loss else None),
               "tlb_cnn_train_step")
        self._keep = t
        return loss.value if want_loss else None


def learn_stats(data, stream=None):
    """(sum, sum of squares) of each of the 4 channels of a float32 device tensor [..., 4]."""
    import torch
    lib = load_library()
    out = (ctypes.c_double * 8)()
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib, lib.tlb_learn_stats(_f32(data), int(data.numel() // 4), ctypes.c_void_p(s.cuda_stream), out),
           "tlb_learn_stats")
    return np.array(out[:4]), np.array(out[4:])


def restrict(fine, coarse):
    """Overwrite coarse's state with the full-weighting restriction of fine's (tlb_restrict)."""
    _check(fine.lib, fine.lib.tlb_restrict(fine._h, coarse._h), "tlb_restrict")


def learn_pair(grid, truth=None, moments=None, targets=None):
    """Moments of grid's state [nt, np, 4], and with truth also moments(truth) - moments(grid)."""
    import torch
    shape = grid.shape + (4,)
    m = moments if moments is not None else torch.empty(shape, dtype=torch.float32, device="cuda")
    y = None
    if truth is not None:
        y = targets if targets is not None else torch.empty(shape, dtype=torch.float32, device="cuda")
    _check(grid.lib, grid.lib.tlb_learn_pair(grid._h, truth._h if truth is not None else None,
                                             _f32(m, shape), _f32(y, shape) if y is not None else None),
           "tlb_learn_pair")
    return m, y


def apply_correction(grid, corrections):
    _check(grid.lib, grid.lib.tlb_apply_correction(grid._h, _f32(corrections, grid.shape + (4,))),
           "tlb_apply_correction")


def learned_step(grid, net, nsteps):
    _check(grid.lib, grid.lib.tlb_learned_step_n(grid._h, net._h, int(nsteps)), "tlb_learned_step_n")


STREAM_COPY, STREAM_ADD, STREAM_READ = 0, 1, 2


def hbm_stream(mode, x, y, z, stream=None):
    """tlb_hbm_stream on torch device tensors (16-byte aligned, contiguous): mode 0 copies x to
    z, mode 1 writes x + y (as floats) to z, mode 2 reads x (z receives one 16-byte partial per
    workgroup).  Enqueued on `stream` (default: the current stream); returns the bytes moved."""
    import torch
    lib = load_library()
    n16 = x.numel() * x.element_size() // 16
    s = stream if stream is not None else torch.cuda.current_stream()
    _check(lib, lib.tlb_hbm_stream(int(mode), _ptr(x), _ptr(y), _ptr(z), int(n16),
                                   ctypes.c_void_p(s.cuda_stream)), "tlb_hbm_stream")
    return 16 * n16 * (2 if mode == STREAM_COPY else 3 if mode == STREAM_ADD else 1)
