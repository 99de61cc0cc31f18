"""MI355X dense-field phase-to-space turbulence renderer: Python binding.

Thin ctypes binding over ``libtsim.so`` (declared in ``include/tsim.h``).
The functions here only marshal arguments -- torch tensors become device
pointers, the current torch stream becomes the HIP stream -- and every step
of the renderer runs in the library's HIP kernels.  There is no CPU fallback:
importing fails if the library has not been built.
"""
import ctypes
import os

import numpy as np
import torch  # loaded first so the library shares torch's HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsim.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_2210_06713_amd/build.py` "
        "(the renderer has no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

N_MODES = 35
OK, EINVAL, ENOMEM, EDEVICE, EARTEFACT, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
P2S_EXACT, P2S_LEARNED = 0, 1
FP32, BF16 = 0, 1


class _Params(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("C", ctypes.c_int32),
                ("Gh", ctypes.c_int32), ("Gw", ctypes.c_int32), ("n_modes", ctypes.c_int32),
                ("pixel_pitch_over_d", ctypes.c_double), ("aperture_d_m", ctypes.c_double),
                ("wavelength_m", ctypes.c_double), ("path_length_m", ctypes.c_double),
                ("alias_fold", ctypes.c_int32), ("pupil_n", ctypes.c_int32),
                ("psf_t", ctypes.c_int32), ("basis_k", ctypes.c_int32),
                ("basis", ctypes.POINTER(ctypes.c_double)), ("p2s_mode", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("subharmonic_levels", ctypes.c_int32)]


_vp = ctypes.c_void_p
_i = ctypes.c_int
_u64 = ctypes.c_uint64


class _BatchItem(ctypes.Structure):
    _fields_ = [("plan", _vp), ("frames", ctypes.c_int32), ("d_over_r0", ctypes.POINTER(ctypes.c_float)),
                ("frame0", ctypes.c_uint64), ("img", _vp), ("zern", _vp), ("beta", _vp), ("blur", _vp),
                ("out", _vp), ("ws", _vp)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_lib_plan_create = _sig("tsim_plan_create", _i, [ctypes.POINTER(_Params), ctypes.POINTER(_vp)])
_lib_plan_destroy = _sig("tsim_plan_destroy", _i, [_vp])
_lib_ws = _sig("tsim_workspace_bytes", _i, [_vp, _i, ctypes.POINTER(ctypes.c_size_t)])
_lib_table = _sig("tsim_plan_table", _i, [_vp, _i, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t])
_lib_sample = _sig("tsim_sample_zernike", _i,
                   [_vp, _i, ctypes.POINTER(ctypes.c_float), _u64, _u64, _vp, _vp, _vp])
_lib_autotune = _sig("tsim_plan_autotune", _i, [_vp, _i, _vp, _vp, _vp])
_lib_set_tuning = _sig("tsim_plan_set_tuning", _i, [_vp, _i, _i])
_lib_tuning = _sig("tsim_plan_tuning", _i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i)])
_lib_sample_noalloc = _sig("tsim_sample_zernike_noalloc", _i,
                           [_vp, _i, ctypes.POINTER(ctypes.c_float), _u64, _u64, _vp, _vp])
_lib_sample_ar = _sig("tsim_sample_zernike_ar", _i, [_vp, _i, ctypes.POINTER(ctypes.c_float), _u64, _u64,
                                                     ctypes.c_float, _vp, ctypes.c_float, _vp, _vp, _vp])
_lib_stats_ws = _sig("tsim_tilt_stats_ws_bytes", _i, [_vp, _i, _i, ctypes.POINTER(ctypes.c_size_t)])
_lib_stats = _sig("tsim_tilt_stats", _i, [_vp, _i, _vp, _i, ctypes.POINTER(ctypes.c_double), _vp, _vp])
_lib_sf_ws = _sig("tsim_structure_function_ws_bytes", _i, [_vp, _i, ctypes.POINTER(ctypes.c_size_t)])
_lib_sf = _sig("tsim_structure_function", _i, [_vp, _i, _vp, ctypes.POINTER(ctypes.c_double),
                                               ctypes.POINTER(ctypes.c_double), _vp, _vp])
_lib_otf_ws = _sig("tsim_otf_ws_bytes", _i, [_vp, _i, ctypes.POINTER(ctypes.c_size_t)])
_lib_otf = _sig("tsim_otf", _i, [_vp, _i, _vp, _i, ctypes.POINTER(ctypes.c_double), _vp, _vp])
_lib_p2s = _sig("tsim_p2s", _i, [_vp, _i, _vp, _vp, _vp, _vp])
_lib_render = _sig("tsim_render", _i, [_vp, _i, _vp, _vp, _vp, _vp, _vp])
_lib_warp = _sig("tsim_warp", _i, [_vp, _i, _vp, _vp, _vp, _vp])
_lib_psf = _sig("tsim_psf_exact", _i, [_vp, _i, _vp, _vp, _vp])
_lib_status = _sig("tsim_status_string", ctypes.c_char_p, [_i])
_lib_basis = _sig("tsim_basis_build", _i, [_vp, _i, _u64, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)])
_lib_trace_enable = _sig("tsim_trace_enable", _i, [_i])
_lib_trace_count = _sig("tsim_trace_count", _i, [ctypes.POINTER(_i)])
_lib_trace_get = _sig("tsim_trace_get", _i, [_i, ctypes.c_char_p, ctypes.c_size_t,
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i)])
_f = ctypes.c_float
_fp = ctypes.POINTER(ctypes.c_float)
_lib_mlp_create = _sig("tsim_mlp_create", _i, [_vp, _i, _u64, ctypes.POINTER(_vp)])
_lib_mlp_destroy = _sig("tsim_mlp_destroy", _i, [_vp])
_lib_mlp_count = _sig("tsim_mlp_param_count", _i, [_vp, ctypes.POINTER(ctypes.c_size_t)])
_lib_mlp_layout = _sig("tsim_mlp_layout", _i, [_vp, ctypes.POINTER(ctypes.c_size_t),
                                              ctypes.POINTER(ctypes.c_size_t)])
_lib_mlp_get = _sig("tsim_mlp_get", _i, [_vp, _i, _fp, ctypes.c_size_t])
_lib_mlp_set = _sig("tsim_mlp_set", _i, [_vp, _i, _fp, ctypes.c_size_t])
_lib_mlp_data = _sig("tsim_mlp_make_data", _i, [_vp, _i, _u64, _f, _f, _vp, _vp, _vp, _vp])
_lib_mlp_data_ws = _sig("tsim_mlp_data_ws_bytes", _i, [_vp, _i, ctypes.POINTER(ctypes.c_size_t)])
_lib_mlp_grad = _sig("tsim_mlp_grad", _i, [_vp, _i, _vp, _vp, _fp, _vp])
_lib_mlp_train = _sig("tsim_mlp_train", _i, [_vp, _vp, _vp, _i, _i, _f, _f, _fp, _vp])
_lib_set_mlp = _sig("tsim_plan_set_mlp", _i, [_vp, _vp])
_lib_mlp_fit = _sig("tsim_mlp_fit_output", _i, [_vp, _vp, _i, _vp])
_lib_mlp_predict = _sig("tsim_mlp_predict", _i, [_vp, _i, _vp, _vp, _vp])
_lib_host_tables = _sig("tsim_host_tables", _i,
                        [ctypes.POINTER(_Params), _i, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t])
_lib_p2s_form = _sig("tsim_p2s_form", _i, [_vp, ctypes.POINTER(_i)])
_lib_batch_create = _sig("tsim_batch_create", _i, [ctypes.POINTER(_BatchItem), _i, _u64, ctypes.POINTER(_vp)])
_lib_batch_launch = _sig("tsim_batch_launch", _i, [_vp, _vp])
_lib_batch_destroy = _sig("tsim_batch_destroy", _i, [_vp])
_lib_last_error = _sig("tsim_last_error", _i, [ctypes.c_char_p, ctypes.c_size_t])
_lib_sync = _sig("tsim_sync", _i, [_vp])
_lib_frame_group = _sig("tsim_frame_group", _i, [_vp, ctypes.POINTER(_i)])
_lib_frame_ws = _sig("tsim_frame_workspace_bytes", _i, [_vp, _i, ctypes.POINTER(ctypes.c_size_t)])
_lib_frame = _sig("tsim_frame", _i, [_vp, _i, _i, ctypes.POINTER(ctypes.c_float), _u64, _u64, _vp, _vp, _vp,
                                     _vp, _vp])

EXPORTED = ["tsim_plan_create", "tsim_plan_destroy", "tsim_workspace_bytes", "tsim_plan_table",
            "tsim_plan_autotune", "tsim_plan_set_tuning", "tsim_plan_tuning",
            "tsim_sample_zernike", "tsim_sample_zernike_ar", "tsim_p2s", "tsim_render", "tsim_warp", "tsim_psf_exact",
            "tsim_status_string", "tsim_host_tables", "tsim_basis_build", "tsim_trace_enable",
            "tsim_trace_count", "tsim_trace_get", "tsim_mlp_create", "tsim_mlp_destroy",
            "tsim_mlp_param_count", "tsim_mlp_layout", "tsim_mlp_get", "tsim_mlp_set",
            "tsim_mlp_data_ws_bytes", "tsim_mlp_make_data", "tsim_mlp_grad", "tsim_mlp_train", "tsim_plan_set_mlp",
            "tsim_mlp_fit_output", "tsim_mlp_predict", "tsim_tilt_stats_ws_bytes", "tsim_tilt_stats",
            "tsim_structure_function_ws_bytes", "tsim_structure_function", "tsim_p2s_form",
            "tsim_last_error", "tsim_sync", "tsim_sample_zernike_noalloc", "tsim_batch_create",
            "tsim_batch_launch", "tsim_batch_destroy", "tsim_otf_ws_bytes", "tsim_otf", "tsim_frame_group",
            "tsim_frame_workspace_bytes", "tsim_frame"]


def last_error():
    """(status, text) of the last failing library call on this thread, then
    cleared; (0, "") if none."""
    buf = ctypes.create_string_buffer(256)
    st = _lib_last_error(buf, 256)
    return st, buf.value.decode()


def sync(stream=None):
    """Wait for the stream; an asynchronous device fault raises TsimError."""
    _check(_lib_sync(_stream(stream)), "tsim_sync")


def trace_enable(on=True):
    """Start (clearing old counts) or stop per-kernel event timing."""
    _check(_lib_trace_enable(1 if on else 0), "tsim_trace_enable")


def trace_report():
    """{kernel name: (launches, total ms)} for launches since trace_enable()."""
    n = _i()
    _check(_lib_trace_count(ctypes.byref(n)), "tsim_trace_count")
    out = {}
    for i in range(n.value):
        buf = ctypes.create_string_buffer(128)
        ms = ctypes.c_double()
        cnt = _i()
        _check(_lib_trace_get(i, buf, 128, ctypes.byref(ms), ctypes.byref(cnt)), "tsim_trace_get")
        out[buf.value.decode()] = (cnt.value, ms.value)
    return out


class TsimError(RuntimeError):
    def __init__(self, status, what):
        super().__init__(f"{what}: {_lib_status(status).decode()} ({status})")
        self.status = status


def _check(status, what):
    if status != OK:
        raise TsimError(status, what)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _expect(t, name, shape, dtype, device=None):
    """Raise ValueError unless `t` is a contiguous device tensor of exactly
    `shape` and `dtype` (on `device` if given).  The C ABI receives bare
    pointers and cannot check extents, so every buffer is checked here,
    before any launch."""
    if t is None:
        raise ValueError(f"{name}: tensor expected")
    if not t.is_cuda:
        raise ValueError(f"{name}: device tensor expected")
    if device is not None and t.device != device:
        raise ValueError(f"{name}: on {t.device}, expected {device}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: contiguous tensor expected")


def _expect_bytes(t, name, nbytes, device):
    """A workspace: a contiguous device tensor of at least `nbytes` bytes."""
    if t is None or not t.is_cuda:
        raise ValueError(f"{name}: device tensor expected")
    if t.device != device:
        raise ValueError(f"{name}: on {t.device}, expected {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: contiguous tensor expected")
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"{name}: {t.numel() * t.element_size()} bytes, {nbytes} needed")


def kpad(k):
    """BF16 weight-row width for K basis functions: K rounded up to 32, 64,
    112 or 128."""
    return 32 if k <= 32 else 64 if k <= 64 else 112 if k <= 112 else 128


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_params(H, W, C=1, Gh=None, Gw=None, pixel_pitch_over_d=0.125, aperture_d_m=0.0,
                wavelength_m=0.0, path_length_m=0.0, alias_fold=2, pupil_n=64, psf_t=33,
                basis_k=1, p2s_mode=P2S_EXACT, precision=FP32, subharmonic_levels=0, n_modes=N_MODES):
    if Gh is None:
        Gh = 1 << int(np.ceil(np.log2(2 * H)))
    if Gw is None:
        Gw = 1 << int(np.ceil(np.log2(2 * W)))
    return _Params(H, W, C, Gh, Gw, n_modes, pixel_pitch_over_d, aperture_d_m, wavelength_m,
                   path_length_m, alias_fold, pupil_n, psf_t, basis_k, None, p2s_mode, precision,
                   subharmonic_levels)


def host_tables(params, what):
    """Run the host half of plan creation (no device) and return one table:
    0 = A_0, 1 = L, 2 = sqrt quarter spectra [N][Gw/2+1][Gh/2+1], 3 = pitch,
    4 = subharmonic amplitudes [2][4][4]."""
    N = params.n_modes
    sizes = {0: N * N, 1: N * N, 2: N * (params.Gw // 2 + 1) * (params.Gh // 2 + 1), 3: 1, 4: 32}
    out = np.zeros(sizes[what], dtype=np.float64)
    _check(_lib_host_tables(ctypes.byref(params), what,
                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.size),
           "tsim_host_tables")
    if what in (0, 1):
        return out.reshape(N, N)
    if what == 2:
        return out.reshape(N, params.Gw // 2 + 1, params.Gh // 2 + 1)
    if what == 4:
        return out.reshape(2, 4, 4)
    return out[0]


class Plan:
    """A renderer plan (``tsim_plan``): FP64 tables built once, then
    immutable.  Sizes follow ``tsim_params`` in ``include/tsim.h``."""

    def __init__(self, H, W, C=1, Gh=None, Gw=None, pixel_pitch_over_d=0.125,
                 aperture_d_m=0.0, wavelength_m=0.0, path_length_m=0.0, alias_fold=2,
                 pupil_n=64, psf_t=33, basis=None, basis_k=None, p2s_mode=P2S_EXACT,
                 precision=FP32, subharmonic_levels=0, n_modes=N_MODES):
        if Gh is None:
            Gh = 1 << int(np.ceil(np.log2(2 * H)))
        if Gw is None:
            Gw = 1 << int(np.ceil(np.log2(2 * W)))
        self._basis = None
        bptr = None
        if basis is not None:
            self._basis = np.ascontiguousarray(basis, dtype=np.float64)
            basis_k = self._basis.shape[0]
            bptr = self._basis.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        if basis_k is None:
            basis_k = 1
        self.params = _Params(H, W, C, Gh, Gw, n_modes, pixel_pitch_over_d, aperture_d_m,
                              wavelength_m, path_length_m, alias_fold, pupil_n, psf_t, basis_k,
                              bptr, p2s_mode, precision, subharmonic_levels)
        self.H, self.W, self.C, self.Gh, self.Gw = H, W, C, Gh, Gw
        self.N = n_modes
        self.T, self.K, self.P = psf_t, basis_k, pupil_n
        self.p2s_mode, self.precision = p2s_mode, precision
        self.KP = kpad(basis_k)
        h = _vp()
        _check(_lib_plan_create(ctypes.byref(self.params), ctypes.byref(h)), "tsim_plan_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _lib_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- plan tables -------------------------------------------------
    def table(self, what):
        N = self.N
        sizes = {0: N * N, 1: N * N, 2: N * (self.Gw // 2 + 1) * (self.Gh // 2 + 1), 3: 1, 4: 32}
        out = np.zeros(sizes[what], dtype=np.float64)
        _check(_lib_table(self._h, what, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          out.size), "tsim_plan_table")
        if what in (0, 1):
            return out.reshape(N, N)
        if what == 2:
            return out.reshape(N, self.Gw // 2 + 1, self.Gh // 2 + 1)
        if what == 4:
            return out.reshape(2, 4, 4)
        return out[0]

    def workspace_bytes(self, frames):
        n = ctypes.c_size_t()
        _check(_lib_ws(self._h, frames, ctypes.byref(n)), "tsim_workspace_bytes")
        return n.value

    def workspace(self, frames, device="cuda"):
        """Allocate a device workspace (plumbing only) for `frames` frames."""
        n = max(self.workspace_bytes(frames), 256)
        return torch.empty(n, dtype=torch.uint8, device=device)

    # ---- buffer checks (shapes the kernels assume) -----------------
    def _zern(self, zern, name="zern"):
        if zern is None or zern.dim() != 4:
            raise ValueError(f"{name}: [frames, n_modes, H, W] tensor expected")
        _expect(zern, name, (zern.shape[0], self.N, self.H, self.W), torch.float32)
        return zern.shape[0], zern.device

    def _frames_img(self, img, name, frames, device):
        _expect(img, name, (frames, self.C, self.H, self.W), torch.float32, device)

    def _beta(self, beta, frames, device):
        """Weights as tsim_p2s writes and tsim_render reads them: float32
        [F][H][W][K], or bfloat16 [F][H][W][KP] in BF16 plans."""
        if self.precision == BF16:
            _expect(beta, "beta", (frames, self.H, self.W, self.KP), torch.bfloat16, device)
        else:
            _expect(beta, "beta", (frames, self.H, self.W, self.K), torch.float32, device)

    def _ws(self, ws, frames, device):
        _expect_bytes(ws, "ws", self.workspace_bytes(frames), device)

    # ---- hot path ----------------------------------------------------
    def sample_zernike(self, d_over_r0, seed, frame0, zern, ws, stream=None):
        d = np.ascontiguousarray(np.atleast_1d(d_over_r0), dtype=np.float32)
        frames, dev = self._zern(zern)
        if d.size != frames:
            raise ValueError("one D/r0 per frame expected")
        if frames > 0:
            self._ws(ws, frames, dev)
        _check(_lib_sample(self._h, frames, d.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                           int(seed), int(frame0), _ptr(zern), _ptr(ws), _stream(stream)),
               "tsim_sample_zernike")

    def autotune(self, frames, zern, ws, stream=None):
        """Times the sampler's launch forms on these buffers and keeps the
        fastest (tsim_plan_autotune); returns (pass-1 columns, pass-2 form)."""
        f, dev = self._zern(zern)
        if f != frames or frames < 1:
            raise ValueError("zern must hold `frames` frames")
        self._ws(ws, frames, dev)
        _check(_lib_autotune(self._h, frames, _ptr(zern), _ptr(ws), _stream(stream)), "tsim_plan_autotune")
        return self.tuning()

    def set_tuning(self, columns=0, rows_form=0):
        """Forces the sampler's launch forms (0 = the built-in choice)."""
        _check(_lib_set_tuning(self._h, int(columns), int(rows_form)), "tsim_plan_set_tuning")

    def tuning(self):
        """(pass-1 columns per block, pass-2 form) in effect."""
        c, r = _i(), _i()
        _check(_lib_tuning(self._h, ctypes.byref(c), ctypes.byref(r)), "tsim_plan_tuning")
        return c.value, r.value

    def sample_zernike_noalloc(self, d_over_r0, seed, frame0, zern, stream=None):
        """tsim_sample_zernike without a workspace and without any allocation
        (the library's fixed scratch array holds the intermediate)."""
        d = np.ascontiguousarray(np.atleast_1d(d_over_r0), dtype=np.float32)
        frames, _ = self._zern(zern)
        if d.size != frames:
            raise ValueError("one D/r0 per frame expected")
        _check(_lib_sample_noalloc(self._h, frames, d.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   int(seed), int(frame0), _ptr(zern), _stream(stream)),
               "tsim_sample_zernike_noalloc")

    def sample_zernike_ar(self, d_over_r0, seed, frame0, alpha, zern, ws, zern_prev=None,
                          d_over_r0_prev=0.0, stream=None):
        """Auto-regressively correlated frames (tsim_sample_zernike_ar)."""
        d = np.ascontiguousarray(np.atleast_1d(d_over_r0), dtype=np.float32)
        frames, dev = self._zern(zern)
        if d.size != frames:
            raise ValueError("one D/r0 per frame expected")
        if frames > 0:
            self._ws(ws, frames, dev)
        if zern_prev is not None:
            _expect(zern_prev, "zern_prev", (self.N, self.H, self.W), torch.float32, dev)
        _check(_lib_sample_ar(self._h, frames, d.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                              int(seed), int(frame0), float(alpha), _ptr(zern_prev),
                              float(d_over_r0_prev), _ptr(zern), _ptr(ws), _stream(stream)),
               "tsim_sample_zernike_ar")

    def tilt_stats(self, zern, max_lag, ws=None, stream=None):
        """Spatial tilt statistics (tsim_tilt_stats): returns (corr, dtv), each
        [2 modes (Noll 2, 3)][2 axes (x, y)][max_lag + 1] float64."""
        frames, dev = self._zern(zern)
        n = ctypes.c_size_t()
        if frames > 0:
            _check(_lib_stats_ws(self._h, frames, int(max_lag), ctypes.byref(n)), "tsim_tilt_stats_ws_bytes")
        if ws is None:
            ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=dev)
        _expect_bytes(ws, "ws", n.value, dev)
        out = np.zeros(8 * (int(max_lag) + 1), dtype=np.float64)
        _check(_lib_stats(self._h, frames, _ptr(zern), int(max_lag),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(ws), _stream(stream)),
               "tsim_tilt_stats")
        out = out.reshape(2, 2, 2, int(max_lag) + 1)
        return out[:, :, 0].copy(), out[:, :, 1].copy()

    def structure_function(self, zern, ws=None, stream=None):
        """Phase structure function over the aperture (tsim_structure_function):
        returns (D [31] for r = 0..30 pupil samples, r/D = r/32, and the
        coefficients' second moments [35][35])."""
        frames, dev = self._zern(zern)
        n = ctypes.c_size_t()
        if frames > 0:
            _check(_lib_sf_ws(self._h, frames, ctypes.byref(n)), "tsim_structure_function_ws_bytes")
        if ws is None:
            ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=dev)
        _expect_bytes(ws, "ws", n.value, dev)
        D = np.zeros(31, dtype=np.float64)
        C = np.zeros((35, 35), dtype=np.float64)
        _check(_lib_sf(self._h, frames, _ptr(zern), D.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                       C.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(ws), _stream(stream)),
               "tsim_structure_function")
        return D, C

    def otf(self, zern, short_exposure=False, ws=None, stream=None):
        """Mean optical transfer function over all pixels of the frames
        (tsim_otf): complex [64][64], lag (dy, dx) at (32 + dy, 32 + dx),
        H(0) = 1; the short-exposure form removes the Zernike tilts."""
        frames, dev = self._zern(zern)
        n = ctypes.c_size_t()
        if frames > 0:
            _check(_lib_otf_ws(self._h, frames, ctypes.byref(n)), "tsim_otf_ws_bytes")
        if ws is None:
            ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=dev)
        _expect_bytes(ws, "ws", n.value, dev)
        out = np.zeros((2, 64, 64), dtype=np.float64)
        _check(_lib_otf(self._h, frames, _ptr(zern), 1 if short_exposure else 0,
                        out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(ws), _stream(stream)),
               "tsim_otf")
        return out[0] + 1j * out[1]

    def p2s_form(self):
        """P2S_LEARNED if tsim_p2s runs the network now, else P2S_EXACT."""
        f = _i()
        _check(_lib_p2s_form(self._h, ctypes.byref(f)), "tsim_p2s_form")
        return f.value

    def p2s(self, zern, beta, ws, stream=None):
        frames, dev = self._zern(zern)
        self._beta(beta, frames, dev)
        if frames > 0:
            self._ws(ws, frames, dev)
        _check(_lib_p2s(self._h, frames, _ptr(zern), _ptr(beta), _ptr(ws), _stream(stream)),
               "tsim_p2s")

    def render(self, img, beta, out, ws=None, stream=None):
        if img is None or img.dim() != 4:
            raise ValueError("img: [frames, C, H, W] tensor expected")
        frames, dev = img.shape[0], img.device
        self._frames_img(img, "img", frames, dev)
        self._frames_img(out, "out", frames, dev)
        self._beta(beta, frames, dev)
        _check(_lib_render(self._h, frames, _ptr(img), _ptr(beta), _ptr(out), _ptr(ws),
                           _stream(stream)), "tsim_render")

    def warp(self, img, zern, out, stream=None):
        frames, dev = self._zern(zern)
        self._frames_img(img, "img", frames, dev)
        self._frames_img(out, "out", frames, dev)
        _check(_lib_warp(self._h, frames, _ptr(img), _ptr(zern), _ptr(out), _stream(stream)),
               "tsim_warp")

    # ---- the whole path in one call ----------------------------------
    def frame_group(self):
        g = _i()
        _check(_lib_frame_group(self._h, ctypes.byref(g)), "tsim_frame_group")
        return g.value

    def frame_workspace_bytes(self, group):
        n = ctypes.c_size_t()
        _check(_lib_frame_ws(self._h, group, ctypes.byref(n)), "tsim_frame_workspace_bytes")
        return n.value

    def frame_workspace(self, group, device="cuda"):
        """Allocate a device workspace (plumbing only) for tsim_frame."""
        return torch.empty(self.frame_workspace_bytes(group), dtype=torch.uint8, device=device)

    def frame(self, d_over_r0, seed, frame0, img, out, ws, group=None, zern_out=None, stream=None):
        if img is None or img.dim() != 4:
            raise ValueError("img: [frames, C, H, W] tensor expected")
        frames, dev = img.shape[0], img.device
        if group is None:
            group = self.frame_group()
        self._frames_img(img, "img", frames, dev)
        self._frames_img(out, "out", frames, dev)
        if zern_out is not None:
            _expect(zern_out, "zern_out", (frames, self.N, self.H, self.W), torch.float32, dev)
        _expect_bytes(ws, "ws", self.frame_workspace_bytes(group), dev)
        if len(d_over_r0) != frames:
            raise ValueError("d_over_r0: one value per frame expected")
        d = (ctypes.c_float * frames)(*[float(v) for v in d_over_r0])
        _check(_lib_frame(self._h, frames, group, d, int(seed), int(frame0), _ptr(img),
                          _ptr(zern_out) if zern_out is not None else None, _ptr(out), _ptr(ws),
                          _stream(stream)), "tsim_frame")

    def basis_build(self, n_psf=20000, seed=0, dr_lo=0.5, dr_hi=5.0):
        """PCA PSF basis (K x T*T float64) and its eigenvalues, computed by
        the library (device PSFs and Gram matrix, host eigen-solver)."""
        out = np.zeros((self.K, self.T * self.T), dtype=np.float64)
        eig = np.zeros(self.K, dtype=np.float64)
        _check(_lib_basis(self._h, int(n_psf), int(seed), float(dr_lo), float(dr_hi),
                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          eig.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "tsim_basis_build")
        return out, eig

    def psf_exact(self, zvec, psf, stream=None):
        if zvec is None or zvec.dim() != 2:
            raise ValueError("zvec: [n, n_modes] tensor expected")
        n = zvec.shape[0]
        _expect(zvec, "zvec", (n, self.N), torch.float32)
        _expect(psf, "psf", (n, self.T * self.T), torch.float32, zvec.device)
        _check(_lib_psf(self._h, n, _ptr(zvec), _ptr(psf), _stream(stream)),
               "tsim_psf_exact")


class Mlp:
    """The learned P2S network (``tsim_mlp``): 35 -> 256 -> 256 -> 256 -> K."""

    def __init__(self, plan, batch=8192, seed=0):
        h = _vp()
        _check(_lib_mlp_create(plan._h, int(batch), int(seed), ctypes.byref(h)), "tsim_mlp_create")
        self._h = h
        self.K = plan.K
        self.batch = batch
        n = ctypes.c_size_t()
        _check(_lib_mlp_count(self._h, ctypes.byref(n)), "tsim_mlp_param_count")
        self.n_params = n.value
        ow = (ctypes.c_size_t * 4)()
        ob = (ctypes.c_size_t * 4)()
        _check(_lib_mlp_layout(self._h, ow, ob), "tsim_mlp_layout")
        self.off_w = list(ow)
        self.off_b = list(ob)
        self.dims = [N_MODES, 256, 256, 256, self.K]

    def close(self):
        if getattr(self, "_h", None):
            _lib_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _count(self, what):
        return {0: self.n_params, 1: self.n_params, 2: N_MODES, 3: self.K, 4: 1,
                5: self.n_params, 6: self.n_params, 7: 2}[what]

    def get(self, what):
        """what: 0 parameters, 1 gradients, 2 inv_s, 3 mu, 4 s_out, 5/6 AdamW
        first/second moments, 7 [steps taken, schedule length]."""
        n = self._count(what)
        out = np.zeros(n, dtype=np.float32)
        _check(_lib_mlp_get(self._h, what, out.ctypes.data_as(_fp), n), "tsim_mlp_get")
        return out

    def set(self, what, values):
        v = np.ascontiguousarray(values, dtype=np.float32).ravel()
        _check(_lib_mlp_set(self._h, what, v.ctypes.data_as(_fp), v.size), "tsim_mlp_set")

    def unpack(self, flat):
        """[(W [out][in], b [out])] views of a flat parameter array."""
        out = []
        for l in range(4):
            i, o = self.dims[l], self.dims[l + 1]
            out.append((flat[self.off_w[l]:self.off_w[l] + o * i].reshape(o, i),
                        flat[self.off_b[l]:self.off_b[l] + o]))
        return out

    def pack(self, layers):
        flat = np.zeros(self.n_params, dtype=np.float32)
        for l, (W, b) in enumerate(layers):
            flat[self.off_w[l]:self.off_w[l] + W.size] = np.asarray(W, dtype=np.float32).ravel()
            flat[self.off_b[l]:self.off_b[l] + b.size] = b
        return flat

    def checkpoint(self):
        """Training state: parameters, AdamW moments and counters (host)."""
        return {w: self.get(w) for w in (0, 5, 6, 7)} | {"inv_s": self.get(2), "mu": self.get(3),
                                                        "s_out": self.get(4)}

    def restore(self, state):
        for w in (0, 5, 6, 7):
            self.set(w, state[w])
        self.set(2, state["inv_s"])
        self.set(3, state["mu"])
        self.set(4, state["s_out"])

    def _pairs(self, zvec, target, n=None):
        if zvec is None or zvec.dim() != 2:
            raise ValueError("zvec: [n, 35] tensor expected")
        n = zvec.shape[0] if n is None else n
        _expect(zvec, "zvec", (n, N_MODES), torch.float32)
        _expect(target, "target", (n, self.K), torch.float32, zvec.device)

    def grad(self, zvec, target, stream=None):
        self._pairs(zvec, target)
        if zvec.shape[0] > self.batch:
            raise ValueError(f"at most {self.batch} pairs per gradient call")
        loss = ctypes.c_float()
        _check(_lib_mlp_grad(self._h, zvec.shape[0], _ptr(zvec), _ptr(target), ctypes.byref(loss),
                             _stream(stream)), "tsim_mlp_grad")
        return loss.value

    def fit_output(self, target, stream=None):
        if target is None or target.dim() != 2:
            raise ValueError("target: [n, K] tensor expected")
        _expect(target, "target", (target.shape[0], self.K), torch.float32)
        _check(_lib_mlp_fit(self._h, _ptr(target), target.shape[0], _stream(stream)),
               "tsim_mlp_fit_output")

    def train(self, zvec, target, steps, lr_max=1e-3, lr_min=1e-5, stream=None):
        self._pairs(zvec, target)
        losses = np.zeros(steps, dtype=np.float32)
        _check(_lib_mlp_train(self._h, _ptr(zvec), _ptr(target), zvec.shape[0], int(steps),
                              float(lr_max), float(lr_min), losses.ctypes.data_as(_fp),
                              _stream(stream)), "tsim_mlp_train")
        return losses


class Batch:
    """Mixed-size frames through the whole path in one library-built HIP
    graph (``tsim_batch``).  ``items``: dicts with keys plan, d_over_r0
    (one per frame), frame0, img, zern, beta, blur, out, ws (device tensors,
    shaped as for the individual calls).  The tensors are kept referenced
    for the batch's lifetime."""

    def __init__(self, items, seed):
        self._keep = []
        arr = (_BatchItem * len(items))()
        for k, it in enumerate(items):
            pl = it["plan"]
            d = np.ascontiguousarray(np.atleast_1d(it["d_over_r0"]), dtype=np.float32)
            frames, dev = pl._zern(it["zern"])
            if d.size != frames:
                raise ValueError("one D/r0 per frame expected")
            pl._frames_img(it["img"], "img", frames, dev)
            pl._frames_img(it["blur"], "blur", frames, dev)
            pl._frames_img(it["out"], "out", frames, dev)
            pl._beta(it["beta"], frames, dev)
            pl._ws(it["ws"], frames, dev)
            self._keep += [pl, d, it["img"], it["zern"], it["beta"], it["blur"], it["out"], it["ws"]]
            arr[k] = _BatchItem(pl._h, frames, d.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                int(it.get("frame0", 0)), _ptr(it["img"]).value, _ptr(it["zern"]).value,
                                _ptr(it["beta"]).value, _ptr(it["blur"]).value, _ptr(it["out"]).value,
                                _ptr(it["ws"]).value)
        h = _vp()
        _check(_lib_batch_create(arr, len(items), int(seed), ctypes.byref(h)), "tsim_batch_create")
        self._h = h

    def launch(self, stream=None):
        _check(_lib_batch_launch(self._h, _stream(stream)), "tsim_batch_launch")

    def close(self):
        if getattr(self, "_h", None):
            _lib_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_training_data(plan, n_pairs, seed=0, dr_lo=0.5, dr_hi=5.0, stream=None):
    """(zvec [n][35], beta [n][K]) device tensors from the exact path."""
    z = torch.empty((n_pairs, N_MODES), dtype=torch.float32, device="cuda")
    b = torch.empty((n_pairs, plan.K), dtype=torch.float32, device="cuda")
    nb = ctypes.c_size_t(0)
    _check(_lib_mlp_data_ws(plan._h, int(n_pairs), ctypes.byref(nb)), "tsim_mlp_data_ws_bytes")
    ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device="cuda")
    _check(_lib_mlp_data(plan._h, int(n_pairs), int(seed), float(dr_lo), float(dr_hi), _ptr(z),
                         _ptr(b), _ptr(ws), _stream(stream)), "tsim_mlp_make_data")
    return z, b


def mlp_predict(plan, zvec, stream=None):
    """The plan's network on Zernike vectors [n][35] -> beta [n][K] (float32)."""
    if zvec is None or zvec.dim() != 2:
        raise ValueError("zvec: [n, 35] tensor expected")
    _expect(zvec, "zvec", (zvec.shape[0], N_MODES), torch.float32)
    out = torch.empty((zvec.shape[0], plan.K), dtype=torch.float32, device="cuda")
    _check(_lib_mlp_predict(plan._h, zvec.shape[0], _ptr(zvec), _ptr(out), _stream(stream)),
           "tsim_mlp_predict")
    return out


def plan_set_mlp(plan, mlp):
    _check(_lib_set_mlp(plan._h, mlp._h), "tsim_plan_set_mlp")
