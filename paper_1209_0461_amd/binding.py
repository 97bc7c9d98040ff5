"""ctypes binding of libpmnu.so (include/pm_nu.h): argument marshalling only.

Functions carry the C names (pm_nu_init, pm_nu_deposit, ...). Device arrays are passed as
torch tensors (their data_ptr()); host arrays as NumPy arrays. All device work runs in
the library's HIP kernels; nothing here computes any part of the step.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpmnu.so")

PM_NU_OK = 0
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "EHISTORY",
          -6: "ENODEV", -7: "ESURROGATE", -8: "ENONFINITE"}
SUR_IN = 16
STAGE_CAP = 32


class PMNuError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pm_nu error {code} ({ERRORS.get(code, '?')}): {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("n_mesh", ctypes.c_int32), ("n_boxes", ctypes.c_int32),
                ("n_particles", ctypes.c_int64), ("box_size", ctypes.c_double),
                ("omega_m", ctypes.c_double), ("hubble", ctypes.c_double),
                ("n_kbins", ctypes.c_int32), ("max_history", ctypes.c_int32),
                ("substeps", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("deconvolve", ctypes.c_int32), ("response_mode", ctypes.c_int32),
                ("n_species", ctypes.c_int32), ("stream", ctypes.c_void_p)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_INT = ctypes.c_int
_F = ctypes.POINTER(ctypes.c_float)

SIGNATURES = {
    "pm_nu_default_config": (None, [ctypes.POINTER(Config)]),
    "pm_nu_init": (_INT, [ctypes.POINTER(Config), _D, ctypes.POINTER(_P)]),
    "pm_nu_destroy": (None, [_P]),
    "pm_nu_last_error": (ctypes.c_char_p, []),
    "pm_nu_get_bins": (_INT, [_P, _I64, _D, _D]),
    "pm_nu_set_history": (_INT, [_P, _INT, _INT, _D, _D, _D, _D, _D]),
    "pm_nu_get_history": (_INT, [_P, _INT, ctypes.POINTER(_INT), _D, _D, _D]),
    "pm_nu_deposit": (_INT, [_P, _P]),
    "pm_nu_response": (_INT, [_P, ctypes.c_double]),
    "pm_nu_force": (_INT, [_P, _P, _P, ctypes.c_double]),
    "pm_nu_step": (_INT, [_P, _P, _P, ctypes.c_double]),
    "pm_nu_get_spectrum": (_INT, [_P, _INT, _D, _D, _D]),
    "pm_nu_copy_density": (_INT, [_P, _INT, _P]),
    "pm_nu_set_keep_density": (_INT, [_P, _INT]),
    "pm_nu_set_inverse_xy": (_INT, [_P, _INT]),
    "pm_nu_set_forward_zy": (_INT, [_P, _INT]),
    "pm_nu_set_inverse_yz": (_INT, [_P, _INT]),
    "pm_nu_side_grid_uses": (_INT, [_P, _I64]),
    "pm_nu_binned_power_noalloc": (_INT, [_P, ctypes.c_int64, _INT, ctypes.c_double, _INT, _P,
                                          _P]),
    "pm_nu_copy_modes": (_INT, [_P, _INT, _P]),
    "pm_nu_copy_force_grid": (_INT, [_P, _INT, _INT, _P]),
    "pm_nu_set_timing": (_INT, [_P, _INT]),
    "pm_nu_set_species": (_INT, [_P, _INT, _INT, _D, _D]),
    "pm_nu_set_background": (_INT, [_P, _INT]),
    "pm_nu_set_kernel": (_INT, [_P, _INT]),
    "pm_nu_set_iterations": (_INT, [_P, _INT]),
    "pm_nu_advance": (_INT, [_P, _P, _P, _P, _D, _INT]),
    "pm_nu_kernel_values": (_INT, [_P, ctypes.c_int64, _INT, _P, _P]),
    "pm_nu_set_timing_mask": (_INT, [_P, ctypes.c_uint32]),
    "pm_nu_read_timing": (_INT, [_P, ctypes.POINTER(_INT), ctypes.POINTER(ctypes.c_char_p), _D, _I64]),
    "pm_nu_graph_capture": (_INT, [_P, _P, _P, ctypes.c_double]),
    "pm_nu_graph_launch": (_INT, [_P]),
    "pm_nu_autotune": (_INT, [_P, _P, _P, ctypes.c_double, ctypes.c_char_p]),
    "pm_nu_tuning": (_INT, [_P, ctypes.c_char_p, ctypes.c_size_t]),
    "pm_nu_set_launch": (_INT, [_P, _INT, _INT, _INT, _INT]),
    "pm_nu_set_fft_tiles": (_INT, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "pm_nu_surrogate_blob_floats": (ctypes.c_int64, []),
    "pm_nu_surrogate_load": (_INT, [_P, _F, ctypes.c_int64]),
    "pm_nu_surrogate_save": (_INT, [_P, _F, ctypes.c_int64]),
    "pm_nu_surrogate_init": (_INT, [_P, _P, _P, ctypes.c_int64, ctypes.c_uint64]),
    "pm_nu_surrogate_train": (_INT, [_P, _P, _P, ctypes.c_int64, _INT, _INT, ctypes.c_float,
                                     ctypes.c_uint64, _F]),
    "pm_nu_surrogate_train_part": (_INT, [_P, _P, _P, ctypes.c_int64, _INT, _INT, _INT, _INT,
                                          ctypes.c_float, ctypes.c_uint64, _F]),
    "pm_nu_surrogate_predict": (_INT, [_P, _P, _P, ctypes.c_int64]),
    "pm_nu_surrogate_grad": (_INT, [_P, _P, _P, ctypes.c_int64, _P, _F]),
    "pm_nu_surrogate_dataset": (_INT, [_P, ctypes.c_double, _P, _P]),
    "pm_nu_set_power": (_INT, [_P, _INT, _D]),
    "pm_nu_set_mass": (_INT, [_P, _INT, ctypes.c_double]),
    "pm_nu_set_response_mode": (_INT, [_P, _INT]),
    "pm_nu_get_surrogate_check": (_INT, [_P, _INT, _D, _D]),
}

_lib = None


def load_library(path=None):
    """Load libpmnu.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_1209_0461_amd.build`"
                           " (the step has no CPU fallback)")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def _check(rc):
    if rc != PM_NU_OK:
        msg = load_library().pm_nu_last_error()
        raise PMNuError(rc, msg.decode() if msg else "")
    return rc


def _dptr(a):
    """Host double array pointer (contiguous float64 copy kept alive by the caller)."""
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def _dev(t):
    """Device pointer of a torch tensor on a GPU."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def current_stream_handle():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------- C-named calls ----
def pm_nu_default_config():
    cfg = Config()
    load_library().pm_nu_default_config(ctypes.byref(cfg))
    return cfg


def pm_nu_init(cfg, m_nu_total):
    m = _f64(m_nu_total).reshape(-1)
    if m.size != cfg.n_boxes:
        raise ValueError("one neutrino mass per box is required")
    h = _P()
    _check(load_library().pm_nu_init(ctypes.byref(cfg), _dptr(m), ctypes.byref(h)))
    return h


def pm_nu_destroy(h):
    if h:
        load_library().pm_nu_destroy(h)


def pm_nu_get_bins(h, n_kbins):
    edges = np.zeros(n_kbins + 1, dtype=np.int64)
    counts = np.zeros(n_kbins)
    kmean = np.zeros(n_kbins)
    _check(load_library().pm_nu_get_bins(h, edges.ctypes.data_as(_I64), _dptr(counts),
                                         _dptr(kmean)))
    return edges, counts, kmean


def pm_nu_set_history(h, box, a, pm_half, pnu_half, pnu_half_init, theta_over_delta_init):
    a = _f64(a).reshape(-1)
    n = a.size
    pm = _f64(pm_half)
    pn = _f64(pnu_half)
    pi = _f64(pnu_half_init).reshape(-1)
    th = _f64(theta_over_delta_init).reshape(-1)
    if pm.shape[0] != n or pn.shape[0] != n:
        raise ValueError("history arrays must have one row per node")
    _check(load_library().pm_nu_set_history(h, box, n, _dptr(a), _dptr(pm), _dptr(pn),
                                            _dptr(pi), _dptr(th)))


def pm_nu_get_history(h, box, max_history, n_kbins):
    n = _INT()
    a = np.zeros(max_history)
    pm = np.zeros((max_history, n_kbins))
    pn = np.zeros((max_history, n_kbins))
    _check(load_library().pm_nu_get_history(h, box, ctypes.byref(n), _dptr(a), _dptr(pm),
                                            _dptr(pn)))
    k = n.value
    return a[:k].copy(), pm[:k].copy(), pn[:k].copy()


def pm_nu_deposit(h, pos):
    _check(load_library().pm_nu_deposit(h, _dev(pos)))


def pm_nu_response(h, a_now):
    _check(load_library().pm_nu_response(h, float(a_now)))


def pm_nu_force(h, pos, acc, a_now):
    _check(load_library().pm_nu_force(h, _dev(pos), _dev(acc), float(a_now)))


def pm_nu_step(h, pos, acc, a_now):
    _check(load_library().pm_nu_step(h, _dev(pos), _dev(acc), float(a_now)))


def pm_nu_get_spectrum(h, box, n_kbins):
    p = np.zeros(n_kbins)
    pn = np.zeros(n_kbins)
    r = np.zeros(n_kbins)
    _check(load_library().pm_nu_get_spectrum(h, box, _dptr(p), _dptr(pn), _dptr(r)))
    return p, pn, r


def pm_nu_binned_power_noalloc(pos, n_mesh, box_size, n_kbins, p_cdm, stream=None):
    """Binned P_cdm of one box without a context or any allocation: pos a float32 device
    tensor [n][3], p_cdm a float64 device tensor [n_kbins] (written on the stream)."""
    import torch
    if pos.dtype != torch.float32 or pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be a float32 tensor of shape (n, 3)")
    if p_cdm.dtype != torch.float64 or p_cdm.numel() != n_kbins:
        raise ValueError("p_cdm must be a float64 tensor of n_kbins values")
    st = stream if stream is not None else current_stream_handle()
    _check(load_library().pm_nu_binned_power_noalloc(_dev(pos), int(pos.shape[0]), int(n_mesh),
                                                     float(box_size), int(n_kbins),
                                                     _dev(p_cdm), st))


def pm_nu_side_grid_uses(h):
    n = ctypes.c_int64(0)
    _check(load_library().pm_nu_side_grid_uses(h, ctypes.byref(n)))
    return int(n.value)


def pm_nu_copy_density(h, box, out):
    _check(load_library().pm_nu_copy_density(h, box, _dev(out)))


def pm_nu_set_keep_density(h, on):
    _check(load_library().pm_nu_set_keep_density(h, int(bool(on))))


def pm_nu_set_inverse_xy(h, fused):
    _check(load_library().pm_nu_set_inverse_xy(h, int(bool(fused))))


def pm_nu_set_inverse_yz(h, fused):
    _check(load_library().pm_nu_set_inverse_yz(h, int(bool(fused))))


def pm_nu_set_forward_zy(h, fused):
    _check(load_library().pm_nu_set_forward_zy(h, int(bool(fused))))


def pm_nu_copy_modes(h, box, out):
    _check(load_library().pm_nu_copy_modes(h, box, _dev(out)))


def pm_nu_copy_force_grid(h, box, axis, out):
    _check(load_library().pm_nu_copy_force_grid(h, box, axis, _dev(out)))


def pm_nu_set_timing(h, enable):
    _check(load_library().pm_nu_set_timing(h, 1 if enable else 0))


def pm_nu_set_species(h, box, masses, pnu_half_init=None):
    """Species masses of one box [eV] (mass hierarchy); optional initial amplitudes
    [n_species][B]."""
    m = np.ascontiguousarray(masses, dtype=np.float64)
    ic = None if pnu_half_init is None else np.ascontiguousarray(pnu_half_init, dtype=np.float64)
    _check(load_library().pm_nu_set_species(h, int(box), len(m), _dptr(m),
                                            None if ic is None else _dptr(ic)))


def pm_nu_set_background(h, relativistic):
    """Background of the time grid: 0 matter + Lambda, 1 with radiation and relativistic
    neutrinos (eq. (relativistic))."""
    _check(load_library().pm_nu_set_background(h, 1 if relativistic else 0))


def pm_nu_set_kernel(h, series):
    """I(x) in the history integral: 0 the fit eq. (fit), 1 the exact series (Appendix C)."""
    _check(load_library().pm_nu_set_kernel(h, 1 if series else 0))


def pm_nu_set_iterations(h, iterations):
    """Iterations of the implicit current node (Appendix B), 1..16."""
    _check(load_library().pm_nu_set_iterations(h, int(iterations)))


def pm_nu_advance(h, pos, vel, acc, a_steps):
    """Kick-drift-kick steps through a_steps (host sequence, len n_steps + 1); pos, vel, acc
    are device tensors updated in place (acc must hold the force at a_steps[0])."""
    a = np.ascontiguousarray(a_steps, dtype=np.float64)
    _check(load_library().pm_nu_advance(h, _dev(pos), _dev(vel), _dev(acc), _dptr(a),
                                        len(a) - 1))


def pm_nu_kernel_values(x, out, series, stream=None):
    """I(x) on the device: x and out are float64 device tensors of the same length."""
    import torch
    if x.dtype != torch.float64 or out.dtype != torch.float64 or out.numel() != x.numel():
        raise ValueError("x and out must be float64 tensors of the same length")
    st = stream if stream is not None else current_stream_handle()
    _check(load_library().pm_nu_kernel_values(_dev(x), int(x.numel()), 1 if series else 0,
                                              _dev(out), st))


def pm_nu_set_timing_mask(h, stage_mask):
    _check(load_library().pm_nu_set_timing_mask(h, int(stage_mask) & 0xFFFFFFFF))


def pm_nu_read_timing(h):
    n = _INT(STAGE_CAP)
    names = (ctypes.c_char_p * STAGE_CAP)()
    ms = np.zeros(STAGE_CAP)
    cnt = np.zeros(STAGE_CAP, dtype=np.int64)
    _check(load_library().pm_nu_read_timing(h, ctypes.byref(n), names, _dptr(ms),
                                            cnt.ctypes.data_as(_I64)))
    return {names[i].decode(): (float(ms[i]), int(cnt[i])) for i in range(n.value)}


def pm_nu_graph_capture(h, pos, acc, a_now):
    _check(load_library().pm_nu_graph_capture(h, _dev(pos), _dev(acc), float(a_now)))


def pm_nu_graph_launch(h):
    _check(load_library().pm_nu_graph_launch(h))


def pm_nu_autotune(h, pos, acc, a_now, cache_path=None):
    cp = cache_path.encode() if cache_path else None
    _check(load_library().pm_nu_autotune(h, _dev(pos), _dev(acc), float(a_now), cp))


def pm_nu_set_launch(h, deposit_mode, deposit_block, interp_mode, interp_block):
    _check(load_library().pm_nu_set_launch(h, int(deposit_mode), int(deposit_block),
                                           int(interp_mode), int(interp_block)))


def pm_nu_set_fft_tiles(h, candidates):
    """Tile candidate (0, 1 or 2) of each FFT pass: fwd_z, fwd_y, fwd_x, inv_x, inv_y, inv_z."""
    c = np.ascontiguousarray(candidates, dtype=np.int32).reshape(-1)
    if c.size != 6:
        raise ValueError("six candidates are needed")
    _check(load_library().pm_nu_set_fft_tiles(h, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))


def pm_nu_tuning(h):
    buf = ctypes.create_string_buffer(1024)
    _check(load_library().pm_nu_tuning(h, buf, 1024))
    return buf.value.decode()


def pm_nu_surrogate_blob_floats():
    return int(load_library().pm_nu_surrogate_blob_floats())


def pm_nu_surrogate_load(h, blob):
    b = np.ascontiguousarray(np.asarray(blob, dtype=np.float32)).reshape(-1)
    _check(load_library().pm_nu_surrogate_load(h, b.ctypes.data_as(_F), b.size))


def pm_nu_surrogate_save(h):
    b = np.zeros(pm_nu_surrogate_blob_floats(), dtype=np.float32)
    _check(load_library().pm_nu_surrogate_save(h, b.ctypes.data_as(_F), b.size))
    return b


def pm_nu_surrogate_init(h, x, y, seed):
    _check(load_library().pm_nu_surrogate_init(h, _dev(x), _dev(y), x.shape[0], int(seed)))


def pm_nu_surrogate_train(h, x, y, epochs, batch, lr, seed):
    loss = ctypes.c_float(0.0)
    _check(load_library().pm_nu_surrogate_train(h, _dev(x), _dev(y), x.shape[0], int(epochs),
                                                int(batch), float(lr), int(seed),
                                                ctypes.byref(loss)))
    return float(loss.value)


def pm_nu_surrogate_train_part(h, x, y, first_epoch, epochs, total_epochs, batch, lr, seed):
    loss = ctypes.c_float(0.0)
    _check(load_library().pm_nu_surrogate_train_part(h, _dev(x), _dev(y), x.shape[0],
                                                     int(first_epoch), int(epochs),
                                                     int(total_epochs), int(batch), float(lr),
                                                     int(seed), ctypes.byref(loss)))
    return float(loss.value)


def pm_nu_surrogate_predict(h, x, y):
    _check(load_library().pm_nu_surrogate_predict(h, _dev(x), _dev(y), x.shape[0]))


def pm_nu_surrogate_grad(h, x, y, grad):
    loss = ctypes.c_float(0.0)
    _check(load_library().pm_nu_surrogate_grad(h, _dev(x), _dev(y), x.shape[0], _dev(grad),
                                               ctypes.byref(loss)))
    return float(loss.value)


def pm_nu_surrogate_dataset(h, a_now, x, y):
    _check(load_library().pm_nu_surrogate_dataset(h, float(a_now), _dev(x), _dev(y)))


def pm_nu_set_response_mode(h, mode):
    _check(load_library().pm_nu_set_response_mode(h, int(mode)))


def pm_nu_set_mass(h, box, m_nu_total):
    _check(load_library().pm_nu_set_mass(h, box, float(m_nu_total)))


def pm_nu_set_power(h, box, p_cdm):
    p = _f64(p_cdm).reshape(-1)
    _check(load_library().pm_nu_set_power(h, box, _dptr(p)))


def pm_nu_get_surrogate_check(h, box, n_kbins):
    ex = np.zeros(n_kbins)
    su = np.zeros(n_kbins)
    _check(load_library().pm_nu_get_surrogate_check(h, box, _dptr(ex), _dptr(su)))
    return ex, su


# --------------------------------------------------------------- convenience class ----
class PMNu:
    """One library context. Device tensors in, device tensors out."""

    def __init__(self, n_mesh, n_particles, box_size, n_kbins, max_history, m_nu_total,
                 omega_m=0.3, hubble=0.7, substeps=8, iterations=1, deconvolve=True,
                 response_mode=0, n_species=3, stream=None):
        m = np.atleast_1d(np.asarray(m_nu_total, dtype=np.float64))
        cfg = pm_nu_default_config()
        cfg.n_mesh = int(n_mesh)
        cfg.n_boxes = int(m.size)
        cfg.n_particles = int(n_particles)
        cfg.box_size = float(box_size)
        cfg.omega_m = float(omega_m)
        cfg.hubble = float(hubble)
        cfg.n_kbins = int(n_kbins)
        cfg.max_history = int(max_history)
        cfg.substeps = int(substeps)
        cfg.iterations = int(iterations)
        cfg.deconvolve = 1 if deconvolve else 0
        cfg.response_mode = int(response_mode)
        cfg.n_species = int(n_species)
        cfg.stream = stream if stream is not None else current_stream_handle()
        self.cfg = cfg
        self.m_nu = m
        self.h = pm_nu_init(cfg, m)

    def close(self):
        if getattr(self, "h", None):
            pm_nu_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def n_boxes(self):
        return self.cfg.n_boxes

    def bins(self):
        return pm_nu_get_bins(self.h, self.cfg.n_kbins)

    def set_history(self, box, hist):
        pm_nu_set_history(self.h, box, hist["a"], hist["pm_half"], hist["pnu_half"],
                          hist["pnu_half_init"], hist["theta_over_delta_init"])

    def history(self, box):
        return pm_nu_get_history(self.h, box, self.cfg.max_history, self.cfg.n_kbins)

    def advance(self, pos, vel, acc, a_steps):
        """Kick-drift-kick steps through a_steps; acc must hold the force at a_steps[0]."""
        for t, name in ((pos, "pos"), (vel, "vel"), (acc, "acc")):
            self._check_particles(t, name)
        pm_nu_advance(self.h, pos, vel, acc, a_steps)

    def _check_particles(self, t, name):
        import torch
        want = self.cfg.n_boxes * self.cfg.n_particles * 3
        if t.dtype != torch.float32 or t.numel() != want:
            raise ValueError(f"{name} must be float32 with n_boxes*n_particles*3 = {want} "
                             f"elements (got {t.dtype}, {t.numel()})")

    def deposit(self, pos):
        self._check_particles(pos, "pos")
        pm_nu_deposit(self.h, pos)

    def response(self, a_now):
        pm_nu_response(self.h, a_now)

    def force(self, pos, acc, a_now):
        self._check_particles(pos, "pos")
        self._check_particles(acc, "acc")
        pm_nu_force(self.h, pos, acc, a_now)

    def step(self, pos, acc, a_now):
        self._check_particles(pos, "pos")
        self._check_particles(acc, "acc")
        pm_nu_step(self.h, pos, acc, a_now)

    def spectrum(self, box=0):
        p, pn, r = pm_nu_get_spectrum(self.h, box, self.cfg.n_kbins)
        return dict(p_cdm=p, pnu_half=pn, ratio=r)
