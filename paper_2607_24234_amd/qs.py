"""Python binding of libqs (include/qs.h): argument marshalling only.

Every step of the solver runs in the HIP library.  torch provides device memory (the
workspace and output buffers) and the HIP stream; if libqs.so is missing or cannot be
loaded, importing this module's ``lib()`` raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("QS_LIBRARY", os.path.join(PKG, "libqs.so"))

# mirrored from include/qs.h
QS_OK = 0
QS_ERR_ARG = -1
QS_ERR_ALLOC = -2
QS_ERR_HIP = -3
QS_ERR_NUMERIC = -4
QS_ERR_UNSUPPORTED = -5
QS_ERR_STATE = -6
QS_FP64 = 0
QS_FP32 = 1
PROFILE_FLATTOP, PROFILE_GAUSSIAN, PROFILE_TABLE = 0, 1, 2
GEOM_SPECTRAL, GEOM_TRANSVERSE_GRID = 0, 1
SEED_NOISE, SEED_UNIFORM, SEED_FRONT_IMPULSE, SEED_CENTROID, SEED_NONE = 0, 1, 2, 3, 4
FLAG_DROP_LONGITUDINAL, FLAG_NO_RESTORING, FLAG_STEADY_INFLOW, FLAG_FPERP_SNAPSHOTS = 1, 2, 4, 8
FLAG_STATIONARY_FRONT = 16

_D = ctypes.POINTER(ctypes.c_double)


class QSParams(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32),
                ("q", _D), ("m", _D), ("nb_over_np", _D),
                ("gamma_b", ctypes.c_double),
                ("length", ctypes.c_double),
                ("profile", ctypes.c_int32),
                ("sigma_xi", ctypes.c_double),
                ("xi_center", ctypes.c_double),
                ("profile_table", _D),
                ("geometry", ctypes.c_int32),
                ("n_modes", ctypes.c_int64),
                ("kx", _D), ("ky", _D),
                ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("sigma_r", ctypes.c_double),
                ("n_xi", ctypes.c_int32),
                ("d_tau", ctypes.c_double),
                ("precision", ctypes.c_int32),
                ("seed_kind", ctypes.c_int32),
                ("seed_amp", ctypes.c_double),
                ("rng_seed", ctypes.c_uint64),
                ("centroid_offset", ctypes.c_double),
                ("flags", ctypes.c_int32)]


class QSPlan(ctypes.Structure):
    _fields_ = [("columns_per_lane", ctypes.c_int32),
                ("segment_cells", ctypes.c_int32),
                ("max_segments", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class QSGrowthInstance(ctypes.Structure):
    _fields_ = [("nb_over_np", ctypes.c_double), ("gamma_b", ctypes.c_double),
                ("length", ctypes.c_double), ("d_tau", ctypes.c_double),
                ("seed_amp", ctypes.c_double), ("n_xi", ctypes.c_int32),
                ("n_modes", ctypes.c_int32), ("k", _D)]


GROWTH_SURROGATE, GROWTH_SOLVER, GROWTH_AUTO = 0, 1, 2
GROWTH_BINS = 32768


class QSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libqs status %d: %s" % (status, msg))
        self.status = status


_lib = None

EXPORTS = ["qs_abi_version", "qs_last_error", "qs_workspace_size", "qs_workspace_size_ex", "qs_init",
           "qs_init_ex", "qs_get_plan", "qs_tune", "qs_graph_create", "qs_graph_launch", "qs_graph_free",
           "qs_step_tau", "qs_grid_get_state", "qs_grid_set_state", "qs_mlp_param_count", "qs_mlp_create", "qs_mlp_set_params", "qs_mlp_get_params",
           "qs_mlp_forward", "qs_mlp_grads", "qs_mlp_get_grads", "qs_mlp_set_grads", "qs_mlp_adamw",
           "qs_mlp_train_step", "qs_mlp_free", "qs_growth_targets", "qs_growth_sample",
           "qs_growth_features", "qs_growth_calibrate", "qs_growth_map", "qs_growth_map_noalloc",
           "qs_sync_check", "qs_set_rollback", "qs_set_snapshot_align", "qs_debug_set_wait_budget", "qs_steps_done", "qs_get_state", "qs_set_state", "qs_free",
           "qs_debug_splitmix64", "qs_debug_mlp_gemm_check", "qs_checkpoint_size", "qs_save_checkpoint", "qs_load_checkpoint",
           "qs_svea_coefficients", "qs_svea_seed_impulse", "qs_svea_step", "qs_svea_ln_envelope",
           "qs_regime_map", "qs_surrogate_train", "qs_surrogate_load", "qs_surrogate_net", "qs_surrogate_table",
           "qs_surrogate_free"]


def lib():
    """Load libqs.so (raises if it is missing: build it with paper_2607_24234_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqs.so not found at %s; run `python -m paper_2607_24234_amd.build` "
                          "(or __graft_entry__.build())" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER(QSParams)
    vp = ctypes.c_void_p
    L.qs_abi_version.restype = ctypes.c_int32
    L.qs_last_error.restype = ctypes.c_char_p
    L.qs_workspace_size.restype = ctypes.c_size_t
    L.qs_workspace_size.argtypes = [P, ctypes.c_int32]
    L.qs_init.restype = ctypes.c_int
    L.qs_init.argtypes = [P, ctypes.c_int32, vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    PP = ctypes.POINTER(QSPlan)
    L.qs_workspace_size_ex.restype = ctypes.c_size_t
    L.qs_workspace_size_ex.argtypes = [P, ctypes.c_int32, PP]
    L.qs_init_ex.restype = ctypes.c_int
    L.qs_init_ex.argtypes = [P, ctypes.c_int32, PP, vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.qs_get_plan.restype = ctypes.c_int
    L.qs_get_plan.argtypes = [vp, PP, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]
    L.qs_tune.restype = ctypes.c_int
    L.qs_tune.argtypes = [P, ctypes.c_int32, ctypes.c_int32, PP, ctypes.POINTER(ctypes.c_double)]
    L.qs_graph_create.restype = ctypes.c_int
    L.qs_graph_create.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, ctypes.POINTER(vp)]
    L.qs_graph_launch.restype = ctypes.c_int
    L.qs_graph_launch.argtypes = [vp]
    L.qs_graph_free.restype = None
    L.qs_graph_free.argtypes = [vp]
    L.qs_mlp_param_count.restype = ctypes.c_int64
    L.qs_mlp_create.restype = ctypes.c_int
    L.qs_mlp_create.argtypes = [ctypes.c_int32, vp, ctypes.POINTER(vp)]
    F = ctypes.POINTER(ctypes.c_float)
    for name in ("qs_mlp_set_params", "qs_mlp_get_params", "qs_mlp_get_grads", "qs_mlp_set_grads"):
        getattr(L, name).restype = ctypes.c_int
        getattr(L, name).argtypes = [vp, F]
    L.qs_mlp_forward.restype = ctypes.c_int
    L.qs_mlp_forward.argtypes = [vp, vp, ctypes.c_int64, vp]
    L.qs_mlp_grads.restype = ctypes.c_int
    L.qs_mlp_grads.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    L.qs_mlp_adamw.restype = ctypes.c_int
    L.qs_mlp_adamw.argtypes = [vp] + [ctypes.c_double] * 5
    L.qs_mlp_train_step.restype = ctypes.c_int
    L.qs_mlp_train_step.argtypes = [vp, vp, vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
    L.qs_mlp_free.restype = None
    L.qs_mlp_free.argtypes = [vp]
    GI = ctypes.POINTER(QSGrowthInstance)
    L.qs_growth_targets.restype = ctypes.c_int
    L.qs_growth_targets.argtypes = [GI, ctypes.c_int32, vp, vp, ctypes.c_int32, vp, vp]
    L.qs_growth_sample.restype = ctypes.c_int
    L.qs_growth_sample.argtypes = [GI, ctypes.c_int32, vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.c_uint64, ctypes.c_int64, vp, vp, vp]
    L.qs_growth_features.restype = ctypes.c_int
    L.qs_growth_features.argtypes = [vp, ctypes.c_int64, vp, vp, vp]
    L.qs_growth_calibrate.restype = ctypes.c_int
    L.qs_growth_calibrate.argtypes = [vp, vp, vp, ctypes.c_int64, vp]
    L.qs_growth_map.restype = ctypes.c_int
    L.qs_growth_map.argtypes = [vp, vp, ctypes.c_float, vp, ctypes.c_int64, ctypes.c_int32, vp, vp, vp]
    L.qs_growth_map_noalloc.restype = ctypes.c_int
    L.qs_growth_map_noalloc.argtypes = [vp, vp, ctypes.c_float, vp, ctypes.c_int64, vp, vp]
    for name in ("qs_grid_get_state", "qs_grid_set_state"):
        getattr(L, name).restype = ctypes.c_int
        getattr(L, name).argtypes = [vp, _D, _D, _D, _D]
    L.qs_step_tau.restype = ctypes.c_int
    L.qs_step_tau.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    L.qs_sync_check.restype = ctypes.c_int
    L.qs_sync_check.argtypes = [vp]
    L.qs_set_rollback.restype = ctypes.c_int
    L.qs_set_rollback.argtypes = [vp, ctypes.c_int32]
    L.qs_set_snapshot_align.restype = ctypes.c_int
    L.qs_set_snapshot_align.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
    L.qs_debug_set_wait_budget.restype = ctypes.c_int
    L.qs_debug_set_wait_budget.argtypes = [vp, ctypes.c_double]
    L.qs_debug_mlp_gemm_check.restype = ctypes.c_int32
    L.qs_debug_mlp_gemm_check.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p, ctypes.c_int32]
    L.qs_steps_done.restype = ctypes.c_int64
    L.qs_steps_done.argtypes = [vp]
    L.qs_get_state.restype = ctypes.c_int
    L.qs_get_state.argtypes = [vp, _D, _D, _D, _D]
    L.qs_set_state.restype = ctypes.c_int
    L.qs_set_state.argtypes = [vp, _D, _D, _D, _D]
    L.qs_free.restype = None
    L.qs_free.argtypes = [vp]
    L.qs_checkpoint_size.restype = ctypes.c_size_t
    L.qs_checkpoint_size.argtypes = [vp]
    L.qs_save_checkpoint.restype = ctypes.c_int
    L.qs_save_checkpoint.argtypes = [vp, vp, ctypes.c_size_t]
    L.qs_load_checkpoint.restype = ctypes.c_int
    L.qs_load_checkpoint.argtypes = [vp, vp, ctypes.c_size_t]
    L.qs_debug_splitmix64.restype = ctypes.c_uint64
    L.qs_debug_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    L.qs_svea_coefficients.restype = ctypes.c_int
    L.qs_svea_coefficients.argtypes = [ctypes.c_int32, _D, _D, _D, ctypes.c_double, ctypes.c_int64, _D, _D]
    L.qs_svea_seed_impulse.restype = ctypes.c_int
    L.qs_svea_seed_impulse.argtypes = [ctypes.c_int64, ctypes.c_int32, vp, vp, vp, vp]
    L.qs_svea_step.restype = ctypes.c_int
    L.qs_svea_step.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_double, vp, ctypes.c_double, ctypes.c_int32,
                               vp, vp, vp, vp]
    L.qs_svea_ln_envelope.restype = ctypes.c_int
    L.qs_svea_ln_envelope.argtypes = [ctypes.c_int64, ctypes.c_int32, vp, vp, vp, vp]
    L.qs_surrogate_train.restype = ctypes.c_int
    L.qs_surrogate_train.argtypes = [ctypes.c_char_p, ctypes.c_char_p, vp, ctypes.POINTER(ctypes.c_double)]
    L.qs_surrogate_load.restype = ctypes.c_int
    L.qs_surrogate_load.argtypes = [ctypes.c_char_p, vp, ctypes.POINTER(vp)]
    L.qs_surrogate_net.restype = vp
    L.qs_surrogate_net.argtypes = [vp]
    L.qs_surrogate_table.restype = vp
    L.qs_surrogate_table.argtypes = [vp]
    L.qs_surrogate_free.restype = None
    L.qs_surrogate_free.argtypes = [vp]
    L.qs_regime_map.restype = ctypes.c_int
    L.qs_regime_map.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
    _lib = L
    return L


def _check(status):
    if status != QS_OK:
        raise QSError(status, lib().qs_last_error().decode(errors="replace"))


def _dp(a):
    return None if a is None else a.ctypes.data_as(_D)


class _Instance:
    """Keeps the numpy arrays behind one QSParams alive."""

    def __init__(self, inst, precision):
        sp = inst["species"]
        self.q = np.ascontiguousarray([s[0] for s in sp], np.float64)
        self.m = np.ascontiguousarray([s[1] for s in sp], np.float64)
        self.nb = np.ascontiguousarray([s[2] for s in sp], np.float64)
        self.kx = np.ascontiguousarray(inst.get("kx", np.zeros(0)), np.float64)
        ky = inst.get("ky")
        self.ky = None if ky is None else np.ascontiguousarray(ky, np.float64)
        tab = inst.get("profile_table")
        self.tab = None if tab is None else np.ascontiguousarray(tab, np.float64)
        p = QSParams()
        p.n_species = len(sp)
        p.q, p.m, p.nb_over_np = _dp(self.q), _dp(self.m), _dp(self.nb)
        p.gamma_b = float(inst["gamma"])
        p.length = float(inst["length"])
        p.profile = int(inst.get("profile", PROFILE_TABLE if self.tab is not None else PROFILE_FLATTOP))
        p.sigma_xi = float(inst.get("sigma_xi", 0.0))
        p.xi_center = float(inst.get("xi_center", 0.0))
        p.profile_table = _dp(self.tab)
        p.geometry = int(inst.get("geometry", GEOM_SPECTRAL))
        p.n_modes = len(self.kx)
        p.kx, p.ky = _dp(self.kx), _dp(self.ky)
        p.n_xi = int(inst["n_xi"])
        p.d_tau = float(inst["d_tau"])
        p.precision = precision
        p.seed_kind = int(inst.get("seed_kind", SEED_NOISE))
        p.seed_amp = float(inst.get("seed_amp", 1e-6))
        p.rng_seed = int(inst.get("rng_seed", 0)) & (2**64 - 1)
        p.flags = int(inst.get("flags", 0))
        p.nx, p.ny = int(inst.get("nx", 0)), int(inst.get("ny", 0))
        p.lx, p.ly = float(inst.get("lx", 0.0)), float(inst.get("ly", 0.0))
        p.sigma_r = float(inst.get("sigma_r", 0.0))
        p.centroid_offset = float(inst.get("centroid_offset", 0.0))
        self.p = p
        self.n_modes = len(self.kx)
        self.n_xi = p.n_xi


def _plan(columns_per_lane=0, segment_cells=0):
    if not columns_per_lane and not segment_cells:
        return None
    return QSPlan(int(columns_per_lane), int(segment_cells), 0, 0)


def workspace_size(instances, precision=QS_FP32, columns_per_lane=0, segment_cells=0):
    insts = [_Instance(i, precision) for i in instances]
    arr = (QSParams * len(insts))(*[x.p for x in insts])
    pl = _plan(columns_per_lane, segment_cells)
    return int(lib().qs_workspace_size_ex(arr, len(insts), ctypes.byref(pl) if pl else None))


MLP_DIMS = (5, 512, 512, 512, 512, 1)


def pack_params(params):
    """[(W [out, in], b [out]), ...] -> flat float32 array in the library's layout."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(), np.asarray(b, np.float32).ravel()])
                           for W, b in params]).astype(np.float32)


def unpack_params(flat, dims=MLP_DIMS):
    out, o = [], 0
    for i in range(len(dims) - 1):
        n_w = dims[i + 1] * dims[i]
        W = np.asarray(flat[o:o + n_w], np.float64).reshape(dims[i + 1], dims[i])
        o += n_w
        b = np.asarray(flat[o:o + dims[i + 1]], np.float64)
        o += dims[i + 1]
        out.append((W, b))
    return out


class MLP:
    """The surrogate network (include/qs_mlp.h) on one device; tensors are torch CUDA
    float32 tensors, parameters host numpy arrays."""

    def __init__(self, max_batch=65536, stream=None):
        import torch
        self.torch = torch
        self.stream = torch.cuda.current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        _check(lib().qs_mlp_create(int(max_batch), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.max_batch = int(max_batch)
        self.n_params = int(lib().qs_mlp_param_count())

    def _f(self, a):
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))

    def set_params(self, params):
        flat = np.ascontiguousarray(params if isinstance(params, np.ndarray) else pack_params(params), np.float32)
        assert flat.size == self.n_params
        _check(lib().qs_mlp_set_params(self.h, self._f(flat)))

    def get_params(self):
        flat = np.empty(self.n_params, np.float32)
        _check(lib().qs_mlp_get_params(self.h, self._f(flat)))
        return flat

    def get_grads(self):
        flat = np.empty(self.n_params, np.float32)
        _check(lib().qs_mlp_get_grads(self.h, self._f(flat)))
        return flat

    def set_grads(self, flat):
        flat = np.ascontiguousarray(flat, np.float32)
        _check(lib().qs_mlp_set_grads(self.h, self._f(flat)))

    def forward(self, x, out=None):
        t = self.torch
        x = x.contiguous()
        y = t.empty(x.shape[0], dtype=t.float32, device=x.device) if out is None else out
        _check(lib().qs_mlp_forward(self.h, ctypes.c_void_p(x.data_ptr()), int(x.shape[0]), ctypes.c_void_p(y.data_ptr())))
        return y

    def grads(self, x, target, want_loss=True):
        loss = ctypes.c_double()
        _check(lib().qs_mlp_grads(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                  int(x.shape[0]), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def adamw(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.01):
        _check(lib().qs_mlp_adamw(self.h, lr, beta1, beta2, eps, weight_decay))

    def train_step(self, x, target, lr, want_loss=False):
        loss = ctypes.c_double()
        _check(lib().qs_mlp_train_step(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(target.data_ptr()),
                                       int(x.shape[0]), lr, ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().qs_mlp_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BorrowedMLP(MLP):
    """A network owned by another handle (qs_surrogate_net): same calls, never freed here."""

    def __init__(self, handle, stream=None):
        import torch
        self.torch = torch
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self.h = ctypes.c_void_p(handle)
        self.max_batch = 128
        self.n_params = int(lib().qs_mlp_param_count())

    def close(self):
        self.h = None


SURROGATE_STATS = 8
SURROGATE_STAT_NAMES = ("heldout_rms", "heldout_p99", "heldout_max", "heldout_within_1e-2", "bins_trusted_1e-2",
                        "final_loss", "seconds_data", "seconds_train")


def surrogate_train(path, cfg=None, stream=None):
    """qs_surrogate_train: the whole training pipeline in the library; cfg is a dict of the
    configuration keys of include/qs_surrogate.h.  Returns the statistics as a dict."""
    import json
    import torch
    text = json.dumps(cfg or {}).encode()
    st = (ctypes.c_double * SURROGATE_STATS)()
    s = torch.cuda.current_stream() if stream is None else stream
    _check(lib().qs_surrogate_train(text, os.fsencode(path), ctypes.c_void_p(s.cuda_stream), st))
    return dict(zip(SURROGATE_STAT_NAMES, list(st)))


class Surrogate:
    """A trained surrogate file loaded on the current device (qs_surrogate_load): `net` for
    qs_growth_map and `table`, the device address of its error table."""

    def __init__(self, path, stream=None):
        import torch
        s = torch.cuda.current_stream() if stream is None else stream
        h = ctypes.c_void_p()
        _check(lib().qs_surrogate_load(os.fsencode(path), ctypes.c_void_p(s.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.net = BorrowedMLP(lib().qs_surrogate_net(h), s)
        self.table = int(lib().qs_surrogate_table(h))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().qs_surrogate_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GrowthInstances:
    """qs_growth_instance descriptions of solver instances (dicts from inputs.py with a
    single species); keeps the k arrays alive."""

    def __init__(self, instances):
        self._k = []
        arr = (QSGrowthInstance * len(instances))()
        for i, inst in enumerate(instances):
            (q, m, nb), = inst["species"]
            k = np.asarray(inst["kx"], np.float64)
            ky = inst.get("ky")
            kk = np.ascontiguousarray(np.abs(k) if ky is None else np.hypot(k, np.asarray(ky, np.float64)), np.float64)
            self._k.append(kk)
            arr[i] = QSGrowthInstance(nb, inst["gamma"], inst["length"], inst["d_tau"], inst.get("seed_amp", 1e-6),
                                      inst["n_xi"], len(kk), _dp(kk))
        self.arr = arr
        self.n = len(instances)


def _vp(t):
    """Device pointer of a torch tensor, or a raw address (int), or None."""
    if t is None:
        return None
    if isinstance(t, int):
        return ctypes.c_void_p(t)
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    return ctypes.c_void_p(stream.cuda_stream) if stream is not None else None


def growth_targets(gi, ln_e, ln_b, G, stream=None):
    n_snap = ln_e.shape[0]
    _check(lib().qs_growth_targets(gi.arr, gi.n, _vp(ln_e), _vp(ln_b), int(n_snap), _vp(G), _stream_ptr(stream)))


def growth_sample(gi, G, snap_steps, seed, n, Q, T, stream=None):
    """Examples: queries Q [n, 5] (ln n_b, ln gamma, k, xi, tau) and their targets T [n]."""
    st = np.ascontiguousarray(snap_steps, np.int32)
    _check(lib().qs_growth_sample(gi.arr, gi.n, _vp(G), len(st), st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  int(seed), int(n), _vp(Q), _vp(T), _stream_ptr(stream)))


def growth_features(q, x=None, baseline=None, stream=None):
    """Network inputs x [n, 5] and baseline [n] of queries q [n, 5] (either output optional)."""
    _check(lib().qs_growth_features(_vp(q), int(q.shape[0]), _vp(x), _vp(baseline), _stream_ptr(stream)))


def growth_calibrate(net, Q, T, table):
    _check(lib().qs_growth_calibrate(net.h, _vp(Q), _vp(T), int(Q.shape[0]), _vp(table)))


def growth_map(net, table, tol, q, mode, out, used_solver=None, stream=None):
    _check(lib().qs_growth_map(net.h if net is not None else None, _vp(table), float(tol), _vp(q), int(q.shape[0]),
                               int(mode), _vp(out), _vp(used_solver), _stream_ptr(stream)))


GROWTH_NOALLOC_MAX = 262144  # mirrored from include/qs_growth.h


def growth_map_noalloc(net, table, tol, q, out, needs_solver):
    """Network answers and routing flags with no allocation (qs_growth_map_noalloc), queued
    on the network's stream."""
    _check(lib().qs_growth_map_noalloc(net.h, _vp(table), float(tol), _vp(q), int(q.shape[0]), _vp(out),
                                       _vp(needs_solver)))


class GridSolver:
    """A finite-width context (geometry TRANSVERSE_GRID, FP32) over one instance dict with
    keys nx, ny, lx, ly, sigma_r, centroid_offset besides the usual ones."""

    def __init__(self, inst, device=None, stream=None):
        import torch
        self.torch = torch
        inst = dict(inst)
        inst["geometry"] = GEOM_TRANSVERSE_GRID
        self._inst = _Instance(inst, QS_FP32)
        self._params = (QSParams * 1)(self._inst.p)
        self.shape = (int(inst["n_xi"]), int(inst["ny"]), int(inst["nx"]))
        self.cells = int(np.prod(self.shape))
        L = lib()
        nbytes = int(L.qs_workspace_size(self._params, 1))
        if nbytes == 0:
            _check(L.qs_init(self._params, 1, None, None, 0, ctypes.byref(ctypes.c_void_p())))
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream() if stream is None else stream
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            ctx = ctypes.c_void_p()
            _check(L.qs_init(self._params, 1, ctypes.c_void_p(self.stream.cuda_stream),
                             ctypes.c_void_p(self.workspace.data_ptr()), nbytes, ctypes.byref(ctx)))
        self.ctx = ctx

    def step(self, n_steps, out_every=1, snapshots=False, max_ln_a=False, out=None):
        t = self.torch
        res = {} if out is None else out
        if snapshots:
            n_snap = 1 if n_steps == 0 else -(-n_steps // max(1, out_every))
            if "ln_e" not in res:
                res["ln_e"] = t.empty((n_snap,) + self.shape, dtype=t.float32, device=self.device)
                res["ln_b"] = t.empty((n_snap,) + self.shape, dtype=t.float32, device=self.device)
        if max_ln_a and n_steps > 0 and "max_ln_a" not in res:
            res["max_ln_a"] = t.empty(n_steps, dtype=t.float32, device=self.device)
        pe = ctypes.c_void_p(res["ln_e"].data_ptr()) if snapshots else None
        pb = ctypes.c_void_p(res["ln_b"].data_ptr()) if snapshots else None
        pm = ctypes.c_void_p(res["max_ln_a"].data_ptr()) if (max_ln_a and n_steps > 0) else None
        _check(lib().qs_step_tau(self.ctx, int(n_steps), int(max(1, out_every)), pe, pb, pm))
        return res

    def sync_check(self):
        _check(lib().qs_sync_check(self.ctx))

    def get_state(self):
        arrs = [np.empty(self.shape) for _ in range(4)]
        _check(lib().qs_grid_get_state(self.ctx, *[_dp(a) for a in arrs]))
        return dict(zip(("rho", "j_par", "j_x", "j_y"), arrs))

    def set_state(self, st):
        arrs = [np.ascontiguousarray(st[k], np.float64).reshape(self.shape) for k in ("rho", "j_par", "j_x", "j_y")]
        _check(lib().qs_grid_set_state(self.ctx, *[_dp(a) for a in arrs]))

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().qs_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune(instances, precision=QS_FP32, steps_per_call=100):
    """Autotuned launch plan for these instances (qs_tune): dict with columns_per_lane,
    segment_cells and ms_per_step; pass the first two to Solver."""
    insts = [_Instance(i, precision) for i in instances]
    arr = (QSParams * len(insts))(*[x.p for x in insts])
    best = QSPlan()
    ms = ctypes.c_double()
    _check(lib().qs_tune(arr, len(insts), int(steps_per_call), ctypes.byref(best), ctypes.byref(ms)))
    return {"columns_per_lane": best.columns_per_lane, "segment_cells": best.segment_cells,
            "ms_per_step": ms.value}


class Graph:
    """A captured qs_step_tau call (qs_graph_create); replay() advances the solver by
    n_steps and rewrites the same output tensors."""

    def __init__(self, solver, n_steps, out_every=1, snapshots=False, max_ln_a=False):
        t = solver.torch
        self.solver = solver
        self.out = {}
        if snapshots:
            n_snap = -(-n_steps // max(1, out_every))
            self.out["ln_e"] = t.empty((n_snap, solver.snap_elems), dtype=solver.dtype, device=solver.device)
            self.out["ln_b"] = t.empty((n_snap, solver.snap_elems), dtype=solver.dtype, device=solver.device)
        if max_ln_a:
            self.out["max_ln_a"] = t.empty((n_steps, solver.total_modes), dtype=solver.dtype, device=solver.device)
        ptr = lambda k: ctypes.c_void_p(self.out[k].data_ptr()) if k in self.out else None
        g = ctypes.c_void_p()
        _check(lib().qs_graph_create(solver.ctx, int(n_steps), int(max(1, out_every)), ptr("ln_e"), ptr("ln_b"),
                                     ptr("max_ln_a"), ctypes.byref(g)))
        self.g = g

    def replay(self):
        _check(lib().qs_graph_launch(self.g))
        return self.out

    def close(self):
        if getattr(self, "g", None) is not None and self.g.value:
            lib().qs_graph_free(self.g)
            self.g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """A qs_ctx over one or more instances, with torch-owned device memory.

    instances: list of dicts as produced by ``paper_2607_24234_amd.inputs`` (keys species,
    gamma, length, n_xi, kx, ky, d_tau, seed_kind, seed_amp, rng_seed, flags, ...).
    columns_per_lane / segment_cells: launch plan overrides (0 = the library's choice).
    """

    def __init__(self, instances, precision=QS_FP32, device=None, stream=None, columns_per_lane=0,
                 segment_cells=0):
        import torch
        if isinstance(instances, dict):
            instances = [instances]
        L = lib()
        self.torch = torch
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self._insts = [_Instance(i, precision) for i in instances]
        self._params = (QSParams * len(self._insts))(*[x.p for x in self._insts])
        self._plan = _plan(columns_per_lane, segment_cells)
        pp = ctypes.byref(self._plan) if self._plan else None
        nbytes = int(L.qs_workspace_size_ex(self._params, len(self._insts), pp))
        if nbytes == 0:
            _check(L.qs_init_ex(self._params, len(self._insts), pp, None, None, 0, ctypes.byref(ctypes.c_void_p())))
        self.n_modes = [x.n_modes for x in self._insts]
        self.n_xi = [x.n_xi for x in self._insts]
        self.total_modes = sum(self.n_modes)
        self.state_elems = sum(m * n for m, n in zip(self.n_modes, self.n_xi))
        self.snap_ld = list(self.n_modes)   # snapshot row length per instance (qs_set_snapshot_align)
        self.snap_elems = self.state_elems
        self.dtype = torch.float64 if precision == QS_FP64 else torch.float32
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream() if stream is None else stream
            # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            ctx = ctypes.c_void_p()
            _check(L.qs_init_ex(self._params, len(self._insts), pp, ctypes.c_void_p(self.stream.cuda_stream),
                                ctypes.c_void_p(self.workspace.data_ptr()), nbytes, ctypes.byref(ctx)))
        self.ctx = ctx

    def plan(self):
        """Launch plan the library chose: dict columns_per_lane, segment_cells, max_segments,
        workgroups, waves_per_workgroup."""
        p = QSPlan()
        nwg, wpw = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().qs_get_plan(self.ctx, ctypes.byref(p), ctypes.byref(nwg), ctypes.byref(wpw)))
        return {"columns_per_lane": p.columns_per_lane, "segment_cells": p.segment_cells,
                "max_segments": p.max_segments, "workgroups": nwg.value, "waves_per_workgroup": wpw.value}

    # -------------------------------------------------------------- stepping
    def step(self, n_steps, out_every=1, snapshots=False, max_ln_a=False, out=None):
        """Advance every instance by n_steps tau-steps.  Returns a dict of torch tensors:
        'ln_e', 'ln_b' [n_snap, snap_elems] (if snapshots) and 'max_ln_a' [n_steps, total_modes]."""
        t = self.torch
        res = {} if out is None else out
        n_snap = 0
        if snapshots:
            n_snap = 1 if n_steps == 0 else -(-n_steps // max(1, out_every))
            if "ln_e" not in res:
                res["ln_e"] = t.empty((n_snap, self.snap_elems), dtype=self.dtype, device=self.device)
                res["ln_b"] = t.empty((n_snap, self.snap_elems), dtype=self.dtype, device=self.device)
        if max_ln_a and n_steps > 0 and "max_ln_a" not in res:
            res["max_ln_a"] = t.empty((n_steps, self.total_modes), dtype=self.dtype, device=self.device)
        pe = ctypes.c_void_p(res["ln_e"].data_ptr()) if snapshots else None
        pb = ctypes.c_void_p(res["ln_b"].data_ptr()) if snapshots else None
        pm = ctypes.c_void_p(res["max_ln_a"].data_ptr()) if (max_ln_a and n_steps > 0) else None
        _check(lib().qs_step_tau(self.ctx, int(n_steps), int(max(1, out_every)), pe, pb, pm))
        return res

    def snapshot_view(self, flat, instance=0):
        """View of one instance's block of a snapshot row as [n_xi, n_modes] (the padding of
        aligned rows left out)."""
        off = sum(ld * n for ld, n in zip(self.snap_ld[:instance], self.n_xi[:instance]))
        n, m, ld = self.n_xi[instance], self.n_modes[instance], self.snap_ld[instance]
        return flat[..., off:off + n * ld].reshape(*flat.shape[:-1], n, ld)[..., :m]

    def set_snapshot_align(self, align):
        """Pad each instance's snapshot rows to a multiple of `align` modes
        (qs_set_snapshot_align; 1 = dense)."""
        elems = ctypes.c_int64()
        _check(lib().qs_set_snapshot_align(self.ctx, int(align), ctypes.byref(elems)))
        self.snap_ld = [-(-m // align) * align for m in self.n_modes]
        self.snap_elems = int(elems.value)
        assert self.snap_elems == sum(ld * n for ld, n in zip(self.snap_ld, self.n_xi))

    def sync_check(self):
        _check(lib().qs_sync_check(self.ctx))

    def set_rollback(self, enable=True):
        """Keep a device copy of the last good state for qs_sync_check to restore."""
        _check(lib().qs_set_rollback(self.ctx, 1 if enable else 0))

    def debug_wait_budget(self, seconds):
        """Test hook: the hand-off wait budget of the march launches (-1 = default)."""
        _check(lib().qs_debug_set_wait_budget(self.ctx, float(seconds)))

    @property
    def steps_done(self):
        return int(lib().qs_steps_done(self.ctx))

    # -------------------------------------------------------------- state
    def get_state(self):
        """Canonical state: list (per instance) of dicts rho, j_par, j_perp [n_modes, n_xi]
        complex128 and log2_scale [n_modes]."""
        tot = self.state_elems
        rho = np.empty(2 * tot)
        jpa = np.empty(2 * tot)
        jpe = np.empty(2 * tot)
        l2 = np.empty(self.total_modes)
        _check(lib().qs_get_state(self.ctx, _dp(rho), _dp(jpa), _dp(jpe), _dp(l2)))
        out, o, mo = [], 0, 0
        for m, n in zip(self.n_modes, self.n_xi):
            sl = slice(2 * o, 2 * (o + m * n))
            out.append({"rho": rho[sl].view(np.complex128).reshape(m, n).copy(),
                        "j_par": jpa[sl].view(np.complex128).reshape(m, n).copy(),
                        "j_perp": jpe[sl].view(np.complex128).reshape(m, n).copy(),
                        "log2_scale": l2[mo:mo + m].copy()})
            o += m * n
            mo += m
        return out

    def set_state(self, states):
        rho = np.concatenate([np.ascontiguousarray(s["rho"], np.complex128).ravel() for s in states])
        jpa = np.concatenate([np.ascontiguousarray(s["j_par"], np.complex128).ravel() for s in states])
        jpe = np.concatenate([np.ascontiguousarray(s["j_perp"], np.complex128).ravel() for s in states])
        l2 = np.concatenate([np.ascontiguousarray(s["log2_scale"], np.float64).ravel() for s in states])
        _check(lib().qs_set_state(self.ctx, _dp(rho.view(np.float64)), _dp(jpa.view(np.float64)),
                                  _dp(jpe.view(np.float64)), _dp(l2)))

    def save_checkpoint(self):
        """Opaque bitwise image of the state (bytes)."""
        n = int(lib().qs_checkpoint_size(self.ctx))
        buf = np.empty(n, np.uint8)
        _check(lib().qs_save_checkpoint(self.ctx, buf.ctypes.data_as(ctypes.c_void_p), n))
        return buf

    def load_checkpoint(self, buf):
        buf = np.ascontiguousarray(buf, np.uint8)
        _check(lib().qs_load_checkpoint(self.ctx, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes))

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().qs_free(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def svea_coefficients(species, gamma, k):
    """(i/2) Gamma_CFI(k)^2 per wavenumber (include/qs_svea.h), as a complex numpy array."""
    q = np.ascontiguousarray([sp[0] for sp in species], np.float64)
    m = np.ascontiguousarray([sp[1] for sp in species], np.float64)
    nb = np.ascontiguousarray([sp[2] for sp in species], np.float64)
    k = np.ascontiguousarray(k, np.float64).ravel()
    a = np.empty(2 * len(k), np.float64)
    _check(lib().qs_svea_coefficients(len(q), _dp(q), _dp(m), _dp(nb), float(gamma), len(k), _dp(k), _dp(a)))
    return a[0::2] + 1j * a[1::2]


def half_window_cells(half_width, h):
    """Cells within half_width of a cell centre on either side: floor(half_width / h), with a
    relative allowance of 1e-9 for a ratio that is an integer up to rounding."""
    return int(math.floor(half_width / h * (1.0 + 1e-9)))


def regime_map(ln_e, ln_b, half_window, log_ratio=True, first_e_cell=True, stream=None):
    """E/B regime diagnostic (include/qs_regime.h) of one snapshot pair: ln_e, ln_b are torch
    device tensors [n_xi][n_modes] (float32 or float64, contiguous), half_window the window's
    half width in cells.  Returns (R [n_xi][n_modes] of the same type or None, first
    electrically dominated cell int32 [n_modes] or None)."""
    import torch
    if ln_e.shape != ln_b.shape or ln_e.dtype != ln_b.dtype or ln_e.dim() != 2:
        raise ValueError("ln_e and ln_b must be [n_xi][n_modes] tensors of one type")
    if not (ln_e.is_contiguous() and ln_b.is_contiguous()):
        raise ValueError("ln_e and ln_b must be contiguous")
    prec = {torch.float32: QS_FP32, torch.float64: QS_FP64}.get(ln_e.dtype)
    if prec is None:
        raise ValueError("ln_e and ln_b must be float32 or float64")
    n_xi, n_modes = ln_e.shape
    R = torch.empty_like(ln_e) if log_ratio else None
    F = torch.empty(n_modes, dtype=torch.int32, device=ln_e.device) if first_e_cell else None
    s = torch.cuda.current_stream() if stream is None else stream
    _check(lib().qs_regime_map(_vp(ln_e), _vp(ln_b), n_modes, n_xi, int(half_window), prec,
                               _vp(R) if R is not None else None, _vp(F) if F is not None else None,
                               _stream_ptr(s)))
    return R, F


class SVEASolver:
    """The envelope-approximation variant (include/qs_svea.h) for one beam and a list of
    wavenumbers: FP64 state n, m (complex, blocks of 64 modes) in torch device memory, seeded by
    the front impulse; state() returns them as [n_xi][n_modes]."""

    def __init__(self, species, gamma, k, length, n_xi, d_tau, stream=None):
        import torch
        self.torch = torch
        self.stream = torch.cuda.current_stream() if stream is None else stream
        self.k = np.ascontiguousarray(k, np.float64).ravel()
        self.n_modes, self.n_xi = len(self.k), int(n_xi)
        self.h = float(length) / self.n_xi
        self.d_tau = float(d_tau)
        a = svea_coefficients(species, gamma, self.k)
        self.a = torch.as_tensor(np.stack([a.real, a.imag], 1), device="cuda").contiguous()
        self.n_blocks = (self.n_modes + 63) // 64
        self.n = torch.empty((self.n_blocks, self.n_xi, 64, 2), dtype=torch.float64, device="cuda")
        self.m = torch.empty_like(self.n)
        self.log2 = torch.empty(self.n_modes, dtype=torch.int32, device="cuda")
        self.seed_impulse()

    def _s(self):
        return _stream_ptr(self.stream)

    def seed_impulse(self):
        _check(lib().qs_svea_seed_impulse(self.n_modes, self.n_xi, _vp(self.n), _vp(self.m), _vp(self.log2), self._s()))

    def step(self, n_steps):
        _check(lib().qs_svea_step(self.n_modes, self.n_xi, self.h, _vp(self.a), self.d_tau, int(n_steps), _vp(self.n),
                                  _vp(self.m), _vp(self.log2), self._s()))

    def ln_envelope(self, out=None):
        out = self.torch.empty((self.n_xi, self.n_modes), dtype=self.torch.float64, device="cuda") if out is None else out
        _check(lib().qs_svea_ln_envelope(self.n_modes, self.n_xi, _vp(self.n), _vp(self.log2), _vp(out), self._s()))
        return out

    def state(self):
        """(n, m) as complex numpy arrays [n_xi][n_modes] including the power-of-two scale."""
        self.torch.cuda.synchronize()
        sc = np.ldexp(1.0, self.log2.cpu().numpy().astype(np.int64))
        def unblock(t):
            a = t.cpu().numpy()                                   # [block][cell][lane][2]
            a = a.transpose(1, 0, 2, 3).reshape(self.n_xi, self.n_blocks * 64, 2)[:, :self.n_modes]
            return a[..., 0] + 1j * a[..., 1]
        return unblock(self.n) * sc[None, :], unblock(self.m) * sc[None, :]
