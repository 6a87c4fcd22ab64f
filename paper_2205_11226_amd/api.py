"""ctypes binding of the C ABI in include/skmmse.h (same names, same order).

Host arrays are NumPy; device buffers are PyTorch tensors (``torch`` is used
only for device memory and the current HIP stream).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libskmmse.so")

MODES = {"profile": 0, "cnn": 1, "brl": 2, "idl": 3, "full": 4, "plain": 5}
LAYER_FILL, LAYER_BRL, LAYER_IDL, LAYER_HQL = -1, 0, 1, 2
FLAG_CTX_RELAXED, FLAG_NO_HQL, FLAG_NO_CAND, FLAG_EMPTY_CTX, FLAG_HQL_SINGULAR = 1, 2, 4, 8, 16

EXPORTS = ("skm_default_params", "skm_patch_params", "skm_create", "skm_destroy", "skm_conceal",
           "skm_conceal_device", "skm_conceal_device_noalloc", "skm_distances_device", "skm_cnn_init", "skm_cnn_set_weights",
           "skm_cnn_get_weights", "skm_cnn_set_thresholds", "skm_save_cnn", "skm_load_cnn",
           "skm_cnn_inputs", "skm_cnn_forward", "skm_cnn_gradients", "skm_cnn_train_step",
           "skm_cnn_last_predictions", "skm_conceal_batch", "skm_set_option", "skm_get_option",
           "skm_autotune", "skm_autotune_save", "skm_autotune_load", "skm_profile_enable",
           "skm_profile_read", "skm_last_error")
OPT_GRAPHS, OPT_BATCH_STREAMS, OPT_GATE_GRID, OPT_HQL_GRID = 1, 2, 3, 4
OPT_BATCH_MODE, OPT_EST_VARIANT, OPT_GROUP_SPLIT = 5, 6, 7
CNN_PARAMS = 20898


class SkmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"skmmse status {status}: {msg}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32), ("ring", ctypes.c_int32), ("window", ctypes.c_int32),
        ("expand_step", ctypes.c_int32), ("min_overlap_pct", ctypes.c_int32),
        ("min_hql_cands", ctypes.c_int32), ("mode", ctypes.c_int32),
        ("max_rounds", ctypes.c_int32), ("sigma2", ctypes.c_double),
        ("t_phi", ctypes.c_double), ("t_nu", ctypes.c_double), ("ridge_rel", ctypes.c_double),
        ("hql_partial", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


class BlockInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in (
        "bx", "by", "layer", "round", "n_cand", "n_complete", "radius", "flags", "phi",
        "n_ctx")] + [("log_nu", ctypes.c_double)]


class FrameDesc(ctypes.Structure):
    _fields_ = [
        ("frame", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("out", ctypes.c_void_p),
        ("width", ctypes.c_int32), ("height", ctypes.c_int32), ("stride", ctypes.c_int32),
        ("params", ctypes.POINTER(Params)), ("info", ctypes.c_void_p), ("xhat", ctypes.c_void_p),
        ("cap", ctypes.c_int32), ("n_lost", ctypes.c_int32), ("rounds", ctypes.c_int32),
        ("status", ctypes.c_int32), ("reserved", ctypes.c_int32),
    ]


BLOCK_INFO_DTYPE = np.dtype([(n, "<i4") for n in (
    "bx", "by", "layer", "round", "n_cand", "n_complete", "radius", "flags", "phi",
    "n_ctx")] + [("log_nu", "<f8")])
assert BLOCK_INFO_DTYPE.itemsize == ctypes.sizeof(BlockInfo) == 48


def _load():
    # PyTorch ships its own HIP runtime under the same soname as the system
    # one the library links; loading torch first makes the process use one
    # runtime for both (the other order leaves torch without devices).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2205_11226_amd/build.py`")
    so = ctypes.CDLL(LIB_PATH)
    p, i32, vp = ctypes.POINTER, ctypes.c_int32, ctypes.c_void_p
    so.skm_default_params.argtypes = [p(Params)]
    so.skm_default_params.restype = None
    so.skm_patch_params.argtypes = [p(Params)]
    so.skm_patch_params.restype = None
    so.skm_create.argtypes = [i32, p(vp)]
    so.skm_create.restype = i32
    so.skm_destroy.argtypes = [vp]
    so.skm_destroy.restype = None
    so.skm_conceal.argtypes = [vp, vp, vp, i32, i32, i32, p(Params), vp, vp, i32, p(i32)]
    so.skm_conceal.restype = i32
    so.skm_conceal_device.argtypes = [vp, vp, vp, i32, i32, i32, p(Params), vp, vp, vp, i32,
                                      p(i32), vp]
    so.skm_conceal_device.restype = i32
    so.skm_conceal_device_noalloc.argtypes = so.skm_conceal_device.argtypes
    so.skm_conceal_device_noalloc.restype = so.skm_conceal_device.restype
    so.skm_distances_device.argtypes = [vp, vp, vp, i32, i32, i32, p(Params), vp, vp, i32,
                                        p(i32), vp]
    so.skm_distances_device.restype = i32
    f32, f64, cp = ctypes.c_float, ctypes.c_double, ctypes.c_char_p
    so.skm_cnn_init.argtypes = [vp, ctypes.c_uint64]
    so.skm_cnn_set_weights.argtypes = [vp, vp, i32]
    so.skm_cnn_get_weights.argtypes = [vp, vp, i32]
    so.skm_cnn_set_thresholds.argtypes = [vp, f64, f64]
    so.skm_save_cnn.argtypes = [vp, cp]
    so.skm_load_cnn.argtypes = [vp, cp]
    so.skm_cnn_inputs.argtypes = [vp, vp, vp, i32, i32, i32, p(Params), vp, i32, p(i32), vp]
    so.skm_cnn_forward.argtypes = [vp, vp, i32, vp, vp]
    so.skm_cnn_gradients.argtypes = [vp, vp, vp, i32, vp, p(f32), vp]
    so.skm_cnn_train_step.argtypes = [vp, vp, vp, i32, f32, p(f32), vp]
    so.skm_cnn_last_predictions.argtypes = [vp, vp, i32]
    for n in ("skm_cnn_init", "skm_cnn_set_weights", "skm_cnn_get_weights",
              "skm_cnn_set_thresholds", "skm_save_cnn", "skm_load_cnn", "skm_cnn_inputs",
              "skm_cnn_forward", "skm_cnn_gradients", "skm_cnn_train_step",
              "skm_cnn_last_predictions"):
        getattr(so, n).restype = i32
    so.skm_conceal_batch.argtypes = [vp, p(FrameDesc), i32, vp]
    so.skm_conceal_batch.restype = i32
    so.skm_set_option.argtypes = [vp, i32, ctypes.c_int64]
    so.skm_set_option.restype = i32
    so.skm_get_option.argtypes = [vp, i32, p(ctypes.c_int64)]
    so.skm_get_option.restype = i32
    so.skm_autotune.argtypes = [vp, p(FrameDesc), i32, i32, p(ctypes.c_double)]
    so.skm_autotune.restype = i32
    so.skm_autotune_save.argtypes = [vp, cp]
    so.skm_autotune_save.restype = i32
    so.skm_autotune_load.argtypes = [vp, cp]
    so.skm_autotune_load.restype = i32
    so.skm_profile_enable.argtypes = [vp, i32]
    so.skm_profile_enable.restype = i32
    so.skm_profile_read.argtypes = [vp, p(ctypes.c_double), p(i32)]
    so.skm_profile_read.restype = i32
    so.skm_last_error.argtypes = []
    so.skm_last_error.restype = ctypes.c_char_p
    return so


lib = _load()


def exported_symbols() -> tuple:
    return tuple(n for n in EXPORTS if hasattr(lib, n))


def _check(status: int):
    if status != 0:
        raise SkmError(status, lib.skm_last_error().decode(errors="replace"))


def default_params(**kw) -> Params:
    """Paper defaults; keyword overrides (``mode`` may be a name)."""
    prm = Params()
    lib.skm_default_params(ctypes.byref(prm))
    return _override(prm, kw)


def patch_params(**kw) -> Params:
    """The paper's 2 x 2 patch geometry (B 2, ring 2); keyword overrides."""
    prm = Params()
    lib.skm_patch_params(ctypes.byref(prm))
    return _override(prm, kw)


def _override(prm: Params, kw: dict) -> Params:
    profile = kw.pop("profile", None)
    if profile is not None:
        tphi, tnu = {"express": (20.0, 0.01), "efficient": (20.0, 0.1),
                     "excellent": (20.0, 100.0)}[profile]
        prm.t_phi, prm.t_nu = tphi, tnu
    for k, v in kw.items():
        if k == "mode" and isinstance(v, str):
            v = MODES[v]
        if not hasattr(prm, k):
            raise KeyError(k)
        setattr(prm, k, v)
    return prm


class Context:
    """Owns an ``skm_ctx`` on one HIP device."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib.skm_create(int(device), ctypes.byref(h)))
        self._h = h
        self.device = int(device)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib.skm_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------- timing
    def profile_enable(self, on: bool = True):
        _check(lib.skm_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """(summed ms, launches) of the estimation kernel since the last read."""
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int32(0)
        _check(lib.skm_profile_read(self._h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    # ------------------------------------------------------------ options
    def set_option(self, option: int, value: int):
        _check(lib.skm_set_option(self._h, int(option), int(value)))

    def get_option(self, option: int) -> int:
        v = ctypes.c_int64(0)
        _check(lib.skm_get_option(self._h, int(option), ctypes.byref(v)))
        return v.value

    # -------------------------------------------------------------- batch
    @staticmethod
    def _frame_descs(jobs):
        """jobs: sequence of (frame, mask, out, params[, info, xhat, cap])."""
        descs = (FrameDesc * len(jobs))()
        keep = []
        for k, job in enumerate(jobs):
            frame, mask, out, prm = job[:4]
            _dev_check(frame, mask)
            d = descs[k]
            d.frame, d.mask, d.out = frame.data_ptr(), mask.data_ptr(), out.data_ptr()
            d.height, d.width = frame.shape
            d.stride = frame.stride(0)
            d.params = ctypes.pointer(prm)
            keep.append(prm)
            if len(job) > 4:
                info, xhat, cap = job[4:7]
                d.info = info.data_ptr() if info is not None else None
                d.xhat = xhat.data_ptr() if xhat is not None else None
                d.cap = cap
        return descs, keep

    def conceal_batch(self, jobs, stream=None):
        """Conceal several device frames; jobs as in _frame_descs.  Returns
        the list of (n_lost, rounds, status) per frame; raises on the first
        error."""
        import torch
        descs, keep = self._frame_descs(jobs)
        dev = jobs[0][0].device if jobs else None
        s = (torch.cuda.current_stream(dev) if stream is None else stream) if jobs else None
        st = lib.skm_conceal_batch(self._h, descs, len(jobs),
                                   ctypes.c_void_p(s.cuda_stream) if s is not None else None)
        res = [(d.n_lost, d.rounds, d.status) for d in descs]
        _check(st)
        del keep
        return res

    def autotune(self, jobs, reps: int = 3) -> float:
        """Pick the fastest launch configuration for these frames; returns the
        best batch time in ms."""
        descs, keep = self._frame_descs(jobs)
        ms = ctypes.c_double(0.0)
        _check(lib.skm_autotune(self._h, descs, len(jobs), int(reps), ctypes.byref(ms)))
        del keep
        return ms.value

    def autotune_save(self, path: str):
        """Write the launch options and per-geometry tile table as JSON."""
        _check(lib.skm_autotune_save(self._h, os.fsencode(path)))

    def autotune_load(self, path: str):
        """Read a tuning file written by autotune_save."""
        _check(lib.skm_autotune_load(self._h, os.fsencode(path)))

    # ------------------------------------------------------- learned gate
    def cnn_init(self, seed: int = 0):
        _check(lib.skm_cnn_init(self._h, int(seed)))

    def cnn_set_weights(self, w):
        w = np.ascontiguousarray(w, dtype=np.float32)
        _check(lib.skm_cnn_set_weights(self._h, w.ctypes.data, int(w.size)))

    def cnn_get_weights(self) -> np.ndarray:
        w = np.empty(CNN_PARAMS, dtype=np.float32)
        _check(lib.skm_cnn_get_weights(self._h, w.ctypes.data, CNN_PARAMS))
        return w

    def cnn_set_thresholds(self, tau1: float, tau2: float):
        _check(lib.skm_cnn_set_thresholds(self._h, float(tau1), float(tau2)))

    def cnn_save(self, path: str):
        _check(lib.skm_save_cnn(self._h, os.fsencode(path)))

    def cnn_load(self, path: str):
        _check(lib.skm_load_cnn(self._h, os.fsencode(path)))

    def cnn_inputs(self, frame, mask, params: Params, stream=None):
        """bf16 bit patterns (int16 tensor) [n_lost, 8, 24, 24] of every lost block
        (the 48 x 48 two-channel window, space to depth)."""
        import torch
        _dev_check(frame, mask)
        h, w = frame.shape
        cap = max((h // params.block) * (w // params.block), 1)
        out = torch.empty((cap, 8, 24, 24), dtype=torch.int16, device=frame.device)
        n = ctypes.c_int32(0)
        s = torch.cuda.current_stream(frame.device) if stream is None else stream
        _check(lib.skm_cnn_inputs(self._h, frame.data_ptr(), mask.data_ptr(), w, h,
                                  frame.stride(0), ctypes.byref(params), out.data_ptr(), cap,
                                  ctypes.byref(n), ctypes.c_void_p(s.cuda_stream)))
        return out[:n.value]

    def cnn_forward(self, x, stream=None):
        import torch
        x = x.contiguous()
        out = torch.empty((x.shape[0], 2), dtype=torch.float32, device=x.device)
        s = torch.cuda.current_stream(x.device) if stream is None else stream
        _check(lib.skm_cnn_forward(self._h, x.data_ptr(), int(x.shape[0]), out.data_ptr(),
                                   ctypes.c_void_p(s.cuda_stream)))
        return out

    def cnn_gradients(self, x, t, stream=None):
        import torch
        x, t = x.contiguous(), t.contiguous().float()
        g = np.empty(CNN_PARAMS, dtype=np.float32)
        loss = ctypes.c_float(0.0)
        s = torch.cuda.current_stream(x.device) if stream is None else stream
        _check(lib.skm_cnn_gradients(self._h, x.data_ptr(), t.data_ptr(), int(x.shape[0]),
                                     g.ctypes.data, ctypes.byref(loss),
                                     ctypes.c_void_p(s.cuda_stream)))
        return loss.value, g

    def cnn_train_step(self, x, t, lr: float, want_loss=True, stream=None):
        import torch
        loss = ctypes.c_float(float("nan"))
        s = torch.cuda.current_stream(x.device) if stream is None else stream
        _check(lib.skm_cnn_train_step(self._h, x.data_ptr(), t.data_ptr(), int(x.shape[0]),
                                      float(lr), ctypes.byref(loss) if want_loss else None,
                                      ctypes.c_void_p(s.cuda_stream)))
        return loss.value

    def cnn_last_predictions(self, cap: int) -> np.ndarray:
        out = np.empty((max(cap, 1), 2), dtype=np.float32)
        _check(lib.skm_cnn_last_predictions(self._h, out.ctypes.data, int(max(cap, 1))))
        return out[:cap]

    # ---------------------------------------------------------------- host
    def conceal(self, frame: np.ndarray, mask: np.ndarray, params: Params,
                want_info: bool = True):
        """Host entry point; returns (out uint8, info structured array)."""
        frame = np.ascontiguousarray(frame, dtype=np.uint8)
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if frame.ndim != 2 or frame.shape != mask.shape:
            raise ValueError("frame and mask must be 2-D of the same shape")
        h, w = frame.shape
        out = np.empty_like(frame)
        cap = (h // params.block) * (w // params.block)
        info = np.zeros(max(cap, 1), dtype=BLOCK_INFO_DTYPE) if want_info else None
        n = ctypes.c_int32(0)
        _check(lib.skm_conceal(self._h, frame.ctypes.data, mask.ctypes.data, w, h, w,
                               ctypes.byref(params), out.ctypes.data,
                               info.ctypes.data if want_info else None, cap,
                               ctypes.byref(n)))
        return out, (info[:n.value] if want_info else None)

    # -------------------------------------------------------------- device
    def conceal_device(self, frame, mask, params: Params, out=None, want_info=True,
                       want_xhat=True, stream=None):
        """Device entry point on torch uint8 CUDA tensors (H, W).

        Returns (out tensor, info structured array or None, xhat float32
        tensor (n_lost, B, B) or None).
        """
        return self._conceal_device(lib.skm_conceal_device, frame, mask, params, out,
                                    want_info, want_xhat, stream)

    def conceal_device_noalloc(self, frame, mask, params: Params, out=None, want_info=True,
                               want_xhat=True, stream=None):
        """skm_conceal_device_noalloc: as conceal_device, with the library's
        workspace taken from its fixed per-GPU array (no device allocation by
        the library; the output tensors here are the caller's)."""
        return self._conceal_device(lib.skm_conceal_device_noalloc, frame, mask, params, out,
                                    want_info, want_xhat, stream)

    def _conceal_device(self, entry, frame, mask, params, out, want_info, want_xhat, stream):
        import torch
        _dev_check(frame, mask)
        h, w = frame.shape
        if out is None:
            out = torch.empty_like(frame)
        b = params.block
        cap = (h // b) * (w // b)
        dinfo = (torch.zeros(max(cap, 1) * BLOCK_INFO_DTYPE.itemsize, dtype=torch.uint8,
                             device=frame.device) if want_info else None)
        dx = (torch.zeros((max(cap, 1), b, b), dtype=torch.float32, device=frame.device)
              if want_xhat else None)
        n = ctypes.c_int32(0)
        s = torch.cuda.current_stream(frame.device) if stream is None else stream
        _check(entry(
            self._h, frame.data_ptr(), mask.data_ptr(), w, h, frame.stride(0),
            ctypes.byref(params), out.data_ptr(),
            dinfo.data_ptr() if dinfo is not None else None,
            dx.data_ptr() if dx is not None else None, cap, ctypes.byref(n),
            ctypes.c_void_p(s.cuda_stream)))
        info = None
        if dinfo is not None:
            info = dinfo.cpu().numpy().view(BLOCK_INFO_DTYPE)[:n.value].copy()
        return out, info, (dx[:n.value] if dx is not None else None)

    def distances_device(self, frame, mask, params: Params, stream=None):
        """Exact distance table: (d, n) int32 tensors (n_lost, 2W+1, 2W+1)."""
        import torch
        _dev_check(frame, mask)
        h, w = frame.shape
        b, W = params.block, params.window
        cap = max((h // b) * (w // b), 1)
        D = 2 * W + 1
        d = torch.empty((cap, D, D), dtype=torch.int32, device=frame.device)
        c = torch.empty((cap, D, D), dtype=torch.int32, device=frame.device)
        n = ctypes.c_int32(0)
        s = torch.cuda.current_stream(frame.device) if stream is None else stream
        _check(lib.skm_distances_device(
            self._h, frame.data_ptr(), mask.data_ptr(), w, h, frame.stride(0),
            ctypes.byref(params), d.data_ptr(), c.data_ptr(), cap, ctypes.byref(n),
            ctypes.c_void_p(s.cuda_stream)))
        return d[:n.value], c[:n.value]


def _dev_check(frame, mask):
    import torch
    for t in (frame, mask):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.uint8
                and t.dim() == 2 and t.stride(1) == 1):
            raise ValueError("frame and mask must be 2-D row-contiguous uint8 CUDA tensors")
    if frame.shape != mask.shape or frame.stride(0) != mask.stride(0):
        raise ValueError("frame and mask must have the same shape and stride")
