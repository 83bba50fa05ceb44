"""ctypes binding of the warm-start MLP entry points of ``libhrelax.so``
(``hr_mlp_*``, ``hr_warm_start``); every network step runs in the library's
HIP kernels, torch only owns the device buffers."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _check, _dp, load_library

_fp = ctypes.POINTER(ctypes.c_float)

N_FEAT = 15

_SIG = {
    "hr_mlp_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_ulonglong, ctypes.POINTER(ctypes.c_void_p)]),
    "hr_mlp_param_count": (ctypes.c_size_t, [ctypes.c_void_p]),
    "hr_mlp_workspace_bytes": (ctypes.c_size_t, [ctypes.c_void_p, ctypes.c_int]),
    "hr_mlp_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                   ctypes.c_void_p]),
    "hr_mlp_destroy": (None, [ctypes.c_void_p]),
    "hr_mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, _fp, ctypes.c_size_t]),
    "hr_mlp_set_params": (ctypes.c_int, [ctypes.c_void_p, _fp, ctypes.c_size_t]),
    "hr_mlp_set_output_map": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_float, ctypes.c_float]),
    "hr_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, _fp, ctypes.c_int, _fp]),
    "hr_mlp_gradients": (ctypes.c_int, [ctypes.c_void_p, _fp, _fp, ctypes.c_int, _fp, _fp]),
    "hr_mlp_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int, ctypes.c_float, _fp]),
    "hr_mlp_grid_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _dp, ctypes.c_void_p]),
    "hr_warm_start": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, _dp, ctypes.c_double]),
}


def _lib():
    L = load_library()
    if not getattr(L, "_mlp_sigs", False):
        for name, (res, args) in _SIG.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        L._mlp_sigs = True
    return L


def config_features(q: float, chi1, chi2, P: float, D: float) -> np.ndarray:
    """The 9 configuration inputs, scaled to O(1): (q - 5.5)/4.5, chi1 (3), chi2 (3),
    10 |P|, (D - 13)/7."""
    chi1 = np.asarray(chi1, dtype=np.float64).reshape(3)
    chi2 = np.asarray(chi2, dtype=np.float64).reshape(3)
    return np.concatenate([[(q - 5.5) / 4.5], chi1, chi2, [10.0 * P, (D - 13.0) / 7.0]])


class MLP:
    def __init__(self, width: int = 256, seed: int = 0, max_batch: int = 65536, device=None):
        import torch

        L = _lib()
        h = ctypes.c_void_p()
        _check(L.hr_mlp_create(int(width), int(seed), ctypes.byref(h)), "hr_mlp_create")
        self._h = h
        self.width = width
        self.max_batch = max_batch
        self.n_params = L.hr_mlp_param_count(h)
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = L.hr_mlp_workspace_bytes(h, int(max_batch))
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (self._ws.data_ptr() + 255) // 256 * 256
        self.stream = torch.cuda.Stream(device=dev)
        self.device = dev
        with torch.cuda.device(dev):
            _check(L.hr_mlp_bind(h, ctypes.c_void_p(aligned), nbytes, int(max_batch),
                                 ctypes.c_void_p(self.stream.cuda_stream)), "hr_mlp_bind")

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib().hr_mlp_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(_lib().hr_mlp_get_params(self._h, out.ctypes.data_as(_fp), out.size), "hr_mlp_get_params")
        return out

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        _check(_lib().hr_mlp_set_params(self._h, p.ctypes.data_as(_fp), p.size), "hr_mlp_set_params")

    def set_output_map(self, scale: float, shift: float) -> None:
        self.out_scale, self.out_shift = float(scale), float(shift)
        _check(_lib().hr_mlp_set_output_map(self._h, float(scale), float(shift)), "hr_mlp_set_output_map")

    def forward(self, x) -> np.ndarray:
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
        y = np.zeros(len(x), dtype=np.float32)
        _check(_lib().hr_mlp_forward(self._h, x.ctypes.data_as(_fp), len(x), y.ctypes.data_as(_fp)),
               "hr_mlp_forward")
        return y

    def gradients(self, x, t):
        x = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
        t = np.ascontiguousarray(np.asarray(t, dtype=np.float32))
        g = np.zeros(self.n_params, dtype=np.float32)
        loss = ctypes.c_float()
        _check(_lib().hr_mlp_gradients(self._h, x.ctypes.data_as(_fp), t.ctypes.data_as(_fp),
                                       len(x), g.ctypes.data_as(_fp), ctypes.byref(loss)),
               "hr_mlp_gradients")
        return float(loss.value), g

    def train_step(self, x_dev, t_dev, lr: float) -> float:
        """x_dev (B x 15) and t_dev (B) are contiguous float32 torch tensors on the device.

        The library copies them on the network's stream; that stream first waits
        for the work already queued on torch's current stream (where the caller
        produced the batch), so the copy never reads a half-written batch."""
        import torch

        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        loss = ctypes.c_float()
        _check(_lib().hr_mlp_train_step(self._h, ctypes.c_void_p(x_dev.data_ptr()),
                                        ctypes.c_void_p(t_dev.data_ptr()), int(x_dev.shape[0]),
                                        float(lr), ctypes.byref(loss)), "hr_mlp_train_step")
        return float(loss.value)

    def grid_features(self, grid, cfg9):
        import torch

        cfg9 = np.ascontiguousarray(np.asarray(cfg9, dtype=np.float64))
        out = torch.empty((grid.n_extended, N_FEAT), dtype=torch.float32, device=self.device)
        # `out` comes from torch's allocator on the current stream and the library
        # writes it on the grid's stream: order that write after the current
        # stream's pending work (an earlier reader of the same memory).
        grid.stream.wait_stream(torch.cuda.current_stream(self.device))
        _check(_lib().hr_mlp_grid_features(self._h, grid.handle, cfg9.ctypes.data_as(_dp),
                                           ctypes.c_void_p(out.data_ptr())), "hr_mlp_grid_features")
        return out

    def warm_start(self, grid, cfg9, eta: float) -> None:
        cfg9 = np.ascontiguousarray(np.asarray(cfg9, dtype=np.float64))
        _check(_lib().hr_warm_start(grid.handle, self._h, cfg9.ctypes.data_as(_dp), float(eta)),
               "hr_warm_start")
