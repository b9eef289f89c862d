"""Thin ctypes binding of libzoomhash (include/zoomhash.h).

Functions keep the C names; arrays are passed as torch CUDA/HIP tensors (their
device pointers are handed to the library), host arrays as numpy arrays.
Nothing here computes any part of the zoom path: every step runs in the HIP
kernels of libzoomhash.so, and loading fails loudly when the library is
missing or no GPU is present.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libzoomhash.so")

ZH_OK, ZH_EINVAL, ZH_ESTATE, ZH_ENOMEM, ZH_EDEVICE, ZH_EUNSUPPORTED, ZH_EIO = range(7)
ZH_FEAT_MEANREM, ZH_FEAT_GRAD4 = 0, 1
STATUS_NAMES = {0: "ZH_OK", 1: "ZH_EINVAL", 2: "ZH_ESTATE", 3: "ZH_ENOMEM", 4: "ZH_EDEVICE",
                5: "ZH_EUNSUPPORTED", 6: "ZH_EIO"}


class ZHError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class zh_dictionary(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int32), ("scale", ctypes.c_int32),
                ("feat_mode", ctypes.c_int32), ("feat", ctypes.c_void_p),
                ("resid", ctypes.c_void_p)]


class zh_query_opts(ctypes.Structure):
    _fields_ = [("cap", ctypes.c_int32), ("rerank", ctypes.c_int32), ("proj", ctypes.c_int32),
                ("lle_fp64", ctypes.c_int32)]


class zh_stats_t(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_uint64), ("codes_fixed", ctypes.c_uint64),
                ("rank_fallbacks", ctypes.c_uint64), ("deferred", ctypes.c_uint64),
                ("streamed", ctypes.c_uint64), ("lle_fp64", ctypes.c_uint64),
                ("dict_bytes", ctypes.c_uint64), ("truncated", ctypes.c_uint64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class zh_batch(ctypes.Structure):
    _fields_ = [("n_images", ctypes.c_int32), ("lr", ctypes.POINTER(ctypes.c_void_p)),
                ("hr_out", ctypes.POINTER(ctypes.c_void_p)), ("h", ctypes.POINTER(ctypes.c_int32)),
                ("w", ctypes.POINTER(ctypes.c_int32)), ("scale", ctypes.POINTER(ctypes.c_int32)),
                ("K", ctypes.c_int32), ("lam", ctypes.c_double), ("bp_iters", ctypes.c_int32),
                ("sigma_s", ctypes.c_float), ("sigma_r", ctypes.c_float)]


class zh_batch_tuning(ctypes.Structure):
    _fields_ = [("bp_tile", ctypes.c_int32), ("bp_grid_per_cu", ctypes.c_int32), ("bp_ms", ctypes.c_float * 6),
                ("synth_rows", ctypes.c_int32), ("synth_ms", ctypes.c_float * 2), ("from_cache", ctypes.c_int32)]


_V, _I, _I64, _U64, _F = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_float
SIGNATURES = {
    "zh_create": [ctypes.POINTER(_V), _I, _V],
    "zh_destroy": [_V],
    "zh_set_stream": [_V, _V],
    "zh_sync": [_V],
    "zh_last_error": [_V],
    "zh_degrade": [_V, _V, _I, _I, _I, _I, _F, _V],
    "zh_make_dictionary": [_V, _V, _I, _I, _I, _V, _I64, _I, _F, _I, _V, _V],
    "zh_features": [_V, _V, _I, _I, _I, _V, _V],
    "zh_upsample": [_V, _V, _I, _I, _I, _V],
    "zh_make_dictionary_interp": [_V, _V, _I, _I, _I, _V, _I64, _I, _F, _I, _V, _V],
    "zh_backproject_lr": [_V, _V, _V, _I, _I, _I, _I, _F, _F],
    "zh_sample_crops": [_V, _V, _I, _I, _I, _V, _I, _I, _V, _V],
    "zh_table_entropy": [_V, _I, _V, _I],
    "zh_knn_l1": [_V],
    "zh_knn_t": [_V, _I],
    "zh_candidates_t": [_V, _I, _I, _V, _V],
    "zh_build_tables": [_V, ctypes.POINTER(zh_dictionary), _I, _I, _F, _U64],
    "zh_save_tables": [_V, _I, ctypes.c_char_p],
    "zh_load_tables": [_V, ctypes.POINTER(zh_dictionary), ctypes.c_char_p],
    "zh_get_hash_params": [_V, _I, _V, _V],
    "zh_hash": [_V, _I, _V, _I64, _V, _V],
    "zh_hash_noalloc": [_V, _I, _V, _I64, _V, _V],
    "zh_set_query_opts": [_V, ctypes.POINTER(zh_query_opts)],
    "zh_set_query_metric": [_V, _I],
    "zh_query": [_V, _V, _I, _I, _I, _I],
    "zh_lle_weights": [_V, ctypes.c_double],
    "zh_lle_all": [_V, ctypes.c_double, _V, _V],
    "zh_reconstruct": [_V, _V],
    "zh_backproject": [_V, _V, _I, _F, _F],
    "zh_backward": [_V, _V, _V, _V],
    "zh_run_batch": [_V, ctypes.POINTER(zh_batch)],
    "zh_tune_batch": [_V, ctypes.POINTER(zh_batch), ctypes.POINTER(zh_batch_tuning)],
    "zh_get_results": [_V, _V, _V, _V, _V, _V],
    "zh_survivors": [_V, _V],
    "zh_query_shape": [_V, ctypes.POINTER(_I64), ctypes.POINTER(ctypes.c_int32)],
    "zh_candidates": [_V, ctypes.c_int32, _V, _V],
    "zh_stats": [_V, ctypes.POINTER(zh_stats_t)],
    "zh_set_timing": [_V, _I],
    "zh_set_timing_stages": [_V, ctypes.c_uint32],
    "zh_get_timing": [_V, _V, _V],
}
STAGES = ["features", "hash", "search", "lle", "synth", "blend", "bp_error", "bp_update", "rotate", "probe"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libzoomhash.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with paper_1004_3980_amd/build.py")
        lib = ctypes.CDLL(path)
        for name, args in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = None if name == "zh_destroy" else (
                ctypes.c_char_p if name == "zh_last_error" else ctypes.c_int32)
        _lib = lib
    return _lib


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    if not t.is_cuda:
        raise ValueError("libzoomhash takes device tensors")
    if not t.is_contiguous():
        raise ValueError("libzoomhash takes contiguous tensors")
    return t.data_ptr()


class Context:
    """Owns one zh_ctx; raises ZHError on a nonzero status."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        st = self.lib.zh_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != ZH_OK:
            raise ZHError(st, "zh_create failed")
        self.h = h
        self.device = device
        self._keep = []

    def _chk(self, st):
        if st != ZH_OK:
            raise ZHError(st, self.lib.zh_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.zh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls with the C names (minus the zh_ prefix on the method) --
    def sync(self):
        self._chk(self.lib.zh_sync(self.h))

    def degrade(self, hr, n_img, H, W, scale, sigma, lr):
        self._chk(self.lib.zh_degrade(self.h, _ptr(hr), n_img, H, W, scale, sigma, _ptr(lr)))

    def make_dictionary(self, hr, n_img, H, W, pos, n, scale, sigma, feat_mode, feat, resid):
        self._chk(self.lib.zh_make_dictionary(self.h, _ptr(hr), n_img, H, W, _ptr(pos), n, scale,
                                              sigma, feat_mode, _ptr(feat), _ptr(resid)))

    def upsample(self, lr, h, w, scale, out):
        self._chk(self.lib.zh_upsample(self.h, _ptr(lr), h, w, scale, _ptr(out)))

    def make_dictionary_interp(self, hr, n_img, H, W, pos, n, scale, sigma, feat_mode, feat, resid):
        self._chk(self.lib.zh_make_dictionary_interp(self.h, _ptr(hr), n_img, H, W, _ptr(pos), n, scale, sigma,
                                                     feat_mode, _ptr(feat), _ptr(resid)))

    def backproject_lr(self, hr, lr, h, w, scale, iters, sigma_s, sigma_r):
        self._chk(self.lib.zh_backproject_lr(self.h, _ptr(hr), _ptr(lr), h, w, scale, iters, sigma_s, sigma_r))

    def sample_crops(self, imgs, n_img, H, W, draws, m, side, corners, crops=None):
        self._chk(self.lib.zh_sample_crops(self.h, _ptr(imgs), n_img, H, W, _ptr(draws), m, side,
                                           _ptr(corners), _ptr(crops) if crops is not None else None))

    def candidates_t(self, t, cap_per_query, counts, ids):
        self._chk(self.lib.zh_candidates_t(self.h, t, cap_per_query, _ptr(counts), _ptr(ids)))

    def knn_t(self, t):
        self._chk(self.lib.zh_knn_t(self.h, t))

    def knn_l1(self):
        self._chk(self.lib.zh_knn_l1(self.h))

    def table_entropy(self, scale, L):
        out = np.zeros(L, dtype=np.float64)
        self._chk(self.lib.zh_table_entropy(self.h, scale, out.ctypes.data_as(ctypes.c_void_p), L))
        return out

    def features(self, lr, h, w, feat_mode, feat, mu=None):
        self._chk(self.lib.zh_features(self.h, _ptr(lr), h, w, feat_mode, _ptr(feat), _ptr(mu)))

    def build_tables(self, feat, resid, n, dim, scale, feat_mode, L, k, w, seed):
        d = zh_dictionary(n, dim, scale, feat_mode, _ptr(feat), _ptr(resid))
        self._chk(self.lib.zh_build_tables(self.h, ctypes.byref(d), L, k, w, seed))
        self._keep = [t for t in self._keep if getattr(t, "_zh_scale", None) != scale]
        for t in (feat, resid):
            try:
                t._zh_scale = scale
            except AttributeError:
                pass
            self._keep.append(t)

    def save_tables(self, scale, path):
        self._chk(self.lib.zh_save_tables(self.h, scale, os.fsencode(path)))

    def load_tables(self, feat, resid, n, dim, scale, feat_mode, path):
        d = zh_dictionary(n, dim, scale, feat_mode, _ptr(feat), _ptr(resid))
        self._chk(self.lib.zh_load_tables(self.h, ctypes.byref(d), os.fsencode(path)))
        self._keep = [t for t in self._keep if getattr(t, "_zh_scale", None) != scale]
        for t in (feat, resid):
            try:
                t._zh_scale = scale
            except AttributeError:
                pass
            self._keep.append(t)

    def get_hash_params(self, scale, L, k, D):
        a = np.empty(L * k * D, dtype=np.float32)
        b = np.empty(L * k, dtype=np.float32)
        self._chk(self.lib.zh_get_hash_params(self.h, scale, a.ctypes.data, b.ctypes.data))
        return a.reshape(L * k, D), b

    def hash(self, scale, feat, n, codes=None, keys=None):
        self._chk(self.lib.zh_hash(self.h, scale, _ptr(feat), n, _ptr(codes), _ptr(keys)))

    def hash_noalloc(self, scale, feat, n, codes, keys):
        self._chk(self.lib.zh_hash_noalloc(self.h, scale, _ptr(feat), n, _ptr(codes), _ptr(keys)))

    def set_query_opts(self, cap=0, rerank=0, proj=1, lle_fp64=1):
        o = zh_query_opts(cap, rerank, proj, lle_fp64)
        self._chk(self.lib.zh_set_query_opts(self.h, ctypes.byref(o)))

    def set_query_metric(self, metric):
        """metric: "l2" or "l1" (the ranking of zh_query)."""
        self._chk(self.lib.zh_set_query_metric(self.h, {"l2": 0, "l1": 1}[metric]))

    def query(self, lr, h, w, scale, K):
        self._chk(self.lib.zh_query(self.h, _ptr(lr), h, w, scale, K))

    def lle_weights(self, lam):
        self._chk(self.lib.zh_lle_weights(self.h, lam))

    def lle_all(self, lam, ids=None, w=None):
        self._chk(self.lib.zh_lle_all(self.h, lam, _ptr(ids), _ptr(w)))

    def reconstruct(self, hr_out):
        self._chk(self.lib.zh_reconstruct(self.h, _ptr(hr_out)))

    def backproject(self, hr, iters, sigma_s, sigma_r):
        self._chk(self.lib.zh_backproject(self.h, _ptr(hr), iters, sigma_s, sigma_r))

    def backward(self, g_hr, g_resid, g_lambda):
        self._chk(self.lib.zh_backward(self.h, _ptr(g_hr), _ptr(g_resid), _ptr(g_lambda)))

    def _batch(self, lrs, outs, scales, K, lam, bp_iters, sigma_s, sigma_r):
        n = len(lrs)
        if not (n == len(outs) == len(scales)) or n == 0:
            raise ValueError("lrs, outs and scales must be non-empty and of one length")
        for t in list(lrs) + list(outs):
            _ptr(t)
        arrs = ((ctypes.c_void_p * n)(*[t.data_ptr() for t in lrs]),
                (ctypes.c_void_p * n)(*[t.data_ptr() for t in outs]),
                (ctypes.c_int32 * n)(*[t.shape[0] for t in lrs]),
                (ctypes.c_int32 * n)(*[t.shape[1] for t in lrs]),
                (ctypes.c_int32 * n)(*[int(s) for s in scales]))
        return arrs, zh_batch(n, *arrs, K, lam, bp_iters, sigma_s, sigma_r)

    def run_batch(self, lrs, outs, scales, K, lam, bp_iters, sigma_s, sigma_r):
        """Zoom many LR images (device tensors [h, w]) into outs ([s h, s w])."""
        keep, b = self._batch(lrs, outs, scales, K, lam, bp_iters, sigma_s, sigma_r)
        self._chk(self.lib.zh_run_batch(self.h, ctypes.byref(b)))

    def tune_batch(self, lrs, outs, scales, K, lam, bp_iters, sigma_s, sigma_r):
        keep, b = self._batch(lrs, outs, scales, K, lam, bp_iters, sigma_s, sigma_r)
        t = zh_batch_tuning()
        self._chk(self.lib.zh_tune_batch(self.h, ctypes.byref(b), ctypes.byref(t)))
        return {"bp_tile": t.bp_tile, "bp_grid_per_cu": t.bp_grid_per_cu, "bp_ms": list(t.bp_ms),
                "synth_rows": t.synth_rows, "synth_ms": list(t.synth_ms), "from_cache": t.from_cache}

    def get_results(self, ids=None, d2=None, m=None, w=None, ncand=None):
        self._chk(self.lib.zh_get_results(self.h, _ptr(ids), _ptr(d2), _ptr(m), _ptr(w), _ptr(ncand)))

    def survivors(self, out):
        self._chk(self.lib.zh_survivors(self.h, _ptr(out)))

    def query_shape(self):
        Q = ctypes.c_int64()
        D = ctypes.c_int32()
        self._chk(self.lib.zh_query_shape(self.h, ctypes.byref(Q), ctypes.byref(D)))
        return Q.value, D.value

    def candidates(self, cap_per_query, counts, ids):
        self._chk(self.lib.zh_candidates(self.h, cap_per_query, _ptr(counts), _ptr(ids)))

    def set_timing(self, on: bool, stages=None):
        """stages: names from STAGES to time (None: all)."""
        if stages is None:
            self._chk(self.lib.zh_set_timing(self.h, 1 if on else 0))
        else:
            mask = 0
            for n in stages:
                mask |= 1 << STAGES.index(n)
            self._chk(self.lib.zh_set_timing_stages(self.h, mask if on else 0))

    def get_timing(self):
        ms = np.zeros(len(STAGES), dtype=np.float64)
        n = np.zeros(len(STAGES), dtype=np.int32)
        self._chk(self.lib.zh_get_timing(self.h, ms.ctypes.data, n.ctypes.data))
        return {s: (float(ms[i]), int(n[i])) for i, s in enumerate(STAGES)}

    def stats(self):
        s = zh_stats_t()
        self._chk(self.lib.zh_stats(self.h, ctypes.byref(s)))
        return s.as_dict()
