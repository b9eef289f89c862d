"""Run a workload through libzoomhash on one GPU.

Inputs come from the seeded generator in `synthdata` (images and sampling
positions only); every step of the method runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import zoomhash as zb


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libzoomhash needs a GPU (torch.cuda.is_available() is False)")
    return torch


class GpuWorkload:
    """Dictionary, tables and test image of one workload resident on the GPU."""

    def __init__(self, wl, ctx: zb.Context | None = None, device: int = 0, proj: int = 1):
        torch = _torch()
        self.torch = torch
        self.wl = wl
        self.dev = torch.device("cuda", device)
        self.ctx = ctx or zb.Context(device)
        s = wl.scale
        hr = torch.from_numpy(wl.dictionary_images()).to(self.dev)
        pos = torch.from_numpy(wl.positions().astype(np.int32)).to(self.dev)
        n = pos.shape[0]
        self.D = wl.D
        self.ps2 = (5 * s) ** 2
        self.feat = torch.empty((n, self.D), dtype=torch.float32, device=self.dev)
        self.resid = torch.empty((n, self.ps2), dtype=torch.float32, device=self.dev)
        self.ctx.make_dictionary(hr, hr.shape[0], hr.shape[1], hr.shape[2], pos, n, s,
                                 wl.blur_sigma, wl.feat_mode, self.feat, self.resid)
        del hr
        self._cap = wl.cap
        self.ctx.set_query_opts(cap=wl.cap, rerank=0, proj=proj, lle_fp64=1)
        self.ctx.build_tables(self.feat, self.resid, n, self.D, s, wl.feat_mode, wl.L, wl.k,
                              wl.w, wl.hash_seed)
        self.n = n
        if wl.test_h == 0:        # dictionary only
            self.hr_gt = self.lr = self.hr_out = None
            return
        img = torch.from_numpy(wl.test_image()).to(self.dev)
        if wl.test_lr_direct:
            self.hr_gt = None
            self.lr = img.contiguous()
        else:
            self.hr_gt = img
            h = (img.shape[0] + s - 1) // s
            w = (img.shape[1] + s - 1) // s
            self.lr = torch.empty((h, w), dtype=torch.float32, device=self.dev)
            self.ctx.degrade(img, 1, img.shape[0], img.shape[1], s, wl.blur_sigma, self.lr)
        self.h, self.w = self.lr.shape
        self.Q = (self.h - 4) * (self.w - 4)
        self.hr_out = torch.empty((s * self.h, s * self.w), dtype=torch.float32, device=self.dev)

    def set_mode(self, cap=None, rerank=0, proj=1, lle_fp64=1):
        self._cap = self.wl.cap if cap is None else cap
        self.ctx.set_query_opts(cap=self._cap, rerank=rerank, proj=proj, lle_fp64=lle_fp64)

    def zoom(self, lr=None, K=None, lam=None, out=None, metric="l2"):
        """hash + K-NN + LLE + blend for the test image; returns the HR image.
        metric "l1": neighbours re-ranked under l1 after the l2 query
        (zh_knn_l1); "l1q": the query itself ranks under l1
        (zh_set_query_metric), the same neighbours without the l2 ranking
        (both need the early stop); "t=<t>": neighbours among the t-of-L
        candidates."""
        wl = self.wl
        lr = self.lr if lr is None else lr
        out = self.hr_out if out is None else out
        if metric == "l1q":
            self.ctx.set_query_metric("l1")
        try:
            self.ctx.query(lr, lr.shape[0], lr.shape[1], wl.scale, wl.K if K is None else K)
        finally:
            if metric == "l1q":
                self.ctx.set_query_metric("l2")
        if metric == "l1":
            self.ctx.knn_l1()
        elif metric.startswith("t="):
            self.ctx.knn_t(int(metric[2:]))
        self.ctx.lle_weights(wl.lam if lam is None else lam)
        self.ctx.reconstruct(out)
        return out

    token = 0

    def forward_record(self, lr, lam, K=None, iters=None, out=None):
        """Query, weights, reconstruction and back-projection of `lr` into a
        new image (or `out`), recorded for zh_backward."""
        wl = self.wl
        s = wl.scale
        out = self.torch.empty((s * lr.shape[0], s * lr.shape[1]), dtype=self.torch.float32,
                               device=self.dev) if out is None else out
        self.ctx.query(lr, lr.shape[0], lr.shape[1], s, wl.K if K is None else K)
        self.ctx.lle_weights(lam)
        self.ctx.reconstruct(out)
        self.ctx.backproject(out, wl.bp_iters if iters is None else iters, wl.sigma_s, wl.sigma_r)
        self.token += 1
        return out

    def backproject(self, hr, iters=None):
        wl = self.wl
        self.ctx.backproject(hr, wl.bp_iters if iters is None else iters, wl.sigma_s, wl.sigma_r)
        return hr

    def results(self, K=None):
        torch = self.torch
        K = self.wl.K if K is None else K
        Q, _ = self.ctx.query_shape()
        ids = torch.empty((Q, K), dtype=torch.int32, device=self.dev)
        d2 = torch.empty((Q, K), dtype=torch.float32, device=self.dev)
        m = torch.empty(Q, dtype=torch.int32, device=self.dev)
        w = torch.empty((Q, K), dtype=torch.float32, device=self.dev)
        nc = torch.empty(Q, dtype=torch.int32, device=self.dev)
        self.ctx.get_results(ids, d2, m, w, nc)
        out = {}
        if self.ctx_cap() > 0:
            sv = torch.empty(Q, dtype=torch.int32, device=self.dev)
            self.ctx.survivors(sv)
            out["nsurv"] = sv
        self.ctx.sync()
        out = {k: v.cpu().numpy() for k, v in out.items()}
        out.update({"ids": ids.cpu().numpy(), "d2": d2.cpu().numpy(), "m": m.cpu().numpy(),
                    "w": w.cpu().numpy(), "ncand": nc.cpu().numpy()})
        return out

    def ctx_cap(self):
        return self._cap
