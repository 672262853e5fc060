"""One optimisation step of the per-Gaussian parameters, assembled from the
library's calls (argument marshalling and buffer ownership only; every step
runs in the HIP kernels behind include/legs.h).

  render   project -> bin/sort -> blend forward of every view (Sec. 3.1 Eq. 1,
           with R_s and R_u of Sec. 3.4); the forward launch also zeroes the
           gradient buffers (legs_render_forward_zero)
  loss     per view, mean |out - target| over RGB and s_G plus lambda_u times
           the mean rendered uncertainty (the L_u regulariser of Eq. 11),
           and dL/d(out) (legs_l1_loss_grad)
  backward blend backward from (T_final, last), projection backward
           (legs_render_backward, legs_project_backward)
  update   one fused Adam launch over means, log-scales, quaternions, opacity
           logits and channels, the uncertainty clamped to [0, 1] (Sec. 4:
           Adam, lr 1e-3, betas (0.9, 0.999); u in [0, 1] of Sec. 3.4.2)

Every call is capturable, so the whole step can be recorded once as a HIP
graph (capture()) and replayed. A captured step keeps the Adam step number of
its capture (the bias correction); eager steps advance it.
"""
from __future__ import annotations

import ctypes as ct

import torch

from . import _lib as L
from . import raster as R
from .decode import adam as _adam, l1_loss_grad as _l1

GROUPS = ("mean", "log_scale", "quat", "opacity_logit", "channels")


class TrainStep:
    def __init__(self, cams, params: dict, target, d_sem: int, o: L.Opts | None = None,
                 lambda_u: float = 1.0, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8,
                 capacity_slack: float = 1.15):
        self.rast = R.Rasterizer(cams, o if o is not None else R.opts())
        ctx, views, o = self.rast.ctx, self.rast.views, self.rast.o
        for k in GROUPS:
            t = params[k]
            assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous(), k
        self.p = params
        n, C = params["channels"].shape
        self.n, self.C, self.n_fit = int(n), int(C), 3 + int(d_sem)
        assert self.n_fit < self.C, "the last channel is the uncertainty u"
        self.lambda_u, self.lr, self.betas, self.eps = lambda_u, lr, betas, eps
        dev = params["mean"].device
        self.target = target
        self.proj = R.project(ctx, params["mean"], params["log_scale"], params["quat"],
                              params["opacity_logit"], views, o)
        sized = R.bin_sort(ctx, self.proj, views, o)
        self.bins = R.BinsBuf(int(sized.n_instances * capacity_slack) + 4096, views.total_tiles, dev)
        del sized
        px = views.total_pixels
        self.out = torch.empty(C * px, dtype=torch.float32, device=dev)
        self.T = torch.empty(px, dtype=torch.float32, device=dev)
        self.last = torch.empty(px, dtype=torch.int32, device=dev)
        self.d_out = torch.empty(C * px, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        G = n * views.n_views
        # gradients: one allocation (zeroed once per step by the forward launch)
        sizes = {"grad2d": 8 * G, "channels": n * C, "mean": 3 * n, "log_scale": 3 * n, "quat": 4 * n,
                 "opacity_logit": n}
        self.gflat = torch.zeros(sum(sizes.values()), dtype=torch.float32, device=dev)
        self.g, at = {}, 0
        for k, sz in sizes.items():
            self.g[k] = self.gflat[at:at + sz]
            at += sz
        self.g["grad2d"] = self.g["grad2d"].view(G, 8)
        self.g["channels"] = self.g["channels"].view(n, C)
        for k in ("mean", "log_scale", "quat", "opacity_logit"):
            self.g[k] = self.g[k].view(params[k].shape)
        self.m = {k: torch.zeros_like(params[k]) for k in GROUPS}
        self.v = {k: torch.zeros_like(params[k]) for k in GROUPS}
        self.step_count = 0
        self.graph = None

    def _groups(self):
        gr = []
        for k in GROUPS:
            d = dict(param=self.p[k], grad=self.g[k], m=self.m[k], v=self.v[k])
            if k == "channels":
                d["clamp"] = (self.C, self.C - 1, 0.0, 1.0)     # u in [0, 1]
            gr.append(d)
        return gr

    def enqueue(self, step_number: int):
        ctx, views, o, p = self.rast.ctx, self.rast.views, self.rast.o, self.p
        R.project(ctx, p["mean"], p["log_scale"], p["quat"], p["opacity_logit"], views, o, out=self.proj)
        R.bin_sort(ctx, self.proj, views, o, self.bins, sync_count=False)
        # the forward launch also zeroes the gradients the backward accumulates into
        R.render_forward(ctx, self.proj, self.bins, views, p["channels"], o, self.out, self.T, self.last,
                         zero=self.gflat)
        _l1(ctx, self.out, self.target, views, self.C, self.n_fit, self.lambda_u, self.d_out, self.loss)
        R.render_backward(ctx, self.proj, self.bins, views, p["channels"], o, self.T, self.last, self.d_out,
                          self.g["grad2d"], self.g["channels"])
        R.project_backward(ctx, p["mean"], p["log_scale"], p["quat"], p["opacity_logit"], views, o, self.proj,
                           self.g["grad2d"], {k: self.g[k] for k in ("mean", "log_scale", "quat", "opacity_logit")})
        _adam(ctx, self._groups(), step_number, lr=self.lr, betas=self.betas, eps=self.eps)

    def step(self):
        """One eager step (advances the Adam step number)."""
        self.step_count += 1
        self.enqueue(self.step_count)
        return self.loss

    def overflowed(self) -> bool:
        return int(self.bins.count.item()) > self.bins.capacity

    def capture(self, step_number: int = 1):
        """Record one step as a HIP graph (on a side stream) and return it."""
        g = R.Graph(self.rast.ctx)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            with g.capture():
                self.enqueue(step_number)
        torch.cuda.current_stream().wait_stream(side)
        self.graph = g
        return g
