"""Python face of the splatting calls of liblegs.so (same names as the C ABI
without the `legs_` prefix) plus a torch.autograd.Function.

PyTorch only provides device memory and the current stream here; every step
of projection, binning, sorting, blending and their backward runs in the HIP
kernels behind include/legs.h.
"""
from __future__ import annotations

import ctypes as ct
import dataclasses

import torch

from . import _lib as L


def _p(t):
    return ct.c_void_p(t.data_ptr()) if t is not None else ct.c_void_p(0)


def _stream(device=None):
    return ct.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def opts(tile=16, lds_batch=256, alpha_max=0.99, alpha_min=1.0 / 255.0, t_min=1e-4,
         lowpass=0.3, z_near=0.2, guard=1.3, persistent=False, full_sort=False, full_box=False,
         ids_only=False) -> L.Opts:
    o = L.Opts()
    L.lib().legs_opts_default(ct.byref(o))
    o.tile, o.lds_batch = int(tile), int(lds_batch)
    o.flags = ((L.LEGS_FLAG_PERSISTENT if persistent else 0) | (L.LEGS_FLAG_FULL_SORT if full_sort else 0)
               | (L.LEGS_FLAG_FULL_BOX if full_box else 0) | (L.LEGS_FLAG_IDS_ONLY if ids_only else 0))
    o.alpha_max, o.alpha_min, o.t_min = alpha_max, alpha_min, t_min
    o.lowpass, o.z_near, o.guard = lowpass, z_near, guard
    return o


class Context:
    """A library context bound to one GPU (legs_create / legs_destroy)."""

    def __init__(self, device: int = 0):
        h = ct.c_void_p()
        code = L.lib().legs_create(int(device), ct.byref(h))
        if code != L.LEGS_OK:
            raise L.LegsError(code, f"legs_create({device}) failed")
        self.handle = h
        self.device = torch.device("cuda", int(device))

    def check(self, code):
        return L.check(self.handle, code)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                L.lib().legs_destroy(h)
            except Exception:
                pass
            self.handle = None


@dataclasses.dataclass
class Views:
    host: object            # ctypes array of L.View
    dev: torch.Tensor       # the same bytes in device memory
    n_views: int
    total_tiles: int
    total_pixels: int
    sizes: list             # [(W, H)] per view
    pixel_offsets: list
    tile: int


def to_camera(c) -> L.Camera:
    W, H, fx, fy, cx, cy, R, t = c.as_tuple()
    return L.Camera(W, H, fx, fy, cx, cy, (ct.c_double * 9)(*R), (ct.c_double * 3)(*t))


def views_build(cams, o: L.Opts, device) -> Views:
    n = len(cams)
    carr = (L.Camera * n)(*[to_camera(c) for c in cams])
    varr = (L.View * n)()
    tt, tp = ct.c_int64(), ct.c_int64()
    code = L.lib().legs_views_build(carr, n, ct.byref(o), varr, ct.byref(tt), ct.byref(tp))
    if code != L.LEGS_OK:
        raise L.LegsError(code, "legs_views_build: invalid cameras")
    raw = bytes(ct.string_at(ct.addressof(varr), ct.sizeof(varr)))
    dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(device)
    return Views(varr, dev, n, int(tt.value), int(tp.value),
                 [(varr[i].cam.width, varr[i].cam.height) for i in range(n)],
                 [int(varr[i].pixel_offset) for i in range(n)], int(o.tile))


class ProjectedBuf:
    def __init__(self, n, n_views, device):
        G = max(n * n_views, 1)       # never a NULL device pointer, even when empty
        nb = int(L.lib().legs_projected_blocks(n, n_views))
        self.n, self.n_views = n, n_views
        self.mean2d = torch.empty((G, 2), dtype=torch.float64, device=device)
        self.conic = torch.empty((G, 4), dtype=torch.float32, device=device)
        self.box = torch.empty((G, 4), dtype=torch.int32, device=device)
        self.depth = torch.empty(G, dtype=torch.float32, device=device)
        self.ntiles = torch.empty(G, dtype=torch.int32, device=device)
        self.block_offsets = torch.empty(2 * (nb + 1), dtype=torch.int64, device=device)
        ob = int(L.lib().legs_order_scratch_bytes(n, n_views))
        self.order = torch.empty(max(ob, 256), dtype=torch.uint8, device=device)

    def struct(self):
        return L.Projected(self.mean2d.data_ptr(), self.conic.data_ptr(), self.box.data_ptr(),
                           self.depth.data_ptr(), self.ntiles.data_ptr(),
                           self.block_offsets.data_ptr(), self.order.data_ptr())


class BinsBuf:
    def __init__(self, capacity, total_tiles, device):
        capacity = max(int(capacity), 1)
        self.capacity = capacity
        self.keys = torch.empty(capacity, dtype=torch.int64, device=device)
        self.keys_alt = torch.empty(capacity, dtype=torch.int64, device=device)
        self.ids = torch.empty(capacity, dtype=torch.int32, device=device)
        self.ids_alt = torch.empty(capacity, dtype=torch.int32, device=device)
        self.ranges = torch.empty((total_tiles, 2), dtype=torch.int32, device=device)
        nbytes = int(L.lib().legs_sort_scratch_bytes(capacity, total_tiles))
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.count = torch.zeros(1, dtype=torch.int64, device=device)
        self.n_instances = None

    def struct(self):
        return L.Bins(self.keys.data_ptr(), self.keys_alt.data_ptr(), self.ids.data_ptr(),
                      self.ids_alt.data_ptr(), self.ranges.data_ptr(), self.scratch.data_ptr(),
                      self.count.data_ptr(), self.capacity)


def project(ctx: Context, mean, log_scale, quat, opacity_logit, views: Views, o: L.Opts,
            out: ProjectedBuf | None = None) -> ProjectedBuf:
    n = int(mean.shape[0])
    for t in (mean, log_scale, quat, opacity_logit):
        assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    out = out or ProjectedBuf(n, views.n_views, mean.device)
    s = out.struct()
    ctx.check(L.lib().legs_project(ctx.handle, _p(mean), _p(log_scale), _p(quat),
                                   _p(opacity_logit), n, _p(views.dev), views.n_views,
                                   ct.byref(o), ct.byref(s), _stream()))
    return out


def bin_sort(ctx: Context, proj: ProjectedBuf, views: Views, o: L.Opts,
             bins: BinsBuf | None = None, sync_count: bool = True) -> BinsBuf:
    """Bin and sort. With sync_count the instance total is read back and the
    buffers grown (and the call repeated) if it exceeds their capacity."""
    device = proj.mean2d.device
    if bins is None:
        bins = BinsBuf(max(1 << 16, proj.n * views.n_views * 4), views.total_tiles, device)
    ps = proj.struct()
    while True:
        bs = bins.struct()
        cnt = ct.c_int64(0)
        code = L.lib().legs_bin_sort(ctx.handle, ct.byref(ps), proj.n, _p(views.dev),
                                     views.n_views, views.total_tiles, ct.byref(o), ct.byref(bs),
                                     ct.byref(cnt) if sync_count else None, _stream())
        if code == L.LEGS_ERR_CAPACITY and sync_count:
            bins = BinsBuf(int(cnt.value * 1.15) + 1024, views.total_tiles, device)
            continue
        ctx.check(code)
        if sync_count:
            bins.n_instances = int(cnt.value)
        return bins


def render_forward(ctx: Context, proj: ProjectedBuf, bins: BinsBuf, views: Views, channels,
                   o: L.Opts, out=None, T=None, last=None, zero=None):
    """legs_render_forward; with zero (a contiguous device tensor), the same
    launch also sets zero to 0 (legs_render_forward_zero)."""
    assert channels.is_cuda and channels.dtype == torch.float32 and channels.is_contiguous()
    n, C = channels.shape
    device = channels.device
    if out is None:
        out = torch.empty(C * views.total_pixels, dtype=torch.float32, device=device)
    if T is None:
        T = torch.empty(views.total_pixels, dtype=torch.float32, device=device)
    if last is None:
        last = torch.empty(views.total_pixels, dtype=torch.int32, device=device)
    ps, bs = proj.struct(), bins.struct()
    if zero is None:
        ctx.check(L.lib().legs_render_forward(ctx.handle, ct.byref(ps), n, ct.byref(bs), _p(views.dev),
                                              views.n_views, views.total_tiles, _p(channels), C,
                                              ct.byref(o), _p(out), _p(T), _p(last), _stream()))
    else:
        assert zero.is_cuda and zero.is_contiguous()
        ctx.check(L.lib().legs_render_forward_zero(ctx.handle, ct.byref(ps), n, ct.byref(bs), _p(views.dev),
                                                   views.n_views, views.total_tiles, _p(channels), C,
                                                   ct.byref(o), _p(out), _p(T), _p(last), _p(zero),
                                                   zero.numel() * zero.element_size(), _stream()))
    return out, T, last


def render_backward(ctx: Context, proj: ProjectedBuf, bins: BinsBuf, views: Views, channels,
                    o: L.Opts, T, last, d_out, grad2d=None, d_channels=None):
    n, C = channels.shape
    device = channels.device
    if grad2d is None:
        grad2d = torch.zeros((n * views.n_views, 8), dtype=torch.float32, device=device)
    if d_channels is None:
        d_channels = torch.zeros((n, C), dtype=torch.float32, device=device)
    d_out = d_out.contiguous()
    ps, bs = proj.struct(), bins.struct()
    ctx.check(L.lib().legs_render_backward(ctx.handle, ct.byref(ps), n, ct.byref(bs),
                                           _p(views.dev), views.n_views, views.total_tiles,
                                           _p(channels), C, ct.byref(o), _p(T), _p(last),
                                           _p(d_out), _p(grad2d), _p(d_channels), _stream()))
    return grad2d, d_channels


def clear(ctx: Context, t):
    """Zero a contiguous device tensor with the library's fill kernel."""
    assert t.is_cuda and t.is_contiguous()
    ctx.check(L.lib().legs_clear(ctx.handle, _p(t), t.numel() * t.element_size(), _stream()))
    return t


def render_counts(ctx: Context, proj: ProjectedBuf, bins: BinsBuf, views: Views, o: L.Opts):
    """(forward alpha evaluations, blended entries, backward alpha evaluations,
    list positions walked) for these lists."""
    counts = torch.zeros(4, dtype=torch.int64, device=proj.mean2d.device)
    ps, bs = proj.struct(), bins.struct()
    ctx.check(L.lib().legs_render_counts(ctx.handle, ct.byref(ps), proj.n, ct.byref(bs),
                                         _p(views.dev), views.n_views, views.total_tiles,
                                         ct.byref(o), _p(counts), _stream()))
    return [int(x) for x in counts.cpu()]


def project_backward(ctx: Context, mean, log_scale, quat, opacity_logit, views: Views, o: L.Opts,
                     proj: ProjectedBuf, grad2d, grads=None):
    n = int(mean.shape[0])
    if grads is None:
        grads = dict(mean=torch.zeros_like(mean), log_scale=torch.zeros_like(log_scale),
                     quat=torch.zeros_like(quat), opacity_logit=torch.zeros_like(opacity_logit))
    ps = proj.struct()
    ctx.check(L.lib().legs_project_backward(ctx.handle, _p(mean), _p(log_scale), _p(quat),
                                            _p(opacity_logit), n, _p(views.dev), views.n_views,
                                            ct.byref(o), ct.byref(ps), _p(grad2d),
                                            _p(grads["mean"]), _p(grads["log_scale"]),
                                            _p(grads["quat"]), _p(grads["opacity_logit"]),
                                            _stream()))
    return grads


class Rasterizer:
    """Holds a context, a view table and options.

    forward() reuses one set of bin buffers: its lists are overwritten by the
    next forward(). The autograd path (rasterize) instead takes a set of its
    own for every call and returns it to a pool when its backward has been
    enqueued, so several renders may be alive before any backward runs."""

    def __init__(self, cams, o: L.Opts | None = None, device: int = 0):
        self.ctx = Context(device)
        self.o = o if o is not None else opts()
        self.views = views_build(cams, self.o, self.ctx.device)
        self.bins = None
        self._pool = []

    def forward(self, mean, log_scale, quat, opacity_logit, channels):
        proj = project(self.ctx, mean, log_scale, quat, opacity_logit, self.views, self.o)
        self.bins = bin_sort(self.ctx, proj, self.views, self.o, self.bins)
        out, T, last = render_forward(self.ctx, proj, self.bins, self.views, channels, self.o)
        return proj, self.bins, out, T, last

    def forward_owned(self, mean, log_scale, quat, opacity_logit, channels):
        """Like forward(), with bin buffers that belong to the caller until
        it hands them back with release()."""
        proj = project(self.ctx, mean, log_scale, quat, opacity_logit, self.views, self.o)
        bins = bin_sort(self.ctx, proj, self.views, self.o, self._pool.pop() if self._pool else None)
        out, T, last = render_forward(self.ctx, proj, bins, self.views, channels, self.o)
        return proj, bins, out, T, last

    def release(self, bins):
        self._pool.append(bins)


class RasterizeFn(torch.autograd.Function):
    """out (planar, views concatenated), T_final = rasterize(...).
    Saves only the projected records, the tile lists, T_final and last; each
    call holds its own tile lists until its backward."""

    @staticmethod
    def forward(fctx, mean, log_scale, quat, opacity_logit, channels, rast: Rasterizer):
        proj, bins, out, T, last = rast.forward_owned(mean, log_scale, quat, opacity_logit, channels)
        fctx.rast, fctx.proj, fctx.bins = rast, proj, bins
        fctx.save_for_backward(mean, log_scale, quat, opacity_logit, channels, T, last)
        fctx.mark_non_differentiable(T)
        return out, T

    @staticmethod
    def backward(fctx, d_out, d_T):
        mean, log_scale, quat, opacity_logit, channels, T, last = fctx.saved_tensors
        r = fctx.rast
        grad2d, d_ch = render_backward(r.ctx, fctx.proj, fctx.bins, r.views, channels, r.o, T, last,
                                       d_out)
        g = project_backward(r.ctx, mean, log_scale, quat, opacity_logit, r.views, r.o, fctx.proj,
                             grad2d)
        # the lists are no longer read after the kernels enqueued above (same stream)
        r.release(fctx.bins)
        fctx.bins = None
        return g["mean"], g["log_scale"], g["quat"], g["opacity_logit"], d_ch, None


def rasterize(mean, log_scale, quat, opacity_logit, channels, rast: Rasterizer):
    return RasterizeFn.apply(mean, log_scale, quat, opacity_logit, channels, rast)


class Graph:
    """A captured HIP graph (legs_capture_begin / legs_capture_end). Use as

        g = Graph(ctx)
        with torch.cuda.stream(side_stream):
            with g.capture():
                ...  # calls of this module, with bin_sort(sync_count=False)
        g.launch()   # on the current stream
    """

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.handle = None

    class _Cap:
        def __init__(self, g):
            self.g = g

        def __enter__(self):
            self.g.ctx.check(L.lib().legs_capture_begin(self.g.ctx.handle, _stream()))
            return self.g

        def __exit__(self, et, ev, tb):
            h = ct.c_void_p()
            code = L.lib().legs_capture_end(self.g.ctx.handle, _stream(), ct.byref(h))
            if et is None:
                self.g.ctx.check(code)
                self.g.handle = h
            return False

    def capture(self):
        return Graph._Cap(self)

    def launch(self):
        self.ctx.check(L.lib().legs_graph_launch(self.ctx.handle, self.handle, _stream()))

    def __del__(self):
        if getattr(self, "handle", None):
            try:
                L.lib().legs_graph_destroy(self.handle)
            except Exception:
                pass
            self.handle = None


def autotune(ctx: Context, mean, log_scale, quat, opacity_logit, channels, cams, base: L.Opts,
             d_out=None, reps=3):
    """Returns (best options, {(tile, lds_batch): ms})."""
    n, C = channels.shape
    carr = (L.Camera * len(cams))(*[to_camera(c) for c in cams])
    best = L.Opts()
    table = (ct.c_float * 9)()
    ctx.check(L.lib().legs_autotune(ctx.handle, _p(mean), _p(log_scale), _p(quat),
                                    _p(opacity_logit), _p(channels), n, C, carr, len(cams),
                                    ct.byref(base), _p(d_out) if d_out is not None else None,
                                    reps, ct.byref(best), table, _stream()))
    times = {(t, b): float(table[3 * i + j]) for i, t in enumerate((8, 16, 32))
             for j, b in enumerate((64, 128, 256))}
    return best, times
