"""Python face of the FP64 CPU oracle (test infrastructure only).

Loads oracle/liblegs_oracle.so (plain C, see legs_oracle.c) with ctypes and
exposes numpy-level calls. Nothing here touches the GPU or the product
library; the product path never imports this module.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liblegs_oracle.so")

ALPHA_MAX = 0.99
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4


class OCam(ct.Structure):
    _fields_ = [("W", ct.c_int32), ("H", ct.c_int32), ("fx", ct.c_double), ("fy", ct.c_double),
                ("cx", ct.c_double), ("cy", ct.c_double), ("R", ct.c_double * 9),
                ("t", ct.c_double * 3)]


class OOpts(ct.Structure):
    _fields_ = [("lowpass", ct.c_double), ("z_near", ct.c_double), ("guard", ct.c_double),
                ("alpha_max", ct.c_double), ("alpha_min", ct.c_double), ("t_min", ct.c_double),
                ("eps_alpha", ct.c_double), ("eps_t", ct.c_double), ("eps_alpha_mag", ct.c_double),
                ("tile", ct.c_int32), ("pad", ct.c_int32)]


PROJ_DTYPE = np.dtype([
    ("ntiles", np.int64), ("tx", np.float64), ("ty", np.float64), ("tz", np.float64),
    ("mx", np.float64), ("my", np.float64), ("a", np.float64), ("b", np.float64),
    ("c", np.float64), ("A", np.float64), ("B", np.float64), ("C", np.float64),
    ("sig", np.float64), ("lam", np.float64), ("radius", np.float64),
    ("valid", np.int32), ("clampx", np.int32), ("clampy", np.int32),
    ("x0", np.int32), ("x1", np.int32), ("y0", np.int32), ("y1", np.int32),
    ("tx0", np.int32), ("tx1", np.int32), ("ty0", np.int32), ("ty1", np.int32),
    ("depth32", np.float32)], align=True)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from oracle import build as _b
            _b.build()
        L = ct.CDLL(_LIB_PATH)
        P = ct.c_void_p
        i64, i32 = ct.c_int64, ct.c_int32
        L.oracle_project.argtypes = [i64, P, P, P, P, ct.POINTER(OCam), ct.POINTER(OOpts), P]
        L.oracle_project.restype = None
        L.oracle_count.argtypes = [i64, P]
        L.oracle_count.restype = i64
        L.oracle_bin.argtypes = [i32, i64, P, P, P, i64, i64, P, P, P]
        L.oracle_bin.restype = None
        L.oracle_render.argtypes = [P, ct.POINTER(OCam), ct.POINTER(OOpts), P, i32, P, P, i64, i64,
                                    P, P, P, P, P, P, P]
        L.oracle_render.restype = None
        L.oracle_render_region.argtypes = [i64, P, ct.POINTER(OCam), ct.POINTER(OOpts), P, i32, i32,
                                           i32, i32, i32, P, P, P, P]
        L.oracle_render_region.restype = ct.c_double
        L.oracle_render_backward.argtypes = [i64, P, ct.POINTER(OCam), ct.POINTER(OOpts), P, i32, P,
                                             P, i64, P, P, P, P, P, P, ct.c_double]
        L.oracle_render_backward.restype = None
        L.oracle_project_backward.argtypes = [i64, P, P, P, P, ct.POINTER(OCam), ct.POINTER(OOpts),
                                              P, P, P, P, P]
        L.oracle_project_backward.restype = None
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = i32
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_set_threads.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ct.c_void_p) if a is not None else None


def make_cam(cam) -> OCam:
    W, H, fx, fy, cx, cy, R, t = cam.as_tuple()
    return OCam(W, H, fx, fy, cx, cy, (ct.c_double * 9)(*R), (ct.c_double * 3)(*t))


def make_opts(tile=16, lowpass=0.3, z_near=0.2, guard=1.3, eps_alpha=1e-5, eps_t=1e-4,
              eps_alpha_mag=0.0) -> OOpts:
    return OOpts(lowpass, z_near, guard, ALPHA_MAX, ALPHA_MIN, T_MIN, eps_alpha, eps_t, eps_alpha_mag, int(tile), 0)


class Params:
    """Per-Gaussian parameters promoted to float64 (the oracle's working precision)."""

    def __init__(self, mean, log_scale, quat, opacity_logit):
        self.mean = np.ascontiguousarray(mean, np.float64)
        self.log_scale = np.ascontiguousarray(log_scale, np.float64)
        self.quat = np.ascontiguousarray(quat, np.float64)
        self.omega = np.ascontiguousarray(opacity_logit, np.float64)

    @classmethod
    def from_scene(cls, scene):
        return cls(scene.mean, scene.log_scale, scene.quat, scene.opacity_logit)

    @property
    def n(self):
        return self.mean.shape[0]

    def copy(self):
        return Params(self.mean.copy(), self.log_scale.copy(), self.quat.copy(), self.omega.copy())


def project(params: Params, cam, opts: OOpts) -> np.ndarray:
    out = np.zeros(params.n, PROJ_DTYPE)
    c = make_cam(cam)
    lib().oracle_project(params.n, _p(params.mean), _p(params.log_scale), _p(params.quat),
                         _p(params.omega), ct.byref(c), ct.byref(opts), _p(out))
    return out


def view_tables(cams, tile):
    tiles_x = np.array([(c.width + tile - 1) // tile for c in cams], np.int32)
    tiles_y = np.array([(c.height + tile - 1) // tile for c in cams], np.int32)
    counts = tiles_x.astype(np.int64) * tiles_y
    offsets = np.concatenate([[0], np.cumsum(counts)[:-1]]).astype(np.int64)
    return tiles_x, tiles_y, offsets, int(counts.sum())


def project_views(params: Params, cams, opts: OOpts) -> np.ndarray:
    """[n_views, n] projected records."""
    return np.stack([project(params, c, opts) for c in cams], axis=0)


def bin_lists(proj: np.ndarray, cams, opts: OOpts):
    """Sorted keys (u64), ids (u32) and ranges ([tiles, 2] u32) over all views."""
    n_views, n = proj.shape
    tiles_x, _, offsets, total_tiles = view_tables(cams, opts.tile)
    flat = np.ascontiguousarray(proj.reshape(-1))
    total = int(lib().oracle_count(flat.shape[0], _p(flat)))
    keys = np.zeros(max(total, 1), np.uint64)
    ids = np.zeros(max(total, 1), np.uint32)
    ranges = np.zeros((total_tiles, 2), np.uint32)
    lib().oracle_bin(n_views, n, _p(flat), _p(offsets), _p(tiles_x), total_tiles, total,
                     _p(keys), _p(ids), _p(ranges))
    return keys[:total], ids[:total], ranges


def render_view(proj_v, cam, opts, channels, ids, ranges, tile_offset, pix=None, flip_mask=None):
    """Render one view from its tile lists. Returns dict with out [C, npix],
    T [npix], last [npix], n_amb [npix], margin [npix] (npix = H*W if pix is None)."""
    ch = np.ascontiguousarray(channels, np.float64)
    C = ch.shape[1]
    assert C <= 64
    c = make_cam(cam)
    npix = cam.width * cam.height if pix is None else len(pix)
    pix_a = None if pix is None else np.ascontiguousarray(pix, np.int64)
    fm = None if flip_mask is None else np.ascontiguousarray(flip_mask, np.uint32)
    out = np.zeros((C, npix))
    T = np.zeros(npix)
    last = np.zeros(npix, np.int64)
    namb = np.zeros(npix, np.int32)
    margin = np.zeros(npix)
    pv = np.ascontiguousarray(proj_v)
    idv = np.ascontiguousarray(ids if len(ids) else np.zeros(1, np.uint32))
    lib().oracle_render(_p(pv), ct.byref(c), ct.byref(opts), _p(ch), C, _p(idv), _p(ranges),
                        int(tile_offset), npix, _p(pix_a), _p(fm), _p(out), _p(T), _p(last),
                        _p(namb), _p(margin))
    return dict(out=out, T=T, last=last, n_amb=namb, margin=margin)


def render_region(proj_v, cam, opts, channels, x0, y0, w, h, G=None):
    ch = np.ascontiguousarray(channels, np.float64)
    C = ch.shape[1]
    c = make_cam(cam)
    out = np.zeros((C, h, w))
    T = np.zeros((h, w))
    hsh = ct.c_uint64(0)
    Gd = None if G is None else np.ascontiguousarray(G, np.float64)
    pv = np.ascontiguousarray(proj_v)
    loss = lib().oracle_render_region(pv.shape[0], _p(pv), ct.byref(c), ct.byref(opts), _p(ch), C,
                                      int(x0), int(y0), int(w), int(h), _p(Gd), _p(out), _p(T),
                                      ct.byref(hsh))
    return dict(out=out, T=T, loss=float(loss), hash=int(hsh.value))


def render_backward_view(proj_v, cam, opts, channels, ids, ranges, tile_offset, G_view,
                         flip_mask=None, dch=None, mag=None, mag_cond=0.0):
    """Returns (grad2d [n, 6] for this view, dch [n, C] accumulated). mag
    (optional dict with "g2" [n, 6] and "channels" [n, C]) receives the
    magnitude sums sum |term| of those gradients (g2 overwritten, channels
    accumulated), each pixel's terms weighted by 1 + mag_cond * S, S the sum of
    1 / (1 - alpha) over the pixel's blended entries (how strongly rounding
    errors of the alphas reach the pixel's terms through T and the suffix)."""
    ch = np.ascontiguousarray(channels, np.float64)
    n, C = ch.shape
    c = make_cam(cam)
    g2 = np.zeros((n, 6))
    if dch is None:
        dch = np.zeros((n, C))
    Gd = np.ascontiguousarray(G_view, np.float64)
    fm = None if flip_mask is None else np.ascontiguousarray(flip_mask, np.uint32)
    pv = np.ascontiguousarray(proj_v)
    idv = np.ascontiguousarray(ids if len(ids) else np.zeros(1, np.uint32))
    m2 = mc = None
    if mag is not None:
        mag["g2"] = m2 = np.zeros((n, 6))
        mc = mag.setdefault("channels", np.zeros((n, C)))
    lib().oracle_render_backward(n, _p(pv), ct.byref(c), ct.byref(opts), _p(ch), C, _p(idv),
                                 _p(ranges), int(tile_offset), _p(Gd), _p(fm), _p(g2), _p(dch),
                                 _p(m2), _p(mc), float(mag_cond))
    return g2, dch


def project_backward(params: Params, cam, opts, grad2d, acc=None):
    n = params.n
    if acc is None:
        acc = dict(mean=np.zeros((n, 3)), log_scale=np.zeros((n, 3)), quat=np.zeros((n, 4)),
                   opacity_logit=np.zeros(n))
    c = make_cam(cam)
    g2 = np.ascontiguousarray(grad2d, np.float64)
    lib().oracle_project_backward(n, _p(params.mean), _p(params.log_scale), _p(params.quat),
                                  _p(params.omega), ct.byref(c), ct.byref(opts), _p(g2),
                                  _p(acc["mean"]), _p(acc["log_scale"]), _p(acc["quat"]),
                                  _p(acc["opacity_logit"]))
    return acc


def threads() -> int:
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


# ---- whole-pipeline helpers --------------------------------------------------

def forward(scene, cams, opts, params: Params | None = None):
    """Project, bin and render every view. Returns dict with proj [V, n],
    keys, ids, ranges, per-view renders and the concatenated planar outputs."""
    params = params or Params.from_scene(scene)
    proj = project_views(params, cams, opts)
    keys, ids, ranges = bin_lists(proj, cams, opts)
    _, _, offsets, _ = view_tables(cams, opts.tile)
    views = []
    for v, cam in enumerate(cams):
        views.append(render_view(proj[v], cam, opts, scene.channels, ids, ranges, offsets[v]))
    return dict(params=params, proj=proj, keys=keys, ids=ids, ranges=ranges, offsets=offsets,
                views=views)


GEO_GROUPS = ("mean", "log_scale", "quat", "opacity_logit")


def backward(scene, cams, opts, fwd, G_flat, flip_masks=None, magnitudes=False, mag_cond=0.0):
    """Gradients of sum(G * out) w.r.t. every per-Gaussian parameter (float64).

    With magnitudes, also acc["mag"]: for every gradient entry the scale of
    the rounding error of a floating-point evaluation of it. The blend sums
    are the only long sums of the gradient (every other step is a fixed short
    formula), so this is sum |term| of the per-view screen-space and channel
    sums, carried to the per-Gaussian groups through the magnitude of the
    projection's chain rule: for each view and screen-space component k,
    |J e_k| (the chain rule applied to a unit gradient in k) times the
    magnitude sum of component k. mag_cond weights each pixel's terms as in
    render_backward_view."""
    params = fwd["params"]
    n, C = scene.channels.shape
    dch = np.zeros((n, C))
    acc = None
    grad2d_all = []
    mag = dict(channels=np.zeros((n, C))) if magnitudes else None
    mags = {k: 0.0 for k in GEO_GROUPS}
    mag2d_all = []
    off = 0
    for v, cam in enumerate(cams):
        hw = cam.width * cam.height
        Gv = G_flat[off:off + C * hw].reshape(C, hw)
        off += C * hw
        fm = None if flip_masks is None else flip_masks[v]
        g2, dch = render_backward_view(fwd["proj"][v], cam, opts, scene.channels, fwd["ids"],
                                       fwd["ranges"], fwd["offsets"][v], Gv, fm, dch, mag, mag_cond)
        grad2d_all.append(g2)
        acc = project_backward(params, cam, opts, g2, acc)
        if magnitudes:
            mag2d_all.append(mag["g2"])
            for k in range(6):
                unit = np.zeros((n, 6))
                unit[:, k] = 1.0
                col = project_backward(params, cam, opts, unit)
                for grp in GEO_GROUPS:
                    mags[grp] = mags[grp] + np.abs(col[grp]) * mag["g2"][:, k].reshape((n,) + (1,) * (col[grp].ndim - 1))
    acc["channels"] = dch
    acc["grad2d"] = np.stack(grad2d_all, axis=0)
    if magnitudes:
        acc["mag"] = dict(mags, channels=mag["channels"], grad2d=np.stack(mag2d_all, axis=0))
    return acc
