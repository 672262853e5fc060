"""Central finite differences of L = sum(G * out) in float64 (test
infrastructure only).

For a chosen Gaussian and parameter, the Gaussian is re-projected at
theta + s h for s in (-2, -1, 1, 2) and only the rectangle covering its pixel
boxes in all of these states is re-rendered from the tile-free definition
(every other pixel does not contain it in any state, so its output is
unchanged). The derivative is the five-point stencil
(-L(+2h) + 8 L(+h) - 8 L(-h) + L(-2h)) / (12 h), error O(h^4); it is accepted
only if every box / skip / blend / clamp / stop decision inside that rectangle
is identical in all five states; otherwise h is halved (down to h_min) and the
entry is reported as unpinned if no step qualifies.
"""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

GROUPS = (("mean", 3), ("log_scale", 3), ("quat", 4), ("opacity_logit", 1))


def _param_array(params: O.Params, group):
    return {"mean": params.mean, "log_scale": params.log_scale, "quat": params.quat,
            "opacity_logit": params.omega}[group]


def _project_single(params: O.Params, g, cam, opts):
    sub = O.Params(params.mean[g:g + 1], params.log_scale[g:g + 1], params.quat[g:g + 1],
                   params.omega[g:g + 1])
    return O.project(sub, cam, opts)[0]


def _region(states, cam):
    xs0, xs1, ys0, ys1 = [], [], [], []
    for s in states:
        if s["valid"]:
            xs0.append(s["x0"]); xs1.append(s["x1"]); ys0.append(s["y0"]); ys1.append(s["y1"])
    if not xs0:
        return None
    return min(xs0), min(ys0), max(xs1) - min(xs0) + 1, max(ys1) - min(ys0) + 1


class _Local:
    """The Gaussians whose pixel boxes intersect a margin around Gaussian g,
    kept in id order (so depth ties resolve exactly as over the full set).
    Any region inside the margin renders identically from this subset."""

    def __init__(self, proj_v, g, cam, channels, margin=24):
        p = proj_v[g]
        self.x0 = max(0, int(p["x0"]) - margin)
        self.y0 = max(0, int(p["y0"]) - margin)
        self.x1 = min(cam.width - 1, int(p["x1"]) + margin)
        self.y1 = min(cam.height - 1, int(p["y1"]) + margin)
        v = proj_v["valid"] == 1
        hit = v & (proj_v["x1"] >= self.x0) & (proj_v["x0"] <= self.x1) & \
            (proj_v["y1"] >= self.y0) & (proj_v["y0"] <= self.y1)
        hit[g] = True
        self.idx = np.nonzero(hit)[0]
        self.k = int(np.searchsorted(self.idx, g))
        self.proj = np.ascontiguousarray(proj_v[self.idx])
        self.channels = np.ascontiguousarray(np.asarray(channels, np.float64)[self.idx])

    def covers(self, region):
        x0, y0, w, h = region
        return x0 >= self.x0 and y0 >= self.y0 and x0 + w - 1 <= self.x1 and y0 + h - 1 <= self.y1


def _loss_state(local, state, cam, opts, Gv, region, channels=None):
    pv = local.proj.copy()
    pv[local.k] = state
    x0, y0, w, h = region
    assert local.covers(region)
    Gr = Gv.reshape(Gv.shape[0], cam.height, cam.width)[:, y0:y0 + h, x0:x0 + w]
    ch = local.channels if channels is None else channels
    r = O.render_region(pv, cam, opts, ch, x0, y0, w, h, np.ascontiguousarray(Gr))
    return r["loss"], r["hash"]


def fd_gaussian(params: O.Params, channels, cams, opts, proj, G_flat, g,
                h_rel=1e-4, h_min=1e-8):
    """FD gradient of one Gaussian's geometric parameters and channels.
    Returns dict group -> (values [k], valid mask [k])."""
    C = channels.shape[1]
    Gvs = []
    off = 0
    for cam in cams:
        hw = cam.width * cam.height
        Gvs.append(G_flat[off:off + C * hw].reshape(C, hw))
        off += C * hw
    res = {}
    locals_ = [(_Local(proj[v], g, cam, channels) if proj[v][g]["valid"] else None)
               for v, cam in enumerate(cams)]
    steps = (2.0, 1.0, -1.0, -2.0)
    coef = (-1.0, 8.0, -8.0, 1.0)
    for group, k in GROUPS:
        vals = np.zeros(k)
        ok = np.zeros(k, bool)
        arr = _param_array(params, group)
        for comp in range(k):
            theta = float(arr.reshape(params.n, -1)[g, comp])
            h = h_rel * max(1.0, abs(theta))
            while h >= h_min:
                total = 0.0
                valid = True
                for v, cam in enumerate(cams):
                    pp = O.Params(params.mean[g:g + 1], params.log_scale[g:g + 1],
                                  params.quat[g:g + 1], params.omega[g:g + 1]).copy()
                    pa = _param_array(pp, group).reshape(1, -1)
                    states = []
                    for st in steps:
                        pa[0, comp] = theta + st * h
                        states.append(_project_single(pp, 0, cam, opts))
                    s0 = proj[v][g]
                    reg = _region([s0] + states, cam)
                    if reg is None:
                        continue
                    loc = locals_[v]
                    if loc is None or not loc.covers(reg):
                        loc = _Local(proj[v], g, cam, channels, margin=10 ** 6)
                    _, h0 = _loss_state(loc, s0, cam, opts, Gvs[v], reg)
                    acc = 0.0
                    for st, cf, sx in zip(steps, coef, states):
                        l, hx = _loss_state(loc, sx, cam, opts, Gvs[v], reg)
                        if hx != h0:
                            valid = False
                            break
                        acc += cf * l
                    if not valid:
                        break
                    total += acc / (12.0 * h)
                if valid:
                    vals[comp] = total
                    ok[comp] = True
                    break
                h *= 0.5
        res[group] = (vals, ok)
    # channels: out is linear in them, a central difference is exact up to rounding
    vals = np.zeros(C)
    for comp in range(C):
        theta = float(channels[g, comp])
        h = max(1.0, abs(theta))
        total = 0.0
        for v, cam in enumerate(cams):
            s0 = proj[v][g]
            reg = _region([s0], cam)
            if reg is None:
                continue
            loc = locals_[v]
            chp = loc.channels.copy()
            chp[loc.k, comp] = theta + h
            lp, _ = _loss_state(loc, s0, cam, opts, Gvs[v], reg, chp)
            chp[loc.k, comp] = theta - h
            lm, _ = _loss_state(loc, s0, cam, opts, Gvs[v], reg, chp)
            total += (lp - lm) / (2.0 * h)
        vals[comp] = total
    res["channels"] = (vals, np.ones(C, bool))
    return res


def blended_gaussians(bwd):
    """Ids of Gaussians blended into at least one pixel of some view: exactly
    those with a non-zero channel gradient under a generic upstream G."""
    return np.nonzero(np.abs(bwd["channels"]).sum(axis=1) > 0)[0]
