"""Shared helpers for GPU-vs-oracle parity tests (not collected by pytest).

Comparison rules
  - integer work (boxes, tile counts, keys, ids, ranges, last): bit-exact;
  - rendered channels and final transmittance: |gpu - oracle| <= 1e-4 per
    pixel and channel. Where a skip (alpha vs 1/255) or stop (T (1 - alpha) vs
    1e-4) decision lies within a relative margin of 1e-5 / 1e-4 of its
    threshold, float32 and float64 may legitimately take different branches:
    such a pixel also passes if it matches the oracle with that decision
    inverted (up to the first four ambiguous events, any combination);
  - gradients: per Gaussian and parameter group,
    ||g - g_ref|| <= 1e-3 * max(||g_ref||, f * RMS of the group) + k * ||m||
    with f = 1e-3 (f = 1e-2 for the quaternion), the oracle replaying each
    pixel along the branch the GPU took, and ||G - G_ref|| / ||G_ref|| <= 1e-5
    over the whole group. m is the oracle's magnitude of the sums that form
    the gradient (sum |term| of each blend sum, carried through the
    magnitude of the projection's chain rule) and k = 3e-5: a float32 sum can
    only be as exact as its terms, whose float32 evaluation is good to a
    relative 3e-5 (a few ulps per operation, and the transmittance recovered
    back to front by up to a few hundred divisions). The term matters only
    where the terms cancel (|sum| much smaller than sum |term|); elsewhere
    the 1e-3 relative bound decides. The quaternion's larger floor covers a
    cancellation by construction: the quaternion gradient of a nearly
    isotropic Gaussian is a difference of nearly equal terms (it vanishes
    for an isotropic one), so float32 rounding of its conic gradients,
    amplified by the ratio of the two scales, dominates it.
"""
from __future__ import annotations

import numpy as np
import torch

from oracle import oracle as O

GROUPS = ("mean", "log_scale", "quat", "opacity_logit", "channels")


def to_dev(scene, device="cuda"):
    return dict(mean=torch.from_numpy(scene.mean).to(device),
                log_scale=torch.from_numpy(scene.log_scale).to(device),
                quat=torch.from_numpy(scene.quat).to(device),
                opacity_logit=torch.from_numpy(scene.opacity_logit).to(device),
                channels=torch.from_numpy(scene.channels).to(device))


# Skip decisions a float32 evaluation may take either way: within a relative
# 1e-5 of 1/255 (the rounding of alpha itself, ~|power| 2^-24), plus 16 ulps
# (2^-24 each) per unit of the exponent's magnitude sum, which bounds the
# effect of rounding the conic and the mean offsets to float32 where the
# exponent's terms cancel (needle-shaped Gaussians: a sum of 600 for a power
# of -5 moves alpha by ~1.7e-5, measured in float32).
EPS_ALPHA_MAG = 16.0 * 2.0 ** -24


def oracle_opts(o, eps_alpha=1e-5, eps_t=1e-4, eps_alpha_mag=EPS_ALPHA_MAG):
    return O.make_opts(tile=o.tile, lowpass=o.lowpass, z_near=o.z_near, guard=o.guard,
                       eps_alpha=eps_alpha, eps_t=eps_t, eps_alpha_mag=eps_alpha_mag)


def compare_projection(proj_gpu, fwd, n):
    """GPU projected records vs the oracle's: integers exact, floats close."""
    P = fwd["proj"].reshape(-1)
    box = proj_gpu.box.cpu().numpy()
    nt = proj_gpu.ntiles.cpu().numpy().astype(np.int64)
    valid = P["valid"] == 1
    want_box = np.stack([P["x0"], P["x1"], P["y0"], P["y1"]], 1)
    assert np.array_equal(nt, np.where(valid, P["ntiles"], 0)), "tile counts differ"
    assert np.array_equal(box[valid], want_box[valid]), "pixel boxes differ"
    assert (box[~valid, 0] > box[~valid, 1]).all(), "culled Gaussians must have empty boxes"
    depth = proj_gpu.depth.cpu().numpy()
    assert np.array_equal(depth[valid].view(np.uint32), P["depth32"][valid].view(np.uint32))
    m2 = proj_gpu.mean2d.cpu().numpy()
    assert np.allclose(m2[valid, 0], P["mx"][valid], rtol=1e-13, atol=1e-9)
    assert np.allclose(m2[valid, 1], P["my"][valid], rtol=1e-13, atol=1e-9)
    cn = proj_gpu.conic.cpu().numpy().astype(np.float64)
    scale = np.maximum(np.abs(P["A"]), np.abs(P["C"]))
    for k, f in enumerate(("A", "B", "C")):
        assert (np.abs(cn[valid, k] - P[f][valid]) <= 2.5e-7 * scale[valid]).all(), f"conic {f}"
    assert np.allclose(cn[valid, 3], P["sig"][valid], rtol=2e-7, atol=0)
    return int(valid.sum())


def compare_bins(bins_gpu, fwd, ids_only=False):
    """Tile lists bit-exact: count, keys (unless the binning wrote ids only),
    ids and ranges."""
    n_inst = int(bins_gpu.count.item())
    assert n_inst == len(fwd["keys"]), (n_inst, len(fwd["keys"]))
    ids = bins_gpu.ids[:n_inst].cpu().numpy().view(np.uint32)
    if not ids_only:
        keys = bins_gpu.keys[:n_inst].cpu().numpy().view(np.uint64)
        assert np.array_equal(keys, fwd["keys"]), "sorted keys differ"
    assert np.array_equal(ids, fwd["ids"]), "sorted ids differ"
    rg = bins_gpu.ranges.cpu().numpy().view(np.uint32)
    empty_o = fwd["ranges"][:, 0] == fwd["ranges"][:, 1]
    empty_g = rg[:, 0] == rg[:, 1]
    assert np.array_equal(empty_o, empty_g)
    assert np.array_equal(rg[~empty_g], fwd["ranges"][~empty_o])
    return n_inst


def compare_render(out_g, T_g, last_g, scene, cams, oo, fwd, tol=1e-4, pix_subset=None):
    """Per-pixel parity with the ambiguity rule. A pixel without ambiguous
    decisions must match the oracle (channels and T within tol, last exact).
    A pixel with some must match one of its branches (the oracle with any
    combination of its first four ambiguous decisions inverted) the same way;
    of the branches that do, the one whose final T is closest to the GPU's in
    relative terms is taken as the GPU's branch (flipping a decision moves T
    by a factor 1 - alpha, far beyond float32 rounding, even where the
    channels move by less than tol), and the backward replays it. Returns
    (flip masks per view, stats). pix_subset: optional per-view arrays of
    linear pixel indices to check (the oracle renders only those)."""
    C = scene.n_channels
    out_g = out_g.cpu().numpy()
    T_g = T_g.cpu().numpy()
    last_g = last_g.cpu().numpy().astype(np.int64)
    off_pix = 0
    masks = []
    stats = dict(pixels=0, ambiguous=0, flipped=0, max_err=0.0)
    for v, cam in enumerate(cams):
        hw = cam.width * cam.height
        go = out_g[C * off_pix:C * (off_pix + hw)].reshape(C, hw)
        gT = T_g[off_pix:off_pix + hw]
        gl = last_g[off_pix:off_pix + hw]
        if pix_subset is None:
            r = fwd["views"][v]
            pix = np.arange(hw)
        else:
            pix = np.asarray(pix_subset[v], np.int64)
            r = O.render_view(fwd["proj"][v], cam, oo, scene.channels, fwd["ids"], fwd["ranges"],
                              fwd["offsets"][v], pix=pix)
        go, gT, gl = go[:, pix], gT[pix], gl[pix]
        err = np.maximum(np.abs(go - r["out"]).max(axis=0), np.abs(gT - r["T"]))
        ok = (err <= tol) & (gl == r["last"])
        mask = np.zeros(len(pix), np.uint32)
        stats["pixels"] += len(pix)
        bad = np.nonzero(~ok)[0]
        unresolved = bad[r["n_amb"][bad] == 0]
        assert len(unresolved) == 0, (
            f"view {v}: {len(unresolved)} unambiguous pixels differ; first {pix[unresolved[:5]]},"
            f" err {err[unresolved[:5]]}, last gpu {gl[unresolved[:5]]} oracle {r['last'][unresolved[:5]]}")
        amb = np.nonzero(r["n_amb"] > 0)[0]
        stats["ambiguous"] += len(amb)
        if len(amb):
            def rel_T(t_branch, idx):
                return np.abs(gT[idx] - t_branch) / np.maximum(t_branch, 1e-30)
            best = np.where(ok[amb], rel_T(r["T"][amb], amb), np.inf)
            for m in range(1, 16):
                si = np.nonzero(r["n_amb"][amb] >= m.bit_length())[0]
                if len(si) == 0:
                    continue
                sel = amb[si]
                rf = O.render_view(fwd["proj"][v], cam, oo, scene.channels, fwd["ids"],
                                   fwd["ranges"], fwd["offsets"][v], pix=pix[sel],
                                   flip_mask=np.full(len(sel), m, np.uint32))
                e2 = np.maximum(np.abs(go[:, sel] - rf["out"]).max(axis=0), np.abs(gT[sel] - rf["T"]))
                sc = rel_T(rf["T"], sel)
                upd = (e2 <= tol) & (gl[sel] == rf["last"]) & (sc < best[si])
                best[si[upd]] = sc[upd]
                mask[sel[upd]] = m
            nomatch = amb[~np.isfinite(best)]
            assert len(nomatch) == 0, (f"view {v}: {len(nomatch)} ambiguous pixels match no branch; "
                                       f"first {pix[nomatch[:5]]} err {err[nomatch[:5]]}")
            stats["flipped"] += int((mask[amb] != 0).sum())
        stats["max_err"] = max(stats["max_err"], float(err[ok].max()) if ok.any() else 0.0)
        full = np.zeros(hw, np.uint32)
        full[pix] = mask
        masks.append(full)
        off_pix += hw
    return masks, stats


def gpu_grads_to_np(grads, d_ch):
    out = {k: grads[k].cpu().numpy().astype(np.float64) for k in ("mean", "log_scale", "quat", "opacity_logit")}
    out["channels"] = d_ch.cpu().numpy().astype(np.float64)
    return out


FLOOR = {"quat": 1e-2}
FLOOR_DEFAULT = 1e-3


def group_floor(grp):
    return FLOOR.get(grp, FLOOR_DEFAULT)


# Rounding-error model of a float32 evaluation of the gradient sums, in units
# of the oracle's magnitude sums (sum |term|, each pixel's terms weighted by
# 1 + MAG_COND * S with S = sum 1 / (1 - alpha) over its blended entries).
# A term's own float32 arithmetic and the summation of up to ~1e5 terms per
# Gaussian (wave reductions, then atomics) stay within MAG_KAPPA = 3e-5 (about
# 250 float32 half-ulps) of sum |term|. The transmittance and the suffix are
# products over the list: a rounding error of a few half-ulps in alpha_j moves
# them by about 5 u / (1 - alpha_j) relative, u = 2^-24, so a pixel's terms
# carry up to about 5 u S relative error; MAG_KAPPA * MAG_COND = 1e-6 (about
# 16 u) covers that with a factor of 3 to spare.
MAG_KAPPA = 3e-5
MAG_COND = 1.0 / 30.0


def compare_grads(g, ref, n, tol=1e-3, groups=GROUPS, subset=None, floor=None, global_tol=1e-5, mag=None):
    """Per-Gaussian group check; returns worst ratio err / bound and the
    global relative error per group (asserted <= global_tol unless None).
    mag (optional): per group, the magnitude sums of the reference gradient
    (same shape), adding MAG_KAPPA * ||mag|| to each bound."""
    worst = {}
    for grp in groups:
        fl = group_floor(grp) if floor is None else floor
        a = np.asarray(g[grp], np.float64).reshape(n, -1)
        r = np.asarray(ref[grp], np.float64).reshape(n, -1)
        m = None if mag is None else np.asarray(mag[grp], np.float64).reshape(n, -1)
        if subset is not None:
            a, r = a[subset], r[subset]
            m = None if m is None else m[subset]
        nz = np.abs(r).sum(axis=1) > 0
        rms = np.sqrt(np.mean(r[nz] ** 2)) if nz.any() else 0.0
        err = np.linalg.norm(a - r, axis=1)
        bound = tol * np.maximum(np.linalg.norm(r, axis=1), fl * rms)
        if m is not None:
            bound = bound + MAG_KAPPA * np.linalg.norm(m, axis=1)
        bad = err > bound
        if nz.any() or bad.any():
            k = int(np.argmax(err / np.maximum(bound, 1e-300)))
            worst[grp] = dict(ratio=float(err[k] / max(bound[k], 1e-300)),
                              global_rel=float(np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-300)),
                              worst_norm_over_rms=float(np.linalg.norm(r[k]) / max(rms, 1e-300)),
                              index=int(k), err=float(err[k]), norm=float(np.linalg.norm(r[k])),
                              mag_norm=None if m is None else float(np.linalg.norm(m[k])))
        assert not bad.any(), (f"{grp}: {int(bad.sum())} of {len(a)} Gaussians exceed tolerance; "
                               f"worst {worst[grp]}")
        if global_tol is not None and grp in worst:
            assert worst[grp]["global_rel"] <= global_tol, (grp, worst[grp])
    return worst


def check_mlp_probs(pr_gpu, feat, ws, bs, normalize, tol=2e-5, max_unresolved_frac=0.002,
                    hidden_out=None):
    """GPU decoder probabilities [P][N] against the oracle. A pixel none of
    whose bf16-rounded values lies near a rounding midpoint must be within tol
    of the oracle's softmax; every other pixel within tol of the softmax of
    one of its rounding branches (oracle.decode.mlp_branches), which fixes the
    logits used for it. Pixels with more ambiguous values than the branch
    enumeration follows (at most max_unresolved_frac of them) are left out.
    Returns (logits [P][N] of the matched branches, resolved mask, number of
    ambiguous pixels). With hidden_out a list, it receives the oracle's
    rounded layer inputs [x, h1, ...] ([P][width] each) of the matched
    branches (the plain forward's where a pixel is unresolved)."""
    from oracle import decode as D
    ref = D.mlp_forward(feat, ws, bs, normalize=normalize)
    logits = ref["logits"].copy()
    if hidden_out is not None:
        hidden_out[:] = [h.copy() for h in ref["hs"]]
    M = D.softmax(logits)
    ok = ~ref["ambiguous"]
    err = np.abs(pr_gpu - M).max(axis=1)
    assert (err[ok] < tol).all(), (int((err[ok] >= tol).sum()), float(err[ok].max()))
    resolved = ok.copy()
    unresolved = 0
    for i in np.nonzero(~ok)[0]:
        br, complete, hid = D.mlp_branches(feat[i], ws, bs, normalize=normalize, return_hidden=True)
        errs = [np.abs(pr_gpu[i] - D.softmax(b[None])[0]).max() for b in br]
        k = int(np.argmin(errs))
        if errs[k] < tol:
            logits[i] = br[k]
            resolved[i] = True
            if hidden_out is not None:
                for h, v in zip(hidden_out, hid[k]):
                    h[i] = v
        else:
            assert not complete, (i, errs[k])
            unresolved += 1
    assert unresolved <= max_unresolved_frac * len(feat), unresolved
    return logits, resolved, int((~ok).sum())

