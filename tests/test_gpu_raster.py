"""GPU parity of the splatting path (projection, binning, blending and their
backward) against the FP64 CPU oracle, through the C ABI of liblegs.so.

Renderer: Sec. 3.1 Eq. 1 with the semantic (Sec. 3.4.1, R_s) and
uncertainty (Sec. 3.4.2, R_u) channels blended alongside RGB.
"""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import fd
from oracle import oracle as O
from tests import parity as PT

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def R():
    from paper_2311_18482_amd import raster
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return raster


def run_forward(R, scene, cams, o):
    rast = R.Rasterizer(cams, o)
    d = PT.to_dev(scene)
    proj, bins, out, T, last = rast.forward(d["mean"], d["log_scale"], d["quat"],
                                            d["opacity_logit"], d["channels"])
    torch.cuda.synchronize()
    return rast, d, proj, bins, out, T, last


def run_backward(R, rast, d, proj, bins, T, last, G):
    Gd = torch.from_numpy(G).cuda()
    grad2d, d_ch = R.render_backward(rast.ctx, proj, bins, rast.views, d["channels"], rast.o, T,
                                     last, Gd)
    grads = R.project_backward(rast.ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"],
                               rast.views, rast.o, proj, grad2d)
    torch.cuda.synchronize()
    return grad2d, grads, d_ch


def full_check(R, scene, cams, tile=16, batch=256, grads=True, seed_g=200):
    o = R.opts(tile=tile, lds_batch=batch)
    oo = PT.oracle_opts(o)
    note(f"forward n={scene.n} views={len(cams)} tile={tile} batch={batch}")
    rast, d, proj, bins, out, T, last = run_forward(R, scene, cams, o)
    fwd = O.forward(scene, cams, oo)
    PT.compare_projection(proj, fwd, scene.n)
    PT.compare_bins(bins, fwd)
    masks, stats = PT.compare_render(out, T, last, scene, cams, oo, fwd)
    note(f"render stats {stats}")
    if not grads:
        return stats
    G = synth.upstream_grads(cams, scene.n_channels, seed_g)
    note("backward")
    grad2d, g, d_ch = run_backward(R, rast, d, proj, bins, T, last, G)
    ref = O.backward(scene, cams, oo, fwd, G.astype(np.float64), flip_masks=masks, magnitudes=True, mag_cond=PT.MAG_COND)
    # per-G-view screen-space gradients: an intermediate mixing units (mean,
    # conic and opacity gradients), whose largest entries are conic gradients
    # of the smallest Gaussians, sums with cancellation: its global error is
    # bounded at 3e-5
    g2 = grad2d.cpu().numpy()[:, :6].astype(np.float64)
    ref2 = ref["grad2d"].reshape(-1, 6)
    PT.compare_grads({"g2": g2}, {"g2": ref2}, g2.shape[0], groups=("g2",), global_tol=3e-5,
                     mag={"g2": ref["mag"]["grad2d"].reshape(-1, 6)})
    worst = PT.compare_grads(PT.gpu_grads_to_np(g, d_ch), ref, scene.n, mag=ref["mag"])
    note(f"gradient worst ratios {worst}")
    return stats


def test_c1_forward_backward(R):
    scene, cams = synth.workload_c1()
    full_check(R, scene, cams)


@pytest.mark.parametrize("tile,batch", [(8, 64), (32, 128), (16, 64)])
def test_c1_other_tiles(R, tile, batch):
    scene, cams = synth.workload_c1()
    full_check(R, scene, cams, tile=tile, batch=batch)


def test_ragged_multiview(R):
    """Views whose sizes are not multiples of the tile, seen from different poses."""
    scene = synth.make_scene(6000, 12, synth.VOL_C1, d_sem=8)
    cams = [synth.camera_front(100, 75, 110.0), synth.camera_front(37, 53, 40.0)]
    R2, t2 = synth.look_at((2.0, 1.0, -2.0), target=(0.0, 0.0, 4.0))
    cams.append(synth.Camera(150, 90, 140.0, 150.0, 70.0, 47.0, R2, t2))
    for tile in (8, 16, 32):
        full_check(R, scene, cams, tile=tile, batch=128)


def test_many_views_index_apart_from_depth_keys(R):
    """520 small views: the G-view depth keys need 6 digit passes (10 view bits
    above the 32 depth bits) and the G-view index 17 bits, more than 64 in all,
    so the index travels in an array of its own beside the keys (the depth
    sort's other path; every other scene packs it into the keys' low bits)."""
    scene = synth.make_scene(200, 12, synth.VOL_C1, d_sem=8)
    rng = np.random.default_rng(520)
    cams = []
    for v in range(520):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        Rv, tv = synth.look_at(tuple(np.array([0.0, 0.0, 4.0]) + 6.0 * u), target=(0.0, 0.0, 4.0))
        w, h = 16 + v % 5, 12 + v % 3
        cams.append(synth.Camera(w, h, 18.0, 18.0, w / 2, h / 2, Rv, tv))
    G = 200 * len(cams)
    gpass = (32 + int(np.ceil(np.log2(len(cams)))) + 7) // 8
    assert int(np.ceil(np.log2(G))) + 8 * gpass > 64
    full_check(R, scene, cams, tile=8, batch=64)


def test_uncommon_channel_counts(R):
    for d_sem in (0, 5, 16, 30):
        scene = synth.make_scene(3000, 13 + d_sem, synth.VOL_C1, d_sem=d_sem)
        cams = [synth.camera_front(64, 48, 64.0)]
        full_check(R, scene, cams, tile=16, batch=64)


def test_degenerate_scenes(R):
    # everything behind the camera, or nothing at all touches the image
    scene = synth.make_scene(500, 14, synth.VOL_C1, d_sem=2)
    scene.mean[:, 2] = -3.0
    cams = [synth.camera_front(64, 64, 64.0)]
    stats = full_check(R, scene, cams)
    assert stats["pixels"] == 64 * 64
    # a single anisotropic Gaussian (an isotropic one has an identically zero
    # quaternion gradient, leaving nothing but rounding to compare)
    one = synth.make_scene(1, 15, synth.VOL_C1, d_sem=3)
    one.mean[0] = (0.0, 0.0, 3.0)
    one.log_scale[0] = (-1.2, -1.9, -1.5)
    full_check(R, one, cams)


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_c2_forward_backward_and_fd(R):
    scene, cams = synth.workload_c2()
    o = R.opts(tile=16, lds_batch=256)
    oo = PT.oracle_opts(o)
    note("c2 forward")
    rast, d, proj, bins, out, T, last = run_forward(R, scene, cams, o)
    fwd = O.forward(scene, cams, oo)
    PT.compare_projection(proj, fwd, scene.n)
    PT.compare_bins(bins, fwd)
    masks, stats = PT.compare_render(out, T, last, scene, cams, oo, fwd)
    note(f"c2 render stats {stats}")
    G = synth.upstream_grads(cams, scene.n_channels, 202)
    note("c2 backward")
    grad2d, g, d_ch = run_backward(R, rast, d, proj, bins, T, last, G)
    ref = O.backward(scene, cams, oo, fwd, G.astype(np.float64), flip_masks=masks, magnitudes=True, mag_cond=PT.MAG_COND)
    gg = PT.gpu_grads_to_np(g, d_ch)
    worst = PT.compare_grads(gg, ref, scene.n, mag=ref["mag"])
    note(f"c2 gradient worst ratios {worst}")
    # central finite differences on 64 seeded Gaussians blended somewhere: 8
    # outside the guard band (Jacobian at the clamped point), 8 with radius in
    # (40, 100] px, 48 with radius <= 40 px
    ids = fd.blended_gaussians(ref)
    P = fwd["proj"][0]
    rng = np.random.default_rng(302)
    clamped = ids[(P["clampx"][ids] == 1) | (P["clampy"][ids] == 1)]
    clamped = clamped[np.argsort(P["radius"][clamped], kind="stable")][:24]
    large = ids[(P["radius"][ids] > 40) & (P["radius"][ids] <= 100)]
    small = ids[(P["radius"][ids] <= 40)]
    assert len(clamped) >= 8 and len(large) >= 8
    sel = np.concatenate([rng.choice(clamped, 8, replace=False), rng.choice(large, 8, replace=False),
                          rng.choice(small, 48, replace=False)])
    n_valid = 0
    for k, gidx in enumerate(sel):
        if k % 4 == 0:
            note(f"c2 fd gaussian {k}/64 (radius {P['radius'][gidx]:.0f}, guard-band clamp "
                 f"{bool(P['clampx'][gidx] or P['clampy'][gidx])})")
        r = fd.fd_gaussian(fwd["params"], scene.channels, cams, oo, fwd["proj"], G.astype(np.float64), gidx)
        for grp in PT.GROUPS:
            vals, ok = r[grp]
            a = gg[grp].reshape(scene.n, -1)[gidx][ok]
            rms = np.sqrt(np.mean(ref[grp][ids] ** 2))
            err = np.linalg.norm(a - vals[ok])
            bound = 1e-3 * max(np.linalg.norm(vals[ok]), PT.group_floor(grp) * rms)
            assert err <= bound, (int(gidx), grp, err, bound)
            n_valid += int(ok.sum())
    note(f"c2 fd entries checked {n_valid}")
    assert n_valid >= 64 * 20


def alpha_clamp_scene(seed=23):
    """C1 plus 120 Gaussians in front of it (z = 1.75, nearer than every C1
    Gaussian) whose means project onto pixel centres and whose opacities
    exceed alpha_max (logits in [5, 9]): at and near those centres alpha is
    clamped to 0.99, the front Gaussian leaves T = 0.01, and stacked ones reach
    the stop rule right at its threshold."""
    base, cams = synth.workload_c1()
    rng = np.random.default_rng(seed)
    n = 120
    cam = cams[0]
    i = rng.integers(6, cam.width - 6, n)
    j = rng.integers(6, cam.height - 6, n)
    z = np.full(n, 1.75)
    mean = np.stack([(i + 0.5 - cam.cx) / cam.fx * z, (j + 0.5 - cam.cy) / cam.fy * z, z], 1)
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    special = synth.Scene(mean.astype(np.float32), rng.uniform(-3.0, -2.0, (n, 3)).astype(np.float32),
                          q.astype(np.float32), rng.uniform(5.0, 9.0, n).astype(np.float32),
                          base.channels[:n].copy(), base.d_sem)
    both = synth.Scene(*(np.concatenate([getattr(special, k), getattr(base, k)])
                         for k in ("mean", "log_scale", "quat", "opacity_logit", "channels")), base.d_sem)
    return both, cams, i, j


def test_alpha_clamp_scene(R):
    """Forward and backward parity where alpha is clamped to alpha_max (the
    forward's clamp and the backward's gate that stops the chain through a
    clamped alpha), against the oracle."""
    scene, cams, i, j = alpha_clamp_scene()
    oo = PT.oracle_opts(R.opts())
    fwd = O.forward(scene, cams, oo)
    T = fwd["views"][0]["T"]
    centre = j * cams[0].width + i
    # the oracle clamps at the centres: one front Gaussian leaves T <= 0.01
    assert (T[centre] <= 0.01 * (1 + 1e-9)).mean() > 0.9
    for tile, batch in ((16, 256), (32, 256), (8, 64)):
        stats = full_check(R, scene, cams, tile=tile, batch=batch)
        note(f"alpha clamp tile={tile}: {stats}")


@pytest.mark.timeout(900)
def test_target_1m_1080p(R):
    """The benchmark's own workload and launch setting (1M Gaussians, one
    1920x1080 view, 32-pixel tiles, LDS batch 256) against the oracle:
    projection and tile lists bit-exact, images, T and last within 1e-4 under
    the ambiguity rule, per-G-view screen-space and per-Gaussian gradients
    within the gradient bound."""
    scene, cams = synth.workload_1m_1080p()
    stats = full_check(R, scene, cams, tile=32, batch=256)
    note(f"1m@1080p: {stats}")
    assert stats["pixels"] == 1920 * 1080


def test_autograd_two_renders_one_loss(R):
    """Two renders through the autograd function before one backward (two
    scenes' images in one loss): each call keeps its own tile lists, so both
    gradients match the oracle."""
    cams = [synth.camera_front(96, 80, 96.0)]
    o = R.opts(tile=16, lds_batch=128)
    rast = R.Rasterizer(cams, o)
    oo = PT.oracle_opts(o)
    scenes = [synth.make_scene(3000, 71 + k, synth.VOL_C1, d_sem=8) for k in range(2)]
    params, outs = [], []
    for sc in scenes:
        p = {k: v.clone().requires_grad_(True) for k, v in PT.to_dev(sc).items()}
        out, _ = R.rasterize(p["mean"], p["log_scale"], p["quat"], p["opacity_logit"], p["channels"], rast)
        params.append(p)
        outs.append(out)
    Gs = [synth.upstream_grads(cams, scenes[0].n_channels, 230 + k) for k in range(2)]
    loss = sum((out * torch.from_numpy(G).cuda()).sum() for out, G in zip(outs, Gs))
    loss.backward()
    torch.cuda.synchronize()
    for sc, p, out, G in zip(scenes, params, outs, Gs):
        fwd = O.forward(sc, cams, oo)
        # the outputs must be those of each scene (the second render did not
        # overwrite what the first one's backward reads)
        _, _, _, _, o2, T2, l2 = run_forward(R, sc, cams, o)
        assert torch.equal(out.detach(), o2)
        masks, _ = PT.compare_render(o2, T2, l2, sc, cams, oo, fwd)
        ref = O.backward(sc, cams, oo, fwd, G.astype(np.float64), flip_masks=masks, magnitudes=True, mag_cond=PT.MAG_COND)
        got = {k: p[k].grad.cpu().numpy().astype(np.float64) for k in ("mean", "log_scale", "quat", "opacity_logit")}
        got["channels"] = p["channels"].grad.cpu().numpy().astype(np.float64)
        PT.compare_grads(got, ref, sc.n, mag=ref["mag"])


def test_tile_and_batch_invariance(R):
    """Images and final transmittance are bit-identical for every tile size and
    LDS batch size (the per-pixel box rule makes them tile-free)."""
    scene = synth.make_scene(50_000, 16, synth.VOL_C2, d_sem=8)
    cams = [synth.camera_front(333, 250, 300.0)]
    ref = None
    for tile in (8, 16, 32):
        for batch in (64, 128, 256):
            note(f"invariance tile={tile} batch={batch}")
            _, _, _, _, out, T, _ = run_forward(R, scene, cams, R.opts(tile=tile, lds_batch=batch))
            cur = (out.cpu().numpy(), T.cpu().numpy())
            if ref is None:
                ref = cur
            else:
                assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1])


def test_reach_cut_changes_no_result(R):
    """Skipping the pixels outside the reach of alpha_min changes nothing:
    images, final transmittance and last index are bit-identical to
    evaluating the whole 3-sigma box (LEGS_FLAG_FULL_BOX), gradients agree to
    float32 summation order, on a scene with near-threshold and transparent
    opacities and strongly elongated Gaussians; only the work counts drop."""
    scene = synth.make_scene(30_000, 19, synth.VOL_C2, d_sem=8)
    scene.opacity_logit[::7] = -6.5                 # opacity 0.0015 < alpha_min
    scene.opacity_logit[3::7] = -5.52               # opacity just above alpha_min
    scene.log_scale[::5, 0] += 2.0                  # needles
    scene.log_scale[1::5, 1] -= 1.5
    cams = [synth.camera_front(320, 240, 300.0), synth.camera_front(150, 110, 140.0)]
    G = synth.upstream_grads(cams, scene.n_channels, 210)
    res = {}
    for full in (False, True):
        note(f"reach cut full_box={full}")
        o = R.opts(full_box=full)
        rast, d, proj, bins, out, T, last = run_forward(R, scene, cams, o)
        grad2d, g, d_ch = run_backward(R, rast, d, proj, bins, T, last, G)
        counts = R.render_counts(rast.ctx, proj, bins, rast.views, o)
        res[full] = (out.cpu().numpy(), T.cpu().numpy(), last.cpu().numpy(), PT.gpu_grads_to_np(g, d_ch), counts)
    a, b = res[False], res[True]
    for i in range(3):
        assert np.array_equal(a[i], b[i])
    for k in a[3]:
        x, y = a[3][k], b[3][k]
        scale = np.abs(y).max() + 1e-30
        assert np.abs(x - y).max() <= 1e-4 * scale, k
    note(f"counts reach {a[4]} full box {b[4]}")
    assert a[4][1] == b[4][1] and a[4][3] == b[4][3]
    assert a[4][0] < 0.9 * b[4][0] and a[4][2] < 0.9 * b[4][2]


def test_determinism_and_permutation(R):
    scene = synth.make_scene(40_000, 17, synth.VOL_C2, d_sem=8)
    cams = [synth.camera_front(300, 200, 280.0)]
    o = R.opts()
    _, _, _, _, out1, T1, l1 = run_forward(R, scene, cams, o)
    _, _, _, _, out2, T2, l2 = run_forward(R, scene, cams, o)
    assert torch.equal(out1, out2) and torch.equal(T1, T2) and torch.equal(l1, l2)
    perm = np.random.default_rng(3).permutation(scene.n)
    _, _, _, _, out3, T3, l3 = run_forward(R, scene.subset(perm), cams, o)
    assert torch.equal(out1, out3) and torch.equal(T1, T3) and torch.equal(l1, l3)


def test_capacity_overflow_is_reported(R):
    from paper_2311_18482_amd import _lib as L
    scene, cams = synth.workload_c1()
    o = R.opts()
    rast = R.Rasterizer(cams, o)
    d = PT.to_dev(scene)
    proj = R.project(rast.ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"], rast.views, o)
    small = R.BinsBuf(1000, rast.views.total_tiles, d["mean"].device)
    import ctypes as ct
    cnt = ct.c_int64(0)
    ps, bs = proj.struct(), small.struct()
    code = L.lib().legs_bin_sort(rast.ctx.handle, ct.byref(ps), scene.n, R._p(rast.views.dev), 1,
                                 rast.views.total_tiles, ct.byref(o), ct.byref(bs), ct.byref(cnt),
                                 R._stream())
    assert code == L.LEGS_ERR_CAPACITY and cnt.value > 1000
    # without the host read-back, kernels truncate to the capacity and flag it on device
    code = L.lib().legs_bin_sort(rast.ctx.handle, ct.byref(ps), scene.n, R._p(rast.views.dev), 1,
                                 rast.views.total_tiles, ct.byref(o), ct.byref(bs), None, R._stream())
    assert code == L.LEGS_OK
    torch.cuda.synchronize()
    assert int(small.count.item()) == cnt.value
    # the wrapper grows its buffers and gets the exact lists
    bins = R.bin_sort(rast.ctx, proj, rast.views, o, small)
    assert bins.n_instances == cnt.value and bins.capacity >= cnt.value


def test_invalid_arguments(R):
    from paper_2311_18482_amd import _lib as L
    import ctypes as ct
    scene, cams = synth.workload_c1()
    rast = R.Rasterizer(cams, R.opts())
    d = PT.to_dev(scene)
    bad = R.opts(tile=12)
    proj = R.ProjectedBuf(scene.n, 1, d["mean"].device)
    ps = proj.struct()
    code = L.lib().legs_project(rast.ctx.handle, R._p(d["mean"]), R._p(d["log_scale"]),
                                R._p(d["quat"]), R._p(d["opacity_logit"]), scene.n,
                                R._p(rast.views.dev), 1, ct.byref(bad), ct.byref(ps), R._stream())
    assert code == L.LEGS_ERR_ARG
    assert b"tile" in L.lib().legs_last_error(rast.ctx.handle)
    code = L.lib().legs_project(rast.ctx.handle, None, R._p(d["log_scale"]), R._p(d["quat"]),
                                R._p(d["opacity_logit"]), scene.n, R._p(rast.views.dev), 1,
                                ct.byref(rast.o), ct.byref(ps), R._stream())
    assert code == L.LEGS_ERR_ARG


def test_autograd_function(R):
    scene, cams = synth.workload_c1()
    rast = R.Rasterizer(cams, R.opts())
    d = PT.to_dev(scene)
    params = {k: v.clone().requires_grad_(True) for k, v in d.items()}
    out, T = R.rasterize(params["mean"], params["log_scale"], params["quat"],
                         params["opacity_logit"], params["channels"], rast)
    G = torch.from_numpy(synth.upstream_grads(cams, scene.n_channels, 203)).cuda()
    (out * G).sum().backward()
    _, _, proj, bins, _, T2, last = run_forward(R, scene, cams, rast.o)
    grad2d, g, d_ch = run_backward(R, rast, d, proj, bins, T2, last, G.cpu().numpy())
    # same kernels, float atomics in a different order
    got = {k: params[k].grad.cpu().numpy().astype(np.float64) for k in ("mean", "log_scale", "quat", "opacity_logit")}
    got["channels"] = params["channels"].grad.cpu().numpy().astype(np.float64)
    PT.compare_grads(got, PT.gpu_grads_to_np(g, d_ch), scene.n, tol=1e-4)


@pytest.mark.parametrize("persistent", [False, True])
def test_forward_zero_matches_and_zeroes(R, persistent):
    """legs_render_forward_zero composites exactly like legs_render_forward
    (out, T and last bit-identical, one workgroup per tile and persistent) and
    sets the whole given range to 0 (a float count that leaves a 3-float tail
    after the float4 stores), nothing past it; it rejects a misaligned range
    and a byte count that is not a multiple of 4."""
    scene, cams = synth.workload_c1()
    o = R.opts(tile=32, lds_batch=128, persistent=persistent)
    rast, d, proj, bins, out, T, last = run_forward(R, scene, cams, o)
    n_zero = 1_000_003
    buf = torch.full((n_zero + 8,), 7.0, device="cuda")
    out2, T2, last2 = (torch.full_like(out, -1.0), torch.full_like(T, -1.0), torch.full_like(last, -1))
    R.render_forward(rast.ctx, proj, bins, rast.views, d["channels"], o, out2, T2, last2, zero=buf[:n_zero])
    torch.cuda.synchronize()
    assert torch.equal(out2, out) and torch.equal(T2, T) and torch.equal(last2, last)
    assert (buf[:n_zero] == 0.0).all() and (buf[n_zero:] == 7.0).all()
    with pytest.raises(RuntimeError):
        R.render_forward(rast.ctx, proj, bins, rast.views, d["channels"], o, out2, T2, last2, zero=buf[1:101])
    with pytest.raises(RuntimeError):
        R.render_forward(rast.ctx, proj, bins, rast.views, d["channels"], o, out2, T2, last2,
                         zero=buf.view(torch.uint8)[:7])
    torch.cuda.synchronize()
    assert (buf[n_zero:] == 7.0).all()


def test_persistent_launch_matches(R):
    """One persistent launch over the tiles of several uneven views gives the
    same images, T and last as one workgroup per tile (bit for bit: each pixel
    runs the same arithmetic), and both launches' gradients match the oracle
    within the gradient bound (their float32 sums are taken in different
    orders, so they are compared with the exact result, not with each other)."""
    scene = synth.make_scene(60_000, 18, synth.VOL_CUBE, d_sem=8)
    cams = synth.cameras_sphere(4, 118, 8.0, ((320, 240), (200, 150), (480, 270)))
    G = synth.upstream_grads(cams, scene.n_channels, 218)
    res = []
    for persistent in (False, True):
        note(f"persistent={persistent}")
        o = R.opts(persistent=persistent)
        rast, d, proj, bins, out, T, last = run_forward(R, scene, cams, o)
        grad2d, g, d_ch = run_backward(R, rast, d, proj, bins, T, last, G)
        res.append((out.clone(), T.clone(), last.clone(), PT.gpu_grads_to_np(g, d_ch)))
    assert torch.equal(res[0][0], res[1][0]) and torch.equal(res[0][1], res[1][1])
    assert torch.equal(res[0][2], res[1][2])
    oo = PT.oracle_opts(o)
    fwd = O.forward(scene, cams, oo)
    masks, stats = PT.compare_render(res[1][0], res[1][1], res[1][2], scene, cams, oo, fwd)
    ref = O.backward(scene, cams, oo, fwd, G.astype(np.float64), flip_masks=masks, magnitudes=True,
                     mag_cond=PT.MAG_COND)
    for persistent in (False, True):
        worst = PT.compare_grads(res[int(persistent)][3], ref, scene.n, mag=ref["mag"])
        note(f"persistent={persistent}: {stats} {worst}")


def test_graph_replay(R):
    """A captured forward + backward step replays to the eager result, with
    eager work and synchronisation between replays."""
    scene = synth.make_scene(50_000, 19, synth.VOL_CUBE, d_sem=8)
    cams = synth.cameras_sphere(3, 119, 8.0, ((256, 192), (320, 180), (200, 200)))
    o = R.opts(persistent=True)
    rast = R.Rasterizer(cams, o)
    d = PT.to_dev(scene)
    n, C = scene.channels.shape
    views = rast.views
    proj = R.project(rast.ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"], views, o)
    bins = R.bin_sort(rast.ctx, proj, views, o)
    bins = R.BinsBuf(bins.n_instances + 4096, views.total_tiles, d["mean"].device)
    out = torch.empty(C * views.total_pixels, device="cuda")
    T = torch.empty(views.total_pixels, device="cuda")
    last = torch.empty(views.total_pixels, dtype=torch.int32, device="cuda")
    G = torch.from_numpy(synth.upstream_grads(cams, C, 219)).cuda()
    grad2d = torch.zeros((n * views.n_views, 8), device="cuda")
    d_ch = torch.zeros((n, C), device="cuda")
    grads = {k: torch.zeros_like(d[k]) for k in ("mean", "log_scale", "quat", "opacity_logit")}

    def step():
        R.project(rast.ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"], views, o, out=proj)
        R.bin_sort(rast.ctx, proj, views, o, bins, sync_count=False)
        R.render_forward(rast.ctx, proj, bins, views, d["channels"], o, out, T, last)
        grad2d.zero_()
        d_ch.zero_()
        for t in grads.values():
            t.zero_()
        R.render_backward(rast.ctx, proj, bins, views, d["channels"], o, T, last, G, grad2d, d_ch)
        R.project_backward(rast.ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"],
                           views, o, proj, grad2d, grads)

    step()
    torch.cuda.synchronize()
    ref = (out.clone(), T.clone(), last.clone(), d_ch.clone(), {k: v.clone() for k, v in grads.items()})
    g = R.Graph(rast.ctx)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with g.capture():
            step()
    torch.cuda.current_stream().wait_stream(side)
    for rep in range(4):
        out.fill_(-1.0)
        T.fill_(-1.0)
        d_ch.fill_(123.0)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        note(f"graph replay {rep}")
        assert torch.equal(out, ref[0]) and torch.equal(T, ref[1]) and torch.equal(last, ref[2])
        # float atomics accumulate in a different order on every run
        got = {k: v.cpu().numpy().astype(np.float64) for k, v in grads.items()}
        got["channels"] = d_ch.cpu().numpy().astype(np.float64)
        want = {k: v.cpu().numpy().astype(np.float64) for k, v in ref[4].items()}
        want["channels"] = ref[3].cpu().numpy().astype(np.float64)
        PT.compare_grads(got, want, n, tol=1e-4)


def graph_replays_match_oracle(R, scene, cams, o, reps, seed_g):
    """Captures one forward + backward step (project, bin, blend forward,
    gradient clear, blend backward, project backward) as a HIP graph and
    replays it reps times with eager work and synchronisation in between;
    every replay matches the oracle (lists bit-exact, images, T and last
    under the ambiguity rule, per-Gaussian gradients within the gradient
    bound)."""
    oo = PT.oracle_opts(o)
    rast = R.Rasterizer(cams, o)
    d = PT.to_dev(scene)
    n, C = scene.channels.shape
    views = rast.views
    proj = R.project(rast.ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"], views, o)
    sized = R.bin_sort(rast.ctx, proj, views, o)
    bins = R.BinsBuf(sized.n_instances + 4096, views.total_tiles, d["mean"].device)
    del sized
    out = torch.empty(C * views.total_pixels, device="cuda")
    T = torch.empty(views.total_pixels, device="cuda")
    last = torch.empty(views.total_pixels, dtype=torch.int32, device="cuda")
    G = synth.upstream_grads(cams, C, seed_g)
    Gd = torch.from_numpy(G).cuda()
    gflat = torch.zeros(n * views.n_views * 8 + n * (C + 11), device="cuda")
    grad2d = gflat[:n * views.n_views * 8].view(-1, 8)
    rest = gflat[n * views.n_views * 8:]
    d_ch = rest[:n * C].view(n, C)
    grads = {"mean": rest[n * C:n * (C + 3)].view(n, 3), "log_scale": rest[n * (C + 3):n * (C + 6)].view(n, 3),
             "quat": rest[n * (C + 6):n * (C + 10)].view(n, 4), "opacity_logit": rest[n * (C + 10):]}

    def step():
        R.project(rast.ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"], views, o, out=proj)
        R.bin_sort(rast.ctx, proj, views, o, bins, sync_count=False)
        R.render_forward(rast.ctx, proj, bins, views, d["channels"], o, out, T, last)
        R.clear(rast.ctx, gflat)
        R.render_backward(rast.ctx, proj, bins, views, d["channels"], o, T, last, Gd, grad2d, d_ch)
        R.project_backward(rast.ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"],
                           views, o, proj, grad2d, grads)

    g = R.Graph(rast.ctx)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with g.capture():
            step()
    torch.cuda.current_stream().wait_stream(side)
    fwd = O.forward(scene, cams, oo)
    ref = None
    for rep in range(reps):
        out.fill_(-1.0)
        T.fill_(-1.0)
        d_ch.fill_(123.0)
        torch.cuda.synchronize()
        g.launch()
        torch.cuda.synchronize()
        note(f"{len(cams)}-view graph replay {rep} (tile {o.tile}, batch {o.lds_batch}, flags {o.flags})")
        PT.compare_bins(bins, fwd, ids_only=bool(o.flags & R.L.LEGS_FLAG_IDS_ONLY))
        masks, stats = PT.compare_render(out, T, last, scene, cams, oo, fwd)
        if ref is None:
            ref = O.backward(scene, cams, oo, fwd, G.astype(np.float64), flip_masks=masks, magnitudes=True,
                             mag_cond=PT.MAG_COND)
        got = PT.gpu_grads_to_np(grads, d_ch)
        worst = PT.compare_grads(got, ref, n, mag=ref["mag"])
        note(f"replay {rep}: {stats} {worst}")


def test_persistent_graph_six_views_matches_oracle(R):
    """A captured forward + backward step over 6 views of uneven resolution
    with both blend kernels launched persistently (one queue of every view's
    tiles, heaviest first), replayed several times: every replay matches the
    oracle."""
    scene = synth.make_scene(60_000, 24, synth.VOL_CUBE, d_sem=8)
    sizes = ((320, 240), (200, 150), (480, 270), (256, 256), (160, 120), (400, 300))
    cams = synth.cameras_sphere(6, 124, 8.0, (320, 240))
    for c, (w, h) in zip(cams, sizes):
        c.width, c.height, c.fx, c.fy, c.cx, c.cy = w, h, float(w), float(w), w / 2.0, h / 2.0
    graph_replays_match_oracle(R, scene, cams, R.opts(tile=16, lds_batch=128, persistent=True), 3, 224)


@pytest.mark.timeout(1200)
def test_c3_sixteen_views_autotuned_persistent_graph(R):
    """The 16-view batch as the bench times it: 1M Gaussians, 16 views of
    uneven resolution on the r=8 sphere, the autotuner's choice of tile and
    LDS batch, both blend kernels persistent, ids-only binning, the step
    captured and replayed: every replay against the oracle."""
    scene, cams = synth.workload_c3()
    d = PT.to_dev(scene)
    G = torch.from_numpy(synth.upstream_grads(cams, scene.n_channels, 203)).cuda()
    ctx = R.Context(0)
    best, table = R.autotune(ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"], d["channels"], cams,
                             R.opts(persistent=True, ids_only=True), d_out=G, reps=1)
    del d, G
    torch.cuda.empty_cache()
    note(f"c3 autotune: best tile {best.tile} batch {best.lds_batch}")
    o = R.opts(tile=best.tile, lds_batch=best.lds_batch, persistent=True, ids_only=True)
    graph_replays_match_oracle(R, scene, cams, o, 2, 203)


def test_autotune_returns_a_valid_setting(R):
    scene = synth.make_scene(40_000, 20, synth.VOL_CUBE, d_sem=8)
    cams = synth.cameras_sphere(2, 120, 8.0, ((320, 240), (256, 256)))
    d = PT.to_dev(scene)
    G = torch.from_numpy(synth.upstream_grads(cams, scene.n_channels, 220)).cuda()
    ctx = R.Context(0)
    best, times = R.autotune(ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"],
                             d["channels"], cams, R.opts(persistent=True), d_out=G, reps=2)
    note(f"autotune {best.tile} {best.lds_batch} {times}")
    assert best.tile in (8, 16, 32) and best.lds_batch in (64, 128, 256)
    assert all(t > 0 for t in times.values())
    assert times[(best.tile, best.lds_batch)] == min(times.values())


def _super_tiles(cams, tile):
    n = 0
    for c in cams:
        tx, ty = (c.width + tile - 1) // tile, (c.height + tile - 1) // tile
        n += ((tx + 7) // 8) * ((ty + 3) // 4)
    return n


@pytest.mark.parametrize("rig", ["small", "wide"])
def test_depth_first_and_full_sort_lists_identical(R, rig):
    """Sorting the depth digits per G-view before expansion gives the same
    instance lists as sorting all eight key digits over the instances. The
    small rig has at most 256 super-tiles (one coarse pass), the wide one
    more (two coarse passes)."""
    scene = synth.make_scene(80_000, 21, synth.VOL_CUBE, d_sem=8)
    if rig == "small":
        cams = synth.cameras_sphere(3, 121, 8.0, ((320, 240), (640, 360), (200, 150)))
        assert _super_tiles(cams, 8) <= 256 and _super_tiles(cams, 16) <= 256
    else:
        cams = synth.cameras_sphere(4, 121, 8.0, ((320, 240), (640, 360), (200, 150), (1280, 720)))
        assert _super_tiles(cams, 8) > 256 and _super_tiles(cams, 16) > 256
    lists = []
    for full in (False, True):
        for tile in (8, 16):
            note(f"rig={rig} full_sort={full} tile={tile}")
            o = R.opts(tile=tile, full_sort=full)
            rast, d, proj, bins, out, T, last = run_forward(R, scene, cams, o)
            n_inst = int(bins.count.item())
            lists.append((tile, bins.keys[:n_inst].cpu().numpy(), bins.ids[:n_inst].cpu().numpy(),
                          bins.ranges.cpu().numpy(), out.cpu().numpy()))
            if not full and tile == 16:
                fwd = O.forward(scene, cams, PT.oracle_opts(o))
                PT.compare_bins(bins, fwd)
    for a, b in zip(lists[:2], lists[2:]):
        assert a[0] == b[0]
        for x, y in zip(a[1:], b[1:]):
            assert np.array_equal(x, y)
    # ids only: the same lists, ranges and images; the keys left as they were
    for tile, keys, ids, ranges, img in lists[:2]:
        note(f"rig={rig} ids_only tile={tile}")
        o = R.opts(tile=tile, ids_only=True)
        rast, d, proj, bins, out, T, last = run_forward(R, scene, cams, o)
        n_inst = int(bins.count.item())
        assert n_inst == len(ids)
        assert np.array_equal(bins.ids[:n_inst].cpu().numpy(), ids)
        assert np.array_equal(bins.ranges.cpu().numpy(), ranges)
        assert np.array_equal(out.cpu().numpy(), img)
        bins.keys.fill_(0x5A5A5A5A5A5A5A5A)
        R.bin_sort(rast.ctx, proj, rast.views, o, bins)
        torch.cuda.synchronize()
        assert (bins.keys == 0x5A5A5A5A5A5A5A5A).all()
        assert np.array_equal(bins.ids[:n_inst].cpu().numpy(), ids)


def _expected_counts(proj_v, cam, ids, ranges, tile_offset, tile, amin, amax, tmin):
    """Per-pixel walk of the tile lists in FP64 (numpy over the pixels of one
    tile at a time): alpha evaluations of the forward, blended entries, alpha
    evaluations of the backward and list positions walked, with evaluations
    counted inside the box, and inside the box cut to the bounding box of the
    ellipse where opacity * exp(power) >= alpha_min (the reach)."""
    tx_n = (cam.width + tile - 1) // tile
    ty_n = (cam.height + tile - 1) // tile
    tot = np.zeros(4)
    reach = np.zeros(4)
    for t in range(tx_n * ty_n):
        s, e = ranges[tile_offset + t]
        if e <= s:
            continue
        g = ids[s:e].astype(np.int64)
        p = proj_v[g]
        x0, y0 = (t % tx_n) * tile, (t // tx_n) * tile
        xs, ys = np.meshgrid(np.arange(x0, min(x0 + tile, cam.width)),
                             np.arange(y0, min(y0 + tile, cam.height)))
        px, py = xs.reshape(-1, 1), ys.reshape(-1, 1)
        inbox = ((p["valid"] != 0) & (px >= p["x0"]) & (px <= p["x1"]) & (py >= p["y0"])
                 & (py <= p["y1"]))
        dx, dy = p["mx"] - (px + 0.5), p["my"] - (py + 0.5)
        # A dx^2 + 2 B dx dy + C dy^2 <= K, K = 2 ln(opacity / alpha_min): its
        # bounding box has half widths sqrt(K C / det) and sqrt(K A / det)
        K = 2.0 * np.log(np.maximum(p["sig"], 1e-300) / amin)
        det = p["A"] * p["C"] - p["B"] ** 2
        with np.errstate(invalid="ignore", divide="ignore"):
            hw = np.sqrt(np.maximum(K, 0.0) * p["C"] / det)
            hh = np.sqrt(np.maximum(K, 0.0) * p["A"] / det)
        inreach = inbox & (K >= 0.0) & (np.abs(dx) <= hw) & (np.abs(dy) <= hh)
        power = np.minimum(-0.5 * (p["A"] * dx * dx + p["C"] * dy * dy) - p["B"] * dx * dy, 0.0)
        alpha = np.minimum(p["sig"] * np.exp(power), amax)
        blend = inbox & (alpha >= amin)
        f = np.where(blend, 1.0 - alpha, 1.0)
        T_before = np.concatenate([np.ones((len(px), 1)), np.cumprod(f, axis=1)[:, :-1]], axis=1)
        stop = blend & (T_before * (1.0 - alpha) < tmin)
        L = len(g)
        has = stop.any(axis=1)
        k_stop = np.where(has, stop.argmax(axis=1), L)          # position of the stop (or L)
        pos = np.arange(L)[None, :]
        before_stop = pos < k_stop[:, None]
        blended = blend & before_stop
        last = np.where(blended.any(axis=1), L - 1 - np.argmax(blended[:, ::-1], axis=1), -1)
        tot[0] += (inbox & (pos <= k_stop[:, None])).sum()
        tot[1] += blended.sum()
        tot[2] += (inbox & (pos <= last[:, None])).sum()
        tot[3] += np.minimum(k_stop + 1, L).sum()
        reach[0] += (inreach & (pos <= k_stop[:, None])).sum()
        reach[2] += (inreach & (pos <= last[:, None])).sum()
    reach[1], reach[3] = tot[1], tot[3]
    return tot, reach


def test_render_counts_match_a_per_pixel_walk(R):
    """The work counts behind the blend kernels' ALU roofline against a plain
    per-pixel walk of the same lists (FP64; up to the rare decisions that FP32
    and FP64 take differently): blended entries and list positions are equal;
    alpha evaluations, which the kernels skip outside the reach of alpha_min,
    lie between the walk's counts inside the exact reach and inside the full
    box, and within 3 % of the former (the reach is widened for rounding)."""
    scene = synth.make_scene(20_000, 31, synth.VOL_C1, d_sem=8)
    cams = [synth.camera_front(256, 192, 240.0), synth.camera_front(200, 150, 190.0)]
    for tile in (8, 16):
        note(f"render_counts tile={tile}")
        o = R.opts(tile=tile)
        rast, d, proj, bins, out, T, last = run_forward(R, scene, cams, o)
        counts = R.render_counts(rast.ctx, proj, bins, rast.views, o)
        fwd = O.forward(scene, cams, PT.oracle_opts(o))
        box, reach = np.zeros(4), np.zeros(4)
        for v, cam in enumerate(cams):
            b_, r_ = _expected_counts(fwd["proj"][v], cam, fwd["ids"], fwd["ranges"],
                                      fwd["offsets"][v], tile, o.alpha_min, o.alpha_max, o.t_min)
            box += b_
            reach += r_
        note(f"counts {counts} reach {reach.tolist()} box {box.tolist()}")
        assert reach[1] > 0 and reach[0] >= reach[2] >= reach[1]
        assert box[0] > 1.2 * reach[0]              # the cut matters on this scene
        for q in (1, 3):
            assert abs(counts[q] - reach[q]) <= 1e-4 * reach[q] + 2, (counts, reach)
        for q in (0, 2):
            tol = 1e-4 * reach[q] + 2
            assert reach[q] - tol <= counts[q] <= min(box[q], 1.03 * reach[q]) + tol, (counts, reach, box)


def _truncated_lists(fwd, cams, tile, n, capacity):
    """The first `capacity` instances of the depth-ordered stream (G-views by
    (view, depth bits), ties by Gaussian; each G-view's tiles row-major),
    stably sorted by tile: keys, ids and ranges, from the oracle projection."""
    _, _, offsets, total_tiles = O.view_tables(cams, tile)
    recs = []
    for v, cam in enumerate(cams):
        p = fwd["proj"][v]
        txn = (cam.width + tile - 1) // tile
        bits = p["depth32"].view(np.uint32).astype(np.uint64)
        for g in np.nonzero(p["ntiles"] > 0)[0]:
            recs.append((v, int(bits[g]), int(g), txn, int(offsets[v])))
    recs.sort(key=lambda r: (r[0], r[1], r[2]))
    tiles, ids, dbits = [], [], []
    for v, db, g, txn, toff in recs:
        p = fwd["proj"][v][g]
        for ty in range(p["ty0"], p["ty1"] + 1):
            for tx in range(p["tx0"], p["tx1"] + 1):
                tiles.append(toff + ty * txn + tx)
                ids.append(g)
                dbits.append(db)
        if len(tiles) >= capacity:
            break
    tiles, ids, dbits = (np.array(a[:capacity], np.uint64) for a in (tiles, ids, dbits))
    order = np.argsort(tiles, kind="stable")
    keys = (tiles[order] << np.uint64(32)) | dbits[order]
    ranges = np.zeros((total_tiles, 2), np.int64)
    t_sorted = tiles[order].astype(np.int64)
    starts = np.searchsorted(t_sorted, np.arange(total_tiles), "left")
    ends = np.searchsorted(t_sorted, np.arange(total_tiles), "right")
    ranges[:, 0], ranges[:, 1] = starts, ends
    return keys, ids[order].astype(np.uint32), ranges


def test_truncated_lists_without_host_count(R):
    """Without the host read-back an overflowing binning keeps the first
    `capacity` instances of the depth-ordered stream, sorted by tile, with
    ranges inside the capacity (so the blend kernels stay in bounds)."""
    import ctypes as ct
    from paper_2311_18482_amd import _lib as L
    scene = synth.make_scene(3000, 41, synth.VOL_C1, d_sem=8)
    cams = [synth.camera_front(160, 120, 150.0), synth.camera_front(96, 80, 90.0)]
    for tile in (8, 16):
        o = R.opts(tile=tile)
        rast = R.Rasterizer(cams, o)
        d = PT.to_dev(scene)
        proj = R.project(rast.ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"],
                         rast.views, o)
        full = R.bin_sort(rast.ctx, proj, rast.views, o)
        total = full.n_instances
        fwd = O.forward(scene, cams, PT.oracle_opts(o))
        for cap in (total // 3, total - 7):
            note(f"truncated lists tile={tile} capacity={cap} of {total}")
            small = R.BinsBuf(cap, rast.views.total_tiles, d["mean"].device)
            ps, bs = proj.struct(), small.struct()
            code = L.lib().legs_bin_sort(rast.ctx.handle, ct.byref(ps), scene.n, R._p(rast.views.dev),
                                         len(cams), rast.views.total_tiles, ct.byref(o), ct.byref(bs),
                                         None, R._stream())
            assert code == L.LEGS_OK
            torch.cuda.synchronize()
            assert int(small.count.item()) == total
            keys, ids, ranges = _truncated_lists(fwd, cams, tile, scene.n, cap)
            assert np.array_equal(small.keys.cpu().numpy().view(np.uint64), keys)
            assert np.array_equal(small.ids.cpu().numpy().view(np.uint32), ids)
            assert np.array_equal(small.ranges.cpu().numpy().astype(np.int64), ranges)
