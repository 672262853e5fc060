"""Pins for the FP64 CPU oracle, checked against things other than itself:
closed forms, library routines (scipy rotations, numpy eigen/inverse, torch),
finite differences, brute force over all Gaussians, and invariants.

Rasteriser pins follow the renderer of Sec. 3.1 (Eq. 1) with the extra
semantic and uncertainty channels of Sec. 3.4; decoder pins follow Eq. 4 and
Eq. 8-9; Adam follows Sec. 4.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from oracle import decode as D
from oracle import fd
from oracle import oracle as O

H_LOWPASS = 0.3


def params1(mean, ls, q=(1, 0, 0, 0), omega=0.0):
    return O.Params(np.array([mean], float), np.array([ls], float), np.array([q], float),
                    np.array([omega], float))


def scene_from(mean, ls, q, omega, ch):
    return synth.Scene(np.asarray(mean, np.float32), np.asarray(ls, np.float32),
                       np.asarray(q, np.float32), np.asarray(omega, np.float32),
                       np.asarray(ch, np.float32), 0)


def pinhole(cam, t):
    return np.array([cam.fx * t[0] / t[2] + cam.cx, cam.fy * t[1] / t[2] + cam.cy])


def fd_jacobian(cam, t, h=1e-6):
    J = np.zeros((2, 3))
    for k in range(3):
        e = np.zeros(3)
        e[k] = h * max(1.0, abs(t[k]))
        J[:, k] = (pinhole(cam, t + e) - pinhole(cam, t - e)) / (2 * e[k])
    return J


def sigma3(ls, q):
    Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()   # scipy is scalar-last
    S = np.diag(np.exp(ls))
    return Rm @ S @ S.T @ Rm.T


# ---------------------------------------------------------------- projection

def test_isotropic_on_axis_closed_form(oracle_lib):
    cam = synth.camera_front(128, 128, 128.0)
    opts = O.make_opts(16)
    for z, ls in [(4.0, -2.0), (2.5, -3.0), (10.0, -1.0)]:
        p = O.project(params1((0, 0, z), (ls, ls, ls)), cam, opts)[0]
        s = np.exp(ls)
        want = (128.0 * s / z) ** 2 + H_LOWPASS
        assert p["valid"] == 1
        assert p["mx"] == 64.0 and p["my"] == 64.0
        assert p["a"] == pytest.approx(want, rel=1e-13)
        assert p["c"] == pytest.approx(want, rel=1e-13)
        assert abs(p["b"]) < 1e-15 * want
        assert p["A"] == pytest.approx(1 / want, rel=1e-13)
        assert p["depth32"] == np.float32(z)


def test_anisotropic_axis_aligned_and_z_rotation(oracle_lib):
    cam = synth.camera_front(200, 100, 150.0)
    cam.fy = 120.0
    opts = O.make_opts(16)
    ls = (-2.0, -1.5, -2.5)
    z = 5.0
    sx, sy = np.exp(ls[0]), np.exp(ls[1])
    p = O.project(params1((0, 0, z), ls), cam, opts)[0]
    assert p["a"] == pytest.approx((150.0 * sx / z) ** 2 + H_LOWPASS, rel=1e-13)
    assert p["c"] == pytest.approx((120.0 * sy / z) ** 2 + H_LOWPASS, rel=1e-13)
    # a 90 degree rotation about the optical axis swaps the screen axes
    q = (np.cos(np.pi / 4), 0.0, 0.0, np.sin(np.pi / 4))
    p2 = O.project(params1((0, 0, z), ls, q), cam, opts)[0]
    assert p2["a"] == pytest.approx((150.0 * sy / z) ** 2 + H_LOWPASS, rel=1e-12)
    assert p2["c"] == pytest.approx((120.0 * sx / z) ** 2 + H_LOWPASS, rel=1e-12)
    assert abs(p2["b"]) < 1e-12


def test_quaternion_sign_and_scale_invariance(oracle_lib):
    rng = np.random.default_rng(7)
    cam = synth.camera_front(128, 128, 128.0)
    opts = O.make_opts(16)
    for _ in range(20):
        mean = (rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(2, 6))
        ls = rng.normal(-2, 0.5, 3)
        q = rng.normal(size=4)
        ps = [O.project(params1(mean, ls, qq), cam, opts)[0] for qq in (q, -q, 2.5 * q)]
        for f in ("a", "b", "c", "A", "B", "C", "mx", "my"):
            assert ps[1][f] == pytest.approx(ps[0][f], rel=1e-12, abs=1e-14)
            assert ps[2][f] == pytest.approx(ps[0][f], rel=1e-12, abs=1e-14)


def test_covariance_matches_fd_jacobian_and_scipy_rotation(oracle_lib):
    """Sigma' = J W Sigma W^T J^T + h with J the numerical Jacobian of the
    pinhole map and Sigma built from scipy's rotation of the quaternion."""
    rng = np.random.default_rng(11)
    R, t = synth.look_at((3.0, -2.0, 7.0))
    cam = synth.Camera(640, 480, 600.0, 580.0, 320.0, 240.0, R, t)
    opts = O.make_opts(16)
    n_checked = 0
    for _ in range(40):
        mean = rng.uniform(-1.5, 1.5, 3)
        ls = rng.normal(-2, 0.5, 3)
        q = rng.normal(size=4)
        p = O.project(params1(mean, ls, q), cam, opts)[0]
        tc = R @ mean + t
        if not p["valid"] or p["clampx"] or p["clampy"]:
            continue
        J = fd_jacobian(cam, tc)
        S2 = J @ R @ sigma3(ls, q / np.linalg.norm(q)) @ R.T @ J.T
        assert p["a"] == pytest.approx(S2[0, 0] + H_LOWPASS, rel=1e-6)
        assert p["b"] == pytest.approx(S2[0, 1], rel=1e-6, abs=1e-6 * S2[0, 0])
        assert p["c"] == pytest.approx(S2[1, 1] + H_LOWPASS, rel=1e-6)
        m = pinhole(cam, tc)
        assert p["mx"] == pytest.approx(m[0], rel=1e-14)
        assert p["my"] == pytest.approx(m[1], rel=1e-14)
        inv = np.linalg.inv(np.array([[p["a"], p["b"]], [p["b"], p["c"]]]))
        assert np.allclose([p["A"], p["B"], p["C"]], [inv[0, 0], inv[0, 1], inv[1, 1]], rtol=1e-12)
        lam = np.linalg.eigvalsh(np.array([[p["a"], p["b"]], [p["b"], p["c"]]]))[-1]
        assert p["lam"] == pytest.approx(lam, rel=1e-12)
        n_checked += 1
    assert n_checked > 20


def test_covariance_monte_carlo(oracle_lib):
    """For a small Gaussian the projected covariance (minus the low-pass) equals
    the sample covariance of pinhole-projected 3D samples."""
    rng = np.random.default_rng(3)
    cam = synth.camera_front(512, 512, 500.0)
    opts = O.make_opts(16)
    mean = np.array([0.4, -0.3, 6.0])
    ls = np.array([-4.0, -4.6, -5.0])
    q = np.array([0.8, 0.3, -0.4, 0.2])
    p = O.project(params1(mean, ls, q), cam, opts)[0]
    S = sigma3(ls, q / np.linalg.norm(q))
    x = rng.multivariate_normal(mean, S, size=200_000)
    uv = np.stack([cam.fx * x[:, 0] / x[:, 2] + cam.cx, cam.fy * x[:, 1] / x[:, 2] + cam.cy], 1)
    cov = np.cov(uv.T)
    assert p["a"] - H_LOWPASS == pytest.approx(cov[0, 0], rel=0.02)
    assert p["c"] - H_LOWPASS == pytest.approx(cov[1, 1], rel=0.02)
    assert p["b"] == pytest.approx(cov[0, 1], abs=0.02 * np.sqrt(cov[0, 0] * cov[1, 1]))


def test_guard_band_clamp_uses_jacobian_at_clamped_point(oracle_lib):
    cam = synth.camera_front(128, 128, 128.0)
    opts = O.make_opts(16)
    lim = 1.3 * 0.5 * 128 / 128
    mean = np.array([3.0, 0.1, 2.0])                 # tx/tz = 1.5 > lim
    ls = np.array([0.0, 0.0, 0.0])                   # large enough to still touch the image
    p = O.project(params1(mean, ls), cam, opts)[0]
    assert p["clampx"] == 1 and p["clampy"] == 0
    tcl = np.array([lim * mean[2], mean[1], mean[2]])
    J = fd_jacobian(cam, tcl)
    S2 = J @ sigma3(ls, np.array([1.0, 0, 0, 0])) @ J.T
    assert p["a"] == pytest.approx(S2[0, 0] + H_LOWPASS, rel=1e-6)
    assert p["c"] == pytest.approx(S2[1, 1] + H_LOWPASS, rel=1e-6)
    assert p["mx"] == pytest.approx(128 * 3.0 / 2.0 + 64, rel=1e-15)   # mean itself unclamped


def test_culling(oracle_lib):
    cam = synth.camera_front(128, 128, 128.0)
    opts = O.make_opts(16)
    assert O.project(params1((0, 0, 0.1), (-2, -2, -2)), cam, opts)[0]["valid"] == 0   # near plane
    assert O.project(params1((0, 0, -3), (-2, -2, -2)), cam, opts)[0]["valid"] == 0    # behind
    assert O.project(params1((0, 0, 3), (-2, -2, -2), (0, 0, 0, 0)), cam, opts)[0]["valid"] == 0
    assert O.project(params1((np.nan, 0, 3), (-2, -2, -2)), cam, opts)[0]["valid"] == 0
    assert O.project(params1((0, 0, 3), (np.inf, -2, -2)), cam, opts)[0]["valid"] == 0
    assert O.project(params1((50, 0, 3), (-3, -3, -3)), cam, opts)[0]["valid"] == 0    # off-screen
    assert O.project(params1((0, 0, 3), (-2, -2, -2)), cam, opts)[0]["valid"] == 1


def test_pixel_box_definition(oracle_lib):
    scene, cams = synth.workload_c1()
    opts = O.make_opts(16)
    proj = O.project(O.Params.from_scene(scene), cams[0], opts)
    W, H = cams[0].width, cams[0].height
    ii = np.arange(W) + 0.5
    jj = np.arange(H) + 0.5
    v = proj[proj["valid"] == 1]
    assert len(v) > 9000
    for p in v[:2000]:
        assert p["radius"] == np.ceil(3.0 * np.sqrt(p["lam"]))
        inx = np.abs(ii - p["mx"]) <= p["radius"]
        iny = np.abs(jj - p["my"]) <= p["radius"]
        bx = (np.arange(W) >= p["x0"]) & (np.arange(W) <= p["x1"])
        by = (np.arange(H) >= p["y0"]) & (np.arange(H) <= p["y1"])
        assert np.array_equal(inx, bx) and np.array_equal(iny, by)
        assert p["depth32"] == np.float32(p["tz"])


# ------------------------------------------------------------------- binning

def brute_force_lists(proj, cams, tile):
    tiles_x, tiles_y, offsets, total_tiles = O.view_tables(cams, tile)
    items = []
    for v in range(proj.shape[0]):
        for g in range(proj.shape[1]):
            p = proj[v, g]
            if not p["valid"]:
                continue
            for ty in range(tiles_y[v]):
                for tx in range(tiles_x[v]):
                    # rect test written from the tile's pixel extent and the box
                    tx_lo, tx_hi = tx * tile, tx * tile + tile - 1
                    ty_lo, ty_hi = ty * tile, ty * tile + tile - 1
                    if p["x1"] >= tx_lo and p["x0"] <= tx_hi and p["y1"] >= ty_lo and p["y0"] <= ty_hi:
                        gt = int(offsets[v] + ty * tiles_x[v] + tx)
                        bits = int(np.float32(p["depth32"]).view(np.uint32))
                        items.append((gt, bits, g))
    items.sort()
    return items, total_tiles


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_bin_lists_brute_force(oracle_lib, tile):
    scene = synth.make_scene(150, 21, synth.VOL_C1)
    cams = [synth.camera_front(80, 56, 90.0), synth.camera_front(48, 40, 60.0)]
    cams[1].R, cams[1].t = synth.look_at((0.5, 0.3, -1.0), target=(0.0, 0.0, 4.0))
    opts = O.make_opts(tile)
    params = O.Params.from_scene(scene)
    proj = O.project_views(params, cams, opts)
    keys, ids, ranges = O.bin_lists(proj, cams, opts)
    items, total_tiles = brute_force_lists(proj, cams, tile)
    assert len(items) == len(keys) == int(proj["ntiles"][proj["valid"] == 1].sum())
    want_keys = np.array([(t << 32) | b for t, b, _ in items], np.uint64)
    want_ids = np.array([g for _, _, g in items], np.uint32)
    assert np.array_equal(keys, want_keys)
    assert np.array_equal(ids, want_ids)
    for t in range(total_tiles):
        sel = [k for k, it in enumerate(items) if it[0] == t]
        if sel:
            assert ranges[t, 0] == sel[0] and ranges[t, 1] == sel[-1] + 1
        else:
            assert ranges[t, 0] == ranges[t, 1]


# ------------------------------------------------------------------ blending

def np_project(params, cam, lowpass=H_LOWPASS, z_near=0.2, guard=1.3):
    """Independent vectorised projection used by the brute-force renderer."""
    R = np.asarray(cam.R)
    tc = params.mean @ R.T + np.asarray(cam.t)
    q = params.quat / np.linalg.norm(params.quat, axis=1, keepdims=True)
    Rq = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    S = np.exp(params.log_scale)
    M = Rq * S[:, None, :]
    Sig = M @ np.transpose(M, (0, 2, 1))
    limx = guard * 0.5 * cam.width / cam.fx
    limy = guard * 0.5 * cam.height / cam.fy
    ux = np.clip(tc[:, 0] / tc[:, 2], -limx, limx) * tc[:, 2]
    uy = np.clip(tc[:, 1] / tc[:, 2], -limy, limy) * tc[:, 2]
    z = tc[:, 2]
    J = np.zeros((len(z), 2, 3))
    J[:, 0, 0] = cam.fx / z
    J[:, 0, 2] = -cam.fx * ux / z ** 2
    J[:, 1, 1] = cam.fy / z
    J[:, 1, 2] = -cam.fy * uy / z ** 2
    T = J @ R
    S2 = T @ Sig @ np.transpose(T, (0, 2, 1))
    S2[:, 0, 0] += lowpass
    S2[:, 1, 1] += lowpass
    Q = np.linalg.inv(S2)
    mx = cam.fx * tc[:, 0] / z + cam.cx
    my = cam.fy * tc[:, 1] / z + cam.cy
    lam = np.linalg.eigvalsh(S2)[:, -1]
    r = np.ceil(3 * np.sqrt(lam))
    sig = 1 / (1 + np.exp(-params.omega))
    valid = (z > z_near)
    return dict(mx=mx, my=my, Q=Q, r=r, sig=sig, valid=valid, depth32=z.astype(np.float32))


def np_render(params, channels, cam, return_last=False):
    """Per pixel, over ALL Gaussians ordered by (depth32 bits, id): the
    front-to-back rule written out directly. With return_last, also the id of
    the last Gaussian blended at each pixel (-1 if none)."""
    P = np_project(params, cam)
    order = np.lexsort((np.arange(params.n), P["depth32"].view(np.uint32)))
    C = channels.shape[1]
    out = np.zeros((C, cam.height, cam.width))
    Tf = np.ones((cam.height, cam.width))
    last_id = np.full((cam.height, cam.width), -1, np.int64)
    ch = channels.astype(np.float64)
    for j in range(cam.height):
        for i in range(cam.width):
            T = 1.0
            acc = np.zeros(C)
            for g in order:
                if not P["valid"][g]:
                    continue
                dx = P["mx"][g] - (i + 0.5)
                dy = P["my"][g] - (j + 0.5)
                if abs(dx) > P["r"][g] or abs(dy) > P["r"][g]:
                    continue
                Q = P["Q"][g]
                pw = min(0.0, -0.5 * (Q[0, 0] * dx * dx + Q[1, 1] * dy * dy) - Q[0, 1] * dx * dy)
                a = min(0.99, P["sig"][g] * np.exp(pw))
                if a < 1 / 255:
                    continue
                if T * (1 - a) < 1e-4:
                    break
                acc += a * T * ch[g]
                T *= (1 - a)
                last_id[j, i] = g
            out[:, j, i] = acc
            Tf[j, i] = T
    if return_last:
        return out, Tf, last_id
    return out, Tf


def test_blend_brute_force_all_gaussians(oracle_lib):
    scene = synth.make_scene(120, 31, synth.VOL_C1, d_sem=8)
    cams = [synth.camera_front(40, 32, 40.0)]
    opts = O.make_opts(16)
    f = O.forward(scene, cams, opts)
    out, T = np_render(O.Params.from_scene(scene), scene.channels, cams[0])
    r = f["views"][0]
    assert np.allclose(r["out"].reshape(out.shape), out, rtol=1e-11, atol=1e-12)
    assert np.allclose(r["T"].reshape(T.shape), T, rtol=1e-11, atol=1e-14)
    assert (r["T"] < 0.5).any()                 # the scene is dense enough to matter


def test_single_gaussian_closed_form(oracle_lib):
    cam = synth.camera_front(96, 96, 96.0)
    opts = O.make_opts(16)
    ch = np.array([[0.3, -1.2, 2.0, 0.5]])
    sc = scene_from([[0.21, -0.13, 3.0]], [[-2.2, -2.6, -2.9]], [[0.9, 0.1, -0.3, 0.2]], [0.7], ch)
    f = O.forward(sc, [cam], opts)
    p = f["proj"][0][0]
    jj, ii = np.mgrid[0:96, 0:96]
    dx = p["mx"] - (ii + 0.5)
    dy = p["my"] - (jj + 0.5)
    pw = np.minimum(0.0, -0.5 * (p["A"] * dx * dx + p["C"] * dy * dy) - p["B"] * dx * dy)
    a = np.minimum(0.99, p["sig"] * np.exp(pw))
    inbox = (np.abs(dx) <= p["radius"]) & (np.abs(dy) <= p["radius"])
    a = np.where(inbox & (a >= 1 / 255), a, 0.0)
    out = f["views"][0]["out"].reshape(4, 96, 96)
    for c in range(4):
        assert np.allclose(out[c], float(sc.channels[0, c]) * a, rtol=1e-14, atol=1e-16)
    assert np.allclose(f["views"][0]["T"].reshape(96, 96), 1 - a, rtol=1e-14)


def test_alpha_clamp_at_exact_centre(oracle_lib):
    cam = synth.camera_front(128, 128, 128.0)
    opts = O.make_opts(16)
    # mean projects exactly onto the centre of pixel (64, 64); opacity 0.9975 > 0.99
    sc = scene_from([[1 / 64, 1 / 64, 4.0]], [[-2.0, -2.0, -2.0]], [[1, 0, 0, 0]], [6.0],
                    [[1.0, 2.0]])
    f = O.forward(sc, [cam], opts)
    p = f["proj"][0][0]
    assert p["mx"] == 64.5 and p["my"] == 64.5
    out = f["views"][0]["out"].reshape(2, 128, 128)
    assert out[0, 64, 64] == 0.99 and out[1, 64, 64] == 1.98
    assert f["views"][0]["T"].reshape(128, 128)[64, 64] == pytest.approx(0.01, rel=1e-15)


def test_two_overlapping_gaussians(oracle_lib):
    cam = synth.camera_front(64, 64, 64.0)
    opts = O.make_opts(16)
    ch = np.array([[1.0, 0.0], [0.0, 1.0]])
    sc = scene_from([[0.0, 0.0, 3.0], [0.0, 0.0, 5.0]], [[-1.8] * 3, [-1.6] * 3],
                    [[1, 0, 0, 0]] * 2, [0.4, 1.1], ch)
    f = O.forward(sc, [cam], opts)
    P = f["proj"][0]
    jj, ii = np.mgrid[0:64, 0:64]

    def alpha(p):
        dx = p["mx"] - (ii + 0.5)
        dy = p["my"] - (jj + 0.5)
        pw = np.minimum(0, -0.5 * (p["A"] * dx * dx + p["C"] * dy * dy) - p["B"] * dx * dy)
        a = np.minimum(0.99, p["sig"] * np.exp(pw))
        inb = (np.abs(dx) <= p["radius"]) & (np.abs(dy) <= p["radius"])
        return np.where(inb & (a >= 1 / 255), a, 0.0)

    a1, a2 = alpha(P[0]), alpha(P[1])
    out = f["views"][0]["out"].reshape(2, 64, 64)
    assert np.allclose(out[0], a1, rtol=1e-14, atol=1e-16)
    assert np.allclose(out[1], a2 * (1 - a1), rtol=1e-14, atol=1e-16)


def test_invariants_ones_channel_T_bounds_and_low_opacity(oracle_lib):
    scene = synth.make_scene(3000, 41, synth.VOL_C1, d_sem=2)
    scene.channels[:, 0] = 1.0
    cams = [synth.camera_front(96, 80, 96.0)]
    opts = O.make_opts(16)
    f = O.forward(scene, cams, opts)
    r = f["views"][0]
    assert np.allclose(r["out"][0], 1.0 - r["T"], atol=1e-12)
    assert (r["T"] <= 1.0).all() and (r["T"] >= 1e-4).all()
    assert (r["T"] < 1e-3).any()
    # Gaussians with opacity below 1/255 can never be blended
    extra = synth.make_scene(500, 42, synth.VOL_C1, d_sem=2)
    extra.opacity_logit[:] = -6.0
    both = synth.Scene(np.concatenate([scene.mean, extra.mean]),
                       np.concatenate([scene.log_scale, extra.log_scale]),
                       np.concatenate([scene.quat, extra.quat]),
                       np.concatenate([scene.opacity_logit, extra.opacity_logit]),
                       np.concatenate([scene.channels, extra.channels]), 2)
    f2 = O.forward(both, cams, opts)
    assert np.array_equal(f2["views"][0]["out"], r["out"])
    assert np.array_equal(f2["views"][0]["T"], r["T"])


def test_permutation_and_tile_invariance(oracle_lib):
    scene = synth.make_scene(2000, 51, synth.VOL_C1, d_sem=4)
    cams = [synth.camera_front(100, 72, 100.0)]
    base = O.forward(scene, cams, O.make_opts(16))["views"][0]
    perm = np.random.default_rng(5).permutation(scene.n)
    d = O.forward(scene.subset(perm), cams, O.make_opts(16))["views"][0]
    assert np.array_equal(d["out"], base["out"]) and np.array_equal(d["T"], base["T"])
    assert np.array_equal(d["last"], base["last"])
    for tile in (8, 32):
        d = O.forward(scene, cams, O.make_opts(tile))["views"][0]
        assert np.array_equal(d["out"], base["out"]) and np.array_equal(d["T"], base["T"])


def test_region_render_matches_tile_lists(oracle_lib):
    scene = synth.make_scene(4000, 61, synth.VOL_C1, d_sem=8)
    cams = [synth.camera_front(128, 128, 128.0)]
    opts = O.make_opts(16)
    f = O.forward(scene, cams, opts)
    rr = O.render_region(f["proj"][0], cams[0], opts, scene.channels, 13, 29, 70, 50)
    full = f["views"][0]["out"].reshape(-1, 128, 128)[:, 29:79, 13:83]
    assert np.array_equal(rr["out"], full)


def test_ambiguous_skip_flip(oracle_lib):
    cam = synth.camera_front(64, 64, 64.0)
    opts = O.make_opts(16)
    s0 = 1.0 / 255.0
    omega = np.float32(np.log(s0 / (1 - s0)))
    sig = 1.0 / (1.0 + np.exp(-float(omega)))
    assert abs(sig - s0) / s0 < 1e-6           # within the ambiguity margin of the skip rule
    above = sig >= s0
    # centred on pixel (32, 32): alpha there equals sig (power 0)
    sc = scene_from([[1.5 / 64, 1.5 / 64, 3.0]], [[-1.0] * 3], [[1, 0, 0, 0]], [omega], [[2.0]])
    f = O.forward(sc, [cam], opts)
    assert f["proj"][0][0]["mx"] == 32.5 and f["proj"][0][0]["my"] == 32.5
    lin = 32 * 64 + 32
    r0 = O.render_view(f["proj"][0], cam, opts, sc.channels, f["ids"], f["ranges"], 0, pix=[lin])
    r1 = O.render_view(f["proj"][0], cam, opts, sc.channels, f["ids"], f["ranges"], 0, pix=[lin],
                       flip_mask=[1])
    assert r0["n_amb"][0] == 1
    blended, skipped = (r0, r1) if above else (r1, r0)
    assert blended["out"][0, 0] == pytest.approx(2.0 * sig, rel=1e-12)
    assert blended["last"][0] == 1
    assert skipped["out"][0, 0] == 0.0 and skipped["T"][0] == 1.0 and skipped["last"][0] == 0


def test_skip_window_grows_with_exponent_magnitude(oracle_lib):
    """The skip decision counts as ambiguous within eps_alpha (relative) of
    1/255, widened by eps_alpha_mag per unit of the exponent's magnitude sum
    0.5 |A dx^2| + |B dx dy| + 0.5 |C dy^2|. A needle-shaped footprint (terms
    of ~1188 cancelling to a power of -5.2) with alpha 2e-5 below 1/255 is
    ambiguous only with the widening; a round footprint at the same alpha and
    power (magnitude sum 5.2) is not ambiguous either way. Both are skipped."""
    cam = synth.camera_front(64, 64, 64.0)
    sc = scene_from([[1.5 / 64, 1.5 / 64, 3.0]], [[-1.0] * 3], [[1, 0, 0, 0]], [0.0], [[2.0]])
    f = O.forward(sc, [cam], O.make_opts(16))
    lin = 32 * 64 + 32
    dx, dy = 10.0, -9.9
    target = (1.0 / 255.0) * (1.0 - 2e-5)
    got = {}
    for name in ("needle", "round"):
        rec = f["proj"][0].copy()
        if name == "needle":
            A = C = 12.0
            B = (0.5 * (A * dx * dx + C * dy * dy) - 5.2) / (-dx * dy)
            assert A * C - B * B > 0.0
        else:
            A = C = 10.4 / (dx * dx + dy * dy)
            B = 0.0
        power = -0.5 * (A * dx * dx + C * dy * dy) - B * dx * dy
        assert power == pytest.approx(-5.2, rel=1e-12)
        rec["mx"], rec["my"] = 32.5 + dx, 32.5 + dy
        rec["A"], rec["B"], rec["C"] = A, B, C
        rec["sig"] = target / np.exp(power)
        rec["x0"], rec["x1"], rec["y0"], rec["y1"] = 0, 63, 0, 63
        for widen in (False, True):
            opts = O.make_opts(16, eps_alpha_mag=16 * 2.0 ** -24 if widen else 0.0)
            r = O.render_view(rec, cam, opts, sc.channels, f["ids"], f["ranges"], 0, pix=[lin])
            got[(name, widen)] = int(r["n_amb"][0])
            assert r["out"][0, 0] == 0.0 and r["T"][0] == 1.0
    assert got == {("needle", False): 0, ("needle", True): 1, ("round", False): 0, ("round", True): 0}


# ------------------------------------------------------------------ backward

def _group_err(an, ref, floor):
    return np.linalg.norm(an - ref) / max(np.linalg.norm(ref), floor)


def test_backward_matches_finite_differences(oracle_lib):
    scene = synth.make_scene(3000, 71, synth.VOL_C1, d_sem=8)
    cams = [synth.camera_front(96, 96, 96.0)]
    cams.append(synth.Camera(96, 80, 90.0, 90.0, 48.0, 40.0, *synth.look_at((1.0, 0.5, -2.0), (0, 0, 4.0))))
    opts = O.make_opts(16)
    f = O.forward(scene, cams, opts)
    G = synth.upstream_grads(cams, scene.n_channels, 271)
    b = O.backward(scene, cams, opts, f, G)
    ids = fd.blended_gaussians(b)
    sel = np.random.default_rng(3).choice(ids, 12, replace=False)
    groups = ("mean", "log_scale", "quat", "opacity_logit", "channels")
    rms = {g: np.sqrt(np.mean(b[g].reshape(scene.n, -1)[ids] ** 2)) for g in groups}
    n_valid = 0
    for g in sel:
        r = fd.fd_gaussian(f["params"], scene.channels, cams, opts, f["proj"], G, g)
        for grp in groups:
            vals, ok = r[grp]
            an = b[grp].reshape(scene.n, -1)[g]
            n_valid += int(ok.sum())
            err = _group_err(an[ok], vals[ok], 1e-3 * rms[grp])
            assert err < 1e-5, (g, grp, err)
    assert n_valid > 12 * 20


def test_channel_gradient_is_blend_weight(oracle_lib):
    """out is linear in the channels: with channels = identity the render gives
    each Gaussian's weight alpha * T per pixel, and dL/dch = sum_px G * weight."""
    n = 40
    scene = synth.make_scene(n, 81, synth.VOL_C1, d_sem=0)
    scene.log_scale[:] += 1.0
    cams = [synth.camera_front(48, 48, 48.0)]
    opts = O.make_opts(16)
    G = synth.upstream_grads(cams, scene.n_channels, 281)
    f = O.forward(scene, cams, opts)
    b = O.backward(scene, cams, opts, f, G)
    eye = synth.Scene(scene.mean, scene.log_scale, scene.quat, scene.opacity_logit,
                      np.eye(n, dtype=np.float32), 0)
    w = O.forward(eye, cams, opts)["views"][0]["out"]          # [n, HW]
    Gv = G.reshape(scene.n_channels, -1)
    want = w @ Gv.T                                             # [n, C]
    assert np.allclose(b["channels"], want, rtol=1e-12, atol=1e-13)
    assert np.abs(want).max() > 0.1


def test_isolated_gaussian_opacity_gradient(oracle_lib):
    cam = synth.camera_front(64, 64, 64.0)
    opts = O.make_opts(16)
    sc = scene_from([[0.1, -0.05, 3.0]], [[-1.5, -1.9, -1.7]], [[0.7, 0.2, 0.1, -0.3]], [-0.4],
                    [[0.8, -1.1]])
    f = O.forward(sc, [cam], opts)
    G = synth.upstream_grads([cam], 2, 5)
    b = O.backward(sc, [cam], opts, f, G)
    p = f["proj"][0][0]
    jj, ii = np.mgrid[0:64, 0:64]
    dx = p["mx"] - (ii + 0.5)
    dy = p["my"] - (jj + 0.5)
    ep = np.exp(np.minimum(0, -0.5 * (p["A"] * dx * dx + p["C"] * dy * dy) - p["B"] * dx * dy))
    a = p["sig"] * ep
    use = (np.abs(dx) <= p["radius"]) & (np.abs(dy) <= p["radius"]) & (a >= 1 / 255) & (a <= 0.99)
    Gv = G.reshape(2, 64, 64).astype(np.float64)
    s = p["sig"]
    c0, c1 = float(sc.channels[0, 0]), float(sc.channels[0, 1])
    want = float(((Gv[0] * c0 + Gv[1] * c1) * ep * s * (1 - s))[use].sum())
    assert b["opacity_logit"][0] == pytest.approx(want, rel=1e-12)


# ------------------------------------------------------------------- decoding

def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 3, 20000), rng.normal(0, 1e-3, 2000)]).astype(np.float32)
    # exact ties (low 16 bits = 0x8000) on normal numbers of both signs
    e = rng.integers(100, 150, 500).astype(np.uint32)
    m = rng.integers(0, 128, 500).astype(np.uint32)
    sg = rng.integers(0, 2, 500).astype(np.uint32)
    ties = (sg << 31) | (e << 23) | (m << 16) | np.uint32(0x8000)
    x = np.concatenate([x, ties.view(np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(D.bf16(x.astype(np.float64)), ref)


def test_decode_plain_reduces_to_folded_argmax_and_torch_softmax():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    feat = rng.normal(0, 1, (3000, 8)).astype(np.float32)
    feat[0] = 0.0
    Pm = synth.projection(512, 8, 9)
    Cb = synth.codebook(128, 512, 10)
    probs, top1 = D.decode_plain(feat, Pm, Cb)
    folded = feat.astype(np.float64) @ (Cb.astype(np.float64) @ Pm.astype(np.float64)).T
    s = np.sort(folded, axis=1)
    clear = (s[:, -1] - s[:, -2]) > 1e-6 * np.abs(s[:, -1])
    assert top1[0] == 0
    assert np.array_equal(top1[1:][clear[1:]], np.argmax(folded, axis=1)[1:][clear[1:]])
    z = torch.from_numpy(feat.astype(np.float64)) @ torch.from_numpy(Pm.astype(np.float64)).T
    cos = torch.nn.functional.cosine_similarity(z[:, None, :], torch.from_numpy(Cb.astype(np.float64))[None], dim=2)
    ref = torch.softmax(cos, dim=1).numpy()
    assert np.allclose(probs[1:], ref[1:], rtol=1e-12, atol=1e-15)


def _torch_mlp(torch, x, ws, bs):
    xt = torch.from_numpy(x.astype(np.float64))
    h = torch.from_numpy(D.bf16(torch.nn.functional.normalize(xt, dim=1).numpy()))
    for l, (W, b) in enumerate(zip(ws, bs)):
        h = torch.nn.functional.linear(h, W, b)
        if l < len(ws) - 1:
            r = torch.relu(h)
            h = r + (torch.from_numpy(D.bf16(r.detach().numpy())) - r).detach()
    return h


def test_raw_input_decoder_matches_torch():
    """Without the input normalisation the decoder is Eq. 8 applied to R_s."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    x = rng.normal(0, 1, (300, 8)).astype(np.float32)
    ws, bs = synth.mlp_init((8, 64, 64, 64), 13)
    fw = D.mlp_forward(x, ws, bs, normalize=False)
    h = torch.from_numpy(D.bf16(x.astype(np.float64)))
    for l, (W, b) in enumerate(zip(ws, bs)):
        h = torch.nn.functional.linear(h, torch.from_numpy(D.bf16(W.astype(np.float64))),
                                       torch.from_numpy(b.astype(np.float64)))
        if l < 2:
            h = torch.from_numpy(D.bf16(torch.relu(h).numpy()))
    assert np.allclose(fw["logits"], h.numpy(), rtol=1e-12, atol=1e-13)
    assert not np.allclose(fw["logits"], D.mlp_forward(x, ws, bs)["logits"])


def test_mlp_forward_and_grads_match_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(2)
    x = rng.normal(0, 1, (500, 8)).astype(np.float32)
    y = rng.integers(0, 128, 500)
    ws, bs = synth.mlp_init((8, 64, 64, 128), 4)
    fw = D.mlp_forward(x, ws, bs)
    Wt = [torch.tensor(D.bf16(w.astype(np.float64)), requires_grad=True) for w in ws]
    bt = [torch.tensor(b.astype(np.float64), requires_grad=True) for b in bs]
    logits = _torch_mlp(torch, x, Wt, bt)
    assert np.allclose(fw["logits"], logits.detach().numpy(), rtol=1e-12, atol=1e-13)
    loss = torch.nn.functional.cross_entropy(logits, torch.from_numpy(y))
    loss.backward()
    l2, gW, gb = D.mlp_grads(x, y, ws, bs)
    assert l2 == pytest.approx(loss.item(), rel=1e-12)
    for l in range(3):
        assert np.allclose(gW[l], Wt[l].grad.numpy(), rtol=1e-10, atol=1e-14)
        assert np.allclose(gb[l], bt[l].grad.numpy(), rtol=1e-10, atol=1e-14)


def test_mlp_input_is_scale_free():
    """The decoder sees only the feature's direction: a positive rescale of a
    feature leaves its logits unchanged, and a zero feature gives the logits
    of a zero input (the biases pushed through the layers)."""
    rng = np.random.default_rng(5)
    x = rng.normal(0, 1, (300, 8)).astype(np.float32)
    ws, bs = synth.mlp_init((8, 64, 64, 32), 6)
    a = D.mlp_forward(x, ws, bs)
    b = D.mlp_forward((x * np.float32(4.0)), ws, bs)    # exact rescale by a power of two
    assert np.array_equal(a["logits"], b["logits"])
    z = D.mlp_forward(np.zeros((1, 8), np.float32), ws, bs)["logits"][0]
    h = np.zeros(8)
    for l, (W, bb) in enumerate(zip(ws, bs)):
        h = D.bf16(W.astype(np.float64)) @ h + bb.astype(np.float64)
        if l < 2:
            h = D.bf16(np.maximum(h, 0.0))
    assert np.allclose(z, h, rtol=0, atol=1e-12)


def test_adam_first_step_closed_form_and_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    p0 = rng.normal(0, 1, 1000)
    g = rng.normal(0, 1, 1000)
    p1, m, v = D.adam(p0, g, np.zeros(1000), np.zeros(1000), 1, lr=1e-3)
    assert np.allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-16)
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(1000), np.zeros(1000)
    for step in range(1, 6):
        gs = rng.normal(0, 1, 1000)
        pt.grad = torch.tensor(gs)
        opt.step()
        p, m, v = D.adam(p, gs, m, v, step)
    assert np.allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_l1_loss_gradient_fd():
    rng = np.random.default_rng(4)
    cams = [synth.camera_front(6, 5, 6.0), synth.camera_front(4, 3, 4.0)]
    C, ds = 6, 2
    out = rng.normal(0, 1, sum(C * c.width * c.height for c in cams))
    tgt = rng.normal(0, 1, out.shape)
    loss, grad = D.l1_loss_grad(out, tgt, cams, C, ds, lambda_u=1.0)
    for k in rng.choice(out.size, 40, replace=False):
        e = np.zeros_like(out)
        e[k] = 1e-6
        lp, _ = D.l1_loss_grad(out + e, tgt, cams, C, ds)
        lm, _ = D.l1_loss_grad(out - e, tgt, cams, C, ds)
        assert grad[k] == pytest.approx((lp - lm) / 2e-6, rel=1e-6, abs=1e-9)


def _guard_band_scene(seed, n_out=40, n_in=300):
    """Gaussians whose means lie outside the guard band (|x/z| > 1.3 W / (2 f))
    but whose footprints still reach the image, mixed with ordinary ones."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(2.5, 4.0, n_out)
    u = rng.uniform(0.68, 0.85, n_out) * rng.choice([-1.0, 1.0], n_out)
    v = rng.uniform(-0.3, 0.3, n_out)
    out_mean = np.stack([u * z, v * z, z], 1)
    inner = synth.make_scene(n_in, seed + 1, synth.VOL_C1, d_sem=2)
    q = rng.normal(size=(n_out, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return synth.Scene(
        np.concatenate([out_mean.astype(np.float32), inner.mean]),
        np.concatenate([rng.normal(-1.0, 0.2, (n_out, 3)).astype(np.float32), inner.log_scale]),
        np.concatenate([q.astype(np.float32), inner.quat]),
        np.concatenate([rng.normal(0.0, 1.0, n_out).astype(np.float32), inner.opacity_logit]),
        np.concatenate([rng.normal(0.0, 1.0, (n_out, inner.n_channels)).astype(np.float32),
                        inner.channels]), 2)


def test_guard_band_backward_matches_finite_differences(oracle_lib):
    """The Jacobian of a Gaussian outside the guard band is evaluated at the
    clamped point (x/z held at the limit), so its derivative with respect to the
    camera-space x or y is zero and only z moves it. The oracle's analytic
    gradient of such Gaussians (mean, log-scale, quaternion, opacity, channels)
    agrees with float64 central finite differences of the rendered loss."""
    scene = _guard_band_scene(91)
    cams = [synth.camera_front(96, 96, 96.0)]
    opts = O.make_opts(16)
    f = O.forward(scene, cams, opts)
    P = f["proj"][0]
    G = synth.upstream_grads(cams, scene.n_channels, 291)
    b = O.backward(scene, cams, opts, f, G)
    blended = set(fd.blended_gaussians(b).tolist())
    clamped = [g for g in range(40) if P["valid"][g] and (P["clampx"][g] or P["clampy"][g])
               and g in blended]
    assert len(clamped) >= 20
    groups = ("mean", "log_scale", "quat", "opacity_logit", "channels")
    ids = np.array(sorted(blended))
    rms = {g: np.sqrt(np.mean(b[g].reshape(scene.n, -1)[ids] ** 2)) for g in groups}
    n_valid = 0
    for g in clamped[:10]:
        r = fd.fd_gaussian(f["params"], scene.channels, cams, opts, f["proj"], G, g)
        for grp in groups:
            vals, ok = r[grp]
            an = b[grp].reshape(scene.n, -1)[g]
            n_valid += int(ok.sum())
            err = _group_err(an[ok], vals[ok], 1e-3 * rms[grp])
            assert err < 1e-5, (g, grp, err)
    assert n_valid >= 10 * 14


def test_l1_loss_closed_form_values():
    """Constant maps give the loss in closed form: with |out - target| = d on
    every fitted channel and a rendered uncertainty u in each remaining
    channel, each view contributes d + lambda_u * u per uncertainty channel,
    and dL/dout = sign(out - target) / (n_fit H W) or lambda_u / (H W)."""
    cams = [synth.camera_front(7, 5, 7.0), synth.camera_front(3, 4, 3.0)]
    C, ds = 7, 3                        # RGB + 3 semantic + 1 uncertainty
    n_fit = 3 + ds
    parts_o, parts_t, want_g = [], [], []
    rng = np.random.default_rng(12)
    for cam in cams:
        hw = cam.width * cam.height
        t = rng.normal(0, 1, (C, hw))
        sign = rng.choice([-1.0, 1.0], (C, hw))
        o = t + 0.375 * sign
        o[n_fit:] = 0.625
        parts_o.append(o.reshape(-1))
        parts_t.append(t.reshape(-1))
        g = np.concatenate([sign[:n_fit] / (n_fit * hw), np.full((C - n_fit, hw), 2.0 / hw)])
        want_g.append(g.reshape(-1))
    loss, grad = D.l1_loss_grad(np.concatenate(parts_o), np.concatenate(parts_t), cams, C, ds,
                                lambda_u=2.0)
    assert loss == pytest.approx(len(cams) * (0.375 + 2.0 * 0.625), rel=1e-14)
    assert np.allclose(grad, np.concatenate(want_g), rtol=1e-15, atol=0)
    # equal maps: no L1 term and a zero sign gradient
    o = np.concatenate(parts_t).copy()
    loss0, grad0 = D.l1_loss_grad(o, o, cams, C, ds, lambda_u=0.0)
    assert loss0 == 0.0 and not grad0.any()


def _tile_positions(items, tile_of_pixel):
    """Position of each Gaussian in each tile's list, from brute-force lists."""
    pos = {}
    k_in_tile = {}
    for t, _, g in items:
        k = k_in_tile.get(t, 0)
        pos[(t, g)] = k
        k_in_tile[t] = k + 1
    return pos


def test_last_index_multi_entry_brute_force(oracle_lib):
    """`last` = 1 + the tile-list position of the last Gaussian blended at a
    pixel. A direct per-pixel walk over all Gaussians (depth order) names that
    Gaussian; its position in the brute-force tile list gives the expected
    value, on a scene dense enough that many pixels blend several entries and
    some stop."""
    scene = synth.make_scene(150, 33, synth.VOL_C1, d_sem=1)
    scene.opacity_logit[:] += 2.0
    cam = synth.camera_front(40, 32, 40.0)
    for tile in (8, 16):
        opts = O.make_opts(tile)
        f = O.forward(scene, [cam], opts)
        r = f["views"][0]
        params = O.Params.from_scene(scene)
        _, _, last_id = np_render(params, scene.channels, cam, return_last=True)
        items, _ = brute_force_lists(f["proj"], [cam], tile)
        pos = _tile_positions(items, None)
        tiles_x = (cam.width + tile - 1) // tile
        want = np.zeros(cam.width * cam.height, np.int64)
        for j in range(cam.height):
            for i in range(cam.width):
                g = last_id[j, i]
                if g >= 0:
                    want[j * cam.width + i] = 1 + pos[((j // tile) * tiles_x + i // tile, g)]
        assert np.array_equal(r["last"], want)
        assert (want > 1).mean() > 0.5 and want.max() > 10


def test_ambiguous_stop_flip_and_backward_replay(oracle_lib):
    """Two Gaussians with opacity above alpha_max centred on one pixel: both
    clamp to 0.99, so after the second T (1 - alpha) = 1e-4 up to rounding,
    the stop rule's threshold. The oracle flags the decision ambiguous; with
    it inverted the second Gaussian stops unblended. The backward along the
    inverted branch equals the backward of the same scene with t_min nudged
    so that the stop happens without inversion (and, for the skip rule, with
    alpha_min nudged), so a flip mask replays exactly the other decision."""
    cam = synth.camera_front(64, 64, 64.0)
    opts = O.make_opts(16)
    # centred on pixel (32, 32); opacities above 0.99 only within half a pixel
    # of the centre, so the centre is the only pixel where both clamp
    c = 1.5 / 64
    sc = scene_from([[c, c, 3.0], [c * 4 / 3, c * 4 / 3, 4.0]], [[-1.0] * 3, [-0.9] * 3],
                    [[1, 0, 0, 0]] * 2, [5.5, 5.0], [[1.0, 0.5], [0.25, 2.0]])
    f = O.forward(sc, [cam], opts)
    P = f["proj"][0]
    assert P["mx"][0] == pytest.approx(32.5, abs=1e-12) and P["mx"][1] == pytest.approx(32.5, abs=1e-12)
    lin = 32 * 64 + 32
    r0 = O.render_view(P, cam, opts, sc.channels, f["ids"], f["ranges"], 0, pix=[lin])
    r1 = O.render_view(P, cam, opts, sc.channels, f["ids"], f["ranges"], 0, pix=[lin], flip_mask=[1])
    assert r0["n_amb"][0] == 1
    a = 0.99
    # without the flip both blend (T'= (1 - 0.99)^2 rounds above 1e-4 in float64)
    assert r0["last"][0] == 2 and r0["out"][0, 0] == pytest.approx(a * 1.0 + a * (1 - a) * 0.25, rel=1e-12)
    assert r0["T"][0] == pytest.approx((1 - a) ** 2, rel=1e-12)
    assert r1["last"][0] == 1 and r1["out"][0, 0] == pytest.approx(a, rel=1e-12)
    assert r1["T"][0] == pytest.approx(1 - a, rel=1e-12)
    # backward replay of the flipped branch = backward with the stop taken naturally
    G = synth.upstream_grads([cam], 2, 17).astype(np.float64)
    fm = np.zeros(64 * 64, np.uint32)
    fm[lin] = 1
    b_flip = O.backward(sc, [cam], opts, f, G, flip_masks=[fm])
    o2 = O.make_opts(16)
    o2.t_min = 1.0000001e-4
    f2 = O.forward(sc, [cam], o2)
    assert f2["views"][0]["last"][lin] == 1
    b_nat = O.backward(sc, [cam], o2, f2, G)
    b_plain = O.backward(sc, [cam], opts, f, G)
    for grp in ("mean", "log_scale", "quat", "opacity_logit", "channels"):
        assert np.allclose(b_flip[grp], b_nat[grp], rtol=1e-12, atol=1e-15), grp
    assert not np.allclose(b_flip["channels"], b_plain["channels"])


def test_skip_flip_backward_replay(oracle_lib):
    """A Gaussian whose alpha at one pixel sits at 1/255 within the ambiguity
    margin: the backward along the inverted skip decision equals the backward
    with alpha_min nudged so that the other decision is taken naturally."""
    cam = synth.camera_front(64, 64, 64.0)
    opts = O.make_opts(16)
    s0 = 1.0 / 255.0
    omega = np.float32(np.log(s0 / (1 - s0)))
    sig = 1.0 / (1.0 + np.exp(-float(omega)))
    sc = scene_from([[1.5 / 64, 1.5 / 64, 3.0], [0.1, 0.05, 2.5]], [[-1.0] * 3, [-1.6, -1.2, -1.4]],
                    [[1, 0, 0, 0], [0.9, 0.2, -0.1, 0.3]], [omega, 0.3], [[2.0, 1.0], [0.5, -1.0]])
    f = O.forward(sc, [cam], opts)
    lin = 32 * 64 + 32
    G = synth.upstream_grads([cam], 2, 18).astype(np.float64)
    fm = np.zeros(64 * 64, np.uint32)
    fm[lin] = 1
    r = O.render_view(f["proj"][0], cam, opts, sc.channels, f["ids"], f["ranges"], 0, pix=[lin])
    assert r["n_amb"][0] == 1
    b_flip = O.backward(sc, [cam], opts, f, G, flip_masks=[fm])
    o2 = O.make_opts(16)
    # move alpha_min across alpha so that the natural decision is the inverted one
    o2.alpha_min = sig * (1 + 1e-9) if sig >= s0 else sig * (1 - 1e-9)
    o2.eps_alpha = 1e-12
    f2 = O.forward(sc, [cam], o2)
    b_nat = O.backward(sc, [cam], o2, f2, G)
    for grp in ("mean", "log_scale", "quat", "opacity_logit", "channels"):
        assert np.allclose(b_flip[grp], b_nat[grp], rtol=1e-10, atol=1e-15), grp


# ------------------------------------------------------- semantic loss (Eqs. 10-12)

def _torch_semantic(torch, f, ru, y, ws, bs, inv_hw, lam_ce, lam_u, round_bf16, normalize=True):
    """The same loss written with torch ops, differentiated by autograd
    (straight-through roundings via the detach trick)."""
    ft = torch.tensor(f.astype(np.float64), requires_grad=True)
    rt = torch.tensor(ru.astype(np.float64), requires_grad=True)
    Wt = [torch.tensor(D.bf16(w.astype(np.float64)) if round_bf16 else w.astype(np.float64), requires_grad=True)
          for w in ws]
    bt = [torch.tensor(b.astype(np.float64), requires_grad=True) for b in bs]

    def st(x):
        return x + (torch.from_numpy(D.bf16(x.detach().numpy())) - x).detach() if round_bf16 else x
    h = st(torch.nn.functional.normalize(ft, dim=1) if normalize else ft)
    for l, (W, b) in enumerate(zip(Wt, bt)):
        h = torch.nn.functional.linear(h, W, b)
        if l < len(Wt) - 1:
            h = st(torch.relu(h))
    ce = torch.nn.functional.cross_entropy(h, torch.from_numpy(y.astype(np.int64)), reduction="none")
    loss = lam_ce * (ce * (1.0 - rt)).sum() * inv_hw + lam_u * rt.sum() * inv_hw
    loss.backward()
    return loss.item(), ft.grad.numpy(), rt.grad.numpy(), [w.grad.numpy() for w in Wt], [b.grad.numpy() for b in bt]


def test_rounding_branches_and_followed_gradients():
    """mlp_branches: the first branch of a pixel is the plain forward; every
    branch rounds each value (the normalised input, each hidden activation
    computed from the branch's previous layer) to one of its two bf16
    neighbours, and differs from round-to-nearest only where the value lies
    within amb_tol of a rounding midpoint; its logits are the forward of its
    own activations. Following a branch's activations (hidden=) gives the
    straight-through gradients torch autograd computes with the roundings
    forced to those values, for mlp_grads (Eq. 9) and semantic_loss_grad
    (Eqs. 10-12)."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(14)
    P, K, tol = 400, 32, 2e-6
    f = rng.normal(0, 1, (P, 8)).astype(np.float32)
    ru = rng.uniform(0, 1, P)
    y = rng.integers(0, K, P)
    ws, bs = synth.mlp_init((8, 64, 64, K), 15)
    fw = D.mlp_forward(f, ws, bs, amb_tol=tol)
    amb = np.nonzero(fw["ambiguous"])[0]
    assert len(amb) >= 5
    Wb = [D.bf16(w.astype(np.float64)) for w in ws]
    b64 = [b.astype(np.float64) for b in bs]
    hid = [h.copy() for h in fw["hs"]]
    moved = 0
    for i in amb:
        lg, complete, trails = D.mlp_branches(f[i], ws, bs, amb_tol=tol, return_hidden=True)
        assert complete and len(lg) >= 2 and len(trails) == len(lg)
        assert all(np.array_equal(a, b[i]) for a, b in zip(trails[0], fw["hs"]))
        u = f[i].astype(np.float64) / np.linalg.norm(f[i].astype(np.float64))
        for z, tr in zip(lg, trails):
            assert np.allclose(z, tr[-1] @ Wb[-1].T + b64[-1], rtol=0, atol=1e-12)
            for l, h in enumerate(tr):
                v = u if l == 0 else np.maximum(tr[l - 1] @ Wb[l - 1].T + b64[l - 1], 0.0)
                lo, hi = D.bf16(v * (1 - tol)), D.bf16(v * (1 + tol))
                near = lo != hi
                assert np.array_equal(h[~near], D.bf16(v)[~near])
                assert ((h[near] == lo[near]) | (h[near] == hi[near])).all()
        for l, h in enumerate(trails[-1]):
            hid[l][i] = h
        moved += any(not np.array_equal(a, b) for a, b in zip(trails[-1], trails[0]))
    assert moved == len(amb)

    def forced(normalize):
        ft = torch.tensor(f.astype(np.float64), requires_grad=True)
        Wt = [torch.tensor(w, requires_grad=True) for w in Wb]
        bt = [torch.tensor(b, requires_grad=True) for b in b64]

        def force(x, v):
            return x + (torch.from_numpy(v) - x).detach()
        h = force(torch.nn.functional.normalize(ft, dim=1) if normalize else ft, hid[0])
        for l, (W, b) in enumerate(zip(Wt, bt)):
            h = torch.nn.functional.linear(h, W, b)
            if l < len(Wt) - 1:
                h = force(torch.relu(h), hid[l + 1])
        return ft, Wt, bt, h
    ft, Wt, bt, z = forced(True)
    loss = torch.nn.functional.cross_entropy(z, torch.from_numpy(y))
    loss.backward()
    l2, gW, gb = D.mlp_grads(f, y, ws, bs, hidden=hid)
    assert l2 == pytest.approx(loss.item(), rel=1e-12)
    for l in range(3):
        assert np.allclose(gW[l], Wt[l].grad.numpy(), rtol=1e-10, atol=1e-14)
        assert np.allclose(gb[l], bt[l].grad.numpy(), rtol=1e-10, atol=1e-14)
    plain = D.mlp_grads(f, y, ws, bs)
    assert not np.allclose(plain[1][0], gW[0], rtol=1e-12, atol=0)      # the branches matter
    ft, Wt, bt, z = forced(True)
    rt = torch.tensor(ru, requires_grad=True)
    inv_hw = 1.0 / 613.0
    ce = torch.nn.functional.cross_entropy(z, torch.from_numpy(y), reduction="none")
    sl = 1.5 * (ce * (1.0 - rt)).sum() * inv_hw + 0.5 * rt.sum() * inv_hw
    sl.backward()
    r = D.semantic_loss_grad(f, ru, y, ws, bs, inv_hw, 1.5, 0.5, hidden=hid)
    assert r["loss"] == pytest.approx(sl.item(), rel=1e-12)
    assert np.allclose(r["d_feat"], ft.grad.numpy(), rtol=1e-9, atol=1e-15)
    assert np.allclose(r["d_ru"], rt.grad.numpy(), rtol=1e-12, atol=1e-16)
    for l in range(3):
        assert np.allclose(r["gW"][l], Wt[l].grad.numpy(), rtol=1e-9, atol=1e-15)
        assert np.allclose(r["gb"][l], bt[l].grad.numpy(), rtol=1e-9, atol=1e-15)


@pytest.mark.parametrize("round_bf16,normalize", [(True, True), (False, True), (True, False)])
def test_semantic_loss_matches_torch_autograd(round_bf16, normalize):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(8)
    P, K = 400, 64
    f = rng.normal(0, 1, (P, 8)).astype(np.float32)
    ru = rng.uniform(0, 1, P).astype(np.float32)
    y = rng.integers(0, K, P)
    ws, bs = synth.mlp_init((8, 64, 64, K), 9)
    inv_hw = 1.0 / 517.0
    r = D.semantic_loss_grad(f, ru, y, ws, bs, inv_hw, 1.0, 1.0, round_bf16=round_bf16, normalize=normalize)
    lt, gf, gr, gW, gb = _torch_semantic(torch, f, ru, y, ws, bs, inv_hw, 1.0, 1.0, round_bf16, normalize)
    assert r["loss"] == pytest.approx(lt, rel=1e-12)
    assert np.allclose(r["d_feat"], gf, rtol=1e-9, atol=1e-15)
    assert np.allclose(r["d_ru"], gr, rtol=1e-12, atol=1e-16)
    for l in range(3):
        assert np.allclose(r["gW"][l], gW[l], rtol=1e-9, atol=1e-15)
        assert np.allclose(r["gb"][l], gb[l], rtol=1e-9, atol=1e-15)


def test_semantic_loss_special_cases_and_fd():
    """R_u = 0 reduces L_CE to the plain mean cross-entropy (Eq. 9 with H W
    pixels), whose gradients mlp_grads gives; R_u = 1 removes every CE term,
    leaving L_u alone; dL/dR_u is exact in closed form ((lambda_u - lambda_CE
    CE) / (H W), L is linear in R_u); and without the roundings the feature
    gradient matches central finite differences."""
    rng = np.random.default_rng(10)
    P, K = 300, 32
    f = rng.normal(0, 1, (P, 8)).astype(np.float32)
    y = rng.integers(0, K, P)
    ws, bs = synth.mlp_init((8, 64, 64, K), 11)
    r0 = D.semantic_loss_grad(f, np.zeros(P), y, ws, bs, 1.0 / P, 1.0, 1.0)
    l2, gW, gb = D.mlp_grads(f, y, ws, bs)
    assert r0["loss"] == pytest.approx(l2, rel=1e-12)
    for l in range(3):
        assert np.allclose(r0["gW"][l], gW[l], rtol=1e-12, atol=1e-16)
        assert np.allclose(r0["gb"][l], gb[l], rtol=1e-12, atol=1e-16)
    r1 = D.semantic_loss_grad(f, np.ones(P), y, ws, bs, 1.0 / P, 1.0, 0.5)
    assert r1["loss"] == pytest.approx(0.5, rel=1e-14)
    assert not r1["d_feat"].any() and all(not g.any() for g in r1["gW"])
    ru = rng.uniform(0, 1, P)
    r = D.semantic_loss_grad(f, ru, y, ws, bs, 1.0 / 777.0, 2.0, 0.25, round_bf16=False)
    assert np.allclose(r["d_ru"], (0.25 - 2.0 * r["ce"]) / 777.0, rtol=1e-14)
    ff = f.astype(np.float64)
    for p, c in zip(rng.integers(0, P, 20), rng.integers(0, 8, 20)):
        hstep = 1e-4
        fp, fm = ff.copy(), ff.copy()
        fp[p, c] += hstep
        fm[p, c] -= hstep
        lp = D.semantic_loss_grad(fp.astype(np.float64), ru, y, ws, bs, 1.0 / 777.0, 2.0, 0.25, False)["loss"]
        lm = D.semantic_loss_grad(fm.astype(np.float64), ru, y, ws, bs, 1.0 / 777.0, 2.0, 0.25, False)["loss"]
        assert r["d_feat"][p, c] == pytest.approx((lp - lm) / (2 * hstep), rel=1e-5, abs=1e-10)


def test_gradient_magnitude_sums(oracle_lib):
    """The magnitude sums behind the float32-aware gradient bound bound the
    gradients they belong to (|sum t| <= sum |t|, and through the chain
    rule's magnitude), and equal them when no term cancels: a positive
    upstream gradient on positive channels gives channel-gradient terms
    alpha T G > 0 only."""
    scene = synth.make_scene(800, 92, synth.VOL_C1, d_sem=2)
    cams = [synth.camera_front(64, 56, 64.0), synth.camera_front(48, 48, 50.0)]
    opts = O.make_opts(16)
    f = O.forward(scene, cams, opts)
    G = synth.upstream_grads(cams, scene.n_channels, 93).astype(np.float64)
    b = O.backward(scene, cams, opts, f, G, magnitudes=True)
    m = b["mag"]
    for grp in ("mean", "log_scale", "quat", "opacity_logit", "channels"):
        assert (np.abs(b[grp]) <= m[grp] * (1 + 1e-12) + 1e-300).all(), grp
        assert (m[grp] > 0).any()
    assert (np.abs(b["grad2d"]) <= m["grad2d"] * (1 + 1e-12) + 1e-300).all()
    bp = O.backward(scene, cams, opts, f, np.abs(G), magnitudes=True)
    pos = scene.channels >= 0
    assert np.allclose(bp["channels"][pos], bp["mag"]["channels"][pos], rtol=1e-12, atol=0)
