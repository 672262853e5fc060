#!/usr/bin/env python
"""Throughput of the splatting hot path on one MI355X.

One step = project -> bin/sort -> blend forward -> blend backward ->
project backward for every view of the workload (the forward + backward
rasteriser pass of Sec. 3.1 Eq. 1 with the R_s and R_u channels of Sec. 3.4),
inputs resident in HBM. value = total view pixels / median step time, in
Mpixels/s. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload 1m_1080p]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd Mpixels/s, 1M Gaussians @1080p; learned vs plain decode @\u226599% top-1"
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
FLOPS_EVAL = 16        # one alpha evaluation: offsets, quadratic form, clamp, exp, opacity, tests


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name):
    import synth
    if name == "1m_1080p":
        scene, cams = synth.workload_1m_1080p()
        desc = "1M Gaussians in [-4,4]^3, 1 view 1920x1080 on the r=8 sphere, C=12 (RGB+8 sem+u)"
    elif name == "c2":
        scene, cams = synth.workload_c2()
        desc = "300k Gaussians, 1 view 1080x720, C=12"
    elif name == "c3":
        scene, cams = synth.workload_c3()
        desc = "1M Gaussians, 16 uneven views on the r=8 sphere, C=12"
    else:
        raise SystemExit(f"unknown workload {name}")
    return scene, cams, desc


# kernel of each stage and the source file it is built from
STAGE_KERNEL = {"blend_bwd": ("k_blend_bwd", "blend.hip"), "blend_fwd": ("k_blend_fwd", "blend.hip"),
                "project": ("k_project", "project.hip"), "project_bwd": ("k_project_backward", "project.hip")}


def measured_traffic(stage, args):
    """HBM bytes per launch of the stage's kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known
    size), or None when there is none for this workload or the kernel's source
    has changed since the counters were taken."""
    import hashlib
    if stage not in STAGE_KERNEL:
        return None
    kernel, src = STAGE_KERNEL[stage]
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{args.workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_2311_18482_amd", "csrc", src), "rb").read()).hexdigest()
    if rec.get("source_sha256") != sha or rec.get("tile") != args.tile or rec.get("lds_batch") != args.lds_batch:
        return None
    return rec["hbm_bytes_per_launch"]


def decode_leg(log_fn, epochs=200):
    """Learned vs plain decode on the 32-view 1080p workload (Sec. 3.3 Eq. 4 plain
    codebook decode; Eq. 8/9 MLP decoder trained on the GPU by this library):
    render the 8-dim semantic maps of all views, label 10M pixels sampled from
    views 0-15 with the plain decode, train the 8-64-64-128 decoder on them,
    then report top-1 agreement on views 16-31 and Mpixels/s of the learned,
    plain and folded-plain decodes over all 32 views (top-1 output)."""
    import math
    import torch
    import synth
    from paper_2311_18482_amd import raster as R, decode as DEC
    scene, cams = synth.workload_c4()
    dev = torch.device("cuda:0")
    d = {k: torch.from_numpy(getattr(scene, k)).to(dev)
         for k in ("mean", "log_scale", "quat", "opacity_logit", "channels")}
    C = scene.channels.shape[1]
    feats = []
    for v in range(len(cams)):
        rast = R.Rasterizer([cams[v]], R.opts())
        _, _, out, _, _ = rast.forward(d["mean"], d["log_scale"], d["quat"], d["opacity_logit"],
                                       d["channels"])
        hw = cams[v].width * cams[v].height
        feats.append(out.view(C, hw)[3:11].t().contiguous())   # [P][8] semantic channels
        del rast, out
    ntr = sum(f.shape[0] for f in feats[:16])
    ftr_all = torch.cat(feats[:16])
    fev = torch.cat(feats[16:])
    fall = torch.cat([ftr_all, fev])
    del feats
    ctx = R.Context(0)
    K = 128
    Pm = torch.from_numpy(synth.projection(512, 8, 4 + 400)).to(dev)
    Cb = torch.from_numpy(synth.codebook(K, 512, 4 + 401)).to(dev)
    g = torch.Generator(device=dev)
    g.manual_seed(4 + 402)
    pick = torch.randperm(ntr, device=dev, generator=g)[:10_000_000]
    ftr = ftr_all[pick].contiguous()
    del ftr_all
    ytr, _ = DEC.decode_plain(ctx, DEC.rowmajor_features(ftr), Pm, Cb)
    yev, _ = DEC.decode_plain(ctx, DEC.rowmajor_features(fev), Pm, Cb)
    B, lr0 = 65536, 1e-2
    n = ftr.shape[0]

    def train(normalize):
        ws, bs = synth.mlp_init((8, 64, 64, K), 4 + 403)
        tr = DEC.MlpTrainer(ctx, DEC.mlp_pack(ws, bs), K, B, lr=lr0, normalize=normalize)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        for ep in range(epochs):
            tr.lr = lr0 * 0.5 * (1.0 + math.cos(math.pi * ep / epochs))
            perm = torch.randperm(n, device=dev, generator=g)
            fs, ys = ftr[perm], ytr[perm]
            for i in range(0, n - B + 1, B):
                tr.step(DEC.rowmajor_features(fs[i:i + B]), ys[i:i + B])
                steps += 1
            if ep % 50 == 49 or ep == epochs - 1:
                log_fn(f"decoder ({'normalised' if normalize else 'raw'} input) epoch {ep + 1}/{epochs}")
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        top, _ = DEC.decode_mlp(ctx, DEC.rowmajor_features(fev), tr.params, K, normalize=normalize)
        return tr, float((top == yev).float().mean().item()), steps, train_s

    tr, agree, steps, train_s = train(True)
    tr_raw, agree_raw, _, _ = train(False)
    P = fall.shape[0]
    folded = DEC.decode_fold(ctx, Pm, Cb)
    top1 = torch.empty(P, dtype=torch.int32, device=dev)

    def tm(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    f_all = DEC.rowmajor_features(fall)
    ms = {"learned": tm(lambda: DEC.decode_mlp(ctx, f_all, tr.params, K, top1=top1)),
          "learned_raw_input": tm(lambda: DEC.decode_mlp(ctx, f_all, tr_raw.params, K, top1=top1, normalize=False)),
          "plain": tm(lambda: DEC.decode_plain(ctx, f_all, Pm, Cb)),
          "folded": tm(lambda: DEC.decode_folded(ctx, f_all, folded, K))}
    # the full distribution as well (float32 softmax of every class, with the top-1)
    probs = torch.empty((P, K), dtype=torch.float32, device=dev)
    lib = __import__("paper_2311_18482_amd._lib", fromlist=["lib"])
    st = R._stream()

    def learned_probs():
        ctx.check(lib.lib().legs_decode_mlp(ctx.handle, R._p(fall), P, 1, 8, R._p(tr.params), K,
                                            lib.LEGS_MLP_NORMALIZE_INPUT, R._p(probs), R._p(top1), st))
    ms["learned_probs"] = tm(learned_probs)
    del probs
    torch.cuda.empty_cache()
    mpx = {k: P / (v * 1e-3) / 1e6 for k, v in ms.items()}
    probs_bytes = P * (8 * 4 + K * 4 + 4)        # features read, float32 distribution and top-1 written
    return dict(workload="1M Gaussians, 32 views 1920x1080 (C=12, 8-dim semantic maps), codebook "
                         "128 x 512, projection 512 x 8, decoder 8-64-64-128 bf16 on the L2-normalised "
                         "rendered feature (top-1 output)",
                pixels=int(P), top1_agreement=agree, top1_agreement_raw_input=agree_raw,
                train_pairs=int(n), train_steps=steps, train_s=train_s,
                learned_mpx_s=mpx["learned"], learned_raw_input_mpx_s=mpx["learned_raw_input"],
                plain_mpx_s=mpx["plain"], folded_mpx_s=mpx["folded"],
                learned_over_plain=mpx["learned"] / mpx["plain"],
                learned_over_folded=mpx["learned"] / mpx["folded"],
                learned_probs_mpx_s=mpx["learned_probs"],
                learned_probs_roofline=dict(bound="hbm", unit="GB/s", bytes_per_px=8 * 4 + K * 4 + 4,
                                            achieved=probs_bytes / (ms["learned_probs"] * 1e-3) / 1e9,
                                            peak=HBM_PEAK_GBS,
                                            frac=probs_bytes / (ms["learned_probs"] * 1e-3) / 1e9 / HBM_PEAK_GBS),
                ms=ms)


BF16_MFMA_PEAK_TFLOPS = 2500.0    # dense bf16 / fp16 MFMA


def _timer(reps=5):
    import torch

    def tm(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))
    return tm


def language_leg(log_fn):
    """Rows beyond the rasteriser, each on its own synthetic input of the
    paper's shapes (random-init weights; what is timed is the kernel work):
      paper_decoder  Table 3 decoder 8-128-256-128 over four 1920x1080 views of
                     8-d rendered features (top-1 only, and the fp16
                     distribution M_infer), then F = M_infer S with S 128 x 512
                     (supplementary inference equations), F planar float32 / half;
      quantize       1M hybrid features (512 CLIP + 384 DINO dims, half) against
                     a 128-code feature space: Eqs. 4-7 with the gradient;
      smooth         L_smo (Eqs. 13-14) with every gradient over the 1M Gaussians
                     of the 1080p scene."""
    import torch
    import synth
    from paper_2311_18482_amd import raster as R, decode as DEC
    dev = torch.device("cuda:0")
    ctx = R.Context(0)
    tm = _timer()
    res = {}
    # --- Table 3 decoder and F = M S
    P, N, d = 4 * 1920 * 1080, 128, 512
    g = torch.Generator(device=dev).manual_seed(190)
    feat = torch.randn((P, 8), generator=g, device=dev)
    ws, bs = synth.mlp_init((8, 128, 256, N), 191)
    params = DEC.mlp_pack(ws, bs).to(dev)
    S = torch.from_numpy(synth.codebook(N, d, 192)).to(dev)
    fr = DEC.rowmajor_features(feat)
    top1 = torch.empty(P, dtype=torch.int32, device=dev)
    p16 = torch.empty((P, N), dtype=torch.float16, device=dev)
    F32 = torch.empty((d, P), dtype=torch.float32, device=dev)
    lib = __import__("paper_2311_18482_amd._lib", fromlist=["lib"]).lib()
    st = R._stream()

    def dec_top1():
        ctx.check(lib.legs_decode_dmlp(ctx.handle, R._p(feat), P, 1, 8, R._p(params), N, 0, None, None,
                                       R._p(top1), st))

    def dec_probs():
        ctx.check(lib.legs_decode_dmlp(ctx.handle, R._p(feat), P, 1, 8, R._p(params), N, 0, None, R._p(p16),
                                       R._p(top1), st))
    ms_t = tm(dec_top1)
    ms_p = tm(dec_probs)
    ms_f = tm(lambda: DEC.language_features(ctx, p16, S, F=F32))
    F16 = F32.view(-1).view(torch.float16)[: d * P].view(d, P)
    ms_h = tm(lambda: DEC.language_features(ctx, p16, S, out_f16=True, F=F16))
    flop_px = 2 * (8 * 128 + 128 * 256 + 256 * N)
    fbytes = lambda ob: P * (N * 2 * ((d + 511) // 512) + d * ob)   # M read once per 512-dimension chunk
    res["paper_decoder"] = dict(
        workload=f"Table 3 decoder 8-128-256-{N} (bf16) on {P} px (4 views 1920x1080) of N(0,1) features; "
                 f"F = M S with S {N} x {d}",
        pixels=P, ms=dict(top1=ms_t, probs_f16=ms_p, features_f32=ms_f, features_f16=ms_h),
        mpx_s=dict(top1=P / ms_t / 1e3, probs_f16=P / ms_p / 1e3, features_f32=P / ms_f / 1e3),
        roofline=dict(decoder=dict(bound="mfma", unit="TFLOP/s", achieved=P * flop_px / ms_t / 1e9,
                                   peak=BF16_MFMA_PEAK_TFLOPS,
                                   frac=P * flop_px / ms_t / 1e9 / BF16_MFMA_PEAK_TFLOPS,
                                   flop_per_px=flop_px),
                      features_f32=dict(bound="hbm", unit="GB/s", achieved=fbytes(4) / ms_f / 1e6, peak=HBM_PEAK_GBS,
                                        frac=fbytes(4) / ms_f / 1e6 / HBM_PEAK_GBS, bytes_per_px=fbytes(4) / P),
                      features_f16=dict(bound="hbm", unit="GB/s", achieved=fbytes(2) / ms_h / 1e6, peak=HBM_PEAK_GBS,
                                        frac=fbytes(2) / ms_h / 1e6 / HBM_PEAK_GBS, bytes_per_px=fbytes(2) / P)))
    log_fn(f"paper decoder: {json.dumps(res['paper_decoder'])}")
    del feat, top1, p16, F32, F16
    torch.cuda.empty_cache()
    # --- quantisation
    K, N, dc, dd = 1 << 20, 128, 512, 384
    d = dc + dd
    rng = np.random.default_rng(193)
    Sq = rng.normal(0, 1, (N, d)).astype(np.float32)
    Ft = (torch.from_numpy(Sq).to(dev)[torch.randint(0, N, (K,), generator=g, device=dev)] +
          1.5 * torch.randn((K, d), generator=g, device=dev)).half().contiguous()
    Sd = torch.from_numpy(Sq).to(dev)
    wsq = torch.empty(int(lib.legs_quantize_workspace_bytes(K, N, d)), dtype=torch.uint8, device=dev)
    ms_a = tm(lambda: DEC.quantize(ctx, Ft, Sd, dc, grad=False, workspace=wsq))
    ms_g = tm(lambda: DEC.quantize(ctx, Ft, Sd, dc, grad=True, workspace=wsq))
    fl = 2 * K * N * d
    res["quantize"] = dict(
        workload=f"{K} hybrid features ({dc} CLIP + {dd} DINO dims, half) scattered around a {N}-code space; "
                 f"lambda_DINO = lambda_lb = 0.5, lambda_cos = 1",
        features=K, ms=dict(assign=ms_a, assign_and_grad=ms_g),
        mfeat_s=dict(assign=K / ms_a / 1e3, assign_and_grad=K / ms_g / 1e3),
        roofline=dict(assign=dict(bound="hbm", unit="GB/s", achieved=K * d * 2 / ms_a / 1e6, peak=HBM_PEAK_GBS,
                                  frac=K * d * 2 / ms_a / 1e6 / HBM_PEAK_GBS, bytes_per_feature=d * 2,
                                  mfma_frac=fl / ms_a / 1e9 / BF16_MFMA_PEAK_TFLOPS),
                      assign_and_grad=dict(bound="hbm", unit="GB/s", achieved=2 * K * d * 2 / ms_g / 1e6,
                                           peak=HBM_PEAK_GBS, frac=2 * K * d * 2 / ms_g / 1e6 / HBM_PEAK_GBS,
                                           bytes_per_feature=2 * d * 2,
                                           mfma_frac=3 * fl / ms_g / 1e9 / BF16_MFMA_PEAK_TFLOPS)))
    log_fn(f"quantize: {json.dumps(res['quantize'])}")
    del Ft, Sd, wsq
    torch.cuda.empty_cache()
    # --- smoothing
    scene, _ = synth.workload_1m_1080p()
    n, C = scene.channels.shape
    mean = torch.from_numpy(scene.mean).to(dev)
    chans = torch.from_numpy(scene.channels).to(dev)
    ws3, bs3 = synth.mlp_init((3, 128, 128, 128, 8), 194)
    sp = torch.cat([torch.from_numpy(np.concatenate([W.reshape(-1), b])) for W, b in zip(ws3, bs3)]).to(dev)
    grad = torch.zeros_like(sp)
    dch = torch.zeros_like(chans)
    loss = torch.zeros(1, device=dev)
    wss = DEC.smooth_workspace(ctx, n)
    ms_s = tm(lambda: DEC.smooth_loss_grad(ctx, mean, chans, 3, C - 1, sp, grad, dch, loss, workspace=wss))
    flop_g = 2 * (3 * 128 + 2 * 128 * 128 + 128 * 8) * 3       # forward, input-side backward, weight gradient
    # HBM bytes per Gaussian: the workspace planes written by the forward and
    # read by the weight gradient (x 16 rows, h1-h3 128 rows bf16, dz1-dz3 128
    # rows and dz4 8 rows as two bf16 parts), position and s_G, u read, and the
    # read-modify-write of the 8 channel-gradient floats
    planes_b = 16 * 2 + 3 * 128 * 2 + 3 * 128 * 4 + 8 * 4
    bytes_g = 2 * planes_b + 12 + 9 * 4 + 2 * 8 * 4
    res["smooth"] = dict(
        workload=f"L_smo and its gradients over {n} Gaussians (the 1080p scene), MLP 3-128-128-128-8 bf16",
        gaussians=int(n), ms=ms_s, mgauss_s=n / ms_s / 1e3,
        roofline=dict(bound="hbm", unit="GB/s", achieved=n * bytes_g / ms_s / 1e6, peak=HBM_PEAK_GBS,
                      frac=n * bytes_g / ms_s / 1e6 / HBM_PEAK_GBS, bytes_per_gaussian=bytes_g,
                      mfma_frac=n * flop_g / ms_s / 1e9 / BF16_MFMA_PEAK_TFLOPS, flop_per_gaussian=flop_g))
    log_fn(f"smooth: {json.dumps(res['smooth'])}")
    return res


def c5_leg(log_fn, steps, warmup):
    """One optimisation step of every per-Gaussian parameter (render, L1 +
    L_u, backward, fused Adam) at 3M Gaussians x 4 views 1920x1080, C = 20,
    replayed as one HIP graph."""
    import torch
    import synth
    from paper_2311_18482_amd import raster as R
    from paper_2311_18482_amd.train import TrainStep
    dev = torch.device("cuda:0")
    scene, cams = synth.workload_c5()
    n, C = scene.channels.shape
    d_sem = C - 4
    target = torch.from_numpy(synth.targets_l1(cams, C, d_sem, 205)).to(dev)
    params = {k: torch.from_numpy(np.ascontiguousarray(v)).to(dev) for k, v in
              (("mean", scene.mean), ("log_scale", scene.log_scale), ("quat", scene.quat),
               ("opacity_logit", scene.opacity_logit), ("channels", scene.channels))}
    torch.cuda.reset_peak_memory_stats()
    ts = TrainStep(cams, params, target, d_sem, o=R.opts(tile=32, lds_batch=256, ids_only=True))
    for _ in range(warmup):
        ts.step()
    torch.cuda.synchronize()
    g = ts.capture(step_number=warmup + 1)
    g.launch()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        g.launch()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    px = sum(c.width * c.height for c in cams)
    res = dict(workload=f"{n} Gaussians in [-4,4]^3, {len(cams)} views 1920x1080, C={C} (RGB + {d_sem} sem + u); "
                        f"per-view L1 + L_u, Adam on all {n * (11 + C)} floats",
               ms_per_step=ms, mpx_s=px / ms / 1e3, instances=int(ts.bins.count.item()),
               overflowed=bool(ts.overflowed()), peak_mem_gib=torch.cuda.max_memory_allocated() / 2 ** 30)
    log_fn(f"c5: {json.dumps(res)}")
    return res


def _oracle_step(O, scene, cams, oo, G):
    """One forward + backward of the oracle, stage by stage; returns seconds per stage."""
    t = {}
    t0 = time.perf_counter()
    params = O.Params.from_scene(scene)
    proj = O.project_views(params, cams, oo)
    t["project"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    keys, ids, ranges = O.bin_lists(proj, cams, oo)
    t["bin_sort"] = time.perf_counter() - t0
    _, _, offsets, _ = O.view_tables(cams, oo.tile)
    t0 = time.perf_counter()
    for v, cam in enumerate(cams):
        O.render_view(proj[v], cam, oo, scene.channels, ids, ranges, offsets[v])
    t["blend_fwd"] = time.perf_counter() - t0
    n, C = scene.channels.shape
    dch = np.zeros((n, C))
    acc = None
    t["blend_bwd"] = t["project_bwd"] = 0.0
    off = 0
    for v, cam in enumerate(cams):
        hw = cam.width * cam.height
        t0 = time.perf_counter()
        g2, dch = O.render_backward_view(proj[v], cam, oo, scene.channels, ids, ranges, offsets[v],
                                         G[off:off + C * hw].reshape(C, hw), None, dch)
        t["blend_bwd"] += time.perf_counter() - t0
        t0 = time.perf_counter()
        acc = O.project_backward(params, cam, oo, g2, acc)
        t["project_bwd"] += time.perf_counter() - t0
        off += C * hw
    return t


def cpu_baseline(scene, cams, tile):
    """The FP64 oracle as it stands, on this host's cores: one full forward +
    backward of the same workload (projection, lists, blending, backward) on
    every thread OpenMP gives it, then the same step on one thread, both with
    per-stage times."""
    import synth
    from oracle import oracle as O
    oo = O.make_opts(tile)
    px = sum(c.width * c.height for c in cams)
    G = synth.upstream_grads(cams, scene.n_channels, 200).astype(np.float64)
    nth = O.threads()
    st = _oracle_step(O, scene, cams, oo, G)
    dt = sum(st.values())
    O.set_threads(1)
    try:
        st1 = _oracle_step(O, scene, cams, oo, G)
    finally:
        O.set_threads(nth)
    dt1 = sum(st1.values())
    # the oracle's decodes (Eq. 4 plain, Eq. 8 learned with the bf16 roundings
    # emulated; numpy, its BLAS on this host's threads) on a pixel sample
    from oracle import decode as D
    npx = 200_000
    fs = np.random.default_rng(400).normal(0, 1, (npx, 8)).astype(np.float32)
    Pm, Cb = synth.projection(512, 8, 404), synth.codebook(128, 512, 405)
    ws, bs = synth.mlp_init((8, 64, 64, 128), 407)
    t0 = time.perf_counter()
    D.decode_plain(fs, Pm, Cb)
    t_plain = time.perf_counter() - t0
    t0 = time.perf_counter()
    np.argmax(D.mlp_forward(fs, ws, bs)["logits"], axis=1)
    t_learned = time.perf_counter() - t0
    decode = dict(sample=f"{npx} pixels of 8-d features, codebook 128 x 512, decoder 8-64-64-128",
                  plain_mpx_s=npx / t_plain / 1e6, learned_mpx_s=npx / t_learned / 1e6,
                  plain_s=t_plain, learned_s=t_learned)
    return dict(value=px / dt / 1e6, unit="Mpixels/s", cores=nth, kind="oracle",
                sample=f"one full forward+backward step of the same workload ({px} px), {dt:.1f} s on {nth} "
                       f"threads",
                stage_s=st,
                single_thread=dict(value=px / dt1 / 1e6, unit="Mpixels/s", cores=1,
                                   sample=f"the same step on one thread, {dt1:.1f} s", stage_s=st1),
                decode=decode)


def coarse_entries(proj, tile, sx=8, sy=4):
    """Super-tile entries of the two-level binning (8 x 4-tile super-tiles):
    statistics for the byte model, computed on the host from the boxes."""
    box = proj.box.cpu().numpy().astype(np.int64)
    vis = proj.ntiles.cpu().numpy() > 0
    tx0, tx1, ty0, ty1 = (box[vis, k] // tile for k in range(4))
    return int(((tx1 // sx - tx0 // sx + 1) * (ty1 // sy - ty0 // sy + 1)).sum())


class StepRunner:
    """Buffers and the captured HIP graph of one forward + backward step
    (project -> bin/sort -> blend forward -> blend backward -> project
    backward) for a scene and a camera rig, inputs resident in HBM. Every
    kernel of the step is the library's; the blend forward also zeroes the
    gradient buffers the backward accumulates into (legs_render_forward_zero)."""

    STAGES = ("project", "bin_sort", "blend_fwd", "blend_bwd", "project_bwd")

    def __init__(self, R, scene, cams, o, G, dev):
        import torch
        self.R, self.o = R, o
        self.rast = R.Rasterizer(cams, o)
        ctx, views = self.rast.ctx, self.rast.views
        self.d = {k: torch.from_numpy(getattr(scene, k)).to(dev)
                  for k in ("mean", "log_scale", "quat", "opacity_logit", "channels")}
        n, C = scene.channels.shape
        self.n, self.C = n, C
        self.proj = R.ProjectedBuf(n, views.n_views, dev)
        R.project(ctx, self.d["mean"], self.d["log_scale"], self.d["quat"], self.d["opacity_logit"], views, o,
                  out=self.proj)
        bins = R.bin_sort(ctx, self.proj, views, o)            # sizes the lists once (host read-back)
        self.n_inst = bins.n_instances
        del bins
        self.bins = R.BinsBuf(int(self.n_inst * 1.05) + 4096, views.total_tiles, dev)
        self.out = torch.empty(C * views.total_pixels, dtype=torch.float32, device=dev)
        self.T = torch.empty(views.total_pixels, dtype=torch.float32, device=dev)
        self.last = torch.empty(views.total_pixels, dtype=torch.int32, device=dev)
        self.G = G
        # every gradient buffer is a slice of one flat allocation, zeroed by the forward launch
        gshapes = {"grad2d": (n * views.n_views, 8), "d_ch": (n, C)}
        gshapes.update({k: tuple(self.d[k].shape) for k in ("mean", "log_scale", "quat", "opacity_logit")})
        self.gflat = torch.zeros(sum(int(np.prod(sh)) for sh in gshapes.values()), dtype=torch.float32, device=dev)
        self.gv, at = {}, 0
        for k, sh in gshapes.items():
            self.gv[k] = self.gflat[at:at + int(np.prod(sh))].view(sh)
            at += int(np.prod(sh))
        self.graph = None

    def step(self, ev=None):
        R, ctx, views, o, d = self.R, self.rast.ctx, self.rast.views, self.o, self.d

        def mark(i):
            if ev is not None:
                ev[i].record()
        mark(0)
        R.project(ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"], views, o, out=self.proj)
        mark(1)
        R.bin_sort(ctx, self.proj, views, o, self.bins, sync_count=False)
        mark(2)
        R.render_forward(ctx, self.proj, self.bins, views, d["channels"], o, self.out, self.T, self.last,
                         zero=self.gflat)
        mark(3)
        R.render_backward(ctx, self.proj, self.bins, views, d["channels"], o, self.T, self.last, self.G,
                          self.gv["grad2d"], self.gv["d_ch"])
        mark(4)
        grads = {k: self.gv[k] for k in ("mean", "log_scale", "quat", "opacity_logit")}
        R.project_backward(ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"], views, o, self.proj,
                           self.gv["grad2d"], grads)
        mark(5)

    def time_eager(self, steps, warmup):
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        assert int(self.bins.count.item()) <= self.bins.capacity, "instance list overflowed"
        evs = [[torch.cuda.Event(enable_timing=True) for _ in range(6)] for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            self.step(evs[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_step = np.array([evs[k][0].elapsed_time(evs[k][5]) for k in range(steps)])
        stage_ms = {s_: float(np.median([evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(steps)]))
                    for i, s_ in enumerate(self.STAGES)}
        return float(np.median(per_step)), stage_ms, wall

    def time_graph(self, steps, warmup):
        """The same step captured once as a HIP graph (every call is capturable:
        the binning reads its sizes on the device) and replayed: each timed
        step is one graph launch doing the whole step's work."""
        import torch
        if self.graph is None:
            self.graph = self.R.Graph(self.rast.ctx)
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                with self.graph.capture():
                    self.step()
            torch.cuda.current_stream().wait_stream(side)
        for _ in range(warmup):
            self.graph.launch()
        torch.cuda.synchronize()
        gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e0, e1 in gev:
            e0.record()
            self.graph.launch()
            e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        assert int(self.bins.count.item()) <= self.bins.capacity, "instance list overflowed"
        return float(np.median([e0.elapsed_time(e1) for e0, e1 in gev])), wall


def c3_leg(log_fn, steps, warmup):
    """The 16-view batch: 1M Gaussians seen by 16 cameras of uneven resolution
    on the r=8 sphere, forward + backward of all views per step. The
    autotuner sweeps tile {8, 16, 32} x LDS batch {64, 128, 256}; the chosen
    setting is then timed as a replayed HIP graph with the blend kernels
    launched one workgroup per tile and as persistent launches."""
    import torch
    import synth
    from paper_2311_18482_amd import raster as R
    scene, cams = synth.workload_c3()
    dev = torch.device("cuda:0")
    C = scene.n_channels
    G = torch.from_numpy(synth.upstream_grads(cams, C, 203)).to(dev)
    d = {k: torch.from_numpy(getattr(scene, k)).to(dev)
         for k in ("mean", "log_scale", "quat", "opacity_logit", "channels")}
    ctx = R.Context(0)
    log_fn("c3: autotune over tile x LDS batch")
    best, table = R.autotune(ctx, d["mean"], d["log_scale"], d["quat"], d["opacity_logit"], d["channels"], cams,
                             R.opts(persistent=True, ids_only=True), d_out=G, reps=2)
    del d
    torch.cuda.empty_cache()
    px = sum(c.width * c.height for c in cams)
    res = dict(workload="1M Gaussians in [-4,4]^3, 16 views of uneven resolution on the r=8 sphere, C=12",
               views=len(cams), pixels=int(px), resolutions=[[c.width, c.height] for c in cams],
               autotune=dict(ms={f"tile{t}_batch{b}": v for (t, b), v in table.items()},
                             best=dict(tile=int(best.tile), lds_batch=int(best.lds_batch))))
    for persistent in (False, True):
        o = R.opts(tile=best.tile, lds_batch=best.lds_batch, persistent=persistent, ids_only=True)
        run = StepRunner(R, scene, cams, o, G, dev)
        eager_ms, stage_ms, _ = run.time_eager(steps, warmup)
        graph_ms, _ = run.time_graph(steps, warmup)
        key = "persistent" if persistent else "one_workgroup_per_tile"
        res[key] = dict(ms_per_step=graph_ms, mpx_s=px / (graph_ms * 1e-3) / 1e6, eager_ms_per_step=eager_ms,
                        stage_ms=stage_ms, instances=int(run.n_inst))
        log_fn(f"c3 {key}: {json.dumps(res[key])}")
        del run
        torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="1m_1080p")
    ap.add_argument("--tile", type=int, default=32)
    ap.add_argument("--lds-batch", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-decode", action="store_true", help="skip the learned-vs-plain decode leg")
    ap.add_argument("--no-c3", action="store_true", help="skip the 16-view batch leg")
    ap.add_argument("--no-language", action="store_true",
                    help="skip the Table 3 decoder / feature map, quantisation and smoothing legs")
    ap.add_argument("--no-c5", action="store_true", help="skip the 3M-Gaussian training-step leg")
    ap.add_argument("--decode-epochs", type=int, default=200,
                    help="decoder training epochs of the decode leg (fewer only to profile its kernels)")
    ap.add_argument("--eager", action="store_true",
                    help="report the eagerly launched step instead of the replayed HIP graph of the step")
    ap.add_argument("--persistent", action="store_true", help="persistent blend kernels (tiles from a counter)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed steps, run one plain 1 GiB elementwise copy (torch.neg), "
                         "the reference dispatch that scales FETCH_SIZE / WRITE_SIZE to bytes")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the rasteriser would shard by view with one gradient all-reduce).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2311_18482_amd import raster as R

    scene, cams, desc = workload(args.workload)
    log(f"workload {desc}")
    # the blend kernels read the tile lists' ids and ranges; the 64-bit keys are
    # not written (LEGS_FLAG_IDS_ONLY)
    o = R.opts(tile=args.tile, lds_batch=args.lds_batch, persistent=args.persistent, ids_only=True)
    dev = torch.device("cuda:0")
    n, C = scene.channels.shape
    G = torch.from_numpy(__import__("synth").upstream_grads(cams, C, 200)).to(dev)
    run = StepRunner(R, scene, cams, o, G, dev)
    rast, views, proj, bins, n_inst = run.rast, run.rast.views, run.proj, run.bins, run.n_inst
    eager_ms, stage_ms, wall = run.time_eager(args.steps, args.warmup)
    log(f"eager step {eager_ms:.3f} ms; stages (median ms): {json.dumps(stage_ms)}; wall {wall:.3f}s for "
        f"{args.steps} steps; instances {n_inst}")
    graph_ms = None
    if not args.eager:
        graph_ms, gwall = run.time_graph(args.steps, args.warmup)
        log(f"graph step {graph_ms:.3f} ms; wall {gwall:.3f}s for {args.steps} replays")
    ms = eager_ms if graph_ms is None else graph_ms
    px = views.total_pixels
    value = px / (ms * 1e-3) / 1e6

    # Algorithmic work per stage (section "Roofline" of the design notes):
    #  - bin_sort: bytes of emission, the onesweep passes and the ranges per instance;
    #  - project / project_bwd: bytes read and written per (Gaussian, view);
    #  - blend_fwd / blend_bwd: FP32 vector flops per alpha evaluation and per
    #    blended entry, from the work counts of the lists (a statistics pass run
    #    once, outside the timed steps).
    ev, blended, ev_bwd, _walked = R.render_counts(rast.ctx, proj, bins, views, o)
    G_views = n * views.n_views
    # depth passes of the G-view sort: 8-bit digits over the 32 depth bits and
    # the view bits, ceil(log2(views)) (none for one view)
    gpasses = (32 + int(np.ceil(np.log2(views.n_views))) + 7) // 8
    # bytes per G-view and pass: the G-view index travels in the key's low bits
    # (8 B each way) when the index and the digits fit in 64 bits, else a
    # separate 4 B id follows the 8 B key
    gbits = int(np.ceil(np.log2(G_views))) if G_views > 1 else 0
    pass_b = 16 if 0 < gbits and gbits + 8 * gpasses <= 64 else 24
    n_coarse = coarse_entries(proj, args.tile)
    work = {
        "project": ("hbm", G_views * (44 + 16 + 16 + 16 + 4 + 4)),
        # per G-view: the depth sort (pass_b per pass), the records (36 B read,
        # 32 B written), the cell counts (32 B) and the coarse emission (16 B);
        # per super-tile entry: the coarse pass writes 8 B, the compaction reads
        # the list and the tile record twice (40 B); per instance: the
        # compaction writes the 4 B id (no key: ids only)
        "bin_sort": ("hbm", G_views * (pass_b * gpasses + 68 + 32 + 16) + n_coarse * 48 + n_inst * 4),
        "project_bwd": ("hbm", G_views * (44 + 32 + 44 + 4)),
        "blend_fwd": ("alu", ev * FLOPS_EVAL + blended * (4 + 2 * C)),
        "blend_bwd": ("alu", ev_bwd * FLOPS_EVAL + blended * (40 + 7 * C)),
    }

    def roof(stage):
        bound, amount = work[stage]
        sec = stage_ms[stage] * 1e-3
        if bound == "hbm":
            ach = amount / sec / 1e9
            return dict(bound="hbm", kernel=stage, achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=ach / HBM_PEAK_GBS, traffic=None)
        ach = amount / sec / 1e12
        return dict(bound="alu", kernel=stage, achieved=ach, peak=FP32_VECTOR_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=ach / FP32_VECTOR_PEAK_TFLOPS, traffic=None)

    # the dominant kernel among the single-kernel stages (bin_sort is a chain of
    # kernels and is reported with the other stages)
    dom = max((s_ for s_ in work if s_ != "bin_sort"), key=lambda s_: stage_ms[s_])
    roofline = roof(dom)
    roofline["traffic"] = measured_traffic(dom, args)
    roofline["other_stages"] = {s_: {k: roof(s_)[k] for k in ("bound", "achieved", "unit", "frac")}
                                for s_ in work if s_ != dom}
    log(f"work counts: evaluations {ev} blended {blended} bwd evaluations {ev_bwd}; "
        f"roofline {json.dumps(roofline)}")

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.neg(src, out=dst)          # one elementwise dispatch: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        log("copy calibration: 1 GiB read, 1 GiB written (neg kernel)")
        del src, dst

    del run, rast, proj, bins
    torch.cuda.empty_cache()
    c3 = None
    if not args.no_c3 and args.workload == "1m_1080p":
        log("16-view leg: autotune, then one-workgroup-per-tile and persistent blend launches")
        c3 = c3_leg(log, max(5, args.steps // 2), 2)
        torch.cuda.empty_cache()

    dec = None
    if not args.no_decode and args.workload == "1m_1080p":
        log("decode leg: render 32 views, label, train the decoder, time the decodes")
        dec = decode_leg(log, epochs=args.decode_epochs)
        log(f"decode: {json.dumps(dec)}")

    lang = None
    if not args.no_language and args.workload == "1m_1080p":
        log("language legs: Table 3 decoder and F, quantisation, smoothing")
        lang = language_leg(log)
        torch.cuda.empty_cache()

    c5 = None
    if not args.no_c5 and args.workload == "1m_1080p":
        log("c5 leg: training step at 3M Gaussians x 4 views")
        c5 = c5_leg(log, max(5, args.steps // 2), 2)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        cpu = cpu_baseline(scene, cams, args.tile)

    rec = dict(metric=METRIC, value=value, unit="Mpixels/s",
               n_gpus=1, steps=args.steps, warmup=args.warmup, ms_per_step=ms,
               higher_is_better=True, scaling="weak", vs_baseline=None, dtype="f32",
               data="synthetic",
               config=dict(workload=desc, n_gaussians=int(n), views=len(cams), pixels=int(px),
                           channels=int(C), tile=args.tile, lds_batch=args.lds_batch,
                           instances=int(n_inst), super_tile_entries=int(n_coarse), alpha_evaluations=int(ev),
                           blended_entries=int(blended), stage_ms=stage_ms,
                           launch="eager" if graph_ms is None else "hip graph replay of the whole step",
                           eager_ms_per_step=eager_ms, persistent_blend=bool(args.persistent)),
               roofline=roofline, c3=c3, decode=dec, language=lang, c5=c5, cpu_baseline=cpu)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
