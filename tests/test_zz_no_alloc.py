"""The allocation-free semantic loss (legs_semantic_loss_grad_noalloc, whose
workspace is the library's fixed per-GPU array) against the entry point that
takes a caller-allocated workspace (legs_semantic_loss_grad), through the C
ABI, on two calls in a row, the second with fewer pixels; both are also
checked against the FP64 oracle of Sec. 3.4.2, Eqs. 10-12."""
import ctypes as ct
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import decode as D

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def _run(ctx, DEC, f, ru, y, params, K, inv_hw, noalloc):
    P = f.shape[0]
    grad = torch.zeros_like(params)
    loss = torch.zeros(1, device="cuda")
    d_feat = torch.full((P, 8), 7.0, device="cuda")
    d_ru = torch.full((P,), 7.0, device="cuda")
    fd = DEC.rowmajor_features(torch.from_numpy(f).cuda())
    rud, yd = torch.from_numpy(ru).cuda(), torch.from_numpy(y).cuda()
    if noalloc:
        DEC.semantic_loss_grad_noalloc(ctx, fd, rud, yd, params, K, inv_hw, grad, (d_feat, 1, 8), d_ru, loss)
    else:
        ws = DEC.workspace(ctx, P, K)
        DEC.semantic_loss_grad(ctx, fd, rud, yd, params, K, inv_hw, ws, grad, (d_feat, 1, 8), d_ru, loss)
    torch.cuda.synchronize()
    return (grad.cpu().numpy().astype(np.float64), loss.item(), d_feat.cpu().numpy(), d_ru.cpu().numpy())


def test_noalloc_matches_workspace_entry_point():
    from paper_2311_18482_amd import raster, decode as DEC, _lib as L
    ctx = raster.Context(0)
    K = 128
    ws_, bs_ = synth.mlp_init((8, 64, 64, K), 81)
    params = DEC.mlp_pack(ws_, bs_).cuda()
    rng = np.random.default_rng(80)
    for P in (DEC.NOALLOC_MAX_PIXELS, 3001):          # the second call is smaller
        note(f"noalloc semantic loss P={P}")
        f = rng.normal(0, 1, (P, 8)).astype(np.float32)
        ru = rng.uniform(0, 1, P).astype(np.float32)
        y = rng.integers(0, K, P).astype(np.int32)
        inv_hw = 1.0 / (2 * P)
        g_ws, l_ws, df_ws, dr_ws = _run(ctx, DEC, f, ru, y, params, K, inv_hw, noalloc=False)
        g_na, l_na, df_na, dr_na = _run(ctx, DEC, f, ru, y, params, K, inv_hw, noalloc=True)
        # per-pixel outputs: the same kernels on the same inputs, bit for bit
        assert np.array_equal(df_na, df_ws) and np.array_equal(dr_na, dr_ws)
        # the loss and the decoder gradient are float32 atomic sums (order varies)
        assert l_na == pytest.approx(l_ws, rel=1e-5)
        off = 0
        ref = D.semantic_loss_grad(f, ru, y, ws_, bs_, inv_hw, 1.0, 1.0)
        assert l_na == pytest.approx(ref["loss"], rel=1e-5)
        for w, b in zip(ref["gW"], ref["gb"]):
            for part in (w.reshape(-1), b):
                seg_na, seg_ws = g_na[off:off + part.size], g_ws[off:off + part.size]
                assert np.linalg.norm(seg_na - seg_ws) <= 1e-5 * np.linalg.norm(part), off
                assert np.linalg.norm(seg_na - part) <= 2e-3 * np.linalg.norm(part), off
                off += part.size
    # more pixels than the fixed workspace holds: refused, nothing launched
    P = DEC.NOALLOC_MAX_PIXELS + 1
    t = torch.zeros(P * 8, device="cuda")
    rc = L.lib().legs_semantic_loss_grad_noalloc(ctx.handle, t.data_ptr(), t.data_ptr(), P, 1, 8,
                                                 t.data_ptr(), K, 1, params.data_ptr(), 1.0, 1.0, 1.0,
                                                 t.data_ptr(), t.data_ptr(), 1, 8, t.data_ptr(), t.data_ptr(),
                                                 None)
    assert rc == -1
