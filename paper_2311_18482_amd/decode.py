"""Python face of the decoding, decoder-training, Adam and loss calls of
liblegs.so (names of the C ABI without the `legs_` prefix). Marshalling only:
every step runs in the HIP kernels behind include/legs.h.

Feature arguments are (tensor, P, c_stride, p_stride): element (p, c) of a
rendered compact feature is tensor[c * c_stride + p * p_stride].
"""
from __future__ import annotations

import ctypes as ct

import torch

from . import _lib as L
from .raster import Context, _p, _stream

DIN = 8


def planar_features(out, views, C, first_channel, view=None):
    """Feature view into render_forward's planar output: returns
    (base tensor, P, c_stride, p_stride) for one view (or for all pixels when
    the output holds a single view)."""
    v = 0 if view is None else view
    W, H = views.sizes[v]
    hw = W * H
    off = C * views.pixel_offsets[v] + first_channel * hw
    return out[off:], hw, hw, 1


def rowmajor_features(feat):
    assert feat.dim() == 2 and feat.shape[1] == DIN and feat.is_contiguous()
    return feat, int(feat.shape[0]), 1, DIN


def _feat_args(f):
    t, P, cs, ps = f
    assert t.is_cuda and t.dtype == torch.float32
    return _p(t), int(P), int(cs), int(ps)


def decode_plain(ctx: Context, f, proj, codebook, probs=False):
    tp, P, cs, ps = _feat_args(f)
    K, D = codebook.shape
    top1 = torch.empty(max(P, 1), dtype=torch.int32, device=ctx.device)
    pr = torch.empty((P, K), dtype=torch.float32, device=ctx.device) if probs else None
    ctx.check(L.lib().legs_decode_plain(ctx.handle, tp, P, cs, ps, _p(proj), D, _p(codebook), K,
                                        _p(pr), _p(top1), _stream()))
    return top1[:P], pr


def decode_fold(ctx: Context, proj, codebook):
    K, D = codebook.shape
    folded = torch.empty((K + DIN) * DIN, dtype=torch.float32, device=ctx.device)
    ctx.check(L.lib().legs_decode_fold(ctx.handle, _p(proj), D, _p(codebook), K, _p(folded),
                                       _stream()))
    return folded


def decode_folded(ctx: Context, f, folded, K, probs=False):
    tp, P, cs, ps = _feat_args(f)
    top1 = torch.empty(max(P, 1), dtype=torch.int32, device=ctx.device)
    pr = torch.empty((P, K), dtype=torch.float32, device=ctx.device) if probs else None
    ctx.check(L.lib().legs_decode_folded(ctx.handle, tp, P, cs, ps, _p(folded), K, _p(pr),
                                         _p(top1), _stream()))
    return top1[:P], pr


def mlp_param_count(K):
    return int(L.lib().legs_mlp_param_count(K))


def mlp_pack(ws, bs):
    """Pack [W1, W2, W3], [b1, b2, b3] (float32, W as [out][in]) in ABI order."""
    parts = []
    for W, b in zip(ws, bs):
        parts += [torch.as_tensor(W, dtype=torch.float32).reshape(-1),
                  torch.as_tensor(b, dtype=torch.float32).reshape(-1)]
    return torch.cat(parts)


def mlp_flags(normalize: bool) -> int:
    return L.LEGS_MLP_NORMALIZE_INPUT if normalize else 0


def decode_mlp(ctx: Context, f, params, K, probs=False, top1=None, normalize=True):
    tp, P, cs, ps = _feat_args(f)
    if top1 is None:
        top1 = torch.empty(max(P, 1), dtype=torch.int32, device=ctx.device)
    pr = torch.empty((P, K), dtype=torch.float32, device=ctx.device) if probs else None
    ctx.check(L.lib().legs_decode_mlp(ctx.handle, tp, P, cs, ps, _p(params), K, mlp_flags(normalize),
                                      _p(pr), _p(top1), _stream()))
    return top1[:P], pr


def dmlp_param_count(N):
    return int(L.lib().legs_dmlp_param_count(N))


def decode_dmlp(ctx: Context, f, params, N, probs=False, probs_f16=False, top1=True, normalize=False):
    """Table 3 decoder (legs_decode_dmlp). Returns (top1 [P] int32 or None,
    probs [P][N] float32 or None, probs_f16 [P][N] float16 or None)."""
    tp, P, cs, ps = _feat_args(f)
    dev = ctx.device
    t1 = torch.empty(max(P, 1), dtype=torch.int32, device=dev) if top1 else None
    pr = torch.empty((P, N), dtype=torch.float32, device=dev) if probs else None
    p16 = torch.empty((P, N), dtype=torch.float16, device=dev) if probs_f16 else None
    ctx.check(L.lib().legs_decode_dmlp(ctx.handle, tp, P, cs, ps, _p(params), N, mlp_flags(normalize),
                                       _p(pr), _p(p16), _p(t1), _stream()))
    return (t1[:P] if t1 is not None else None), pr, p16


def language_features(ctx: Context, probs_f16, S, out_f16=False, F=None):
    """F = M S planar [d][P] (legs_language_features); probs_f16 [P][N]
    float16, S [N][d] float32."""
    assert probs_f16.dtype == torch.float16 and probs_f16.is_contiguous()
    assert S.dtype == torch.float32 and S.is_contiguous()
    P, N = probs_f16.shape
    d = S.shape[1]
    if F is None:
        F = torch.empty((d, P), dtype=torch.float16 if out_f16 else torch.float32, device=ctx.device)
    ctx.check(L.lib().legs_language_features(ctx.handle, _p(probs_f16), P, N, _p(S), d, int(bool(out_f16)),
                                             _p(F), _stream()))
    return F


def quantize(ctx: Context, feat, S, d_clip, lambda_dino=0.5, lambda_cos=1.0, lambda_lb=0.5, grad=True,
             workspace=None):
    """Codebook quantisation (legs_quantize). feat [K][d] float16, S [N][d]
    float32. Returns dict with index [K] int32, counts [N] int32 (uint32
    bits), prob_mean [N], losses [3] = (L_cos, L_lb, L_q) and grad [N][d]
    (None without the gradient pass)."""
    assert feat.dtype == torch.float16 and feat.is_contiguous() and S.dtype == torch.float32
    K, d = feat.shape
    N = S.shape[0]
    dev = ctx.device
    if workspace is None:
        workspace = torch.empty(max(int(L.lib().legs_quantize_workspace_bytes(K, N, d)), 16), dtype=torch.uint8,
                                device=dev)
    out = dict(index=torch.empty(max(K, 1), dtype=torch.int32, device=dev),
               counts=torch.empty(N, dtype=torch.int32, device=dev),
               prob_mean=torch.empty(N, dtype=torch.float32, device=dev),
               losses=torch.empty(3, dtype=torch.float32, device=dev),
               grad=torch.empty((N, d), dtype=torch.float32, device=dev) if grad else None)
    ctx.check(L.lib().legs_quantize(ctx.handle, _p(feat), K, d, int(d_clip), _p(S), N, float(lambda_dino),
                                    float(lambda_cos), float(lambda_lb), _p(workspace), _p(out["index"]),
                                    _p(out["counts"]), _p(out["prob_mean"]), _p(out["losses"]), _p(out["grad"]),
                                    _stream()))
    out["index"] = out["index"][:K]
    return out


def smooth_param_count():
    return int(L.lib().legs_smooth_param_count())


def smooth_workspace(ctx: Context, n):
    return torch.empty(max(int(L.lib().legs_smooth_workspace_bytes(n)), 16), dtype=torch.uint8, device=ctx.device)


def smooth_loss_grad(ctx: Context, mean, channels, sem_channel, u_channel, params, grad, d_channels, loss,
                     w_s=0.1, lambda_smo=1.0, workspace=None):
    """Adaptive spatial smoothing loss and gradients (legs_smooth_loss_grad);
    loss, grad and d_channels are accumulated. Returns the workspace (which
    holds the bf16 input and hidden activations, Gaussians padded to a
    multiple of 64, each R-row plane in MFMA operand order
    [Gp / 16][ceil(R / 32)][2][min(R, 32)][8])."""
    n, C = channels.shape
    if workspace is None:
        workspace = smooth_workspace(ctx, n)
    ctx.check(L.lib().legs_smooth_loss_grad(ctx.handle, _p(mean), _p(channels), C, int(sem_channel), int(u_channel),
                                            n, _p(params), float(w_s), float(lambda_smo), _p(workspace), _p(grad),
                                            _p(d_channels), _p(loss), _stream()))
    return workspace


class MlpTrainer:
    """Decoder parameters, Adam moments and scratch for legs_mlp_train_step."""

    def __init__(self, ctx: Context, params, K, batch, lr=1e-3, betas=(0.9, 0.999), eps=1e-8,
                 normalize=True):
        self.ctx, self.K, self.lr, self.betas, self.eps = ctx, K, lr, betas, eps
        self.flags = mlp_flags(normalize)
        self.params = params.to(ctx.device).contiguous().clone()
        n = mlp_param_count(K)
        assert self.params.numel() == n
        self.m = torch.zeros(n, dtype=torch.float32, device=ctx.device)
        self.v = torch.zeros(n, dtype=torch.float32, device=ctx.device)
        self.grad = torch.zeros(n, dtype=torch.float32, device=ctx.device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=ctx.device)
        nbytes = int(L.lib().legs_mlp_workspace_bytes(batch, K))
        self.ws = torch.empty(max(nbytes, 4), dtype=torch.uint8, device=ctx.device)
        self.batch = batch
        self.step_count = 0

    def grad_only(self, f, labels):
        tp, P, cs, ps = _feat_args(f)
        assert P <= self.batch
        self.ctx.check(L.lib().legs_mlp_grad(self.ctx.handle, tp, P, cs, ps, _p(labels), self.K,
                                             self.flags, _p(self.params), _p(self.ws), _p(self.grad),
                                             _p(self.loss), _stream()))
        return self.grad, self.loss

    def step(self, f, labels):
        tp, P, cs, ps = _feat_args(f)
        assert P <= self.batch
        self.step_count += 1
        self.ctx.check(L.lib().legs_mlp_train_step(
            self.ctx.handle, tp, P, cs, ps, _p(labels), self.K, self.flags, _p(self.params), _p(self.m),
            _p(self.v), _p(self.grad), self.step_count, self.lr, self.betas[0], self.betas[1],
            self.eps, _p(self.ws), _p(self.loss), _stream()))
        return self.loss


def semantic_loss_grad(ctx: Context, f, ru, labels, params, K, inv_hw, workspace, grad, d_feat, d_ru, loss,
                       lambda_ce=1.0, lambda_u=1.0, normalize=True):
    """Eqs. 10-12 over the pixels of one view (legs_semantic_loss_grad).
    f: feature argument like the decode calls; d_feat: (tensor, c_stride,
    p_stride) receiving dL_s/dR_s; ru, d_ru: [P] tensors; grad and loss are
    accumulated."""
    tp, P, cs, ps = _feat_args(f)
    dt, dcs, dps = d_feat
    ctx.check(L.lib().legs_semantic_loss_grad(ctx.handle, tp, _p(ru), P, cs, ps, _p(labels), K,
                                              mlp_flags(normalize), _p(params), lambda_ce, lambda_u, inv_hw,
                                              _p(workspace), _p(grad), _p(dt), int(dcs), int(dps), _p(d_ru),
                                              _p(loss), _stream()))


def semantic_loss_grad_noalloc(ctx: Context, f, ru, labels, params, K, inv_hw, grad, d_feat, d_ru, loss,
                               lambda_ce=1.0, lambda_u=1.0, normalize=True):
    """semantic_loss_grad without a workspace (legs_semantic_loss_grad_noalloc):
    the library's own fixed per-GPU array serves as workspace; at most
    max_noalloc_pixels() pixels per call."""
    tp, P, cs, ps = _feat_args(f)
    dt, dcs, dps = d_feat
    ctx.check(L.lib().legs_semantic_loss_grad_noalloc(ctx.handle, tp, _p(ru), P, cs, ps, _p(labels), K,
                                                      mlp_flags(normalize), _p(params), lambda_ce, lambda_u,
                                                      inv_hw, _p(grad), _p(dt), int(dcs), int(dps), _p(d_ru),
                                                      _p(loss), _stream()))


NOALLOC_MAX_PIXELS = 16384      # LEGS_NOALLOC_MAX_PIXELS of include/legs.h


def workspace(ctx: Context, P, K):
    nbytes = int(L.lib().legs_mlp_workspace_bytes(P, K))
    return torch.empty(max(nbytes, 4), dtype=torch.uint8, device=ctx.device)


def adam(ctx: Context, groups, step, lr=1e-3, betas=(0.9, 0.999), eps=1e-8):
    """groups: list of dicts with param, grad, m, v (float32 tensors) and
    optional clamp=(every, offset, lo, hi)."""
    arr = (L.AdamGroup * len(groups))()
    for i, g in enumerate(groups):
        ce, co, lo, hi = g.get("clamp", (0, 0, 0.0, 0.0))
        arr[i] = L.AdamGroup(g["param"].data_ptr(), g["grad"].data_ptr(), g["m"].data_ptr(),
                             g["v"].data_ptr(), g["param"].numel(), ce, co, lo, hi)
    ctx.check(L.lib().legs_adam(ctx.handle, arr, len(groups), int(step), lr, betas[0], betas[1],
                                eps, _stream()))


def l1_loss_grad(ctx: Context, out, target, views, C, n_fit, lambda_u=1.0, d_out=None, loss=None):
    if d_out is None:
        d_out = torch.empty_like(out)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=out.device)
    ctx.check(L.lib().legs_l1_loss_grad(ctx.handle, _p(out), _p(target), _p(views.dev),
                                        views.n_views, views.total_pixels, C, n_fit, lambda_u,
                                        _p(d_out), _p(loss), _stream()))
    return d_out, loss
