"""FP64 numpy oracle for the language-feature side of the method (test
infrastructure only; never imported by the product path).

  language_features  supplementary inference equations: the decoder of
                     Table 3 (1x1 convolutions 8 -> 128 -> 256 -> N, ReLU
                     between them) gives M_infer = softmax(D_MLP(R_s)) per
                     pixel, and the language feature map is F = M_infer S with
                     S [N][d] the discrete feature space.
  quantize           Sec. 3.3: the two-part cosine distance of Eq. 4 between
                     hybrid (CLIP | DINO) features and the discrete feature
                     space, the argmax index of each feature, its quantisation
                     (Eq. 5), the cosine loss of Eq. 6, the load-balancing loss
                     of Eq. 7 (utilisation ratio r and mean selection
                     probability p as the supplementary section defines them),
                     L_q of the quantisation summary equation, and the
                     gradient of L_q with respect to the feature space.
  smoothing          Sec. 3.4.2 adaptive spatial smoothing: s_MLP =
                     MLP(PE(p)) (Eq. 13; PE and MLP of Table 4) and
                     L_smo = |s_MLP - s_G*| + max(u*, w_s) |s_MLP* - s_G| (Eq.
                     14), with its gradients with respect to the MLP and s_G.

Roundings emulated where the GPU path has them (bf16 weights and hidden
activations of the MLPs, float32 accumulation aside); everything else in
float64.
"""
from __future__ import annotations

import numpy as np

from oracle.decode import bf16, mlp_forward, softmax


# ---------------------------------------------------------------- inference

def language_features(feat, weights, biases, S, normalize=False):
    """feat [P, 8] rendered compact features, weights/biases of the decoder
    (any depth; Table 3 has 8 -> 128 -> 256 -> N), S [N, d].
    Returns dict: logits, M (softmax, float64), top1 (lowest index on ties),
    F = M S, F_abs = M |S| (the scale of a rounding error of F)."""
    fw = mlp_forward(feat, weights, biases, normalize=normalize)
    logits = fw["logits"]
    M = softmax(logits)
    Sd = np.asarray(S, np.float64)
    return dict(logits=logits, M=M, top1=np.argmax(logits, axis=1), F=M @ Sd, F_abs=M @ np.abs(Sd),
                ambiguous=fw["ambiguous"])


# ------------------------------------------------------------- quantisation

def _unit_rows(X):
    n = np.sqrt(np.sum(X * X, axis=1))
    return X / np.where(n > 0.0, n, 1.0)[:, None], n


def quantize(F, S, d_clip, lambda_dino=0.5, lambda_cos=1.0, lambda_lb=0.5, m=None):
    """F [K, d] hybrid features (columns [0, d_clip) CLIP, the rest DINO),
    S [N, d] the discrete feature space with the same split.

    D_ij = cos(F_i^C, f_j^C) + lambda_dino cos(F_i^D, f_j^D)        (Eq. 4)
    m_i = argmax_j D_ij (lowest index on ties);  F^_i = f_{m_i}    (Eq. 5)
    L_cos = mean_i [(1 - cos(F_i^C, F^_i^C)) + lambda_dino (1 - cos(F_i^D, F^_i^D))]   (Eq. 6)
    r = (sum_i onehot(m_i)) / K, p = (sum_i softmax_j(D_ij)) / K,
    L_lb = sum_j r_j p_j                                           (Eq. 7)
    L_q = lambda_cos L_cos + lambda_lb L_lb

    The gradient is with respect to S (the optimised feature space); the
    argmax and therefore r are piecewise constant (no gradient). m (optional)
    replaces the argmax (to follow another evaluation's choice among
    near-equal distances). A zero row
    (feature or code part) has cosine 0 and no gradient through it.
    Returns dict with D, cos_c, cos_d, m, r, p, L_cos, L_lb, L_q, dD (dL_q/dD),
    grad [N, d] and margin (top-1 minus top-2 of each row of D)."""
    F = np.asarray(F, np.float64)
    S = np.asarray(S, np.float64)
    K, d = F.shape
    N = S.shape[0]
    Fc, nFc = _unit_rows(F[:, :d_clip])
    Fd, nFd = _unit_rows(F[:, d_clip:])
    Sc, nSc = _unit_rows(S[:, :d_clip])
    Sd, nSd = _unit_rows(S[:, d_clip:])
    cos_c = Fc @ Sc.T
    cos_d = Fd @ Sd.T
    D = cos_c + lambda_dino * cos_d
    m = np.argmax(D, axis=1) if m is None else np.asarray(m, np.int64)
    srt = np.sort(D, axis=1)
    margin = srt[:, -1] - srt[:, -2] if N > 1 else np.full(K, np.inf)
    rows = np.arange(K)
    L_cos = float(np.mean((1.0 - cos_c[rows, m]) + lambda_dino * (1.0 - cos_d[rows, m])))
    r = np.bincount(m, minlength=N).astype(np.float64) / K
    s = softmax(D)
    p = s.mean(axis=0)
    L_lb = float(np.sum(r * p))
    L_q = lambda_cos * L_cos + lambda_lb * L_lb
    # dL/dD: the cosine loss of row i is (1 + lambda_dino) - D_{i m_i}; the
    # load-balancing loss is sum_j r_j mean_i s_ij, and d s_ij / d D_il =
    # s_ij (delta_jl - s_il).
    dD = lambda_lb / K * s * (r[None, :] - (s @ r)[:, None])
    dD[rows, m] -= lambda_cos / K
    # d cos(a, b) / d b = (a^ - cos(a, b) b^) / |b| for the unit vectors a^, b^
    gc = (dD.T @ Fc - np.sum(dD * cos_c, axis=0)[:, None] * Sc) / np.where(nSc > 0, nSc, np.inf)[:, None]
    gd = lambda_dino * (dD.T @ Fd - np.sum(dD * cos_d, axis=0)[:, None] * Sd) / \
        np.where(nSd > 0, nSd, np.inf)[:, None]
    grad = np.concatenate([gc, gd], axis=1)
    return dict(D=D, cos_c=cos_c, cos_d=cos_d, m=m, r=r, p=p, L_cos=L_cos, L_lb=L_lb, L_q=L_q, dD=dD,
                grad=grad, margin=margin)


# ------------------------------------------------------------- smoothing

def positional_encoding(pos, n_freq):
    """NeRF positional encoding of positions [n, 3]: the position followed by
    sin(2^k pi p), cos(2^k pi p) for k < n_freq; n_freq = 0 is the position
    itself (Table 4's configuration 0)."""
    p = np.asarray(pos, np.float64)
    parts = [p]
    for k in range(n_freq):
        parts.append(np.sin((2.0 ** k) * np.pi * p))
        parts.append(np.cos((2.0 ** k) * np.pi * p))
    return np.concatenate(parts, axis=1)


def smooth_forward(pos, weights, biases, n_freq=0, round_bf16=True, hidden=None):
    """s_MLP = MLP(PE(p)) (Eq. 13): fully connected layers with ReLU between
    them (Table 4: PE -> 128 -> 128 -> 128 -> 8). Weights and the hidden
    activations are rounded to bf16 (round_bf16); the encoded position enters
    the first layer unrounded. hidden (optional): the hidden activations to
    use instead of the computed ones (another evaluation's rounding choices);
    the pre-activations are still computed from the previous layer's.
    Returns dict with hs (layer inputs), zs (pre-activations) and out (float64)."""
    rnd = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    h = positional_encoding(np.asarray(pos, np.float32), n_freq)
    hs, zs = [h], []
    L = len(weights)
    for l in range(L):
        W = rnd(np.asarray(weights[l], np.float32).astype(np.float64))
        b = np.asarray(biases[l], np.float32).astype(np.float64)
        z = h @ W.T + b
        zs.append(z)
        if l < L - 1:
            h = rnd(np.maximum(z, 0.0)) if hidden is None else np.asarray(hidden[l], np.float64)
            hs.append(h)
    return dict(hs=hs, zs=zs, out=zs[-1])


def smoothing_loss_grad(pos, s_g, u, weights, biases, w_s=0.1, n_freq=0, round_bf16=True, hidden=None):
    """Adaptive spatial smoothing loss (Eq. 14) averaged over the Gaussians:
      L_smo = mean_g [ |s_MLP - s_G*|_2 + max(u_G*, w_s) |s_MLP* - s_G|_2 ]
    (* = stop gradient; unsquared Euclidean norms). The positions are inputs,
    not optimised by this loss. Gradients: the first term reaches the MLP, the
    second reaches s_G; u gets none. A Gaussian with s_MLP = s_G contributes
    zero loss and zero gradient. hidden: as in smooth_forward. The ReLU gate
    of a unit is open where its (rounded) activation is positive, which is
    where its pre-activation is.
    Returns dict with loss, s_mlp, d_sg [n, d_s], gW, gb (lists per layer)."""
    fw = smooth_forward(pos, weights, biases, n_freq, round_bf16, hidden)
    sg = np.asarray(s_g, np.float64)
    uu = np.asarray(u, np.float64)
    n = sg.shape[0]
    diff = fw["out"] - sg
    nrm = np.sqrt(np.sum(diff * diff, axis=1))
    wgt = np.maximum(uu, w_s)
    loss = float(np.sum(nrm * (1.0 + wgt)) / n)
    unit = diff / np.where(nrm > 0.0, nrm, np.inf)[:, None]
    dz = unit / n
    d_sg = -(wgt / n)[:, None] * unit
    rnd = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    L = len(weights)
    gW, gb = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        gW[l] = dz.T @ fw["hs"][l]
        gb[l] = dz.sum(axis=0)
        if l > 0:
            W = rnd(np.asarray(weights[l], np.float32).astype(np.float64))
            dz = (dz @ W) * (fw["hs"][l] > 0.0)
    return dict(loss=loss, s_mlp=fw["out"], d_sg=d_sg, gW=gW, gb=gb, norm=nrm, hs=fw["hs"], zs=fw["zs"])
