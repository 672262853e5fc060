"""FP64 numpy oracle for decoding, decoder training, Adam and the training-step
loss (test infrastructure only; never imported by the product path).

  decode_plain   Sec. 3.3 Eq. 4 (cosine max-similarity search over the
                 discrete feature space S) applied to a rendered compact
                 feature lifted to the codebook dimension by a fixed projection;
                 softmax over the scores, top-1 = argmax (lowest index on ties).
  mlp_forward    Eq. 8 / supplementary inference equation: softmax(D_MLP(R_s)),
                 D_MLP a stack of 1x1 convolutions = per-pixel linear layers
                 with ReLU (Table 3 gives the layer pattern), applied to the
                 feature divided by its norm; bf16 rounding of the input,
                 weights and hidden activations is emulated exactly,
                 accumulation is in float64.
  mlp_train_step Eq. 9 cross-entropy against index labels, gradients by the
                 chain rule (straight through the bf16 roundings), then Adam.
  adam           Sec. 4: Adam, lr 1e-3, betas (0.9, 0.999); no weight decay.
  l1_loss_grad   per-view mean absolute error over RGB and semantic channels
                 plus lambda_u * mean(R_u) (Eq. 11) and its gradient.
"""
from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    Works directly from float64 (a single rounding); normal range only
    (no subnormal, overflow or NaN handling: activations here stay normal)."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)                        # x = m * 2**e, 0.5 <= |m| < 1
    r = np.round(np.ldexp(m, 8))              # 8 significant bits, half to even
    return np.ldexp(r, e - 8)


def decode_plain(feat, proj, codebook):
    """feat [P, d_s], proj [D, d_s], codebook [K, D] (unit rows).
    Returns (probs [P, K] float64, top1 [P] int64)."""
    f = np.asarray(feat, np.float64)
    Pm = np.asarray(proj, np.float64)
    Cb = np.asarray(codebook, np.float64)
    z = f @ Pm.T                              # lifted feature, [P, D]
    nz = np.sqrt(np.sum(z * z, axis=1))
    dots = z @ Cb.T
    cn = np.sqrt(np.sum(Cb * Cb, axis=1))
    with np.errstate(invalid="ignore", divide="ignore"):
        s = dots / (nz[:, None] * cn[None, :])
    s[nz == 0] = 0.0
    s = s - s.max(axis=1, keepdims=True)
    e = np.exp(s)
    probs = e / e.sum(axis=1, keepdims=True)
    top1 = np.argmax(dots / np.where(nz == 0, 1.0, nz)[:, None] / cn[None, :], axis=1)
    top1[nz == 0] = 0
    return probs, top1


def mlp_forward(feat, weights, biases, amb_tol=2e-6, normalize=True):
    """Per-pixel MLP with ReLU between layers. weights[l] is [out, in] (float32
    master), biases[l] [out] (float32). With normalize (the default) the
    feature is first divided by its Euclidean norm (a zero feature stays
    zero): the codes it is trained to predict depend only on the feature's
    direction (cosine scores, Eq. 4); without it the decoder sees R_s itself,
    as Eq. 8 writes it.
    Returns a dict with the bf16-rounded input, pre-activations z_l,
    post-activations h_l and float64 logits.

    `ambiguous` flags pixels with an input or hidden activation within a
    relative amb_tol of a bf16 rounding midpoint: a float32 computation (error
    ~1e-7 relative) may round such a value to the other neighbour, so those
    pixels are checked only loosely against an implementation in float32."""
    f = np.asarray(feat, np.float32).astype(np.float64)
    if normalize:
        nrm = np.sqrt(np.sum(f * f, axis=1, keepdims=True))
        u = np.where(nrm > 0.0, f / np.where(nrm > 0.0, nrm, 1.0), 0.0)
    else:
        u = f
    x = bf16(u)
    hs = [x]
    zs = []
    h = x
    amb = np.any(bf16(u * (1 + amb_tol)) != bf16(u * (1 - amb_tol)), axis=1)
    L = len(weights)
    for l in range(L):
        W = bf16(np.asarray(weights[l], np.float32).astype(np.float64))
        b = np.asarray(biases[l], np.float32).astype(np.float64)
        z = h @ W.T + b
        zs.append(z)
        if l < L - 1:
            r = np.maximum(z, 0.0)
            h = bf16(r)
            amb |= np.any(bf16(r * (1 + amb_tol)) != bf16(r * (1 - amb_tol)), axis=1)
            hs.append(h)
    return dict(x=x, hs=hs, zs=zs, logits=zs[-1], ambiguous=amb)


def mlp_branches(feat_row, weights, biases, normalize=True, amb_tol=2e-6, max_states=64,
                 return_hidden=False):
    """Every logit vector a float32 evaluation of mlp_forward can produce for
    one pixel: wherever a value that is rounded to bf16 (the input, each
    hidden activation) lies within a relative amb_tol of a rounding midpoint,
    both neighbours are followed. Returns (list of logits, complete) with
    complete False when more than max_states branches would arise (the list
    then holds the branches of the first ambiguous values only). With
    return_hidden, also the rounded layer inputs [x, h1, ...] of each branch
    (a third list, same order)."""
    f = np.asarray(feat_row, np.float32).astype(np.float64)[None, :]
    if normalize:
        nrm = np.sqrt(np.sum(f * f))
        u = f / nrm if nrm > 0.0 else np.zeros_like(f)
    else:
        u = f
    complete = True

    def roundings(v):
        nonlocal complete
        lo, hi = bf16(v * (1 - amb_tol)), bf16(v * (1 + amb_tol))
        base = bf16(v)
        amb = np.nonzero(lo != hi)[1] if v.ndim == 2 else np.nonzero(lo != hi)[0]
        outs = [base]
        for j in amb:
            alt = []
            for o in outs:
                for cand in (lo[..., j], hi[..., j]):
                    if cand != o[..., j]:
                        q = o.copy()
                        q[..., j] = cand
                        alt.append(q)
            if len(outs) + len(alt) > max_states:
                complete = False
                break
            outs += alt
        return outs

    states = [(h, [h[0]]) for h in roundings(u)]
    L = len(weights)
    Ws = [bf16(np.asarray(w, np.float32).astype(np.float64)) for w in weights]
    bs = [np.asarray(b, np.float32).astype(np.float64) for b in biases]
    for l in range(L):
        nxt = []
        for h, trail in states:
            z = h @ Ws[l].T + bs[l]
            if l < L - 1:
                nxt += [(q, trail + [q[0]]) for q in roundings(np.maximum(z, 0.0))]
            else:
                nxt.append((z[0], trail))
        if len(nxt) > max_states:
            complete = False
            nxt = nxt[:max_states]
        states = nxt
    logits = [z for z, _ in states]
    if return_hidden:
        return logits, complete, [trail for _, trail in states]
    return logits, complete


def softmax(z):
    z = z - z.max(axis=1, keepdims=True)
    e = np.exp(z)
    return e / e.sum(axis=1, keepdims=True)


def _follow(fw, hidden, weights, biases):
    """Replace the rounded layer inputs of a forward pass by given ones
    (another evaluation's rounding choices: hidden = [x, h1, h2, ...]) and
    recompute every pre-activation from them in float64."""
    hs = [np.asarray(h, np.float64) for h in hidden]
    zs = []
    for l in range(len(weights)):
        W = bf16(np.asarray(weights[l], np.float32).astype(np.float64))
        zs.append(hs[l] @ W.T + np.asarray(biases[l], np.float32).astype(np.float64))
    return dict(fw, x=hs[0], hs=hs, zs=zs, logits=zs[-1])


def mlp_grads(feat, labels, weights, biases, normalize=True, hidden=None):
    """Mean cross-entropy over the batch and its gradients w.r.t. every weight
    and bias (straight-through for the bf16 roundings). hidden (optional): the
    decoder input and hidden activations to follow ([x, h1, h2]) instead of
    this forward's roundings; a ReLU gate is open where its activation is
    positive, which is where its pre-activation is."""
    fw = mlp_forward(feat, weights, biases, normalize=normalize)
    if hidden is not None:
        fw = _follow(fw, hidden, weights, biases)
    B = feat.shape[0]
    p = softmax(fw["logits"])
    y = np.asarray(labels, np.int64)
    loss = float(-np.mean(np.log(p[np.arange(B), y])))
    dz = p.copy()
    dz[np.arange(B), y] -= 1.0
    dz /= B
    L = len(weights)
    gW = [None] * L
    gb = [None] * L
    for l in range(L - 1, -1, -1):
        h_in = fw["hs"][l]
        gW[l] = dz.T @ h_in
        gb[l] = dz.sum(axis=0)
        if l > 0:
            W = bf16(np.asarray(weights[l], np.float32).astype(np.float64))
            dh = dz @ W
            dz = dh * (fw["hs"][l] > 0.0)
    return loss, gW, gb


def adam(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected, no weight decay). Returns (p, m, v) float64."""
    p = np.asarray(p, np.float64)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    p = p - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def l1_loss_grad(out_flat, target_flat, cams, n_channels, d_sem, lambda_u=1.0):
    """out/target planar [C][H][W] per view, concatenated. Loss per view:
    mean |out - target| over the RGB and semantic channels, plus lambda_u times
    the mean rendered uncertainty; summed over views. Returns (loss, grad)."""
    out = np.asarray(out_flat, np.float64)
    tgt = np.asarray(target_flat, np.float64)
    grad = np.zeros_like(out)
    loss = 0.0
    off = 0
    n_fit = 3 + d_sem
    for cam in cams:
        hw = cam.width * cam.height
        o = out[off:off + n_channels * hw].reshape(n_channels, hw)
        t = tgt[off:off + n_channels * hw].reshape(n_channels, hw)
        g = grad[off:off + n_channels * hw].reshape(n_channels, hw)
        d = o[:n_fit] - t[:n_fit]
        loss += float(np.abs(d).sum() / (n_fit * hw))
        g[:n_fit] = np.sign(d) / (n_fit * hw)
        for c in range(n_fit, n_channels):
            loss += lambda_u * float(o[c].sum() / hw)
            g[c] = lambda_u / hw
        off += n_channels * hw
    return loss, grad


def semantic_loss_grad(feat, ru, labels, weights, biases, inv_hw, lambda_ce=1.0, lambda_u=1.0,
                       round_bf16=True, normalize=True, hidden=None):
    """Semantic loss of Sec. 3.4.2 for the pixels of one view and its gradients:
      L_CE = sum_px CE(softmax(D_MLP(R_s)), M) (1 - R_u) / (H W)      (Eq. 10)
      L_u  = sum_px R_u / (H W)                                        (Eq. 11)
      L_s  = lambda_CE L_CE + lambda_u L_u                             (Eq. 12)
    feat [P, 8] = R_s, ru [P] = R_u, labels [P] = M (code indices), inv_hw =
    1 / (H W) of the view. The decoder is mlp_forward's (input divided by its
    norm, bf16 roundings emulated unless round_bf16 is False). Gradients pass
    straight through the roundings. hidden (optional): the rounded decoder
    input and hidden activations to follow ([x, h1, ...], another
    evaluation's rounding choices) instead of this forward's. Returns dict
    with loss, ce [P], d_feat [P, 8] = dL_s/dR_s, d_ru [P] = dL_s/dR_u, gW, gb
    (lists per layer)."""
    f = np.asarray(feat).astype(np.float64)     # float32 maps promote exactly
    u_r = np.asarray(ru).astype(np.float64)
    y = np.asarray(labels, np.int64)
    P = f.shape[0]
    nrm = np.sqrt(np.sum(f * f, axis=1, keepdims=True))
    u = np.where(nrm > 0.0, f / np.where(nrm > 0.0, nrm, 1.0), 0.0) if normalize else f
    rnd = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
    h = rnd(u)
    hs, zs, Ws = [h], [], []
    L = len(weights)
    for l in range(L):
        W = rnd(np.asarray(weights[l], np.float32).astype(np.float64))
        b = np.asarray(biases[l], np.float32).astype(np.float64)
        Ws.append(W)
        z = h @ W.T + b
        zs.append(z)
        if l < L - 1:
            h = rnd(np.maximum(z, 0.0))
            hs.append(h)
    if hidden is not None:
        hs = [np.asarray(v, np.float64) for v in hidden]
        zs = [hs[l] @ Ws[l].T + np.asarray(biases[l], np.float32).astype(np.float64) for l in range(L)]
    p = softmax(zs[-1])
    ce = -np.log(p[np.arange(P), y])
    wpx = lambda_ce * (1.0 - u_r) * inv_hw                # weight of each pixel's CE
    loss = float(np.sum(wpx * ce) + lambda_u * inv_hw * np.sum(u_r))
    d_ru = (-lambda_ce * ce + lambda_u) * inv_hw
    dz = p.copy()
    dz[np.arange(P), y] -= 1.0
    dz *= wpx[:, None]
    gW, gb = [None] * L, [None] * L
    for l in range(L - 1, -1, -1):
        gW[l] = dz.T @ hs[l]
        gb[l] = dz.sum(axis=0)
        dh = dz @ Ws[l]
        if l > 0:
            dz = dh * (hs[l] > 0.0)            # ReLU gate: open where its activation is positive
    # dh is now dL/d(decoder input); a normalised input f / |f| has the
    # Jacobian (I - u u^T) / |f| (zero for a zero feature)
    if normalize:
        d_feat = np.where(nrm > 0.0,
                          (dh - np.sum(dh * u, axis=1, keepdims=True) * u) / np.where(nrm > 0.0, nrm, 1.0), 0.0)
    else:
        d_feat = dh
    return dict(loss=loss, ce=ce, d_feat=d_feat, d_ru=d_ru, gW=gW, gb=gb)
