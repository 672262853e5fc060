"""GPU parity of the codebook quantisation of Sec. 3.3 (Eqs. 4-7 and the
supplementary load-balancing loss) against the FP64 oracle, through the C
ABI: indices, histogram, mean selection probability, L_cos, L_lb, L_q and the
gradient with respect to the discrete feature space."""
import sys

import numpy as np
import pytest
import torch

from oracle import language as LG

pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    from paper_2311_18482_amd import raster
    assert torch.cuda.is_available()
    return raster.Context(0)


def hybrid(K, N, d, d_clip, seed, noise=1.5):
    """Features scattered around the codes (so the argmax is mostly clear but
    some features sit near a tie), a zero feature and one with a zero DINO part."""
    rng = np.random.default_rng(seed)
    S = rng.normal(0, 1, (N, d)).astype(np.float32)
    c = rng.integers(0, N, K)
    F = (S[c] + noise * rng.normal(0, 1, (K, d))).astype(np.float16)
    F[0] = 0
    F[1, d_clip:] = 0
    return F, S


@pytest.mark.parametrize("N,d,d_clip,K", [(128, 896, 512, 20000 + 77), (64, 896, 512, 9001),
                                          (32, 256, 256, 3000 + 5), (128, 384, 128, 257)])
def test_quantize_matches_oracle(ctx, N, d, d_clip, K):
    from paper_2311_18482_amd import decode as DEC
    F, S = hybrid(K, N, d, d_clip, 170 + N + d)
    note(f"quantize N={N} d={d} d_clip={d_clip} K={K}")
    out = DEC.quantize(ctx, torch.from_numpy(F).cuda(), torch.from_numpy(S).cuda(), d_clip)
    torch.cuda.synchronize()
    m = out["index"].cpu().numpy().astype(np.int64)
    counts = out["counts"].cpu().numpy().astype(np.int64)
    F64 = F.astype(np.float64)
    S16 = S.astype(np.float16).astype(np.float64)
    q = LG.quantize(F64, S16, d_clip, 0.5, 1.0, 0.5)
    # index: the oracle's wherever the two best distances differ by more than
    # float32 rounding can move them; else one of the near-best codes
    clear = q["margin"] > 1e-4
    assert np.array_equal(m[clear], q["m"][clear])
    rows = np.arange(K)
    assert (q["D"][rows, m] >= q["D"].max(axis=1) - 1e-4).all()
    assert np.array_equal(counts, np.bincount(m, minlength=N))
    pm = out["prob_mean"].cpu().numpy().astype(np.float64)
    assert np.allclose(pm, q["p"], rtol=1e-4, atol=1e-7)
    # losses and gradient along the GPU's indices
    q2 = LG.quantize(F64, S16, d_clip, 0.5, 1.0, 0.5, m=m)
    L = out["losses"].cpu().numpy().astype(np.float64)
    assert L[0] == pytest.approx(q2["L_cos"], rel=1e-5)
    assert L[1] == pytest.approx(q2["L_lb"], rel=1e-4)
    assert L[2] == pytest.approx(q2["L_q"], rel=1e-5)
    g = out["grad"].cpu().numpy().astype(np.float64)
    # the gradient's contraction runs on half precision: the weights 2^10 K dL/dD
    # and the unit feature rows each round by at most 2^-11 relative (plus
    # 2^-25 absolute per element where a half is subnormal), the sums are
    # float32; per code and part the error is then at most
    # (2^-10 + 2e-6) sum_i |dL/dD_ij| / |S_j| + 2^-34 / |S_j|
    dD = q2["dD"]
    for lo, hi, lam in ((0, d_clip, 1.0), (d_clip, d, 0.5)):
        if hi == lo:
            continue
        nS = np.linalg.norm(S16[:, lo:hi], axis=1)
        inv = 1.0 / np.where(nS > 0, nS, np.inf)
        scale = lam * np.abs(dD).sum(axis=0) * inv
        bound = (2.0 ** -10 + 2e-6) * scale + 2.0 ** -34 * inv
        err = np.linalg.norm(g[:, lo:hi] - q2["grad"][:, lo:hi], axis=1)
        assert (err <= bound).all(), float((err / bound).max())
    note(f"ambiguous indices {int((~clear).sum())}, flipped {int((m != q['m']).sum())}, "
         f"losses {L.tolist()} vs {[q2['L_cos'], q2['L_lb'], q2['L_q']]}")


def test_quantize_rejects_bad_shapes(ctx):
    from paper_2311_18482_amd import decode as DEC
    F = torch.zeros((10, 200), dtype=torch.float16, device="cuda")
    S = torch.zeros((32, 200), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError):
        DEC.quantize(ctx, F, S, 128)                    # d not a multiple of 128
    F = torch.zeros((10, 256), dtype=torch.float16, device="cuda")
    S = torch.zeros((48, 256), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError):
        DEC.quantize(ctx, F, S, 128)                    # N not in {32, 64, 128}


def test_quantize_at_bench_size(ctx):
    """1M hybrid features (512 CLIP + 384 DINO dims, half) against a 128-code
    feature space: the shape and launch configuration the bench times. The
    indices of 20000 sampled features (and the first, zero-DINO and last ones)
    against the oracle (clear margins exactly, else a near-best code), the
    histogram against the indices, and the mean selection probability, the
    three losses and the gradient against the oracle over all features along
    the GPU's indices. Bounds as in the small test, with the float32 sums
    over 1M features allowed for: the loss and probability sums take one
    rounding per feature (or per wave) in the worst case (the tolerances
    below cover their random walk, about sqrt(adds) 2^-24), and each gradient
    element is a float32 sum of at most per_block / 16 MFMA steps plus one
    atomic per workgroup (under 600 roundings: 4e-5)."""
    from paper_2311_18482_amd import decode as DEC
    K, N, d, d_clip = 1_000_000, 128, 896, 512
    rng = np.random.default_rng(196)
    S = rng.normal(0, 1, (N, d)).astype(np.float32)
    F = np.empty((K, d), np.float16)
    for lo in range(0, K, 125_000):
        hi = min(lo + 125_000, K)
        c = rng.integers(0, N, hi - lo)
        F[lo:hi] = (S[c] + 1.5 * rng.normal(0, 1, (hi - lo, d))).astype(np.float16)
    F[0] = 0
    F[1, d_clip:] = 0
    note(f"quantize at K={K} N={N} d={d} d_clip={d_clip}")
    out = DEC.quantize(ctx, torch.from_numpy(F).cuda(), torch.from_numpy(S).cuda(), d_clip)
    torch.cuda.synchronize()
    m = out["index"].cpu().numpy().astype(np.int64)
    counts = out["counts"].cpu().numpy().astype(np.int64)
    pm = out["prob_mean"].cpu().numpy().astype(np.float64)
    L = out["losses"].cpu().numpy().astype(np.float64)
    g = out["grad"].cpu().numpy().astype(np.float64)
    del out
    torch.cuda.empty_cache()
    assert np.array_equal(counts, np.bincount(m, minlength=N))
    S16 = S.astype(np.float16).astype(np.float64)
    idx = np.unique(np.concatenate([[0, 1], np.arange(K - 40, K), rng.integers(0, K, 20000)]))
    qs = LG.quantize(F[idx], S16, d_clip, 0.5, 1.0, 0.5)
    clear = qs["margin"] > 1e-4
    assert np.array_equal(m[idx][clear], qs["m"][clear])
    rows = np.arange(len(idx))
    assert (qs["D"][rows, m[idx]] >= qs["D"].max(axis=1) - 1e-4).all()
    del qs
    q2 = LG.quantize(F, S16, d_clip, 0.5, 1.0, 0.5, m=m)
    assert np.allclose(pm, q2["p"], rtol=2e-4, atol=1e-7)
    assert L[0] == pytest.approx(q2["L_cos"], rel=2e-4)
    assert L[1] == pytest.approx(q2["L_lb"], rel=2e-4)
    assert L[2] == pytest.approx(q2["L_q"], rel=2e-4)
    dD = q2["dD"]
    for lo, hi, lam in ((0, d_clip, 1.0), (d_clip, d, 0.5)):
        nS = np.linalg.norm(S16[:, lo:hi], axis=1)
        inv = 1.0 / np.where(nS > 0, nS, np.inf)
        scale = lam * np.abs(dD).sum(axis=0) * inv
        bound = (2.0 ** -10 + 4e-5) * scale + 2.0 ** -34 * inv
        err = np.linalg.norm(g[:, lo:hi] - q2["grad"][:, lo:hi], axis=1)
        assert (err <= bound).all(), float((err / bound).max())
    note(f"sampled {len(idx)}: ambiguous {int((~clear).sum())}; losses {L.tolist()} vs "
         f"{[q2['L_cos'], q2['L_lb'], q2['L_q']]}")
