"""The parity helpers themselves, on the CPU: a rendering taken from the
oracle with planted branch choices (decisions inverted at some ambiguous
pixels) stands in for a GPU rendering, and the forward comparison must name
exactly the planted branches, also where they move the channels by less
than its tolerance (the final T tells them apart)."""
import numpy as np
import torch

import synth
from oracle import oracle as O
from tests import parity as PT


def test_compare_render_recovers_planted_branches(oracle_lib):
    scene, cams = synth.workload_c1()
    # a wide skip window, so that many pixels have ambiguous decisions
    oo = O.make_opts(16, eps_alpha=3e-2)
    fwd = O.forward(scene, cams, oo)
    r = fwd["views"][0]
    cam = cams[0]
    hw = cam.width * cam.height
    amb = np.nonzero(r["n_amb"] > 0)[0]
    assert len(amb) > 200, len(amb)
    rng = np.random.default_rng(5)
    planted = np.zeros(hw, np.uint32)
    pick = amb[rng.random(len(amb)) < 0.5]
    planted[pick] = 1
    fl = O.render_view(fwd["proj"][0], cam, oo, scene.channels, fwd["ids"], fwd["ranges"], 0, pix=pick,
                       flip_mask=np.ones(len(pick), np.uint32))
    out, T, last = r["out"].copy(), r["T"].copy(), r["last"].copy()
    out[:, pick], T[pick], last[pick] = fl["out"], fl["T"], fl["last"]
    moved = np.abs(fl["out"] - r["out"][:, pick]).max(axis=0)
    tol = 1e-2
    assert (moved < tol).sum() > 50            # flips the channels alone cannot tell apart
    masks, stats = PT.compare_render(torch.from_numpy(out.astype(np.float32).reshape(-1)),
                                     torch.from_numpy(T.astype(np.float32)),
                                     torch.from_numpy(last.astype(np.int32)), scene, cams, oo, fwd, tol=tol)
    # the planted branch, or one that renders identically (flipping a skip can
    # change nothing when the blend would have tripped the stop rule)
    diff = np.nonzero(masks[0] != planted)[0]
    assert len(diff) <= len(pick) // 20, len(diff)
    for q in diff:
        a, b = (O.render_view(fwd["proj"][0], cam, oo, scene.channels, fwd["ids"], fwd["ranges"], 0, pix=[q],
                              flip_mask=[m]) for m in (masks[0][q], planted[q]))
        assert np.array_equal(a["out"], b["out"]) and a["T"][0] == b["T"][0] and a["last"][0] == b["last"][0], q
