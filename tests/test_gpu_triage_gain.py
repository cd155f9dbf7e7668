"""What the trained network gains over the plain search (learned triage).

The network is trained on the GPU by the library's own forward and backward
kernels, on cutouts of candidates that the GPU pipeline finds on seeded
synthetic beams (the realistic band and sampling, injected pulses, narrowband
bursts and zero-DM spikes), labelled by their injections.  On held-out beams
(disjoint beam numbers: independent noise, pulses and RFI) the test compares
the events (friends-of-friends groups of candidates) the plain search passes
on with those whose representative the network accepts, at a logit threshold
fixed on separate validation beams:

  recall (injected pulses with a passed event that matches them) with the
  network >= 0.99 x the plain search's, with fewer events passed on.

The plain threshold search stays the judge of recall: the network only drops
events."""
import json
import time

import numpy as np
import pytest

from paper_2110_12749_amd import synth, triage
from tests._util import say

pytestmark = pytest.mark.gpu

TRAIN_BEAMS, VAL_BEAMS, TEST_BEAMS = 32, 12, 24
STEPS, BATCH, LR = 1500, 256, 1e-3
MARGIN = 2.0  # logits below the weakest validation pulse's best event


@pytest.mark.timeout(900)
def test_trained_network_keeps_recall_and_cuts_events(dev):
    import torch
    from paper_2110_12749_amd import gsp
    rng = np.random.default_rng(1)
    ctx = gsp.Context(0)
    t0 = time.perf_counter()
    xs, ys = [], []
    for k in range(TRAIN_BEAMS):
        b = triage.Beam(ctx, synth.triage_beam(k, "train"), torch)
        pick = triage.pick_candidates(b, 16, 256, rng, neg_per_pos=3.0)
        if len(pick):
            xs.append(gsp.cutouts(ctx, b.fb, b.w.freqs, b.dmt, b.desc, b.cands[pick]))
            ys.append((b.pulse[pick] >= 0).astype(np.float32))
        b.release()
    x, y, npos, nneg = triage.balance(torch, xs, ys, rng)
    del xs
    say(f"[case] triage gain: {x.shape[0]} balanced training cutouts ({npos} positive, {nneg} negative), "
        f"{time.perf_counter() - t0:.0f} s")
    net = gsp.Cnn(ctx, seed=1)
    losses = triage.train(net, x, y, STEPS, BATCH, LR, rng, torch)
    del x, y
    torch.cuda.empty_cache()
    say(f"  trained {STEPS} steps: loss {losses[0][1]:.3f} -> {losses[-1][1]:.3f}")
    assert losses[-1][1] < 0.5 * losses[0][1]

    def scored(split, n):
        out = []
        for k in range(n):
            b = triage.Beam(ctx, synth.triage_beam(k, split), torch)
            ev, z = triage.event_scores(ctx, net, torch, b)
            out.append((b, ev, z))
            b.release()
        return out

    val = scored("val", VAL_BEAMS)
    best = []
    for b, ev, z in val:
        k = b.pulse[ev]
        best += [float(z[k == pk].max()) for pk in np.unique(k[k >= 0])]
    tau = min(best) - MARGIN
    test = scored("test", TEST_BEAMS)
    r_plain, e_plain, n_pulses = triage.recall_and_events(test, None)
    r_cnn, e_cnn, _ = triage.recall_and_events(test, tau)
    lost = []
    for b, ev, z in test:
        k = b.pulse[ev]
        for pk in np.unique(k[k >= 0]):
            zb = float(z[k == pk].max())
            if zb <= tau:
                p = b.w.pulses[int(pk)]
                lost.append((round(p.dm, 1), round(p.fwhm_s * 1e3, 2), round(p.snr, 1), round(zb, 2)))
    summary = {"pulses": n_pulses, "lost (dm, fwhm ms, snr, best logit)": lost, "found_plain": round(r_plain * n_pulses), "found_cnn": round(r_cnn * n_pulses),
               "recall_plain": r_plain, "recall_cnn": r_cnn, "events_plain": e_plain, "events_cnn": e_cnn,
               "tau": tau, "seconds": round(time.perf_counter() - t0, 1)}
    say("  " + json.dumps(summary))
    net.close()
    ctx.close()
    assert r_plain > 0.5
    assert r_cnn >= 0.99 * r_plain, summary
    assert e_cnn < e_plain, summary
