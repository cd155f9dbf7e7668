"""Every dedispersion launch shape the autotuner may pick gives bit-exact
results (ragged channels, trials and samples; uint8 and uint16 staging)."""
import numpy as np
import pytest

import oracle
from paper_2110_12749_amd import synth
from tests._util import say

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4, 8, 16), (4, 4, 8, 32), (4, 8, 4, 16), (4, 8, 4, 32), (2, 8, 8, 16), (2, 8, 4, 32),
          (4, 4, 4, 16), (8, 4, 8, 16), (4, 4, 1, 3), (2, 8, 1, 1)]


@pytest.fixture(scope="module")
def case(dev):
    import torch
    from paper_2110_12749_amd import gsp
    w = synth.small(nchan=203, nsamp=7001, segments=[(0.0, 0.7, 45, 1), (31.5, 2.0, 13, 4)], n_pulses=2)
    X = w.generate()
    ref = oracle.dedisperse(X, w.freqs, w.tsamp, w.segments)
    fb = torch.from_numpy(X).to("cuda")
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    ctx = gsp.Context(0)
    yield gsp, ctx, w, fb, desc, ref, torch
    torch.cuda.synchronize()
    ctx.close()


@pytest.mark.parametrize("shape", SHAPES)
def test_shape_bit_exact(case, shape):
    gsp, ctx, w, fb, desc, ref, torch = case
    say(f"[case] shape {shape}")
    for s in range(desc.n_seg):
        ctx.set_row_shape(w.freqs, desc, s, *shape)
    dmt = ctx.dedisperse(fb, w.freqs, desc)
    views = gsp.segment_views(desc, dmt)
    for s in range(desc.n_seg):
        assert (views[s].cpu().numpy() == ref[s]).all(), (shape, s)


def test_autotune_then_parity(case):
    gsp, ctx, w, fb, desc, ref, torch = case
    shapes = ctx.autotune(fb, w.freqs, desc, n_reps=1)
    say(f"  tuned {shapes}")
    dmt = ctx.dedisperse(fb, w.freqs, desc)
    views = gsp.segment_views(desc, dmt)
    for s in range(desc.n_seg):
        assert (views[s].cpu().numpy() == ref[s]).all()
