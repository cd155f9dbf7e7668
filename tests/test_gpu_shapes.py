"""Every dedispersion launch shape the autotuner may pick gives bit-exact
results (ragged channels, trials and samples; uint8 and uint16 staging; the
16-bit tile and the byte-quad tile)."""
import numpy as np
import pytest

import oracle
from paper_2110_12749_amd import synth
from tests._util import say

pytestmark = pytest.mark.gpu

SHAPES = [(4, 4, 8, 16), (4, 4, 8, 32), (4, 8, 4, 16), (4, 8, 4, 32), (2, 8, 8, 16), (2, 8, 4, 32),
          (4, 4, 4, 16), (8, 4, 8, 16), (4, 4, 1, 3), (2, 8, 1, 1)]
# byte-quad tile (groups, tpw, waves, quads per pass, kind): the autotuner's
# candidates, one-quad and three-quad passes, a single summing wave
QUAD_SHAPES = [(8, 4, 8, 64, 1), (8, 4, 16, 64, 1), (8, 2, 16, 64, 1), (8, 2, 8, 64, 1), (4, 8, 8, 64, 1),
               (16, 2, 16, 64, 1), (4, 4, 8, 64, 1), (8, 4, 16, 3, 1), (8, 4, 8, 1, 1), (8, 2, 1, 64, 1),
               # kind 2: 4 staging waves besides `waves` summing waves
               (4, 8, 8, 64, 2), (8, 4, 8, 64, 2), (4, 8, 12, 64, 2), (4, 8, 1, 64, 2), (8, 4, 8, 3, 2)]


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
    # a sentinel in every output: an output no tile writes cannot pass
    dmt = ctx.dedisperse(fb, w.freqs, desc, out=torch.full((desc.total,), -1, dtype=torch.int32, device="cuda"))
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


@pytest.fixture(scope="module")
def quad_case(dev):
    """A multiple of 4 channels, ragged trials and samples, a D = 1 row (the
    byte-quad tile's) and a D = 2 row (which keeps the 16-bit tile)."""
    import torch
    from paper_2110_12749_amd import gsp
    w = synth.small(nchan=516, nsamp=9001, segments=[(0.0, 0.3, 71, 1), (21.3, 1.0, 13, 2)], tsamp=98.304e-6,
                    n_pulses=2)
    X = w.generate()
    ref = oracle.dedisperse(X, w.freqs, w.tsamp, w.segments)
    fb = torch.from_numpy(X).to("cuda")
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    ctx = gsp.Context(0)
    yield gsp, ctx, w, fb, desc, ref, torch
    torch.cuda.synchronize()
    ctx.close()


def test_quad_is_default_for_d1(quad_case):
    gsp, ctx, w, fb, desc, ref, torch = quad_case
    assert ctx.row_shape(w.freqs, desc, 0)[4] == 2
    assert ctx.row_shape(w.freqs, desc, 1)[4] == 0
    with pytest.raises(gsp.GspError):  # D = 2 rows are summed as 16-bit samples
        ctx.set_row_shape(w.freqs, desc, 1, 8, 4, 8, 64, 1)


@pytest.mark.parametrize("shape", QUAD_SHAPES)
def test_quad_shape_bit_exact(quad_case, shape):
    gsp, ctx, w, fb, desc, ref, torch = quad_case
    say(f"[case] quad shape {shape}")
    ctx.set_row_shape(w.freqs, desc, 0, *shape)
    used = ctx.row_shape(w.freqs, desc, 0)
    assert used[4] == shape[4] and used[3] <= shape[3], used
    dmt = ctx.dedisperse(fb, w.freqs, desc, out=torch.full((desc.total,), -1, dtype=torch.int32, device="cuda"))
    views = gsp.segment_views(desc, dmt)
    for s in range(desc.n_seg):
        assert (views[s].cpu().numpy() == ref[s]).all(), (shape, s)


def test_quad_shape_rejected_when_copies_do_not_fit(quad_case):
    """1024 outputs per wave and a single wave: a quad's copies exceed what
    one wave's staging registers hold, so the shape is refused with an error
    and the row keeps its previous tables."""
    gsp, ctx, w, fb, desc, ref, torch = quad_case
    ctx.set_row_shape(w.freqs, desc, 0, 8, 4, 8, 64, 1)
    with pytest.raises(gsp.GspError):
        ctx.set_row_shape(w.freqs, desc, 0, 16, 2, 1, 64, 1)
    assert ctx.row_shape(w.freqs, desc, 0)[:3] == (8, 4, 8)
    dmt = ctx.dedisperse(fb, w.freqs, desc)
    views = gsp.segment_views(desc, dmt)
    assert (views[0].cpu().numpy() == ref[0]).all()


@pytest.mark.parametrize("nchan,nsamp,tsamp,seg,kind", [
    (4, 3000, 196.608e-6, (0.0, 1.0, 3, 1), 2),      # one channel quad
    (8, 5000, 98.304e-6, (0.0, 0.5, 1, 1), 2),       # two quads, a single trial
    (12, 4097, 98.304e-6, (5.0, 0.7, 70, 1), 0),     # quad copies too wide: the 16-bit tile
])
def test_quad_default_on_few_channels(dev, nchan, nsamp, tsamp, seg, kind):
    """The D = 1 default on very few channels: the byte-quad tile where its
    copies fit, else the 16-bit tile; bit-exact either way."""
    import torch
    from paper_2110_12749_amd import gsp
    w = synth.small(nchan=nchan, nsamp=nsamp, segments=[seg], tsamp=tsamp, n_pulses=1)
    X = w.generate()
    ref = oracle.dedisperse(X, w.freqs, w.tsamp, w.segments)
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    ctx = gsp.Context(0)
    try:
        assert ctx.row_shape(w.freqs, desc, 0)[4] == kind
        fb = torch.from_numpy(X).to("cuda")
        dmt = ctx.dedisperse(fb, w.freqs, desc, out=torch.full((desc.total,), -1, dtype=torch.int32, device="cuda"))
        assert (gsp.segment_views(desc, dmt)[0].cpu().numpy() == ref[0]).all()
    finally:
        torch.cuda.synchronize()
        ctx.close()


@pytest.fixture(scope="module")
def split_case(dev):
    """A wide band (256 channels over 270-1620 MHz): on the D = 1 row the
    lowest quads' delay copies do not fit the byte-quad tile, so the row's
    band is split between the two tiles; a D = 2 row keeps the 16-bit tile."""
    import torch
    from paper_2110_12749_amd import gsp
    w = synth.small(nchan=256, nsamp=40000, segments=[(0.0, 0.1, 200, 1), (20.0, 0.3, 40, 2)], f_lo=270.0,
                    f_hi=1620.0, n_pulses=2, seed_offset=33)
    X = w.generate()
    ref = oracle.dedisperse(X, w.freqs, w.tsamp, w.segments)
    fb = torch.from_numpy(X).to("cuda")
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    ctx = gsp.Context(0)
    yield gsp, ctx, w, fb, desc, ref, torch
    torch.cuda.synchronize()
    ctx.close()


def _check_rows(gsp, ctx, w, fb, desc, ref, torch):
    dmt = ctx.dedisperse(fb, w.freqs, desc, out=torch.full((desc.total,), -1, dtype=torch.int32, device="cuda"))
    views = gsp.segment_views(desc, dmt)
    for s in range(desc.n_seg):
        got = views[s].cpu().numpy()
        bad = np.argwhere(got != ref[s])
        assert len(bad) == 0, f"row {s}: {len(bad)} mismatches, first {bad[:5].tolist()}"


def test_split_is_default_on_a_wide_band(split_case):
    gsp, ctx, w, fb, desc, ref, torch = split_case
    say(f"[case] split default, shapes {ctx.row_shape(w.freqs, desc, 0)} {ctx.row_shape(w.freqs, desc, 1)}")
    assert ctx.row_shape(w.freqs, desc, 0)[4] == 3
    assert ctx.row_shape(w.freqs, desc, 1)[4] == 0
    _check_rows(gsp, ctx, w, fb, desc, ref, torch)


@pytest.mark.parametrize("descending", [False, True])
def test_split_either_band_order(dev, descending):
    """Channels in descending frequency: the quads that do not fit are at the
    high-index end, and the 16-bit tile takes that end."""
    import torch
    from paper_2110_12749_amd import gsp
    w = synth.small(nchan=128, nsamp=30000, segments=[(0.0, 0.2, 70, 1)], f_lo=270.0, f_hi=1620.0, n_pulses=1,
                    seed_offset=34)
    X, freqs = w.generate(), w.freqs
    if descending:  # the same data with the channel axis reversed
        X, freqs = np.ascontiguousarray(X[:, ::-1]), freqs[::-1].copy()
    ref = oracle.dedisperse(X, freqs, w.tsamp, w.segments)
    desc = gsp.plan_shape(w.nsamp, freqs, w.tsamp, w.segments)
    ctx = gsp.Context(0)
    try:
        say(f"[case] split, descending={descending}: shape {ctx.row_shape(freqs, desc, 0)}")
        assert ctx.row_shape(freqs, desc, 0)[4] == 3
        dmt = ctx.dedisperse(torch.from_numpy(X).to("cuda"), freqs, desc,
                             out=torch.full((desc.total,), -1, dtype=torch.int32, device="cuda"))
        got = gsp.segment_views(desc, dmt)[0].cpu().numpy()
        bad = np.argwhere(got != ref[0])
        assert len(bad) == 0, f"{len(bad)} mismatches, first {bad[:5].tolist()}"
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_split_rejected_where_every_quad_fits(quad_case):
    gsp, ctx, w, fb, desc, ref, torch = quad_case
    with pytest.raises(gsp.GspError):
        ctx.set_row_shape(w.freqs, desc, 0, 4, 8, 8, 64, 3)


def test_split_tuned_then_parity(split_case):
    """The autotuner times the split tile against the others on this row
    (whichever wins, the sums stay exact)."""
    gsp, ctx, w, fb, desc, ref, torch = split_case
    shapes = ctx.autotune(fb, w.freqs, desc, n_reps=1)
    say(f"  tuned {shapes}")
    _check_rows(gsp, ctx, w, fb, desc, ref, torch)
