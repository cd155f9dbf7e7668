"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Dedispersion: bit-exact (integer sums).  Statistics: relative 1e-9 (both
sides use the same exact integer moments; only double rounding may differ).
Candidates: the match rule of tests/_util.match_candidates with a relative
SNR tolerance of 1e-5.
"""
import numpy as np
import pytest

import oracle
from paper_2110_12749_amd import synth
from tests._util import match_candidates, oracle_cands_with_seg, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(dev):
    import torch
    from paper_2110_12749_amd import gsp
    ctx = gsp.Context(0)
    yield gsp, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def _run(env, w, X=None):
    gsp, ctx, torch = env
    if X is None:
        X = w.generate()
    fb = torch.from_numpy(X).to("cuda")
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    # a sentinel in every output: an output no tile writes cannot pass
    out = torch.full((desc.total,), -1, dtype=torch.int32, device="cuda")
    dmt = ctx.dedisperse(fb, w.freqs, desc, out=out)
    torch.cuda.synchronize()
    return X, desc, dmt


def _full_parity(env, w, search=True):
    gsp, ctx, torch = env
    say(f"[case] {w.name} nchan={w.nchan} nsamp={w.nsamp} segs={w.segments}")
    X, desc, dmt = _run(env, w)
    views = gsp.segment_views(desc, dmt)
    ref = oracle.dedisperse(X, w.freqs, w.tsamp, w.segments)
    for s in range(desc.n_seg):
        got = views[s].cpu().numpy()
        assert got.shape == ref[s].shape
        bad = np.argwhere(got != ref[s])
        assert len(bad) == 0, f"row {s}: {len(bad)} mismatches, first {bad[:5].tolist()}"
    mu, sg = ctx.trial_stats(dmt, desc)
    k = 0
    for s in range(desc.n_seg):
        for i in range(ref[s].shape[0]):
            m, g = oracle.stats(ref[s][i])
            assert abs(mu[k] - m) <= 1e-9 * abs(m) and abs(sg[k] - g) <= 1e-9 * g, (s, i)
            k += 1
    if search:
        cg = ctx.single_pulse_search(dmt, desc, w.widths, w.threshold)
        co = oracle_cands_with_seg([(s, c) for s in range(desc.n_seg)
                                    for c in [_ora_search_rows(ref[s], w.widths, w.threshold)]])
        n_exact = match_candidates(cg, co, w.threshold)
        say(f"  candidates gpu={len(cg)} oracle={len(co)} exact={n_exact}")
        return cg, co
    return None, None


def _ora_search_rows(arr, widths, thr):
    rows = [oracle.search_series(arr[i], widths, thr, trial=i) for i in range(arr.shape[0])]
    rows = [r for r in rows if len(r)]
    return np.concatenate(rows) if rows else np.zeros(0, oracle.CAND_DTYPE)


def test_tiny_full_parity_and_pulse(env):
    w = synth.tiny()
    cg, co = _full_parity(env, w)
    assert len(cg) == len(co)
    best = cg[np.argmax(cg["snr"])]
    assert abs(int(best["dm_index"]) - 57) <= 1
    assert abs(best["time_s"] - 1.5) < 2e-3


@pytest.mark.parametrize("nchan,nsamp,segs", [
    (64, 8192, [(0.0, 1.0, 64, 1)]),                     # exact tiles
    (37, 5000, [(0.0, 1.3, 45, 1)]),                     # ragged channels, time and trials
    (96, 9001, [(0.0, 2.0, 33, 2), (66.0, 3.0, 7, 3)]),  # D = 2, 3 with ragged tails
    (200, 12345, [(0.0, 0.5, 40, 1), (20.0, 1.0, 30, 4), (50.0, 4.0, 17, 8)]),
    (300, 4099, [(0.0, 0.25, 5, 1)]),                    # more channels than one flush of 256
    (1, 3000, [(0.0, 1.0, 3, 1)]),                       # one channel
    (8192, 4000, [(0.0, 0.5, 40, 1), (20.0, 1.0, 24, 2)]),  # two 64-lane groups per cutout band, long passes
])
def test_small_plans_parity(env, nchan, nsamp, segs):
    w = synth.small(nchan=nchan, nsamp=nsamp, segments=segs, n_pulses=2)
    _full_parity(env, w)


def test_saturated_input_no_overflow(env):
    """All-255 input: the largest sums of every row, through every flush."""
    gsp, ctx, torch = env
    w = synth.small(nchan=600, nsamp=6000, segments=[(0.0, 1.0, 20, 1), (20.0, 1.0, 10, 8)])
    X = np.full((w.nsamp, w.nchan), 255, np.uint8)
    X, desc, dmt = _run(env, w, X)
    views = gsp.segment_views(desc, dmt)
    assert (views[0].cpu().numpy() == 255 * 600).all()
    assert (views[1].cpu().numpy() == 255 * 600 * 8).all()
    # constant series: sigma 0 and no candidates
    assert len(ctx.single_pulse_search(dmt, desc, [1, 2, 4], 3.0)) == 0


@pytest.fixture(scope="module")
def full_cache(env):
    """One full-size workload at a time: (workload, input, plan, DM-time array
    on the device, the search's candidates)."""
    gsp, ctx, torch = env
    cache = {}
    yield cache
    cache.clear()
    torch.cuda.empty_cache()


def _full(env, cache, name):
    gsp, ctx, torch = env
    if name not in cache:
        cache.clear()
        torch.cuda.empty_cache()
        w = getattr(synth, name)()
        say(f"[case] {name} full size: generate, dedisperse, search")
        X, desc, dmt = _run(env, w)
        cg = ctx.single_pulse_search(dmt, desc, w.widths, w.threshold)
        cache[name] = (w, X, desc, dmt, cg)
    return cache[name]


def parity_trials(n_dm):
    """The first, the last and every 37th trial of a plan row."""
    return sorted(set([0, n_dm - 1] + list(range(0, n_dm, 37))))


FULL_ROWS = [("realistic", r) for r in range(4)] + [("wideband", r) for r in range(4)]


@pytest.mark.parametrize("name,row", FULL_ROWS, ids=[f"{n}-row{r}" for n, r in FULL_ROWS])
def test_full_size_rows_parity(env, full_cache, name, row):
    """The realistic workload (4096 ch over 1000-1500 MHz, 2^20 samples, 3850
    trials in 4 rows) and the wideband large-delay workload (4096 ch over
    270-1620 MHz, 2^19 samples, 3350 trials, maximum delay 84,250 samples at
    D = 4, RFI bursts and zero-DM spikes) at full size: whole dedispersed
    series of the first, the last and every 37th trial of the row, and of the
    trials nearest the injected pulses, bit-exact against the oracle, the search's candidates of those trials matched
    against the oracle's search of its own series, and corners plus 300
    random outputs of the row bit-exact."""
    gsp, ctx, torch = env
    w, X, desc, dmt, cg = _full(env, full_cache, name)
    seg = w.segments[row]
    views = gsp.segment_views(desc, dmt)
    n_dm, n_out = seg[2], desc.n_out[row]
    # and the trial nearest each injected pulse whose DM lies in this row
    lo, st = seg[0], seg[1]
    near = [int(round((p.dm - lo) / st)) for p in w.pulses]
    trials = sorted(set(parity_trials(n_dm)) | {i for i in near if 0 <= i < n_dm})
    say(f"[case] {name} row {row}: {len(trials)} whole trials of {n_dm}, {n_out} outputs each")
    n_c = 0
    for i in trials:
        ref = oracle.dedisperse_segment(X, w.freqs, w.tsamp, seg, trials=(i, i + 1))[0]
        got = views[row][i].cpu().numpy()
        bad = np.flatnonzero(got != ref)
        assert len(bad) == 0, f"row {row} trial {i}: {len(bad)} mismatches, first {bad[:5].tolist()}"
        co = oracle_cands_with_seg([(row, oracle.search_series(ref, w.widths, w.threshold, trial=i))])
        match_candidates(cg[(cg["seg"] == row) & (cg["dm_index"] == i)], co, w.threshold)
        n_c += len(co)
    say(f"  {len(trials)} trials bit-exact, {n_c} oracle candidates matched")
    rng = np.random.default_rng(1 + row)
    tr = np.concatenate([[0, n_dm - 1, 0, n_dm - 1], rng.integers(0, n_dm, 300)])
    tt = np.concatenate([[0, 0, n_out - 1, n_out - 1], rng.integers(0, n_out, 300)])
    ref = oracle.dedisperse_points(X, w.freqs, w.tsamp, seg, tr, tt)
    got = views[row][torch.from_numpy(tr).long().cuda(), torch.from_numpy(tt).long().cuda()].cpu().numpy()
    assert (got.astype(np.int64) == ref).all(), f"row {row}"
