"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test fixes the oracle to something independent: exact rational
arithmetic, brute-force Python loops, closed forms, conservation laws, the
paper's own DDplan tables (tests/golden/ddplan_tables.json) and recovery of
injected pulses.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2110_12749_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
K = Fraction("4148.808")


def frac_delay(dm: Fraction, f: Fraction, fref: Fraction, tsamp: Fraction, D: int):
    """floor(r + 1/2) in exact rational arithmetic, and the exact r."""
    r = K * dm * (1 / (f * f) - 1 / (fref * fref)) / (tsamp * D)
    return math.floor(r + Fraction(1, 2)), r


def frac_centres(lo, hi, nchan):
    lo, hi = Fraction(lo), Fraction(hi)
    return [lo + (Fraction(2 * c + 1, 2)) * (hi - lo) / nchan for c in range(nchan)]


# --- delay table -------------------------------------------------------------

def test_delay_table_tiny_matches_exact_rationals():
    """All 200 x 128 delays of the tiny workload equal floor(r + 1/2) of the
    exact rational r, and no r lies near a rounding tie."""
    w = synth.tiny()
    fr = frac_centres("1000", "1500", 128)
    fref = fr[-1]
    ts = Fraction("196.608e-6")
    d = oracle.delay_table(w.freqs, w.tsamp, w.segments[0])
    margin = 1.0
    for i in range(200):
        for c in range(128):
            exact, r = frac_delay(Fraction(i), fr[c], fref, ts, 1)
            assert d[i, c] == exact, (i, c)
            if i:
                margin = min(margin, abs(float(r - math.floor(r)) - 0.5))
    assert margin > 1e-6


def test_delay_worked_values():
    """Worked delays of the tiny workload (channels 0, 32, 64, 96, 126, 127),
    from exact rational evaluation of the dispersion law."""
    w = synth.tiny()
    f = w.freqs
    fref = oracle.fref(f)
    chans = [0, 32, 64, 96, 126, 127]
    expect = {1.0: [12, 7, 4, 2, 0, 0], 57.3: [666, 413, 233, 99, 3, 0],
              100.0: [1162, 721, 406, 173, 5, 0], 199.0: [2312, 1435, 808, 344, 10, 0]}
    fr = frac_centres("1000", "1500", 128)
    for dm, vals in expect.items():
        got = [oracle.delay(dm, f[c], fref, w.tsamp, 1) for c in chans]
        assert got == vals
        exact = [frac_delay(Fraction(str(dm)), fr[c], fr[-1], Fraction("196.608e-6"), 1)[0] for c in chans]
        assert exact == vals
    md, no = oracle.plan_shape(w.nsamp, f, w.tsamp, w.segments)
    assert md[0] == 2312 and no[0] == 16384 - 2312


@pytest.mark.parametrize("D", [2, 4, 8])
def test_delay_downsampled_rows_match_rationals(D):
    """Rows with downsampling round at D * tsamp (wideband band, sampled DMs)."""
    nchan = 64
    fr = frac_centres("270", "1620", nchan)
    f = np.array([float(x) for x in fr])
    ts = "196.608e-6"
    seg = (450.0, 1.0, 40, D)
    d = oracle.delay_table(f, float(ts), seg)
    for i in range(0, 40, 3):
        for c in range(0, nchan, 5):
            exact, _ = frac_delay(Fraction(450) + i, fr[c], fr[-1], Fraction(ts), D)
            assert d[i, c] == exact


def test_delay_reference_is_highest_channel_any_order():
    """f_ref is the highest frequency wherever it sits; delays are >= 0 and
    zero only there (DM > 0)."""
    f = np.array([1400.0, 1100.0, 1500.0, 1000.0, 1250.0])
    assert oracle.fref(f) == 1500.0
    d = oracle.delay_table(f, 1e-4, (10.0, 5.0, 4, 1))
    assert (d >= 0).all()
    assert (d[:, 2] == 0).all() and (d[:, [0, 1, 3, 4]] > 0).all()
    # descending-frequency ordering gives the mirrored table
    d2 = oracle.delay_table(f[::-1], 1e-4, (10.0, 5.0, 4, 1))
    assert (d2 == d[:, ::-1]).all()


# --- plan rows (paper Tables 2 and 3) ---------------------------------------

def test_ddplan_tables_row_counts_and_half_open_grid():
    """N_DM = (high - low) / dDM for every row of the paper's two DM plans;
    rows are contiguous, and the oracle's grid lo + i * step, i < N_DM,
    stays below the row's high DM, whose value starts the next row."""
    g = json.load(open(os.path.join(GOLDEN, "ddplan_tables.json")))
    for band in ("band1", "band2"):
        rows = g[band]
        for k, (lo, hi, step, D, n) in enumerate(rows):
            lo_, hi_, st = Fraction(lo), Fraction(hi), Fraction(step)
            assert (hi_ - lo_) / st == n
            if k + 1 < len(rows):
                assert rows[k + 1][0] == hi
            seg = (float(lo), float(step), n, D)
            assert oracle.trial_dm(seg, 0) == float(lo)
            assert oracle.trial_dm(seg, n - 1) < float(hi)
            assert abs(oracle.trial_dm(seg, n) - float(hi)) < 1e-9
    # sum of the Band1 / Band2 DM counts
    assert sum(r[4] for r in g["band1"]) == 3462
    assert sum(r[4] for r in g["band2"]) == 10730


def test_band1_plan_shape_downsampling_scales_delays():
    """Band1 (Table 1: 512 ch over 271-398 MHz) with its first four plan
    rows: the maximum delay of each row is the exact-rational maximum."""
    g = json.load(open(os.path.join(GOLDEN, "ddplan_tables.json")))
    b = g["bands"]["band1"]
    fr = frac_centres(str(b["f_lo_mhz"]), str(b["f_hi_mhz"]), b["nchan"])
    f = np.array([float(x) for x in fr])
    ts = Fraction("98e-6")
    segs = [(float(lo), float(st), n, D) for lo, hi, st, D, n in g["band1"][:4]]
    md, no = oracle.plan_shape(1 << 19, f, float(ts), segs)
    for s, (lo, hi, st, D, n) in enumerate(g["band1"][:4]):
        dm_last = Fraction(lo) + (n - 1) * Fraction(st)
        exact, _ = frac_delay(dm_last, fr[0], fr[-1], ts, D)
        assert md[s] == exact
        assert no[s] == (1 << 19) // D - exact


# --- dedispersion sums ------------------------------------------------------

def brute_dedisperse(X, delays, D, n_out):
    """Independent triple loop straight from the definition."""
    nsamp, nchan = X.shape
    n_dm = delays.shape[0]
    out = np.zeros((n_dm, n_out), dtype=np.int64)
    for i in range(n_dm):
        for t in range(n_out):
            s = 0
            for c in range(nchan):
                base = (t + int(delays[i][c])) * D
                for m in range(D):
                    s += int(X[base + m][c])
            out[i][t] = s
    return out


@pytest.mark.parametrize("D", [1, 3])
def test_dedisperse_brute_force_tiny(D):
    rng = np.random.default_rng(7 + D)
    nchan, nsamp = 12, 256
    # wide band so delays span 0 .. large within 8 trials
    fr = frac_centres("300", "900", nchan)
    f = np.array([float(x) for x in fr])
    tsamp = 1e-3
    seg = (0.0, 0.3, 8, D)
    X = rng.integers(0, 256, size=(nsamp, nchan), dtype=np.uint8)
    d = np.array([[frac_delay(Fraction(3, 10) * i, fr[c], fr[-1], Fraction(1, 1000), D)[0] for c in range(nchan)]
                  for i in range(8)])
    assert d.min() == 0 and d.max() > 10
    n_out = nsamp // D - d.max()
    ref = brute_dedisperse(X, d, D, n_out)
    got = oracle.dedisperse_segment(X, f, tsamp, seg)
    assert got.shape == ref.shape
    assert (got == ref).all()
    # individual points straight from the raw filterbank
    tr = rng.integers(0, 8, 50)
    tt = rng.integers(0, n_out, 50)
    pts = oracle.dedisperse_points(X, f, tsamp, seg, tr, tt)
    assert (pts == ref[tr, tt]).all()


def test_dm_zero_is_channel_sum():
    w = synth.small(nchan=32, nsamp=2048, segments=[(0.0, 2.0, 4, 1)])
    X = w.generate()
    out = oracle.dedisperse_segment(X, w.freqs, w.tsamp, w.segments[0])
    n_out = out.shape[1]
    assert (out[0] == X[:n_out].astype(np.int64).sum(axis=1)).all()
    # D = 2: the channel sum of row pairs
    out2 = oracle.dedisperse_segment(X, w.freqs, w.tsamp, (0.0, 2.0, 4, 2))
    pair = X[: 2 * out2.shape[1]].astype(np.int64).reshape(-1, 2, 32).sum(axis=(1, 2))
    assert (out2[0] == pair).all()


@pytest.mark.parametrize("D", [1, 2])
def test_single_sample_delta_shift_direction(D):
    """A single nonzero pixel X[t*][c*] = v shows up in trial i only at
    t = t*//D - d[i][c*]."""
    nchan, nsamp = 16, 1024
    f = np.linspace(1000, 1500, nchan)
    tsamp = 2e-4
    seg = (0.0, 7.0, 6, D)
    d = oracle.delay_table(f, tsamp, seg)
    for cs in (0, 5, 15):
        X = np.zeros((nsamp, nchan), np.uint8)
        ts = 600
        X[ts, cs] = 201
        out = oracle.dedisperse_segment(X, f, tsamp, seg)
        n_out = out.shape[1]
        for i in range(6):
            nz = np.nonzero(out[i])[0]
            t_exp = ts // D - d[i, cs]
            if 0 <= t_exp < n_out:
                assert list(nz) == [t_exp] and out[i, t_exp] == 201
            else:
                assert len(nz) == 0


def test_conservation_over_valid_range():
    """sum_t out[i][t] = sum_c (Q_c[d_ic + n_out] - Q_c[d_ic]), Q_c the
    per-channel prefix sums of the downsampled data."""
    w = synth.small(nchan=48, nsamp=4096, segments=[(0.0, 3.0, 10, 2)])
    X = w.generate()
    seg = w.segments[0]
    out = oracle.dedisperse_segment(X, w.freqs, w.tsamp, seg)
    d = oracle.delay_table(w.freqs, w.tsamp, seg)
    n_out = out.shape[1]
    Y = X[: (X.shape[0] // 2) * 2].astype(np.int64).reshape(-1, 2, 48).sum(axis=1).T  # [c][j]
    Q = np.concatenate([np.zeros((48, 1), np.int64), np.cumsum(Y, axis=1)], axis=1)
    for i in range(10):
        exp = sum(Q[c, d[i, c] + n_out] - Q[c, d[i, c]] for c in range(48))
        assert out[i].astype(np.int64).sum() == exp


def test_downsample_against_reshape_sum():
    rng = np.random.default_rng(3)
    X = rng.integers(0, 256, size=(1001, 7), dtype=np.uint8)
    for D in (1, 2, 3, 8):
        Y = oracle.downsample(X, D)
        n = 1001 // D
        ref = X[: n * D].astype(np.int64).reshape(n, D, 7).sum(axis=1).T
        assert (Y == ref).all()


def test_linearity_without_clipping():
    rng = np.random.default_rng(11)
    f = np.linspace(1200, 1500, 24)
    seg = (0.0, 20.0, 5, 1)
    A = rng.integers(0, 128, size=(3000, 24), dtype=np.uint8)
    B = rng.integers(0, 128, size=(3000, 24), dtype=np.uint8)
    oa = oracle.dedisperse_segment(A, f, 1e-4, seg).astype(np.int64)
    ob = oracle.dedisperse_segment(B, f, 1e-4, seg).astype(np.int64)
    oab = oracle.dedisperse_segment(A + B, f, 1e-4, seg).astype(np.int64)
    assert (oab == oa + ob).all()


# --- statistics --------------------------------------------------------------

def test_stats_exact_moments_vs_fractions():
    rng = np.random.default_rng(5)
    for n in (2, 3, 17, 500):
        x = rng.integers(-3_000_000, 3_000_000, size=n).astype(np.int32)
        mu, sg = oracle.stats(x)
        m = Fraction(int(x.astype(np.int64).sum()), n)
        var = sum((Fraction(int(v)) - m) ** 2 for v in x) / n
        assert abs(mu - float(m)) <= 1e-12 * max(1.0, abs(float(m)))
        assert abs(sg - math.sqrt(float(var))) <= 1e-9 * math.sqrt(float(var))


def test_stats_large_offset_no_cancellation():
    """A large constant offset does not spoil sigma (moments about x[0])."""
    x = (2_000_000_000 + np.array([0, 1, 2, 3, 4] * 100)).astype(np.int64).astype(np.int32)
    mu, sg = oracle.stats(x)
    assert abs(sg - math.sqrt(2.0)) < 1e-12
    assert abs(mu - 2_000_000_002) < 1e-6


# --- boxcar search -----------------------------------------------------------

def test_spike_snr_closed_form():
    """Constant series with one spike of height h: SNR at w = 1 is sqrt(n-1),
    at a width-w box covering it (n - w) / (sqrt(n-1) sqrt(w))."""
    n, k, h = 1000, 400, 37
    x = np.full(n, 5000, np.int32)
    x[k] += h
    c = oracle.search_series(x, [1], 6.0)
    assert len(c) == 1 and c[0]["t_peak"] == k and c[0]["width"] == 1
    assert abs(c[0]["snr"] - math.sqrt(n - 1)) < 1e-9
    mu, sg = oracle.stats(x)
    for wdt in (2, 4, 8):
        r = oracle.search_range(x, k + wdt - 1, k + wdt, mu, sg, [wdt], 0.0)
        assert len(r) == 1
        assert abs(r[0]["snr"] - (n - wdt) / (math.sqrt(n - 1) * math.sqrt(wdt))) < 1e-9
    # best over widths is the narrowest box: it is the peak of the run
    c = oracle.search_series(x, [1, 2, 4, 8], 6.0)
    assert len(c) == 1 and c[0]["width"] == 1 and c[0]["t_peak"] == k
    # the run covers every box end whose best box still holds the spike
    assert c[0]["t_first"] == k and c[0]["t_last"] == k + 7


def test_constant_series_has_no_candidates():
    assert len(oracle.search_series(np.full(100, 7, np.int32), [1, 2, 4], 0.0)) == 0


def _balanced_series(n, base, devs):
    """base + deviations, with compensating -1s far away so the mean is base."""
    x = np.full(n, base, np.int64)
    for p, v in devs.items():
        x[p] += v
    excess = sum(devs.values())
    for j in range(excess):
        x[10 + 7 * j] -= 1
    assert x.sum() == base * n
    return x.astype(np.int32)


def test_tie_rules_width_and_time():
    # equal snr for w = 1 and w = 4 at the same end: the smaller width wins
    x = _balanced_series(2000, 300, {800: 1, 801: 1, 802: 0, 803: 2})
    mu, sg = oracle.stats(x)
    assert mu == 300.0
    r = oracle.search_range(x, 803, 804, mu, sg, [4, 1], 0.0)
    s1 = (2.0) / (sg * 1.0)
    s4 = (4.0) / (sg * 2.0)
    assert s1 == s4
    assert len(r) == 1 and r[0]["width"] == 1 and r[0]["t_peak"] == 803
    # two equal peaks inside one run: the earlier box end wins
    x = _balanced_series(2000, 300, {900: 3, 901: 3})
    c = oracle.search_series(x, [1], 6.0)
    assert len(c) == 1 and c[0]["t_first"] == 900 and c[0]["t_last"] == 901 and c[0]["t_peak"] == 900


def test_threshold_is_inclusive_and_widths_are_a_set():
    x = _balanced_series(1500, 100, {700: 4})
    mu, sg = oracle.stats(x)
    snr = (104 - mu) / sg
    thr = np.float32(snr)
    if float(thr) > snr:
        thr = np.nextafter(thr, np.float32(-np.inf))
    # the largest float32 threshold not above the peak SNR flags it ...
    c = oracle.search_series(x, [1], float(thr))
    assert len(c) == 1 and c[0]["t_peak"] == 700
    # ... the next float32 up does not
    assert len(oracle.search_series(x, [1], float(np.nextafter(thr, np.float32(np.inf))))) == 0
    a = oracle.search_series(x, [2, 1, 2, 1, 4], 5.0)
    b = oracle.search_series(x, [1, 2, 4], 5.0)
    assert (a == b).all()


def test_boxes_never_start_before_zero():
    x = _balanced_series(1000, 50, {0: 9, 1: 9})
    c = oracle.search_series(x, [1, 2, 4, 8], 6.0)
    assert len(c) >= 1 and c[0]["t_peak"] >= 0
    # at e = 0 only w = 1 is valid
    mu, sg = oracle.stats(x)
    r = oracle.search_range(x, 0, 1, mu, sg, [8, 2, 1], 0.0)
    assert r[0]["width"] == 1


def test_window_search_covers_series_when_whole():
    rng = np.random.default_rng(1)
    x = rng.normal(1000, 30, size=5000).astype(np.int32)
    x[2500:2510] += 100
    a = oracle.search_series(x, [1, 2, 4, 8], 4.0)
    b = oracle.search_window(x, 0, len(x), [1, 2, 4, 8], 4.0)
    assert (a == b).all()


def _brute_window(x, w0, w1, widths, thr, clip_at_window=False, stats_span=None):
    """Pure-Python window search: statistics (population mean and sigma in
    exact rationals) over x[w0:w1] (or over `stats_span`), every box end e in
    [w0, w1), boxes [e-w+1, e] reaching back before w0 (or clipped at w0 when
    asked, a deliberately wrong rule), best over the sorted width set (ties to
    the smaller width), one candidate per maximal run at its argmax (ties to
    the earlier end).  Returns [(t_peak, width, t_first, t_last, snr)]."""
    a, b = stats_span if stats_span else (w0, w1)
    seg = [int(v) for v in x[a:b]]
    n = len(seg)
    mean = Fraction(sum(seg), n)
    var = Fraction(sum(v * v for v in seg), n) - mean * mean
    mu, sg = float(mean), math.sqrt(float(var))
    ws = sorted(set(widths))
    best = []
    for e in range(w0, w1):
        bw, bs = 0, None
        for w in ws:
            lo = e - w + 1
            if lo < 0 or (clip_at_window and lo < w0):
                continue
            snr = (sum(int(v) for v in x[lo:e + 1]) - w * mu) / (sg * math.sqrt(w))
            if bs is None or snr > bs:
                bw, bs = w, snr
        best.append((e, bw, bs))
    out, run = [], None
    for e, bw, bs in best + [(w1, 0, None)]:
        if bs is not None and bs >= thr:
            if run is None:
                run = [e, e, bw, bs, e]
            else:
                run[1] = e
                if bs > run[3]:
                    run[2], run[3], run[4] = bw, bs, e
        elif run is not None:
            first, last, bw_, bs_, ep = run
            out.append((ep - bw_ + 1, bw_, first, last, bs_))
            run = None
    return out


def test_window_search_reaches_back_and_takes_window_statistics():
    """orc_search_window with w0 > 0 equals a brute-force loop: statistics
    over [w0, w1) only, boxes ending in the window reaching back before w0,
    runs cut at both window edges.  The case is built so that the two
    plausible mistakes (boxes clipped at w0, statistics over the whole
    series) give different candidates."""
    rng = np.random.default_rng(4)
    x = rng.normal(1000, 20, size=3000).round().astype(np.int32)
    x[:1200] += 60                      # before the window: a different level
    w0, w1 = 1200, 2400
    x[1190:1203] += 120                 # a pulse straddling the window start
    x[1700:1712] += 90                  # one inside
    x[2395:2400] += 150                 # one touching the window end
    widths = [1, 2, 4, 8, 16, 32]
    thr = 6.0
    got = oracle.search_window(x, w0, w1, widths, thr)
    want = _brute_window(x, w0, w1, widths, thr)
    assert len(got) == len(want) >= 3
    for g, (tp, w, tf, tl, snr) in zip(got, want):
        assert (g["t_peak"], g["width"], g["t_first"], g["t_last"]) == (tp, w, tf, tl)
        assert g["snr"] == pytest.approx(snr, rel=1e-12)
    assert want[0][0] < w0 and want[0][2] == w0       # its peak box starts before the window
    assert want[-1][3] == w1 - 1                      # the last run is cut at the window end
    # the wrong readings differ from the right one on this case
    assert _brute_window(x, w0, w1, widths, thr, clip_at_window=True) != want
    assert _brute_window(x, w0, w1, widths, thr, stats_span=(0, len(x))) != want


# --- grouping ----------------------------------------------------------------

def test_group_friends_of_friends():
    c = np.zeros(6, oracle.CAND_DTYPE)
    # chain 0-1-2 over neighbouring trials with overlapping runs; 3 isolated in
    # time; 4 two trials away from 2 (not linked); 5 overlaps 4
    rows = [(10, 100, 105, 7.0), (11, 104, 108, 9.0), (12, 108, 110, 8.0), (11, 300, 301, 6.5),
            (14, 100, 110, 6.1), (15, 110, 112, 6.2)]
    for k, (tr, a, b, s) in enumerate(rows):
        c[k] = (tr, 1, a, a, b, s)
    g = oracle.group(c)
    assert list(g) == [1, 1, 1, 3, 5, 5]


# --- end to end: injected pulse ---------------------------------------------

def test_tiny_injected_pulse_recovered():
    """The tiny workload's pulse (DM 57.3, FWHM 2 ms, SNR 15) is the top
    candidate: trial within one of 57, width within x2 of the optimal
    boxcar 1.19 FWHM / tsamp, SNR close to the injected value."""
    w = synth.tiny()
    X = w.generate()
    out = oracle.dedisperse(X, w.freqs, w.tsamp, w.segments)
    assert out[0].shape == (200, 14072)
    c = oracle.search(out, w.widths, w.threshold)
    best = c[np.argmax(c["snr"])]
    assert abs(int(best["trial"]) - 57) <= 1
    opt = 1.19 * 2e-3 / w.tsamp
    assert opt / 2 <= best["width"] <= opt * 2
    assert 0.94 * 15 - 1.5 <= best["snr"] <= 0.94 * 15 + 1.5
    t_s = (best["t_peak"] + best["width"] / 2) * w.tsamp
    assert abs(t_s - 1.5) < 2e-3


def test_noise_only_false_alarms_are_rare():
    w = synth.tiny()
    X = w.generate(noise_only=True)
    out = oracle.dedisperse(X, w.freqs, w.tsamp, w.segments)
    c = oracle.search(out, w.widths, w.threshold)
    assert len(c) < 20
    assert (c["snr"] < 7.5).all() if len(c) else True
