"""Pins of the sub-band (two-stage) dedispersion oracle against facts
outside it: the special cases that reduce to the pinned brute-force
oracle, a pure-Python brute force over exact-rational composite delays on
tiny inputs, the bound on how far composite delays may move from the
brute-force ones, and recovery of the tiny workload's injected pulse."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2110_12749_amd import synth

K = Fraction("4148.808")


def _fr(x):
    return Fraction(repr(float(x)))


def _rdelay(dm, f, fb, tsamp, D):
    r = K * dm * (1 / (f * f) - 1 / (fb * fb)) / (tsamp * D)
    return math.floor(r + Fraction(1, 2)), r


def _bands(nchan, n_sub):
    return [list(range(b * nchan // n_sub, (b + 1) * nchan // n_sub)) for b in range(n_sub)]


def test_one_channel_per_band_is_brute_force():
    """n_sub = nchan: no stage-1 shift, stage-2 delays are the channels'
    own, so the output is the brute-force dedispersion."""
    w = synth.small(nchan=24, nsamp=3000, segments=[(0.0, 2.0, 20, 1)], n_pulses=1, seed_offset=301)
    X = w.generate()
    for group in (1, 4, 7):
        got = oracle.dedisperse_subband(X, w.freqs, w.tsamp, w.segments[0], 24, group)
        assert np.array_equal(got, oracle.dedisperse_segment(X, w.freqs, w.tsamp, w.segments[0]))


@pytest.mark.parametrize("D", [1, 2])
def test_one_band_one_trial_groups_is_brute_force(D):
    """n_sub = 1 and groups of one trial: the band's reference is fref, the
    nominal DM is the trial's own, so stage 1 is the brute-force sum."""
    w = synth.small(nchan=20, nsamp=4000, segments=[(3.0, 1.5, 12, D)], n_pulses=1, seed_offset=302)
    X = w.generate()
    got = oracle.dedisperse_subband(X, w.freqs, w.tsamp, w.segments[0], 1, 1)
    assert np.array_equal(got, oracle.dedisperse_segment(X, w.freqs, w.tsamp, w.segments[0]))


@pytest.mark.parametrize("nchan,n_sub,group,D", [(12, 3, 3, 1), (10, 4, 4, 2), (9, 2, 5, 3)])
def test_two_stages_equal_python_brute_force(nchan, n_sub, group, D):
    """Tiny inputs: a pure-Python triple loop over the composite delays
    computed in exact rationals (nominal DM at the group centre, band
    reference = the band's highest channel) equals the oracle's two
    stages; ragged last groups and unequal bands included."""
    rng = np.random.default_rng(nchan * 100 + D)
    nsamp, n_dm, lo, step = 400, 11, Fraction(2), Fraction(3)
    freqs = [Fraction(1000) + Fraction(500) * (2 * c + 1) / (2 * nchan) for c in range(nchan)]
    fref = max(freqs)
    ts = Fraction("1e-3")
    X = rng.integers(0, 256, size=(nsamp, nchan), dtype=np.uint8)
    seg = (float(lo), float(step), n_dm, D)
    fl = np.array([float(f) for f in freqs])
    bands = _bands(nchan, n_sub)
    comp = np.zeros((n_dm, nchan), np.int64)
    for i in range(n_dm):
        g0 = (i // group) * group
        ng = min(group, n_dm - g0)
        dmg = lo + (Fraction(g0) + Fraction(ng - 1, 2)) * step
        dmi = lo + i * step
        for bl in bands:
            fb = max(freqs[c] for c in bl)
            d2, _ = _rdelay(dmi, fb, fref, ts, D)
            for c in bl:
                d1, _ = _rdelay(dmg, freqs[c], fb, ts, D)
                comp[i, c] = d2 + d1
    N = nsamp // D
    n_out = N - int(comp.max())
    d_or, n_or = oracle.subband_delays(fl, nsamp, float(ts), seg, n_sub, group)
    assert np.array_equal(d_or, comp) and n_or == n_out
    Y = X[:N * D].reshape(N, D, nchan).sum(axis=1, dtype=np.int64)
    want = np.zeros((n_dm, n_out), np.int64)
    for i in range(n_dm):
        for t in range(n_out):
            want[i, t] = sum(int(Y[t + comp[i, c], c]) for c in range(nchan))
    got = oracle.dedisperse_subband(X, fl, float(ts), seg, n_sub, group)
    assert np.array_equal(got, want)
    # a group's nominal DM sits at its centre
    assert oracle.group_dm(seg, group, 0) == pytest.approx(float(lo + Fraction(group - 1, 2) * step))


def test_composite_delays_within_smearing_bound_of_brute_force():
    """Each composite delay differs from the brute-force delay by at most
    the in-band smearing K |DM_i - DM_g| (f_c^-2 - f_b^-2) / (D tsamp) plus
    1.5 samples (three roundings of at most half a sample each: the two
    stage delays and the brute-force delay), on the realistic band."""
    nchan, n_sub, group = 256, 16, 8
    freqs = 1000.0 + (np.arange(nchan) + 0.5) * 500.0 / nchan
    for seg in [(0.0, 0.1, 96, 1), (150.0, 0.3, 64, 2)]:
        d_sub, _ = oracle.subband_delays(freqs, 1 << 16, 49.152e-6, seg, n_sub, group)
        d_bf = oracle.delay_table(freqs, 49.152e-6, seg)
        fb = np.array([freqs[bl].max() for bl in map(np.array, _bands(nchan, n_sub))])
        band_of = np.repeat(np.arange(n_sub), nchan // n_sub)
        for i in range(seg[2]):
            dmg = oracle.group_dm(seg, group, i // group)
            dmi = seg[0] + i * seg[1]
            smear = 4148.808 * abs(dmi - dmg) * (freqs ** -2 - fb[band_of] ** -2) / (seg[3] * 49.152e-6)
            assert np.all(np.abs(d_sub[i] - d_bf[i]) <= smear + 1.5 + 1e-9), i


def test_tiny_pulse_recovered_by_subband():
    """The tiny workload's pulse (DM 57.3, FWHM 2 ms, SNR 15) through
    16 sub-bands of 8 channels and groups of 8 trials: found at trial
    57 +- 1 with at least 0.9 of the brute-force SNR."""
    w = synth.tiny()
    X = w.generate()
    seg = w.segments[0]
    bf = oracle.search(oracle.dedisperse(X, w.freqs, w.tsamp, w.segments), w.widths, w.threshold)
    sb = oracle.search([oracle.dedisperse_subband(X, w.freqs, w.tsamp, seg, 16, 8)], w.widths, w.threshold)
    b_bf = bf[np.argmax(bf["snr"])]
    b_sb = sb[np.argmax(sb["snr"])]
    assert abs(int(b_sb["trial"]) - 57) <= 1
    assert b_sb["snr"] >= 0.9 * b_bf["snr"]
    assert abs(int(b_sb["t_peak"]) - int(b_bf["t_peak"])) <= 2
