"""Pins of the integer RFI-mitigation oracle (clip of outlying zero-DM
spectra, zero-DM filter) against facts outside it: a hand-computed case,
exact invariants (a constant added to a spectrum leaves the zero-DM output
unchanged; filtered spectra have rounded mean 128; a huge threshold
changes nothing), and recovery of a dispersed pulse through both."""
from fractions import Fraction

import numpy as np

import oracle
from paper_2110_12749_amd import synth


def test_clip_hand_computed():
    """6 spectra x 4 channels, one block.  Zero-DM sums s = (8, 8, 8, 8, 8, 48):
    mean 14.67, population sigma 14.91; |48 - 14.67| = 33.3 > 2 sigma, the
    rest 6.67 < 2 sigma, so only spectrum 5 is flagged (1.5 sigma would
    flag nothing else either).  It becomes the channel means of the other
    five spectra, rounded half up: channel sums (10, 10, 10, 10) / 5 = 2."""
    X = np.array([[2, 2, 2, 2], [1, 3, 1, 3], [3, 1, 3, 1], [2, 2, 2, 2], [2, 2, 2, 2], [12, 12, 12, 12]], np.uint8)
    s = [int(v) for v in X.sum(axis=1)]
    mu = Fraction(sum(s), 6)
    var = Fraction(sum(v * v for v in s), 6) - mu * mu
    assert abs(48 - mu) ** 2 > 4 * var and all((v - mu) ** 2 <= 4 * var for v in s[:5])
    out, n = oracle.rfi_clean(X, clip_sigma=2.0, block=6)
    assert n == 1
    assert (out[:5] == X[:5]).all() and (out[5] == [2, 2, 2, 2]).all()
    # rounding half up of the means: channel sums 7 over 2 unflagged spectra -> 4 (3.5 up)
    Y = np.array([[3, 0], [4, 0], [90, 90]], np.uint8)
    out, n = oracle.rfi_clean(Y, clip_sigma=1.0, block=3)
    assert n == 1 and (out[2] == [4, 0]).all()


def test_huge_threshold_changes_nothing():
    w = synth.small(nchan=64, nsamp=3000, n_pulses=1, seed_offset=401)
    X = w.generate()
    out, n = oracle.rfi_clean(X, clip_sigma=1e9, block=512)
    assert n == 0 and (out == X).all()


def test_zero_dm_invariants():
    rng = np.random.default_rng(402)
    X = rng.integers(60, 196, size=(500, 37), dtype=np.uint8)  # no clamping can occur
    out, _ = oracle.rfi_clean(X, zero_dm=True)
    # each filtered spectrum has rounded mean 128
    z = (2 * out.astype(np.int64).sum(axis=1) + 37) // (2 * 37)
    assert (z == 128).all()
    # a constant added to a spectrum (a zero-DM broadband spike) is removed exactly
    Y = X.copy()
    Y[100] += 40
    Y[300:303] -= 17
    out2, _ = oracle.rfi_clean(Y, zero_dm=True)
    assert (out2 == out).all()
    # and filtering twice changes nothing more
    out3, _ = oracle.rfi_clean(out, zero_dm=True)
    assert (out3 == out).all()


def test_clip_flags_exactly_the_broadband_spikes():
    """Noise plus three strong zero-DM spikes: exactly those spectra are
    flagged, and each becomes the per-channel rounded means of its block's
    other spectra (exact rationals)."""
    w = synth.small(nchan=128, nsamp=4096, n_pulses=0, seed_offset=403)
    X = w.generate()
    spikes = [100, 2000, 3999]
    for j in spikes:
        X[j] = np.minimum(255, X[j].astype(np.int32) + 60).astype(np.uint8)
    out, n = oracle.rfi_clean(X, clip_sigma=6.0, block=1024)
    assert n == len(spikes)
    changed = np.flatnonzero((out != X).any(axis=1))
    assert list(changed) == spikes
    for j in spikes:
        b0 = (j // 1024) * 1024
        rows = [r for r in range(b0, min(b0 + 1024, 4096)) if r != j]
        sums = X[rows].astype(np.int64).sum(axis=0)
        want = [int(Fraction(int(v), len(rows)) + Fraction(1, 2)) for v in sums]  # floor(mean + 1/2)
        assert list(out[j]) == want


def test_dispersed_pulse_survives_mitigation():
    """A DM-300 pulse (FWHM 2 ms, SNR 20) over the tiny band, with zero-DM
    spikes: after clip and zero-DM filter the pulse keeps >= 0.9 of its
    SNR at its trial and the spikes' DM-0 candidates are gone."""
    w = synth.small(nchan=128, nsamp=20000, segments=[(0.0, 10.0, 40, 1)], n_pulses=0, seed_offset=404)
    w.pulses = [synth.Pulse(300.0, 2.0, 2e-3, 20.0)]
    w.spikes = [(3000, 2, 40.0), (9000, 1, 40.0), (15000, 3, 40.0)]
    synth._with_amps(w)
    X = w.generate()
    seg = w.segments[0]
    raw = oracle.search(oracle.dedisperse(X, w.freqs, w.tsamp, w.segments), w.widths, w.threshold)
    Xc, n = oracle.rfi_clean(X, clip_sigma=6.0, block=2048, zero_dm=True)
    cl = oracle.search(oracle.dedisperse(Xc, w.freqs, w.tsamp, w.segments), w.widths, w.threshold)
    assert n >= 3
    assert (raw["trial"] == 0).sum() >= 3 and (cl["trial"] == 0).sum() == 0

    def best(c):
        near = c[np.abs(c["trial"] - 30) <= 1]
        return float(near["snr"].max()) if len(near) else 0.0
    assert best(cl) >= 0.9 * best(raw) > 10
