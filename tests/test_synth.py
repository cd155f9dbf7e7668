"""The seeded input generator: Philox4x32-10 known answers, noise model,
block-wise regeneration, injected-pulse geometry."""
import math

import numpy as np

from paper_2110_12749_amd import synth


def test_philox_known_answers():
    # Known-answer vectors of Philox4x32-10 (Salmon et al., SC'11; Random123).
    assert synth.philox4x32_10((0, 0, 0, 0), (0, 0)) == (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)
    assert synth.philox4x32_10((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2) == (0x408F276D, 0x41C83B0E, 0xA20BC7C6,
                                                                          0x6D5451FD)
    assert synth.philox4x32_10((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0)) == (
        0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)


def test_noise_moments():
    w = synth.small(nchan=256, nsamp=8192)
    X = w.generate(noise_only=True).astype(np.float64)
    # quantised N(128, 16): mean 128, variance 256 + 1/12 (no clipping at 8 sigma)
    assert abs(X.mean() - 128.0) < 0.05
    assert abs(X.var() - (256.0 + 1.0 / 12.0)) < 1.0
    z = (X - 128.0) / 16.0
    assert abs((z ** 3).mean()) < 0.02
    assert abs((z ** 4).mean() - 3.0) < 0.05


def test_blocks_regenerate_identically():
    w = synth.small(nchan=64, nsamp=4096, n_pulses=2)
    w.bursts = [(3, 0.1, 0.3, 40.0, 7.0, 0.5), (60, 0.0, 2.0, 25.0, 3.0, 0.0)]
    w.spikes = [(999, 3, 40.0), (2000, 1, 40.0)]
    whole = w.generate()
    assert (whole != w.generate(noise_only=True)).any()
    parts = [w.generate(t_begin=a, nrows=b - a) for a, b in [(0, 1000), (1000, 1001), (1001, 4096)]]
    assert (np.concatenate(parts) == whole).all()


def test_pulse_lands_at_dispersed_time():
    w = synth.small(nchan=16, nsamp=4096, n_pulses=1)
    p = w.pulses[0]
    p.amp = 100.0  # bright but below clipping
    p.fwhm_s = 1.5 * w.tsamp
    X = w.generate().astype(np.int64) - w.generate(noise_only=True).astype(np.int64)
    fmax = w.freqs.max()
    for c in range(16):
        t = (p.t0_s + 4148.808 * p.dm * (w.freqs[c] ** -2 - fmax ** -2)) / w.tsamp
        col = X[:, c]
        assert abs(int(np.argmax(col)) - t) <= 1.0


def test_pulse_amplitude_matches_target_snr():
    """A * sqrt(nchan) * sqrt(sum g^2) / std equals the requested SNR."""
    tsamp, fwhm, nchan = 49.152e-6, 5e-3, 4096
    a = synth.pulse_amplitude(12.0, fwhm, tsamp, nchan)
    sig = fwhm / (2 * math.sqrt(2 * math.log(2))) / tsamp
    t = np.arange(-2000, 2000)
    g2 = np.exp(-(t / sig) ** 2).sum()
    assert abs(a * math.sqrt(nchan) * math.sqrt(g2) / 16.0 - 12.0) < 1e-3


def test_plans():
    assert sum(s[2] for s in synth.realistic(nsamp=1 << 16).segments) == 3850
    assert sum(s[2] for s in synth.wideband(nsamp=1 << 16).segments) == 3350
    for n in (1000, 2600, 3850, 4000):
        assert sum(s[2] for s in synth.ladder(n_trials=n)) == n
