"""Seeded synthetic workloads: filterbanks with injected pulses and RFI.

This module makes inputs only.  It holds none of the dedispersion or search
arithmetic; the CPU oracle and the GPU library both consume what it writes.

Input recipe (the paper's CRAFTS data are not available; these stand in):
  * uint8 time-major filterbank [nsamp][nchan], noise N(128, 16) quantised by
    rint-half-even and clipped to 0..255;
  * channel centres f_c = lo + (c + 1/2) * (hi - lo) / nchan, ascending;
  * pulses: unit-peak Gaussians of a given FWHM, dispersed with
    4148.808 s * DM * (f^-2 - f_max^-2), integrated over each sample; the
    per-channel peak A is set from a target matched-filter SNR as
    A = SNR * std / (sqrt(nchan) * sqrt(sigma_g * sqrt(pi) / tsamp));
  * RFI (wideband workload): narrowband sinusoid bursts in 5 % of the
    channels and zero-DM broadband spikes;
  * noise from Philox4x32-10 keyed by the seed, so any block of rows
    regenerates independently (used by the streaming tests).

DM plans follow the DDplan row layout of the paper's Tables 2-3
(low DM, DM step, number of DMs, downsampling).
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libgsp_synth.so")
SRC = os.path.join(HERE, "synth.c")
BASE_SEED = 2110127490


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Pulse(C.Structure):
    _fields_ = [("dm", C.c_double), ("t0_s", C.c_double), ("fwhm_s", C.c_double), ("amp", C.c_double)]


class _Burst(C.Structure):
    _fields_ = [("chan", C.c_int32), ("pad_", C.c_int32), ("t_start_s", C.c_double),
                ("dur_s", C.c_double), ("amp", C.c_double), ("period_samp", C.c_double),
                ("phase", C.c_double)]


class _Spike(C.Structure):
    _fields_ = [("t_sample", C.c_int64), ("n_samp", C.c_int32), ("pad_", C.c_int32), ("amp", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.gsps_filterbank.restype = C.c_int
        L.gsps_filterbank.argtypes = [P, C.c_int64, C.c_int64, C.c_int32, P, C.c_double, C.c_uint64,
                                      C.c_uint32, C.c_double, C.c_double, P, C.c_int32, P, C.c_int32, P,
                                      C.c_int32]
        L.gsps_philox4x32_10.restype = None
        L.gsps_philox4x32_10.argtypes = [P, P, P]
        L.gsps_normal.restype = C.c_double
        L.gsps_normal.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
        _lib = L
    return _lib


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().gsps_philox4x32_10(C.addressof(c), C.addressof(k), C.addressof(o))
    return tuple(int(v) for v in o)


def normal(seed: int, beam: int, flat_index: int) -> float:
    return float(lib().gsps_normal(seed, beam, flat_index))


@dataclass
class Pulse:
    dm: float
    t0_s: float      # arrival time at the highest channel frequency
    fwhm_s: float
    snr: float       # target matched-filter SNR at native resolution
    amp: float = 0.0  # per-channel peak, counts (derived from snr)


@dataclass
class Workload:
    """One beam's input and plan.  ``segments`` rows are (dm_lo, dm_step, n_dm, downsamp)."""
    name: str
    nchan: int
    f_lo: float
    f_hi: float
    tsamp: float
    nsamp: int
    segments: list
    widths: list
    threshold: float
    seed: int
    beam: int = 0
    mean: float = 128.0
    std: float = 16.0
    pulses: list = field(default_factory=list)
    bursts: list = field(default_factory=list)   # (chan, t_start_s, dur_s, amp, period_samp, phase)
    spikes: list = field(default_factory=list)   # (t_sample, n_samp, amp)

    @property
    def freqs(self) -> np.ndarray:
        c = np.arange(self.nchan, dtype=np.float64)
        return self.f_lo + (c + 0.5) * ((self.f_hi - self.f_lo) / self.nchan)

    @property
    def n_trials(self) -> int:
        return int(sum(s[2] for s in self.segments))

    def generate(self, t_begin: int = 0, nrows: int | None = None, out: np.ndarray | None = None,
                 noise_only: bool = False) -> np.ndarray:
        """Rows [t_begin, t_begin + nrows) as uint8 [nrows][nchan] (time-major)."""
        if nrows is None:
            nrows = self.nsamp - t_begin
        if out is None:
            out = np.empty((nrows, self.nchan), np.uint8)
        assert out.dtype == np.uint8 and out.shape == (nrows, self.nchan) and out.flags.c_contiguous
        f = np.ascontiguousarray(self.freqs)
        pulses = [] if noise_only else self.pulses
        bursts = [] if noise_only else self.bursts
        spikes = [] if noise_only else self.spikes
        pa = (_Pulse * max(1, len(pulses)))(*[_Pulse(p.dm, p.t0_s, p.fwhm_s, p.amp) for p in pulses])
        ba = (_Burst * max(1, len(bursts)))(*[_Burst(int(b[0]), 0, *map(float, b[1:])) for b in bursts])
        sa = (_Spike * max(1, len(spikes)))(*[_Spike(int(s[0]), int(s[1]), 0, float(s[2])) for s in spikes])
        rc = lib().gsps_filterbank(out.ctypes.data, t_begin, nrows, self.nchan, f.ctypes.data, self.tsamp,
                                   self.seed, self.beam, self.mean, self.std, C.addressof(pa), len(pulses),
                                   C.addressof(ba), len(bursts), C.addressof(sa), len(spikes))
        if rc != 0:
            raise RuntimeError(f"synthetic generator failed ({rc})")
        return out


def pulse_amplitude(snr: float, fwhm_s: float, tsamp: float, nchan: int, std: float = 16.0) -> float:
    """Per-channel peak giving matched-filter SNR `snr` on the true-DM series."""
    sig = fwhm_s / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    sum_g2 = sig * math.sqrt(math.pi) / tsamp
    return snr * std / (math.sqrt(nchan) * math.sqrt(sum_g2))


def _with_amps(w: Workload) -> Workload:
    for p in w.pulses:
        p.amp = pulse_amplitude(p.snr, p.fwhm_s, w.tsamp, w.nchan, w.std)
    return w


# DDplan-style ladder used by the realistic workloads: steps 0.1/0.3/1/3 pc cm^-3
# with downsampling 1/2/4/8 over 0-150/150-450/450-1200/1200-3000.
LADDER = [(0.0, 150.0, 0.1, 1), (150.0, 450.0, 0.3, 2), (450.0, 1200.0, 1.0, 4), (1200.0, 3000.0, 3.0, 8)]


def ladder(max_dm: float = 3000.0, n_trials: int | None = None) -> list:
    """Plan rows of the ladder truncated at max_dm (or at a total trial count;
    a count above the full ladder extends its last row)."""
    rows = []
    total = 0
    for k, (lo, hi, step, d) in enumerate(LADDER):
        if n_trials is not None:
            n = int(round((hi - lo) / step))
            if k == len(LADDER) - 1:
                n = n_trials - total
            n = min(n, n_trials - total)
        else:
            if lo >= max_dm:
                break
            n = int(round((min(hi, max_dm) - lo) / step))
        if n <= 0:
            break
        rows.append((lo, step, n, d))
        total += n
    return rows


def tiny(seed_offset: int = 0) -> Workload:
    """128 ch over 1000-1500 MHz, tsamp 196.608 us, 16384 samples, DM 0-199
    step 1, one pulse at DM 57.3 (FWHM 2 ms, SNR 15), widths 1..32, 6 sigma."""
    w = Workload("tiny", 128, 1000.0, 1500.0, 196.608e-6, 16384, [(0.0, 1.0, 200, 1)],
                 [1, 2, 4, 8, 16, 32], 6.0, BASE_SEED + 0 + seed_offset)
    w.pulses = [Pulse(57.3, 1.5, 2e-3, 15.0)]
    return _with_amps(w)


WIDTHS_512 = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]


def _random_pulses(rng, n, t_lo, t_hi, dm_lo=10.0, dm_hi=2000.0):
    t0s = np.linspace(t_lo, t_hi, n)
    jitter = (t0s[1] - t0s[0]) * 0.25 if n > 1 else 0.0
    out = []
    for k in range(n):
        dm = float(math.exp(rng.uniform(math.log(dm_lo), math.log(dm_hi))))
        fwhm = float(math.exp(rng.uniform(math.log(0.5e-3), math.log(20e-3))))
        snr = float(rng.uniform(6.0, 30.0))
        t0 = float(t0s[k] + rng.uniform(-jitter, jitter))
        out.append(Pulse(dm, t0, fwhm, snr))
    return out


def realistic(nsamp: int = 1 << 20, seed_offset: int = 0) -> Workload:
    """4096 ch over 1000-1500 MHz, tsamp 49.152 us, 2^20 samples, the ladder
    0-3000 (3850 trials), 20 pulses (DM log-uniform 10-2000, FWHM log-uniform
    0.5-20 ms, SNR uniform 6-30), widths 1..512, 6 sigma."""
    w = Workload("realistic", 4096, 1000.0, 1500.0, 49.152e-6, nsamp, ladder(3000.0), WIDTHS_512, 6.0,
                 BASE_SEED + 1 + seed_offset)
    rng = np.random.default_rng(w.seed)
    span = nsamp * w.tsamp
    # last segment (D=8, DM 3000) keeps about 0.866 of the data valid
    w.pulses = _random_pulses(rng, 20, 0.03 * span, 0.80 * span)
    return _with_amps(w)


def wideband(nsamp: int = 1 << 19, seed_offset: int = 0) -> Workload:
    """4096 ch over 270-1620 MHz, tsamp 196.608 us, 2^19 samples, the ladder
    truncated at DM 1500 (3350 trials), RFI in 5 % of the channels and 30
    zero-DM spikes, pulses as in the realistic workload (DM up to 1500)."""
    w = Workload("wideband", 4096, 270.0, 1620.0, 196.608e-6, nsamp, ladder(1500.0), WIDTHS_512, 6.0,
                 BASE_SEED + 2 + seed_offset)
    rng = np.random.default_rng(w.seed)
    span = nsamp * w.tsamp
    # the D=4 row's largest delay (DM 1200 at 270 MHz) is about 66 s
    w.pulses = _random_pulses(rng, 20, 0.02 * span, 0.30 * span, 10.0, 1500.0)
    chans = rng.choice(w.nchan, size=int(round(0.05 * w.nchan)), replace=False)
    for c in chans:
        for _ in range(3):
            dur = float(rng.uniform(0.1, 2.0))
            t0 = float(rng.uniform(0.0, span - dur))
            w.bursts.append((int(c), t0, dur, float(rng.uniform(20, 60)), float(rng.uniform(2, 50)),
                             float(rng.uniform(0, 2 * math.pi))))
    for _ in range(30):
        w.spikes.append((int(rng.integers(0, nsamp - 4)), int(rng.integers(1, 4)), 40.0))
    return _with_amps(w)


def small(nchan=64, nsamp=8192, segments=None, tsamp=196.608e-6, f_lo=1000.0, f_hi=1500.0, n_pulses=1,
          seed_offset=0, widths=(1, 2, 4, 8, 16, 32), threshold=6.0) -> Workload:
    """Scaled-down workloads for quick parity runs (same noise model)."""
    if segments is None:
        segments = [(0.0, 1.0, 64, 1)]
    w = Workload("small", nchan, f_lo, f_hi, tsamp, nsamp, list(segments), list(widths), threshold,
                 BASE_SEED + 100 + seed_offset)
    rng = np.random.default_rng(w.seed)
    dm_max = max(s[0] + s[1] * (s[2] - 1) for s in segments)
    span = nsamp * tsamp
    w.pulses = [Pulse(float(rng.uniform(0.2, 0.8) * max(dm_max, 1.0)), float(span * (0.1 + 0.25 * k)),
                      float(rng.uniform(1e-3, 4e-3)), float(rng.uniform(10, 20))) for k in range(n_pulses)]
    return _with_amps(w)


def stream_beams(n_beams: int = 19, seed_offset: int = 0) -> list:
    """The 19-beam streaming workload: realistic band, uneven lengths in
    2^18..2^20 samples, per-beam ladders of 1000-4000 trials."""
    rng = np.random.default_rng(BASE_SEED + 3 + seed_offset)
    beams = []
    for b in range(n_beams):
        nsamp = int(rng.integers(1 << 18, (1 << 20) + 1))
        n_trials = int(rng.integers(1000, 4001))
        w = Workload(f"beam{b}", 4096, 1000.0, 1500.0, 49.152e-6, nsamp, ladder(n_trials=n_trials), WIDTHS_512,
                     6.0, BASE_SEED + 3 + seed_offset, beam=b)
        span = nsamp * w.tsamp
        # the largest delay of a 4000-trial ladder is about 8 s
        w.pulses = _random_pulses(rng, 4, 0.05 * span, max(0.05 * span + 1.0, span - 9.0), 10.0, 1500.0)
        beams.append(_with_amps(w))
    return beams


def triage_beam(k: int, split: str = "train", nsamp: int = 1 << 17, n_pulses: int = 8, n_spikes: int = 6,
                burst_frac: float = 0.05) -> Workload:
    """Beams for training and testing the triage network: the realistic band
    and sampling, 2^17 samples (6.44 s), the ladder truncated at DM 1500
    (3350 trials), `n_pulses` pulses (DM log-uniform 10-1500, FWHM
    log-uniform 0.5-20 ms, SNR uniform 6-30) and RFI of the wideband kind:
    sinusoid bursts in 5 % of the channels and zero-DM broadband spikes of
    +40 over 1-3 samples.  `split` ("train", "val", "test") selects disjoint
    beam numbers, hence independent noise, pulses and RFI."""
    beam = {"train": 1000, "val": 300000, "test": 600000}[split] + k
    w = Workload(f"triage-{split}{k}", 4096, 1000.0, 1500.0, 49.152e-6, nsamp, ladder(1500.0), WIDTHS_512, 6.0,
                 BASE_SEED + 5, beam=beam)
    rng = np.random.default_rng([BASE_SEED + 5, beam])
    span = nsamp * w.tsamp
    # the D=8 row's largest delay (DM 1500) is about 3.45 s
    w.pulses = _random_pulses(rng, n_pulses, 0.15, span - 3.6, 10.0, 1500.0)
    chans = rng.choice(w.nchan, size=int(round(burst_frac * w.nchan)), replace=False)
    for c in chans:
        dur = float(rng.uniform(0.1, 2.0))
        t0 = float(rng.uniform(0.0, span - dur))
        w.bursts.append((int(c), t0, dur, float(rng.uniform(20, 60)), float(rng.uniform(2, 50)),
                         float(rng.uniform(0, 2 * math.pi))))
    for _ in range(n_spikes):
        w.spikes.append((int(rng.integers(0, nsamp - 4)), int(rng.integers(1, 4)), 40.0))
    return _with_amps(w)


def search_cases(n: int = 30000, seed: int = 0) -> np.ndarray:
    """Hand-shaped int32 series [trials][n] for the boxcar search alone (no
    dedispersion): noise of sigma 1000 around 10^6 plus, per trial,
      0  noise only;
      1  a +3 sigma plateau over samples 5000-24999 (one run across many
         segments and blocks) and a bright spike on it;
      2  a noise-free +6 sigma shelf over 990-1019 carrying two equal spikes
         at 1000 and 1006 (equal box sums: a tie inside one run), and spikes
         at the first and last sample and on both sides of 8192;
      3  the same shapes around 2^30 with sigma 2^20 (sums beyond 2^32);
      4  a constant (sigma 0: no candidates);
      5  negative values (noise around -10^6) with a one-sample pulse every
         2500 samples;
      6  a wide Gaussian pulse (FWHM 300) next to a narrow one.
    """
    rng = np.random.default_rng([BASE_SEED + 9, seed])
    x = np.rint(1e6 + 1000.0 * rng.standard_normal((7, n))).astype(np.int64)
    x[1, 5000:25000] += 3000
    x[1, 15000 % n] += 60000
    for i, (base, sig) in ((2, (1e6, 1000)), (3, (float(1 << 30), float(1 << 20)))):
        if i == 3:
            x[i] = np.rint(base + sig * rng.standard_normal(n)).astype(np.int64)
        x[i, 990:1020] = int(base + 6 * sig)
        x[i, [t for t in (1000, 1006) if t < n]] += int(40 * sig)
        for t in (0, 8191, 8192, n - 1):
            if t < n:
                x[i, t] += int(40 * sig)
    x[4] = 123456
    x[5] = np.rint(-1e6 + 1000.0 * rng.standard_normal(n)).astype(np.int64)
    x[5, ::2500] += 20000
    t = np.arange(n)
    x[6] += np.rint(800.0 * np.exp(-0.5 * ((t - 12000) / (300 / 2.355)) ** 2)).astype(np.int64)
    x[6, 12500 % n] += 30000
    assert np.abs(x).max() < 2 ** 31
    return x.astype(np.int32)
