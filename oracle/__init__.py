"""CPU oracle: plain C loops behind ctypes, for tests and the CPU baseline only.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use this package.  It shares no code with
the GPU library (``paper_2110_12749_amd``) and imports nothing from it.

Every function follows the definitions written at the top of ``oracle.c``
(the shift-and-sum of Section 2.3 / Algorithms 2-3 of the paper, applied per
DDplan row of Tables 2-3, plus the boxcar search the paper leaves
unspecified).  The CNN oracle lives in ``oracle/cnn.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = os.path.join(HERE, "oracle.c")


def build(verbose: bool = False) -> str:
    """Compile liboracle.so with gcc (plain -O2, OpenMP, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-std=gnu11", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class Seg(C.Structure):
    _fields_ = [("dm_lo", C.c_double), ("dm_step", C.c_double), ("n_dm", C.c_int32),
                ("downsamp", C.c_int32)]


class Cand(C.Structure):
    _fields_ = [("trial", C.c_int32), ("width", C.c_int32), ("t_peak", C.c_int64),
                ("t_first", C.c_int64), ("t_last", C.c_int64), ("snr", C.c_double)]


CAND_DTYPE = np.dtype([("trial", np.int32), ("width", np.int32), ("t_peak", np.int64),
                       ("t_first", np.int64), ("t_last", np.int64), ("snr", np.float64)])
assert CAND_DTYPE.itemsize == C.sizeof(Cand)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_num_threads.restype = C.c_int
        L.orc_num_threads.argtypes = []
        L.orc_set_threads.restype = None
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_fref.restype = C.c_double
        L.orc_fref.argtypes = [P, C.c_int32]
        L.orc_trial_dm.restype = C.c_double
        L.orc_trial_dm.argtypes = [Seg, C.c_int32]
        L.orc_delay.restype = C.c_int64
        L.orc_delay.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32]
        L.orc_delay_table.restype = None
        L.orc_delay_table.argtypes = [P, C.c_int32, C.c_double, Seg, P]
        L.orc_plan_shape.restype = None
        L.orc_plan_shape.argtypes = [C.c_int64, P, C.c_int32, C.c_double, P, C.c_int32, P, P]
        L.orc_downsample.restype = None
        L.orc_downsample.argtypes = [P, C.c_int64, C.c_int32, C.c_int32, P]
        L.orc_dedisperse_segment.restype = C.c_int
        L.orc_dedisperse_segment.argtypes = [P, C.c_int64, C.c_int32, P, C.c_double, Seg, C.c_int32,
                                             C.c_int32, C.c_int64, P]
        L.orc_dedisperse_points.restype = None
        L.orc_dedisperse_points.argtypes = [P, C.c_int64, C.c_int32, P, C.c_double, Seg, P, P,
                                            C.c_int64, P]
        L.orc_stats.restype = None
        L.orc_stats.argtypes = [P, C.c_int64, P, P]
        L.orc_search_range.restype = C.c_int64
        L.orc_search_range.argtypes = [P, C.c_int64, C.c_int64, C.c_int64, C.c_double, C.c_double, P,
                                       C.c_int32, C.c_float, C.c_int32, P, C.c_int64]
        L.orc_search_series.restype = C.c_int64
        L.orc_search_series.argtypes = [P, C.c_int64, P, C.c_int32, C.c_float, C.c_int32, P, C.c_int64]
        L.orc_search_window.restype = C.c_int64
        L.orc_search_window.argtypes = [P, C.c_int64, C.c_int64, C.c_int64, P, C.c_int32, C.c_float,
                                        C.c_int32, P, C.c_int64]
        L.orc_delay_ref.restype = C.c_int64
        L.orc_delay_ref.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int32]
        L.orc_group_dm.restype = C.c_double
        L.orc_group_dm.argtypes = [Seg, C.c_int32, C.c_int32]
        L.orc_subband_delays.restype = None
        L.orc_subband_delays.argtypes = [P, C.c_int32, C.c_int64, C.c_double, Seg, C.c_int32, C.c_int32, P, P]
        L.orc_dedisperse_subband.restype = C.c_int
        L.orc_dedisperse_subband.argtypes = [P, C.c_int64, C.c_int32, P, C.c_double, Seg, C.c_int32, C.c_int32,
                                             C.c_int32, C.c_int32, C.c_int64, P]
        L.orc_rfi_clean.restype = C.c_int64
        L.orc_rfi_clean.argtypes = [P, C.c_int64, C.c_int32, C.c_double, C.c_int64, C.c_int32, P]
        L.orc_group.restype = None
        L.orc_group.argtypes = [P, C.c_int64, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _seg(s) -> Seg:
    dm_lo, dm_step, n_dm, d = s
    return Seg(float(dm_lo), float(dm_step), int(n_dm), int(d))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timings)."""
    lib().orc_set_threads(int(n))


def fref(freqs) -> float:
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    return lib().orc_fref(_ptr(f), len(f))


def trial_dm(seg, i: int) -> float:
    return float(lib().orc_trial_dm(_seg(seg), i))


def delay(dm: float, f: float, fref_mhz: float, tsamp: float, D: int = 1) -> int:
    return int(lib().orc_delay(dm, f, fref_mhz, tsamp, D))


def delay_table(freqs, tsamp: float, seg) -> np.ndarray:
    """int64 [n_dm][nchan] delays of one plan row (dm_lo, dm_step, n_dm, D)."""
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    out = np.empty((int(seg[2]), len(f)), dtype=np.int64)
    lib().orc_delay_table(_ptr(f), len(f), tsamp, _seg(seg), _ptr(out))
    return out


def plan_shape(nsamp: int, freqs, tsamp: float, segs):
    """(max_delay[n_seg], n_out[n_seg]) as int64 arrays."""
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    arr = (Seg * len(segs))(*[_seg(s) for s in segs])
    md = np.empty(len(segs), np.int64)
    no = np.empty(len(segs), np.int64)
    lib().orc_plan_shape(nsamp, _ptr(f), len(f), tsamp, arr, len(segs), _ptr(md), _ptr(no))
    return md, no


def downsample(X: np.ndarray, D: int) -> np.ndarray:
    """uint32 [nchan][nsamp // D] channel-major sums of D samples."""
    X = np.ascontiguousarray(X, dtype=np.uint8)
    nsamp, nchan = X.shape
    Y = np.empty((nchan, nsamp // D), np.uint32)
    lib().orc_downsample(_ptr(X), nsamp, nchan, D, _ptr(Y))
    return Y


def dedisperse_segment(X: np.ndarray, freqs, tsamp: float, seg, trials=None) -> np.ndarray:
    """int32 [n_trials][n_out] for trials [i0, i1) of one segment (all by default)."""
    X = np.ascontiguousarray(X, dtype=np.uint8)
    nsamp, nchan = X.shape
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    _, n_out = plan_shape(nsamp, f, tsamp, [seg])
    n_out = int(n_out[0])
    if n_out <= 0:
        raise ValueError("input shorter than the segment's maximum delay")
    i0, i1 = (0, int(seg[2])) if trials is None else trials
    out = np.empty((i1 - i0, n_out), np.int32)
    rc = lib().orc_dedisperse_segment(_ptr(X), nsamp, nchan, _ptr(f), tsamp, _seg(seg), i0, i1, n_out,
                                      _ptr(out))
    if rc:
        raise MemoryError("oracle allocation failed")
    return out


def dedisperse(X: np.ndarray, freqs, tsamp: float, segs):
    """List of per-segment int32 [n_dm][n_out] arrays for a whole plan."""
    return [dedisperse_segment(X, freqs, tsamp, s) for s in segs]


def dedisperse_points(X: np.ndarray, freqs, tsamp: float, seg, trial, t) -> np.ndarray:
    """int64 values of individual outputs (trial[k], t[k]) of one segment."""
    X = np.ascontiguousarray(X, dtype=np.uint8)
    nsamp, nchan = X.shape
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    tr = np.ascontiguousarray(trial, dtype=np.int32)
    tt = np.ascontiguousarray(t, dtype=np.int64)
    out = np.empty(len(tr), np.int64)
    lib().orc_dedisperse_points(_ptr(X), nsamp, nchan, _ptr(f), tsamp, _seg(seg), _ptr(tr), _ptr(tt),
                                len(tr), _ptr(out))
    return out


def group_dm(seg, group: int, g: int) -> float:
    """Nominal DM of trial group g of a row in sub-band dedispersion."""
    return float(lib().orc_group_dm(_seg(seg), int(group), int(g)))


def subband_delays(freqs, nsamp: int, tsamp: float, seg, n_sub: int, group: int):
    """(int64 [n_dm][nchan] composite delays d2(i, b(c)) + d1(g(i), c), n_out) of a row."""
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    d = np.empty((int(seg[2]), len(f)), np.int64)
    n_out = C.c_int64()
    lib().orc_subband_delays(_ptr(f), len(f), nsamp, tsamp, _seg(seg), int(n_sub), int(group), _ptr(d),
                             C.byref(n_out))
    return d, int(n_out.value)


def dedisperse_subband(X: np.ndarray, freqs, tsamp: float, seg, n_sub: int, group: int, trials=None) -> np.ndarray:
    """int32 [n_trials][n_out] of sub-band dedispersion, trials [i0, i1) of one row."""
    X = np.ascontiguousarray(X, dtype=np.uint8)
    nsamp, nchan = X.shape
    f = np.ascontiguousarray(freqs, dtype=np.float64)
    _, n_out = subband_delays(f, nsamp, tsamp, seg, n_sub, group)
    if n_out <= 0:
        raise ValueError("input shorter than the row's largest composite delay")
    i0, i1 = (0, int(seg[2])) if trials is None else trials
    out = np.empty((i1 - i0, n_out), np.int32)
    rc = lib().orc_dedisperse_subband(_ptr(X), nsamp, nchan, _ptr(f), tsamp, _seg(seg), int(n_sub), int(group), i0,
                                      i1, n_out, _ptr(out))
    if rc:
        raise MemoryError("oracle allocation failed")
    return out


def rfi_clean(X: np.ndarray, clip_sigma: float = 0.0, block: int = 2048, zero_dm: bool = False):
    """(cleaned uint8 [nsamp][nchan], flagged spectra): clip of outlying
    zero-DM spectra per block, then the zero-DM filter (oracle.c)."""
    X = np.ascontiguousarray(X, dtype=np.uint8)
    out = np.empty_like(X)
    n = lib().orc_rfi_clean(_ptr(X), X.shape[0], X.shape[1], float(clip_sigma), int(block), int(bool(zero_dm)),
                            _ptr(out))
    return out, int(n)


def stats(x: np.ndarray):
    x = np.ascontiguousarray(x, dtype=np.int32)
    mu = C.c_double()
    sg = C.c_double()
    lib().orc_stats(_ptr(x), len(x), C.byref(mu), C.byref(sg))
    return mu.value, sg.value


def _cands(buf: np.ndarray, n: int) -> np.ndarray:
    return buf[:n].copy()


def search_series(x: np.ndarray, widths, threshold: float, trial: int = 0) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.int32)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    cap = 1024
    while True:
        buf = np.zeros(cap, CAND_DTYPE)
        n = lib().orc_search_series(_ptr(x), len(x), _ptr(w), len(w), threshold, trial, _ptr(buf), cap)
        if n <= cap:
            return _cands(buf, n)
        cap = int(n)


def search_range(x, e0, e1, mu, sigma, widths, threshold, trial=0) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.int32)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    cap = 1024
    while True:
        buf = np.zeros(cap, CAND_DTYPE)
        n = lib().orc_search_range(_ptr(x), len(x), e0, e1, mu, sigma, _ptr(w), len(w), threshold, trial,
                                   _ptr(buf), cap)
        if n <= cap:
            return _cands(buf, n)
        cap = int(n)


def search_window(x, w0, w1, widths, threshold, trial=0) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.int32)
    w = np.ascontiguousarray(widths, dtype=np.int32)
    cap = 1024
    while True:
        buf = np.zeros(cap, CAND_DTYPE)
        n = lib().orc_search_window(_ptr(x), len(x), w0, w1, _ptr(w), len(w), threshold, trial, _ptr(buf),
                                    cap)
        if n <= cap:
            return _cands(buf, n)
        cap = int(n)


def search(dmt_segments, widths, threshold: float):
    """Candidates of a whole plan: list over segments of per-trial searches, concatenated.

    Returns a structured array with an extra ``seg`` column, sorted by
    (seg, trial, t_peak)."""
    rows = []
    for s, arr in enumerate(dmt_segments):
        for i in range(arr.shape[0]):
            c = search_series(arr[i], widths, threshold, trial=i)
            if len(c):
                rows.append((s, c))
    dt = np.dtype([("seg", np.int32)] + [(n, CAND_DTYPE[n]) for n in CAND_DTYPE.names])
    if not rows:
        return np.zeros(0, dt)
    out = np.zeros(sum(len(c) for _, c in rows), dt)
    k = 0
    for s, c in rows:
        out["seg"][k:k + len(c)] = s
        for n in CAND_DTYPE.names:
            out[n][k:k + len(c)] = c[n]
        k += len(c)
    order = np.lexsort((out["t_peak"], out["trial"], out["seg"]))
    return out[order]


def group(cands: np.ndarray) -> np.ndarray:
    """Representative index per candidate (friends-of-friends, one segment)."""
    c = np.ascontiguousarray(cands[list(CAND_DTYPE.names)].astype(CAND_DTYPE))
    g = np.empty(len(c), np.int64)
    lib().orc_group(_ptr(c), len(c), _ptr(g))
    return g
