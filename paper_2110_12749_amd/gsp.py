"""Python binding of libgsp.so (include/gsp.h): argument marshalling only.

Every step of the path runs in the library's HIP kernels; torch supplies
device memory and streams.  Importing this module fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
# torch first: it ships its own HIP runtime (same soname as ROCm's), and the
# library must bind to that one; loading the library first would bring a
# second HIP/HSA runtime into the process.
import torch  # noqa: F401

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsp.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
_L = C.CDLL(LIB_PATH)

GSP_OK, GSP_EINVAL, GSP_ETOOSHORT, GSP_EOVERFLOW, GSP_ECAPACITY, GSP_ENOMEM, GSP_EDEVICE, GSP_EAGAIN = (
    0, -1, -2, -3, -4, -5, -6, -7)
MAX_SEG = 16


class Segment(C.Structure):
    _fields_ = [("dm_lo", C.c_double), ("dm_step", C.c_double), ("n_dm", C.c_int32), ("downsamp", C.c_int32)]


class DmtDesc(C.Structure):
    _fields_ = [("nsamp", C.c_int64), ("nchan", C.c_int32), ("n_seg", C.c_int32), ("tsamp", C.c_double),
                ("fref_mhz", C.c_double), ("seg", Segment * MAX_SEG), ("max_delay", C.c_int64 * MAX_SEG),
                ("n_out", C.c_int64 * MAX_SEG), ("offset", C.c_int64 * MAX_SEG), ("trial0", C.c_int32 * MAX_SEG),
                ("n_trials", C.c_int32), ("kind", C.c_int32), ("total", C.c_int64)]


class Candidate(C.Structure):
    _fields_ = [("seg", C.c_int32), ("dm_index", C.c_int32), ("dm", C.c_double), ("t_peak", C.c_int64),
                ("t_first", C.c_int64), ("t_last", C.c_int64), ("width", C.c_int32), ("snr", C.c_float),
                ("time_s", C.c_double)]


CAND_DTYPE = np.dtype([("seg", np.int32), ("dm_index", np.int32), ("dm", np.float64), ("t_peak", np.int64),
                       ("t_first", np.int64), ("t_last", np.int64), ("width", np.int32), ("snr", np.float32),
                       ("time_s", np.float64)])
assert CAND_DTYPE.itemsize == C.sizeof(Candidate)

P = C.c_void_p
_L.gsp_create.restype = C.c_int
_L.gsp_create.argtypes = [C.c_int, C.POINTER(P)]
_L.gsp_destroy.restype = None
_L.gsp_destroy.argtypes = [P]
_L.gsp_strerror.restype = C.c_char_p
_L.gsp_strerror.argtypes = [C.c_int]
_L.gsp_last_error.restype = C.c_char_p
_L.gsp_last_error.argtypes = [P]
_L.gsp_plan_shape.restype = C.c_int
_L.gsp_plan_shape.argtypes = [C.c_int64, C.c_int32, P, C.c_double, P, C.c_int32, C.POINTER(DmtDesc)]
_L.gsp_delay_table.restype = C.c_int
_L.gsp_delay_table.argtypes = [C.POINTER(DmtDesc), P, C.c_int32, P]
_L.gsp_dedisperse.restype = C.c_int
_L.gsp_dedisperse.argtypes = [P, P, P, C.POINTER(DmtDesc), P, P]
_L.gsp_subband_plan_shape.restype = C.c_int
_L.gsp_subband_plan_shape.argtypes = [C.c_int64, C.c_int32, P, C.c_double, P, C.c_int32, P, P, C.POINTER(DmtDesc)]
_L.gsp_dedisperse_subband.restype = C.c_int
_L.gsp_dedisperse_subband.argtypes = [P, P, P, C.POINTER(DmtDesc), P, P, P, P]
_L.gsp_rank_groups.restype = C.c_int
_L.gsp_rank_groups.argtypes = [P, C.c_int64, P, C.POINTER(DmtDesc), P, C.c_int64, C.POINTER(C.c_int64)]
for _n, _a in (("gsp_store_create", [P]), ("gsp_store_add_file", [P, C.c_char_p, C.c_int32, C.c_int32, C.c_int64,
                                                                   C.c_double, C.c_double, C.c_double, P]),
               ("gsp_store_add_groups", [P, C.c_int64, C.c_int64, P, C.c_int64, P]),
               ("gsp_store_add_pulsar", [P, C.c_char_p, C.c_double, P]),
               ("gsp_store_match_pulsars", [P, C.c_int64, C.c_double, C.c_int32, P]),
               ("gsp_store_add_picture", [P, C.c_int64, C.c_char_p]),
               ("gsp_store_query", [P, C.c_int32, C.c_double, C.c_double, P, C.c_int64, P]),
               ("gsp_store_count", [P, C.c_int32, P]), ("gsp_store_save", [P, C.c_char_p]),
               ("gsp_store_load", [P, C.c_char_p])):
    getattr(_L, _n).restype = C.c_int
    getattr(_L, _n).argtypes = _a
_L.gsp_store_destroy.restype = None
_L.gsp_store_destroy.argtypes = [P]
_L.gsp_store_last_error.restype = C.c_char_p
_L.gsp_store_last_error.argtypes = [P]
_L.gsp_rfi_clean.restype = C.c_int
_L.gsp_rfi_clean.argtypes = [P, P, C.c_int64, C.c_int32, C.c_double, C.c_int64, C.c_int32, P, C.POINTER(C.c_int64), P]
_L.gsp_trial_stats.restype = C.c_int
_L.gsp_trial_stats.argtypes = [P, P, C.POINTER(DmtDesc), P, P, P]
_L.gsp_single_pulse_search_noalloc.restype = C.c_int
_L.gsp_single_pulse_search_noalloc.argtypes = [P, P, C.POINTER(DmtDesc), P, C.c_int32, C.c_float, P, C.c_int64,
                                               C.POINTER(C.c_int64), P]
_L.gsp_single_pulse_search.restype = C.c_int
_L.gsp_single_pulse_search.argtypes = [P, P, C.POINTER(DmtDesc), P, C.c_int32, C.c_float, P, C.c_int64,
                                       C.POINTER(C.c_int64), P]
class Shape(C.Structure):
    _fields_ = [("groups", C.c_int32), ("tpw", C.c_int32), ("waves", C.c_int32), ("chunk", C.c_int32),
                ("kind", C.c_int32)]


_L.gsp_autotune.restype = C.c_int
_L.gsp_autotune.argtypes = [P, P, P, C.POINTER(DmtDesc), P, C.c_int32, P]
_L.gsp_row_shape.restype = C.c_int
_L.gsp_row_shape.argtypes = [P, P, C.POINTER(DmtDesc), C.c_int32, C.POINTER(Shape)]
_L.gsp_set_row_shape.restype = C.c_int
_L.gsp_set_row_shape.argtypes = [P, P, C.POINTER(DmtDesc), C.c_int32, C.POINTER(Shape)]
_L.gsp_tuning_save.restype = C.c_int
_L.gsp_tuning_save.argtypes = [P, C.c_char_p]
_L.gsp_tuning_load.restype = C.c_int
_L.gsp_tuning_load.argtypes = [P, C.c_char_p]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double), ("work", C.c_double)]


_L.gsp_profile_enable.restype = C.c_int
_L.gsp_profile_enable.argtypes = [P, C.c_int]
_L.gsp_profile_read.restype = C.c_int
_L.gsp_profile_read.argtypes = [P, P, C.c_int32, C.POINTER(C.c_int32), C.c_int]
_L.gsp_group_candidates.restype = C.c_int
_L.gsp_group_candidates.argtypes = [P, C.c_int64, P, C.POINTER(C.c_int64)]


class GspError(RuntimeError):
    def __init__(self, status: int, msg: str = ""):
        self.status = status
        text = _L.gsp_strerror(status).decode()
        super().__init__(f"{text} ({status})" + (f": {msg}" if msg else ""))


def lib():
    return _L


def _check(status: int, ctx=None):
    if status != GSP_OK:
        msg = _L.gsp_last_error(ctx).decode() if ctx else ""
        raise GspError(status, msg)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _segs(segments):
    arr = (Segment * len(segments))()
    for k, (lo, st, n, d) in enumerate(segments):
        arr[k] = Segment(float(lo), float(st), int(n), int(d))
    return arr


def _stream_handle(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def plan_shape(nsamp: int, freqs, tsamp: float, segments) -> DmtDesc:
    """Validate a plan and return its output descriptor (gsp_plan_shape)."""
    f = _f64(freqs)
    d = DmtDesc()
    segs = _segs(segments)
    _check(_L.gsp_plan_shape(int(nsamp), len(f), f.ctypes.data, float(tsamp), C.addressof(segs), len(segments),
                             C.byref(d)))
    return d


def _row_ints(v, n_seg, what):
    a = np.full(n_seg, int(v), np.int32) if np.isscalar(v) else np.ascontiguousarray(v, dtype=np.int32)
    assert a.shape == (n_seg,), what
    return a


def subband_plan_shape(nsamp: int, freqs, tsamp: float, segments, n_sub, group) -> DmtDesc:
    """Descriptor of a sub-band plan (gsp_subband_plan_shape); n_sub and
    group: one value for every row, or one per row."""
    f = _f64(freqs)
    d = DmtDesc()
    segs = _segs(segments)
    ns = _row_ints(n_sub, len(segments), "n_sub")
    gr = _row_ints(group, len(segments), "group")
    _check(_L.gsp_subband_plan_shape(int(nsamp), len(f), f.ctypes.data, float(tsamp), C.addressof(segs),
                                     len(segments), ns.ctypes.data, gr.ctypes.data, C.byref(d)))
    return d


def delay_table(desc: DmtDesc, freqs, seg: int) -> np.ndarray:
    f = _f64(freqs)
    out = np.empty((desc.seg[seg].n_dm, desc.nchan), np.int32)
    _check(_L.gsp_delay_table(C.byref(desc), f.ctypes.data, int(seg), out.ctypes.data))
    return out


def segment_views(desc: DmtDesc, dmt):
    """Per-row [n_dm][n_out] views of a flat DM-time array."""
    return [dmt[desc.offset[s]: desc.offset[s] + desc.seg[s].n_dm * desc.n_out[s]].view(desc.seg[s].n_dm,
                                                                                         desc.n_out[s])
            for s in range(desc.n_seg)]


def group_candidates(cands: np.ndarray):
    """(representative index per candidate, number of groups)."""
    c = np.ascontiguousarray(cands, dtype=CAND_DTYPE)
    rep = np.empty(len(c), np.int64)
    ng = C.c_int64()
    _check(_L.gsp_group_candidates(c.ctypes.data, len(c), rep.ctypes.data, C.byref(ng)))
    return rep, int(ng.value)


GROUP_DTYPE = np.dtype([("rep", np.int64), ("seg", np.int32), ("rank", np.int32), ("n_events", np.int32),
                        ("n_trials", np.int32), ("dm_min", np.float64), ("dm_max", np.float64),
                        ("dm_peak", np.float64), ("snr_max", np.float32), ("snr_lo", np.float32),
                        ("snr_hi", np.float32), ("reserved", np.int32), ("time_s", np.float64),
                        ("width_s", np.float64), ("start_s", np.float64), ("duration_s", np.float64)])
STORE_CAND_DTYPE = np.dtype([("id", np.int64), ("file_id", np.int64), ("g", GROUP_DTYPE)])
T_FITS_INFO, T_SINGLEPULSE_GROUPS, T_SINGLEPULSE_CANDIDATES, T_PULSAR, T_FILE_PULSAR, T_SINGLEPULSE_PIC = range(6)


def rank_groups(cands: np.ndarray, rep, desc: DmtDesc) -> np.ndarray:
    """Ranked groups (GROUP_DTYPE), one per group of gsp_group_candidates."""
    c = np.ascontiguousarray(cands, dtype=CAND_DTYPE)
    r = np.ascontiguousarray(rep, dtype=np.int64)
    cap = max(1, len(np.unique(r))) if len(r) else 1
    out = np.zeros(cap, GROUP_DTYPE)
    n = C.c_int64()
    _check(_L.gsp_rank_groups(c.ctypes.data, len(c), r.ctypes.data, C.byref(desc), out.ctypes.data, cap,
                              C.byref(n)))
    return out[: n.value]


class Store:
    """Candidate store with the paper's six tables (gsp_store_*)."""

    def __init__(self):
        self.h = P()
        _check(_L.gsp_store_create(C.byref(self.h)))

    def _check(self, st):
        if st != GSP_OK:
            raise GspError(st, _L.gsp_store_last_error(self.h).decode())

    def close(self):
        if self.h:
            _L.gsp_store_destroy(self.h)
            self.h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_file(self, name, beam, nchan, nsamp, tsamp, f_lo, f_hi) -> int:
        i = C.c_int64()
        self._check(_L.gsp_store_add_file(self.h, name.encode(), int(beam), int(nchan), int(nsamp), float(tsamp),
                                          float(f_lo), float(f_hi), C.byref(i)))
        return int(i.value)

    def add_groups(self, file_id, n_candidates, groups) -> int:
        g = np.ascontiguousarray(groups, dtype=GROUP_DTYPE)
        i = C.c_int64()
        self._check(_L.gsp_store_add_groups(self.h, int(file_id), int(n_candidates), g.ctypes.data, len(g),
                                            C.byref(i)))
        return int(i.value)

    def add_pulsar(self, name, dm) -> int:
        i = C.c_int64()
        self._check(_L.gsp_store_add_pulsar(self.h, name.encode(), float(dm), C.byref(i)))
        return int(i.value)

    def match_pulsars(self, file_id, dm_tol, min_rank=3) -> int:
        n = C.c_int64()
        self._check(_L.gsp_store_match_pulsars(self.h, int(file_id), float(dm_tol), int(min_rank), C.byref(n)))
        return int(n.value)

    def add_picture(self, cand_id, path):
        self._check(_L.gsp_store_add_picture(self.h, int(cand_id), path.encode()))

    def query(self, min_rank=1, dm_lo=-np.inf, dm_hi=np.inf) -> np.ndarray:
        n = C.c_int64()
        st = _L.gsp_store_query(self.h, int(min_rank), float(dm_lo), float(dm_hi), None, 0, C.byref(n))
        if st not in (GSP_OK, GSP_ECAPACITY):
            self._check(st)
        out = np.zeros(max(1, n.value), STORE_CAND_DTYPE)
        self._check(_L.gsp_store_query(self.h, int(min_rank), float(dm_lo), float(dm_hi), out.ctypes.data,
                                       len(out), C.byref(n)))
        return out[: n.value]

    def count(self, table) -> int:
        n = C.c_int64()
        self._check(_L.gsp_store_count(self.h, int(table), C.byref(n)))
        return int(n.value)

    def save(self, path):
        self._check(_L.gsp_store_save(self.h, str(path).encode()))

    def load(self, path):
        self._check(_L.gsp_store_load(self.h, str(path).encode()))


class Context:
    """A library context (gsp_create) bound to one device."""

    def __init__(self, device: int = 0):
        h = P()
        _check(_L.gsp_create(int(device), C.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            _L.gsp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, fb, freqs, desc: DmtDesc, out=None, n_reps: int = 2, stream=None):
        """Time every candidate launch shape per plan row; keep the fastest."""
        import torch
        if out is None:
            out = torch.empty(desc.total, dtype=torch.int32, device=fb.device)
        f = _f64(freqs)
        _check(_L.gsp_autotune(self.h, C.c_void_p(fb.data_ptr()), f.ctypes.data, C.byref(desc),
                               C.c_void_p(out.data_ptr()), int(n_reps), _stream_handle(stream)), self.h)
        return [self.row_shape(freqs, desc, s) for s in range(desc.n_seg)]

    def row_shape(self, freqs, desc: DmtDesc, seg: int) -> tuple:
        f = _f64(freqs)
        sh = Shape()
        _check(_L.gsp_row_shape(self.h, f.ctypes.data, C.byref(desc), int(seg), C.byref(sh)), self.h)
        return (sh.groups, sh.tpw, sh.waves, sh.chunk, sh.kind)

    def set_row_shape(self, freqs, desc: DmtDesc, seg: int, groups: int, tpw: int, waves: int, chunk: int,
                      kind: int = 0):
        f = _f64(freqs)
        sh = Shape(int(groups), int(tpw), int(waves), int(chunk), int(kind))
        _check(_L.gsp_set_row_shape(self.h, f.ctypes.data, C.byref(desc), int(seg), C.byref(sh)), self.h)

    def tuning_save(self, path: str):
        _check(_L.gsp_tuning_save(self.h, path.encode()), self.h)

    def tuning_load(self, path: str):
        _check(_L.gsp_tuning_load(self.h, path.encode()), self.h)

    def profile_enable(self, on: bool = True):
        _check(_L.gsp_profile_enable(self.h, int(bool(on))), self.h)

    def profile_read(self, reset: bool = True) -> dict:
        """{kernel name: (launches, total_ms, work)} of the timed launches."""
        cap = 32
        arr = (KernelStat * cap)()
        n = C.c_int32()
        _check(_L.gsp_profile_read(self.h, C.addressof(arr), cap, C.byref(n), int(bool(reset))), self.h)
        return {arr[k].name.decode(): (int(arr[k].launches), float(arr[k].total_ms), float(arr[k].work))
                for k in range(min(n.value, cap))}

    def dedisperse(self, fb, freqs, desc: DmtDesc, out=None, stream=None):
        """fb: torch uint8 [nsamp][nchan] on the device.  Returns int32 [total]."""
        import torch
        assert fb.dtype == torch.uint8 and fb.is_cuda and fb.is_contiguous()
        assert tuple(fb.shape) == (desc.nsamp, desc.nchan)
        if out is None:
            out = torch.empty(desc.total, dtype=torch.int32, device=fb.device)
        assert out.dtype == torch.int32 and out.is_contiguous() and out.numel() >= desc.total
        f = _f64(freqs)
        _check(_L.gsp_dedisperse(self.h, C.c_void_p(fb.data_ptr()), f.ctypes.data, C.byref(desc),
                                 C.c_void_p(out.data_ptr()), _stream_handle(stream)), self.h)
        return out

    def dedisperse_subband(self, fb, freqs, desc: DmtDesc, n_sub, group, out=None, stream=None):
        """Sub-band dedispersion (desc from subband_plan_shape with the same
        n_sub and group).  Returns int32 [total]."""
        import torch
        assert fb.dtype == torch.uint8 and fb.is_cuda and fb.is_contiguous()
        assert tuple(fb.shape) == (desc.nsamp, desc.nchan)
        if out is None:
            out = torch.empty(desc.total, dtype=torch.int32, device=fb.device)
        assert out.dtype == torch.int32 and out.is_contiguous() and out.numel() >= desc.total
        f = _f64(freqs)
        ns = _row_ints(n_sub, desc.n_seg, "n_sub")
        gr = _row_ints(group, desc.n_seg, "group")
        _check(_L.gsp_dedisperse_subband(self.h, C.c_void_p(fb.data_ptr()), f.ctypes.data, C.byref(desc),
                                         ns.ctypes.data, gr.ctypes.data, C.c_void_p(out.data_ptr()),
                                         _stream_handle(stream)), self.h)
        return out

    def trial_stats(self, dmt, desc: DmtDesc, stream=None):
        mu = np.empty(desc.n_trials, np.float64)
        sg = np.empty(desc.n_trials, np.float64)
        _check(_L.gsp_trial_stats(self.h, C.c_void_p(dmt.data_ptr()), C.byref(desc), mu.ctypes.data, sg.ctypes.data,
                                  _stream_handle(stream)), self.h)
        return mu, sg

    def rfi_clean(self, fb, clip_sigma: float = 0.0, block: int = 2048, zero_dm: bool = False, out=None,
                  count: bool = True, stream=None):
        """RFI mitigation of a device uint8 [nsamp][nchan] filterbank (in
        place when out is fb).  Returns (out, spectra replaced by the clip,
        or None with count=False: then the call stays asynchronous)."""
        import torch
        assert fb.is_cuda and fb.dtype == torch.uint8 and fb.dim() == 2 and fb.is_contiguous()
        if out is None:
            out = torch.empty_like(fb)
        n = C.c_int64()
        _check(_L.gsp_rfi_clean(self.h, C.c_void_p(fb.data_ptr()), fb.shape[0], fb.shape[1], float(clip_sigma),
                                int(block), int(bool(zero_dm)), C.c_void_p(out.data_ptr()),
                                C.byref(n) if count else None, _stream_handle(stream)), self.h)
        return out, (int(n.value) if count else None)

    def single_pulse_search(self, dmt, desc: DmtDesc, widths, threshold: float, capacity: int = 1 << 16,
                            stream=None) -> np.ndarray:
        w = np.ascontiguousarray(widths, dtype=np.int32)
        # start from the largest count seen on this context, so that a
        # repeated search of similar data does not run twice
        capacity = max(capacity, getattr(self, "_cap_hint", 0))
        while True:
            out = np.empty(capacity, CAND_DTYPE)
            n = C.c_int64()
            st = _L.gsp_single_pulse_search(self.h, C.c_void_p(dmt.data_ptr()), C.byref(desc), w.ctypes.data, len(w),
                                            float(threshold), out.ctypes.data, capacity, C.byref(n),
                                            _stream_handle(stream))
            if st == GSP_ECAPACITY:
                capacity = int(n.value)
                self._cap_hint = capacity
                continue
            _check(st, self.h)
            return out[: n.value]

    def single_pulse_search_noalloc(self, dmt, desc: DmtDesc, widths, threshold: float, capacity: int = 1 << 16,
                                    stream=None) -> np.ndarray:
        """The same search with no device allocation (the library's static
        scratch; the candidate array doubles as host workspace)."""
        w = np.ascontiguousarray(widths, dtype=np.int32)
        while True:
            out = np.empty(capacity, CAND_DTYPE)
            n = C.c_int64()
            st = _L.gsp_single_pulse_search_noalloc(self.h, C.c_void_p(dmt.data_ptr()), C.byref(desc),
                                                    w.ctypes.data, len(w), float(threshold), out.ctypes.data,
                                                    capacity, C.byref(n), _stream_handle(stream))
            if st == GSP_ECAPACITY and n.value > capacity:
                capacity = int(n.value)
                continue
            _check(st, self.h)
            return out[: n.value]


_default = {}


def context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def dedisperse(fb, freqs, tsamp: float, segments, ctx: Context | None = None, stream=None):
    """dedisperse(filterbank, freqs, tsamp, dm_plan) -> (int32 DM-time array, descriptor)."""
    desc = plan_shape(fb.shape[0], freqs, tsamp, segments)
    ctx = ctx or context(fb.device.index or 0)
    return ctx.dedisperse(fb, freqs, desc, stream=stream), desc


def single_pulse_search(dmt, desc: DmtDesc, widths, threshold: float, ctx: Context | None = None, stream=None):
    """single_pulse_search(dmt, widths, threshold) -> candidate array (CAND_DTYPE)."""
    ctx = ctx or context(dmt.device.index or 0)
    return ctx.single_pulse_search(dmt, desc, widths, threshold, stream=stream)


def trial_stats(dmt, desc: DmtDesc, ctx: Context | None = None, stream=None):
    ctx = ctx or context(dmt.device.index or 0)
    return ctx.trial_stats(dmt, desc, stream=stream)


# ---------------------------------------------------------------------------
# streaming (continuous batching of beams arriving in blocks)
# ---------------------------------------------------------------------------
class StreamCandidate(C.Structure):
    _fields_ = [("beam", C.c_int32), ("block", C.c_int32), ("c", Candidate), ("score", C.c_float),
                ("reserved", C.c_int32)]


class StreamStats(C.Structure):
    _fields_ = [("lat_p50_s", C.c_double), ("lat_p99_s", C.c_double), ("lat_max_s", C.c_double),
                ("blocks", C.c_int64), ("steps", C.c_int64), ("busy_s", C.c_double), ("mem_used", C.c_int64),
                ("mem_budget", C.c_int64), ("beams_active", C.c_int32), ("beams_queued", C.c_int32),
                ("blocks_pending", C.c_int64), ("triage_scored", C.c_int64), ("triage_rejected", C.c_int64),
                ("triage_s", C.c_double), ("search_repeats", C.c_int64)]


STREAM_CAND_DTYPE = np.dtype([("beam", np.int32), ("block", np.int32)] + [(n, CAND_DTYPE[n]) for n in CAND_DTYPE.names]
                             + [("score", np.float32), ("reserved", np.int32)])
assert STREAM_CAND_DTYPE.itemsize == C.sizeof(StreamCandidate)

_L.gsp_stream_create.restype = C.c_int
_L.gsp_stream_create.argtypes = [P, C.c_int64, C.c_int32, P, C.c_int32, C.c_float, C.POINTER(P)]
_L.gsp_stream_destroy.restype = None
_L.gsp_stream_destroy.argtypes = [P]
_L.gsp_stream_last_error.restype = C.c_char_p
_L.gsp_stream_last_error.argtypes = [P]
_L.gsp_stream_open_beam.restype = C.c_int
_L.gsp_stream_open_beam.argtypes = [P, C.c_int32, P, C.c_double, P, C.c_int32, C.POINTER(C.c_int32)]
_L.gsp_stream_push.restype = C.c_int
_L.gsp_stream_push.argtypes = [P, C.c_int32, P, C.c_int64]
_L.gsp_stream_close_beam.restype = C.c_int
_L.gsp_stream_close_beam.argtypes = [P, C.c_int32]
_L.gsp_stream_step.restype = C.c_int
_L.gsp_stream_step.argtypes = [P, C.POINTER(C.c_int64)]
for _n in ("gsp_stream_start", "gsp_stream_stop", "gsp_stream_flush"):
    getattr(_L, _n).restype = C.c_int
    getattr(_L, _n).argtypes = [P]
_L.gsp_stream_poll.restype = C.c_int
_L.gsp_stream_poll.argtypes = [P, P, C.c_int64, C.POINTER(C.c_int64)]
_L.gsp_stream_report.restype = C.c_int
_L.gsp_stream_report.argtypes = [P, C.POINTER(StreamStats)]
_L.gsp_stream_window.restype = C.c_int
_L.gsp_stream_window.argtypes = [P, C.c_int32, C.c_int32, P, C.c_int64, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
_L.gsp_stream_snapshot.restype = C.c_int
_L.gsp_stream_snapshot.argtypes = [P, C.c_int32, P, C.c_int64, C.POINTER(C.c_int64)]
_L.gsp_stream_restore.restype = C.c_int
_L.gsp_stream_restore.argtypes = [P, C.c_int32, P, C.c_int64]
_L.gsp_stream_set_graph.restype = C.c_int
_L.gsp_stream_set_graph.argtypes = [P, C.c_int]
_L.gsp_stream_set_fragment_capacity.restype = C.c_int
_L.gsp_stream_set_fragment_capacity.argtypes = [P, C.c_int64]
_L.gsp_stream_set_triage.restype = C.c_int
_L.gsp_stream_set_triage.argtypes = [P, P, C.c_float]


class Stream:
    """A streaming engine (gsp_stream_create) on a context."""

    def __init__(self, ctx: Context, mem_budget: int, block_nsamp: int, widths, threshold: float):
        w = np.ascontiguousarray(widths, dtype=np.int32)
        h = P()
        _check(_L.gsp_stream_create(ctx.h, int(mem_budget), int(block_nsamp), w.ctypes.data, len(w),
                                    float(threshold), C.byref(h)), ctx.h)
        self.h = h
        self.ctx = ctx
        self.block = int(block_nsamp)
        self.nchan = {}

    def _check(self, st):
        if st != GSP_OK:
            raise GspError(st, _L.gsp_stream_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            _L.gsp_stream_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def open_beam(self, nchan: int, freqs, tsamp: float, segments):
        """Returns (beam_id, admitted)."""
        f = _f64(freqs)
        segs = _segs(segments)
        bid = C.c_int32()
        st = _L.gsp_stream_open_beam(self.h, int(nchan), f.ctypes.data, float(tsamp), C.addressof(segs),
                                     len(segments), C.byref(bid))
        if st not in (GSP_OK, GSP_EAGAIN):
            self._check(st)
        self.nchan[bid.value] = int(nchan)
        return bid.value, st == GSP_OK

    def push(self, beam: int, block: np.ndarray):
        b = np.ascontiguousarray(block, dtype=np.uint8)
        assert b.ndim == 2 and b.shape[1] == self.nchan[beam]
        self._check(_L.gsp_stream_push(self.h, int(beam), b.ctypes.data, b.shape[0]))

    def close_beam(self, beam: int):
        self._check(_L.gsp_stream_close_beam(self.h, int(beam)))

    def step(self) -> int:
        n = C.c_int64()
        self._check(_L.gsp_stream_step(self.h, C.byref(n)))
        return n.value

    def start(self):
        self._check(_L.gsp_stream_start(self.h))

    def stop(self):
        self._check(_L.gsp_stream_stop(self.h))

    def flush(self):
        self._check(_L.gsp_stream_flush(self.h))

    def set_graph(self, on: bool):
        self._check(_L.gsp_stream_set_graph(self.h, int(bool(on))))

    def set_fragment_capacity(self, cap: int):
        self._check(_L.gsp_stream_set_fragment_capacity(self.h, int(cap)))

    def set_triage(self, cnn, threshold: float = 0.0):
        """Attach a trained Cnn (None: the plain search) scoring each step's candidates."""
        self._triage = cnn  # keep the network alive while attached
        self._check(_L.gsp_stream_set_triage(self.h, cnn.h if cnn is not None else None, float(threshold)))

    def poll(self) -> np.ndarray:
        rows = []
        while True:
            buf = np.zeros(4096, STREAM_CAND_DTYPE)
            n = C.c_int64()
            self._check(_L.gsp_stream_poll(self.h, buf.ctypes.data, len(buf), C.byref(n)))
            rows.append(buf[: n.value])
            if n.value < len(buf):
                break
        return np.concatenate(rows)

    def report(self) -> dict:
        r = StreamStats()
        self._check(_L.gsp_stream_report(self.h, C.byref(r)))
        return {f: getattr(r, f) for f, _ in StreamStats._fields_}

    def window(self, beam: int, seg: int, n_dm: int):
        """(t_first, int32 [n_dm][n_t]) of the last step's window of a row."""
        t0 = C.c_int64()
        nt = C.c_int64()
        st = _L.gsp_stream_window(self.h, int(beam), int(seg), None, 0, C.byref(t0), C.byref(nt))
        if st not in (GSP_OK, GSP_ECAPACITY):
            self._check(st)
        out = np.empty((n_dm, nt.value), np.int32)
        if nt.value > 0:
            self._check(_L.gsp_stream_window(self.h, int(beam), int(seg), out.ctypes.data, out.size, C.byref(t0),
                                             C.byref(nt)))
        return t0.value, out

    def snapshot(self, beam: int) -> bytes:
        n = C.c_int64()
        st = _L.gsp_stream_snapshot(self.h, int(beam), None, 0, C.byref(n))
        if st not in (GSP_OK, GSP_ECAPACITY):
            self._check(st)
        buf = C.create_string_buffer(n.value)
        self._check(_L.gsp_stream_snapshot(self.h, int(beam), buf, n.value, C.byref(n)))
        return buf.raw

    def restore(self, beam: int, data: bytes):
        self._check(_L.gsp_stream_restore(self.h, int(beam), data, len(data)))


# --- learned triage ------------------------------------------------------------
_L.gsp_cutouts.argtypes = [P, P, P, P, C.POINTER(DmtDesc), P, C.c_int64, P, P]
_L.gsp_cutouts.restype = C.c_int
_L.gsp_cnn_num_params.argtypes = []
_L.gsp_cnn_num_params.restype = C.c_int64
_L.gsp_cnn_create.argtypes = [P, C.c_uint64, C.POINTER(P)]
_L.gsp_cnn_create.restype = C.c_int
_L.gsp_cnn_destroy.argtypes = [P]
_L.gsp_cnn_destroy.restype = None
for _n in ("gsp_cnn_get_params", "gsp_cnn_set_params"):
    getattr(_L, _n).argtypes = [P, P, C.c_int64]
    getattr(_L, _n).restype = C.c_int
for _n in ("gsp_cnn_save", "gsp_cnn_load"):
    getattr(_L, _n).argtypes = [P, C.c_char_p]
    getattr(_L, _n).restype = C.c_int
_L.gsp_cnn_forward.argtypes = [P, P, C.c_int64, P, P]
_L.gsp_cnn_forward.restype = C.c_int
_L.gsp_cnn_gradients.argtypes = [P, P, P, C.c_int64, P, P, P]
_L.gsp_cnn_gradients.restype = C.c_int
_L.gsp_cnn_train_step.argtypes = [P, P, P, C.c_int64, C.c_float, P, P]
_L.gsp_cnn_train_step.restype = C.c_int
_L.gsp_cnn_activation.argtypes = [P, C.c_int32, P, C.c_int64]
_L.gsp_cnn_activation.restype = C.c_int


def cutouts(ctx: Context, fb, freqs, dmt, desc: DmtDesc, cands: np.ndarray, out=None, stream=None):
    """bf16 (torch.int16 storage of the bit patterns) [n][2][64][64] cutouts
    of candidates (CAND_DTYPE, host) on the device."""
    import torch
    n = len(cands)
    if out is None:
        out = torch.empty((n, 2, 64, 64), dtype=torch.int16, device=fb.device)
    if n == 0:
        return out
    c = np.ascontiguousarray(cands, dtype=CAND_DTYPE)
    cd = torch.from_numpy(c.view(np.uint8).copy()).to(fb.device)
    f = _f64(freqs)
    _check(_L.gsp_cutouts(ctx.h, C.c_void_p(fb.data_ptr()), f.ctypes.data, C.c_void_p(dmt.data_ptr()),
                          C.byref(desc), C.c_void_p(cd.data_ptr()), n, C.c_void_p(out.data_ptr()),
                          _stream_handle(stream)), ctx.h)
    if stream is None:
        torch.cuda.current_stream().synchronize()  # keep `cd` alive until the kernel has read it
    else:
        stream.synchronize()
    return out


class Cnn:
    """Triage network on the device (parameters as one float vector, in the
    library's documented order)."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        self.h = P()
        _check(_L.gsp_cnn_create(ctx.h, C.c_uint64(seed), C.byref(self.h)), ctx.h)
        self.n_params = int(_L.gsp_cnn_num_params())

    def close(self):
        if self.h:
            _L.gsp_cnn_destroy(self.h)
            self.h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, np.float32)
        _check(_L.gsp_cnn_get_params(self.h, out.ctypes.data, self.n_params), self.ctx.h)
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.n_params
        _check(_L.gsp_cnn_set_params(self.h, p.ctypes.data, self.n_params), self.ctx.h)

    def save(self, path: str):
        _check(_L.gsp_cnn_save(self.h, path.encode()), self.ctx.h)

    def load(self, path: str):
        _check(_L.gsp_cnn_load(self.h, path.encode()), self.ctx.h)

    @staticmethod
    def _x(x):
        import torch
        assert x.is_cuda and x.is_contiguous() and x.dtype in (torch.int16, torch.bfloat16)
        assert tuple(x.shape[1:]) == (2, 64, 64)
        return C.c_void_p(x.data_ptr()), int(x.shape[0])

    def forward(self, x, out=None, stream=None):
        import torch
        xp, n = self._x(x)
        if out is None:
            out = torch.empty(n, dtype=torch.float32, device=x.device)
        _check(_L.gsp_cnn_forward(self.h, xp, n, C.c_void_p(out.data_ptr()), _stream_handle(stream)), self.ctx.h)
        return out

    def gradients(self, x, labels, stream=None):
        xp, n = self._x(x)
        assert labels.is_cuda and labels.numel() == n
        g = np.empty(self.n_params, np.float32)
        loss = C.c_float()
        _check(_L.gsp_cnn_gradients(self.h, xp, C.c_void_p(labels.data_ptr()), n, g.ctypes.data, C.byref(loss),
                                    _stream_handle(stream)), self.ctx.h)
        return g, float(loss.value)

    def train_step(self, x, labels, lr: float, want_loss: bool = True, stream=None):
        xp, n = self._x(x)
        assert labels.is_cuda and labels.numel() == n
        loss = C.c_float()
        _check(_L.gsp_cnn_train_step(self.h, xp, C.c_void_p(labels.data_ptr()), n, float(lr),
                                     C.byref(loss) if want_loss else None, _stream_handle(stream)), self.ctx.h)
        return float(loss.value) if want_loss else None

    def activation(self, which: int, n: int) -> np.ndarray:
        """A stored tensor of the last forward / backward pass (the header's
        table of `which`): bf16 values as float64, float32 logits and
        dloss/dlogit, uint8 max-pool choices."""
        if which < 4 or 6 <= which < 10:
            l = which % 6
            h = 32 >> l
            shape, dt = (n, h, h, 16 << l), np.uint16
        elif which in (4, 10):
            shape, dt = (n, 192), np.uint16
        elif which in (5, 11):
            shape, dt = (n,), np.float32
        elif 12 <= which < 16:
            l = which - 12
            h = 64 >> l
            shape, dt = (n, h, h, 16 << l), np.uint16
        elif 16 <= which < 20:
            l = which - 16
            h = 32 >> l
            shape, dt = (n, h, h, 16 << l), np.uint8
        else:
            raise ValueError(which)
        out = np.empty(shape, dt)
        _check(_L.gsp_cnn_activation(self.h, int(which), out.ctypes.data, out.nbytes), self.ctx.h)
        if dt == np.uint16:
            return (out.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
        return out
