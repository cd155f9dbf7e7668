"""The search entry point that allocates nothing (static device scratch,
host work in the caller's buffer) gives exactly what
gsp_single_pulse_search gives, on two calls in a row, the second on a
smaller input, and rejects what its scratch cannot hold."""
import numpy as np
import pytest

from paper_2110_12749_amd import synth
from tests._util import say

pytestmark = pytest.mark.gpu

KEY = ["seg", "dm_index", "dm", "t_peak", "t_first", "t_last", "width", "snr", "time_s"]


def _case(ctx, gsp, torch, w):
    X = w.generate()
    fb = torch.from_numpy(X).cuda()
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    dmt = ctx.dedisperse(fb, w.freqs, desc)
    return desc, dmt


def test_noalloc_search_equals_search_on_two_calls(dev):
    import torch
    from paper_2110_12749_amd import gsp
    ctx = gsp.Context(0)
    big = synth.small(nchan=256, nsamp=40000, segments=[(0.0, 0.5, 120, 1), (60.0, 1.0, 60, 2), (120.0, 2.0, 30, 4)],
                      n_pulses=4, seed_offset=80, widths=[1, 2, 4, 8, 16, 32, 64])
    small = synth.small(nchan=64, nsamp=5000, segments=[(0.0, 1.0, 40, 1)], n_pulses=2, seed_offset=81,
                        widths=[1, 2, 4, 8, 16])
    for name, w in (("larger", big), ("smaller", small)):
        desc, dmt = _case(ctx, gsp, torch, w)
        ref = ctx.single_pulse_search(dmt, desc, w.widths, w.threshold)
        got = ctx.single_pulse_search_noalloc(dmt, desc, w.widths, w.threshold)
        say(f"[case] no-alloc search, {name} input: {len(ref)} candidates")
        assert len(ref) > 0
        assert len(got) == len(ref)
        for k in KEY:
            assert np.array_equal(got[k], ref[k]), k
    # a candidate buffer too small: nothing written, a sufficient capacity reported
    desc, dmt = _case(ctx, gsp, torch, big)
    ref = ctx.single_pulse_search(dmt, desc, big.widths, big.threshold)
    out = np.zeros(2, gsp.CAND_DTYPE)
    import ctypes as C
    n = C.c_int64()
    w = np.ascontiguousarray(big.widths, dtype=np.int32)
    st = gsp._L.gsp_single_pulse_search_noalloc(ctx.h, C.c_void_p(dmt.data_ptr()), C.byref(desc), w.ctypes.data,
                                                len(w), float(big.threshold), out.ctypes.data, 2, C.byref(n), None)
    assert st == gsp.GSP_ECAPACITY and n.value >= len(ref)
    assert (out == np.zeros(2, gsp.CAND_DTYPE)).all()
    got = ctx.single_pulse_search_noalloc(dmt, desc, big.widths, big.threshold, capacity=int(n.value))
    assert len(got) == len(ref) and all(np.array_equal(got[k], ref[k]) for k in KEY)
    ctx.close()
