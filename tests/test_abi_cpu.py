"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every declared symbol; plan shapes and delay tables equal the
oracle's entry for entry; argument errors come back as status codes; the
host grouping equals the oracle's."""
import ctypes as C

import numpy as np
import pytest

import oracle
from paper_2110_12749_amd import synth
from tests._util import header_functions


@pytest.fixture(scope="module")
def gsp():
    from paper_2110_12749_amd import gsp as g
    return g


def test_library_exports_every_declared_symbol(gsp):
    names = header_functions()
    assert "gsp_dedisperse" in names and "gsp_single_pulse_search" in names
    for n in names:
        assert hasattr(gsp.lib(), n), n


def _check_plan(gsp, w, nsamp=None):
    nsamp = nsamp or w.nsamp
    d = gsp.plan_shape(nsamp, w.freqs, w.tsamp, w.segments)
    md, no = oracle.plan_shape(nsamp, w.freqs, w.tsamp, w.segments)
    assert d.n_seg == len(w.segments)
    off = 0
    for s in range(d.n_seg):
        assert d.max_delay[s] == md[s] and d.n_out[s] == no[s]
        assert d.offset[s] == off
        off += w.segments[s][2] * no[s]
    assert d.total == off and d.n_trials == w.n_trials
    return d


def test_plan_shape_matches_oracle(gsp):
    for w in (synth.tiny(), synth.realistic(), synth.wideband()):
        _check_plan(gsp, w)
    d = _check_plan(gsp, synth.tiny())
    assert d.n_out[0] == 14072 and d.max_delay[0] == 2312


@pytest.mark.parametrize("name", ["tiny", "realistic", "wideband"])
def test_delay_tables_bit_exact_vs_oracle(gsp, name):
    w = getattr(synth, name)() if name == "tiny" else getattr(synth, name)(nsamp=1 << 20 if name == "realistic" else 1 << 19)
    d = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    for s, seg in enumerate(w.segments):
        lib = gsp.delay_table(d, w.freqs, s)
        ref = oracle.delay_table(w.freqs, w.tsamp, seg)
        assert (lib.astype(np.int64) == ref).all()


def test_plan_errors(gsp):
    f = np.linspace(1000, 1500, 16)
    with pytest.raises(gsp.GspError) as e:
        gsp.plan_shape(100, f, 1e-3, [(0.0, 100.0, 10, 1)])
    assert e.value.status == gsp.GSP_ETOOSHORT
    for bad in ([(0.0, 0.0, 4, 1)], [(0.0, 1.0, 0, 1)], [(-1.0, 1.0, 4, 1)], [(0.0, 1.0, 4, 0)],
                [(0.0, 1.0, 4, 258)], [(0.0, float("nan"), 4, 1)]):
        with pytest.raises(gsp.GspError) as e:
            gsp.plan_shape(10000, f, 1e-3, bad)
        assert e.value.status == gsp.GSP_EINVAL
    with pytest.raises(gsp.GspError) as e:
        gsp.plan_shape(10000, np.array([1000.0, -5.0]), 1e-3, [(0.0, 1.0, 4, 1)])
    assert e.value.status == gsp.GSP_EINVAL
    with pytest.raises(gsp.GspError) as e:
        gsp.plan_shape(10000, f, 0.0, [(0.0, 1.0, 4, 1)])
    assert e.value.status == gsp.GSP_EINVAL
    with pytest.raises(gsp.GspError) as e:
        gsp.plan_shape(1 << 20, np.linspace(1000, 1500, 70000), 1e-3, [(0.0, 1.0, 4, 128)])
    assert e.value.status == gsp.GSP_EOVERFLOW
    with pytest.raises(gsp.GspError) as e:
        gsp.plan_shape(10000, f, 1e-3, [(0.0, 1.0, 4, 1)] * 17)
    assert e.value.status == gsp.GSP_EINVAL
    assert gsp.lib().gsp_strerror(-4) == b"output capacity too small"


def test_dedisperse_rejects_bad_pointers_without_gpu(gsp):
    # a null context is rejected before any device call
    d = gsp.plan_shape(4096, np.linspace(1000, 1500, 16), 1e-3, [(0.0, 1.0, 4, 1)])
    rc = gsp.lib().gsp_dedisperse(None, None, None, C.byref(d), None, None)
    assert rc == gsp.GSP_EINVAL


def _rand_cands(rng, n, n_trials=12, T=400):
    import paper_2110_12749_amd.gsp as g
    c = np.zeros(n, g.CAND_DTYPE)
    c["seg"] = rng.integers(0, 2, n)
    c["dm_index"] = rng.integers(0, n_trials, n)
    c["t_first"] = rng.integers(0, T, n)
    c["t_last"] = c["t_first"] + rng.integers(0, 6, n)
    c["t_peak"] = c["t_first"]
    c["width"] = 1
    c["snr"] = rng.choice(np.arange(6, 12, 0.5), n).astype(np.float32)
    # runs of one trial must be disjoint (as a search produces them)
    keep = []
    seen = {}
    for k in np.lexsort((c["t_first"], c["dm_index"], c["seg"])):
        key = (int(c["seg"][k]), int(c["dm_index"][k]))
        if key in seen and c["t_first"][k] <= seen[key]:
            continue
        seen[key] = int(c["t_last"][k])
        keep.append(k)
    return c[np.array(sorted(keep))]


@pytest.mark.parametrize("search_order", [False, True])
def test_grouping_matches_oracle(gsp, search_order):
    """Any candidate order, and the search's own (seg, dm_index, t_peak)
    order, whose trials the grouping then orders one by one."""
    rng = np.random.default_rng(0)
    for trial in range(30):
        c = _rand_cands(rng, 200)
        if search_order:
            c = c[np.lexsort((c["t_first"], c["t_peak"], c["dm_index"], c["seg"]))]
        rep, ng = gsp.group_candidates(c)
        for s in (0, 1):
            idx = np.nonzero(c["seg"] == s)[0]
            oc = np.zeros(len(idx), oracle.CAND_DTYPE)
            oc["trial"] = c["dm_index"][idx]
            oc["t_first"] = c["t_first"][idx]
            oc["t_last"] = c["t_last"][idx]
            oc["t_peak"] = c["t_peak"][idx]
            oc["snr"] = c["snr"][idx].astype(np.float64)
            og = oracle.group(oc)
            assert (idx[og] == rep[idx]).all()
        assert ng == len(np.unique(rep))


def test_subband_plan_shape_matches_oracle(gsp):
    """Sub-band plans: per-row valid lengths and largest composite delays
    equal the oracle's; the descriptor is marked as a sub-band plan; the
    16-bit limit on the sub-band series and bad n_sub / group are rejected."""
    w = synth.realistic()
    n_sub, group = [64, 64, 64, 128], [8, 16, 16, 16]
    d = gsp.subband_plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments, n_sub, group)
    assert d.kind == 1
    off = 0
    for s, seg in enumerate(w.segments):
        dd, n_out = oracle.subband_delays(w.freqs, w.nsamp, w.tsamp, seg, n_sub[s], group[s])
        assert d.n_out[s] == n_out
        assert d.max_delay[s] == w.nsamp // seg[3] - n_out
        assert d.offset[s] == off
        off += seg[2] * n_out
    assert d.total == off
    assert gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments).kind == 0
    for bad in ([64, 64, 64, 64], [0, 64, 64, 128], [64, 64, 64, 4097]):  # D = 8 with 64 channels per band; range
        with pytest.raises(gsp.GspError) as e:
            gsp.subband_plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments, bad, 16)
        assert e.value.status == gsp.GSP_EINVAL
    for bad in (0, 65):
        with pytest.raises(gsp.GspError):
            gsp.subband_plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments, n_sub, bad)
    with pytest.raises(gsp.GspError) as e:
        gsp.subband_plan_shape(20000, w.freqs, w.tsamp, w.segments, n_sub, 16)
    assert e.value.status == gsp.GSP_ETOOSHORT
