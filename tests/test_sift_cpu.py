"""Sifting (ranking of grouped events) and the candidate store, host only.

The ranking oracle (oracle/sift.py) is pinned by hand-built groups whose
rank follows from the stated rules by hand, and by what the rules are for:
an injected dispersed pulse ranks high, zero-DM spikes rank as RFI.  The
library's gsp_rank_groups equals the oracle record for record on the
oracle's candidates of a synthetic beam.  The store keeps the six tables,
matches known sources by DM, answers queries and survives a save/load."""
import numpy as np
import pytest

import oracle
from oracle import sift
from paper_2110_12749_amd import synth


@pytest.fixture(scope="module")
def gsp():
    from paper_2110_12749_amd import gsp as g
    return g


def _cands(gsp, rows):
    """rows: (seg, dm_index, dm, t_first, t_last, width, snr) -> CAND_DTYPE, t_peak = t_last - width + 1."""
    c = np.zeros(len(rows), gsp.CAND_DTYPE)
    for k, (s, i, dm, t0, t1, wd, snr) in enumerate(rows):
        c[k] = (s, i, dm, t1 - wd + 1, t0, t1, wd, snr, (t1 - wd + 1 + wd / 2) * 1e-3)
    return c


def test_hand_built_groups_rank_by_the_rules(gsp):
    # group A: 2 trials only -> noise (1)
    # group B: peak at DM 0.5 over 4 trials -> RFI (2), before any other rule
    # group C: 5 trials, SNR 10 at the peak, 9.5 / 9.2 at the ends: f = 0.05 -> 3
    # group D: ends 8.5 and 8.2 of 10: f = min(0.15, 0.18) = 0.15 -> 4
    # group E: ends 7 and 6.2 of 10: f = 0.3 -> 5
    # group F: ends 6.1 and 6.0 of 15: f = 0.593 -> 6
    rows = [(0, 10, 10.0, 100, 105, 4, 7.0), (0, 11, 11.0, 100, 104, 4, 6.5),
            (0, 0, 0.0, 500, 501, 2, 20.0), (0, 1, 0.5, 500, 501, 2, 22.0), (0, 2, 1.0, 500, 500, 2, 15.0),
            (0, 3, 1.5, 500, 500, 2, 9.0)]

    def peaked(t, ends, top, i0=40):
        lo, hi = ends
        return [(0, i0, float(i0), t, t + 3, 8, lo), (0, i0 + 1, i0 + 1.0, t, t + 3, 8, (lo + top) / 2),
                (0, i0 + 2, i0 + 2.0, t, t + 4, 8, top), (0, i0 + 3, i0 + 3.0, t + 1, t + 4, 8, (hi + top) / 2),
                (0, i0 + 4, i0 + 4.0, t + 1, t + 4, 8, hi)]
    rows += peaked(1000, (9.5, 9.2), 10.0) + peaked(2000, (8.5, 8.2), 10.0) + peaked(3000, (7.0, 6.2), 10.0) \
        + peaked(4000, (6.1, 6.0), 15.0)
    c = _cands(gsp, rows)
    order = np.lexsort((c["t_peak"], c["dm_index"], c["seg"]))
    c = c[order]
    rep, ng = gsp.group_candidates(c)
    assert ng == 6
    ranks = {}
    for g in sift.rank_groups(c, rep, [1], 1e-3):
        ranks[int(round(g["time_s"]))] = g["rank"]
    # representatives' times: (t_peak + w/2) * 1e-3 s -> 0, 0, 1, 2, 3, 4 (rounded)
    got = sorted(g["rank"] for g in sift.rank_groups(c, rep, [1], 1e-3))
    assert got == [1, 2, 3, 4, 5, 6]
    by_dm = {round(g["dm_peak"], 1): g["rank"] for g in sift.rank_groups(c, rep, [1], 1e-3)}
    assert by_dm[0.5] == 2 and by_dm[10.0] == 1
    # the group spans and counts
    F = [g for g in sift.rank_groups(c, rep, [1], 1e-3) if g["rank"] == 6][0]
    assert F["n_events"] == 5 and F["n_trials"] == 5 and F["dm_min"] == 40.0 and F["dm_max"] == 44.0
    assert F["start_s"] == pytest.approx((4000 - 8 + 1) * 1e-3) and F["duration_s"] == pytest.approx(12e-3)


def _oracle_candidates(gsp, w, X):
    """The oracle's candidates of a whole plan in the library's layout, sorted
    as gsp_single_pulse_search sorts them, and its grouping."""
    rows = oracle.dedisperse(X, w.freqs, w.tsamp, w.segments)
    o = oracle.search(rows, w.widths, w.threshold)
    c = np.zeros(len(o), gsp.CAND_DTYPE)
    c["seg"] = o["seg"]
    c["dm_index"] = o["trial"]
    for k in range(len(o)):
        seg = w.segments[int(o["seg"][k])]
        c["dm"][k] = oracle.trial_dm(seg, int(o["trial"][k]))
        c["time_s"][k] = (int(o["t_peak"][k]) + 0.5 * int(o["width"][k])) * seg[3] * w.tsamp
    for f in ("t_peak", "t_first", "t_last", "width", "snr"):
        c[f] = o[f]
    rep = np.empty(len(c), np.int64)
    for s in range(len(w.segments)):
        idx = np.flatnonzero(c["seg"] == s)
        if len(idx):
            rep[idx] = idx[oracle.group(o[idx])]
    return c, rep


def test_library_ranks_equal_oracle_and_mean_something(gsp):
    """The tiny workload's pulse (DM 57.3, SNR 15) plus three zero-DM
    broadband spikes: record-for-record equality of library and oracle;
    the pulse's group ranks 5 or 6, the spikes' groups rank 2."""
    w = synth.tiny()
    w.spikes = [(3000, 2, 40.0), (9000, 1, 40.0), (12000, 3, 40.0)]
    X = w.generate()
    c, rep = _oracle_candidates(gsp, w, X)
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    lib = gsp.rank_groups(c, rep, desc)
    ora = sift.rank_groups(c, rep, [s[3] for s in w.segments], w.tsamp)
    assert len(lib) == len(ora) > 3
    for a, b in zip(lib, ora):
        for f in ("rep", "seg", "rank", "n_events", "n_trials"):
            assert int(a[f]) == b[f], f
        for f in ("dm_min", "dm_max", "dm_peak", "snr_max", "snr_lo", "snr_hi", "time_s", "width_s", "start_s",
                  "duration_s"):
            assert float(a[f]) == pytest.approx(b[f], rel=1e-12, abs=1e-12), f
    pulse = max(ora, key=lambda g: g["snr_max"] if abs(g["dm_peak"] - 57.3) < 3 else 0)
    assert abs(pulse["dm_peak"] - 57.3) < 3 and pulse["rank"] >= 5
    for t in (3000, 9000, 12000):
        near = [g for g in ora if abs(g["time_s"] - t * w.tsamp) < 0.05 and g["dm_peak"] < 1.0]
        assert near and all(g["rank"] == 2 for g in near), t


def test_store_tables_queries_and_roundtrip(gsp, tmp_path):
    w = synth.tiny()
    X = w.generate()
    c, rep = _oracle_candidates(gsp, w, X)
    desc = gsp.plan_shape(w.nsamp, w.freqs, w.tsamp, w.segments)
    groups = gsp.rank_groups(c, rep, desc)
    st = gsp.Store()
    f1 = st.add_file("beam0_tiny", 0, w.nchan, w.nsamp, w.tsamp, 1000.0, 1500.0)
    first = st.add_groups(f1, len(c), groups)
    assert first == 1 and st.count(gsp.T_SINGLEPULSE_CANDIDATES) == len(groups)
    with pytest.raises(gsp.GspError):
        st.add_groups(f1, len(c), groups)  # each input once
    with pytest.raises(gsp.GspError):
        st.add_file("bad,name", 0, 1, 1, 1.0, 1.0, 2.0)
    st.add_pulsar("J_test_57", 57.3)
    st.add_pulsar("J_none", 900.0)
    assert st.match_pulsars(f1, dm_tol=2.0, min_rank=5) == 1
    st.add_picture(first, "cutouts/cand1.png")
    best = st.query(min_rank=5)
    assert len(best) >= 1 and all(b["g"]["rank"] >= 5 for b in best)
    near = st.query(min_rank=1, dm_lo=55.0, dm_hi=60.0)
    assert all(55.0 <= b["g"]["dm_peak"] <= 60.0 for b in near) and len(near) >= 1
    counts = [st.count(t) for t in range(6)]
    assert counts == [1, 1, len(groups), 2, 1, 1]
    st.save(tmp_path)
    names = sorted(p.name for p in tmp_path.iterdir())
    assert names == sorted(["T_FITS_INFO.csv", "T_SINGLEPULSE_GROUPS.csv", "T_SINGLEPULSE_CANDIDATES.csv",
                            "T_PULSAR.csv", "T_FILE_PULSAR.csv", "T_SINGLEPULSE_PIC.csv"])
    st2 = gsp.Store()
    st2.load(tmp_path)
    assert [st2.count(t) for t in range(6)] == counts
    a, b = st.query(), st2.query()
    assert len(a) == len(b)
    for f in gsp.GROUP_DTYPE.names:
        assert np.array_equal(a["g"][f], b["g"][f]), f
    st.close()
    st2.close()
