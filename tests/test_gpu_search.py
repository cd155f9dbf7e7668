"""The boxcar search alone on hand-shaped series (synth.search_cases), through
the C ABI, against the oracle's search of the same series.

Runs that cross the search kernel's internal boundaries (64-sample steps,
512-sample blocks, segments of box ends handled by different waves), ties of
equal box sums, boxes at the first and last sample, sums beyond 2^32 and
negative samples.  Candidates must agree exactly: same runs (first and last
box end), same peak (box end and width) and the same SNR to float32
rounding."""
import numpy as np
import pytest

import oracle
from paper_2110_12749_amd import synth
from tests._util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env(dev):
    import torch
    from paper_2110_12749_amd import gsp
    ctx = gsp.Context(0)
    yield gsp, ctx, torch
    torch.cuda.synchronize()
    ctx.close()


def run_case(env, x, widths, thr):
    gsp, ctx, torch = env
    n_tr, n = x.shape
    # one channel, D = 1: n outputs per trial, the DM-time rows are x itself
    desc = gsp.plan_shape(n, [1400.0], 1e-4, [(0.0, 1.0, n_tr, 1)])
    assert desc.n_out[0] == n and desc.total == x.size
    dmt = torch.from_numpy(np.ascontiguousarray(x).reshape(-1)).cuda()
    cg = ctx.single_pulse_search(dmt, desc, widths, thr)
    rows = [oracle.search_series(x[i], widths, thr, trial=i) for i in range(n_tr)]
    co = np.concatenate(rows)
    say(f"  widths {list(widths)[:4]}..{max(widths)} thr {thr}: gpu {len(cg)} oracle {len(co)}")
    kg = np.lexsort((cg["t_first"], cg["dm_index"]))
    ko = np.lexsort((co["t_first"], co["trial"]))
    cg, co = cg[kg], co[ko]
    assert len(cg) == len(co)
    for f_g, f_o in (("dm_index", "trial"), ("t_first", "t_first"), ("t_last", "t_last"), ("t_peak", "t_peak"),
                     ("width", "width")):
        bad = np.flatnonzero(cg[f_g].astype(np.int64) != co[f_o].astype(np.int64))
        assert len(bad) == 0, (f_g, cg[bad[:3]], co[bad[:3]])
    so = co["snr"].astype(np.float64)
    assert np.all(np.abs(cg["snr"].astype(np.float64) - so) <= 1e-6 * np.abs(so))
    return cg


@pytest.mark.parametrize("widths,thr", [
    ([1, 2, 4, 8, 16, 32, 64, 128, 256, 512], 5.0),
    ([1, 3, 7, 100, 333, 1000], 4.0),   # a longer ring
    ([1, 2, 5, 40, 4000], 4.5),         # one segment per trial
    ([1, 2, 4], 5.0),                   # no box holds both shelf spikes: a tie
])
def test_search_cases_exact(env, widths, thr):
    say(f"[case] search cases widths {widths} thr {thr}")
    x = synth.search_cases()
    c = run_case(env, x, widths, thr)
    assert not (c["dm_index"] == 4).any()  # constant trial
    if max(widths) >= 64:  # boxes long enough to lift the plateau over the threshold
        # the plateau trial gives one run spanning segment and block boundaries
        long = c[(c["dm_index"] == 1) & (c["t_last"] - c["t_first"] > 16384)]
        assert len(long) >= 1
    if max(widths) > 4:
        return
    # the tie on the shelf goes to the earlier box end
    for tr in (2, 3):
        shelf = c[(c["dm_index"] == tr) & (c["t_first"] <= 1000) & (c["t_last"] >= 1006)]
        assert len(shelf) == 1 and shelf["t_peak"][0] == 1000 and shelf["width"][0] == 1, shelf


def test_search_tail_lengths(env):
    """Series lengths around the step, block and segment sizes."""
    x = synth.search_cases(n=30000, seed=1)
    for n in (1, 63, 64, 65, 511, 512, 513, 8191, 8192, 8193, 8192 + 511, 16385):
        say(f"[case] search length {n}")
        run_case(env, x[:, :n], [1, 2, 4, 8, 16, 32, 64], 4.0)
