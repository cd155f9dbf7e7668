"""RFI mitigation on the GPU (gsp_rfi_clean) against the oracle
(oracle.rfi_clean): bit-exact cleaned filterbanks and equal counts of
replaced spectra, in place and out of place, clip alone, zero-DM filter
alone and both, ragged last blocks, channel counts that are and are not
multiples of 16, and the wideband workload at full size."""
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


def _check(env, X, clip, block, zero_dm, in_place):
    gsp, ctx, torch = env
    ref, n_ref = oracle.rfi_clean(X, clip_sigma=clip, block=block, zero_dm=zero_dm)
    fb = torch.from_numpy(X).cuda()
    if in_place:
        out, n = ctx.rfi_clean(fb, clip, block, zero_dm, out=fb)
    else:
        out, n = ctx.rfi_clean(fb, clip, block, zero_dm)
        assert torch.equal(fb.cpu(), torch.from_numpy(X)), "input changed"
    got = out.cpu().numpy()
    bad = np.argwhere(got != ref)
    assert len(bad) == 0, f"{len(bad)} bytes differ, first {bad[:5].tolist()}"
    assert n == n_ref
    return n


def test_hand_case(env):
    X = np.array([[2, 2, 2, 2], [1, 3, 1, 3], [3, 1, 3, 1], [2, 2, 2, 2], [2, 2, 2, 2], [12, 12, 12, 12]], np.uint8)
    assert _check(env, X, 2.0, 6, False, False) == 1
    Y = np.array([[3, 0], [4, 0], [90, 90]], np.uint8)
    assert _check(env, Y, 1.0, 3, False, True) == 1


@pytest.mark.parametrize("nchan,nsamp,block", [(128, 5000, 1024), (100, 3001, 700), (4096, 9000, 2048),
                                               (37, 2500, 1)])
@pytest.mark.parametrize("mode", ["clip", "zerodm", "both"])
def test_spikes_and_bursts(env, nchan, nsamp, block, mode):
    """Noise with zero-DM spikes (some saturating) and narrowband bursts;
    ragged last blocks; block 1 (every block a single spectrum: nothing to
    replace)."""
    w = synth.small(nchan=nchan, nsamp=nsamp, n_pulses=1, seed_offset=500 + nchan % 13)
    X = w.generate()
    rng = np.random.default_rng(nchan + nsamp)
    for j in rng.choice(nsamp, 6, replace=False):
        X[j] = np.minimum(255, X[j].astype(np.int32) + int(rng.integers(30, 200))).astype(np.uint8)
    for c in rng.choice(nchan, max(1, nchan // 20), replace=False):
        t0 = int(rng.integers(0, nsamp - 200))
        X[t0:t0 + 200, c] = np.minimum(255, X[t0:t0 + 200, c].astype(np.int32) + 60).astype(np.uint8)
    clip = 0.0 if mode == "zerodm" else 4.0
    zero_dm = mode != "clip"
    say(f"[case] rfi {nchan}x{nsamp} block {block} {mode}")
    n1 = _check(env, X, clip, block, zero_dm, False)
    n2 = _check(env, X, clip, block, zero_dm, True)
    assert n1 == n2
    if mode != "zerodm" and block > 1:
        assert n1 >= 1


def test_wideband_full_size(env):
    """The wideband workload (4096 channels, 2^19 samples, bursts in 5 % of
    the channels, 30 zero-DM spikes), cleaned in place by both steps."""
    w = synth.wideband()
    say("[case] rfi wideband full size: generate")
    X = w.generate()
    n = _check(env, X, 6.0, 2048, True, True)
    say(f"  {n} spectra replaced")
    assert n >= 1
