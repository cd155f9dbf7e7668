"""Host logic of the triage module: labelling candidates by injections."""
import numpy as np

from paper_2110_12749_amd import gsp, synth, triage


def cands(rows):
    c = np.zeros(len(rows), gsp.CAND_DTYPE)
    for k, (seg, dm, t, w) in enumerate(rows):
        c[k]["seg"], c[k]["dm"], c[k]["time_s"], c[k]["width"] = seg, dm, t, w
    return c


def test_match_pulses_windows():
    w = synth.triage_beam(0, "train")
    w.pulses = [synth.Pulse(300.0, 1.0, 2e-3, 10.0), synth.Pulse(20.0, 2.0, 1e-3, 10.0)]
    span = triage.K_DISP * (1 / 1000.0 ** 2 - 1 / 1500.0 ** 2)
    c = cands([
        (1, 300.0, 1.0, 4),                     # on the pulse
        (1, 310.0, 1.0 - 0.5 * span * 10, 8),   # higher DM: arrives early, inside the window
        (1, 310.0, 1.0 + 0.05, 8),              # higher DM but late: outside
        (1, 290.0, 1.0 + 0.5 * span * 10, 8),   # lower DM: arrives late, inside
        (0, 20.5, 2.0, 2),                      # second pulse
        (0, 17.5, 2.0, 2),                      # DM too far from 20 (|dd| > max(2, 0.05 * 20))
        (0, 20.0, 3.0, 2),                      # no pulse at that time
        (0, 20.0, 2.0, 512),                    # box far longer than the pulse
        (1, 320.0, 1.0, 8),                     # DM too far from 300 (|dd| > 15)
    ])
    got = triage.match_pulses(c, w)
    assert got.tolist() == [0, 0, -1, 0, 1, -1, -1, -1, -1]


def test_triage_beams_are_disjoint_and_seeded():
    a = synth.triage_beam(3, "train")
    b = synth.triage_beam(3, "test")
    c = synth.triage_beam(3, "train")
    assert a.beam != b.beam and [p.dm for p in a.pulses] != [p.dm for p in b.pulses]
    assert [p.dm for p in a.pulses] == [p.dm for p in c.pulses] and a.spikes == c.spikes
    assert a.n_trials == 3350 and all(10.0 <= p.dm <= 1500.0 for p in a.pulses)
