"""CPU oracle of candidate sifting: ranking of grouped single-pulse events.

TEST INFRASTRUCTURE.  Only ``tests/`` uses this module.  It shares no code
with the GPU library and imports nothing from it.

The paper sifts its single-pulse events with RRATtrap (Section 2.2: events
of nearby DMs and times are grouped, the groups ranked and scored by rules;
Section 3.2 reports ranks 3 to 6 with 6 the best and a class of RFI or
noise) but states none of the rules.  The rules below are this project's
reading, written out plainly; parity unpinned by the paper (pinned here by
hand-built groups and by injected pulses and zero-DM spikes in the tests):

  Per group (a friends-of-friends component of the candidates of one plan
  row, identified by its representative: the member of highest SNR):
    n_events  members; n_trials distinct trials among them;
    dm_min, dm_max over the members; the peak = the representative
      (dm_peak, snr_max, time_s, width_s = width * D * tsamp);
    span: start = min over members of (t_first - width + 1) * D * tsamp,
          end = max over members of (t_last + 1) * D * tsamp;
          duration = end - start;
    snr_lo / snr_hi: best member SNR at the group's lowest / highest DM.
  rank 2 (RFI):   dm_peak < 1 pc cm^-3 (interference at zero DM);
  rank 1 (noise): otherwise, n_trials < 3;
  otherwise the fall-off of SNR toward both ends of the group's DM range,
    f = min(1 - snr_lo / snr_max, 1 - snr_hi / snr_max), gives
    rank 3 (f < 0.1), 4 (f < 0.2), 5 (f < 0.35) or 6.
"""
from __future__ import annotations

import numpy as np

RFI_DM = 1.0
FALLOFF = (0.1, 0.2, 0.35)


def rank_groups(cands, rep, downsamp, tsamp):
    """cands: structured array with seg, dm_index, dm, t_peak, t_first,
    t_last, width, snr, time_s; rep[k] = index of candidate k's group
    representative; downsamp[seg] = D of each plan row.  Returns a list of
    dicts, one per group, in order of the representative's index."""
    members = {}
    for k in range(len(cands)):
        members.setdefault(int(rep[k]), []).append(k)
    out = []
    for r in sorted(members):
        ks = members[r]
        c0 = cands[r]
        D = int(downsamp[int(c0["seg"])])
        trials = set()
        dm_min, dm_max = float("inf"), float("-inf")
        start, end = float("inf"), float("-inf")
        for k in ks:
            c = cands[k]
            trials.add((int(c["seg"]), int(c["dm_index"])))
            dm_min = min(dm_min, float(c["dm"]))
            dm_max = max(dm_max, float(c["dm"]))
            start = min(start, (int(c["t_first"]) - int(c["width"]) + 1) * D * tsamp)
            end = max(end, (int(c["t_last"]) + 1) * D * tsamp)
        snr_lo = max(float(cands[k]["snr"]) for k in ks if float(cands[k]["dm"]) == dm_min)
        snr_hi = max(float(cands[k]["snr"]) for k in ks if float(cands[k]["dm"]) == dm_max)
        snr_max = float(c0["snr"])
        if float(c0["dm"]) < RFI_DM:
            rank = 2
        elif len(trials) < 3:
            rank = 1
        else:
            f = min(1.0 - snr_lo / snr_max, 1.0 - snr_hi / snr_max)
            rank = 3 if f < FALLOFF[0] else (4 if f < FALLOFF[1] else (5 if f < FALLOFF[2] else 6))
        out.append({"rep": r, "seg": int(c0["seg"]), "n_events": len(ks), "n_trials": len(trials),
                    "dm_min": dm_min, "dm_max": dm_max, "dm_peak": float(c0["dm"]), "snr_max": snr_max,
                    "snr_lo": snr_lo, "snr_hi": snr_hi, "time_s": float(c0["time_s"]),
                    "width_s": int(c0["width"]) * D * tsamp, "start_s": start, "duration_s": end - start,
                    "rank": rank})
    return out
