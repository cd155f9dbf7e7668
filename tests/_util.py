"""Shared test helpers (not collected by pytest)."""
import re
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(path=os.path.join(ROOT, "include", "gsp.h")):
    """Names of the functions declared in a C header."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(gsp_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def say(*a):
    """Progress line that reaches the log even if the process dies next."""
    print(*a, flush=True)


def match_candidates(gpu, ora, thr, tol=1e-5, trial_key=("seg", "dm_index")):
    """Candidate-list match rule.

    gpu: CAND_DTYPE array of the library; ora: oracle candidates with fields
    seg, trial, t_peak, t_first, t_last, width, snr.
    (i) every oracle run whose peak is above the tolerance band around the
    threshold overlaps a GPU run of the same trial, and the best such GPU peak
    has the same SNR within `tol` (relative); (ii) the same from the GPU side;
    (iii) where the peaks are matched, (t_peak, width) agree unless the two
    sides' peak SNRs are within `tol` of each other (a near tie).
    Returns the number of exactly matched peaks."""
    hi = thr * (1 + tol)

    def index(arr, seg_f, trial_f):
        d = {}
        for k in range(len(arr)):
            d.setdefault((int(arr[seg_f][k]), int(arr[trial_f][k])), []).append(k)
        return d

    gi = index(gpu, "seg", "dm_index")
    oi = index(ora, "seg", "trial")
    exact = 0
    for (s, t), ks in oi.items():
        for k in ks:
            o = ora[k]
            if o["snr"] < hi:
                continue
            cand = [j for j in gi.get((s, t), []) if gpu["t_last"][j] >= o["t_first"] and gpu["t_first"][j] <= o["t_last"]]
            assert cand, f"oracle candidate {o} has no GPU run"
            j = max(cand, key=lambda j: gpu["snr"][j])
            g = gpu[j]
            assert abs(float(g["snr"]) - o["snr"]) <= tol * abs(o["snr"]) + 1e-6, (g, o)
            if int(g["t_peak"]) == int(o["t_peak"]) and int(g["width"]) == int(o["width"]):
                exact += 1
    for (s, t), ks in gi.items():
        for j in ks:
            g = gpu[j]
            if g["snr"] < hi:
                continue
            cand = [k for k in oi.get((s, t), []) if ora["t_last"][k] >= g["t_first"] and ora["t_first"][k] <= g["t_last"]]
            assert cand, f"GPU candidate {g} has no oracle run"
    return exact


def oracle_cands_with_seg(ora_list):
    """Concatenate per-segment oracle candidate arrays adding a seg column."""
    import oracle
    dt = np.dtype([("seg", np.int32)] + [(n, oracle.CAND_DTYPE[n]) for n in oracle.CAND_DTYPE.names])
    rows = [(s, c) for s, c in ora_list]
    n = sum(len(c) for _, c in rows)
    out = np.zeros(n, dt)
    k = 0
    for s, c in rows:
        out["seg"][k:k + len(c)] = s
        for f in oracle.CAND_DTYPE.names:
            out[f][k:k + len(c)] = c[f]
        k += len(c)
    return out
