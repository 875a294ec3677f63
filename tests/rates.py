"""Exponential rates of the electric energy from its peaks (the paper's
damping/growth-rate fits, Sec. 6.2 and 6.3), shared by the CPU and GPU
physics tests.  Test infrastructure only."""
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_golden(name):
    """key value pairs of a golden fixture (comment lines start with #)."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split()
            out[k] = float(v)
    return out


def peaks(t, E):
    i = [j for j in range(1, len(E) - 1) if E[j] > E[j - 1] and E[j] >= E[j + 1]]
    return np.asarray(t)[i], np.asarray(E)[i]


def trapping_growth_rate(t, E):
    """Growth rate of the field amplitude sqrt(E): least-squares slope of
    log E at the peaks from the minimum of the peak envelope on, halved."""
    tp, Ep = peaks(t, E)
    m = int(np.argmin(Ep))
    return 0.5 * np.polyfit(tp[m:], np.log(Ep[m:]), 1)[0]
