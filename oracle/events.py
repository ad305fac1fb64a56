"""Event detection oracle: raw nanopore samples -> events (TEST INFRASTRUCTURE
ONLY; the same rules as the package doc of ``oracle``).

Section 4.1 (software processing layer) segments each read's raw samples
into events before normalisation, to shrink the query; section 5.2 takes the
R9.4 event-detection parameters from f5c and nanopolish, whose detector is a
two-window t-test.  The paper prints neither the algorithm nor its numbers,
so this module follows a reading of that detector, stated in full.  Parity
unpinned against the paper: nothing the paper prints fixes these events;
the tests pin the reading itself (hand-worked detector traces, window
statistics against closed forms).

1. t statistic at every boundary position i (between samples i-1 and i), for
   a window length w: with m1, v1 the mean and population variance of
   x[i-w .. i-1] and m2, v2 those of x[i .. i+w-1],
       t_w(i) = |m2 - m1| / max(sqrt((v1 + v2) / w), 1e-30)
   for w <= i <= L - w, else 0.  Sums run in index order in float64 (means
   first, then the squared deviations).
2. Two peak detectors, short (w = 3, threshold 1.4) and long (w = 6,
   threshold 9.0), peak height 0.2, scan i = 0 .. L-1, short first at each
   i.  A detector skips positions up to its mask.  Without a candidate it
   tracks the running minimum of t and opens a candidate at i once t rises
   more than the peak height above it.  With a candidate it moves the
   candidate to any higher t; while the short detector's candidate exceeds
   its threshold, the long detector is masked up to (candidate + 6) and its
   own candidate dropped; a candidate above its threshold becomes valid once
   t has fallen more than the peak height below it, and a valid candidate is
   emitted as an event boundary once i is more than w / 2 (integer) past
   it; the detector then restarts from the current t.
3. Events are the segments between consecutive distinct boundaries (with 0
   and L as the outer ends); an event's value is the float32 rounding of
   the float64 mean of its samples (summed in index order).
4. Prefix trimming (section 4.1's footnote: the first events of a read
   belong to the adaptor): the first ``trim`` events are dropped and the
   next ``keep`` returned.

Everything is plain Python over float64 values, written for clarity, not
speed (reads of a few thousand samples).
"""
from __future__ import annotations

import math

import numpy as np

W_SHORT, W_LONG = 3, 6
T_SHORT, T_LONG = 1.4, 9.0
PEAK_HEIGHT = 0.2
DEN_FLOOR = 1e-30


def tstat(x, w: int) -> np.ndarray:
    """t_w(i) for i = 0 .. L-1 (step 1 of the module doc)."""
    v = [float(a) for a in np.asarray(x, np.float32)]
    L = len(v)
    t = np.zeros(L, np.float64)
    for i in range(w, L - w + 1):
        s1 = 0.0
        s2 = 0.0
        for k in range(w):
            s1 += v[i - w + k]
            s2 += v[i + k]
        m1 = s1 / w
        m2 = s2 / w
        q1 = 0.0
        q2 = 0.0
        for k in range(w):
            d1 = v[i - w + k] - m1
            d2 = v[i + k] - m2
            q1 += d1 * d1
            q2 += d2 * d2
        v1 = q1 / w
        v2 = q2 / w
        den = max(math.sqrt((v1 + v2) / w), DEN_FLOOR)
        t[i] = abs(m2 - m1) / den
    return t


class _Detector:
    def __init__(self, t, w, threshold):
        self.t, self.w, self.threshold = t, w, threshold
        self.masked_to = -1
        self.peak_pos = -1
        self.peak_val = math.inf
        self.valid = False


def boundaries(x) -> list[int]:
    """Sorted distinct event boundaries of raw samples x (steps 1 and 2)."""
    return peaks(tstat(x, W_SHORT), tstat(x, W_LONG))


def peaks(t_short, t_long) -> list[int]:
    """Step 2 of the module doc on given t statistics of both detectors."""
    short = _Detector(np.asarray(t_short, np.float64), W_SHORT, T_SHORT)
    long_ = _Detector(np.asarray(t_long, np.float64), W_LONG, T_LONG)
    found = []
    L = len(short.t)
    for i in range(L):
        for det in (short, long_):
            if det.masked_to >= i:
                continue
            v = float(det.t[i])
            if det.peak_pos < 0:
                if v < det.peak_val:
                    det.peak_val = v
                elif v - det.peak_val > PEAK_HEIGHT:
                    det.peak_val = v
                    det.peak_pos = i
                continue
            if v > det.peak_val:
                det.peak_val = v
                det.peak_pos = i
            if det is short and det.peak_val > det.threshold:
                long_.masked_to = det.peak_pos + long_.w
                long_.peak_pos = -1
                long_.peak_val = math.inf
                long_.valid = False
            if det.peak_val - v > PEAK_HEIGHT and det.peak_val > det.threshold:
                det.valid = True
            if det.valid and i - det.peak_pos > det.w // 2:
                found.append(det.peak_pos)
                det.peak_pos = -1
                det.peak_val = v
                det.valid = False
    return sorted(set(found))


def events(x) -> np.ndarray:
    """Event values (float32) of a whole read (step 3)."""
    v = [float(a) for a in np.asarray(x, np.float32)]
    if not v:
        return np.zeros(0, np.float32)  # no samples, no segment
    cuts = [0] + [b for b in boundaries(x) if 0 < b < len(v)] + [len(v)]
    out = []
    for a, b in zip(cuts[:-1], cuts[1:]):
        s = 0.0
        for k in range(a, b):
            s += v[k]
        out.append(s / (b - a))
    return np.asarray(out, np.float64).astype(np.float32)


def query_events(x, trim: int = 50, keep: int = 250) -> np.ndarray:
    """Events trim .. trim+keep-1 of a read (step 4); fewer if it has fewer."""
    return events(x)[trim:trim + keep]
