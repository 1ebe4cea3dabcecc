"""Generalised multi-time-scale integrator schedule (FP64 oracle).

Test infrastructure only (see ``oracle/__init__.py``).

Sec. 3.2: with a single kind of time step T[h] moving monotonically from 0 to
tau, each action term i gets its own second-order scheme for H_i = T + S_i;
the schemes are overlaid by placing every S_i[w] update at its own time t and
applying T[dt] for the gaps between consecutive distinct times.  The paper's
worked example (a two-step and a three-step leapfrog) is reproduced by
``merge`` exactly (see the golden test).

Per-term schemes (times and weights in units of tau):

* leapfrog (Sec. 3.2): S[h/2] T[h] S[h/2] per step, h = 1/n: weight h/2 at
  t = 0 and t = 1, h at interior step boundaries;
* Omelyan (the HMC workload asks for it; not in the paper):
  S[lam h] T[h/2] S[(1-2 lam) h] T[h/2] S[lam h] per step: weight lam h at the
  ends, 2 lam h at interior step boundaries, (1 - 2 lam) h at step midpoints.

Updates at one time commute (each only changes P using the current U).  The
order among them is chosen mirror-symmetric: ascending term index before the
midpoint, descending after it (the paper's example has this order).
"""
from __future__ import annotations

from fractions import Fraction

OMELYAN_LAMBDA = 0.1931833275037836


def scheme_events(kind: str, n: int, lam: float = OMELYAN_LAMBDA):
    """List of (time, weight) for one term, time a Fraction of tau."""
    ev = []
    h = Fraction(1, n)
    if kind == "leapfrog":
        ev.append((Fraction(0), h / 2))
        for k in range(1, n):
            ev.append((k * h, h))
        ev.append((Fraction(1), h / 2))
    elif kind == "omelyan":
        hf = 1.0 / n
        ev.append((Fraction(0), lam * hf))
        for k in range(n):
            ev.append((k * h + h / 2, (1 - 2 * lam) * hf))
            if k < n - 1:
                ev.append(((k + 1) * h, 2 * lam * hf))
        ev.append((Fraction(1), lam * hf))
    else:
        raise ValueError(kind)
    return ev


def merge(schemes):
    """Overlay per-term schemes.

    ``schemes``: list over terms of (time, weight) lists.  Returns a list of
    ('S', term, weight) and ('T', dt) steps, times and weights in units of tau.
    """
    by_time = {}
    for i, ev in enumerate(schemes):
        for t, w in ev:
            by_time.setdefault(t, []).append((i, w))
    out = []
    prev = Fraction(0)
    for t in sorted(by_time):
        if t > prev:
            out.append(("T", t - prev))
            prev = t
        group = sorted(by_time[t], key=lambda iw: iw[0], reverse=(2 * t > 1))
        for i, w in group:
            out.append(("S", i, w))
    if prev < 1:
        out.append(("T", Fraction(1) - prev))
    return out
