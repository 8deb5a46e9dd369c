"""Exact binary32 helpers for the independent checks (numpy, no oracle code)."""
import numpy as np


def fmaf(a, b, c):
    """Correctly rounded binary32 a*b + c.  The binary64 product of two binary32
    values is exact; the binary64 sum is corrected with TwoSum so that a value
    that lands exactly on a binary32 midpoint is nudged towards the true sum."""
    a = np.asarray(a, np.float32).astype(np.float64)
    b = np.asarray(b, np.float32).astype(np.float64)
    c = np.asarray(c, np.float32).astype(np.float64)
    p = a * b
    s = p + c
    bb = s - p
    e = (p - (s - bb)) + (c - bb)
    r = s.astype(np.float32)
    # midpoint test: s exactly halfway between two binary32 neighbours
    lo = np.where(r.astype(np.float64) <= s, r, np.nextafter(r, np.float32(-np.inf)))
    hi = np.nextafter(lo, np.float32(np.inf))
    mid = (lo.astype(np.float64) + hi.astype(np.float64)) * 0.5
    fix = (e != 0) & (s == mid) & np.isfinite(s)
    if np.any(fix):
        s2 = np.where(fix, np.nextafter(s, s + e), s)
        r = np.where(fix, s2.astype(np.float32), r)
    return r.astype(np.float32)
