"""Nested-loop restatement of the search for tiny inputs (oracle; test infrastructure).

Every quantity is formed by explicit Python loops over scalars, directly from
the definitions in `search` (section 2.2 of the paper), with no array
operations, so that the vectorised oracle can be checked against it on cubes
of a few pixels, sub-bands and tens of samples.
"""
import math


def dedisperse_boxcar_brute(z, delays, widths):
    """z: nested lists z[t][s][p] of floats. Returns (smax, toa) as nested lists [d][w][p]."""
    nt, ns, npix = len(z), len(z[0]), len(z[0][0])
    nd, nw = len(delays), len(widths)
    smax = [[[-math.inf] * npix for _ in range(nw)] for _ in range(nd)]
    toa = [[[-1] * npix for _ in range(nw)] for _ in range(nd)]
    for d in range(nd):
        dmax = max(delays[d])
        for iw in range(nw):
            w = widths[iw]
            for p in range(npix):
                best, best_t = -math.inf, -1
                t = 0
                while t + w - 1 + dmax <= nt - 1:
                    total = 0.0
                    for k in range(w):
                        for s in range(ns):
                            total += z[t + k + delays[d][s]][s][p]
                    snr = total / math.sqrt(ns * w)
                    if snr > best:
                        best, best_t = snr, t
                    t += 1
                smax[d][iw][p] = best
                toa[d][iw][p] = best_t
    return smax, toa


def best_brute(smax, toa):
    nd, nw, npix = len(smax), len(smax[0]), len(smax[0][0])
    out = []
    for p in range(npix):
        b, bd, bw, bt = -math.inf, -1, -1, -1
        for d in range(nd):
            for w in range(nw):
                if smax[d][w][p] > b:
                    b, bd, bw, bt = smax[d][w][p], d, w, toa[d][w][p]
        out.append((b, bd, bw, bt))
    return out


def median_brute(vals):
    v = sorted(float(a) for a in vals)
    n = len(v)
    if n % 2:
        return v[n // 2]
    return (v[n // 2 - 1] + v[n // 2]) / 2.0
