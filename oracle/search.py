"""De-dispersion / boxcar / S/N / candidate search (oracle; test infrastructure).

Follows section 2.2 of the paper: median subtraction and noise normalisation
per pixel, incoherent de-dispersion of every pixel's time series over a grid
of DM trials with precomputed integer shifts, boxcar filtering over a set of
widths, conversion to S/N, the maximum S/N over time with its time of arrival
(TOA), and a threshold that yields candidates. Section 2.3: the S/N and TOA
maps for all pixels, widths and DM trials are kept, and post-processing takes
the ten highest-S/N candidates. Section 3.1: the survey threshold is 6 sigma.

The method reaches a result with a plain definition, so this module writes
that definition out in FP64:

  z[t][s][p]   = cast((x - med[p][s]) / sigma[p][s])        (FP64, then cast)
  D_d[t][p]    = sum_s z[t + delta[d][s]][s][p],   0 <= t < L_d
  L_d          = n_t - max_s delta[d][s]
  B_dw[t][p]   = sum_{k<w} D_d[t+k][p],            0 <= t <= L_d - w
  S_dw[t][p]   = B_dw[t][p] / sqrt(n_sub * w)
  snr_max      = max_t S_dw,  toa = smallest t attaining it
  best[p]      = max over (d, w) of snr_max, ties to smallest d, then w
  candidates   = pixels with best >= theta, sorted by (-S/N, p), first K

Readings taken where the paper is open (each also listed in the design notes):
  * sigma scales the MAD to a Gaussian sigma (see `stats`); S/N divides the
    boxcar sum by sqrt(n_sub * w), the noise of a sum of n_sub*w unit-sigma
    samples, instead of a running standard deviation of the filtered series.
  * only windows that lie wholly inside the cube are searched (no wrap, no
    zero padding); a trial with no such window has snr_max = -inf, toa = -1.
  * the threshold is inclusive (S/N >= theta).
  * one candidate per pixel: its best (d, w) and that trial's TOA.
  * cast chain: FP64 -> FP32 (round to nearest even) -> FP16 / BF16 (round to
    nearest even from the FP32 value).
  * a series whose statistics are not usable (sigma == 0 or not finite, or a
    non-finite sample in it) is written as z = 0 and counted as flagged.
"""
import numpy as np

from .delays import delay_table
from .stats import robust_stats

STORE_DTYPES = ("f32", "f16", "bf16")


# ---------------------------------------------------------------- casting
def round_f32_to_bf16(x32):
    """Round FP32 values to BF16, nearest even; returned as float32 values.

    BF16 keeps the top 16 bits of an FP32 word. Rounding to nearest even adds
    0x7FFF plus the lowest kept bit before truncation; NaNs stay NaN.
    """
    a = np.ascontiguousarray(np.asarray(x32, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), np.float32(np.nan), out)


def cast_store(z64, store):
    """FP64 -> stored dtype; returns the stored values as exact float64.
    store "f64" keeps z unquantised (the reference for the precision forms)."""
    if store == "f64":
        return np.asarray(z64, dtype=np.float64)
    z32 = np.asarray(z64, dtype=np.float64).astype(np.float32)
    if store == "f32":
        return z32.astype(np.float64)
    if store == "f16":
        return z32.astype(np.float16).astype(np.float64)
    if store == "bf16":
        return round_f32_to_bf16(z32).astype(np.float64)
    raise ValueError(f"unknown store dtype {store!r}")


# ---------------------------------------------------------- normalisation
def normalize(cube_tsp, norm="pixel_subband", store="f32", med=None, sigma=None):
    """Raw cube [t][s][p] -> (z as FP64 values of the stored dtype, med, sigma, n_flagged).

    norm: 'pixel_subband' | 'pixel' | 'external' | 'none'.
    'external' takes med/sigma ([n_pix][n_sub], FP64) from the caller.
    """
    x = np.asarray(cube_tsp)
    x64 = x.astype(np.float64)
    nt, ns, npix = x.shape
    finite = np.isfinite(x64)
    if norm == "none":
        z = np.where(finite, x64, 0.0)
        return cast_store(z, store), None, None, int((~finite).sum())
    if norm in ("pixel_subband", "pixel"):
        bad_series = ~finite.all(axis=0)                     # [s][p]
        if norm == "pixel":
            bad_series = np.broadcast_to(bad_series.any(axis=0)[None], bad_series.shape)
        xs = np.where(finite, x64, 0.0)
        med, sig = robust_stats(xs, norm)                     # [p][s]
        med = np.where(bad_series.T, np.nan, med)
        sig = np.where(bad_series.T, np.nan, sig)
    elif norm == "external":
        med = np.asarray(med, dtype=np.float64).reshape(npix, ns)
        sig = np.asarray(sigma, dtype=np.float64).reshape(npix, ns)
    else:
        raise ValueError(f"unknown normalisation {norm!r}")
    usable = np.isfinite(med) & np.isfinite(sig) & (sig > 0)   # [p][s]
    m = np.where(usable, med, 0.0).T[None]                      # [1][s][p]
    sg = np.where(usable, sig, 1.0).T[None]
    z = (x64 - m) / sg
    ok = usable.T[None] & finite
    if norm == "external":
        z = np.where(ok, z, 0.0)
        n_flag = int((~usable).sum()) + int((usable.T[None] & ~finite).sum())
    else:
        z = np.where(usable.T[None], z, 0.0)
        n_flag = int((~usable).sum())
    return cast_store(z, store), med, sig, n_flag


# --------------------------------------------------------- de-dispersion
def dedisperse(z_tsp, delays):
    """Shift-and-sum over sub-bands. Returns list over d of D_d[t][p] (FP64)."""
    z = np.asarray(z_tsp, dtype=np.float64)
    nt, ns, npix = z.shape
    out = []
    for d in range(delays.shape[0]):
        dmax = int(delays[d].max())
        L = nt - dmax
        if L <= 0:
            out.append(np.zeros((0, npix)))
            continue
        acc = np.zeros((L, npix))
        for s in range(ns):
            sh = int(delays[d, s])
            acc += z[sh:sh + L, s, :]
        out.append(acc)
    return out


# ----------------------------------------------------------------- boxcar
def boxcar_sums(D_tp, w):
    """B[t][p] = sum_{k<w} D[t+k][p] for 0 <= t <= L - w, by an FP64 running sum."""
    L = D_tp.shape[0]
    if L - w + 1 <= 0:
        return np.zeros((0, D_tp.shape[1]))
    P = np.zeros((L + 1, D_tp.shape[1]))
    P[1:] = np.cumsum(D_tp, axis=0)
    return P[w:] - P[:-w]


def snr_series(D_tp, w, n_sub):
    """S/N time series for one (DM, width): boxcar sum / sqrt(n_sub * w)."""
    return boxcar_sums(D_tp, w) / np.sqrt(np.float64(n_sub) * np.float64(w))


def snr_toa_maps(z_tsp, delays, widths):
    """snr_max[d][w][p] (FP64, -inf if no window) and toa[d][w][p] (int32, -1)."""
    z = np.asarray(z_tsp, dtype=np.float64)
    nt, ns, npix = z.shape
    nd, nw = delays.shape[0], len(widths)
    smax = np.full((nd, nw, npix), -np.inf)
    toa = np.full((nd, nw, npix), -1, dtype=np.int32)
    for d, D in enumerate(dedisperse(z, delays)):
        for iw, w in enumerate(widths):
            S = snr_series(D, int(w), ns)
            if S.shape[0] == 0:
                continue
            smax[d, iw] = S.max(axis=0)
            toa[d, iw] = np.argmax(S, axis=0).astype(np.int32)  # first maximum
    return smax, toa


# ------------------------------------------------------------- candidates
def best_per_pixel(smax, toa):
    """Best (d, w) per pixel by S/N; ties to the smallest d, then smallest w."""
    nd, nw, npix = smax.shape
    flat = smax.reshape(nd * nw, npix)          # row index = d * nw + w
    idx = np.argmax(flat, axis=0)               # first maximum in (d, w) order
    best = flat[idx, np.arange(npix)]
    valid = np.isfinite(best)
    bd = np.where(valid, idx // nw, -1).astype(np.int32)
    bw = np.where(valid, idx % nw, -1).astype(np.int32)
    bt = np.where(valid, toa.reshape(nd * nw, npix)[idx, np.arange(npix)], -1).astype(np.int32)
    return best, bd, bw, bt


def candidates(best, bd, bw, bt, nx, theta, k_max):
    """Pixels with best >= theta, sorted by (-S/N, p); returns (list, n_total)."""
    sel = np.nonzero(np.isfinite(best) & (best >= theta))[0]
    order = sorted(sel.tolist(), key=lambda p: (-best[p], p))
    recs = [dict(x=int(p % nx), y=int(p // nx), dm_index=int(bd[p]),
                 width_index=int(bw[p]), toa=int(bt[p]), snr=float(best[p]))
            for p in order[:k_max]]
    return recs, len(sel)


# ------------------------------------------------------------ full search
def search(cube_tsp, freqs_ghz, f_ref_ghz, dt_ms, dms, widths, nx,
           norm="pixel_subband", store="f32", theta=6.0, k_max=10,
           med=None, sigma=None, k_dm_ms=4.15):
    """The whole search on a raw cube [t][s][p]. Returns a dict of results."""
    delays = delay_table(freqs_ghz, f_ref_ghz, dt_ms, dms, k_dm_ms)
    z, m, sg, nflag = normalize(cube_tsp, norm, store, med, sigma)
    smax, toa = snr_toa_maps(z, delays, widths)
    best, bd, bw, bt = best_per_pixel(smax, toa)
    cands, ntot = candidates(best, bd, bw, bt, nx, theta, k_max)
    return dict(delays=delays, z=z, med=m, sigma=sg, n_flagged=nflag,
                snr_max=smax, toa=toa, best=best, best_d=bd, best_w=bw,
                best_toa=bt, candidates=cands, n_total=ntot)


def snr_toa_margin_maps(z_tsp, delays, widths):
    """Like `snr_toa_maps`, plus the gap between the best and the second-best
    S/N over time (inf where only one window exists, nan where none)."""
    z = np.asarray(z_tsp, dtype=np.float64)
    nt, ns, npix = z.shape
    nd, nw = delays.shape[0], len(widths)
    smax = np.full((nd, nw, npix), -np.inf)
    toa = np.full((nd, nw, npix), -1, dtype=np.int32)
    margin = np.full((nd, nw, npix), np.nan)
    for d, D in enumerate(dedisperse(z, delays)):
        for iw, w in enumerate(widths):
            S = snr_series(D, int(w), ns)
            if S.shape[0] == 0:
                continue
            smax[d, iw] = S.max(axis=0)
            t = np.argmax(S, axis=0)
            toa[d, iw] = t.astype(np.int32)
            if S.shape[0] == 1:
                margin[d, iw] = np.inf
            else:
                S2 = S.copy()
                S2[t, np.arange(npix)] = -np.inf
                margin[d, iw] = smax[d, iw] - S2.max(axis=0)
    return smax, toa, margin


def trial_margin(smax):
    """Per pixel, the gap between the best and the second-best snr_max over all
    (DM, width) trials: inf where one trial alone has a window (or there is one
    trial in all), nan where no trial has one. Decides where the best trial is
    unambiguous."""
    nd, nw, npix = smax.shape
    if nd * nw == 1:
        return np.full(npix, np.inf)
    flat = np.where(np.isfinite(smax), smax, -np.inf).reshape(nd * nw, npix)
    top2 = np.sort(flat, axis=0)[-2:]
    out = np.full(npix, np.nan)
    ok = np.isfinite(top2[1])
    out[ok] = top2[1][ok] - top2[0][ok]          # second best -inf: inf
    return out


def bin_time(cube_tsp, factor):
    """Time binning for the longer search timescales (section 2.2: the images
    are also searched binned by 5 and by 75 samples).

    out[t'][s][p] = x[t' f][s][p] + ... + x[t' f + f - 1][s][p], added in FP64
    in that order and rounded once to FP32, for t' < n_t // f; a trailing
    partial bin is dropped (reading: the paper bins whole groups of samples).
    """
    x = np.asarray(cube_tsp)
    f = int(factor)
    nb = x.shape[0] // f
    acc = np.zeros((nb,) + x.shape[1:], dtype=np.float64)
    for k in range(f):
        acc = acc + x[k:nb * f:f].astype(np.float64)
    return acc.astype(np.float32)


def multiscale_search(cube_tsp, freqs_ghz, f_ref_ghz, dt_ms, dms, widths, nx, factors, dm_scales,
                      **kw):
    """The search at several timescales (section 2.2): timescale i bins the raw
    cube by factors[i] and searches it with dt * factors[i] and the DM trials
    times dm_scales[i], or DM 0 alone when dm_scales[i] == 0 (the longest
    timescale bypasses de-dispersion). Returns one `search` result per
    timescale."""
    out = []
    for f, k in zip(factors, dm_scales):
        xb = np.asarray(cube_tsp) if f == 1 else bin_time(cube_tsp, f)
        d = np.zeros(1) if k == 0 else np.asarray(dms, dtype=np.float64) * k
        out.append(search(xb, freqs_ghz, f_ref_ghz, dt_ms * f, d, widths, nx, **kw))
    return out
