"""PSF-based reduction of an image's top candidates (oracle; test infrastructure).

Section 2.3 of the paper: the simulated PSF is thresholded at its 90th
percentile into a binary mask; the mask is centred on each of the top
candidates in turn, that candidate taken as the central lobe and every other
candidate inside the mask as a possible sidelobe; the weighted mean S/N over
the central and sidelobe candidates is computed; the candidate whose weighted
mean S/N is largest is the final one.

Readings (the paper does not give them):
  * the weights are the PSF's amplitude at each member's offset from the
    central candidate (1 for the central one), the PSF normalised to its centre;
  * "weighted mean S/N" is read as the S/N of the weighted mean of the members'
    S/N values: each S/N carries unit noise, so the weighted mean
    sum(w S) / sum(w) has noise sqrt(sum(w^2)) / sum(w), and its S/N is
    sum(w S) / sqrt(sum(w^2)) (the PSF-matched filter over the candidates).
    A point source then scores highest on its own pixel (its sidelobes' S/N
    scale with w). The plain mean sum(w S) / sum(w) was tried first: sidelobes
    pull the source's mean down, and on simulated snapshot beams it kept a
    sidelobe in most images, against the paper's report that off-axis picks
    are a small fraction;
  * the percentile is NumPy's default (linear interpolation between order
    statistics) over every PSF pixel, and the mask keeps pixels >= it;
  * an offset outside the PSF image is outside the mask;
  * ties go to the earlier candidate in the list (the higher S/N).
"""
import numpy as np


def psf_reduce(cands, psf, percentile=90.0):
    """cands: sequence of (x, y, snr); psf: [2hy+1][2hx+1], centre at (hx, hy).
    Returns (index of the final candidate, the S/N of its weighted mean)."""
    psf = np.asarray(psf, dtype=np.float64)
    hy, hx = psf.shape[0] // 2, psf.shape[1] // 2
    w = psf / psf[hy, hx]
    q = np.percentile(psf, percentile)
    best_i, best_s = -1, -np.inf
    for i, (xi, yi, si) in enumerate(cands):
        weights, snrs = [1.0], [float(si)]
        for j, (xj, yj, sj) in enumerate(cands):
            if j == i:
                continue
            dx, dy = xj - xi, yj - yi
            if abs(dx) > hx or abs(dy) > hy:
                continue
            if psf[hy + dy, hx + dx] >= q:
                weights.append(float(w[hy + dy, hx + dx]))
                snrs.append(float(sj))
        wv, sv = np.array(weights), np.array(snrs)
        mean = (wv * sv).sum() / wv.sum()                 # weighted mean of the S/N values
        noise = np.sqrt((wv * wv).sum()) / wv.sum()       # its noise (each S/N has unit noise)
        score = mean / noise
        if score > best_s:
            best_i, best_s = i, score
    return best_i, best_s
