"""PSF-based reduction of an image's top candidates (oracle; test infrastructure).

Section 2.3 of the paper: the simulated PSF is thresholded at its 90th
percentile into a binary mask; the mask is centred on each of the top
candidates in turn, that candidate taken as the central lobe and every other
candidate inside the mask as a possible sidelobe; the weighted mean S/N over
the central and sidelobe candidates is computed; the candidate whose weighted
mean is largest is the final one.

Readings (the paper does not give them):
  * the weights are the PSF's amplitude at each member's offset from the
    central candidate (1 for the central one), the PSF normalised to its centre;
  * the percentile is NumPy's default (linear interpolation between order
    statistics) over every PSF pixel, and the mask keeps pixels >= it;
  * an offset outside the PSF image is outside the mask;
  * ties go to the earlier candidate in the list (the higher S/N).
"""
import numpy as np


def psf_reduce(cands, psf, percentile=90.0):
    """cands: sequence of (x, y, snr); psf: [2hy+1][2hx+1], centre at (hx, hy).
    Returns (index of the final candidate, its weighted mean S/N)."""
    psf = np.asarray(psf, dtype=np.float64)
    hy, hx = psf.shape[0] // 2, psf.shape[1] // 2
    w = psf / psf[hy, hx]
    q = np.percentile(psf, percentile)
    best_i, best_s = -1, -np.inf
    for i, (xi, yi, si) in enumerate(cands):
        num, den = float(si), 1.0
        for j, (xj, yj, sj) in enumerate(cands):
            if j == i:
                continue
            dx, dy = xj - xi, yj - yi
            if abs(dx) > hx or abs(dy) > hy:
                continue
            if psf[hy + dy, hx + dx] >= q:
                num += w[hy + dy, hx + dx] * float(sj)
                den += w[hy + dy, hx + dx]
        score = num / den
        if score > best_s:
            best_i, best_s = i, score
    return best_i, best_s
