"""Robust noise statistics (oracle; test infrastructure).

Paper section 2.2: the data are median-subtracted in each pixel before the
search and the filtered series are normalised by a noise estimate. Section
3.2 notes that a plain (non-robust) instantaneous noise estimate is biased
high by wide (8-16 sample) pulses, which lowers their S/N. The reading taken
here: the noise of each series is the median absolute deviation scaled to a
Gaussian standard deviation, sigma = MAD / Phi^-1(3/4).

Definitions (textbook, written out):
  median of n values sorted ascending as v_0..v_{n-1}:
      v_{(n-1)/2}                       if n is odd
      (v_{n/2-1} + v_{n/2}) / 2         if n is even  (FP64 add, then halve)
  MAD = median(|x - median(x)|), every difference formed in FP64.

Granularity (open in the paper, which says "in each pixel"):
  'pixel_subband'  one (median, sigma) per (pixel, sub-band) over time
  'pixel'          one (median, sigma) per pixel over (time, sub-band)
"""
import numpy as np

MAD_TO_SIGMA = 1.482602218505602  # 1 / Phi^-1(3/4), rounded to FP64


def median_fp64(values):
    """Median of a 1-D array, by the textbook definition, in FP64."""
    v = np.sort(np.asarray(values, dtype=np.float64).ravel(), kind="stable")
    n = v.size
    if n == 0:
        raise ValueError("median of an empty series")
    if n % 2 == 1:
        return np.float64(v[(n - 1) // 2])
    return np.float64((v[n // 2 - 1] + v[n // 2]) / 2.0)


def mad_fp64(values, med):
    """Median absolute deviation about `med` (FP64)."""
    x = np.asarray(values, dtype=np.float64).ravel()
    return median_fp64(np.abs(x - np.float64(med)))


def median_axis0(x):
    """Vectorised textbook median over axis 0 (FP64), same definition."""
    v = np.sort(np.asarray(x, dtype=np.float64), axis=0, kind="stable")
    n = v.shape[0]
    if n % 2 == 1:
        return v[(n - 1) // 2].copy()
    return (v[n // 2 - 1] + v[n // 2]) / 2.0


def robust_stats(cube_tsp, mode="pixel_subband"):
    """Median and sigma for a raw cube laid out [t][s][p].

    Returns (med, sigma), each float64 of shape [n_pix, n_sub]. In 'pixel'
    mode the per-pixel value is repeated across sub-bands.
    """
    x = np.asarray(cube_tsp)
    nt, ns, npix = x.shape
    x64 = x.astype(np.float64)
    if mode == "pixel_subband":
        med = median_axis0(x64)                       # [s][p]
        mad = median_axis0(np.abs(x64 - med[None]))   # [s][p]
        sig = MAD_TO_SIGMA * mad
        return med.T.copy(), sig.T.copy()
    if mode == "pixel":
        flat = x64.reshape(nt * ns, npix)             # rows ordered (t, s)
        med = median_axis0(flat)                      # [p]
        mad = median_axis0(np.abs(flat - med[None]))
        sig = MAD_TO_SIGMA * mad
        return (np.repeat(med[:, None], ns, axis=1),
                np.repeat(sig[:, None], ns, axis=1))
    raise ValueError(f"unknown statistics mode {mode!r}")
