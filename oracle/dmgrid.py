"""DM-trial grid from a smearing tolerance (oracle; test infrastructure).

Section 2.2 of the paper searches DM trials chosen with a "DM tolerance" and
models a pulse's effective width as the quadrature sum of its intrinsic
width W_int, the sampling time t_s, the dispersive smearing inside the
lowest-frequency channel t_dnu = 0.0083 ms * dnu_MHz * DM * nu_min^-3 and the
residual delay across the band after de-dispersion to a trial,
t_BW = 4.15 ms * |DM - DM_trial| * (nu_min^-2 - nu_max^-2); the relative S/N
is sqrt(t_s / W_eff) (reading: the printed ratio is upside down, since the
text has the relative S/N falling below 60% at high DM).

Readings (the paper names the tolerance but gives no rule):
  * the worst-placed pulse sits midway between two trials; consecutive trials
    DM_i, DM_{i+1} = DM_i + 2h are spaced so that at DM_mid = DM_i + h the
    effective width with the residual delay of h exceeds the width without it
    by exactly the factor tol:  W_eff(DM_mid, h) = tol * W_eff(DM_mid, 0);
  * the grid starts at dm_min and ends with the first trial >= dm_max.

This module finds each spacing by bisection on that defining equation (the
library solves the equivalent quadratic in closed form).
"""
import math

K_DM_MS = 4.15          # dispersion delay constant, ms GHz^2 cm^3 / pc
K_CHAN_MS = 0.0083      # intra-channel smearing constant, ms GHz^3 / (MHz pc cm^-3)


def w_eff(dm, ddm, nu_min, nu_max, dnu_mhz, t_s, w_int):
    """Effective width (ms) of a pulse at `dm` searched at a trial `ddm` away."""
    t_dnu = K_CHAN_MS * dnu_mhz * dm * nu_min ** -3
    t_bw = K_DM_MS * abs(ddm) * (nu_min ** -2 - nu_max ** -2)
    return math.sqrt(w_int ** 2 + t_s ** 2 + t_dnu ** 2 + t_bw ** 2)


def snr_rel(dm, ddm, nu_min, nu_max, dnu_mhz, t_s, w_int):
    """S/N relative to a narrow pulse at DM 0 (the paper's Eq. 2, read as sqrt(t_s / W_eff))."""
    return math.sqrt(t_s / w_eff(dm, ddm, nu_min, nu_max, dnu_mhz, t_s, w_int))


def half_spacing(dm, nu_min, nu_max, dnu_mhz, t_s, w_int, tol):
    """h > 0 with w_eff(dm + h, h) = tol * w_eff(dm + h, 0), by bisection."""
    f = lambda h: (w_eff(dm + h, h, nu_min, nu_max, dnu_mhz, t_s, w_int)
                   - tol * w_eff(dm + h, 0.0, nu_min, nu_max, dnu_mhz, t_s, w_int))
    lo, hi = 0.0, 1.0
    while f(hi) < 0.0:
        hi *= 2.0
        if hi > 1e12:
            raise ValueError("the tolerance cannot be met (channel smearing grows faster than the residual delay)")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if f(mid) < 0.0:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def dm_grid(freqs_ghz, dnu_mhz, t_s, w_int, tol, dm_min, dm_max):
    """Trials dm_min = DM_0 < DM_1 < ... , the last the first one >= dm_max."""
    nu_min, nu_max = min(freqs_ghz), max(freqs_ghz)
    out = [float(dm_min)]
    while out[-1] < dm_max:
        out.append(out[-1] + 2.0 * half_spacing(out[-1], nu_min, nu_max, dnu_mhz, t_s, w_int, tol))
    return out
