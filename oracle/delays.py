"""Dispersion delay table (oracle; test infrastructure).

Paper section 2.2: the cold-plasma delay between two frequencies is
4.15 ms * DM * (nu_lo^-2 - nu_hi^-2) with nu in GHz (this is the law inside
the t_BW definition that precedes Eq. 2). The search precomputes integer
shift indices per channel and keeps them resident on the GPU (section 2.2 and
its footnote on reusing the table at 5x coarser sampling).

Reading taken here (open in the paper): each sub-band is referenced to the
highest frequency f_ref, so all delays are >= 0, and a delay in samples is the
FP64 value of  k * DM * (1/(f*f) - 1/(f_ref*f_ref)) / dt  evaluated left to
right, rounded half-to-even.
"""
import numpy as np

K_DM_MS = 4.15  # ms GHz^2 cm^3 / pc, the constant printed in section 2.2


def delay_samples_real(freqs_ghz, f_ref_ghz, dt_ms, dms, k_dm_ms=K_DM_MS):
    """Unrounded delays in samples, shape [n_dm, n_sub], FP64.

    Evaluated in the fixed order ((k*DM) * (1/(f*f) - 1/(fr*fr))) / dt.
    """
    f = np.asarray(freqs_ghz, dtype=np.float64)
    dm = np.asarray(dms, dtype=np.float64)
    fr = np.float64(f_ref_ghz)
    inv = 1.0 / (f * f) - 1.0 / (fr * fr)          # [n_sub]
    kd = np.float64(k_dm_ms) * dm                   # [n_dm]
    return (kd[:, None] * inv[None, :]) / np.float64(dt_ms)


def delay_table(freqs_ghz, f_ref_ghz, dt_ms, dms, k_dm_ms=K_DM_MS):
    """Integer delay table delta[d][s] (int32), rounded half to even."""
    real = delay_samples_real(freqs_ghz, f_ref_ghz, dt_ms, dms, k_dm_ms)
    return np.rint(real).astype(np.int32)
