"""Pins for the DM-grid oracle: closed forms without channel smearing, the
defining width ratio at every midpoint, monotone spacing, and the paper's
sensitivity statements (section 2.2)."""
import math

import numpy as np
import pytest

from oracle import dmgrid

NU = (1.311, 1.499)


def test_linear_grid_without_channel_smearing():
    """dnu = 0: h = sqrt(tol^2 - 1) * sqrt(t_s^2 + W_int^2) / (4.15 * (nu_min^-2 - nu_max^-2))."""
    for t_s, w_int, tol in ((134.2, 0.0, 1.6), (670.0, 50.0, 1.25), (10.0, 3.0, 2.0)):
        g = dmgrid.dm_grid(NU, 0.0, t_s, w_int, tol, 0.0, 5000.0)
        a = 4.15 * (NU[0] ** -2 - NU[1] ** -2)
        h = math.sqrt(tol * tol - 1.0) * math.hypot(t_s, w_int) / a
        np.testing.assert_allclose(np.diff(g), 2 * h, rtol=1e-12)
        assert g[-1] >= 5000.0 > g[-2]


def test_width_ratio_at_every_midpoint_is_the_tolerance():
    g = dmgrid.dm_grid(NU, 11.71875, 134.2, 6.6, 1.6, 0.0, 20000.0)
    for a, b in zip(g[:-1], g[1:]):
        mid, h = 0.5 * (a + b), 0.5 * (b - a)
        r = dmgrid.w_eff(mid, h, *NU, 11.71875, 134.2, 6.6) / dmgrid.w_eff(mid, 0.0, *NU, 11.71875, 134.2, 6.6)
        assert r == pytest.approx(1.6, rel=1e-12)


def test_spacing_grows_with_dm_when_channels_smear():
    g = np.array(dmgrid.dm_grid(NU, 11.71875, 134.2, 0.0, 1.6, 0.0, 20000.0))
    d = np.diff(g)
    assert (d[1:] > d[:-1]).all()


def test_relative_snr_is_one_at_dm0_and_falls_with_offset_and_width():
    """Eq. 2 (read as sqrt(t_s / W_eff)): 1 for a narrow pulse at DM 0 on its own trial, and
    strictly smaller for any residual DM offset, channel smearing or intrinsic width; at the
    grid's midpoints it is 1/sqrt(tol) of its on-trial value (the tolerance on width)."""
    f = lambda dm, ddm, w: dmgrid.snr_rel(dm, ddm, *NU, 11.71875, 134.2, w)
    assert f(0.0, 0.0, 0.0) == 1.0
    assert f(0.0, 50.0, 0.0) < 1.0 and f(500.0, 0.0, 0.0) < 1.0 and f(0.0, 0.0, 10.0) < 1.0
    g = dmgrid.dm_grid(NU, 11.71875, 134.2, 0.0, 1.6, 0.0, 4000.0)
    for a, b in zip(g[:-1], g[1:]):
        m = 0.5 * (a + b)
        assert f(m, 0.5 * (b - a), 0.0) == pytest.approx(f(m, 0.0, 0.0) / math.sqrt(1.6), rel=1e-12)
