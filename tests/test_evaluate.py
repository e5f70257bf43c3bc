"""The host-side dose evaluation (Sec. II.D) against closed forms.

* gamma (Eqs. 14-15): identical doses give 0 everywhere; a uniform offset of
  f x D_max on a flat field gives exactly f / 2% (no shift helps); a linear
  ramp of slope a shifted by delta has the continuous minimum
  gamma = delta / sqrt(dd^2 + (dD / a)^2), which the searched grid reaches
  from above within its spacing;
* s (Eq. 12) and the histories for 1% from s ~ 1/sqrt(N);
* the FP32-vs-FP64 precision summary on a known relative error;
* the z-test on Gaussian estimates with known sigma, and its failure on a
  5-sigma offset.
"""
import math

import numpy as np
import pytest

from paper_1101_1245_amd import evaluate as E

VOX = (0.25, 0.25, 0.25)   # cm (dx, dy, dz)


def test_gamma_identical_is_zero():
    rng = np.random.default_rng(3)
    d = rng.random((8, 9, 10)) + 0.5
    g = E.gamma_index(d, d.copy(), VOX)
    assert g.n_voxels == int(np.sum(d > 0.1 * d.max()))
    assert g.pass_rate == 1.0 and g.gamma_max == 0.0


@pytest.mark.parametrize("f", [0.01, 0.03])
def test_gamma_uniform_offset(f):
    ref = np.ones((6, 6, 6))
    g = E.gamma_index(ref, ref + f, VOX)
    assert np.allclose(g.gamma, f / 0.02, rtol=1e-12)
    assert g.pass_rate == (1.0 if f < 0.02 else 0.0)


def test_gamma_shifted_ramp_closed_form():
    nx = 40
    x = (np.arange(nx) + 0.5) * VOX[0]                 # voxel centres along x (cm)
    a = 0.5                                            # dose per cm, D_max = a * x[-1]
    delta = 0.08                                       # shift (cm), a multiple of the 0.04 cm search step
    ref = np.broadcast_to(a * x, (5, 5, nx)).copy()
    ev = np.broadcast_to(a * (x - delta), (5, 5, nx)).copy()
    g = E.gamma_index(ref, ev, VOX)
    sel = np.argwhere(ref > 0.1 * ref.max())
    dD = 0.02 * ref.max()
    exact = delta / math.sqrt(0.2 ** 2 + (dD / a) ** 2)
    # interior voxels, where neither the shift nor the search leaves the grid
    inner = (sel[:, 2] >= 4) & (sel[:, 2] <= nx - 5)
    gi = g.gamma[inner]
    assert np.all(gi >= exact - 1e-9)
    assert np.all(gi <= exact + 0.02), (gi.max(), exact)
    # a pure distance shift at a steep gradient tends to delta / 2 mm
    steep = E.gamma_index(ref * 100.0, ev * 100.0, VOX)
    assert steep.gamma[inner].max() <= delta / 0.2 + 1e-9


def test_uncertainty_s_and_histories():
    d = np.array([10.0, 5.0, 1.0, 0.5])
    s = np.array([0.2, 0.2, 0.5, 0.5])
    # voxels above 20% of D_max: 10 and 5, relative 0.02 and 0.04
    assert E.uncertainty_s(d, s) == pytest.approx(0.03)
    assert E.histories_for(0.02, 1000) == 4000
    assert E.efficiency(0.01, 2.0) == pytest.approx(5000.0)


def test_precision_error_known_offset():
    rng = np.random.default_rng(5)
    ref = rng.random((7, 7, 7)) + 1.0
    ev = ref * (1.0 + 1e-4)
    p = E.precision_error(ev, ref)
    assert p.n == ref.size
    assert p.sum_rel == pytest.approx(1e-4, rel=1e-9)
    assert p.max_abs == pytest.approx(1e-4, rel=1e-9)           # the maximum voxel carries the largest change
    assert p.mean_abs == pytest.approx(1e-4 * ref.mean() / ref.max(), rel=1e-9)


def test_z_test_gaussian_and_offset():
    rng = np.random.default_rng(11)
    shape = (20, 20, 20)
    mu = np.full(shape, 10.0)
    sa, sb = np.full(shape, 0.3), np.full(shape, 0.4)
    da = mu + sa * rng.standard_normal(shape)
    db = mu + sb * rng.standard_normal(shape)
    zt = E.z_test(da, sa, db, sb, dof=10 ** 6)
    assert zt.passed and zt.n == mu.size
    bad = E.z_test(da + 2.5, sa, db, sb, dof=10 ** 6)           # 5 combined sigma
    assert not bad.passed and bad.frac_over_3 > 0.9
