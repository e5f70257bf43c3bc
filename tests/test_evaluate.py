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


def test_z_test_batch_sigma_tails_and_mean_offset():
    # sigma of one estimate from K = 32 batches (31 degrees of freedom), the
    # other known: |z| > 3 occurs more often than for a normal variate, and
    # the t-adjusted bounds accept it; a 0.1 sigma offset of every voxel is a
    # mean z far beyond 3/sqrt(n)
    rng = np.random.default_rng(12)
    n, K = 40000, 32
    batches = rng.standard_normal((K, n))
    da = batches.mean(axis=0)
    sa = batches.std(axis=0, ddof=1) / math.sqrt(K)
    sb = np.full(n, 1.0 / math.sqrt(K))
    db = sb * rng.standard_normal(n)
    zt = E.z_test(da, sa, db, sb, ref_for_mask=np.ones(n), dof=K - 1)
    assert zt.passed, E.describe(zt)
    assert zt.frac_limit > 0.0027
    off = E.z_test(da + 0.1 * np.sqrt(sa ** 2 + sb ** 2), sa, db, sb, ref_for_mask=np.ones(n), dof=K - 1)
    assert not off.passed and abs(off.mean) > off.mean_limit
    # same streams: a variance far below one is accepted, above 1.25 is not
    same = E.z_test(da, sa, da + 0.01 * sa, sa, ref_for_mask=np.ones(n), dof=K - 1, same_streams=True)
    assert same.passed and same.var < 0.01
    wide = E.z_test(da, sa / 1.3, db, sb / 1.3, ref_for_mask=np.ones(n), dof=K - 1)
    assert not wide.passed and wide.var > 1.25


def test_z_test_mean_bound_with_correlated_voxels():
    # Every batch of an estimate shifts all voxels together by a common
    # amount (as one history deposits in many voxels): mean z then scatters
    # far more than 1/sqrt(n) between independent runs.  The bound from the
    # batches' own spread accepts such runs and still rejects a real offset.
    rng = np.random.default_rng(21)
    n, K, trials = 3000, 32, 40
    strict_fail = batch_fail = 0
    for _ in range(trials):
        runs = []
        for _ in range(2):
            b = 10.0 + 0.2 * rng.standard_normal((K, 1)) + rng.standard_normal((K, n))
            nk = np.full(K, 100.0)
            d = b.mean(axis=0)
            s = b.std(axis=0, ddof=1) / math.sqrt(K)
            runs.append((d, s, (b, nk)))
        (da, sa, ba), (db, sb, bb) = runs
        mask = np.ones(n)
        strict_fail += not E.z_test(da, sa, db, sb, ref_for_mask=mask, dof=K - 1).passed
        batch_fail += not E.z_test(da, sa, db, sb, ref_for_mask=mask, dof=K - 1, batches=(ba, bb)).passed
    assert strict_fail > trials // 2 and batch_fail <= 2, (strict_fail, batch_fail)
    (da, sa, ba), (db, sb, bb) = runs
    off = E.z_test(da + 0.25, sa, db, sb, ref_for_mask=np.ones(n), dof=K - 1,
                   batches=((ba[0] + 0.25, ba[1]), bb))
    assert not off.passed and abs(off.mean) > off.mean_limit


def test_batch_doses_match_the_dose():
    rng = np.random.default_rng(4)
    K, N = 8, 1003
    e = rng.random((K, 3, 4, 5))
    rho = np.full((3, 4, 5), 1.5)
    dk, nk = E.batch_doses(e, rho, (0.5, 0.5, 0.5), N, h0=5)
    assert nk.sum() == N and nk.max() - nk.min() <= 1
    assert nk[5 % K] == np.ceil(N / K)                      # the first history (5) is in batch 5
    d = (nk[:, None, None, None] * dk).sum(axis=0) / N
    want = e.sum(axis=0) / N * E.MEV_TO_J / (1.5 * 0.125 * 1e-3)
    assert np.allclose(d, want, rtol=1e-13)
