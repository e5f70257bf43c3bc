"""GPU: the paper's second and third geometries (Sec. III.A: a lung box in
water; tissue, lung and bone slabs) and the divergence-reduction settings of
its Table VI, through the C ABI.

* Parity against the FP64 oracle: 15 MeV electrons on the lung box and 15 MeV
  photons on the slabs, per-voxel z-test with the combined sigma on the same
  streams and on independent streams (the bar of the water tests); event
  counts within 6 sigma + 1% of the oracle's.  The voxels compared (above 10%
  of the maximum) are chosen from a separate GPU run with its own seed:
  choosing them by one of the estimates being compared favours voxels where
  that estimate ran high, which biases the mean z of independent runs.
* The base, compaction, pool and combined settings, and the engine default,
  give bit-identical doses and sigmas on both geometries for both particle
  types (each particle carries its own stream and tallies are integer sums);
  the integer energy ledger closes exactly in every run.
"""
import numpy as np
import pytest

from paper_1101_1245_amd import evaluate as E
from paper_1101_1245_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    from paper_1101_1245_amd import gpumcd
    return gpumcd


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("make,particle,n", [(I.lung_box, I.ELECTRON, 100_000),
                                             (I.tissue_lung_bone, I.PHOTON, 200_000)],
                         ids=["electron-lung-box", "photon-tissue-lung-bone"])
def test_geometry_matches_oracle(ctx, G, oracle, make, particle, n):
    w = make(particle, n_hist=n)
    print("\n%s n=%d seed=%d" % (w.name, n, w.seed), flush=True)
    d, s, st = G.run_workload(ctx, w)
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    ref, _, _ = G.run_workload(ctx, w, seed=101)                      # voxel mask only
    res = oracle.run_parallel(w.materials, w.phantom, w.source, w.physics, w.seed, n)
    do, so = oracle.dose(res, w.phantom)
    zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=w.physics.n_batches - 1, same_streams=True)
    assert zt.passed, (zt.n, zt.frac_over_3, zt.max_abs, zt.mean, zt.var)
    r2 = oracle.run_parallel(w.materials, w.phantom, w.source, w.physics, w.seed + 1, n)
    do2, so2 = oracle.dose(r2, w.phantom)
    zi = E.z_test(d, s, do2, so2, ref_for_mask=ref, dof=w.physics.n_batches - 1)
    assert zi.passed, (zi.n, zi.frac_over_3, zi.max_abs, zi.mean, zi.var)
    for k in ("n_e_steps", "n_photon_events", "n_secondaries", "n_hard"):
        a, b = st[k], res.stats[k]
        assert abs(a - b) < 6 * np.sqrt(b) + 0.01 * b, (k, a, b)


@pytest.mark.parametrize("make", [I.lung_box, I.tissue_lung_bone], ids=["lung-box", "tissue-lung-bone"])
@pytest.mark.parametrize("particle", [I.ELECTRON, I.PHOTON], ids=["electron", "photon"])
def test_divergence_settings_bit_identical(ctx, G, make, particle):
    w = make(particle, n_hist=20_000 if particle == I.ELECTRON else 60_000)
    print("\n%s n=%d" % (w.name, w.n_hist), flush=True)
    d0, s0, st0 = G.run_workload(ctx, w)
    assert st0["ledger_residual_lsb"] == 0
    for name, tuning in I.ABLATION_TUNINGS.items():
        d, s, st = G.run_workload(ctx, w, tuning=tuning)
        assert st["ledger_residual_lsb"] == 0, name
        assert np.array_equal(d0, d) and np.array_equal(s0, s), name
        for k in ("n_e_steps", "n_photon_events", "n_secondaries", "n_hard"):
            assert st[k] == st0[k], (name, k)
