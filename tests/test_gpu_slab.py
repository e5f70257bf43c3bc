"""GPU: the heterogeneous slab phantom against the FP64 oracle.

128^3 voxels of 0.25 cm: water 0-3 cm, bone (1.85 g/cm^3) 3-5 cm, lung
(0.26 g/cm^3) 5-12 cm, water beyond; 6 MeV photons, 10 x 10 cm field, the
full 4e7 histories on both sides (the oracle over the host cores, in worker
processes over disjoint history ranges).

Voxel masks and dose bands (each slab x dose above 50% and 10-50% of the
maximum) come from a separate GPU run with its own seed: choosing voxels by
the very estimates being compared favours voxels where one of them ran high.

* FP32 vs FP64 (GPU and oracle on the same 4e7 histories): the z-test passes,
  event counts agree within 1e-3, and in every band the GPU/oracle ratio of
  the band's summed dose is within 0.1% of 1 -- the stated FP32-vs-FP64
  error, printed per band with -s.
* Gamma 2%/2 mm (Eqs. 14-15) of the same-stream GPU dose against the
  oracle's, voxels above 10% of the maximum: at least 99% pass.  Histories
  whose FP32 and FP64 trajectories part after a flipped decision become
  independent samples; at 4e7 histories their voxel-to-voxel noise is well
  inside the 2% criterion.
* Statistical agreement (GPU on 4e7 other histories): the z-test with the
  t-adjusted bounds of the evaluation module.
* The integer ledger closes and no majorant is violated.
"""
import numpy as np
import pytest

from paper_1101_1245_amd import evaluate as E
from paper_1101_1245_amd import inputs as I

pytestmark = pytest.mark.gpu

SLABS = (("water 0-3 cm", 0.0, 3.0), ("bone 3-5 cm", 3.0, 5.0), ("lung 5-12 cm", 5.0, 12.0),
         ("water 12-32 cm", 12.0, 32.0))
BANDS = (("> 50%", 0.5, np.inf), ("10-50%", 0.1, 0.5))


def band_ratios(d, do, ref, voxel):
    """Per slab x dose band of ref: voxels and the ratio of summed doses d / do."""
    zc = (np.arange(d.shape[0]) + 0.5) * voxel
    rmax = ref.max()
    rows = []
    for name, z0, z1 in SLABS:
        zsel = ((zc >= z0) & (zc < z1))[:, None, None]
        for bname, lo, hi in BANDS:
            sel = zsel & (ref > lo * rmax) & (ref <= hi * rmax)
            n = int(sel.sum())
            rows.append((name, bname, n, float(d[sel].sum() / do[sel].sum()) if n else np.nan))
    return rows


def show(title, rows, zt):
    print("\n%s: z-test %s" % (title, E.describe(zt)))
    for name, bname, n, ratio in rows:
        print("  %-15s %-7s %7d voxels  sum ratio %.5f" % (name, bname, n, ratio))


N_FULL = 40_000_000


@pytest.fixture(scope="module")
def runs(oracle):
    from paper_1101_1245_amd import gpumcd as G
    w = I.slab_6mev()
    assert w.n_hist == N_FULL
    with G.Context(0) as ctx:
        ref, _, _ = G.run_workload(ctx, w, seed=101)                       # masks and bands only
        full = G.run_workload(ctx, w, seed=1)
        other = G.run_workload(ctx, w, seed=5)
    print("\nslab: GPU runs done; oracle on %d histories" % N_FULL, flush=True)
    r = oracle.run_parallel(w.materials, w.phantom, w.source, w.physics, 1, N_FULL, batches=False)
    do, so = oracle.dose(r, w.phantom)
    return w, ref, full, other, (do, so, r)


@pytest.mark.timeout(900)
def test_slab_fp32_vs_fp64_same_streams(runs):
    w, ref, (d, s, st), _, (do, so, r) = runs
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    assert st["n_hist"] == N_FULL
    for k in ("n_photon_events", "n_e_steps", "n_hard", "n_secondaries"):
        assert abs(st[k] - r.stats[k]) < 1e-3 * r.stats[k], k      # the same trajectories, up to FP32 flips
    zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=w.physics.n_batches - 1, same_streams=True)
    rows = band_ratios(d, do, ref, w.phantom.voxel[2])
    show("same 4e7 histories (FP32 - FP64)", rows, zt)
    assert zt.passed, E.describe(zt)
    for name, bname, n, ratio in rows:
        assert n >= 50 and abs(ratio - 1.0) < 1e-3, (name, bname, n, ratio)


@pytest.mark.timeout(900)
def test_slab_gamma_same_streams(runs):
    # gamma 2%/2 mm (Eqs. 14-15) of the GPU dose against the oracle's on the
    # same 4e7 histories, over voxels above 10% of the oracle's maximum
    w, ref, (d, s, st), _, (do, so, r) = runs
    g = E.gamma_index(do, d, w.phantom.voxel)
    p = E.precision_error(d, do)
    print("\nslab, same 4e7 histories: summed dose %+.2e, voxel |diff| mean %.2e max %.2e of D_max over %d voxels; "
          "gamma 2%%/2 mm pass %.5f, max %.3f" % (p.sum_rel, p.mean_abs, p.max_abs, p.n, g.pass_rate, g.gamma_max))
    assert g.pass_rate >= 0.99, (g.pass_rate, g.gamma_max, g.n_voxels)


@pytest.mark.timeout(900)
def test_slab_statistical_agreement(runs):
    w, ref, _, (d, s, st), (do, so, r) = runs
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=w.physics.n_batches - 1)
    show("independent 4e7 histories", band_ratios(d, do, ref, w.phantom.voxel[2]), zt)
    assert zt.passed, E.describe(zt)
    for k in ("n_photon_events", "n_e_steps", "n_secondaries"):
        assert abs(st[k] / r.stats[k] - 1.0) < 2e-3, (k, st[k], r.stats[k])
