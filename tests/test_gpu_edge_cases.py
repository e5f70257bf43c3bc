"""GPU: degenerate inputs of the transport (Secs. II.A-II.C) against the FP64
oracle, through the C ABI.

* A phantom of zero density: photons see a zero majorant (Eq. 3) and leave
  at once, electrons cross it voxel by voxel with no energy loss (Eq. 8 with
  rho = 0), no deflection and no hard event; nothing is deposited and the
  whole incident energy escapes, in the plain and the batched forms.
* Primary electrons below the cutoff deposit their whole energy in the voxel
  they enter; the GPU's per-voxel energy equals the oracle's, history for
  history.
* A vacuum gap between two water slabs: photons cross it as fictitious
  events only, electrons stream through it; not one unit of energy lands in
  the gap, and the doses on both sides agree with the oracle on the same
  streams (z-test) with event counts within 2e-3.
* The largest batch count accepted (n_batches = 1024): a run's 1024 batch
  tallies fold (k mod 32) into exactly those of the same run with 32 batches
  (history h in batch h mod K), the deposited energy is the same, the dose
  of the 1024-batch finalize equals the 32-batch one bit for bit, and Eq. 12's
  s of the two agree within 10%.
* The largest history count one call accepts (2^32 - 1): the plain form
  runs every history and closes the ledger; the batched form with the same
  histories split over two beams (the second starting at history 2^31) gives
  the same dose and sigma bit for bit; 2^32 histories are refused by both.
* The smallest and ragged grids (one voxel; 7 x 5 x 3 voxels, fewer than one
  finalize block and not a whole number of the tally's 16-voxel blocks, whose
  raw batch tallies finalize to the run's own dose and sigma) and the fewest
  histories allowed (n = n_batches), and
  beams at the largest energy accepted (30 MeV): the ledger closes exactly
  and the doses agree with the oracle.
"""
import dataclasses

import numpy as np
import pytest

from paper_1101_1245_amd import evaluate as E
from paper_1101_1245_amd import inputs as I

pytestmark = pytest.mark.gpu
LSB = 2.0 ** -27


@pytest.fixture(scope="module")
def G():
    from paper_1101_1245_amd import gpumcd
    return gpumcd


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def loaded(ctx, materials, phantom, physics):
    return ctx.load_tables(materials, physics), ctx.load_phantom(phantom)


def release(ctx, *ids):
    for i in ids:
        ctx.release(i)


@pytest.mark.parametrize("particle,e", [(I.PHOTON, 1.0), (I.ELECTRON, 15.0)], ids=["photon", "electron"])
def test_zero_density_phantom_deposits_nothing(ctx, G, oracle, particle, e):
    ph = I.homogeneous((8, 8, 8), 0.5, density=0.0)
    phys = I.Physics(ecut=0.2, pcut=0.01)
    src = I.centred(ph, I.Source(particle, e=e, wx=2.0, wy=2.0))
    n = 1000
    print("\nvacuum 8^3, particle %d, %g MeV, n=%d" % (particle, e, n), flush=True)
    tid, pid = loaded(ctx, (I.WATER,), ph, phys)
    try:
        d, s, st = ctx.run_beam(pid, tid, src, n, 5)
        pb, _, db, sb, stb = ctx.run_beams(pid, tid, [src], [n], 5, per_beam=True)
    finally:
        release(ctx, pid, tid)
    for dose, sig, stats in ((d, s, st), (db, sb, stb)):
        assert not dose.any() and not sig.any()
        assert stats["ledger_residual_lsb"] == 0 and stats["e_dep_mev"] == 0.0
        assert stats["e_esc_mev"] == pytest.approx(n * e, rel=1e-9)
        assert stats["n_hard"] == 0 and stats["n_secondaries"] == 0
        assert np.isnan(stats["s_rel"])                   # Eq. 12 has no voxel to average over
    assert not pb.any()
    if particle == I.ELECTRON:
        # straight through the 8 voxels of depth, one boundary-limited step each
        assert st["n_e_steps"] == 8 * n
    res = oracle.run((I.WATER,), ph, src, phys, seed=5, n_hist=n)
    assert res.e1.sum() == 0.0 and res.stats["e_esc"] == pytest.approx(n * e, rel=1e-12)


def test_sub_cutoff_electrons_deposit_where_they_enter(ctx, oracle):
    ph = I.homogeneous((4, 4, 4), 0.5)
    phys = I.Physics(ecut=0.2, pcut=0.01)
    src = I.centred(ph, I.Source(I.ELECTRON, e=0.1))
    n = 640
    tid, pid = loaded(ctx, (I.WATER,), ph, phys)
    try:
        t, st = ctx.run_beam_tally(pid, tid, src, n, 3)
    finally:
        release(ctx, pid, tid)
    got = t.sum(axis=0)                                   # 2^-27 MeV units per voxel
    assert st["ledger_residual_lsb"] == 0 and st["n_e_steps"] == 0
    assert not got[1:].any()
    e_lsb = int(round(0.1 / LSB))
    assert int(got.sum()) == n * e_lsb
    res = oracle.run((I.WATER,), ph, src, phys, seed=3, n_hist=n)
    assert not res.e1[1:].any()
    # the same histories enter the same voxels: equal up to the units' rounding
    assert np.array_equal(np.rint(res.e1[0] / 0.1).astype(np.int64), got[0] // e_lsb)
    assert np.array_equal(got[0] % e_lsb, np.zeros_like(got[0]))


def gap_phantom():
    """32 x 32 x 48 voxels of 0.5 cm: water 0-6 cm, vacuum 6-12 cm, water 12-24 cm."""
    return I.z_slabs((32, 32, 48), 0.5, [(6.0, 0, 1.0), (12.0, 0, 0.0), (24.0, 0, 1.0)])


@pytest.mark.parametrize("particle,e,n", [(I.PHOTON, 6.0, 200_000), (I.ELECTRON, 15.0, 100_000)],
                         ids=["photon-6MeV", "electron-15MeV"])
def test_vacuum_gap_matches_oracle(ctx, oracle, particle, e, n):
    ph = gap_phantom()
    phys = I.Physics(ecut=0.7, pcut=0.01)
    src = I.centred(ph, I.Source(particle, e=e, wx=5.0, wy=5.0))
    gap = slice(12, 24)                                   # depth voxels 6-12 cm
    print("\nvacuum gap, particle %d, %g MeV, n=%d" % (particle, e, n), flush=True)
    tid, pid = loaded(ctx, (I.WATER,), ph, phys)
    try:
        t, st = ctx.run_beam_tally(pid, tid, src, n, 21)
        d, s, _ = ctx.finalize_tally(pid, tid, t, 0, n)
        ref, _, _ = ctx.run_beam(pid, tid, src, n, 22)     # voxel mask only
    finally:
        release(ctx, pid, tid)
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    assert not t[:, gap].any()
    # the far slab is reached (photons always, 15 MeV electrons by their bremsstrahlung photons)
    assert t[:, 24:].sum() > 0
    res = oracle.run_parallel((I.WATER,), ph, src, phys, 21, n, batches=False)
    assert not res.e1[gap].any()
    do, so = oracle.dose(res, ph)
    zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=phys.n_batches - 1, same_streams=True)
    print("same streams: z-test %s" % E.describe(zt))
    assert zt.passed, E.describe(zt)
    for k in ("n_e_steps", "n_photon_events", "n_secondaries", "n_hard"):
        a, b = st[k], res.stats[k]
        assert abs(a - b) < 2e-3 * b + 10, (k, a, b)


@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 5, 3)], ids=["one-voxel", "7x5x3"])
def test_smallest_grids_and_fewest_histories(ctx, oracle, shape):
    ph = I.homogeneous(shape, 1.0)
    phys = I.Physics(ecut=0.2, pcut=0.01)
    src = I.centred(ph, I.Source(I.PHOTON, e=2.0, wx=1.0, wy=1.0))
    K = phys.n_batches
    tid, pid = loaded(ctx, (I.WATER,), ph, phys)
    try:
        d0, s0, st0 = ctx.run_beam(pid, tid, src, K, 9)       # the fewest histories allowed
        n = 40_000
        d, s, st = ctx.run_beam(pid, tid, src, n, 9)
        ref, _, _ = ctx.run_beam(pid, tid, src, n, 10)
        # the raw batch tallies of the same run (slice-major at the C ABI, whatever the
        # voxel count) give the same dose and sigma through the finalize entry point
        t, _ = ctx.run_beam_tally(pid, tid, src, n, 9)
        dt, st_, _ = ctx.finalize_tally(pid, tid, t, 0, n)
    finally:
        release(ctx, pid, tid)
    assert d0.shape == ph.shape and np.all(np.isfinite(d0)) and np.all(np.isfinite(s0))
    assert st0["ledger_residual_lsb"] == 0 and st["ledger_residual_lsb"] == 0
    assert t.shape == (K,) + ph.shape
    assert np.array_equal(dt, d) and np.array_equal(st_, s)
    # and hold exactly the energy the run deposited
    e_total = float(t.sum()) * LSB
    assert e_total == pytest.approx(st["e_dep_mev"], rel=1e-12)
    res = oracle.run((I.WATER,), ph, src, phys, seed=9, n_hist=n, batches=False)
    do, so = oracle.dose(res, ph)
    zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=K - 1, same_streams=True)
    print("\n%s: same streams: z-test %s" % (shape, E.describe(zt)))
    assert zt.passed, E.describe(zt)


@pytest.mark.parametrize("particle,n", [(I.PHOTON, 100_000), (I.ELECTRON, 20_000)], ids=["photon", "electron"])
def test_largest_energy(ctx, G, oracle, particle, n):
    ph = I.homogeneous((24, 24, 48), 0.5)
    phys = I.Physics(ecut=0.7, pcut=0.01)
    src = I.centred(ph, I.Source(particle, e=30.0, wx=4.0, wy=4.0))
    print("\n30 MeV, particle %d, n=%d" % (particle, n), flush=True)
    tid, pid = loaded(ctx, (I.WATER,), ph, phys)
    try:
        d, s, st = ctx.run_beam(pid, tid, src, n, 31)
        ref, _, _ = ctx.run_beam(pid, tid, src, n, 32)
        with pytest.raises(G.GpumcdError):
            ctx.run_beam(pid, tid, I.centred(ph, I.Source(particle, e=30.5)), n, 31)
    finally:
        release(ctx, pid, tid)
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    res = oracle.run_parallel((I.WATER,), ph, src, phys, 31, n, batches=False)
    do, so = oracle.dose(res, ph)
    zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=phys.n_batches - 1, same_streams=True)
    print("same streams: z-test %s" % E.describe(zt))
    assert zt.passed, E.describe(zt)


def test_largest_batch_count_folds_into_fewer_batches(ctx):
    ph = I.homogeneous((16, 10, 12), 0.5)
    src = I.centred(ph, I.Source(I.PHOTON, e=6.0, wx=3.0, wy=3.0))
    n = 150_000
    print("\nn_batches 1024 vs 32, %s, n=%d" % (ph.shape, n), flush=True)
    t_big = ctx.load_tables((I.WATER,), I.Physics(ecut=0.7, pcut=0.01, n_batches=1024))
    t_small = ctx.load_tables((I.WATER,), I.Physics(ecut=0.7, pcut=0.01, n_batches=32))
    pid = ctx.load_phantom(ph)
    try:
        a, sa = ctx.run_beam_tally(pid, t_big, src, n, 41)
        b, sb = ctx.run_beam_tally(pid, t_small, src, n, 41)
        da, _, ra = ctx.finalize_tally(pid, t_big, a, 0, n)
        db, _, rb = ctx.finalize_tally(pid, t_small, b, 0, n)
    finally:
        release(ctx, pid, t_big, t_small)
    assert a.shape == (1024,) + ph.shape and b.shape == (32,) + ph.shape
    assert sa["ledger_residual_lsb"] == 0 and sb["ledger_residual_lsb"] == 0
    assert sa["e_dep_mev"] == sb["e_dep_mev"]
    # batch k = 32 j + k' of 1024 holds the histories h = k' (mod 32) with h = k (mod 1024)
    assert np.array_equal(a.reshape((32, 32) + ph.shape).sum(axis=0), b)
    assert np.array_equal(da, db)
    print("s of Eq. 12: %.5f with 1024 batches, %.5f with 32" % (ra, rb))
    assert abs(ra / rb - 1.0) < 0.1


def test_largest_history_count(ctx, G):
    ph = I.homogeneous((32, 32, 32), 0.5)
    phys = I.Physics(ecut=0.7, pcut=0.01)
    src = I.centred(ph, I.Source(I.PHOTON, e=1.0, wx=4.0, wy=4.0))
    second = dataclasses.replace(src, first_history=1 << 31)
    n = (1 << 32) - 1
    print("\n2^32 - 1 photons of 1 MeV on 32^3 water, plain and split over two beams", flush=True)
    tid, pid = loaded(ctx, (I.WATER,), ph, phys)
    try:
        d, s, st = ctx.run_beam(pid, tid, src, n, 51)
        _, _, db, sb, stb = ctx.run_beams(pid, tid, [src, second], [1 << 31, (1 << 31) - 1], 51, tuning={})
        with pytest.raises(G.GpumcdError):
            ctx.run_beam(pid, tid, src, 1 << 32, 51)
        with pytest.raises(G.GpumcdError):
            ctx.run_beams(pid, tid, [src, second], [1 << 31, 1 << 31], 51, tuning={})
    finally:
        release(ctx, pid, tid)
    for stats in (st, stb):
        assert stats["n_hist"] == n and stats["ledger_residual_lsb"] == 0
        assert stats["e_in_mev"] == pytest.approx(float(n), rel=1e-12)
        assert 0.0 < stats["s_rel"] < 0.01
    print("s of Eq. 12: plain %.2e, batched %.2e; %.2f s and %.2f s on the device"
          % (st["s_rel"], stb["s_rel"], st["t_device_s"], stb["t_device_s"]))
    assert np.array_equal(db, d)
    # the second beam's histories keep their batches (off + h = 2^32 + i and 2^31 + i agree mod 32)
    assert np.array_equal(sb, s)
