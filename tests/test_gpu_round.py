"""GPU: the persistent round kernel (tuning ``persistent``), the batched
form's pool of persistent wavefronts (Sec. II.C.3) drained from a device work
queue.

Every particle carries its own stream and tallies are integer sums, so
whichever wavefront claims a chunk -- and in whichever round a particle is
transported -- the dose cannot change.  The bar is therefore bit identity
with the pass kernels:

* two-beam batched jobs (15 MeV electrons and photons on water, per-beam
  doses and sigmas) and plain single-beam runs, at the default sizes and with
  tiny passes, chunks and visit budgets that force many rounds, carried-over
  particles and partial chunks;
* a three-material slab job and a four-material beamlet job (the most
  materials whose two table blocks fit in LDS beside each other);
* tables of more than four materials run the passes instead, with the same
  result;
* the stuck-queue fixed point is detected in this form too.
The event counters agree exactly and the round kernel is the only transport
kernel launched.
"""
import numpy as np
import pytest

from paper_1101_1245_amd import inputs as I

pytestmark = pytest.mark.gpu

ROUND = {"persistent": 1}


@pytest.fixture(scope="module")
def G():
    from paper_1101_1245_amd import gpumcd
    return gpumcd


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def same_counts(a, b):
    for k in ("n_e_steps", "n_photon_events", "n_secondaries", "n_hard", "n_fictitious", "e_dep_mev", "e_esc_mev"):
        assert a[k] == b[k], (k, a[k], b[k])


def only_rounds(st):
    assert st["n_round_launches"] > 0 and st["n_electron_launches"] == 0 and st["n_photon_launches"] == 0, st


@pytest.mark.parametrize("extra", [{}, {"pass_items": 5000, "chunk": 7919, "events_per_visit": 3, "wave_items": 64,
                                        "rounds_per_check": 2}],
                         ids=["defaults", "tiny-rounds"])
def test_round_kernel_batched_bit_identical(ctx, extra):
    we, wg = I.water_15mev(I.ELECTRON, n_hist=150_000), I.water_15mev(I.PHOTON, n_hist=600_000)
    tid = ctx.load_tables(we.materials, we.physics)
    pid = ctx.load_phantom(we.phantom)
    try:
        srcs, counts = [we.source, I.centred(we.phantom, I.Source(I.PHOTON, e=15.0, wx=10, wy=10, beam_id=1))], \
            [we.n_hist, wg.n_hist]
        base = dict(extra, chunk=extra.get("chunk", 1 << 20), pass_items=extra.get("pass_items", 1 << 21))
        ref = ctx.run_beams(pid, tid, srcs, counts, 3, per_beam=True, per_beam_sigma=True, tuning=base)
        got = ctx.run_beams(pid, tid, srcs, counts, 3, per_beam=True, per_beam_sigma=True, tuning=dict(base, **ROUND))
    finally:
        ctx.release(pid)
        ctx.release(tid)
    for r in (ref, got):
        assert r[4]["ledger_residual_lsb"] == 0
    only_rounds(got[4])
    for i in range(4):
        assert np.array_equal(ref[i], got[i]), i
    same_counts(ref[4], got[4])


def test_round_kernel_plain_and_slabs(ctx):
    w = I.slab_6mev(n_hist=400_000)
    w.phantom = I.z_slabs((48, 48, 96), 0.25, [(3.0, 0, 1.0), (5.0, 1, 1.85), (12.0, 2, 0.26), (24.0, 0, 1.0)])
    w.source = I.centred(w.phantom, I.Source(I.PHOTON, I.TRIANGULAR, 10.0, e_lo=2.0, e_mode=10.0, e_hi=18.0,
                                             wx=6.0, wy=6.0))
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    try:
        d0, s0, st0 = ctx.run_beam(pid, tid, w.source, w.n_hist, 5)
        d1, s1, st1 = ctx.run_beam(pid, tid, w.source, w.n_hist, 5, tuning=ROUND)
        d2, s2, st2 = ctx.run_beam(pid, tid, w.source, w.n_hist, 5,
                                   tuning=dict(ROUND, pass_items=3000, chunk=5000, wave_items=128))
    finally:
        ctx.release(pid)
        ctx.release(tid)
    only_rounds(st1)
    only_rounds(st2)
    for d, s, st in ((d1, s1, st1), (d2, s2, st2)):
        assert st["ledger_residual_lsb"] == 0
        assert np.array_equal(d, d0) and np.array_equal(s, s0)
        same_counts(st0, st)


def test_round_kernel_four_material_beamlets(ctx):
    j = I.beamlet_job(n_beamlets=16, shape=(64, 64, 64), voxel=0.4, count_scale=0.05, min_count=64)
    tid = ctx.load_tables(j.materials, j.physics)
    pid = ctx.load_phantom(j.phantom)
    try:
        tu = {"chunk": 1 << 18, "pass_items": 1 << 19}
        ref = ctx.run_beams(pid, tid, j.sources, j.counts, 2, per_beam=True, tuning=tu)
        got = ctx.run_beams(pid, tid, j.sources, j.counts, 2, per_beam=True, tuning=dict(tu, **ROUND))
    finally:
        ctx.release(pid)
        ctx.release(tid)
    only_rounds(got[4])
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[2], got[2]) and np.array_equal(ref[3], got[3])
    same_counts(ref[4], got[4])


def test_round_kernel_falls_back_beyond_four_materials(ctx):
    mats = I.DEFAULT_MATERIALS + (I.WATER,)        # five materials: two table blocks do not fit in LDS
    ph = I.ellipsoids(32, 0.5, seed=3)
    src = I.centred(ph, I.Source(I.PHOTON, e=8.0, wx=4.0, wy=4.0))
    tid = ctx.load_tables(mats, I.serving_physics())
    pid = ctx.load_phantom(ph)
    try:
        d0, s0, st0 = ctx.run_beam(pid, tid, src, 100_000, 1)
        d1, s1, st1 = ctx.run_beam(pid, tid, src, 100_000, 1, tuning=ROUND)
    finally:
        ctx.release(pid)
        ctx.release(tid)
    assert st1["n_round_launches"] == 0 and st1["n_electron_launches"] > 0
    assert np.array_equal(d0, d1) and np.array_equal(s0, s1)


def test_round_kernel_stuck_queues_reported(ctx, G):
    ph = I.homogeneous(24, 0.5)
    src = I.centred(ph, I.Source(I.PHOTON, e=6.0, wx=4.0, wy=4.0))
    tid = ctx.load_tables((I.WATER,), I.Physics(ecut=0.2, pcut=0.01))
    pid = ctx.load_phantom(ph)
    tight = dict(ROUND, queue_items=64, secondaries_per_visit=64, chunk=64, pass_items=1024)
    try:
        for fn in (lambda: ctx.run_beam(pid, tid, src, 20_000, 3, tuning=tight),
                   lambda: ctx.run_beams(pid, tid, [src], [20_000], 3, tuning=dict(tight, rounds_per_check=2))):
            with pytest.raises(G.GpumcdError) as e:
                fn()
            assert e.value.code == G.GMC_EOVERFLOW and "too full" in str(e.value)
        d, s, st = ctx.run_beam(pid, tid, src, 20_000, 3, tuning=ROUND)
        d0, s0, _ = ctx.run_beam(pid, tid, src, 20_000, 3)
        assert np.array_equal(d, d0) and np.array_equal(s, s0)
    finally:
        ctx.release(pid)
        ctx.release(tid)
