"""GPU: triangular and tabulated (histogram) energy spectra of the source
(Sec. II.C.2), through the C ABI, against the FP64 oracle.

* Triangular 2-10-18 MeV photons (the served stream's polyenergetic beam):
  first real interaction per history on the slab phantom -- the same stream
  word count and the same point to 1e-3 cm for at least 99.9% of histories,
  which checks the FP32 inverse-CDF energy of every history -- and the
  incident energy per history equal to the oracle's to FP32 rounding.
* Triangular photon and electron beams on 64^3 water: per-voxel z-tests on
  the same and on independent streams (voxel mask from a separate run),
  event counts, closed ledger; the FP32-vs-FP64 error and the gamma 2%/2 mm
  pass rate of the same-stream comparison are printed with -s.

* First real photon interaction per history, from a tabulated 6 MV-like
  photon spectrum on the slab phantom: the same stream word count and the
  same point to 1e-3 cm for at least 99.9% of histories (the interaction
  point depends on the sampled energy through the attenuation coefficient).
* A tabulated electron beam on 64^3 water: per-voxel z-tests with the
  combined sigma on the same and on independent streams (voxel mask from a
  separate run), event counts within 6 sigma + 1% of the oracle's, closed
  ledger.
* Batched jobs mixing tabulated and monoenergetic beams, and the served form,
  give each beam's plain-form dose bit for bit (each beam's table is found at
  its own offset of the job's table buffer; the server copies the tables at
  submission).
* Invalid tables are refused with GMC_EINVAL.
"""
import numpy as np
import pytest

from paper_1101_1245_amd import evaluate as E
from paper_1101_1245_amd import inputs as I

pytestmark = pytest.mark.gpu

PHOTON_EDGES = np.array([0.25, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 5.0, 6.0])
PHOTON_WEIGHTS = np.array([0.6, 1.0, 0.9, 0.75, 1.1, 0.7, 0.4, 0.15])
ELECTRON_EDGES = np.array([4.0, 8.0, 12.0, 16.0])
ELECTRON_WEIGHTS = np.array([1.0, 2.0, 1.0])


@pytest.fixture(scope="module")
def G():
    from paper_1101_1245_amd import gpumcd
    return gpumcd


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def tab_source(ph, particle, edges, weights, field=10.0, beam_id=0):
    return I.centred(ph, I.Source(particle, I.TABULATED, 0.0, wx=field, wy=field, beam_id=beam_id,
                                  tab_e=edges, tab_w=weights))


def tri_source(ph, particle, field=10.0, beam_id=0):
    return I.centred(ph, I.Source(particle, I.TRIANGULAR, 10.0, e_lo=2.0, e_mode=10.0, e_hi=18.0, wx=field,
                                  wy=field, beam_id=beam_id))


def test_first_events_triangular_photons(ctx, oracle):
    w = I.slab_6mev()
    src = tri_source(w.phantom, I.PHOTON, field=4.0)
    n = 40000
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    try:
        gx, gn = ctx.first_events(pid, tid, src, w.seed, 0, n)
    finally:
        ctx.release(pid)
        ctx.release(tid)
    ox, on = oracle.first_events(w.materials, w.phantom, src, w.physics, w.seed, 0, n)
    both = np.isfinite(ox[:, 0]) & np.isfinite(gx[:, 0])
    close = both & (np.max(np.abs(gx - ox), axis=1) < 1e-3)
    esc_both = ~np.isfinite(ox[:, 0]) & ~np.isfinite(gx[:, 0])
    agree = (gn == on) & (close | esc_both)
    assert both.sum() > 10000
    assert agree.mean() >= 0.999, agree.mean()


@pytest.mark.parametrize("particle,n", [(I.PHOTON, 2_000_000), (I.ELECTRON, 300_000)], ids=["photon", "electron"])
def test_triangular_beam_matches_oracle(ctx, oracle, batched_run, particle, n):
    from conftest import oracle_batches
    w = I.water_15mev(particle, n_hist=n)
    src = tri_source(w.phantom, particle)
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    try:
        d, s, st, bg = batched_run(ctx, pid, tid, src, n, w.seed, w.phantom)
        ref, _, _ = ctx.run_beam(pid, tid, src, n, 101, shape=w.phantom.shape)   # voxel mask only
    finally:
        ctx.release(pid)
        ctx.release(tid)
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    res = oracle.run_parallel(w.materials, w.phantom, src, w.physics, w.seed, n, batches=False)
    # the same primaries: incident energy equal to FP32 rounding of each history's energy
    assert st["e_in_mev"] == pytest.approx(res.stats["e_in"], rel=1e-6)
    assert abs(res.stats["e_in"] / n - 10.0) < 0.02
    do, so = oracle.dose(res, w.phantom)
    zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=w.physics.n_batches - 1, same_streams=True)
    g = E.gamma_index(do, d, w.phantom.voxel)
    p = E.precision_error(d, do)
    print("\ntriangular %s, same %d histories: z-test %s; summed dose %+.2e, voxel |diff| mean %.2e max %.2e of "
          "D_max; gamma 2%%/2 mm pass %.5f" % (w.name, n, E.describe(zt), p.sum_rel, p.mean_abs, p.max_abs,
                                             g.pass_rate))
    assert zt.passed, E.describe(zt)
    for k in ("n_e_steps", "n_photon_events", "n_secondaries", "n_hard"):
        a, b = st[k], res.stats[k]
        assert abs(a - b) < 2e-3 * b + 10, (k, a, b)
    r2 = oracle.run_parallel(w.materials, w.phantom, src, w.physics, w.seed + 1, n)
    do2, so2 = oracle.dose(r2, w.phantom)
    zi = E.z_test(d, s, do2, so2, ref_for_mask=ref, dof=w.physics.n_batches - 1,
                  batches=(bg, oracle_batches(r2, w.phantom, n)))
    print("triangular %s, independent: z-test %s" % (w.name, E.describe(zi)))
    assert zi.passed, E.describe(zi)


def test_first_events_tabulated_photons(ctx, oracle):
    w = I.slab_6mev()
    src = tab_source(w.phantom, I.PHOTON, PHOTON_EDGES, PHOTON_WEIGHTS, field=4.0)
    n = 40000
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    try:
        gx, gn = ctx.first_events(pid, tid, src, w.seed, 0, n)
    finally:
        ctx.release(pid)
        ctx.release(tid)
    ox, on = oracle.first_events(w.materials, w.phantom, src, w.physics, w.seed, 0, n)
    both = np.isfinite(ox[:, 0]) & np.isfinite(gx[:, 0])
    close = both & (np.max(np.abs(gx - ox), axis=1) < 1e-3)
    esc_both = ~np.isfinite(ox[:, 0]) & ~np.isfinite(gx[:, 0])
    agree = (gn == on) & (close | esc_both)
    assert both.sum() > 10000
    assert agree.mean() >= 0.999, agree.mean()


def test_tabulated_electrons_match_oracle(ctx, G, oracle, batched_run):
    from conftest import oracle_batches
    w = I.water_15mev(I.ELECTRON, n_hist=100_000)
    src = tab_source(w.phantom, I.ELECTRON, ELECTRON_EDGES, ELECTRON_WEIGHTS)
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    try:
        d, s, st, bg = batched_run(ctx, pid, tid, src, w.n_hist, w.seed, w.phantom)
        ref, _, _ = ctx.run_beam(pid, tid, src, w.n_hist, 101, shape=w.phantom.shape)   # voxel mask only
    finally:
        ctx.release(pid)
        ctx.release(tid)
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    # incident energy: the histogram's mean (weighted bin centres) per history
    mean = np.sum(ELECTRON_WEIGHTS * 0.5 * (ELECTRON_EDGES[:-1] + ELECTRON_EDGES[1:])) / ELECTRON_WEIGHTS.sum()
    assert abs(st["e_in_mev"] / w.n_hist - mean) < 0.02
    res = oracle.run_parallel(w.materials, w.phantom, src, w.physics, w.seed, w.n_hist)
    do, so = oracle.dose(res, w.phantom)
    assert st["e_in_mev"] == pytest.approx(res.stats["e_in"], rel=1e-6)
    zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=w.physics.n_batches - 1, same_streams=True)
    print("\ntabulated electrons, same streams: z-test %s" % E.describe(zt))
    assert zt.passed, E.describe(zt)
    r2 = oracle.run_parallel(w.materials, w.phantom, src, w.physics, w.seed + 1, w.n_hist)
    do2, so2 = oracle.dose(r2, w.phantom)
    zi = E.z_test(d, s, do2, so2, ref_for_mask=ref, dof=w.physics.n_batches - 1,
                  batches=(bg, oracle_batches(r2, w.phantom, w.n_hist)))
    print("tabulated electrons, independent: z-test %s" % E.describe(zi))
    assert zi.passed, E.describe(zi)
    for k in ("n_e_steps", "n_photon_events", "n_secondaries", "n_hard"):
        a, b = st[k], res.stats[k]
        assert abs(a - b) < 6 * np.sqrt(b) + 0.01 * b, (k, a, b)


def test_batched_and_served_tabulated_beams_equal_plain(ctx, G):
    w = I.water_15mev(I.PHOTON)
    ph = w.phantom
    srcs = [tab_source(ph, I.PHOTON, PHOTON_EDGES, PHOTON_WEIGHTS, field=5.0, beam_id=0),
            I.centred(ph, I.Source(I.ELECTRON, I.MONO, 9.0, wx=3.0, wy=3.0, beam_id=1)),
            tab_source(ph, I.ELECTRON, ELECTRON_EDGES, ELECTRON_WEIGHTS, field=3.0, beam_id=2),
            tab_source(ph, I.PHOTON, np.array([10.0, 12.0, 15.0]), np.array([1.0, 3.0]), field=2.0, beam_id=3)]
    counts = [200_000, 30_000, 40_000, 100_000]
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(ph)
    try:
        pb, ps, d, s, st = ctx.run_beams(pid, tid, srcs, counts, 7, shape=ph.shape, per_beam=True,
                                         per_beam_sigma=True)
        assert st["ledger_residual_lsb"] == 0
        plain = [ctx.run_beam(pid, tid, sb, n, 7, shape=ph.shape) for sb, n in zip(srcs, counts)]
        for b, (db, sb, _) in enumerate(plain):
            assert np.array_equal(pb[b], db) and np.array_equal(ps[b], sb), b
        ctx.server_start(max_slots=2)
        try:
            tickets = [ctx.submit(pid, tid, sb, n, 7) for sb, n in zip(srcs, counts)]
            for t, (db, sb, _) in zip(tickets, plain):
                done, dd, ss, _ = ctx.poll(t, ph.shape, wait=True)
                assert done and np.array_equal(dd, db) and np.array_equal(ss, sb)
        finally:
            ctx.server_stop()
    finally:
        ctx.release(pid)
        ctx.release(tid)


@pytest.mark.parametrize("edges,weights", [([1.0, 1.0, 2.0], [1.0, 1.0]), ([2.0, 1.0], [1.0]),
                                           ([1.0, 2.0], [-1.0]), ([1.0, 2.0, 3.0], [0.0, 0.0]),
                                           ([1.0, 31.0], [1.0]), ([0.0, 2.0], [1.0])])
def test_invalid_tables_are_refused(ctx, G, edges, weights):
    w = I.small_photon_water(n_hist=1000)
    src = tab_source(w.phantom, I.PHOTON, np.array(edges), np.array(weights))
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    try:
        with pytest.raises(G.GpumcdError) as e:
            ctx.run_beam(pid, tid, src, w.n_hist, 1, shape=w.phantom.shape)
        assert e.value.code == G.GMC_EINVAL
    finally:
        ctx.release(pid)
        ctx.release(tid)
