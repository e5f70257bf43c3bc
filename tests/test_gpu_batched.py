"""GPU: the batched form (several beams in one job, graph-replayed rounds).

Bars:
* each beam's dose and sigma from the batched form are bit-identical to the
  plain form run of that beam alone (same seed, same beam id): every
  particle draws from its own stream and tallies are integer sums, so
  neither the other beams in the job nor the tuning can change them;
* the combined dose is the history-weighted sum of the per-beam doses (to
  FP64 rounding of the two conversions) and, for one beam, bit-identical to
  the plain form's dose and sigma; it does not depend on the tally layout
  (per-beam batched tallies, or single per-beam tallies beside a combined
  one, or the combined one alone);
* the combined dose agrees with the oracle's combined dose by the
  same-stream z-test;
* with more beams than the kernels keep in LDS (300), per-beam results stay
  bit-identical to the plain form's;
* at the full beamlet size (256 beamlets, 200x200x160, about 5.8e7
  histories, default tuning as timed by the benchmark): the integer ledger
  closes, no majorant is violated, and sampled beams are bit-identical to
  their plain-form runs; the smallest beam also passes the z-test against
  the oracle;
* at the benchmark's water size (5.25e6 electrons + 6.5e7 photons in one
  batched job): per-beam results equal the plain runs, and each beam agrees
  with an independent oracle run at the paper's counts.
"""
import types

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


@pytest.fixture(scope="module")
def small_job():
    return I.beamlet_job(16, (48, 48, 40), 0.5, count_scale=0.01, min_count=200)


@pytest.fixture(scope="module")
def loaded(ctx, small_job):
    tid = ctx.load_tables(small_job.materials, small_job.physics)
    pid = ctx.load_phantom(small_job.phantom)
    yield pid, tid
    ctx.release(pid)
    ctx.release(tid)


@pytest.fixture(scope="module")
def batched(ctx, small_job, loaded):
    pid, tid = loaded
    j = small_job
    return ctx.run_beams(pid, tid, j.sources, j.counts, j.seed, shape=j.phantom.shape, per_beam=True,
                         per_beam_sigma=True)


def test_per_beam_bit_identical_to_plain(ctx, small_job, loaded, batched):
    pid, tid = loaded
    j = small_job
    pb, ps, d, s, st = batched
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    e_in = 0.0
    for b, (src, n) in enumerate(zip(j.sources, j.counts)):
        db, sb, stb = ctx.run_beam(pid, tid, src, int(n), j.seed, shape=j.phantom.shape)
        assert np.array_equal(pb[b], db) and np.array_equal(ps[b], sb), b
        e_in += stb["e_in_mev"]
    assert st["e_in_mev"] == pytest.approx(e_in, rel=1e-12)


def test_combined_is_history_weighted_sum(small_job, batched):
    j = small_job
    pb, ps, d, s, st = batched
    n = j.counts.astype(np.float64)
    want = np.tensordot(n, pb, axes=1) / n.sum()
    assert np.allclose(d, want, rtol=1e-12, atol=1e-30)
    assert st["n_hist"] == int(j.counts.sum())
    assert np.all(s >= 0) and np.all(s[d == 0] == 0)


def test_single_beam_matches_plain_exactly(ctx, small_job, loaded):
    pid, tid = loaded
    j = small_job
    src, n = j.sources[1], int(j.counts[1])
    for per_beam in (False, True):
        pb, ps, d, s, _ = ctx.run_beams(pid, tid, [src], [n], 5, shape=j.phantom.shape, per_beam=per_beam,
                                        per_beam_sigma=per_beam)
        d1, s1, _ = ctx.run_beam(pid, tid, src, n, 5, shape=j.phantom.shape)
        assert np.array_equal(d, d1) and np.array_equal(s, s1)
        if per_beam:
            assert np.array_equal(pb[0], d1) and np.array_equal(ps[0], s1)


def test_tally_layouts_agree(ctx, G, small_job, loaded, batched):
    pid, tid = loaded
    j = small_job
    pb, ps, d, s, st = batched
    # combined tally only
    _, _, dc, sc, _ = ctx.run_beams(pid, tid, j.sources, j.counts, j.seed, shape=j.phantom.shape)
    assert np.array_equal(dc, d)
    # a beam with fewer histories than batches: single per-beam tallies beside the combined one
    counts = j.counts.copy()
    counts[3] = 20
    pb2, _, d2, s2, st2 = ctx.run_beams(pid, tid, j.sources, counts, j.seed, shape=j.phantom.shape, per_beam=True)
    assert st2["ledger_residual_lsb"] == 0
    _, _, d3, s3, _ = ctx.run_beams(pid, tid, j.sources, counts, j.seed, shape=j.phantom.shape)
    assert np.array_equal(d2, d3) and np.array_equal(s2, s3)
    for b in range(len(j.sources)):
        if b != 3:
            assert np.array_equal(pb2[b], pb[b]), b
    with pytest.raises(G.GpumcdError):
        ctx.run_beams(pid, tid, j.sources, counts, j.seed, shape=j.phantom.shape, per_beam_sigma=True)


def test_tuning_replay_and_output_kind_invariance(ctx, small_job, loaded, batched):
    pid, tid = loaded
    j = small_job
    pb, ps, d, s, st = batched
    tunings = [
        {"chunk": 3001, "pass_items": 4096, "wave_items": 256, "rounds_per_check": 1, "events_per_visit": 5,
         "secondaries_per_visit": 2, "wg_size": 128, "refill_lanes": 64},
        {"rounds_per_check": 9, "chunk": 20000, "wave_items": 64, "refill_lanes": 17},
        {"energy_sort": 1, "chunk": 5000, "pass_items": 20000},
    ]
    for tu in tunings:
        pb2, ps2, d2, s2, st2 = ctx.run_beams(pid, tid, j.sources, j.counts, j.seed, shape=j.phantom.shape,
                                              per_beam=True, per_beam_sigma=True, tuning=tu)
        assert np.array_equal(pb, pb2) and np.array_equal(ps, ps2), tu
        assert np.array_equal(d, d2) and np.array_equal(s, s2), tu
        assert st2["ledger_residual_lsb"] == 0
    pb3, ps3, d3, s3, _ = ctx.run_beams(pid, tid, j.sources, j.counts, j.seed, shape=j.phantom.shape,
                                        per_beam=True, per_beam_sigma=True, out="torch")
    assert np.array_equal(pb3.cpu().numpy(), pb) and np.array_equal(ps3.cpu().numpy(), ps)
    assert np.array_equal(d3.cpu().numpy(), d) and np.array_equal(s3.cpu().numpy(), s)
    _, _, d4, _, _ = ctx.run_beams(pid, tid, j.sources, j.counts, j.seed + 1, shape=j.phantom.shape)
    assert not np.array_equal(d, d4)


def test_combined_matches_oracle(small_job, batched, oracle):
    j = small_job
    pb, ps, d, s, st = batched
    e1 = e2 = 0.0
    stats = {}
    for src, n in zip(j.sources, j.counts):
        r = oracle.run_parallel(j.materials, j.phantom, src, j.physics, j.seed, int(n), batches=False)
        e1 = e1 + r.e1
        e2 = e2 + r.e2
        for k, v in r.stats.items():
            stats[k] = stats.get(k, 0) + v
    comb = types.SimpleNamespace(e1=e1, e2=e2, n_hist=int(j.counts.sum()))
    do, so = oracle.dose(comb, j.phantom)
    zt = E.z_test(d, s, do, so, dof=j.physics.n_batches - 1, same_streams=True)
    print("\n" + E.describe(zt))
    assert zt.passed, E.describe(zt)
    assert st["e_in_mev"] == pytest.approx(stats["e_in"], rel=1e-6)
    for k in ("n_e_steps", "n_photon_events", "n_secondaries"):
        a, b = st[k], stats[k]
        assert abs(a - b) < 6 * np.sqrt(b) + 0.02 * b, (k, a, b)


def test_errors(ctx, G, small_job, loaded):
    pid, tid = loaded
    j = small_job
    with pytest.raises(G.GpumcdError):
        ctx.run_beams(pid, tid, j.sources[:2], [100, 0], 1, shape=j.phantom.shape)
    with pytest.raises(G.GpumcdError):
        ctx.run_beams(pid, tid, j.sources[:2], [3, 4], 1, shape=j.phantom.shape)    # fewer than n_batches
    with pytest.raises(ValueError):
        ctx.run_beams(pid, tid, j.sources[:2], [100], 1, shape=j.phantom.shape)
    with pytest.raises(ValueError):
        ctx.run_beams(pid, tid, j.sources[:1], [100], 1, shape=j.phantom.shape, tuning={"chunks": 5})


def test_more_beams_than_the_lds_beam_table(ctx):
    """Jobs of more than 256 beams read the beam table from memory instead of
    LDS: per-beam results stay bit-identical to the plain form's."""
    j = I.beamlet_job(300, (48, 48, 40), 0.5, count_scale=0.002, min_count=100)
    tid = ctx.load_tables(j.materials, j.physics)
    pid = ctx.load_phantom(j.phantom)
    try:
        pb, ps, d, s, st = ctx.run_beams(pid, tid, j.sources, j.counts, j.seed, shape=j.phantom.shape,
                                         per_beam=True, per_beam_sigma=True)
        assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
        for b in (0, 1, 255, 256, 299):
            db, sb, _ = ctx.run_beam(pid, tid, j.sources[b], int(j.counts[b]), j.seed, shape=j.phantom.shape)
            assert np.array_equal(pb[b], db) and np.array_equal(ps[b], sb), b
    finally:
        ctx.release(pid)
        ctx.release(tid)


def test_full_beamlet_job(ctx, oracle):
    torch = pytest.importorskip("torch")
    j = I.beamlet_job()
    tid = ctx.load_tables(j.materials, j.physics)
    pid = ctx.load_phantom(j.phantom)
    try:
        pb, _, d, s, st = ctx.run_beams(pid, tid, j.sources, j.counts, j.seed, shape=j.phantom.shape,
                                        per_beam=True, out="torch")
        assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
        assert st["n_hist"] == int(j.counts.sum())
        order = np.argsort(j.counts)
        kinds = np.array([src.particle for src in j.sources])
        picks = [int(order[0]), int(order[-1]),
                 int(next(b for b in order if kinds[b] == I.ELECTRON)),
                 int(next(b for b in order if kinds[b] == I.PHOTON))]
        for b in picks:
            db, _, _ = ctx.run_beam(pid, tid, j.sources[b], int(j.counts[b]), j.seed, shape=j.phantom.shape,
                                    sigma=False, out="torch")
            assert torch.equal(pb[b], db), b
        # the smallest beamlet against the oracle (same streams)
        b = int(order[0])
        r = oracle.run_parallel(j.materials, j.phantom, j.sources[b], j.physics, j.seed, int(j.counts[b]),
                                batches=False)
        do, so = oracle.dose(r, j.phantom)
        zt = E.z_test(pb[b].cpu().numpy(), so, do, so, dof=10 ** 6, same_streams=True)
        pe = E.precision_error(pb[b].cpu().numpy(), do)
        print("\nsmallest beamlet (%d histories), same streams: summed dose %+.2e, voxel |diff| mean %.2e max %.2e "
              "of D_max over %d voxels" % (int(j.counts[b]), pe.sum_rel, pe.mean_abs, pe.max_abs, pe.n))
        print("\n" + E.describe(zt))
        assert zt.passed, E.describe(zt)
        del pb, d, s
        torch.cuda.empty_cache()
    finally:
        ctx.release(pid)
        ctx.release(tid)


def test_autotuner_choice_is_cached_and_result_invariant(ctx, G, small_job, loaded):
    pid, tid = loaded
    j = small_job
    counts = j.counts * 2            # another job class than the fixture's (tuned when it ran)
    tun, rep = ctx.autotune(pid, tid, j.sources, counts, budget_s=20.0)
    assert rep["from_cache"] == 0 and rep["trials"] >= 3 and rep["complete"] == 1
    assert rep["t_best_s"] <= rep["t_default_s"]
    assert tun["wg_size"] in (0, 256, 512, 1024) and 1 <= tun["refill_lanes"] <= 64 and tun["chunk"] > 0
    tun2, rep2 = ctx.autotune(pid, tid, j.sources, counts)
    assert rep2["from_cache"] == 1 and rep2["trials"] == 0 and tun2 == tun
    # tuning=None runs with the cached choice; the result does not depend on it
    pb, ps, d, s, _ = ctx.run_beams(pid, tid, j.sources, counts, j.seed, shape=j.phantom.shape, per_beam=True,
                                    per_beam_sigma=True, tuning=None)
    pb2, ps2, d2, s2, _ = ctx.run_beams(pid, tid, j.sources, counts, j.seed, shape=j.phantom.shape, per_beam=True,
                                        per_beam_sigma=True, tuning={"chunk": 4099, "refill_lanes": 3})
    assert np.array_equal(pb, pb2) and np.array_equal(ps, ps2) and np.array_equal(d, d2) and np.array_equal(s, s2)


def test_beam_outside_the_phantom_ahead_of_another(ctx):
    """Primaries that start outside the phantom are stored with zero energy and
    skipped.  A whole beam of them admitted ahead of another beam's primaries
    fills many chunks with nothing to transport; every wavefront must go on to
    the next chunk rather than stop, so that the other beam is transported in
    full (closed ledger, dose bit-identical to its plain run)."""
    from dataclasses import replace
    w = I.water_15mev(I.ELECTRON)
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    try:
        outside = replace(w.source, cx=-40.0, beam_id=0)
        inside = replace(w.source, beam_id=1)
        pb, ps, d, s, st = ctx.run_beams(pid, tid, [outside, inside], [400_000, 600_000], 3,
                                         shape=w.phantom.shape, per_beam=True, per_beam_sigma=True)
        assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
        assert not pb[0].any()
        d1, s1, st1 = ctx.run_beam(pid, tid, inside, 600_000, 3, shape=w.phantom.shape)
        assert np.array_equal(pb[1], d1) and np.array_equal(ps[1], s1)
        assert st["n_e_steps"] == st1["n_e_steps"] and st["n_photon_events"] == st1["n_photon_events"]
    finally:
        ctx.release(pid)
        ctx.release(tid)


def test_water_beams_at_the_benchmark_size(ctx, oracle):
    """The benchmark's job as it times it: the 15 MeV electron and photon
    beams on 64^3 water at their 1% history counts (5.25e6 + 6.5e7) in one
    batched job with per-beam doses and sigmas.  Each beam equals its plain
    run bit for bit (through the raw batch tallies), the ledger closes, and
    each beam's dose agrees with an independent FP64 oracle run at the
    paper's counts (1e6 electrons, 4e6 photons): z-test with the mean bound
    from both sides' batch spreads."""
    from conftest import oracle_batches
    we, wg = I.water_15mev(I.ELECTRON), I.water_15mev(I.PHOTON)
    counts = [5_250_000, 65_000_000]
    seed = 23
    print("\nwater beams at the benchmark size: %d electrons + %d photons" % tuple(counts), flush=True)
    tid = ctx.load_tables(we.materials, we.physics)
    pid = ctx.load_phantom(we.phantom)
    shape = we.phantom.shape
    try:
        pb, ps, d, s, st = ctx.run_beams(pid, tid, [we.source, wg.source], counts, seed, per_beam=True,
                                         per_beam_sigma=True)
        plain = []
        for w, n in zip((we, wg), counts):
            t, stt = ctx.run_beam_tally(pid, tid, w.source, n, seed)
            dt, stg, _ = ctx.finalize_tally(pid, tid, t, 0, n)
            bg = E.batch_doses(t.astype(np.float64) * E.LSB_MEV, we.phantom.rho, we.phantom.voxel, n)
            ref, _, _ = ctx.run_beam(pid, tid, w.source, w.n_hist, seed + 100)   # voxel mask only
            plain.append((dt, stg, stt, bg, ref))
    finally:
        ctx.release(pid)
        ctx.release(tid)
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    assert st["n_hist"] == sum(counts)
    for b, (w, (dt, stg, stt, bg, ref)) in enumerate(zip((we, wg), plain)):
        assert stt["ledger_residual_lsb"] == 0
        assert np.array_equal(pb[b], dt) and np.array_equal(ps[b], stg), b
        res = oracle.run_parallel(w.materials, w.phantom, w.source, w.physics, seed + 1, w.n_hist)
        do, so = oracle.dose(res, w.phantom)
        zi = E.z_test(dt, stg, do, so, ref_for_mask=ref, dof=w.physics.n_batches - 1,
                      batches=(bg, oracle_batches(res, w.phantom, w.n_hist)))
        print("%s, %d GPU histories against %d in the oracle: z-test %s" % (w.name, counts[b], w.n_hist,
                                                                           E.describe(zi)))
        assert zi.passed, E.describe(zi)
