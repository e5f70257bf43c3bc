"""GPU: a beam split into history shards, the one-GPU part of the multi-GPU
scheme (Sec. II.C.3: histories are independent, so several GPUs can each run
a share of them and add their tallies).

Every history draws from its own counter-based stream keyed by its number
and falls into batch (number mod K), and tallies are integer sums.  So:

* the uint64 batch tallies of G runs over consecutive history ranges
  (``first_history``), added as integers, equal the tally of one run over
  all of them bit for bit, and their finalize gives that run's dose and sigma
  bit for bit -- the exchange of a sharded run is one integer reduction;
* the shards as beams of one batched job (per-beam outputs) give each
  shard's own dose and the whole run's combined dose and sigma bit for bit;
* a shard in the middle of the range agrees with the FP64 oracle run over
  the same history numbers (same-stream z-test).
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


@pytest.fixture(scope="module")
def setup(ctx):
    # 6 MeV photons on the slab phantom at 0.25 cm (electrons, photons, three materials)
    w = I.slab_6mev(n_hist=600_000)
    w.phantom = I.z_slabs((48, 48, 96), 0.25, [(3.0, 0, 1.0), (5.0, 1, 1.85), (12.0, 2, 0.26), (24.0, 0, 1.0)])
    w.source = I.centred(w.phantom, I.Source(I.PHOTON, e=6.0, wx=6.0, wy=6.0, beam_id=2))
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    yield w, tid, pid
    ctx.release(pid)
    ctx.release(tid)


EDGES = (0, 123_457, 400_001, 600_000)   # three shards of uneven, non-multiple-of-K sizes


def shard(src, h0):
    from dataclasses import replace
    return replace(src, first_history=h0)


def test_shard_tallies_add_up_to_one_run(ctx, setup):
    w, tid, pid = setup
    n = EDGES[-1]
    full_t, st = ctx.run_beam_tally(pid, tid, w.source, n, 9)
    assert st["ledger_residual_lsb"] == 0
    d, s, st_d = ctx.run_beam(pid, tid, w.source, n, 9)
    total = np.zeros_like(full_t)
    for a, b in zip(EDGES[:-1], EDGES[1:]):
        t, st_g = ctx.run_beam_tally(pid, tid, shard(w.source, a), b - a, 9)
        assert st_g["ledger_residual_lsb"] == 0 and st_g["n_hist"] == b - a
        total += t
    assert np.array_equal(total, full_t)
    df, sf, srel = ctx.finalize_tally(pid, tid, total, 0, n)
    assert np.array_equal(df, d) and np.array_equal(sf, s)
    assert srel == st_d["s_rel"]
    # the same from device-resident tallies
    tt, _ = ctx.run_beam_tally(pid, tid, w.source, n, 9, out="torch")
    dt, st_, _ = ctx.finalize_tally(pid, tid, tt, 0, n)
    assert np.array_equal(dt, d) and np.array_equal(st_, s)


def test_shards_as_beams_of_one_batched_job(ctx, setup):
    w, tid, pid = setup
    n = EDGES[-1]
    d, s, _ = ctx.run_beam(pid, tid, w.source, n, 9)
    srcs = [shard(w.source, a) for a in EDGES[:-1]]
    counts = [b - a for a, b in zip(EDGES[:-1], EDGES[1:])]
    pb, ps, dc, sc, st = ctx.run_beams(pid, tid, srcs, counts, 9, per_beam=True, per_beam_sigma=True)
    assert st["ledger_residual_lsb"] == 0
    assert np.array_equal(dc, d) and np.array_equal(sc, s)
    for i, (src, m) in enumerate(zip(srcs, counts)):
        dg, sg, _ = ctx.run_beam(pid, tid, src, m, 9)
        assert np.array_equal(pb[i], dg) and np.array_equal(ps[i], sg), i


def test_middle_shard_matches_oracle(ctx, setup, oracle):
    w, tid, pid = setup
    a, b = EDGES[1], EDGES[2]
    d, s, st = ctx.run_beam(pid, tid, shard(w.source, a), b - a, 9)
    mask, _, _ = ctx.run_beam(pid, tid, w.source, b - a, 101)
    res = oracle.run(w.materials, w.phantom, w.source, w.physics, 9, EDGES[-1], h_begin=a, h_end=b, batches=False)
    assert st["e_in_mev"] == pytest.approx(res.stats["e_in"], rel=1e-6)
    do, so = oracle.dose(res, w.phantom)
    zt = E.z_test(d, s, do, so, ref_for_mask=mask, dof=w.physics.n_batches - 1, same_streams=True)
    print("\nshard [%d, %d) vs oracle, same streams: %s" % (a, b, E.describe(zt)))
    assert zt.passed, E.describe(zt)
    for k in ("n_photon_events", "n_e_steps", "n_secondaries"):
        assert abs(st[k] - res.stats[k]) < 2e-3 * res.stats[k] + 10, (k, st[k], res.stats[k])


def test_shard_ranges_are_checked(ctx, G, setup):
    w, tid, pid = setup
    with pytest.raises(G.GpumcdError) as e:
        ctx.run_beam(pid, tid, shard(w.source, (1 << 32) - 1000), 2000, 1)
    assert e.value.code == G.GMC_EINVAL
    t, _ = ctx.run_beam_tally(pid, tid, w.source, 1000, 1)
    for a, b in ((0, 0), (5, 3), (0, 10), (0, (1 << 32) + 1)):
        with pytest.raises(G.GpumcdError) as e:
            ctx.finalize_tally(pid, tid, t, a, b)
        assert e.value.code == G.GMC_EINVAL
    with pytest.raises(ValueError):
        ctx.finalize_tally(pid, tid, t[:-1], 0, 1000)
