"""GPU: the served form (continuous batching of dose requests).

Bars:
* every request's dose and sigma are bit-identical to running the same
  request alone through the plain form (same phantom, tables, source,
  histories and seed), whatever ran beside it;
* requests submitted together overlap: with several slots, later requests
  start before earlier ones finish; with a budget that fits one slot, they
  run one after another;
* a request whose footprint can never fit is refused (GMC_EBUSY), ids held by
  queued requests cannot be released, and bad requests are rejected at
  submission;
* served requests of the request stream's kind -- an ellipsoid phantom with
  four materials, triangular 2-10-18 MeV photon and electron beams --
  submitted together with others agree with the FP64 oracle: per-voxel
  z-tests on the same and on independent streams, event counts;
* a request on the largest grid of the request stream (256^3 voxels) served
  beside a small one equals the plain form bit for bit and agrees with the
  oracle on the same histories; the stream's largest request (1e8 histories
  on 256^3 voxels) equals the plain form bit for bit with an exact ledger.
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
def stream(ctx):
    pool, reqs = I.request_stream(seed=5, n_requests=10, n_phantoms=3, grid=(24, 48), log10_hist=(4.0, 5.3))
    tid = ctx.load_tables(I.DEFAULT_MATERIALS, I.serving_physics())
    pids = [ctx.load_phantom(p) for p in pool]
    yield pool, reqs, tid, pids
    for p in pids:
        ctx.release(p)
    ctx.release(tid)


def run_all(ctx, pool, reqs, tid, pids):
    tickets = [ctx.submit(pids[r.phantom], tid, r.source, r.n_hist, r.seed) for r in reqs]
    out = []
    for t, r in zip(tickets, reqs):
        done, d, s, st = ctx.poll(t, pool[r.phantom].shape, wait=True)
        assert done
        out.append((d, s, st))
    return out


def test_results_equal_alone(ctx, stream):
    pool, reqs, tid, pids = stream
    ctx.server_start(max_slots=4)
    try:
        res = run_all(ctx, pool, reqs, tid, pids)
    finally:
        ctx.server_stop()
    for (d, s, st), r in zip(res, reqs):
        assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
        da, sa, sta = ctx.run_beam(pids[r.phantom], tid, r.source, r.n_hist, r.seed, shape=pool[r.phantom].shape)
        assert np.array_equal(d, da) and np.array_equal(s, sa), r
        assert st["s_rel"] == sta["s_rel"] or (np.isnan(st["s_rel"]) and np.isnan(sta["s_rel"])), r
    # overlap: some request started before an earlier one finished
    starts = [st["t_queue_s"] for _, _, st in res]
    ends = [st["t_latency_s"] for _, _, st in res]
    assert any(starts[j] < ends[i] for i in range(len(res)) for j in range(i + 1, len(res)))


def test_one_slot_budget_serialises(ctx, G, stream):
    pool, reqs, tid, pids = stream
    sub = reqs[:4]
    ctx.server_start(max_slots=1)
    try:
        tickets = [ctx.submit(pids[r.phantom], tid, r.source, r.n_hist, r.seed) for r in sub]
        # the last request waits behind the others on the single slot: its phantom is held
        with pytest.raises(G.GpumcdError) as e:
            ctx.release(pids[sub[-1].phantom])
        assert e.value.code == G.GMC_EBUSY
        res = [ctx.poll(t, pool[r.phantom].shape, wait=True)[1:] for t, r in zip(tickets, sub)]
    finally:
        ctx.server_stop()
    for i in range(1, len(res)):
        assert res[i][2]["t_queue_s"] >= res[i - 1][2]["t_latency_s"] - 1e-4
    ctx.server_start(max_slots=2, hbm_budget_bytes=1 << 20)
    try:
        with pytest.raises(G.GpumcdError) as e:
            ctx.submit(pids[0], tid, reqs[0].source, reqs[0].n_hist, 1)
        assert e.value.code == G.GMC_EBUSY
    finally:
        ctx.server_stop()


def test_results_wait_in_device_memory_and_move_to_host_at_stop(ctx, stream):
    """Finished results stay in the server's device result pool until polled;
    stopping the server moves the unpolled ones to host memory.  Either way
    the polled dose and sigma equal the plain form's bit for bit, delivered to
    host or to device memory."""
    import time
    pool, reqs, tid, pids = stream
    sub = reqs[:6]
    ctx.server_start(max_slots=2)
    try:
        tickets = [ctx.submit(pids[r.phantom], tid, r.source, r.n_hist, r.seed) for r in sub]
        # the first two polled at once (device results), the rest after the stop
        early = [ctx.poll(t, pool[r.phantom].shape, wait=True, out=o)
                 for t, r, o in zip(tickets[:2], sub[:2], ("numpy", "torch"))]
        t_end = time.time() + 120
        while ctx.server_status()["finished_unpolled"] < len(sub) - 2 and time.time() < t_end:
            time.sleep(0.01)
        assert ctx.server_status()["finished_unpolled"] == len(sub) - 2
    finally:
        ctx.server_stop()
    late = [ctx.poll(t, pool[r.phantom].shape, wait=True, out=o)
            for t, r, o in zip(tickets[2:], sub[2:], ("numpy", "torch") * 2)]
    for (done, d, s, st), r in zip(early + late, sub):
        assert done and st["ledger_residual_lsb"] == 0
        d = d.cpu().numpy() if hasattr(d, "cpu") else d
        s = s.cpu().numpy() if hasattr(s, "cpu") else s
        da, sa, _ = ctx.run_beam(pids[r.phantom], tid, r.source, r.n_hist, r.seed, shape=pool[r.phantom].shape)
        assert np.array_equal(d, da) and np.array_equal(s, sa), r


def test_bad_requests_and_device_output(ctx, G, stream):
    pool, reqs, tid, pids = stream
    ctx.server_start()
    try:
        with pytest.raises(G.GpumcdError):
            ctx.submit(pids[0], tid, reqs[0].source, 5, 1)                 # fewer histories than batches
        with pytest.raises(G.GpumcdError):
            ctx.submit(9999, tid, reqs[0].source, 1000, 1)                 # unknown phantom
        with pytest.raises(G.GpumcdError):
            ctx.submit(pids[0], tid, I.Source(I.PHOTON, e=45.0), 1000, 1)  # energy out of range
        r = reqs[1]
        t = ctx.submit(pids[r.phantom], tid, r.source, r.n_hist, r.seed)
        done, d, s, st = ctx.poll(t, pool[r.phantom].shape, wait=True, out="torch")
        assert done
        with pytest.raises(G.GpumcdError):
            ctx.poll(t, pool[r.phantom].shape)                             # retired
    finally:
        ctx.server_stop()
    da, sa, _ = ctx.run_beam(pids[r.phantom], tid, r.source, r.n_hist, r.seed, shape=pool[r.phantom].shape)
    assert np.array_equal(d.cpu().numpy(), da) and np.array_equal(s.cpu().numpy(), sa)


def test_served_triangular_requests_match_oracle(ctx, oracle, batched_run):
    from conftest import oracle_batches
    ph = I.ellipsoids(40, 0.4, seed=23)
    phys = I.serving_physics()
    reqs = [(I.centred(ph, I.Source(I.PHOTON, I.TRIANGULAR, 10.0, e_lo=2.0, e_mode=10.0, e_hi=18.0, wx=6.0, wy=6.0,
                                    beam_id=3)), 1_000_000, 7),
            (I.centred(ph, I.Source(I.ELECTRON, I.TRIANGULAR, 10.0, e_lo=2.0, e_mode=10.0, e_hi=18.0, wx=4.0,
                                    wy=4.0, beam_id=4)), 200_000, 8),
            (I.centred(ph, I.Source(I.PHOTON, I.MONO, 12.0, wx=3.0, wy=3.0, beam_id=5)), 300_000, 9)]
    tid = ctx.load_tables(I.DEFAULT_MATERIALS, phys)
    pid = ctx.load_phantom(ph)
    try:
        ctx.server_start(max_slots=3)
        try:
            tickets = [ctx.submit(pid, tid, src, n, seed) for src, n, seed in reqs]
            out = [ctx.poll(t, ph.shape, wait=True) for t in tickets]
        finally:
            ctx.server_stop()
        masks = [ctx.run_beam(pid, tid, src, n, 101, shape=ph.shape)[0] for src, n, _ in reqs[:2]]
        # the same requests through the raw-tally entry points: the batches for the mean bound
        batches = []
        for (src, n, seed), (_, d, s, _) in zip(reqs[:2], out[:2]):
            db, sb, _, bg = batched_run(ctx, pid, tid, src, n, seed, ph)
            assert np.array_equal(db, d) and np.array_equal(sb, s)
            batches.append(bg)
    finally:
        ctx.release(pid)
        ctx.release(tid)
    for (src, n, seed), (done, d, s, st), ref, bg in zip(reqs[:2], out[:2], masks, batches):
        assert done and st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
        res = oracle.run_parallel(I.DEFAULT_MATERIALS, ph, src, phys, seed, n, batches=False)
        assert st["e_in_mev"] == pytest.approx(res.stats["e_in"], rel=1e-6)
        do, so = oracle.dose(res, ph)
        zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=phys.n_batches - 1, same_streams=True)
        p = E.precision_error(d, do)
        print("\nserved triangular %s, same %d histories: z-test %s; summed dose %+.2e, voxel |diff| max %.2e of "
              "D_max" % ("electrons" if src.particle else "photons", n, E.describe(zt), p.sum_rel, p.max_abs))
        assert zt.passed, E.describe(zt)
        for k in ("n_e_steps", "n_photon_events", "n_secondaries"):
            assert abs(st[k] - res.stats[k]) < 2e-3 * res.stats[k] + 10, (k, st[k], res.stats[k])
        r2 = oracle.run_parallel(I.DEFAULT_MATERIALS, ph, src, phys, seed + 100, n)
        do2, so2 = oracle.dose(r2, ph)
        zi = E.z_test(d, s, do2, so2, ref_for_mask=ref, dof=phys.n_batches - 1,
                      batches=(bg, oracle_batches(r2, ph, n)))
        print("served triangular, independent: z-test %s" % E.describe(zi))
        assert zi.passed, E.describe(zi)


def test_largest_grid_request_matches_plain_and_oracle(ctx, oracle):
    """A request on the request stream's largest grid, 256^3 voxels of
    0.25 cm (16.8M voxels, 4.3 GB of batch tallies), served beside a small
    one: bit-identical to the plain form, the ledger exact, and the dose in
    agreement with the FP64 oracle on the same histories."""
    big = I.ellipsoids(256, 0.25, seed=31)
    small = I.ellipsoids(32, 0.5, seed=32)
    phys = I.serving_physics()
    src = I.centred(big, I.Source(I.PHOTON, I.TRIANGULAR, 10.0, e_lo=2.0, e_mode=10.0, e_hi=18.0, wx=10.0, wy=10.0,
                                  beam_id=6))
    src_small = I.centred(small, I.Source(I.ELECTRON, I.MONO, 8.0, wx=4.0, wy=4.0, beam_id=7))
    n = 1_000_000
    print("\n256^3 request, n=%d" % n, flush=True)
    tid = ctx.load_tables(I.DEFAULT_MATERIALS, phys)
    pid = ctx.load_phantom(big)
    pid_s = ctx.load_phantom(small)
    try:
        ctx.server_start(max_slots=2)
        try:
            t_big = ctx.submit(pid, tid, src, n, 17)
            t_small = ctx.submit(pid_s, tid, src_small, 50_000, 18)
            done, d, s, st = ctx.poll(t_big, big.shape, wait=True)
            done_s, d_s, s_s, _ = ctx.poll(t_small, small.shape, wait=True)
        finally:
            ctx.server_stop()
        assert done and done_s
        da, sa, _ = ctx.run_beam(pid, tid, src, n, 17)
        ref, _, _ = ctx.run_beam(pid, tid, src, n, 117)        # voxel mask only
        ds, ss, _ = ctx.run_beam(pid_s, tid, src_small, 50_000, 18)
    finally:
        ctx.release(pid)
        ctx.release(pid_s)
        ctx.release(tid)
    assert np.array_equal(d, da) and np.array_equal(s, sa)
    assert np.array_equal(d_s, ds) and np.array_equal(s_s, ss)
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0
    res = oracle.run_parallel(I.DEFAULT_MATERIALS, big, src, phys, 17, n, batches=False)
    assert st["e_in_mev"] == pytest.approx(res.stats["e_in"], rel=1e-6)
    do, so = oracle.dose(res, big)
    zt = E.z_test(d, s, do, so, ref_for_mask=ref, dof=phys.n_batches - 1, same_streams=True)
    p = E.precision_error(d, do)
    print("256^3 served request, same histories: z-test %s; summed dose %+.2e, voxel |diff| max %.2e of D_max"
          % (E.describe(zt), p.sum_rel, p.max_abs))
    assert zt.passed, E.describe(zt)
    for k in ("n_e_steps", "n_photon_events", "n_secondaries"):
        assert abs(st[k] - res.stats[k]) < 2e-3 * res.stats[k] + 10, (k, st[k], res.stats[k])


def test_largest_request_served_equals_plain(ctx):
    """The request stream's largest request, 1e8 histories on a 256^3 grid,
    served beside a small one: bit-identical to the plain form, the ledger
    exact (the oracle cannot follow 1e8 histories; these properties hold at
    any size)."""
    big = I.ellipsoids(256, 0.25, seed=33)
    phys = I.serving_physics()
    src = I.centred(big, I.Source(I.PHOTON, I.MONO, 20.0, wx=10.0, wy=10.0, beam_id=8))
    small = I.ellipsoids(32, 0.5, seed=34)
    src_small = I.centred(small, I.Source(I.ELECTRON, I.TRIANGULAR, 10.0, e_lo=2.0, e_mode=10.0, e_hi=18.0, wx=3.0,
                                          wy=3.0, beam_id=9))
    n = 100_000_000
    print("\n256^3 request, n=%d" % n, flush=True)
    tid = ctx.load_tables(I.DEFAULT_MATERIALS, phys)
    pid = ctx.load_phantom(big)
    pid_s = ctx.load_phantom(small)
    try:
        ctx.server_start(max_slots=2)
        try:
            t_big = ctx.submit(pid, tid, src, n, 41)
            t_small = ctx.submit(pid_s, tid, src_small, 100_000, 42)
            done, d, s, st = ctx.poll(t_big, big.shape, wait=True)
            done_s, d_s, s_s, st_s = ctx.poll(t_small, small.shape, wait=True)
        finally:
            ctx.server_stop()
        da, sa, sta = ctx.run_beam(pid, tid, src, n, 41)
        ds, ss, _ = ctx.run_beam(pid_s, tid, src_small, 100_000, 42)
    finally:
        ctx.release(pid)
        ctx.release(pid_s)
        ctx.release(tid)
    assert done and done_s
    assert st["ledger_residual_lsb"] == 0 and st["n_majorant_violations"] == 0 and st_s["ledger_residual_lsb"] == 0
    assert st["n_hist"] == n and st["e_in_mev"] == pytest.approx(20.0 * n, rel=1e-6)
    assert np.array_equal(d, da) and np.array_equal(s, sa)
    assert np.array_equal(d_s, ds) and np.array_equal(s_s, ss)
    assert st["s_rel"] == sta["s_rel"]
