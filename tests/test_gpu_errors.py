"""GPU: the failure paths of the engine, each forced from the host so that
every kernel still runs to its normal end.

* A job whose 64-bit tallies could overflow (histories x highest energy at or
  above 2^63 units of 2^-27 MeV) is refused before anything runs, in the
  plain, batched and served forms.
* A queue too small for the per-visit output budget (tuning queue_items)
  leaves neither pass able to move: the plain and the graph-replayed batched
  form both detect the fixed point and return GMC_EOVERFLOW instead of
  looping; the context runs the next job normally, bit-identical to a fresh
  run.
* A majorant below the real attenuation (physics majorant_margin < 1) is
  counted in n_majorant_violations, photon and electron side, while the
  ledger still closes; at the default margin the count is zero.
* Output shapes that do not match the phantom are refused by the binding
  before the library writes nx*ny*nz doubles.
"""
import numpy as np
import pytest

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
def water(ctx):
    ph = I.homogeneous(24, 0.5)
    tid = ctx.load_tables((I.WATER,), I.Physics(ecut=0.2, pcut=0.01))
    pid = ctx.load_phantom(ph)
    yield ph, tid, pid
    ctx.release(pid)
    ctx.release(tid)


def test_tally_overflow_refused_up_front(ctx, G, water):
    ph, tid, pid = water
    src = I.centred(ph, I.Source(I.PHOTON, e=30.0, wx=2.0, wy=2.0))
    n = 3_000_000_000          # 3e9 x 30 MeV x 2^27 > 2^63
    with pytest.raises(G.GpumcdError) as e:
        ctx.run_beam(pid, tid, src, n, 1)
    assert e.value.code == G.GMC_EOVERFLOW
    with pytest.raises(G.GpumcdError) as e:
        ctx.run_beams(pid, tid, [src, src], [n // 2, n // 2], 1, tuning={"chunk": 1 << 20})
    assert e.value.code == G.GMC_EOVERFLOW
    ctx.server_start(max_slots=1)
    try:
        with pytest.raises(G.GpumcdError) as e:
            ctx.submit(pid, tid, src, n, 1)
        assert e.value.code == G.GMC_EOVERFLOW
    finally:
        ctx.server_stop()


def test_stuck_queues_are_reported(ctx, G, water):
    ph, tid, pid = water
    src = I.centred(ph, I.Source(I.PHOTON, e=6.0, wx=4.0, wy=4.0))
    ref_d, ref_s, _ = ctx.run_beam(pid, tid, src, 20_000, 3)
    # a soft capacity of 64 particles with 64 secondaries per visit: once both
    # queues hold a particle, neither pass may take one
    tight = {"queue_items": 64, "secondaries_per_visit": 64, "chunk": 64, "pass_items": 1024}
    with pytest.raises(G.GpumcdError) as e:
        ctx.run_beam(pid, tid, src, 20_000, 3, tuning=tight)
    assert e.value.code == G.GMC_EOVERFLOW and "too full" in str(e.value)
    with pytest.raises(G.GpumcdError) as e:
        ctx.run_beams(pid, tid, [src], [20_000], 3, tuning=dict(tight, rounds_per_check=2))
    assert e.value.code == G.GMC_EOVERFLOW and "too full" in str(e.value)
    # the context is usable afterwards and gives the same result as before
    d, s, st = ctx.run_beam(pid, tid, src, 20_000, 3)
    assert st["ledger_residual_lsb"] == 0
    assert np.array_equal(d, ref_d) and np.array_equal(s, ref_s)
    # a small but workable queue finishes with the same dose
    d2, s2, st2 = ctx.run_beam(pid, tid, src, 20_000, 3, tuning={"queue_items": 4096, "chunk": 512})
    assert np.array_equal(d2, ref_d) and np.array_equal(s2, ref_s)


@pytest.mark.parametrize("particle", [I.PHOTON, I.ELECTRON], ids=["photon", "electron"])
def test_undersized_majorant_is_counted(ctx, particle):
    ph = I.homogeneous(24, 0.5)
    src = I.centred(ph, I.Source(particle, e=6.0, wx=4.0, wy=4.0))
    counts = {}
    for margin in (0.0, 0.5):
        tid = ctx.load_tables((I.WATER,), I.Physics(ecut=0.2, pcut=0.01, majorant_margin=margin))
        pid = ctx.load_phantom(ph)
        try:
            _, _, st = ctx.run_beam(pid, tid, src, 20_000, 4)
        finally:
            ctx.release(pid)
            ctx.release(tid)
        assert st["ledger_residual_lsb"] == 0
        counts[margin] = st["n_majorant_violations"]
    assert counts[0.0] == 0 and counts[0.5] > 0, counts


def test_bad_margin_and_shapes_refused(ctx, G, water):
    ph, tid, pid = water
    with pytest.raises(G.GpumcdError) as e:
        ctx.load_tables((I.WATER,), I.Physics(majorant_margin=1e-3))
    assert e.value.code == G.GMC_EINVAL
    assert ctx.phantom_shape(pid) == ph.shape
    src = I.centred(ph, I.Source(I.PHOTON, e=1.0))
    with pytest.raises(ValueError):
        ctx.run_beam(pid, tid, src, 1000, 1, shape=(24, 24, 23))
    ctx.server_start(max_slots=1)
    try:
        t = ctx.submit(pid, tid, src, 1000, 1)
        with pytest.raises(ValueError):
            ctx.poll(t, (10, 10, 10))
        done, d, s, _ = ctx.poll(t)
        assert done and d.shape == ph.shape
    finally:
        ctx.server_stop()
    with pytest.raises(G.GpumcdError) as e:
        ctx.phantom_shape(9999)
    assert e.value.code == G.GMC_ENOTFOUND
