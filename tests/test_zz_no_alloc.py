"""GPU: the allocation-free finalize (gmc_finalize_tally_noalloc) against
gmc_finalize_tally, called through the C ABI.

The two share the finalize kernels (Sec. II.D: dose per history and the
batch uncertainty of Eq. 13, s of Eq. 12); the allocation-free one keeps its
work (histories per batch, the partial sums of s) in the library's per-device
array instead of allocated memory.  On the same device tallies and history
range the results must agree bit for bit -- dose, sigma and s -- on two calls
in a row, the second on a smaller phantom and a shifted, shorter history
range, so that stale contents of the shared work array would show.
"""
from dataclasses import replace

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


def _case(ctx, shape, n, h0, seed):
    """A photon beam's device tallies over histories [h0, h0 + n) on a
    water phantom of `shape` (nz, ny, nx) at 0.5 cm."""
    w = I.small_photon_water(n_hist=n)
    w.phantom = I.z_slabs(shape, 0.5, [(1e3, 0, 1.0)])
    w.source = replace(I.centred(w.phantom, I.Source(I.PHOTON, e=2.0, wx=2.0, wy=2.0, beam_id=5)),
                       first_history=h0)
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    t, st = ctx.run_beam_tally(pid, tid, w.source, n, seed, out="torch")
    assert st["ledger_residual_lsb"] == 0
    return w, tid, pid, t


def _compare(ctx, tid, pid, t, h0, h1):
    import torch
    shape = ctx.phantom_shape(pid)
    d_ref, s_ref, srel_ref = ctx.finalize_tally(pid, tid, t, h0, h1)
    # outputs prefilled with NaN: every voxel must be written
    dose = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    sigma = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    srel = ctx.finalize_tally_noalloc(pid, tid, t, h0, h1, dose, sigma)
    torch.cuda.synchronize()
    d, s = dose.cpu().numpy(), sigma.cpu().numpy()
    print("\nno-alloc finalize %s, histories [%d, %d): s %.6e (reference %.6e)" % (shape, h0, h1, srel, srel_ref),
          flush=True)
    assert np.array_equal(d.view(np.uint64), d_ref.view(np.uint64))
    assert np.array_equal(s.view(np.uint64), s_ref.view(np.uint64))
    assert np.float64(srel).view(np.uint64) == np.float64(srel_ref).view(np.uint64)
    assert d.max() > 0 and np.isfinite(srel)
    # without sigma: dose unchanged, s NaN
    dose2 = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")
    srel2 = ctx.finalize_tally_noalloc(pid, tid, t, h0, h1, dose2, None)
    assert np.array_equal(dose2.cpu().numpy().view(np.uint64), d_ref.view(np.uint64))
    assert np.isnan(srel2)


def test_noalloc_finalize_equals_finalize_twice_smaller_second(ctx):
    # first call: 24 x 20 x 16 voxels, histories [0, 60000)
    w, tid, pid, t = _case(ctx, (24, 20, 16), 60_000, 0, 3)
    _compare(ctx, tid, pid, t, 0, 60_000)
    # second call: smaller phantom, shorter range not starting at 0 (other batch sizes)
    w2, tid2, pid2, t2 = _case(ctx, (10, 8, 6), 20_003, 777, 4)
    _compare(ctx, tid2, pid2, t2, 777, 777 + 20_003)
    # the first case again after the smaller one
    _compare(ctx, tid, pid, t, 0, 60_000)
    for h in (pid, tid, pid2, tid2):
        ctx.release(h)


def test_noalloc_finalize_rejects_bad_arguments(ctx, G):
    import torch
    w, tid, pid, t = _case(ctx, (8, 8, 8), 5_000, 0, 5)
    shape = ctx.phantom_shape(pid)
    dose = torch.zeros(shape, dtype=torch.float64, device="cuda")
    K = w.physics.n_batches
    with pytest.raises(G.GpumcdError) as e:    # fewer histories than batches
        ctx.finalize_tally_noalloc(pid, tid, t, 0, K - 1, dose)
    assert e.value.code == G.GMC_EINVAL
    with pytest.raises(G.GpumcdError) as e:    # beyond 2^32 histories
        ctx.finalize_tally_noalloc(pid, tid, t, 0, 1 << 33, dose)
    assert e.value.code == G.GMC_EINVAL
    L = G.lib()
    assert L.gmc_finalize_tally_noalloc(ctx._h, pid, tid, None, 0, 5_000, dose.data_ptr(), None, None) == G.GMC_EINVAL
    assert L.gmc_finalize_tally_noalloc(ctx._h, pid, tid, t.data_ptr(), 0, 5_000, None, None, None) == G.GMC_EINVAL
    assert L.gmc_finalize_tally_noalloc(ctx._h, 999999, tid, t.data_ptr(), 0, 5_000, dose.data_ptr(), None,
                                        None) == G.GMC_ENOTFOUND
    ctx.release(pid)
    ctx.release(tid)
