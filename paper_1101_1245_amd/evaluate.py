"""Dose-distribution evaluation of Sec. II.D: the statistical uncertainty s
(Eq. 12), the efficiency epsilon = 1/(s^2 T) (Eq. 11), the gamma index
(Eqs. 14-15) with the summary of Sec. III.A, and the z-test used to compare
two Monte Carlo estimates voxel by voxel.

Host-side numpy analysis of finished dose arrays; not part of the transport.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy import stats


def uncertainty_s(dose: np.ndarray, sigma: np.ndarray, frac: float = 0.2) -> float:
    """Eq. 12: mean relative uncertainty over voxels with D > frac * D_max."""
    sel = dose > frac * dose.max()
    if not np.any(sel):
        return float("nan")
    return float(np.mean(sigma[sel] / dose[sel]))


def efficiency(s: float, t: float) -> float:
    """Eq. 11."""
    return 1.0 / (s * s * t)


def histories_for(s0: float, n0: int, target: float = 0.01) -> int:
    """Histories needed to reach uncertainty ``target`` given s0 at n0 (s ~ 1/sqrt(N))."""
    return int(math.ceil(n0 * (s0 / target) ** 2))


# ------------------------------------------------------------------ gamma
def _trilinear(d: np.ndarray, pts: np.ndarray) -> np.ndarray:
    """Trilinear interpolation of d[z, y, x] at fractional voxel-centre indices pts (n, 3) in (z, y, x);
    values outside the grid are clamped to the edge voxels."""
    nz, ny, nx = d.shape
    p = np.empty_like(pts)
    p[:, 0] = np.clip(pts[:, 0], 0, nz - 1)
    p[:, 1] = np.clip(pts[:, 1], 0, ny - 1)
    p[:, 2] = np.clip(pts[:, 2], 0, nx - 1)
    i0 = np.minimum(np.floor(p).astype(np.int64), np.array([nz - 2, ny - 2, nx - 2]).clip(min=0))
    f = p - i0
    out = np.zeros(len(pts))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (f[:, 0] if dz else 1 - f[:, 0]) * (f[:, 1] if dy else 1 - f[:, 1]) * (f[:, 2] if dx else 1 - f[:, 2])
                iz = np.minimum(i0[:, 0] + dz, nz - 1)
                iy = np.minimum(i0[:, 1] + dy, ny - 1)
                ix = np.minimum(i0[:, 2] + dx, nx - 1)
                out += w * d[iz, iy, ix]
    return out


@dataclass
class GammaResult:
    gamma: np.ndarray          # per selected reference voxel
    pass_rate: float           # fraction with gamma <= 1
    gamma_max: float
    gamma_avg: float
    n_voxels: int
    n_fail_1: int              # gamma > 1.0
    n_fail_12: int             # gamma > 1.2


def gamma_index(ref: np.ndarray, ev: np.ndarray, voxel, dose_tol: float = 0.02, dist_tol_cm: float = 0.2,
                threshold: float = 0.1, step_cm: float = None, radius_factor: float = 3.0) -> GammaResult:
    """Global gamma (Eqs. 14-15) of the evaluated dose ``ev`` against ``ref``.

    Dose criterion dose_tol * max(ref); distance criterion dist_tol_cm; the
    evaluated dose is trilinearly interpolated and searched on a grid of
    spacing step_cm (default dist_tol/5) within radius_factor * dist_tol of
    each reference voxel centre with ref > threshold * max(ref).
    """
    voxel = np.asarray(voxel, dtype=np.float64)  # (dx, dy, dz)
    dmax = float(ref.max())
    dD = dose_tol * dmax
    sel = np.argwhere(ref > threshold * dmax)     # (n, 3) as (z, y, x)
    if step_cm is None:
        step_cm = dist_tol_cm / 5.0
    r = radius_factor * dist_tol_cm
    k = int(math.ceil(r / step_cm))
    ax = np.arange(-k, k + 1) * step_cm
    oz, oy, ox = np.meshgrid(ax, ax, ax, indexing="ij")
    off = np.stack([oz.ravel(), oy.ravel(), ox.ravel()], axis=1)
    dist2 = (off ** 2).sum(axis=1)
    keep = dist2 <= r * r + 1e-12
    off, dist2 = off[keep], dist2[keep]
    order = np.argsort(dist2)
    off, dist2 = off[order], dist2[order]
    scale = np.array([voxel[2], voxel[1], voxel[0]])   # cm per index along z, y, x
    refv = ref[sel[:, 0], sel[:, 1], sel[:, 2]]
    best = np.full(len(sel), np.inf)
    base = sel.astype(np.float64)
    for o, d2 in zip(off, dist2):
        g_dist = d2 / dist_tol_cm ** 2
        active = best > g_dist
        if not np.any(active):
            break
        pts = base[active] + o / scale
        val = _trilinear(ev, pts)
        g2 = g_dist + ((val - refv[active]) / dD) ** 2
        idx = np.nonzero(active)[0]
        best[idx] = np.minimum(best[idx], g2)
    g = np.sqrt(best)
    return GammaResult(g, float(np.mean(g <= 1.0)), float(g.max()) if g.size else 0.0,
                       float(g.mean()) if g.size else 0.0, int(g.size), int(np.sum(g > 1.0)), int(np.sum(g > 1.2)))


# ------------------------------------------------------------------ precision
@dataclass
class PrecisionError:
    n: int               # voxels with ref > threshold * max(ref)
    sum_rel: float       # sum(ev) / sum(ref) - 1 over those voxels
    mean_abs: float      # mean |ev - ref| / max(ref) over those voxels
    max_abs: float       # max |ev - ref| / max(ref) over those voxels


def precision_error(ev: np.ndarray, ref: np.ndarray, threshold: float = 0.1) -> PrecisionError:
    """Difference of a dose ``ev`` from a reference dose ``ref`` computed on
    the same random streams (FP32 transport against the FP64 one): the
    relative difference of the summed dose and the mean and largest voxel
    difference in units of the reference maximum, over voxels above
    ``threshold`` of that maximum."""
    dmax = float(ref.max())
    sel = ref > threshold * dmax
    n = int(sel.sum())
    if n == 0:
        return PrecisionError(0, 0.0, 0.0, 0.0)
    diff = np.abs(ev[sel] - ref[sel]) / dmax
    return PrecisionError(n, float(ev[sel].sum() / ref[sel].sum() - 1.0), float(diff.mean()), float(diff.max()))


# ------------------------------------------------------------------ z-test
@dataclass
class ZTest:
    n: int
    z: np.ndarray
    frac_over_3: float
    frac_limit: float
    max_abs: float
    max_limit: float
    mean: float
    mean_limit: float
    var: float
    var_range: tuple
    passed: bool


LSB_MEV = 2.0 ** -27
MEV_TO_J = 1.602176634e-13


def batch_doses(batch_energy, rho, voxel, n_hist_total: int, h0: int = 0):
    """Per-batch dose per history D_k[v] (Gy) and the batch sizes n_k from
    batch energy sums (MeV; history h in batch h mod K), for histories
    [h0, h0 + N)."""
    e = np.asarray(batch_energy, dtype=np.float64)
    K = e.shape[0]
    h = np.arange(h0, h0 + n_hist_total, dtype=np.int64)
    nk = np.bincount(h % K, minlength=K).astype(np.float64)
    rho = np.asarray(rho, dtype=np.float64)
    vol = float(np.prod(voxel))
    with np.errstate(divide="ignore", invalid="ignore"):
        conv = np.where(rho > 0, MEV_TO_J / (rho * vol * 1e-3), 0.0)
    return e / nk.reshape((K,) + (1,) * (e.ndim - 1)) * conv, nk


def weighted_sum_se(dk, nk, w):
    """Standard error of sum_v w_v D_v, D = sum_k n_k D_k / N, from the spread
    of the K batch values Y_k = sum_v w_v D_k,v (the batch estimator of Eq.
    13): var = sum_k n_k^2 (Y_k - Y)^2 / (N^2 (K - 1)/K).  It carries every
    covariance between voxels that share histories."""
    K = dk.shape[0]
    y = np.array([np.sum(w * dk[k]) for k in range(K)])
    n = nk.sum()
    m = np.sum(nk * y) / n
    return math.sqrt(np.sum(nk * nk * (y - m) ** 2) / (n * n * (K - 1) / K))


def z_test(d_a, s_a, d_b, s_b, ref_for_mask=None, threshold: float = 0.1, dof: int = 31,
           same_streams: bool = False, dof_b: float = None, batches=None) -> ZTest:
    """Voxel-by-voxel agreement of two Monte Carlo estimates.

    Over voxels with ref > threshold * max(ref) (ref defaults to d_b),
    z = (d_a - d_b)/sqrt(s_a^2 + s_b^2).  A literal "every voxel within 3
    sigma" fails voxels by chance, so the test asks:

    * the fraction with |z| > 3 is at most p + 3 sqrt(p/n), p the expected
      fraction: the mean over the voxels of P(|t_nu| > 3), nu each voxel's
      Welch-Satterthwaite degrees of freedom (``dof`` for s_a, a batch
      estimate; ``dof_b`` for s_b, None for a history-by-history estimate,
      whose degrees of freedom are practically infinite) -- with an
      estimated sigma z has heavier tails than a normal variate, and
      P(|t_31| > 3) = 0.53% against 0.27%;
    * max |z| below the two-sided Bonferroni bound at alpha = 1e-3 over the n
      voxels, for the smallest nu;
    * |mean z| <= 3/sqrt(n) -- or, with ``batches`` = ((Dk_a, nk_a), (Dk_b,
      nk_b)) the per-batch doses of both estimates (independent runs), within
      t(K - 1) at the 3-sigma level of its own standard error: mean z is the
      weighted sum sum_v (d_a - d_b)_v / (n sigma_v) of dose differences,
      whose batch spread includes the correlation of voxels that share
      histories (a photon history deposits in many voxels), which 3/sqrt(n)
      -- the bound for independent voxels -- leaves out;
    * var z in [0.8, 1.25].

    With ``same_streams`` the two runs drew the same random streams, so their
    estimates are positively correlated and z has a variance below one
    (equal to zero for identical trajectories); the lower variance bound is
    then dropped and the other bounds, which only tighten, are kept.
    """
    ref = d_b if ref_for_mask is None else ref_for_mask
    sel = ref > threshold * ref.max()
    va, vb = s_a[sel] ** 2, s_b[sel] ** 2
    den = np.sqrt(va + vb)
    den = np.where(den > 0, den, np.inf)
    z = (d_a[sel] - d_b[sel]) / den
    n = int(z.size)
    with np.errstate(divide="ignore", invalid="ignore"):
        tail_b = vb * vb / dof_b if dof_b else 0.0
        nu = np.where(va > 0, (va + vb) ** 2 / (va * va / dof + tail_b), np.inf)
    nu = np.clip(np.nan_to_num(nu, nan=1e9, posinf=1e9), dof, 1e9)
    p3 = float(np.mean(2.0 * stats.t.sf(3.0, nu))) if n else 0.0027
    frac = float(np.mean(np.abs(z) > 3.0)) if n else 0.0
    frac_lim = p3 + 3.0 * math.sqrt(p3 / max(n, 1))
    max_lim = float(stats.t.isf(1e-3 / (2.0 * max(n, 1)), float(nu.min()) if n else dof))
    mean = float(np.mean(z)) if n else 0.0
    mean_lim = 3.0 / math.sqrt(max(n, 1))
    if batches is not None and n:
        (dka, nka), (dkb, nkb) = batches
        w = np.zeros(np.shape(d_a))
        w[sel] = 1.0 / (n * den)
        se = math.hypot(weighted_sum_se(dka, nka, w), weighted_sum_se(dkb, nkb, w))
        kk = min(dka.shape[0], dkb.shape[0]) - 1
        mean_lim = float(stats.t.isf(0.00135, kk)) * se
    var = float(np.var(z)) if n else 1.0
    vr = (0.0 if same_streams else 0.8, 1.25)
    ok = n > 0 and frac <= frac_lim and float(np.max(np.abs(z))) <= max_lim and abs(mean) <= mean_lim \
        and vr[0] <= var <= vr[1]
    return ZTest(n, z, frac, frac_lim, float(np.max(np.abs(z))) if n else 0.0, max_lim, mean, mean_lim, var, vr, ok)


def describe(zt: ZTest) -> str:
    """One line with the z-test's statistics and their bounds."""
    return ("n %d, frac |z|>3 %.5f (<= %.5f), max |z| %.2f (<= %.2f), mean z %+.4f (<= %.4f), var z %.3f in "
            "[%.2f, %.2f] -> %s" % (zt.n, zt.frac_over_3, zt.frac_limit, zt.max_abs, zt.max_limit, zt.mean,
                                     zt.mean_limit, zt.var, zt.var_range[0], zt.var_range[1],
                                     "pass" if zt.passed else "FAIL"))
