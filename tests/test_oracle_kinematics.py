"""Pins of the oracle's event kinematics: the outgoing particles of each
interaction, as produced by the very routines the transport calls
(``oracle.event``), against the conservation laws they must obey.

* Compton (Sec. II.A): E = E' + T; the photon's energy follows the Compton
  relation E' = E / (1 + (E/mc^2)(1 - cos theta)); the recoil electron carries
  the momentum the photon gave up, E d = E' d' + p_e d_e with
  p_e = sqrt(T (T + 2 mc^2)) -- which holds only if the relation and the
  electron's direction are both right.
* Moller (Sec. II.B.1): T = W + T'; both electrons' momenta add up to the
  incoming one (two-body kinematics on a free electron at rest), which fixes
  their polar angles and puts their azimuths pi apart.
* Bremsstrahlung (Sec. II.B.1): k + T' = T, the electron keeps its direction,
  the photon leaves at the polar angle mc^2/E.
* Pair: T1 + T2 = E - 2 mc^2, T1 uniform, azimuths pi apart; photoelectric:
  T = E.
* Every azimuth is uniform about the incoming direction.

The incoming direction is a general unit vector, so the rotation about it is
exercised with all three components non-zero.
"""
import numpy as np
import pytest
from scipy import stats

MC2 = 0.51099895
D0 = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])


def unit_ok(d):
    return np.allclose(np.linalg.norm(d, axis=1), 1.0, rtol=0, atol=1e-12)


def p_of(t):
    return np.sqrt(t * (t + 2 * MC2))


def azimuth(d, axis=D0):
    """Azimuth of each row of d about `axis` in a fixed transverse frame."""
    e1 = np.cross(axis, [1.0, 0.0, 0.0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(axis, e1)
    return np.arctan2(d @ e2, d @ e1)


def uniform_azimuth(phi):
    return stats.kstest((phi + np.pi) / (2 * np.pi), "uniform").pvalue > 1e-3


@pytest.mark.parametrize("e", [0.05, 1.0, 6.0, 15.0])
def test_compton_conservation(oracle, e):
    ev = oracle.event("compton", e, direction=D0, count=20000)
    e1, d1, t, dt = ev[:, 0], ev[:, 1:4], ev[:, 4], ev[:, 5:8]
    assert unit_ok(d1) and unit_ok(dt)
    assert np.allclose(e1 + t, e, rtol=1e-14, atol=0)
    cos = d1 @ D0
    assert np.allclose(e1, e / (1 + e / MC2 * (1 - cos)), rtol=1e-10, atol=0)
    mom = e * D0[None, :] - e1[:, None] * d1 - p_of(t)[:, None] * dt
    assert np.max(np.abs(mom)) < 1e-9 * e
    assert uniform_azimuth(azimuth(d1))
    # the electron leaves at the opposite azimuth and never backwards
    assert np.all(dt @ D0 > -1e-12)


@pytest.mark.parametrize("t,kcut", [(1.0, 0.2), (6.0, 0.7), (15.0, 0.7), (15.0, 0.01)])
def test_moller_two_body_kinematics(oracle, t, kcut):
    ev = oracle.event("moller", t, kcut, direction=D0, count=20000)
    w, dd, tp, dp = ev[:, 0], ev[:, 1:4], ev[:, 4], ev[:, 5:8]
    assert unit_ok(dd) and unit_ok(dp)
    assert np.allclose(w + tp, t, rtol=1e-14, atol=0)
    assert np.all(w >= kcut * (1 - 1e-12)) and np.all(w <= 0.5 * t * (1 + 1e-12))
    mom = p_of(t) * D0[None, :] - p_of(w)[:, None] * dd - p_of(tp)[:, None] * dp
    assert np.max(np.abs(mom)) < 1e-9 * p_of(t)
    assert uniform_azimuth(azimuth(dd))
    # both leave forward, on opposite sides of the incoming direction
    assert np.all(dd @ D0 > 0) and np.all(dp @ D0 > 0)
    tr_d = dd - (dd @ D0)[:, None] * D0
    tr_p = dp - (dp @ D0)[:, None] * D0
    assert np.all(np.sum(tr_d * tr_p, axis=1) <= 1e-12)


@pytest.mark.parametrize("t,kc", [(1.0, 0.01), (15.0, 0.01), (6.0, 0.5)])
def test_brems_photon_angle(oracle, t, kc):
    ev = oracle.event("brems", t, kc, direction=D0, count=20000)
    k, dg, te, de = ev[:, 0], ev[:, 1:4], ev[:, 4], ev[:, 5:8]
    assert unit_ok(dg)
    assert np.allclose(k + te, t, rtol=1e-14, atol=0)
    assert np.all(k >= kc * (1 - 1e-12)) and np.all(k <= t * (1 + 1e-12))
    assert np.array_equal(de, np.broadcast_to(D0, de.shape))
    assert np.allclose(dg @ D0, np.cos(MC2 / (t + MC2)), rtol=0, atol=1e-12)
    assert uniform_azimuth(azimuth(dg))


@pytest.mark.parametrize("e", [1.5, 6.0, 15.0])
def test_pair_energy_split_and_azimuths(oracle, e):
    ev = oracle.event("pair", e, direction=D0, count=20000)
    t1, d1, t2, d2 = ev[:, 0], ev[:, 1:4], ev[:, 4], ev[:, 5:8]
    avail = e - 2 * MC2
    assert unit_ok(d1) and unit_ok(d2)
    assert np.allclose(t1 + t2, avail, rtol=1e-13, atol=0)
    assert stats.kstest(t1 / avail, "uniform").pvalue > 1e-3
    tr1 = d1 - (d1 @ D0)[:, None] * D0
    tr2 = d2 - (d2 @ D0)[:, None] * D0
    n1, n2 = np.linalg.norm(tr1, axis=1), np.linalg.norm(tr2, axis=1)
    ok = (n1 > 1e-6) & (n2 > 1e-6)
    cosphi = np.sum(tr1[ok] * tr2[ok], axis=1) / (n1[ok] * n2[ok])
    assert np.allclose(cosphi, -1.0, atol=1e-9)
    assert uniform_azimuth(azimuth(d1))


def test_photoelectron_takes_the_photon_energy(oracle):
    ev = oracle.event("photo", 0.08, direction=D0, count=20000)
    assert np.all(ev[:, 0] == 0.08) and unit_ok(ev[:, 1:4])
    assert uniform_azimuth(azimuth(ev[:, 1:4]))


def test_events_refuse_below_threshold(oracle):
    with pytest.raises(ValueError):
        oracle.event("pair", 1.0, direction=D0, count=1)
    with pytest.raises(ValueError):
        oracle.event("moller", 0.3, 0.2, direction=D0, count=1)
    with pytest.raises(ValueError):
        oracle.event("brems", 0.01, 0.01, direction=D0, count=1)
