"""Seeded synthetic inputs: materials, phantoms, beams, physics settings.

This module holds data and seeded generators only -- no transport or
cross-section arithmetic -- so that the HIP path and the CPU oracle can be fed
identical inputs without sharing any of the method's code.

Workloads follow the paper's set-ups (Sec. II.D and Sec. III): monoenergetic
parallel beams entering a voxelized phantom along +z, a 64^3 grid of 0.5 cm
water voxels at 15 MeV (Table IV), slab heterogeneities of water, bone and lung
(Sec. III.A), plus ellipsoid phantoms with several materials for beamlet
batches and request streams.  No public dataset is involved; every array is
generated from a numpy ``default_rng`` seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

PHOTON, ELECTRON = 0, 1
MONO, TRIANGULAR, TABULATED = 0, 1, 2


@dataclass(frozen=True)
class Material:
    """Effective-element material: Z/A (mol/g), effective Z, mean excitation energy (eV)."""
    name: str
    z_over_a: float
    z_eff: float
    i_ev: float


# Approximate standard tissue values; any self-consistent set works because both
# sides read the same numbers.
WATER = Material("water", 0.55509, 7.42, 75.0)
LUNG = Material("lung", 0.55509, 7.42, 75.0)        # water composition, low density
BONE = Material("bone", 0.5213, 13.8, 106.4)
SOFT_TISSUE = Material("soft_tissue", 0.5512, 7.2, 72.3)
DEFAULT_MATERIALS: Tuple[Material, ...] = (LUNG, WATER, SOFT_TISSUE, BONE)


@dataclass
class Phantom:
    """Voxel densities (g/cm^3) and material indices, arrays [nz, ny, nx] (x fastest)."""
    rho: np.ndarray
    mat: np.ndarray
    voxel: Tuple[float, float, float]   # (dx, dy, dz) cm

    @property
    def shape(self):
        return self.rho.shape

    @property
    def extent(self):
        nz, ny, nx = self.rho.shape
        return (nx * self.voxel[0], ny * self.voxel[1], nz * self.voxel[2])


@dataclass
class Source:
    """Parallel beam along +z entering at z = 0 over a rectangular field."""
    particle: int = PHOTON
    spectrum: int = MONO
    e: float = 1.0
    e_lo: float = 0.0
    e_mode: float = 0.0
    e_hi: float = 0.0
    cx: float = 0.0
    cy: float = 0.0
    wx: float = 1.0
    wy: float = 1.0
    beam_id: int = 0
    tab_e: Optional[np.ndarray] = None   # TABULATED: tab_n + 1 increasing bin edges (MeV)
    tab_w: Optional[np.ndarray] = None   # TABULATED: tab_n bin weights
    first_history: int = 0               # number of the first history (a shard of a larger run)


@dataclass
class Physics:
    """Transport cutoffs (kinetic, MeV) and run options."""
    ecut: float = 0.2
    pcut: float = 0.01
    kcut: float = 0.0          # <= 0: equal to ecut
    kc: float = 0.0            # <= 0: equal to pcut
    esmax_gcm2: float = 0.0    # <= 0: no user step bound
    n_batches: int = 32
    test_mode: int = 0         # 0 full, 1 photon first collision, 2 electron CSDA straight-ahead
    majorant_margin: float = 0.0   # <= 0: the default 1.001


# ------------------------------------------------------------------ phantoms
def homogeneous(n: Sequence[int], voxel: float, material_index: int = 0, density: float = 1.0) -> Phantom:
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    rho = np.full((nz, ny, nx), density, np.float32)
    mat = np.full((nz, ny, nx), material_index, np.uint8)
    return Phantom(rho, mat, (float(voxel),) * 3)


def z_slabs(n: Sequence[int], voxel: float, slabs: Sequence[Tuple[float, int, float]]) -> Phantom:
    """Slabs along depth: ``slabs`` = [(z_end_cm, material_index, density), ...];
    the last slab runs to the end of the phantom."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    zc = (np.arange(nz) + 0.5) * voxel
    rho = np.empty((nz, ny, nx), np.float32)
    mat = np.empty((nz, ny, nx), np.uint8)
    start = 0.0
    for i, (zend, m, d) in enumerate(slabs):
        sel = (zc >= start) & ((zc < zend) | (i == len(slabs) - 1))
        rho[sel] = d
        mat[sel] = m
        start = zend
    return Phantom(rho, mat, (float(voxel),) * 3)


def material_from_density(rho: np.ndarray) -> np.ndarray:
    """Index into DEFAULT_MATERIALS: < 0.6 lung, < 1.1 water, < 1.4 soft tissue, else bone."""
    return np.select([rho < 0.6, rho < 1.1, rho < 1.4], [0, 1, 2], 3).astype(np.uint8)


def ellipsoids(n: Sequence[int], voxel: float, seed: int, count: int = 12,
               rho_range=(0.2, 1.9), axis_frac=(0.05, 0.35)) -> Phantom:
    """Water box with ``count`` seeded axis-aligned ellipsoids (later ones
    overwrite earlier ones); densities U(rho_range), materials from density."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else tuple(n)
    rng = np.random.default_rng(seed)
    ext = np.array([nx, ny, nz], np.float64) * voxel
    rho = np.ones((nz, ny, nx), np.float32)
    zc = ((np.arange(nz) + 0.5) * voxel)[:, None, None]
    yc = ((np.arange(ny) + 0.5) * voxel)[None, :, None]
    xc = ((np.arange(nx) + 0.5) * voxel)[None, None, :]
    def span(cen, axis, ncell):   # voxel centres within the ellipsoid's bounding box on one axis
        lo = max(int(np.floor((cen - axis) / voxel - 0.5)), 0)
        hi = min(int(np.ceil((cen + axis) / voxel + 0.5)) + 1, ncell)
        return slice(lo, max(lo, hi))

    for _ in range(count):
        c = rng.uniform(0, 1, 3) * ext
        a = rng.uniform(axis_frac[0], axis_frac[1], 3) * ext
        d = rng.uniform(*rho_range)
        sx, sy, sz = span(c[0], a[0], nx), span(c[1], a[1], ny), span(c[2], a[2], nz)
        inside = (((xc[:, :, sx] - c[0]) / a[0]) ** 2 + ((yc[:, sy, :] - c[1]) / a[1]) ** 2
                  + ((zc[sz, :, :] - c[2]) / a[2]) ** 2 <= 1.0)
        rho[sz, sy, sx][inside] = d
    return Phantom(rho, material_from_density(rho), (float(voxel),) * 3)


# ------------------------------------------------------------------ workloads
@dataclass
class Workload:
    name: str
    materials: Tuple[Material, ...]
    phantom: Phantom
    source: Source
    physics: Physics
    n_hist: int
    seed: int = 1
    extra: dict = field(default_factory=dict)


def centred(ph: Phantom, src: Source) -> Source:
    ex, ey, _ = ph.extent
    return replace(src, cx=ex / 2.0, cy=ey / 2.0)


def small_photon_water(n_hist: int = 100000) -> Workload:
    """1 MeV photons, 0.5 x 0.5 cm beam on 32^3 water at 0.5 cm; ECUT 0.2, PCUT 0.01."""
    ph = homogeneous(32, 0.5, 0)
    src = centred(ph, Source(PHOTON, MONO, 1.0, wx=0.5, wy=0.5))
    return Workload("photon_1MeV_water_32^3", (WATER,), ph, src, Physics(ecut=0.2, pcut=0.01), n_hist)


def water_15mev(particle: int, n_hist: int = None) -> Workload:
    """15 MeV parallel beam, 10 x 10 cm field, 64^3 water at 0.5 cm (Table IV set-up);
    1e6 electrons or 4e6 photons; ECUT 0.7 (kinetic), PCUT 0.01."""
    ph = homogeneous(64, 0.5, 0)
    src = centred(ph, Source(particle, MONO, 15.0, wx=10.0, wy=10.0))
    if n_hist is None:
        n_hist = 1_000_000 if particle == ELECTRON else 4_000_000
    name = "%s_15MeV_water_64^3" % ("electron" if particle == ELECTRON else "photon")
    return Workload(name, (WATER,), ph, src, Physics(ecut=0.7, pcut=0.01), n_hist)


def lung_box(particle: int, n_hist: int = None, lung_density: float = 0.26) -> Workload:
    """The paper's second geometry (Sec. III.A): 64^3 water at 0.5 cm with a lung
    box centred on the beam axis, 4.5 x 4.5 cm across; for electrons 4 cm long
    from a depth of 3 cm, for photons 6.5 cm long from 5.5 cm.  A voxel is lung
    when its centre lies inside the box or on its faces; the lateral faces fall
    on voxel centres of the 0.5 cm grid, so the box is 5 cm across here.  15 MeV, 10 x 10 cm field, 1e6
    electrons or 4e6 photons, ECUT 0.7 (kinetic), PCUT 0.01.  The lung density
    (not stated in the paper) is 0.26 g/cm^3, as in the slab phantom."""
    ph = homogeneous(64, 0.5, 0)
    z0, length = (3.0, 4.0) if particle == ELECTRON else (5.5, 6.5)
    ex, ey, _ = ph.extent
    nz, ny, nx = ph.shape
    c = (np.arange(64) + 0.5) * 0.5
    inx = np.abs(c - ex / 2.0) <= 2.25
    iny = np.abs(c - ey / 2.0) <= 2.25
    inz = (c >= z0) & (c < z0 + length)
    box = inz[:, None, None] & iny[None, :, None] & inx[None, None, :]
    ph.rho[box] = lung_density
    ph.mat[box] = 1
    src = centred(ph, Source(particle, MONO, 15.0, wx=10.0, wy=10.0))
    if n_hist is None:
        n_hist = 1_000_000 if particle == ELECTRON else 4_000_000
    name = "%s_15MeV_lung_box_64^3" % ("electron" if particle == ELECTRON else "photon")
    return Workload(name, (WATER, LUNG), ph, src, Physics(ecut=0.7, pcut=0.01), n_hist)


def tissue_lung_bone(particle: int, n_hist: int = None, tissue_density: float = 1.0,
                     lung_density: float = 0.26, bone_density: float = 1.85) -> Workload:
    """The paper's third geometry (Sec. III.A): 64^3 slabs at 0.5 cm along the
    beam, in the order the text gives (soft tissue, lung, bone, soft tissue):
    for electrons 2 cm of tissue, 2 cm of lung and 2 cm of bone; for photons 3,
    2 and 7 cm; soft tissue beyond.  15 MeV, 10 x 10 cm field, 1e6 electrons or
    4e6 photons, ECUT 0.7 (kinetic), PCUT 0.01.  The densities are not stated:
    soft tissue 1.0, lung 0.26 and bone 1.85 g/cm^3, as in the slab phantom."""
    t, l, b = (2.0, 2.0, 2.0) if particle == ELECTRON else (3.0, 2.0, 7.0)
    ph = z_slabs(64, 0.5, [(t, 0, tissue_density), (t + l, 1, lung_density), (t + l + b, 2, bone_density),
                           (32.0, 0, tissue_density)])
    src = centred(ph, Source(particle, MONO, 15.0, wx=10.0, wy=10.0))
    if n_hist is None:
        n_hist = 1_000_000 if particle == ELECTRON else 4_000_000
    name = "%s_15MeV_tissue_lung_bone_64^3" % ("electron" if particle == ELECTRON else "photon")
    return Workload(name, (SOFT_TISSUE, LUNG, BONE), ph, src, Physics(ecut=0.7, pcut=0.01), n_hist)


# The paper's divergence-reduction study (Sec. II.C.3, Table VI) as tunings of
# this engine.  "base": a particle stays on its lane until it ends and a
# wavefront takes new particles only when all 64 lanes are idle;
# "compaction_nN": particles are requeued after N events per visit (an
# electron's events are its steps, a photon's its interactions; the paper does
# not state its N); "pool": every lane takes the next particle as soon as it is
# idle; "both": requeue cadence 64 and refills at 4 idle lanes (the engine's
# defaults).  All of them allow 16 secondaries per visit (a particle that
# creates more is requeued); hard-event and absorption parking are part of
# every pass.
def _ablation(events: int, refill: int) -> dict:
    # the paper's two techniques alone: no requeue at the tail of a share
    return {"events_per_visit": events, "secondaries_per_visit": 16, "refill_lanes": refill, "tail_lanes": -1}


ABLATION_TUNINGS = {
    "base": _ablation(1 << 15, 64),
    "compaction_n4": _ablation(4, 64),
    "compaction_n16": _ablation(16, 64),
    "compaction_n64": _ablation(64, 64),
    "pool": _ablation(1 << 15, 1),
    "both": _ablation(64, 4),
}


def slab_6mev(n_hist: int = 40_000_000) -> Workload:
    """6 MeV photons, 10 x 10 cm, 128^3 at 0.25 cm: water 0-3 cm, bone (1.85) 3-5,
    lung (0.26) 5-12, water to the end."""
    mats = (WATER, BONE, LUNG)
    ph = z_slabs(128, 0.25, [(3.0, 0, 1.0), (5.0, 1, 1.85), (12.0, 2, 0.26), (32.0, 0, 1.0)])
    src = centred(ph, Source(PHOTON, MONO, 6.0, wx=10.0, wy=10.0))
    return Workload("photon_6MeV_slabs_128^3", mats, ph, src, Physics(ecut=0.7, pcut=0.01), n_hist)


def beamlets(seed: int = 11, phantom_seed: int = 7, n_beamlets: int = 256, shape=(200, 200, 160),
             voxel: float = 0.25) -> Tuple[Phantom, List[Source], np.ndarray]:
    """Pencil beamlets 0.5 x 0.5 cm on a 16 x 16 grid at 1 cm pitch, centred on an
    ellipsoid phantom; energies U(1, 20) MeV; photons:electrons 3:1 by seeded
    permutation; history counts log-uniform on [1e4, 1e6]."""
    ph = ellipsoids(shape, voxel, phantom_seed)
    rng = np.random.default_rng(seed)
    ex, ey, _ = ph.extent
    side = int(round(np.sqrt(n_beamlets)))
    kinds = np.array([PHOTON] * (n_beamlets * 3 // 4) + [ELECTRON] * (n_beamlets - n_beamlets * 3 // 4))
    kinds = rng.permutation(kinds)
    energies = rng.uniform(1.0, 20.0, n_beamlets)
    counts = np.round(10.0 ** rng.uniform(4.0, 6.0, n_beamlets)).astype(np.uint64)
    srcs = []
    for i in range(n_beamlets):
        gx, gy = i % side, i // side
        cx = ex / 2.0 + (gx - (side - 1) / 2.0) * 1.0
        cy = ey / 2.0 + (gy - (side - 1) / 2.0) * 1.0
        srcs.append(Source(int(kinds[i]), MONO, float(energies[i]), cx=cx, cy=cy, wx=0.5, wy=0.5, beam_id=i))
    return ph, srcs, counts


@dataclass
class BeamJob:
    """Several beams on one phantom, run as one job (the batched form)."""
    name: str
    materials: Tuple[Material, ...]
    phantom: Phantom
    sources: List[Source]
    counts: np.ndarray           # histories per beam, uint64
    physics: Physics
    seed: int = 1


def beamlet_job(n_beamlets: int = 256, shape=(200, 200, 160), voxel: float = 0.25, count_scale: float = 1.0,
                min_count: int = 1, seed: int = 11, phantom_seed: int = 7) -> BeamJob:
    """The pencil-beamlet batch on the ellipsoid phantom (four materials:
    lung, water, soft tissue, bone), ECUT 0.7 (kinetic) and PCUT 0.01 MeV as
    in the 15 MeV and slab set-ups.  ``count_scale`` shrinks every history
    count (for oracle-sized cases), never below ``min_count``."""
    ph, srcs, counts = beamlets(seed, phantom_seed, n_beamlets, shape, voxel)
    if count_scale != 1.0:
        counts = np.maximum(np.round(counts * count_scale), min_count).astype(np.uint64)
    name = "beamlets_%d_%dx%dx%d" % (n_beamlets, shape[0], shape[1], shape[2])
    return BeamJob(name, DEFAULT_MATERIALS, ph, srcs, counts, Physics(ecut=0.7, pcut=0.01))



@dataclass
class DoseRequest:
    """One request of the served form: a beam on one phantom of the pool."""
    phantom: int                 # index into the request stream's phantom pool
    source: Source
    n_hist: int
    seed: int


def request_stream(seed: int = 13, n_requests: int = 200, n_phantoms: int = 16, grid=(32, 256),
                   voxel=(0.25, 0.5), log10_hist=(5.0, 8.0)) -> Tuple[List[Phantom], List[DoseRequest]]:
    """Seeded dose requests: a pool of ellipsoid phantoms (cubic grids of
    U{grid} voxels of U(voxel) cm) that requests draw from, photons or
    electrons at 3:1, energy monoenergetic U(1, 20) MeV or triangular on
    [2, 18] MeV with mode 10 (even odds), square field U(1, 10) cm centred on
    the entry face, 10^U(log10_hist) histories.  ECUT/PCUT as in
    ``serving_physics``."""
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(n_phantoms):
        n = int(rng.integers(grid[0], grid[1] + 1))
        pool.append(ellipsoids(n, float(rng.uniform(*voxel)), seed=10_000 + 97 * seed + i))
    reqs = []
    for j in range(n_requests):
        k = int(rng.integers(n_phantoms))
        particle = ELECTRON if rng.random() < 0.25 else PHOTON
        side = float(rng.uniform(1.0, 10.0))
        if rng.random() < 0.5:
            src = Source(particle, MONO, float(rng.uniform(1.0, 20.0)), wx=side, wy=side, beam_id=j)
        else:
            src = Source(particle, TRIANGULAR, 10.0, e_lo=2.0, e_mode=10.0, e_hi=18.0, wx=side, wy=side, beam_id=j)
        reqs.append(DoseRequest(k, centred(pool[k], src), int(round(10.0 ** rng.uniform(*log10_hist))), 1 + j))
    return pool, reqs


def serving_physics() -> Physics:
    """Cutoffs of the served requests (as in the 15 MeV and slab set-ups)."""
    return Physics(ecut=0.7, pcut=0.01)


def poisson_arrivals(rate: float, n: int, seed: int = 17) -> np.ndarray:
    """Arrival times (s from the first) of a Poisson stream of n requests at ``rate`` per second."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n)
    gaps[0] = 0.0
    return np.cumsum(gaps)
