"""Python access to the FP64 CPU oracle (``gmc_oracle.c``).

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this module.  It never imports the
HIP package: inputs are duck-typed objects (phantom, materials, source,
physics) from the seeded input generators, and every number it returns comes
from the C oracle plus the plain statistics of the paper's Sec. II.D written
out below.

Statistics (Sec. II.D):
  * dose per history D_v = (1/N) sum_h E_vh / (rho_v V), converted to Gy;
  * Eq. 13: Delta D^2 = (<D^2> - <D>^2) / (N - 1), history by history;
  * the batch estimate over K batches, for cross-checking the HIP path's
    estimator.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gmc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liboracle.so")

MEV_TO_J = 1.602176634e-13


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
        os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "gmc_oracle.h"))
    ):
        os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
             "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Material(C.Structure):
    _fields_ = [("z_over_a", C.c_double), ("z_eff", C.c_double), ("i_ev", C.c_double)]


class _Phantom(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("rho", C.POINTER(C.c_float)), ("mat", C.POINTER(C.c_uint8))]


class _Source(C.Structure):
    _fields_ = [("particle", C.c_int), ("spectrum", C.c_int),
                ("e", C.c_double), ("e_lo", C.c_double), ("e_mode", C.c_double), ("e_hi", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("wx", C.c_double), ("wy", C.c_double),
                ("beam_id", C.c_uint32), ("tab_e", C.POINTER(C.c_double)), ("tab_w", C.POINTER(C.c_double)),
                ("tab_n", C.c_int)]


class _Physics(C.Structure):
    _fields_ = [("ecut", C.c_double), ("pcut", C.c_double), ("kcut", C.c_double), ("kc", C.c_double),
                ("esmax_gcm2", C.c_double), ("n_batches", C.c_int), ("test_mode", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("e_in", C.c_double), ("e_dep", C.c_double), ("e_esc", C.c_double), ("e_sink", C.c_double),
                ("n_hist", C.c_uint64), ("n_photon_events", C.c_uint64), ("n_fictitious", C.c_uint64),
                ("n_e_steps", C.c_uint64), ("n_hard", C.c_uint64), ("n_secondaries", C.c_uint64),
                ("n_majorant_violations", C.c_uint64)]


_lib = None

XS = {"mu_C": 0, "mu_pe": 1, "mu_pair": 2, "S_col": 3, "Sigma_M": 4, "E_M_hard": 5, "L_col": 6,
      "Sigma_B": 7, "L_rad": 8, "S_rad": 9, "L": 10, "inv_lambda1": 11, "eta": 12}
SAMPLERS = {"kn": 0, "sauter": 1, "pair": 2, "moller": 3, "brems": 4, "wentzel": 5}
EVENTS = {"compton": 0, "photo": 1, "pair": 2, "moller": 3, "brems": 4}


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        dp = C.POINTER(C.c_double)
        u32p = C.POINTER(C.c_uint32)
        u64p = C.POINTER(C.c_uint64)
        L.orc_philox4x32.argtypes = [u32p, u32p, u32p]
        L.orc_philox4x64.argtypes = [u64p, u64p, u64p]
        L.orc_child_path.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32]
        L.orc_child_path.restype = C.c_uint64
        L.orc_stream_words.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, C.c_int,
                                       u32p, dp]
        L.orc_xs.argtypes = [C.POINTER(_Material), C.c_int, dp, C.c_int, C.c_double, C.c_double, dp]
        L.orc_sample.argtypes = [C.c_int, C.c_double, C.c_double, C.c_uint64, C.c_int, dp, dp]
        L.orc_ms_screening_A.argtypes = [C.c_double]
        L.orc_ms_screening_A.restype = C.c_double
        L.orc_rotate.argtypes = [dp, C.c_double, C.c_double, dp]
        L.orc_grid_size.restype = C.c_int
        L.orc_majorants.argtypes = [C.POINTER(_Material), C.c_int, C.POINTER(_Phantom), C.POINTER(_Physics),
                                    dp, dp]
        L.orc_run.argtypes = [C.POINTER(_Material), C.c_int, C.POINTER(_Phantom), C.POINTER(_Source),
                              C.POINTER(_Physics), C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64,
                              dp, dp, dp, C.POINTER(_Stats)]
        L.orc_sample_source.argtypes = [C.POINTER(_Source), C.c_uint64, C.c_uint64, C.c_uint64, dp]
        L.orc_first_events.argtypes = [C.POINTER(_Material), C.c_int, C.POINTER(_Phantom), C.POINTER(_Source),
                                       C.POINTER(_Physics), C.c_uint64, C.c_uint64, C.c_uint64, dp, u32p]
        L.orc_event.argtypes = [C.c_int, C.c_double, C.c_double, dp, C.c_uint64, C.c_int, dp]
        L.orc_electron_tracks.argtypes = [C.POINTER(_Material), C.c_int, C.POINTER(_Phantom), C.POINTER(_Source),
                                          C.POINTER(_Physics), C.c_uint64, C.c_uint64, C.c_uint64, C.c_double, C.c_double,
                                          dp]
        L.orc_set_skin_fraction.argtypes = [C.c_double]
        L.orc_set_skin_fraction.restype = None
        _lib = L
    return _lib


def _ptr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


# ---------------------------------------------------------------- marshalling
def _materials(mats):
    arr = (_Material * len(mats))()
    for i, m in enumerate(mats):
        arr[i] = _Material(float(m.z_over_a), float(m.z_eff), float(m.i_ev))
    return arr


def _phantom(ph):
    rho = np.ascontiguousarray(ph.rho, dtype=np.float32)
    mat = np.ascontiguousarray(ph.mat, dtype=np.uint8)
    nz, ny, nx = rho.shape
    dx, dy, dz = ph.voxel
    p = _Phantom(nx, ny, nz, float(dx), float(dy), float(dz), _ptr(rho, C.c_float), _ptr(mat, C.c_uint8))
    return p, (rho, mat)


def _source(src):
    s = _Source(int(src.particle), int(src.spectrum), float(src.e), float(src.e_lo), float(src.e_mode),
                float(src.e_hi), float(src.cx), float(src.cy), float(src.wx), float(src.wy),
                int(src.beam_id))
    tab_e, tab_w = getattr(src, "tab_e", None), getattr(src, "tab_w", None)
    if tab_e is not None and tab_w is not None:
        e = np.ascontiguousarray(tab_e, dtype=np.float64)
        w = np.ascontiguousarray(tab_w, dtype=np.float64)
        s.tab_e, s.tab_w, s.tab_n = _ptr(e, C.c_double), _ptr(w, C.c_double), int(w.size)
        s._keep = (e, w)   # the arrays live as long as the structure
    return s


def sample_source(source, seed: int, h_begin: int, h_end: int) -> np.ndarray:
    """Primaries of histories [h_begin, h_end): rows (x, y, kinetic energy)."""
    src = _source(source)
    out = np.zeros((h_end - h_begin, 3))
    rc = lib().orc_sample_source(C.byref(src), C.c_uint64(seed), C.c_uint64(h_begin), C.c_uint64(h_end),
                                 _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError("invalid source")
    return out


def _physics(phys):
    return _Physics(float(phys.ecut), float(phys.pcut), float(phys.kcut), float(phys.kc),
                    float(phys.esmax_gcm2), int(phys.n_batches), int(phys.test_mode))


# ------------------------------------------------------------------- helpers
def philox4x32(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(o, C.c_uint32))
    return o


def philox4x64(ctr, key):
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    o = np.zeros(4, np.uint64)
    lib().orc_philox4x64(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(o, C.c_uint64))
    return o


def child_path(parent_path: int, parent_n: int, child_idx: int) -> int:
    return int(lib().orc_child_path(parent_path, parent_n, child_idx))


def stream_words(seed: int, beam: int, hist: int, path: int, n0: int, count: int):
    w = np.zeros(count, np.uint32)
    u = np.zeros(count, np.float64)
    lib().orc_stream_words(seed, beam, hist, path, n0, count, _ptr(w, C.c_uint32), _ptr(u, C.c_double))
    return w, u


def xs(material, which: str, energies, kcut: float = 0.0, kc: float = 0.0):
    e = np.ascontiguousarray(energies, dtype=np.float64)
    out = np.zeros_like(e)
    m = _Material(float(material.z_over_a), float(material.z_eff), float(material.i_ev))
    rc = lib().orc_xs(C.byref(m), XS[which], _ptr(e, C.c_double), e.size, kcut, kc, _ptr(out, C.c_double))
    assert rc == 0
    return out


def sample(which: str, p1: float, p2: float = 0.0, seed: int = 1, count: int = 100000):
    out = np.zeros(count)
    out2 = np.zeros(count)
    rc = lib().orc_sample(SAMPLERS[which], p1, p2, seed, count, _ptr(out, C.c_double), _ptr(out2, C.c_double))
    assert rc == 0
    return (out, out2) if which == "kn" else out


def event(which: str, e: float, p2: float = 0.0, direction=(0.0, 0.0, 1.0), seed: int = 1, count: int = 10000):
    """Outgoing particles of `count` events of kind `which` (compton, photo,
    pair, moller with p2 = kcut, brems with p2 = kc) for an incoming particle
    of energy e along `direction`, each on its own stream: rows (E_a, d_a,
    E_b, d_b) as returned by the transport's own event routine."""
    d = np.ascontiguousarray(direction, dtype=np.float64)
    out = np.zeros((count, 8))
    rc = lib().orc_event(EVENTS[which], e, p2, _ptr(d, C.c_double), seed, count, _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError("event below threshold or unknown")
    return out


def electron_tracks(materials, phantom, source, physics, seed: int, h_begin: int, h_end: int, path_cm: float,
                    z_start: float = 0.0):
    """Primary electrons of histories [h_begin, h_end) in test mode 3 or 4,
    started at depth z_start along +z and stopped after path_cm of path: rows
    (u, v, w, T, z), NaN where the electron left the phantom or fell below
    the cutoff first."""
    n = h_end - h_begin
    out = np.zeros((n, 5))
    mats = _materials(materials)
    ph, keep = _phantom(phantom)
    src = _source(source)
    phy = _physics(physics)
    rc = lib().orc_electron_tracks(mats, len(materials), C.byref(ph), C.byref(src), C.byref(phy), seed, h_begin,
                                   h_end, path_cm, z_start, _ptr(out, C.c_double))
    if rc != 0:
        raise ValueError("oracle rejected the input (code %d)" % rc)
    return out


def set_skin_fraction(f: float) -> None:
    """The electron voxel skin as a fraction of the smallest voxel width
    (default 1e-4), for this process and the workers it forks later."""
    lib().orc_set_skin_fraction(float(f))


def ms_screening_A(g1: float) -> float:
    return float(lib().orc_ms_screening_A(g1))


def rotate(d, cost: float, phi: float):
    a = np.ascontiguousarray(d, dtype=np.float64)
    o = np.zeros(3)
    lib().orc_rotate(_ptr(a, C.c_double), cost, phi, _ptr(o, C.c_double))
    return o


def grid_size() -> int:
    return int(lib().orc_grid_size())


def majorants(materials, phantom, physics):
    n = grid_size()
    mu = np.zeros(n)
    sg = np.zeros(n)
    mats = _materials(materials)
    ph, keep = _phantom(phantom)
    phy = _physics(physics)
    rc = lib().orc_majorants(mats, len(materials), C.byref(ph), C.byref(phy), _ptr(mu, C.c_double),
                             _ptr(sg, C.c_double))
    assert rc == 0
    return mu, sg


# ----------------------------------------------------------------- transport
@dataclass
class OracleResult:
    n_hist: int
    e1: np.ndarray            # sum_h E_vh, MeV, [nz, ny, nx]
    e2: np.ndarray            # sum_h E_vh^2
    eb: Optional[np.ndarray]  # per-batch sums [K, nz, ny, nx]
    stats: dict = field(default_factory=dict)


def run(materials, phantom, source, physics, seed: int, n_hist: int, h_begin: int = 0,
        h_end: Optional[int] = None, batches: bool = True) -> OracleResult:
    """Run histories [h_begin, h_end) of an n_hist-history beam."""
    if h_end is None:
        h_end = n_hist
    rho = np.asarray(phantom.rho)
    shape = rho.shape
    nv = rho.size
    K = max(int(physics.n_batches), 1)
    e1 = np.zeros(nv)
    e2 = np.zeros(nv)
    eb = np.zeros(K * nv) if batches else None
    st = _Stats()
    mats = _materials(materials)
    ph, keep = _phantom(phantom)
    src = _source(source)
    phy = _physics(physics)
    rc = lib().orc_run(mats, len(materials), C.byref(ph), C.byref(src), C.byref(phy), seed, h_begin, h_end,
                       n_hist, _ptr(e1, C.c_double), _ptr(e2, C.c_double),
                       _ptr(eb, C.c_double) if eb is not None else None, C.byref(st))
    if rc != 0:
        raise ValueError("oracle rejected the input (code %d)" % rc)
    stats = {name: getattr(st, name) for name, _ in _Stats._fields_}
    return OracleResult(h_end - h_begin, e1.reshape(shape), e2.reshape(shape),
                        eb.reshape((K,) + shape) if eb is not None else None, stats)


def _run_range(args):
    return run(*args)


def run_parallel(materials, phantom, source, physics, seed: int, n_hist: int, workers: int = 0,
                 batches: bool = True) -> OracleResult:
    """The plain oracle over disjoint history ranges in worker processes.

    Each worker runs the single-threaded oracle on its own range; the
    per-voxel sums are added.  Identical (up to FP64 summation order) to one
    run over all histories, because every history depends on its index only.
    """
    import multiprocessing as mp

    workers = workers or min(os.cpu_count() or 1, 16)
    if workers <= 1 or n_hist < 2 * workers:
        return run(materials, phantom, source, physics, seed, n_hist, batches=batches)
    build()
    edges = np.linspace(0, n_hist, workers + 1).astype(np.int64)
    jobs = [(materials, phantom, source, physics, seed, n_hist, int(a), int(b), batches)
            for a, b in zip(edges[:-1], edges[1:]) if b > a]
    ctx = mp.get_context("fork")
    with ctx.Pool(len(jobs)) as pool:
        parts = pool.map(_run_range, jobs)
    out = parts[0]
    for p in parts[1:]:
        out.e1 += p.e1
        out.e2 += p.e2
        if out.eb is not None:
            out.eb += p.eb
        for k in out.stats:
            out.stats[k] += p.stats[k]
        out.n_hist += p.n_hist
    return out


def first_events(materials, phantom, source, physics, seed: int, h_begin: int, h_end: int):
    n = h_end - h_begin
    xyz = np.zeros(3 * n)
    nu = np.zeros(n, np.uint32)
    mats = _materials(materials)
    ph, keep = _phantom(phantom)
    src = _source(source)
    phy = _physics(physics)
    rc = lib().orc_first_events(mats, len(materials), C.byref(ph), C.byref(src), C.byref(phy), seed, h_begin,
                                h_end, _ptr(xyz, C.c_double), _ptr(nu, C.c_uint32))
    if rc != 0:
        raise ValueError("oracle rejected the input (code %d)" % rc)
    return xyz.reshape(n, 3), nu


# ---------------------------------------------------------------- statistics
def dose(result: OracleResult, phantom, n_total: Optional[int] = None):
    """Dose per history (Gy) and its Eq. 13 uncertainty, history by history.

    D = <E>/(rho V); Delta D^2 = (<D^2> - <D>^2)/(N - 1).  Voxels with zero
    density report zero dose.
    """
    n = float(n_total if n_total is not None else result.n_hist)
    rho = np.asarray(phantom.rho, dtype=np.float64)
    vol = float(np.prod(phantom.voxel))
    with np.errstate(divide="ignore", invalid="ignore"):
        conv = np.where(rho > 0, MEV_TO_J / (rho * vol * 1e-3), 0.0)
    mean = result.e1 / n * conv
    mean2 = result.e2 / n * conv * conv
    var = np.maximum(mean2 - mean * mean, 0.0) / (n - 1.0)
    return mean, np.sqrt(var)


def batch_sigma(result: OracleResult, phantom, n_total: int):
    """Batch estimate of the uncertainty of the mean dose, K batches of
    histories h with k = h mod K: sigma^2 = sum_k n_k^2 (m_k - m)^2 /
    (N^2 (K-1)/K), m_k the per-history mean of batch k (equal-size batches
    give the textbook sum_k (m_k - m)^2 / (K (K-1)))."""
    K = result.eb.shape[0]
    h = np.arange(n_total, dtype=np.int64)
    nk = np.bincount(h % K, minlength=K).astype(np.float64)
    rho = np.asarray(phantom.rho, dtype=np.float64)
    vol = float(np.prod(phantom.voxel))
    with np.errstate(divide="ignore", invalid="ignore"):
        conv = np.where(rho > 0, MEV_TO_J / (rho * vol * 1e-3), 0.0)
    m = result.eb.sum(axis=0) / n_total
    mk = result.eb / nk[:, None, None, None]
    var = (nk[:, None, None, None] ** 2 * (mk - m) ** 2).sum(axis=0) / (n_total ** 2 * (K - 1) / K)
    return np.sqrt(var) * conv
