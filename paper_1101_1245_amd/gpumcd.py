"""Thin ctypes binding of the C ABI in ``include/gpumcd.h``.

Argument marshalling only: every step of the transport runs in the gfx950
kernels of ``libgpumcd.so``.  There is no CPU fallback -- if the library is not
built, or no GPU is present, these functions raise.

PyTorch is used, when asked for, only to own device output buffers and to hand
the library the current HIP stream.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libgpumcd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gpumcd.h")

GMC_OK, GMC_EINVAL, GMC_ENOMEM, GMC_EDEVICE, GMC_ENOTFOUND, GMC_EBUSY, GMC_EOVERFLOW, GMC_EINTERNAL = \
    0, -1, -2, -3, -4, -5, -6, -7
GMC_HOST, GMC_DEVICE = 0, 1
_CODES = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ENOTFOUND", -5: "EBUSY", -6: "EOVERFLOW",
          -7: "EINTERNAL"}


class GpumcdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("gpumcd %s (%d): %s" % (_CODES.get(code, "?"), code, msg))
        self.code = code


class gmc_material(C.Structure):
    _fields_ = [("z_over_a", C.c_double), ("z_eff", C.c_double), ("i_ev", C.c_double)]


class gmc_physics(C.Structure):
    _fields_ = [("ecut_mev", C.c_double), ("pcut_mev", C.c_double), ("kcut_mev", C.c_double),
                ("kc_mev", C.c_double), ("esmax_gcm2", C.c_double), ("n_batches", C.c_int),
                ("test_mode", C.c_int), ("majorant_margin", C.c_double)]


class gmc_source(C.Structure):
    _fields_ = [("particle", C.c_int), ("spectrum", C.c_int), ("e_mev", C.c_double), ("e_lo", C.c_double),
                ("e_mode", C.c_double), ("e_hi", C.c_double), ("cx_cm", C.c_double), ("cy_cm", C.c_double),
                ("wx_cm", C.c_double), ("wy_cm", C.c_double), ("beam_id", C.c_uint32),
                ("tab_e", C.POINTER(C.c_double)), ("tab_w", C.POINTER(C.c_double)), ("tab_n", C.c_int),
                ("first_history", C.c_uint64)]


class gmc_run_stats(C.Structure):
    _fields_ = [("t_total_s", C.c_double), ("t_device_s", C.c_double), ("e_in_mev", C.c_double),
                ("e_dep_mev", C.c_double), ("e_esc_mev", C.c_double), ("e_sink_mev", C.c_double),
                ("n_hist", C.c_uint64), ("n_photon_events", C.c_uint64), ("n_fictitious", C.c_uint64),
                ("n_e_steps", C.c_uint64), ("n_hard", C.c_uint64), ("n_secondaries", C.c_uint64),
                ("n_majorant_violations", C.c_uint64), ("n_passes", C.c_uint64),
                ("ledger_residual_lsb", C.c_int64), ("t_photon_pass_s", C.c_double),
                ("t_electron_pass_s", C.c_double), ("n_photon_launches", C.c_uint64),
                ("n_electron_launches", C.c_uint64), ("s_rel", C.c_double), ("t_round_s", C.c_double),
                ("n_round_launches", C.c_uint64), ("n_photon_interactions", C.c_uint64)]


class gmc_tuning(C.Structure):
    _fields_ = [("events_per_visit", C.c_int), ("secondaries_per_visit", C.c_int), ("chunk", C.c_int),
                ("wg_size", C.c_int), ("pass_items", C.c_int), ("wave_items", C.c_int),
                ("rounds_per_check", C.c_int), ("refill_lanes", C.c_int), ("energy_sort", C.c_int),
                ("tail_lanes", C.c_int), ("queue_items", C.c_int), ("persistent", C.c_int),
                ("aggregate", C.c_int)]


class gmc_autotune_report(C.Structure):
    _fields_ = [("trials", C.c_int), ("from_cache", C.c_int), ("complete", C.c_int),
                ("sample_histories", C.c_uint64), ("t_default_s", C.c_double), ("t_best_s", C.c_double)]


class gmc_server_config(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("max_slots", C.c_int)]


class gmc_request_stats(C.Structure):
    _fields_ = [("t_queue_s", C.c_double), ("t_run_s", C.c_double), ("t_latency_s", C.c_double),
                ("run", gmc_run_stats)]


class gmc_server_status_t(C.Structure):
    _fields_ = [("running", C.c_int), ("pending", C.c_int), ("in_flight", C.c_int),
                ("finished_unpolled", C.c_int), ("budget_bytes", C.c_size_t)]


_lib = None


def header_symbols():
    """Names of the functions declared in include/gpumcd.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gmc_[a-z_0-9]+)\s*\(", text)))


def lib():
    """Load libgpumcd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libgpumcd.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    try:
        # torch bundles its own HIP runtime under the same soname; loading it
        # first makes the library bind to that copy, so the process has a
        # single HIP runtime and torch tensors/streams stay usable beside it.
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    dp = C.POINTER(C.c_double)
    L.gmc_create.argtypes = [C.c_int, vp, C.POINTER(vp)]
    L.gmc_destroy.argtypes = [vp]
    L.gmc_destroy.restype = None
    L.gmc_last_error.argtypes = [vp]
    L.gmc_last_error.restype = C.c_char_p
    L.gmc_load_tables.argtypes = [vp, C.POINTER(gmc_material), C.c_int, C.POINTER(gmc_physics),
                                  C.POINTER(C.c_int32)]
    L.gmc_load_phantom.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, vp, vp,
                                   C.c_int, C.POINTER(C.c_int32)]
    L.gmc_release.argtypes = [vp, C.c_int32]
    L.gmc_run_beam.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(gmc_source), C.c_uint64, C.c_uint64, vp, vp,
                               C.c_int, C.POINTER(gmc_tuning), C.POINTER(gmc_run_stats)]
    L.gmc_run_beams.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(gmc_source), C.POINTER(C.c_uint64), C.c_int,
                                C.c_uint64, C.POINTER(vp), C.POINTER(vp), vp, vp, C.c_int, C.POINTER(gmc_tuning),
                                C.POINTER(gmc_run_stats)]
    L.gmc_autotune.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(gmc_source), C.POINTER(C.c_uint64), C.c_int,
                               C.c_double, C.POINTER(gmc_tuning), C.POINTER(gmc_autotune_report)]
    L.gmc_server_start.argtypes = [vp, C.POINTER(gmc_server_config)]
    L.gmc_server_stop.argtypes = [vp]
    L.gmc_submit.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(gmc_source), C.c_uint64, C.c_uint64,
                             C.POINTER(C.c_uint64)]
    L.gmc_poll.argtypes = [vp, C.c_uint64, C.c_int, C.POINTER(C.c_int), vp, vp, C.c_int,
                           C.POINTER(gmc_request_stats)]
    L.gmc_server_status.argtypes = [vp, C.POINTER(gmc_server_status_t)]
    L.gmc_rng_words.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, C.c_int,
                                C.POINTER(C.c_uint32)]
    L.gmc_table_eval.argtypes = [vp, C.c_int32, C.c_int, C.c_int, dp, C.c_int, dp]
    L.gmc_atomic_rate.argtypes = [vp, C.c_int, C.c_int, C.POINTER(C.c_double)]
    L.gmc_first_events.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(gmc_source), C.c_uint64, C.c_uint32,
                                   C.c_uint32, C.POINTER(C.c_float), C.POINTER(C.c_uint32)]
    L.gmc_run_beam_tally.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(gmc_source), C.c_uint64, C.c_uint64, vp,
                                     C.c_int, C.POINTER(gmc_tuning), C.POINTER(gmc_run_stats)]
    L.gmc_finalize_tally.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_int, C.c_uint64, C.c_uint64, vp, vp, C.c_int,
                                     C.POINTER(C.c_double)]
    L.gmc_finalize_tally_noalloc.argtypes = [vp, C.c_int32, C.c_int32, vp, C.c_uint64, C.c_uint64, vp, vp,
                                             C.POINTER(C.c_double)]
    L.gmc_phantom_dims.argtypes = [vp, C.c_int32, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    _lib = L
    return L


def _src(s, keep: list) -> gmc_source:
    """The C source of `s`; a tabulated spectrum's tables go into `keep`,
    which the caller holds until the call that reads them has returned."""
    out = gmc_source(int(s.particle), int(s.spectrum), float(s.e), float(s.e_lo), float(s.e_mode), float(s.e_hi),
                     float(s.cx), float(s.cy), float(s.wx), float(s.wy), int(s.beam_id))
    out.first_history = int(getattr(s, "first_history", 0))
    tab_e, tab_w = getattr(s, "tab_e", None), getattr(s, "tab_w", None)
    if tab_e is not None and tab_w is not None:
        e = np.ascontiguousarray(tab_e, dtype=np.float64)
        w = np.ascontiguousarray(tab_w, dtype=np.float64)
        keep.append((e, w))
        out.tab_e = e.ctypes.data_as(C.POINTER(C.c_double))
        out.tab_w = w.ctypes.data_as(C.POINTER(C.c_double))
        out.tab_n = int(w.size)
    return out


def _phys(p) -> gmc_physics:
    return gmc_physics(float(p.ecut), float(p.pcut), float(p.kcut), float(p.kc), float(p.esmax_gcm2),
                       int(p.n_batches), int(p.test_mode), float(getattr(p, "majorant_margin", 0.0)))


def _tuning(t) -> Optional[gmc_tuning]:
    if t is None:
        return None
    if isinstance(t, gmc_tuning):
        return t
    unknown = set(t) - {f for f, _ in gmc_tuning._fields_}
    if unknown:
        raise ValueError("unknown tuning keys: %s" % sorted(unknown))
    return gmc_tuning(*[int(t.get(f, 0)) for f, _ in gmc_tuning._fields_])


def stats_dict(st: gmc_run_stats) -> dict:
    return {name: getattr(st, name) for name, _ in gmc_run_stats._fields_}


class Context:
    """One gmc_context on a HIP device (optionally on torch's current stream)."""

    def __init__(self, device: int = 0, use_torch_stream: bool = False):
        L = lib()
        stream = None
        if use_torch_stream:
            import torch
            stream = C.c_void_p(torch.cuda.current_stream(device).cuda_stream)
        h = C.c_void_p()
        rc = L.gmc_create(device, stream, C.byref(h))
        if rc != GMC_OK:
            raise GpumcdError(rc, "gmc_create failed (no HIP device %d?)" % device)
        self._h = h
        self._L = L
        self._tickets = {}   # ticket -> phantom id, for the output shape of gmc_poll
        self._nbatch = {}    # tables id -> n_batches

    def close(self):
        if getattr(self, "_h", None):
            self._L.gmc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, rc):
        if rc != GMC_OK:
            msg = self._L.gmc_last_error(self._h)
            raise GpumcdError(rc, msg.decode() if msg else "")

    # ------------------------------------------------------------ handles
    def load_tables(self, materials, physics) -> int:
        arr = (gmc_material * len(materials))(*[gmc_material(m.z_over_a, m.z_eff, m.i_ev) for m in materials])
        tid = C.c_int32()
        ph = _phys(physics)
        self._check(self._L.gmc_load_tables(self._h, arr, len(materials), C.byref(ph), C.byref(tid)))
        self._nbatch[tid.value] = int(physics.n_batches) if int(physics.n_batches) > 0 else 32
        return tid.value

    def load_phantom(self, phantom) -> int:
        rho = np.ascontiguousarray(phantom.rho, dtype=np.float32)
        mat = np.ascontiguousarray(phantom.mat, dtype=np.uint8)
        nz, ny, nx = rho.shape
        dx, dy, dz = phantom.voxel
        pid = C.c_int32()
        self._check(self._L.gmc_load_phantom(self._h, nx, ny, nz, dx, dy, dz, rho.ctypes.data, mat.ctypes.data,
                                             GMC_HOST, C.byref(pid)))
        return pid.value

    def release(self, handle: int):
        self._check(self._L.gmc_release(self._h, handle))

    def phantom_shape(self, phantom_id: int):
        """(nz, ny, nx) of a loaded phantom: the shape of every dose output on it."""
        nx, ny, nz = C.c_int(), C.c_int(), C.c_int()
        self._check(self._L.gmc_phantom_dims(self._h, phantom_id, C.byref(nx), C.byref(ny), C.byref(nz)))
        return (nz.value, ny.value, nx.value)

    def _out_shape(self, phantom_id: int, shape):
        """The phantom's (nz, ny, nx); a given shape must hold exactly its voxels
        (the library writes nx*ny*nz doubles into every output)."""
        real = self.phantom_shape(phantom_id)
        if shape is not None and int(np.prod(shape)) != int(np.prod(real)):
            raise ValueError("output shape %s does not match the phantom's %s" % (tuple(shape), real))
        return tuple(shape) if shape is not None else real

    # --------------------------------------------------------------- runs
    def run_beam(self, phantom_id: int, tables_id: int, source, n_hist: int, seed: int, shape=None,
                 tuning=None, sigma: bool = True, out: str = "numpy"):
        """Dose (Gy/history) and sigma per voxel, plus run statistics.

        out="numpy": host arrays; out="torch": float64 tensors on the context's
        GPU written directly by the finalize kernel."""
        st = gmc_run_stats()
        keep = []
        src = _src(source, keep)
        tun = _tuning(tuning)
        tun_p = C.byref(tun) if tun is not None else None
        shape = self._out_shape(phantom_id, shape)
        n = int(np.prod(shape))
        if out == "torch":
            import torch
            d = torch.empty(n, dtype=torch.float64, device="cuda")
            s = torch.empty(n, dtype=torch.float64, device="cuda") if sigma else None
            rc = self._L.gmc_run_beam(self._h, phantom_id, tables_id, C.byref(src), n_hist, seed, d.data_ptr(),
                                      s.data_ptr() if s is not None else None, GMC_DEVICE, tun_p, C.byref(st))
            self._check(rc)
            return d.view(*shape), (s.view(*shape) if s is not None else None), stats_dict(st)
        d = np.empty(n, np.float64)
        s = np.empty(n, np.float64) if sigma else None
        rc = self._L.gmc_run_beam(self._h, phantom_id, tables_id, C.byref(src), n_hist, seed, d.ctypes.data,
                                  s.ctypes.data if s is not None else None, GMC_HOST, tun_p, C.byref(st))
        self._check(rc)
        return d.reshape(shape), (s.reshape(shape) if s is not None else None), stats_dict(st)

    def run_beams(self, phantom_id: int, tables_id: int, sources, n_hist, seed: int, shape=None, tuning=None,
                  per_beam: bool = False, per_beam_sigma: bool = False, sigma: bool = True, out: str = "numpy"):
        """Batched form: several beams in one job.  Returns (per_beam_dose or
        None, per_beam_sigma or None, combined_dose, combined_sigma or None,
        stats); per-beam arrays have shape (n_beams, nz, ny, nx)."""
        shape = self._out_shape(phantom_id, shape)
        nb = len(sources)
        if nb != len(n_hist):
            raise ValueError("one history count per source")
        st = gmc_run_stats()
        keep = []
        srcs = (gmc_source * nb)(*[_src(s, keep) for s in sources])
        counts = (C.c_uint64 * nb)(*[int(n) for n in n_hist])
        tun = _tuning(tuning)
        tun_p = C.byref(tun) if tun is not None else None
        n = int(np.prod(shape))
        if out == "torch":
            import torch
            mk = lambda *sz: torch.empty(*sz, dtype=torch.float64, device="cuda")  # noqa: E731
            ptr = lambda a: a.data_ptr()  # noqa: E731
            kind = GMC_DEVICE
        else:
            mk = lambda *sz: np.empty(sz, np.float64)  # noqa: E731
            ptr = lambda a: a.ctypes.data  # noqa: E731
            kind = GMC_HOST
        d = mk(n)
        s = mk(n) if sigma else None

        def rows(a):
            return (C.c_void_p * nb)(*[ptr(a) + b * n * 8 for b in range(nb)]) if a is not None else None

        pb = mk(nb, n) if per_beam else None
        ps = mk(nb, n) if per_beam_sigma else None
        rc = self._L.gmc_run_beams(self._h, phantom_id, tables_id, srcs, counts, nb, seed, rows(pb), rows(ps), ptr(d),
                                   ptr(s) if s is not None else None, kind, tun_p, C.byref(st))
        self._check(rc)
        rs = lambda a, sh: a.reshape(*sh) if a is not None else None  # noqa: E731
        per = (nb,) + tuple(shape)
        return rs(pb, per), rs(ps, per), rs(d, tuple(shape)), rs(s, tuple(shape)), stats_dict(st)

    def run_beam_tally(self, phantom_id: int, tables_id: int, source, n_hist: int, seed: int, tuning=None,
                       out: str = "numpy"):
        """Raw integer batch tallies (uint64, 2^-27 MeV units, shape (K, nz, ny,
        nx)) of a plain run, and its statistics; K is the tables' n_batches."""
        st = gmc_run_stats()
        keep = []
        src = _src(source, keep)
        tun = _tuning(tuning)
        shape = self.phantom_shape(phantom_id)
        n = int(np.prod(shape))
        K = self._batches(tables_id)
        if out == "torch":
            import torch
            t = torch.empty(K * n, dtype=torch.int64, device="cuda")
            ptr, kind = t.data_ptr(), GMC_DEVICE
        else:
            t = np.empty(K * n, np.uint64)
            ptr, kind = t.ctypes.data, GMC_HOST
        self._check(self._L.gmc_run_beam_tally(self._h, phantom_id, tables_id, C.byref(src), int(n_hist), int(seed),
                                               ptr, kind, C.byref(tun) if tun is not None else None, C.byref(st)))
        return t.reshape((K,) + shape), stats_dict(st)

    def finalize_tally(self, phantom_id: int, tables_id: int, tally, h_begin: int, h_end: int, sigma: bool = True):
        """Dose and sigma (host arrays) and s of Eq. 12 of batch tallies covering
        histories [h_begin, h_end): a numpy uint64 array or a torch int64
        tensor on the GPU, shape (K, nz, ny, nx)."""
        shape = self.phantom_shape(phantom_id)
        n = int(np.prod(shape))
        if hasattr(tally, "data_ptr"):
            if tally.numel() != self._batches(tables_id) * n or not tally.is_contiguous():
                raise ValueError("tally must be a contiguous (K, nz, ny, nx) tensor")
            tp, tk = tally.data_ptr(), GMC_DEVICE
        else:
            tally = np.ascontiguousarray(tally, dtype=np.uint64)
            if tally.size != self._batches(tables_id) * n:
                raise ValueError("tally must hold (K, nz, ny, nx) values")
            tp, tk = tally.ctypes.data, GMC_HOST
        d = np.empty(n, np.float64)
        s = np.empty(n, np.float64) if sigma else None
        srel = C.c_double()
        self._check(self._L.gmc_finalize_tally(self._h, phantom_id, tables_id, tp, tk, int(h_begin), int(h_end),
                                               d.ctypes.data, s.ctypes.data if s is not None else None, GMC_HOST,
                                               C.byref(srel)))
        return d.reshape(shape), (s.reshape(shape) if s is not None else None), srel.value

    def finalize_tally_noalloc(self, phantom_id: int, tables_id: int, tally, h_begin: int, h_end: int, dose,
                               sigma=None, want_s: bool = True):
        """gmc_finalize_tally_noalloc: tally, dose and sigma are contiguous torch
        tensors on the GPU ((K, nz, ny, nx) int64, (nz, ny, nx) float64);
        writes dose and sigma in place and returns s of Eq. 12 (NaN without
        sigma or when not wanted)."""
        shape = self.phantom_shape(phantom_id)
        n = int(np.prod(shape))
        if tally.numel() != self._batches(tables_id) * n or not tally.is_contiguous():
            raise ValueError("tally must be a contiguous (K, nz, ny, nx) tensor")
        for t in (dose, sigma):
            if t is not None and (t.numel() != n or not t.is_contiguous()):
                raise ValueError("dose and sigma must be contiguous tensors of nx*ny*nz values")
        srel = C.c_double(float("nan"))
        self._check(self._L.gmc_finalize_tally_noalloc(self._h, phantom_id, tables_id, tally.data_ptr(),
                                                       int(h_begin), int(h_end), dose.data_ptr(),
                                                       sigma.data_ptr() if sigma is not None else None,
                                                       C.byref(srel) if want_s else None))
        return srel.value

    def _batches(self, tables_id: int) -> int:
        return self._nbatch[tables_id]

    def autotune(self, phantom_id: int, tables_id: int, sources, n_hist, budget_s: float = 0.0):
        """The autotuner's choice for this job (cached per job class): (tuning dict, report dict)."""
        nb = len(sources)
        keep = []
        srcs = (gmc_source * nb)(*[_src(s, keep) for s in sources])
        counts = (C.c_uint64 * nb)(*[int(n) for n in n_hist])
        tun = gmc_tuning()
        rep = gmc_autotune_report()
        self._check(self._L.gmc_autotune(self._h, phantom_id, tables_id, srcs, counts, nb, budget_s, C.byref(tun),
                                         C.byref(rep)))
        return ({f: getattr(tun, f) for f, _ in gmc_tuning._fields_},
                {f: getattr(rep, f) for f, _ in gmc_autotune_report._fields_})

    # --------------------------------------------------------- served form
    def server_start(self, hbm_budget_bytes: int = 0, max_slots: int = 0):
        cfg = gmc_server_config(int(hbm_budget_bytes), int(max_slots))
        self._check(self._L.gmc_server_start(self._h, C.byref(cfg)))

    def server_stop(self):
        self._check(self._L.gmc_server_stop(self._h))

    def server_status(self) -> dict:
        st = gmc_server_status_t()
        self._check(self._L.gmc_server_status(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in gmc_server_status_t._fields_}

    def submit(self, phantom_id: int, tables_id: int, source, n_hist: int, seed: int) -> int:
        keep = []
        src = _src(source, keep)
        t = C.c_uint64()
        self._check(self._L.gmc_submit(self._h, phantom_id, tables_id, C.byref(src), int(n_hist), int(seed),
                                       C.byref(t)))
        self._tickets[t.value] = phantom_id
        return t.value

    def poll(self, ticket: int, shape=None, wait: bool = True, sigma: bool = True, out: str = "numpy"):
        """(done, dose, sigma, stats); dose/sigma None while not done.  A
        finished ticket is retired by the call that returns it.  shape
        defaults to the request's phantom's and must hold as many voxels."""
        if ticket in self._tickets:
            shape = self._out_shape(self._tickets[ticket], shape)
        elif shape is None:
            raise ValueError("unknown ticket %d: give the output shape" % ticket)
        n = int(np.prod(shape))
        if out == "torch":
            import torch
            d = torch.empty(n, dtype=torch.float64, device="cuda")
            s = torch.empty(n, dtype=torch.float64, device="cuda") if sigma else None
            dp, sp, kind = d.data_ptr(), (s.data_ptr() if s is not None else None), GMC_DEVICE
        else:
            d = np.empty(n, np.float64)
            s = np.empty(n, np.float64) if sigma else None
            dp, sp, kind = d.ctypes.data, (s.ctypes.data if s is not None else None), GMC_HOST
        done = C.c_int()
        st = gmc_request_stats()
        self._check(self._L.gmc_poll(self._h, int(ticket), 1 if wait else 0, C.byref(done), dp, sp, kind,
                                     C.byref(st)))
        if not done.value:
            return False, None, None, None
        self._tickets.pop(ticket, None)
        stats = {"t_queue_s": st.t_queue_s, "t_run_s": st.t_run_s, "t_latency_s": st.t_latency_s}
        stats.update(stats_dict(st.run))
        return True, d.reshape(*shape), (s.reshape(*shape) if s is not None else None), stats

    # ------------------------------------------------------------- checks
    def rng_words(self, seed: int, beam: int, hist: int, path: int, n0: int, count: int) -> np.ndarray:
        out = np.zeros(count, np.uint32)
        self._check(self._L.gmc_rng_words(self._h, seed, beam, hist, path, n0, count,
                                          out.ctypes.data_as(C.POINTER(C.c_uint32))))
        return out

    def table_eval(self, tables_id: int, which: int, mat: int, energies) -> np.ndarray:
        e = np.ascontiguousarray(energies, dtype=np.float64)
        out = np.zeros_like(e)
        self._check(self._L.gmc_table_eval(self._h, tables_id, which, mat, e.ctypes.data_as(C.POINTER(C.c_double)),
                                           e.size, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def atomic_rate(self, log2_words: int, hot: int = 0) -> float:
        """Measured 64-bit atomic additions per second into 2^log2_words words
        (hashed addresses, or hot > 0: t mod hot)."""
        r = C.c_double()
        self._check(self._L.gmc_atomic_rate(self._h, int(log2_words), int(hot), C.byref(r)))
        return r.value

    def first_events(self, phantom_id: int, tables_id: int, source, seed: int, h_begin: int, h_end: int):
        n = h_end - h_begin
        xyz = np.zeros(3 * n, np.float32)
        nu = np.zeros(n, np.uint32)
        keep = []
        src = _src(source, keep)
        self._check(self._L.gmc_first_events(self._h, phantom_id, tables_id, C.byref(src), seed, h_begin, h_end,
                                             xyz.ctypes.data_as(C.POINTER(C.c_float)),
                                             nu.ctypes.data_as(C.POINTER(C.c_uint32))))
        return xyz.reshape(n, 3), nu


def run_workload(ctx: Context, w, n_hist: Optional[int] = None, seed: Optional[int] = None, tuning=None,
                 out: str = "numpy"):
    """Load a Workload's tables and phantom, run its beam, release the handles."""
    tid = ctx.load_tables(w.materials, w.physics)
    pid = ctx.load_phantom(w.phantom)
    try:
        return ctx.run_beam(pid, tid, w.source, n_hist or w.n_hist, w.seed if seed is None else seed,
                            shape=w.phantom.rho.shape, tuning=tuning, out=out)
    finally:
        ctx.release(pid)
        ctx.release(tid)
