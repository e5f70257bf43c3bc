#!/usr/bin/env python3
"""Throughput benchmark: histories/s at 1% statistical uncertainty, plain vs batched.

Default workload (the paper's Table IV set-up): 15 MeV monoenergetic parallel
beams, 10 x 10 cm field, on a 64^3 water phantom of 0.5 cm voxels, ECUT 0.7
MeV (kinetic), PCUT 0.01 MeV: one electron beam and one photon beam.  A pilot
run at the paper's counts (1e6 electrons, 4e6 photons) measures the
uncertainty s of Eq. 12 for each beam; each beam is then run with the
histories N_1% that bring s to 1%.  One step = both beams at N_1%:

* plain leg: two gmc_run_beam calls (one beam per sequence of passes);
* batched leg: one gmc_run_beams call holding both beams (graph-replayed
  rounds), with each beam's own dose as well as the combined one.

`value` is the batched leg's rate; the plain leg's is reported beside it.
Inputs are resident in HBM and outputs stay in device memory.

Served leg (``served``): a seeded Poisson stream of 200 dose requests
(ellipsoid phantoms of 32^3-256^3 voxels from a resident pool, mixed beams,
1e5-1e8 histories) at 0.7 x the capacity measured by a closed-loop pilot,
through the continuous-batching server; p50/p99 latency from submission to
result and the aggregate histories/s.

``--workload beamlets``: 256 pencil beamlets (0.5 x 0.5 cm, 1-20 MeV,
photons:electrons 3:1, 1e4-1e6 histories each) on a 200x200x160 ellipsoid
phantom at 0.25 cm; plain = 256 gmc_run_beam calls, batched = one
gmc_run_beams call with per-beamlet doses.

``--workload geometries``: the paper's timing tables on this GPU -- one 15 MeV
beam (1e6 electrons or 4e6 photons, 10 x 10 cm) on each of the three 64^3
geometries (water, lung box, tissue-lung-bone slabs; Table IV), and on the lung
box the base, compaction (N = 4, 16, 64), pool, combined and default
settings (Table VI; A_comp is the best N).

``--workload atomics``: the library's 64-bit atomic-add microbenchmark (the
tally path's second roof), random addresses into 0.26 MB-1 GiB arrays and hot
sets of 1-4096 words.

``--workload regroup``: energy regrouping before every pass against none, in
the batched form (monoenergetic water beams, triangular-spectrum beams,
beamlets).

Prints one JSON line with the throughput, the roofline of the dominant kernel
(average launch duration from the HIP event pairs around every pass launch in
the timed plain and batched legs) and, for the default workload, the oracle's
CPU rate on a bounded sample.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work per unit (lane operations): one condensed electron step and
# one photon flight + interaction decision (derivation in the design notes).
OPS_PER_E_STEP = 400.0
OPS_PER_PH_EVENT = 175.0
# ... and, on top of its flight, one real photon interaction (a Compton event:
# 400-600 operations more; photoelectric and pair events taken alike)
OPS_PER_PH_INTERACTION = 500.0
# 32-bit VALU lane operations: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (no packed FP32).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
# HBM bytes per unit of algorithmic work (electron step / photon event) of the
# pass kernels, from two rocprofv3 counter runs (FETCH_SIZE, then WRITE_SIZE)
# over the timed legs of the water workload, each scaled by the same counter
# on a 1 GiB device copy (fetched bytes x2.0, written x1.0), and the tally
# additions per electron step (TCP_TCC_ATOMIC_WITHOUT_RET_REQ over the same
# legs).  Valid only for the kernel and engine sources they were measured on
# (their digest); per launch they are multiplied by this run's work per
# launch.
TRAFFIC = {"sources_sha256": "9e39638eb02b1fb17234828d06de818ee4dd27b87fb381394cb8ad690d9150e4",
           "k_electron_pass": 57.98, "k_electron_pass_atomics": 0.614}
# Words of the array the atomic roof is measured on: 2^23 uint64 (67 MB), the
# size of the water job's 32-batch tally.
ATOMIC_ROOF_LOG2_WORDS = 23
MEASURED_SOURCES = ("paper_1101_1245_amd/csrc/gmc_kernels.hip",
                    "paper_1101_1245_amd/csrc/gmc_device.hpp",
                    "paper_1101_1245_amd/csrc/gmc_internal.hpp",
                    "paper_1101_1245_amd/csrc/gmc_engine.cpp",
                    "paper_1101_1245_amd/csrc/gmc_host.hpp")


def measured_traffic(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in MEASURED_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC.get(kernel) if h.hexdigest() == TRAFFIC["sources_sha256"] else None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or platform.machine()


def cpu_baseline(n1=None):
    """The FP64 oracle, single-threaded, on a bounded sample of the same beams;
    with n1 (histories per beam at 1%), the time the oracle would take to reach
    1% on both beams at the sampled per-beam rates."""
    from oracle import oracle as O
    from paper_1101_1245_amd import inputs as I
    we = I.water_15mev(I.ELECTRON)
    wg = I.water_15mev(I.PHOTON)
    ne, ng = 70000, 280000
    t0 = time.perf_counter()
    O.run(we.materials, we.phantom, we.source, we.physics, we.seed, ne, batches=False)
    t1 = time.perf_counter()
    O.run(wg.materials, wg.phantom, wg.source, wg.physics, wg.seed, ng, batches=False)
    t2 = time.perf_counter()
    out = {"value": (ne + ng) / (t2 - t0), "unit": "histories/s", "cores": 1, "kind": "oracle",
           "sample": "%d electrons (%.1f s) + %d photons (%.1f s), 15 MeV, 64^3 water, one host core of %d (%s)" %
                     (ne, t1 - t0, ng, t2 - t1, os.cpu_count() or 0, cpu_model())}
    if n1:
        out["time_to_1pct_s"] = n1["electron"] * (t1 - t0) / ne + n1["photon"] * (t2 - t1) / ng
    return out


class Acc:
    """Sums of pass-kernel times and work units over runs."""

    def __init__(self):
        self.t = [0.0, 0.0, 0.0]  # photon pass, electron pass, persistent round kernel seconds
        self.n = [0, 0, 0]        # launches
        self.steps = 0
        self.events = 0
        self.interactions = 0
        self.resid = 0
        self.hist = 0
        self.atomic_roof = None   # additions/s of the atomic microbenchmark, when measured

    def add(self, st):
        self.t[0] += st["t_photon_pass_s"]
        self.t[1] += st["t_electron_pass_s"]
        self.n[0] += st["n_photon_launches"]
        self.n[1] += st["n_electron_launches"]
        self.t[2] += st["t_round_s"]
        self.n[2] += st["n_round_launches"]
        self.steps += st["n_e_steps"]
        self.events += st["n_photon_events"]
        self.interactions += st["n_photon_interactions"]
        self.resid |= st["ledger_residual_lsb"]
        self.hist += st["n_hist"]

    def merge(self, o):
        for i in range(3):
            self.t[i] += o.t[i]
            self.n[i] += o.n[i]
        self.steps += o.steps
        self.events += o.events
        self.interactions += o.interactions
        self.resid |= o.resid
        self.hist += o.hist


def roofline(acc, workload="water"):
    """Dominant pass kernel (most device time), its average launch duration and
    algorithmic lane-ops per launch against the VALU lane-op peak; for the
    water workload also its measured HBM bytes and its tally additions
    against the atomic rate measured in the same run."""
    ph_ops = acc.events * OPS_PER_PH_EVENT + acc.interactions * OPS_PER_PH_INTERACTION
    if acc.t[2] > max(acc.t[0], acc.t[1]):
        # persistent round kernels: both particle types in each launch
        name, t, n = "k_round", acc.t[2], acc.n[2]
        ops = acc.steps * OPS_PER_E_STEP + ph_ops
    elif acc.t[1] >= acc.t[0]:
        name, t, n, ops = "k_electron_pass", acc.t[1], acc.n[1], acc.steps * OPS_PER_E_STEP
    else:
        name, t, n, ops = "k_photon_pass", acc.t[0], acc.n[0], ph_ops
    n = max(n, 1)
    avg = t / n
    achieved = ops / n / avg / 1e12 if avg > 0 else 0.0
    peak = PEAK_LANE_OPS / 1e12
    per_unit = measured_traffic(name) if workload == "water" else None
    units = (acc.steps if name != "k_photon_pass" else acc.events) / n
    traffic = per_unit * units if per_unit else None
    out = {"bound": "alu", "kernel": name, "achieved": achieved, "peak": peak, "unit": "TOP/s",
           "frac": achieved / peak, "traffic": traffic, "avg_launch_ms": avg * 1e3, "launches": n,
           "share_of_pass_time": t / max(acc.t[0] + acc.t[1] + acc.t[2], 1e-30)}
    if traffic:
        out["traffic_unit"] = "HBM bytes per launch (%.2f per unit of work x %.3g units)" % (per_unit, units)
        out["hbm_GBps"] = traffic / avg / 1e9
        out["hbm_frac"] = traffic / avg / 8.0e12
    # the tally's second roof: additions per second against what random 64-bit
    # atomics reach on an array the size of the tally, measured in the same run
    adds = measured_traffic(name + "_atomics") if workload == "water" else None
    if adds and acc.atomic_roof and avg > 0:
        a = adds * units / avg
        out["atomics"] = {"achieved": a, "peak": acc.atomic_roof, "unit": "additions/s", "frac": a / acc.atomic_roof,
                          "per_unit": adds,
                          "peak_from": "k_atomic_rate: 2^%d uint64 words at hashed addresses, best of 3 launches"
                                       % ATOMIC_ROOF_LOG2_WORDS}
    # the other pass kernel against the same peak (in a job run by round
    # kernels the pass counts cover only the legs that ran passes)
    if name != "k_round":
        for other, i, ops_i in (("k_photon_pass", 0, ph_ops), ("k_electron_pass", 1, acc.steps * OPS_PER_E_STEP)):
            if other != name and acc.n[i] > 0 and acc.t[i] > 0:
                a = ops_i / acc.t[i] / 1e12
                out[other] = {"achieved": a, "frac": a / peak, "avg_launch_ms": acc.t[i] / acc.n[i] * 1e3,
                              "launches": acc.n[i]}
                if other == "k_photon_pass":
                    out[other]["ops"] = "%g per flight + %g per real interaction" % (OPS_PER_PH_EVENT,
                                                                                     OPS_PER_PH_INTERACTION)
    return out


def sync():
    import torch
    torch.cuda.synchronize()


def bench_water(args, G, E, I):
    we = I.water_15mev(I.ELECTRON)
    wg = I.water_15mev(I.PHOTON)
    ctx = G.Context(0)
    tid = ctx.load_tables(we.materials, we.physics)
    pid = ctx.load_phantom(we.phantom)
    shape = we.phantom.shape

    # pilot at the paper's counts -> histories for the target s (Eq. 12)
    n1, s_pilot = {}, {}
    for key, w in (("electron", we), ("photon", wg)):
        d, s, st = ctx.run_beam(pid, tid, w.source, w.n_hist, 1, shape=shape, out="torch")
        sv = E.uncertainty_s(d.cpu().numpy(), s.cpu().numpy())
        s_pilot[key] = sv
        n1[key] = min(E.histories_for(sv, w.n_hist, args.target), (1 << 31) - 1)
        print("pilot %s: N=%d s=%.4f -> N=%d for s=%.3f (device %.1f ms)" %
              (key, w.n_hist, sv, n1[key], args.target, st["t_device_s"] * 1e3), file=sys.stderr, flush=True)
    srcs = [we.source, wg.source]
    counts = [n1["electron"], n1["photon"]]

    def plain(seed):
        out = []
        for w, key in ((we, "electron"), (wg, "photon")):
            out.append(ctx.run_beam(pid, tid, w.source, n1[key], seed, shape=shape, out="torch"))
        return out

    def batched(seed):
        return ctx.run_beams(pid, tid, srcs, counts, seed, shape=shape, per_beam=True, per_beam_sigma=True,
                             tuning=args.tuning, out="torch")

    # the alternate electron cutoff first, so that the timed legs and the
    # host-output leg stay the water workload's last launches
    alt = None if args.no_alt_ecut else alt_ecut(args, ctx, pid, shape, G, E, I)

    for i in range(args.warmup):
        plain(100 + i)
        batched(100 + i)

    legs = {}
    last = {}
    t_beam = {"electron": 0.0, "photon": 0.0}   # device time per beam, plain leg
    for leg, fn in (("plain", plain), ("batched", batched)):
        acc = Acc()
        sync()
        t0 = time.perf_counter()
        for k in range(args.steps):
            r = fn(1000 + k)
            if leg == "plain":
                for (_, _, st), key in zip(r, ("electron", "photon")):
                    acc.add(st)
                    t_beam[key] += st["t_device_s"] / args.steps
            else:
                acc.add(r[4])
            last[leg] = r
        sync()
        el = time.perf_counter() - t0
        legs[leg] = (acc, el)
        print("%s: %.1f ms/step, %.3e histories/s" % (leg, el / args.steps * 1e3, acc.hist / el),
              file=sys.stderr, flush=True)

    # the batched leg's per-beam uncertainty is that of the plain leg's runs with the same seed
    s_final = {}
    for (d, s, _), key in zip(last["plain"], ("electron", "photon")):
        s_final[key] = E.uncertainty_s(d.cpu().numpy(), s.cpu().numpy())
    pb, ps = last["batched"][0], last["batched"][1]
    same = all(bool((pb[i] == last["plain"][i][0]).all()) and bool((ps[i] == last["plain"][i][1]).all())
               for i in range(2))

    # the paper's timings include the transfer of the results: the plain leg
    # once more with dose and sigma copied to host memory
    sync()
    t0 = time.perf_counter()
    for k in range(args.steps):
        for w, key in ((we, "electron"), (wg, "photon")):
            ctx.run_beam(pid, tid, w.source, n1[key], 1000 + k, shape=shape, out="numpy")
    el_h = time.perf_counter() - t0

    acc_b, el_b = legs["batched"]
    acc_p, el_p = legs["plain"]
    both = Acc()
    both.merge(acc_p)
    both.merge(acc_b)
    out = {
        "metric": "histories/s at 1% stat. unc. (plain vs batched); served dose p50/p99 latency",
        "value": acc_b.hist / el_b,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el_b / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "15 MeV electron + photon parallel beams, 10x10 cm, 64^3 water at 0.5 cm, "
                        "ECUT 0.7 / PCUT 0.01 MeV, each beam at N_1%; value = batched form (both beams "
                        "in one gmc_run_beams job)",
            "n_electrons": n1["electron"], "n_photons": n1["photon"],
            "s_pilot": s_pilot, "s_timed": s_final,
            "tallies": "int64 fixed point, 32 batches",
            "batched_tuning": args.tuning if args.tuning is not None else "autotuned",
            "outputs": "device memory (no PCIe in the timed region)",
        },
        "plain": {"value": acc_p.hist / el_p, "ms_per_step": el_p / args.steps * 1e3},
        "batched_over_plain": (acc_b.hist / el_b) / (acc_p.hist / el_p),
        "batched_equals_plain_per_beam": same,
        "plain_host_outputs": {"value": acc_p.hist / el_h, "ms_per_step": el_h / args.steps * 1e3,
                               "note": "plain leg with dose and sigma copied to host memory in the timed region"},
        "efficiency_per_s": {key: 1.0 / (s_final[key] ** 2 * t_beam[key]) for key in ("electron", "photon")},
        "efficiency_note": "epsilon = 1 / (s^2 T) (Eq. 11) per beam, T its plain-form device time",
    }
    if alt is not None:
        out["alt_ecut_0p189"] = alt
    # the atomic roof on an array the size of this job's tally (after the
    # timed legs, outside them)
    both.atomic_roof = max(ctx.atomic_rate(ATOMIC_ROOF_LOG2_WORDS) for _ in range(3))
    ctx.close()
    return out, both


def alt_ecut(args, ctx, pid, shape, G, E, I):
    """The same two beams with the electron cutoff read as EGSnrc's total-energy
    ECUT 0.7 MeV, i.e. 0.189 MeV kinetic (K_cut with it): pilot at the paper's
    counts, histories for s = 1%, then timed batched steps."""
    we = I.water_15mev(I.ELECTRON)
    wg = I.water_15mev(I.PHOTON)
    phys = I.Physics(ecut=0.189, pcut=0.01)
    tid = ctx.load_tables(we.materials, phys)
    n1 = {}
    for key, w in (("electron", we), ("photon", wg)):
        d, s, _ = ctx.run_beam(pid, tid, w.source, w.n_hist, 1, shape=shape, out="torch")
        n1[key] = min(E.histories_for(E.uncertainty_s(d.cpu().numpy(), s.cpu().numpy()), w.n_hist, args.target),
                      (1 << 31) - 1)
    srcs, counts = [we.source, wg.source], [n1["electron"], n1["photon"]]
    ctx.run_beams(pid, tid, srcs, counts, 100, shape=shape, per_beam=True, per_beam_sigma=True, tuning=args.tuning,
                  out="torch")
    steps = max(1, min(args.steps, 3))
    acc = Acc()
    sync()
    t0 = time.perf_counter()
    for k in range(steps):
        acc.add(ctx.run_beams(pid, tid, srcs, counts, 1000 + k, shape=shape, per_beam=True, per_beam_sigma=True,
                              tuning=args.tuning, out="torch")[4])
    sync()
    el = time.perf_counter() - t0
    ctx.release(tid)
    print("alternate ECUT 0.189 MeV: %.1f ms/step, %.3e histories/s" % (el / steps * 1e3, acc.hist / el),
          file=sys.stderr, flush=True)
    return {"value": acc.hist / el, "unit": "histories/s", "ms_per_step": el / steps * 1e3, "steps": steps,
            "n_electrons": n1["electron"], "n_photons": n1["photon"],
            "electron_steps_per_history": acc.steps / max(acc.hist, 1),
            "note": "batched leg of the water workload with ECUT 0.189 MeV kinetic (EGSnrc's ECUT 0.7 read as a "
                    "total energy), each beam at its own N_1%"}


def bench_beamlets(args, G, E, I):
    import torch
    j = I.beamlet_job()
    ctx = G.Context(0)
    tid = ctx.load_tables(j.materials, j.physics)
    pid = ctx.load_phantom(j.phantom)
    shape = j.phantom.shape
    total = int(j.counts.sum())

    def plain(seed):
        acc = Acc()
        for src, n in zip(j.sources, j.counts):
            d, _, st = ctx.run_beam(pid, tid, src, int(n), seed, shape=shape, sigma=False, out="torch")
            acc.add(st)
            del d
        return acc

    def batched(seed):
        acc = Acc()
        pb, _, d, s, st = ctx.run_beams(pid, tid, j.sources, j.counts, seed, shape=shape, per_beam=True,
                                        tuning=args.tuning, out="torch")
        acc.add(st)
        del pb, d, s
        return acc

    for i in range(args.warmup):
        batched(100 + i)
        torch.cuda.empty_cache()
    legs = {}
    for leg, fn in (("plain", plain), ("batched", batched)):
        acc = Acc()
        sync()
        t0 = time.perf_counter()
        for k in range(args.steps):
            acc.merge(fn(1000 + k))
        sync()
        el = time.perf_counter() - t0
        legs[leg] = (acc, el)
        torch.cuda.empty_cache()
        print("%s: %.1f ms/step, %.3e histories/s" % (leg, el / args.steps * 1e3, acc.hist / el),
              file=sys.stderr, flush=True)
    acc_b, el_b = legs["batched"]
    acc_p, el_p = legs["plain"]
    both = Acc()
    both.merge(acc_p)
    both.merge(acc_b)
    out = {
        "metric": "histories/s (plain vs batched), beamlet batch",
        "value": acc_b.hist / el_b,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el_b / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "256 pencil beamlets 0.5x0.5 cm, 1-20 MeV, photons:electrons 3:1, 1e4-1e6 histories "
                        "each (%d in total), 200x200x160 ellipsoid phantom at 0.25 cm, ECUT 0.7 / PCUT 0.01 MeV; "
                        "value = one gmc_run_beams job with per-beamlet doses" % total,
            "beamlets": len(j.sources), "histories": total,
            "batched_tuning": args.tuning if args.tuning is not None else "autotuned",
            "outputs": "device memory (no PCIe in the timed region)",
        },
        "plain": {"value": acc_p.hist / el_p, "ms_per_step": el_p / args.steps * 1e3,
                  "roofline": roofline(acc_p, "beamlets")},
        "batched_over_plain": (acc_b.hist / el_b) / (acc_p.hist / el_p),
        # the launches that produce `value`: the batched leg's (the plain leg's
        # 256 short jobs have a roofline of their own under "plain")
        "roofline": roofline(acc_b, "beamlets"),
        "ledger_residual_lsb": both.resid,
    }
    ctx.close()
    return out


def bench_geometries(args, G, E, I):
    """The paper's timing tables on this GPU: the time of one 15 MeV beam (1e6
    electrons or 4e6 photons) on each of the three geometries (Table IV), and on
    the lung box the divergence-reduction settings against the base one
    (Table VI: A = T_base / T)."""
    geoms = (("water", I.water_15mev), ("lung_box", I.lung_box), ("tissue_lung_bone", I.tissue_lung_bone))
    reps = max(4 * args.steps, 10)
    ctx = G.Context(0)
    acc_all = Acc()

    def timed(w, tuning):
        tid = ctx.load_tables(w.materials, w.physics)
        pid = ctx.load_phantom(w.phantom)
        shape = w.phantom.shape
        for i in range(args.warmup):
            ctx.run_beam(pid, tid, w.source, w.n_hist, 100 + i, shape=shape, sigma=False, tuning=tuning,
                         out="torch")
        acc = Acc()
        sync()
        t0 = time.perf_counter()
        for k in range(reps):
            d, _, st = ctx.run_beam(pid, tid, w.source, w.n_hist, 1000 + k, shape=shape, sigma=False,
                                    tuning=tuning, out="torch")
            acc.add(st)
        sync()
        el = (time.perf_counter() - t0) / reps
        acc_all.merge(acc)
        ctx.release(pid)
        ctx.release(tid)
        return el, d, acc

    table_iv = {}
    hist = 0
    secs = 0.0
    for gname, make in geoms:
        row = {}
        for pname, p in (("electron", I.ELECTRON), ("photon", I.PHOTON)):
            w = make(p)
            el, _, acc = timed(w, None)
            row[pname + "_s"] = el
            hist += w.n_hist
            secs += el
            print("Table IV %-17s %-8s %8.2f ms  (%.3e histories/s)" % (gname, pname, el * 1e3, w.n_hist / el),
                  file=sys.stderr, flush=True)
        table_iv[gname] = row

    # the other fixed-count set-ups: 1 MeV photons on 32^3 water (1e5) and
    # 6 MeV photons on the 128^3 slab phantom (4e7)
    fixed = {}
    for w in (I.small_photon_water(), I.slab_6mev()):
        el, _, _ = timed(w, None)
        fixed[w.name] = {"histories": w.n_hist, "s": el, "histories_per_s": w.n_hist / el}
        print("fixed count %-24s %9.2f ms  (%.3e histories/s)" % (w.name, el * 1e3, w.n_hist / el),
              file=sys.stderr, flush=True)

    table_vi = {}
    identical = True
    settings = list(I.ABLATION_TUNINGS.items()) + [("default", None)]
    for pname, p in (("electron", I.ELECTRON), ("photon", I.PHOTON)):
        w = I.lung_box(p)
        t = {}
        ref = None
        for tname, tuning in settings:
            el, d, acc = timed(w, tuning)
            t[tname] = el
            if ref is None:
                ref = d
            else:
                identical &= bool(torch_equal(ref, d))
            print("Table VI %-8s %-15s %8.2f ms  launches %d/%d" % (pname, tname, el * 1e3, acc.n[0], acc.n[1]),
                  file=sys.stderr, flush=True)
        comp = min((k for k in t if k.startswith("compaction")), key=lambda k: t[k])
        table_vi[pname] = {
            "T_base_s": t["base"],
            "A_comp": t["base"] / t[comp], "A_comp_setting": comp,
            "A_pool": t["base"] / t["pool"],
            "A_both": t["base"] / t["both"],
            "A_default": t["base"] / t["default"],
            "T_s": t,
        }

    out = {
        "metric": "histories/s over the three geometries' beams; Table IV times and Table VI factors",
        "value": hist / secs,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "ms_per_step": secs * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "15 MeV parallel beams, 10x10 cm, 64^3 at 0.5 cm: water, water with a lung box, "
                        "tissue-lung-bone slabs; 1e6 electrons or 4e6 photons per run; ECUT 0.7 / PCUT 0.01 "
                        "MeV; one step = the six runs (plain form, engine defaults); outputs in device memory",
            "ablation": "lung box, tunings " + json.dumps(I.ABLATION_TUNINGS),
        },
        "table_iv_s": table_iv,
        "fixed_count": fixed,
        "table_vi": table_vi,
        "ablation_doses_bit_identical": identical,
        "roofline": roofline(acc_all, "geometries"),
        "ledger_residual_lsb": acc_all.resid,
    }
    ctx.close()
    return out


def bench_regroup(args, G, E, I):
    """Energy regrouping before every pass (the grouping of similar energies
    that Sec. IV.B proposes for polyenergetic beams) against none, in the
    batched form with one fixed tuning otherwise: the water beams at the
    histories of 1% uncertainty (monoenergetic), the same phantom with
    triangular 2-10-18 MeV spectra, and the 256 beamlets (1-20 MeV)."""
    import torch
    we, wg = I.water_15mev(I.ELECTRON), I.water_15mev(I.PHOTON)
    tri = [I.centred(we.phantom, I.Source(p, I.TRIANGULAR, 10.0, e_lo=2.0, e_mode=10.0, e_hi=18.0,
                                          wx=10.0, wy=10.0, beam_id=b)) for b, p in enumerate((I.ELECTRON, I.PHOTON))]
    j = I.beamlet_job()
    cases = (("water 15 MeV e + photons", we, [we.source, wg.source], [5_248_287, 64_951_300], False),
             ("water 2-10-18 MeV e + photons", we, tri, [5_000_000, 50_000_000], False),
             ("256 beamlets 1-20 MeV", j, j.sources, list(j.counts), True))
    reps = max(args.steps, 2)
    ctx = G.Context(0)
    rows = {}
    acc_all = Acc()
    identical = True
    for name, w, srcs, counts, per_beam in cases:
        tid = ctx.load_tables(w.materials, w.physics)
        pid = ctx.load_phantom(w.phantom)
        shape = w.phantom.shape
        row = {}
        ref = None
        for sort in (0, 1):
            tuning = {"chunk": 1 << 22, "pass_items": 1 << 23, "energy_sort": sort}
            for i in range(args.warmup):
                ctx.run_beams(pid, tid, srcs, counts, 100 + i, shape=shape, per_beam=per_beam, tuning=tuning,
                              out="torch")
            acc = Acc()
            sync()
            t0 = time.perf_counter()
            for k in range(reps):
                r = ctx.run_beams(pid, tid, srcs, counts, 1000 + k, shape=shape, per_beam=per_beam, tuning=tuning,
                                  out="torch")
                acc.add(r[4])
            sync()
            el = (time.perf_counter() - t0) / reps
            acc_all.merge(acc)
            if ref is None:
                ref = r[2]
            else:
                identical &= bool(torch_equal(ref, r[2]))
            key = "sorted" if sort else "unsorted"
            row[key] = {"ms_per_step": el * 1e3, "electron_pass_ms": acc.t[1] / reps * 1e3,
                        "photon_pass_ms": acc.t[0] / reps * 1e3}
            print("%-30s %-8s %7.1f ms/step  e-pass %6.1f ms  photon pass %6.1f ms" %
                  (name, key, el * 1e3, acc.t[1] / reps * 1e3, acc.t[0] / reps * 1e3), file=sys.stderr, flush=True)
            del r
            torch.cuda.empty_cache()
        row["speedup"] = row["unsorted"]["ms_per_step"] / row["sorted"]["ms_per_step"]
        rows[name] = row
        ctx.release(pid)
        ctx.release(tid)
    total = sum(int(sum(c[3])) for c in cases)
    t_sorted = sum(r["sorted"]["ms_per_step"] for r in rows.values())
    out = {
        "metric": "histories/s with energy regrouping before every pass (vs without)",
        "value": total / (t_sorted * 1e-3),
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": reps,
        "warmup": args.warmup,
        "ms_per_step": t_sorted,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "batched form, chunk 2^22, pass 2^23: 15 MeV e (5.2e6) + photons (6.5e7) on 64^3 water; "
                        "triangular 2-10-18 MeV e (5e6) + photons (5e7) on 64^3 water; 256 beamlets 1-20 MeV on a "
                        "200x200x160 ellipsoid phantom; one step = the three jobs with regrouping",
        },
        "cases": rows,
        "doses_bit_identical": identical,
        "roofline": roofline(acc_all, "regroup"),
        "ledger_residual_lsb": acc_all.resid,
    }
    ctx.close()
    return out


def bench_atomics(args, G):
    """The tally path's second roof: 64-bit atomic additions per second into
    arrays from L2 size to HBM size at hashed addresses, and into hot sets of
    1, 64 and 4096 words (the library's own microbenchmark kernel)."""
    ctx = G.Context(0)
    sizes = {}
    for lg in (15, 18, 21, 23, 25, 27, 29, 31):
        rate = max(ctx.atomic_rate(lg) for _ in range(max(args.steps, 1)))
        sizes["%.3g MB" % ((1 << lg) * 8 / 1e6)] = rate
        print("random atomics into %8.3g MB: %.3e /s" % ((1 << lg) * 8 / 1e6, rate), file=sys.stderr, flush=True)
    hot = {}
    for h in (1, 64, 4096):
        hot[str(h)] = max(ctx.atomic_rate(15, h) for _ in range(max(args.steps, 1)))
        print("hot set of %4d words: %.3e /s" % (h, hot[str(h)]), file=sys.stderr, flush=True)
    ctx.close()
    big = sizes["%.3g MB" % ((1 << 27) * 8 / 1e6)]
    return {
        "metric": "64-bit atomic additions/s at hashed addresses of a 1 GiB array",
        "value": big,
        "unit": "additions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": (1 << 26) / big * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "2^20 lanes x 64 atomic adds of 1 into uint64 arrays of 2^15..2^31 words at hashed "
                               "addresses, and into hot sets of 1 / 64 / 4096 words; best of --steps launches"},
        "random_by_array_size": sizes,
        "hot_set": hot,
    }


def torch_equal(a, b):
    import torch
    return torch.equal(a, b)


def bench_serve(args, G, I):
    """Served form: a Poisson stream of dose requests at 0.7 x the capacity of
    a closed-loop pilot; latency from submission to result."""
    import threading
    import numpy as np
    pool, reqs = I.request_stream(seed=13, n_requests=args.serve_requests)
    ctx = G.Context(0)
    tid = ctx.load_tables(I.DEFAULT_MATERIALS, I.serving_physics())
    pids = [ctx.load_phantom(p) for p in pool]
    acc = Acc()

    def drain(tickets, sub, out_kind="torch"):
        out = []
        for t, r in zip(tickets, sub):
            _, _, _, st = ctx.poll(t, pool[r.phantom].shape, wait=True, sigma=True, out=out_kind)
            acc.add(st)
            out.append(st)
        return out

    ctx.server_start(max_slots=args.serve_slots)
    try:
        # closed-loop pilot: a batch of requests submitted at once
        pilot = reqs[:min(len(reqs), 40)]
        t0 = time.perf_counter()
        drain([ctx.submit(pids[r.phantom], tid, r.source, r.n_hist, 10_000 + r.seed) for r in pilot], pilot)
        capacity = len(pilot) / (time.perf_counter() - t0)
        rate = 0.7 * capacity
        arrivals = I.poisson_arrivals(rate, len(reqs), seed=17)
        acc = Acc()
        tickets = [None] * len(reqs)
        ready = [threading.Event() for _ in reqs]

        def submitter():
            start = time.perf_counter()
            for i, r in enumerate(reqs):
                delay = start + arrivals[i] - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                tickets[i] = ctx.submit(pids[r.phantom], tid, r.source, r.n_hist, r.seed)
                ready[i].set()

        th = threading.Thread(target=submitter)
        t0 = time.perf_counter()
        th.start()
        stats = []
        for i, r in enumerate(reqs):
            ready[i].wait()
            stats.extend(drain([tickets[i]], [r]))
        el = time.perf_counter() - t0
        th.join()
    finally:
        ctx.server_stop()
    acc_stream, acc = acc, Acc()      # the closed loop below is not part of the stream's kernel statistics
    lat = np.array([st["t_latency_s"] for st in stats])
    queue = np.array([st["t_queue_s"] for st in stats])
    hist = sum(r.n_hist for r in reqs)

    # the same requests as a closed loop (all submitted at once) and through
    # the plain form one after another: throughput of the two forms on
    # identical work, with the outputs in device memory and in host memory
    def closed_loop(out_kind):
        ctx.server_start(max_slots=args.serve_slots)
        try:
            sync()
            t0 = time.perf_counter()
            tickets = [ctx.submit(pids[r.phantom], tid, r.source, r.n_hist, 20_000 + r.seed) for r in reqs]
            drain(tickets, reqs, out_kind)
            sync()
            return time.perf_counter() - t0
        finally:
            ctx.server_stop()

    def plain_sequential(out_kind):
        sync()
        t0 = time.perf_counter()
        for r in reqs:
            ctx.run_beam(pids[r.phantom], tid, r.source, r.n_hist, 20_000 + r.seed, sigma=True, out=out_kind)
        sync()
        return time.perf_counter() - t0

    el_closed = closed_loop("torch")
    el_plain = plain_sequential("torch")
    el_closed_h = closed_loop("numpy")
    el_plain_h = plain_sequential("numpy")
    for p in pids:
        ctx.release(p)
    ctx.close()
    out = {
        "requests": len(reqs), "slots": args.serve_slots, "phantom_pool": len(pool),
        "capacity_req_per_s": capacity, "rate_req_per_s": rate,
        "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
        "mean_latency_s": float(lat.mean()), "p99_queue_s": float(np.percentile(queue, 99)),
        "histories_per_s": hist / el, "histories": hist, "elapsed_s": el,
        "closed_loop": {"histories_per_s": hist / el_closed, "elapsed_s": el_closed,
                        "note": "all requests submitted at once to the server, results polled into device memory"},
        "plain_sequential": {"histories_per_s": hist / el_plain, "elapsed_s": el_plain,
                             "note": "the same requests through gmc_run_beam one after another, outputs on the "
                                     "device"},
        "closed_loop_over_plain": el_plain / el_closed,
        "host_outputs": {"closed_loop_histories_per_s": hist / el_closed_h,
                         "plain_sequential_histories_per_s": hist / el_plain_h,
                         "closed_loop_over_plain": el_plain_h / el_closed_h,
                         "note": "both legs again with dose and sigma delivered to host memory (numpy)"},
        "workload": "Poisson stream of %d requests (seed 13) at 0.7 x closed-loop capacity: cubic ellipsoid "
                    "phantoms 32^3-256^3 at 0.25-0.5 cm (pool of %d), photons:electrons 3:1, 1-20 MeV mono or "
                    "2-10-18 MeV triangular, 1-10 cm fields, 1e5-1e8 histories" % (len(reqs), len(pool)),
    }
    print("served closed loop %.3e histories/s, plain one after another %.3e histories/s (x%.2f); host outputs "
          "%.3e vs %.3e (x%.2f)" % (hist / el_closed, hist / el_plain, el_plain / el_closed, hist / el_closed_h,
                                    hist / el_plain_h, el_plain_h / el_closed_h), file=sys.stderr, flush=True)
    print("served: p50 %.3f s p99 %.3f s, %.3e histories/s at %.2f req/s" %
          (out["p50_latency_s"], out["p99_latency_s"], out["histories_per_s"], rate), file=sys.stderr, flush=True)
    return out, acc_stream


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("water", "beamlets", "geometries", "regroup", "atomics"), default="water")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-form leg")
    ap.add_argument("--no-beamlets", action="store_true", help="skip the 256-beamlet leg of the default workload")
    ap.add_argument("--no-alt-ecut", action="store_true",
                    help="skip the water workload's alternate run at ECUT 0.189 MeV kinetic")
    ap.add_argument("--beamlet-steps", type=int, default=3,
                    help="timed steps of the 256-beamlet leg of the default workload (each ~0.8 s)")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--copy-reference", type=int, default=0, metavar="MIB",
                    help="first run one device-to-device copy of MIB MiB: a kernel of known traffic that "
                         "hardware byte counters can be scaled by")
    ap.add_argument("--target", type=float, default=0.01, help="statistical uncertainty s of Eq. 12")
    ap.add_argument("--tuning", type=json.loads, default=None, metavar="JSON",
                    help="tuning of the batched legs (water, beamlets) as a JSON object of gmc_tuning fields, "
                         "e.g. '{\"persistent\": 1}'; default: the autotuner's choice")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the per-GPU transport is what is measured; how it would shard "
              "across GPUs is described in the design notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_1101_1245_amd import evaluate as E
    from paper_1101_1245_amd import gpumcd as G
    from paper_1101_1245_amd import inputs as I

    if args.copy_reference > 0:
        import torch
        src = torch.ones(args.copy_reference << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload == "water":
        out, acc = bench_water(args, G, E, I)
        # the roofline covers the plain and batched legs, where each pass kernel has
        # the GPU to itself; served requests overlap on purpose (up to 4 slots), which
        # stretches every kernel's duration
        out["roofline"] = roofline(acc)
        out["ledger_residual_lsb"] = acc.resid
        if not args.no_beamlets:
            import copy
            bargs = copy.copy(args)
            bargs.steps, bargs.warmup = max(1, args.beamlet_steps), 1
            bl = bench_beamlets(bargs, G, E, I)
            out["beamlets"] = {k: bl[k] for k in ("value", "unit", "steps", "ms_per_step", "plain",
                                                   "batched_over_plain", "roofline", "ledger_residual_lsb")}
            out["beamlets"]["workload"] = bl["config"]["workload"]
            out["ledger_residual_lsb"] |= bl["ledger_residual_lsb"]
        if not args.no_serve:
            out["served"], acc_s = bench_serve(args, G, I)
            out["served"]["electron_pass_launches"] = acc_s.n[1]
            out["served"]["electron_pass_ms_mean_overlapped"] = acc_s.t[1] / max(acc_s.n[1], 1) * 1e3
            out["ledger_residual_lsb"] |= acc_s.resid
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline({"electron": out["config"]["n_electrons"],
                                                "photon": out["config"]["n_photons"]})
    elif args.workload == "beamlets":
        out = bench_beamlets(args, G, E, I)
    elif args.workload == "geometries":
        out = bench_geometries(args, G, E, I)
    elif args.workload == "regroup":
        out = bench_regroup(args, G, E, I)
    else:
        out = bench_atomics(args, G)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
