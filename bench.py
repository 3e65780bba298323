#!/usr/bin/env python3
"""Throughput of the stabilised fermion determinant on one MI355X.

Headline (the largest configuration): one HMC step of 32 auxiliary fields on
the honeycomb lattice L = 16 (N = 512 sites), N_t = 512, beta = 64, U = 3,
QR every s = 16 slices, checkpoints every c = 16 slices.  One step = for
every field: the slice exponential exp(+-dk K), the stabilised checkpoint
interval products, the prefix / suffix products, log det M, G = M^-1 and the
full force d log det M / d phi (N_t x N).  The step is a prepared force plan
(exponential included) captured once in a graph and replayed on inputs
resident in HBM; `value` counts field evaluations (log det + G + force of one
field) per second.

Printed as one JSON line, with
  roofline      the step's dominant kernel (largest summed launch time per
                step): model FLOP per launch / average launch time from HIP
                events around every launch on the launch stream (a pass of
                eager calls of the same plan) against the FP64 MFMA peak;
                HBM bytes per launch from committed rocprofv3 counters;
  cpu_baseline  the CPU oracle on the host cores: its own per-slice steps
                timed on a bounded sample at N = 512 and scaled to one field;
and further legs: lowT_L6 (det+G of one N = 72 field, N_t = 256), force
(N = 128 checkpointed adjoint vs the plain per-slice inversion), batched
(256 mixed configurations in one launch sequence vs one call per
configuration), observables, an HMC trajectory, the intermediate-volume
variant (matrix-free product-form slices) against the dense slices, the
time-displaced G(t, t0) (with the CPU oracle's time per pair), and the force
sweep with the per-slice trace of a dense operator against the force alone.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_MFMA = 78.6e12      # MI355X dense FP64 matrix, FLOP/s
PEAK_HBM = 8.0e12             # bytes/s
METRIC = "det+G evals/s & FP64 MFMA %peak; HMC force evals/s, batched/adjoint vs plain"


# ---------------------------------------------------------------------------
# model FLOP counts (complex multiply-add = 8 real FLOP; LAPACK counts)
# ---------------------------------------------------------------------------

def chain_flops(N, rows, s):
    """Slice products 4N^3 each (real E times complex X) and, per chunk of s
    slices, pivoted QR 16/3 N^3 + explicit Q 16/3 N^3 + T update 4 N^3."""
    return N ** 3 * (4.0 * rows + (16 / 3 + 16 / 3 + 4.0) * math.ceil(rows / s))


def combine_flops(N):
    """Bracket 8N^3, QR 16/3, Q 16/3, X1 Q 8N^3, T update 4N^3."""
    return N ** 3 * (8.0 + 16 / 3 + 16 / 3 + 8.0 + 4.0)


def close_flops(N, want_g=True):
    """T X 8N^3, QR 16/3 N^3 and, for G, Q^H 8N^3, R^-1 4N^3, X (.) 8N^3."""
    return N ** 3 * (8.0 + 16 / 3 + ((8.0 + 4.0 + 8.0) if want_g else 0.0))


def expm_flops(N):
    """Six real products of the Paterson-Stockmeyer Taylor polynomial."""
    return 12.0 * N ** 3


def alg_det_flops(N, Nt, s):
    """Algorithmic FLOP of one det+G evaluation: N^3 [4 Nt + 14.67 ceil(Nt/s)
    + 33.3] (slices, per-chunk QR / Q / T update, close with G); the one-time
    exponential and the extra work of time segments are not counted."""
    return chain_flops(N, Nt, s) + close_flops(N)


def det_flops(N, Nt, s, nseg):
    """FLOP the segmented evaluation executes: segment chains, nseg - 1
    combines, the close with G and the exponential."""
    bounds = [Nt * k // nseg for k in range(nseg + 1)]
    f = sum(chain_flops(N, bounds[k + 1] - bounds[k], s) for k in range(nseg))
    return f + (nseg - 1) * combine_flops(N) + close_flops(N) + expm_flops(N)


def alg_force_flops(N, Nt, s, c):
    """Algorithmic FLOP of one force evaluation (log det, G and the force):
    F_det + N^3 Nt (12 + 14.67/s + 64/c) -- a suffix chain, two products per
    carried slice and a recomputation of G~ at every checkpoint."""
    return alg_det_flops(N, Nt, s) + N ** 3 * Nt * (12.0 + (16 / 3 + 16 / 3 + 4.0) / s + 64.0 / c)


def force_item_flops(N, Nt, c, fields):
    """Model FLOP of the force launch: per checkpoint a stabilised product and
    a close with G (the checkpoint's G~), and two real x complex products per
    carried slice (N_t - nc carried slices per field)."""
    nc = math.ceil(Nt / c)
    return fields * (nc * (combine_flops(N) + close_flops(N)) + (Nt - nc) * 8.0 * N ** 3)


def phase_split(call):
    """Launch times of one eager call by phase: [(phase, work items, ms)],
    from HIP events around every launch on the launch stream."""
    import torch
    import paper_2604_02130_amd as fd
    fd.profile_start()
    call()
    torch.cuda.synchronize()
    return [(name, n, round(ms, 4)) for name, n, ms in fd.profile_stop()]


def src_digest():
    from paper_2604_02130_amd import build
    return build.source_digest()


def traffic_from_profiles(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter summaries, only if
    they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("src_digest") != src_digest():
        return None
    return rec.get("bytes_per_launch")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_threads():
    try:
        import threadpoolctl
        return max(i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()) or 1
    except Exception:
        return os.cpu_count()


# ---------------------------------------------------------------------------
# headline: the 32-field N = 512 HMC step
# ---------------------------------------------------------------------------

def headline(args, fd, torch, dev):
    from workload import hmc_batch
    hb = hmc_batch(32)
    w0 = hb[0]
    N, Nt, s, c = w0.N, w0.Nt, w0.s, w0.c
    Kh = torch.from_numpy(w0.K()).to(dev)
    hprobs = [(Kh, torch.from_numpy(wb.phi()).to(dev), wb.dk) for wb in hb]
    a = time.perf_counter()
    plan = fd.Plan("force", hprobs, s=s, checkpoint=c, want_g=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.launch()
    torch.cuda.synchronize()
    setup = time.perf_counter() - a
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    log(f"headline set up in {setup:.1f} s; warmup done; timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = plan.status.cpu()
    if int(st.min()) < 0:
        raise SystemExit(f"HMC step status {st.tolist()}")
    ld_graph = plan.ld.clone()
    step_s = (t1 - t0) / args.steps
    log(f"HMC step (32 fields, N=512): {step_s:.3f} s")

    # per-launch times from HIP events on the launch stream: eager launches
    # of the same plan
    fd.profile_start()
    reps = 1
    for _ in range(reps):
        plan.launch()
    torch.cuda.synchronize()
    phases = fd.profile_stop()
    if not torch.equal(ld_graph, plan.ld):
        raise SystemExit("graph replay and eager launch disagree")
    nc = math.ceil(Nt / c)
    fields = len(hb)
    per_kind = {}
    for name, nitems, ms in phases:
        rec = per_kind.setdefault(name, {"launches": 0, "items": 0, "ms": 0.0})
        rec["launches"] += 1
        rec["items"] += nitems
        rec["ms"] += ms
    model = {
        "expm": 2 * fields * expm_flops(N),
        "chain": fields * nc * chain_flops(N, c, s),
        "combine": per_kind.get("combine", {"items": 0})["items"] * combine_flops(N),
        "force": force_item_flops(N, Nt, c, fields) * reps,
    }
    for name, rec in per_kind.items():
        rec["launches"] //= reps
        rec["items"] //= reps
        rec["ms_per_step"] = rec.pop("ms") / reps
        if name in model and rec["ms_per_step"] > 0:
            rate = model[name] / reps / (rec["ms_per_step"] * 1e-3)
            rec["model_tflop_s"] = rate / 1e12
            rec["frac_fp64_mfma_peak"] = rate / PEAK_FP64_MFMA
    dom = max(per_kind, key=lambda k: per_kind[k]["ms_per_step"])
    drec = per_kind[dom]
    avg_ms = drec["ms_per_step"] / drec["launches"]
    flop_per_launch = model[dom] / reps / drec["launches"]
    achieved = flop_per_launch / (avg_ms * 1e-3)
    kernel = f"k_{dom}<512>"
    roofline = {
        "bound": "mfma",
        "kernel": kernel,
        "achieved": achieved / 1e12,
        "peak": PEAK_FP64_MFMA / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_MFMA,
        "traffic": traffic_from_profiles(f"k_{dom}", "hmc_L16"),
        "avg_launch_ms": avg_ms,
        "model_flop_per_launch": flop_per_launch,
        "phases_per_step": per_kind,
    }
    alg = sum(alg_force_flops(wb.N, wb.Nt, wb.s, wb.c) for wb in hb)
    result = {
        "metric": METRIC,
        "value": fields / step_s,
        "unit": "det+G+force evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "hmc_L16: 32 auxiliary fields, honeycomb L=16 (N=512), Nt=512, beta=64, "
                        "kappa=1, U=3, phi~N(0, delta*U) seeds 5000..5031, s=16, c=16; per step and "
                        "field: exp(+-dk K), log det M, G and the full force dlogdetM/dphi",
            "fields": fields,
            "timed": "graph replay of a prepared force plan (exponential included every step)",
            "parallelism": "single GPU",
        },
        "fp64_mfma_pct_peak": 100.0 * alg / step_s / PEAK_FP64_MFMA,
        "alg_flop_per_step": alg,
        "roofline": roofline,
        "setup_s": setup,
    }
    del graph, plan
    torch.cuda.empty_cache()
    return result, hb


def cpu_baseline_hmc(hb):
    """The oracle's own force method (stabilised prefix and suffix products
    of single slices, one stabilised inversion per row) timed on a bounded
    sample of its steps at N = 512 and scaled to one field: 2 N_t slice
    products and N_t row inversions (row 1 is G, its close gives log det)."""
    import numpy as np
    from oracle import fdet_oracle as F
    w = hb[0]
    K, phi = w.K(), w.phi()
    N, Nt = w.N, w.Nt
    U, e = F._slice_factors(K, w.dk)
    slices = [F._slice_udv(U, e, np.exp(1j * phi[t])) for t in range(24)]
    P = F.udv_product(slices[0], F.udv_identity(N))      # warm-up
    n_prod, t_prod = 0, 0.0
    a = time.perf_counter()
    for t in range(1, 21):
        P = F.udv_product(slices[t], P)
        n_prod += 1
    t_prod = (time.perf_counter() - a) / n_prod
    S = F.udv_product(F.udv_identity(N), slices[23])
    F.udv_close(F.udv_product(P, S))                    # warm-up
    n_close = 8
    a = time.perf_counter()
    for _ in range(n_close):
        F.udv_close(F.udv_product(P, S))
    t_close = (time.perf_counter() - a) / n_close
    per_field = 2 * Nt * t_prod + Nt * t_close
    return {
        "value": 1.0 / per_field,
        "unit": "det+G+force evals/s",
        "cores": host_threads(),
        "kind": "oracle",
        "sample": f"extrapolated from a timed sample of the oracle's own steps at N={N}: "
                  f"{n_prod} stabilised single-slice products ({t_prod:.3f} s each) and "
                  f"{n_close} row inversions (product + close, {t_close:.3f} s each); one field "
                  f"= 2*{Nt} products + {Nt} inversions = {per_field:.0f} s",
    }


# ---------------------------------------------------------------------------
# further legs
# ---------------------------------------------------------------------------

def leg_lowT(args, fd, torch, dev):
    """det + G of the low-temperature single configuration (N = 72)."""
    from workload import WORKLOADS
    w = WORKLOADS["lowT_L6"]
    N, Nt, s = w.N, w.Nt, w.s
    Kd = torch.from_numpy(w.K()).to(dev)
    pd = torch.from_numpy(w.phi()).to(dev)
    tuned = fd.autotune([(Kd, pd, w.dk)], what="greens", s=s)
    nseg = tuned["segments"]
    plan = fd.Plan("greens", [(Kd, pd, w.dk)], s=s, segments=nseg)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.launch()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        plan.launch()
    for _ in range(5):
        graph.replay()
    torch.cuda.synchronize()
    reps = 50
    a = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - a) / reps
    phases = phase_split(plan.launch)
    per = {}
    for name, nitems, ms in phases:
        per.setdefault(name, []).append(ms)
    out = {
        "workload": "lowT_L6: honeycomb L=6 (N=72), Nt=256, beta=32, U=3, s=8; log det M and G",
        "evals_per_s": 1.0 / dt,
        "ms": dt * 1e3,
        "segments": nseg,
        "fp64_mfma_pct_peak": 100.0 * alg_det_flops(N, Nt, s) / dt / PEAK_FP64_MFMA,
        "phases_ms": {k: v for k, v in per.items()},
    }
    if not args.no_cpu:
        import oracle
        K, phi = w.K(), w.phi()
        oracle.sporadic_logdet_greens(K, w.dk, phi, s)
        n, a = 0, time.perf_counter()
        while True:
            oracle.sporadic_logdet_greens(K, w.dk, phi, s)
            n += 1
            if time.perf_counter() - a > 5.0:
                break
        dtc = time.perf_counter() - a
        out["cpu_oracle"] = {"evals_per_s": n / dtc, "cores": host_threads(),
                             "sample": f"{n} det+G evals (QR every {s} slices), {dtc:.1f} s"}
    log(f"lowT_L6 det+G: {dt * 1e3:.3f} ms")
    return out


def leg_force(fd, torch, dev):
    from workload import WORKLOADS
    wf = WORKLOADS["force_L8"]
    Kf = torch.from_numpy(wf.K()).to(dev)
    pf = torch.from_numpy(wf.phi()).to(dev)
    wsf = fd.Workspace()
    out = {}
    for label, c, reps in (("adjoint_c16", wf.c, 5), ("plain_c1", 1, 2)):
        fd.force(Kf, pf, wf.dk, s=wf.s, checkpoint=c, check=False, ws=wsf)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            fd.force(Kf, pf, wf.dk, s=wf.s, checkpoint=c, check=False, ws=wsf)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - a) / reps
        out[label] = {"force_evals_per_s": 1.0 / dt, "ms": dt * 1e3,
                      "alg_tflop_s": alg_force_flops(wf.N, wf.Nt, wf.s, 16) / dt / 1e12,
                      "phases_ms": phase_split(lambda: fd.force(
                          Kf, pf, wf.dk, s=wf.s, checkpoint=c, check=False, ws=wsf))}
        log(f"force {label}: {dt * 1e3:.2f} ms")
    trf = fd.Trajectory(Kf, pf, wf.dk, s=wf.s, checkpoint=wf.c)
    trf.replay()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(10):
        trf.replay()
    torch.cuda.synchronize()
    out["adjoint_c16"]["graph_ms"] = (time.perf_counter() - a) / 10 * 1e3
    del trf
    out["workload"] = "force_L8: honeycomb L=8 (N=128), Nt=256, beta=32, U=3, s=8"
    out["adjoint_vs_plain"] = out["adjoint_c16"]["force_evals_per_s"] / out["plain_c1"]["force_evals_per_s"]
    return out


def leg_batched(fd, torch, dev):
    from workload import batched_mix
    mix = batched_mix()
    cache = {}
    probs = []
    for wb in mix:
        if wb.L not in cache:
            cache[wb.L] = torch.from_numpy(wb.K()).to(dev)
        probs.append((cache[wb.L], torch.from_numpy(wb.phi()).to(dev), wb.dk))
    wsb = fd.Workspace()
    fd.greens_batched(probs, s=8, check=False, ws=wsb)
    torch.cuda.synchronize()
    reps = 3
    a = time.perf_counter()
    for _ in range(reps):
        fd.greens_batched(probs, s=8, check=False, ws=wsb)
    torch.cuda.synchronize()
    dtb = (time.perf_counter() - a) / reps
    plain = {}
    # one call per configuration: the library's single-configuration default
    # segments, and one segment (one sequential chain per call); one warm-up
    # pass per form
    for label, seg in (("plain_default_segments", 0), ("plain_one_segment", 1)):
        for (Kb, pb, dkb) in probs:
            fd.greens(Kb, pb, dkb, s=8, segments=seg, check=False, ws=wsb)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for (Kb, pb, dkb) in probs:
            fd.greens(Kb, pb, dkb, s=8, segments=seg, check=False, ws=wsb)
        torch.cuda.synchronize()
        plain[label] = time.perf_counter() - a
    bflops = sum(alg_det_flops(wb.N, wb.Nt, 8) for wb in mix)
    bphases = phase_split(lambda: fd.greens_batched(probs, s=8, check=False, ws=wsb))
    log(f"batched {dtb * 1e3:.1f} ms vs plain {plain['plain_default_segments'] * 1e3:.1f} ms "
        f"(default segments) / {plain['plain_one_segment'] * 1e3:.1f} ms (one segment)")
    return {
        "workload": "256 configs, L in {3,5,6,7,8}, Nt in {32..512}, delta=0.125, U=3, s=8",
        "batched_evals_per_s": len(mix) / dtb,
        "batched_ms": dtb * 1e3,
        "plain_default_segments_evals_per_s": len(mix) / plain["plain_default_segments"],
        "plain_one_segment_evals_per_s": len(mix) / plain["plain_one_segment"],
        "batched_vs_plain_default_segments": plain["plain_default_segments"] / dtb,
        "batched_vs_plain_one_segment": plain["plain_one_segment"] / dtb,
        "fp64_mfma_pct_peak": 100.0 * bflops / dtb / PEAK_FP64_MFMA,
        "phases_ms": bphases,
    }


def leg_observables(fd, torch, dev):
    import numpy as np
    obs = {"workload": "tr((1 - G) A) of one random complex G and A (k_trace_tiles + "
                       "k_trace_final); algorithmic bytes 2 N^2 x 16 B read"}
    rng = np.random.default_rng(5)
    for No in (72, 512):
        Go = torch.from_numpy(rng.normal(size=(No, No)) + 1j * rng.normal(size=(No, No))).to(dev)
        Ao = torch.from_numpy(rng.normal(size=(No, No)) + 1j * rng.normal(size=(No, No))).to(dev)
        wso = fd.Workspace()
        for _ in range(10):
            fd.response_trace(Go, Ao, ws=wso)
        reps = 200
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fd.response_trace(Go, Ao, ws=wso)
        ev1.record()
        torch.cuda.synchronize()
        us = ev0.elapsed_time(ev1) * 1e3 / reps
        gr = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fd.response_trace(Go, Ao, ws=wso)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(gr):
            for _ in range(20):
                fd.response_trace(Go, Ao, ws=wso)
        gr.replay()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(10):
            gr.replay()
        ev1.record()
        torch.cuda.synchronize()
        us_g = ev0.elapsed_time(ev1) * 1e3 / 200
        del gr
        nbytes = 2 * No * No * 16
        obs[f"N{No}"] = {"us_per_call": us, "us_per_call_graph": us_g,
                         "hbm_gb_s": nbytes / (us_g * 1e-6) / 1e9,
                         "frac_hbm_peak": nbytes / (us_g * 1e-6) / PEAK_HBM}
        log(f"response trace N={No}: {us:.1f} us per call, {us_g:.1f} us in a graph")
    return obs


def leg_trajectory(fd, torch, dev):
    """One leapfrog trajectory of the force_L8 field; the step size keeps the
    energy error of order one (it grows as eps^2)."""
    import numpy as np
    from workload import WORKLOADS
    wm = WORKLOADS["force_L8"]
    Km = torch.from_numpy(wm.K()).to(dev)
    pm = torch.from_numpy(wm.phi()).to(dev)
    rng = np.random.default_rng(6)
    pim = torch.from_numpy(rng.standard_normal(wm.phi().shape).reshape(-1)).to(dev)
    wsm = fd.Workspace()
    nmd, epsm, dUm = 4, 0.0015, wm.dk * 3.0
    fd.hmc_leapfrog([(Km, pm, wm.dk)], pim.clone(), dUm, epsm, nmd, s=wm.s, checkpoint=wm.c,
                    ws=wsm)
    torch.cuda.synchronize()
    reps = 3
    a = time.perf_counter()
    for _ in range(reps):
        dHm = fd.hmc_leapfrog([(Km, pm, wm.dk)], pim.clone(), dUm, epsm, nmd, s=wm.s,
                              checkpoint=wm.c, ws=wsm)
    torch.cuda.synchronize()
    dtm = (time.perf_counter() - a) / reps
    hplan = fd.HmcPlan([(Km, pm, wm.dk)], dUm, epsm, nmd, s=wm.s, checkpoint=wm.c)
    hplan.pi.copy_(pim)
    hplan.capture()
    hplan.replay()
    torch.cuda.synchronize()
    a = time.perf_counter()
    for _ in range(reps):
        hplan.replay()
    torch.cuda.synchronize()
    dtg = (time.perf_counter() - a) / reps
    hplan.close()
    log(f"HMC trajectory (4 steps, N=128): {dtm * 1e3:.1f} ms, graph {dtg * 1e3:.1f} ms, "
        f"dH {float(dHm[0]):.3f}")
    return {
        "workload": f"force_L8 field (N=128, Nt=256, s=8, c=16), leapfrog of {nmd} steps "
                    f"({nmd + 1} force evaluations), eps={epsm}, dU=delta*U",
        "ms": dtm * 1e3,
        "ms_per_force_eval": dtm * 1e3 / (nmd + 1),
        "graph_ms": dtg * 1e3,
        "dH": float(dHm[0]),
    }


# ---------------------------------------------------------------------------

def leg_sparse(args, fd, torch, dev):
    """Intermediate-volume low-temperature variant (Sec. 9 with the product-form
    slices of Sec. 8, n = 4): det + G of field 0 of the headline batch
    (N = 512, N_t = 512, beta = 64, s = 16) with matrix-free slices, against
    det + G of the same field with the dense exponential, both with the
    library's default time segments."""
    from workload import hmc_batch
    w = hmc_batch()[0]
    N, Nt, s, n = w.N, w.Nt, w.s, 4
    Kd = torch.from_numpy(w.K()).to(dev)
    pd = torch.from_numpy(w.phi()).to(dev)
    col, val = fd.ell(Kd)
    q = int(col.shape[1])
    ws = fd.Workspace()
    out = {"workload": "field 0 of hmc_L16 (N=512, Nt=512, beta=64, U=3), s=16; log det M and G; "
                       "sparse: degree-4 product-form Taylor slices applied matrix-free (q=3)"}
    for label, call in (("sparse", lambda: fd.sparse_greens(col, val, pd, w.dk, n=n, s=s, ws=ws,
                                                            check=False)),
                        ("dense", lambda: fd.greens(Kd, pd, w.dk, s=s, ws=ws, check=False))):
        call()
        torch.cuda.synchronize()
        reps = 5
        a = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - a) / reps
        out[label] = {"ms": dt * 1e3, "evals_per_s": 1.0 / dt, "phases_ms": phase_split(call)}
        log(f"sparse leg {label}: {dt * 1e3:.2f} ms")
    # the matrix-free slices: per slice and matrix element one field phase
    # (6 FLOP) and n stencil steps of q real x complex terms plus the complex
    # scale (4 q + 8 FLOP); LDS traffic (q + 2) x 16 B per step + 32 B per phase
    chain_ms = sum(ms for name, _, ms in out["sparse"]["phases_ms"] if name == "chain")
    flop = Nt * N * N * (n * (4 * q + 8) + 6)
    lds = Nt * N * N * (n * (q + 2) * 16 + 32)
    out["sparse"]["stencil_model_flop"] = flop
    out["sparse"]["stencil_model_lds_bytes"] = lds
    out["sparse"]["chain_ms"] = chain_ms
    out["sparse_vs_dense"] = out["dense"]["ms"] / out["sparse"]["ms"]
    if not args.no_cpu:
        import scipy.sparse as sp
        import oracle
        Ks = sp.csr_matrix(w.K())
        a = time.perf_counter()
        oracle.sparse_logdet_greens(Ks, w.dk, w.phi(), n, s)
        dtc = time.perf_counter() - a
        out["cpu_oracle"] = {"evals_per_s": 1.0 / dtc, "cores": host_threads(),
                             "sample": f"1 det+G eval of the same field (sparse K, QR every {s} "
                                       f"slices), {dtc:.1f} s"}
    return out


def force_cpu_oracle():
    """The oracle's force (stabilised prefix and suffix products of single
    slices, one stabilised inversion per row) on the force_L8 field, timed on
    a bounded sample of its steps and scaled to one evaluation: 2 N_t slice
    products and N_t row inversions (as the headline's cpu_baseline does at
    N = 512)."""
    import numpy as np
    from oracle import fdet_oracle as F
    from workload import WORKLOADS
    w = WORKLOADS["force_L8"]
    K, phi = w.K(), w.phi()
    N, Nt = w.N, w.Nt
    U, e = F._slice_factors(K, w.dk)
    slices = [F._slice_udv(U, e, np.exp(1j * phi[t])) for t in range(24)]
    P = F.udv_product(slices[0], F.udv_identity(N))      # warm-up
    n_prod = 20
    a = time.perf_counter()
    for t in range(1, n_prod + 1):
        P = F.udv_product(slices[t], P)
    t_prod = (time.perf_counter() - a) / n_prod
    S = F.udv_product(F.udv_identity(N), slices[23])
    F.udv_close(F.udv_product(P, S))                    # warm-up
    n_close = 8
    a = time.perf_counter()
    for _ in range(n_close):
        F.udv_close(F.udv_product(P, S))
    t_close = (time.perf_counter() - a) / n_close
    per_eval = 2 * Nt * t_prod + Nt * t_close
    return {"force_evals_per_s": 1.0 / per_eval, "s_per_eval": per_eval, "cores": host_threads(),
            "kind": "oracle",
            "sample": f"extrapolated from {n_prod} stabilised single-slice products "
                      f"({t_prod:.4f} s each) and {n_close} row inversions ({t_close:.4f} s each) "
                      f"at N={N}; one evaluation = 2*{Nt} products + {Nt} inversions"}


def leg_displaced(args, fd, torch, dev):
    """Time-displaced G(t, t0) (two slice chains per pair and a scale-split
    close, Sec. 7 steps 7-9) on the lowT_L6 field for the pairs its parity test
    checks, beside the CPU oracle's split close of one pair.  Model FLOP per
    pair: the slice chains over all N_t slices with their QRs, one stabilised
    product and a close with G."""
    from workload import WORKLOADS
    w = WORKLOADS["lowT_L6"]
    K = torch.from_numpy(w.K()).to(dev)
    ph = torch.from_numpy(w.phi()).to(dev)
    pairs = [(1, 1), (130, 3), (3, 130), (256, 1), (1, 256), (77, 76)]
    ws = fd.Workspace()
    fd.greens_displaced(K, ph, w.dk, pairs, s=w.s, ws=ws)   # checks the status
    torch.cuda.synchronize()
    reps = 5
    a = time.perf_counter()
    for _ in range(reps):
        fd.greens_displaced(K, ph, w.dk, pairs, s=w.s, check=False, ws=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - a) / reps
    flop = len(pairs) * (chain_flops(w.N, w.Nt, w.s) + combine_flops(w.N) + close_flops(w.N))
    out = {"workload": f"lowT_L6 field (N={w.N}, Nt={w.Nt}, beta={w.beta}, s={w.s}), "
                       f"{len(pairs)} (t, t0) pairs per call",
           "ms_per_call": dt * 1e3, "pairs_per_s": len(pairs) / dt,
           "model_tflop_s": flop / dt / 1e12,
           "phases_ms": phase_split(lambda: fd.greens_displaced(K, ph, w.dk, pairs, s=w.s,
                                                                check=False, ws=ws))}
    log(f"displaced G: {dt * 1e3:.2f} ms per call of {len(pairs)} pairs")
    if not args.no_cpu:
        import oracle
        a = time.perf_counter()
        oracle.dsplit_displaced_greens(w.K(), w.dk, w.phi(), 130, 3)
        cpu = time.perf_counter() - a
        out["cpu_oracle_s_per_pair"] = cpu
        out["vs_cpu_oracle"] = cpu / (dt / len(pairs))
    return out


def leg_force_response(fd, torch, dev):
    """The force sweep with the per-slice trace tr((1 - G~_t) A) of a dense
    complex A (eq. response_simple before its slice average) on the lowT_L6
    field, against the same force without the trace."""
    import numpy as np
    from workload import WORKLOADS
    w = WORKLOADS["lowT_L6"]
    K = torch.from_numpy(w.K()).to(dev)
    ph = torch.from_numpy(w.phi()).to(dev)
    rng = np.random.default_rng(2700)
    A = torch.from_numpy(rng.normal(size=(w.N, w.N)) + 1j * rng.normal(size=(w.N, w.N))).to(dev)
    ws = fd.Workspace()
    fd.force_response(K, ph, w.dk, A, s=w.s, checkpoint=16, ws=ws)   # checks the status
    torch.cuda.synchronize()
    out = {"workload": f"lowT_L6 field (N={w.N}, Nt={w.Nt}, beta={w.beta}, s={w.s}, c=16), "
                       "dense complex A"}
    reps = 5
    for label, call in (
            ("with_trace", lambda: fd.force_response(K, ph, w.dk, A, s=w.s, checkpoint=16,
                                                     check=False, ws=ws)),
            ("force_only", lambda: fd.force(K, ph, w.dk, s=w.s, checkpoint=16, check=False,
                                            ws=ws))):
        call()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(reps):
            call()
        torch.cuda.synchronize()
        out[label] = {"ms": (time.perf_counter() - a) / reps * 1e3}
    out["trace_overhead"] = out["with_trace"]["ms"] / out["force_only"]["ms"]
    log(f"force with trace {out['with_trace']['ms']:.2f} ms, without {out['force_only']['ms']:.2f} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baselines")
    ap.add_argument("--no-extra", action="store_true", help="only the headline")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} (WORLD_SIZE={world}) "
              "is not supported by this single-GPU build", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2604_02130_amd as fd

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(2)
    fd.load_library()
    dev = torch.device("cuda:0")

    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    result, hb = headline(args, fd, torch, dev)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline_hmc(hb)
        log(f"cpu oracle: {result['cpu_baseline']['value']:.3e} evals/s (extrapolated)")
    if not args.no_extra:
        result["lowT_L6"] = leg_lowT(args, fd, torch, dev)
        result["force"] = leg_force(fd, torch, dev)
        if not args.no_cpu:
            try:
                result["force"]["cpu_oracle"] = force_cpu_oracle()
            except Exception as e:  # noqa: BLE001
                result["force"]["cpu_oracle"] = {"error": f"{type(e).__name__}: {e}"}
        result["batched"] = leg_batched(fd, torch, dev)
        result["observables"] = leg_observables(fd, torch, dev)
        result["hmc_trajectory"] = leg_trajectory(fd, torch, dev)
        result["sparse"] = leg_sparse(args, fd, torch, dev)
        # an error in one of these legs is reported in its key; the line is printed anyway
        for key, leg in (("displaced", lambda: leg_displaced(args, fd, torch, dev)),
                         ("force_response", lambda: leg_force_response(fd, torch, dev))):
            try:
                result[key] = leg()
            except Exception as e:  # noqa: BLE001
                result[key] = {"error": f"{type(e).__name__}: {e}"}
                log(f"{key} leg failed: {e}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
