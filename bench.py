"""Benchmark of the per-step particle loop on one MI355X.

A step is one pass of the whole loop (injection, lepton pass, photon pass,
field, periodic re-sort) over the production gap: 65536 cells, alpha = 1.5,
b = 0.1, R_curv = 1e7 cm, surface injection 0.1 n_co dx per step, started from
the seeded initial state and grown (untimed) by the physics itself until the
stores hold at least --grow-to particles.  Then --warmup untimed steps and
--steps timed steps; inputs are resident in HBM throughout.

Prints one JSON line.  `value` is particle-steps/s (leptons + photons
advanced by one step) over the timed steps, which run without any
instrumentation.  Right after them the same number of steps runs again with a
HIP event pair around every kernel group (on the library's stream): that pass
gives the per-kernel average launch times.  `roofline` is the dominant
kernel's algorithmic HBM bytes per launch over its average launch time;
`step_roofline` is the whole step's algorithmic bytes over the timed step
time.  `cpu_baseline` is the FP64 oracle on a bounded sample of the same
grown state, on this host.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KERNEL_SOURCES = ("gap_device.hpp", "gap_kernels.hpp")   # code of the two particle kernels
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_leptons_k_photons_production.txt")
# algorithmic bytes per unit of work: a lepton-step reads position, momentum
# and weight and writes position and momentum (20 B); a lepton-step that
# evaluates emission also reads the 8-byte id.  A photon-step reads position,
# energy, weight, birth step and id and writes position (28 B).
B_LEP, B_EMIT_EVAL, B_PHO = 20, 8, 28
# bytes the photon kernel must move at least: position, energy and birth step
# read and position written for every photon (16 B); id and weight only for
# the photons that draw a conversion (12 B)
B_PHO_MIN, B_CONV_EVAL_MIN = 16, 12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def grow(g, target, max_steps, block=1000):
    t0 = time.time()
    while True:
        c = g.counts()
        n = c["n_lep"] + c["n_pho"]
        if n >= target or c["step"] >= max_steps:
            log("grown: step %d leptons %d photons %d (%.1f s)" % (c["step"], c["n_lep"], c["n_pho"], time.time() - t0))
            return c
        g.step(block)
        g.sync()
        log("  grow: step %d particles %d" % (c["step"] + block, n))


def kernel_source_hash():
    """sha256 over the sources of the particle kernels, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_21920_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary.

    The summary holds FETCH_SIZE + WRITE_SIZE per dispatch, already scaled by
    the copy calibration, and the hash of the kernel sources it was taken
    with; a summary taken with other sources gives None."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    kv = {}
    for ln in lines:
        m = re.match(r"^(\S+)\s*=\s*(\S+)\s*$", ln)
        if m:
            kv[m.group(1)] = m.group(2)
    if kv.get("kernel_source_sha256") != kernel_source_hash():
        return None
    v = kv.get("hbm_bytes_per_launch." + kernel)
    return float(v) if v is not None else None


class ProfilerRegion:
    """roctx resume/pause around the timed steps, so that a profiler run with
    --selected-regions collects exactly the timed launches (no-op otherwise)."""

    def __init__(self):
        import ctypes
        self.lib = None
        for name in ("librocprofiler-sdk-roctx.so.1", "librocprofiler-sdk-roctx.so"):
            try:
                self.lib = ctypes.CDLL(name)
                break
            except OSError:
                continue
        if self.lib is not None:
            for fn in (self.lib.roctxProfilerResume, self.lib.roctxProfilerPause):
                fn.argtypes = [ctypes.c_uint64]
                fn.restype = ctypes.c_int

    def resume(self):
        if self.lib is not None:
            self.lib.roctxProfilerResume(0)

    def pause(self):
        if self.lib is not None:
            self.lib.roctxProfilerPause(0)


def cpu_baseline(cfg, step, budget_s=15.0, sample=400_000):
    """Oracle particle-steps/s on a seeded discharge-like sample of the
    production gap (4e5 particles, 39% leptons as in the grown state)."""
    from oracle.oracle import Oracle
    from paper_2608_21920_amd import inputs
    nl = int(0.39 * sample)
    L, P = inputs.discharge_sample(7, cfg["n_cells"], cfg.get("h_gap_frac", 0.8), nl, sample - nl, step)
    o = Oracle(cfg)
    o.set_state(inputs.leptons_as_oracle(L), inputs.photons_as_oracle(P), Es=0.0, step=step)
    c_start = o.counts()
    t0 = time.time()
    done = 0
    ps = 0
    while time.time() - t0 < budget_s:
        c0 = o.counts()
        o.step(1)
        ps += c0["n_lep"] + c0["n_pho"]
        done += 1
    el = time.time() - t0
    c_end = o.counts()
    ev = (c_end["n_emit_eval"] - c_start["n_emit_eval"]) / max(1, ps)
    cv = (c_end["n_conv_eval"] - c_start["n_conv_eval"]) / max(1, ps)
    return dict(value=ps / el, unit="particle-steps/s", cores=1, kind="oracle",
                sample="seeded discharge-like state of the production gap: %d leptons (gamma log-uniform in "
                       "[1, 1e8] over the QED zone) + %d photons (x log-uniform in [2, 1e8]), %d steps in %.1f s; "
                       "emission / conversion evaluations per particle-step %.3f / %.3f" % (nl, sample - nl, done, el, ev, cv))


def bench_batched(plain_value, n_tubes=256):
    """The batched ensemble (uneven tubes in one set of launches), autotuned,
    timed over graph replays of twice the re-sort interval (so that every
    replay starts from the same layout and reuses one captured graph), then
    over as many eager steps (the photon side on the library's second
    stream; a captured graph keeps every kernel on one stream).  `value` is
    the faster of the two, both are reported."""
    import torch
    from paper_2608_21920_amd import Gap, workloads
    cfgs = workloads.batched_tubes(n_tubes, seed=1)
    t0 = time.time()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = Gap(cfgs, stream=s)
        g.sync()
        t_init = time.time() - t0
        tune = g.autotune(16)
        log("batched: %d tubes built in %.1f s, autotune %s" % (n_tubes, t_init, tune))
        steps = 2 * tune["resort_every"]
        g.step_graph(steps)          # capture and a first replay
        g.sync()

        def totals():
            tot = dict(lep=0, pho=0, emit=0, conv=0, n_lep=0, n_pho=0)
            for t in range(n_tubes):
                c = g.counts(t)
                tot["lep"] += c["lep_steps"]
                tot["pho"] += c["pho_steps"]
                tot["emit"] += c["n_emit_eval"]
                tot["conv"] += c["n_conv_eval"]
                tot["n_lep"] += c["n_lep"]
                tot["n_pho"] += c["n_pho"]
                assert c["err"] == 0, (t, c)
            return tot
        c0 = totals()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        g.step_graph(steps)
        g.step_graph(steps)
        e1.record(s)
        g.sync()
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1)
        c1 = totals()
        e0.record(s)
        g.step(2 * steps)
        e1.record(s)
        g.sync()
        torch.cuda.synchronize()
        ms_eager = e0.elapsed_time(e1)
        c2 = totals()
        g.close()
    n = 2 * steps
    ps_g = (c1["lep"] - c0["lep"]) + (c1["pho"] - c0["pho"])
    ps_e = (c2["lep"] - c1["lep"]) + (c2["pho"] - c1["pho"])
    graph = ps_g / ms_graph >= ps_e / ms_eager
    a, b = (c0, c1) if graph else (c1, c2)
    ms = ms_graph if graph else ms_eager
    ps = ps_g if graph else ps_e
    alg = B_LEP * (b["lep"] - a["lep"]) + B_EMIT_EVAL * (b["emit"] - a["emit"]) + B_PHO * (b["pho"] - a["pho"])
    value = ps / (ms / 1e3)
    return dict(value=value, unit="particle-steps/s", tubes=n_tubes, steps=n, ms_per_step=ms / n,
                ms_per_step_graph=ms_graph / n, ms_per_step_eager=ms_eager / n,
                leptons=c0["n_lep"], photons=c0["n_pho"], graph=graph, autotune=tune,
                hbm_frac_whole_step=alg / (ms / 1e3) / 1e9 / PEAK_HBM_GBS,
                vs_plain=value / plain_value if plain_value else None,
                config="256 tubes: cells uniform in [2048, 16384], alpha uniform in [-1, 2], B/B_Q log-uniform "
                       "in [0.01, 0.3], ppc uniform in [4, 64] per species, seed 1; uniform e+- start, "
                       "physical QED")


def bench_adjoint(window=2000, ckpt=100):
    """The differentiable window: forward (checkpoints) + reverse pass, and the
    same number of plain steps of the same gap."""
    import torch
    from paper_2608_21920_amd import Gap, workloads
    from paper_2608_21920_amd import gap as G
    cfg = dict(workloads.ADJOINT, flags=G.INJ_FIXED)
    g = Gap(cfg)
    g.sync()
    c0 = g.counts()
    t0 = time.time()
    loss = g.window_forward(window, ckpt)[0]
    t1 = time.time()
    da, dn = g.backward()
    t2 = time.time()
    c1 = g.counts()
    assert c1["err"] == 0, c1
    g.close()
    p = Gap(cfg)
    p.sync()
    torch.cuda.synchronize()
    t3 = time.time()
    p.step(window)
    p.sync()
    t4 = time.time()
    p.close()
    ps = (c1["lep_steps"] - c0["lep_steps"]) + (c1["pho_steps"] - c0["pho_steps"])
    fwd, bwd, plain = (t1 - t0) * 1e3, (t2 - t1) * 1e3, (t4 - t3) * 1e3
    return dict(value=ps / ((fwd + bwd) / 1e3), unit="particle-steps/s (window forward + backward)",
                window_steps=window, ckpt_every=ckpt, leptons_start=c0["n_lep"], particle_steps=ps,
                forward_ms=fwd, backward_ms=bwd, plain_ms=plain, fwd_bwd_over_plain=(fwd + bwd) / plain,
                loss=loss, dL_dalpha=float(da[0]), dL_dninj=float(dn[0]),
                config="16384 cells, 122 e- + 122 e+ per cell, rescaled QED (tiny preset), injection 0.1 "
                       "n_co dx per step, frozen QED, loss = time-averaged <E^2>")


def bench_filter(steps=200):
    """The current filter (8 binomial passes per step) on the production grid:
    the same start state of the production gap stepped with and without it,
    wall time per step and the field update's share (HIP-event timing of
    the field group, which then includes the filter kernel)."""
    from paper_2608_21920_amd import Gap, workloads
    from paper_2608_21920_amd import gap as G
    out = {}
    for name, extra in (("plain", 0), ("filtered", G.FILTER)):
        cfg = dict(workloads.PRODUCTION)
        cfg["flags"] = cfg.get("flags", 0) | extra
        g = Gap(cfg)
        g.step(20)
        g.sync()
        t0 = time.perf_counter()
        g.step(steps)
        g.sync()
        wall = (time.perf_counter() - t0) * 1e3 / steps
        g.set_timing(True)
        g.step(steps)
        g.sync()
        n, tms = g.timing()["field"]
        g.set_timing(False)
        out[name] = dict(ms_per_step=wall, field_us=tms / max(n, 1) * 1e3, leptons=g.counts()["n_lep"])
        g.close()
    out["filter_us_per_step"] = (out["filtered"]["field_us"] - out["plain"]["field_us"])
    out["config"] = "production gap start state (65536 cells), %d steps each" % steps
    return out


def bench_diagnostics(g, calls=5):
    """The discharge diagnostics on the grown production state: wall time of
    one peak-multiplicity call (bins of 64 cells: zeroing the sums, the profile
    pass over both stores, the peak kernel, the 48-byte copy back), with 12 B
    per particle read (position, momentum or energy, weight) as its bytes; and
    the step time with the waterfall recorded after every step."""
    g.set_profile_bin(64)
    pk = g.peak()
    g.sync()
    t0 = time.perf_counter()
    for _ in range(calls):
        g.peak()
    ms = (time.perf_counter() - t0) * 1e3 / calls
    c = g.counts()
    n = c["n_lep"] + c["n_pho"]

    # the E^2 waterfall (Fig. 4) recorded after every step in bins of 64
    # cells: wall time per step with and without it, over two re-sort
    # intervals each
    def wall(k):
        g.sync()
        t0 = time.perf_counter()
        g.step(k)
        g.sync()
        return (time.perf_counter() - t0) * 1e3 / k

    # the power spectrum of E (65536 cells -> one FP64 FFT of 2^16 points)
    g.e_spectrum()
    g.sync()
    t0 = time.perf_counter()
    for _ in range(calls):
        g.e_spectrum()
    spec_ms = (time.perf_counter() - t0) * 1e3 / calls
    # the momentum spectra of both species (one pass over both stores)
    g.spectra()
    g.sync()
    t0 = time.perf_counter()
    for _ in range(calls):
        g.spectra()
    mspec_ms = (time.perf_counter() - t0) * 1e3 / calls
    # phase space (bins of 64 cells x 180 signed momentum columns)
    g.phase_space()
    g.sync()
    t0 = time.perf_counter()
    for _ in range(calls):
        g.phase_space()
    phase_ms = (time.perf_counter() - t0) * 1e3 / calls

    k = 2 * 136
    plain = wall(k)
    g.set_waterfall(1, 64, 64)
    rec = wall(k)
    ws, we = g.waterfall()
    g.set_waterfall(0)
    return dict(peak_call_ms=ms, particles=n, gbs_at_12_bytes=12.0 * n / (ms / 1e3) / 1e9,
                m_pairs_peak=pk["m_pairs"], h_peak=pk["h"], g3_at_peak=pk["g3"], e_min=pk["e_min"],
                e_max=pk["e_max"], e_spectrum_call_ms=spec_ms, momentum_spectra_call_ms=mspec_ms, phase_space_call_ms=phase_ms, waterfall=dict(ms_per_step_without=plain, ms_per_step_with=rec,
                                                  records_read=int(ws.size), bins=int(we.shape[1]),
                                                  max_e2=float(we.max()) if we.size else None))


def copy_calibration(nbytes):
    """A plain device copy of known size, for scaling HBM traffic counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--grow-to", type=float, default=2.0e7)
    ap.add_argument("--max-grow-steps", type=int, default=90000)
    ap.add_argument("--graph", action="store_true", help="time graph replays instead of eager steps")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calib", type=int, default=0, help="only run a device copy of this many bytes")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched ensemble")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiable window")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d refused)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.copy_calib:
        copy_calibration(a.copy_calib)
        return

    import torch
    from paper_2608_21920_amd import Gap, workloads
    cfg = dict(workloads.PRODUCTION)
    g = Gap(cfg)
    grow(g, a.grow_to, a.max_grow_steps)
    g.step(a.warmup)
    g.sync()

    s = g.stream
    region = ProfilerRegion()

    def run(steps, timing):
        c_a = g.counts()
        g.set_timing(timing)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        if not timing:
            region.resume()
        e0.record(s)
        if a.graph:
            g.step_graph(steps)
        else:
            g.step(steps)
        e1.record(s)
        g.sync()
        torch.cuda.synchronize()
        if not timing:
            region.pause()
        tim = g.timing() if timing else None
        g.set_timing(False)
        c_b = g.counts()
        assert c_b["err"] == 0, c_b
        return e0.elapsed_time(e1), {k: c_b[k] - c_a[k] for k in c_b}, tim, c_a

    # timed steps (no instrumentation), then the same number with kernel events
    ms, dA, _, c0 = run(a.steps, False)
    c1 = g.counts()
    psteps = dA["lep_steps"] + dA["pho_steps"]
    value = psteps / (ms / 1e3)
    step_bytes = B_LEP * dA["lep_steps"] + B_EMIT_EVAL * dA["n_emit_eval"] + B_PHO * dA["pho_steps"]
    step_roof = dict(bound="hbm", achieved=step_bytes / (ms / 1e3) / 1e9, peak=PEAK_HBM_GBS, unit="GB/s",
                     frac=step_bytes / (ms / 1e3) / 1e9 / PEAK_HBM_GBS, bytes_per_step=step_bytes / a.steps)
    kern, roof, tim, ms_i = {}, None, None, None
    if not a.graph:
        ms_i, d, tim, _ = run(a.steps, True)
        # algorithmic bytes of the sorted-region kernels and of the tail kernels
        # (the tail passes of both species are one launch)
        lep_b = lambda n_steps, n_eval: B_LEP * n_steps + B_EMIT_EVAL * n_eval
        pho_b = lambda n_steps, n_eval: B_PHO * n_steps
        pho_min = lambda n_steps, n_eval: B_PHO_MIN * n_steps + B_CONV_EVAL_MIN * n_eval
        lt, pt = (d["lep_steps_tail"], d["emit_eval_tail"]), (d["pho_steps_tail"], d["conv_eval_tail"])
        units = dict(leptons=(lep_b(d["lep_steps"] - lt[0], d["n_emit_eval"] - lt[1]),) * 2,
                     photons=(pho_b(d["pho_steps"] - pt[0], 0), pho_min(d["pho_steps"] - pt[0], d["n_conv_eval"] - pt[1])),
                     tails=(lep_b(*lt) + pho_b(*pt), lep_b(*lt) + pho_min(*pt)))
        for name, (byt, byt_min) in units.items():
            n, tms = tim[name]
            if name == "photons":
                # the sorted photon pass is two launches: streaming, then the
                # conversion draws of the photons it queued
                tms += tim["conversions"][1]
            per = tms / max(n, 1)
            kern[name] = dict(launches=n, avg_ms=per, bytes_per_launch=byt / max(n, 1),
                              gbs=(byt / max(n, 1)) / (per / 1e3) / 1e9 if tms > 0 else None,
                              min_bytes_per_launch=byt_min / max(n, 1))
        dom = max(("leptons", "photons"), key=lambda k: kern[k]["avg_ms"])
        kname = {"leptons": ("k_leptons",), "photons": ("k_photons", "k_conversions")}[dom]
        tr = [measured_traffic(k) for k in kname]
        roof = dict(bound="hbm", achieved=kern[dom]["gbs"], peak=PEAK_HBM_GBS, unit="GB/s",
                    frac=kern[dom]["gbs"] / PEAK_HBM_GBS, traffic=None if None in tr else sum(tr),
                    kernel="+".join(kname), bytes_per_launch=kern[dom]["bytes_per_launch"],
                    avg_launch_ms=kern[dom]["avg_ms"])
        kern["conversions"] = dict(launches=tim["conversions"][0],
                                   avg_ms=tim["conversions"][1] / max(tim["conversions"][0], 1))
    out = {
        "metric": "particle-steps/s (leptons + photons), % of HBM roofline of the dominant kernel",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms / a.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded initial gap grown by the simulation itself)",
        "config": {"workload": "production gap: 65536 cells, alpha 1.5, b 0.1, R_curv 1e7 cm, surface "
                               "injection 0.1 n_co dx/step, caps 5e7 per species",
                   "n_cells": cfg["n_cells"], "step_at_start": c0["step"], "leptons": c0["n_lep"],
                   "photons": c0["n_pho"], "parallelism": "single GPU", "graph": a.graph,
                   "emit_eval_per_particle_step": round(dA["n_emit_eval"] / max(1, psteps), 4),
                   "conv_eval_per_particle_step": round(dA["n_conv_eval"] / max(1, psteps), 4)},
        "roofline": roof,
        "step_roofline": step_roof,
        "kernels": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kern.items()},
        "timing_ms": {k: round(v[1], 3) for k, v in tim.items()} if tim else None,
        "ms_per_step_with_kernel_events": ms_i / a.steps if ms_i else None,
        "diagnostics": bench_diagnostics(g),
    }
    g.close()
    out["filter"] = bench_filter()
    if not a.no_batched:
        out["batched"] = bench_batched(value)
    if not a.no_adjoint:
        out["adjoint"] = bench_adjoint()
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cfg, c1["step"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
