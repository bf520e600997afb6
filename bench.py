"""Benchmark of the per-step particle loop on one MI355X.

A step is one pass of the whole loop (injection, lepton pass, photon pass,
field, and the periodic re-sort and merge check) over the production gap:
65536 cells, alpha = 1.5, b = 0.1, R_curv = 1e7 cm, surface injection
0.1 n_co dx per step, started from the seeded initial state and grown
(untimed) by the physics itself until the stores hold at least --grow-to
particles.  Then --warmup untimed steps and --steps timed steps; inputs are
resident in HBM throughout.

Prints one JSON line.
 * `ms_per_step` is the timed window's step time with the re-sort and the
   merge check at their average rate: the window's own re-sorts and merge
   checks (a window may hold none) are replaced by the measured cost of one
   re-sort every `resort_every` steps and one merge check every
   `merge_every` steps.  The costs come from a separate run of one whole
   re-sort period with HIP events around each kernel group.  `value` is the
   window's particle-steps (leptons + photons advanced by one step) over
   `steps` x `ms_per_step`; the raw window figures are in `window`.
 * `roofline` is the dominant kernel's algorithmic HBM bytes per launch over
   its average launch time (HIP events on its stream); `step_roofline` is the
   whole step's algorithmic bytes over `ms_per_step`, with `counter_frac`
   from the FETCH_SIZE + WRITE_SIZE bytes of a whole re-sort period when the
   committed counter summary matches the kernel sources.
 * `full_scale`, `batched` and `adjoint` are the other configurations;
   `cpu_baseline` is the FP64 oracle on the GPU's own grown state, on this
   host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# sources of every kernel a step launches (the counter summary is keyed by them)
KERNEL_SOURCES = ("gap_device.hpp", "gap_kernels.hpp", "gap_merge.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step_production.txt")
# algorithmic bytes per unit of work: a lepton-step reads position, momentum
# and weight and writes position and momentum (20 B); a lepton-step that
# evaluates emission also reads the 8-byte id.  A photon-step reads position,
# energy, weight, birth step and id and writes position (28 B).
B_LEP, B_EMIT_EVAL, B_PHO = 20, 8, 28
# bytes the photon kernel must move at least: position, energy and birth step
# read and position written for every photon (16 B); id and weight only for
# the photons that draw a conversion (12 B)
B_PHO_MIN, B_CONV_EVAL_MIN = 16, 12
# the reverse pass of the differentiable window: per lepton-step it reads the
# taped position and momentum of both ends and the three adjoints and writes
# the adjoints back (48 B)
B_ADJ_REV = 48
CPU_WORKERS_MAX = 16        # the host share of one GPU


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def grow(g, target, max_steps, block=1000, tube=0):
    t0 = time.time()
    while True:
        c = g.counts(tube)
        n = c["n_lep"] + c["n_pho"]
        if n >= target or c["step"] >= max_steps:
            log("grown: step %d leptons %d photons %d (%.1f s)" % (c["step"], c["n_lep"], c["n_pho"], time.time() - t0))
            return c
        g.step(block)
        g.sync()


def kernel_source_hash():
    """sha256 over the kernel sources, in a fixed order."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2608_21920_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes from the committed counter summary: per launch of each step
    kernel and per step over a whole re-sort period (FETCH_SIZE + WRITE_SIZE,
    scaled by the copy calibration).  None when the summary was taken with
    other kernel sources."""
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
    out = {k.split(".", 1)[1]: float(v) for k, v in kv.items() if k.startswith("hbm_bytes_per_launch.")}
    if "hbm_bytes_per_step" in kv:
        out["_per_step"] = float(kv["hbm_bytes_per_step"])
    return out


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


def _window(g, torch, steps, timing=False, graph=False, region=None):
    """Run `steps` steps bracketed by synchronisations and events on the
    library's stream: (ms, counter deltas of tube 0, timing record or None,
    counts before)."""
    s = g.stream
    c_a = g.counts()
    g.set_timing(timing)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    if region is not None:
        region.resume()
    e0.record(s)
    if graph:
        g.step_graph(steps)
    else:
        g.step(steps)
    e1.record(s)
    g.sync()
    torch.cuda.synchronize()
    if region is not None:
        region.pause()
    tim = g.timing() if timing else None
    g.set_timing(False)
    c_b = g.counts()
    assert c_b["err"] == 0, c_b
    return e0.elapsed_time(e1), {k: c_b[k] - c_a[k] for k in c_b}, tim, c_a


def _alg_bytes(d):
    return B_LEP * d["lep_steps"] + B_EMIT_EVAL * d["n_emit_eval"] + B_PHO * d["pho_steps"]


def measure_gap(g, torch, cfg, steps, warmup, grow_to, max_grow, graph=False, region=None, kernels=True):
    """The plain step of one grown gap: the timed window (uninstrumented),
    the same number of steps with kernel events, and one whole re-sort period
    with kernel events for the amortised costs of the re-sort and merge
    check."""
    grow(g, grow_to, max_grow)
    g.step(warmup)
    g.sync()
    R = int(g.launch()["resort_every"])
    merge_every = int(cfg.get("merge_every", 64)) if cfg.get("merge") or (cfg.get("flags", 0) & 32) else 0
    ms, d, _, c0 = _window(g, torch, steps, graph=graph, region=region)
    psteps = d["lep_steps"] + d["pho_steps"]
    n_rs = d["rebuckets"]
    n_mg = 0
    if merge_every:
        n_mg = sum(1 for n in range(c0["step"], c0["step"] + steps) if n % merge_every == 0)
    # one whole re-sort period with kernel events: the cost of one re-sort
    # and of the merge checks that fall in it
    ms_p, d_p, tim_p, _ = _window(g, torch, R, timing=True)
    resort_ms = tim_p["resort"][1] / max(tim_p["resort"][0], 1)
    merge_ms = tim_p["merge"][1] / max(tim_p["merge"][0], 1) if tim_p["merge"][0] else 0.0
    body = (ms - n_rs * resort_ms - n_mg * merge_ms) / steps
    amort = resort_ms / R + (merge_ms / merge_every if merge_every else 0.0)
    ms_step = body + amort
    out = dict(ms_per_step=ms_step, value=psteps / (ms_step * steps / 1e3), psteps=psteps, counts_before=c0,
               delta=d, window=dict(ms_per_step=ms / steps, value=psteps / (ms / 1e3), resorts=n_rs, merge_checks=n_mg),
               amortized=dict(resort_ms=resort_ms, resort_every=R, merge_check_ms=merge_ms, merge_every=merge_every,
                              ms_per_step_period_with_events=ms_p / R))
    sb = _alg_bytes(d) / steps
    out["step_roofline"] = dict(bound="hbm", achieved=sb / (ms_step / 1e3) / 1e9, peak=PEAK_HBM_GBS, unit="GB/s",
                                frac=sb / (ms_step / 1e3) / 1e9 / PEAK_HBM_GBS, bytes_per_step=sb)
    if not kernels:
        return out
    # the same number of steps with an event pair around every kernel group
    ms_i, di, tim, _ = _window(g, torch, steps, timing=True)
    lep_b = lambda n_steps, n_eval: B_LEP * n_steps + B_EMIT_EVAL * n_eval
    pho_b = lambda n_steps, n_eval: B_PHO * n_steps
    pho_min = lambda n_steps, n_eval: B_PHO_MIN * n_steps + B_CONV_EVAL_MIN * n_eval
    lt, pt = (di["lep_steps_tail"], di["emit_eval_tail"]), (di["pho_steps_tail"], di["conv_eval_tail"])
    units = dict(leptons=(lep_b(di["lep_steps"] - lt[0], di["n_emit_eval"] - lt[1]),) * 2,
                 photons=(pho_b(di["pho_steps"] - pt[0], 0), pho_min(di["pho_steps"] - pt[0], di["n_conv_eval"] - pt[1])),
                 tails=(lep_b(*lt) + pho_b(*pt), lep_b(*lt) + pho_min(*pt)))
    kern = {}
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
    kern["conversions"] = dict(launches=tim["conversions"][0], avg_ms=tim["conversions"][1] / max(tim["conversions"][0], 1))
    for k in ("field", "prologue"):
        kern[k] = dict(launches=tim[k][0], avg_ms=tim[k][1] / max(tim[k][0], 1))
    out["kernels"] = kern
    out["timing_ms"] = {k: round(v[1], 4) for k, v in tim.items()}
    out["ms_per_step_with_kernel_events"] = ms_i / steps
    return out


def dominant_roofline(res, traffic):
    kern = res["kernels"]
    dom = max(("leptons", "photons"), key=lambda k: kern[k]["avg_ms"])
    kname = {"leptons": ("k_leptons",), "photons": ("k_photons", "k_conversions")}[dom]
    tr = None
    if traffic is not None and all(k in traffic for k in kname):
        tr = sum(traffic[k] for k in kname)
    return dict(bound="hbm", achieved=kern[dom]["gbs"], peak=PEAK_HBM_GBS, unit="GB/s",
                frac=kern[dom]["gbs"] / PEAK_HBM_GBS, traffic=tr, kernel="+".join(kname),
                bytes_per_launch=kern[dom]["bytes_per_launch"], avg_launch_ms=kern[dom]["avg_ms"])


def copy_bandwidth(torch, nbytes=4 << 30, reps=10):
    """Achievable device-copy bandwidth: read + write bytes of a plain copy
    over its time (HIP events)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (ms / 1e3) / 1e9


def export_state(g):
    """The GPU's whole particle state in the oracle's arrays (exact
    conversions), with E_s and the step index."""
    from paper_2608_21920_amd import inputs
    c = g.counts()
    return dict(L=inputs.leptons_as_oracle(g.leptons()), P=inputs.photons_as_oracle(g.photons()), Es=g.es(),
                step=c["step"])


def _oracle_steps(cfg, L, P, Es, step, budget_s, min_steps=1):
    """Step the oracle from a state for about budget_s seconds: (particle-steps,
    seconds, steps, emission and conversion evaluations)."""
    from oracle.oracle import Oracle
    o = Oracle(cfg)
    o.set_state(L, P, Es=Es, step=step)
    c_s = o.counts()
    t0 = time.time()
    ps, done = 0, 0
    while done < min_steps or time.time() - t0 < budget_s:
        c0 = o.counts()
        o.step(1)
        ps += c0["n_lep"] + c0["n_pho"]
        done += 1
    el = time.time() - t0
    c_e = o.counts()
    return ps, el, done, c_e["n_emit_eval"] - c_s["n_emit_eval"], c_e["n_conv_eval"] - c_s["n_conv_eval"]


def _worker(args):
    path, cfg, budget = args
    z = np.load(path)
    L = {k[2:]: z[k] for k in z.files if k.startswith("L_")}
    P = {k[2:]: z[k] for k in z.files if k.startswith("P_")}
    ps, el, done, ev, cv = _oracle_steps(cfg, L, P, float(z["Es"]), int(z["step"]), budget)
    return ps, el, done


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(cfg, state, budget_s=15.0):
    """The FP64 oracle on the GPU's own grown state: one process on the whole
    state (the same particles, field and evaluation mix as the GPU window),
    then one process per core, each on a disjoint random share of the
    particles (aggregate particle-steps/s over the wall time)."""
    import multiprocessing as mp
    L, P = state["L"], state["P"]
    nl, npho = L["id"].size, P["id"].size
    ps, el, done, ev, cv = _oracle_steps(cfg, L, P, state["Es"], state["step"], budget_s)
    one = ps / el
    nproc = os.cpu_count() or 1
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = nproc
    workers = max(1, min(CPU_WORKERS_MAX, affinity))
    rng = np.random.default_rng(11)
    lw, pw = rng.integers(0, workers, nl), rng.integers(0, workers, npho)
    paths = []
    tmp = os.environ.get("TMPDIR", "/tmp")
    for i in range(workers):
        path = os.path.join(tmp, "gap_cpu_share_%d_%d.npz" % (os.getpid(), i))
        np.savez(path, **{"L_" + k: v[lw == i] for k, v in L.items()}, **{"P_" + k: v[pw == i] for k, v in P.items()},
                 Es=state["Es"], step=state["step"])
        paths.append(path)
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_worker, [(p, cfg, budget_s) for p in paths])
    wall = time.time() - t0
    for p in paths:
        os.remove(p)
    allc = sum(r[0] for r in res) / max(r[1] for r in res)
    return dict(value=one, unit="particle-steps/s", cores=1, kind="oracle",
                sample="the GPU's grown production state exported whole (%d leptons, %d photons at step %d): %d "
                       "oracle steps in %.1f s on one core; emission / conversion evaluations per particle-step "
                       "%.4f / %.4f" % (nl, npho, state["step"], done, el, ev / max(ps, 1), cv / max(ps, 1)),
                all_cores=dict(value=allc, cores=workers, wall_s=wall,
                               note="one oracle process per core, each stepping a disjoint random share of the "
                                    "same state for about %.0f s; aggregate particle-steps over the longest "
                                    "process time" % budget_s),
                host=dict(nproc=nproc, affinity=affinity, cpu_model=cpu_model()),
                build="gcc -O2, single-threaded FP64")


def bench_full_scale(torch, steps, warmup, grow_to, max_grow, region=None):
    """The full-scale gap (262144 cells, b = 0.2, caps 2e8), grown by the
    physics to at least grow_to particles, measured like the production gap."""
    from paper_2608_21920_amd import Gap, workloads
    cfg = dict(workloads.FULL)
    g = Gap(cfg)
    res = measure_gap(g, torch, cfg, steps, warmup, grow_to, max_grow, region=region)
    g.close()
    c0 = res["counts_before"]
    return dict(value=res["value"], unit="particle-steps/s", ms_per_step=res["ms_per_step"], steps=steps,
                leptons=c0["n_lep"], photons=c0["n_pho"], step_at_start=c0["step"], window=res["window"],
                amortized=res["amortized"], step_roofline=res["step_roofline"], roofline=dominant_roofline(res, None),
                kernels=res["kernels"],
                emit_eval_per_particle_step=round(res["delta"]["n_emit_eval"] / max(1, res["psteps"]), 4),
                conv_eval_per_particle_step=round(res["delta"]["n_conv_eval"] / max(1, res["psteps"]), 4),
                config="full-scale gap: 262144 cells, alpha 1.5, b 0.2, R_curv 1e7 cm, surface injection 0.1 n_co "
                       "dx/step, caps 2e8 per species with merging; grown by the simulation to %.0e particles" % grow_to)


def _batched_totals(g, n_tubes):
    tot = dict(lep=0, pho=0, emit=0, conv=0, n_lep=0, n_pho=0, n_emit=0, n_conv=0)
    for t in range(n_tubes):
        c = g.counts(t)
        tot["lep"] += c["lep_steps"]
        tot["pho"] += c["pho_steps"]
        tot["emit"] += c["n_emit_eval"]
        tot["conv"] += c["n_conv_eval"]
        tot["n_lep"] += c["n_lep"]
        tot["n_pho"] += c["n_pho"]
        tot["n_emit"] += c["n_emit"]
        tot["n_conv"] += c["n_conv"]
        assert c["err"] == 0, (t, c)
    return tot


def bench_batched(torch, plain_value, cfgs, label, ignite_steps=0, n_tubes=256, launch=None, region=None):
    """An ensemble of uneven tubes in one set of launches, autotuned, timed
    over graph replays of twice the re-sort interval (each replay starts from
    the same store layout, so one captured graph serves them all) and over as
    many eager steps; `value` is the faster of the two.  ignite_steps untimed
    steps run first (QED ignition)."""
    from paper_2608_21920_amd import Gap
    t0 = time.time()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = Gap(cfgs, stream=s)
        g.sync()
        t_init = time.time() - t0
        if ignite_steps:
            g.step(ignite_steps)
            g.sync()
        if launch is None:
            tune = g.autotune(16)
        else:
            g.set_launch(launch["grid_leptons"], launch["grid_photons"], launch["grid_tails"], launch["resort_every"])
            tune = g.launch()
        log("batched (%s): %d tubes built in %.1f s, launch %s" % (label[:40], n_tubes, t_init, tune))
        steps = 2 * tune["resort_every"]
        g.step_graph(steps)          # capture and a first replay
        g.sync()
        c0 = _batched_totals(g, n_tubes)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        g.step_graph(steps)
        g.step_graph(steps)
        e1.record(s)
        g.sync()
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1)
        c1 = _batched_totals(g, n_tubes)
        if region is not None:
            region.resume()
        e0.record(s)
        g.step(2 * steps)
        e1.record(s)
        g.sync()
        torch.cuda.synchronize()
        if region is not None:
            region.pause()
        ms_eager = e0.elapsed_time(e1)
        c2 = _batched_totals(g, n_tubes)
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
                ms_per_step_graph=ms_graph / n, ms_per_step_eager=ms_eager / n, graph=graph, autotune=tune,
                leptons=a["n_lep"], photons=a["n_pho"], ignite_steps=ignite_steps,
                emissions_in_window=b["n_emit"] - a["n_emit"], conversions_in_window=b["n_conv"] - a["n_conv"],
                emit_eval_per_particle_step=round((b["emit"] - a["emit"]) / max(ps, 1), 4),
                conv_eval_per_particle_step=round((b["conv"] - a["conv"]) / max(ps, 1), 4),
                hbm_frac_whole_step=alg / (ms / 1e3) / 1e9 / PEAK_HBM_GBS,
                vs_plain=value / plain_value if plain_value else None, config=label)


def bench_qed_active(torch, plain_value, region=None):
    """The 256 tubes of the batched recipe with the QED rescaled (the
    cascade-heavy ensemble), timed after ignition."""
    from paper_2608_21920_amd import workloads
    return bench_batched(
        torch, plain_value, workloads.batched_qed_active(workloads.batched_tubes(256, seed=1)), ignite_steps=400,
        region=region,
        label="256 tubes: cells uniform in [2048, 16384], alpha uniform in [-1, 2], B/B_Q log-uniform in "
              "[0.01, 0.3], ppc uniform in [4, 64] per species, seed 1; uniform e+- start, QED rescaled "
              "(lambda~ x 3e3, R~ x 3e-3) so that emission, photon transport and conversion run, merge check every "
              "32 steps above 70 % of the cap; "
              "timed after 400 steps, past ignition, with its own autotuned launch shape")


def bench_adjoint(torch, window=2000, ckpt=100):
    """The differentiable window: forward (checkpoints) + reverse pass, and the
    same number of plain steps of the same gap."""
    from paper_2608_21920_amd import Gap, workloads
    from paper_2608_21920_amd import gap as G
    cfg = dict(workloads.ADJOINT, flags=G.INJ_FIXED)
    g = Gap(cfg)
    g.sync()
    c0 = g.counts()
    t0 = time.time()
    loss = g.window_forward(window, ckpt)[0]
    t1 = time.time()
    c1 = g.counts()
    da, dn = g.backward()
    t2 = time.time()
    assert g.counts()["err"] == 0
    g.close()
    p = Gap(cfg)
    p.sync()
    torch.cuda.synchronize()
    t3 = time.time()
    p.step(window)
    p.sync()
    t4 = time.time()
    p.close()
    d = {k: c1[k] - c0[k] for k in c1}
    ps = d["lep_steps"] + d["pho_steps"]
    fwd, bwd, plain = (t1 - t0) * 1e3, (t2 - t1) * 1e3, (t4 - t3) * 1e3
    # bytes: the forward window, its recomputation in the reverse pass (the
    # same algorithmic bytes again) and the reverse step over the leptons
    fwd_b = _alg_bytes(d)
    alg = 2 * fwd_b + B_ADJ_REV * d["lep_steps"]
    return dict(value=ps / ((fwd + bwd) / 1e3), unit="particle-steps/s (window forward + backward)",
                window_steps=window, ckpt_every=ckpt, leptons_start=c0["n_lep"], particle_steps=ps,
                forward_ms=fwd, backward_ms=bwd, plain_ms=plain, fwd_bwd_over_plain=(fwd + bwd) / plain,
                hbm_frac=alg / ((fwd + bwd) / 1e3) / 1e9 / PEAK_HBM_GBS, bytes_fwd_bwd=alg,
                bytes_note="forward window and its recomputation at 20 B + 8 B per evaluation per lepton-step and "
                           "28 B per photon-step each, plus 48 B per lepton-step for the reverse step",
                loss=loss, dL_dalpha=float(da[0]), dL_dninj=float(dn[0]),
                config="16384 cells, 122 e- + 122 e+ per cell, rescaled QED, injection 0.1 n_co dx per step, "
                       "frozen QED, loss = time-averaged <E^2>")


def bench_filter(steps=200):
    """The current filter (8 binomial passes per step) on the production grid:
    the same start state of the production gap stepped with and without it,
    wall time per step and the field update's share."""
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
    one call of each (peak multiplicity, E power spectrum, momentum spectra,
    phase space) and the step time with the E^2 waterfall recorded after
    every step."""
    g.set_profile_bin(64)
    pk = g.peak()
    g.sync()

    def per_call(fn):
        fn()
        g.sync()
        t0 = time.perf_counter()
        for _ in range(calls):
            fn()
        return (time.perf_counter() - t0) * 1e3 / calls

    ms = per_call(g.peak)
    c = g.counts()
    n = c["n_lep"] + c["n_pho"]
    spec_ms = per_call(g.e_spectrum)
    mspec_ms = per_call(g.spectra)
    phase_ms = per_call(g.phase_space)

    def wall(k):
        g.sync()
        t0 = time.perf_counter()
        g.step(k)
        g.sync()
        return (time.perf_counter() - t0) * 1e3 / k

    k = 2 * 136
    plain = wall(k)
    g.set_waterfall(1, 64, 64)
    rec = wall(k)
    ws, we = g.waterfall()
    g.set_waterfall(0)
    return dict(peak_call_ms=ms, particles=n, gbs_at_12_bytes=12.0 * n / (ms / 1e3) / 1e9,
                m_pairs_peak=pk["m_pairs"], h_peak=pk["h"], g3_at_peak=pk["g3"], e_min=pk["e_min"],
                e_max=pk["e_max"], e_spectrum_call_ms=spec_ms, momentum_spectra_call_ms=mspec_ms,
                phase_space_call_ms=phase_ms,
                waterfall=dict(ms_per_step_without=plain, ms_per_step_with=rec, records_read=int(ws.size),
                               bins=int(we.shape[1]), max_e2=float(we.max()) if we.size else None))


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
    ap.add_argument("--no-batched", action="store_true", help="skip the batched ensembles")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the differentiable window")
    ap.add_argument("--no-full", action="store_true", help="skip the full-scale gap")
    ap.add_argument("--only-main", action="store_true", help="the production gap only (profiling runs)")
    ap.add_argument("--only-batched", action="store_true",
                    help="the QED-active ensemble only, its eager timed steps inside the profiler region (profiling runs)")
    ap.add_argument("--only-full", action="store_true",
                    help="the full-scale gap only, its timed steps inside the profiler region (profiling runs)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (--gpus %d refused)" % a.gpus,
              file=sys.stderr)
        sys.exit(2)
    if a.copy_calib:
        copy_calibration(a.copy_calib)
        return
    if a.only_main:
        a.no_cpu = a.no_batched = a.no_adjoint = a.no_full = True
    if a.only_batched:
        import torch
        print(json.dumps({"batched": bench_qed_active(torch, None, region=ProfilerRegion())}))
        return
    if a.only_full:
        import torch
        full = bench_full_scale(torch, a.steps, a.warmup, a.grow_to, a.max_grow_steps, region=ProfilerRegion())
        print(json.dumps({"full_scale": full}))
        return

    import torch
    from paper_2608_21920_amd import Gap, workloads
    cfg = dict(workloads.PRODUCTION)
    # graph capture needs a stream other than the legacy default one
    g = Gap(cfg, stream=torch.cuda.Stream() if a.graph else None)
    region = ProfilerRegion()
    res = measure_gap(g, torch, cfg, a.steps, a.warmup, a.grow_to, a.max_grow_steps, graph=a.graph, region=region,
                      kernels=not a.graph)
    traffic = measured_traffic()
    c0, d = res["counts_before"], res["delta"]
    psteps = res["psteps"]
    step_roof = res["step_roofline"]
    if traffic is not None and "_per_step" in traffic:
        step_roof["counter_bytes_per_step"] = traffic["_per_step"]
        step_roof["counter_frac"] = traffic["_per_step"] / (res["ms_per_step"] / 1e3) / 1e9 / PEAK_HBM_GBS
    else:
        step_roof["counter_bytes_per_step"] = None
        step_roof["counter_frac"] = None
    out = {
        "metric": "particle-steps/s (leptons + photons), % of HBM roofline of the dominant kernel",
        "value": res["value"], "unit": "particle-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": res["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic (seeded initial gap grown by the simulation itself)",
        "config": {"workload": "production gap: 65536 cells, alpha 1.5, b 0.1, R_curv 1e7 cm, surface "
                               "injection 0.1 n_co dx/step, caps 5e7 per species",
                   "n_cells": cfg["n_cells"], "step_at_start": c0["step"], "leptons": c0["n_lep"],
                   "photons": c0["n_pho"], "parallelism": "single GPU", "graph": a.graph,
                   "emit_eval_per_particle_step": round(d["n_emit_eval"] / max(1, psteps), 4),
                   "conv_eval_per_particle_step": round(d["n_conv_eval"] / max(1, psteps), 4)},
        "roofline": dominant_roofline(res, traffic) if "kernels" in res else None,
        "step_roofline": step_roof,
        "window": res["window"],
        "amortized": res["amortized"],
        "kernels": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in res.get("kernels", {}).items()},
        "timing_ms": res.get("timing_ms"),
        "ms_per_step_with_kernel_events": res.get("ms_per_step_with_kernel_events"),
    }
    if not a.only_main:
        out["diagnostics"] = bench_diagnostics(g)
    state = None if a.no_cpu else export_state(g)
    g.close()
    torch.cuda.empty_cache()
    out["copy_gbs"] = copy_bandwidth(torch)
    if out["roofline"] is not None:
        out["roofline"]["achievable_copy_gbs"] = out["copy_gbs"]
    if not a.only_main:
        out["filter"] = bench_filter()
    if not a.no_full:
        out["full_scale"] = bench_full_scale(torch, a.steps, a.warmup, a.grow_to, a.max_grow_steps)
        torch.cuda.empty_cache()
    if not a.no_batched:
        recipe = workloads.batched_tubes(256, seed=1)
        phys = bench_batched(
            torch, res["value"], recipe,
            label="256 tubes of the batched recipe with physical QED (R_curv 1e7 cm): no emission in the timed "
                  "window")
        torch.cuda.empty_cache()
        out["batched"] = bench_qed_active(torch, res["value"])
        out["batched_physical_qed"] = phys
        torch.cuda.empty_cache()
    if not a.no_adjoint:
        out["adjoint"] = bench_adjoint(torch)
    if state is not None:
        out["cpu_baseline"] = cpu_baseline(cfg, state)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
