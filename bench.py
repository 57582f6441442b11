"""Benchmark: ion-pack steps per second on one MI355X.

Workload (the space-charge configuration on the 256 x 1024 grid): ring
electrode fields at 0.05 mm spacing, 1e6 packs injected at 500 per step and
weighted to a 10 nA current, ion m = 5000 Da, z = +5, CCS 1500 A^2, N2 gas at
1e5 -> 200 Pa, collisions on, CIC deposit + Poisson every 10 steps,
dt = 0.5 ns.  A step is one pass of the whole path (emission, RK4 push,
classification, collisions, dissociation, tallies, and the space-charge
update every 10th step).

The run first advances the workload through its emission ramp (steps
0..1999, untimed set-up that does not depend on --warmup), so the population
is the full 1e6 packs; then `warmup` untimed steps; then exactly `steps`
steps timed with the device synchronised on both sides, with no per-kernel
timing events (the kernel times behind the rooflines come from the next
`steps` steps, timed with them).  value = active
pack-steps advanced in the timed window / wall seconds, FP64 path; the FP32
form (FP32 math, BF16 tables, two-float positions) is timed the same way
and reported beside it, and so is the hybrid form (the FP32 form with the
Langevin branch taking the dense first millimetre).

Also reported: the dominant kernel's roofline (HIP events around every
launch of the fused step kernel), the deposit's, windows of the masked
Poisson solve, the snapshots and the adaptive step (`next_rows`), the large
1024 x 8192 configuration, the plain 128 x 512 configuration over its whole
horizon with the oracle timed beside it, serving latency under overload and
at a sustainable load with the oracle's service time on a sample of the
queries, and the CPU oracle's rate on a bounded sample of the same workload
on this host's cores.  On request (--population-sweep), the hybrid form's
step kernel at several populations, fitted as a fixed cost per launch plus a
cost per pack.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "ion-pack steps/s (push+collision+PIC) FP32 vs FP64 GPU; serving p50/p99 latency"
WORKLOAD = ("256x1024 ring-electrode grid (0.05 mm), 1e6 packs injected at 500/step over steps 0-1999 weighted "
            "to 10 nA, m=5000 Da z=+5 CCS 1500 A^2 N2 1e5->200 Pa, CIC+Poisson every 10 steps, dt=0.5 ns; "
            "timed window after the emission ramp and the warmup steps (full 1e6-pack population)")

# Published MI355X vector peaks: FP64 78.6 TFLOP/s, FP32 157.3 TFLOP/s (256
# CUs x 2.4 GHz; an FMA counts as two operations).  The fused step is bound
# by vector-ALU issue; each form is priced against the peak of its own
# arithmetic type.  (Measured issue rates: unpacked FP32, 64-bit integer
# products and three-input XORs issue at the FP64 rate, so the FP32 form's
# ceiling in practice is the FP64 figure; the published FP32 figure counts
# packed instructions, which the build disables.)
PEAK_OPS = {"fp64": 78.6e12, "fp32": 157.3e12}

# Algorithmic operation counts of the fused step kernel: each add, multiply,
# compare/select, integer xor/add/multiply half, conversion and elementary
# function evaluation of the method counts as one operation (a Philox4x32-10
# block is 104).  Per event:
OPS_PACK_STEP = 567       # RK4 with four bilinear field gathers, classification, gas gather and
                          # collision setup, the final wait that ends the step, dissociation
OPS_CANDIDATE = 276       # every candidate inside the step: two Philox blocks, wait, partner draw, test
OPS_ACCEPTED = 161        # accepted candidate: third block, impulsive update, scattering
OPS_EXCHANGE = 18         # internal-energy exchange (taken with probability alpha)

# Algorithmic HBM bytes per active pack-step of the fused step kernel in a
# context that defines one species (every workload timed here): read status,
# id, position, velocity, internal energy and hazard; write back position,
# velocity, internal energy and hazard.  FP64: 76 + 64 B.  FP32 form
# (two-float position and internal energy, FP32 velocity and hazard):
# 60 + 48 B.  With several species each pack also reads its 4-byte tag.  An
# inactive slot costs its status word (4 B).
BYTES_STEP = {"fp64": 140, "fp32": 108}
# A pack on the hybrid Langevin branch neither reads nor writes its internal
# energy and hazard: FP32 form 48 B read (status, id, position, velocity) +
# 36 B written (position, velocity).
BYTES_LANGEVIN = {"fp64": 108, "fp32": 84}
# Deposit: status, position (FP64, or the FP32 form's hi+lo pairs) and the
# int64 charge of every active pack (the LDS-aggregated grid atomics are
# counted as L2 traffic, not HBM), plus one write of the int64 grid.
BYTES_DEPOSIT = {"fp64": 36, "fp32": 36}
GRID_BYTES = 256 * 1024 * 8
HBM_PEAK = 8.0e12

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_step_c2_traffic.txt")
VALU_FILE = os.path.join(ROOT, "profiles", "k_step_c2_valu.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2609_31258_amd", "csrc", f)
                  for f in ("mc_kernels.hpp", "mc_device.hpp", "mc_math64.hpp")]


def _code_only(text: str) -> str:
    """C++ source without its comments and blank lines (string and character
    literals kept), so that the hash below changes with the code only."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            i = text.find("\n", i)
            i = n if i < 0 else i
        elif text.startswith("/*", i):
            i = text.find("*/", i + 2)
            i = n if i < 0 else i + 2
        else:
            out.append(c)
            i += 1
    return "\n".join(line.rstrip() for line in "".join(out).splitlines() if line.strip())


def kernel_source_hash() -> str:
    """sha256[:16] of the step and deposit kernels' code (comments excluded)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(_code_only(open(f, encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def _profile_values(path: str):
    """key: value lines of a committed rocprofv3 summary, or {} when the
    kernels changed after it was taken."""
    if not os.path.exists(path):
        return {}
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv if kv.get("kernel_source_sha256") == kernel_source_hash() else {}


def measured_traffic(precision: str):
    """HBM bytes per step launch from the committed rocprofv3 counter summary,
    or None when the kernels changed after the counters were taken."""
    v = _profile_values(TRAFFIC_FILE).get(f"{precision}_hbm_bytes_per_launch")
    return float(v) if v else None


def measured_issue(form: str):
    """Vector-ALU busy share and lane utilisation of the step kernel from the
    committed rocprofv3 summary (None when stale)."""
    kv = _profile_values(VALU_FILE)
    b, u = kv.get(f"{form}_valu_busy"), kv.get(f"{form}_lane_utilization")
    return {"valu_busy": float(b), "lane_utilization": float(u)} if b and u else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20,
                    help="untimed steps after the 2000-step emission ramp (the ramp always runs)")
    ap.add_argument("--forms", default="fp64,fp32,hybrid",
                    help="comma list of the forms to time: fp64 (plain FP64 path), fp32 (FP32 math, BF16 tables, "
                         "two-float positions), hybrid (FP32 form with the Langevin branch in 0-1 mm)")
    ap.add_argument("--sort-every", type=int, default=100,
                    help="reorder the pack slots by species and cell every N steps (0 = never); the sorts fall "
                         "inside the timed windows")
    ap.add_argument("--large-sort-every", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=300,
                    help="steps of the workload's emission ramp the oracle runs for the CPU baseline")
    ap.add_argument("--serving-queries", type=int, default=256)
    ap.add_argument("--serving-rate", type=float, default=20.0)
    ap.add_argument("--serving-steps", type=int, default=2000)
    ap.add_argument("--serving-budget-gib", type=float, default=64.0)
    ap.add_argument("--sustained-queries", type=int, default=48,
                    help="queries of the serving run at a load the GPU sustains")
    ap.add_argument("--sustained-rate", type=float, default=4.0)
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-next-rows", action="store_true",
                    help="skip the windows of the masked Poisson solve, the snapshots and the adaptive step")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the window of the large configuration (1024x8192 grid, 1.6e7 packs of ten species)")
    ap.add_argument("--large-steps", type=int, default=20)
    ap.add_argument("--large-fill", action="store_true",
                    help="large configuration: run its 1e4-step emission ramp instead of starting from a snapshot")
    ap.add_argument("--no-c1", action="store_true", help="skip the 128x512 full-horizon run and its oracle timing")
    ap.add_argument("--population-sweep", default="",
                    help="comma list of pack counts: time the hybrid form's step kernel at each population "
                         "(HIP events) and fit its per-launch time as intercept + slope x packs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (calibrates HBM byte counters)")
    return ap.parse_args()


def _say(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _fill(sim, n_steps: int, label: str) -> None:
    """Untimed stepping in chunks, one progress line per chunk."""
    t0 = time.time()
    done = 0
    while done < n_steps:
        k = min(500, n_steps - done)
        sim.step(k)
        sim.synchronize()
        done += k
        _say(f"{label} {done}/{n_steps} ({time.time() - t0:.1f} s)")


def _timed(sim, steps: int, events: bool = True):
    """Exactly `steps` steps between two device synchronisations; the
    tallies of the window and, with `events`, its per-kernel HIP-event
    times (the events add a stream marker on both sides of every launch)."""
    import torch
    sim.set_timing(events)
    sim.reset_timing()
    before = sim.read_tallies()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sim.step(steps)
    sim.synchronize()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    after = sim.read_tallies()
    tim = sim.read_timing()
    info = sim.info()
    d = lambda k: after[k] - before[k]
    return dict(wall=t2 - t1, pack_steps=d("pack_steps"), cand=d("n_cand"), coll=d("n_coll"), exch=d("n_exchange"),
                langevin=d("n_langevin"), timing=tim, slots=info["n_slots"], active=int(after["class_n"][0]),
                classes=after["class_n"].tolist(), tallies=after, steps=steps, start_step=info["step"] - steps)


def run_gpu(precision: int, steps: int, warmup: int, langevin: bool = False, sort_every: int = 0):
    """The workload from step 0: its emission ramp (2000 steps, 500 packs per
    step), `warmup` more steps, then the timed window on the full population."""
    from paper_2609_31258_amd import mucite, synth
    f, ions, srcs, op, _ = synth.config_c2()
    op.sort_every = sort_every
    if langevin:  # hybrid form: aggregated relaxation in the dense first millimetre
        op.langevin_on, op.lv_z_lo, op.lv_z_hi, op.lv_switch = 1, 0.0, 1e-3, 0.05
    ramp = srcs[0].n_total // srcs[0].packs_per_step
    name = ("fp64" if precision == 0 else "fp32") + (" hybrid" if langevin else "")
    sim = mucite.Sim(seed=synth.SEED, pack_capacity=srcs[0].n_total, precision=precision, timing=False)
    sim.setup(f, ions, srcs, op)
    _fill(sim, ramp, f"{name} emission ramp")
    if warmup:
        _fill(sim, warmup, f"{name} warmup")
    # the headline window runs without per-kernel events; the kernel times
    # (rooflines) come from the next window of as many steps, with them
    r = _timed(sim, steps, events=False)
    r["ev"] = _timed(sim, steps, events=True)
    r["ramp_steps"] = ramp
    sim.close()
    _say(f"{name}: {r['pack_steps'] / r['wall']:.3e} pack-steps/s, {r['wall'] * 1e3 / steps:.3f} ms/step, "
         f"{r['active']} active")
    return r


def run_population_sweep(populations, steps: int, sort_every: int):
    """The hybrid form's step kernel at several populations of the 256x1024
    workload (its emission ramp cut to each population, then `steps` steps
    with HIP events): per-launch time against packs, fitted as intercept +
    slope x packs.  The slope is the marginal cost of a pack (its bytes over
    it give the bandwidth the kernel sustains once it is full); the intercept
    is what a launch costs beyond that (ramp-up, drain, the events)."""
    import numpy as np
    from paper_2609_31258_amd import mucite, synth
    rows = []
    for n in populations:
        f, ions, srcs, op, _ = synth.config_c2()
        srcs[0].n_total = n
        op.sort_every = sort_every
        op.langevin_on, op.lv_z_lo, op.lv_z_hi, op.lv_switch = 1, 0.0, 1e-3, 0.05
        sim = mucite.Sim(seed=synth.SEED, pack_capacity=n, precision=1, timing=False)
        sim.setup(f, ions, srcs, op)
        _fill(sim, (n + srcs[0].packs_per_step - 1) // srcs[0].packs_per_step + 20, f"sweep {n} ramp")
        r = _timed(sim, steps, events=True)
        sim.close()
        t = r["timing"]
        ms = t["ms"]["step"] / max(t["launches"]["step"], 1)
        rows.append({"packs": n, "active": r["active"], "wavefronts": (n + 63) // 64, "step_ms": ms,
                     "langevin_fraction": r["langevin"] / max(r["pack_steps"], 1)})
        _say(f"sweep: {n} packs, step kernel {ms:.5f} ms")
    out = {"kernel": "k_step (hybrid form)", "steps_per_population": steps, "rows": rows}
    if len(rows) >= 2:
        x = np.array([q["active"] for q in rows], dtype=np.float64)
        y = np.array([q["step_ms"] for q in rows], dtype=np.float64)
        slope, icpt = np.polyfit(x, y, 1)
        out["fit"] = {"slope_ps_per_pack": slope * 1e9, "intercept_us": icpt * 1e3,
                      "marginal_GBps": BYTES_LANGEVIN["fp32"] / (slope * 1e-3) / 1e9 if slope > 0 else None,
                      "bytes_per_pack_step": BYTES_LANGEVIN["fp32"]}
    return out


def hbm_roofline(r, precision: str, kernel: str, traffic_key=None):
    """HBM roofline of a bandwidth-bound kernel from its algorithmic bytes."""
    key = {"step": "step", "deposit": "deposit"}[kernel]
    ms, launches = r["timing"]["ms"][key], max(r["timing"]["launches"][key], 1)
    avg_s = ms / 1e3 / launches
    if kernel == "step":
        idle = max(r["slots"] * r["steps"] - r["pack_steps"], 0)
        lang = r.get("langevin", 0)
        nbytes = ((r["pack_steps"] - lang) * BYTES_STEP[precision] + lang * BYTES_LANGEVIN[precision] +
                  4 * idle) / launches
    else:
        nbytes = r["active"] * BYTES_DEPOSIT[precision] + GRID_BYTES  # population nearly constant in the window
    achieved = nbytes / avg_s if avg_s > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": achieved / HBM_PEAK, "traffic": measured_traffic(traffic_key) if traffic_key else None,
            "kernel": "deposit (k_deposit)" if kernel == "deposit" else "k_step", "avg_launch_ms": avg_s * 1e3,
            "launches": launches, "bytes_per_launch": nbytes,
            "issue": measured_issue(traffic_key) if kernel == "step" and traffic_key else None}


def roofline(r, precision: str, alpha: float):
    """Vector-ALU roofline of the fused step: algorithmic operations per
    launch over the launch's average HIP-event duration, against the
    published vector peak of the form's arithmetic type."""
    ms = r["timing"]["ms"]["step"]
    launches = max(r["timing"]["launches"]["step"], 1)
    avg_s = ms / 1e3 / launches
    ops = (r["pack_steps"] * OPS_PACK_STEP + r["cand"] * OPS_CANDIDATE +
           r["coll"] * OPS_ACCEPTED + r.get("exch", alpha * r["coll"]) * OPS_EXCHANGE)
    ops_per_launch = ops / launches
    achieved = ops_per_launch / avg_s
    peak = PEAK_OPS[precision if precision in PEAK_OPS else "fp32"]
    return {"bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": measured_traffic(precision),
            "kernel": "k_step (fused push/classify/collide)", "avg_launch_ms": avg_s * 1e3, "launches": launches,
            "ops_per_launch": ops_per_launch, "issue": measured_issue(precision)}


def default_alpha() -> float:
    """Internal-exchange probability of the workload's ion (default rule
    4 mg ma / (mg + ma)^2, ma = m / n_atoms)."""
    from paper_2609_31258_amd import synth
    _, ions, _, _, _ = synth.config_c2()
    mg, ma = synth.M_N2_DA, ions[0].mass_da / ions[0].n_atoms
    return 4 * mg * ma / (mg + ma) ** 2


def precision_report(t64, t32, hists=("act_hist_ke", "act_hist_teff")):
    """Error of a run's tallies (t32) against a reference run's (t64) on the
    same packs, seed and steps: relative differences of the weighted mean
    kinetic and internal energies of the active population, total-variation
    distance and Kolmogorov-Smirnov statistic of the histograms named, class
    fractions by count and by weight."""
    import numpy as np
    out = {}
    w64, w32 = t64["class_w"][0], t32["class_w"][0]
    for k in ("sum_w_ke_active", "sum_w_eint_active"):
        a, b = t64[k] / max(w64, 1), t32[k] / max(w32, 1)
        out[k.replace("sum_w_", "rel_err_mean_")] = abs(b - a) / abs(a) if a else None
    ew64, ew32 = max(t64["emitted_w"], 1), max(t32["emitted_w"], 1)
    out["class_weight_fraction_diff"] = [float(a / ew64 - b / ew32) for a, b in zip(t64["class_w"], t32["class_w"])]
    for h in hists:
        p, q = np.asarray(t64[h], float), np.asarray(t32[h], float)
        p, q = p / max(p.sum(), 1), q / max(q.sum(), 1)
        out["tv_" + h] = 0.5 * float(np.abs(p - q).sum())
        out["ks_" + h] = float(np.abs(np.cumsum(p) - np.cumsum(q)).max())
    n64, n32 = max(t64["class_n"].sum(), 1), max(t32["class_n"].sum(), 1)
    out["class_fraction_diff"] = [float(a / n64 - b / n32) for a, b in zip(t64["class_n"], t32["class_n"])]
    out["candidates_rel_diff"] = abs(t32["n_cand"] - t64["n_cand"]) / max(t64["n_cand"], 1)
    return out


def precision_vs_oracle():
    """Each GPU form's error against the FP64 oracle on the same packs, seed
    and steps, in two runs the oracle finishes in seconds: the space-charge
    workload at a twentieth of its pack rate (25 packs per step, weights x20,
    the same 10 nA) over 300 steps (30 space-charge updates; read-time
    histograms of the active population), and the terminal-event variant of
    the low-pressure fields (6000 packs in two bursts, 1200 steps of 5 ns:
    every terminal class, transmitted KE/T_eff/exit-radius histograms)."""
    from oracle.binding import OracleSim
    from paper_2609_31258_amd import mucite, synth
    out = {}
    runs = {"space_charge": (lambda: synth.config_c2(n_packs=7500, packs_per_step=25), 300, None),
            "terminal_events": (lambda: synth.config_c1x(4000, 2000), 1200, (4000, 2000))}
    for name, (cfg, steps, bursts) in runs.items():
        tallies = {}
        for form, prec in (("oracle", None), ("fp64", 0), ("fp32", 1)):
            f, ions, srcs, op, _ = cfg()
            sim = OracleSim(synth.SEED) if prec is None else mucite.Sim(seed=synth.SEED, pack_capacity=7500, precision=prec)
            sim.setup(f, ions, srcs, op)
            for k, nb in enumerate(bursts or ()):
                sim.inject(k, nb)
            sim.step(steps)
            tallies[form] = sim.read_tallies()
            sim.close()
        hists = ("act_hist_ke", "act_hist_teff") + (("hist_ke", "hist_teff", "hist_r", "exit_bins") if bursts else ())
        out[name] = {form: precision_report(tallies["oracle"], tallies[form], hists) for form in ("fp64", "fp32")}
        cls = tallies["oracle"]["class_n"]
        out[name]["classes_oracle"] = cls.tolist()
        # the statistical scale of the FP32 form's differences, whose paths
        # part from the FP64 ones: two-sample KS critical values at alpha =
        # 1e-3 for the active and the transmitted populations
        ks = lambda n: 1.95 * math.sqrt(2.0 / n) if n > 0 else None
        out[name]["ks_critical_active"] = ks(int(cls[0]))
        out[name]["ks_critical_transmitted"] = ks(int(cls[1]))
        _say(f"precision vs oracle, {name}: classes {tallies['oracle']['class_n'].tolist()}")
    return out


def cpu_baseline(n_steps: int):
    """The oracle as it stands, on this host's cores, on a bounded sample of
    the same workload: its first n_steps steps from step 0 (emission at 500
    packs per step, the space-charge update every 10 steps), all of it timed."""
    from oracle.binding import OracleSim, num_threads
    from paper_2609_31258_amd import synth
    f, ions, srcs, op, _ = synth.config_c2()
    o = OracleSim(synth.SEED)
    o.setup(f, ions, srcs, op)
    t0 = time.perf_counter()
    done = 0
    while done < n_steps:
        k = min(50, n_steps - done)
        o.step(k)
        done += k
        _say(f"oracle (cpu baseline) {done}/{n_steps} steps ({time.perf_counter() - t0:.1f} s)")
    wall = time.perf_counter() - t0
    T = o.read_tallies()
    o.close()
    ps = sum(min(n, srcs[0].n_total // srcs[0].packs_per_step) * srcs[0].packs_per_step for n in range(1, n_steps + 1))
    return {"value": ps / wall, "unit": "pack-steps/s", "cores": num_threads(), "kind": "oracle",
            "sample": f"the workload's first {n_steps} steps from step 0 (emission ramp to "
                      f"{n_steps * srcs[0].packs_per_step} packs, {(n_steps + 9) // 10} space-charge updates), "
                      f"{ps:.3e} pack-steps in {wall:.1f} s",
            "collisions_per_s": T["n_coll"] / wall, "wall_s": wall}


def run_c1_full():
    """The plain 128x512 configuration over its whole horizon (1e4 packs,
    2000 steps of 1 ns, collisions on, no space charge) on the GPU (FP64) and
    in the oracle on this host's cores; whole-run wall times."""
    import torch
    from oracle.binding import OracleSim, num_threads
    from paper_2609_31258_amd import mucite, synth
    f, ions, srcs, op, meta = synth.config_c1()
    n, steps = meta["burst"], meta["steps"]
    g = mucite.Sim(seed=synth.SEED, pack_capacity=n, precision=0, timing=True)
    g.setup(f, ions, srcs, op)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.inject(0, n)
    g.step(steps)
    g.synchronize()
    wall_g = time.perf_counter() - t0
    tg = g.read_tallies()
    g.close()
    _say(f"128x512 full run on the GPU: {wall_g:.3f} s")
    o = OracleSim(synth.SEED)
    o.setup(f, ions, srcs, op)
    t0 = time.perf_counter()
    o.inject(0, n)
    for k in range(0, steps, 500):
        o.step(500)
        _say(f"128x512 full run, oracle {k + 500}/{steps} ({time.perf_counter() - t0:.1f} s)")
    wall_o = time.perf_counter() - t0
    to = o.read_tallies()
    o.close()
    ps = n * steps
    return {"workload": "128x512 grid, 1e4 packs of 500 Da z=+1 at step 0, 2000 x 1 ns, collisions on, "
                        "no space charge, FP64",
            "gpu": {"wall_s": wall_g, "value": tg["pack_steps"] / wall_g, "unit": "pack-steps/s",
                    "collisions": int(tg["n_coll"]), "classes": tg["class_n"].tolist()},
            "oracle": {"wall_s": wall_o, "value": ps / wall_o, "unit": "pack-steps/s", "cores": num_threads(),
                       "collisions": int(to["n_coll"]), "classes": to["class_n"].tolist()},
            "speedup": wall_o / wall_g}


def run_large(steps: int, fill: bool, n_packs: int = 16_000_000, sort_every: int = 0):
    """The large configuration in the FP32 form (1024x8192 grid, 1.6e7 packs
    of ten species, space charge every 5 steps): a timed window of `steps`
    steps on the full population, started from a seeded snapshot of the
    post-ramp state (or after the 1e4-step emission ramp with --large-fill);
    and the oracle's rate on a 1e5-pack slice of the same snapshot (push,
    collisions and dissociation; the oracle's direct O(nz^2) sine sums take
    minutes per space-charge update on this grid, so the slice runs without
    them)."""
    from oracle.binding import OracleSim, num_threads
    from paper_2609_31258_amd import mucite, synth
    f, ions, srcs, op, meta = synth.config_c5(n_packs=n_packs)
    op.sort_every = sort_every
    w = synth.config_c5_pack_weights(ions, srcs, op)
    sim = mucite.Sim(seed=synth.SEED, pack_capacity=n_packs, precision=1, timing=True)
    if fill:
        sim.setup(f, ions, srcs, op)
        _fill(sim, meta["emit_steps"], "large emission ramp")
        start = "after its 1e4-step emission ramp"
    else:
        sim.setup(f, ions, [], op)
        snap = synth.c5_post_ramp_snapshot(f, ions, w, n_packs, synth.SEED)
        sim.write_packs(snap)
        del snap
        _fill(sim, 5, "large warmup")
        start = "from a seeded snapshot of the post-ramp state (3 mm x 0.3 mm, ten species)"
    r = _timed(sim, steps)
    sim.close()
    ps = r["pack_steps"]
    alpha = sum(4 * synth.M_N2_DA * (i.mass_da / i.n_atoms) / (synth.M_N2_DA + i.mass_da / i.n_atoms) ** 2
                for i in ions) / len(ions)
    _say(f"large: {ps / r['wall']:.3e} pack-steps/s, {r['wall'] * 1e3 / steps:.3f} ms/step")
    # oracle slice
    n_cpu, cpu_steps = 100_000, 100
    o = OracleSim(synth.SEED)
    op.sc_on = 0
    o.setup(f, ions, [], op)
    o.write_packs(synth.c5_post_ramp_snapshot(f, ions, w, n_cpu, synth.SEED + 3))
    t0 = time.perf_counter()
    o.step(cpu_steps)
    wall_o = time.perf_counter() - t0
    to = o.read_tallies()
    o.close()
    _say(f"large: oracle slice {n_cpu * cpu_steps / wall_o:.3e} pack-steps/s ({wall_o:.1f} s)")
    return {"workload": "1024x8192 grid, 1.6e7 packs of ten species (200-5e4 Da, Arrhenius), 50 nA, "
                        "SC every 5 steps, dt=0.25 ns, FP32 form (BF16 tables); window " + start,
            "steps": steps, "sort_every": sort_every, "value": ps / r["wall"], "unit": "pack-steps/s",
            "ms_per_step": r["wall"] * 1e3 / steps, "active": r["active"], "classes": r["classes"],
            "collisions_per_s": r["coll"] / r["wall"], "candidates_per_pack_step": r["cand"] / max(ps, 1),
            "kernel_ms": r["timing"]["ms"], "roofline": roofline(r, "fp32", alpha),
            "cpu_slice": {"value": n_cpu * cpu_steps / wall_o, "unit": "pack-steps/s", "cores": num_threads(),
                          "kind": "oracle", "sample": f"{n_cpu} packs of the same snapshot, {cpu_steps} steps, "
                                                      f"no space-charge update, {wall_o:.1f} s",
                          "collisions_per_s": to["n_coll"] / wall_o}}


def serving_query(f, q, steps: int):
    """One design query of the serving workload: emission over the first half of
    the horizon at the query's current, space charge every 10 steps."""
    from paper_2609_31258_amd import synth
    ion = synth.Ion(q["mass_da"], q["charge_z"], q["ccs_m2"], max(3, q["n_atoms"]), act_kind=1, act_p1=100e3,
                    act_p2=-80.0)
    pps = max(1, int(round(q["n_packs"] / (steps // 2))))
    src = synth.Source(kind=1, current_a=q["current_a"], packs_per_step=pps, n_total=q["n_packs"], sigma_r=1e-4,
                       r_trunc=3e-4)
    op = synth.Operating(dt=0.5e-9, v_rf=q["v_rf"], f_rf=1e6, v_off=q["v_off"], sc_on=1, sc_every=10,
                         z_det=f.grid.L, r_det=f.grid.R, exit_bin_dt=1e-7, n_exit_bins=100)
    return ion, src, op


def full_occupancy_snapshot(n_packs: int):
    """The workload's full-occupancy state as a pack snapshot: n_packs packs
    within 0.3 mm of the injection plane, thermal about the gas flow, at the
    source's pack weight."""
    from paper_2609_31258_amd import synth
    f, ions, srcs, op, _ = synth.config_c2()
    snap = synth.pack_snapshot(n_packs, f, seed=synth.SEED, z_hi=3e-4, r_hi=3e-4, v_sigma=22.0, v_drift=300.0,
                               e_lo=1.7e-18, e_hi=1.9e-18, weight=srcs[0].current_a * op.dt / (5 * 1.602176634e-19) / 500)
    return f, ions, op, snap


def run_variant(name: str, steps: int, n_packs: int, precision: int = 1, sample_capacity: int = 0, sort_every: int = 0,
                **op_changes):
    """One timed window of a full-population snapshot with some operating
    fields changed (the next rows: masked Poisson, snapshots, adaptive step).
    The first step (and with it the first space-charge update, where the
    capacitance matrix of the masked solve is built) is timed on its own."""
    import torch
    from paper_2609_31258_amd import mucite, synth
    f, ions, op, snap = full_occupancy_snapshot(n_packs)
    op.sort_every = sort_every
    for k, v in op_changes.items():
        setattr(op, k, v)
    sim = mucite.Sim(seed=synth.SEED, pack_capacity=n_packs, precision=precision, timing=True,
                     sample_capacity=sample_capacity)
    sim.setup(f, ions, [], op)
    sim.write_packs(snap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(1)
    sim.synchronize()
    first = time.perf_counter() - t0
    sim.step(9)
    sim.synchronize()
    t_sim0 = sim.info()["time"]
    r = _timed(sim, steps)
    sim_time = sim.info()["time"] - t_sim0
    n_samples = len(sim.read_samples()) if sample_capacity else 0
    sim.close()
    tim = r["timing"]
    wall = r["wall"]
    updates = max(tim["launches"]["poisson"], 1)
    _say(f"{name}: {r['pack_steps'] / wall:.3e} pack-steps/s, {wall * 1e3 / steps:.3f} ms per step")
    return {"value": r["pack_steps"] / wall, "unit": "pack-steps/s", "ms_per_step": wall * 1e3 / steps,
            "steps": steps, "first_step_s": first, "mean_dt_s": sim_time / steps,
            "simulated_s_per_wall_s": sim_time / wall, "space_charge_updates": tim["launches"]["poisson"],
            "update_ms": (tim["ms"]["deposit"] + tim["ms"]["poisson"] + tim["ms"]["field"]) / updates,
            "samples": n_samples, "kernel_ms": tim["ms"]}


def run_next_rows(steps: int, n_packs: int = 1_000_000, sort_every: int = 0):
    """The next rows on a full-population snapshot of the workload, FP32 form:
    a plain window, the masked Poisson solve (potential zero on the ring
    electrodes' mask nodes), full-population snapshots every 20 steps, and
    the adaptive step of Eq. 1 with explicit collisions and on the hybrid
    branch (largest step 2 ns, the Langevin cap)."""
    f, _, _, _ = full_occupancy_snapshot(1)
    g = f.grid
    mask = f.mask.reshape(g.nz, g.nr)
    out = {"state": f"{n_packs} packs, seeded snapshot of the full population (FP32 form, BF16 tables)"}
    out["plain"] = run_variant("plain", steps, n_packs, sort_every=sort_every)
    out["masked_poisson"] = run_variant("masked poisson", steps, n_packs, sc_mask=1, sort_every=sort_every)
    out["masked_poisson"]["mask_nodes"] = int(mask[1:-1, :-1].sum())
    out["snapshots"] = run_variant("snapshots", steps, n_packs, sample_capacity=n_packs * (steps // 20 + 2),
                                   sample_every=20, sample_stride=1, sort_every=sort_every)
    out["adaptive_explicit"] = run_variant("adaptive (explicit collisions)", steps, n_packs, adaptive=1, sort_every=sort_every)
    out["hybrid_fixed"] = run_variant("hybrid, fixed 0.5 ns", steps, n_packs, langevin_on=1, lv_z_lo=0.0,
                                      lv_z_hi=1e-3, lv_switch=0.05, sort_every=sort_every)
    out["adaptive_hybrid"] = run_variant("adaptive hybrid", steps, n_packs, langevin_on=1, lv_z_lo=0.0,
                                         lv_z_hi=1e-3, lv_switch=0.05, adaptive=1, dt=2e-9, lv_dt_max=2e-9,
                                         sort_every=sort_every)
    return out


def run_serving(n_queries: int, rate_hz: float, steps: int, precision: int, budget_gib: float, max_resident: int,
                label: str = "serving"):
    """Poisson arrivals of design queries into one server (shared 256x1024 field
    set, FP32 form); latency = completion - submission on the server clock."""
    from paper_2609_31258_amd import mucite, synth
    f = synth.ring_fields(256, 1024)
    qs = synth.serving_queries(n_queries, rate_hz=rate_hz)
    srv = mucite.Server(f, hbm_budget=int(budget_gib * (1 << 30)), precision=precision, max_resident=max_resident,
                        steps_per_sync=20)
    t0 = time.perf_counter()
    ids = []
    for k, q in enumerate(qs):
        delay = q["arrival_s"] - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        ion, src, op = serving_query(f, q, steps)
        ids.append(srv.submit(ion, src, op, n_steps=steps, seed=q["seed"]))
        if (k + 1) % 16 == 0:
            _say(f"{label} submitted {k + 1}/{n_queries}")
    res = []
    for k, i in enumerate(ids):
        res.append(srv.wait(i, 3600.0))
        if (k + 1) % 16 == 0:
            _say(f"{label} completed {k + 1}/{n_queries} ({time.perf_counter() - t0:.1f} s)")
    st = srv.stats()
    srv.close()
    lat = [r["t_done"] - r["t_submit"] for r in res if r["state"] == mucite.Q_DONE]
    lat.sort()
    pct = lambda p: lat[min(len(lat) - 1, int(math.ceil(p * len(lat))) - 1)] if lat else None
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    ps = sum(r["tallies"]["pack_steps"] for r in res if r["state"] == mucite.Q_DONE)
    # offered load: the work that arrived per second of arrivals, over the
    # rate at which the GPU served it while busy
    service_rate = ps / st["busy_s"] if st["busy_s"] > 0 else None
    arrival_span = qs[-1]["arrival_s"] if len(qs) > 1 else None
    return {"queries": n_queries, "completed": len(lat), "arrival_rate_hz": rate_hz, "steps_per_query": steps,
            "p50_latency_s": pct(0.50), "p99_latency_s": pct(0.99), "mean_latency_s": sum(lat) / len(lat),
            "throughput_pack_steps_per_s": ps / span, "pack_steps": ps, "span_s": span,
            "offered_load": (ps / arrival_span) / service_rate if service_rate and arrival_span else None,
            "max_resident_seen": st["max_resident_seen"], "pool_peak_bytes": st["pool_peak"],
            "dtype": "f32 (BF16 tables)" if precision == 1 else "f64"}


def serving_oracle_sample(n_queries: int, rate_hz: float, steps: int, precision: int, n_sample: int = 8,
                          budget_pack_steps: float = 2e6):
    """The oracle's service time on a seeded sample of the serving queries
    (the first n_sample of the same list): each query runs alone on the GPU
    (one context, the serving form) over its whole horizon, which gives its
    GPU service time and its pack-steps; its packs at the end of emission
    (half the horizon) are handed to the oracle, timed over about
    budget_pack_steps pack-steps at that occupancy on this host's cores, and
    the query's oracle service time is its pack-steps over that rate."""
    import torch
    from paper_2609_31258_amd import mucite, synth
    from oracle.binding import OracleSim, num_threads
    f = synth.ring_fields(256, 1024)
    qs = synth.serving_queries(n_queries, rate_hz=rate_hz)[:n_sample]
    rows = []
    for k, q in enumerate(qs):
        ion, src, op = serving_query(f, q, steps)
        sim = mucite.Sim(seed=q["seed"], pack_capacity=src.n_total, precision=precision)
        sim.setup(f, [ion], [src], op)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps // 2)
        sim.synchronize()
        t_half = time.perf_counter() - t0
        p = sim.read_packs()
        t0 = time.perf_counter()
        sim.step(steps - steps // 2)
        sim.synchronize()
        gpu_s = t_half + time.perf_counter() - t0
        ps = int(sim.read_tallies()["pack_steps"])
        sim.close()
        act = p["status"] == 0
        snap = {key: p[key][act] for key in ("x", "y", "z", "vx", "vy", "vz", "e_int", "h", "w", "id", "tag")}
        n_act = int(act.sum())
        o = OracleSim(q["seed"])
        o.setup(f, [ion], [], op)  # the packs as they stand; the source has finished emitting
        o.write_packs(snap)
        o_steps = max(1, int(budget_pack_steps // max(n_act, 1)))
        t0 = time.perf_counter()
        o.step(o_steps)
        wall_o = time.perf_counter() - t0
        o.close()
        rate_o = n_act * o_steps / wall_o
        rows.append({"n_packs": q["n_packs"], "mass_da": q["mass_da"], "charge_z": q["charge_z"], "pack_steps": ps,
                     "gpu_service_s": gpu_s, "oracle_rate": rate_o, "oracle_service_s": ps / rate_o,
                     "oracle_timed_steps": o_steps, "oracle_timed_packs": n_act})
        _say(f"serving oracle sample {k + 1}/{n_sample}: {q['n_packs']} packs, GPU {gpu_s:.2f} s, "
             f"oracle {ps / rate_o:.1f} s (extrapolated from {o_steps} steps)")
    tot_g = sum(r["gpu_service_s"] for r in rows)
    tot_o = sum(r["oracle_service_s"] for r in rows)
    return {"queries": rows, "gpu_service_s_total": tot_g, "oracle_service_s_total": tot_o,
            "speedup": tot_o / tot_g if tot_g > 0 else None, "cores": num_threads(), "kind": "oracle",
            "sample": f"the first {n_sample} queries of the serving list, each alone; oracle timed on about "
                      f"{budget_pack_steps:.0e} pack-steps from its end-of-emission state"}


def copy_calibration():
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    _say(f"copy calibration: {n} bytes read, {n} bytes written")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "bench.py runs on one GPU: --gpus above 1 is not supported (no multi-GPU path)"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench needs a GPU"
    if args.copy_calibration:
        copy_calibration()
    res = {}
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    if not forms or any(f not in ("fp64", "fp32", "hybrid") for f in forms):
        print(json.dumps({"error": f"unknown form list {args.forms!r}"}))
        sys.exit(2)
    if "fp64" in forms:
        res["fp64"] = run_gpu(0, args.steps, args.warmup, sort_every=args.sort_every)
    if "fp32" in forms:
        res["fp32"] = run_gpu(1, args.steps, args.warmup, sort_every=args.sort_every)
    if "hybrid" in forms:
        res["hybrid"] = run_gpu(1, args.steps, args.warmup, langevin=True, sort_every=args.sort_every)
    main_key = "fp64" if "fp64" in res else ("fp32" if "fp32" in res else "hybrid")
    r = res[main_key]
    value = r["pack_steps"] / r["wall"]
    out = {
        "metric": METRIC, "value": value, "unit": "pack-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["wall"] * 1e3 / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64" if main_key == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "grid": [256, 1024], "packs": r["slots"], "active": r["active"],
                   "ramp_steps": r["ramp_steps"], "first_timed_step": r["start_step"], "sc_every": 10,
                   "sort_every": args.sort_every,
                   "dt_s": 0.5e-9, "precision": main_key},
        "roofline": hbm_roofline(r["ev"], "fp32", "step", "hybrid") if main_key == "hybrid"
        else roofline(r["ev"], main_key, default_alpha()),
        "collisions_per_s": r["coll"] / r["wall"],
        "candidates_per_pack_step": r["cand"] / max(r["pack_steps"], 1),
        "kernel_ms": r["ev"]["timing"]["ms"],
        "ms_per_step_with_kernel_events": r["ev"]["wall"] * 1e3 / args.steps,
    }
    if main_key != "hybrid":
        out["deposit_roofline"] = hbm_roofline(r["ev"], main_key, "deposit", "deposit_" + main_key)
    if "fp32" in res and main_key == "fp64":
        q = res["fp32"]
        out["fp32_form"] = {"value": q["pack_steps"] / q["wall"], "unit": "pack-steps/s",
                            "ms_per_step": q["wall"] * 1e3 / args.steps, "dtype": "f32 (BF16 tables)",
                            "active": q["active"], "speedup_vs_fp64": (q["pack_steps"] / q["wall"]) / value,
                            "roofline": roofline(q["ev"], "fp32", default_alpha()), "collisions_per_s": q["coll"] / q["wall"],
                            "deposit_roofline": hbm_roofline(q["ev"], "fp32", "deposit", "deposit_fp32"),
                            "kernel_ms": q["ev"]["timing"]["ms"],
                            "ms_per_step_with_kernel_events": q["ev"]["wall"] * 1e3 / args.steps,
                            "error_vs_fp64": precision_report(r["tallies"], q["tallies"])}
    if "hybrid" in res and main_key != "hybrid":
        h = res["hybrid"]
        ref = res.get("fp32")
        out["hybrid_form"] = {"value": h["pack_steps"] / h["wall"], "unit": "pack-steps/s",
                              "ms_per_step": h["wall"] * 1e3 / args.steps, "dtype": "f32 (BF16 tables)",
                              "active": h["active"], "langevin_fraction": h["langevin"] / max(h["pack_steps"], 1),
                              "speedup_vs_explicit_fp32": (h["pack_steps"] / h["wall"]) / (ref["pack_steps"] / ref["wall"])
                              if ref else None,
                              "roofline": hbm_roofline(h["ev"], "fp32", "step", "hybrid"),
                              "kernel_ms": h["ev"]["timing"]["ms"],
                              "ms_per_step_with_kernel_events": h["ev"]["wall"] * 1e3 / args.steps}
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(args.cpu_steps)
    if not args.no_cpu_baseline:
        out["error_vs_oracle"] = precision_vs_oracle()
    if not args.no_c1:
        out["c1_full"] = run_c1_full()
    if not args.no_large:
        out["large"] = run_large(args.large_steps, args.large_fill, sort_every=args.large_sort_every)
    if not args.no_next_rows:
        out["next_rows"] = run_next_rows(args.steps, sort_every=args.sort_every)
    if args.population_sweep:
        pops = [int(v) for v in args.population_sweep.split(",") if v.strip()]
        out["hybrid_population_sweep"] = run_population_sweep(pops, args.steps, args.sort_every)
    if not args.no_serving:
        out["serving"] = run_serving(args.serving_queries, args.serving_rate, args.serving_steps, 1,
                                     args.serving_budget_gib, 64)
        out["serving_sustained"] = run_serving(args.sustained_queries, args.sustained_rate, args.serving_steps, 1,
                                               args.serving_budget_gib, 64, label="serving (sustained)")
        if not args.no_cpu_baseline:
            out["serving"]["oracle_sample"] = serving_oracle_sample(args.serving_queries, args.serving_rate,
                                                                    args.serving_steps, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
