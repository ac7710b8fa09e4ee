"""Benchmark: all-pairs Coulomb velocity-Verlet step at N = 100000 on one MI355X.

One step = one md step of the whole hot path on the N = 100000 workload
(cloud100k: Gaussian cloud, 1% of ions at +2e, static pseudo-potential trap,
dt = 1 ns): the force stage (by default each unordered pair once, applied to
both ions), then the fixed-order finish fused with the trap, the
velocity-Verlet kick and the next drift.  ``value`` is pair interactions per
second, N^2 per step (the paper's loop count).

Prints one JSON line with the contract fields plus ``roofline`` (the force
stage against the FP64 vector peak at the method's own FLOP count: 27 per
unordered pair on the default Newton's-third-law stage, 20 per ordered pair on
the direct kernel), ``cpu_baseline`` (the oracle's plain double loop timed on
this host on a bounded sample), ``mixed`` (the FP32-seeded one-Newton-step
path: speed and its force error), ``mixed_f32d_ablation`` (FP32 displacements:
speed and error) and ``after_200_steps`` (the workload's 200-step run and the
force errors at its final positions).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n N] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic FLOPs, counted on the paper's section 3 double loop with each +, -, *, /, sqrt
# counted once and the softening add included:
#  - 20 per ordered pair evaluated on its own (3 sub, r^2 + eps2 in 6, sqrt, divide, cube in 2,
#    times q_j, 3 mul + 3 add into the sums);
#  - 27 per unordered pair evaluated once for both ions by Newton's third law (the 20, plus the
#    other ion's charge multiply and its 3 mul + 3 add).
# A force evaluation of N ions is 20 N (N - 1) FLOPs on the direct kernel and 27 N (N - 1) / 2
# on the Newton's-third-law stage: the work the kernel performs, not a dense-equivalent count.
FLOPS_PER_PAIR = 20
FLOPS_PER_SYM_PAIR = 27
SYM_ALGOS = (1, 2, 4)


# Hessian-vector products, counted the same way, per ordered pair and B vectors: geometry and
# scales 16 (d 3, r^2 + eps2 6, sqrt and divide 2, y^3 2, times q_j 1, 3 y^5 from y^3 and y^2 2),
# and per vector 21 (u = v_i - v_j 3, d.u 5, its scale 1, 3 d c - u y^3 components 9,
# accumulation 3).  Per unordered pair applied to both ions: 15 + 30 B (no q_j multiply in the
# shared scales; per vector the 21 minus the one accumulation, plus 3 mul + 3 add into each ion).
def hvp_eval_flops(n: int, nvec: int, sym: bool) -> float:
    if sym:
        return (15 + 30 * nvec) * n * (n - 1) / 2.0
    return (16 + 21 * nvec) * float(n) * (n - 1)


def force_eval_flops(n: int, algo: int) -> float:
    """Algorithmic FLOPs of one force evaluation of n ions on the given path."""
    if algo in SYM_ALGOS:
        return FLOPS_PER_SYM_PAIR * n * (n - 1) / 2.0
    return FLOPS_PER_PAIR * float(n) * (n - 1)
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# sources of the default force stage (the counter summary is valid only for these as committed)
KERNEL_SOURCES = ("paper_2106_11143_amd/csrc/pair_sym.hpp", "paper_2106_11143_amd/csrc/pair_sym.hip",
                  "paper_2106_11143_amd/csrc/wave_reduce.hpp", "paper_2106_11143_amd/csrc/rsqrt.hpp",
                  "paper_2106_11143_amd/csrc/step_common.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_stage_fp64_cloud100k_traffic.json")
STAGE_KERNELS = {
    0: "cb::k_pair<FP64> (all-pairs force, j-split partials)",
    1: "force stage cb::k_sym_plan + cb::k_pair_sym<FP64> + cb::k_sym_finish<FP64> (each unordered pair "
       "evaluated once and applied to both ions, reactions summed by cross-lane permutes; tile partials summed "
       "in fixed order)",
    2: "force stage cb::k_sym_plan + cb::k_pair_sym<FP64> + cb::k_sym_finish<FP64> (each unordered pair "
       "evaluated once and applied to both ions, reactions summed through LDS; tile partials summed in fixed "
       "order)",
    4: "force stage cb::k_sym_plan + cb::k_pair_sym_rows<FP64> + cb::k_sym_finish<FP64> (each unordered pair "
       "evaluated once and applied to both ions; four i-blocks per workgroup share each j-segment and add their "
       "reactions in LDS before one store; tile partials summed in fixed order)",
}


def kernel_hash() -> str:
    """Hash of the force stage's source code, comments and whitespace removed
    (a comment edit leaves the committed counter summary valid)."""
    import re

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        src = re.sub(r"//[^\n]*", "", src)
        h.update(re.sub(r"\s+", " ", src).strip().encode())
    return h.hexdigest()[:16]


def stage_counters(cfg):
    """The committed rocprofv3 counter summary of one FP64 force evaluation
    (all kernels of the stage): HBM bytes and executed FP64 FLOPs, or None if
    absent, taken on other code or on another launch configuration."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    if t.get("config") != {k: cfg[k] for k in ("algo", "p", "wg", "splits")}:
        return None
    return t


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=100000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this size (rocprofv3 counter calibration)")
    ap.add_argument("--workload", default="cloud100k",
                    choices=["cloud100k", "cloud1024", "rf32768", "kz512", "crystal8192", "hvp8192", "rsqrt_sweep",
                             "recording", "uniform_tiles"],
                    help="cloud100k is the headline; the others time the remaining workloads")
    ap.add_argument("--no-extras", action="store_true",
                    help="cloud100k: only the timed legs (steps, force stage, mixed), no error or 200-step legs "
                         "(for profiler runs)")
    ap.add_argument("--stage-only", action="store_true",
                    help="cloud100k: only FP64 force-stage evaluations of the headline input (--steps of them, "
                         "after the clock warm-up), for counter runs that must see one kernel configuration only")
    ap.add_argument("--ungrouped", action="store_true",
                    help="time cloud100k in its seeded ion order (species interleaved) instead of grouped by "
                         "species")
    ap.add_argument("--algo", type=int, choices=[1, 2, 4], default=None,
                    help="force one Newton's-third-law variant for cloud100k (1: reactions by permutes, 2: through "
                         "LDS, one wave per tile; 4: four i-blocks per workgroup sharing each j-segment) at the "
                         "default tile shape")
    ap.add_argument("--direct", action="store_true",
                    help="force the direct kernel (every ordered pair, j-split partials) instead of the "
                         "default Newton's-third-law stage, at the direct kernel's default launch")
    args = ap.parse_args()
    if args.workload != "cloud100k":
        if args.gpus != 1:
            print("bench.py runs on one GPU only", file=sys.stderr)
            sys.exit(2)
        print(json.dumps(OTHER_WORKLOADS[args.workload](args)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding is "
              "not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2106_11143_amd import api, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    d_seeded = inputs.cloud100k(n=args.n)
    # the same ions relabelled so that each species is contiguous (the paper's split
    # of species into separate N-body sub-problems); --ungrouped keeps the seeded order
    d = d_seeded if args.ungrouped else inputs.group_by_charge(d_seeded)
    n = d["n"]
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    q, m = dev(d["q"]), dev(d["m"])
    trap, dt = d["trap"], d["dt"]
    if args.algo is not None:
        for op in ("md_run", "forces", "energy"):
            for prec in ("fp64", "mixed"):
                c = api.get_config(op, n, prec)
                api.set_config(op, n, prec, p=c["p"] if c["algo"] in (1, 2, 4) else 8, wg=4,
                               splits=c["splits"] if c["algo"] in (1, 2, 4) else 512, algo=args.algo)
    if args.direct:
        waves = -(-n // 64)
        splits = max(1, min(64, -(-65536 // waves), max(1, n // 64)))
        for op in ("md_run", "forces"):
            for prec in ("fp64", "mixed"):
                api.set_config(op, n, prec, p=1, wg=64, splits=splits, algo=0)

    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    def fresh_state():
        st = inputs.state9(d)
        return [dev(st[k]) for k in range(9)]

    def time_steps(prec, K, W):
        st = fresh_state()
        api.md_run(st, q, m, trap, 0.0, dt, 0, prec=prec, init_accel=True)  # a_0
        if W:
            api.md_run(st, q, m, trap, 0.0, dt, W, prec=prec, init_accel=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        api.md_run(st, q, m, trap, W * dt, dt, K, prec=prec, init_accel=False)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), st

    def time_pair_kernel(prec, reps, dd=None):
        dd = d if dd is None else dd
        x, y, z, q = (dev(dd[k]) for k in ("x", "y", "z", "q"))
        api.coulomb_pair_stage(x, y, z, q, prec=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            api.coulomb_pair_stage(x, y, z, q, prec=prec)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    # the engine clock ramps over the first few hundred ms of FP64 load: settle it
    # with force evaluations before anything is timed (not part of any timed region)
    prewarm(torch, lambda: time_pair_kernel("fp64", 1), 0.5)
    if args.stage_only:
        print(json.dumps({"kernel_ms": time_pair_kernel("fp64", args.steps), "evaluations": args.steps,
                          "config": api.get_config("forces", n, "fp64"),
                          "note": "profiling run (--stage-only): not a bench line"}), flush=True)
        return
    ms_fp64, st64 = time_steps("fp64", args.steps, args.warmup)
    ms_mixed, _ = time_steps("mixed", args.steps, args.warmup)
    reps = max(10, args.steps // 2)
    kt64 = time_pair_kernel("fp64", reps)
    kt_mixed = time_pair_kernel("mixed", reps)
    other = d_seeded if not args.ungrouped else inputs.group_by_charge(d_seeded)
    kt_other = time_pair_kernel("fp64", reps, other)
    if args.no_extras:
        print(json.dumps({"ms_per_step": ms_fp64 / args.steps, "kernel_ms": kt64, "mixed_ms_per_step":
                          ms_mixed / args.steps, "mixed_kernel_ms": kt_mixed, "other_order_kernel_ms": kt_other,
                          "note": "profiling run (--no-extras): not a bench line"}), flush=True)
        return
    cfg = api.get_config("md_run", n, "fp64")
    pairs_step = float(n) * float(n)
    ms_per_step = ms_fp64 / args.steps
    value = pairs_step * args.steps / (ms_fp64 * 1e-3)
    flops_eval = force_eval_flops(n, cfg["algo"])
    achieved = flops_eval / (kt64 * 1e-3) / 1e12
    counters = stage_counters(cfg)
    traffic = counters.get("bytes_per_launch") if counters else None
    executed = counters.get("executed_fp64_flops_per_launch") if counters else None

    # one GPU's share of an 8-way split by ion index: forces on N/8 ions from all N
    xs, ys, zs = (dev(d[k]) for k in ("x", "y", "z"))
    i0, i1 = 3 * n // 8, 4 * n // 8
    api.coulomb_forces_range(xs, ys, zs, q, i0, i1)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        api.coulomb_forces_range(xs, ys, zs, q, i0, i1)
    e1.record()
    torch.cuda.synchronize()
    ms_share = e0.elapsed_time(e1) / reps
    share = {"i_range": [i0, i1], "ms": ms_share, "pairs_per_s": float(i1 - i0) * n / (ms_share * 1e-3),
             "note": "coulomb_forces_range (direct kernel, every ordered pair of the range) on one GPU; the "
                     "position all-gather of a multi-GPU run is not included"}

    # force error of the mixed path against the FP64 path, all ions
    x, y, z = (dev(d[k]) for k in ("x", "y", "z"))
    F64 = torch.stack(api.coulomb_forces(x, y, z, q, prec="fp64")).cpu().numpy()
    Fmx = torch.stack(api.coulomb_forces(x, y, z, q, prec="mixed")).cpu().numpy()
    emx = np.linalg.norm(Fmx - F64, axis=0) / np.linalg.norm(F64, axis=0)

    # the literal FP32-displacement reading of the mixed path (ablation, direct kernel): time and error
    api.coulomb_forces(x, y, z, q, prec="mixed_f32d")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(3):
        Ff = api.coulomb_forces(x, y, z, q, prec="mixed_f32d")
    e1.record()
    torch.cuda.synchronize()
    ms_f32d = e0.elapsed_time(e1) / 3
    Ff = torch.stack(Ff).cpu().numpy()
    ef = np.linalg.norm(Ff - F64, axis=0) / np.linalg.norm(F64, axis=0)

    # the workload's 200-step run (FP64 and mixed), then the forces at the final
    # FP64 positions on both paths: the mixed path's force error after the run
    nlong = d["nsteps"]
    st_long = {}
    for prec in ("fp64", "mixed"):
        st = fresh_state()
        api.md_run(st, q, m, trap, 0.0, dt, nlong, prec=prec, init_accel=True)
        st_long[prec] = st
    xl, yl, zl = st_long["fp64"][:3]
    F64l = torch.stack(api.coulomb_forces(xl, yl, zl, q, prec="fp64")).cpu().numpy()
    Fmxl = torch.stack(api.coulomb_forces(xl, yl, zl, q, prec="mixed")).cpu().numpy()
    emxl = np.linalg.norm(Fmxl - F64l, axis=0) / np.linalg.norm(F64l, axis=0)
    r64 = torch.stack(st_long["fp64"][:3]).cpu().numpy()
    rmx = torch.stack(st_long["mixed"][:3]).cpu().numpy()
    after = {"steps": nlong, "positions": "final positions of the FP64 run",
             "mixed_vs_fp64": {"max_rel": float(emxl.max()), "rms_rel": float(np.sqrt(np.mean(emxl ** 2))),
                               "ions": n},
             "mixed_vs_fp64_trajectory_max_abs_m": float(np.abs(rmx - r64).max()),
             "position_scale_m": float(np.abs(r64).max())}

    out = {
        "metric": "pair interactions/s (FP64, N=100000, one velocity-Verlet step per step)",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded Gaussian ion cloud, inputs.cloud100k)",
        "config": {
            "workload": f"cloud100k: N={n} ions, Gaussian sigma=(150,150,800) um, 1% at +2e, static trap "
                        "2pi(1,1,0.2) MHz, dt=1 ns, FP64 all-pairs Coulomb + velocity-Verlet; ions "
                        + ("in the seeded order (species interleaved)" if args.ungrouped else
                           "grouped by species (the seeded ions relabelled, the +2e ions last)"),
            "n": n, "launch": cfg,
            "flops_per_unordered_pair": FLOPS_PER_SYM_PAIR if cfg["algo"] in SYM_ALGOS else None,
            "flops_per_ordered_pair": FLOPS_PER_PAIR if cfg["algo"] not in SYM_ALGOS else None,
        },
        "roofline": {
            "bound": "alu",
            "kernel": STAGE_KERNELS.get(cfg["algo"], "?"),
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "frac_fp32_peak": achieved / PEAK_FP32_TFLOPS,
            "traffic": traffic,
            "kernel_ms": kt64,
            "algorithmic_flops_per_launch": flops_eval,
            "flop_convention": ("the method's own work: 27 FLOP per unordered pair x N(N-1)/2 pairs (each pair "
                                "evaluated once and applied to both ions)" if cfg["algo"] in SYM_ALGOS else
                                "the method's own work: 20 FLOP per ordered pair x N(N-1) pairs"),
            "dense_equivalent_tflops": FLOPS_PER_PAIR * pairs_step / (kt64 * 1e-3) / 1e12,
            "dense_equivalent_note": "20 FLOP x N^2 ordered pairs per evaluation whatever the kernel does; "
                                     "a throughput figure, not a fraction of peak",
            "executed_fp64_tflops": executed / (kt64 * 1e-3) / 1e12 if executed else None,
        },
        "other_ion_order": {
            "order": "grouped by species" if args.ungrouped else "seeded order (species interleaved)",
            "kernel_ms": kt_other,
            "frac": force_eval_flops(n, cfg["algo"]) / (kt_other * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
            "note": "the same system relabelled; tiles of one charge per side take the charge-free pair loop",
        },
        "one_gpu_share_of_8": share,
        "mixed": {
            "pairs_per_s": pairs_step * args.steps / (ms_mixed * 1e-3),
            "ms_per_step": ms_mixed / args.steps,
            "kernel_ms": kt_mixed,
            "kernel_tflops": flops_eval / (kt_mixed * 1e-3) / 1e12,
            "speedup_vs_fp64_step": ms_fp64 / ms_mixed,
            "speedup_vs_fp64_kernel": kt64 / kt_mixed,
            "max_rel_force_err_vs_fp64": float(emx.max()),
            "rms_rel_force_err_vs_fp64": float(np.sqrt(np.mean(emx ** 2))),
        },
        "mixed_f32d_ablation": {
            "what": "mixed refinement on displacements rounded to FP32 (in r^2 and in the numerator); "
                    "direct kernel, forces only",
            "kernel_ms": ms_f32d, "speedup_vs_fp64_kernel": kt64 / ms_f32d,
            "max_rel_force_err_vs_fp64": float(ef.max()),
            "rms_rel_force_err_vs_fp64": float(np.sqrt(np.mean(ef ** 2))),
        },
        "after_200_steps": after,
    }
    if not args.no_cpu:
        out["cpu_baseline"], out["oracle_error"] = cpu_leg(d, F64, Fmx, args.cpu_seconds, Ff)
        # the force error after the 200-step run, against the oracle at the same positions
        _, err_l = cpu_leg(dict(d, x=r64[0], y=r64[1], z=r64[2]), F64l, Fmxl, 0.0, None, time_it=False)
        after["oracle_error"] = err_l
    print(json.dumps(out), flush=True)


def prewarm(torch, fn, seconds):
    """Runs fn until `seconds` of wall time have passed (GPU clock settling)."""
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        fn()
    torch.cuda.synchronize()


def cpu_leg(d, F64, Fmx, seconds, Ff32d=None, time_it=True):
    """The oracle on this host: its plain double loop timed on a bounded sample
    of rows (all j for ions 0..k-1), and the GPU force errors against its
    compensated forces on a sample of ions."""
    import numpy as np

    from oracle import oracle as O

    n = d["n"]
    args = (d["x"], d["y"], d["z"], d["q"])
    base = None
    if time_it:
        base = _time_plain(O, n, args, seconds)
    g = np.random.Generator(np.random.PCG64(5))
    idx = np.sort(g.choice(n, min(n, 1000), replace=False))
    ref = np.stack(O.forces(*args, idx=idx))
    err = {}
    for name, F in (("fp64", F64), ("mixed", Fmx), ("mixed_f32d", Ff32d)):
        if F is None:
            continue
        e = np.linalg.norm(F[:, idx] - ref, axis=0) / np.linalg.norm(ref, axis=0)
        err[name] = {"max_rel": float(e.max()), "rms_rel": float(np.sqrt(np.mean(e ** 2))), "ions": len(idx)}
    return base, err


def _time_plain(O, n, args, seconds):
    """The plain double loop timed on a bounded sample of rows."""
    t0 = time.perf_counter()
    k0 = min(n, 2000)
    O.forces_plain_range(*args, 0, k0)
    t_cal = time.perf_counter() - t0
    k = int(min(n, max(k0, k0 * seconds / max(t_cal, 1e-6))))
    reps = max(1, int(seconds / max(t_cal * k / k0, 1e-6)))
    t0 = time.perf_counter()
    used = 0
    for _ in range(reps):
        _, _, _, used = O.forces_plain_range(*args, 0, k)
    t = time.perf_counter() - t0
    pairs = float(reps) * k * (n - 1)
    return {"value": pairs / t, "unit": "pairs/s", "cores": int(used), "kind": "oracle",
            "sample": f"plain FP64 double loop (SQRT+DIV), rows 0..{k - 1} x all {n} ions, {reps} pass(es), "
                      f"{t:.1f} s"}


# ----------------------------------------------------------------------------
# The other workloads (not the headline line): same JSON contract fields.
def _setup():
    import numpy as np
    import torch

    from paper_2106_11143_amd import api, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a), device="cuda")
    return np, torch, api, inputs, dev


def _timer(torch):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    return e0, e1


def _line(metric, value, unit, steps, warmup, ms_per_step, workload, extra, higher=True):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps, "warmup": warmup,
           "ms_per_step": ms_per_step, "higher_is_better": higher, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic (seeded, paper_2106_11143_amd.inputs)",
           "config": {"workload": workload}}
    out.update(extra)
    return out


def _roof(flops, seconds, what, convention):
    """Roofline object for a secondary workload: the whole timed region's
    algorithmic FLOP rate (the method's own work, as `convention` states)
    against the FP64 vector peak; a lower bound on the dominant kernel's own
    rate, since it includes the other kernels and the launch gaps."""
    achieved = flops / seconds / 1e12
    return {"bound": "alu", "kernel": what, "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None, "flop_convention": convention}


def _force_convention(algo):
    return ("27 FLOP per unordered pair x n(n-1)/2 per force evaluation (Newton's third law)" if algo in SYM_ALGOS
            else "20 FLOP per ordered pair x n(n-1) per force evaluation")


def bench_md_single(args, which):
    """cloud1024 (100 steps, energies every step) or rf32768 (explicit RF,
    energies every 50 steps): time of whole runs, pairs/s = N^2 per step."""
    np, torch, api, inputs, dev = _setup()
    d = inputs.cloud1024() if which == "cloud1024" else inputs.rf32768()
    n, nsteps = d["n"], d["nsteps"]
    every = 1 if which == "cloud1024" else 50
    q, m = dev(d["q"]), dev(d["m"])
    st0 = inputs.state9(d)
    reps = max(1, args.steps if which == "cloud1024" else 1)

    def one():
        ts = [dev(st0[k]) for k in range(9)]
        return api.md_run(ts, q, m, d["trap"], 0.0, d["dt"], nsteps, every=every), ts

    for _ in range(max(1, args.warmup if which == "cloud1024" else 1)):
        one()
    torch.cuda.synchronize()
    e0, e1 = _timer(torch)
    e0.record()
    for _ in range(reps):
        en, ts = one()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    E = en[0, :, 3].cpu().numpy()
    cfg = api.get_config("md_run", n, "fp64")
    extra = {"energy_rel_range": float((E.max() - E.min()) / abs(E[0])), "nsteps_per_run": nsteps,
             "launch": cfg,
             "roofline": _roof(force_eval_flops(n, cfg["algo"]) * nsteps, ms * 1e-3,
                               "whole md_run (force stage + fused epilogue per step, energies as recorded)",
                               _force_convention(cfg["algo"]))}
    if not args.no_cpu:
        from oracle import oracle as O

        k = 3 if which == "rf32768" else nsteps
        t0 = time.perf_counter()
        O.md_run(st0, d["q"], d["m"], d["trap"], 0.0, d["dt"], k, every=every if which == "cloud1024" else 0)
        t = time.perf_counter() - t0
        extra["cpu_baseline"] = {"value": float(n) * n * k / t, "unit": "pairs/s", "cores": len(os.sched_getaffinity(0)),
                                 "kind": "oracle", "sample": f"oracle md_run (compensated sums), {k} steps, {t:.1f} s"}
    wl = ("cloud1024: N=1024, Gaussian 20 um, 10 mK, static trap 2pi(1,1,0.2) MHz, dt=1 ns, 100 steps, energies "
          "every step" if which == "cloud1024" else
          "rf32768: N=32768 uniform ellipsoid (150,150,1000) um, RF a=0 q=0.3 Omega=2pi 10 MHz, wz=2pi 0.1 MHz, "
          "dt=5 ns, 1000 steps, energies every 50")
    return _line("pair interactions/s (FP64 velocity-Verlet run)", float(n) * n * nsteps / (ms * 1e-3), "pairs/s",
                 reps, args.warmup, ms / nsteps, wl, extra)


def bench_kz(args):
    """kz512: 512 runs, N uniform in [64, 4096], ramp, in one md_run; FP64
    and mixed on the default (stepped) ensemble path, FP64 captured in a HIP
    graph and replayed, and FP64 on the persistent kernel for comparison.  --steps sets the steps per run (10000
    in the full workload)."""
    np, torch, api, inputs, dev = _setup()
    from paper_2106_11143_amd import drivers

    nsteps = args.steps if args.steps != 50 else 10000
    d = inputs.kz512(nsteps=nsteps)
    offs = d["offsets"]
    ns = np.diff(offs)
    pairs = float((ns.astype(np.float64) ** 2).sum()) * nsteps
    st0 = inputs.state9(d)
    q, m = dev(d["q"]), dev(d["m"])
    res = {}
    ntot = int(offs[-1])
    # the default path (the stepped one for this ensemble), then the
    # persistent kernel forced, for comparison
    # (the persistent kernel over at most 1000 steps: its rate per step is steady)
    for key, prec, force in (("fp64", "fp64", False), ("mixed", "mixed", False), ("fp64_persistent", "fp64", True)):
        k = min(nsteps, 1000) if force else nsteps
        if force:
            api.set_config("md_ensemble", ntot, prec, p=4, wg=512, splits=1, algo=0)
        ts = [dev(st0[c]) for c in range(9)]
        torch.cuda.synchronize()
        e0, e1 = _timer(torch)
        e0.record()
        api.md_run(ts, q, m, d["traps"], 0.0, d["dt"], k, offsets=offs, prec=prec)
        e1.record()
        torch.cuda.synchronize()
        if force:
            api.reset_config("md_ensemble", ntot, prec)
        ms = e0.elapsed_time(e1)
        got = np.stack([t.cpu().numpy() for t in ts[:3]])
        defects = [drivers.count_defects(*got[:, offs[r]:offs[r + 1]]) for r in range(d["nrun"])]
        kp = pairs / nsteps * k
        res[key] = {"ms": ms, "steps": k, "ms_per_step": ms / k, "runs_per_s": d["nrun"] / (ms * 1e-3),
                    "pairs_per_s": kp / (ms * 1e-3), "defects_mean": float(np.mean(defects)),
                    "finite": bool(np.isfinite(got).all())}
    # the default path captured in a HIP graph (at most 1000 steps: two
    # launches per step), replayed once, against the same steps run eagerly
    k = min(nsteps, 1000)
    ts_eager = [dev(st0[c]) for c in range(9)]
    api.md_run(ts_eager, q, m, d["traps"], 0.0, d["dt"], k, offsets=offs)
    ts_g = [dev(st0[c]) for c in range(9)]
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        api.md_run(ts_g, q, m, d["traps"], 0.0, d["dt"], k, offsets=offs)
    for c in range(9):
        ts_g[c].copy_(dev(st0[c]))
    torch.cuda.synchronize()
    e0, e1 = _timer(torch)
    e0.record()
    graph.replay()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    res["fp64_graph"] = {"ms": ms, "steps": k, "ms_per_step": ms / k,
                         "pairs_per_s": pairs / nsteps * k / (ms * 1e-3),
                         "bitwise_equal_eager": bool(torch.equal(torch.stack(ts_g), torch.stack(ts_eager)))}
    del graph
    extra = {"mixed": res["mixed"], "fp64": res["fp64"], "fp64_graph_replay": res["fp64_graph"],
             "fp64_persistent_kernel": res["fp64_persistent"],
             "path": "stepped (p = 4; JL = 512, the default shape for ensembles of 2^30 or more ordered pairs)",
             "nrun": d["nrun"],
             "nsteps_per_run": nsteps,
             "sum_N2": float((ns.astype(np.float64) ** 2).sum()),
             "roofline": _roof(FLOPS_PER_SYM_PAIR * float((ns.astype(np.float64) * (ns - 1) / 2).sum()) * nsteps,
                               res["fp64"]["ms"] * 1e-3,
                               "whole md_run: per step k_pair_sym_ens<FP64> over every run's tiles + k_ens_step<FP64>",
                               "27 FLOP per unordered pair x sum over runs of n(n-1)/2 per step (Newton's third law)")}
    if not args.no_cpu:
        from oracle import oracle as O

        order = np.argsort(-ns)[:16]
        k = 2
        t0 = time.perf_counter()
        cpairs = 0.0
        for r in order:
            sl = slice(offs[r], offs[r + 1])
            O.md_run(st0[:, sl], d["q"][sl], d["m"][sl], d["trap"], 0.0, d["dt"], k)
            cpairs += float(ns[r]) ** 2 * k
        t = time.perf_counter() - t0
        extra["cpu_baseline"] = {"value": cpairs / t, "unit": "pairs/s", "cores": len(os.sched_getaffinity(0)),
                                 "kind": "oracle", "sample": f"oracle md_run, 16 largest runs x {k} steps, {t:.1f} s"}
    return _line("pair interactions/s (FP64 batched ensemble)", res["fp64"]["pairs_per_s"], "pairs/s", 1, 0,
                 res["fp64"]["ms"] / nsteps,
                 f"kz512: 512 runs, N~U[64,4096], wx,wy 2pi 1.5->0.6 MHz over 20 us, wz 2pi 0.15 MHz, dt 2 ns, "
                 f"{nsteps} steps", extra)


def bench_crystal(args):
    """crystal8192: minimised crystal, 32 lowest normal modes by block
    Lanczos on the HVP kernel, and the 2000-step trajectory gradient with
    checkpoints every 50 steps, checked against central differences."""
    np, torch, api, inputs, dev = _setup()
    from paper_2106_11143_amd import drivers

    d = inputs.crystal8192()
    n, trap = d["n"], d["trap"]
    q, m = dev(d["q"]), dev(d["m"])
    t0 = time.perf_counter()
    r, info = drivers.minimise(dev(np.stack([d["x"], d["y"], d["z"]])), q, m, trap, ftol_rel=1e-10)
    torch.cuda.synchronize()
    t_min = time.perf_counter() - t0
    # HVP throughput at 8 vectors per pass
    V = dev(np.random.Generator(np.random.PCG64(1)).normal(size=(8, 3, n)))
    rows = [r[c].contiguous() for c in range(3)]
    api.coulomb_hvp(*rows, q, V, m, trap)
    torch.cuda.synchronize()
    e0, e1 = _timer(torch)
    e0.record()
    for _ in range(10):
        api.coulomb_hvp(*rows, q, V, m, trap)
    e1.record()
    torch.cuda.synchronize()
    ms_hvp = e0.elapsed_time(e1) / 10
    t0 = time.perf_counter()
    lam, vecs, resid, lan_info = drivers.lanczos_lowest(r, q, m, trap, k=32, block=8, maxdim=12000)
    torch.cuda.synchronize()
    t_lan = time.perf_counter() - t0
    wz2 = trap["wz"] ** 2
    # Kohn: a uniform axial displacement is an exact eigenvector with omega_z^2
    U = torch.zeros(3, n, dtype=torch.float64, device="cuda")
    U[2] = 1.0
    kohn = float((api.coulomb_hvp(*rows, q, U, m, trap)[2] / m).sub(wz2).abs().max()) / wz2
    lam = lam.cpu().numpy()
    st = np.zeros((9, n))
    st[:3] = r.cpu().numpy()
    st[3], st[4], st[5] = d["vx"], d["vy"], d["vz"]
    t0 = time.perf_counter()
    L, g, _ = drivers.traj_grad(dev(st), q, m, trap, d["dt"], d["nsteps"], checkpoint_every=d["checkpoint_every"])
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    g = g.cpu().numpy()

    def loss(tr):
        s = [dev(st[k]) for k in range(9)]
        api.md_run(s, q, m, tr, 0.0, d["dt"], d["nsteps"])
        return float(sum(((s[c] - dev(st[c])) ** 2).sum() for c in range(3))) / n

    fd = {}
    for c, key in ((0, "wx"), (2, "wz")):
        h = 1e-6 * trap[key]
        tp, tm = dict(trap), dict(trap)
        tp[key] += h
        tm[key] -= h
        fd[key] = {"adjoint": float(g[c]), "central_fd": (loss(tp) - loss(tm)) / (2 * h)}
    hcfg = api.get_config("hvp", n, "fp64")
    hsym = hcfg["algo"] in SYM_ALGOS
    extra = {"roofline": _roof(hvp_eval_flops(n, 8, hsym), ms_hvp * 1e-3,
                               "cb::k_hvp<FP64> + epilogue, 8 vectors" if not hsym else
                               "cb::k_hvp_sym<FP64> + finish, 8 vectors",
                               ("15 + 30 B FLOP per unordered pair (B = 8 vectors) x n(n-1)/2" if hsym else
                                "16 + 21 B FLOP per ordered pair (B = 8 vectors) x n(n-1)")),
             "hvp_launch": hcfg,
             "minimise_s": t_min, "minimise": info, "hvp_ms_8vec": ms_hvp, "lanczos_s": t_lan,
             "lowest_over_wz2": [float(v) for v in lam[:6] / wz2],
             "zero_mode_rel": float(abs(lam[0]) / wz2), "kohn_axial_rel": kohn,
             "lanczos_max_residual": float(resid.max()), "lanczos": lan_info, "traj_grad_s": t_grad, "msd": L, "grad_fd": fd}
    if not args.no_cpu:
        from oracle import oracle as O

        rc = r.cpu().numpy()
        v8 = np.random.Generator(np.random.PCG64(2)).normal(size=(8, 3, n))
        t0 = time.perf_counter()
        passes = 0
        while passes == 0 or time.perf_counter() - t0 < 3.0:
            O.hvp(rc[0], rc[1], rc[2], d["q"], v8, m=d["m"], trap=trap)
            passes += 1
        t = time.perf_counter() - t0
        extra["cpu_baseline"] = {"value": float(n) * n * 8 * passes / t, "unit": "pairs*vectors/s",
                                 "cores": len(os.sched_getaffinity(0)), "kind": "oracle",
                                 "sample": f"oracle exact HVP (compensated), 8 vectors at N={n}, {passes} pass(es), "
                                           f"{t:.1f} s"}
    return _line("HVP pair-vector interactions/s (FP64, 8 vectors per pass)", float(n) * n * 8 / (ms_hvp * 1e-3),
                 "pairs*vectors/s", 10, 1, ms_hvp,
                 "crystal8192: N=8192 minimised crystal, 2pi(1,1,0.05) MHz; Lanczos 32 lowest; 2000-step adjoint "
                 "gradient, checkpoints every 50", extra)


def bench_hvp(args):
    """hvp8192: Hessian-vector products with 8 vectors at N = 8192 (the
    crystal8192 ions before relaxation: the cost does not depend on the
    configuration), in the default launch and in the all-pairs kernel's for
    comparison; a short workload for profiler runs."""
    np, torch, api, inputs, dev = _setup()
    d = inputs.crystal8192()
    n, trap = d["n"], d["trap"]
    q, m = dev(d["q"]), dev(d["m"])
    rows = [dev(d[k]) for k in ("x", "y", "z")]
    V = dev(np.random.Generator(np.random.PCG64(1)).normal(size=(8, 3, n)))
    reps = max(3, args.steps if args.steps != 50 else 20)

    def timed():
        api.coulomb_hvp(*rows, q, V, m, trap)
        torch.cuda.synchronize()
        e0, e1 = _timer(torch)
        e0.record()
        for _ in range(reps):
            out = api.coulomb_hvp(*rows, q, V, m, trap)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps, out

    cfg = api.get_config("hvp", n, "fp64")
    prewarm(torch, lambda: api.coulomb_hvp(*rows, q, V, m, trap), 0.5)
    ms, hv = timed()
    waves = -(-n // 64)
    api.set_config("hvp", n, "fp64", p=1, wg=256, splits=max(1, min(64, -(-3072 // waves))), algo=0)
    ms_direct, hv_d = timed()
    api.reset_config("hvp", n, "fp64")
    diff = float(((hv - hv_d).norm(dim=1) / hv_d.norm(dim=1)).max())
    sym = cfg["algo"] in SYM_ALGOS
    extra = {"launch": cfg, "direct_kernel_ms": ms_direct, "speedup_vs_direct": ms_direct / ms,
             "max_rel_vs_direct": diff,
             "roofline": _roof(hvp_eval_flops(n, 8, sym), ms * 1e-3,
                               "cb::k_hvp_sym<FP64> + pack + finish, 8 vectors" if sym else
                               "cb::k_hvp<FP64> + epilogue, 8 vectors",
                               ("15 + 30 B FLOP per unordered pair (B = 8 vectors) x n(n-1)/2" if sym else
                                "16 + 21 B FLOP per ordered pair (B = 8 vectors) x n(n-1)"))}
    return _line("HVP pair-vector interactions/s (FP64, 8 vectors)", float(n) * n * 8 / (ms * 1e-3),
                 "pairs*vectors/s", reps, 1, ms, "hvp8192: N=8192 ions, 8 vectors, static trap 2pi(1,1,0.05) MHz",
                 extra)


def bench_rsqrt_sweep(args):
    """Speed and accuracy of the four 1/sqrt variants against N (the paper's
    comparison of SQRT+DIV with the approximate inverse square root plus 0, 1
    or 2 Newton-Raphson steps, sections 4 and 6): time per force evaluation
    in the default launch of each size, and the per-ion relative force error
    against the oracle on a sample of ions."""
    np, torch, api, inputs, dev = _setup()
    from oracle import oracle as O

    variants = {"ieee": "SQRT+DIV (IEEE sqrt, division)", "fp64": "FP32 seed + 2nd-order refinement",
                "mixed": "FP32 seed + one Newton step", "fp32": "FP32 seed only",
                "mixed_f32d": "ablation: one Newton step on FP32-rounded displacements (direct kernel)"}
    sizes = [1024, 4096, 16384, 32768, 65536, 100000]
    rows = []
    for n in sizes:
        d = inputs.cloud100k(n=n)
        x, y, z, q = (dev(d[k]) for k in ("x", "y", "z", "q"))
        g = np.random.Generator(np.random.PCG64(11))
        idx = np.sort(g.choice(n, min(n, 256), replace=False))
        ref = np.stack(O.forces(d["x"], d["y"], d["z"], d["q"], idx=idx))
        for prec in variants:
            F = api.coulomb_forces(x, y, z, q, prec=prec)
            torch.cuda.synchronize()
            reps = max(3, int(0.05 / (n * n * 2e-13)))
            e0, e1 = _timer(torch)
            e0.record()
            for _ in range(reps):
                api.coulomb_forces(x, y, z, q, prec=prec)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            Fh = np.stack([t.cpu().numpy() for t in F])[:, idx]
            err = np.linalg.norm(Fh - ref, axis=0) / np.linalg.norm(ref, axis=0)
            cfg = api.get_config("forces", n, prec)
            rows.append({"n": n, "variant": prec, "ms": ms, "pairs_per_s": float(n) * n / (ms * 1e-3),
                         "max_rel_err": float(err.max()), "rms_rel_err": float(np.sqrt(np.mean(err ** 2))),
                         "algo": cfg["algo"]})
            print(f"n={n:6d} {prec:5s} {ms:9.4f} ms {float(n) * n / (ms * 1e-3):.3e} pairs/s "
                  f"max_err {err.max():.2e}", file=sys.stderr, flush=True)
    top = [r for r in rows if r["n"] == sizes[-1]]
    best = {r["variant"]: r["pairs_per_s"] for r in top}
    return _line("pair interactions/s per 1/sqrt variant (cloud100k-shaped clouds, coulomb_forces)",
                 best["fp64"], "pairs/s", 1, 1, [r["ms"] for r in top if r["variant"] == "fp64"][0],
                 f"rsqrt sweep: Gaussian clouds N in {sizes}, 1% at +2e, four 1/sqrt variants", 
                 {"variants": variants, "table": rows})


def bench_recording(args):
    """Energy-recording steps against plain steps on cloud100k (grouped by
    species, FP64, default launch): md_run of --steps steps without records
    and with a record every step, alternated three times after a clock
    pre-warm; the line's value is the recording step's rate."""
    np, torch, api, inputs, dev = _setup()
    d = inputs.group_by_charge(inputs.cloud100k())
    st = inputs.state9(d)
    ts = [dev(st[k]) for k in range(9)]
    q, m = dev(d["q"]), dev(d["m"])
    x, y, z = (dev(d[k]) for k in "xyz")
    prewarm(torch, lambda: api.coulomb_pair_stage(x, y, z, q), 1.0)
    api.md_run(ts, q, m, d["trap"], 0.0, d["dt"], 0, init_accel=True)
    K = args.steps if args.steps != 50 else 30
    rows = []
    for _ in range(3):
        for every in (0, 1):
            e0, e1 = _timer(torch)
            e0.record()
            api.md_run(ts, q, m, d["trap"], 0.0, d["dt"], K, init_accel=False, every=every)
            e1.record()
            torch.cuda.synchronize()
            rows.append({"every": every, "ms_per_step": e0.elapsed_time(e1) / K})
            print(f"md_run cloud100k every={every}: {rows[-1]['ms_per_step']:.4f} ms per step", file=sys.stderr,
                  flush=True)
    plain = [r["ms_per_step"] for r in rows if r["every"] == 0]
    rec = [r["ms_per_step"] for r in rows if r["every"] == 1]
    n = d["n"]
    return _line("pair interactions/s (FP64 velocity-Verlet steps recording the energies)",
                 float(n) * n / (np.mean(rec) * 1e-3), "pairs/s", K, 0, float(np.mean(rec)),
                 "cloud100k grouped by species: md_run steps with an energy record every step vs none",
                 {"plain_ms_per_step": plain, "recording_ms_per_step": rec,
                  "recording_over_plain": float(np.mean(rec) / np.mean(plain))})


def bench_uniform_tiles(args):
    """The charge-free tile loop on the single-species workloads: rf32768's
    force stage, timed (20 evaluations after a clock pre-warm), and 3 kz512
    md_run steps (for counter runs; not timed), first with their uniform
    charges, then with every other charge scaled by 1 + 1e-7 (no tile
    uniform: the per-j charge path everywhere)."""
    np, torch, api, inputs, dev = _setup()
    d = inputs.rf32768()
    x, y, z = (dev(d[k]) for k in "xyz")
    qm = d["q"].copy()
    qm[1::2] *= 1 + 1e-7
    qs = {"uniform": dev(d["q"]), "perturbed": dev(qm)}
    prewarm(torch, lambda: api.coulomb_pair_stage(x, y, z, qs["uniform"]), 0.5)
    res = {}
    reps = 20
    for rnd in range(2):
        for tag, q in qs.items():
            e0, e1 = _timer(torch)
            e0.record()
            for _ in range(reps):
                api.coulomb_pair_stage(x, y, z, q)
            e1.record()
            torch.cuda.synchronize()
            key = f"rf32768_{tag}_stage_ms"
            res[key] = min(res.get(key, 1e9), e0.elapsed_time(e1) / reps)
    k = inputs.kz512(nsteps=3)
    st0 = inputs.state9(k)
    m = dev(k["m"])
    for tag in ("uniform", "perturbed"):
        qh = k["q"].copy()
        if tag == "perturbed":
            qh[1::2] *= 1 + 1e-7
        ts = [dev(st0[c]) for c in range(9)]
        api.md_run(ts, dev(qh), m, k["traps"], 0.0, k["dt"], 3, offsets=k["offsets"])
        torch.cuda.synchronize()
    n = d["n"]
    return _line("pair interactions/s (rf32768 force stage, charge-free tiles)",
                 float(n) * n / (res["rf32768_uniform_stage_ms"] * 1e-3), "pairs/s", reps, 0,
                 res["rf32768_uniform_stage_ms"],
                 "rf32768 force stage, uniform charges vs every other charge scaled by 1+1e-7 (and 3 kz512 steps "
                 "of each, untimed, for counter runs)", res)


OTHER_WORKLOADS = {
    "cloud1024": lambda a: bench_md_single(a, "cloud1024"),
    "rf32768": lambda a: bench_md_single(a, "rf32768"),
    "kz512": bench_kz,
    "crystal8192": bench_crystal,
    "hvp8192": bench_hvp,
    "rsqrt_sweep": bench_rsqrt_sweep,
    "recording": bench_recording,
    "uniform_tiles": bench_uniform_tiles,
}


if __name__ == "__main__":
    main()
