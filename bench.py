"""Throughput of the D3Q19 binary-fluid LB step on one MI355X.

Default workload: the 256^3 periodic tanh droplet (radius 64, width
sqrt(-2 kappa/A), +-1e-3 seeded noise) with A=-0.00625, B=0.00625,
kappa=0.004, tau_f=tau_g=1, Gamma=0.5, stepped in FP32 deviation storage (the
headline line) and in FP64 on the same input; plus the adjoint/forward cost
of the reverse mode (64^3 FP64 and 128^3 FP32 rollouts) and the oracle timed
on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line.  A "step" is one full timestep of the lattice (order
parameter, gradients, chemical stress, collision of f and g, propagation).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# Algorithmic HBM bytes per lattice-site update of one step (one launch of the
# single-pass kernel processes every site once).  The method must read and
# write the 19 f and 19 g populations once: 76 words of the storage type,
# 304 B (FP32 storage) or 608 B (FP64) -- the roofline's basis.  In FP32 mode
# the stored time level also carries the reference order parameter phi_c
# (one 32-bit word, read once and written once: 8 B), which the kernel moves
# on top of that.
def step_bytes_per_site(elem_bytes: int) -> dict:
    extra = 8 if elem_bytes == 4 else 0
    return {"method_min": 76 * elem_bytes, "kernel": 76 * elem_bytes + extra}


# HBM bytes per launch of the single-pass step kernel on the 256^3 droplet,
# from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) over
# `bench.py --steps 5 --warmup 1 --no-adjoint --no-cpu-baseline
# --spinodal-steps 0 --force-steps 5 --fd-steps 5 --shard-steps 0
# --error-steps 0`, each scaled by the same counter's reading for the
# library's copy kernel of known size (FETCH x 2.000, WRITE x 1.000).
# They hold only for the kernel sources they were taken on (the hash below);
# after any change to those sources the traffic is reported as null.
TRAFFIC_SOURCES = ("lb_kernels.hip", "lb_device.h", "lb_internal.h")
TRAFFIC_SHA256 = "d86d933167066445c0fd4198305be13ba6339a49ff7f7524e314d0ba5395c23f"
TRAFFIC_BYTES = {"fp32_dev": 5350005418, "fp64": 10363384056}


def sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1609_01479_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(prec: str, n: int, layout: str = "rows"):
    if n != 256 or layout != "rows" or TRAFFIC_SHA256 is None or prec not in TRAFFIC_BYTES:
        return None
    if sources_sha256() != TRAFFIC_SHA256:
        return None
    return TRAFFIC_BYTES[prec]


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def settle(lb, calls: int, step=None) -> None:
    """`calls` untimed steps (or `step()` calls) on the library's stream.
    After host work, allocations or an idle spell the GPU runs its first
    tens of milliseconds of work slowly (the 256^3 step 1.02-1.06 ms, then
    0.97 ms twenty launches later); the legs beside the headline settle
    first, for some 30-60 ms, so that they report the steady state.  A count,
    not a time: legs that compare the two precisions step both alike."""
    step = step or (lambda: lb.step(1))
    for _ in range(calls):
        step()
    lb.synchronize()


def time_steps(lb, steps: int, warmup: int, sums=None):
    """ms for `steps` steps on the library's stream (HIP events on that
    stream).  With `sums` (a (steps, 5) FP64 device tensor) every step also
    reduces its conserved sums (lb_step_sums)."""
    import torch
    lb.step(warmup)
    lb.synchronize()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(lb.stream)
    if sums is None:
        lb.step(steps)
    else:
        lb.step_sums(steps, sums)
    e1.record(lb.stream)
    e1.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def adjoint_ratio(shape, T, interval, precision, phi0, tgt, params, order_param="lb",
                  coupling="stress", extra=None):
    """(forward ms for T plain steps, backward ms incl. recompute, grads);
    extra (a dict, optional) receives the checkpoint interval used and the
    rollout's own forward time (the T steps, writing its checkpoints)."""
    import torch
    from paper_1609_01479_amd import LB
    from paper_1609_01479_amd.rollout import rollout
    dev = torch.device("cuda:0")
    lb = LB(shape, precision=precision, device=dev, order_param=order_param, coupling=coupling,
            **params)
    lb.init_phi(phi0)
    settle(lb, 30 * (256 // shape[0]) ** 3)
    fwd_ms = time_steps(lb, T, 0)
    del lb
    rest = {k: params[k] for k in ("gamma", "tau_f", "tau_g", "rho0")}
    tgt_t = torch.tensor(tgt, device=dev)

    info = {}

    def forward():
        p0 = torch.tensor(phi0, dtype=torch.float64, device=dev, requires_grad=True)
        th = [torch.tensor(params[k], dtype=torch.float64, device=dev, requires_grad=True)
              for k in ("A", "B", "kappa")]
        phiT = rollout(p0, *th, T, interval=interval, precision=precision,
                       order_param=order_param, coupling=coupling, info=info, **rest)
        return p0, th, 0.5 * ((phiT - tgt_t) ** 2).sum()

    # one untimed rollout first (kernel loading, allocator), as every timed
    # region here has its warm-up
    forward()[2].backward()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p0, th, loss = forward()
    torch.cuda.synchronize()
    if extra is not None:
        extra["interval"] = info.get("interval")
        extra["rollout_forward_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    t0 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    bwd_ms = (time.perf_counter() - t0) * 1e3
    grads = (p0.grad.detach().cpu().numpy(), [float(t.grad) for t in th])
    return fwd_ms, bwd_ms, grads


def mixed_rollout_grads(shape, T, k, fwd_prec, adj_prec, phi0, tgt, params):
    """dL/dphi0 and dL/d(A, B, kappa) of the LB-scheme rollout (stress
    coupling, loss 1/2 sum (phi_T - tgt)^2) with the trajectory stepped in
    fwd_prec storage and the adjoint steps taken in adj_prec storage: every
    (recomputed) state of the trajectory is exported as dense FP64
    distributions and imported into the adjoint's context, whose reverse step
    then linearises the step there.  Separates the error of an FP32 forward
    trajectory from that of FP32 adjoint arithmetic and storage."""
    import torch
    from paper_1609_01479_amd import LB
    dev = torch.device("cuda:0")
    fw = LB(shape, precision=fwd_prec, device=dev, **params)
    ad = LB(shape, precision=adj_prec, adjoint=True, device=dev, **params)
    fw.init_phi(phi0)
    ckpts, t = [], 0
    while t < T:
        ckpts.append(fw.get_state())
        n = min(k, T - t)
        fw.step(n)
        t += n
    phiT = fw.phi()
    ad.adjoint_seed(phiT - torch.tensor(tgt, device=dev))
    dtheta = torch.zeros(3, dtype=torch.float64, device=dev)
    seg = [None] + [fw.new_state() for _ in range(min(k, T) - 1)]
    buf = ad.new_state()
    for si in reversed(range(len(ckpts))):
        t0, t1 = si * k, min(T, si * k + k)
        seg[0] = ckpts[si]
        for j in range(1, t1 - t0):
            fw.step_from(seg[j - 1], seg[j])
        for t in reversed(range(t0, t1)):
            fw.set_state(seg[t - t0])
            f, g = fw.export_dist()
            ad.import_dist(f, g)
            ad.get_state(buf)
            ad.adjoint_step(buf, dtheta)
    dphi0 = ad.adjoint_phi0()
    torch.cuda.synchronize()
    return dphi0.cpu().numpy(), [float(v) for v in dtheta.cpu()]


def footprint_sweep(args):
    """Achieved bandwidth against the bytes a launch touches: the library's
    streaming copy (read B, write B) and the single-pass step and its
    memory-only twin (read one time level, write the other) on droplet
    lattices of growing size.  GB/s count the kernels' own bytes (FP32
    storage: 312 B per site with phi_c; FP64: 608)."""
    import torch

    import lbinputs
    from paper_1609_01479_amd import LB
    from paper_1609_01479_amd.lb import copy_probe_gbps
    params = dict(lbinputs.SPINODAL_PARAMS)
    xi = lbinputs.interface_width(params["A"], params["kappa"])
    steps = max(args.steps, 20)
    out = {"metric": "bandwidth against footprint", "copy": [], "lattice": []}
    for gb in (0.25, 0.5, 1.0, 2.0, 2.62, 4.0, 8.0):
        nbytes = int(gb * 1e9)
        log(f"copy probe {gb} GB")
        out["copy"].append({"read_GB": gb, "footprint_GB": 2 * gb,
                            "GBps": round(copy_probe_gbps(nbytes, reps=10), 1)})
        torch.cuda.empty_cache()
    for n in (128, 192, 256, 320):
        shape = (n, n, n)
        nsites = n ** 3
        phi0 = lbinputs.droplet_phi0(shape, n / 4.0, xi, noise=1e-3, seed=lbinputs.SEED_DROPLET)
        for prec in ("fp32_dev", "fp64"):
            row = {"n": n, "precision": prec}
            # the step and its twin on the same buffers, timed alternately
            # (3 rounds, medians; even step counts keep both on one level)
            lb = LB(shape, precision=prec, device="cuda:0", **params)
            lb.init_phi(phi0)
            twin = lb.sibling("stream")
            e = int(lb.sizes.elem_bytes)
            kb = step_bytes_per_site(e)["kernel"]
            row["footprint_GB"] = round(kb * nsites / 1e9, 3)
            k = steps + steps % 2
            log(f"{prec} {shape}: step and twin, 3 x {k} steps each")
            settle(lb, 30, lambda: lb.step(2))  # even: both contexts stay on one level
            time_steps(lb, 0, 2 * (args.warmup // 2 + 1))
            time_steps(twin, 0, 2 * (args.warmup // 2 + 1))
            tm = {"fused": [], "stream": []}
            for _ in range(3):
                tm["fused"].append(time_steps(lb, k, 0) / k)
                tm["stream"].append(time_steps(twin, k, 0) / k)
            for kern, v in tm.items():
                ms = sorted(v)[1]
                row[kern + "_ms"] = round(ms, 4)
                row[kern + "_GBps"] = round(kb * nsites / (ms * 1e-3) / 1e9, 1)
            twin.close()
            del lb, twin
            torch.cuda.empty_cache()
            row["step_over_twin"] = round(row["fused_ms"] / row["stream_ms"], 4)
            out["lattice"].append(row)
    return out


def fp32_vs_fp64_run(shape, phi0, params, lay, steps):
    """FP32 deviation storage against FP64 on the same droplet over a fixed
    number of steps (2000 by default, whatever --steps is): steps both
    precisions, with max and RMS of |phi32 - phi64| at a quarter and half of
    the run; fp32_vs_fp64_finish() takes the end point."""
    from paper_1609_01479_amd import LB
    log(f"FP32 vs FP64: {steps} steps of both")
    l32 = LB(shape, precision="fp32_dev", device="cuda:0", **lay, **params)
    l64 = LB(shape, precision="fp64", device="cuda:0", **lay, **params)
    l32.init_phi(phi0)
    l64.init_phi(phi0)
    marks = sorted({m for m in (steps // 4, steps // 2, steps) if m > 0})
    done, phi_hist = 0, {}
    for m in marks:
        l32.step(m - done)
        l64.step(m - done)
        done = m
        if m < steps:
            d = (l32.phi() - l64.phi()).abs()
            phi_hist[str(m)] = {"max": float(d.max()), "rms": float(d.square().mean().sqrt())}
            del d
    return l32, l64, phi_hist, done


def fp32_vs_fp64_finish(l32, l64, phi_hist, done):
    """The end point of fp32_vs_fp64_run: |phi32 - phi64| and |u32 - u64|."""
    import torch
    _, u32, p32 = l32.moments()
    _, u64, p64 = l64.moments()
    dphi = (p32 - p64).abs()
    du = (u32 - u64).abs()
    phi_hist[str(done)] = {"max": float(dphi.max()), "rms": float(dphi.square().mean().sqrt())}
    err = {"after_steps": done,
           "phi_max": float(dphi.max()),
           "phi_rms": float(dphi.square().mean().sqrt()),
           "u_max": float(du.max()),
           "u_rms": float(du.square().mean().sqrt()),
           "u64_max": float(u64.abs().max()),
           "phi_by_step": phi_hist,
           "target_phi_max": 1e-5}
    del u32, u64, p32, p64, dphi, du
    torch.cuda.empty_cache()
    return err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-legs", default="",
                    help="comma-separated names of the adjoint legs to run (default: all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=2,
                    help="oracle steps of the 256^3 CPU baseline sample")
    ap.add_argument("--layout", default="rows", choices=["rows", "soa", "aos", "aosoa"],
                    help="distribution layout of the 256^3 legs (default: row-blocked)")
    ap.add_argument("--aosoa-len", type=int, default=64, help="z-sites per block for --layout aosoa")
    ap.add_argument("--force-steps", type=int, default=200,
                    help="steps of the 256^3 force-coupling lines (0: skip)")
    ap.add_argument("--fd-steps", type=int, default=200,
                    help="steps of the 256^3 finite-difference order-parameter lines (0: skip)")
    ap.add_argument("--shard-steps", type=int, default=500,
                    help="steps of the one-GPU-share lines (32 x 256 x 256, 0: skip)")
    ap.add_argument("--grad-attribution", action="store_true",
                    help="attribute the FP32 adjoint's gradient error (128^3, T=1000, k=32) "
                         "to the trajectory or the adjoint precision")
    ap.add_argument("--error-steps", type=int, default=2000,
                    help="steps of the FP32-vs-FP64 error leg on the 256^3 droplet (0: skip)")
    ap.add_argument("--spinodal-steps", type=int, default=1000,
                    help="steps of the extra 128^3 FP64 spinodal throughput line (0: skip)")
    ap.add_argument("--footprint-sweep", action="store_true",
                    help="only the bandwidth-against-footprint sweep: the copy probe over "
                         "0.25-8 GB and the single-pass step and its memory-only twin on "
                         "droplet lattices of 128^3 to 320^3 (both storage precisions)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(a step shards as x-slabs with one halo exchange per step; not built)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lbinputs
    from paper_1609_01479_amd import LB

    if args.footprint_sweep:
        print(json.dumps(footprint_sweep(args)), flush=True)
        return

    n = args.size
    shape = (n, n, n)
    params = dict(lbinputs.SPINODAL_PARAMS)
    xi = lbinputs.interface_width(params["A"], params["kappa"])
    radius = n / 4.0
    log(f"droplet {shape} radius {radius} xi {xi:.5f}")
    phi0 = lbinputs.droplet_phi0(shape, radius, xi, noise=1e-3, seed=lbinputs.SEED_DROPLET)
    nsites = n ** 3

    lay = dict(layout=args.layout, aosoa_len=args.aosoa_len if args.layout == "aosoa" else 0)
    # The contexts of the headline legs are created first, then the
    # FP32-vs-FP64 error leg steps, and the headline legs follow it at once.
    # A GPU that has idled, or stepped at a light load, for some
    # milliseconds (allocations, host-side copies and reductions between
    # legs) runs its first tens of milliseconds of the step slowly: the
    # kernel measured 1.02-1.06 ms at the first launches after such gaps and
    # 0.97 ms twenty launches later.  Created beforehand and started while
    # the GPU is busy, the headline's timed steps see its steady state.
    precs = ["fp32_dev"] + ([] if args.no_fp64 else ["fp64"])
    ctxs = {}
    for prec in precs:
        ctxs[prec] = LB(shape, precision=prec, device="cuda:0", **lay, **params)
        ctxs[prec].init_phi(phi0)
    errrun = None
    if not args.no_fp64 and args.error_steps > 0:
        errrun = fp32_vs_fp64_run(shape, phi0, params, lay, args.error_steps)

    runs = {}
    for prec in precs:
        lb = ctxs.pop(prec)
        hist = torch.empty((args.steps, 5), dtype=torch.float64, device="cuda:0")
        log(f"{prec}: warmup {args.warmup}, timing {args.steps} steps (with per-step sums)")
        ms = time_steps(lb, args.steps, args.warmup, sums=hist)
        torch.cuda.synchronize()
        h = hist.cpu().numpy()
        # the same number of steps without the per-step reduction: one launch
        # of the single-pass kernel per step, timed with HIP events on the
        # library's stream -- the kernel's average launch duration; and five
        # repeats of a tenth of them (min and median per step)
        ms_plain = time_steps(lb, args.steps, 0)
        kr = max(args.steps // 10, 1)
        reps = sorted(time_steps(lb, kr, 0) / kr for _ in range(5))
        runs[prec] = dict(ms=ms, ms_plain=ms_plain, reps=reps, elem=int(lb.sizes.elem_bytes),
                          max_drift=np.abs(h - h[0]).max(axis=0))
        log(f"{prec}: {ms:.1f} ms -> {nsites * args.steps / (ms * 1e-3) / 1e6:.1f} MLUPS "
            f"(plain steps {ms_plain:.1f} ms)")
        del lb, hist
        torch.cuda.empty_cache()

    prim = runs["fp32_dev"]
    ms_step = prim["ms"] / args.steps
    mlups = nsites / (ms_step * 1e-3) / 1e6

    def roof(run, prec):
        e = run["elem"]
        b = step_bytes_per_site(e)
        # achieved = the method's algorithmic bytes per launch (304 or 608 B
        # per site times the N sites one launch updates) / the kernel's
        # average launch duration (plain steps: one launch each)
        t = run["ms_plain"] / args.steps * 1e-3
        achieved = b["method_min"] * nsites / t / 1e9
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                "traffic": measured_traffic(prec, n, args.layout),
                "bytes_per_site": b["method_min"],
                "algorithmic_bytes_per_launch": b["method_min"] * nsites,
                "kernel": "k_step_fused_f32" if e == 4 else "k_step_fused_f64",
                "kernel_ms": round(t * 1e3, 4),
                "kernel_time_source": f"HIP events around {args.steps} plain steps "
                                      "(one launch each) on the library's stream",
                "kernel_bytes_per_site": b["kernel"],
                "achieved_kernel_bytes_GBps": round(b["kernel"] * nsites / t / 1e9, 1)}

    out = {
        "metric": "MLUPS & % peak HBM GB/s, D3Q19 binary 256^3: FP32 vs FP64; adjoint/forward cost",
        "value": round(mlups, 1), "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded tanh droplet + noise)",
        "config": {"workload": f"D3Q19 binary-fluid droplet {n}^3 periodic, FP32 deviation storage",
                   "lattice": list(shape), "layout": args.layout
                   + (f":{args.aosoa_len}" if args.layout == "aosoa" else ""),
                   "radius": radius, "xi": round(xi, 6),
                   "noise": 1e-3, "seed": lbinputs.SEED_DROPLET, **params},
        "roofline": roof(prim, "fp32_dev"),
    }
    out["ms_per_step_without_sums"] = round(prim["ms_plain"] / args.steps, 4)
    out["ms_per_step_without_sums_5_repeats"] = {"min": round(prim["reps"][0], 4),
                                                 "median": round(prim["reps"][2], 4)}
    out["conservation"] = {"fp32_max_abs_drift_over_run": {
        k: float(v) for k, v in zip(("rho", "phi", "jx", "jy", "jz"), prim["max_drift"])}}
    if "fp64" in runs:
        r64 = runs["fp64"]
        ms64 = r64["ms"] / args.steps
        out["fp64"] = {"value": round(nsites / (ms64 * 1e-3) / 1e6, 1), "unit": "MLUPS",
                       "ms_per_step": round(ms64, 4),
                       "ms_per_step_without_sums": round(r64["ms_plain"] / args.steps, 4),
                       "ms_per_step_without_sums_5_repeats": {"min": round(r64["reps"][0], 4),
                                                              "median": round(r64["reps"][2], 4)},
                       "roofline": roof(r64, "fp64")}
        out["conservation"]["fp64_max_abs_drift_over_run"] = {
            k: float(v) for k, v in zip(("rho", "phi", "jx", "jy", "jz"), r64["max_drift"])}
        out["fp32_over_fp64_speedup"] = round(ms64 / ms_step, 3)

    # the single-pass kernel's memory-only twin (LB_KERNEL_STREAM: the same
    # loads, phi sums and stores with the collision left out) on the same
    # lattice: the memory-bound floor of this kernel's access pattern
    out["stream_twin"] = {}
    for prec in precs:
        # the twin as a second context on the step's own buffers, the two
        # timed alternately (5 rounds; even step counts keep both contexts on
        # the same time level): same memory, same moment, so the ratio does
        # not carry placement or drift between separate allocations
        lb = LB(shape, precision=prec, device="cuda:0", **lay, **params)
        lb.init_phi(phi0)
        twin = lb.sibling("stream")
        k = max(args.steps, 20)
        k += k % 2
        log(f"{prec}: step and memory-only twin on the same buffers, 5 x {k} steps each")
        settle(lb, 30, lambda: lb.step(2))  # even: both contexts stay on one level
        time_steps(lb, 0, 2 * (args.warmup // 2 + 1))
        time_steps(twin, 0, 2 * (args.warmup // 2 + 1))
        ts, tt = [], []
        for _ in range(5):
            ts.append(time_steps(lb, k, 0) / k)
            tt.append(time_steps(twin, k, 0) / k)
        ts.sort()
        tt.sort()
        e = int(lb.sizes.elem_bytes)
        kb = step_bytes_per_site(e)["kernel"]
        key = "fp32_dev" if e == 4 else "fp64"
        out["stream_twin"][key] = {
            "step_ms_median": round(ts[2], 4), "twin_ms_median": round(tt[2], 4),
            "twin_GBps_kernel_bytes": round(kb * nsites / (tt[2] * 1e-3) / 1e9, 1),
            "step_over_twin": round(ts[2] / tt[2], 4), "rounds": 5, "steps_per_round": k}
        twin.close()
        del lb, twin
        torch.cuda.empty_cache()

    if errrun is not None:
        out["fp32_vs_fp64_error"] = fp32_vs_fp64_finish(*errrun)
        del errrun
    del runs

    # force coupling (body force -div Pi) on the same 256^3 droplet: one
    # marching kernel per step (phi from its own pulls), f and g read and
    # written once: the method's 608 B per site in FP64 and 304 in FP32
    # storage (the kernel's own 312 with its reference field phi_c)
    if args.force_steps > 0:
        out["force_coupling"] = {}
        force_phi = {}
        for prec, minimum, kbytes in (("fp32_dev", 304, 312), ("fp64", 608, 608)):
            lb = LB(shape, precision=prec, coupling="force", device="cuda:0", **lay, **params)
            lb.init_phi(phi0)
            log(f"{prec} force coupling {shape}: {args.force_steps} steps")
            settle(lb, 60)
            ms = time_steps(lb, args.force_steps, args.warmup)
            t = ms / args.force_steps * 1e-3
            out["force_coupling"][prec] = {
                "value": round(nsites / t / 1e6, 1), "unit": "MLUPS", "steps": args.force_steps,
                "ms_per_step": round(ms / args.force_steps, 4),
                "achieved_GBps": round(minimum * nsites / t / 1e9, 1),
                "frac": round(minimum * nsites / t / 1e9 / HBM_PEAK_GBPS, 4),
                "bytes_per_site": minimum,
                "kernel_bytes_per_site": kbytes,
                "kernels": "k_force_fused"}
            force_phi[prec] = lb.phi().cpu().numpy()
            del lb
            torch.cuda.empty_cache()
        out["force_coupling"]["phi_fp32_vs_fp64_max"] = float(
            np.abs(force_phi["fp32_dev"] - force_phi["fp64"]).max())
        del force_phi

    # finite-difference order parameter (a phi field, no g) on the same 256^3
    # droplet, single-pass kernel: f read and written once (FP64 304, FP32
    # storage 152 B per site) and phi read and written once (16): 320 and 168
    # B per site, the scheme's minimum.
    if args.fd_steps > 0:
        out["fd_order_parameter"] = {}
        fd_phi = {}
        for prec, moved in (("fp32_dev", 168), ("fp64", 320)):
            lb = LB(shape, precision=prec, order_param="fd", device="cuda:0", **lay, **params)
            lb.init_phi(phi0)
            log(f"{prec} finite-difference order parameter {shape}: {args.fd_steps} steps")
            settle(lb, 60)
            ms = time_steps(lb, args.fd_steps, args.warmup)
            t = ms / args.fd_steps * 1e-3
            fd_phi[prec] = lb.phi().cpu().numpy()
            out["fd_order_parameter"][prec] = {
                "value": round(nsites / t / 1e6, 1), "unit": "MLUPS", "steps": args.fd_steps,
                "ms_per_step": round(ms / args.fd_steps, 4),
                "achieved_GBps": round(moved * nsites / t / 1e9, 1),
                "frac": round(moved * nsites / t / 1e9 / HBM_PEAK_GBPS, 4),
                "bytes_per_site": moved,
                "kernels": "k_fd_fused"}
            del lb
            torch.cuda.empty_cache()
        out["fd_order_parameter"]["phi_fp32_vs_fp64_max"] = float(
            np.abs(fd_phi["fp32_dev"] - fd_phi["fp64"]).max())
        del fd_phi
        # with the force coupling: one marching kernel as well, f and phi
        # read and written once (the scheme's minimum, 320 / 168 B per site;
        # Pi, the force and the face ring's mu and u formed on chip)
        out["fd_order_parameter"]["force_coupling"] = {}
        for prec, moved in (("fp32_dev", 168), ("fp64", 320)):
            lb = LB(shape, precision=prec, order_param="fd", coupling="force", device="cuda:0",
                    **lay, **params)
            lb.init_phi(phi0)
            log(f"{prec} finite-difference order parameter + force coupling {shape}: "
                f"{args.fd_steps} steps")
            settle(lb, 60)
            ms = time_steps(lb, args.fd_steps, args.warmup)
            t = ms / args.fd_steps * 1e-3
            out["fd_order_parameter"]["force_coupling"][prec] = {
                "value": round(nsites / t / 1e6, 1), "unit": "MLUPS", "steps": args.fd_steps,
                "ms_per_step": round(ms / args.fd_steps, 4),
                "achieved_GBps": round(moved * nsites / t / 1e9, 1),
                "frac": round(moved * nsites / t / 1e9 / HBM_PEAK_GBPS, 4),
                "bytes_per_site": moved, "kernels": "k_fd_force_fused"}
            del lb
            torch.cuda.empty_cache()

    # one GPU's share of the 256^3 droplet split into 8 x-slabs: a shard of
    # 32 x 256 x 256 (halo_x) whose step reads halo planes instead of the
    # periodic wrap; here it receives its own faces (pack + unpack on the
    # same GPU stand in for the exchange with its neighbours).  Timed: the
    # step with its face copies, and the face copies alone.
    if args.shard_steps > 0 and n == 256:
        out["shard_32x256x256"] = {}
        sh = (32, 256, 256)
        nsh = 32 * 256 * 256
        lo, hi = n // 2 - 16, n // 2 + 16  # the slab through the centre
        phish = np.ascontiguousarray(phi0[lo - 1:hi + 1])
        for prec, moved in (("fp32_dev", 304), ("fp64", 608)):
            lb = LB(sh, precision=prec, device="cuda:0", halo_x=True, **lay, **params)
            lb.init_phi(phish)
            faces = (lb.new_face(), lb.new_face())

            def exchange():
                lb.pack_faces(*faces)
                lb.unpack_faces(faces[1], faces[0])

            def timed(k, step):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                lb.synchronize()
                e0.record(lb.stream)
                for _ in range(k):
                    exchange()
                    if step:
                        lb.step(1)
                e1.record(lb.stream)
                e1.synchronize()
                return e0.elapsed_time(e1)

            log(f"{prec} shard {sh}: {args.shard_steps} steps with face exchange")
            settle(lb, 240, lambda: (exchange(), lb.step(1)))
            timed(args.warmup, True)
            ms = timed(args.shard_steps, True)
            ms_faces = timed(args.shard_steps, False)
            t = ms / args.shard_steps * 1e-3
            ts = (ms - ms_faces) / args.shard_steps * 1e-3
            out["shard_32x256x256"][prec] = {
                "value": round(nsh / t / 1e6, 1), "unit": "MLUPS", "steps": args.shard_steps,
                "ms_per_step": round(ms / args.shard_steps, 4),
                "faces_ms_per_step": round(ms_faces / args.shard_steps, 4),
                "face_bytes": int(lb.sizes.face_bytes),
                "step_ms_without_faces": round(ts * 1e3, 4),
                "achieved_GBps": round(moved * nsh / ts / 1e9, 1),
                "frac": round(moved * nsh / ts / 1e9 / HBM_PEAK_GBPS, 4)}
            del lb, faces
            torch.cuda.empty_cache()

    # FP64 on the 128^3 spinodal-decomposition lattice (phi0 ~ U(-0.05, 0.05))
    if not args.no_fp64 and args.spinodal_steps > 0:
        sh = (128, 128, 128)
        lb = LB(sh, precision="fp64", device="cuda:0", **params)
        lb.init_phi(lbinputs.spinodal_phi0(sh))
        log(f"fp64 spinodal {sh}: {args.spinodal_steps} steps")
        settle(lb, 240)
        ms = time_steps(lb, args.spinodal_steps, args.warmup)
        t = ms / args.spinodal_steps * 1e-3
        n128 = 128 ** 3
        out["fp64_spinodal_128"] = {
            "value": round(n128 / t / 1e6, 1), "unit": "MLUPS", "steps": args.spinodal_steps,
            "ms_per_step": round(ms / args.spinodal_steps, 4),
            "achieved_GBps": round(step_bytes_per_site(8)["method_min"] * n128 / t / 1e9, 1),
            "frac": round(step_bytes_per_site(8)["method_min"] * n128 / t / 1e9 / HBM_PEAK_GBPS, 4)}
        del lb
        torch.cuda.empty_cache()

    # the library's streaming copy over 2 GiB (read 1 GiB + write 1 GiB): the
    # practical HBM ceiling, measured in the same job
    from paper_1609_01479_amd.lb import copy_probe_gbps
    probe = copy_probe_gbps(1024 ** 3)
    out["copy_probe_GBps"] = round(probe, 1)
    # the kernels' own bytes (FP32: with phi_c) over the copy's rate
    out["roofline"]["kernel_frac_of_copy_probe"] = round(
        out["roofline"]["achieved_kernel_bytes_GBps"] / probe, 4)
    if "fp64" in out:
        out["fp64"]["roofline"]["kernel_frac_of_copy_probe"] = round(
            out["fp64"]["roofline"]["achieved_kernel_bytes_GBps"] / probe, 4)
    # the same copy at the footprint of the FP32 step (read one time level,
    # write another: 2 x 312/2 B per site)
    probe_fp = copy_probe_gbps(156 * nsites, reps=10)
    out["copy_probe_same_footprint_GBps"] = round(probe_fp, 1)
    out["roofline"]["kernel_frac_of_copy_probe_same_footprint"] = round(
        out["roofline"]["achieved_kernel_bytes_GBps"] / probe_fp, 4)

    if not args.no_adjoint:
        adj = {}
        # the sqrt(T) checkpoint intervals of the two configurations, the
        # 64^3 one with every state kept (200 x 81 MB: no recomputation), and
        # the same two configurations for the finite-difference scheme and
        # for the force coupling (the larger one for both together)
        for name, nn, T, k, prec, op, cp in (
                ("64^3_fp64_T200", 64, 200, 15, "fp64", "lb", "stress"),
                ("64^3_fp64_T200_every_state", 64, 200, 1, "fp64", "lb", "stress"),
                ("128^3_fp32_T1000", 128, 1000, 32, "fp32_dev", "lb", "stress"),
                ("fd_64^3_fp64_T200", 64, 200, 15, "fp64", "fd", "stress"),
                ("fd_128^3_fp32_T1000", 128, 1000, 32, "fp32_dev", "fd", "stress"),
                ("force_64^3_fp64_T200", 64, 200, 15, "fp64", "lb", "force"),
                ("force_128^3_fp32_T1000", 128, 1000, 32, "fp32_dev", "lb", "force"),
                ("fd_force_128^3_fp32_T1000", 128, 1000, 32, "fp32_dev", "fd", "force"),
                # as many checkpoints as HBM holds (at most 90% of the free
                # memory): k = 2 for these 336 MB states, 168 GB of them
                ("128^3_fp32_T1000_hbm_checkpoints", 128, 1000, "auto", "fp32_dev", "lb",
                 "stress")):
            if args.adjoint_legs and name not in args.adjoint_legs.split(","):
                continue
            sh = (nn, nn, nn)
            ph0 = lbinputs.spinodal_phi0(sh)
            tgt = lbinputs.lamellar_target(sh, 32, xi)
            log(f"adjoint {name}")
            ex = {}
            fwd, bwd, g = adjoint_ratio(sh, T, k, prec, ph0, tgt, params, op, cp, extra=ex)
            entry = {"forward_ms": round(fwd, 2), "backward_ms": round(bwd, 2),
                     "adjoint_over_forward": round(bwd / fwd, 3), "interval": ex["interval"],
                     "rollout_forward_ms": ex["rollout_forward_ms"],
                     "order_param": op, "coupling": cp, "warmup_rollouts": 1}
            if prec == "fp32_dev" and k != "auto":
                _, _, g64 = adjoint_ratio(sh, T, k, "fp64", ph0, tgt, params, op, cp)
                entry["grad_rel_err_vs_fp64"] = {
                    "phi0_l2": float(np.linalg.norm(g[0] - g64[0]) / np.linalg.norm(g64[0])),
                    "A": g[1][0] / g64[1][0] - 1, "B": g[1][1] / g64[1][1] - 1,
                    "kappa": g[1][2] / g64[1][2] - 1}
            adj[name] = entry
            torch.cuda.empty_cache()
        out["adjoint"] = adj

    if args.grad_attribution:
        # every (trajectory, adjoint) precision pair of the 128^3, T = 1000,
        # k = 32 configuration against the all-FP64 pair
        sh = (128, 128, 128)
        ph0 = lbinputs.spinodal_phi0(sh)
        tgt = lbinputs.lamellar_target(sh, 32, xi)
        res = {}
        for fp_, ap_ in (("fp64", "fp64"), ("fp32_dev", "fp32_dev"), ("fp32_dev", "fp64"),
                         ("fp64", "fp32_dev")):
            log(f"gradient attribution: trajectory {fp_}, adjoint {ap_}")
            res[(fp_, ap_)] = mixed_rollout_grads(sh, 1000, 32, fp_, ap_, ph0, tgt, params)
            torch.cuda.empty_cache()
        g64 = res[("fp64", "fp64")]
        out["grad_attribution"] = {
            f"trajectory_{a}_adjoint_{b}": {
                "phi0_l2": float(np.linalg.norm(g[0] - g64[0]) / np.linalg.norm(g64[0])),
                "A": g[1][0] / g64[1][0] - 1, "B": g[1][1] / g64[1][1] - 1,
                "kappa": g[1][2] / g64[1][2] - 1}
            for (a, b), g in res.items() if (a, b) != ("fp64", "fp64")}

    if not args.no_cpu_baseline:
        # The FP64 oracle as it stands (plain per-site C loops; OpenMP over
        # sites in its gradient and collision loops; the order-parameter sum,
        # chemical potential and stress, and streaming serial) on the host cores: a bounded sample of the
        # headline workload (cpu_steps steps of the same 256^3 droplet), the
        # 128^3 spinodal input of the FP64 throughput line (5 steps), and one
        # thread on a 64^3 droplet.  A baseline, not the target.
        import oracle
        cores = len(os.sched_getaffinity(0))
        cores = oracle.set_threads(cores)
        cpu = host_cpu_model()
        p = oracle.Params(*shape, **params)
        f, g = oracle.init(p, phi0)
        log(f"oracle: {args.cpu_steps} steps at {shape} on {cores} threads ({cpu})")
        t0 = time.perf_counter()
        oracle.run(p, f, g, args.cpu_steps)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(nsites * args.cpu_steps / dt / 1e6, 3),
                               "unit": "MLUPS", "cores": cores, "kind": "oracle",
                               "sample": f"{args.cpu_steps} FP64 steps of the same {n}^3 droplet "
                                         f"lattice ({dt:.1f} s) on {cpu}; the oracle's OpenMP "
                                         f"covers its gradient and collision loops, its "
                                         f"order-parameter sum, chemical stress and "
                                         f"streaming run serially"}
        del f, g
        s2 = (128, 128, 128)
        p2 = oracle.Params(*s2, **params)
        f2, g2 = oracle.init(p2, lbinputs.spinodal_phi0(s2))
        t0 = time.perf_counter()
        oracle.run(p2, f2, g2, 5)
        dt2 = time.perf_counter() - t0
        out["cpu_baseline_spinodal_128"] = {"value": round(128 ** 3 * 5 / dt2 / 1e6, 3),
                                            "unit": "MLUPS", "cores": cores, "kind": "oracle",
                                            "sample": f"5 FP64 steps of the 128^3 spinodal "
                                                      f"lattice ({dt2:.1f} s)"}
        del f2, g2
        # single-thread figure on a 64^3 droplet of the same recipe
        s1 = (64, 64, 64)
        p1 = oracle.Params(*s1, **params)
        f1, g1 = oracle.init(p1, lbinputs.droplet_phi0(s1, 16.0, xi, noise=1e-3,
                                                        seed=lbinputs.SEED_DROPLET))
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.run(p1, f1, g1, 1)
        dt1 = time.perf_counter() - t0
        oracle.set_threads(cores)
        out["cpu_baseline_1thread"] = {"value": round(64 ** 3 / dt1 / 1e6, 3), "unit": "MLUPS",
                                       "cores": 1, "kind": "oracle",
                                       "sample": f"1 FP64 step of a 64^3 droplet ({dt1:.1f} s)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
