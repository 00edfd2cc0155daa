#!/usr/bin/env python3
"""Throughput of the D3Q19 central-moment LBM step on one MI355X.

Workload (timed): periodic 256^3 lattice, Taylor-Green field U0 = 0.05 plus
seeded uniform noise +-1e-4, nu = 1e-3, Kolmogorov body force
F_x = 1e-6 sin(2 pi y / L), FP32 populations (shifted storage) and FP32
collision.  One step = one fused gather-collide-store launch over all nodes.

Prints one JSON line: MLUPS of the whole job, the roofline of the step kernel
(algorithmic bytes / kernel time from HIP events on the lattice's stream),
the FP16/BF16 shifted-storage variants measured the same way, and the FP64
CPU oracle timed on a bounded sample of the same workload on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2010_01628_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def elem_bytes(precision: str) -> int:
    return {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}[precision]


def time_variant(L, inputs, torch, size, precision, streaming, steps, warmup, fields):
    nu = 1e-3
    p = L.make_params(size, size, size, precision=precision, streaming=streaming,
                      omega=inputs.omega_from_nu(nu), force_mode=L.LBM_FORCE_KOLMOGOROV,
                      kolmogorov_amp=1e-6)
    lat = L.Lattice(p)
    rho_d, u_d = fields
    lat.init(rho_d, u_d)
    lat.step(warmup)
    torch.cuda.synchronize()
    stream = lat.stream
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev0[k].record(stream)
        lat.step(1)
        ev1[k].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms = [a.elapsed_time(b) for a, b in zip(ev0, ev1)]
    _, _, diag = lat.moments(want_fields=False)
    nbytes = lat.device_bytes
    lat.close()
    N = size ** 3
    kms = sorted(kernel_ms)
    avg_ms = sum(kernel_ms) / len(kernel_ms)
    algo_bytes = N * 2 * 19 * elem_bytes(precision)
    return {
        "precision": precision,
        "streaming": streaming,
        "mlups": N * steps / wall / 1e6,
        "ms_per_step": wall / steps * 1e3,
        "kernel_ms_avg": avg_ms,
        "kernel_ms_median": kms[len(kms) // 2],
        "algo_bytes_per_launch": algo_bytes,
        "achieved_GBs": algo_bytes / (avg_ms * 1e-3) / 1e9,
        "device_bytes": nbytes,
        "sum_rho": diag[0],
        "finite": bool(all(x == x for x in diag)),
    }


def cpu_baseline(inputs, size, seconds_target=20.0):
    """FP64 oracle (closed-form mode, OpenMP on all host cores) on a bounded
    sample: whole-lattice steps of the same 256^3 workload."""
    import numpy as np

    import oracle

    nu = 1e-3
    rho, u = inputs.taylor_green_noise(size, 0.05, 1e-4, seed=20101628)
    F = inputs.kolmogorov_force(size, size, size, 1e-6)
    Kd = oracle.K(inputs.omega_from_nu(nu))
    f = oracle.init(rho, u)
    del rho, u
    out = np.empty_like(f)
    steps = 0
    t0 = time.perf_counter()
    while True:
        oracle.step(f, Kd, F=F, out=out)
        f, out = out, f
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds_target / 2 or steps >= 4:
            break
    N = size ** 3
    return {
        "value": N * steps / el / 1e6,
        "unit": "MLUPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{steps} full steps of the {size}^3 workload (FP64, closed-form App. C path), {el:.1f} s",
    }


def load_traffic(precision: str, streaming: str, size: int, launches_algo_bytes: float):
    path = os.path.join(ROOT, "profiles", f"traffic_d3q19_step_{precision}_{streaming}_{size}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None  # counters were taken on another version of the kernels
    return t.get("hbm_bytes_per_launch")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--precision", default="fp32", choices=["fp64", "fp32", "fp16", "bf16"])
    ap.add_argument("--streaming", default="ab", choices=["ab", "aa"])
    ap.add_argument("--variants", default="fp16:ab,bf16:ab,fp32:aa,fp16:aa,fp64:ab",
                    help="extra precision:streaming pairs to time ('' = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        return 2
    if "RANK" in os.environ and os.environ.get("WORLD_SIZE", "1") != "1":
        print(json.dumps({"error": "single-GPU build: launch without torch.distributed"}))
        return 2

    import torch

    from paper_2010_01628_amd import inputs
    from paper_2010_01628_amd import lbm as L

    L.lib()  # fail loudly if the HIP library is missing
    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        return 3
    size = args.size
    log(f"bench: generating {size}^3 fields")
    rho, u = inputs.taylor_green_noise(size, 0.05, 1e-4, seed=20101628)
    fields = (torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
    del rho, u

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1.0)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    log(f"bench: timing {args.precision}/{args.streaming} {args.steps} steps")
    head = time_variant(L, inputs, torch, size, args.precision, args.streaming, args.steps, args.warmup, fields)
    variants = {}
    for spec in [v for v in args.variants.split(",") if v]:
        prec, _, strm = spec.partition(":")
        strm = strm or args.streaming
        if (prec, strm) == (args.precision, args.streaming):
            continue
        log(f"bench: timing variant {prec}/{strm}")
        variants[f"{prec}_{strm}"] = time_variant(L, inputs, torch, size, prec, strm, max(20, args.steps // 4),
                                                  max(5, args.warmup // 4), fields)
    del fields
    torch.cuda.empty_cache()

    traffic = load_traffic(args.precision, args.streaming, size, head["algo_bytes_per_launch"])
    roof = {
        "bound": "hbm",
        "achieved": round(head["achieved_GBs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(head["achieved_GBs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": "lbm::k_step (fused gather-collide-store)",
        "kernel_ms_avg": round(head["kernel_ms_avg"], 5),
        "algo_bytes_per_launch": head["algo_bytes_per_launch"],
    }
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: CPU oracle baseline")
        cpu = cpu_baseline(inputs, size)

    line = {
        "metric": "MLUPS & % HBM roofline, D3Q19 CM-LBM 256^3; FP16/learned vs plain FP32",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.precision if args.precision != "fp32" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"D3Q19 CM-LBM periodic {size}^3, Taylor-Green U0=0.05 + seeded noise 1e-4, nu=1e-3, "
                        f"Kolmogorov force 1e-6, {args.precision} storage, {args.streaming.upper()} streaming",
            "nodes": size ** 3,
            "storage": args.precision,
            "streaming": args.streaming,
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "variants": {k: {"mlups": round(v["mlups"], 1), "achieved_GBs": round(v["achieved_GBs"], 1),
                         "frac": round(v["achieved_GBs"] / HBM_PEAK_GBS, 4),
                         "kernel_ms_avg": round(v["kernel_ms_avg"], 5),
                         "speedup_vs_head": round(v["mlups"] / head["mlups"], 3)} for k, v in variants.items()},
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
