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
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def kernel_source_hash() -> str:
    from paper_2010_01628_amd.traffic import kernel_source_hash as h

    return h()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def elem_bytes(precision: str) -> int:
    return {"fp64": 8, "fp32": 4, "fp16": 2, "bf16": 2}[precision]


def time_variant(L, inputs, torch, size, precision, streaming, steps, warmup, fields, mlp=None, tune=True,
                 moments="central", rounding="nearest"):
    nu = 1e-3
    p = L.make_params(size, size, size, precision=precision, streaming=streaming,
                      omega=inputs.omega_from_nu(nu), force_mode=L.LBM_FORCE_KOLMOGOROV,
                      kolmogorov_amp=1e-6, moments=moments, rounding=rounding, seed=20101628)
    lat = L.Lattice(p)
    rho_d, u_d = fields
    lat.init(rho_d, u_d)
    launch = None
    if mlp is not None:
        lat.attach_mlp(mlp)
    elif tune:
        launch = lat.tune(10)  # work-group shape and cache hints, timed on real steps
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
    fallbacks = lat.fallback_count() if mlp is not None else None
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
        "fallbacks": fallbacks,
        "launch": launch,
    }


def stream_copy_bandwidth(torch, L, n, eb=4, q=19, reps=10, lane=0):
    """Rate of the library's bandwidth reference (lbm_stream_copy): q arrays
    of n elements copied with the step's access pattern and streaming hints
    (lane: bytes per thread and array, 0 = one element as the step), read +
    write bytes per second, HIP events on the stream it runs on, best of
    `reps` after two untimed launches."""
    dt = {2: torch.int16, 4: torch.int32, 8: torch.int64}[eb]
    a = torch.zeros(q * n, dtype=dt, device="cuda")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for _ in range(2):
        L.lbm_stream_copy(a.data_ptr(), b.data_ptr(), n, q, eb, True, st.cuda_stream, lane_bytes=lane)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        L.lbm_stream_copy(a.data_ptr(), b.data_ptr(), n, q, eb, True, st.cuda_stream, lane_bytes=lane)
        e1.record(st)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * q * n * eb / (best * 1e-3) / 1e9


def copy_bandwidth(torch, nbytes=2 << 30, reps=10):
    """Device copy bandwidth (read + write bytes per second) of torch's copy
    of a 2 GiB buffer, HIP events, best of `reps`: a measured copy rate the
    step kernel is compared with beside the nominal 8 TB/s (one read and one
    write stream; a copy of 19 streams in and 19 out, the step's access
    pattern, runs faster)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def time_ensemble(L, inputs, torch, steps, warmup, mlp, tune=True):
    """The 64-box ensemble workload (sides 48/64/96, random-phase fields,
    u_rms 0.04, nu log-uniform in [1e-4, 1e-3]): MLUPS of plain D3Q19, learned
    D3Q19 and D3Q27, FP32 storage, one persistent launch per step replayed
    from a HIP graph."""
    spec = inputs.ensemble_boxes()
    boxes = [(n, inputs.omega_from_nu(nu)) for n, nu, _ in spec]
    fields = [inputs.random_phase_field(n, 0.04, seed=sd) for n, _, sd in spec]
    out = {}
    for name, q, net in (("q19", 19, None), ("q19_learned", 19, mlp), ("q27", 27, None)):
        ens = L.Ensemble(boxes, q=q, precision="fp32")
        for b, (rho, u) in enumerate(fields):
            ens.init(b, rho, u)
        if net is not None:
            ens.set_mlp(net)
        grid = ens.tune(10) if tune else None  # work-groups per launch (times real steps)
        ens.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ens.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        bpn = 2 * q * 4
        out[name] = {"mlups": round(ens.nodes * steps / wall / 1e6, 1),
                     "achieved_GBs": round(ens.nodes * bpn * steps / wall / 1e9, 1),
                     "algo_bytes_per_node": bpn, "grid": grid}
        if net is not None:
            out[name]["fallback_rate"] = ens.fallback_count() / float(ens.nodes * (steps + warmup))
        out["nodes"] = ens.nodes
        ens.close()
    out["boxes"] = len(boxes)
    out["steps"] = steps
    return out


def time_coupled(L, inputs, torch, steps, warmup):
    """Coupled-lattice workloads: the two-phase droplet (192^3, R = 32,
    density ratio 10, sigma = 1e-3, W = 4, FP32), the Hartmann channel
    (32 x 128 x 32, Ha = 10, FP32), the Shan-Chen static bubble (100^3,
    R = 20, G = -5, nu = 0.0333, FP32) and the colour-gradient Rayleigh-Taylor
    case (64 x 256 x 64, FP32).  Algorithmic bytes per node and step:
    two-phase 244 (flow 152, phase 56, phi 32 + 4), magnetic 320, Shan-Chen
    236 (psi launch 76 + 4, step 152 + 4), colour gradient 464 (phi launch
    152 + 4, step 304 + 4)."""
    import numpy as np

    out = {}
    n = 192
    phi = inputs.droplet((n, n, n), 32.0, 4.0, noise=1e-3, seed=192)
    par = L.make_params(n, n, n, precision="fp32", omega=1.25,
                        phase=dict(rho_light=1.0, rho_heavy=10.0, sigma=1e-3, width=4.0, mobility=0.1))
    lat = L.Lattice(par)
    lat.init_phase(phi, np.full(phi.shape, 1.0 / 3.0), np.zeros((3,) + phi.shape))
    del phi
    out["phase_192"] = _time_lattice(lat, torch, steps, warmup, n ** 3, 244)
    lat.close()
    nx, ny, nz = 32, 128, 32
    b0 = 10.0 * 2 * 0.1 / ny
    F = 0.02 * b0 ** 2 * np.tanh(10.0) / (0.1 * 10.0 * (1 - 1 / np.cosh(10.0)))
    par = L.make_params(nx, ny, nz, precision="fp32", omega=1.0 / 0.8, walls_y=True, force_mode=L.LBM_FORCE_UNIFORM,
                        force=(F, 0.0, 0.0), magnetic=dict(eta=0.1, b_wall=(0.0, b0, 0.0)))
    lat = L.Lattice(par)
    b = np.zeros((3, nz, ny, nx))
    b[1] = b0
    lat.init_magnetic(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)), b)
    out["hartmann_32x128x32"] = _time_lattice(lat, torch, 4 * steps, warmup, nx * ny * nz, 320)
    lat.close()
    n = 100
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - n / 2) ** 2)
    rho = 0.15 + 1.8 * 0.5 * (1 - np.tanh((r - 20.0) / 2.0))
    par = L.make_params(n, n, n, precision="fp32", omega=inputs.omega_from_nu(0.0333), shan_chen=dict(G=-5.0))
    lat = L.Lattice(par)
    lat.init(rho, np.zeros((3,) + rho.shape))
    out["shan_chen_bubble_100"] = _time_lattice(lat, torch, 4 * steps, warmup, n ** 3, 236)
    lat.close()
    from paper_2010_01628_amd import rayleigh_taylor

    par, rr, rb, _ = rayleigh_taylor.setup(64)
    lat = L.Lattice(par)
    lat.init_colour(rr, rb, np.zeros((3,) + rr.shape))
    out["rayleigh_taylor_64x256x64"] = _time_lattice(lat, torch, 4 * steps, warmup, rr.size, 464)
    lat.close()
    return out


def _time_lattice(lat, torch, steps, warmup, nodes, bytes_per_node):
    lat.step(warmup)
    st = lat.stream
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record(st)
    lat.step(steps)
    b.record(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = a.elapsed_time(b) / steps
    gbs = nodes * bytes_per_node / (ms * 1e-3) / 1e9
    _, _, diag = lat.moments(want_fields=False)
    return {"mlups": round(nodes * steps / wall / 1e6, 1), "ms_per_step": round(ms, 5),
            "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "algo_bytes_per_node": bytes_per_node, "finite": all(x == x for x in diag)}


def bench_network(L):
    """A fixed network for throughput runs: random hidden layers and a small
    random output layer, so the rates spread around 1 without fallbacks (the
    cost does not depend on the weights otherwise)."""
    import numpy as np

    from paper_2010_01628_amd import learned

    P = learned.initial_params(seed=0)
    P[1440:1728] = np.random.default_rng(1).normal(size=288) * 0.02
    scales = np.array([0.05, 0.02, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3])
    return L.Mlp(P, scales)


def cpu_baseline(inputs, size, seconds_target=12.0):
    """FP64 oracle (f* = T(u)^-1 k* by a dense solve per node, OpenMP on all
    host cores) on a bounded sample: whole-lattice steps of the same 256^3
    workload."""
    import numpy as np

    import oracle

    nu = 1e-3
    rho, u = inputs.taylor_green_noise(size, 0.05, 1e-4, seed=20101628)
    F = inputs.kolmogorov_force(size, size, size, 1e-6)
    Kd = oracle.K(inputs.omega_from_nu(nu))
    f = oracle.init(rho, u)
    del rho, u
    out = np.empty_like(f)
    # two untimed steps: first touch of the output pages, then one warm step
    for _ in range(2):
        oracle.step(f, Kd, F=F, out=out)
        f, out = out, f
    steps = 0
    t0 = time.perf_counter()
    while True:
        oracle.step(f, Kd, F=F, out=out)
        f, out = out, f
        steps += 1
        el = time.perf_counter() - t0
        if el > seconds_target or steps >= 64:
            break
    N = size ** 3
    return {
        "value": N * steps / el / 1e6,
        "unit": "MLUPS",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": f"{steps} full steps of the {size}^3 workload after 2 untimed steps (FP64, dense T(u) "
                  f"solve per node), {el:.1f} s",
        "cpu_model": cpu_model(),
        "cpus_visible": os.cpu_count(),
    }


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def kernel_label(streaming: str, launch) -> str:
    """Name of the timed step kernel for a launch (block_x, block_y, cache
    policy, staged) as lbm_tune reports it (None: the library default,
    which stages wherever whole-row work-groups allow it)."""
    staged = launch is None or bool(launch[3])
    if streaming == "ab":
        name = "lbm::k_step_ab_rows" if staged else "lbm::k_step_ab"
    else:
        name = "lbm::k_step_aa (even) + lbm::k_step_aa_odd_rows" if staged else "lbm::k_step_aa"
    return name + " (fused gather-collide-store" + (", x-moving populations staged through LDS)" if staged else ")")


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
    ap.add_argument("--variants",
                    default="fp16:ab,bf16:ab,fp32:aa,fp16:aa,bf16:aa,fp64:ab,fp32+mlp:ab,fp16+mlp:ab,fp32+raw:ab,"
                            "fp16+raw:ab,bf16+sr:ab",
                    help="extra precision[+mlp|+raw|+sr]:streaming pairs to time ('' = none); +mlp = learned "
                         "rates, +raw = raw-moment collision (the N = I variant), +sr = stochastic rounding")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 64-box ensemble workload")
    ap.add_argument("--no-coupled", action="store_true", help="skip the two-phase and magnetic workloads")
    ap.add_argument("--no-tune", action="store_true", help="keep the library's default launch shape")
    ap.add_argument("--no-mem-check", action="store_true",
                    help="skip the 512^3 AA FP32 and FP16 memory check (device bytes and MLUPS)")
    ap.add_argument("--no-cost-table", action="store_true",
                    help="skip the D3Q19/D3Q27 x raw/central cost table over D = 32..128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain 1 GiB device copy (calibrates HBM counters)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        return 2
    if "RANK" in os.environ and os.environ.get("WORLD_SIZE", "1") != "1":
        print(json.dumps({"error": "one-GPU benchmark: launch without torch.distributed"}))
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
    head = time_variant(L, inputs, torch, size, args.precision, args.streaming, args.steps, args.warmup, fields,
                        tune=not args.no_tune)
    variants = {}
    mlp = None
    for spec in [v for v in args.variants.split(",") if v]:
        prec, _, strm = spec.partition(":")
        strm = strm or args.streaming
        prec, _, plus = prec.partition("+")
        if (prec, strm) == (args.precision, args.streaming) and not plus:
            continue
        if plus not in ("", "mlp", "raw", "sr"):
            raise SystemExit(f"unknown variant modifier +{plus}")
        if plus == "mlp" and mlp is None:
            mlp = bench_network(L)
        log(f"bench: timing variant {spec}")
        tag = {"": "", "mlp": "_learned", "raw": "_raw", "sr": "_stochastic"}[plus]
        variants[f"{prec}{tag}_{strm}"] = time_variant(
            L, inputs, torch, size, prec, strm, max(20, args.steps // 4), max(5, args.warmup // 4), fields,
            mlp=mlp if plus == "mlp" else None, tune=not args.no_tune, moments="raw" if plus == "raw" else "central",
            rounding="stochastic" if plus == "sr" else "nearest")
    del fields
    torch.cuda.empty_cache()
    ensemble = None
    if not args.no_ensemble:
        if mlp is None:
            mlp = bench_network(L)
        log("bench: ensemble workload")
        ensemble = time_ensemble(L, inputs, torch, max(20, args.steps // 2), max(4, args.warmup // 2), mlp,
                                 tune=not args.no_tune)
    coupled = None
    if not args.no_coupled:
        log("bench: coupled-lattice workloads")
        coupled = time_coupled(L, inputs, torch, max(20, args.steps // 2), max(4, args.warmup // 2))
    cost = None
    if not args.no_cost_table:
        from paper_2010_01628_amd import taylor_green

        log("bench: cost table (Taylor-Green, D = 32..128)")
        cost = taylor_green.cost_table()
    mem = None
    if not args.no_mem_check:
        log("bench: 512^3 memory check")
        rho, u = inputs.taylor_green_noise(512, 0.05, 1e-4, seed=20101628)
        f512 = (torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
        del rho, u
        mem = {}
        for prec in ("fp32", "fp16"):
            r = time_variant(L, inputs, torch, 512, prec, "aa", 20, 4, f512)
            mem[f"{prec}_aa"] = {"mlups": round(r["mlups"], 1), "device_bytes": r["device_bytes"],
                                 "achieved_GBs": round(r["achieved_GBs"], 1), "finite": r["finite"]}
        del f512
        torch.cuda.empty_cache()

    traffic = load_traffic(args.precision, args.streaming, size, head["algo_bytes_per_launch"])
    copy_gbs = copy_bandwidth(torch)
    ref_gbs = stream_copy_bandwidth(torch, L, size ** 3, eb=elem_bytes(args.precision))
    # the same copy with wider accesses per thread: does the ceiling itself rise?
    lane_gbs = {str(w): round(stream_copy_bandwidth(torch, L, size ** 3, eb=elem_bytes(args.precision), lane=w), 1)
                for w in (8, 16) if w > elem_bytes(args.precision)}
    lane_gbs[str(elem_bytes(args.precision))] = round(ref_gbs, 1)
    roof = {
        "bound": "hbm",
        "achieved": round(head["achieved_GBs"], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(head["achieved_GBs"] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "kernel": kernel_label(args.streaming, head["launch"]),
        "kernel_ms_avg": round(head["kernel_ms_avg"], 5),
        "algo_bytes_per_launch": head["algo_bytes_per_launch"],
        "launch": head["launch"],
        "torch_copy_GBs": round(copy_gbs, 1),
        "frac_of_torch_copy": round(head["achieved_GBs"] / copy_gbs, 4),
        "stream_copy_GBs": round(ref_gbs, 1),
        "frac_of_stream_copy": round(head["achieved_GBs"] / ref_gbs, 4),
        "stream_copy_GBs_by_lane_bytes": lane_gbs,
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
                         "speedup_vs_head": round(v["mlups"] / head["mlups"], 3), "launch": v["launch"],
                         **({"fallbacks": v["fallbacks"]} if v["fallbacks"] is not None else {})}
                     for k, v in variants.items()},
        "ensemble": ensemble,
        "coupled": coupled,
        "cost_table": cost,
        "mem_check_512": mem,
        "kernel_source_hash": kernel_source_hash(),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
