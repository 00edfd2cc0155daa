"""Conditioning of the timed workload under storage rounding, measured with
the FP64 oracle only (writes tests/golden/conditioning_config2.json).

Workload: the 3-D Taylor-Green field of Sec. III (U0 = 0.05, x = 2 pi i / L)
plus seeded uniform noise 1e-4, nu = 1e-3, Kolmogorov force
F_x = 1e-6 sin(2 pi y / L), periodic L^3, 1000 steps.  The exact FP64 run is
the reference; each variant perturbs the stored state, which (as on the GPU)
is the deviation s_i = f_i - w_i from the rest populations:

  init_eps    s_i(0) -> s_i(0) (1 + 2^-24 xi), xi uniform in [-1, 1], once
  step_eps    the same relative noise on s_i after every step
  fp32        s_i rounded to FP32 after every step (round to nearest even)
  fp16        s_i rounded to FP32, then FP16 (nearest even), every step
  bf16        s_i rounded to FP32, then BF16 (nearest even), every step
  bf16_sr     s_i rounded to FP32, then BF16 with stochastic rounding (a
              uniform 16-bit integer added to the FP32 bit pattern before the
              low 16 bits are cut), every step

Every other operation is the oracle's FP64 arithmetic, so each variant's
distance from the reference is what that storage alone costs on this
workload: relative L2 of u and of rho - mean(rho) at steps 200 and 1000.

    python tests/golden/conditioning.py 64 [128 ...] [--only fp32,bf16,...]

Random numbers come from numpy (seeded); nothing here runs on a GPU or calls
the GPU library.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2010_01628_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "conditioning_config2.json")
STEPS, NU, U0, NOISE, SEED, KOLM = 1000, 1e-3, 0.05, 1e-4, 20101628, 1e-6
RECORD = (200, 1000)
EPS = 2.0 ** -24


def bf16_rne(x32: np.ndarray) -> np.ndarray:
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def bf16_sr(x32: np.ndarray, rng: np.random.Generator) -> np.ndarray:
    b = x32.view(np.uint32).astype(np.uint64)
    b = (b + rng.integers(0, 1 << 16, size=b.shape, dtype=np.uint64)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def make_perturb(kind: str, w: np.ndarray, seed: int):
    rng = np.random.default_rng(seed)
    wb = w[:, None, None, None]

    def perturb(f: np.ndarray) -> None:
        s = f - wb
        if kind in ("init_eps", "step_eps"):
            s *= 1.0 + EPS * rng.uniform(-1.0, 1.0, size=s.shape)
        else:
            s32 = s.astype(np.float32)
            if kind == "fp16":
                s32 = s32.astype(np.float16).astype(np.float32)
            elif kind == "bf16":
                s32 = bf16_rne(s32)
            elif kind == "bf16_sr":
                s32 = bf16_sr(s32, rng)
            s = s32.astype(np.float64)
        np.add(s, wb, out=f)

    return perturb


def fields(f, F):
    rho, u = oracle.moments(f, F)
    return rho, u


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rel_l2_fluct(ra, rb):
    da, db = ra - ra.mean(), rb - rb.mean()
    return float(np.linalg.norm((da - db).ravel()) / np.linalg.norm(db.ravel()))


def run(N: int, kind: str | None, f0, Kd, F, w, refs=None):
    f = f0.copy()
    if kind == "init_eps":
        make_perturb(kind, w, 1)(f)
        per_step = None
    elif kind is not None:
        per_step = make_perturb(kind, w, 2)
    else:
        per_step = None
    out = np.empty_like(f)
    rec = {}
    t0 = time.time()
    for t in range(1, STEPS + 1):
        oracle.step(f, Kd, F=F, out=out)
        f, out = out, f
        if per_step is not None:
            per_step(f)
        if t in RECORD:
            rho, u = fields(f, F)
            if refs is None:
                rec[t] = (rho, u)
            else:
                rr, ur = refs[t]
                rec[t] = {"u": rel_l2(u, ur), "rho_fluct": rel_l2_fluct(rho, rr)}
        if t % 100 == 0:
            print(f"  {N}^3 {kind or 'reference'}: step {t} ({time.time() - t0:.0f} s)", flush=True)
    return rec


KINDS = ("init_eps", "step_eps", "fp32", "fp16", "bf16", "bf16_sr")


def main(sizes, kinds=KINDS):
    res = json.load(open(OUT)) if os.path.exists(OUT) else {}
    c, w, _ = oracle.tables()
    for N in sizes:
        rho, u = inputs.taylor_green_noise(N, U0, NOISE, seed=SEED)
        F = inputs.kolmogorov_force(N, N, N, KOLM)
        Kd = oracle.K(inputs.omega_from_nu(NU))
        f0 = oracle.init(rho, u)
        refs = run(N, None, f0, Kd, F, w)
        entry = {"steps": list(RECORD), "oracle_threads": oracle.num_threads()}
        for kind in kinds:
            rec = run(N, kind, f0, Kd, F, w, refs)
            entry[kind] = {str(t): v for t, v in rec.items()}
            print(f"{N}^3 {kind}: {entry[kind]}", flush=True)
            res[str(N)] = entry
            with open(OUT, "w") as fh:
                json.dump(res, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    args = sys.argv[1:]
    kinds = KINDS
    if "--only" in args:
        i = args.index("--only")
        kinds = tuple(args[i + 1].split(","))
        args = args[:i] + args[i + 2:]
    main([int(a) for a in args] or [64], kinds)
