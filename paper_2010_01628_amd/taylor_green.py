"""Three-dimensional Taylor-Green vortex of Sec. III, the paper's single-phase
comparison of the D3Q19 and D3Q27 CM lattices and the workload of its cost
study (App. D): kinetic-energy decay for given Re = u0 D / nu and
Ma = u0 / cs, and the per-step cost of the four collision variants the paper
times (D3Q19/D3Q27, raw/central moments) over box sizes D.

Only orders library calls: every lattice operation runs in the HIP library.
"""
from __future__ import annotations

import math

import numpy as np

from . import inputs
from . import lbm as L

CS = math.sqrt(1.0 / 3.0)


def parameters(D: int, Re: float, Ma: float):
    """(u0, nu, omega, t0 = D / u0 in steps)."""
    u0 = Ma * CS
    nu = u0 * D / Re
    return u0, nu, 1.0 / (3.0 * nu + 0.5), D / u0


def ke_decay(D: int, Re: float, Ma: float, q: int = 19, moments: str = "central", precision: str = "fp32",
             t_end: float = 3.0, samples: int = 60, check_every: int = 50):
    """Run the vortex (rho = 1, velocity of Sec. III at x = 2 pi i / D) to
    t / t0 = t_end.  Returns dict(t = t / t0 at the samples, ke = KE / KE(0),
    stable, t_fail): a run that the library's stability check stops
    (non-finite or non-positive density) is marked unstable at that time."""
    u0, _, om, t0 = parameters(D, Re, Ma)
    rho, u = inputs.taylor_green_noise(D, u0, 0.0)
    p = L.make_params(D, D, D, precision=precision, q=q, omega=om, moments=moments, check_every=check_every)
    lat = L.Lattice(p)
    try:
        lat.init(rho, u)
        _, _, d = lat.moments(want_fields=False)
        ke0 = d[4]
        total = int(round(t_end * t0))
        t, ke = [0.0], [1.0]
        done = 0
        stable, t_fail = True, None
        for k in range(1, samples + 1):
            target = int(round(k * total / samples))
            try:
                lat.step(target - done)
            except L.LbmError as e:
                if e.code != L.LBM_EUNSTABLE:
                    raise
                stable, t_fail = False, lat.step_count / t0
                break
            done = target
            _, _, d = lat.moments(want_fields=False)
            if not np.isfinite(d[4]):
                stable, t_fail = False, done / t0
                break
            t.append(done / t0)
            ke.append(d[4] / ke0)
        return {"t": np.array(t), "ke": np.array(ke), "stable": stable, "t_fail": t_fail, "steps_per_t0": t0}
    finally:
        lat.close()


VARIANTS = (("q19_rm", 19, "raw"), ("q19_cm", 19, "central"), ("q27_rm", 27, "raw"), ("q27_cm", 27, "central"))


def cost_table(sizes=(32, 48, 64, 96, 128), precision: str = "fp32", steps: int = 200, warmup: int = 20):
    """Time per step (HIP events on the lattice's stream) of each variant at
    each D, A-B streaming, default launch; and the paper's normalisation: cost
    of a whole run with T_ite proportional to D (acoustic scaling), relative to
    D3Q19 raw moments at the smallest D."""
    import torch

    ms = {}
    for D in sizes:
        rho, u = inputs.taylor_green_noise(D, 0.2 * CS, 0.0)
        for name, q, mom in VARIANTS:
            _, _, om, _ = parameters(D, 1600.0, 0.2)
            lat = L.Lattice(L.make_params(D, D, D, precision=precision, q=q, omega=om, moments=mom))
            lat.init(rho, u)
            lat.step(warmup)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(lat.stream)
            lat.step(steps)
            b.record(lat.stream)
            torch.cuda.synchronize()
            ms[(D, name)] = a.elapsed_time(b) / steps
            lat.close()
    base = ms[(sizes[0], "q19_rm")] * sizes[0]
    rows = []
    for D in sizes:
        rows.append({"D": D, **{name: round(ms[(D, name)] * D / base, 3) for name, _, _ in VARIANTS},
                     "ms_per_step": {name: round(ms[(D, name)], 5) for name, _, _ in VARIANTS},
                     "mlups": {name: round(D ** 3 / (ms[(D, name)] * 1e-3) / 1e6, 1) for name, _, _ in VARIANTS}})
    big = sizes[-1]
    ratios = {"q27_cm/q19_cm": round(ms[(big, "q27_cm")] / ms[(big, "q19_cm")], 3),
              "q19_cm/q19_rm": round(ms[(big, "q19_cm")] / ms[(big, "q19_rm")], 3),
              "q27_cm/q27_rm": round(ms[(big, "q27_cm")] / ms[(big, "q27_rm")], 3)}
    return {"precision": precision, "rows": rows, "ratios_at_largest_D": ratios}

