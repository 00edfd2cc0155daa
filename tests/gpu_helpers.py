"""Shared helpers of the GPU parity tests (run GPU lattice, run oracle, compare)."""
import sys

import numpy as np

from paper_2010_01628_amd import inputs
from paper_2010_01628_amd import lbm as L


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


def rel_l2_fluct(rho_a, rho_b):
    """relative L2 of rho - mean(rho), the meaningful density error."""
    da = rho_a - rho_a.mean()
    db = rho_b - rho_b.mean()
    return float(np.linalg.norm((da - db).ravel()) / max(np.linalg.norm(db.ravel()), 1e-300))


def gpu_run(nx, ny, nz, rho, u, steps, precision="fp64", streaming="ab", omega=1.0, omega_bulk=1.0,
            omega_hi=None, force=None, force_mode=L.LBM_FORCE_NONE, kolmogorov_amp=0.0, walls=False,
            uniform=(0.0, 0.0, 0.0), block=(0, 0), want_pops=True, q=19, moments="central", rounding="nearest",
            cache_policy=0):
    """Run the GPU library; returns dict(rho, u, f, diag) as numpy float64."""
    import torch

    ff = None
    if force is not None:
        ff = torch.from_numpy(np.ascontiguousarray(force, dtype=np.float64)).cuda()
        force_mode = L.LBM_FORCE_FIELD
    p = L.make_params(nx, ny, nz, precision=precision, streaming=streaming, omega=omega, omega_bulk=omega_bulk,
                      omega_hi=omega_hi, force_mode=force_mode, force=uniform, kolmogorov_amp=kolmogorov_amp,
                      force_field_ptr=None if ff is None else ff.data_ptr(), walls_y=walls, block=block,
                      moments=moments, rounding=rounding, seed=20101628, cache_policy=cache_policy)
    p.q = q
    lat = L.Lattice(p, force_field=ff)
    try:
        lat.init(rho, u)
        lat.step(steps)
        r, v, diag = lat.moments()
        out = {"rho": r.cpu().numpy(), "u": v.cpu().numpy(), "diag": diag}
        if want_pops:
            out["f"] = lat.get_populations().cpu().numpy()
        torch.cuda.synchronize()
        return out
    finally:
        lat.close()


def oracle_run(orc, rho, u, steps, omega=1.0, omega_bulk=1.0, omega_hi=None, F=None, walls=False,
               mode=None):
    Kd = orc.K(omega, omega_bulk, omega_hi)
    f = orc.run(orc.init(rho, u), steps, Kd, F=F, walls_y=walls, mode=orc.DEFINITION if mode is None else mode)
    r, v = orc.moments(f, F)
    return {"rho": r, "u": v, "f": f}
