"""Rayleigh-Taylor instability of Sec. III with the colour-gradient lattice of
App. E: a heavy fluid (rho_h = 3, red) over a light one (rho_l = 1, blue) in a
W x 4W x W box with no-slip walls at the bottom and top, periodic sideways,
gravity along -y with sqrt(g W) = 0.04, Re = W sqrt(g W) / nu = 512,
At = 0.5.  Reports the spike (the lowest point of the heavy fluid, on the
column x = z = W/2 where the initial interface is lowest) in units of W at
t / t0 = 0, 0.5, ..., 4, t0 = W / sqrt(g W).

Only orders library calls: every lattice operation runs in the HIP library.
"""
from __future__ import annotations

import numpy as np

from . import lbm as L

RHO_H, RHO_L = 3.0, 1.0
ALPHA_B = 1.0 / 3.0
ALPHA_R = 1.0 - (1.0 - ALPHA_B) * RHO_L / RHO_H  # rho_h (1 - alpha_r) = rho_l (1 - alpha_b)


def setup(W: int = 64, Re: float = 512.0, u_ref: float = 0.04, precision: str = "fp32", beta: float = 0.7,
          A: float = 0.0):
    """(params, rho_red, rho_blue, steps per t0)."""
    nx, ny, nz = W, 4 * W, W
    g = u_ref * u_ref / W
    nu = W * u_ref / Re
    omega = 1.0 / (3.0 * nu + 0.5)
    p = L.make_params(nx, ny, nz, precision=precision, omega=omega, walls_y=True,
                      colour=dict(alpha_red=ALPHA_R, alpha_blue=ALPHA_B, A=A, beta=beta, gravity=(0.0, -g, 0.0),
                                  rho_ref=0.5 * (RHO_H + RHO_L)))
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    top = y > 2 * W + 0.05 * W * (np.cos(2 * np.pi * x / W) + np.cos(2 * np.pi * z / W))
    rr = np.where(top, RHO_H, 0.0)
    rb = np.where(top, 0.0, RHO_L)
    return p, rr, rb, W / u_ref


def spike(rho_red, rho_blue, W: int) -> float:
    """Lowest crossing of phi = 0 on the column x = z = W/2, in units of W
    (node y, linear interpolation between nodes)."""
    c = W // 2
    rr = np.asarray(rho_red)[c, :, c]
    rb = np.asarray(rho_blue)[c, :, c]
    phi = (rr - rb) / (rr + rb)
    for y in range(len(phi) - 1):
        if phi[y] <= 0.0 < phi[y + 1]:
            return (y + phi[y] / (phi[y] - phi[y + 1])) / W
    return float("nan")


def run(W: int = 64, times=(0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0), precision: str = "fp32", **kw):
    """Spike positions at the given t / t0; returns (times, positions)."""
    import torch

    p, rr, rb, t0 = setup(W, precision=precision, **kw)
    lat = L.Lattice(p)
    try:
        lat.init_colour(rr, rb, np.zeros((3,) + rr.shape))
        out = []
        done = 0
        for t in times:
            target = int(round(t * t0))
            if target > done:
                lat.step(target - done)
                done = target
            a, b = lat.colour_fields()
            out.append(spike(a.cpu().numpy(), b.cpu().numpy(), W))
        torch.cuda.synchronize()
        return np.array(times), np.array(out)
    finally:
        lat.close()
