"""Design check of the z-slab decomposition (CPU, oracle only).

A periodic lattice split into G z-slabs, each advancing only its own planes,
reproduces the unsplit run bit for bit when, before every step, each slab
receives from its two neighbours only the five populations that cross the
shared face: with pull streaming a node at the slab's lowest plane reads
f*_i(x - c_i) one plane below for the five c_i with c_z = +1, and the highest
plane one plane above for the five with c_z = -1.  The other 14 populations
of a boundary plane never leave their slab, so the halo is 5 x nx x ny values
per face and direction.

State here, as in the GPU's A-B storage, is the post-collision field P_i(x)
(pre-collision f_i(x) = P_i(x - c_i)).  Each slab's collision uses the
oracle's step on the slab's own planes: its push streaming wraps within the
slab, which this test undoes (a pure permutation), so only the collision --
local to each node -- is taken from it.
"""
import numpy as np
import pytest

from paper_2010_01628_amd import inputs


def pull(P, c, lo=None, hi=None):
    """Pre-collision f_i(x) = P_i(x - c_i) on a slab's planes (axis order
    z, y, x), periodic in x and y; across z from the halo planes lo (one
    plane below, only the populations with c_z = +1 are read) and hi (one
    plane above, c_z = -1).  lo = hi = None: periodic in z as well."""
    out = np.empty_like(P)
    for i in range(19):
        cx, cy, cz = c[i]
        s = np.roll(P[i], shift=(cy, cx), axis=(1, 2))
        if lo is None:
            out[i] = np.roll(s, shift=cz, axis=0)
        elif cz == 0:
            out[i] = s
        elif cz == 1:
            out[i, 1:] = s[:-1]
            out[i, 0] = np.roll(lo[i], shift=(cy, cx), axis=(0, 1))
        else:
            out[i, :-1] = s[1:]
            out[i, -1] = np.roll(hi[i], shift=(cy, cx), axis=(0, 1))
    return out


def collide_only(orc, f, Kd, F):
    """Post-collision populations at each node: the oracle's step (collide,
    then push with periodic wrap inside the array) followed by the inverse
    of that push."""
    c, _, _ = orc.tables()
    g = orc.step(f, Kd, F=F)
    return np.stack([np.roll(g[i], shift=(-c[i, 2], -c[i, 1], -c[i, 0]), axis=(0, 1, 2)) for i in range(19)])


@pytest.mark.parametrize("nz,cuts", [(12, (6,)), (12, (4, 8)), (12, (3, 6, 9)), (10, (4, 7))])
def test_slab_split_with_five_population_halos_is_bitwise(orc, nz, cuts):
    nx, ny, steps = 6, 5, 4
    c, _, _ = orc.tables()
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=31, umax=0.06, drho=0.02)
    F = inputs.kolmogorov_force(nx, ny, nz, 2e-4)
    Kd = orc.K(1.7, omega_bulk=1.3)
    # post-collision field of the first step, the state both runs start from
    P0 = collide_only(orc, orc.init(rho, u), Kd, F)

    # unsplit
    P = P0.copy()
    for _ in range(steps):
        P = collide_only(orc, pull(P, c), Kd, F)

    # split: slab g owns planes [b[g], b[g+1])
    b = [0, *cuts, nz]
    G = len(b) - 1
    slabs = [P0[:, b[g]:b[g + 1]].copy() for g in range(G)]
    up = [i for i in range(19) if c[i, 2] == 1]
    down = [i for i in range(19) if c[i, 2] == -1]
    assert len(up) == len(down) == 5
    halo_values = 0
    for _ in range(steps):
        # exchange: only the five crossing populations of each boundary plane
        lo, hi = [], []
        for g in range(G):
            below, above = slabs[(g - 1) % G], slabs[(g + 1) % G]
            L = np.full((19, ny, nx), np.nan)  # populations never read stay NaN
            H = np.full((19, ny, nx), np.nan)
            L[up] = below[up, -1]
            H[down] = above[down, 0]
            halo_values += 2 * 5 * nx * ny
            lo.append(L)
            hi.append(H)
        slabs = [collide_only(orc, pull(slabs[g], c, lo[g], hi[g]), Kd, F[:, b[g]:b[g + 1]]) for g in range(G)]
    assert np.array_equal(np.concatenate(slabs, axis=1), P)
    assert halo_values == steps * G * 2 * 5 * nx * ny


def test_slab_split_detects_a_missing_population(orc):
    """The check is sharp: leaving out one crossing population of the halo
    (it stays NaN) spoils the split run."""
    nx, ny, nz = 6, 5, 8
    c, _, _ = orc.tables()
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=32, umax=0.06, drho=0.02)
    Kd = orc.K(1.6)
    P0 = collide_only(orc, orc.init(rho, u), Kd, None)
    up = [i for i in range(19) if c[i, 2] == 1]
    down = [i for i in range(19) if c[i, 2] == -1]
    a, bb = P0[:, :4], P0[:, 4:]
    L = np.full((19, ny, nx), np.nan)
    H = np.full((19, ny, nx), np.nan)
    L[up[1:]] = bb[up[1:], -1]  # one of the five left out
    H[down] = bb[down, 0]
    out = collide_only(orc, pull(a, c, L, H), Kd, None)
    assert np.isnan(out[:, 0]).any() and not np.isnan(out[:, 1:-1]).any()
