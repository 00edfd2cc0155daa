"""Seeded synthetic input fields shared by the GPU path, the tests and the bench.

This module holds no arithmetic of the lattice Boltzmann method itself: it
only builds the initial macroscopic fields (density, velocity) and body-force
fields that define a problem, in float64 numpy arrays with the node layout
n = x + nx*(y + ny*z), i.e. arrays shaped (nz, ny, nx) and (3, nz, ny, nx).

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), keyed by (seed, node,
component), so any subset of nodes can be regenerated independently.
"""
from __future__ import annotations

import numpy as np

_GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to state x + golden gamma (uint64)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform_pm1(seed: int, node: np.ndarray, comp: int) -> np.ndarray:
    """Uniform numbers in [-1, 1) keyed by (seed, node index, component)."""
    with np.errstate(over="ignore"):
        key = (np.uint64(seed) * np.uint64(0xD1B54A32D192ED03)) ^ (
            np.asarray(node, dtype=np.uint64) * np.uint64(4) + np.uint64(comp))
        bits = splitmix64(splitmix64(key))
    return (bits >> np.uint64(11)).astype(np.float64) * (2.0 / 2.0 ** 53) - 1.0


def omega_from_nu(nu: float) -> float:
    """Shear relaxation rate for kinematic viscosity nu, cs^2 = 1/3."""
    return 1.0 / (3.0 * nu + 0.5)


def shear_wave(n: int = 32, amp: float = 0.01, nx: int | None = None, ny: int | None = None):
    """rho = 1, u_x(z) = amp sin(2 pi z / n), u_y = u_z = 0 on nx*ny*n nodes."""
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    z = np.arange(n, dtype=np.float64)
    rho = np.ones((n, ny, nx))
    u = np.zeros((3, n, ny, nx))
    u[0] = (amp * np.sin(2.0 * np.pi * z / n))[:, None, None]
    return rho, u


def taylor_green_noise(L: int, U0: float = 0.05, noise: float = 1e-4, seed: int = 20101628,
                       shape: tuple[int, int, int] | None = None):
    """3D Taylor-Green field u0 (cos x sin y sin z, -1/2 sin x cos y sin z,
    -1/2 sin x sin y cos z), x = 2 pi i / L at node index i, plus uniform
    noise in [-noise, noise] per component; rho = 1."""
    nx, ny, nz = shape if shape is not None else (L, L, L)
    x = 2.0 * np.pi * np.arange(nx) / L
    y = 2.0 * np.pi * np.arange(ny) / L
    z = 2.0 * np.pi * np.arange(nz) / L
    sx, cx = np.sin(x)[None, None, :], np.cos(x)[None, None, :]
    sy, cy = np.sin(y)[None, :, None], np.cos(y)[None, :, None]
    sz, cz = np.sin(z)[:, None, None], np.cos(z)[:, None, None]
    u = np.empty((3, nz, ny, nx))
    u[0] = U0 * cx * sy * sz
    u[1] = -0.5 * U0 * sx * cy * sz
    u[2] = -0.5 * U0 * sx * sy * cz
    if noise:
        nodes = np.arange(nx * ny * nz, dtype=np.uint64).reshape(nz, ny, nx)
        for d in range(3):
            u[d] += noise * uniform_pm1(seed, nodes, d)
    rho = np.ones((nz, ny, nx))
    return rho, u


def kolmogorov_force(nx: int, ny: int, nz: int, amp: float = 1e-6) -> np.ndarray:
    """Body-force density F_x = amp sin(2 pi y / ny), F_y = F_z = 0; (3,nz,ny,nx)."""
    F = np.zeros((3, nz, ny, nx))
    F[0] = (amp * np.sin(2.0 * np.pi * np.arange(ny) / ny))[None, :, None]
    return F


def uniform_force(nx: int, ny: int, nz: int, F) -> np.ndarray:
    out = np.zeros((3, nz, ny, nx))
    for d in range(3):
        out[d] = F[d]
    return out


def random_lattice_fields(nx: int, ny: int, nz: int, seed: int, umax: float = 0.05,
                          drho: float = 0.05, fmax: float = 0.0):
    """Random (rho, u, F) fields for parity tests that exercise every wrap."""
    nodes = np.arange(nx * ny * nz, dtype=np.uint64).reshape(nz, ny, nx)
    rho = 1.0 + drho * uniform_pm1(seed, nodes, 3)
    u = np.stack([umax * uniform_pm1(seed, nodes, d) for d in range(3)])
    F = np.stack([fmax * uniform_pm1(seed + 1, nodes, d) for d in range(3)])
    return rho, u, F


def random_phase_field(L: int, u_rms: float = 0.04, seed: int = 0, k0: float = 4.0, shape=None):
    """Solenoidal velocity field with random phases and energy spectrum
    E(k) ~ k^4 exp(-2 (k/k0)^2) on a periodic box, rescaled so that
    sqrt(<|u|^2>/3) = u_rms; rho = 1.  Built from seeded white noise filtered
    in Fourier space (numpy FFT) and projected onto zero divergence."""
    nx, ny, nz = shape if shape is not None else (L, L, L)
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((3, nz, ny, nx))
    U = np.fft.fftn(noise, axes=(1, 2, 3))
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.fftfreq(nx) * nx
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    k2 = KX ** 2 + KY ** 2 + KZ ** 2
    k = np.sqrt(k2)
    # white noise has a flat |U|^2 per mode; E(k) = 4 pi k^2 |U(k)|^2 ~ k^4 exp(-2 (k/k0)^2)
    amp = np.where(k > 0, k * np.exp(-(k / k0) ** 2), 0.0)
    U *= amp[None]
    kd = np.where(k2 > 0, k2, 1.0)
    div = (KX * U[0] + KY * U[1] + KZ * U[2]) / kd
    U[0] -= KX * div
    U[1] -= KY * div
    U[2] -= KZ * div
    u = np.real(np.fft.ifftn(U, axes=(1, 2, 3)))
    u -= u.mean(axis=(1, 2, 3), keepdims=True)
    u *= u_rms / np.sqrt(np.mean(np.sum(u ** 2, axis=0)) / 3.0)
    return np.ones((nz, ny, nx)), u


def ensemble_boxes(n_boxes: int = 64, sizes=(48, 64, 96), nu_range=(1e-4, 1e-3), seed: int = 2010):
    """Seeded box list of the ensemble workload: side lengths drawn from
    `sizes`, viscosities log-uniform in nu_range.  Returns [(L, nu, field_seed)]."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(n_boxes):
        L = int(rng.choice(sizes))
        nu = float(np.exp(rng.uniform(np.log(nu_range[0]), np.log(nu_range[1]))))
        out.append((L, nu, seed * 1000 + b))
    return out


def droplet(shape, R: float, W: float = 4.0, noise: float = 0.0, seed: int = 192, center=None):
    """Phase field of a drop of radius R: phi = 1/2 + 1/2 tanh(2 (R - r)/W)
    (phi = 1 inside), r the distance from `center` (default: the box centre
    (nx/2, ny/2, nz/2); with nz = 1 the drop is a cylinder along z), plus
    seeded uniform noise in [-noise, noise].  shape = (nx, ny, nz);
    returns (nz, ny, nx)."""
    nx, ny, nz = shape
    cx, cy, cz = center if center is not None else (nx / 2, ny / 2, nz / 2 if nz > 1 else 0.0)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    phi = 0.5 + 0.5 * np.tanh(2.0 * (R - r) / W)
    if noise:
        nodes = np.arange(nx * ny * nz, dtype=np.uint64).reshape(nz, ny, nx)
        phi = phi + noise * uniform_pm1(seed, nodes, 0)
    return phi


def slab(shape, thickness: float, W: float = 4.0):
    """Planar layer phi = 1 for |x - nx/2| < thickness/2 (tanh edges of width
    W), uniform in y and z; (nz, ny, nx)."""
    nx, ny, nz = shape
    x = np.arange(nx, dtype=np.float64)
    d = thickness / 2 - np.abs(x - nx / 2)
    phi = 0.5 + 0.5 * np.tanh(2.0 * d / W)
    return np.broadcast_to(phi[None, None, :], (nz, ny, nx)).copy()
