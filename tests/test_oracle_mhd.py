"""Pins of the magnetohydrodynamics oracle (D3Q7 vector magnetic lattice
coupled to the D3Q19 CM flow) against facts outside its own code: moments of
the magnetic equilibrium, the current of a measured field against curl b,
magnetic diffusion against the linear (von Neumann) mode of the lattice
computed with numpy, reduction to the paper's scheme without a field, flux
conservation, and the Hartmann profile and amplitude."""
import numpy as np
import pytest

import oracle
from paper_2010_01628_amd import inputs

M = oracle.mhd
rng = np.random.default_rng(569)
C7 = np.array([[0, 0, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
W7 = np.array([0.25] + [0.125] * 6)


def test_equilibrium_moments():
    """sum_i g_eq = b, sum_i c g_eq = u b - b u (the induction flux), second
    moment cs^2 b I with cs^2 = 1/4."""
    for _ in range(5):
        b = rng.normal(size=3) * 0.1
        u = rng.normal(size=3) * 0.05
        ge = M.geq(b, u)  # [a, i]
        assert np.allclose(ge.sum(axis=1), b, atol=1e-16)
        lam = np.einsum("ic,ai->ca", C7, ge)
        assert np.allclose(lam, np.outer(u, b) - np.outer(b, u), atol=1e-16)
        m2 = np.einsum("ic,id,ai->acd", C7, C7, ge)
        for a in range(3):
            assert np.allclose(m2[a], 0.25 * b[a] * np.eye(3), atol=1e-16)


def test_current_is_curl_b():
    """After the non-equilibrium has settled, j from the non-equilibrium
    moments equals curl b of the measured field (spectral derivative):
    b = (0, A sin(kx), A sin(kz)) gives j = (A k cos(kz)... ) per component."""
    n = 64
    eta, A = 0.05, 1e-4
    prm = M.params(eta)
    k = 2 * np.pi / n
    x = np.arange(n)
    b = np.zeros((3, n, 1, n))  # (3, nz, ny, nx), ny = 1
    b[1] = (A * np.sin(k * x))[None, None, :]  # b_y(x): curl_z = d_x b_y
    b[0] = (A * np.cos(k * x))[:, None, None]  # b_x(z): curl_y = d_z b_x
    f, g = M.init(np.ones((n, 1, n)), np.zeros((3, n, 1, n)), b)
    f, g = M.run(prm, 1.0, f, g, 40)
    _, _, bb, jj = M.fields(prm, f, g)
    kx = np.fft.fftfreq(n) * 2 * np.pi
    dby_dx = np.real(np.fft.ifft(1j * kx[None, None, :] * np.fft.fft(bb[1], axis=2), axis=2))
    dbx_dz = np.real(np.fft.ifft(1j * kx[:, None, None] * np.fft.fft(bb[0], axis=0), axis=0))
    err_z = np.linalg.norm(jj[2] - dby_dx) / np.linalg.norm(dby_dx)
    err_y = np.linalg.norm(jj[1] - dbx_dz) / np.linalg.norm(dbx_dz)
    assert err_z < 2e-2 and err_y < 2e-2, (err_z, err_y)
    assert np.abs(jj[0]).max() < 1e-3 * np.abs(jj[2]).max()


def test_magnetic_diffusion_matches_linear_mode():
    """Fluid at rest, b_x = A sin(kz) with A tiny (the Lorentz force is O(A^2)):
    the field decays exactly as the linear mode of the D3Q7 BGK lattice,
    computed here as a 7x7 matrix power with numpy."""
    n, T, eta, A = 16, 60, 0.08, 1e-6
    wm = M.omega_m(eta)
    k = 2 * np.pi / n
    z = np.arange(n)
    b = np.zeros((3, n, 1, 1))
    b[0] = (A * np.sin(k * z))[:, None, None]
    f, g = M.init(np.ones((n, 1, 1)), np.zeros((3, n, 1, 1)), b)
    f, g = M.run(M.params(eta), 1.0, f, g, T)
    _, _, bb, _ = M.fields(M.params(eta), f, g)
    amp = 2 * np.abs(np.fft.fft(bb[0, :, 0, 0])[1]) / n
    Cm = (1 - wm) * np.eye(7) + wm * np.outer(W7, np.ones(7))
    S = np.diag(np.exp(-1j * k * C7[:, 2]))
    G = np.linalg.matrix_power(S @ Cm, T) @ W7
    want = A * np.abs(G.sum())
    assert abs(amp - want) < 1e-6 * want, (amp, want)
    # and the continuum rate is close (not exact): exp(-eta k^2 T)
    assert abs(amp / A - np.exp(-eta * k * k * T)) < 0.05


@pytest.mark.parametrize("walls", [False, True])
def test_zero_field_is_paper_scheme(orc, walls):
    nx, ny, nz = 8, 6, 5
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=4, umax=0.04, fmax=1e-4)
    om = 1.6
    f, g = M.init(rho, u, np.zeros((3, nz, ny, nx)))
    f, g = M.run(M.params(0.1), om, f, g, 7, F=F, walls_y=walls)
    want = orc.run(orc.init(rho, u), 7, orc.K(om), F=F, walls_y=walls)
    assert np.abs(f - want).max() < 1e-15
    assert np.abs(g).max() == 0.0


def test_magnetic_flux_conserved():
    nx, ny, nz = 9, 7, 6
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=8, umax=0.03)
    b = np.stack([0.02 * inputs.uniform_pm1(9, np.arange(nx * ny * nz, dtype=np.uint64), d).reshape(nz, ny, nx)
                  for d in range(3)])
    f, g = M.init(rho, u, b)
    f, g = M.run(M.params(0.07), 1.4, f, g, 25)
    _, _, bb, _ = M.fields(M.params(0.07), f, g)
    assert np.allclose(bb.sum(axis=(1, 2, 3)), b.sum(axis=(1, 2, 3)), rtol=0, atol=1e-14)


def hartmann(ny=128, Ha=10.0, nu=0.1, eta=0.1, u_max=0.02):
    """Hartmann channel (walls at y = -1/2, ny - 1/2; field b_y0 imposed there),
    width L = ny, Ha = b_y0 L / sqrt(4 rho nu eta); body force for the given
    u_max with b_x = 0 on both walls: u_max = (F eta / b0^2)(Ha / tanh Ha)(1 - 1/cosh Ha)."""
    b0 = Ha * 2 * np.sqrt(nu * eta) / ny
    F = u_max * b0 ** 2 * np.tanh(Ha) / (eta * Ha * (1 - 1 / np.cosh(Ha)))
    y = np.arange(ny)
    yp = 2 * (y + 0.5) - ny
    shape = (1 - np.cosh(Ha * yp / ny) / np.cosh(Ha)) / (1 - 1 / np.cosh(Ha))
    return b0, F, shape


def test_hartmann_profile():
    ny, Ha, nu, eta = 128, 10.0, 0.1, 0.1
    b0, F, shape = hartmann(ny, Ha, nu, eta)
    prm = M.params(eta, (0.0, b0, 0.0))
    b = np.zeros((3, 1, ny, 1))
    b[1] = b0
    Fx = np.zeros((3, 1, ny, 1))
    Fx[0] = F
    f, g = M.init(np.ones((1, ny, 1)), np.zeros((3, 1, ny, 1)), b)
    f, g = M.run(prm, 1.0 / (3 * nu + 0.5), f, g, 30000, F=Fx, walls_y=True)
    _, u, bb, _ = M.fields(prm, f, g, F=Fx)
    ux = u[0, 0, :, 0]
    err = np.linalg.norm(ux / ux.max() - shape) / np.linalg.norm(shape)
    print(f"Hartmann: shape rel L2 {err:.2e}, u_max {ux.max():.6f} (analytic 0.02)")
    assert err < 1e-3
    assert abs(ux.max() / 0.02 - 1) < 5e-3
    assert np.abs(bb[1] - b0).max() < 1e-6 * b0  # div b = 0 keeps b_y uniform
