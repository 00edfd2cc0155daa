"""Lattice-level pins of the FP64 oracle: closed forms, linear theory and
conservation laws.  All run on the CPU in a few seconds."""
import numpy as np
import pytest

from paper_2010_01628_amd import inputs

CS2 = 1.0 / 3.0


def printed_M():
    import os

    return np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "d3q19_M_printed.txt"))


def sin_amplitude(ux, n):
    """Projection of u_x(z) on sin(2 pi z / n), averaged over x and y."""
    z = np.arange(n)
    prof = ux.mean(axis=(1, 2))
    return 2.0 / n * np.sum(prof * np.sin(2 * np.pi * z / n)), 2.0 / n * np.sum(prof * np.cos(2 * np.pi * z / n))


def test_shear_wave_tau1_closed_form(orc):
    """32^3 shear wave, nu = 1/6 (w = 1), higher-order rates 1, 200 steps.
    With every rate equal to 1, f* = f_eq(rho, u) and the mode u_x = A sin(kz)
    obeys A(t) = A0 ((2 + cos k)/3)^t exactly while rho stays uniform; the
    continuum decay exp(-nu k^2 t) is within 4e-6 relative after 200 steps."""
    n, A0, steps = 32, 0.01, 200
    k = 2 * np.pi / n
    rho, u = inputs.shear_wave(n, A0)
    f = orc.run(orc.init(rho, u), steps, orc.K(1.0))
    rho_t, u_t = orc.moments(f)
    A, B = sin_amplitude(u_t[0], n)
    exact = A0 * ((2 + np.cos(k)) / 3) ** steps
    assert abs(A - exact) / exact < 1e-12
    assert abs(B) < 1e-15
    assert np.isclose(exact / A0, 0.2766225906958, rtol=0, atol=1e-13)
    nu = 1.0 / 6.0
    assert abs(A - A0 * np.exp(-nu * k * k * steps)) / A < 4e-6
    # uniform density, no transverse flow, mass and momentum conserved
    assert np.abs(rho_t - 1.0).max() < 1e-14
    assert np.abs(u_t[1:]).max() < 1e-15
    assert abs(f.sum() - n ** 3) / n ** 3 < 1e-14
    # u_x independent of x and y
    assert np.abs(u_t[0] - u_t[0].mean(axis=(1, 2), keepdims=True)).max() < 1e-15


def linear_operator(orc, Kdiag, kvec):
    """Linearised one-step map about rest (rho = 1, u = 0, F = 0) for a Fourier
    mode exp(i k.x): stream(S) o collide(C), C = J + M^-1 (I - K) M (I - J),
    J the projection on the linear equilibrium w_i (drho + 3 c_i.dj)."""
    c, w, _ = orc.tables()
    M = printed_M()
    J = w[:, None] * (1.0 + 3.0 * (c @ c.T))
    C = J + np.linalg.solve(M, np.diag(1.0 - Kdiag) @ M) @ (np.eye(19) - J)
    S = np.diag(np.exp(-1j * (c @ kvec)))
    return S @ C


@pytest.mark.parametrize("seed", [0, 1])
def test_linear_modes_match_von_neumann(orc, seed):
    """Any small perturbation of the rest state on an 8^3 periodic lattice
    evolves as L(k)^t (von Neumann analysis) with L built from the printed M
    and the rates alone.  Random rates (w, w_b, w_hi) and a random 19-vector
    of initial perturbations; the symmetric difference of +-A runs cancels the
    even nonlinear orders.  Pins K's row placement, the equilibrium's linear
    part and the streaming direction."""
    rng = np.random.default_rng(seed)
    n, steps, A = 8, 12, 1e-5
    kvec = 2 * np.pi * np.array([1, 2, 3]) / n
    Kd = orc.K(rng.uniform(0.6, 1.9), rng.uniform(0.6, 1.9), rng.uniform(0.6, 1.9, 9))
    c, w, _ = orc.tables()
    v0 = rng.normal(size=19) + 1j * rng.normal(size=19)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    phase = np.exp(1j * (kvec[0] * x + kvec[1] * y + kvec[2] * z))
    pert = np.real(v0[:, None, None, None] * phase[None])
    runs = []
    for sgn in (+1, -1):
        f0 = w[:, None, None, None] + sgn * A * pert
        runs.append(orc.run(f0, steps, Kd))
    lin = (runs[0] - runs[1]) / (2 * A)
    vt = np.linalg.matrix_power(linear_operator(orc, Kd, kvec), steps) @ v0
    want = np.real(vt[:, None, None, None] * phase[None])
    assert np.abs(lin - want).max() / np.abs(want).max() < 1e-7


def test_shear_wave_general_rate_linear_theory(orc):
    """Shear wave at nu = 0.05 (w ~ 1.538) on 2x2x32: the u_x amplitude follows
    the linearised operator, while the continuum law is off by ~0.3 %."""
    n, A0, steps, nu = 32, 1e-4, 200, 0.05
    om = inputs.omega_from_nu(nu)
    kz = 2 * np.pi / n
    rho, u = inputs.shear_wave(n, A0, nx=2, ny=2)
    Kd = orc.K(om)
    f = orc.run(orc.init(rho, u), steps, Kd)
    _, ut = orc.moments(f)
    A, B = sin_amplitude(ut[0], n)
    c, w, _ = orc.tables()
    v0 = 3.0 * w * c[:, 0]  # linear part of f_eq for u_x = Im(exp(ikz))
    vt = np.linalg.matrix_power(linear_operator(orc, Kd, np.array([0.0, 0.0, kz])), steps) @ v0
    a = np.sum(c[:, 0] * vt)
    assert abs(A / A0 - a.real) < 1e-7
    assert abs(B / A0 - a.imag) < 1e-7
    cont = np.exp(-nu * kz * kz * steps)
    assert 1e-3 < abs(A / A0 - cont) / cont < 1e-2


@pytest.mark.parametrize("mode", [0, 2])
def test_lattice_conservation_with_random_force(orc, mode):
    """Random 6x5x7 lattice, random force field, random rates: total mass is
    conserved to round-off and total momentum sum f c grows by exactly sum F."""
    nx, ny, nz = 6, 5, 7
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=5, umax=0.05, fmax=1e-3)
    rng = np.random.default_rng(3)
    Kd = orc.K(rng.uniform(0.5, 1.9), rng.uniform(0.5, 1.9), rng.uniform(0.5, 1.9, 9))
    c, _, _ = orc.tables()
    f = orc.init(rho, u)
    m0 = f.sum()
    for _ in range(5):
        p0 = np.einsum("iabc,id->d", f, c)
        f = orc.step(f, Kd, F=F, mode=mode)
        p1 = np.einsum("iabc,id->d", f, c)
        assert np.allclose(p1 - p0, F.reshape(3, -1).sum(axis=1), rtol=0, atol=1e-13)
        assert abs(f.sum() - m0) / m0 < 1e-14


def test_uniform_flow_is_steady_and_translation(orc):
    """Galilean check: a uniform flow at equilibrium is an exact steady state
    for any rates, and a stream-wise translated field stays translated."""
    nx, ny, nz = 4, 3, 5
    rho = np.full((nz, ny, nx), 1.03)
    u = np.zeros((3, nz, ny, nx))
    u[0], u[1], u[2] = 0.07, -0.04, 0.02
    Kd = orc.K(1.93, 0.7, np.full(9, 1.4))
    f0 = orc.init(rho, u)
    f = orc.run(f0, 7, Kd)
    assert np.abs(f - f0).max() < 1e-15


def test_halfway_bounce_back_poiseuille(orc):
    """Walls at y = -1/2 and y = ny - 1/2 (halfway bounce-back), uniform force
    F_x, w = 1: the steady profile matches the parabola
    u(y) = F (y + 1/2)(ny - 1/2 - y) / (2 rho nu) within 1 % of its maximum,
    mass is conserved and the wall shear balances the body force."""
    ny, Fx = 16, 1e-6
    nu = 1.0 / 6.0
    rho = np.ones((1, ny, 1))
    u = np.zeros((3, 1, ny, 1))
    F = inputs.uniform_force(1, ny, 1, (Fx, 0.0, 0.0))
    Kd = orc.K(inputs.omega_from_nu(nu))
    f = orc.init(rho, u)
    m0 = f.sum()
    f = orc.run(f, 4000, Kd, F=F, walls_y=True)
    r, ut = orc.moments(f, F)
    y = np.arange(ny)
    exact = Fx * (y + 0.5) * (ny - 0.5 - y) / (2 * nu)
    prof = ut[0, 0, :, 0]
    assert np.abs(prof - exact).max() < 1e-2 * exact.max()
    # mirror symmetry about the channel centre: a wrong wall index breaks it at
    # O(1e-2); round-off of the O(0.1) populations (~1e-17 per step, carried
    # by the pivoted solve's non-mirror-symmetric order) builds up to ~3e-12
    # of the maximum over the 4000 steps
    assert np.allclose(prof, prof[::-1], rtol=0, atol=1e-10 * exact.max())
    assert abs(f.sum() - m0) < 1e-13
    # steady: one more step changes nothing (to the decay of the slowest mode)
    g = orc.step(f, Kd, F=F, walls_y=True)
    assert np.abs(g - f).max() < 1e-12


def test_step_at_matches_full_step(orc):
    """The sampled single-step routine equals the full lattice step at every node."""
    nx, ny, nz = 5, 6, 4
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=21, umax=0.05, fmax=1e-3)
    Kd = orc.K(1.6, 1.1, np.linspace(0.9, 1.2, 9))
    for walls in (False, True):
        f = orc.run(orc.init(rho, u), 3, Kd, F=F, walls_y=walls)
        full = orc.step(f, Kd, F=F, walls_y=walls)
        nodes = np.arange(nx * ny * nz)
        got = orc.step_at(f, nodes, Kd, F=F, walls_y=walls)
        assert np.array_equal(got, full.reshape(19, -1).T)
