"""Pins of the colour-gradient oracle (App. E on the paper's D3Q19 CM
collision; readings G1-G6) against facts outside its own code: moments of
the weights phi_i, the printed post-collision central moments of h_eq, the
reduction to the paper's scheme for one colour, conservation, the moments of
the perturbation operator in closed form, the recolouring's conservation and
direction, the pressure balance of a flat interface at rest, the linear
(von Neumann) operator of a pure colour with its sound speed, and the
Young-Laplace law with the printed sigma = (2/9) A / omega."""
import numpy as np
import pytest

import oracle

C = oracle.colour_gradient
CS2 = 1.0 / 3.0


def c2_of(c):
    return (c * c).sum(axis=1)


@pytest.mark.parametrize("alpha", [0.0, 1.0 / 3.0, 0.6, 7.0 / 9.0])
def test_phi_weights_moments(orc, alpha):
    """sum phi_i = 1, sum phi_i c_i = 0, sum phi_i c_i c_i = (1 - alpha)/2 I:
    the equation of state p = rho (1 - alpha)/2; alpha = 1/3 gives w_i."""
    c, w, _ = orc.tables()
    phi = np.array([C.phi_i(k, alpha) for k in c2_of(c)])
    assert abs(phi.sum() - 1) < 1e-15
    assert np.abs(phi @ c).max() < 1e-16
    assert np.allclose(np.einsum("i,ia,ib->ab", phi, c, c), 0.5 * (1 - alpha) * np.eye(3), atol=1e-16)
    if alpha == 1.0 / 3.0:
        assert np.allclose(phi, w, atol=1e-16)


def test_heq_central_moments_match_printed_list(orc):
    """App. E's post-collision CMs of the equilibrium part: k4 = 3 rho (1 -
    alpha)/2, k10..15 = rho u (3 alpha - 1)/6 (with the u component of each
    printed row), k16..18 = rho [1 + ua^2 + ub^2 - alpha (1 + 3 ua^2 + 3 ub^2)]
    / 6 (the factor 1/6 restored: without it alpha = 1/3 would give 2 rho/3
    instead of the rho cs^4 of the standard equilibrium), deviatoric and
    mixed second-order ones 0."""
    rng = np.random.default_rng(2)
    for _ in range(30):
        rho = rng.uniform(0.5, 3.0)
        u = rng.uniform(-0.1, 0.1, 3)
        alpha = rng.uniform(0.0, 0.9)
        k = orc.T(u) @ C.heq(rho, u, alpha)
        ux, uy, uz = u
        assert abs(k[0] - rho) < 1e-14
        assert np.abs(k[1:4]).max() < 1e-15
        assert abs(k[4] - 1.5 * rho * (1 - alpha)) < 1e-14
        assert np.abs(k[5:10]).max() < 1e-15
        t = rho * (3 * alpha - 1) / 6
        assert np.allclose(k[10:16], [t * uy, t * ux, t * uz, t * ux, t * uz, t * uy], atol=1e-15)
        row = lambda a, b: rho * (1 + a * a + b * b - alpha * (1 + 3 * a * a + 3 * b * b)) / 6
        assert np.allclose(k[16:19], [row(ux, uy), row(ux, uz), row(uy, uz)], atol=1e-15)


@pytest.mark.parametrize("walls", [False, True])
def test_single_colour_is_the_papers_scheme(orc, walls):
    """Blue only with alpha_b = 1/3: h_eq = f_eq, phi = -1 everywhere (no
    perturbation, no recolouring bias): the paper's step with the body force
    (rho - rho_ref) g, to FP64 round-off (the two sides reach f_eq and f* by
    different linear solves, each rounding at ~1e-16 times the condition
    number of T(u), about 10)."""
    from paper_2010_01628_amd import inputs

    nx, ny, nz = 6, 5, 4
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=12, umax=0.05)
    g, rref = np.array([1e-4, -2e-4, 5e-5]), 1.02
    prm = C.params(1.6, 7.0 / 9.0, A=0.01, g=g, rho_ref=rref)
    fr, fb = C.init(prm, np.zeros_like(rho), rho, u)
    F = (rho - rref)[None] * g[:, None, None, None]
    want = orc.step(orc.init(rho, u), orc.K(1.6), F=F, walls_y=walls)
    ar, ab = C.step(prm, fr, fb, walls_y=walls)
    assert np.abs(ar).max() == 0.0
    assert np.abs(ab - want).max() < 5e-15


def random_mixture(shape, seed):
    from paper_2010_01628_amd import inputs

    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    s = np.tanh(np.sin(2 * np.pi * x / nx) + np.cos(2 * np.pi * y / ny) * 0.8 + 0.3 * np.sin(2 * np.pi * z / nz))
    rr = 1.5 * (1 + s) + 1e-3 * rng.uniform(size=s.shape)
    rb = 0.5 * (1 - s) + 1e-3 * rng.uniform(size=s.shape)
    _, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=seed, umax=0.03)
    return rr, rb, u


def test_colour_mass_and_momentum_conserved(orc):
    rr, rb, u = random_mixture((7, 6, 5), 3)
    g = np.array([0.0, -3e-5, 1e-5])
    prm = C.params(1.7, 7.0 / 9.0, A=0.02, g=g, rho_ref=2.0)
    fr, fb = C.init(prm, rr, rb, u)
    c, _, _ = orc.tables()
    mr, mb = fr.sum(), fb.sum()
    j0 = c.T @ (fr + fb).reshape(19, -1).sum(axis=1)
    steps = 10
    Fsum = np.zeros(3)
    for _ in range(steps):
        rho = (fr + fb).sum(axis=0)
        Fsum += (rho - 2.0).sum() * g
        fr, fb = C.step(prm, fr, fb)
    assert abs(fr.sum() - mr) / mr < 1e-14 and abs(fb.sum() - mb) / mb < 1e-14
    j = c.T @ (fr + fb).reshape(19, -1).sum(axis=1)
    assert np.allclose(j - j0, Fsum, atol=1e-12)


def test_perturbation_moments_closed_form(orc):
    """The perturbation added to the total populations has zero mass and
    momentum and second moment -(A/9)|grad phi| (I - n n) (from sum_i w_i
    c_a c_b c_c c_d = cs^4 (delta delta + ...) and sum_i B_i c_a c_b = I/3)."""
    c, _, _ = orc.tables()
    rng = np.random.default_rng(4)
    for _ in range(20):
        rr, rb = rng.uniform(0.2, 2.0, 2)
        rho = rr + rb
        u = rng.uniform(-0.05, 0.05, 3)
        a = 7.0 / 9.0
        h = C.heq(rho, u, (rr * a + rb / 3) / rho) * (1 + 0.02 * rng.uniform(-1, 1, 19))
        fr, fb = rr / rho * h, rb / rho * h
        grad = rng.normal(size=3) * 0.1
        A = rng.uniform(0.001, 0.05)
        p1 = C.params(1.5, a, A=A)
        p0 = C.params(1.5, a, A=0.0)
        d = sum(C.collide(p1, fr, fb, grad)[:2]) - sum(C.collide(p0, fr, fb, grad)[:2])
        gn = np.linalg.norm(grad)
        n = grad / gn
        assert abs(d.sum()) < 1e-15
        assert np.abs(c.T @ d).max() < 1e-15
        want = -(A / 9.0) * gn * (np.eye(3) - np.outer(n, n))
        assert np.allclose(np.einsum("ia,ib,i->ab", c, c, d), want, atol=1e-15)


def test_recolouring_conserves_and_separates(orc):
    """The recolouring leaves the total populations and each colour's mass
    unchanged, and moves red momentum along +grad phi."""
    c, _, _ = orc.tables()
    rng = np.random.default_rng(5)
    for _ in range(20):
        rr, rb = rng.uniform(0.2, 2.0, 2)
        rho = rr + rb
        h = C.heq(rho, rng.uniform(-0.05, 0.05, 3), 0.5) * (1 + 0.02 * rng.uniform(-1, 1, 19))
        fr, fb = rr / rho * h, rb / rho * h
        grad = rng.normal(size=3) * 0.1
        ar, ab, _, _ = C.collide(C.params(1.3, 0.6, beta=0.7), fr, fb, grad)
        br, bb, _, _ = C.collide(C.params(1.3, 0.6, beta=0.0), fr, fb, grad)
        assert np.abs((ar + ab) - (br + bb)).max() < 1e-16
        assert abs(ar.sum() - fr.sum()) < 1e-15 and abs(ab.sum() - fb.sum()) < 1e-15
        assert (c @ grad) @ (ar - br) > 0


def test_flat_interface_at_rest_balances_pressure():
    """A red slab (rho 3, alpha_r = 7/9) in blue (rho 1, alpha_b = 1/3): the
    densities satisfy rho_r (1 - alpha_r) = rho_b (1 - alpha_b), so the layer
    stays at rest with p = rho (1 - alpha)/2 equal in both bulks."""
    nx, ny, nz = 2, 40, 1
    y = np.arange(ny)
    red = ((y >= 10) & (y < 30))[None, :, None] * np.ones((nz, ny, nx))
    prm = C.params(1.0 / (3 * 0.05 + 0.5), 7.0 / 9.0)
    fr, fb = C.init(prm, 3.0 * red, 1.0 - red, np.zeros((3, nz, ny, nx)))
    fr, fb = C.run(prm, fr, fb, 5000)
    rr, rb, phi, u, p = C.fields(prm, fr, fb)
    assert abs(p[0, 20, 0] - p[0, 0, 0]) < 1e-11
    assert np.abs(u).max() < 1e-10
    assert abs(rr[0, 20, 0] - 3.0) < 1e-4 and abs(rb[0, 0, 0] - 1.0) < 1e-4
    assert phi[0, 20, 0] > 0.999 and phi[0, 0, 0] < -0.999


def test_pure_colour_linear_modes_and_sound_speed():
    """Red only (phi = 1: neither perturbation nor recolouring) with
    alpha = 0.6: small perturbations follow the linear operator
    J + M^-1 (I - K) M (I - J) with J built from phi_i (the linear part of
    h_eq) and the printed M; its sound mode travels at sqrt((1 - alpha)/2)."""
    import os

    M = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "d3q19_M_printed.txt"))
    c, w, _ = oracle.tables()
    alpha, om = 0.6, 1.5
    phi = np.array([C.phi_i(k, alpha) for k in c2_of(c)])
    J = phi[:, None] * np.ones(19)[None, :] + 3.0 * w[:, None] * (c @ c.T)
    Kd = oracle.K(om)
    Cop = J + np.linalg.solve(M, np.diag(1.0 - Kd) @ M) @ (np.eye(19) - J)
    n, steps, A = 32, 10, 1e-6
    kv = np.array([2 * np.pi / n, 0.0, 0.0])
    Lop = np.diag(np.exp(-1j * (c @ kv))) @ Cop
    rng = np.random.default_rng(6)
    v0 = rng.normal(size=19) + 1j * rng.normal(size=19)
    x = np.arange(n)
    pert = np.real(v0[:, None] * np.exp(1j * kv[0] * x)[None, :])[:, None, None, :]
    prm = C.params(om, alpha)
    base = phi[:, None, None, None] * np.ones((19, 1, 1, n))
    runs = [C.run(prm, base + s * A * pert, np.zeros_like(base), steps)[0] for s in (1, -1)]
    lin = (runs[0] - runs[1]) / (2 * A)
    want = np.real((np.linalg.matrix_power(Lop, steps) @ v0)[:, None] * np.exp(1j * kv[0] * x)[None, :])
    assert np.abs(lin[:, 0, 0, :] - want).max() / np.abs(want).max() < 1e-7
    ev = np.linalg.eigvals(Lop)
    speeds = np.sort(np.abs(np.angle(ev[np.abs(ev) > 0.9]))) / kv[0]
    cs = np.sqrt((1 - alpha) / 2)
    assert np.min(np.abs(speeds - cs)) < 2e-3 * cs


def test_young_laplace_printed_sigma():
    """Equal densities, cylinder of radius 10 in a 40^2 box, A = 0.01: the
    steady pressure jump times R equals sigma = (2/9) A / omega within 8 %
    (measured 4-6 % above, shrinking with R)."""
    n, R, A = 40, 10.0, 0.01
    om = 1.0 / (3 * 0.05 + 0.5)
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    inside = (np.hypot(xx - n / 2 + 0.5, yy - n / 2 + 0.5) < R)[None].astype(float)
    prm = C.params(om, 1.0 / 3.0, A=A)
    fr, fb = C.init(prm, inside, 1.0 - inside, np.zeros((3, 1, n, n)))
    fr, fb = C.run(prm, fr, fb, 4000)
    _, _, _, u, p = C.fields(prm, fr, fb)
    dp = p[0, n // 2, n // 2] - p[0, 0, 0]
    sigma = (2.0 / 9.0) * A / om
    assert abs(dp * R / sigma - 1) < 0.08, dp * R / sigma
    assert np.abs(u).max() < 1e-4
