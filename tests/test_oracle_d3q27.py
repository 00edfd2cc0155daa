"""Pins of the D3Q27 part of the oracle (App. D; readings Q1-Q3, Q6)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(__file__))

from paper_2010_01628_amd import inputs  # noqa: E402


@pytest.fixture(scope="module")
def q27(orc):
    return orc.d3q27


def test_velocity_set(q27):
    c, w, opp = q27.tables()
    assert {tuple(v) for v in c} == {(a, b, d) for a in (-1, 0, 1) for b in (-1, 0, 1) for d in (-1, 0, 1)}
    for i in range(1, 27):
        assert opp[i] == (i + 13 if i <= 13 else i - 13)
        assert np.array_equal(c[opp[i]], -c[i])
    # tensor-product weights: moments of D1Q3 (1, 1/3) per axis
    assert np.isclose(w.sum(), 1.0)
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3)
    assert np.isclose(np.sum(w * c[:, 0] ** 2 * c[:, 1] ** 2 * c[:, 2] ** 2), 1 / 27)
    assert np.isclose(np.sum(w * c[:, 0] ** 4), 1 / 3)


def test_equilibrium_raw_moments_are_products(q27):
    """Reading Q1: raw moments of f_eq are rho prod_a mu_{p_a}(u_a) with mu_0 = 1,
    mu_1 = u, mu_2 = u^2 + 1/3 for every exponent up to 2 per axis."""
    c, _, _ = q27.tables()
    rng = np.random.default_rng(1)
    mu = lambda p, u: (1.0, u, u * u + 1.0 / 3.0)[p]
    for _ in range(20):
        rho = 1 + 0.1 * rng.uniform(-1, 1)
        u = rng.uniform(-0.3, 0.3, 3)
        fe = q27.feq(rho, u)
        for p in range(3):
            for q in range(3):
                for r in range(3):
                    m = np.sum(fe * c[:, 0] ** p * c[:, 1] ** q * c[:, 2] ** r)
                    assert np.isclose(m, rho * mu(p, u[0]) * mu(q, u[1]) * mu(r, u[2]), atol=1e-15)


def test_equilibrium_cms_galilean(q27):
    """T27(u) f_eq(rho, u): k0 = rho, k9 = rho, k17 = rho/3, k18 = rho/9,
    k26 = rho/27, all others 0, for every u."""
    rng = np.random.default_rng(2)
    for _ in range(20):
        rho = 1 + 0.1 * rng.uniform(-1, 1)
        u = rng.uniform(-0.3, 0.3, 3)
        k = q27.T(u) @ q27.feq(rho, u)
        want = np.zeros(27)
        want[[0, 9, 17, 18, 26]] = [rho, rho, rho / 3, rho / 9, rho / 27]
        assert np.allclose(k, want, atol=1e-14)
        assert np.allclose(q27.keq(rho), want, atol=1e-16)


def test_forcing_cms_match_d3q19_list(orc, q27):
    """Reading Q3 reproduces App. B eq. (CMQ19) on the monomials both lattices
    share (rows of D3Q27 combined back to single monomials)."""
    F = np.array([0.3, -0.7, 1.1])
    R27 = q27.Rcm(F)
    R19 = orc.Rcm(F)
    assert np.allclose(R27[1:4], F)
    mono27 = {  # monomial -> value from D3Q27 rows
        "210": (R27[11] + R27[14]) / 2, "012": (R27[11] - R27[14]) / 2,
        "120": (R27[10] + R27[13]) / 2, "102": (R27[10] - R27[13]) / 2,
        "201": (R27[12] + R27[15]) / 2, "021": (R27[12] - R27[15]) / 2,
    }
    assert np.isclose(mono27["210"], R19[10]) and np.isclose(mono27["120"], R19[11])
    assert np.isclose(mono27["201"], R19[12]) and np.isclose(mono27["102"], R19[13])
    assert np.isclose(mono27["021"], R19[14]) and np.isclose(mono27["012"], R19[15])
    assert np.allclose(R27[[0, 4, 5, 6, 7, 8, 9, 16, 17, 18, 19, 20, 21, 22, 26]], 0.0)
    # fifth order: R_122 = Fx/9, R_212 = Fy/9, R_221 = Fz/9
    assert np.allclose(R27[[23, 24, 25]], F / 9)


def test_collision_fixed_point_and_conservation(q27):
    c, _, _ = q27.tables()
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = 1 + 0.1 * rng.uniform(-1, 1)
        u = rng.uniform(-0.2, 0.2, 3)
        K = q27.K(rng.uniform(0.2, 1.99))
        fe = q27.feq(rho, u)
        fs, _, _ = q27.collide(fe, (0, 0, 0), K)
        assert np.allclose(fs, fe, atol=1e-15)
        f = fe * (1 + 0.05 * rng.uniform(-1, 1, 27))
        F = 1e-2 * rng.normal(size=3)
        fs, _, _ = q27.collide(f, F, K)
        assert np.isclose(fs.sum(), f.sum(), atol=1e-15)
        assert np.allclose(fs @ c, f @ c + F, atol=1e-15)


D3Q19_MONOS = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1),
               (0, 1, 1), (2, 1, 0), (1, 2, 0), (2, 0, 1), (1, 0, 2), (0, 2, 1), (0, 1, 2), (2, 2, 0), (2, 0, 2),
               (0, 2, 2)]


def project_to_q19(orc, q27, f27):
    """D3Q19 populations with the same 19 raw moments as the D3Q27 ones."""
    c27, _, _ = q27.tables()
    c19, _, _ = orc.tables()
    A27 = np.array([[c27[i, 0] ** p * c27[i, 1] ** q * c27[i, 2] ** r for i in range(27)] for p, q, r in D3Q19_MONOS])
    A19 = np.array([[c19[i, 0] ** p * c19[i, 1] ** q * c19[i, 2] ** r for i in range(19)] for p, q, r in D3Q19_MONOS])
    return np.linalg.solve(A19, A27 @ f27), A19, A27


def test_d3q27_and_d3q19_agree_on_the_shared_moments(orc, q27):
    """With the paper's rates, a D3Q27 collision leaves the 19 shared raw
    moments exactly where a D3Q19 collision of the projected state puts them:
    the two lattices differ only through the streaming of the 8 corners."""
    rng = np.random.default_rng(4)
    for _ in range(20):
        rho = 1 + 0.1 * rng.uniform(-1, 1)
        u = rng.uniform(-0.1, 0.1, 3)
        f27 = q27.feq(rho, u) * (1 + 0.1 * rng.uniform(-1, 1, 27))
        F = 1e-2 * rng.normal(size=3)
        om = rng.uniform(0.3, 1.99)
        f27s, _, _ = q27.collide(f27, F, q27.K(om))
        f19, A19, A27 = project_to_q19(orc, q27, f27)
        f19s, _, _, _ = orc.collide(f19, F, orc.K(om), 0)
        assert np.allclose(A19 @ f19s, A27 @ f27s, atol=2e-15)


def test_shear_wave_tau1_closed_form_d3q27(q27):
    n, A0, steps = 16, 0.01, 60
    k = 2 * np.pi / n
    rho, u = inputs.shear_wave(n, A0, nx=2, ny=2)
    f = q27.run(q27.init(rho, u), steps, q27.K(1.0))
    r, ut = q27.moments(f)
    prof = ut[0].mean(axis=(1, 2))
    A = 2.0 / n * np.sum(prof * np.sin(k * np.arange(n)))
    assert abs(A / (A0 * ((2 + np.cos(k)) / 3) ** steps) - 1) < 1e-12
    assert np.abs(r - 1).max() < 1e-14


def test_linear_modes_match_von_neumann_d3q27(q27):
    """Random small perturbations follow the linearised D3Q27 operator built
    from T27(0), the rates and the linear equilibrium w (drho + 3 c.dj)."""
    c, w, _ = q27.tables()
    rng = np.random.default_rng(5)
    n, steps, A = 6, 8, 1e-5
    kvec = 2 * np.pi * np.array([1, 2, -1]) / n
    om = 1.7
    Kd = q27.K(om)
    M = q27.T([0.0, 0.0, 0.0])
    J = w[:, None] * (1.0 + 3.0 * (c @ c.T))
    C = J + np.linalg.solve(M, np.diag(1.0 - Kd) @ M) @ (np.eye(27) - J)
    L = np.diag(np.exp(-1j * (c @ kvec))) @ C
    v0 = rng.normal(size=27) + 1j * rng.normal(size=27)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    phase = np.exp(1j * (kvec[0] * x + kvec[1] * y + kvec[2] * z))
    pert = np.real(v0[:, None, None, None] * phase[None])
    runs = [q27.run(w[:, None, None, None] + s * A * pert, steps, Kd) for s in (1, -1)]
    lin = (runs[0] - runs[1]) / (2 * A)
    want = np.real((np.linalg.matrix_power(L, steps) @ v0)[:, None, None, None] * phase[None])
    assert np.abs(lin - want).max() / np.abs(want).max() < 1e-7


def test_lattice_conservation_d3q27(q27):
    nx, ny, nz = 5, 4, 6
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=8, umax=0.05, fmax=1e-3)
    c, _, _ = q27.tables()
    Kd = q27.K(1.6)
    f = q27.init(rho, u)
    m0 = f.sum()
    for walls in (False, True):
        g = f.copy()
        for _ in range(3):
            p0 = np.einsum("iabc,id->d", g, c)
            g = q27.step(g, Kd, F=F, walls_y=walls)
            if not walls:
                assert np.allclose(np.einsum("iabc,id->d", g, c) - p0, F.reshape(3, -1).sum(axis=1), atol=1e-13)
        assert abs(g.sum() - m0) / m0 < 1e-14


# --------------------------------------------------------------------------
# Raw-moment variant (reading Q6: N = I with the same equilibrium and force)
# --------------------------------------------------------------------------
def test_raw_equilibrium_is_M_times_population_equilibrium(q27):
    """The raw equilibrium moments in the App. D basis equal T27(0) f_eq with
    the tensor-product populations (pinned above as products of D1Q3
    moments)."""
    rng = np.random.default_rng(21)
    M = q27.T([0.0, 0.0, 0.0])
    for _ in range(30):
        rho = 1 + 0.2 * rng.uniform(-1, 1)
        u = rng.uniform(-0.3, 0.3, 3)
        assert np.allclose(q27.keq_rm(rho, u), M @ q27.feq(rho, u), atol=1e-15)


def test_raw_forcing_is_raw_moments_of_the_cm_forcing(q27):
    """Raw forcing moments = M T27(u)^-1 R^CM: the same velocity-space forcing
    term as the central-moment scheme."""
    rng = np.random.default_rng(22)
    M = q27.T([0.0, 0.0, 0.0])
    for _ in range(30):
        u = rng.uniform(-0.3, 0.3, 3)
        F = rng.normal(size=3)
        Fi = np.linalg.solve(q27.T(u), q27.Rcm(F))
        assert np.allclose(q27.Rrm(u, F), M @ Fi, atol=1e-14)


def test_raw_unit_rates_equal_cm_and_conserve(q27):
    c, _, _ = q27.tables()
    rng = np.random.default_rng(23)
    for _ in range(20):
        rho = 1 + 0.1 * rng.uniform(-1, 1)
        u = rng.uniform(-0.1, 0.1, 3)
        f = q27.feq(rho, u) * (1 + 0.05 * rng.uniform(-1, 1, 27))
        F = 1e-2 * rng.normal(size=3)
        a, _, _ = q27.collide(f, F, q27.K(1.0))
        b, _, _ = q27.collide(f, F, q27.K(1.0), raw=True)
        assert np.abs(a - b).max() < 1e-15
        K = q27.K(rng.uniform(0.3, 1.95))
        fs, _, _ = q27.collide(f, F, K, raw=True)
        assert np.isclose(fs.sum(), f.sum(), atol=1e-15)
        assert np.allclose(fs @ c, f @ c + F, atol=1e-15)
        fe = q27.feq(rho, u)
        assert np.allclose(q27.collide(fe, (0, 0, 0), K, raw=True)[0], fe, atol=1e-15)
        # and differs from the CM scheme away from unit rates
        assert np.abs(q27.collide(f, F, K, raw=True)[0] - q27.collide(f, F, K)[0]).max() > 1e-9


def test_raw_d3q27_and_raw_d3q19_agree_on_the_shared_moments(orc, q27):
    """Raw variants of both lattices relax the same second-order raw moments
    towards the same equilibrium with the same forcing; all other shared
    moments go to equilibrium plus half the forcing: identical post-collision
    values on the 19 shared raw moments."""
    rng = np.random.default_rng(24)
    for _ in range(20):
        rho = 1 + 0.1 * rng.uniform(-1, 1)
        u = rng.uniform(-0.1, 0.1, 3)
        f27 = q27.feq(rho, u) * (1 + 0.1 * rng.uniform(-1, 1, 27))
        F = 1e-2 * rng.normal(size=3)
        om = rng.uniform(0.3, 1.99)
        f27s, _, _ = q27.collide(f27, F, q27.K(om), raw=True)
        f19, A19, A27 = project_to_q19(orc, q27, f27)
        f19s, _, _, _ = orc.collide(f19, F, orc.K(om), orc.RM_DEFINITION)
        assert np.allclose(A19 @ f19s, A27 @ f27s, atol=2e-15)


def test_raw_linear_modes_match_von_neumann_d3q27(q27):
    """About rest the raw and central bases coincide to first order: the
    same linear operator as above."""
    c, w, _ = q27.tables()
    rng = np.random.default_rng(25)
    n, steps, A = 6, 8, 1e-5
    kvec = 2 * np.pi * np.array([2, -1, 1]) / n
    Kd = q27.K(1.45)
    M = q27.T([0.0, 0.0, 0.0])
    J = w[:, None] * (1.0 + 3.0 * (c @ c.T))
    C = J + np.linalg.solve(M, np.diag(1.0 - Kd) @ M) @ (np.eye(27) - J)
    L = np.diag(np.exp(-1j * (c @ kvec))) @ C
    v0 = rng.normal(size=27) + 1j * rng.normal(size=27)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    phase = np.exp(1j * (kvec[0] * x + kvec[1] * y + kvec[2] * z))
    pert = np.real(v0[:, None, None, None] * phase[None])
    runs = [q27.run(w[:, None, None, None] + s * A * pert, steps, Kd, raw=True) for s in (1, -1)]
    lin = (runs[0] - runs[1]) / (2 * A)
    want = np.real((np.linalg.matrix_power(L, steps) @ v0)[:, None, None, None] * phase[None])
    assert np.abs(lin - want).max() / np.abs(want).max() < 1e-7
