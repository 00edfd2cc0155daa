"""Pins of the oracle's raw-moment variant (App. C with N = I: the classical
raw-moment MRT in the paper's basis) against facts outside its own code: the
printed matrix M, the shifted-product raw moments of the equilibrium and the
Gaussian-rule raw moments of the forcing term (App. B, C), the App. C
post-collision rule, invariants and the linear (von Neumann) modes about
rest."""
import numpy as np
import pytest

import moment_forms as mf
from test_oracle_physics import linear_operator, printed_M

CS2 = 1.0 / 3.0
RM_MODES = [2]  # oracle.RM_DEFINITION


def rand_pops(orc, rng, amp=0.08, neq=0.01):
    rho = 1.0 + 0.1 * rng.uniform(-1, 1)
    u = amp * rng.uniform(-1, 1, 3)
    return orc.feq(rho, u) * (1.0 + neq * rng.uniform(-1, 1, 19))


def rand_K(orc, rng):
    return orc.K(rng.uniform(0.5, 1.95), rng.uniform(0.5, 1.95), rng.uniform(0.5, 1.95, 9))


def test_M_is_the_printed_matrix(orc):
    assert np.array_equal(orc.M(), printed_M())


def test_raw_equilibrium_is_the_shifted_product(orc):
    """The raw-moment variant's equilibrium (App. C's list) is the raw moments
    of the Galilean-invariant equilibrium: rho prod_a mu_{p_a}(u_a)."""
    rng = np.random.default_rng(11)
    for _ in range(50):
        rho = 1.0 + 0.2 * rng.uniform(-1, 1)
        u = 0.3 * rng.uniform(-1, 1, 3)
        assert np.allclose(orc.keq_rm(rho, u), mf.eq_raw(rho, u), atol=1e-15)


def test_raw_forcing_is_the_gaussian_rule(orc):
    """App. B: R^RM (eq. RMQ19) are the raw moments of the forcing term whose
    CMs are R^CM; both follow the Gaussian rule on the equilibrium moments."""
    rng = np.random.default_rng(12)
    for _ in range(30):
        u = 0.3 * rng.uniform(-1, 1, 3)
        F = rng.normal(size=3)
        assert np.allclose(orc.Rrm(u, F), mf.forcing_raw(u, F), atol=1e-14)


@pytest.mark.parametrize("mode", RM_MODES)
def test_unit_rates_equal_the_cm_scheme(orc, mode):
    """K = I: both schemes set every moment to equilibrium plus half the
    forcing, the same populations whichever basis is used."""
    rng = np.random.default_rng(13)
    for _ in range(30):
        f = rand_pops(orc, rng)
        F = 1e-3 * rng.normal(size=3)
        want, *_ = orc.collide(f, F, orc.K(1.0), mode=0)
        got, *_ = orc.collide(f, F, orc.K(1.0), mode=mode)
        assert np.abs(got - want).max() < 1e-15


@pytest.mark.parametrize("mode", RM_MODES)
def test_equilibrium_is_fixed_point(orc, mode):
    rng = np.random.default_rng(15)
    for _ in range(20):
        rho = 1.0 + 0.1 * rng.uniform(-1, 1)
        u = 0.1 * rng.uniform(-1, 1, 3)
        fe = orc.feq(rho, u)
        fs, *_ = orc.collide(fe, (0.0, 0.0, 0.0), rand_K(orc, rng), mode=mode)
        assert np.abs(fs - fe).max() < 1e-15


@pytest.mark.parametrize("mode", RM_MODES)
def test_collision_conserves_mass_and_adds_force(orc, mode):
    rng = np.random.default_rng(16)
    c, _, _ = orc.tables()
    for _ in range(30):
        f = rand_pops(orc, rng)
        F = 1e-3 * rng.normal(size=3)
        fs, *_ = orc.collide(f, F, rand_K(orc, rng), mode=mode)
        assert abs(fs.sum() - f.sum()) < 1e-15
        assert np.abs(c.T @ fs - (c.T @ f + F)).max() < 1e-15


def test_post_collision_matches_printed_list_without_force(orc):
    """App. C post-collision raw moments with the paper's rates and F = 0:
    k5..k9 relax with w towards their equilibrium, all other rows are set to
    it (the shifted-product raw equilibrium); k5..k9 are the sums over f of
    eq. (PreCollCMS)."""
    rng = np.random.default_rng(17)
    M = printed_M()
    c, _, _ = orc.tables()
    cx, cy, cz = c[:, 0], c[:, 1], c[:, 2]
    for _ in range(30):
        f = rand_pops(orc, rng, neq=0.05)
        om = rng.uniform(0.5, 1.95)
        rho = f.sum()
        ux, uy, uz = (c.T @ f) / rho
        k5 = np.sum(f * (cx ** 2 - cy ** 2))
        k6 = np.sum(f * (cy ** 2 - cz ** 2))
        k7, k8, k9 = np.sum(f * cx * cy), np.sum(f * cx * cz), np.sum(f * cy * cz)
        want = mf.eq_raw(rho, (ux, uy, uz))
        want[5:10] = (1 - om) * np.array([k5, k6, k7, k8, k9]) + om * want[5:10]
        fs, *_ = orc.collide(f, (0.0, 0.0, 0.0), orc.K(om), mode=2)
        assert np.allclose(M @ fs, want, atol=1e-15)


def test_differs_from_cm_away_from_unit_rates(orc):
    """Not a pin: with w != 1 and a finite velocity the two bases relax
    different non-equilibrium combinations, so the variants must differ."""
    rng = np.random.default_rng(18)
    f = rand_pops(orc, rng, amp=0.1, neq=0.05)
    a, *_ = orc.collide(f, (0.0, 0.0, 0.0), orc.K(1.7), mode=0)
    b, *_ = orc.collide(f, (0.0, 0.0, 0.0), orc.K(1.7), mode=2)
    assert np.abs(a - b).max() > 1e-7


def test_linear_modes_match_von_neumann(orc):
    """About rest both bases coincide to first order (T(u) = M + O(u)), so a
    small perturbation evolves as the same L(k)^t built from the printed M
    and the rates alone."""
    rng = np.random.default_rng(19)
    n, steps, A = 8, 12, 1e-5
    kvec = 2 * np.pi * np.array([2, 1, 3]) / n
    Kd = rand_K(orc, rng)
    c, w, _ = orc.tables()
    v0 = rng.normal(size=19) + 1j * rng.normal(size=19)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    phase = np.exp(1j * (kvec[0] * x + kvec[1] * y + kvec[2] * z))
    pert = np.real(v0[:, None, None, None] * phase[None])
    runs = [orc.run(w[:, None, None, None] + s * A * pert, steps, Kd, mode=2) for s in (+1, -1)]
    lin = (runs[0] - runs[1]) / (2 * A)
    vt = np.linalg.matrix_power(linear_operator(orc, Kd, kvec), steps) @ v0
    want = np.real(vt[:, None, None, None] * phase[None])
    assert np.abs(lin - want).max() / np.abs(want).max() < 1e-7


@pytest.mark.parametrize("walls", [False, True])
def test_lattice_conservation_with_random_force(orc, walls):
    """Periodic lattice: total mass constant and total momentum grows by the
    summed force every step (walls: mass only)."""
    from paper_2010_01628_amd import inputs

    nx, ny, nz = 6, 5, 4
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=31, umax=0.05, fmax=1e-3)
    f = orc.init(rho, u)
    c, _, _ = orc.tables()
    mass0 = f.sum()
    mom0 = c.T @ f.reshape(19, -1).sum(axis=1)
    steps = 5
    f = orc.run(f, steps, orc.K(1.6, 1.3, np.full(9, 1.2)), F=F, walls_y=walls, mode=2)
    assert abs(f.sum() - mass0) / mass0 < 1e-14
    if not walls:
        mom = c.T @ f.reshape(19, -1).sum(axis=1)
        assert np.allclose(mom - mom0, steps * F.reshape(3, -1).sum(axis=1), atol=1e-13)
