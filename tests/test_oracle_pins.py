"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these tests compares the oracle with itself: each one checks an
oracle routine against a different printed passage, a closed form, a library
routine, or an invariant, so that a dropped term, a wrong sign or index or a
transposed operand in the oracle fails at least one of them.
"""
import os

import numpy as np
import pytest

import moment_forms as mf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CS2 = 1.0 / 3.0


def printed_M():
    return np.loadtxt(os.path.join(GOLDEN, "d3q19_M_printed.txt"))


def rand_state(rng, amp=0.05):
    rho = 1.0 + 0.1 * rng.uniform(-1, 1)
    u = amp * rng.uniform(-1, 1, 3)
    return rho, u


# --------------------------------------------------------------------------
# Lattice (Sec. II.A)
# --------------------------------------------------------------------------
def test_lattice_isotropy(orc):
    """Textbook D3Q19 moment isotropy: sum w = 1, sum w c = 0,
    sum w c_a c_b = cs^2 delta_ab, sum w cx^2 cy^2 = cs^4, odd moments vanish."""
    c, w, opp = orc.tables()
    assert np.isclose(w.sum(), 1.0, atol=1e-15)
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    second = np.einsum("i,ia,ib->ab", w, c, c)
    assert np.allclose(second, CS2 * np.eye(3), atol=1e-16)
    assert np.isclose(np.sum(w * c[:, 0] ** 2 * c[:, 1] ** 2), CS2 ** 2, atol=1e-16)
    assert np.isclose(np.sum(w * c[:, 0] ** 4), 3 * CS2 ** 2, atol=1e-16)
    third = np.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert np.allclose(third, 0.0, atol=1e-16)
    # swap-trick ordering: opposite(i) = i +- 9 and c_opp = -c
    for i in range(1, 19):
        assert opp[i] == (i + 9 if i <= 9 else i - 9)
        assert np.array_equal(c[opp[i]], -c[i])
    # 19 distinct velocities, none of the (+-1,+-1,+-1) corners
    assert len({tuple(v) for v in c}) == 19
    assert np.all(np.sum(np.abs(c), axis=1) <= 2)


def test_T_at_rest_is_printed_M(orc):
    """T(0) built from the monomials of Sec. II.B equals the numeric M printed
    in App. C (this also fixes the last row as cy^2 cz^2)."""
    assert np.array_equal(orc.T([0.0, 0.0, 0.0]), printed_M())


def test_shift_matrix_lower_unitriangular(orc):
    """App. C: T = N M with N lower triangular (unit diagonal)."""
    rng = np.random.default_rng(1)
    M = printed_M()
    for _ in range(5):
        u = rng.uniform(-0.3, 0.3, 3)
        N = orc.T(u) @ np.linalg.inv(M)
        assert np.allclose(np.triu(N, 1), 0.0, atol=1e-13)
        assert np.allclose(np.diag(N), 1.0, atol=1e-13)


# --------------------------------------------------------------------------
# Equilibrium (Sec. II.A eq. EqQ19RM; Sec. II.B; App. C raw equilibrium list)
# --------------------------------------------------------------------------
def test_equilibrium_cms_galilean(orc):
    """Sec. II.B: T(u) f_eq(rho, u) = [rho,0,0,0,3 rho cs^2,0..0, rho cs^4 x3]
    for every u (the printed list of equilibrium CMs, also the product form)."""
    rng = np.random.default_rng(2)
    for _ in range(50):
        rho, u = rand_state(rng, 0.3)
        k = orc.T(u) @ orc.feq(rho, u)
        want = np.zeros(19)
        want[0] = rho
        want[4] = 3 * rho * CS2
        want[16:19] = rho * CS2 ** 2
        assert np.allclose(k, want, atol=1e-14)
        assert np.allclose(orc.keq(rho), want, atol=0)
        assert np.allclose(mf.eq_central(rho), want, atol=1e-16)


def test_equilibrium_raw_moments_are_shifted_products(orc):
    """Raw moments of the equilibrium with the printed M: Galilean-invariant
    product CMs shifted by u give rho prod_a mu_{p_a}(u_a), mu = (1, u,
    u^2 + cs^2) (binomial theorem); App. C lists these as the raw-moment
    variant's equilibrium, which the oracle takes as M f_eq."""
    rng = np.random.default_rng(3)
    M = printed_M()
    for _ in range(50):
        rho, u = rand_state(rng, 0.3)
        want = mf.eq_raw(rho, u)
        assert np.allclose(M @ orc.feq(rho, u), want, atol=1e-15)
        assert np.allclose(orc.keq_rm(rho, u), want, atol=1e-15)


def test_equilibrium_hydrodynamic_moments_match_qian(orc):
    """Sec. II.A: the extended equilibrium and the textbook second-order one
    (eq. 2ndEquilibrium) carry the same mass, momentum and momentum flux
    rho (cs^2 I + u u), exactly and for any u; they differ only in the
    higher-order moments (third and fourth order)."""
    c, w, _ = orc.tables()
    rng = np.random.default_rng(13)
    for _ in range(30):
        rho, uu = rand_state(rng, 0.3)
        cu = c @ uu
        qian = rho * w * (1 + cu / CS2 + cu ** 2 / (2 * CS2 ** 2) - uu @ uu / (2 * CS2))
        ext = orc.feq(rho, uu)
        for f in (qian, ext):
            assert np.isclose(f.sum(), rho, atol=1e-15)
            assert np.allclose(f @ c, rho * uu, atol=1e-15)
            assert np.allclose(np.einsum("i,ia,ib->ab", f, c, c),
                               rho * (CS2 * np.eye(3) + np.outer(uu, uu)), atol=1e-15)
        # the third-order moment sum f cx^2 cy differs: rho uy (ux^2 + cs^2) for the
        # extended one (App. C list), rho cs^2 uy for the second-order one
        m210 = lambda f: np.sum(f * c[:, 0] ** 2 * c[:, 1])
        assert np.isclose(m210(ext), rho * uu[1] * (uu[0] ** 2 + CS2), atol=1e-15)
        assert np.isclose(m210(qian), rho * uu[1] * CS2, atol=1e-15)


# --------------------------------------------------------------------------
# Forcing term (App. B) and the dense solve of the back-transform
# --------------------------------------------------------------------------
def test_forcing_moments_gaussian_rule(orc):
    """App. B: the forcing CMs (eq. CMQ19, the oracle's R^CM) and the raw
    moments of the same forcing term (eq. RMQ19; the oracle's M T(u)^-1 R^CM)
    both follow the Gaussian rule R_pqr = sum_a p_a F_a m_{pqr-e_a}/rho on the
    central and raw equilibrium moments; the velocity-space term
    F_i = M^-1 R^RM carries zero mass, momentum F and momentum flux
    u F + F u (Guo's forcing moments)."""
    rng = np.random.default_rng(6)
    M = printed_M()
    c, _, _ = orc.tables()
    for _ in range(20):
        u = rng.uniform(-0.3, 0.3, 3)
        F = rng.normal(size=3)
        assert np.allclose(orc.Rcm(F), mf.forcing_central(F), atol=1e-15)
        Rrm = orc.Rrm(u, F)
        assert np.allclose(Rrm, mf.forcing_raw(u, F), atol=1e-14)
        Fi = np.linalg.solve(M, Rrm)
        assert abs(Fi.sum()) < 1e-14
        assert np.allclose(Fi @ c, F, atol=1e-14)
        assert np.allclose(np.einsum("i,ia,ib->ab", Fi, c, c), np.outer(u, F) + np.outer(F, u), atol=1e-14)


def test_dense_solve_matches_library_solve(orc):
    """f* from the oracle's elimination solves T(u) f* = k*: it equals
    numpy.linalg.solve on the same system (k* rebuilt from the returned
    pre-collision moments and the printed relaxation rule)."""
    rng = np.random.default_rng(4)
    for _ in range(50):
        rho, u = rand_state(rng, 0.2)
        f = orc.feq(rho, u) * (1 + 0.1 * rng.uniform(-1, 1, 19))
        F = 1e-2 * rng.normal(size=3)
        K = orc.K(rng.uniform(0.1, 1.99), rng.uniform(0.1, 1.99), rng.uniform(0.1, 1.99, 9))
        fs, k, rr, uu = orc.collide(f, F, K, 0)
        ks = (1 - K) * k + K * mf.eq_central(rr) + (1 - K / 2) * mf.forcing_central(F)
        assert np.allclose(fs, np.linalg.solve(orc.T(uu), ks), rtol=0, atol=1e-13)


# --------------------------------------------------------------------------
# Collision (Sec. II.B eqs. posColl0, system)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("mode", [0, 2])
def test_equilibrium_is_fixed_point(orc, mode):
    """collide(f_eq) = f_eq for any rates when F = 0."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        rho, u = rand_state(rng, 0.2)
        K = orc.K(rng.uniform(0.1, 1.99), rng.uniform(0.1, 1.99), rng.uniform(0.1, 1.99, 9))
        fe = orc.feq(rho, u)
        fs, _, _, _ = orc.collide(fe, (0, 0, 0), K, mode)
        assert np.allclose(fs, fe, atol=1e-15)


@pytest.mark.parametrize("mode", [0, 2])
def test_collision_conserves_mass_and_adds_force(orc, mode):
    """sum f* = sum f and sum f* c = sum f c + F at every node (reading R2)."""
    c, w, _ = orc.tables()
    rng = np.random.default_rng(8)
    for _ in range(50):
        rho, u = rand_state(rng, 0.1)
        f = orc.feq(rho, u) * (1 + 0.05 * rng.uniform(-1, 1, 19))
        F = 1e-3 * rng.normal(size=3)
        K = orc.K(rng.uniform(0.1, 1.99), rng.uniform(0.1, 1.99), rng.uniform(0.1, 1.99, 9))
        fs, _, _, _ = orc.collide(f, F, K, mode)
        assert np.isclose(fs.sum(), f.sum(), rtol=0, atol=1e-15)
        assert np.allclose(fs @ c, f @ c + F, rtol=0, atol=1e-15)


def test_single_rate_is_bgk_with_guo_forcing(orc):
    """Sec. II.B: with every non-conserved rate equal to w, Lambda = T^-1 K T = w I
    and the scheme is BGK with the extended equilibrium and the (1 - w/2) F_i
    forcing, F_i = M^-1 R^RM (App. B).  Built here from the printed M and the
    product / Gaussian-rule moment forms -- none of the CM machinery."""
    c, w, _ = orc.tables()
    M = printed_M()
    rng = np.random.default_rng(10)
    for _ in range(30):
        rho, u = rand_state(rng, 0.1)
        f = orc.feq(rho, u) * (1 + 0.05 * rng.uniform(-1, 1, 19))
        F = 1e-2 * rng.normal(size=3)
        om = rng.uniform(0.2, 1.95)
        K = orc.K(om, om, np.full(9, om))
        fs, _, rho_o, u_o = orc.collide(f, F, K, 0)
        # macroscopic fields, force-shifted (reading R2)
        rr = f.sum()
        uu = (f @ c + 0.5 * F) / rr
        assert np.isclose(rho_o, rr) and np.allclose(u_o, uu)
        feq = np.linalg.solve(M, mf.eq_raw(rr, uu))
        Fi = np.linalg.solve(M, mf.forcing_raw(uu, F))
        bgk = f + om * (feq - f) + (1 - om / 2) * Fi
        assert np.allclose(fs, bgk, rtol=0, atol=1e-14)


def test_precollision_cms_by_binomial_shift(orc):
    """Moment sums brute-forced on a 4^3 lattice of random positive f: the
    oracle's k = T(u) f equals central moments obtained from raw moments
    sum_i f_i cx^a cy^b cz^c by the binomial theorem, an independent route."""
    from math import comb

    c, w, _ = orc.tables()
    rng = np.random.default_rng(11)
    basis = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), None, None, None,
             (1, 1, 0), (1, 0, 1), (0, 1, 1), (2, 1, 0), (1, 2, 0), (2, 0, 1),
             (1, 0, 2), (0, 2, 1), (0, 1, 2), (2, 2, 0), (2, 0, 2), (0, 2, 2)]

    def raw(f, a, b, cc):
        return sum(f[i] * c[i, 0] ** a * c[i, 1] ** b * c[i, 2] ** cc for i in range(19))

    def central(f, u, a, b, cc):
        tot = 0.0
        for p in range(a + 1):
            for q in range(b + 1):
                for r in range(cc + 1):
                    tot += (comb(a, p) * comb(b, q) * comb(cc, r) * (-u[0]) ** (a - p)
                            * (-u[1]) ** (b - q) * (-u[2]) ** (cc - r) * raw(f, p, q, r))
        return tot

    for _ in range(64):  # the 4^3 nodes
        f = rng.uniform(0.01, 0.2, 19)
        F = 1e-2 * rng.normal(size=3)
        _, k, rho, u = orc.collide(f, F, orc.K(1.3), 0)
        for r, b in enumerate(basis):
            if b is None:
                continue
            assert np.isclose(k[r], central(f, u, *b), rtol=0, atol=1e-14), r
        X, Y, Z = (central(f, u, 2, 0, 0), central(f, u, 0, 2, 0), central(f, u, 0, 0, 2))
        assert np.isclose(k[4], X + Y + Z, atol=1e-14)
        assert np.isclose(k[5], X - Y, atol=1e-14)
        assert np.isclose(k[6], Y - Z, atol=1e-14)
        # first-order CMs are -F/2 with the force-shifted velocity
        assert np.allclose(k[1:4], -0.5 * F, atol=1e-15)


def test_post_collision_cms_match_printed_list(orc):
    """Sec. II.B eq. (posColl0) with the paper's rates: T(u) f* equals the
    printed list k0*=rho, k1..3*=F/2, k4*=3 rho cs^2, k5..9*=(1-w) k5..9,
    k10..15* = cs^2 F/2 in the printed pattern, k16..18*=rho cs^4."""
    rng = np.random.default_rng(12)
    for _ in range(30):
        rho, u = rand_state(rng, 0.1)
        f = orc.feq(rho, u) * (1 + 0.05 * rng.uniform(-1, 1, 19))
        Fx, Fy, Fz = 1e-2 * rng.normal(size=3)
        om = rng.uniform(0.2, 1.95)
        fs, k, rho_o, u_o = orc.collide(f, (Fx, Fy, Fz), orc.K(om), 0)
        ks = orc.T(u_o) @ fs
        want = np.array([
            rho_o, Fx / 2, Fy / 2, Fz / 2, 3 * rho_o * CS2,
            (1 - om) * k[5], (1 - om) * k[6], (1 - om) * k[7], (1 - om) * k[8], (1 - om) * k[9],
            Fy * CS2 / 2, Fx * CS2 / 2, Fz * CS2 / 2, Fx * CS2 / 2, Fz * CS2 / 2, Fy * CS2 / 2,
            rho_o * CS2 ** 2, rho_o * CS2 ** 2, rho_o * CS2 ** 2,
        ])
        assert np.allclose(ks, want, atol=1e-14)
