"""Closed forms of the moments of the paper's D3Q19 equilibrium and forcing
term, used as pins of the oracle (they share no code with it).

Sec. II.B states that the equilibrium CMs are Galilean invariant: in the
basis of T they are those of a product over the three axes of 1-D factors
with central moments (1, 0, cs^2) for exponents (0, 1, 2).  Shifting a
product by u (binomial theorem, axis by axis) gives raw moments
rho * prod_a mu_{p_a}(u_a) with mu_0 = 1, mu_1 = u, mu_2 = u^2 + cs^2.  The
forcing term of App. B has the moments of -(F/rho).grad_xi f_eq (a Gaussian,
or Hermite, forcing): R_pqr = sum_a p_a F_a m_{pqr - e_a} / rho, with m the
central (R^CM) or raw (R^RM) equilibrium moments.  Every row of T has
exponents of at most 2 per axis, so these forms cover all 19 rows.
"""
import numpy as np

CS2 = 1.0 / 3.0

# rows of T (Sec. II.B, eq. "matrix"): a monomial c_x^p c_y^q c_z^r, or one of
# the three combinations of the second-order diagonal monomials (rows 4..6)
ROWS = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), "trace", "xx-yy", "yy-zz", (1, 1, 0), (1, 0, 1), (0, 1, 1),
        (2, 1, 0), (1, 2, 0), (2, 0, 1), (1, 0, 2), (0, 2, 1), (0, 1, 2), (2, 2, 0), (2, 0, 2), (0, 2, 2)]


def central_1d(p):
    return (1.0, 0.0, CS2)[p]


def raw_1d(p, u):
    return (1.0, u, u * u + CS2)[p]


def _rows(mono):
    out = np.zeros(19)
    for r, e in enumerate(ROWS):
        if e == "trace":
            out[r] = mono((2, 0, 0)) + mono((0, 2, 0)) + mono((0, 0, 2))
        elif e == "xx-yy":
            out[r] = mono((2, 0, 0)) - mono((0, 2, 0))
        elif e == "yy-zz":
            out[r] = mono((0, 2, 0)) - mono((0, 0, 2))
        else:
            out[r] = mono(e)
    return out


def eq_central(rho):
    """Equilibrium CMs in the rows of T (product form)."""
    return _rows(lambda e: rho * central_1d(e[0]) * central_1d(e[1]) * central_1d(e[2]))


def eq_raw(rho, u):
    """Equilibrium raw moments in the rows of M = T(0) (shifted product form)."""
    return _rows(lambda e: rho * raw_1d(e[0], u[0]) * raw_1d(e[1], u[1]) * raw_1d(e[2], u[2]))


def _gauss(F, m):
    def mono(e):
        tot = 0.0
        for a in range(3):
            if e[a] > 0:
                low = list(e)
                low[a] -= 1
                tot += e[a] * F[a] * m(tuple(low))
        return tot

    return _rows(mono)


def forcing_central(F):
    """CMs of the forcing term (Gaussian rule on the central product form)."""
    return _gauss(F, lambda e: central_1d(e[0]) * central_1d(e[1]) * central_1d(e[2]))


def forcing_raw(u, F):
    """Raw moments of the forcing term (Gaussian rule on the raw product form)."""
    return _gauss(F, lambda e: raw_1d(e[0], u[0]) * raw_1d(e[1], u[1]) * raw_1d(e[2], u[2]))
