"""FP64 diagnostics of lbm_moments (the totals the paper tracks in time:
mass, momentum and the kinetic energy 1/2 sum rho |u|^2 of Sec. III, plus
max |u|) against the same totals computed from the oracle's rho and
force-shifted u, on random forced lattices with and without walls, in both
streaming patterns.

A total that may cancel (momentum) is compared against the sum of the
magnitudes of its terms, the scale its rounding error is proportional to."""
import numpy as np
import pytest

from gpu_helpers import gpu_run, oracle_run, say
from paper_2010_01628_amd import inputs
from paper_2010_01628_amd import lbm as L

pytestmark = pytest.mark.gpu

# relative bounds: FP64 storage and collision differ from the oracle by
# rounding order only; FP32 storage rounds every population to 2^-24 of its
# deviation each step, a few 1e-8 of the totals after these few steps
TOL = {"fp64": 1e-12, "fp32": 1e-6}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def oracle_totals(rho, u):
    ru = rho[None] * u
    speed = np.sqrt(np.sum(u * u, axis=0))
    return {
        "mass": float(rho.sum()),
        "mom": ru.reshape(3, -1).sum(axis=1),
        "mom_scale": np.abs(ru).reshape(3, -1).sum(axis=1),
        "ke": 0.5 * float(np.sum(rho * np.sum(u * u, axis=0))),
        "umax": float(speed.max()),
    }


def check(diag, o, tol, label):
    err_mass = abs(diag[0] - o["mass"]) / o["mass"]
    err_mom = np.abs(diag[1:4] - o["mom"]) / o["mom_scale"]
    err_ke = abs(diag[4] - o["ke"]) / o["ke"]
    err_max = abs(diag[5] - o["umax"]) / o["umax"]
    say(f"  {label}: mass {err_mass:.2e} momentum {err_mom.max():.2e} KE {err_ke:.2e} max|u| {err_max:.2e}")
    assert err_mass <= tol
    assert np.all(err_mom <= tol)
    assert err_ke <= tol
    assert err_max <= tol


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("streaming", ["ab", "aa"])
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape", [(21, 13, 11), (64, 48, 40)])
def test_diag_matches_oracle_totals(orc, precision, streaming, walls, shape):
    nx, ny, nz = shape
    steps = 5
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=41 + nx, umax=0.05, fmax=1e-3)
    g = gpu_run(nx, ny, nz, rho, u, steps, precision=precision, streaming=streaming, omega=1.87, force=F,
                walls=walls, want_pops=False)
    o = oracle_run(orc, rho, u, steps, omega=1.87, F=F, walls=walls)
    check(g["diag"], oracle_totals(o["rho"], o["u"]), TOL[precision],
          f"{precision} {streaming} walls={walls} {nx}x{ny}x{nz}")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_diag_kolmogorov_force(orc, precision):
    """The velocity is shifted by the Kolmogorov force F_x(y) in the totals too."""
    nx, ny, nz = 24, 20, 18
    steps = 7
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=9, umax=0.04)
    amp = 2e-3
    g = gpu_run(nx, ny, nz, rho, u, steps, precision=precision, streaming="ab", omega=1.6,
                force_mode=L.LBM_FORCE_KOLMOGOROV, kolmogorov_amp=amp, want_pops=False)
    F = inputs.kolmogorov_force(nx, ny, nz, amp)
    o = oracle_run(orc, rho, u, steps, omega=1.6, F=F)
    check(g["diag"], oracle_totals(o["rho"], o["u"]), TOL[precision], f"{precision} Kolmogorov")
