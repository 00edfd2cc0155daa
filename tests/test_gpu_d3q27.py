"""GPU D3Q27 lattice (App. D; readings Q1-Q4) against the FP64 oracle."""
import numpy as np
import pytest

from gpu_helpers import gpu_run, rel_l2, say
from paper_2010_01628_amd import inputs
from paper_2010_01628_amd import lbm as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def oracle27(orc, rho, u, steps, omega, F=None, walls=False):
    q = orc.d3q27
    f = q.run(q.init(rho, u), steps, q.K(omega), F=F, walls_y=walls)
    r, v = q.moments(f, F)
    return {"f": f, "rho": r, "u": v}


@pytest.mark.parametrize("nx,ny,nz,walls,streaming,steps", [
    (12, 10, 8, False, "ab", 7), (12, 10, 8, False, "aa", 7), (9, 6, 5, True, "ab", 9), (9, 6, 5, True, "aa", 9),
    (1, 3, 7, False, "aa", 5)])
def test_d3q27_fp64_elementwise(orc, nx, ny, nz, walls, streaming, steps):
    say(f"d3q27 fp64 {nx}x{ny}x{nz} walls={walls} {streaming}")
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=nx + 3 * ny + 7 * nz, umax=0.06, fmax=2e-3)
    om = 1.73
    g = gpu_run(nx, ny, nz, rho, u, steps, "fp64", streaming, omega=om, force=F, walls=walls, q=27)
    o = oracle27(orc, rho, u, steps, om, F=F, walls=walls)
    assert g["f"].shape == o["f"].shape
    assert np.abs(g["f"] - o["f"]).max() < 1e-13
    assert rel_l2(g["u"], o["u"]) < 1e-12


def test_d3q27_fp32_and_ab_aa_bitwise(orc):
    n, steps = 24, 60
    om = inputs.omega_from_nu(1e-3)
    rho, u = inputs.taylor_green_noise(n, 0.05, 1e-4, seed=7)
    a = gpu_run(n, n, n, rho, u, steps, "fp32", "ab", omega=om, q=27, force_mode=L.LBM_FORCE_KOLMOGOROV,
                kolmogorov_amp=1e-6)
    b = gpu_run(n, n, n, rho, u, steps, "fp32", "aa", omega=om, q=27, force_mode=L.LBM_FORCE_KOLMOGOROV,
                kolmogorov_amp=1e-6)
    assert np.array_equal(a["f"], b["f"])
    o = oracle27(orc, rho, u, steps, om, F=inputs.kolmogorov_force(n, n, n, 1e-6))
    err = rel_l2(a["u"], o["u"])
    say(f"  d3q27 fp32 rel L2 u = {err:.3e}")
    assert err < 1e-5
