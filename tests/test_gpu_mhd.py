"""Magnetic coupling (D3Q7 vector magnetic lattice + D3Q19 CM flow) on the
GPU against the FP64 oracle, bitwise reduction to the plain lattice without
a field, and the Hartmann channel workload (32 x 128 x 32, walls in y, Ha =
10, FP32) run to steady state against the analytic profile."""
import numpy as np
import pytest

from gpu_helpers import rel_l2, say
from paper_2010_01628_amd import inputs
from paper_2010_01628_amd import lbm as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def fields(shape, seed, bmax=0.03):
    nx, ny, nz = shape
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=seed, umax=0.04, fmax=1e-4)
    nodes = np.arange(nx * ny * nz, dtype=np.uint64).reshape(nz, ny, nx)
    b = np.stack([bmax * inputs.uniform_pm1(seed + 7, nodes, d) for d in range(3)])
    return rho, u, b, F


def gpu_mhd(shape, rho, u, b, steps, eta, b_wall, omega, walls, F=None, precision="fp64"):
    import torch

    nx, ny, nz = shape
    ff = None if F is None else torch.from_numpy(np.ascontiguousarray(F)).cuda()
    par = L.make_params(nx, ny, nz, precision=precision, omega=omega, walls_y=walls,
                        force_mode=L.LBM_FORCE_FIELD if F is not None else L.LBM_FORCE_NONE,
                        force_field_ptr=None if ff is None else ff.data_ptr(),
                        magnetic=dict(eta=eta, b_wall=b_wall))
    lat = L.Lattice(par, force_field=ff)
    lat.init_magnetic(rho, u, b)
    lat.step(steps)
    f = lat.get_populations().cpu().numpy()
    g = lat.get_coupled_populations().cpu().numpy()
    bb, jj = lat.magnetic_fields()
    r, uu, diag = lat.moments()
    out = dict(f=f, g=g, b=bb.cpu().numpy(), j=jj.cpu().numpy(), rho=r.cpu().numpy(), u=uu.cpu().numpy(), diag=diag)
    lat.close()
    return out


@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("shape,steps", [((12, 10, 8), 1), ((9, 13, 6), 12)])
def test_fp64_matches_oracle(orc, walls, shape, steps):
    say(f"mhd fp64 {shape} walls={walls} steps={steps}")
    rho, u, b, F = fields(shape, 21)
    eta, bw, om = 0.07, (0.01, 0.02, -0.005), 1.6
    prm = orc.mhd.params(eta, bw)
    fo, go = orc.mhd.run(prm, om, *orc.mhd.init(rho, u, b), steps, F=F, walls_y=walls)
    gpu = gpu_mhd(shape, rho, u, b, steps, eta, bw, om, walls, F=F)
    ef, eg = np.abs(gpu["f"] - fo).max(), np.abs(gpu["g"] - go).max()
    say(f"  max |f_gpu - f_oracle| = {ef:.3e}, max |g_gpu - g_oracle| = {eg:.3e}")
    assert ef < 1e-13 and eg < 1e-13
    ro, uo, bo, jo = orc.mhd.fields(prm, fo, go, F=F)
    assert np.abs(gpu["b"] - bo).max() < 1e-14
    assert np.abs(gpu["j"] - jo).max() < 1e-12
    assert np.abs(gpu["u"] - uo).max() < 1e-13
    assert np.abs(gpu["rho"] - ro).max() < 1e-13


def test_fp32_matches_oracle(orc):
    shape, steps = (16, 12, 10), 40
    rho, u, b, F = fields(shape, 5)
    eta, bw, om = 0.1, (0.0, 0.0, 0.0), 1.7
    prm = orc.mhd.params(eta, bw)
    fo, go = orc.mhd.run(prm, om, *orc.mhd.init(rho, u, b), steps, F=F)
    ro, uo, bo, jo = orc.mhd.fields(prm, fo, go, F=F)
    gpu = gpu_mhd(shape, rho, u, b, steps, eta, bw, om, False, F=F, precision="fp32")
    e_u, e_b, e_j = rel_l2(gpu["u"], uo), rel_l2(gpu["b"], bo), rel_l2(gpu["j"], jo)
    say(f"  fp32: rel L2 u {e_u:.2e}, b {e_b:.2e}, j {e_j:.2e}")
    assert e_u < 1e-5 and e_b < 1e-5 and e_j < 1e-4


def test_zero_field_equals_plain_lattice_bitwise():
    """No field: the Lorentz force is exactly zero and the flow equals the
    plain FP32 lattice bit for bit."""
    shape = (20, 14, 9)
    nx, ny, nz = shape
    rho, u, _, _ = fields(shape, 9)
    om = 1.9
    par = L.make_params(nx, ny, nz, precision="fp32", omega=om, walls_y=True, force_mode=L.LBM_FORCE_UNIFORM,
                        force=(1e-5, 0.0, 2e-6), magnetic=dict(eta=0.1))
    a = L.Lattice(par)
    a.init_magnetic(rho, u, np.zeros((3, nz, ny, nx)))
    a.step(6)
    plain = L.Lattice(L.make_params(nx, ny, nz, precision="fp32", omega=om, walls_y=True,
                                    force_mode=L.LBM_FORCE_UNIFORM, force=(1e-5, 0.0, 2e-6)))
    plain.init(rho, u)
    plain.step(6)
    assert np.array_equal(a.get_populations().cpu().numpy(), plain.get_populations().cpu().numpy())
    assert float(np.abs(a.get_coupled_populations().cpu().numpy()).max()) == 0.0
    a.close()
    plain.close()


def hartmann_setup(ny=128, Ha=10.0, nu=0.1, eta=0.1, u_max=0.02):
    b0 = Ha * 2 * np.sqrt(nu * eta) / ny
    F = u_max * b0 ** 2 * np.tanh(Ha) / (eta * Ha * (1 - 1 / np.cosh(Ha)))
    y = np.arange(ny)
    yp = 2 * (y + 0.5) - ny
    shape = (1 - np.cosh(Ha * yp / ny) / np.cosh(Ha)) / (1 - 1 / np.cosh(Ha))
    return b0, F, shape


def test_hartmann_channel():
    """Hartmann workload: 32 x 128 x 32, walls at y = -1/2 and 127.5 with the
    field (0, b0, 0) imposed there, Ha = 10, nu = eta = 0.1, body force for
    U_max ~ 0.02, FP32, run until max|du|/U_max < 1e-6 over 1000 steps (FP32
    resolution; capped at 100k steps).  Profile vs the analytic shape."""
    import torch

    nx, ny, nz = 32, 128, 32
    nu = eta = 0.1
    b0, F, shape = hartmann_setup(ny, 10.0, nu, eta)
    par = L.make_params(nx, ny, nz, precision="fp32", omega=1.0 / (3 * nu + 0.5), walls_y=True,
                        force_mode=L.LBM_FORCE_UNIFORM, force=(F, 0.0, 0.0),
                        magnetic=dict(eta=eta, b_wall=(0.0, b0, 0.0)))
    lat = L.Lattice(par)
    b = np.zeros((3, nz, ny, nx))
    b[1] = b0
    lat.init_magnetic(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)), b)
    prev = None
    steps = 0
    while steps < 100000:
        lat.step(1000)
        steps += 1000
        _, u, _ = lat.moments()
        ux = u[0].mean(dim=(0, 2)).cpu().numpy()
        if prev is not None and np.abs(ux - prev).max() / ux.max() < 1e-6:
            break
        prev = ux
    _, u, _ = lat.moments()
    u = u.cpu().numpy()
    ux = u[0].mean(axis=(0, 2))
    err = np.linalg.norm(ux / ux.max() - shape) / np.linalg.norm(shape)
    spread = np.abs(u[0] - ux[None, :, None]).max()
    say(f"  Hartmann: {steps} steps, u_max {ux.max():.6f} (analytic 0.02), shape rel L2 {err:.2e}, "
        f"x/z spread {spread:.1e}")
    assert steps < 100000
    assert err < 1e-3
    assert abs(ux.max() / 0.02 - 1) < 5e-3
    assert spread < 1e-6
    lat.close()
