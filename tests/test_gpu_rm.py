"""Raw-moment variant (App. C with N = I) on the GPU against the FP64
oracle's raw-moment mode, through the C ABI: element by element in FP64
(ragged, walled, degenerate and AA cases, random force field, general rates),
relative L2 in FP32 / FP16 / BF16 on the config-2 recipe, bitwise identity
of A-B and AA and of row-staged and direct reads, the K = I identity with the
central-moment lattice, and sampled nodes of the 256^3 FP32 lattice in the
launch configuration the benchmark times."""
import numpy as np
import pytest

from gpu_helpers import gpu_run, oracle_run, rel_l2, rel_l2_fluct, say
from paper_2010_01628_amd import inputs
from paper_2010_01628_amd import lbm as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


CASES = [
    # nx, ny, nz, walls, streaming, steps, general rates
    (16, 16, 16, False, "ab", 9, False),
    (16, 16, 16, False, "aa", 9, True),
    (13, 7, 5, True, "ab", 11, True),
    (13, 7, 5, True, "aa", 11, False),
    (70, 3, 2, False, "aa", 6, True),
    (1, 1, 8, False, "ab", 5, False),
    (2, 9, 1, True, "aa", 7, True),
    (64, 10, 3, False, "ab", 8, True),  # whole-row work-groups: row-staged reads
]


@pytest.mark.parametrize("nx,ny,nz,walls,streaming,steps,general", CASES)
def test_random_forced_fp64_elementwise(orc, nx, ny, nz, walls, streaming, steps, general):
    say(f"raw fp64 {nx}x{ny}x{nz} walls={walls} {streaming} steps={steps} general={general}")
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=nx * 17 + ny * 5 + nz, umax=0.06, fmax=2e-3)
    rng = np.random.default_rng(nx * ny + nz)
    om = rng.uniform(0.5, 1.95)
    ob, oh = (rng.uniform(0.5, 1.9), rng.uniform(0.6, 1.9, 9)) if general else (1.0, None)
    g = gpu_run(nx, ny, nz, rho, u, steps, "fp64", streaming, omega=om, omega_bulk=ob, omega_hi=oh, force=F,
                walls=walls, moments="raw")
    o = oracle_run(orc, rho, u, steps, om, ob, oh, F=F, walls=walls, mode=orc.RM_DEFINITION)
    err = np.abs(g["f"] - o["f"]).max()
    say(f"  max |f_gpu - f_oracle| = {err:.3e}")
    assert err < 1e-13
    assert rel_l2(g["u"], o["u"]) < 1e-12
    assert rel_l2_fluct(g["rho"], o["rho"]) < 1e-11


def test_unit_rates_match_central_moment_lattice():
    """K = I: raw and central collisions give the same populations (FP64
    round-off apart)."""
    nx, ny, nz, steps = 12, 9, 7, 6
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=91, umax=0.06, fmax=2e-3)
    a = gpu_run(nx, ny, nz, rho, u, steps, "fp64", "ab", omega=1.0, force=F, moments="raw")
    b = gpu_run(nx, ny, nz, rho, u, steps, "fp64", "ab", omega=1.0, force=F, moments="central")
    assert np.abs(a["f"] - b["f"]).max() < 1e-15
    c = gpu_run(nx, ny, nz, rho, u, steps, "fp64", "ab", omega=1.7, force=F, moments="raw")
    d = gpu_run(nx, ny, nz, rho, u, steps, "fp64", "ab", omega=1.7, force=F, moments="central")
    assert np.abs(c["f"] - d["f"]).max() > 1e-9  # and differ otherwise


HALF_U_TOL = {"fp32": 1e-5, "fp16": 1e-3, "bf16": 5e-3}


@pytest.mark.parametrize("precision,streaming", [("fp32", "ab"), ("fp32", "aa"), ("fp16", "ab"), ("bf16", "aa")])
def test_config2_recipe_vs_oracle(orc, precision, streaming):
    """Config-2 recipe at 32^3 (Taylor-Green U0 = 0.05 + noise, nu = 1e-3,
    Kolmogorov force), 200 steps: relative L2 on u within the bound of the
    storage precision (the same bounds as the central-moment lattice)."""
    n, steps, nu = 32, 200, 1e-3
    om = inputs.omega_from_nu(nu)
    say(f"raw {precision} {streaming} config2 recipe")
    rho, u = inputs.taylor_green_noise(n, 0.05, 1e-4, seed=20101628)
    F = inputs.kolmogorov_force(n, n, n, 1e-6)
    g = gpu_run(n, n, n, rho, u, steps, precision, streaming, omega=om, force_mode=L.LBM_FORCE_KOLMOGOROV,
                kolmogorov_amp=1e-6, want_pops=False, moments="raw")
    o = oracle_run(orc, rho, u, steps, om, F=F, mode=orc.RM_DEFINITION)
    err_u, err_r = rel_l2(g["u"], o["u"]), rel_l2(g["rho"], o["rho"])
    say(f"  rel L2 u = {err_u:.3e}, rho = {err_r:.3e}")
    assert err_u < HALF_U_TOL[precision]
    assert err_r < (1e-5 if precision == "fp32" else 1e-3)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ab_equals_aa_bitwise(precision):
    nx, ny, nz, steps = 24, 10, 6, 13
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=78, umax=0.05, fmax=1e-3)
    kw = dict(omega=1.9, omega_hi=[1.3] * 9, force=F, walls=True, moments="raw")
    a = gpu_run(nx, ny, nz, rho, u, steps, precision, "ab", **kw)
    b = gpu_run(nx, ny, nz, rho, u, steps, precision, "aa", **kw)
    assert np.array_equal(a["f"], b["f"])


def test_row_staged_step_is_bitwise_identical(monkeypatch):
    nx, ny, nz = 64, 44, 12
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=34, umax=0.05)
    kw = dict(omega=1.85, force_mode=L.LBM_FORCE_KOLMOGOROV, kolmogorov_amp=1e-4, moments="raw")
    staged = gpu_run(nx, ny, nz, rho, u, 7, "fp32", "ab", **kw)
    monkeypatch.setenv("LBM_ROW_STAGING", "0")
    direct = gpu_run(nx, ny, nz, rho, u, 7, "fp32", "ab", **kw)
    assert np.array_equal(staged["f"], direct["f"])


def test_network_is_rejected():
    p = L.make_params(16, 16, 16, precision="fp32", moments="raw")
    lat = L.Lattice(p)
    try:
        net = L.Mlp(np.zeros(L.MLP_NPARAM, dtype=np.float32), np.ones(11, dtype=np.float32))
        with pytest.raises(L.LbmError) as e:
            lat.attach_mlp(net)
        assert e.value.code == L.LBM_EUNSUPPORTED
        net.close()
    finally:
        lat.close()


def test_full_size_sampled_single_step(orc):
    """256^3 FP32 A-B, tuned launch (as timed): one step from the GPU's own
    state recomputed by the oracle at sampled nodes, incl. every face, edge
    and corner class."""
    import torch

    S = 256
    say(f"raw full size {S}^3 fp32 ab")
    om = inputs.omega_from_nu(1e-3)
    rho, u = inputs.taylor_green_noise(S, 0.05, 1e-4, seed=20101628)
    p = L.make_params(S, S, S, precision="fp32", streaming="ab", omega=om,
                      force_mode=L.LBM_FORCE_KOLMOGOROV, kolmogorov_amp=1e-6, moments="raw")
    lat = L.Lattice(p)
    try:
        lat.tune(4)
        lat.init(torch.from_numpy(rho).cuda(), torch.from_numpy(u).cuda())
        lat.step(10)
        f_t = lat.get_populations().cpu().numpy()
        lat.step(1)
        rng = np.random.default_rng(10)
        ends = [0, 1, S - 2, S - 1]
        picks = list(rng.integers(0, S ** 3, 2000)) + [x + S * (y + S * z) for x in ends for y in ends for z in ends]
        nodes = np.unique(np.array(picks, dtype=np.int64))
        f1 = lat.get_populations()
        got = f1.reshape(19, -1)[:, torch.from_numpy(nodes).cuda()].T.cpu().numpy()
        del f1
    finally:
        lat.close()
    F = inputs.kolmogorov_force(S, S, S, 1e-6)
    want = orc.step_at(f_t, nodes, orc.K(om), F=F, mode=orc.RM_DEFINITION)
    err = np.abs(got - want).max()
    say(f"  max |f_gpu - f_oracle| over {len(nodes)} nodes = {err:.3e}")
    assert err < 2e-8


# --------------------------------------------------------------------------
# D3Q27 raw-moment variant (the raw moments of the D3Q27 lattice's
# equilibrium and forcing term, N = I)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("nx,ny,nz,walls,streaming,steps", [
    (12, 10, 8, False, "ab", 7), (9, 6, 5, True, "aa", 9), (1, 3, 7, False, "aa", 5)])
def test_d3q27_fp64_elementwise(orc, nx, ny, nz, walls, streaming, steps):
    say(f"raw d3q27 fp64 {nx}x{ny}x{nz} walls={walls} {streaming}")
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=nx + 5 * ny + 3 * nz, umax=0.06, fmax=2e-3)
    om = 1.64
    g = gpu_run(nx, ny, nz, rho, u, steps, "fp64", streaming, omega=om, force=F, walls=walls, q=27, moments="raw")
    q = orc.d3q27
    fo = q.run(q.init(rho, u), steps, q.K(om), F=F, walls_y=walls, raw=True)
    err = np.abs(g["f"] - fo).max()
    say(f"  max |f_gpu - f_oracle| = {err:.3e}")
    assert err < 1e-13


def test_d3q27_fp32_vs_oracle(orc):
    n, steps = 24, 60
    om = inputs.omega_from_nu(1e-3)
    rho, u = inputs.taylor_green_noise(n, 0.05, 1e-4, seed=8)
    g = gpu_run(n, n, n, rho, u, steps, "fp32", "ab", omega=om, q=27, force_mode=L.LBM_FORCE_KOLMOGOROV,
                kolmogorov_amp=1e-6, moments="raw")
    q = orc.d3q27
    F = inputs.kolmogorov_force(n, n, n, 1e-6)
    fo = q.run(q.init(rho, u), steps, q.K(om), F=F, raw=True)
    _, uo = q.moments(fo, F)
    err = rel_l2(g["u"], uo)
    say(f"  raw d3q27 fp32 rel L2 u = {err:.3e}")
    assert err < 1e-5
