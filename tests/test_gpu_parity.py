"""GPU (HIP, gfx950) parity with the FP64 oracle, through the C ABI.

Tolerances (relative L2 on rho and u after the stated steps): 1e-12 for FP64
storage, 1e-5 for FP32, 1e-3 for FP16 shifted storage and 1.5 times the
storage-only error for BF16 (HALF_U_TOL); populations are also compared
element by element where the precision allows.
"""
import json
import os

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


@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_config1_shear_wave_fp64(orc, streaming):
    """32^3 shear wave, FP64, nu = 1/6, 200 steps: GPU = oracle to 1e-12 and the
    u_x amplitude decays as ((2 + cos k)/3)^t."""
    n, A0, steps = 32, 0.01, 200
    say(f"config1 fp64 {streaming}")
    rho, u = inputs.shear_wave(n, A0)
    g = gpu_run(n, n, n, rho, u, steps, "fp64", streaming)
    o = oracle_run(orc, rho, u, steps)
    assert rel_l2(g["u"], o["u"]) < 1e-12
    assert rel_l2(g["rho"], o["rho"]) < 1e-12
    assert np.abs(g["f"] - o["f"]).max() < 1e-13
    k = 2 * np.pi / n
    z = np.arange(n)
    A = 2.0 / n * np.sum(g["u"][0].mean(axis=(1, 2)) * np.sin(k * z))
    assert abs(A / (A0 * ((2 + np.cos(k)) / 3) ** steps) - 1) < 1e-12
    assert abs(g["diag"][0] - n ** 3) < 1e-9  # sum rho


CASES = [
    # nx, ny, nz, walls, streaming, steps
    (16, 16, 16, False, "ab", 9),
    (16, 16, 16, False, "aa", 9),
    (13, 7, 5, True, "ab", 11),   # ragged: nothing a multiple of the block
    (13, 7, 5, True, "aa", 11),
    (70, 3, 2, False, "aa", 6),   # x spans two wavefronts plus a tail
    (1, 1, 8, False, "ab", 5),    # degenerate x, y (every x/y link wraps to itself)
    (2, 9, 1, True, "aa", 7),
    (96, 5, 3, False, "ab", 7),   # rows of 96: two rows per 192-thread work-group, staged
    (48, 6, 4, False, "aa", 7),   # four rows of 48 per work-group, the odd step staged
    (192, 3, 2, False, "ab", 5),  # one 192-node row per work-group
    (320, 2, 2, False, "aa", 5),  # a 320-node row: staged odd step, even step on 64 x 4 work-groups
]


@pytest.mark.parametrize("nx,ny,nz,walls,streaming,steps", CASES)
def test_random_forced_fp64_elementwise(orc, nx, ny, nz, walls, streaming, steps):
    """Random fields, random force field, general rates: every population
    equal to the oracle's within 1e-13 after an odd number of steps."""
    say(f"random fp64 {nx}x{ny}x{nz} walls={walls} {streaming} steps={steps}")
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=nx * 131 + ny * 7 + nz, umax=0.06, fmax=2e-3)
    rng = np.random.default_rng(nx + ny + nz)
    om, ob, oh = rng.uniform(0.5, 1.95), rng.uniform(0.5, 1.9), rng.uniform(0.6, 1.9, 9)
    g = gpu_run(nx, ny, nz, rho, u, steps, "fp64", streaming, omega=om, omega_bulk=ob, omega_hi=oh, force=F,
                walls=walls)
    o = oracle_run(orc, rho, u, steps, om, ob, oh, F=F, walls=walls)
    assert np.abs(g["f"] - o["f"]).max() < 1e-13
    assert rel_l2(g["u"], o["u"]) < 1e-12
    assert rel_l2_fluct(g["rho"], o["rho"]) < 1e-11


@pytest.mark.parametrize("mode", ["uniform", "kolmogorov"])
def test_force_modes_fp64(orc, mode):
    nx, ny, nz, steps = 12, 20, 6, 10
    say(f"force mode {mode}")
    rho, u = inputs.taylor_green_noise(nx, 0.05, 1e-4, seed=3, shape=(nx, ny, nz))
    if mode == "uniform":
        Fv = (1e-4, -2e-4, 5e-5)
        F = inputs.uniform_force(nx, ny, nz, Fv)
        g = gpu_run(nx, ny, nz, rho, u, steps, "fp64", "ab", omega=1.7, force_mode=L.LBM_FORCE_UNIFORM, uniform=Fv)
    else:
        F = inputs.kolmogorov_force(nx, ny, nz, 1e-3)
        g = gpu_run(nx, ny, nz, rho, u, steps, "fp64", "ab", omega=1.7, force_mode=L.LBM_FORCE_KOLMOGOROV,
                    kolmogorov_amp=1e-3)
    o = oracle_run(orc, rho, u, steps, 1.7, F=F)
    assert np.abs(g["f"] - o["f"]).max() < 1e-13
    assert rel_l2(g["u"], o["u"]) < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ab_equals_aa_bitwise(precision):
    """Same arithmetic per node in both patterns: results are bit-identical."""
    nx, ny, nz, steps = 24, 10, 6, 13
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=77, umax=0.05, fmax=1e-3)
    a = gpu_run(nx, ny, nz, rho, u, steps, precision, "ab", omega=1.9, omega_hi=[1.3] * 9, force=F, walls=True)
    b = gpu_run(nx, ny, nz, rho, u, steps, precision, "aa", omega=1.9, omega_hi=[1.3] * 9, force=F, walls=True)
    assert np.array_equal(a["f"], b["f"])
    assert np.array_equal(a["u"], b["u"])


@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_fp32_parity_config2_recipe(orc, streaming):
    """Config-2 recipe at 32^3 (Taylor-Green U0 = 0.05 + seeded noise, nu = 1e-3,
    Kolmogorov force), FP32: relative L2 on u below 1e-5 after 200 steps."""
    n, steps, nu = 32, 200, 1e-3
    om = inputs.omega_from_nu(nu)
    say(f"fp32 config2 recipe {streaming}")
    rho, u = inputs.taylor_green_noise(n, 0.05, 1e-4, seed=20101628)
    F = inputs.kolmogorov_force(n, n, n, 1e-6)
    g = gpu_run(n, n, n, rho, u, steps, "fp32", streaming, omega=om, force_mode=L.LBM_FORCE_KOLMOGOROV,
                kolmogorov_amp=1e-6, want_pops=False)
    o = oracle_run(orc, rho, u, steps, om, F=F)
    err_u = rel_l2(g["u"], o["u"])
    say(f"  fp32 rel L2 u = {err_u:.3e}, rho-fluct {rel_l2_fluct(g['rho'], o['rho']):.3e}")
    assert err_u < 1e-5
    assert rel_l2(g["rho"], o["rho"]) < 1e-5


# Relative-L2 bound on u per storage precision.  The target for 16-bit storage
# is 1e-3, which FP16 meets.  BF16 cannot on this recipe with any arithmetic:
# its storage rounding alone (the FP64 oracle with the stored deviations
# rounded to BF16 after every step, tests/golden/conditioning.py) costs
# 2.96e-3 on u after 200 steps at 32^3.  BF16 is held to 1.5 times that (the
# margin covers rounding decisions that differ between the GPU's FP32 values
# and the oracle's FP64 ones; 3.0e-3 measured).
_COND = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "conditioning_config2.json")))
HALF_U_TOL = {"fp16": 1e-3, "bf16": 1.5 * _COND["32"]["bf16"]["200"]["u"]}


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_half_storage_error_vs_oracle(orc, precision):
    """FP16 / BF16 shifted storage with FP32 collision, config-2 recipe at 32^3,
    200 steps: relative L2 on u against the FP64 oracle within HALF_U_TOL (the
    1e-3 target for FP16; BF16 misses it and is held to its measured level),
    on rho within 1e-3."""
    n, steps, nu = 32, 200, 1e-3
    om = inputs.omega_from_nu(nu)
    say(f"{precision} config2 recipe")
    rho, u = inputs.taylor_green_noise(n, 0.05, 1e-4, seed=20101628)
    F = inputs.kolmogorov_force(n, n, n, 1e-6)
    g = gpu_run(n, n, n, rho, u, steps, precision, "ab", omega=om, force_mode=L.LBM_FORCE_KOLMOGOROV,
                kolmogorov_amp=1e-6, want_pops=False)
    o = oracle_run(orc, rho, u, steps, om, F=F)
    err_u = rel_l2(g["u"], o["u"])
    err_r = rel_l2(g["rho"], o["rho"])
    say(f"  {precision} rel L2 u = {err_u:.3e}, rho = {err_r:.3e}, rho-fluct = {rel_l2_fluct(g['rho'], o['rho']):.3e}")
    assert err_r < 1e-3
    assert err_u < HALF_U_TOL[precision]


@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_checkpoint_resume_bitwise(streaming):
    """n steps, save populations, restore into a fresh lattice, m more steps ==
    n + m steps uninterrupted, bit for bit (odd n exercises the AA parity)."""
    import torch

    nx, ny, nz = 20, 12, 8
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=5, umax=0.05, fmax=0.0)
    ref = gpu_run(nx, ny, nz, rho, u, 12, "fp32", streaming, omega=1.8)
    p = L.make_params(nx, ny, nz, precision="fp32", streaming=streaming, omega=1.8)
    a = L.Lattice(p)
    a.init(rho, u)
    a.step(5)
    saved = a.get_populations().clone()
    a.close()
    b = L.Lattice(p)
    b.init(rho, u)
    b.step(5)  # same parity as the saved state
    b.set_populations(saved)
    b.step(7)
    f = b.get_populations().cpu().numpy()
    assert b.step_count == 12
    b.close()
    torch.cuda.synchronize()
    assert np.array_equal(f, ref["f"])


def test_set_get_roundtrip_fp64():
    nx, ny, nz = 9, 5, 4
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=2)
    for streaming in ("ab", "aa"):
        for walls in (False, True):
            p = L.make_params(nx, ny, nz, precision="fp64", streaming=streaming, walls_y=walls)
            lat = L.Lattice(p)
            lat.init(rho, u)
            lat.step(3)
            f = lat.get_populations()
            f2 = f.clone() * 1.0001
            lat.set_populations(f2)
            assert lat.get_populations().equal(f2)
            lat.close()


def test_instability_is_reported():
    """A non-finite density makes lbm_step fail with LBM_EUNSTABLE at the next check."""
    nx = ny = nz = 8
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=1)
    rho[3, 4, 5] = np.nan
    p = L.make_params(nx, ny, nz, precision="fp32", check_every=2)
    lat = L.Lattice(p)
    lat.init(rho, u)
    with pytest.raises(L.LbmError) as e:
        lat.step(10)
    assert e.value.code == L.LBM_EUNSTABLE
    assert lat.step_count == 2
    lat.close()


def test_stable_run_passes_checks():
    nx = ny = nz = 8
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=1)
    p = L.make_params(nx, ny, nz, precision="fp32", check_every=3)
    lat = L.Lattice(p)
    lat.init(rho, u)
    lat.step(10)
    assert lat.step_count == 10
    lat.close()


@pytest.mark.parametrize("nx,streaming,precision", [(320, "ab", "fp32"), (320, "aa", "fp16"), (300, "aa", "fp64")])
def test_tuned_wide_rows_are_bitwise_identical(nx, streaming, precision):
    """Rows of 257..512 nodes: the tuner also tries one staged work-group of
    nx threads per row; whatever it keeps, the tuned lattice equals one with
    256-wide direct work-groups after the same steps, bit for bit."""
    import os

    ny, nz = 8, 6
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=36, umax=0.05)

    def make():
        p = L.make_params(nx, ny, nz, precision=precision, streaming=streaming, omega=1.8,
                          force_mode=L.LBM_FORCE_KOLMOGOROV, kolmogorov_amp=1e-4)
        lat = L.Lattice(p)
        lat.init(rho, u)
        return lat

    a = make()
    cfg = a.tune(2)
    taken = a.step_count
    say(f"  tuned nx={nx} {streaming} {precision}: block {cfg[0]}x{cfg[1]}, cache policy {cfg[2]}, staged {cfg[3]}")
    assert cfg[0] in (64, 128, 256, nx) and (cfg[0] <= 256 or cfg[3] == 1)
    a.step(5)
    os.environ["LBM_ROW_STAGING"] = "0"
    try:
        b = make()
    finally:
        del os.environ["LBM_ROW_STAGING"]
    b.step(taken + 5)
    assert np.array_equal(a.get_populations().cpu().numpy(), b.get_populations().cpu().numpy())
    a.close()
    b.close()


@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_tuned_launch_is_bitwise_identical(streaming):
    """The autotuner only changes the work-group shape and cache hints: a tuned
    lattice, stepped on, equals an untuned one after the same number of steps,
    bit for bit; a second lattice of the same kind reuses the cached choice
    without running steps."""
    nx, ny, nz = 40, 24, 16
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=31, umax=0.05, fmax=1e-3)
    import torch

    ff = torch.from_numpy(np.ascontiguousarray(F)).cuda()

    def make():
        p = L.make_params(nx, ny, nz, precision="fp32", streaming=streaming, omega=1.8, walls_y=True,
                          force_mode=L.LBM_FORCE_FIELD, force_field_ptr=ff.data_ptr())
        lat = L.Lattice(p, force_field=ff)
        lat.init(rho, u)
        return lat

    a = make()
    cfg = a.tune(4)
    taken = a.step_count
    say(f"  tuned {streaming}: block {cfg[0]}x{cfg[1]}, cache policy {cfg[2]}, {taken} steps")
    assert taken > 0
    a.step(7)
    b = make()
    b.step(taken + 7)
    assert np.array_equal(a.get_populations().cpu().numpy(), b.get_populations().cpu().numpy())
    c = make()
    assert c.tune(4) == cfg and c.step_count == 0
    for lat in (a, b, c):
        lat.close()


def test_xcd_interleaved_grid_is_bitwise_identical(monkeypatch):
    """The optional XCD-interleaved step grid visits every node once: same bits."""
    nx, ny, nz = 64, 48, 32
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=32, umax=0.05)
    ref = gpu_run(nx, ny, nz, rho, u, 9, "fp32", "ab", omega=1.7)
    monkeypatch.setenv("LBM_XCD_CHUNK", "4")
    got = gpu_run(nx, ny, nz, rho, u, 9, "fp32", "ab", omega=1.7)
    assert np.array_equal(ref["f"], got["f"])


@pytest.mark.parametrize("precision,streaming,q", [
    ("fp32", "ab", 19), ("fp16", "ab", 19), ("fp32", "aa", 19), ("fp16", "aa", 19), ("bf16", "aa", 19),
    ("fp64", "aa", 19), ("fp32", "aa", 27), ("fp64", "ab", 27)])
def test_row_staged_step_is_bitwise_identical(precision, streaming, q, monkeypatch):
    """Whole-row work-groups stage the x-moving populations through LDS (the
    A-B reads; the AA odd step's reads and writes); the values are the same
    as direct accesses, bit for bit.  An odd step count ends on an odd AA
    step."""
    nx, ny, nz = 64, 44, 12  # 64-wide rows: one work-group per 4 rows, ragged in y
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=33, umax=0.05)
    kw = dict(omega=1.85, force_mode=L.LBM_FORCE_KOLMOGOROV, kolmogorov_amp=1e-4, q=q)
    monkeypatch.setenv("LBM_ROW_STAGING", "1")
    staged = gpu_run(nx, ny, nz, rho, u, 7, precision, streaming, **kw)
    monkeypatch.setenv("LBM_ROW_STAGING", "0")
    direct = gpu_run(nx, ny, nz, rho, u, 7, precision, streaming, **kw)
    assert np.array_equal(staged["f"], direct["f"])


@pytest.mark.parametrize("nx", [320, 512, 768, 1024])
@pytest.mark.parametrize("precision,streaming,q", [
    ("fp32", "ab", 19), ("fp32", "aa", 19), ("fp16", "ab", 19), ("fp16", "aa", 19), ("fp64", "aa", 19),
    ("fp32", "aa", 27)])
def test_wide_row_staged_step_is_bitwise_identical(nx, precision, streaming, q, monkeypatch):
    """Rows of 257..1024 nodes: one work-group of nx threads per row stages
    the x-moving populations where the staging rows fit in 64 KB of LDS (the
    AA even step runs on 256-wide work-groups of the same launch; FP64 and
    D3Q27 beyond 512 keep direct accesses); the values equal those of
    256-wide work-groups with direct accesses, bit for bit.  An odd step
    count ends on an odd AA step."""
    ny, nz = 6, 5
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=35, umax=0.05)
    kw = dict(omega=1.8, force_mode=L.LBM_FORCE_KOLMOGOROV, kolmogorov_amp=1e-4, q=q)
    monkeypatch.setenv("LBM_ROW_STAGING", "1")
    staged = gpu_run(nx, ny, nz, rho, u, 5, precision, streaming, **kw)
    monkeypatch.setenv("LBM_ROW_STAGING", "0")
    direct = gpu_run(nx, ny, nz, rho, u, 5, precision, streaming, **kw)
    assert np.array_equal(staged["f"], direct["f"])


@pytest.mark.parametrize("precision,streaming,walls,q", [
    ("fp32", "ab", False, 19), ("fp32", "aa", False, 19), ("fp64", "aa", True, 19), ("fp32", "ab", False, 27),
    ("fp16", "ab", False, 19)])
def test_wavefront_cap_is_bitwise_identical(precision, streaming, walls, q, monkeypatch):
    """The step kernels' cap on resident wavefronts per SIMD (an LDS
    allocation; LBM_WAVES_PER_SIMD, default five for 4- and 8-byte storage)
    changes no value, bit for bit: the default against no cap and against a
    cap of two (FP16 storage: no cap by default, against five).  An odd step
    count ends on an odd AA step."""
    nx, ny, nz = 64, 20, 9
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=46, umax=0.05, fmax=1e-3)
    kw = dict(omega=1.8, omega_hi=[1.4] * 9 if q == 19 else None, force=F, walls=walls, q=q)
    a = gpu_run(nx, ny, nz, rho, u, 7, precision, streaming, **kw)
    for cap in ("0", "2", "5"):
        monkeypatch.setenv("LBM_WAVES_PER_SIMD", cap)
        b = gpu_run(nx, ny, nz, rho, u, 7, precision, streaming, **kw)
        assert np.array_equal(a["f"], b["f"])


@pytest.mark.parametrize("precision,walls,moments", [("fp16", False, "central"), ("bf16", False, "central"),
                                                     ("fp16", True, "central"), ("bf16", True, "central"),
                                                     ("fp16", False, "raw")])
def test_aa_even_load_hint_is_bitwise_identical(precision, walls, moments, monkeypatch):
    """With 16-bit storage the AA even step's loads go with or without the
    streaming hint (chosen by lattice size; LBM_AA_EVEN_CACHED forces either);
    the values are the same, bit for bit.  Streaming hints on (cache policy
    1); an odd step count ends on an odd AA step."""
    nx, ny, nz = 64, 20, 9
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=45, umax=0.05, fmax=1e-3)
    kw = dict(omega=1.8, omega_hi=[1.4] * 9, force=F, walls=walls, moments=moments, cache_policy=1)
    monkeypatch.setenv("LBM_AA_EVEN_CACHED", "1")
    a = gpu_run(nx, ny, nz, rho, u, 7, precision, "aa", **kw)
    monkeypatch.setenv("LBM_AA_EVEN_CACHED", "0")
    b = gpu_run(nx, ny, nz, rho, u, 7, precision, "aa", **kw)
    assert np.array_equal(a["f"], b["f"])


@pytest.mark.parametrize("precision,streaming,walls,q", [
    ("fp32", "ab", False, 19), ("fp16", "aa", True, 19), ("fp64", "ab", True, 19), ("bf16", "ab", True, 19),
    ("fp32", "aa", False, 19), ("fp32", "ab", True, 27), ("fp64", "aa", True, 27)])
def test_64bit_addressing_is_bitwise_identical(precision, streaming, walls, q, monkeypatch):
    """Population arrays of 4 GiB and more take 64-bit addresses; smaller ones
    32-bit offsets against the array base (a scalar base where the array is
    the same for the whole wavefront, a per-lane address where a wall picks it
    per node).  Forcing the 64-bit path on a small lattice gives the same
    values, bit for bit."""
    nx, ny, nz = 64, 20, 9
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=44, umax=0.05, fmax=1e-3)
    kw = dict(omega=1.8, omega_hi=[1.4] * 9 if q == 19 else None, force=F, walls=walls, q=q)
    a = gpu_run(nx, ny, nz, rho, u, 6, precision, streaming, **kw)
    monkeypatch.setenv("LBM_OFF32", "0")
    b = gpu_run(nx, ny, nz, rho, u, 6, precision, streaming, **kw)
    assert np.array_equal(a["f"], b["f"])


@pytest.mark.parametrize("q,eb,nt,lane", [(19, 4, True, 0), (19, 2, False, 0), (19, 2, True, 0), (27, 8, True, 0),
                                          (19, 8, False, 0), (19, 4, True, 8), (19, 4, True, 16), (19, 2, True, 16),
                                          (27, 8, False, 16)])
def test_stream_copy_is_exact(q, eb, nt, lane):
    """The bandwidth reference (the step's loads and stores without its
    arithmetic, one element or 8 / 16 bytes per thread and array) copies every
    element of all q arrays; n = 1000 leaves a ragged last work-group."""
    import torch

    n = 1000
    say(f"stream copy q={q} elem_bytes={eb} nt={nt}")
    dt = {2: torch.int16, 4: torch.int32, 8: torch.int64}[eb]
    gen = torch.Generator().manual_seed(5)
    src = torch.randint(-(1 << 15), 1 << 15, (q * n,), generator=gen, dtype=torch.int64).to(dt).cuda()
    dst = torch.zeros_like(src)
    L.lbm_stream_copy(src.data_ptr(), dst.data_ptr(), n, q, eb, nt, torch.cuda.current_stream().cuda_stream,
                      lane_bytes=lane)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
