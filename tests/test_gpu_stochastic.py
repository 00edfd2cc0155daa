"""Stochastic rounding of BF16 storage (lbm_params.rounding): unbiased on
average, counter-based (repeatable, the same in A-B and AA), and a storage
option only (nearest-even rounding elsewhere unchanged)."""
import numpy as np
import pytest

from gpu_helpers import say
from paper_2010_01628_amd import inputs
from paper_2010_01628_amd import lbm as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def bf16_round(x):
    """nearest-even bf16 of float32 values (float64 out)"""
    b = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_down_up(x):
    """the two bf16 neighbours of float32 values (towards and away from zero)"""
    b = np.asarray(x, dtype=np.float32).view(np.uint32)
    lo = (b & np.uint32(0xFFFF0000)).view(np.float32).astype(np.float64)
    hi = ((b & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32).astype(np.float64)
    return lo, hi


def lattice(n, precision, rounding="nearest", seed=0, streaming="ab", **kw):
    p = L.make_params(n, n, n, precision=precision, streaming=streaming, rounding=rounding, seed=seed, **kw)
    return L.Lattice(p)


def test_rounds_up_with_the_discarded_fraction():
    """Every node starts from the same BF16-exact populations and takes one
    step with a uniform force: each post-collision population has one FP32
    value x at every node.  Stochastic rounding stores the upper BF16
    neighbour at a fraction of the nodes equal to x's position between the
    two neighbours (binomial, within 6 standard deviations), so the mean
    stored value is x; nearest-even rounding stores one neighbour everywhere."""
    import torch

    n = 48
    N = n ** 3
    w = np.array([1 / 3] + [1 / 18] * 3 + [1 / 36] * 6 + [1 / 18] * 3 + [1 / 36] * 6)
    c = np.array([[0, 0, 0], [-1, 0, 0], [0, -1, 0], [0, 0, -1], [-1, -1, 0], [-1, 1, 0], [-1, 0, -1], [-1, 0, 1],
                  [0, -1, -1], [0, -1, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, -1, 0], [1, 0, 1],
                  [1, 0, -1], [0, 1, 1], [0, 1, -1]], dtype=float)
    rho, ux = 1.0 + 3.7e-3, 0.031
    cu = c[:, 0] * ux
    feq = rho * w * (1 + 3 * cu + 4.5 * cu ** 2 - 1.5 * ux ** 2)
    s = bf16_round(feq - w)  # deviations exactly representable in BF16 (and FP32)
    f0 = np.broadcast_to((s + w)[:, None, None, None], (19, n, n, n)).copy()
    force = dict(force_mode=L.LBM_FORCE_UNIFORM, force=(2.3e-4, -1.1e-4, 0.7e-4), omega=1.7)
    ref = lattice(n, "fp32", **force)
    ref.set_populations(f0)
    ref.step(1)
    x = ref.get_populations().cpu().numpy()[:, 0, 0, 0] - w  # one FP32 value per population
    ref.close()
    lo, hi = bf16_down_up(x)
    out = {}
    for rounding in ("stochastic", "nearest"):
        lat = lattice(n, "bf16", rounding=rounding, seed=1234, **force)
        lat.set_populations(f0)
        lat.step(1)
        out[rounding] = lat.get_populations().cpu().numpy().reshape(19, N) - w[:, None]
        lat.close()
        torch.cuda.synchronize()
    checked = 0
    for i in range(19):
        if hi[i] == lo[i]:
            continue
        p = (x[i] - lo[i]) / (hi[i] - lo[i])
        if not 1e-3 < p < 1 - 1e-3:  # too close to a BF16 value for the two FP32 collision forms to agree
            continue
        got = out["stochastic"][i]
        assert np.all((np.abs(got - lo[i]) < 1e-12 * abs(lo[i]) + 1e-30) | (np.abs(got - hi[i]) < 1e-12 * abs(hi[i]) + 1e-30))
        frac = np.mean(np.abs(got - hi[i]) < np.abs(got - lo[i]))
        sd = np.sqrt(p * (1 - p) / N)
        say(f"  population {i:2d}: x at {p:.4f} of its BF16 step; rounded up at {frac:.4f} of the nodes "
            f"({(frac - p) / max(sd, 1e-12):+.2f} sd); mean error {np.mean(got) - x[i]:+.2e} of step {hi[i] - lo[i]:.2e}")
        assert abs(frac - p) < 6 * sd + 1e-12
        near = out["nearest"][i]
        assert np.all(near == near[0])  # nearest even: the same value at every node
        checked += 1
    assert checked >= 15


@pytest.mark.parametrize("walls", [False, True])
def test_ab_equals_aa_and_repeats(walls):
    """The random bits depend on (seed, step, node, population) only."""
    nx = 20
    rho, u, F = inputs.random_lattice_fields(nx, nx, nx, seed=5, umax=0.05)
    res = {}
    for key, (streaming, seed) in {"ab": ("ab", 7), "aa": ("aa", 7), "ab2": ("ab", 7), "other": ("ab", 8)}.items():
        lat = lattice(nx, "bf16", rounding="stochastic", seed=seed, streaming=streaming, walls_y=walls, omega=1.85,
                      force_mode=L.LBM_FORCE_UNIFORM, force=(1e-5, 0.0, 0.0))
        lat.init(rho, u)
        lat.step(7)
        res[key] = lat.get_populations().cpu().numpy()
        lat.close()
    assert np.array_equal(res["ab"], res["aa"])
    assert np.array_equal(res["ab"], res["ab2"])
    assert not np.array_equal(res["ab"], res["other"])


def test_only_for_bf16_plain_lattices():
    for bad in (dict(precision="fp16"), dict(precision="fp32"), dict(precision="bf16", q=27),
                dict(precision="bf16", moments="raw")):
        kw = dict(rounding="stochastic")
        kw.update(bad)
        prec = kw.pop("precision")
        with pytest.raises(L.LbmError):
            lattice(8, prec, **kw)
    lat = lattice(8, "bf16", rounding="stochastic")
    mlp = L.Mlp(None, np.ones(11))
    with pytest.raises(L.LbmError):
        lat.attach_mlp(mlp)
    mlp.close()
    lat.close()
