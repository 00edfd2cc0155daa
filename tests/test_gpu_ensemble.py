"""Batched ensemble of periodic boxes (one persistent launch per step, HIP
graph replay) against the FP64 oracle run box by box, and against the
single-lattice path."""
import numpy as np
import pytest

from gpu_helpers import say
from paper_2010_01628_amd import inputs
from paper_2010_01628_amd import lbm as L

pytestmark = pytest.mark.gpu

# sides that leave ragged last tiles (256-node tiles) and one box smaller than a tile
BOXES = [(6, 1.70), (9, 1.90), (5, 1.20), (12, 1.95), (7, 0.80)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


def box_fields(b, n):
    rho, u, _ = inputs.random_lattice_fields(n, n, n, seed=100 + b, umax=0.05)
    return rho, u


def make_ensemble(boxes, q=19, precision="fp64"):
    ens = L.Ensemble(boxes, q=q, precision=precision)
    for b, (n, _) in enumerate(boxes):
        ens.init(b, *box_fields(b, n))
    return ens


def oracle_box(orc, q, b, n, om, steps):
    rho, u = box_fields(b, n)
    mod = orc if q == 19 else orc.d3q27
    return mod.run(mod.init(rho, u), steps, mod.K(om))


@pytest.mark.parametrize("q", [19, 27])
def test_boxes_match_oracle_fp64(orc, q):
    steps = 21  # one 16-step graph replay plus single steps
    say(f"ensemble fp64 q={q}: {len(BOXES)} boxes, {steps} steps")
    ens = make_ensemble(BOXES, q=q)
    ens.step(steps)
    assert ens.step_count == steps
    assert ens.nodes == sum(n ** 3 for n, _ in BOXES)
    for b, (n, om) in enumerate(BOXES):
        g = ens.get_populations(b)
        o = oracle_box(orc, q, b, n, om, steps)
        err = np.abs(g - o).max()
        say(f"  box {b} (L={n}, omega={om}): max |f_gpu - f_oracle| = {err:.3e}")
        assert err < 1e-12
    ens.close()


def test_energy_and_mass_match_oracle(orc):
    steps = 6
    ens = make_ensemble(BOXES, q=19)
    ens.step(steps)
    ke, mass = ens.energy()
    for b, (n, om) in enumerate(BOXES):
        o = oracle_box(orc, 19, b, n, om, steps)
        rho, u = orc.moments(o)
        ke_o = 0.5 * float(np.sum(rho * np.sum(u * u, axis=0)))
        rho0, _ = box_fields(b, n)
        say(f"  box {b}: KE gpu {ke[b]:.12e} oracle {ke_o:.12e}; mass {mass[b]:.15e} initial {rho0.sum():.15e}")
        assert abs(ke[b] - ke_o) <= 1e-11 * ke_o
        assert abs(mass[b] - rho0.sum()) <= 1e-12 * rho0.sum()
    ens.close()


@pytest.mark.parametrize("q", [19, 27])
def test_fp32_matches_single_lattice_bitwise(q):
    """Per node the ensemble runs the same collision as the single-lattice AB
    kernel, so each box equals a standalone FP32 lattice bit for bit."""
    steps = 5
    ens = make_ensemble(BOXES, q=q, precision="fp32")
    ens.step(steps)
    for b, (n, om) in enumerate(BOXES):
        p = L.make_params(n, n, n, precision="fp32", streaming="ab", omega=om, q=q)
        lat = L.Lattice(p)
        lat.init(*box_fields(b, n))
        lat.step(steps)
        want = lat.get_populations().cpu().numpy()
        got = ens.get_populations(b)
        say(f"  q={q} box {b}: max |ensemble - lattice| = {np.abs(got - want).max():.3e}")
        assert np.array_equal(got, want)
        lat.close()
    ens.close()


@pytest.mark.parametrize("q,learned", [(19, False), (27, False), (19, True)])
def test_64bit_addressing_is_bitwise_identical(q, learned, monkeypatch):
    """Boxes whose population arrays are below 4 GiB take 32-bit offsets
    against the box's array base; forcing 64-bit addresses (the path of
    larger boxes) gives the same values, bit for bit."""
    boxes = [(12, 1.85), (7, 1.7), (10, 1.9)]
    mlp = L.Mlp(0.08 * np.random.default_rng(3).normal(size=L.MLP_NPARAM), SCALES) if learned else None
    out = []
    for off32 in ("1", "0"):
        monkeypatch.setenv("LBM_OFF32", off32)
        ens = make_ensemble(boxes, q=q, precision="fp32")
        if mlp is not None:
            ens.set_mlp(mlp)
        ens.step(9)
        out.append([ens.get_populations(b) for b in range(len(boxes))])
        ens.close()
    if mlp is not None:
        mlp.close()
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("q", [19, 27])
def test_wavefront_cap_is_bitwise_identical(q, monkeypatch):
    """The plain step's cap on resident wavefronts per SIMD (an LDS
    allocation; LBM_WAVES_PER_SIMD) changes no value, bit for bit."""
    boxes = [(12, 1.85), (7, 1.7), (10, 1.9)]
    out = []
    for cap in ("5", "0", "2"):
        monkeypatch.setenv("LBM_WAVES_PER_SIMD", cap)
        ens = make_ensemble(boxes, q=q, precision="fp32")
        ens.step(9)
        out.append([ens.get_populations(b) for b in range(len(boxes))])
        ens.close()
    for run in out[1:]:
        for a, b in zip(out[0], run):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("chunk", ["2", "16", "0", "3", "17"])
def test_graph_replay_equals_single_steps(chunk, monkeypatch):
    """Stepping through captured graphs of `chunk` steps (0: no graph; odd
    lengths are rounded down to even) gives the same bits as one call per
    step, including odd totals."""
    boxes = [(16, 1.9), (20, 1.6), (9, 1.3)]
    monkeypatch.setenv("LBM_ENSEMBLE_GRAPH_STEPS", chunk)
    a = make_ensemble(boxes, precision="fp32")
    b = make_ensemble(boxes, precision="fp32")
    a.step(37)
    a.step(3)
    for _ in range(40):
        b.step(1)
    assert a.step_count == b.step_count == 40
    for i in range(len(boxes)):
        assert np.array_equal(a.get_populations(i), b.get_populations(i))
    a.close()
    b.close()


def test_tune_keeps_state(orc):
    """The autotuner times real steps; the state it leaves equals the oracle
    after the same number of steps, and stepping on from there stays exact."""
    boxes = [(24, 1.8), (10, 1.5), (17, 1.2), (8, 1.9)]
    ens = make_ensemble(boxes, precision="fp64")
    grid = ens.tune(4)
    import torch

    ncu = torch.cuda.get_device_properties(0).multi_processor_count
    ntiles = sum((n ** 3 + 255) // 256 for n, _ in boxes)
    assert grid in {min(ncu * m, ntiles) for m in (2, 4, 8, 16, 32, 64)} | {ntiles}
    done = ens.step_count
    assert done % 2 == 0 and done > 0
    ens.step(18)
    say(f"  tuned grid {grid}, steps {ens.step_count}")
    for i, (n, om) in enumerate(boxes):
        o = oracle_box(orc, 19, i, n, om, done + 18)
        assert np.abs(ens.get_populations(i) - o).max() < 1e-12
    ens.close()


SCALES = np.array([0.05, 0.02, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3])


def test_learned_rates_match_single_lattice(orc):
    """Learned-rate ensemble (BF16 MFMA network per node) against a standalone
    lattice with the same network attached (itself checked against the oracle
    in the learned-rate tests)."""
    boxes = [(12, 1.85), (7, 1.7), (10, 1.9)]
    rng = np.random.default_rng(1)
    P = 0.08 * rng.normal(size=L.MLP_NPARAM)
    mlp = L.Mlp(P, SCALES)
    ens = make_ensemble(boxes, precision="fp32")
    ens.set_mlp(mlp)
    steps = 18
    ens.step(steps)
    for b, (n, om) in enumerate(boxes):
        lat = L.Lattice(L.make_params(n, n, n, precision="fp32", streaming="ab", omega=om))
        lat.init(*box_fields(b, n))
        lat.attach_mlp(mlp)
        lat.step(steps)
        want = lat.get_populations().cpu().numpy()
        got = ens.get_populations(b)
        d = np.abs(got - want).max()
        say(f"  box {b}: max |ensemble - lattice| = {d:.3e}")
        assert d == 0.0
        lat.close()
    assert ens.fallback_count() == 0
    ens.close()
    mlp.close()


def test_graph_follows_network_swaps(monkeypatch):
    """Captured step loops carry the attached network's weights: after
    switching between two live networks (and back to the paper's rates)
    between graph-length chunks, replays equal single steps bit for bit."""
    boxes = [(12, 1.85), (7, 1.7), (10, 1.9)]
    rng = np.random.default_rng(8)
    nets = [L.Mlp(0.08 * rng.normal(size=L.MLP_NPARAM), SCALES), L.Mlp(0.08 * rng.normal(size=L.MLP_NPARAM), SCALES)]
    a = make_ensemble(boxes, precision="fp32")
    b = make_ensemble(boxes, precision="fp32")
    for net in (nets[0], nets[1], nets[0], None, nets[1]):
        a.set_mlp(net)
        b.set_mlp(net)
        monkeypatch.setenv("LBM_ENSEMBLE_GRAPH_STEPS", "8")
        a.step(16)
        monkeypatch.setenv("LBM_ENSEMBLE_GRAPH_STEPS", "0")
        b.step(16)
    for i in range(len(boxes)):
        assert np.array_equal(a.get_populations(i), b.get_populations(i))
    # the swaps changed the result: a run with the first network throughout differs
    c = make_ensemble(boxes, precision="fp32")
    c.set_mlp(nets[0])
    c.step(80)
    assert not np.array_equal(a.get_populations(0), c.get_populations(0))
    for x in (a, b, c):
        x.close()
    for net in nets:
        net.close()


def test_learned_fallback_counts():
    """A network whose rates all leave (0, 2) sends every node back to the
    paper's rates: the ensemble then equals the plain one and counts each node."""
    boxes = [(9, 1.7), (6, 1.4)]
    P = np.zeros(L.MLP_NPARAM)
    P[-9:] = 1.5
    mlp = L.Mlp(P, SCALES)
    a = make_ensemble(boxes, precision="fp32")
    b = make_ensemble(boxes, precision="fp32")
    a.set_mlp(mlp)
    a.step(4)
    b.step(4)
    for i in range(len(boxes)):
        assert np.array_equal(a.get_populations(i), b.get_populations(i))
    assert a.fallback_count() == 4 * sum(n ** 3 for n, _ in boxes)
    a.close()
    b.close()
    mlp.close()


def test_ensemble_workload_shapes_run():
    """The seeded ensemble workload (64 boxes of 48/64/96 nodes a side) steps
    and conserves every box's mass in FP32 to round-off."""
    spec = inputs.ensemble_boxes()
    boxes = [(n, inputs.omega_from_nu(nu)) for n, nu, _ in spec]
    ens = L.Ensemble(boxes, q=19, precision="fp32")
    m0 = []
    for b, (n, nu, seed) in enumerate(spec):
        rho, u = inputs.random_phase_field(n, 0.04, seed=seed)
        ens.init(b, rho, u)
        m0.append(rho.sum())
    ke0, mass0 = ens.energy()
    ens.step(20)
    ke, mass = ens.energy()
    say(f"  {len(boxes)} boxes, {ens.nodes} nodes: KE {ke0.sum():.6e} -> {ke.sum():.6e}")
    assert np.all(ke < ke0) and np.all(ke > 0.5 * ke0)
    assert np.max(np.abs(mass - np.array(m0)) / np.array(m0)) < 1e-5
    ens.close()


def test_bad_arguments():
    with pytest.raises(L.LbmError):
        L.Ensemble([(8, 1.0)], q=20)
    with pytest.raises(L.LbmError):
        L.Ensemble([(8, 1.0)], precision="fp16")
    with pytest.raises(L.LbmError):
        L.Ensemble([(8, 2.0)])
    with pytest.raises(L.LbmError):
        L.Ensemble([(1, 1.0)])
    ens = L.Ensemble([(8, 1.0)], q=27)
    mlp = L.Mlp(None, SCALES)
    with pytest.raises(L.LbmError):
        ens.set_mlp(mlp)
    ens.close()
    mlp.close()
