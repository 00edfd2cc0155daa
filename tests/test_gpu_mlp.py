"""Learned higher-order rates on the GPU (BF16 MFMA) against the FP64 oracle
run with the same BF16-rounded weights and BF16 activation rounding."""
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


def gpu_weights(orc, P):
    """What the GPU uses: weight matrices rounded to bf16, biases to float32."""
    Q = np.asarray(P, dtype=np.float32).astype(np.float64)
    u = orc.mlp.unpack(Q)
    for w in ("W1", "W2", "W3"):
        flat = u[w].reshape(-1)
        flat[:] = [orc.mlp.bf16(v) for v in flat]
    return Q


def noneq_state(orc, nx, ny, nz, seed, amp=0.02):
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=seed, umax=0.05)
    rng = np.random.default_rng(seed)
    return orc.init(rho, u) * (1 + amp * rng.uniform(-1, 1, (19, nz, ny, nx)))


def make_lattice(nx, ny, nz, f, omega, **kw):
    p = L.make_params(nx, ny, nz, precision="fp32", streaming=kw.pop("streaming", "ab"), omega=omega, **kw)
    lat = L.Lattice(p)
    lat.init(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    lat.set_populations(f)
    return lat


SCALES = np.array([0.05, 0.02, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3])

# A value the GPU forms in FP32 and rounds to bf16 (a scaled input, a hidden
# activation) can round to the other neighbour than the oracle's FP64 value
# when it lies within the FP32 evaluation error of a bf16 tie.  The oracle
# lists, per node, every rounding within TIE_ULPS x 2^-24 x (the size of the
# terms the value is computed from) of a tie, takes each the other way and
# reports how far the node's post-collision populations move (step_info).  A
# population must then agree with the oracle to FP32 collision accuracy,
# STRICT, plus that possible move of the node it came from.
TIE_ULPS = 64.0
STRICT = 2e-7


def from_source(orc, v, walls):
    """per-node values (nz, ny, nx) -> per population after one step
    (19, nz, ny, nx): the value at the node the population was streamed from
    (the node itself for a population bounced back at a y wall)."""
    c, _, _ = orc.tables()
    out = np.empty((19,) + v.shape, dtype=v.dtype)
    for i in range(19):
        src = np.roll(v, shift=(c[i, 2], c[i, 1], c[i, 0]), axis=(0, 1, 2))
        if walls and c[i, 1] == 1:
            src[:, 0, :] = v[:, 0, :]
        if walls and c[i, 1] == -1:
            src[:, -1, :] = v[:, -1, :]
        out[i] = src
    return out


@pytest.mark.parametrize("streaming,walls,dims", [("ab", False, (16, 12, 8)), ("aa", True, (16, 12, 8)),
                                                  ("ab", False, (96, 5, 3))])
def test_mlp_step_matches_oracle(orc, streaming, walls, dims):
    """(96, 5, 3): two 96-node rows per 192-thread work-group, the x-moving
    populations staged through LDS."""
    nx, ny, nz = dims
    say(f"mlp step parity {streaming} walls={walls}")
    rng = np.random.default_rng(1)
    P = 0.08 * rng.normal(size=L.MLP_NPARAM)
    f0 = noneq_state(orc, nx, ny, nz, 3)
    om = 1.85
    mlp = L.Mlp(P, SCALES)
    lat = make_lattice(nx, ny, nz, f0, om, streaming=streaming, walls_y=walls)
    f0r = lat.get_populations().cpu().numpy()  # FP32-rounded start, shared with the oracle
    lat.attach_mlp(mlp)
    Pg = gpu_weights(orc, P)
    lat.step(1)
    g = lat.get_populations().cpu().numpy()
    o, fb, flip, margin = orc.mlp.step_info(f0r, om, Pg, SCALES, walls_y=walls, tie_ulps=TIE_ULPS)
    bound = STRICT + from_source(orc, flip, walls)
    d = np.abs(g - o)
    say(f"  1 step: max |f_gpu - f_oracle| {d.max():.3e}; max over bound {(d / bound).max():.3f}; "
        f"{(flip > STRICT).sum()} of {flip.size} nodes with a possible tie flip above {STRICT:g} "
        f"(largest {flip.max():.2e}); oracle fallbacks {fb}")
    assert fb == 0 and margin.min() > 1e-2
    assert np.all(d <= bound)
    # three more steps: a flip's effect spreads to the neighbours it streams to
    lat.step(3)
    g4 = lat.get_populations().cpu().numpy()
    o4, fb4 = orc.mlp.run(f0r, 4, om, Pg, SCALES, walls_y=walls, bf16=True)
    d4 = np.abs(g4 - o4)
    say(f"  4 steps: max {d4.max():.3e}, 99.9% quantile {np.quantile(d4, 0.999):.3e}")
    assert fb4 == 0
    assert d4.max() < 4 * (STRICT + flip.max()) and np.quantile(d4, 0.999) < 1e-6
    assert lat.fallback_count() == 0
    lat.close()
    mlp.close()


@pytest.mark.parametrize("precision,unit_roundoff", [("fp16", 2.0 ** -11), ("bf16", 2.0 ** -8)])
def test_mlp_step_16bit_storage_matches_oracle(orc, precision, unit_roundoff):
    """One learned A-B step with FP16- or BF16-shifted storage (the deviation
    s = f - w rho0 stored, rounded to nearest even; the collision in FP32) from
    the decoded start state both sides share: each population agrees with
    the oracle to the FP32 test's bound, plus the stored deviation's
    rounding, at most the unit roundoff u times |s| (plus half the smallest
    FP16 subnormal spacing, 2^-25, for deviations below FP16's normal
    range).  A value within the FP32 bound of a rounding tie may round
    either way; the bound covers that: |fl(x') - x| <= u |x'| + |x' - x|."""
    nx, ny, nz = 16, 12, 8
    say(f"mlp step parity {precision} storage")
    rng = np.random.default_rng(1)
    P = 0.08 * rng.normal(size=L.MLP_NPARAM)
    f0 = noneq_state(orc, nx, ny, nz, 3)
    om = 1.85
    mlp = L.Mlp(P, SCALES)
    lat = L.Lattice(L.make_params(nx, ny, nz, precision=precision, omega=om))
    lat.init(np.ones((nz, ny, nx)), np.zeros((3, nz, ny, nx)))
    lat.set_populations(f0)
    f0r = lat.get_populations().cpu().numpy()  # the stored start, decoded
    assert np.abs(f0r - f0).max() > 0  # the start was rounded to the storage type
    lat.attach_mlp(mlp)
    Pg = gpu_weights(orc, P)
    lat.step(1)
    g = lat.get_populations().cpu().numpy()
    o, fb, flip, margin = orc.mlp.step_info(f0r, om, Pg, SCALES, tie_ulps=TIE_ULPS)
    _, w, _ = orc.tables()
    dev = np.abs(o - w[:, None, None, None])  # rho0 = 1
    fp32_part = STRICT + from_source(orc, flip, False)
    bound = fp32_part * (1 + unit_roundoff) + unit_roundoff * (dev + fp32_part) + 2.0 ** -25
    d = np.abs(g - o)
    say(f"  max |f_gpu - f_oracle| {d.max():.3e}; max over bound {(d / bound).max():.3f}; "
        f"largest stored deviation {dev.max():.2e}; oracle fallbacks {fb}")
    assert fb == 0 and margin.min() > 1e-2
    assert np.all(d <= bound)
    # the rounding is really there: the error is of the storage's size, not FP32's
    assert d.max() > 10 * STRICT
    assert lat.fallback_count() == 0
    lat.close()
    mlp.close()


@pytest.mark.parametrize("bound", ["upper", "lower"])
def test_fallback_decision_near_the_rate_bounds(orc, bound):
    """Output 0 is driven to a rate just inside or just outside 2 (or 0) at
    different nodes.  Where the oracle's rate is farther from the bound than
    the FP32 evaluation error, the GPU takes the same decision (a tie flip
    that changes it is in the oracle's flip effect); there the populations
    agree as in the parity test.  Elsewhere the GPU matches one of the two
    decisions."""
    nx, ny, nz = 16, 12, 8
    rng = np.random.default_rng(21)
    P = 0.05 * rng.normal(size=L.MLP_NPARAM)
    P[1440:1440 + 32] *= 8.0  # row 0 of W3: a wide spread of output 0 over the nodes
    P[1728] = 0.999 if bound == "upper" else -0.999
    f0 = noneq_state(orc, nx, ny, nz, 4)
    om = 1.8
    mlp = L.Mlp(P, SCALES)
    lat = make_lattice(nx, ny, nz, f0, om)
    f0r = lat.get_populations().cpu().numpy()
    lat.attach_mlp(mlp)
    Pg = gpu_weights(orc, P)
    lat.step(1)
    g = lat.get_populations().cpu().numpy()
    o, fb_o, flip, margin = orc.mlp.step_info(f0r, om, Pg, SCALES, tie_ulps=TIE_ULPS)
    plain = orc.step(f0r, orc.K(om))  # every node at the paper's rates
    # a rate is an FP32 sum of 33 terms of size <~ 1 plus one: 2^-18 bounds its error
    ambiguous = np.abs(margin) < 2.0 ** -18
    src_amb = from_source(orc, ambiguous, False)
    bound_p = STRICT + from_source(orc, flip, False)
    fb_g = lat.fallback_count()
    say(f"  {bound}: oracle fallbacks {fb_o}, GPU {fb_g}; nodes within FP32 error of the bound {ambiguous.sum()}; "
        f"margins in [{margin.min():.2e}, {margin.max():.2e}]; largest flip effect {flip.max():.2e}")
    assert 0 < fb_o < nx * ny * nz  # both decisions occur
    assert abs(fb_g - fb_o) <= ambiguous.sum() + (flip > 1e-4).sum()
    d = np.abs(g - o)
    assert np.all(d[~src_amb] <= bound_p[~src_amb])
    either = np.minimum(np.abs(g - o), np.abs(g - plain))
    if src_amb.any():
        assert np.all(either[src_amb] <= bound_p[src_amb])
    lat.close()
    mlp.close()


def test_mlp_64bit_addressing_is_bitwise_identical(orc, monkeypatch):
    """The learned A-B step with 32-bit offsets against each array base and
    with 64-bit addresses (the path of arrays of 4 GiB and more) gives the
    same populations, bit for bit."""
    nx, ny, nz = 64, 10, 6
    rng = np.random.default_rng(2)
    P = 0.08 * rng.normal(size=L.MLP_NPARAM)
    f0 = noneq_state(orc, nx, ny, nz, 9)
    mlp = L.Mlp(P, SCALES)
    out = []
    for off32 in ("1", "0"):
        monkeypatch.setenv("LBM_OFF32", off32)
        lat = make_lattice(nx, ny, nz, f0, 1.8)
        lat.attach_mlp(mlp)
        lat.step(4)
        out.append(lat.get_populations().cpu().numpy())
        assert lat.fallback_count() == 0
        lat.close()
    mlp.close()
    assert np.array_equal(out[0], out[1])


def test_mlp_row_staging_is_bitwise_identical(orc, monkeypatch):
    """The learned A-B step with the x-moving populations staged through
    LDS (work-groups of whole rows, the default where possible) and with
    direct reads gives the same populations, bit for bit."""
    nx, ny, nz = 64, 10, 6
    rng = np.random.default_rng(3)
    P = 0.08 * rng.normal(size=L.MLP_NPARAM)
    f0 = noneq_state(orc, nx, ny, nz, 11)
    mlp = L.Mlp(P, SCALES)
    out = []
    for staging in ("1", "0"):
        monkeypatch.setenv("LBM_ROW_STAGING", staging)
        lat = make_lattice(nx, ny, nz, f0, 1.8)
        assert lat.step_variant == (1 if staging == "1" else 0)
        lat.attach_mlp(mlp)
        lat.step(4)
        out.append(lat.get_populations().cpu().numpy())
        assert lat.fallback_count() == 0
        lat.close()
    mlp.close()
    assert np.array_equal(out[0], out[1])


def test_fallback_is_plain_scheme_bitwise(orc):
    nx, ny, nz = 20, 9, 7
    f0 = noneq_state(orc, nx, ny, nz, 5)
    P = np.zeros(L.MLP_NPARAM)
    P[-9:] = 1.5  # every output rate 2.5: every node falls back
    mlp = L.Mlp(P, SCALES)
    a = make_lattice(nx, ny, nz, f0, 1.7)
    b = make_lattice(nx, ny, nz, f0, 1.7)
    a.attach_mlp(mlp)
    a.step(5)
    b.step(5)
    fa = a.get_populations().cpu().numpy()
    fb_ = b.get_populations().cpu().numpy()
    assert np.array_equal(fa, fb_)
    assert a.fallback_count() == 5 * nx * ny * nz
    a.close()
    b.close()
    mlp.close()


def test_zero_network_is_paper_scheme(orc):
    nx, ny, nz = 16, 8, 6
    f0 = noneq_state(orc, nx, ny, nz, 7)
    mlp = L.Mlp(None, SCALES)
    a = make_lattice(nx, ny, nz, f0, 1.9)
    b = make_lattice(nx, ny, nz, f0, 1.9)
    a.attach_mlp(mlp)
    a.step(4)
    b.step(4)
    assert np.abs(a.get_populations().cpu().numpy() - b.get_populations().cpu().numpy()).max() < 1e-7
    assert a.fallback_count() == 0
    a.close()
    b.close()
    mlp.close()


def test_gradient_matches_oracle(orc):
    """GPU loss and gradient (BF16 products, FP32 accumulation, FP64 sums)
    against the oracle's exact FP64 backpropagation of the same model."""
    import torch

    nx, ny, nz = 16, 8, 8
    rng = np.random.default_rng(11)
    P = 0.1 * rng.normal(size=L.MLP_NPARAM)
    f0 = noneq_state(orc, nx, ny, nz, 9)
    om = 1.8
    mlp = L.Mlp(P, SCALES)
    lat = make_lattice(nx, ny, nz, f0, om)
    f0r = lat.get_populations().cpu().numpy()
    lat.attach_mlp(mlp)
    rho = f0r.sum(axis=0)
    c, _, _ = orc.tables()
    mono = np.stack([np.ones(19), c[:, 0], c[:, 1], c[:, 2], c[:, 0] ** 2, c[:, 1] ** 2, c[:, 2] ** 2,
                     c[:, 0] * c[:, 1], c[:, 0] * c[:, 2], c[:, 1] * c[:, 2]])
    target = np.einsum("ki,iabc->kabc", mono, f0r) + 1e-3 * rng.normal(size=(10, nz, ny, nx))
    sigma = np.array([1e-3, 1e-2, 1e-2, 1e-2, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3])
    mlp.zero_grad()
    tgt = torch.from_numpy(target.astype(np.float32)).cuda()
    loss = lat.accumulate_grad(mlp, tgt, sigma)
    g = mlp.grad()
    Pg = gpu_weights(orc, P)
    tq = target.astype(np.float32).astype(np.float64)
    lo, go, fb = orc.mlp.loss_grad(f0r, tq, om, Pg, SCALES, sigma, bf16=True)
    say(f"  loss gpu {loss:.6e} oracle {lo:.6e}; fallbacks {fb}")
    assert fb == 0
    assert abs(loss - lo) / lo < 1e-4
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    cos = g @ go / (np.linalg.norm(g) * np.linalg.norm(go))
    say(f"  gradient rel L2 err {err:.3e}, cosine {cos:.6f}")
    assert err < 1e-2 and cos > 0.999
    assert lat.step_count == 0  # the state is not advanced
    lat.close()
    mlp.close()


def test_projection_q27_to_q19(orc):
    """GPU projection = solve of the 19 shared raw moments (oracle tables, numpy)."""
    import torch

    n = 12
    rho, u = inputs.random_phase_field(n, 0.04, seed=3)
    p = L.make_params(n, n, n, precision="fp64", q=27, omega=1.9)
    lat = L.Lattice(p)
    lat.init(rho, u)
    lat.step(3)
    f27 = lat.get_populations()
    N = n ** 3
    f19 = torch.empty((19, N), dtype=torch.float64, device="cuda")
    mom = torch.empty((10, N), dtype=torch.float32, device="cuda")
    L.lbm_project_q27(f27.data_ptr(), N, f19.data_ptr(), mom.data_ptr(), lat.stream.cuda_stream)
    torch.cuda.synchronize()
    c27, _, _ = orc.d3q27.tables()
    c19, _, _ = orc.tables()
    monos = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (1, 0, 1),
             (0, 1, 1), (2, 1, 0), (1, 2, 0), (2, 0, 1), (1, 0, 2), (0, 2, 1), (0, 1, 2), (2, 2, 0), (2, 0, 2),
             (0, 2, 2)]
    A27 = np.array([[c27[i, 0] ** a * c27[i, 1] ** b * c27[i, 2] ** d for i in range(27)] for a, b, d in monos])
    A19 = np.array([[c19[i, 0] ** a * c19[i, 1] ** b * c19[i, 2] ** d for i in range(19)] for a, b, d in monos])
    F27 = f27.reshape(27, -1).cpu().numpy()
    want = np.linalg.solve(A19, A27 @ F27)
    assert np.abs(f19.cpu().numpy() - want).max() < 1e-14
    assert np.allclose(mom.cpu().numpy(), (A27 @ F27)[:10], rtol=0, atol=1e-6)
    lat.close()


def test_training_reduces_loss(orc):
    """Adam on the GPU-computed gradient lowers the one-step loss against the
    projected D3Q27 evolution on a 32^3 random-phase field."""
    import torch

    n, nu = 32, 5e-4
    om = inputs.omega_from_nu(nu)
    rho, u = inputs.random_phase_field(n, 0.04, seed=5)
    N = n ** 3
    p27 = L.make_params(n, n, n, precision="fp64", q=27, omega=om)
    q27 = L.Lattice(p27)
    q27.init(rho, u)
    q27.step(20)
    f27 = q27.get_populations()
    f19 = torch.empty((19, N), dtype=torch.float64, device="cuda")
    L.lbm_project_q27(f27.data_ptr(), N, f19.data_ptr(), None, q27.stream.cuda_stream)
    q27.step(1)
    f27b = q27.get_populations()
    tgt = torch.empty((10, N), dtype=torch.float32, device="cuda")
    L.lbm_project_q27(f27b.data_ptr(), N, None, tgt.data_ptr(), q27.stream.cuda_stream)
    torch.cuda.synchronize()
    lat = L.Lattice(L.make_params(n, n, n, precision="fp32", omega=om))
    lat.init(rho, u)
    lat.set_populations(f19)
    rms = lat.feature_rms()
    say(f"  feature rms {np.array2string(rms, precision=2, floatmode='maxprec', formatter={'float_kind': lambda v: f'{v:.2e}'})}")
    scales = np.maximum(rms, 1e-12)
    mlp = L.Mlp(None, scales)
    lat.attach_mlp(mlp)
    sigma = np.array([1e-4, 1e-4, 1e-4, 1e-4, 1e-4, 1e-4, 1e-4, 1e-4, 1e-4, 1e-4])
    losses = []
    for it in range(30):
        mlp.zero_grad()
        losses.append(lat.accumulate_grad(mlp, tgt, sigma))
        mlp.adam_step(3e-3)
    say(f"  loss {losses[0]:.6e} -> {losses[-1]:.6e}")
    assert losses[-1] < losses[0]
    assert lat.fallback_count() >= 0
    lat.close()
    q27.close()
    mlp.close()
