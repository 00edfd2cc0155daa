"""Pins of the learned-rate part of the oracle (readings L1-L5, mlp_oracle.c)."""
import numpy as np
import pytest

from paper_2010_01628_amd import inputs


@pytest.fixture(scope="module")
def M(orc):
    return orc.mlp


def small_params(M, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    return scale * rng.normal(size=M.nparam())


def test_parameter_count_and_layout(M):
    assert M.nparam() == 32 * 11 + 32 + 32 * 32 + 32 + 9 * 32 + 9 == 1737
    P = np.arange(1737.0)
    u = M.unpack(P)
    assert u["W1"][0, 0] == 0 and u["b1"][0] == 352 and u["W2"][0, 0] == 384 and u["b3"][-1] == 1736


def test_bf16_rounding_matches_torch(M):
    """Round-to-nearest-even to bfloat16, checked against torch's converter."""
    import torch

    rng = np.random.default_rng(0)
    vals = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-6, 3, 2000),
                           [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 3.0e-5]])
    want = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    got = np.array([M.bf16(v) for v in vals])
    assert np.array_equal(got, want)


def test_forward_matches_torch_layers(M):
    """The network of reading L2 equals Linear-ReLU-Linear-ReLU-Linear from
    torch.nn in float64 with the same weights."""
    import torch

    P = small_params(M, 1, 0.3)
    u = M.unpack(P)
    net = torch.nn.Sequential(torch.nn.Linear(11, 32), torch.nn.ReLU(), torch.nn.Linear(32, 32), torch.nn.ReLU(),
                              torch.nn.Linear(32, 9)).double()
    with torch.no_grad():
        for layer, (w, b) in zip([net[0], net[2], net[4]], [("W1", "b1"), ("W2", "b2"), ("W3", "b3")]):
            layer.weight.copy_(torch.from_numpy(u[w]))
            layer.bias.copy_(torch.from_numpy(u[b]))
    rng = np.random.default_rng(2)
    for _ in range(20):
        x = rng.normal(size=11)
        z, _ = M.forward(P, x)
        want = net(torch.from_numpy(x)).detach().numpy()
        assert np.allclose(z, want, atol=1e-14)


def test_fallback_rule(M):
    r, fb = M.rates(np.full(9, 0.3))
    assert not fb and np.allclose(r, 1.3)
    z = np.zeros(9)
    z[4] = 1.0  # omega = 2 is outside (0, 2)
    r, fb = M.rates(z)
    assert fb and np.array_equal(r, np.ones(9))
    z[4] = -1.5
    r, fb = M.rates(z)
    assert fb and np.array_equal(r, np.ones(9))


def test_features_vanish_at_equilibrium(orc, M):
    """At f = f_eq every non-equilibrium CM is zero: x = [(rho-1)/s0, 0, ..., 0]."""
    rng = np.random.default_rng(3)
    scales = rng.uniform(0.5, 2.0, 11)
    for _ in range(10):
        rho = 1 + 0.05 * rng.uniform(-1, 1)
        u = rng.uniform(-0.1, 0.1, 3)
        k = orc.T(u) @ orc.feq(rho, u)
        x = M.features(rho, k, scales)
        assert np.isclose(x[0], (rho - 1) / scales[0])
        assert np.allclose(x[1:], 0.0, atol=1e-14)


def test_constant_network_reproduces_fixed_rates(orc, M):
    """W = 0: the network outputs b3 everywhere, so a step equals the plain
    D3Q19 step with omega_hi = 1 + b3 (bitwise) -- output j drives row 10 + j.
    b3 = 0 gives the paper's scheme."""
    nx, ny, nz = 5, 4, 3
    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=4, umax=0.05, fmax=1e-3)
    f = orc.init(rho, u)
    rng = np.random.default_rng(5)
    for b3 in (np.zeros(9), rng.uniform(-0.6, 0.6, 9)):
        P = np.zeros(M.nparam())
        P[-9:] = b3
        g, fb = M.step(f, 1.8, P, np.ones(11), F=F)
        want = orc.step(f, orc.K(1.8, 1.0, 1.0 + b3), F=F)
        assert fb == 0
        assert np.array_equal(g, want)


def test_fallback_reproduces_paper_scheme(orc, M):
    nx, ny, nz = 4, 4, 4
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=6)
    f = orc.init(rho, u)
    P = np.zeros(M.nparam())
    P[-9:] = 1.5  # every rate 2.5: every node falls back
    g, fb = M.step(f, 1.6, P, np.ones(11))
    assert fb == nx * ny * nz
    assert np.array_equal(g, orc.step(f, orc.K(1.6)))


def test_gradient_matches_central_differences(orc, M):
    """FP64 backpropagation (MLP, rate-linear collision, streaming adjoint)
    equals central finite differences of the loss for every parameter."""
    nx, ny, nz = 4, 3, 3
    rng = np.random.default_rng(7)
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=8, umax=0.08, drho=0.05)
    f = orc.init(rho, u) * (1 + 0.05 * rng.uniform(-1, 1, (19, nz, ny, nx)))
    target = np.stack([rho, *(rho * u), *(rho * (u[[0, 1, 2, 0, 0, 1]] * u[[0, 1, 2, 1, 2, 2]]))])
    target[0] += 0.01 * rng.normal(size=rho.shape)
    target[4:7] += 1.0 / 3.0
    P = small_params(M, 9, 0.2)
    scales = rng.uniform(0.2, 0.5, 11)
    sigma = np.array([1e-2, 4e-2, 4e-2, 4e-2, 1e-2, 1e-2, 1e-2, 1e-2, 1e-2, 1e-2])
    loss, g, fb = M.loss_grad(f, target, 1.7, P, scales, sigma)
    assert fb == 0 and loss > 0
    eps = 1e-6
    fd = np.zeros_like(g)
    for p in range(M.nparam()):
        Pp, Pm = P.copy(), P.copy()
        Pp[p] += eps
        Pm[p] -= eps
        fd[p] = (M.loss_grad(f, target, 1.7, Pp, scales, sigma, want_grad=False)[0]
                 - M.loss_grad(f, target, 1.7, Pm, scales, sigma, want_grad=False)[0]) / (2 * eps)
    err = np.abs(fd - g).max() / np.abs(g).max()
    assert err < 1e-6, err
    assert np.abs(g).max() > 0


def test_loss_at_paper_rates_is_plain_step_residual(orc, M):
    """With the constant network (rates 1) the loss is the residual of one
    plain D3Q19 step's moments against the target."""
    nx, ny, nz = 4, 4, 3
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=10)
    f = orc.init(rho, u)
    target = np.zeros((10, nz, ny, nx))
    sigma = np.ones(10)
    loss, _, _ = M.loss_grad(f, target, 1.5, np.zeros(M.nparam()), np.ones(11), sigma, want_grad=False)
    g = orc.step(f, orc.K(1.5))
    c, _, _ = orc.tables()
    mono = np.stack([np.ones(19), c[:, 0], c[:, 1], c[:, 2], c[:, 0] ** 2, c[:, 1] ** 2, c[:, 2] ** 2,
                     c[:, 0] * c[:, 1], c[:, 0] * c[:, 2], c[:, 1] * c[:, 2]])
    m = np.einsum("ki,iabc->kabc", mono, g)
    assert np.isclose(loss, np.mean(np.sum(m ** 2, axis=0)), rtol=1e-13)


def test_step_info_flip_effects(orc, M):
    """step_info returns the populations of the BF16-emulating step unchanged;
    with no rounding listed (tie_ulps = 0) every flip effect is zero; listing
    more roundings (a wider tie band) never lowers a node's effect; a network
    whose hidden layers are zero has only its inputs' roundings to flip and
    they cannot move the rates (the first layer's weights are zero)."""
    nx, ny, nz = 6, 5, 4
    rng = np.random.default_rng(12)
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=13, umax=0.05)
    f = orc.init(rho, u) * (1 + 0.02 * rng.uniform(-1, 1, (19, nz, ny, nx)))
    P = small_params(M, 14, 0.1)
    scales = np.full(11, 5e-3)
    g, fb = M.step(f, 1.8, P, scales, bf16=True)
    o0, fb0, e0, m0 = M.step_info(f, 1.8, P, scales, tie_ulps=0.0)
    o1, fb1, e1, m1 = M.step_info(f, 1.8, P, scales, tie_ulps=64.0)
    o2, fb2, e2, m2 = M.step_info(f, 1.8, P, scales, tie_ulps=4096.0)
    assert np.array_equal(g, o0) and np.array_equal(g, o1) and fb == fb0 == fb1 == 0
    assert np.all(e0 == 0.0)
    assert np.all(e2 >= e1) and e2.max() > 0.0
    assert np.array_equal(m0, m1)
    Z = P.copy()
    Z[0:1728] = 0.0  # W1, b1, W2, b2, W3 zero: z = b3 whatever the inputs
    _, _, ez, mz = M.step_info(f, 1.8, Z, scales, tie_ulps=4096.0)
    assert np.all(ez == 0.0)
    assert np.allclose(mz, np.min(np.minimum(1 + Z[-9:], 1 - Z[-9:])), atol=1e-15)


def test_rollout_loss_reduces_to_the_one_step_loss(orc, M):
    """One step: the rollout loss (oracle steps + numpy moments) equals the
    C one-step loss; several steps: the mean over steps of the one-step
    losses of the states the learned scheme reaches."""
    nx, ny, nz = 4, 4, 3
    rng = np.random.default_rng(3)
    rho, u, _ = inputs.random_lattice_fields(nx, ny, nz, seed=4, umax=0.06, drho=0.03)
    f = orc.init(rho, u) * (1 + 0.03 * rng.uniform(-1, 1, (19, nz, ny, nx)))
    P = small_params(M, 5, 0.2)
    scales = rng.uniform(0.2, 0.5, 11)
    sigma = rng.uniform(0.01, 0.05, 10)
    targets = M.moments10(f)[None] + 0.01 * rng.normal(size=(3, 10, nz, ny, nx))
    for bf16 in (False, True):
        l1, fb = M.rollout_loss(f, targets[:1], 1.6, P, scales, sigma, bf16=bf16)
        lc, _, _ = M.loss_grad(f, targets[0], 1.6, P, scales, sigma, bf16=bf16, want_grad=False)
        assert fb == 0
        assert abs(l1 - lc) <= 1e-13 * lc
    l3, _ = M.rollout_loss(f, targets, 1.6, P, scales, sigma)
    parts, a = [], f
    for k in range(3):
        parts.append(M.loss_grad(a, targets[k], 1.6, P, scales, sigma, want_grad=False)[0])
        a, _ = M.step(a, 1.6, P, scales)
    assert abs(l3 - np.mean(parts)) <= 1e-13 * l3


def test_moments10_are_the_raw_moments(orc, M):
    """rho, j and Pi of populations built from known moments (the Hermite
    equilibrium's second moments: rho (u u + I/3))."""
    rho, u, _ = inputs.random_lattice_fields(3, 3, 3, seed=12, umax=0.07, drho=0.04)
    m = M.moments10(orc.init(rho, u))
    assert np.allclose(m[0], rho, rtol=0, atol=1e-14)
    assert np.allclose(m[1:4], rho * u, rtol=0, atol=1e-14)
    for k, (a, b) in enumerate(((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))):
        want = rho * u[a] * u[b] + (rho / 3.0 if a == b else 0.0)
        assert np.allclose(m[4 + k], want, rtol=0, atol=1e-14)
