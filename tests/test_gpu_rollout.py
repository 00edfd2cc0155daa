"""Rollout training of the learned rates: the loss averaged over several
learned steps and its gradient back-propagated through all of them (the
rates of each step depend on the state it starts from).

The reference is the oracle's FP64 rollout loss (the scheme with the network
evaluated exactly, no BF16 rounding, weights as the GPU holds them): the
GPU's parameter gradient and its gradient with respect to the initial
populations are checked against central differences of that loss along
chosen directions.  The GPU's network runs on BF16 products (activations and
back-propagated errors rounded to BF16), so its gradient differs from the
exact model's by the BF16 rounding of those values.  That difference is
measured on the one-step gradient, whose exact value the oracle gives by
back-propagation in FP64 (test_one_step_against_exact_model_gradient:
4.1e-3 relative L2 on the 16x8x8 case); GRAD_TOL allows 2.5 times it.
"""
import numpy as np
import pytest

from gpu_helpers import say
from paper_2010_01628_amd import inputs
from paper_2010_01628_amd import lbm as L

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-2
NX, NY, NZ = 16, 8, 8
OMEGA = 1.8
SCALES = np.array([0.05, 0.02, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3, 5e-3])
SIGMA = np.array([1e-3, 1e-2, 1e-2, 1e-2, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3, 1e-3])
GROUPS = {"W1": (0, 352), "b1": (352, 384), "W2": (384, 1408), "b2": (1408, 1440), "W3": (1440, 1728),
          "b3": (1728, 1737)}


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


class Case:
    """A non-equilibrium 16x8x8 state, a random network and `steps` targets
    (the moments of the plain scheme's evolution plus noise)."""

    def __init__(self, orc, steps, seed=11):
        import torch

        rng = np.random.default_rng(seed)
        self.P = 0.1 * rng.normal(size=L.MLP_NPARAM)
        rho, u, _ = inputs.random_lattice_fields(NX, NY, NZ, seed=seed + 1, umax=0.05)
        f0 = orc.init(rho, u) * (1 + 0.02 * rng.uniform(-1, 1, (19, NZ, NY, NX)))
        self.mlp = L.Mlp(self.P, SCALES)
        p = L.make_params(NX, NY, NZ, precision="fp32", omega=OMEGA)
        self.lat = L.Lattice(p)
        self.lat.init(np.ones((NZ, NY, NX)), np.zeros((3, NZ, NY, NX)))
        self.lat.set_populations(f0)
        self.f0 = self.lat.get_populations().cpu().numpy()  # as the GPU holds it (FP32)
        self.lat.attach_mlp(self.mlp)
        f, tg = self.f0, []
        for _ in range(steps):
            f = orc.step(f, orc.K(OMEGA))
            tg.append(orc.mlp.moments10(f) + 1e-3 * rng.normal(size=(10, NZ, NY, NX)))
        self.targets = np.array(tg).astype(np.float32).astype(np.float64)
        self.tgt = torch.from_numpy(self.targets.astype(np.float32)).cuda()
        self.Pg = gpu_weights(orc, self.P)

    def close(self):
        self.lat.close()
        self.mlp.close()

    def gpu(self, want_dstate=False):
        self.mlp.zero_grad()
        out = self.lat.accumulate_rollout_grad(self.mlp, self.tgt, SIGMA, want_dstate=want_dstate)
        g = self.mlp.grad()
        self.mlp.zero_grad()
        if want_dstate:
            return out[0], g, out[1].cpu().numpy().astype(np.float64)
        return out, g

    def gpu_weighted(self, w):
        self.mlp.zero_grad()
        loss, per = self.lat.accumulate_rollout_grad(self.mlp, self.tgt, SIGMA, step_weight=w, want_steps=True)
        g = self.mlp.grad()
        self.mlp.zero_grad()
        return loss, per, g

    def loss(self, orc, P=None, f=None, bf16=False):
        P = self.Pg if P is None else P
        f = self.f0 if f is None else f
        lo, fb = orc.mlp.rollout_loss(f, self.targets, OMEGA, P, SCALES, SIGMA, bf16=bf16,
                                      energy_weight=self.energy_weight)
        assert fb == 0
        return lo

    energy_weight = 0.0

    def set_energy_weight(self, w):
        self.energy_weight = w
        self.mlp.set_energy_weight(w)

    def fd_theta(self, orc, v, h=1e-5):
        v = v / np.linalg.norm(v)
        return (self.loss(orc, P=self.Pg + h * v) - self.loss(orc, P=self.Pg - h * v)) / (2 * h)

    def fd_state(self, orc, U, h):
        return (self.loss(orc, f=self.f0 + h * U) - self.loss(orc, f=self.f0 - h * U)) / (2 * h)


def test_one_step_rollout_is_the_one_step_gradient(orc):
    """steps = 1 runs the same kernels as lbm_mlp_accumulate_grad: identical
    loss and gradient."""
    c = Case(orc, 1)
    c.mlp.zero_grad()
    l1 = c.lat.accumulate_grad(c.mlp, c.tgt[0], SIGMA)
    g1 = c.mlp.grad()
    lr, gr = c.gpu()
    assert lr == l1
    assert np.array_equal(gr, g1)
    assert c.lat.step_count == 0
    c.close()


def test_one_step_against_exact_model_gradient(orc):
    """The size of the BF16 effect on the gradient: the GPU's one-step
    gradient against the oracle's exact FP64 back-propagation of the
    unrounded network (the reference the rollout tests use)."""
    c = Case(orc, 1)
    _, g = c.gpu()
    _, ge, fb = orc.mlp.loss_grad(c.f0, c.targets[0], OMEGA, c.Pg, SCALES, SIGMA, bf16=False)
    assert fb == 0
    err = np.linalg.norm(g - ge) / np.linalg.norm(ge)
    say(f"  one-step gradient vs exact FP64 model: rel L2 {err:.3e} (GRAD_TOL {GRAD_TOL})")
    assert err < GRAD_TOL
    c.close()


@pytest.mark.parametrize("steps", [2, 4])
def test_rollout_loss_matches_oracle(orc, steps):
    """The loss against the oracle run with the GPU's BF16 roundings emulated."""
    c = Case(orc, steps)
    lo_gpu, _ = c.gpu()
    lo = c.loss(orc, bf16=True)
    say(f"  {steps} steps: loss gpu {lo_gpu:.8e} oracle {lo:.8e}")
    assert abs(lo_gpu - lo) / lo < 1e-4
    c.close()


@pytest.mark.parametrize("steps", [2, 4])
def test_rollout_parameter_gradient(orc, steps):
    """Directional derivatives of the exact model's rollout loss (central
    differences) along the GPU gradient and along its restriction to each
    parameter block: they equal |g| and |g_block| up to the BF16 effect."""
    c = Case(orc, steps)
    _, g = c.gpu()
    gn = np.linalg.norm(g)
    d = c.fd_theta(orc, g)
    say(f"  {steps} steps: |g| {gn:.6e}, d/dh L(theta + h g/|g|) {d:.6e}")
    assert abs(d - gn) <= GRAD_TOL * gn
    rng = np.random.default_rng(steps)
    for name, (a, b) in GROUPS.items():
        v = np.zeros_like(g)
        v[a:b] = g[a:b]
        nb = np.linalg.norm(v)
        if nb < 1e-6 * gn:
            continue
        d = c.fd_theta(orc, v)
        r = np.zeros_like(g)
        r[a:b] = rng.normal(size=b - a)
        dr = c.fd_theta(orc, r)
        pr = g @ r / np.linalg.norm(r)
        say(f"    {name}: |g| {nb:.4e} fd {d:.4e}; random direction: g.v {pr:+.4e} fd {dr:+.4e}")
        assert abs(d - nb) <= GRAD_TOL * nb
        assert abs(dr - pr) <= GRAD_TOL * nb
    c.close()


@pytest.mark.parametrize("steps", [1, 3])
def test_rollout_state_gradient(orc, steps):
    """dL/df of the initial populations: the derivative along dL/df itself
    is |dL/df|^2, and single entries (the largest ones and random ones, so
    that a misplaced node or population shows) match central differences."""
    c = Case(orc, steps)
    _, _, ds = c.gpu(want_dstate=True)
    n2 = float(np.sum(ds * ds))
    scale = np.abs(c.f0).max()
    h = 1e-7 * scale / np.abs(ds).max()
    d = c.fd_state(orc, ds, h)
    say(f"  {steps} steps: |dL/df|^2 {n2:.6e}, fd along dL/df {d:.6e}")
    assert abs(d - n2) <= GRAD_TOL * n2
    rng = np.random.default_rng(5)
    flat = np.abs(ds).ravel()
    picks = list(np.argsort(flat)[-4:]) + list(rng.integers(0, flat.size, 4))
    for k in picks:
        U = np.zeros_like(ds)
        U.flat[k] = 1.0
        fd = c.fd_state(orc, U, 1e-7 * scale)
        say(f"    entry {np.unravel_index(k, ds.shape)}: gpu {ds.flat[k]:+.6e} fd {fd:+.6e}")
        assert abs(fd - ds.flat[k]) <= GRAD_TOL * flat.max()
    c.close()


def test_step_weights_and_per_step_losses(orc):
    """Per-step losses equal the oracle's (BF16 emulated); weights scale
    each step's loss and its gradient: weights w give sum_k w_k L_k / steps,
    and the gradient is linear in w (the gradient with w = e_1 + 3 e_3 is
    that of e_1 plus three times that of e_3, up to the BF16 rounding of the
    back-propagated errors), which the oracle's weighted loss confirms by
    central differences along the weighted gradient."""
    steps = 3
    c = Case(orc, steps)
    loss, per, g = c.gpu_weighted(None)
    assert abs(loss - per.mean()) <= 1e-12 * loss
    want, _ = orc.mlp.rollout_step_losses(c.f0, c.targets, OMEGA, c.Pg, SCALES, SIGMA, bf16=True)
    say(f"  per-step loss gpu {per} oracle {want}")
    assert np.all(np.abs(per - want) <= 1e-4 * want)
    tiny = 1e-30
    w1 = np.array([1.0, tiny, tiny])
    w3 = np.array([tiny, tiny, 1.0])
    _, p1, g1 = c.gpu_weighted(w1)
    _, p3, g3 = c.gpu_weighted(w3)
    w = w1 + 3 * w3
    lw, pw, gw = c.gpu_weighted(w)
    assert np.allclose(pw, per, rtol=1e-6) and np.allclose(p1, per, rtol=1e-6)
    assert abs(lw - (per[0] + 3 * per[2]) / steps) <= 1e-6 * lw
    # linear up to the BF16 rounding of the back-propagated errors (one BF16
    # step, 2^-8 relative, is the bound: measured 5.6e-4)
    assert np.linalg.norm(gw - (g1 + 3 * g3)) <= 2.0 ** -8 * np.linalg.norm(gw)
    h = 1e-5
    v = gw / np.linalg.norm(gw)
    lp, _ = orc.mlp.rollout_loss(c.f0, c.targets, OMEGA, c.Pg + h * v, SCALES, SIGMA, weights=w)
    lm, _ = orc.mlp.rollout_loss(c.f0, c.targets, OMEGA, c.Pg - h * v, SCALES, SIGMA, weights=w)
    d = (lp - lm) / (2 * h)
    say(f"  weighted: |g| {np.linalg.norm(gw):.6e}, fd {d:.6e}")
    assert abs(d - np.linalg.norm(gw)) <= GRAD_TOL * np.linalg.norm(gw)
    c.close()


def test_energy_term(orc):
    """The kinetic-energy term of the rollout loss: value against the oracle
    (BF16 emulated), parameter gradient and initial-state gradient against
    central differences of the exact model's loss.  The targets' energies
    differ from the scheme's by the noise added to them, and the weight makes
    the term a sizeable part of the loss."""
    steps = 3
    c = Case(orc, steps)
    for bad in (-1.0, float("nan")):
        with pytest.raises(L.LbmError):
            c.mlp.set_energy_weight(bad)
    c.set_energy_weight(2e5)
    lo_gpu, g, ds = c.gpu(want_dstate=True)
    lo = c.loss(orc, bf16=True)
    c.set_energy_weight(0.0)
    lo_moments = c.loss(orc, bf16=True)
    c.set_energy_weight(2e5)
    say(f"  loss gpu {lo_gpu:.8e} oracle {lo:.8e} (moment terms alone {lo_moments:.6e})")
    assert lo > 1.2 * lo_moments
    assert abs(lo_gpu - lo) / lo < 1e-4
    gn = np.linalg.norm(g)
    d = c.fd_theta(orc, g)
    say(f"  |g| {gn:.6e}, d/dh L(theta + h g/|g|) {d:.6e}")
    assert abs(d - gn) <= GRAD_TOL * gn
    n2 = float(np.sum(ds * ds))
    h = 1e-7 * np.abs(c.f0).max() / np.abs(ds).max()
    dsd = c.fd_state(orc, ds, h)
    say(f"  |dL/df|^2 {n2:.6e}, fd along dL/df {dsd:.6e}")
    assert abs(dsd - n2) <= GRAD_TOL * n2
    c.close()
