"""What the trained network gains: D3Q19 with learned higher-order rates
follows D3Q27's kinetic-energy decay more closely than the paper's D3Q19 on
two box sets whose fields it was not trained on -- the seeded 64-box ensemble
workload (sides 48/64/96, 4800 steps) and 16 small boxes (sides 32/48, 1200
steps).  Training: rollouts of 1 to 128 back-propagated steps, each step's
moment loss relative to the paper's scheme, plus the kinetic-energy term.
The held-out one-step and eight-step moment losses are reported and
guarded: matching the energy decay costs some local moment accuracy
(training on the moments alone lowers those losses but raises the small
boxes' decay error).  Over six training seeds of this recipe the learned
losses are 1.01-1.41 (one step) and 1.12-1.47 (eight steps) times the
paper's; the guard, 1.5 and 2 times, catches the runs that trade local
accuracy wholesale (half the energy weight gave eight-step losses of 4.6
and 7.0 times the paper's on two of six seeds, three times the learning
rate one-step losses up to 8.5 times)."""
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


def test_trained_network_tracks_d3q27_better():
    import time

    from paper_2010_01628_amd import learned as LR

    n = 32
    samples = []
    for nu in (1e-4, 3e-4, 1e-3):
        for sd in (1, 2):
            samples += LR.q27_samples(n, nu, 1000 + sd, (10, 150, 300), horizon=128)
    tr = LR.Trainer(samples)
    tr.sigma = tr.per_moment_error()
    assert abs(tr.loss() - 10.0) < 1e-3  # the initial network is the paper's scheme
    t0 = time.perf_counter()
    tr.train(1600, lr=LR.LEARNING_RATE, horizons=LR.ROLLOUT_CURRICULUM, mix=True, normalize=True,
             energy_weight=LR.ENERGY_WEIGHT)
    tr.mlp.set_energy_weight(0.0)  # the held-out losses below are the moment terms
    say(f"  training: {len(samples)} samples, 1600 iterations in {time.perf_counter() - t0:.1f} s")
    held = LR.q27_samples(n, 5e-4, 999, (20, 150), horizon=8)
    for s in held:
        if (s.n, s.omega) not in tr.lats:
            lat = L.Lattice(L.make_params(n, n, n, precision="fp32", omega=s.omega))
            lat.attach_mlp(tr.mlp)
            tr.lats[(s.n, s.omega)] = lat
    trained = tr.mlp.params
    h1, h8 = tr.loss(held), tr.loss(held, horizon=8)
    tr.mlp.set_params(np.zeros(L.MLP_NPARAM))
    p1, p8 = tr.loss(held), tr.loss(held, horizon=8)
    tr.mlp.set_params(trained)
    say(f"  held-out loss, one step: paper rates {p1:.4f}, learned {h1:.4f}; eight steps: {p8:.4f}, {h8:.4f}")
    assert h1 < 1.5 * p1 and h8 < 2.0 * p8

    for label, spec, steps, factor in (
            ("64 boxes 48/64/96", inputs.ensemble_boxes(), 4800, 0.8),
            ("16 boxes 32/48", inputs.ensemble_boxes(n_boxes=16, sizes=(32, 48), seed=4242), 1200, 0.9)):
        res = LR.run_ensembles(spec, steps, 50, mlp=tr.mlp)
        e_plain = LR.decay_error(res.ke["q19"], res.ke["q27"])
        e_learn = LR.decay_error(res.ke["learned"], res.ke["q27"])
        say(f"  {label}, {steps} steps: KE decay error vs D3Q27: paper rates {e_plain:.5f}, learned {e_learn:.5f} "
            f"({e_learn / e_plain:.2f}); fallback rate {res.fallback_rate:.2e}")
        assert e_learn < factor * e_plain
        assert res.fallback_rate < 1e-3
    tr.close()
