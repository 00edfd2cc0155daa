"""What the trained network gains: D3Q19 with learned higher-order rates
follows D3Q27 more closely than the paper's D3Q19, both in the one-step
moment error on held-out data and in the kinetic-energy decay of the ensemble
workload, whose fields it was not trained on."""
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
    from paper_2010_01628_amd import learned as LR

    n = 32
    samples = []
    for nu in (1e-4, 3e-4, 1e-3):
        for sd in (1, 2):
            samples += LR.q27_samples(n, nu, 1000 + sd, (10, 40, 100, 200))
    tr = LR.Trainer(samples)
    tr.sigma = tr.per_moment_error()
    assert abs(tr.loss() - 10.0) < 1e-3  # the initial network is the paper's scheme
    tr.train(800, lr=3e-3)
    held = LR.q27_samples(n, 5e-4, 999, (20, 150))
    for s in held:
        if (s.n, s.omega) not in tr.lats:
            lat = L.Lattice(L.make_params(n, n, n, precision="fp32", omega=s.omega))
            lat.attach_mlp(tr.mlp)
            tr.lats[(s.n, s.omega)] = lat
    trained = tr.mlp.params
    h1 = tr.loss(held)
    tr.mlp.set_params(np.zeros(L.MLP_NPARAM))
    h0 = tr.loss(held)
    tr.mlp.set_params(trained)
    say(f"  held-out one-step loss: paper rates {h0:.4f}, learned {h1:.4f}")
    assert h1 < 0.8 * h0

    # the seeded 64-box workload (sides 48/64/96, nu log-uniform in [1e-4, 1e-3]),
    # none of whose fields was seen in training, over 4800 steps.  (On small
    # 32/48 boxes over 1200 steps the trained network does not reduce this
    # error: the gain is a measured property of this workload.)
    spec = inputs.ensemble_boxes()
    res = LR.run_ensembles(spec, 4800, 50, mlp=tr.mlp)
    e_plain = LR.decay_error(res.ke["q19"], res.ke["q27"])
    e_learn = LR.decay_error(res.ke["learned"], res.ke["q27"])
    say(f"  KE decay error vs D3Q27: paper rates {e_plain:.5f}, learned {e_learn:.5f}; "
        f"fallback rate {res.fallback_rate:.2e}; MLUPS {res.mlups}")
    assert e_learn < 0.9 * e_plain
    assert res.fallback_rate < 1e-3
    tr.close()
