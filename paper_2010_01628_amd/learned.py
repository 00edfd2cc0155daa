"""Learned higher-order relaxation rates: data, training and evaluation.

The network (11 -> 32 -> 32 -> 9, BF16 MFMA, FP32 accumulation) sets the nine
higher-order CM rates of the D3Q19 scheme (the rates the paper fixes to 1,
Sec. II.B); the conserved and viscous rates stay as the paper has them, so
mass and momentum remain exact, and any predicted rate outside (0, 2) sends
the node back to the paper's rates.

Training data come from the D3Q27 CM scheme (App. D) run on the GPU: a D3Q27
state at step t is projected onto the D3Q19 populations with the same 19 raw
moments, and the sample's targets are the 10 low-order raw moments (rho,
rho u, second order) of the D3Q27 states at t + 1 .. t + horizon (same
projection).  A per-node one-step collision target would carry no signal:
with the paper's rates the two lattices give the same post-collision
D3Q19-basis moments, and they differ only through the streaming of the eight
corner populations.  So the loss is taken after D3Q19 steps (collide with the
network's rates, then stream): after one step, or averaged over a rollout of
several learned steps whose gradient is back-propagated through all of them
by the hand-written backward kernels.  The default recipe opens rollouts of
1 to 128 steps over the course of training (ROLLOUT_CURRICULUM); each sample
of a minibatch draws one of the open lengths, every step's moment loss is
taken relative to the paper's scheme at that step (normalize), so that the
long steps, whose errors are larger, do not drown the short ones, and a
kinetic-energy term (ENERGY_WEIGHT) compares the lattice's total kinetic
energy after every step with the D3Q27 target's.  Moment matching alone
lowers the local moment errors and the decay error of large boxes but raises
that of small ones; the energy term lowers the decay error of both box sets,
at a small cost in the local moment errors (the measured trade-off is
recorded with the design notes).

Every lattice operation below runs in the HIP library; this module only
orders the calls and keeps the bookkeeping (which sample, which learning
rate).  Run as `python -m paper_2010_01628_amd.learned` for the comparison
of kinetic-energy decay (plain D3Q19, learned D3Q19 and D3Q27) on the seeded
64-box workload and on a held-out set of 32/48 boxes over 1200 steps.
"""
from __future__ import annotations

import argparse
import json
import time
from dataclasses import dataclass, field

import numpy as np

from . import inputs
from . import lbm as L

N_MOMENTS = 10
N_FEATURES = 11
# rollout curriculum: (fraction of the iterations, steps back-propagated)
ROLLOUT_CURRICULUM = [(0.0, 1), (0.1, 4), (0.2, 16), (0.35, 32), (0.5, 64), (0.75, 128)]
# weight of the rollout loss's kinetic-energy term, and the learning rate the
# recipe uses with it (3e-3 diverged on some seeds)
ENERGY_WEIGHT = 1e4
LEARNING_RATE = 1e-3


@dataclass
class Sample:
    """One training pair on an n^3 periodic box with shear rate omega."""

    n: int
    omega: float
    f19: object  # device float64 (19, n, n, n): projected D3Q27 state at t
    target: object  # device float32 (10, n, n, n): projected moments at t + 1
    t: int
    targets: object = None  # device float32 (horizon, 10, n, n, n): moments at t + 1 .. t + horizon


def q27_samples(n: int, nu: float, seed: int, times, u_rms: float = 0.04, horizon: int = 1):
    """D3Q27 FP64 run from the random-phase field of `seed`; one Sample per
    entry of `times` (steps after initialisation at equilibrium), with the
    projected moments of the `horizon` steps that follow."""
    import torch

    om = inputs.omega_from_nu(nu)
    rho, u = inputs.random_phase_field(n, u_rms, seed=seed)
    lat = L.Lattice(L.make_params(n, n, n, precision="fp64", q=27, omega=om))
    lat.init(rho, u)
    N = n ** 3
    st = lat.stream.cuda_stream
    out, t = [], 0
    for tt in sorted(times):
        if tt < t:
            raise ValueError("sample times closer than the horizon")
        lat.step(tt - t)
        t = tt
        f27 = lat.get_populations()
        f19 = torch.empty((19, n, n, n), dtype=torch.float64, device="cuda")
        L.lbm_project_q27(f27.data_ptr(), N, f19.data_ptr(), None, st)
        tg = torch.empty((horizon, N_MOMENTS, n, n, n), dtype=torch.float32, device="cuda")
        for k in range(horizon):
            lat.step(1)
            t += 1
            f27 = lat.get_populations()
            L.lbm_project_q27(f27.data_ptr(), N, None, tg[k].data_ptr(), st)
        lat.stream.synchronize()
        out.append(Sample(n, om, f19, tg[0], tt, tg))
    lat.close()
    return out


class Trainer:
    """Holds one FP32 D3Q19 lattice per (n, omega) and the network."""

    def __init__(self, samples, scales=None, init_seed: int = 0, hidden_std: float = 1.0):
        self.samples = list(samples)
        self.lats = {}
        for s in self.samples:
            key = (s.n, s.omega)
            if key not in self.lats:
                self.lats[key] = L.Lattice(L.make_params(s.n, s.n, s.n, precision="fp32", omega=s.omega))
        if scales is None:
            scales = self.fit_scales()
        self.scales = np.asarray(scales, dtype=np.float64)
        self.mlp = L.Mlp(initial_params(init_seed, hidden_std), self.scales)
        for lat in self.lats.values():
            lat.attach_mlp(self.mlp)
        self.sigma = np.ones(N_MOMENTS)
        self._paper = {}

    def close(self):
        for lat in self.lats.values():
            lat.close()
        self.mlp.close()

    def _load(self, s: Sample):
        lat = self.lats[(s.n, s.omega)]
        lat.set_populations(s.f19)
        return lat

    def fit_scales(self):
        """Per-feature RMS over the training samples (the frozen input scales)."""
        acc = np.zeros(N_FEATURES)
        for s in self.samples:
            acc += self._load(s).feature_rms() ** 2
        return np.maximum(np.sqrt(acc / len(self.samples)), 1e-12)

    def per_moment_error(self, samples=None):
        """RMS over nodes and samples of each of the 10 moment errors of the
        current network's one-step prediction (the loss with one sigma_k = 1
        and the rest effectively infinite)."""
        samples = self.samples if samples is None else samples
        out = np.zeros(N_MOMENTS)
        for k in range(N_MOMENTS):
            sig = np.full(N_MOMENTS, 1e30)
            sig[k] = 1.0
            tot = 0.0
            for s in samples:
                tot += self._load(s).accumulate_grad(self.mlp, s.target, sig)
            out[k] = np.sqrt(tot / len(samples))
        self.mlp.zero_grad()
        return out

    def paper_step_losses(self, s: Sample):
        """Per-step losses of the paper's scheme on sample s over its whole
        horizon (a zero network, attached to the sample's lattice for the
        call; the trained network and its optimizer state are not touched)."""
        key = (id(s), tuple(self.sigma))
        if key not in self._paper:
            lat = self._load(s)
            zero = L.Mlp(None, self.scales)
            lat.attach_mlp(zero)
            _, per = lat.accumulate_rollout_grad(zero, s.targets, self.sigma, want_steps=True)
            lat.attach_mlp(self.mlp)
            zero.close()
            self._paper[key] = np.maximum(per, 1e-300)
        return self._paper[key]

    def _sample_loss(self, s: Sample, horizon: int, sigma, normalize: bool = False) -> float:
        """Loss of one sample over `horizon` steps (capped by its targets),
        its gradient added to the network's accumulator.  normalize: each
        step's loss is divided by the paper's scheme's loss at that step, so
        every step weighs the same and the paper's scheme scores 1."""
        lat = self._load(s)
        h = 1 if s.targets is None else min(horizon, s.targets.shape[0])
        w = None
        if normalize and s.targets is not None:
            w = 1.0 / self.paper_step_losses(s)[:h]
        if h == 1 and w is None:
            return lat.accumulate_grad(self.mlp, s.target, sigma)
        return lat.accumulate_rollout_grad(self.mlp, s.targets[:h], sigma, step_weight=w)

    def loss(self, samples=None, horizon: int = 1, normalize: bool = False):
        samples = self.samples if samples is None else samples
        tot = 0.0
        for s in samples:
            tot += self._sample_loss(s, horizon, self.sigma, normalize)
        self.mlp.zero_grad()
        return tot / len(samples)

    def train(self, iters: int, lr: float = 3e-3, batch: int = 4, seed: int = 0, log_every: int = 0,
              lr_final: float | None = None, horizons=None, mix: bool = False, normalize: bool = False,
              energy_weight: float = 0.0):
        """Adam over minibatches of samples; cosine learning-rate decay to
        lr_final (default lr / 10).  horizons: the rollout curriculum, a list
        of (start fraction, steps): from iteration start * iters on, each
        sample's loss is the mean over that many learned steps, back-propagated
        through all of them (default: one step throughout).  mix: each sample
        of a minibatch draws its horizon instead, uniformly from those whose
        start has been reached.  normalize: per-step losses relative to the
        paper's scheme (_sample_loss).  energy_weight: weight of the rollouts'
        kinetic-energy term (lbm_mlp_set_energy_weight).  Returns the
        minibatch loss history."""
        self.mlp.set_energy_weight(energy_weight)
        rng = np.random.default_rng(seed)
        lr_final = lr / 10 if lr_final is None else lr_final
        sched = sorted(horizons) if horizons else [(0.0, 1)]
        hist = []
        for it in range(iters):
            open_h = [h for start, h in sched if it >= start * iters] or [1]
            horizon = open_h[-1]
            idx = rng.choice(len(self.samples), size=min(batch, len(self.samples)), replace=False)
            self.mlp.zero_grad()
            tot = 0.0
            for i in idx:
                h = int(rng.choice(open_h)) if mix else horizon
                tot += self._sample_loss(self.samples[i], h, self.sigma / np.sqrt(len(idx)), normalize)
            c = 0.5 * (1 + np.cos(np.pi * it / max(iters - 1, 1)))
            self.mlp.adam_step(lr_final + (lr - lr_final) * c)
            hist.append(tot)
            if log_every and (it % log_every == 0 or it == iters - 1):
                print(f"  iter {it:5d}  steps {horizon}  loss {tot:.6e}", flush=True)
        return hist


def initial_params(seed: int = 0, hidden_std: float = 1.0) -> np.ndarray:
    """Random hidden layers (std hidden_std / sqrt(fan_in)), zero output layer:
    the initial network gives rate 1 everywhere, i.e. the paper's scheme, and
    the output layer still receives a gradient from the first step."""
    rng = np.random.default_rng(seed)
    P = np.zeros(L.MLP_NPARAM)
    P[0:352] = rng.normal(size=352) * hidden_std / np.sqrt(N_FEATURES)
    P[384:1408] = rng.normal(size=1024) * hidden_std / np.sqrt(32)
    return P


# -- evaluation ---------------------------------------------------------------

@dataclass
class DecayResult:
    times: list
    ke: dict = field(default_factory=dict)  # variant -> (n_samples, n_boxes) array
    mlups: dict = field(default_factory=dict)
    fallback_rate: float = 0.0


def run_ensembles(boxes_spec, steps: int, every: int, mlp=None, u_rms: float = 0.04, variants=("q27", "q19", "learned")):
    """Advance the ensemble workload with each variant; sample per-box KE every
    `every` steps.  boxes_spec: [(L, nu, field_seed)]."""
    import torch

    boxes = [(n, inputs.omega_from_nu(nu)) for n, nu, _ in boxes_spec]
    fields = [inputs.random_phase_field(n, u_rms, seed=sd) for n, _, sd in boxes_spec]
    res = DecayResult(times=list(range(0, steps + 1, every)))
    for var in variants:
        if var == "learned" and mlp is None:
            continue
        q = 27 if var == "q27" else 19
        ens = L.Ensemble(boxes, q=q, precision="fp32")
        for b, (rho, u) in enumerate(fields):
            ens.init(b, rho, u)
        if var == "learned":
            ens.set_mlp(mlp)
        kes = [ens.energy()[0]]
        torch.cuda.synchronize()
        busy = 0.0
        for _ in res.times[1:]:
            t0 = time.perf_counter()
            ens.step(every)
            ke = ens.energy()[0]  # synchronizes
            busy += time.perf_counter() - t0
            kes.append(ke)
        res.ke[var] = np.array(kes)
        res.mlups[var] = ens.nodes * steps / busy / 1e6
        if var == "learned":
            res.fallback_rate = ens.fallback_count() / float(ens.nodes * steps)
        ens.close()
    return res


def decay_error(ke: np.ndarray, ke_ref: np.ndarray) -> float:
    """Relative L2 difference of the normalised decay curves KE(t)/KE(0) over
    all samples t > 0 and boxes, divided by the L2 of the reference decay
    1 - KE_ref(t)/KE_ref(0): the fraction of the reference decay that is missed."""
    r = ke[1:] / ke[0]
    rr = ke_ref[1:] / ke_ref[0]
    return float(np.linalg.norm(r - rr) / np.linalg.norm(1.0 - rr))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--train-n", type=int, default=32)
    ap.add_argument("--train-nu", type=float, nargs="+", default=[1e-4, 3e-4, 1e-3])
    ap.add_argument("--train-seeds", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--train-times", type=int, nargs="+", default=[10, 150, 300])
    ap.add_argument("--horizon", type=int, default=128, help="longest rollout (1: one-step training)")
    ap.add_argument("--iters", type=int, default=1600)
    ap.add_argument("--small-boxes", type=int, default=16, help="held-out set of 32/48 boxes, 1200 steps")
    ap.add_argument("--lr", type=float, default=LEARNING_RATE)
    ap.add_argument("--energy-weight", type=float, default=ENERGY_WEIGHT)
    ap.add_argument("--boxes", type=int, default=64)
    ap.add_argument("--steps", type=int, default=4800)
    ap.add_argument("--every", type=int, default=50)
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)

    t0 = time.perf_counter()
    samples = []
    for nu in a.train_nu:
        for sd in a.train_seeds:
            samples += q27_samples(a.train_n, nu, 1000 + sd, a.train_times, horizon=a.horizon)
    tr = Trainer(samples)
    err0 = tr.per_moment_error()
    tr.sigma = np.maximum(err0, 1e-30)  # the paper's scheme scores 1 per moment
    loss0 = tr.loss()
    curriculum = [(f, h) for f, h in ROLLOUT_CURRICULUM if h <= a.horizon]
    tr.train(a.iters, lr=a.lr, log_every=max(a.iters // 10, 1), horizons=curriculum, mix=True, normalize=True,
             energy_weight=a.energy_weight)
    loss1 = tr.loss()
    ratio = tr.per_moment_error() / tr.sigma
    held = q27_samples(a.train_n, a.train_nu[len(a.train_nu) // 2], 999, a.train_times)
    ht = [(s.n, s.omega) for s in held]
    for key in ht:
        if key not in tr.lats:
            tr.lats[key] = L.Lattice(L.make_params(key[0], key[0], key[0], precision="fp32", omega=key[1]))
            tr.lats[key].attach_mlp(tr.mlp)
    held_loss = tr.loss(held)
    trained = tr.mlp.params
    tr.mlp.set_params(np.zeros(L.MLP_NPARAM))  # the paper's rates
    held_loss0 = tr.loss(held)
    tr.mlp.set_params(trained)
    train_s = time.perf_counter() - t0
    print(f"training: {len(samples)} samples, loss {loss0:.4f} -> {loss1:.4f}; held-out {held_loss0:.4f} -> "
          f"{held_loss:.4f} ({train_s:.1f} s)", flush=True)
    small = inputs.ensemble_boxes(n_boxes=a.small_boxes, sizes=(32, 48), seed=4242)
    res_small = run_ensembles(small, 1200, 50, mlp=tr.mlp)
    spec = inputs.ensemble_boxes(n_boxes=a.boxes)
    res = run_ensembles(spec, a.steps, a.every, mlp=tr.mlp)
    report = {
        "train": {"samples": len(samples), "n": a.train_n, "nu": a.train_nu, "iters": a.iters,
                  "loss_plain": loss0, "loss_learned": loss1, "heldout_plain": held_loss0,
                  "heldout_learned": held_loss, "moment_error_ratio": [round(float(v), 4) for v in ratio],
                  "seconds": train_s},
        "ensemble": {"boxes": a.boxes, "steps": a.steps, "every": a.every,
                     "mlups": res.mlups, "fallback_rate": res.fallback_rate,
                     "decay_error_plain": decay_error(res.ke["q19"], res.ke["q27"]),
                     "decay_error_learned": decay_error(res.ke["learned"], res.ke["q27"]) if "learned" in res.ke else None},
        "small_boxes": {"boxes": a.small_boxes, "steps": 1200,
                        "decay_error_plain": decay_error(res_small.ke["q19"], res_small.ke["q27"]),
                        "decay_error_learned": decay_error(res_small.ke["learned"], res_small.ke["q27"])},
    }
    print(json.dumps(report), flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            json.dump(report, fh, indent=1)
    tr.close()


if __name__ == "__main__":
    main()
