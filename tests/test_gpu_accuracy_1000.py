"""Accuracy of every storage precision and streaming pattern over a long run:
the timed workload's recipe (Taylor-Green U0 = 0.05 + seeded noise 1e-4,
nu = 1e-3, Kolmogorov force 1e-6) at 64^3 and 128^3 for 1000 steps against
the FP64 oracle run once per size on the host; relative L2 of u and of
rho - mean(rho).  (The 256^3 lattice is checked at full size step by step in
test_gpu_fullsize.py.)

The bounds come from the workload's own conditioning under storage rounding,
measured with the oracle alone (tests/golden/conditioning.py ->
conditioning_config2.json): the FP64 scheme with its stored deviations
rounded to FP32, FP16 or BF16 after every step.  That is the error the
storage format costs by itself; the GPU adds its FP32 collision arithmetic.

  FP32: the stated tolerance 1e-5 on u and on rho - mean(rho).  The increment
        form of the collision (f* = f + change, the change built from
        non-equilibrium moments) leaves one equilibrium-sized rounding per
        population and step, next to the storage rounding: within
        FP32_FACTOR of the storage-only error.  (The form that rebuilt f* from
        equilibrium-sized moments measured 1.9e-5 / 3.0e-5 at 64^3, 280 and 50
        times the storage-only error.)
  FP16, BF16: the error is the storage's (FP32 arithmetic rounds 2^8 and 2^16
        times finer): within X16_FACTOR of the storage-only error, the margin
        covering rounding decisions that differ between the GPU's FP32 values
        and the oracle's FP64 ones.  FP16 also meets 1e-3 on u; BF16 cannot
        (its storage alone costs 2.8e-2 on u at 64^3 -- reading recorded with
        the measurements).  BF16 with stochastic rounding against the
        storage-only run with stochastic rounding (other random bits, the same
        statistics).
"""
import json
import os

import pytest

from gpu_helpers import gpu_run, rel_l2, rel_l2_fluct, say
from paper_2010_01628_amd import inputs
from paper_2010_01628_amd import lbm as L

pytestmark = pytest.mark.gpu

STEPS, NU = 1000, 1e-3
STATED = {"fp32": 1e-5, "fp16": 1e-3}  # relative L2 on u (and on rho - mean(rho) for FP32)
FP32_FACTOR = {"u": 4.0, "rho_fluct": 8.0}
X16_FACTOR = 1.5
COND = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "conditioning_config2.json")))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.lib()


# storage variants: (lbm precision, rounding, conditioning entry)
VARIANTS = {"fp32": ("fp32", "nearest", "fp32"), "fp16": ("fp16", "nearest", "fp16"),
            "bf16": ("bf16", "nearest", "bf16"), "bf16sr": ("bf16", "stochastic", "bf16_sr")}
# the sizes (64 and 128; the 32^3 entry serves the 200-step parity case)
# whose storage-only errors have been measured for every variant.  128^3 is opt-in (LBM_ACCURACY_128=1): its FP64 oracle run of
# 1000 steps takes ~10 minutes on 16 host threads.
SIZES = sorted(int(k) for k, v in COND.items() if int(k) >= 64 and all(e in v for _, _, e in VARIANTS.values()))
if not os.environ.get("LBM_ACCURACY_128"):
    SIZES = [n for n in SIZES if n < 128]


@pytest.fixture(scope="module", params=SIZES)
def reference(orc, request):
    N = request.param
    say(f"oracle: {N}^3, {STEPS} steps (FP64, host)")
    rho, u = inputs.taylor_green_noise(N, 0.05, 1e-4, seed=20101628)
    F = inputs.kolmogorov_force(N, N, N, 1e-6)
    f = orc.run(orc.init(rho, u), STEPS, orc.K(inputs.omega_from_nu(NU)), F=F,
                progress=lambda t: say(f"  oracle {N}^3: step {t}"))
    r, v = orc.moments(f, F)
    return N, rho, u, r, v


@pytest.mark.parametrize("precision", list(VARIANTS))
@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_long_run_error(reference, precision, streaming):
    N, rho, u, ro, uo = reference
    storage, rounding, entry = VARIANTS[precision]
    cond = COND[str(N)][entry][str(STEPS)]
    say(f"{precision} {streaming}: {N}^3, {STEPS} steps; storage alone: u {cond['u']:.3e}, "
        f"rho - mean(rho) {cond['rho_fluct']:.3e}")
    g = gpu_run(N, N, N, rho, u, STEPS, storage, streaming, omega=inputs.omega_from_nu(NU),
                force_mode=L.LBM_FORCE_KOLMOGOROV, kolmogorov_amp=1e-6, want_pops=False, rounding=rounding)
    err = {"u": rel_l2(g["u"], uo), "rho_fluct": rel_l2_fluct(g["rho"], ro)}
    say(f"  rel L2 u = {err['u']:.3e} ({err['u'] / cond['u']:.2f} x storage alone), rho - mean(rho) = "
        f"{err['rho_fluct']:.3e} ({err['rho_fluct'] / cond['rho_fluct']:.2f} x)")
    for k in ("u", "rho_fluct"):
        factor = FP32_FACTOR[k] if precision == "fp32" else X16_FACTOR
        assert err[k] <= factor * cond[k]
    if precision == "fp32":
        assert err["u"] <= STATED["fp32"] and err["rho_fluct"] <= STATED["fp32"]
    if precision == "fp16":
        assert err["u"] <= STATED["fp16"]
