"""ctypes binding of liblbm.so (the C ABI in include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the ABI.  Loading fails loudly if the library has not been built; there
is no CPU fallback.

The ``lbm_*`` functions mirror the C entry points one to one.  ``Lattice``
wraps a handle for convenience: device memory for inputs and outputs is torch
tensors on the handle's GPU; the handle's stream is torch's current stream at
creation unless another is given.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# LBM_LIBRARY names another build of the same library (the host-sanitized one)
LIB_PATH = os.environ.get("LBM_LIBRARY") or os.path.join(_PKG, "liblbm.so")

ABI_VERSION = 7
LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EDEVICE, LBM_EUNSTABLE, LBM_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
LBM_FP64, LBM_FP32, LBM_FP16_SHIFTED, LBM_BF16_SHIFTED = 0, 1, 2, 3
LBM_AB, LBM_AA = 0, 1
LBM_FORCE_NONE, LBM_FORCE_UNIFORM, LBM_FORCE_FIELD, LBM_FORCE_KOLMOGOROV = 0, 1, 2, 3
LBM_CENTRAL_MOMENTS, LBM_RAW_MOMENTS = 0, 1
LBM_ROUND_NEAREST, LBM_ROUND_STOCHASTIC = 0, 1

PRECISIONS = {"fp64": LBM_FP64, "fp32": LBM_FP32, "fp16": LBM_FP16_SHIFTED, "bf16": LBM_BF16_SHIFTED}
STREAMING = {"ab": LBM_AB, "aa": LBM_AA}
MOMENTS = {"central": LBM_CENTRAL_MOMENTS, "raw": LBM_RAW_MOMENTS}


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class lbm_phase_params(ctypes.Structure):
    _fields_ = [("rho_light", ctypes.c_double), ("rho_heavy", ctypes.c_double), ("sigma", ctypes.c_double),
                ("width", ctypes.c_double), ("mobility", ctypes.c_double)]


class lbm_magnetic_params(ctypes.Structure):
    _fields_ = [("eta", ctypes.c_double), ("b_wall", ctypes.c_double * 3)]


class lbm_shan_chen_params(ctypes.Structure):
    _fields_ = [("G", ctypes.c_double)]


class lbm_colour_params(ctypes.Structure):
    _fields_ = [("alpha_red", ctypes.c_double), ("alpha_blue", ctypes.c_double), ("A", ctypes.c_double),
                ("beta", ctypes.c_double), ("gravity", ctypes.c_double * 3), ("rho_ref", ctypes.c_double)]


LBM_COUPLED_NONE, LBM_COUPLED_PHASE, LBM_COUPLED_MAGNETIC, LBM_COUPLED_SHAN_CHEN, LBM_COUPLED_COLOUR = 0, 1, 2, 3, 4


class lbm_params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("streaming", ctypes.c_int32),
        ("omega", ctypes.c_double),
        ("omega_bulk", ctypes.c_double),
        ("omega_hi", ctypes.c_double * 9),
        ("rho0", ctypes.c_double),
        ("force_mode", ctypes.c_int32),
        ("force", ctypes.c_double * 3),
        ("kolmogorov_amp", ctypes.c_double),
        ("force_field", ctypes.c_void_p),
        ("walls_y", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
        ("cache_policy", ctypes.c_int32),
        ("coupled", ctypes.c_int32),
        ("phase", lbm_phase_params),
        ("magnetic", lbm_magnetic_params),
        ("moments", ctypes.c_int32),
        ("shan_chen", lbm_shan_chen_params),
        ("colour", lbm_colour_params),
        ("rounding", ctypes.c_int32),
        ("seed", ctypes.c_uint32),
    ]


_lib = None


def lib():
    """Load liblbm.so (raises if it is missing: no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2010_01628_amd.build`")
        # torch first: its HIP runtime is then the one the library binds to
        # (one runtime per process, whose devices, streams and pointers both use)
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        P = ctypes.POINTER(lbm_params)
        L.lbm_params_default.argtypes = [P]
        L.lbm_params_default.restype = None
        L.lbm_create.argtypes = [P, vp, ctypes.POINTER(vp)]
        L.lbm_init.argtypes = [vp, vp, vp, i32]
        L.lbm_step.argtypes = [vp, i64]
        L.lbm_moments.argtypes = [vp, vp, vp, vp, i32]
        L.lbm_moments_noalloc.argtypes = [vp, vp, vp, vp]
        L.lbm_get_populations.argtypes = [vp, vp, i32]
        L.lbm_set_populations.argtypes = [vp, vp, i32]
        L.lbm_step_count.argtypes = [vp]
        L.lbm_step_count.restype = i64
        L.lbm_step_variant.argtypes = [vp]
        L.lbm_step_variant.restype = i32
        L.lbm_device_bytes.argtypes = [vp]
        L.lbm_device_bytes.restype = i64
        L.lbm_destroy.argtypes = [vp]
        L.lbm_last_error.restype = ctypes.c_char_p
        L.lbm_abi_version.restype = i32
        fp, dp = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
        L.lbm_mlp_create.argtypes = [fp, fp, vp, ctypes.POINTER(vp)]
        L.lbm_mlp_set_params.argtypes = [vp, fp]
        L.lbm_mlp_get_params.argtypes = [vp, fp]
        L.lbm_mlp_set_scales.argtypes = [vp, fp]
        L.lbm_mlp_destroy.argtypes = [vp]
        L.lbm_set_mlp.argtypes = [vp, vp]
        L.lbm_fallback_count.argtypes = [vp]
        L.lbm_fallback_count.restype = i64
        L.lbm_mlp_zero_grad.argtypes = [vp]
        L.lbm_mlp_accumulate_grad.argtypes = [vp, vp, vp, dp, dp]
        L.lbm_mlp_accumulate_rollout_grad.argtypes = [vp, vp, vp, i32, dp, dp, vp, dp, dp]
        L.lbm_mlp_set_energy_weight.argtypes = [vp, ctypes.c_double]
        L.lbm_mlp_get_grad.argtypes = [vp, dp]
        L.lbm_mlp_adam_step.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.lbm_feature_rms.argtypes = [vp, dp]
        L.lbm_project_q27.argtypes = [vp, i64, vp, vp, vp]
        L.lbm_stream_copy.argtypes = [vp, vp, i64, i32, i32, i32, i32, vp]
        class _box(ctypes.Structure):
            _fields_ = [("n", ctypes.c_int32), ("omega", ctypes.c_double)]

        globals()["lbm_box"] = _box
        BP = ctypes.POINTER(_box)
        L.lbm_ensemble_create.argtypes = [BP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, ctypes.POINTER(vp)]
        L.lbm_ensemble_init.argtypes = [vp, ctypes.c_int32, vp, vp, i32]
        L.lbm_ensemble_set_mlp.argtypes = [vp, vp]
        L.lbm_ensemble_step.argtypes = [vp, i64]
        L.lbm_ensemble_energy.argtypes = [vp, dp, dp]
        L.lbm_ensemble_get_populations.argtypes = [vp, ctypes.c_int32, vp, i32]
        L.lbm_ensemble_nodes.argtypes = [vp]
        L.lbm_ensemble_nodes.restype = i64
        L.lbm_ensemble_step_count.argtypes = [vp]
        L.lbm_ensemble_step_count.restype = i64
        L.lbm_ensemble_fallback_count.argtypes = [vp]
        L.lbm_ensemble_fallback_count.restype = i64
        L.lbm_ensemble_tune.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.lbm_ensemble_destroy.argtypes = [vp]
        for name in ("lbm_ensemble_create", "lbm_ensemble_init", "lbm_ensemble_set_mlp", "lbm_ensemble_step",
                     "lbm_ensemble_energy", "lbm_ensemble_get_populations", "lbm_ensemble_tune",
                     "lbm_ensemble_destroy"):
            getattr(L, name).restype = i32
        ip32 = ctypes.POINTER(ctypes.c_int32)
        L.lbm_tune.argtypes = [vp, ctypes.c_int32, ip32, ip32, ip32, ip32]
        L.lbm_tune.restype = i32
        L.lbm_init_magnetic.argtypes = [vp, vp, vp, vp, i32]
        L.lbm_magnetic_fields.argtypes = [vp, vp, vp, i32]
        L.lbm_init_magnetic.restype = i32
        L.lbm_magnetic_fields.restype = i32
        L.lbm_init_phase.argtypes = [vp, vp, vp, vp, i32]
        L.lbm_phase_fields.argtypes = [vp, vp, vp, i32]
        L.lbm_init_colour.argtypes = [vp, vp, vp, vp, i32]
        L.lbm_colour_fields.argtypes = [vp, vp, vp, i32]
        L.lbm_get_coupled_populations.argtypes = [vp, vp, i32]
        L.lbm_set_coupled_populations.argtypes = [vp, vp, i32]
        for name in ("lbm_init_phase", "lbm_phase_fields", "lbm_get_coupled_populations",
                     "lbm_set_coupled_populations", "lbm_init_colour", "lbm_colour_fields"):
            getattr(L, name).restype = i32
        for name in ("lbm_create", "lbm_init", "lbm_step", "lbm_moments", "lbm_moments_noalloc", "lbm_get_populations",
                     "lbm_set_populations", "lbm_destroy", "lbm_mlp_create", "lbm_mlp_set_params",
                     "lbm_mlp_get_params", "lbm_mlp_set_scales", "lbm_mlp_destroy", "lbm_set_mlp",
                     "lbm_mlp_zero_grad", "lbm_mlp_accumulate_grad", "lbm_mlp_accumulate_rollout_grad",
                     "lbm_mlp_set_energy_weight",
                     "lbm_mlp_get_grad", "lbm_mlp_adam_step",
                     "lbm_feature_rms", "lbm_project_q27", "lbm_stream_copy"):
            getattr(L, name).restype = i32
        if L.lbm_abi_version() != ABI_VERSION:
            raise ImportError("liblbm.so ABI version mismatch")
        _lib = L
    return _lib


def _check(rc: int):
    if rc != LBM_OK:
        raise LbmError(rc, lib().lbm_last_error().decode())
    return rc


# -- one-to-one entry points -------------------------------------------------
def lbm_params_default() -> lbm_params:
    p = lbm_params()
    lib().lbm_params_default(ctypes.byref(p))
    return p


def lbm_create(p: lbm_params, stream: int | None = None) -> int:
    h = ctypes.c_void_p()
    _check(lib().lbm_create(ctypes.byref(p), ctypes.c_void_p(stream or 0), ctypes.byref(h)))
    return h.value


def lbm_init(h: int, rho_ptr: int, u_ptr: int, on_device: bool) -> None:
    _check(lib().lbm_init(h, rho_ptr, u_ptr, int(on_device)))


def lbm_step(h: int, nsteps: int) -> None:
    _check(lib().lbm_step(h, int(nsteps)))


def lbm_moments(h: int, rho_ptr, u_ptr, diag_ptr, on_device: bool) -> None:
    _check(lib().lbm_moments(h, rho_ptr, u_ptr, diag_ptr, int(on_device)))


def lbm_moments_noalloc(h: int, rho_ptr, u_ptr, diag_ptr) -> None:
    """Device pointers only (each may be None); allocates nothing."""
    _check(lib().lbm_moments_noalloc(h, rho_ptr, u_ptr, diag_ptr))


def lbm_get_populations(h: int, f_ptr: int, on_device: bool) -> None:
    _check(lib().lbm_get_populations(h, f_ptr, int(on_device)))


def lbm_set_populations(h: int, f_ptr: int, on_device: bool) -> None:
    _check(lib().lbm_set_populations(h, f_ptr, int(on_device)))


def lbm_step_count(h: int) -> int:
    return lib().lbm_step_count(h)


def lbm_step_variant(h: int) -> int:
    return lib().lbm_step_variant(h)


def lbm_device_bytes(h: int) -> int:
    return lib().lbm_device_bytes(h)


def lbm_destroy(h: int) -> None:
    _check(lib().lbm_destroy(h))


MLP_NPARAM = 1737
MLP_MAX_ROLLOUT = 128


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lbm_mlp_create(params, scales, stream=None) -> int:
    m = ctypes.c_void_p()
    pp = None if params is None else _fptr(np.ascontiguousarray(params, dtype=np.float32))
    sc = np.ascontiguousarray(scales, dtype=np.float32)
    _check(lib().lbm_mlp_create(pp, _fptr(sc), ctypes.c_void_p(stream or 0), ctypes.byref(m)))
    return m.value


def lbm_mlp_set_params(m, params):
    _check(lib().lbm_mlp_set_params(m, _fptr(np.ascontiguousarray(params, dtype=np.float32))))


def lbm_mlp_get_params(m):
    out = np.zeros(MLP_NPARAM, dtype=np.float32)
    _check(lib().lbm_mlp_get_params(m, _fptr(out)))
    return out


def lbm_mlp_set_scales(m, scales):
    _check(lib().lbm_mlp_set_scales(m, _fptr(np.ascontiguousarray(scales, dtype=np.float32))))


def lbm_mlp_destroy(m):
    _check(lib().lbm_mlp_destroy(m))


def lbm_set_mlp(h, m):
    _check(lib().lbm_set_mlp(h, m))


def lbm_fallback_count(h) -> int:
    v = lib().lbm_fallback_count(h)
    if v < 0:
        _check(int(v))
    return int(v)


def lbm_mlp_zero_grad(m):
    _check(lib().lbm_mlp_zero_grad(m))


def lbm_mlp_accumulate_grad(m, h, target_ptr, sigma) -> float:
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    loss = np.zeros(1)
    _check(lib().lbm_mlp_accumulate_grad(m, h, target_ptr, _dptr(sig), _dptr(loss)))
    return float(loss[0])


def lbm_mlp_accumulate_rollout_grad(m, h, targets_ptr, steps, sigma, step_weight=None, dstate_ptr=None):
    """Returns (loss, per-step losses)."""
    sig = np.ascontiguousarray(sigma, dtype=np.float64)
    w = None if step_weight is None else np.ascontiguousarray(step_weight, dtype=np.float64)
    if w is not None and w.size != int(steps):
        raise ValueError("one weight per step")
    loss = np.zeros(1)
    per = np.zeros(int(steps))
    _check(lib().lbm_mlp_accumulate_rollout_grad(m, h, targets_ptr, int(steps), _dptr(sig),
                                                 None if w is None else _dptr(w), dstate_ptr, _dptr(per),
                                                 _dptr(loss)))
    return float(loss[0]), per


def lbm_mlp_set_energy_weight(m, w):
    _check(lib().lbm_mlp_set_energy_weight(m, float(w)))


def lbm_mlp_get_grad(m):
    out = np.zeros(MLP_NPARAM)
    _check(lib().lbm_mlp_get_grad(m, _dptr(out)))
    return out


def lbm_mlp_adam_step(m, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _check(lib().lbm_mlp_adam_step(m, float(lr), float(beta1), float(beta2), float(eps)))


def lbm_feature_rms(h):
    out = np.zeros(11)
    _check(lib().lbm_feature_rms(h, _dptr(out)))
    return out


def lbm_stream_copy(src_ptr, dst_ptr, n, q, elem_bytes, nt=True, stream=None, lane_bytes=0):
    """Copy q arrays of n elements (device pointers) with the step's access
    pattern: a bandwidth reference for the step kernels.  lane_bytes: bytes
    per thread and array (0: one element, as the step; 8 or 16: wider)."""
    _check(lib().lbm_stream_copy(src_ptr, dst_ptr, int(n), int(q), int(elem_bytes), int(lane_bytes), 1 if nt else 0,
                                 ctypes.c_void_p(stream or 0)))


def lbm_project_q27(f27_ptr, n, f19_ptr, moments_ptr, stream=None):
    _check(lib().lbm_project_q27(f27_ptr, int(n), f19_ptr, moments_ptr, ctypes.c_void_p(stream or 0)))


class Mlp:
    """Owns one lbm_mlp (learned higher-order rates)."""

    def __init__(self, params=None, scales=None, stream=None):
        import torch

        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.m = lbm_mlp_create(params, np.ones(11) if scales is None else scales, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "m", None):
            lbm_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    params = property(lambda self: lbm_mlp_get_params(self.m))

    def set_params(self, p):
        lbm_mlp_set_params(self.m, p)

    def set_scales(self, s):
        lbm_mlp_set_scales(self.m, s)

    def zero_grad(self):
        lbm_mlp_zero_grad(self.m)

    def grad(self):
        return lbm_mlp_get_grad(self.m)

    def set_energy_weight(self, w):
        """Weight of the kinetic-energy term of later rollout losses (0: none)."""
        lbm_mlp_set_energy_weight(self.m, w)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        lbm_mlp_adam_step(self.m, lr, beta1, beta2, eps)


def lbm_ensemble_create(boxes, q=19, precision="fp32", stream=None) -> int:
    lib()
    arr = (lbm_box * len(boxes))(*[lbm_box(int(n), float(om)) for n, om in boxes])
    e = ctypes.c_void_p()
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().lbm_ensemble_create(arr, len(boxes), int(q), prec, ctypes.c_void_p(stream or 0), ctypes.byref(e)))
    return e.value


class Ensemble:
    """Owns one lbm_ensemble: boxes = [(side, omega), ...]."""

    def __init__(self, boxes, q=19, precision="fp32"):
        import torch

        self.torch = torch
        self.boxes = list(boxes)
        self.q = q
        self.e = lbm_ensemble_create(self.boxes, q, precision, None)

    def close(self):
        if getattr(self, "e", None):
            _check(lib().lbm_ensemble_destroy(self.e))
            self.e = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, box, rho, u):
        t = self.torch
        n = self.boxes[box][0]
        r = t.from_numpy(np.ascontiguousarray(rho, dtype=np.float64)).cuda()
        v = t.from_numpy(np.ascontiguousarray(u, dtype=np.float64)).cuda()
        assert r.numel() == n ** 3 and v.numel() == 3 * n ** 3
        t.cuda.synchronize()  # the ensemble works on its own stream
        _check(lib().lbm_ensemble_init(self.e, int(box), r.data_ptr(), v.data_ptr(), 1))
        t.cuda.synchronize()  # every stream: r and v stay alive until the init kernel is done

    def set_mlp(self, mlp):
        _check(lib().lbm_ensemble_set_mlp(self.e, None if mlp is None else mlp.m))
        self._mlp = mlp

    def step(self, n):
        _check(lib().lbm_ensemble_step(self.e, int(n)))

    def energy(self):
        ke = np.zeros(len(self.boxes))
        mass = np.zeros(len(self.boxes))
        _check(lib().lbm_ensemble_energy(self.e, _dptr(ke), _dptr(mass)))
        return ke, mass

    def get_populations(self, box):
        n = self.boxes[box][0]
        f = np.zeros((self.q, n, n, n))
        _check(lib().lbm_ensemble_get_populations(self.e, int(box), f.ctypes.data, 0))
        return f

    def tune(self, trial_steps=10):
        g = ctypes.c_int32(0)
        _check(lib().lbm_ensemble_tune(self.e, int(trial_steps), ctypes.byref(g)))
        return g.value

    @property
    def nodes(self):
        return lib().lbm_ensemble_nodes(self.e)

    @property
    def step_count(self):
        return lib().lbm_ensemble_step_count(self.e)

    def fallback_count(self):
        v = lib().lbm_ensemble_fallback_count(self.e)
        if v < 0:
            _check(int(v))
        return int(v)


# -- convenience wrapper -----------------------------------------------------
def make_params(nx, ny, nz, precision="fp32", streaming="ab", omega=1.0, omega_bulk=1.0, omega_hi=None,
                rho0=1.0, force_mode=LBM_FORCE_NONE, force=(0.0, 0.0, 0.0), kolmogorov_amp=0.0,
                force_field_ptr=None, walls_y=False, check_every=0, block=(0, 0), cache_policy=0,
                q=19, phase=None, magnetic=None, moments="central", shan_chen=None, colour=None,
                rounding="nearest", seed=0) -> lbm_params:
    """phase: dict(rho_light, rho_heavy, sigma, width, mobility) makes a
    two-phase lattice (coupled = LBM_COUPLED_PHASE); magnetic: dict(eta,
    b_wall=(bx, by, bz)) a magnetic one (LBM_COUPLED_MAGNETIC); moments:
    "central" (the paper's scheme) or "raw" (its N = I variant); shan_chen:
    dict(G) a Shan-Chen two-phase lattice (LBM_COUPLED_SHAN_CHEN); colour:
    dict(alpha_red, alpha_blue=1/3, A=0, beta=0.7, gravity=(0,0,0), rho_ref=0)
    a colour-gradient lattice (LBM_COUPLED_COLOUR); rounding: "nearest" or
    "stochastic" (BF16 storage), with its random-bit key `seed`."""
    p = lbm_params_default()
    p.q = int(q)
    p.nx, p.ny, p.nz = int(nx), int(ny), int(nz)
    p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    p.streaming = STREAMING[streaming] if isinstance(streaming, str) else int(streaming)
    p.omega = float(omega)
    p.omega_bulk = float(omega_bulk)
    hi = [1.0] * 9 if omega_hi is None else [float(v) for v in omega_hi]
    for j in range(9):
        p.omega_hi[j] = hi[j]
    p.rho0 = float(rho0)
    p.force_mode = int(force_mode)
    for d in range(3):
        p.force[d] = float(force[d])
    p.kolmogorov_amp = float(kolmogorov_amp)
    p.force_field = force_field_ptr
    p.walls_y = int(bool(walls_y))
    p.check_every = int(check_every)
    p.block_x, p.block_y = int(block[0]), int(block[1])
    p.cache_policy = int(cache_policy)
    p.moments = MOMENTS[moments] if isinstance(moments, str) else int(moments)
    p.rounding = {"nearest": LBM_ROUND_NEAREST, "stochastic": LBM_ROUND_STOCHASTIC}[rounding] \
        if isinstance(rounding, str) else int(rounding)
    p.seed = int(seed) & 0xFFFFFFFF
    if magnetic is not None:
        p.coupled = LBM_COUPLED_MAGNETIC
        p.magnetic.eta = float(magnetic["eta"])
        bw = magnetic.get("b_wall", (0.0, 0.0, 0.0))
        for d in range(3):
            p.magnetic.b_wall[d] = float(bw[d])
    if colour is not None:
        p.coupled = LBM_COUPLED_COLOUR
        p.colour.alpha_red = float(colour["alpha_red"])
        p.colour.alpha_blue = float(colour.get("alpha_blue", 1.0 / 3.0))
        p.colour.A = float(colour.get("A", 0.0))
        p.colour.beta = float(colour.get("beta", 0.7))
        gv = colour.get("gravity", (0.0, 0.0, 0.0))
        for d in range(3):
            p.colour.gravity[d] = float(gv[d])
        p.colour.rho_ref = float(colour.get("rho_ref", 0.0))
    if shan_chen is not None:
        p.coupled = LBM_COUPLED_SHAN_CHEN
        p.shan_chen.G = float(shan_chen["G"])
    if phase is not None:
        p.coupled = LBM_COUPLED_PHASE
        for k in ("rho_light", "rho_heavy", "sigma", "width", "mobility"):
            setattr(p.phase, k, float(phase[k]))
    return p


class Lattice:
    """Owns one lbm handle.  Fields are (nz, ny, nx) / (3, nz, ny, nx) float64."""

    def __init__(self, params: lbm_params, stream=None, force_field=None):
        import torch

        self.torch = torch
        self.params = params
        self.shape = (params.nz, params.ny, params.nx)
        self.N = params.nx * params.ny * params.nz
        self.q = params.q
        self._force_field = force_field  # keep the tensor alive
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.h = lbm_create(params, stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device="cuda", dtype=t.float64).contiguous()
        return t.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")

    def init(self, rho, u):
        r = self._dev(rho)
        v = self._dev(u)
        assert r.numel() == self.N and v.numel() == 3 * self.N
        lbm_init(self.h, r.data_ptr(), v.data_ptr(), True)
        self.stream.synchronize()

    def step(self, n: int):
        lbm_step(self.h, n)

    def moments(self, want_fields=True):
        t = self.torch
        diag = np.zeros(6)
        if want_fields:
            rho = t.empty(self.shape, dtype=t.float64, device="cuda")
            u = t.empty((3,) + self.shape, dtype=t.float64, device="cuda")
            lbm_moments(self.h, rho.data_ptr(), u.data_ptr(), diag.ctypes.data, True)
            return rho, u, diag
        lbm_moments(self.h, None, None, diag.ctypes.data, True)
        return None, None, diag

    def get_populations(self):
        t = self.torch
        f = t.empty((self.q,) + self.shape, dtype=t.float64, device="cuda")
        lbm_get_populations(self.h, f.data_ptr(), True)
        self.stream.synchronize()
        return f

    def set_populations(self, f):
        ff = self._dev(f)
        if ff.numel() != self.q * self.N:
            raise ValueError(f"expected {self.q} x {self.N} values, got {ff.numel()}")
        assert ff.numel() == self.q * self.N
        lbm_set_populations(self.h, ff.data_ptr(), True)
        self.stream.synchronize()

    def attach_mlp(self, mlp):
        lbm_set_mlp(self.h, None if mlp is None else mlp.m)
        self._mlp = mlp

    def fallback_count(self):
        return lbm_fallback_count(self.h)

    def feature_rms(self):
        return lbm_feature_rms(self.h)

    def accumulate_grad(self, mlp, target, sigma):
        """target: device float32 tensor (10, nz, ny, nx)."""
        t = target.contiguous()
        assert t.dtype == self.torch.float32 and t.numel() == 10 * self.N
        return lbm_mlp_accumulate_grad(mlp.m, self.h, t.data_ptr(), sigma)

    def accumulate_rollout_grad(self, mlp, targets, sigma, step_weight=None, want_dstate=False, want_steps=False):
        """targets: device float32 tensor (steps, 10, nz, ny, nx), the moments
        after each step; step_weight: one positive weight per step or None.
        Returns the loss; with want_steps also the per-step losses, with
        want_dstate also dL/df (device float32 (19, nz, ny, nx)) of the
        current populations."""
        t = targets.contiguous()
        assert t.dtype == self.torch.float32 and t.numel() % (10 * self.N) == 0
        steps = t.numel() // (10 * self.N)
        ds = self.torch.empty((19,) + self.shape, dtype=self.torch.float32, device=t.device) if want_dstate else None
        loss, per = lbm_mlp_accumulate_rollout_grad(mlp.m, self.h, t.data_ptr(), steps, sigma, step_weight,
                                                    ds.data_ptr() if ds is not None else None)
        out = (loss,)
        if want_steps:
            out += (per,)
        if want_dstate:
            out += (ds,)
        return out if len(out) > 1 else loss

    @property
    def step_count(self):
        return lbm_step_count(self.h)

    @property
    def step_variant(self):
        """0: one node per thread, 1: x-moving populations staged through LDS."""
        return lbm_step_variant(self.h)

    def tune(self, trial_steps=10):
        """Pick the step kernel's work-group shape, cache policy and row
        staging by timing real steps (the state advances); returns
        (block_x, block_y, policy, row_stage)."""
        bx, by, nt, rs = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().lbm_tune(self.h, int(trial_steps), ctypes.byref(bx), ctypes.byref(by), ctypes.byref(nt),
                              ctypes.byref(rs)))
        return bx.value, by.value, nt.value, rs.value

    # -- two-phase lattices ------------------------------------------------
    def init_phase(self, phi, p, u):
        a, b, c = self._dev(phi), self._dev(p), self._dev(u)
        assert a.numel() == self.N and b.numel() == self.N and c.numel() == 3 * self.N
        _check(lib().lbm_init_phase(self.h, a.data_ptr(), b.data_ptr(), c.data_ptr(), 1))
        self.stream.synchronize()

    def phase_fields(self):
        """(phi, p) as device float64 tensors (nz, ny, nx)."""
        t = self.torch
        phi = t.empty(self.shape, dtype=t.float64, device="cuda")
        p = t.empty(self.shape, dtype=t.float64, device="cuda")
        _check(lib().lbm_phase_fields(self.h, phi.data_ptr(), p.data_ptr(), 1))
        self.stream.synchronize()
        return phi, p

    # -- colour-gradient lattices -------------------------------------------
    def init_colour(self, rho_red, rho_blue, u):
        a, b, c = self._dev(rho_red), self._dev(rho_blue), self._dev(u)
        assert a.numel() == self.N and b.numel() == self.N and c.numel() == 3 * self.N
        _check(lib().lbm_init_colour(self.h, a.data_ptr(), b.data_ptr(), c.data_ptr(), 1))
        self.stream.synchronize()

    def colour_fields(self):
        """(rho_red, rho_blue) as device float64 tensors (nz, ny, nx)."""
        t = self.torch
        a = t.empty(self.shape, dtype=t.float64, device="cuda")
        b = t.empty(self.shape, dtype=t.float64, device="cuda")
        _check(lib().lbm_colour_fields(self.h, a.data_ptr(), b.data_ptr(), 1))
        self.stream.synchronize()
        return a, b

    # -- magnetic lattices ---------------------------------------------------
    def init_magnetic(self, rho, u, b):
        a, c, e = self._dev(rho), self._dev(u), self._dev(b)
        assert a.numel() == self.N and c.numel() == 3 * self.N and e.numel() == 3 * self.N
        _check(lib().lbm_init_magnetic(self.h, a.data_ptr(), c.data_ptr(), e.data_ptr(), 1))
        self.stream.synchronize()

    def magnetic_fields(self):
        """(b, j) as device float64 tensors (3, nz, ny, nx)."""
        t = self.torch
        b = t.empty((3,) + self.shape, dtype=t.float64, device="cuda")
        j = t.empty((3,) + self.shape, dtype=t.float64, device="cuda")
        _check(lib().lbm_magnetic_fields(self.h, b.data_ptr(), j.data_ptr(), 1))
        self.stream.synchronize()
        return b, j

    def _coupled_q(self):
        """Populations per node of the coupled lattice (the library writes that
        many arrays of N doubles)."""
        q = {LBM_COUPLED_PHASE: 7, LBM_COUPLED_MAGNETIC: 21, LBM_COUPLED_COLOUR: 19}.get(self.params.coupled)
        if q is None:
            raise LbmError(LBM_EINVAL, "this lattice has no coupled populations")
        return q

    def get_coupled_populations(self):
        q = self._coupled_q()
        t = self.torch
        f = t.empty((q,) + self.shape, dtype=t.float64, device="cuda")
        _check(lib().lbm_get_coupled_populations(self.h, f.data_ptr(), 1))
        self.stream.synchronize()
        return f

    def set_coupled_populations(self, f):
        ff = self._dev(f)
        if ff.numel() != self._coupled_q() * self.N:
            raise ValueError(f"expected {self._coupled_q()} x {self.N} values, got {ff.numel()}")
        _check(lib().lbm_set_coupled_populations(self.h, ff.data_ptr(), 1))
        self.stream.synchronize()

    @property
    def device_bytes(self):
        return lbm_device_bytes(self.h)
