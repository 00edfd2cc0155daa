"""FP64 CPU oracle for the D3Q19 central-moment LBM (arXiv 2010.01628).

TEST INFRASTRUCTURE ONLY: this package is the reference the GPU library is
checked against.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
GPU path (``paper_2010_01628_amd``) and never imports it.

The arithmetic lives in plain C (``d3q19_oracle.c`` and friends), compiled
with gcc and OpenMP into ``liboracle.so``; this module only marshals numpy
arrays.  Each C function cites the paper passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIBRARY names another build of the same sources (the sanitized one)
_SO = os.environ.get("ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_SOURCES = ["d3q19_oracle.c", "d3q27_oracle.c", "mlp_oracle.c", "phase_oracle.c", "mhd_oracle.c",
            "shan_chen_oracle.c", "colour_gradient_oracle.c"]

DEFINITION = 0   # f* = T(u)^-1 k* by a dense solve per node
RM_DEFINITION = 2   # raw-moment variant of App. C (N = I): f* = M^-1 k* by a dense solve

Q = 19


SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def build(force: bool = True, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no HIP, no GPU headers).  ``sanitize``
    builds it with AddressSanitizer and UndefinedBehaviorSanitizer instead of
    -O3 (load it with gcc's libasan preloaded)."""
    so = out or _SO
    if not force and os.path.exists(so):
        return so
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    tmp = so + ".tmp"
    opt = SANITIZE if sanitize else ["-O3"]
    cmd = ["gcc", "-std=c11"] + opt + ["-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
                                       "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, so)
    return so


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        i32, f64 = ctypes.c_int, ctypes.c_double
        L.orc19_tables.argtypes = [ip, dp, ip]
        L.orc19_feq.argtypes = [f64, f64, f64, f64, dp]
        L.orc19_T.argtypes = [f64, f64, f64, dp]
        L.orc19_keq.argtypes = [f64, dp]
        L.orc19_Rcm.argtypes = [f64, f64, f64, dp]
        L.orc19_M.argtypes = [dp]
        L.orc19_keq_rm.argtypes = [f64, f64, f64, f64, dp]
        L.orc19_Rrm.argtypes = [f64, f64, f64, f64, f64, f64, dp]
        L.orc19_collide.argtypes = [dp, dp, dp, i32, dp, dp, dp, dp]
        L.orc19_collide.restype = i32
        L.orc19_K.argtypes = [f64, f64, dp, dp]
        L.orc19_step.argtypes = [i32, i32, i32, i32, dp, dp, dp, dp, i32, i32]
        L.orc19_step.restype = i32
        L.orc19_init.argtypes = [i32, i32, i32, dp, dp, dp]
        L.orc19_moments.argtypes = [i32, i32, i32, dp, dp, dp, dp]
        L.orc19_step_at.argtypes = [i32, i32, i32, i32, dp, dp, dp, i32, i32,
                                    ctypes.POINTER(ctypes.c_int64), i32, dp]
        L.orc19_step_at.restype = i32
        L.orc27_tables.argtypes = [ip, dp, ip]
        L.orc27_feq.argtypes = [f64, f64, f64, f64, dp]
        L.orc27_T.argtypes = [f64, f64, f64, dp]
        L.orc27_keq.argtypes = [f64, dp]
        L.orc27_Rcm.argtypes = [f64, f64, f64, dp]
        L.orc27_K.argtypes = [f64, dp]
        L.orc27_collide.argtypes = [dp, dp, dp, dp, dp, dp]
        L.orc27_collide.restype = i32
        L.orc27_step.argtypes = [i32, i32, i32, i32, dp, dp, dp, dp]
        L.orc27_step.restype = i32
        L.orc27_step_mode.argtypes = [i32, i32, i32, i32, dp, dp, dp, dp, i32]
        L.orc27_step_mode.restype = i32
        L.orc27_collide_mode.argtypes = [dp, dp, dp, i32, dp, dp, dp]
        L.orc27_collide_mode.restype = i32
        L.orc27_keq_rm.argtypes = [f64, f64, f64, f64, dp]
        L.orc27_Rrm.argtypes = [f64, f64, f64, f64, f64, f64, dp]
        L.orc27_init.argtypes = [i32, i32, i32, dp, dp, dp]
        L.orc27_moments.argtypes = [i32, i32, i32, dp, dp, dp, dp]
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.orc_mlp_nparam.restype = i32
        L.orc_bf16.argtypes = [f64]
        L.orc_bf16.restype = f64
        L.orc_mlp_features.argtypes = [f64, dp, dp, dp]
        L.orc_mlp_forward.argtypes = [dp, dp, i32, dp, dp, dp, dp]
        L.orc_mlp_rates.argtypes = [dp, dp]
        L.orc_mlp_rates.restype = i32
        L.orc19_step_mlp.argtypes = [i32, i32, i32, i32, dp, dp, dp, f64, dp, dp, i32]
        L.orc19_step_mlp.restype = ctypes.c_int64
        L.orc19_step_mlp_info.argtypes = [i32, i32, i32, i32, dp, dp, dp, f64, dp, dp, i32, f64, dp, dp]
        L.orc19_step_mlp_info.restype = ctypes.c_int64
        L.orc19_mlp_loss_grad.argtypes = [i32, i32, i32, dp, dp, f64, dp, dp, dp, i32, dp, i64p]
        L.orc19_mlp_loss_grad.restype = f64
        L.orc_pf_tables7.argtypes = [ip, dp]
        L.orc_pf_derivs.argtypes = [dp, dp, dp]
        L.orc_pf_macro.argtypes = [dp, dp, dp, dp]
        L.orc_pf_collide_g.argtypes = [f64, dp, f64, f64, dp, dp, dp, dp]
        L.orc_pf_collide_g.restype = i32
        L.orc_pf_collide_h.argtypes = [f64, f64, dp, dp, dp, dp]
        L.orc_pf_step.argtypes = [i32, i32, i32, dp, dp, dp, dp, dp]
        L.orc_pf_step.restype = i32
        L.orc_pf_init.argtypes = [i32, i32, i32, dp, dp, dp, dp, dp, dp]
        L.orc_pf_fields.argtypes = [i32, i32, i32, dp, dp, dp, dp, dp, dp, dp]
        L.orc_mhd_geq.argtypes = [dp, dp, dp]
        L.orc_mhd_current.argtypes = [dp, dp, f64, dp, dp]
        L.orc_mhd_step.argtypes = [i32, i32, i32, i32, dp, f64, dp, dp, dp, dp, dp]
        L.orc_mhd_step.restype = i32
        L.orc_mhd_init.argtypes = [i32, i32, i32, dp, dp, dp, dp, dp]
        L.orc_mhd_fields.argtypes = [i32, i32, i32, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_sc_psi.argtypes = [f64]
        L.orc_sc_psi.restype = f64
        L.orc_sc_force.argtypes = [i32, i32, i32, dp, f64, dp, dp]
        L.orc_sc_step.argtypes = [i32, i32, i32, f64, dp, dp, dp, dp, dp]
        L.orc_sc_step.restype = i32
        L.orc_sc_fields.argtypes = [i32, i32, i32, f64, dp, dp, dp, dp, dp]
        L.orc_sc_fields.restype = i32
        L.orc_cg_phi_i.argtypes = [i32, f64]
        L.orc_cg_phi_i.restype = f64
        L.orc_cg_heq.argtypes = [f64, f64, f64, f64, f64, dp]
        L.orc_cg_collide.argtypes = [dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_cg_collide.restype = i32
        L.orc_cg_step.argtypes = [i32, i32, i32, i32, dp, dp, dp, dp, dp]
        L.orc_cg_step.restype = i32
        L.orc_cg_init.argtypes = [i32, i32, i32, dp, dp, dp, dp, dp, dp]
        L.orc_cg_fields.argtypes = [i32, i32, i32, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.argtypes = [i32]
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def tables():
    """(c[19,3] int, w[19], opp[19]) in the paper's velocity order."""
    c = np.zeros((Q, 3), dtype=np.int32)
    w = np.zeros(Q)
    opp = np.zeros(Q, dtype=np.int32)
    lib().orc19_tables(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(w),
                       opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return c, w, opp


def feq(rho, u):
    out = np.zeros(Q)
    lib().orc19_feq(float(rho), float(u[0]), float(u[1]), float(u[2]), _p(out))
    return out


def T(u):
    out = np.zeros((Q, Q))
    lib().orc19_T(float(u[0]), float(u[1]), float(u[2]), _p(out))
    return out


def keq(rho):
    out = np.zeros(Q)
    lib().orc19_keq(float(rho), _p(out))
    return out


def Rcm(F):
    out = np.zeros(Q)
    lib().orc19_Rcm(float(F[0]), float(F[1]), float(F[2]), _p(out))
    return out


def M():
    """Raw-moment matrix of App. C (T at u = 0), row-major 19 x 19."""
    out = np.zeros((Q, Q))
    lib().orc19_M(_p(out))
    return out


def keq_rm(rho, u):
    out = np.zeros(Q)
    lib().orc19_keq_rm(float(rho), float(u[0]), float(u[1]), float(u[2]), _p(out))
    return out


def Rrm(u, F):
    out = np.zeros(Q)
    lib().orc19_Rrm(float(u[0]), float(u[1]), float(u[2]), float(F[0]), float(F[1]), float(F[2]), _p(out))
    return out


def K(omega, omega_bulk=1.0, omega_hi=None):
    out = np.zeros(Q)
    hi = None if omega_hi is None else _f64(omega_hi)
    lib().orc19_K(float(omega), float(omega_bulk), _p(hi), _p(out))
    return out


def _check_mode(mode):
    if mode not in (DEFINITION, RM_DEFINITION):
        raise ValueError(f"unknown collision mode {mode}")


def collide(f, F=(0.0, 0.0, 0.0), Kdiag=None, mode=DEFINITION):
    """One node.  Returns (f*, k, rho, u)."""
    _check_mode(mode)
    f = _f64(f)
    F = _f64(F)
    Kd = _f64(Kdiag if Kdiag is not None else K(1.0))
    fs = np.zeros(Q)
    k = np.zeros(Q)
    rho = np.zeros(1)
    u = np.zeros(3)
    rc = lib().orc19_collide(_p(f), _p(F), _p(Kd), int(mode), _p(fs), _p(k), _p(rho), _p(u))
    if rc != 0:
        raise ArithmeticError("singular collision system")
    return fs, k, float(rho[0]), u


def init(rho, u):
    """f = f_eq(rho, u) at every node.  rho: (nz,ny,nx); u: (3,nz,ny,nx)."""
    rho = _f64(rho)
    u = _f64(u)
    nz, ny, nx = rho.shape
    f = np.zeros((Q, nz, ny, nx))
    lib().orc19_init(nx, ny, nz, _p(rho), _p(u), _p(f))
    return f


def step(f, Kdiag, F=None, walls_y=False, mode=DEFINITION, out=None):
    """One collide-and-stream step.  f: (19,nz,ny,nx).  Kdiag: (19,) or (19,nz,ny,nx)."""
    _check_mode(mode)
    f = _f64(f)
    _, nz, ny, nx = f.shape
    Kd = _f64(Kdiag)
    per_node = 1 if Kd.ndim == 4 else 0
    Fa = None if F is None else _f64(F)
    if out is None:
        out = np.empty_like(f)
    rc = lib().orc19_step(nx, ny, nz, int(bool(walls_y)), _p(f), _p(out), _p(Fa), _p(Kd), per_node, int(mode))
    if rc != 0:
        raise ArithmeticError("singular collision system")
    return out


def run(f, nsteps, Kdiag, F=None, walls_y=False, mode=DEFINITION, progress=None, every=100):
    """nsteps steps; progress(t) (optional) is called after every `every` steps."""
    a = _f64(f).copy()
    b = np.empty_like(a)
    for t in range(int(nsteps)):
        step(a, Kdiag, F=F, walls_y=walls_y, mode=mode, out=b)
        a, b = b, a
        if progress is not None and (t + 1) % every == 0:
            progress(t + 1)
    return a


def step_at(f, nodes, Kdiag, F=None, walls_y=False, mode=DEFINITION):
    """f_i(x, t+1) (shape (len(nodes), 19)) at the given node indices only."""
    _check_mode(mode)
    f = _f64(f)
    _, nz, ny, nx = f.shape
    Kd = _f64(Kdiag)
    per_node = 1 if Kd.ndim == 4 else 0
    Fa = None if F is None else _f64(F)
    nd = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros((len(nd), Q))
    rc = lib().orc19_step_at(nx, ny, nz, int(bool(walls_y)), _p(f), _p(Fa), _p(Kd), per_node, int(mode),
                             nd.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(nd), _p(out))
    if rc != 0:
        raise ArithmeticError("singular collision system")
    return out


def moments(f, F=None):
    """(rho (nz,ny,nx), u (3,nz,ny,nx)) with the force-shifted velocity."""
    f = _f64(f)
    _, nz, ny, nx = f.shape
    rho = np.zeros((nz, ny, nx))
    u = np.zeros((3, nz, ny, nx))
    Fa = None if F is None else _f64(F)
    lib().orc19_moments(nx, ny, nz, _p(f), _p(Fa), _p(rho), _p(u))
    return rho, u


# --------------------------------------------------------------------------
# D3Q27 (App. D; readings Q1-Q4 in d3q27_oracle.c)
# --------------------------------------------------------------------------
Q27 = 27


class d3q27:
    @staticmethod
    def tables():
        c = np.zeros((Q27, 3), dtype=np.int32)
        w = np.zeros(Q27)
        opp = np.zeros(Q27, dtype=np.int32)
        lib().orc27_tables(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(w),
                           opp.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        return c, w, opp

    @staticmethod
    def feq(rho, u):
        out = np.zeros(Q27)
        lib().orc27_feq(float(rho), float(u[0]), float(u[1]), float(u[2]), _p(out))
        return out

    @staticmethod
    def T(u):
        out = np.zeros((Q27, Q27))
        lib().orc27_T(float(u[0]), float(u[1]), float(u[2]), _p(out))
        return out

    @staticmethod
    def keq(rho):
        out = np.zeros(Q27)
        lib().orc27_keq(float(rho), _p(out))
        return out

    @staticmethod
    def Rcm(F):
        out = np.zeros(Q27)
        lib().orc27_Rcm(float(F[0]), float(F[1]), float(F[2]), _p(out))
        return out

    @staticmethod
    def keq_rm(rho, u):
        out = np.zeros(Q27)
        lib().orc27_keq_rm(float(rho), float(u[0]), float(u[1]), float(u[2]), _p(out))
        return out

    @staticmethod
    def Rrm(u, F):
        out = np.zeros(Q27)
        lib().orc27_Rrm(float(u[0]), float(u[1]), float(u[2]), float(F[0]), float(F[1]), float(F[2]), _p(out))
        return out

    @staticmethod
    def K(omega):
        out = np.zeros(Q27)
        lib().orc27_K(float(omega), _p(out))
        return out

    @staticmethod
    def collide(f, F=(0.0, 0.0, 0.0), Kdiag=None, raw=False):
        """raw: the raw-moment variant (N = I)."""
        f = _f64(f)
        F = _f64(F)
        Kd = _f64(Kdiag if Kdiag is not None else d3q27.K(1.0))
        fs = np.zeros(Q27)
        rho = np.zeros(1)
        u = np.zeros(3)
        if lib().orc27_collide_mode(_p(f), _p(F), _p(Kd), int(bool(raw)), _p(fs), _p(rho), _p(u)) != 0:
            raise ArithmeticError("singular collision system")
        return fs, float(rho[0]), u

    @staticmethod
    def init(rho, u):
        rho = _f64(rho)
        u = _f64(u)
        nz, ny, nx = rho.shape
        f = np.zeros((Q27, nz, ny, nx))
        lib().orc27_init(nx, ny, nz, _p(rho), _p(u), _p(f))
        return f

    @staticmethod
    def step(f, Kdiag, F=None, walls_y=False, out=None, raw=False):
        f = _f64(f)
        _, nz, ny, nx = f.shape
        if out is None:
            out = np.empty_like(f)
        Fa = None if F is None else _f64(F)
        if lib().orc27_step_mode(nx, ny, nz, int(bool(walls_y)), _p(f), _p(out), _p(Fa), _p(_f64(Kdiag)),
                                 int(bool(raw))) != 0:
            raise ArithmeticError("singular collision system")
        return out

    @staticmethod
    def run(f, nsteps, Kdiag, F=None, walls_y=False, raw=False):
        a = _f64(f).copy()
        b = np.empty_like(a)
        for _ in range(int(nsteps)):
            d3q27.step(a, Kdiag, F=F, walls_y=walls_y, out=b, raw=raw)
            a, b = b, a
        return a

    @staticmethod
    def moments(f, F=None):
        f = _f64(f)
        _, nz, ny, nx = f.shape
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        Fa = None if F is None else _f64(F)
        lib().orc27_moments(nx, ny, nz, _p(f), _p(Fa), _p(rho), _p(u))
        return rho, u


# --------------------------------------------------------------------------
# Learned higher-order rates (readings L1-L5 in mlp_oracle.c)
# --------------------------------------------------------------------------
MLP_NIN, MLP_NH, MLP_NOUT = 11, 32, 9


class mlp:
    @staticmethod
    def nparam():
        return lib().orc_mlp_nparam()

    @staticmethod
    def unpack(P):
        P = _f64(P)
        o = 0
        out = {}
        for name, shape in (("W1", (32, 11)), ("b1", (32,)), ("W2", (32, 32)), ("b2", (32,)), ("W3", (9, 32)),
                            ("b3", (9,))):
            size = int(np.prod(shape))
            out[name] = P[o:o + size].reshape(shape)
            o += size
        return out

    @staticmethod
    def bf16(v):
        return lib().orc_bf16(float(v))

    @staticmethod
    def features(rho, k, scales):
        x = np.zeros(MLP_NIN)
        lib().orc_mlp_features(float(rho), _p(_f64(k)), _p(_f64(scales)), _p(x))
        return x

    @staticmethod
    def forward(P, x, bf16=False):
        xq, h1, h2, z = np.zeros(MLP_NIN), np.zeros(MLP_NH), np.zeros(MLP_NH), np.zeros(MLP_NOUT)
        lib().orc_mlp_forward(_p(_f64(P)), _p(_f64(x)), int(bf16), _p(xq), _p(h1), _p(h2), _p(z))
        return z, (xq, h1, h2)

    @staticmethod
    def rates(z):
        r = np.zeros(MLP_NOUT)
        fb = lib().orc_mlp_rates(_p(_f64(z)), _p(r))
        return r, bool(fb)

    @staticmethod
    def step(f, omega, P, scales, F=None, walls_y=False, bf16=False, out=None):
        f = _f64(f)
        _, nz, ny, nx = f.shape
        if out is None:
            out = np.empty_like(f)
        Fa = None if F is None else _f64(F)
        fb = lib().orc19_step_mlp(nx, ny, nz, int(bool(walls_y)), _p(f), _p(out), _p(Fa), float(omega),
                                  _p(_f64(P)), _p(_f64(scales)), int(bf16))
        if fb < 0:
            raise ArithmeticError("singular collision system")
        return out, int(fb)

    @staticmethod
    def step_info(f, omega, P, scales, F=None, walls_y=False, tie_ulps=64.0):
        """One BF16-emulating step; also returns per node (nz, ny, nx) how far
        its post-collision populations move if its values within tie_ulps of
        a bf16 tie round the other way (summed over those roundings, each
        flipped alone) and the smallest distance of its rates from the ends of
        (0, 2)."""
        f = _f64(f)
        _, nz, ny, nx = f.shape
        out = np.empty_like(f)
        flip = np.empty((nz, ny, nx))
        margin = np.empty((nz, ny, nx))
        Fa = None if F is None else _f64(F)
        fb = lib().orc19_step_mlp_info(nx, ny, nz, int(bool(walls_y)), _p(f), _p(out), _p(Fa), float(omega),
                                       _p(_f64(P)), _p(_f64(scales)), 1, float(tie_ulps), _p(flip), _p(margin))
        if fb < 0:
            raise ArithmeticError("singular collision system")
        return out, int(fb), flip, margin

    @staticmethod
    def run(f, nsteps, omega, P, scales, F=None, walls_y=False, bf16=False):
        a = _f64(f).copy()
        b = np.empty_like(a)
        total = 0
        for _ in range(int(nsteps)):
            _, fb = mlp.step(a, omega, P, scales, F=F, walls_y=walls_y, bf16=bf16, out=b)
            total += fb
            a, b = b, a
        return a, total

    @staticmethod
    def moments10(f):
        """The 10 raw moments of the training loss (rho, j, Pi) of populations
        f (19, nz, ny, nx): component k = sum_i f_i times the monomial k of c_i."""
        c, _, _ = tables()
        mono = np.stack([np.ones(Q), c[:, 0], c[:, 1], c[:, 2], c[:, 0] ** 2, c[:, 1] ** 2, c[:, 2] ** 2,
                         c[:, 0] * c[:, 1], c[:, 0] * c[:, 2], c[:, 1] * c[:, 2]]).astype(np.float64)
        return np.tensordot(mono, _f64(f), axes=(1, 0))

    @staticmethod
    def rollout_step_losses(f, targets, omega, P, scales, sigma, bf16=False):
        """`len(targets)` learned steps from the pre-collision populations f
        (periodic, no force); after step k the squared misfit of the 10
        moments against targets[k-1] in units of sigma, averaged over nodes
        and summed over the moments.  Returns (per-step losses, fallbacks)."""
        a = _f64(f).copy()
        b = np.empty_like(a)
        sig = _f64(sigma).reshape(10, 1, 1, 1)
        out, fbs = [], 0
        for tk in targets:
            _, fb = mlp.step(a, omega, P, scales, bf16=bf16, out=b)
            fbs += fb
            a, b = b, a
            r = (mlp.moments10(a) - _f64(tk)) / sig
            out.append(float(np.sum(r * r)) / (a.size // Q))
        return np.array(out), fbs

    @staticmethod
    def kinetic_energy(rho, j):
        """1/2 sum over the lattice of |j|^2 / rho."""
        return float(0.5 * np.sum((j[0] ** 2 + j[1] ** 2 + j[2] ** 2) / rho))

    @staticmethod
    def rollout_loss(f, targets, omega, P, scales, sigma, bf16=False, weights=None, energy_weight=0.0):
        """Rollout loss: the per-step losses (rollout_step_losses) averaged
        over the steps with weights (default all 1): sum_k w_k L_k / steps;
        with energy_weight w_E > 0 also (w_E / steps) sum_k ((E_k - T_k) /
        T_k)^2, E_k the kinetic energy of the populations after step k and
        T_k that of target k's moments.  Returns (loss, fallbacks)."""
        per, fbs = mlp.rollout_step_losses(f, targets, omega, P, scales, sigma, bf16=bf16)
        w = np.ones(len(per)) if weights is None else _f64(weights)
        loss = float(np.sum(w * per)) / len(per)
        if energy_weight:
            a = _f64(f).copy()
            b = np.empty_like(a)
            for tk in targets:
                mlp.step(a, omega, P, scales, bf16=bf16, out=b)
                a, b = b, a
                m = mlp.moments10(a)
                tk = _f64(tk)
                E = mlp.kinetic_energy(m[0], m[1:4])
                T = mlp.kinetic_energy(tk[0], tk[1:4])
                loss += energy_weight / len(per) * ((E - T) / T) ** 2
        return loss, fbs

    @staticmethod
    def loss_grad(f, target, omega, P, scales, sigma, bf16=False, want_grad=True):
        f = _f64(f)
        _, nz, ny, nx = f.shape
        g = np.zeros(mlp.nparam()) if want_grad else None
        fb = ctypes.c_int64(0)
        loss = lib().orc19_mlp_loss_grad(nx, ny, nz, _p(f), _p(_f64(target)), float(omega), _p(_f64(P)),
                                         _p(_f64(scales)), _p(_f64(sigma)), int(bf16), _p(g), ctypes.byref(fb))
        return loss, g, int(fb.value)


# --------------------------------------------------------------------------
# Two-phase flow: conservative phase field on D3Q7 coupled to velocity-based
# D3Q19 flow populations (readings P1-P6 in phase_oracle.c)
# --------------------------------------------------------------------------
class phase:
    """prm = (rho_l, rho_h, sigma, W, M, omega)."""

    @staticmethod
    def params(rho_l=1.0, rho_h=10.0, sigma=1e-3, W=4.0, M=0.1, omega=1.25):
        return np.array([rho_l, rho_h, sigma, W, M, omega], dtype=np.float64)

    @staticmethod
    def tables7():
        c = np.zeros((7, 3), dtype=np.int32)
        w = np.zeros(7)
        lib().orc_pf_tables7(c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _p(w))
        return c, w

    @staticmethod
    def derivs(phin):
        g = np.zeros(3)
        lap = np.zeros(1)
        lib().orc_pf_derivs(_p(_f64(phin)), _p(g), _p(lap))
        return g, float(lap[0])

    @staticmethod
    def macro(prm, g, phin):
        """dict of the node's Pi (= p/cs^2), rho, u, F, mu and S0."""
        out = np.zeros(10)
        lib().orc_pf_macro(_p(_f64(prm)), _p(_f64(g)), _p(_f64(phin)), _p(out))
        return {"Pi": out[0], "rho": out[1], "u": out[2:5], "F": out[5:8], "mu": out[8], "S0": out[9]}

    @staticmethod
    def collide_g(omega, g, Pi, rho, u, F, grad_rho):
        gs = np.zeros(19)
        if lib().orc_pf_collide_g(float(omega), _p(_f64(g)), float(Pi), float(rho), _p(_f64(u)), _p(_f64(F)),
                                  _p(_f64(grad_rho)), _p(gs)) != 0:
            raise ArithmeticError("singular collision system")
        return gs

    @staticmethod
    def collide_h(W, M, h, phin, u):
        hs = np.zeros(7)
        lib().orc_pf_collide_h(float(W), float(M), _p(_f64(h)), _p(_f64(phin)), _p(_f64(u)), _p(hs))
        return hs

    @staticmethod
    def init(prm, phi, p, u):
        phi = _f64(phi)
        nz, ny, nx = phi.shape
        g = np.zeros((19, nz, ny, nx))
        h = np.zeros((7, nz, ny, nx))
        lib().orc_pf_init(nx, ny, nz, _p(_f64(prm)), _p(phi), _p(_f64(p)), _p(_f64(u)), _p(g), _p(h))
        return g, h

    @staticmethod
    def step(prm, g, h, gout=None, hout=None):
        g = _f64(g)
        h = _f64(h)
        _, nz, ny, nx = g.shape
        gout = np.empty_like(g) if gout is None else gout
        hout = np.empty_like(h) if hout is None else hout
        rc = lib().orc_pf_step(nx, ny, nz, _p(_f64(prm)), _p(g), _p(h), _p(gout), _p(hout))
        if rc != 0:
            raise ArithmeticError("phase-field step failed")
        return gout, hout

    @staticmethod
    def run(prm, g, h, nsteps):
        a, b = _f64(g).copy(), _f64(h).copy()
        a2, b2 = np.empty_like(a), np.empty_like(b)
        for _ in range(int(nsteps)):
            phase.step(prm, a, b, a2, b2)
            a, a2 = a2, a
            b, b2 = b2, b
        return a, b

    @staticmethod
    def fields(prm, g, h):
        """(phi, p, rho, u): p = cs^2 Pi, u force-shifted."""
        g = _f64(g)
        h = _f64(h)
        _, nz, ny, nx = g.shape
        phi = np.zeros((nz, ny, nx))
        p = np.zeros_like(phi)
        rho = np.zeros_like(phi)
        u = np.zeros((3, nz, ny, nx))
        lib().orc_pf_fields(nx, ny, nz, _p(_f64(prm)), _p(g), _p(h), _p(phi), _p(p), _p(rho), _p(u))
        return phi, p, rho, u


# --------------------------------------------------------------------------
# Magnetohydrodynamics: D3Q7 vector magnetic lattice coupled to the D3Q19 CM
# flow (readings M1-M4 in mhd_oracle.c)
# --------------------------------------------------------------------------
class mhd:
    """prm = (eta, b_wall_x, b_wall_y, b_wall_z)."""

    @staticmethod
    def params(eta=0.1, b_wall=(0.0, 0.0, 0.0)):
        return np.array([eta, *b_wall], dtype=np.float64)

    @staticmethod
    def omega_m(eta):
        return 1.0 / (eta / 0.25 + 0.5)

    @staticmethod
    def geq(b, u):
        out = np.zeros(21)
        lib().orc_mhd_geq(_p(_f64(b)), _p(_f64(u)), _p(out))
        return out.reshape(3, 7)

    @staticmethod
    def current(g, u0, omega_m):
        b = np.zeros(3)
        j = np.zeros(3)
        lib().orc_mhd_current(_p(_f64(g).reshape(-1)), _p(_f64(u0)), float(omega_m), _p(b), _p(j))
        return b, j

    @staticmethod
    def init(rho, u, b):
        rho = _f64(rho)
        nz, ny, nx = rho.shape
        f = np.zeros((19, nz, ny, nx))
        g = np.zeros((21, nz, ny, nx))
        lib().orc_mhd_init(nx, ny, nz, _p(rho), _p(_f64(u)), _p(_f64(b)), _p(f), _p(g))
        return f, g

    @staticmethod
    def step(prm, omega, f, g, F=None, walls_y=False, fout=None, gout=None):
        f = _f64(f)
        g = _f64(g)
        _, nz, ny, nx = f.shape
        fout = np.empty_like(f) if fout is None else fout
        gout = np.empty_like(g) if gout is None else gout
        Fa = None if F is None else _f64(F)
        if lib().orc_mhd_step(nx, ny, nz, int(bool(walls_y)), _p(_f64(prm)), float(omega), _p(f), _p(g), _p(Fa),
                              _p(fout), _p(gout)) != 0:
            raise ArithmeticError("collision failed")
        return fout, gout

    @staticmethod
    def run(prm, omega, f, g, nsteps, F=None, walls_y=False):
        a, b = _f64(f).copy(), _f64(g).copy()
        a2, b2 = np.empty_like(a), np.empty_like(b)
        for _ in range(int(nsteps)):
            mhd.step(prm, omega, a, b, F=F, walls_y=walls_y, fout=a2, gout=b2)
            a, a2 = a2, a
            b, b2 = b2, b
        return a, b

    @staticmethod
    def fields(prm, f, g, F=None):
        """(rho, u, b, j): u force-shifted with the Lorentz force."""
        f = _f64(f)
        g = _f64(g)
        _, nz, ny, nx = f.shape
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        b = np.zeros_like(u)
        j = np.zeros_like(u)
        Fa = None if F is None else _f64(F)
        lib().orc_mhd_fields(nx, ny, nz, _p(_f64(prm)), _p(f), _p(g), _p(Fa), _p(rho), _p(u), _p(b), _p(j))
        return rho, u, b, j


class shan_chen:
    """Shan-Chen pseudo-potential two-phase flow (static-bubble case of
    Sec. III) on the paper's D3Q19 CM collision, periodic."""

    @staticmethod
    def psi(rho):
        return lib().orc_sc_psi(float(rho))

    @staticmethod
    def force(rho, G, Fu=None):
        rho = _f64(rho)
        nz, ny, nx = rho.shape
        F = np.zeros((3, nz, ny, nx))
        lib().orc_sc_force(nx, ny, nz, _p(rho), float(G), _p(None if Fu is None else _f64(Fu)), _p(F))
        return F

    @staticmethod
    def step(f, G, omega, Fu=None, out=None, F_out=None):
        """omega: the shear rate (the paper's K) or a full K diagonal (19)."""
        f = _f64(f)
        _, nz, ny, nx = f.shape
        out = np.empty_like(f) if out is None else out
        Kd = _f64(omega) if np.ndim(omega) else K(float(omega))
        if lib().orc_sc_step(nx, ny, nz, float(G), _p(None if Fu is None else _f64(Fu)), _p(Kd), _p(f),
                             _p(out), _p(F_out)) != 0:
            raise ArithmeticError("Shan-Chen step failed")
        return out

    @staticmethod
    def run(f, nsteps, G, omega, Fu=None):
        a = _f64(f).copy()
        b = np.empty_like(a)
        for _ in range(int(nsteps)):
            shan_chen.step(a, G, omega, Fu=Fu, out=b)
            a, b = b, a
        return a

    @staticmethod
    def fields(f, G, Fu=None):
        """(rho, u, p): u force-shifted with the interaction force;
        p = cs^2 rho + G cs^2 psi^2 / 2, the bulk pressure of the model."""
        f = _f64(f)
        _, nz, ny, nx = f.shape
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        p = np.zeros((nz, ny, nx))
        if lib().orc_sc_fields(nx, ny, nz, float(G), _p(None if Fu is None else _f64(Fu)), _p(f), _p(rho), _p(u),
                               _p(p)) != 0:
            raise MemoryError("Shan-Chen fields")
        return rho, u, p


class colour_gradient:
    """Colour-gradient two-phase flow of App. E on the D3Q19 CM collision
    (readings G1-G6 in colour_gradient_oracle.c)."""

    @staticmethod
    def params(omega, alpha_r, alpha_b=1.0 / 3.0, A=0.0, beta=0.7, g=(0.0, 0.0, 0.0), rho_ref=0.0):
        return np.array([omega, alpha_r, alpha_b, A, beta, g[0], g[1], g[2], rho_ref], dtype=np.float64)

    @staticmethod
    def phi_i(c2, alpha):
        return lib().orc_cg_phi_i(int(c2), float(alpha))

    @staticmethod
    def heq(rho, u, alpha):
        out = np.zeros(Q)
        lib().orc_cg_heq(float(rho), float(u[0]), float(u[1]), float(u[2]), float(alpha), _p(out))
        return out

    @staticmethod
    def collide(prm, fr, fb, grad):
        a, b = np.zeros(Q), np.zeros(Q)
        rho, u = np.zeros(1), np.zeros(3)
        if lib().orc_cg_collide(_p(_f64(fr)), _p(_f64(fb)), _p(_f64(grad)), _p(_f64(prm)), _p(a), _p(b), _p(rho),
                                _p(u)) != 0:
            raise ArithmeticError("singular collision system")
        return a, b, float(rho[0]), u

    @staticmethod
    def init(prm, rho_r, rho_b, u):
        rr, rb, uu = _f64(rho_r), _f64(rho_b), _f64(u)
        nz, ny, nx = rr.shape
        fr = np.zeros((Q, nz, ny, nx))
        fb = np.zeros((Q, nz, ny, nx))
        lib().orc_cg_init(nx, ny, nz, _p(_f64(prm)), _p(rr), _p(rb), _p(uu), _p(fr), _p(fb))
        return fr, fb

    @staticmethod
    def step(prm, fr, fb, walls_y=False, frn=None, fbn=None):
        fr, fb = _f64(fr), _f64(fb)
        _, nz, ny, nx = fr.shape
        frn = np.empty_like(fr) if frn is None else frn
        fbn = np.empty_like(fb) if fbn is None else fbn
        if lib().orc_cg_step(nx, ny, nz, int(bool(walls_y)), _p(_f64(prm)), _p(fr), _p(fb), _p(frn), _p(fbn)) != 0:
            raise ArithmeticError("colour-gradient step failed")
        return frn, fbn

    @staticmethod
    def run(prm, fr, fb, nsteps, walls_y=False):
        a, b = _f64(fr).copy(), _f64(fb).copy()
        a2, b2 = np.empty_like(a), np.empty_like(b)
        for _ in range(int(nsteps)):
            colour_gradient.step(prm, a, b, walls_y, a2, b2)
            a, a2 = a2, a
            b, b2 = b2, b
        return a, b

    @staticmethod
    def fields(prm, fr, fb):
        """(rho_r, rho_b, phi, u, p)."""
        fr, fb = _f64(fr), _f64(fb)
        _, nz, ny, nx = fr.shape
        rr, rb, phi, p = (np.zeros((nz, ny, nx)) for _ in range(4))
        u = np.zeros((3, nz, ny, nx))
        lib().orc_cg_fields(nx, ny, nz, _p(_f64(prm)), _p(fr), _p(fb), _p(rr), _p(rb), _p(phi), _p(u), _p(p))
        return rr, rb, phi, u, p
