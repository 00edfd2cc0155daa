"""CPU checks of the C ABI: the library loads, exports every symbol that
include/*.h declares, its parameter struct matches the ctypes mirror, and
parameter validation fails cleanly before any device call."""
import ctypes
import glob
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
INCLUDE = os.path.join(ROOT, "include")


def declared_symbols():
    names = set()
    for hdr in glob.glob(os.path.join(INCLUDE, "*.h")):
        text = open(hdr).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(lbm\w*)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lbm():
    from paper_2010_01628_amd import lbm as L

    L.lib()
    return L


def test_header_declares_entry_points():
    names = declared_symbols()
    for must in ("lbm_create", "lbm_init", "lbm_step", "lbm_moments", "lbm_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(lbm):
    out = subprocess.run(["nm", "-D", "--defined-only", lbm.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = declared_symbols() - exported
    assert not missing, f"declared but not exported: {sorted(missing)}"
    for name in declared_symbols():
        getattr(lbm.lib(), name)  # resolvable through ctypes


def test_params_struct_layout_matches_header(lbm, tmp_path):
    """Compile a C probe against include/lbm.h and compare sizeof/offsetof
    with the ctypes mirror used by the binding."""
    fields = [f for f, _ in lbm.lbm_params._fields_]
    src = tmp_path / "probe.c"
    body = "\n".join(f'printf("{f} %zu\\n", offsetof(lbm_params, {f}));' for f in fields)
    src.write_text(
        "#include <stddef.h>\n#include <stdio.h>\n#include \"lbm.h\"\n"
        "int main(void){" + body + 'printf("sizeof %zu\\n", sizeof(lbm_params)); return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", INCLUDE, str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for f in fields:
        assert int(got[f]) == getattr(lbm.lbm_params, f).offset, f
    assert int(got["sizeof"]) == ctypes.sizeof(lbm.lbm_params)
    # nested parameter blocks of the coupled lattices
    for sname, cls in (("lbm_phase_params", lbm.lbm_phase_params), ("lbm_magnetic_params", lbm.lbm_magnetic_params),
                       ("lbm_shan_chen_params", lbm.lbm_shan_chen_params),
                       ("lbm_colour_params", lbm.lbm_colour_params)):
        body = "\n".join(f'printf("{f} %zu\\n", offsetof({sname}, {f}));' for f, _ in cls._fields_)
        src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"lbm.h\"\n"
                       "int main(void){" + body + f'printf("sizeof %zu\\n", sizeof({sname})); return 0;}}\n')
        subprocess.run(["gcc", "-I", INCLUDE, str(src), "-o", str(exe)], check=True)
        got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
        for f, _ in cls._fields_:
            assert int(got[f]) == getattr(cls, f).offset, (sname, f)
        assert int(got["sizeof"]) == ctypes.sizeof(cls)


def test_defaults(lbm):
    p = lbm.lbm_params_default()
    assert p.abi_version == lbm.ABI_VERSION
    assert (p.nx, p.ny, p.nz, p.q) == (32, 32, 32, 19)
    assert p.omega == 1.0 and p.omega_bulk == 1.0 and list(p.omega_hi) == [1.0] * 9
    assert p.rho0 == 1.0 and p.precision == lbm.LBM_FP32 and p.streaming == lbm.LBM_AB


@pytest.mark.parametrize("field,value,code", [
    ("omega", 2.0, -1), ("omega", 0.0, -1), ("omega", float("nan"), -1),
    ("omega_bulk", 2.5, -1), ("nx", 0, -1), ("q", 15, -1),
    ("precision", 7, -1), ("streaming", 3, -1), ("rho0", -1.0, -1),
    ("force_mode", 2, -1),  # FIELD without a pointer
    ("check_every", -3, -1), ("abi_version", 99, -1),
])
def test_invalid_params_rejected_before_device_use(lbm, field, value, code):
    p = lbm.lbm_params_default()
    setattr(p, field, value)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, None)
    assert e.value.code == code
    assert lbm.lib().lbm_last_error().decode()


def test_d3q27_restrictions(lbm):
    p = lbm.lbm_params_default()
    p.q = 27
    p.precision = lbm.LBM_FP16_SHIFTED
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, None)
    assert e.value.code == lbm.LBM_EUNSUPPORTED
    p.precision = lbm.LBM_FP32
    p.omega_bulk = 1.2
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, None)
    assert e.value.code == lbm.LBM_EUNSUPPORTED


def test_block_shape_validation(lbm):
    p = lbm.lbm_params_default()
    p.block_x, p.block_y = 48, 1
    with pytest.raises(lbm.LbmError):
        lbm.lbm_create(p, None)
    p.block_x, p.block_y = 512, 1
    with pytest.raises(lbm.LbmError):
        lbm.lbm_create(p, None)


def _phase_params(lbm, **kw):
    p = lbm.make_params(16, 16, 16, precision="fp32",
                        phase=dict(rho_light=1.0, rho_heavy=10.0, sigma=1e-3, width=4.0, mobility=0.1))
    for k, v in kw.items():
        if k in ("rho_light", "rho_heavy", "sigma", "width", "mobility"):
            setattr(p.phase, k, v)
        else:
            setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw,code", [
    (dict(q=27), -5), (dict(precision=2), -5), (dict(streaming=1), -5), (dict(walls_y=1), -5),
    (dict(force_mode=1), -5), (dict(omega_bulk=1.5), -5), (dict(rho0=2.0), -1),
    (dict(width=0.0), -1), (dict(mobility=-0.1), -1), (dict(rho_light=0.0), -1), (dict(sigma=-1.0), -1),
    (dict(coupled=7), -1),
])
def test_phase_lattice_validation(lbm, kw, code):
    p = _phase_params(lbm, **kw)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, None)
    assert e.value.code == code, lbm.lib().lbm_last_error().decode()


@pytest.mark.parametrize("kw,code", [
    (dict(q=27), -5), (dict(precision=3), -5), (dict(streaming=1), -5), (dict(omega_bulk=1.2), -5),
    (dict(eta=0.0), -1), (dict(eta=float("nan")), -1),
])
def test_magnetic_lattice_validation(lbm, kw, code):
    p = lbm.make_params(8, 8, 8, precision="fp32", magnetic=dict(eta=0.1, b_wall=(0.0, 0.01, 0.0)))
    for k, v in kw.items():
        if k == "eta":
            p.magnetic.eta = v
        else:
            setattr(p, k, v)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, None)
    assert e.value.code == code, lbm.lib().lbm_last_error().decode()


@pytest.mark.parametrize("kw,code", [
    (dict(moments=2), -1), (dict(moments=-1), -1), (dict(moments=1, q=27, precision=2), -5),
    (dict(moments=1, phase=True), -5), (dict(moments=1, magnetic=True), -5),
])
def test_raw_moment_validation(lbm, kw, code):
    kw = dict(kw)
    extra = {}
    if kw.pop("phase", False):
        extra["phase"] = dict(rho_light=1.0, rho_heavy=10.0, sigma=1e-3, width=4.0, mobility=0.1)
    if kw.pop("magnetic", False):
        extra["magnetic"] = dict(eta=0.1)
    p = lbm.make_params(8, 8, 8, precision="fp32", **extra)
    for k, v in kw.items():
        setattr(p, k, v)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, None)
    assert e.value.code == code, lbm.lib().lbm_last_error().decode()


@pytest.mark.parametrize("kw,code", [
    (dict(q=27), -5), (dict(precision=2), -5), (dict(streaming=1), -5), (dict(walls_y=1), -5),
    (dict(force_mode=3), -5), (dict(G=float("inf")), -1), (dict(moments=1), -5),
])
def test_shan_chen_lattice_validation(lbm, kw, code):
    p = lbm.make_params(8, 8, 8, precision="fp32", shan_chen=dict(G=-5.0))
    for k, v in kw.items():
        if k == "G":
            p.shan_chen.G = v
        else:
            setattr(p, k, v)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, None)
    assert e.value.code == code, lbm.lib().lbm_last_error().decode()


@pytest.mark.parametrize("kw,code", [
    (dict(q=27), -5), (dict(precision=2), -5), (dict(streaming=1), -5), (dict(force_mode=1), -5),
    (dict(omega_bulk=1.3), -5), (dict(alpha_red=1.0), -1), (dict(alpha_blue=-0.1), -1), (dict(A=-1.0), -1),
    (dict(beta=1.5), -1), (dict(rho_ref=float("nan")), -1), (dict(moments=1), -5),
])
def test_colour_lattice_validation(lbm, kw, code):
    p = lbm.make_params(8, 8, 8, precision="fp32", colour=dict(alpha_red=7.0 / 9.0))
    for k, v in kw.items():
        if k in ("alpha_red", "alpha_blue", "A", "beta", "rho_ref"):
            setattr(p.colour, k, v)
        else:
            setattr(p, k, v)
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(p, None)
    assert e.value.code == code, lbm.lib().lbm_last_error().decode()


@pytest.mark.parametrize("src,n,q,eb,lane", [(0, 16, 19, 4, 0), (64, -1, 19, 4, 0), (64, 16, 15, 4, 0),
                                              (64, 16, 19, 3, 0), (64, (1 << 31) * 256 + 1, 19, 4, 0),
                                              (64, 16, 19, 8, 4), (64, 16, 19, 4, 32), (64, 3, 19, 2, 8),
                                              (64, 16, 19, 8, 7)])
def test_stream_copy_validation(lbm, src, n, q, eb, lane):
    """The bandwidth reference rejects bad arguments before any device use
    (the pointers here are never dereferenced)."""
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_stream_copy(src, 64, n, q, eb, lane_bytes=lane)
    assert e.value.code == lbm.LBM_EINVAL
    assert "lbm_stream_copy" in lbm.lib().lbm_last_error().decode()


def test_stream_copy_of_nothing_enqueues_nothing(lbm):
    """n = 0 returns before any device call (so it succeeds without a GPU)."""
    lbm.lbm_stream_copy(64, 64, 0, 19, 4)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises; there is no CPU
    fallback to take its place."""
    from paper_2010_01628_amd import lbm as L

    monkeypatch.setattr(L, "_lib", None)
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "liblbm.so"))
    with pytest.raises(ImportError):
        L.lib()
    with pytest.raises(ImportError):
        L.Lattice(L.make_params(8, 8, 8))


def test_without_a_device_every_create_fails_cleanly(lbm):
    """Valid parameters on a host with no GPU: each create call reports
    LBM_EDEVICE and hands back no handle (nothing is left half-built)."""
    import numpy as np
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    extras = [{}, dict(phase=dict(rho_light=1.0, rho_heavy=10.0, sigma=1e-3, width=4.0, mobility=0.1)),
              dict(magnetic=dict(eta=0.1)), dict(shan_chen=dict(G=-5.0)), dict(colour=dict(alpha_red=7.0 / 9.0))]
    for extra in extras:
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_create(lbm.make_params(16, 16, 16, precision="fp32", **extra), None)
        assert e.value.code == lbm.LBM_EDEVICE
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_mlp_create(None, np.ones(11))
    assert e.value.code == lbm.LBM_EDEVICE
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_ensemble_create([(8, 1.5), (12, 1.2)])
    assert e.value.code == lbm.LBM_EDEVICE


def test_energy_weight_validation(lbm):
    for w in (-1.0, float("nan"), float("inf")):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_mlp_set_energy_weight(0, w)
        assert e.value.code == lbm.LBM_EINVAL


def test_null_handles(lbm):
    """NULL handles: destroy is a no-op, queries report an error."""
    lbm.lbm_destroy(0)
    lbm.lbm_mlp_destroy(0)
    assert lbm.lbm_step_count(0) == -1
    assert lbm.lbm_step_variant(0) == -1
    for call in (lambda: lbm.lbm_step(0, 1), lambda: lbm.lbm_init(0, 0, 0, False),
                 lambda: lbm.lbm_moments(0, 0, 0, 0, False), lambda: lbm.lbm_moments_noalloc(0, 0, 0, 0),
                 lambda: lbm.lbm_get_populations(0, 0, False), lambda: lbm.lbm_set_populations(0, 0, False)):
        with pytest.raises(lbm.LbmError) as e:
            call()
        assert e.value.code == lbm.LBM_EINVAL
