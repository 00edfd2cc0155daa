"""lbm_moments_noalloc (partials in the library's fixed device array, no
allocation) against lbm_moments (partials in handle memory) through the C ABI:
identical per-node fields, totals equal up to the FP64 summation order, on two
calls in a row (the second on a smaller lattice), a lattice whose z planes are
grouped to fit the array, and the size limit."""
import ctypes

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


def make_lattice(nx, ny, nz, precision, streaming, walls, steps, seed):
    import torch

    rho, u, F = inputs.random_lattice_fields(nx, ny, nz, seed=seed, umax=0.05, fmax=1e-3)
    ff = torch.from_numpy(F).cuda()
    p = L.make_params(nx, ny, nz, precision=precision, streaming=streaming, omega=1.83,
                      force_mode=L.LBM_FORCE_FIELD, force_field_ptr=ff.data_ptr(), walls_y=walls)
    lat = L.Lattice(p, force_field=ff)
    lat.init(rho, u)
    lat.step(steps)
    return lat


def both(lat):
    import torch

    rho_a, u_a, diag_a = lat.moments()
    rho_b = torch.full(lat.shape, np.nan, dtype=torch.float64, device="cuda")
    u_b = torch.full((3,) + lat.shape, np.nan, dtype=torch.float64, device="cuda")
    diag_b = torch.full((6,), np.nan, dtype=torch.float64, device="cuda")
    L.lbm_moments_noalloc(lat.h, rho_b.data_ptr(), u_b.data_ptr(), diag_b.data_ptr())
    lat.stream.synchronize()
    return (rho_a.cpu().numpy(), u_a.cpu().numpy(), diag_a), (rho_b.cpu().numpy(), u_b.cpu().numpy(),
                                                              diag_b.cpu().numpy())


def check(lat, label):
    (ra, ua, da), (rb, ub, db) = both(lat)
    # per-node fields come from the same kernel arithmetic: equal bit for bit
    assert np.array_equal(ra, rb) and np.array_equal(ua, ub)
    # totals: same terms, summed in another grouping (1e-12 of the sum of magnitudes)
    scale = np.array([np.abs(ra).sum()] + [np.abs(ra[None] * ua).reshape(3, -1).sum(axis=1)[d] for d in range(3)]
                     + [abs(da[4]), abs(da[5])])
    err = np.abs(da - db) / scale
    say(f"  {label}: max |diag_noalloc - diag| / scale = {err.max():.2e}; max|u| equal: {da[5] == db[5]}")
    assert np.all(err <= 1e-12)
    assert da[5] == db[5]  # a maximum does not depend on the order


def test_two_calls_second_smaller():
    a = make_lattice(70, 45, 33, "fp64", "ab", False, 5, seed=3)
    check(a, "fp64 A-B 70x45x33")
    b = make_lattice(13, 9, 7, "fp32", "aa", True, 3, seed=4)
    check(b, "fp32 AA (odd step) 13x9x7 walls")
    # the array keeps the larger call's partials beyond the smaller one's: a
    # third call on the first lattice still agrees
    check(a, "fp64 A-B 70x45x33 again")
    a.close()
    b.close()


def test_plane_groups_fit_the_array():
    """300x64x400: 2 x 64 work-groups per plane, 400 planes -> 128 plane groups
    of about three planes each."""
    lat = make_lattice(300, 64, 400, "fp32", "ab", False, 2, seed=5)
    check(lat, "fp32 300x64x400 (grouped planes)")
    lat.close()


def test_diag_only_and_null_outputs():
    import torch

    lat = make_lattice(40, 30, 20, "bf16", "aa", False, 4, seed=6)
    _, _, da = lat.moments()
    d = torch.zeros(6, dtype=torch.float64, device="cuda")
    L.lbm_moments_noalloc(lat.h, None, None, d.data_ptr())
    L.lbm_moments_noalloc(lat.h, None, None, None)
    lat.stream.synchronize()
    db = d.cpu().numpy()
    assert abs(db[0] - da[0]) <= 1e-12 * da[0] and db[5] == da[5]
    lat.close()


def test_size_limit_and_coupled_rejected():
    lat = make_lattice(257, 8200, 1, "fp32", "ab", False, 0, seed=7)  # 2 x 8200 work-groups per plane
    d = np.zeros(6)
    import torch

    dd = torch.zeros(6, dtype=torch.float64, device="cuda")
    with pytest.raises(L.LbmError) as e:
        L.lbm_moments_noalloc(lat.h, None, None, dd.data_ptr())
    assert e.value.code == L.LBM_EINVAL and "16384" in str(e.value)
    lat.moments()  # the allocating entry point has no such limit
    lat.close()
    with pytest.raises(L.LbmError):
        L.lbm_moments_noalloc(None, None, None, None)
    del d
