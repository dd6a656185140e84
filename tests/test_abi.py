"""The C-ABI library loads, exports every declared symbol, and validates its
arguments before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2609_07172_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "cylpoisson.h")).read()
    return sorted(set(re.findall(r"\b(cylpoisson_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = P.library()
    names = declared_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(P.EXPORTED_SYMBOLS) == names


@pytest.mark.parametrize("args", [
    (2, 4, 5, 0.02, 0.05, 0.01),        # Nr < 3
    (5, 4, 2, 0.02, 0.05, 0.01),        # Nz < 3
    (5, 0, 5, 0.02, 0.05, 0.01),        # Ntheta < 1
    (5, 4, 5, 0.0, 0.05, 0.01),         # r_in not positive
    (5, 4, 5, 0.05, 0.02, 0.01),        # r_out <= r_in
    (5, 4, 5, 0.02, 0.05, 0.0),         # dz not positive
    (5, 4, 5, 0.02, float("nan"), 0.01),
])
def test_plan_create_rejects_bad_geometry(args):
    with pytest.raises(P.CylPoissonError) as e:
        P.plan_create(*args)
    assert e.value.status == P.EINVAL
    assert P.last_error()


def test_plan_create_rejects_non_finite_bc():
    with pytest.raises(P.CylPoissonError):
        P.plan_create(5, 4, 5, 0.02, 0.05, 0.01, bc=(0.0, float("inf"), 0.0, 0.0))
    assert "finite" in P.last_error()


def test_null_plan_and_status_strings():
    lib = P.library()
    lib.cylpoisson_plan_destroy(None)  # NULL-safe
    assert lib.cylpoisson_solve(None, None, None, 1e-12, None) == P.EINVAL
    assert lib.cylpoisson_apply(None, None, None, None) == P.EINVAL
    assert lib.cylpoisson_dft_forward(None, None, None, None) == P.EINVAL
    assert lib.cylpoisson_dft_inverse(None, None, None, None) == P.EINVAL
    assert lib.cylpoisson_solve_planes(None, None, None, 1e-12, None) == P.EINVAL
    assert lib.cylpoisson_get_stats(None, None) == P.EINVAL
    assert lib.cylpoisson_get_info(None, None) == P.EINVAL
    assert lib.cylpoisson_plan_set_option(None, b"nu1", 2.0) == P.EINVAL
    v = ctypes.c_double()
    assert lib.cylpoisson_plan_get_option(None, b"nu1", ctypes.byref(v)) == P.EINVAL
    assert lib.cylpoisson_autotune(None, None) == P.EINVAL
    # a negative count is rejected before any HIP call
    assert lib.cylpoisson_solve_batch(None, None, None, -1, 1e-12, None, None) == P.EINVAL
    for code in (P.OK, P.NOT_CONVERGED, P.EINVAL, P.ENOMEM, P.EHIP, P.ENONFINITE, P.EDEVICE):
        assert P.status_string(code) != "unknown status"
    assert P.status_string(42) == "unknown status"


@pytest.mark.parametrize("r,z,layout,msg", [
    ([0.02, 0.03, 0.03, 0.05], [0.0, 0.01, 0.02], P.VERTEX, "increasing"),   # repeated radius
    ([0.0, 0.01, 0.02], [0.0, 0.01, 0.02], P.VERTEX, "above 0"),              # the axis
    ([0.02, 0.03, 0.05], [0.0, float("nan"), 0.02], P.VERTEX, "finite"),
    ([0.02, 0.03, 0.05], [0.02, 0.01, 0.0], P.VERTEX, "increasing"),          # decreasing z
    ([1.0e308, 1.5e308, 1.7e308], [0.0, 0.01, 0.02], P.VERTEX, "finite"),     # faces overflow
    ([0.02, 0.05], [0.0, 0.01], P.CELL, "increasing"),                        # wrong count (Python)
])
def test_plan_create_mesh_rejects_bad_meshes(r, z, layout, msg):
    if layout == P.CELL:
        with pytest.raises(ValueError):
            P.plan_create_mesh(len(r), 2, len(z) + 1, r, z, layout)
        return
    with pytest.raises(P.CylPoissonError) as e:
        P.plan_create_mesh(len(r), 2, len(z), r, z, layout)
    assert e.value.status == P.EINVAL
    assert msg in P.last_error()


def test_plan_create_mesh_rejects_null_and_bad_layout():
    lib = P.library()
    bc = P.BC(0.0, 0.0, 0.0, 0.0)
    arr = (ctypes.c_double * 3)(0.02, 0.03, 0.04)
    assert not lib.cylpoisson_plan_create_mesh(3, 2, 3, None, arr, P.VERTEX, ctypes.byref(bc))
    assert "NULL" in P.last_error()
    assert not lib.cylpoisson_plan_create_mesh(3, 2, 3, arr, arr, 7, ctypes.byref(bc))
    assert "layout" in P.last_error()
    assert not lib.cylpoisson_plan_create_mesh(3, 2, 3, arr, arr, P.VERTEX, None)
    assert "bc" in P.last_error()
