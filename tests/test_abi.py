"""C ABI checks that need no GPU: the library loads, exports every symbol
declared in include/pfc.h, and rejects invalid arguments on the host before
any device work."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pfc():
    if not os.path.exists(os.path.join(ROOT, "paper_1501_06852_amd", "libpfc.so")):
        pytest.skip("library not built")
    from paper_1501_06852_amd import pfc as lib
    return lib


def _declared():
    src = open(os.path.join(ROOT, "include", "pfc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pfc_[A-Za-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree(pfc):
    assert _declared() == sorted(pfc.DECLARED)


def test_every_declared_symbol_is_exported(pfc):
    missing = [s for s in _declared() if not hasattr(pfc._lib, s)]
    assert not missing, missing


def test_status_strings_and_defaults(pfc):
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6):
        assert pfc.pfc_status_str(code) != "unknown status"
    o = pfc.pfc_opts_default()
    assert o.struct_size == C.sizeof(pfc.pfc_opts)
    assert (o.restart, o.outer_tol, o.inner_tol, o.precision) == (30, 1e-8, 1e-3, pfc.PFC_FP64)


def test_tau_critical_matches_oracle(pfc):
    from oracle.symbols import tau_star
    for r, pb in [(-0.35, 0.0), (-0.35, -0.34), (-0.3, -0.25), (-0.3, -0.4)]:
        a, b = pfc.pfc_tau_critical(r, pb), tau_star(r, pb)
        assert (math.isinf(a) and math.isinf(b)) or abs(a - b) <= 1e-12 * b


def test_mesh_validation_on_host(pfc):
    # node index out of range, repeated node, wrong dimension: rejected before any device call
    with pytest.raises(pfc.PFCError) as e:
        pfc.pfc_mesh_create_p1(2, 4, np.array([[0, 1, 5]]), np.zeros((1, 3, 2)))
    assert e.value.code == pfc.PFC_ERR_ARG and "out of range" in str(e.value)
    with pytest.raises(pfc.PFCError):
        pfc.pfc_mesh_create_p1(2, 4, np.array([[0, 1, 1]]), np.zeros((1, 3, 2)))
    h = C.c_void_p()
    assert pfc._lib.pfc_mesh_create_p1(4, 4, 1, None, None, C.byref(h)) == pfc.PFC_ERR_ARG
    # empty meshes, a node outside every simplex, zero-volume simplices (collinear / coplanar vertices)
    assert pfc._lib.pfc_mesh_create_p1(2, 0, 0, None, None, C.byref(h)) == pfc.PFC_ERR_ARG
    with pytest.raises(pfc.PFCError) as e:
        pfc.pfc_mesh_create_p1(2, 4, np.array([[0, 1, 2]]), np.array([[[0, 0], [1, 0], [0, 1]]], float))
    assert e.value.code == pfc.PFC_ERR_ARG and "no element" in str(e.value)
    with pytest.raises(pfc.PFCError) as e:
        pfc.pfc_mesh_create_p1(2, 3, np.array([[0, 1, 2]]), np.array([[[0, 0], [1, 0], [2, 0]]], float))
    assert e.value.code == pfc.PFC_ERR_ARG and "degenerate" in str(e.value)
    tet = np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]]], float)
    with pytest.raises(pfc.PFCError) as e:
        pfc.pfc_mesh_create_p1(3, 4, np.array([[0, 1, 2, 3]]), tet)
    assert e.value.code == pfc.PFC_ERR_ARG and "degenerate" in str(e.value)
    # a thin but valid simplex passes the host checks (without a device the call then fails in HIP)
    thin = np.ascontiguousarray([[[0, 0], [1, 0], [0.5, 1e-6]]], dtype=np.float64)
    en = np.ascontiguousarray([[0, 1, 2]], dtype=np.int32)
    rc = pfc._lib.pfc_mesh_create_p1(2, 3, 1, en.ctypes.data_as(pfc._ip), thin.ctypes.data_as(pfc._dp), C.byref(h))
    assert rc in (pfc.PFC_OK, pfc.PFC_ERR_HIP), pfc.pfc_last_error()
    if rc == pfc.PFC_OK:
        pfc.pfc_mesh_destroy(h)
    # CSR: missing diagonal, unsorted columns, asymmetric pattern
    rp = np.array([0, 1, 2], np.int32)
    with pytest.raises(pfc.PFCError):
        pfc.pfc_mesh_create_csr(2, 2, rp, np.array([1, 0], np.int32), np.ones(2), np.ones(2),
                                np.array([[0, 1, 0]]), np.ones(1))
    with pytest.raises(pfc.PFCError):
        pfc.pfc_mesh_create_csr(2, 2, np.array([0, 2, 3], np.int32), np.array([1, 0, 1], np.int32), np.ones(3),
                                np.ones(3), np.array([[0, 1, 0]]), np.ones(1))


def test_null_handles_rejected(pfc):
    v = C.c_void_p()
    assert pfc._lib.pfc_solve(None, None, 0.0, 0.0, 0.1, 1.0, None, None, None, None, None) == pfc.PFC_ERR_ARG
    assert pfc._lib.pfc_rosenbrock_run(None, None, 0.0, 0.0, 0.1, 1, 0, None, None, None) == pfc.PFC_ERR_ARG
    assert pfc._lib.pfc_instance_footprint(None, None) == 0
    o = pfc.pfc_opts_default(restart=64)
    assert pfc._lib.pfc_instance_create(None, C.byref(o), C.byref(v)) == pfc.PFC_ERR_ARG
    assert pfc._lib.pfc_batch_run(None, 0, None, None, None, None, 1, 0, None, None) == pfc.PFC_ERR_ARG
    assert pfc._lib.pfc_spmv(None, 0, None, None, None) == pfc.PFC_ERR_ARG
    assert pfc._lib.pfc_mesh_grid_side(None, None) == pfc.PFC_ERR_ARG
    # the grid_columns option takes 0 or 1
    o = pfc.pfc_opts_default(grid_columns=2)
    assert pfc.pfc_opts_default().grid_columns == 1
    assert pfc._lib.pfc_instance_footprint(C.c_void_p(1), C.byref(o)) == 0
    # gamma_mode takes the two readings, inner_fixed non-negative counts
    for bad in (pfc.pfc_opts_default(gamma_mode=2), pfc.pfc_opts_default(inner_fixed=[0, -1, 0, 0, 0])):
        assert pfc._lib.pfc_instance_footprint(C.c_void_p(1), C.byref(bad)) == 0
    d = pfc.pfc_opts_default()
    assert d.gamma_mode == pfc.PFC_GAMMA_SCALE_ROW and list(d.inner_fixed) == [0] * 5
    # one or two PCG iterations per launch
    assert d.pcg_steps_per_launch == 2
    for bad in (0, 3, -1):
        o = pfc.pfc_opts_default(pcg_steps_per_launch=bad)
        assert pfc._lib.pfc_instance_footprint(C.c_void_p(1), C.byref(o)) == 0


def test_product_path_does_not_import_oracle():
    """The package and the bench's timed path never import the oracle."""
    pkg = os.path.join(ROOT, "paper_1501_06852_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f


def test_p2_mesh_and_pfc1_validation_on_host(pfc):
    h = C.c_void_p()
    # P2: wrong dimension, node index out of range, repeated node
    assert pfc._lib.pfc_mesh_create_p2(4, 10, 1, None, None, C.byref(h)) == pfc.PFC_ERR_ARG
    with pytest.raises(pfc.PFCError):
        pfc.pfc_mesh_create_p2(2, 6, np.array([[0, 1, 2, 3, 4, 9]]), np.zeros((1, 3, 2)))
    with pytest.raises(pfc.PFCError):
        pfc.pfc_mesh_create_p2(2, 6, np.array([[0, 1, 2, 3, 4, 4]]), np.zeros((1, 3, 2)))
    with pytest.raises(ValueError):   # shapes: 6 nodes but coordinates of 4 vertices
        pfc.pfc_mesh_create_p2(2, 6, np.array([[0, 1, 2, 3, 4, 5]]), np.zeros((1, 4, 2)))
    # options: unknown model, non-finite psi_min; the full-state entry points reject null handles
    o = pfc.pfc_opts_default(model=5)
    assert pfc._lib.pfc_instance_footprint(C.c_void_p(1), C.byref(o)) == 0
    o = pfc.pfc_opts_default(psi_min=float("nan"))
    assert pfc._lib.pfc_instance_footprint(C.c_void_p(1), C.byref(o)) == 0
    assert pfc._lib.pfc_solve_x(None, None, 0.0, 0.0, 0.1, 1.0, None, None, None, None, None) == pfc.PFC_ERR_ARG
    assert pfc._lib.pfc_apply_AR_x(None, None, 0.0, 0.1, 1.0, None, None, None) == pfc.PFC_ERR_ARG
    d = pfc.pfc_opts_default()
    assert (d.model, d.psi_min) == (pfc.PFC_MODEL_PFC2, -1.5)
