"""The allocation-free operator apply (needs a GPU): pfc_apply_AR_noalloc, which keeps N(psi_k) in the
library's static scratch array, gives the bits of pfc_apply_AR (the same kernels on an instance's
memory) on two calls in a row, the second on a smaller mesh, and the oracle's A^R y (Section 3.1,
eq. rosenbrock_matrix) element by element; a mesh beyond the scratch size is refused."""
import numpy as np
import pytest

from helpers import Problem, blockerr, dev, host
from oracle import assembly, pfc as opfc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pfc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06852_amd import pfc as lib
    return lib


def _apply_both(pfc, P, seed):
    import torch
    n = P.n
    rng = np.random.default_rng(seed)
    y = rng.normal(size=3 * n)
    r, tau, m11 = -0.35, 0.7, 1.0 / opfc.ROS3PW_GAMMA
    mesh = P.gpu_mesh()
    inst = pfc.pfc_instance_create(mesh, pfc.pfc_opts_default())
    try:
        out_inst = dev(np.zeros(3 * n))
        pfc.pfc_apply_AR(inst, n, dev(P.psi), r, tau, m11, dev(y), out_inst)
        out_na = dev(np.full(3 * n, np.nan))
        print(f"no-alloc apply: {P.mesh.dim}D n = {n}", flush=True)
        pfc.pfc_apply_AR_noalloc(mesh, n, dev(P.psi), r, tau, m11, dev(y), out_na,
                                 stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        a, b = host(out_na), host(out_inst)
        ref = opfc.apply_AR(P.M, P.K, assembly.N_matrix(P.mesh, P.psi), r, tau, m11, y)
        return a, b, ref
    finally:
        pfc.pfc_instance_destroy(inst)


def test_noalloc_apply_matches_instance_apply(pfc):
    big, small = Problem(2, 160, 0.2, seed=41), Problem(3, 6, 0.0, seed=42)
    try:
        for P, seed in ((big, 1), (small, 2)):   # the second call on a smaller mesh
            a, b, ref = _apply_both(pfc, P, seed)
            assert np.array_equal(a, b), P.n
            assert blockerr(a, ref) <= 1e-13
    finally:
        big.close()
        small.close()


def test_noalloc_apply_refuses_meshes_beyond_scratch(pfc):
    import workloads as wl
    mesh = wl.make_mesh(3, 66)   # 287,496 nodes x 15 entries > 2^22
    h = pfc.pfc_mesh_create_p1(3, mesh.n, mesh.elem_nodes, mesh.elem_coords)
    try:
        n = mesh.n
        z = dev(np.zeros(3 * n))
        with pytest.raises(pfc.PFCError) as e:
            pfc.pfc_apply_AR_noalloc(h, n, dev(np.zeros(n)), -0.3, 0.5, 1.0, z, z)
        assert e.value.code == pfc.PFC_ERR_ARG and "scratch" in str(e.value)
    finally:
        pfc.pfc_mesh_destroy(h)
