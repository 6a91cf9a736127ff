"""P2 (quadratic Lagrange) elements on the HIP path against the oracle (needs a GPU).

Section 3 with p = 2 (the degree of Tables 3-5): M, K assembled from the
quadratic basis, N(psi) and the cubic load with degree-8 integrands, the
unchanged FGMRES / P_CH / PCG solver on the wider P2 pattern."""
import numpy as np
import pytest

from helpers import Problem, blockerr, dev, entryerr, host, rel
from oracle import assembly, pfc as opfc, solve as osolve

pytestmark = pytest.mark.gpu
M11 = 1.0 / opfc.ROS3PW_GAMMA
CASES = [(2, 6, 0.2), (2, 9, 0.0), (3, 3, 0.2), (3, 4, 0.1)]   # n = 144, 324, 216, 512


@pytest.fixture(scope="module")
def pfc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06852_amd import pfc as lib
    return lib


@pytest.mark.parametrize("dim,N,jit", CASES)
def test_p2_assembly_N_and_load(pfc, dim, N, jit):
    P = Problem(dim, N, jit, amp=0.3, seed=31, degree=2)
    try:
        m = P.gpu_mesh()
        assert pfc.pfc_mesh_grid_side(m) == 0   # P2 rows differ in width: columns stay stored
        rp, ci, mv, kv = pfc.pfc_mesh_export_csr(m)
        assert np.array_equal(rp, P.M.indptr) and np.array_equal(ci, P.M.indices)
        assert np.abs(mv - P.M.data).max() <= 1e-13 * np.abs(P.M.data).max()
        assert np.abs(kv - P.K.data).max() <= 1e-12 * np.abs(P.K.data).max()
        Nref = assembly.N_matrix(P.mesh, P.psi)
        Nd = dev(np.zeros(P.M.nnz))
        pfc.pfc_assemble_N(m, dev(P.psi), Nd)
        assert np.array_equal(Nref.indptr, P.M.indptr)
        assert np.abs(host(Nd) - Nref.data).max() <= 1e-13 * np.abs(Nref.data).max()
        g = dev(np.zeros(P.n))
        pfc.pfc_load_psi3(m, dev(P.psi), g)
        assert blockerr(host(g), assembly.load_psi3(P.mesh, P.psi), 1) <= 1e-13
    finally:
        P.close()


@pytest.mark.parametrize("dim,N,jit", CASES[:3])
def test_p2_apply_AR_and_stage_rhs(pfc, dim, N, jit):
    P = Problem(dim, N, jit, amp=0.2, seed=32, degree=2)
    inst = None
    try:
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default())
        n = P.n
        rng = np.random.default_rng(2)
        y = rng.normal(size=3 * n)
        r, tau = -0.35, 0.6
        N_ = assembly.N_matrix(P.mesh, P.psi)
        out = dev(np.zeros(3 * n))
        pfc.pfc_apply_AR(inst, n, dev(P.psi), r, tau, M11, dev(y), out)
        assert blockerr(host(out), opfc.apply_AR(P.M, P.K, N_, r, tau, M11, y)) <= 1e-13
        xk = np.concatenate([rng.normal(size=n), P.psi, rng.normal(size=n)])
        ys = rng.normal(size=(3, 3 * n)) * 0.1
        for stage in (1, 2, 3):
            xi = xk + sum(opfc.ROS3PW_A[(stage, j)] * ys[j - 1] for j in range(1, stage))
            c = [opfc.ROS3PW_C[(stage, j)] for j in range(1, stage)]
            bref = opfc.stage_rhs_R(P.mesh, P.M, P.K, r, tau, xi, [ys[j - 1][n:2 * n] for j in range(1, stage)], c)
            b = dev(np.zeros(3 * n))
            pfc.pfc_stage_rhs(inst, n, dev(xk), dev(ys.reshape(-1)), stage, r, tau, b)
            assert blockerr(host(b), bref) <= 1e-12, stage
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


# (2, 40): n = 6400, several workgroups with a ragged last one
@pytest.mark.parametrize("dim,N,jit,tau", [(2, 10, 0.2, 0.5), (3, 4, 0.1, 0.5), (2, 40, 0.2, 1.0)])
def test_p2_solve_replay_and_tolerance(pfc, dim, N, jit, tau):
    P = Problem(dim, N, jit, seed=33, degree=2)
    insts = []
    try:
        n = P.n
        r, psibar = -0.35, -0.3
        x0 = opfc.consistent_init(P.mesh, P.M, P.K, r, P.psi)
        b = opfc.stage_rhs_R(P.mesh, P.M, P.K, r, tau, x0, [], [])
        N_ = assembly.N_matrix(P.mesh, P.psi)
        y_ref, info = osolve.solve_stage(P.M, P.K, N_, r, tau, M11, b, tol=1e-8)
        s = info["schedule"]
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default())
        insts.append(inst)
        x = dev(np.zeros(3 * n))
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x, replay=(s.cycles, s.inner))
        assert gi["outer_iters"] == info["steps"]
        assert entryerr(host(x), y_ref) <= 1e-10
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, N_, r, tau, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8
        im = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(precision=pfc.PFC_MIXED))
        insts.append(im)
        st, gi = pfc.pfc_solve(im, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, N_, r, tau, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8
        # the PFC1 mobility is built for P1 meshes only
        with pytest.raises(pfc.PFCError):
            pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(model=pfc.PFC_MODEL_PFC1))
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        P.close()


@pytest.mark.parametrize("dim,N,jit,tau", [(2, 8, 0.2, 0.5), (3, 3, 0.1, 0.5)])
def test_p2_rosenbrock_replay_parity(pfc, dim, N, jit, tau):
    P = Problem(dim, N, jit, amp=0.05, seed=34, degree=2)
    inst = None
    try:
        r, psibar, steps = -0.35, -0.3, 2
        n = P.n
        x0 = opfc.consistent_init(P.mesh, P.M, P.K, r, P.psi)
        x_ref, infos = osolve.rosenbrock_run(P.mesh, P.M, P.K, x0, r, tau, steps, tol=1e-8)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default())
        state = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        reps = [(i["schedule"].cycles, i["schedule"].inner) for i in infos]
        st, gi = pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau, steps, pfc.PFC_INIT_CONSISTENT, replays=reps)
        assert [g["outer_iters"] for g in gi] == [i["steps"] for i in infos]
        assert entryerr(host(state), x_ref) <= 1e-10
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()
