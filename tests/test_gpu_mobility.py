"""PFC1 mobility model on the HIP path against the oracle (needs a GPU).

K_+(psi_k) and F(mu_k) in the stage matrix, -K_+(psi_i) mu_i in the stage
right-hand side, P_CH built for the time step M0 tau (oracle.mobility).

Solve-level cases start from smooth states (workloads.psi_smooth): with
grid-scale noise the mobility derivative tau F(mu_k) dominates the stage
matrix and P_CH, which drops it (Section 4), no longer makes FGMRES converge,
on the oracle as on the GPU; on the smallest boxes only the longest waves
(kmax = 1) keep the PFC1 time integration itself stable."""
import numpy as np
import pytest

import workloads as wl
from helpers import Problem, blockerr, dev, entryerr, host, rel
from oracle import assembly, mobility as mob, pfc as opfc, solve as osolve

pytestmark = pytest.mark.gpu
M11 = 1.0 / opfc.ROS3PW_GAMMA


@pytest.fixture(scope="module")
def pfc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06852_amd import pfc as lib
    return lib


def _state(P, seed):
    n = P.n
    rng = np.random.default_rng(seed)
    return np.concatenate([0.3 * rng.normal(size=n), P.psi, 0.3 * rng.normal(size=n)])


@pytest.mark.parametrize("dim,N,jit", [(2, 16, 0.2), (3, 5, 0.2), (2, 40, 0.1)])
def test_pfc1_operator_and_stage_rhs(pfc, dim, N, jit):
    P = Problem(dim, N, jit, amp=0.2, seed=21)
    inst = None
    try:
        n = P.n
        r, tau = -0.35, 0.6
        x = _state(P, 1)
        y = np.random.default_rng(2).normal(size=3 * n)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(model=pfc.PFC_MODEL_PFC1))
        out = dev(np.zeros(3 * n))
        pfc.pfc_apply_AR_x(inst, n, dev(x), r, tau, M11, dev(y), out)
        N_ = assembly.N_matrix(P.mesh, x[n:2 * n])
        Kp = mob.K_plus(P.mesh, x[n:2 * n])
        Fm = mob.F_mu(P.mesh, x[:n])
        ref = mob.apply_AR1(P.M, P.K, N_, Kp, Fm, r, tau, M11, y)
        assert blockerr(host(out), ref) <= 1e-12
        # stage right-hand sides at x_i = x_k + sum a_ij y_j
        ys = np.random.default_rng(3).normal(size=(3, 3 * n)) * 0.1
        for stage in (1, 2, 3):
            b = dev(np.zeros(3 * n))
            pfc.pfc_stage_rhs(inst, n, dev(x), dev(ys.reshape(-1)), stage, r, tau, b)
            xi = x.copy()
            prev, crow = [], []
            for j in range(1, stage):
                xi = xi + opfc.ROS3PW_A[(stage, j)] * ys[j - 1]
                prev.append(ys[j - 1][n:2 * n])
                crow.append(opfc.ROS3PW_C[(stage, j)])
            bref = mob.stage_rhs_R1(P.mesh, P.M, P.K, r, tau, xi, prev, crow)
            assert blockerr(host(b), bref) <= 1e-12, stage
        # the psi-only entry points refuse a PFC1 instance
        with pytest.raises(pfc.PFCError):
            pfc.pfc_apply_AR(inst, n, dev(x[n:2 * n]), r, tau, M11, dev(y), out)
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


@pytest.mark.parametrize("dim,N,jit,tau,km", [(2, 16, 0.2, 0.5, 1), (3, 5, 0.2, 0.5, 1), (2, 72, 0.2, 1.0, 2),
                                              (3, 24, 0.1, 0.5, 2)])
def test_pfc1_solve_replay_and_tolerance(pfc, dim, N, jit, tau, km):
    P = Problem(dim, N, jit, seed=22)
    P.psi = wl.psi_smooth(P.mesh, -0.3, 0.2, kmax=km, seed=22)
    insts = []
    try:
        n = P.n
        r, psibar = -0.35, -0.3
        x0 = opfc.consistent_init(P.mesh, P.M, P.K, r, P.psi)
        b = mob.stage_rhs_R1(P.mesh, P.M, P.K, r, tau, x0, [], [])
        N_ = assembly.N_matrix(P.mesh, P.psi)
        Kp = mob.K_plus(P.mesh, P.psi)
        Fm = mob.F_mu(P.mesh, x0[:n])
        m0 = mob.mobility_mean(P.M, P.psi)
        y_ref, info = osolve.solve_stage(P.M, P.K, N_, r, tau, M11, b, tol=1e-8, Kp=Kp, Fm=Fm, m0=m0)
        s = info["schedule"]
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(model=pfc.PFC_MODEL_PFC1))
        insts.append(inst)
        x = dev(np.zeros(3 * n))
        st, gi = pfc.pfc_solve_x(inst, n, dev(x0), r, psibar, tau, M11, dev(b), x, replay=(s.cycles, s.inner))
        assert gi["outer_iters"] == info["steps"]
        assert entryerr(host(x), y_ref) <= 1e-10
        st, gi = pfc.pfc_solve_x(inst, n, dev(x0), r, psibar, tau, M11, dev(b), x)
        res = np.linalg.norm(b - mob.apply_AR1(P.M, P.K, N_, Kp, Fm, r, tau, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8
        # mixed precision reaches the same tolerance
        im = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(model=pfc.PFC_MODEL_PFC1,
                                                                        precision=pfc.PFC_MIXED))
        insts.append(im)
        st, gi = pfc.pfc_solve_x(im, n, dev(x0), r, psibar, tau, M11, dev(b), x)
        res = np.linalg.norm(b - mob.apply_AR1(P.M, P.K, N_, Kp, Fm, r, tau, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8
        with pytest.raises(pfc.PFCError):
            pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        P.close()


@pytest.mark.parametrize("dim,N,jit,tau", [(2, 16, 0.2, 0.5), (3, 6, 0.1, 0.5)])
def test_pfc1_rosenbrock_replay_parity(pfc, dim, N, jit, tau):
    P = Problem(dim, N, jit, seed=23)
    P.psi = wl.psi_smooth(P.mesh, -0.3, 0.2, kmax=1, seed=23)
    inst = None
    try:
        r, psibar, steps = -0.35, -0.3, 2
        n = P.n
        x0 = opfc.consistent_init(P.mesh, P.M, P.K, r, P.psi)
        x_ref, infos = mob.rosenbrock_run1(P.mesh, P.M, P.K, x0, r, tau, steps, tol=1e-8)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(model=pfc.PFC_MODEL_PFC1))
        state = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        reps = [(i["schedule"].cycles, i["schedule"].inner) for i in infos]
        st, gi = pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau, steps, pfc.PFC_INIT_CONSISTENT, replays=reps)
        assert [g["outer_iters"] for g in gi] == [i["steps"] for i in infos]
        assert entryerr(host(state), x_ref) <= 1e-10
        # tolerance mode stays on the oracle's trajectory and conserves int psi_h
        state2 = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        st2, gi2 = pfc.pfc_rosenbrock_run(inst, n, state2, r, psibar, tau, steps, pfc.PFC_INIT_CONSISTENT)
        s2 = host(state2)
        assert st2 == pfc.PFC_OK and all(g["true_rel_res"] <= 1e-8 for g in gi2)
        assert rel(s2, x_ref) <= 1e-6
        mass = np.sum(P.M @ P.psi)
        assert abs(np.sum(P.M @ s2[n:2 * n]) - mass) <= 1e-6 * max(1.0, abs(mass))
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


def test_pfc1_needs_element_geometry(pfc):
    """A mesh given as CSR matrices carries no element gradients: PFC1 instances are refused."""
    P = Problem(2, 8, 0.1, seed=24)
    h = None
    try:
        n = P.n
        M = P.M.tocsr()
        K = P.K.tocsr()
        h = pfc.pfc_mesh_create_csr(2, n, M.indptr, M.indices, M.data, K.data, P.mesh.elem_nodes,
                                    assembly.element_volumes(P.mesh))
        with pytest.raises(pfc.PFCError):
            pfc.pfc_instance_create(h, pfc.pfc_opts_default(model=pfc.PFC_MODEL_PFC1))
    finally:
        if h is not None:
            pfc.pfc_mesh_destroy(h)
        P.close()
