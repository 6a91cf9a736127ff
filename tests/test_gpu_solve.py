"""Solve-level parity of the HIP path against the oracle (needs a GPU)."""
import numpy as np
import pytest

from helpers import Problem, blockerr, dev, entryerr, host, rel
from oracle import assembly, pfc as opfc, reference, solve as osolve

pytestmark = pytest.mark.gpu
M11 = 1.0 / opfc.ROS3PW_GAMMA


@pytest.fixture(scope="module")
def pfc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06852_amd import pfc as lib
    return lib


def _stage1(P, r, tau):
    x0 = opfc.consistent_init(P.mesh, P.M, P.K, r, P.psi)
    b = opfc.stage_rhs_R(P.mesh, P.M, P.K, r, tau, x0, [], [])
    return x0, b


# the last three cases span several workgroups with a ragged last one; the
# first two are smaller than one 64-row slice.  All are periodic grids, whose
# columns the kernel computes; test_column_forms_agree_bitwise ties the stored
# forms (memory, LDS) to these results bit for bit.
@pytest.mark.parametrize("dim,N,jit,tau,prec", [(2, 3, 0.2, 0.5, 0), (3, 3, 0.2, 0.5, 0),
                                                (2, 16, 0.2, 0.1, 0), (2, 10, 0.0, 1.0, 0), (3, 5, 0.2, 0.5, 0),
                                                (2, 24, 0.2, 1.0, 0), (3, 24, 0.1, 0.5, 0), (2, 72, 0.2, 1.0, 0)])
def test_solve_replay_parity(pfc, dim, N, jit, tau, prec):
    P = Problem(dim, N, jit, seed=7)
    inst = None
    try:
        r, psibar = -0.35, -0.3
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(precision=prec))
        n = P.n
        _, b = _stage1(P, r, tau)
        Nm = assembly.N_matrix(P.mesh, P.psi)
        y_ref, info = osolve.solve_stage(P.M, P.K, Nm, r, tau, M11, b, tol=1e-8)
        s = info["schedule"]
        x = dev(np.zeros(3 * n))
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x, replay=(s.cycles, s.inner))
        assert gi["outer_iters"] == info["steps"]
        assert entryerr(host(x), y_ref) <= 1e-10
        assert st == pfc.PFC_OK
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


@pytest.mark.parametrize("dim,N,jit,tau", [(2, 16, 0.2, 0.1), (2, 24, 0.2, 1.0), (3, 5, 0.2, 0.5)])
def test_single_reduction_pcg_replay_parity(pfc, dim, N, jit, tau):
    """The one-launch-per-iteration PCG form reproduces the oracle's standard PCG under replay."""
    P = Problem(dim, N, jit, seed=17)
    inst = None
    try:
        r, psibar = -0.35, -0.3
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(single_reduction=1))
        n = P.n
        _, b = _stage1(P, r, tau)
        Nm = assembly.N_matrix(P.mesh, P.psi)
        y_ref, info = osolve.solve_stage(P.M, P.K, Nm, r, tau, M11, b, tol=1e-8)
        s = info["schedule"]
        x = dev(np.zeros(3 * n))
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x, replay=(s.cycles, s.inner))
        assert entryerr(host(x), y_ref) <= 1e-10
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, tau, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8
        # the inner counts in tolerance mode match the oracle's up to a threshold crossing
        got = pfc.pfc_last_inner_counts(inst)
        ref = np.array(info["schedule"].inner)
        k = min(len(got), len(ref))
        assert np.abs(got[:k] - ref[:k]).max() <= 1
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


@pytest.mark.parametrize("dim,N,jit,tau,prec", [(2, 16, 0.2, 0.1, 0), (2, 16, 0.2, 1.0, 1), (3, 5, 0.2, 0.5, 0),
                                                (3, 6, 0.0, 0.5, 1), (2, 72, 0.2, 1.0, 1)])
def test_solve_tolerance_mode(pfc, dim, N, jit, tau, prec):
    """True residual <= 1e-8 checked with the oracle's operator; error against a tight oracle solve stated."""
    P = Problem(dim, N, jit, seed=8)
    inst = None
    try:
        r, psibar = -0.35, -0.3
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(precision=prec))
        n = P.n
        _, b = _stage1(P, r, tau)
        Nm = assembly.N_matrix(P.mesh, P.psi)
        x = dev(np.zeros(3 * n))
        import time
        t0 = time.perf_counter()
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
        wall = time.perf_counter() - t0
        y = host(x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, tau, M11, y)) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8, (st, res, gi)
        assert abs(gi["true_rel_res"] - res) <= 1e-3 * res + 1e-15
        # the solve's device time lies within the call's wall time
        assert 0.0 < gi["t_solve"] < wall, (gi["t_solve"], wall)
        y_t, _ = osolve.solve_stage(P.M, P.K, Nm, r, tau, M11, b, tol=1e-13)
        fwd = rel(y, y_t)
        y64, i64 = osolve.solve_stage(P.M, P.K, Nm, r, tau, M11, b, tol=1e-8)
        # same accuracy class as the FP64 oracle at the same tolerance
        assert fwd <= max(1e-6, 50 * rel(y64, y_t)), (fwd, rel(y64, y_t))
        # mixed precision at a tight outer tolerance still reaches the FP64 solution
        opts = pfc.pfc_opts_default(precision=prec, outer_tol=1e-12)
        inst2 = pfc.pfc_instance_create(P.gpu_mesh(), opts)
        try:
            st2, _ = pfc.pfc_solve(inst2, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
            assert rel(host(x), y_t) <= 1e-10 if prec == 0 else rel(host(x), y_t) <= 1e-8
        finally:
            pfc.pfc_instance_destroy(inst2)
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


def test_zero_rhs_and_bad_args(pfc):
    P = Problem(2, 8, 0.0, seed=1)
    inst = None
    try:
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default())
        n = P.n
        x = dev(np.ones(3 * n))
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), -0.3, -0.3, 0.5, M11, dev(np.zeros(3 * n)), x)
        assert st == pfc.PFC_OK and gi["outer_iters"] == 0 and not host(x).any()
        with pytest.raises(pfc.PFCError):
            pfc.pfc_solve(inst, n, dev(P.psi), -0.3, -0.3, -1.0, M11, dev(np.zeros(3 * n)), x)
        # a batch that names one instance twice is refused before anything runs
        s0 = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        with pytest.raises(pfc.PFCError) as e:
            pfc.pfc_batch_run([inst, inst], [n, n], [s0, dev(host(s0))], [-0.3] * 2, [-0.3] * 2, [0.5] * 2, 1)
        assert e.value.code == pfc.PFC_ERR_ARG and "distinct" in pfc.pfc_last_error()
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


def test_fft_exact_agreement(pfc):
    """Unjittered mesh, constant psi: the tight GPU solve equals the exact Fourier solution."""
    P = Problem(2, 48, 0.0, amp=0.0, psibar=-0.3, seed=2)
    inst = None
    try:
        r, tau = -0.35, 1.0
        n = P.n
        b = np.random.default_rng(4).normal(size=3 * n)
        yf = reference.fft_exact(P.mesh, P.M, P.K, r, tau, M11, -0.3, b)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(outer_tol=1e-12))
        x = dev(np.zeros(3 * n))
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, -0.3, tau, M11, dev(b), x)
        assert entryerr(host(x), yf) <= 1e-10, gi
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


@pytest.mark.parametrize("dim,N,jit,tau", [(2, 12, 0.2, 0.5), (3, 4, 0.1, 0.5)])
def test_rosenbrock_run_replay_parity(pfc, dim, N, jit, tau):
    P = Problem(dim, N, jit, amp=0.05, seed=9)
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
        # tolerance mode: conservation of int psi_h and closeness to the oracle trajectory
        state2 = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        st2, gi2 = pfc.pfc_rosenbrock_run(inst, n, state2, r, psibar, tau, steps, pfc.PFC_INIT_CONSISTENT)
        s2 = host(state2)
        assert st2 == pfc.PFC_OK and all(g["true_rel_res"] <= 1e-8 for g in gi2)
        # int psi_h changes per stage by gamma * 1^T r_1 <= gamma sqrt(n) ||r|| (residual of block row 1)
        m0 = np.sum(P.M @ P.psi)
        bnd = sum(abs(m) for m in opfc.ROS3PW_M) * steps * opfc.ROS3PW_GAMMA * np.sqrt(n) * 1e-8
        bmax = max(np.linalg.norm(opfc.stage_rhs_R(P.mesh, P.M, P.K, r, tau, x0, [], [])), 1.0)
        assert abs(np.sum(P.M @ s2[n:2 * n]) - m0) <= 10 * bnd * bmax
        assert rel(s2, x_ref) <= 1e-6
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


def test_adaptive_rosenbrock_matches_oracle(pfc):
    """Embedded error estimate and step-size control: same accepted steps and end state as the oracle."""
    from oracle import adaptive
    from oracle.reference import dense_solve
    P = Problem(2, 8, 0.15, amp=0.3, psibar=-0.2, seed=31, h=2.0)
    inst = None
    try:
        r, T, rtol = -0.35, 3.0, 1e-4
        n = P.n
        x0 = opfc.consistent_init(P.mesh, P.M, P.K, r, P.psi)
        prob = opfc.PFCProblem(P.mesh, P.M, P.K, r)

        def lin(N_, tau_, bR, i):
            return dense_solve(opfc.AR_sparse(P.M, P.K, N_, r, tau_, M11), bR)

        xr, taus_r, rej_r = adaptive.rosenbrock_adaptive(prob, x0, 0.5, T, rtol, rtol, lin)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(outer_tol=1e-12))
        state = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        st, taus, rej, infos = pfc.pfc_rosenbrock_adaptive(inst, n, state, r, -0.2, 0.5, T, rtol, rtol)
        assert len(infos) == 3 * (len(taus) + rej) and all(i["true_rel_res"] <= 1e-12 for i in infos)
        assert st >= 0
        assert len(taus) == len(taus_r) and rej == rej_r
        assert np.abs(np.array(taus) - np.array(taus_r)).max() <= 1e-8 * max(taus_r)
        assert abs(sum(taus) - T) <= 1e-12
        assert rel(host(state), xr) <= 1e-8
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


def test_adaptive_rejects_steps_whose_solves_fail(pfc):
    """A stage solve that stops at max_steps rejects the step (tau * 0.2), and the step after a rejection does
    not grow: same accepted steps, rejections and end state as the oracle's controller with the same capped
    FGMRES.  Fixed inner counts make the outer iteration counts a property of the method on both sides; the
    oracle run checks that every count is at least one step from the cap."""
    from oracle import adaptive
    P = Problem(2, 8, 0.15, amp=0.3, psibar=-0.2, seed=31, h=2.0)
    inst = None
    try:
        r, T, rtol, cap, fixed = -0.35, 5.0, 1e-4, 34, [2] * 5
        n = P.n
        x0 = opfc.consistent_init(P.mesh, P.M, P.K, r, P.psi)
        prob = opfc.PFCProblem(P.mesh, P.M, P.K, r)
        kw = dict(tol=1e-8, inner_fixed=fixed)

        def lin(N_, tau_, bR, i):
            y, info = osolve.solve_stage(P.M, P.K, N_, r, tau_, M11, bR, max_steps=cap, **kw)
            if not info["converged"]:
                assert not osolve.solve_stage(P.M, P.K, N_, r, tau_, M11, bR, max_steps=cap + 1, **kw)[1]["converged"]
                raise adaptive.LinearSolveFailed()
            assert info["steps"] <= cap - 1
            return y

        log = []
        xr, taus_r, rej_r = adaptive.rosenbrock_adaptive(prob, x0, 0.5, T, rtol, rtol, lin, log=log)
        n_failed = sum(k == "failed" for _, k in log)
        assert n_failed >= 2 and any(k == "rejected" for _, k in log)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(max_steps=cap, inner_fixed=fixed))
        state = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        st, taus, rej, infos = pfc.pfc_rosenbrock_adaptive(inst, n, state, r, -0.2, 0.5, T, rtol, rtol)
        assert st >= 0
        assert len(taus) == len(taus_r) and rej == rej_r
        assert np.abs(np.array(taus) - np.array(taus_r)).max() <= 1e-8 * max(taus_r)
        assert rel(host(state), xr) <= 1e-8
        # three records per attempt; the attempts the oracle saw fail hold a stage that stopped at the cap
        assert len(infos) == 3 * len(log)
        for a, (_, kind) in enumerate(log):
            att = infos[3 * a:3 * a + 3]
            failed = [i["status"] == pfc.PFC_NOT_CONVERGED for i in att]
            assert any(failed) == (kind == "failed"), (a, kind, att)
            if kind == "failed":
                assert att[failed.index(True)]["outer_iters"] == cap
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


def test_extreme_parameters_and_status_codes(pfc):
    """tau beyond tau* (warning status), tiny tau, short restart, and the Arnoldi-step cap."""
    P = Problem(2, 16, 0.2, seed=41)
    insts = []
    try:
        n = P.n
        r, psibar = -0.35, -0.3
        b = np.random.default_rng(8).normal(size=3 * n)
        Nm = assembly.N_matrix(P.mesh, P.psi)
        x = dev(np.zeros(3 * n))
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default())
        insts.append(inst)
        # the paper accepts steps up to 18 with this preconditioner (Section 7); tau* = 12.26 here
        tau = 18.0
        assert tau >= pfc.pfc_tau_critical(r, psibar)
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, tau, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_WARN_TAU_CRITICAL and res <= 1e-8
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, 1e-5, M11, dev(b), x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, 1e-5, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8
        # restart 3: more cycles, same accuracy
        i3 = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(restart=3))
        insts.append(i3)
        st, gi = pfc.pfc_solve(i3, n, dev(P.psi), r, psibar, 1.0, M11, dev(b), x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, 1.0, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8 and gi["cycles"] > 1
        # cap of 4 Arnoldi steps: not converged, info still valid
        i4 = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(max_steps=4))
        insts.append(i4)
        st, gi = pfc.pfc_solve(i4, n, dev(P.psi), r, psibar, 1.0, M11, dev(b), x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, 1.0, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_NOT_CONVERGED and gi["outer_iters"] == 4 and abs(gi["true_rel_res"] - res) <= 1e-6 * res
        # a non-finite right-hand side is a breakdown
        bad = b.copy()
        bad[3] = np.nan
        with pytest.raises(pfc.PFCError) as e:
            pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, 1.0, M11, dev(bad), x)
        assert e.value.code == pfc.PFC_ERR_BREAKDOWN
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        P.close()


@pytest.mark.parametrize("dim,N,jit,tau,prec", [(2, 16, 0.2, 0.1, 0), (3, 5, 0.1, 0.5, 0), (2, 16, 0.2, 0.5, 1)])
def test_schur_D_variant_parity(pfc, dim, N, jit, tau, prec):
    """P(S_D) with the fixed 20-iteration inner PCG (Table inner_solvers, last row)."""
    P = Problem(dim, N, jit, seed=51)
    inst = None
    try:
        r, psibar = -0.35, -0.3
        n = P.n
        _, b = _stage1(P, r, tau)
        Nm = assembly.N_matrix(P.mesh, P.psi)
        y_ref, info = osolve.solve_stage(P.M, P.K, Nm, r, tau, M11, b, tol=1e-8, schur="D")
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(schur_variant=1, precision=prec))
        x = dev(np.zeros(3 * n))
        if prec == 0:
            s = info["schedule"]
            st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x, replay=(s.cycles, s.inner))
            assert entryerr(host(x), y_ref) <= 1e-10
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, tau, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8
        got = pfc.pfc_last_inner_counts(inst)
        assert (got[:, 2] == 20).all() and (got[:, 3] == 0).all()
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


# 2D float64 reads the columns from memory, 3D float64 and mixed runs stage them in
# LDS; the 3D 24^3 cases span several workgroups with a ragged last one; with 4
# rows per thread every form reads the stored columns from memory
@pytest.mark.parametrize("dim,N,jit,prec,rpt", [(2, 16, 0.2, 0, 1), (3, 5, 0.2, 0, 1), (3, 6, 0.1, 1, 1),
                                                (2, 24, 0.2, 1, 1), (3, 24, 0.1, 0, 1), (2, 40, 0.2, 1, 4),
                                                (3, 24, 0.1, 0, 4)])
def test_column_forms_agree_bitwise(pfc, dim, N, jit, prec, rpt):
    """On periodic grids the kernel computes the columns (grid_columns = 1): the same columns in the
    same order as the stored ones, so a stage solve and a Rosenbrock step give the same bits (one PCG
    iteration per launch in both; the two-iteration form is compared in its own test)."""
    P = Problem(dim, N, jit, seed=61)
    insts = []
    try:
        r, psibar, tau = -0.35, -0.3, 0.5
        n = P.n
        _, b = _stage1(P, r, tau)
        assert pfc.pfc_mesh_grid_side(P.gpu_mesh()) == N
        out = []
        for g in (1, 0):
            inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(precision=prec, grid_columns=g,
                                                                              rows_per_thread=rpt,
                                                                              pcg_steps_per_launch=1))
            insts.append(inst)
            x = dev(np.zeros(3 * n))
            st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
            assert st == pfc.PFC_OK
            s = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
            st, _ = pfc.pfc_rosenbrock_run(inst, n, s, r, psibar, tau, 1, pfc.PFC_INIT_CONSISTENT)
            assert st == pfc.PFC_OK
            out.append((host(x), host(s), gi["outer_iters"]))
        assert out[0][2] == out[1][2]
        assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        P.close()


@pytest.mark.parametrize("dim,N,jit,tau", [(2, 16, 0.2, 0.8), (3, 5, 0.2, 0.5)])
def test_gamma_literal_and_fixed_inner_counts(pfc, dim, N, jit, tau):
    """The literal reading of Section 4 (P_CH(tau) on the unscaled system) and fixed inner iteration
    counts, each against the oracle run the same way."""
    P = Problem(dim, N, jit, seed=71)
    insts = []
    try:
        r, psibar = -0.35, -0.3
        n = P.n
        _, b = _stage1(P, r, tau)
        Nm = assembly.N_matrix(P.mesh, P.psi)
        x = dev(np.zeros(3 * n))
        # literal reading: replay parity, then tolerance mode
        y_ref, info = osolve.solve_stage(P.M, P.K, Nm, r, tau, M11, b, tol=1e-8, gamma_mode="literal")
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(gamma_mode=pfc.PFC_GAMMA_LITERAL))
        insts.append(inst)
        s = info["schedule"]
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x, replay=(s.cycles, s.inner))
        assert gi["outer_iters"] == info["steps"] and entryerr(host(x), y_ref) <= 1e-10
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, tau, M11, host(x))) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8
        # fixed inner counts: every application runs exactly these counts, same iterates as the oracle
        fc = [4, 6, 5, 5, 4]
        y_f, info_f = osolve.solve_stage(P.M, P.K, Nm, r, tau, M11, b, tol=1e-8, inner_fixed=fc)
        inst2 = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(inner_fixed=fc))
        insts.append(inst2)
        st, gi = pfc.pfc_solve(inst2, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
        got = pfc.pfc_last_inner_counts(inst2)
        assert (got == np.array(fc)).all()
        assert gi["outer_iters"] == info_f["steps"] and entryerr(host(x), y_f) <= 1e-10
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        P.close()


# 2D float64 periodic grids: one workgroup smaller than a slice (3^2), one workgroup (16^2, 24^2), several
# workgroups with a ragged last one (72^2: six workgroups of 896 rows, the last 704), and the halo of
# N + 1 rows wrapping round the grid in every case (ranges of rows); sides that are multiples of 64 take
# blocks of 64 x 16 rows whose frames wrap round the grid in both directions (64^2: one block column of
# four blocks; 128^2: 2 x 8 blocks)
@pytest.mark.parametrize("N,jit,tau", [(3, 0.2, 0.5), (16, 0.2, 0.1), (24, 0.2, 1.0), (72, 0.2, 1.0),
                                       (64, 0.2, 1.0), (128, 0.2, 0.5)])
def test_two_pcg_iterations_per_launch(pfc, N, jit, tau):
    """The s-step form (two PCG iterations per launch) against one iteration per launch and the oracle:
    the same inner iteration counts and Arnoldi steps, the same solution to rounding, odd fixed counts
    (a launch that ends after the first of its two iterations), and fewer launches."""
    P = Problem(2, N, jit, seed=71)
    insts = []
    try:
        r, psibar = -0.35, -0.3
        n = P.n
        _, b = _stage1(P, r, tau)
        res = []
        for spl in (2, 1):
            inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(pcg_steps_per_launch=spl))
            insts.append(inst)
            x = dev(np.zeros(3 * n))
            st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
            assert st == pfc.PFC_OK
            counts = pfc.pfc_last_inner_counts(inst)
            launches, _ = pfc.pfc_instance_launch_stats(inst)
            res.append((host(x), gi, counts, launches))
        (x2, g2, c2, l2), (x1, g1, c1, l1) = res
        assert g2["outer_iters"] == g1["outer_iters"] and np.array_equal(c2, c1)
        assert rel(x2, x1) <= 1e-10 and g2["true_rel_res"] <= 1e-8
        if g1["inner_total"] >= 200:
            assert l2 < 0.8 * l1, (l2, l1)
        # against the oracle under replay of its schedule
        Nm = assembly.N_matrix(P.mesh, P.psi)
        y_ref, info = osolve.solve_stage(P.M, P.K, Nm, r, tau, M11, b, tol=1e-8)
        s = info["schedule"]
        x = dev(np.zeros(3 * n))
        st, gi = pfc.pfc_solve(insts[0], n, dev(P.psi), r, psibar, tau, M11, dev(b), x, replay=(s.cycles, s.inner))
        assert gi["outer_iters"] == info["steps"] and entryerr(host(x), y_ref) <= 1e-10
        # odd and even fixed counts, including 1
        fixed = [3, 1, 4, 5, 2]
        y_fix, info_f = osolve.solve_stage(P.M, P.K, Nm, r, tau, M11, b, tol=1e-8, inner_fixed=fixed, max_steps=6)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(inner_fixed=fixed, max_steps=6))
        insts.append(inst)
        x = dev(np.zeros(3 * n))
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
        assert gi["outer_iters"] == info_f["steps"] and entryerr(host(x), y_fix) <= 1e-10
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        P.close()


@pytest.mark.parametrize("N", [64, 128])
def test_two_pcg_iterations_per_launch_2d_blocks_mixed(pfc, N):
    """Mixed precision (float32 inner PCG) on 2D grids of side a multiple of 64 runs two PCG iterations per
    launch on blocks of 64 x 16 rows.  With the oracle's inner counts fixed, odd ones included, one P_CH
    apply in that form reaches the oracle's float64 apply as closely as the one-iteration float32 form
    (both differ from it by float32 rounding of the inner solves), with fewer launches; a tolerance-mode
    stage solve reaches the true residual of the tolerance (the oracle's operator) with the same outer
    iteration count as the one-iteration form."""
    from oracle import precond
    P = Problem(2, N, 0.2, seed=13)
    n = P.n
    tau, r, psibar = 0.5, -0.35, -0.3
    tau_s = tau / M11
    w = np.random.default_rng(5).normal(size=3 * n)
    insts = []
    out = {}
    try:
        _, b = _stage1(P, r, tau)
        Nm = assembly.N_matrix(P.mesh, P.psi)
        for spl in (2, 1):
            inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(precision=1, pcg_steps_per_launch=spl))
            insts.append(inst)
            assert pfc.pfc_instance_config(inst)["pcg_steps_per_launch"] == spl
            for fixed in ([3, 1, 4, 5, 2], [25, 21, 17, 23, 19]):
                ref = precond.pch_apply(precond.InnerSolvers(P.M, P.K, tau_s, mode="pcg", fixed_counts=fixed), w)
                z = dev(np.zeros(3 * n))
                got = pfc.pfc_apply_pch(inst, n, tau_s, dev(w), z, fixed_counts=fixed)
                assert list(got) == list(fixed)
                out[(spl, tuple(fixed))] = (rel(host(z), ref), pfc.pfc_instance_launch_stats(inst)[0])
            x = dev(np.zeros(3 * n))
            st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
            res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, tau, M11, host(x))) / np.linalg.norm(b)
            assert st == pfc.PFC_OK and res <= 1e-8, (spl, st, res)
            out[(spl, "solve")] = gi["outer_iters"]
        for fixed in ([3, 1, 4, 5, 2], [25, 21, 17, 23, 19]):
            (e2, l2), (e1, l1) = out[(2, tuple(fixed))], out[(1, tuple(fixed))]
            assert e2 <= max(1e-5, 3.0 * e1), (fixed, e2, e1)
            if sum(fixed) >= 20:
                assert l2 < 0.8 * l1, (l2, l1)
        assert out[(2, "solve")] == out[(1, "solve")]
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        P.close()


def test_two_pcg_iterations_per_launch_large_team(pfc):
    """A 2D 600^2 grid: a team of 352 workgroups (Gram partials beyond the first 256 per thread group are
    summed by the remainder loop) and a halo of 601 rows.  Both forms (two PCG iterations per launch and
    one) replay the oracle's iteration record and reach its solution element by element; in tolerance
    mode they take the same counts and reach the true residual of the tolerance, the two-iteration form
    with fewer launches."""
    import workloads as wl
    mesh = wl.make_mesh(2, 600, jitter=0.2, seed=5)
    n = mesh.n
    h = pfc.pfc_mesh_create_p1(2, n, mesh.elem_nodes, mesh.elem_coords)
    insts = []
    try:
        assert pfc.pfc_mesh_grid_side(h) == 600
        r, psibar, tau = -0.35, -0.3, 1.0
        psi = wl.psi0(n, psibar, 0.01, seed=5)
        b = np.random.default_rng(9).normal(size=3 * n)
        M, K = assembly.mass_stiffness(mesh)
        Nm = assembly.N_matrix(mesh, psi)
        print("600^2: oracle stage solve", flush=True)
        y_ref, info = osolve.solve_stage(M, K, Nm, r, tau, M11, b, tol=1e-8)
        sch = info["schedule"]
        out = []
        for spl in (2, 1):
            inst = pfc.pfc_instance_create(h, pfc.pfc_opts_default(pcg_steps_per_launch=spl))
            insts.append(inst)
            assert pfc.pfc_instance_config(inst)["pcg_steps_per_launch"] == spl
            x = dev(np.zeros(3 * n))
            print(f"600^2: {spl} PCG iteration(s) per launch, replay", flush=True)
            st, gi = pfc.pfc_solve(inst, n, dev(psi), r, psibar, tau, M11, dev(b), x, replay=(sch.cycles, sch.inner))
            assert gi["outer_iters"] == info["steps"] and entryerr(host(x), y_ref) <= 1e-10, spl
            x = dev(np.zeros(3 * n))
            st, gi = pfc.pfc_solve(inst, n, dev(psi), r, psibar, tau, M11, dev(b), x)
            assert st == pfc.PFC_OK and gi["true_rel_res"] <= 1e-8
            out.append((host(x), gi, pfc.pfc_last_inner_counts(inst), pfc.pfc_instance_launch_stats(inst)[0]))
        (x2, g2, c2, l2), (x1, g1, c1, l1) = out
        assert g2["outer_iters"] == g1["outer_iters"] and np.array_equal(c2, c1)
        assert l2 < 0.8 * l1, (l2, l1)
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        pfc.pfc_mesh_destroy(h)
