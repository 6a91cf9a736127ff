"""Full-size workloads in the launch configuration the benchmark times (needs a GPU).

At these sizes the oracle's full solves take tens of seconds, so each case
checks what the oracle can compute cheaply or what holds at any size:
* the true relative residual of a GPU stage solve, from the oracle's own
  matrices and SpMV (Section 3: A^R y = b^R to 1e-8);
* one P_CH apply with the oracle's inner iteration counts, element by element
  (Section 4.2, steps (1)-(5); S_D variant: Section 4.1);
* a Rosenbrock step through the benchmark's entry point: every stage solve
  converged, and int psi_h conserved (Section 2: the psi equation is in
  divergence form, so 1^T M psi changes only by the solve residuals);
* for the batched workload, replay parity of sampled instances against the
  oracle's whole Rosenbrock step, and bitwise equality of an instance run alone
  and inside the batch.
"""
import numpy as np
import pytest

import workloads as wl
from helpers import Problem, blockerr, dev, entryerr, host, rel
from oracle import assembly, mobility as mob, pfc as opfc, precond, solve as osolve

pytestmark = pytest.mark.gpu
M11 = 1.0 / opfc.ROS3PW_GAMMA


@pytest.fixture(scope="module")
def pfc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06852_amd import pfc as lib
    return lib


def _mass_bound(P, r, tau, x0, steps):
    """Largest change of 1^T M psi that stage solves at relative residual 1e-8 allow: per stage
    gamma 1^T r_1 <= gamma sqrt(n) ||r||, weighted by the step weights m_j."""
    bnd = sum(abs(m) for m in opfc.ROS3PW_M) * steps * opfc.ROS3PW_GAMMA * np.sqrt(P.n) * 1e-8
    bmax = max(np.linalg.norm(opfc.stage_rhs_R(P.mesh, P.M, P.K, r, tau, x0, [], [])), 1.0)
    return 10 * bnd * bmax


# the benchmark's variant workloads: 2D, jitter 0.2, r = -0.35, psibar = -0.3, tau = 1, seed 0
VARIANTS = {
    "p2_256": dict(N=256, degree=2, opts={}),
    "pfc1_512": dict(N=512, degree=1, opts={"model": 1}, smooth=(0.2, 16)),
    "sd_512": dict(N=512, degree=1, opts={"schur_variant": 1}),
}


@pytest.mark.parametrize("name", sorted(VARIANTS))
def test_full_size_variant(pfc, name):
    v = VARIANTS[name]
    r, psibar, tau = -0.35, -0.3, 1.0
    P = Problem(2, v["N"], 0.2, psibar=psibar, seed=0, degree=v["degree"])
    pfc1 = v["opts"].get("model", 0) == 1
    sd = v["opts"].get("schur_variant", 0) == 1
    if "smooth" in v:
        P.psi = wl.psi_smooth(P.mesh, psibar, v["smooth"][0], kmax=v["smooth"][1], seed=0)
    inst = None
    try:
        n = P.n
        print(f"full-size {name}: n = {n}", flush=True)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(**v["opts"]))
        x0 = opfc.consistent_init(P.mesh, P.M, P.K, r, P.psi)
        Nm = assembly.N_matrix(P.mesh, P.psi)
        x = dev(np.zeros(3 * n))
        if pfc1:
            b = mob.stage_rhs_R1(P.mesh, P.M, P.K, r, tau, x0, [], [])
            st, gi = pfc.pfc_solve_x(inst, n, dev(x0), r, psibar, tau, M11, dev(b), x)
            Kp = mob.K_plus(P.mesh, P.psi)
            Fm = mob.F_mu(P.mesh, x0[:n])
            Ay = mob.apply_AR1(P.M, P.K, Nm, Kp, Fm, r, tau, M11, host(x))
        else:
            b = opfc.stage_rhs_R(P.mesh, P.M, P.K, r, tau, x0, [], [])
            st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, M11, dev(b), x)
            Ay = opfc.apply_AR(P.M, P.K, Nm, r, tau, M11, host(x))
        res = np.linalg.norm(b - Ay) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8, (st, res, gi)
        assert abs(gi["true_rel_res"] - res) <= 1e-3 * res + 1e-14
        if not pfc1:
            # one preconditioner apply at the solver's own time step, with the oracle's inner counts
            tau_s = tau / M11
            w = np.random.default_rng(2).normal(size=3 * n)
            inner = precond.InnerSolvers(P.M, P.K, tau_s, mode="pcg", tol=1e-3, schur="D" if sd else "CH")
            z_ref = precond.pch_apply(inner, w)
            z = dev(np.zeros(3 * n))
            got = pfc.pfc_apply_pch(inst, n, tau_s, dev(w), z, fixed_counts=inner.counts[0])
            assert list(got) == list(inner.counts[0])
            assert blockerr(host(z), z_ref) <= 1e-12
        # the benchmark's entry point: one Rosenbrock step from consistent initial values
        state = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        st, gis = pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau, 1, pfc.PFC_INIT_CONSISTENT)
        s = host(state)
        assert st == pfc.PFC_OK and max(g["true_rel_res"] for g in gis) <= 1e-8
        assert np.isfinite(s).all()
        m0 = np.sum(P.M @ P.psi)
        assert abs(np.sum(P.M @ s[n:2 * n]) - m0) <= _mass_bound(P, r, tau, x0, 1)
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


def test_full_size_batched_128_mixed(pfc):
    """256 instances of 2D 128^2 on one mesh, mixed precision, 4 rows per thread, shared operators."""
    import torch
    count, N, rpt = 256, 128, 4
    P = Problem(2, N, 0.0, seed=0)
    n = P.n
    prm = wl.draw_params(count, 7000)
    dv = torch.device("cuda:0")

    def state_of(p):
        s = torch.zeros(3 * n, dtype=torch.float64, device=dv)
        s[n:2 * n] = torch.tensor(wl.psi0(n, p.psibar, 0.01, seed=p.seed), dtype=torch.float64, device=dv)
        return s

    insts = []
    try:
        h = P.gpu_mesh()
        opts = dict(precision=1, shared_ops=1, rows_per_thread=rpt)
        insts = [pfc.pfc_instance_create(h, pfc.pfc_opts_default(**opts)) for _ in range(count)]
        st = [state_of(p) for p in prm]
        args = ([p.r for p in prm], [p.psibar for p in prm], [p.tau for p in prm])
        print("batched: consistent initial values", flush=True)
        pfc.pfc_batch_run(insts, [n] * count, st, *args, 0, pfc.PFC_INIT_CONSISTENT)
        print("batched: one step", flush=True)
        code, infos = pfc.pfc_batch_run(insts, [n] * count, st, *args, 1, pfc.PFC_INIT_GIVEN)
        assert code == pfc.PFC_OK
        assert max(i["true_rel_res"] for row in infos for i in row) <= 1e-8
        # an instance alone gives the bits it has inside the batch
        alone = pfc.pfc_instance_create(h, pfc.pfc_opts_default(**opts))
        insts.append(alone)
        p = prm[0]
        s_alone = state_of(p)
        pfc.pfc_rosenbrock_run(alone, n, s_alone, p.r, p.psibar, p.tau, 0, pfc.PFC_INIT_CONSISTENT)
        pfc.pfc_rosenbrock_run(alone, n, s_alone, p.r, p.psibar, p.tau, 1, pfc.PFC_INIT_GIVEN)
        assert np.array_equal(host(s_alone), host(st[0]))
        # sampled instances against the oracle's Rosenbrock step: the float64 solver in the same
        # launch layout replays the oracle's iteration counts; the batched mixed result is as close
        # as two solves at relative residual 1e-8 can be
        rep = pfc.pfc_instance_create(h, pfc.pfc_opts_default(precision=0, shared_ops=1, rows_per_thread=rpt))
        insts.append(rep)
        for k in (0, 201):
            p = prm[k]
            psi = wl.psi0(n, p.psibar, 0.01, seed=p.seed)
            x0 = opfc.consistent_init(P.mesh, P.M, P.K, p.r, psi)
            x_ref, oinf = osolve.rosenbrock_run(P.mesh, P.M, P.K, x0, p.r, p.tau, 1, tol=1e-8)
            s_rep = state_of(p)
            reps = [(i["schedule"].cycles, i["schedule"].inner) for i in oinf]
            _, gi = pfc.pfc_rosenbrock_run(rep, n, s_rep, p.r, p.psibar, p.tau, 1, pfc.PFC_INIT_CONSISTENT,
                                           replays=reps)
            assert [g["outer_iters"] for g in gi] == [i["steps"] for i in oinf]
            assert entryerr(host(s_rep), x_ref) <= 1e-10, k
            sb = host(st[k])
            assert rel(sb, x_ref) <= 1e-6, k
            m0 = np.sum(P.M @ psi)
            assert abs(np.sum(P.M @ sb[n:2 * n]) - m0) <= _mass_bound(P, p.r, p.tau, x0, 1), k
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        P.close()
