"""The 3D 64^3 mixed-precision workload at full size, against the oracle (needs a GPU).

Workload: periodic 64^3 Kuhn mesh (262,144 nodes, 786,432 unknowns), r = -0.3,
psibar = -0.25, psi_0 = psibar + U[-0.01, 0.01] (seed 0), tau = 0.5, Ros3Pw
stages (m11 = 1/gamma, Table rosenbrock_scheme).  The oracle's matrices, its
consistent initial values and its stage right-hand side define the system
(Section 3.1, eq. rosenbrock_matrix); the oracle solves it to 1e-8 (its
iteration record drives the replays) and to 1e-13 (the reference solution).

* float64 replay: the GPU runs the oracle's cycle lengths and inner counts of
  one stage solve, and of a whole Rosenbrock step, and reaches the oracle's
  iterate element by element within 1e-10 of its largest entry;
* mixed precision (float32 inner PCG, float64 FGMRES; the benchmark's
  instance options) in tolerance mode: the true residual, computed with the
  oracle's own operator, is at most 1e-8, and the forward error against the
  1e-13 reference is at most max(1e-8, 2x the float64 GPU solve's);
* a mixed Rosenbrock step lands within 1e-6 of the oracle's float64 step (two
  runs whose stage solves stop at relative residual 1e-8) and conserves the
  integral of psi to the bound the solve residuals allow.
"""
import numpy as np
import pytest

import workloads as wl
from helpers import Problem, blockerr, dev, entryerr, host, rel
from oracle import assembly, pfc as opfc, solve as osolve

pytestmark = pytest.mark.gpu
M11 = 1.0 / opfc.ROS3PW_GAMMA
R, PSIBAR, TAU = -0.3, -0.25, 0.5


@pytest.fixture(scope="module")
def pfc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06852_amd import pfc as lib
    return lib


@pytest.fixture(scope="module")
def c3(pfc):
    """The oracle's side of the 3D 64^3 stage system (computed once for the module)."""
    print("3D 64^3: oracle matrices, consistent initial values, stage 1 system", flush=True)
    P = Problem(3, 64, 0.0, psibar=PSIBAR, amp=0.01, seed=0)
    x0 = opfc.consistent_init(P.mesh, P.M, P.K, R, P.psi)
    Nm = assembly.N_matrix(P.mesh, P.psi)
    b = opfc.stage_rhs_R(P.mesh, P.M, P.K, R, TAU, x0, [], [])
    print("3D 64^3: oracle stage solve to 1e-8", flush=True)
    y8, info8 = osolve.solve_stage(P.M, P.K, Nm, R, TAU, M11, b, tol=1e-8)
    print("3D 64^3: oracle stage solve to 1e-13", flush=True)
    y13, _ = osolve.solve_stage(P.M, P.K, Nm, R, TAU, M11, b, tol=1e-13)
    yield dict(P=P, x0=x0, Nm=Nm, b=b, y8=y8, info8=info8, y13=y13)
    P.close()


def _residual(c, y):
    P = c["P"]
    return np.linalg.norm(c["b"] - opfc.apply_AR(P.M, P.K, c["Nm"], R, TAU, M11, y)) / np.linalg.norm(c["b"])


def test_c3_stage_solve_fp64_replay_and_mixed_tolerance(pfc, c3):
    P = c3["P"]
    n = P.n
    insts = []
    try:
        mesh = P.gpu_mesh()
        # float64 replay of the oracle's iteration structure
        i64 = pfc.pfc_instance_create(mesh, pfc.pfc_opts_default(precision=0))
        insts.append(i64)
        s = c3["info8"]["schedule"]
        x = dev(np.zeros(3 * n))
        print("3D 64^3: float64 replay", flush=True)
        st, gi = pfc.pfc_solve(i64, n, dev(P.psi), R, PSIBAR, TAU, M11, dev(c3["b"]), x, replay=(s.cycles, s.inner))
        assert gi["outer_iters"] == c3["info8"]["steps"]
        assert entryerr(host(x), c3["y8"]) <= 1e-10
        # float64 in tolerance mode: its forward error sets the accuracy class
        print("3D 64^3: float64 and mixed tolerance-mode solves", flush=True)
        st, gi = pfc.pfc_solve(i64, n, dev(P.psi), R, PSIBAR, TAU, M11, dev(c3["b"]), x)
        y64 = host(x)
        res64 = _residual(c3, y64)
        assert st == pfc.PFC_OK and res64 <= 1e-8, (st, res64)
        fwd64 = rel(y64, c3["y13"])
        # the benchmark's mixed-precision instance
        imp = pfc.pfc_instance_create(mesh, pfc.pfc_opts_default(precision=1))
        insts.append(imp)
        assert pfc.pfc_instance_config(imp)["pcg_steps_per_launch"] == 2   # blocks of the grid
        st, gi = pfc.pfc_solve(imp, n, dev(P.psi), R, PSIBAR, TAU, M11, dev(c3["b"]), x)
        ymp = host(x)
        resmp = _residual(c3, ymp)
        assert st == pfc.PFC_OK and resmp <= 1e-8, (st, resmp, gi)
        assert abs(gi["true_rel_res"] - resmp) <= 1e-3 * resmp + 1e-15
        fwdmp = rel(ymp, c3["y13"])
        print(f"3D 64^3: residual fp64 {res64:.2e} mixed {resmp:.2e}; forward error fp64 {fwd64:.2e} "
              f"mixed {fwdmp:.2e}", flush=True)
        assert fwdmp <= max(1e-8, 2.0 * fwd64), (fwdmp, fwd64)
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)


def test_c3_rosenbrock_step_fp64_replay_and_mixed(pfc, c3):
    P = c3["P"]
    n = P.n
    print("3D 64^3: oracle Rosenbrock step", flush=True)
    x_ref, oinf = osolve.rosenbrock_run(P.mesh, P.M, P.K, c3["x0"], R, TAU, 1, tol=1e-8)
    reps = [(i["schedule"].cycles, i["schedule"].inner) for i in oinf]
    s0 = np.concatenate([np.zeros(n), P.psi, np.zeros(n)])
    insts = []
    try:
        mesh = P.gpu_mesh()
        i64 = pfc.pfc_instance_create(mesh, pfc.pfc_opts_default(precision=0))
        insts.append(i64)
        state = dev(s0)
        print("3D 64^3: float64 Rosenbrock step, replayed", flush=True)
        st, gis = pfc.pfc_rosenbrock_run(i64, n, state, R, PSIBAR, TAU, 1, pfc.PFC_INIT_CONSISTENT, replays=reps)
        assert [g["outer_iters"] for g in gis] == [i["steps"] for i in oinf]
        assert entryerr(host(state), x_ref) <= 1e-10
        # the benchmark's mixed instance, tolerance mode
        imp = pfc.pfc_instance_create(mesh, pfc.pfc_opts_default(precision=1))
        insts.append(imp)
        state = dev(s0)
        print("3D 64^3: mixed Rosenbrock step", flush=True)
        st, gis = pfc.pfc_rosenbrock_run(imp, n, state, R, PSIBAR, TAU, 1, pfc.PFC_INIT_CONSISTENT)
        s = host(state)
        assert st == pfc.PFC_OK and max(g["true_rel_res"] for g in gis) <= 1e-8
        err = rel(s, x_ref)
        print(f"3D 64^3: mixed step against the oracle's float64 step {err:.2e}", flush=True)
        assert err <= 1e-6
        # conservation of int psi_h: per stage the solve residual moves 1^T M psi by at most
        # gamma sqrt(n) ||r||, weighted by the step weights m_j
        bnd = sum(abs(m) for m in opfc.ROS3PW_M) * opfc.ROS3PW_GAMMA * np.sqrt(n) * 1e-8
        bmax = max(np.linalg.norm(c3["b"]), 1.0)
        assert abs(np.sum(P.M @ s[n:2 * n]) - np.sum(P.M @ P.psi)) <= 10 * bnd * bmax
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)


def test_c3_two_pcg_iterations_per_launch_blocks(pfc, c3):
    """The mixed instance's inner PCG runs two iterations per launch on blocks of the grid (4 x 4 x-lines
    per workgroup, one- and two-step frames in LDS).  With the oracle's inner counts fixed, odd ones
    included (a launch that ends after the first of its two iterations), one P_CH apply in that form
    reaches the oracle's float64 apply as closely as the one-iteration float32 form does (both differ
    from it by float32 rounding of the inner solves), and the form takes fewer launches."""
    from oracle import precond
    P = c3["P"]
    n = P.n
    tau_s = TAU / M11
    w = np.random.default_rng(3).normal(size=3 * n)
    inner = precond.InnerSolvers(P.M, P.K, tau_s, mode="pcg", tol=1e-3)
    z_ref = precond.pch_apply(inner, w)
    counts = list(inner.counts[0])
    out = {}
    insts = []
    try:
        mesh = P.gpu_mesh()
        for spl in (2, 1):
            inst = pfc.pfc_instance_create(mesh, pfc.pfc_opts_default(precision=1, pcg_steps_per_launch=spl))
            insts.append(inst)
            assert pfc.pfc_instance_config(inst)["pcg_steps_per_launch"] == spl
            for fixed in (counts, [3, 1, 4, 5, 2]):
                ref = z_ref if fixed is counts else precond.pch_apply(
                    precond.InnerSolvers(P.M, P.K, tau_s, mode="pcg", fixed_counts=fixed), w)
                z = dev(np.zeros(3 * n))
                print(f"3D 64^3: P_CH apply, {spl} PCG iteration(s) per launch, counts {fixed}", flush=True)
                got = pfc.pfc_apply_pch(inst, n, tau_s, dev(w), z, fixed_counts=fixed)
                assert list(got) == list(fixed)
                out[(spl, tuple(fixed))] = (rel(host(z), ref), pfc.pfc_instance_launch_stats(inst)[0])
        for fixed in (counts, [3, 1, 4, 5, 2]):
            (e2, l2), (e1, l1) = out[(2, tuple(fixed))], out[(1, tuple(fixed))]
            print(f"3D 64^3: counts {fixed}: error against the oracle {e2:.2e} (two per launch) "
                  f"{e1:.2e} (one per launch); launches {l2} / {l1}", flush=True)
            assert e2 <= max(1e-5, 3.0 * e1), (e2, e1)
            if sum(fixed) >= 20:
                assert l2 < 0.8 * l1, (l2, l1)
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
