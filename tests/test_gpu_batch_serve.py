"""Batches and the continuous-batching server (needs a GPU).

Each instance gives the same bits alone and inside a batch or a served mix
(fixed-order reductions that depend only on the instance's own team)."""
import time

import numpy as np
import pytest

import workloads as wl
from helpers import Problem, blockerr, dev, entryerr, host, rel
from oracle import pfc as opfc, solve as osolve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pfc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1501_06852_amd import pfc as lib
    return lib


def _problems():
    return [Problem(2, 16, 0.0, seed=11), Problem(2, 10, 0.2, seed=12), Problem(3, 4, 0.0, seed=13)]


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_alone_equals_mix(pfc, prec):
    probs = _problems()
    prm = wl.draw_params(4, 100)
    # two instances on the first mesh (shared M, K), one on each other mesh
    owners = [0, 0, 1, 2]
    insts, states, alone = [], [], []
    try:
        steps = 1
        for k, pi in enumerate(owners):
            P = probs[pi]
            # one PCG iteration per launch alone as in the batch, for the same bits
            o = pfc.pfc_opts_default(precision=prec, shared_ops=1 if pi == 0 else 0, pcg_steps_per_launch=1)
            insts.append(pfc.pfc_instance_create(P.gpu_mesh(), o))
            psi = wl.psi0(P.n, prm[k].psibar, 0.01, seed=prm[k].seed)
            s0 = np.concatenate([np.zeros(P.n), psi, np.zeros(P.n)])
            states.append(dev(s0))
            sa = dev(s0)
            st, _ = pfc.pfc_rosenbrock_run(insts[-1], P.n, sa, prm[k].r, prm[k].psibar, prm[k].tau, steps)
            alone.append(host(sa))
        ns = [probs[pi].n for pi in owners]
        st, infos = pfc.pfc_batch_run(insts, ns, states, [p.r for p in prm], [p.psibar for p in prm],
                                      [p.tau for p in prm], steps)
        assert st >= 0
        for k in range(4):
            assert np.array_equal(host(states[k]), alone[k]), k
            assert all(i["true_rel_res"] <= 1e-8 for i in infos[k])
        # and against the oracle (float64 run at the same tolerance)
        if prec == 0:
            for k, pi in enumerate(owners):
                P = probs[pi]
                psi = wl.psi0(P.n, prm[k].psibar, 0.01, seed=prm[k].seed)
                x0 = opfc.consistent_init(P.mesh, P.M, P.K, prm[k].r, psi)
                xr, _ = osolve.rosenbrock_run(P.mesh, P.M, P.K, x0, prm[k].r, prm[k].tau, steps, tol=1e-8)
                assert rel(alone[k], xr) <= 1e-6
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        for P in probs:
            P.close()


@pytest.mark.parametrize("prec", [0, 1])
def test_batch_2d_blocks_alone_equals_batch(pfc, prec):
    """Instances on 2D grids of side a multiple of 64 run two PCG iterations per launch on blocks of 64 x 16
    rows in a batch as alone (default options), next to an instance without a two-iteration form that runs
    one iteration per launch in the same launches: the batch gives each instance the bits it has alone and the
    step of the one-iteration form to the accuracy of two solves at relative residual 1e-8, and float64
    instances land on the oracle's Rosenbrock step to that accuracy."""
    probs = [Problem(2, 64, 0.2, seed=21), Problem(2, 128, 0.0, seed=22), Problem(3, 4, 0.0, seed=23)]
    prm = wl.draw_params(4, 300)
    owners = [0, 0, 1, 2]   # the 3D instance has no two-iteration form here and runs one per launch
    insts, states, alone = [], [], []
    try:
        steps = 1
        for k, pi in enumerate(owners):
            P = probs[pi]
            insts.append(pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(precision=prec)))
            assert pfc.pfc_instance_config(insts[-1])["pcg_steps_per_launch"] == (2 if P.mesh.dim == 2 else 1)
            psi = wl.psi0(P.n, prm[k].psibar, 0.01, seed=prm[k].seed)
            s0 = np.concatenate([np.zeros(P.n), psi, np.zeros(P.n)])
            states.append(dev(s0))
            sa = dev(s0)
            st, _ = pfc.pfc_rosenbrock_run(insts[-1], P.n, sa, prm[k].r, prm[k].psibar, prm[k].tau, steps)
            assert st == pfc.PFC_OK
            alone.append(host(sa))
        ns = [probs[pi].n for pi in owners]
        args = ([p.r for p in prm], [p.psibar for p in prm], [p.tau for p in prm])
        st, infos = pfc.pfc_batch_run(insts, ns, states, *args, steps)
        assert st >= 0
        for k in range(len(owners)):
            assert np.array_equal(host(states[k]), alone[k]), k
            assert all(i["true_rel_res"] <= 1e-8 for i in infos[k])
        # the same batch with one PCG iteration per launch: the same step to the solves' accuracy
        one = [pfc.pfc_instance_create(probs[pi].gpu_mesh(), pfc.pfc_opts_default(precision=prec, pcg_steps_per_launch=1))
               for pi in owners]
        insts += one
        st1 = [dev(np.concatenate([np.zeros(probs[pi].n), wl.psi0(probs[pi].n, prm[k].psibar, 0.01, seed=prm[k].seed),
                                   np.zeros(probs[pi].n)])) for k, pi in enumerate(owners)]
        st, _ = pfc.pfc_batch_run(one, ns, st1, *args, steps)
        assert st >= 0
        for k in range(len(owners)):
            assert rel(host(st1[k]), host(states[k])) <= 1e-6, k
        if prec == 0:
            for k, pi in enumerate(owners):
                P = probs[pi]
                psi = wl.psi0(P.n, prm[k].psibar, 0.01, seed=prm[k].seed)
                x0 = opfc.consistent_init(P.mesh, P.M, P.K, prm[k].r, psi)
                xr, _ = osolve.rosenbrock_run(P.mesh, P.M, P.K, x0, prm[k].r, prm[k].tau, steps, tol=1e-8)
                assert rel(host(states[k]), xr) <= 1e-6, k
    finally:
        for i in insts:
            pfc.pfc_instance_destroy(i)
        for P in probs:
            P.close()


def _serve(pfc, meshes, reqs, prec, slots, budget, steps=2, rpt=0):
    import ctypes as C
    so = pfc.pfc_server_opts(C.sizeof(pfc.pfc_server_opts), prec, budget, slots, 0, rpt)
    srv = C.c_void_p()
    assert pfc._lib.pfc_server_create(C.byref(so), C.byref(srv)) == 0
    try:
        for rid, (mi, p, psi) in enumerate(reqs):
            a = np.ascontiguousarray(psi)
            rc = pfc._lib.pfc_server_submit(srv, meshes[mi], p.r, p.psibar, p.tau, a.ctypes.data_as(pfc._dp), steps,
                                            rid)
            assert rc == 0, pfc.pfc_last_error()
        assert pfc._lib.pfc_server_drain(srv) == 0
        out = {}
        buf = (pfc.pfc_result * 16)()
        got = C.c_int()
        while True:
            pfc._lib.pfc_server_poll(srv, buf, 16, C.byref(got))
            if got.value == 0:
                break
            for k in range(got.value):
                r = buf[k]
                n = len(reqs[r.req_id][2])
                out[r.req_id] = (r.status, np.ctypeslib.as_array(r.state, shape=(3 * n,)).copy(),
                                 [r.infos[i].true_rel_res for i in range(r.n_stages)], r.t_admit - r.t_submit)
                pfc._lib.pfc_result_free(C.byref(buf[k]))
        return out
    finally:
        pfc._lib.pfc_server_destroy(srv)


@pytest.mark.parametrize("prec", [1, 0])
def test_server_alone_equals_mix_and_admission(pfc, prec):
    probs = _problems()
    meshes = [P.gpu_mesh() for P in probs]
    prm = wl.draw_params(7, 300)
    reqs = []
    for k in range(7):
        mi = k % 3
        reqs.append((mi, prm[k], wl.psi0(probs[mi].n, prm[k].psibar, 0.01, seed=prm[k].seed)))
    try:
        # alone: one instance per request, plain run
        alone = []
        for mi, p, psi in reqs:
            P = probs[mi]
            # served instances run one PCG iteration per launch (their launch sets change while they run)
            inst = pfc.pfc_instance_create(meshes[mi], pfc.pfc_opts_default(precision=prec, pcg_steps_per_launch=1))
            s = dev(np.concatenate([np.zeros(P.n), psi, np.zeros(P.n)]))
            pfc.pfc_rosenbrock_run(inst, P.n, s, p.r, p.psibar, p.tau, 2)
            alone.append(host(s))
            pfc.pfc_instance_destroy(inst)
            # the served precision reaches the oracle's float64 trajectory as closely as two runs
            # whose stage solves stop at relative residual 1e-8 can
            x0 = opfc.consistent_init(P.mesh, P.M, P.K, p.r, psi)
            xr, _ = osolve.rosenbrock_run(P.mesh, P.M, P.K, x0, p.r, p.tau, 2, tol=1e-8)
            assert rel(alone[-1], xr) <= 1e-6
        # served with room for everything, then with a budget that fits about two instances
        fp = max(pfc.pfc_instance_footprint(m, pfc.pfc_opts_default(precision=prec)) for m in meshes)
        for slots, budget in [(8, 64 << 30), (8, int(2.2 * fp))]:
            out = _serve(pfc, meshes, reqs, prec, slots, budget)
            assert sorted(out) == list(range(7))
            for k in range(7):
                st, state, res, _ = out[k]
                assert st >= 0 and max(res) <= 1e-8
                assert np.array_equal(state, alone[k]), (slots, budget, k)
        # a request that can never fit is refused at submission
        import ctypes as C
        so = pfc.pfc_server_opts(C.sizeof(pfc.pfc_server_opts), prec, 1024, 1, 0, 0)
        srv = C.c_void_p()
        assert pfc._lib.pfc_server_create(C.byref(so), C.byref(srv)) == 0
        a = np.zeros(probs[0].n)
        rc = pfc._lib.pfc_server_submit(srv, meshes[0], -0.3, -0.3, 0.5, a.ctypes.data_as(pfc._dp), 1, 0)
        pfc._lib.pfc_server_destroy(srv)
        assert rc == pfc.PFC_ERR_ADMISSION
    finally:
        for P in probs:
            P.close()


def test_full_size_2d_512_stage_solve(pfc):
    """512^2 jittered (the benchmark configuration): replay parity and tolerance-mode residual at full size."""
    from oracle import assembly
    P = Problem(2, 512, 0.2, psibar=-0.3, seed=0)
    inst = None
    try:
        r, psibar, tau = -0.35, -0.3, 1.0
        m11 = 1.0 / opfc.ROS3PW_GAMMA
        n = P.n
        x0 = opfc.consistent_init(P.mesh, P.M, P.K, r, P.psi)
        b = opfc.stage_rhs_R(P.mesh, P.M, P.K, r, tau, x0, [], [])
        Nm = assembly.N_matrix(P.mesh, P.psi)
        y_ref, info = osolve.solve_stage(P.M, P.K, Nm, r, tau, m11, b, tol=1e-8)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default())
        x = dev(np.zeros(3 * n))
        s = info["schedule"]
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, m11, dev(b), x, replay=(s.cycles, s.inner))
        assert entryerr(host(x), y_ref) <= 1e-10
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, psibar, tau, m11, dev(b), x)
        y = host(x)
        res = np.linalg.norm(b - opfc.apply_AR(P.M, P.K, Nm, r, tau, m11, y)) / np.linalg.norm(b)
        assert st == pfc.PFC_OK and res <= 1e-8
        # the benchmark's entry point on this instance: one whole Rosenbrock step (consistent initial
        # values, N(psi_k) reassembly, three stage right-hand sides and solves, the update), replayed
        # with the oracle's iteration counts, then in tolerance mode
        x_ref, oinf = osolve.rosenbrock_run(P.mesh, P.M, P.K, x0, r, tau, 1, tol=1e-8)
        reps = [(i["schedule"].cycles, i["schedule"].inner) for i in oinf]
        state = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        st, gis = pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau, 1, pfc.PFC_INIT_CONSISTENT, replays=reps)
        assert [g["outer_iters"] for g in gis] == [i["steps"] for i in oinf]
        assert entryerr(host(state), x_ref) <= 1e-10
        state = dev(np.concatenate([np.zeros(n), P.psi, np.zeros(n)]))
        st, gis = pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau, 1)
        assert st == pfc.PFC_OK and max(g["true_rel_res"] for g in gis) <= 1e-8
        assert rel(host(state), x_ref) <= 1e-6
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


def test_full_size_3d_64_mixed_vs_fft_exact(pfc):
    """64^3 Kuhn mesh, constant psi: mixed precision at a tight outer tolerance equals the exact Fourier solve."""
    from oracle import reference
    P = Problem(3, 64, 0.0, psibar=-0.25, amp=0.0, seed=0)
    inst = None
    try:
        r, tau = -0.3, 0.5
        m11 = 1.0 / opfc.ROS3PW_GAMMA
        n = P.n
        b = np.random.default_rng(1).normal(size=3 * n)
        yf = reference.fft_exact(P.mesh, P.M, P.K, r, tau, m11, -0.25, b)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(precision=1, outer_tol=1e-11))
        x = dev(np.zeros(3 * n))
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, -0.25, tau, m11, dev(b), x)
        assert rel(host(x), yf) <= 1e-8, gi
        pfc.pfc_instance_destroy(inst)
        inst = pfc.pfc_instance_create(P.gpu_mesh(), pfc.pfc_opts_default(precision=1))
        st, gi = pfc.pfc_solve(inst, n, dev(P.psi), r, -0.25, tau, m11, dev(b), x)
        assert st == pfc.PFC_OK and gi["true_rel_res"] <= 1e-8
    finally:
        if inst is not None:
            pfc.pfc_instance_destroy(inst)
        P.close()


def test_single_slot_server_keeps_two_iterations(pfc):
    """A float64 server with one slot runs every request alone, with two PCG iterations per launch: each
    result equals, bit for bit, a plain run of an instance with the default options (the same form)."""
    P = Problem(2, 24, 0.2, seed=21)
    mesh = P.gpu_mesh()
    prm = wl.draw_params(3, 500)
    reqs = [(0, p, wl.psi0(P.n, p.psibar, 0.01, seed=p.seed)) for p in prm]
    try:
        alone = []
        for _, p, psi in reqs:
            inst = pfc.pfc_instance_create(mesh, pfc.pfc_opts_default(precision=0))
            s = dev(np.concatenate([np.zeros(P.n), psi, np.zeros(P.n)]))
            pfc.pfc_rosenbrock_run(inst, P.n, s, p.r, p.psibar, p.tau, 2)
            alone.append(host(s))
            pfc.pfc_instance_destroy(inst)
        out = _serve(pfc, [mesh], reqs, 0, 1, 64 << 30)
        assert sorted(out) == list(range(len(reqs)))
        for k in range(len(reqs)):
            st, state, res, _ = out[k]
            assert st >= 0 and max(res) <= 1e-8
            assert np.array_equal(state, alone[k]), k
    finally:
        P.close()


def test_server_large_classes_mixed(pfc):
    """A mixed-precision server with a 2D 512^2 and a 3D 48^3 request (the largest served classes) next to
    small ones: every result equals, bit for bit, the same request run alone, and lands on the oracle's
    float64 trajectory as closely as two runs whose stage solves stop at relative residual 1e-8 can."""
    probs = [Problem(2, 512, 0.0, seed=31), Problem(3, 48, 0.0, seed=32), Problem(2, 16, 0.0, seed=33),
             Problem(3, 4, 0.0, seed=34)]
    prm = wl.draw_params(6, 900)
    owners = [0, 2, 1, 3, 2, 3]
    reqs = [(mi, prm[k], wl.psi0(probs[mi].n, prm[k].psibar, 0.01, seed=prm[k].seed)) for k, mi in enumerate(owners)]
    steps = 1
    try:
        meshes = [P.gpu_mesh() for P in probs]
        # served with one row per thread (fixed, so that the alone runs use the same teams)
        print("served large classes: server run", flush=True)
        out = _serve(pfc, meshes, reqs, 1, 8, 64 << 30, steps=steps, rpt=1)
        assert sorted(out) == list(range(len(reqs)))
        for k, (mi, p, psi) in enumerate(reqs):
            P = probs[mi]
            print(f"served large classes: request {k} ({P.mesh.dim}D, n = {P.n}) alone and oracle", flush=True)
            # the server runs 2D grids of side 64k in the block form of two PCG iterations per launch,
            # the others one iteration per launch
            pcg = 2 if (P.mesh.dim == 2 and P.mesh.N % 64 == 0) else 1
            inst = pfc.pfc_instance_create(meshes[mi], pfc.pfc_opts_default(precision=1, rows_per_thread=1,
                                                                            pcg_steps_per_launch=pcg))
            assert pfc.pfc_instance_config(inst)["pcg_steps_per_launch"] == pcg
            s = dev(np.concatenate([np.zeros(P.n), psi, np.zeros(P.n)]))
            pfc.pfc_rosenbrock_run(inst, P.n, s, p.r, p.psibar, p.tau, steps)
            alone = host(s)
            pfc.pfc_instance_destroy(inst)
            st, state, res, _ = out[k]
            assert st >= 0 and max(res) <= 1e-8, (k, st, res)
            assert np.array_equal(state, alone), k
            x0 = opfc.consistent_init(P.mesh, P.M, P.K, p.r, psi)
            xr, _ = osolve.rosenbrock_run(P.mesh, P.M, P.K, x0, p.r, p.tau, steps, tol=1e-8)
            err = rel(state, xr)
            print(f"served large classes: request {k} against the oracle {err:.2e}", flush=True)
            assert err <= 1e-6, (k, err)
    finally:
        for P in probs:
            P.close()
