"""Benchmark of the PFC block-preconditioned FGMRES stage solve on one MI355X.

Default workload (the headline configuration): 2D periodic 512x512 P1 mesh
(262,144 nodes, 786,432 unknowns), node positions jittered by U[-0.2h, 0.2h],
r = -0.35, psibar = -0.3, psi_0 = psibar + U[-0.01, 0.01], Ros3Pw steps with
tau = 1.0, N(psi) reassembled every step, FGMRES(30) to 1e-8 relative
residual, float64.  One "step" is one Rosenbrock step: N reassembly and three
stage solves.  Inputs are synthetic and seeded; everything is resident in HBM
before the timed region starts.

Prints one JSON line.  `value` is stage solves per second.  `roofline` uses the
algorithmic bytes of the solver kernel (paper_1501_06852_amd.roofline) per
launch over the average launch period measured with HIP events on the solver
stream.  `cpu_baseline` times the float64 oracle on one Rosenbrock step of the
same workload on the host (single thread).

Other workloads (`--workload`): 3D 64^3 mixed precision, the P2 / PFC1 / S_D
variants at the headline size, 256 batched 128^2 instances, a served stream of
six mesh classes, adaptive Ros3Pw on the headline problem (t = 0 to 200), and
the device-copy calibration of the traffic counters.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per solver launch from rocprofv3 FETCH_SIZE and WRITE_SIZE runs,
# each scaled by what the counter reads for a plain device copy of known size
# (fetch x2.0, write x1.0), averaged over every launch of a profiled
# `--steps 1 --warmup 0` run (mixed workloads: `--no-precision-check`).  A figure holds only for the kernel sources it
# was taken on: when their digest differs, `traffic` is reported as null.
TRAFFIC = {
    # workload: (sha256 of the kernel sources, bytes per launch, algorithmic bytes per launch of the same run)
    "pfc2d_512_fp64": ("9ff8f5f98174d6032f9200ac3dd8c209432041b5c5084cdcb35e2ea7fc0d6bd8", 46748597.0, 85211856.0),
    "pfc3d_64_mixed": ("9ff8f5f98174d6032f9200ac3dd8c209432041b5c5084cdcb35e2ea7fc0d6bd8", 38870673.0, 71753338.0),
}


# the sources that build the solver kernel and the mesh layout it reads (not the server's host code)
KERNEL_SOURCES = ["include/pfc.h"] + [f"paper_1501_06852_amd/csrc/{f}" for f in
                                      ("device.h", "host.h", "mesh.hip", "pfc_internal.h", "solver.h", "solver.hip")]


def kernel_source_digest():
    import hashlib

    d = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        d.update(rel.encode())
        with open(os.path.join(ROOT, rel), "rb") as f:
            d.update(f.read())
    return d.hexdigest()


def traffic_for(workload):
    rec = TRAFFIC.get(workload)
    if rec is None or rec[0] != kernel_source_digest():
        return None, None
    return rec[1], rec[2]

WORKLOADS = {
    # name: (dim, N, jitter, r, psibar, tau, precision, default steps)
    "pfc2d_512_fp64": (2, 512, 0.2, -0.35, -0.3, 1.0, 0, 20),
    "pfc3d_64_mixed": (3, 64, 0.0, -0.3, -0.25, 0.5, 1, 10),
    "pfc2d_64_fp64": (2, 64, 0.0, -0.35, -0.3, 0.1, 0, 1),
    # the variants of the method beyond the headline path, at the headline size
    "pfc2d_256_p2_fp64": (2, 256, 0.2, -0.35, -0.3, 1.0, 0, 10),      # P2: 262,144 nodes like 512^2 P1
    "pfc2d_512_pfc1_fp64": (2, 512, 0.2, -0.35, -0.3, 1.0, 0, 10),    # PFC1 mobility, smooth initial state
    "pfc2d_512_sd_fp64": (2, 512, 0.2, -0.35, -0.3, 1.0, 0, 10),      # P(S_D) preconditioner
}
# options of the variant workloads: Lagrange degree, model, Schur approximation,
# smooth initial state (amplitude, largest wave number per direction)
VARIANTS = {
    "pfc2d_256_p2_fp64": dict(degree=2),
    "pfc2d_512_pfc1_fp64": dict(model=1, smooth=(0.2, 16)),
    "pfc2d_512_sd_fp64": dict(schur_variant=1),
}


# The paper's own numbers for this path, quoted as context only: a machine the tables do not name, a time
# discretisation they do not single out (implicit Euler or the Rosenbrock scheme, Section 7), h = pi/4,
# about 66,000 DOFs; P_CH with PCG inner solves as in Table inner_solvers, times per linear solve averaged
# over 20 time steps.
PAPER_CONTEXT = {
    2: {"source": "Table direct_iterative_solvers (tau = 0.1, P1) and Table timestep_change (P2, tau = 1.0), 2D",
        "p1_tau0.1": {"seconds_per_solve": 1.65, "outer_iterations": 14},
        "p2_tau1.0": {"seconds_per_solve": 4.53, "outer_iterations": 19},
        "hardware": "not stated (sequential AMDiS/MTL4 runs)", "dofs": "about 66,000"},
    3: {"source": "Table direct_iterative_solvers (tau = 0.1, P1) and Table timestep_change (P2, tau = 1.0), 3D",
        "p1_tau0.1": {"seconds_per_solve": 3.36, "outer_iterations": 18},
        "p2_tau1.0": {"seconds_per_solve": 14.29, "outer_iterations": 24},
        "hardware": "not stated (sequential AMDiS/MTL4 runs)", "dofs": "about 66,000"},
}


def run_cpu_baseline(dim, N, jitter, r, psibar, tau, seed, repeats=3):
    """The oracle as it stands: one Rosenbrock step (three stage solves) of the same workload, timed
    `repeats` times from the same state, median.  The oracle's work is scipy sparse products and numpy
    vector operations; scipy's sparse products run on one thread, so the BLAS pool is pinned to one
    thread as well and the figure is a one-core figure.  A step stands for the timed run because every
    step of a fixed-tau run solves systems of the same size and conditioning (the iteration counts of
    the first step are within a few percent of the later ones')."""
    from threadpoolctl import threadpool_limits

    import workloads as wl
    from oracle import assembly, pfc as opfc, solve as osolve

    mesh = wl.make_mesh(dim, N, jitter=jitter, seed=seed)
    M, K = assembly.mass_stiffness(mesh)
    psi = wl.psi0(mesh.n, psibar, 0.01, seed=seed)
    times = []
    with threadpool_limits(1):
        x0 = opfc.consistent_init(mesh, M, K, r, psi)
        for _ in range(repeats):
            t0 = time.perf_counter()
            x1, infos = osolve.rosenbrock_run(mesh, M, K, x0, r, tau, 1, tol=1e-8)
            times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    return dict(value=3.0 / dt, unit="stage solves/s", cores=1, kind="oracle",
                sample=f"1 Rosenbrock step (3 stage solves, {sum(i['steps'] for i in infos)} Arnoldi steps) of the "
                       f"same workload from its consistent initial state, oracle float64 FGMRES(30)+P_CH+Jacobi-PCG "
                       f"(scipy sparse products, one thread), median of {repeats}: "
                       + ", ".join(f"{t:.1f}" for t in times) + " s")


def oracle_stage_check(pfc, torch, mesh, h, state, r, psibar, tau, precisions, model=0, schur=0):
    """Accuracy against the float64 oracle (untimed).  At the given step state x_k the oracle forms the
    stage-1 system of the next Ros3Pw step (its own M, K, N(psi_k) and right-hand side) and solves it to
    1e-12 as the reference; the GPU solves the same system in tolerance mode (1e-8) in each precision.
    Reported per precision: the true residual computed with the oracle's operator and the forward error
    against the reference."""
    from oracle import assembly, pfc as opfc, solve as osolve

    n = mesh.n
    xk = state.detach().cpu().numpy().astype(np.float64)
    M, K = assembly.mass_stiffness(mesh)
    psi = xk[n:2 * n]
    Nm = assembly.N_matrix(mesh, psi)
    m11 = 1.0 / opfc.ROS3PW_GAMMA
    if model == 1:
        from oracle import mobility as mob
        b = mob.stage_rhs_R1(mesh, M, K, r, tau, xk, [], [])
        Kp, Fm = mob.K_plus(mesh, psi), mob.F_mu(mesh, xk[:n])
        m0 = mob.mobility_mean(M, psi)
        y_ref, _ = osolve.solve_stage(M, K, Nm, r, tau, m11, b, tol=1e-12, Kp=Kp, Fm=Fm, m0=m0,
                                      schur="D" if schur else "CH")

        def op(y):
            return mob.apply_AR1(M, K, Nm, Kp, Fm, r, tau, m11, y)
    else:
        b = opfc.stage_rhs_R(mesh, M, K, r, tau, xk, [], [])
        y_ref, _ = osolve.solve_stage(M, K, Nm, r, tau, m11, b, tol=1e-12, schur="D" if schur else "CH")

        def op(y):
            return opfc.apply_AR(M, K, Nm, r, tau, m11, y)
    dev = state.device
    out = {"reference": "oracle float64 FGMRES(30)+P_CH solve to 1e-12 of the stage-1 system at the final state"}
    for prec in precisions:
        inst = pfc.pfc_instance_create(h, pfc.pfc_opts_default(precision=prec, model=model, schur_variant=schur))
        x = torch.zeros(3 * n, dtype=torch.float64, device=dev)
        bt = torch.tensor(b, dtype=torch.float64, device=dev)
        if model == 1:
            st, gi = pfc.pfc_solve_x(inst, n, state, r, psibar, tau, m11, bt, x)
        else:
            st, gi = pfc.pfc_solve(inst, n, state[n:2 * n].contiguous(), r, psibar, tau, m11, bt, x)
        y = x.cpu().numpy()
        pfc.pfc_instance_destroy(inst)
        out["fp64" if prec == 0 else "mixed"] = dict(
            status=pfc.pfc_status_str(st), outer_iters=gi["outer_iters"],
            true_rel_res_oracle_operator=float(np.linalg.norm(b - op(y)) / np.linalg.norm(b)),
            forward_rel_err=float(np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)))
    return out


def sampled_oracle_errors(mesh, samples, steps):
    """Relative error ||x - x_oracle|| / ||x_oracle|| of GPU results (host arrays) against the float64
    oracle's Ros3Pw run of the same request: consistent initial values from the request's psi_0, then
    `steps` steps with stage solves to 1e-8 (so the figure is the size of the difference between two
    runs whose stage solves stop at that tolerance).  samples: (index, params, state)."""
    import workloads as wl
    from oracle import assembly, pfc as opfc, solve as osolve

    M, K = assembly.mass_stiffness(mesh)
    errs = {}
    for k, p, x in samples:
        psi = wl.psi0(mesh.n, p.psibar, 0.01, seed=p.seed)
        x0 = opfc.consistent_init(mesh, M, K, p.r, psi)
        xr, _ = osolve.rosenbrock_run(mesh, M, K, x0, p.r, p.tau, steps, tol=1e-8)
        errs[str(k)] = float(np.linalg.norm(x - xr) / np.linalg.norm(xr))
    return dict(max=max(errs.values()), per_sample=errs,
                reference=f"oracle float64 Ros3Pw run ({steps} steps, stage solves to 1e-8)")


def bench_batched(args, torch, wl, pfc):
    """256 independent 2D 128^2 instances on one shared mesh, one launch set: mixed batched versus
    the plain float64 solver run instance by instance (same instances, same steps)."""
    count = args.batch
    N = 128
    rpt = 4 if args.rows_per_thread is None else args.rows_per_thread
    mesh = wl.make_mesh(2, N)
    n = mesh.n
    h = pfc.pfc_mesh_create_p1(2, n, mesh.elem_nodes, mesh.elem_coords)
    prm = wl.draw_params(count, 7000)
    steps = args.steps if args.steps is not None else 2
    dev = torch.device("cuda:0")

    def states():
        out = []
        for p in prm:
            s = torch.zeros(3 * n, dtype=torch.float64, device=dev)
            s[n:2 * n] = torch.tensor(wl.psi0(n, p.psibar, 0.01, seed=p.seed), dtype=torch.float64, device=dev)
            out.append(s)
        return out

    res = {}
    # launch configurations: the autotuner's choice for this batch (from the cache, or measured now), and
    # the hand-picked one of earlier measurements (4 rows per thread, operators formed on the fly)
    tuned = {prec: pfc.pfc_autotune(h, prec, count) for prec in (1, 0)}
    runs = [("batched_mixed", 1, pfc.tuned_opts(tuned[1], precision=1)),
            ("batched_fp64", 0, pfc.tuned_opts(tuned[0], precision=0))]
    if not args.no_handpicked:
        runs.append(("batched_mixed_handpicked", 1, pfc.pfc_opts_default(precision=1, shared_ops=1,
                                                                         rows_per_thread=rpt)))
    for label, prec, opts in runs:
        insts = [pfc.pfc_instance_create(h, opts) for _ in range(count)]
        st = states()
        pfc.pfc_batch_run(insts, [n] * count, st, [p.r for p in prm], [p.psibar for p in prm],
                          [p.tau for p in prm], 0, pfc.PFC_INIT_CONSISTENT)
        if args.warmup > 0:   # untimed steps from a copy of the states (the timed steps start from x_0)
            warm = [x.clone() for x in st]
            pfc.pfc_batch_run(insts, [n] * count, warm, [p.r for p in prm], [p.psibar for p in prm],
                              [p.tau for p in prm], args.warmup, pfc.PFC_INIT_GIVEN)
            del warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        code, infos = pfc.pfc_batch_run(insts, [n] * count, st, [p.r for p in prm], [p.psibar for p in prm],
                                        [p.tau for p in prm], steps, pfc.PFC_INIT_GIVEN)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        resid = max(i["true_rel_res"] for row in infos for i in row)
        from paper_1501_06852_amd import roofline
        w = 4 if prec == 1 else 8
        alg = sum(roofline.solve_bytes(n, 7, w, i) for row in infos for i in row)
        res[label] = dict(solves_per_s=3 * steps * count / dt, seconds=dt, status=pfc.pfc_status_str(code),
                          max_true_rel_res=resid, algorithmic_GBps=alg / dt / 1e9,
                          hbm_frac=alg / dt / 1e9 / HBM_PEAK_GBS)
        res[label]["config"] = {k: getattr(opts, k) for k in ("rows_per_thread", "ticks_per_graph",
                                                              "pcg_steps_per_launch", "grid_columns", "shared_ops")}
        if label != "batched_mixed_handpicked" and not args.no_precision_check:
            # sampled instances against the oracle's float64 run of the same steps (not timed)
            res[label]["err_vs_oracle_fp64"] = sampled_oracle_errors(
                mesh, [(k, prm[k], st[k].cpu().numpy()) for k in (0, count // 2, count - 1)], steps)
        for i in insts:
            pfc.pfc_instance_destroy(i)
    # plain float64 solver, one instance at a time, on a sample of the same instances
    sample = min(count, args.plain_sample)
    plain_tuned = pfc.pfc_autotune(h, 0, 1)
    inst = pfc.pfc_instance_create(h, pfc.tuned_opts(plain_tuned, precision=0))
    st = states()[:sample]
    for k in range(sample):
        p = prm[k]
        pfc.pfc_rosenbrock_run(inst, n, st[k], p.r, p.psibar, p.tau, 0, pfc.PFC_INIT_CONSISTENT)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(sample):
        p = prm[k]
        pfc.pfc_rosenbrock_run(inst, n, st[k], p.r, p.psibar, p.tau, steps, pfc.PFC_INIT_GIVEN)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res["plain_fp64_sequential"] = dict(solves_per_s=3 * steps * sample / dt, seconds=dt, instances=sample,
                                        autotune=plain_tuned)
    pfc.pfc_instance_destroy(inst)
    pfc.pfc_mesh_destroy(h)
    out = {"metric": "PFC block solves/s @1e-8 rel residual", "value": res["batched_mixed"]["solves_per_s"],
           "unit": "stage solves/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup, "higher_is_better": True,
           "dtype": "f64 outer / f32 inner", "data": "synthetic",
           "config": {"workload": f"pfc2d_128_batched{count}_mixed", "instances": count, "grid": N, "nodes": n,
                      "launch": res["batched_mixed"]["config"], "launch_chosen_by": "autotuner",
                      "autotune": tuned[1]},
           "speedup_vs_plain_fp64": res["batched_mixed"]["solves_per_s"] / res["plain_fp64_sequential"]["solves_per_s"],
           "detail": res}
    print(json.dumps(out), flush=True)


def bench_served(args, torch, wl, pfc):
    """Served stream: Poisson arrivals of Rosenbrock requests over six mesh classes.  Mixed precision with
    continuous batching versus the plain float64 solver serving one request at a time (FIFO)."""
    import ctypes as C
    classes = wl.SERVED_CLASSES
    meshes = []
    for dim, N in classes:
        m = wl.make_mesh(dim, N)
        meshes.append((m, pfc.pfc_mesh_create_p1(dim, m.n, m.elem_nodes, m.elem_coords)))
    nreq = args.requests
    warm = int(np.ceil(0.05 * nreq))
    steps = args.req_steps
    rpt = 0 if args.rows_per_thread is None else args.rows_per_thread   # 0: chosen per request by load

    def stream(rate):
        return wl.served_stream(nreq, rate, 4242)

    # the autotuner's rows per thread for batches mixing the six classes, at a moderate and at the full
    # load (the tuned servers below give each request the choice for the number of requests then active;
    # below the smallest tuned count they use the load rule)
    hmeshes = [hm for _, hm in meshes]
    tuned = {f"{'mixed' if prec else 'fp64'} mix x{c}": pfc.pfc_autotune_mix(hmeshes, prec, c)
             for prec in (1, 0) for c in sorted({8, args.slots})}

    def serve(prec, slots, rate, rpt, keep=(), use_tuned=1):
        so = pfc.pfc_server_opts(C.sizeof(pfc.pfc_server_opts), prec, 96 << 30, slots, 0, rpt, use_tuned)
        srv = C.c_void_p()
        assert pfc._lib.pfc_server_create(C.byref(so), C.byref(srv)) == 0
        reqs = stream(rate)
        psis = [np.ascontiguousarray(wl.psi0(meshes[c][0].n, p.psibar, 0.01, seed=p.seed)) for _, c, p in reqs]
        t_base = pfc._lib.pfc_server_clock(srv)
        arrive = {}
        for k, (t, c, p) in enumerate(reqs):
            while pfc._lib.pfc_server_clock(srv) - t_base < t:
                time.sleep(0.0005)
            arrive[k] = pfc._lib.pfc_server_clock(srv)
            rc = pfc._lib.pfc_server_submit(srv, meshes[c][1], p.r, p.psibar, p.tau, psis[k].ctypes.data_as(pfc._dp),
                                            steps, k)
            assert rc == 0, pfc.pfc_last_error()
        assert pfc._lib.pfc_server_drain(srv) == 0
        t_end = pfc._lib.pfc_server_clock(srv)
        buf = (pfc.pfc_result * 64)()
        got = C.c_int()
        lat, worst, kept = [], 0.0, {}
        while True:
            pfc._lib.pfc_server_poll(srv, buf, 64, C.byref(got))
            if got.value == 0:
                break
            for k in range(got.value):
                r = buf[k]
                if r.req_id >= warm:   # the first 5% of the stream warm the server up
                    lat.append(r.t_done - arrive[r.req_id])
                worst = max([worst] + [r.infos[i].true_rel_res for i in range(r.n_stages)])
                if r.req_id in keep:
                    nn = meshes[reqs[r.req_id][1]][0].n
                    kept[r.req_id] = np.ctypeslib.as_array(r.state, shape=(3 * nn,)).copy()
                pfc._lib.pfc_result_free(C.byref(buf[k]))
        pfc._lib.pfc_server_destroy(srv)
        lat = np.array(lat)
        return dict(solves_per_s=3 * steps * nreq / (t_end - t_base), wall_s=t_end - t_base,
                    p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    latency_requests=int(lat.size), max_true_rel_res=worst), kept

    # capacity of the plain server (backlogged), then both at 0.8 of that rate
    # the first request of each of the three smallest classes is checked against the oracle
    sample = {}
    for k, (_, c, _) in enumerate(stream(0.0)):
        if c not in sample and meshes[c][0].n <= 32768:
            sample[c] = k
    def leg(name, res):
        print(f"served: {name} done, {res['solves_per_s']:.1f} stage solves/s over {res['wall_s']:.1f} s",
              file=sys.stderr, flush=True)
        return res

    base_bl, _ = serve(0, 1, 0.0, 0)   # a single slot: every request alone (tuned table entries apply from 8)
    leg("float64 FIFO, backlogged", base_bl)
    rate = 0.8 * nreq / base_bl["wall_s"]
    ours_bl, kept = serve(1, args.slots, 0.0, rpt, keep=set(sample.values()))
    leg("mixed continuous, backlogged", ours_bl)
    base, _ = serve(0, 1, rate, 0)
    leg("float64 FIFO, Poisson arrivals", base)
    ours, _ = serve(1, args.slots, rate, rpt)
    leg("mixed continuous, Poisson arrivals", ours)
    # the same backlogged stream with the load rule instead of the table (for comparison)
    ours_rule, _ = serve(1, args.slots, 0.0, rpt, use_tuned=0)
    leg("mixed continuous with the load rule, backlogged", ours_rule)
    if not args.no_precision_check:
        reqs0 = stream(0.0)
        errs = {}
        for c, k in sample.items():
            e = sampled_oracle_errors(meshes[c][0], [(k, reqs0[k][2], kept[k])], steps)
            errs[f"{classes[c][0]}D {classes[c][1]} request {k}"] = e["per_sample"][str(k)]
        ours_bl["err_vs_oracle_fp64"] = dict(
            max=max(errs.values()), per_sample=errs,
            reference=f"oracle float64 Ros3Pw run ({steps} steps, stage solves to 1e-8) of the same request")
    for _, hm in meshes:
        pfc.pfc_mesh_destroy(hm)
    out = {"metric": "PFC block solves/s @1e-8 rel residual; p50/p99 served latency", "value": ours_bl["solves_per_s"],
           "unit": "stage solves/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64 outer / f32 inner",
           "data": "synthetic",
           "config": {"workload": "served_stream", "requests": nreq, "warmup_requests_excluded_from_latency": warm,
                      "rosenbrock_steps": steps,
                      "classes": [f"{d}D {N}" for d, N in classes], "arrival_rate_hz": rate, "slots": args.slots,
                      "rows_per_thread": "autotuner (mixed-batch table entry for the active count)" if rpt == 0
                      else rpt,
                      "autotune": {k: {f: v[f] for f in ("rows_per_thread", "ms_per_step", "ms_default", "from_cache")}
                                   for k, v in tuned.items()}},
           "speedup_vs_plain_fp64_fifo": ours_bl["solves_per_s"] / base_bl["solves_per_s"],
           "backlogged": {"mixed_continuous": ours_bl, "fp64_fifo": base_bl, "mixed_continuous_load_rule": ours_rule},
           "poisson": {"mixed_continuous": ours, "fp64_fifo": base}}
    print(json.dumps(out), flush=True)


def bench_adaptive(args, torch, wl, pfc, roofline):
    """Adaptive Ros3Pw (embedded error estimate, step-size control) on the headline 2D 512^2 float64 problem,
    from t = 0 to t_end: every attempted step, accepted or rejected, costs three stage solves."""
    N, r, psibar, jitter = 512, -0.35, -0.3, 0.2
    tau0, t_end, tol, max_outer = 0.1, 200.0, 1e-3, 300
    max_attempts = args.steps if args.steps is not None else 400
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    mesh = wl.make_mesh(2, N, jitter=jitter, seed=args.seed)
    h = pfc.pfc_mesh_create_p1(2, mesh.n, mesh.elem_nodes, mesh.elem_coords)
    n = mesh.n
    z = pfc.pfc_mesh_query(h)["nnz"] / n
    # a stage solve that needs more than max_outer Arnoldi steps rejects its step (tau * 0.2)
    inst = pfc.pfc_instance_create(h, pfc.pfc_opts_default(precision=0, max_steps=max_outer))
    state = torch.zeros(3 * n, dtype=torch.float64, device=dev)
    state[n:2 * n] = torch.tensor(wl.psi0(n, psibar, 0.01, seed=args.seed), dtype=torch.float64, device=dev)
    # consistent initial values and `warmup` fixed steps of tau0 on a copy (not timed)
    warm = state.clone()
    pfc.pfc_rosenbrock_run(inst, n, warm, r, psibar, tau0, max(args.warmup, 0), pfc.PFC_INIT_CONSISTENT)
    pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau0, 0, pfc.PFC_INIT_CONSISTENT)
    del warm
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    st, taus, rej, infos = pfc.pfc_rosenbrock_adaptive(inst, n, state, r, psibar, tau0, t_end, tol, tol,
                                                       max_attempts, pfc.PFC_INIT_GIVEN)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    launches, graphs = pfc.pfc_instance_launch_stats(inst)
    attempts = len(taus) + rej
    solves = 3 * attempts
    alg = sum(roofline.solve_bytes(n, z, 8, i) for i in infos) + \
        attempts * roofline.step_bytes(n, z, mesh.n_elem, 2, nloc=mesh.elem_nodes.shape[1])
    period_s = gpu_ms * 1e-3 / max(1, launches)
    achieved = alg / max(1, launches) / period_s / 1e9
    failed = [a for a in range(attempts) if any(i["status"] == pfc.PFC_NOT_CONVERGED for i in infos[3 * a:3 * a + 3])]
    res = [i["true_rel_res"] for a in range(attempts) if a not in failed for i in infos[3 * a:3 * a + 3]]
    out = {
        "metric": "PFC block solves/s @1e-8 rel residual",
        "value": solves / wall,
        "unit": "stage solves/s",
        "n_gpus": 1,
        "steps": attempts,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / max(1, attempts),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "pfc2d_512_adaptive_fp64", "dim": 2, "grid": N, "nodes": n, "unknowns": 3 * n,
                   "jitter_h": jitter, "r": r, "psibar": psibar, "tau0": tau0, "t_end": t_end, "rtol": tol,
                   "atol": tol, "max_attempts": max_attempts, "restart": 30, "outer_tol": 1e-8, "inner_tol": 1e-3,
                   "max_outer_steps": max_outer},
        "status": pfc.pfc_status_str(st),
        "t_reached": float(np.sum(taus)),
        "accepted": len(taus), "rejected": rej, "rejected_solve_failed": len(failed),
        "tau_min": float(np.min(taus)) if len(taus) else None, "tau_max": float(np.max(taus)) if len(taus) else None,
        "simulated_time_per_s": float(np.sum(taus)) / wall,
        "max_true_rel_res_converged": max(res) if res else None,
        "outer_iters_mean": float(np.mean([i["outer_iters"] for i in infos])) if infos else None,
        "inner_pcg_per_apply_mean": float(np.mean([i["inner_total"] / max(1, i["inner_applies"]) for i in infos]))
        if infos else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_tick (solver phase launch)", "launches": launches,
                     "algorithmic_bytes": alg, "algorithmic_bytes_per_launch": alg / max(1, launches),
                     "avg_launch_period_us": period_s * 1e6, "kernel_sources_sha256": kernel_source_digest()},
    }
    pfc.pfc_instance_destroy(inst)
    pfc.pfc_mesh_destroy(h)
    print(json.dumps(out), flush=True)


def bench_copy_calibration(torch):
    """Plain device copies (torch's copy kernel, float64): a 1 GiB copy three times, the reference
    kernel whose FETCH_SIZE / WRITE_SIZE counter readings calibrate the solver kernel's, and the
    streaming rates of the two ceilings the roofline discussion uses: arrays far larger than the
    256 MB MALL (1 GiB, read + write), and a 32 MiB working set that stays MALL-resident (copied
    over and over).  Rates count the bytes read plus the bytes written."""
    out = {"workload": "copy_calibration"}
    for label, nbytes, reps in (("hbm_1GiB", 1 << 30, 20), ("mall_32MiB", 32 << 20, 400)):
        n = nbytes // 8
        x = torch.ones(n, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            y.copy_(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[label] = {"bytes_read_per_copy": nbytes, "bytes_written_per_copy": nbytes, "copies": reps,
                      "us_per_copy": ms * 1e3, "GBps": 2 * nbytes / (ms * 1e-3) / 1e9}
        del x, y
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pfc2d_512_fp64", choices=sorted(WORKLOADS) + ["batched", "served", "adaptive", "copy_calibration"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-check", action="store_true",
                    help="skip the untimed float64 comparison step of mixed-precision workloads (profiled runs)")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1501_06852_amd", "tune_cache.json"),
                    help="autotuning table to start from (JSON; missing entries are measured)")
    ap.add_argument("--tune-save", default=None, help="write the autotuning table here afterwards")
    ap.add_argument("--retune", action="store_true", help="start from an empty autotuning table")
    ap.add_argument("--no-handpicked", action="store_true", help="batched: skip the hand-picked comparison run")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--plain-sample", type=int, default=16)
    ap.add_argument("--requests", type=int, default=500)
    ap.add_argument("--req-steps", type=int, default=5)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--rows-per-thread", type=int, default=None,
                    help="rows per thread of the batched (default 4) and served mixed (default 0: by load) instances")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch

    import workloads as wl
    from paper_1501_06852_amd import pfc, roofline

    if args.workload == "copy_calibration":
        return bench_copy_calibration(torch)
    if not args.retune and os.path.exists(args.tune_cache):
        pfc.pfc_tune_load(args.tune_cache)
    if args.tune_save:
        import atexit
        atexit.register(lambda: pfc.pfc_tune_save(args.tune_save))
    if args.workload == "batched":
        return bench_batched(args, torch, wl, pfc)
    if args.workload == "served":
        return bench_served(args, torch, wl, pfc)
    if args.workload == "adaptive":
        return bench_adaptive(args, torch, wl, pfc, roofline)
    dim, N, jitter, r, psibar, tau, prec, dsteps = WORKLOADS[args.workload]
    var = VARIANTS.get(args.workload, {})
    steps = args.steps if args.steps is not None else dsteps
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    mesh = wl.make_mesh(dim, N, jitter=jitter, seed=args.seed)
    if var.get("degree") == 2:
        mesh = wl.p2_mesh(mesh)
        h = pfc.pfc_mesh_create_p2(dim, mesh.n, mesh.elem_nodes, mesh.elem_coords)
    else:
        h = pfc.pfc_mesh_create_p1(dim, mesh.n, mesh.elem_nodes, mesh.elem_coords)
    n = mesh.n
    nnz = pfc.pfc_mesh_query(h)["nnz"]
    gside = pfc.pfc_mesh_grid_side(h)   # the solver computes the columns of periodic grids
    z = nnz / n
    model = var.get("model", 0)
    schur = var.get("schur_variant", 0)
    # the launch configuration of the autotuner for this mesh and precision (its table is keyed by the mesh
    # and precision only: the PFC1 and S_D variants on the headline mesh take the headline's entry)
    tuned = pfc.pfc_autotune(h, prec, 1)
    opts = pfc.tuned_opts(tuned, precision=prec, max_run_steps=max(steps, args.warmup, 1), model=model,
                          schur_variant=schur)
    inst = pfc.pfc_instance_create(h, opts)
    if "smooth" in var:
        psi = wl.psi_smooth(mesh, psibar, var["smooth"][0], kmax=var["smooth"][1], seed=args.seed)
    else:
        psi = wl.psi0(n, psibar, 0.01, seed=args.seed)
    state = torch.zeros(3 * n, dtype=torch.float64, device=dev)
    state[n:2 * n] = torch.tensor(psi, dtype=torch.float64, device=dev)
    # warm-up: consistent initial values and `warmup` steps (not timed)
    pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau, max(args.warmup, 0), pfc.PFC_INIT_CONSISTENT)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    st, infos = pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau, steps, pfc.PFC_INIT_GIVEN)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    launches, graphs = pfc.pfc_instance_launch_stats(inst)
    solves = 3 * steps
    w = 4 if prec == 1 else 8
    z_sd = None
    if schur:
        # entries per row of the second-ring pattern of K M_D^-1 K (host count from the mesh pattern)
        import scipy.sparse as sp
        A = sp.csr_matrix((np.ones(mesh.n_elem * mesh.elem_nodes.shape[1] ** 2),
                           (np.repeat(mesh.elem_nodes, mesh.elem_nodes.shape[1], axis=1).ravel(),
                            np.tile(mesh.elem_nodes, (1, mesh.elem_nodes.shape[1])).ravel())), shape=(n, n))
        A.data[:] = 1.0
        z_sd = (A @ A).nnz / n
    alg = sum(roofline.solve_bytes(n, z, w, i, model=model, z_sd=z_sd) for i in infos) + \
        steps * roofline.step_bytes(n, z, mesh.n_elem, dim, nloc=mesh.elem_nodes.shape[1], model=model)
    period_s = gpu_ms * 1e-3 / max(1, launches)
    achieved = alg / max(1, launches) / period_s / 1e9
    res = [i["true_rel_res"] for i in infos]
    traffic, traffic_alg = traffic_for(args.workload)
    out = {
        "metric": "PFC block solves/s @1e-8 rel residual",
        "value": solves / wall,
        "unit": "stage solves/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f64 outer / f32 inner",
        "data": "synthetic",
        "config": {"workload": args.workload, "dim": dim, "grid": N, "nodes": n, "unknowns": 3 * n,
                   "jitter_h": jitter, "r": r, "psibar": psibar, "tau": tau, "rosenbrock_steps": steps,
                   "stage_solves": solves, "restart": 30, "outer_tol": 1e-8, "inner_tol": 1e-3,
                   "element_degree": mesh.degree, "model": "PFC1" if model == 1 else "PFC2",
                   "schur": "S_D" if schur else "S_CH", "initial_state": "smooth" if "smooth" in var else "noise",
                   "columns": (f"computed from the row (periodic grid, side {gside})" if gside else "read from memory"),
                   "pcg_steps_per_launch": pfc.pfc_instance_config(inst)["pcg_steps_per_launch"],
                   "launch": pfc.pfc_instance_config(inst),
                   "launch_chosen_by": "autotuner", "autotune": tuned},
        "status": pfc.pfc_status_str(st),
        "max_true_rel_res": max(res) if res else None,
        "outer_iters_mean": float(np.mean([i["outer_iters"] for i in infos])),
        "t_solve_mean_ms": float(np.mean([i["t_solve"] for i in infos])) * 1e3,   # device clock, per stage solve
        "inner_pcg_per_apply_mean": float(np.mean([i["inner_total"] / max(1, i["inner_applies"]) for i in infos])),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_over_algorithmic": None if traffic is None else traffic / traffic_alg,
                     "traffic_GBps": None if traffic is None else traffic / period_s / 1e9,
                     "kernel": "k_tick (solver phase launch)", "launches": launches,
                     "algorithmic_bytes": alg, "algorithmic_bytes_per_launch": alg / max(1, launches),
                     "avg_launch_period_us": period_s * 1e6, "kernel_sources_sha256": kernel_source_digest()},
    }
    out["paper_context"] = PAPER_CONTEXT[dim]
    if not args.no_precision_check:
        # accuracy against the float64 oracle at the final state (not timed); a mixed-precision
        # workload also reports the float64 GPU solve of the same system for comparison
        out["err_vs_oracle_fp64"] = oracle_stage_check(pfc, torch, mesh, h, state, r, psibar, tau,
                                                       (1, 0) if prec == 1 else (0,), model=model, schur=schur)
    if not args.no_cpu_baseline and not var:
        out["cpu_baseline"] = run_cpu_baseline(dim, N, jitter, r, psibar, tau, args.seed)
    pfc.pfc_instance_destroy(inst)
    pfc.pfc_mesh_destroy(h)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
