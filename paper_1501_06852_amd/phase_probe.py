"""Launches per solver phase and where a launch spends its time (diagnostics).

Runs one Ros3Pw step of a benchmark workload on the instrumented build of the
library (`python -m paper_1501_06852_amd.build --timing` writes
libpfc_timing.so; PFC_TICK_TIMING), in which workgroup rank 0 of every solver
launch records wall-clock stamps (100 MHz) at its entry, after the prologue's
loads, after the transition, after the phase's work and at its exit, and the
two-iteration PCG forms on 2D grids add stamps inside the phase.  Prints one
JSON object: the launches of each phase and the median time of each part of a
launch, in microseconds.

    python -m paper_1501_06852_amd.phase_probe DIM N PRECISION [DEGREE]

e.g. `2 512 0` (2D 512^2 jittered grid, float64) or `3 64 1` (3D 64^3, mixed).
The workload parameters are those of the benchmark (2D: r = -0.35,
psibar = -0.3, tau = 1; 3D: r = -0.3, psibar = -0.25, tau = 0.5).
"""
from __future__ import annotations

import ctypes as C
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

PHASES = {0: "DONE", 1: "START", 2: "SOLVE_INIT", 3: "RB_BEGIN", 4: "RB_RHS", 5: "RB_UPDATE", 6: "PCG_SETUP",
          7: "PCG_A", 8: "PCG_B", 9: "ASPMV", 10: "GS_UPDATE", 11: "UPDATE_X", 12: "TRUE_RES", 13: "PCH_OUT",
          14: "CG_INIT", 15: "CG_ITER", 16: "SCG_ITER"}
REC = 14          # 64-bit words per launch record
TICK_US = 0.01    # wall clock: 100 MHz


def main(argv):
    if len(argv) < 3:
        print(__doc__)
        return 2
    dim, N, prec = int(argv[0]), int(argv[1]), int(argv[2])
    deg = int(argv[3]) if len(argv) > 3 else 1
    from . import build
    os.environ.setdefault("PFC_LIBRARY", build.LIB_TIMING)
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch
    import workloads as wl
    from . import pfc
    lib = pfc._lib
    if not hasattr(lib, "pfc_debug_trace"):
        raise SystemExit(f"{pfc.LIB_PATH} is not the instrumented build (python -m paper_1501_06852_amd.build --timing)")
    lib.pfc_debug_trace.argtypes = [C.c_void_p, C.c_ulonglong]
    lib.pfc_debug_trace.restype = C.c_int
    lib.pfc_debug_trace_count.restype = C.c_ulonglong

    mesh = wl.make_mesh(dim, N, jitter=0.2 if dim == 2 else 0.0, seed=0)
    if deg == 2:
        mesh = wl.p2_mesh(mesh)
        h = pfc.pfc_mesh_create_p2(dim, mesh.n, mesh.elem_nodes, mesh.elem_coords)
    else:
        h = pfc.pfc_mesh_create_p1(dim, mesh.n, mesh.elem_nodes, mesh.elem_coords)
    n = mesh.n
    inst = pfc.pfc_instance_create(h, pfc.pfc_opts_default(precision=prec))
    r, psibar, tau = (-0.35, -0.3, 1.0) if dim == 2 else (-0.3, -0.25, 0.5)
    state = torch.zeros(3 * n, dtype=torch.float64, device="cuda:0")
    state[n:2 * n] = torch.tensor(wl.psi0(n, psibar, 0.01, seed=0), dtype=torch.float64, device="cuda:0")
    pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau, 1, pfc.PFC_INIT_CONSISTENT)   # warm-up step
    cap = 200000
    buf = torch.zeros(REC * cap, dtype=torch.int64, device="cuda:0")
    if lib.pfc_debug_trace(C.c_void_p(buf.data_ptr()), cap) != 0:
        raise SystemExit("pfc_debug_trace failed")
    pfc.pfc_rosenbrock_run(inst, n, state, r, psibar, tau, 1, pfc.PFC_INIT_GIVEN)
    torch.cuda.synchronize()
    k = min(int(lib.pfc_debug_trace_count()), cap)
    rec = buf[:REC * k].view(k, REC).cpu().numpy()
    phase = rec[:, 0] & 0xff
    rank = (rec[:, 0] >> 8) & 0xffffffff
    t = rec.astype(np.float64)
    own = rank == 0
    med = lambda a, b, m: float(np.median(t[m, b] - t[m, a])) * TICK_US   # noqa: E731
    out = {"workload": {"dim": dim, "N": N, "precision": prec, "degree": deg, "n": n},
           "launches": int(own.sum()), "phases": {}}
    for p in sorted(set(phase[own].tolist())):
        m = own & (phase == p)
        d = {"launches": int(m.sum()), "prologue_us": med(1, 2, m), "transition_us": med(2, 3, m),
             "work_us": med(3, 4, m), "tail_us": med(4, 5, m), "total_us": med(1, 5, m)}
        # stamps inside the two-iteration phase (2D forms): rec[8..11] in the phase, rec[12] after the Gram
        # sums of the previous launch, rec[13] after the transition
        ss = m & (rec[:, 8] >= rec[:, 3]) & (rec[:, 11] >= rec[:, 8]) & (rec[:, 12] >= rec[:, 2])
        if ss.sum():
            d["two_iteration_parts_us"] = {"gram_sums_after_prologue": med(2, 12, ss), "transition": med(12, 13, ss),
                                           "new_p_u_on_frames": med(3, 8, ss), "T_p_on_frame": med(8, 9, ss),
                                           "own_rows_T_u_T2p_products": med(9, 10, ss),
                                           "workgroup_sums_and_store": med(10, 11, ss)}
        out["phases"][PHASES.get(int(p), str(int(p)))] = d
    entries = np.sort(t[own, 1])
    out["launch_period_median_us"] = float(np.median(np.diff(entries))) * TICK_US
    print(json.dumps(out, indent=1))
    pfc.pfc_instance_destroy(inst)
    pfc.pfc_mesh_destroy(h)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
