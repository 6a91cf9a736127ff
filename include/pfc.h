/*
 * pfc.h -- C ABI of the MI355X (gfx950) solver for the block-preconditioned
 * FGMRES solve of the Phase-Field Crystal (PFC2) Rosenbrock stage system.
 *
 * The method is that of Praetorius & Voigt, "Development and Analysis of a
 * Block-Preconditioner for the Phase-Field Crystal Equation":
 *   - P1 finite elements on a simplicial mesh: mass M, stiffness K and the
 *     psi^2-weighted mass matrix N(psi) = -3 (psi^2 phi_j, phi_i)  (Section 3);
 *   - the 3x3 block stage matrix of the Ros3Pw Rosenbrock scheme
 *         A^R = [[M, -(1+r)M + 2K + N(psi_k), K], [tau K, m11 M, 0], [0, K, M]]
 *     (eq. rosenbrock_matrix with the PFC2 mobility, K_+ = K, F = 0), with
 *     m11 = 1/gamma for Rosenbrock stages and m11 = 1 for the linearised Euler
 *     system (eq. systemmatrix);
 *   - right-preconditioned flexible GMRES(restart) with modified Gram-Schmidt
 *     (Section 4 and the solver settings of Section 7), its coefficients for
 *     Arnoldi step j taken from one reduction (the lower-triangular system
 *     (I + L) h = V^T w, L the strictly lower Gram matrix of the basis, which
 *     equals modified Gram-Schmidt in exact arithmetic);
 *   - the preconditioner P_CH = P(S_CH) of eq. preconditioner_S with
 *     S_CH = (M + sqrt(delta) K) M^{-1} (M + sqrt(delta) K), delta = sqrt(tau),
 *     applied in five steps with Jacobi-PCG inner solves (Section 4.2,
 *     Table inner_solvers).
 *
 * Conventions shared by every call
 *   - Block vectors of length 3n are stored block by block:
 *       [mu(0..n-1) | psi(0..n-1) | omega(0..n-1)].
 *   - "device" pointers are HIP device allocations of the current device
 *     (e.g. the data of a torch tensor on cuda:0); "host" pointers are
 *     ordinary host memory.  Each argument below says which.
 *   - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *     Calls that take a stream enqueue their work on it and return only when
 *     that work has completed (they are synchronous towards the caller).
 *   - Inputs are owned by the caller and only read during the call; outputs
 *     are written into caller-owned buffers.  Handles are owned by the
 *     library until the matching *_destroy.  A handle must not be used by
 *     two host threads at once.
 *   - The library never aborts and never prints.  Every int-returning call
 *     returns a status code below; on a negative code, pfc_last_error()
 *     returns a message for the calling thread.
 *   - All arithmetic of the outer solver is float64.  In PFC_MIXED precision
 *     the inner PCG solves and their matrix-vector products use float32.
 *   - A solver call (solve, Rosenbrock run, batch, preconditioner apply)
 *     that has not finished after a wall-clock limit returns PFC_ERR_STATE
 *     once the work already enqueued has drained.  The limit is 600 s per
 *     instance (a batch: per instance of the batch), or the value of the
 *     environment variable PFC_TIMEOUT_S, in seconds, read when an instance
 *     is created.
 */
#ifndef PFC_H
#define PFC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define PFC_OK                 0
#define PFC_NOT_CONVERGED      1  /* max_steps reached; x holds the last iterate, info valid */
#define PFC_WARN_TAU_CRITICAL  2  /* converged, but tau >= tau*(r, psibar) of Lemma 3 */
#define PFC_ERR_ARG           -1  /* invalid argument (nothing was enqueued) */
#define PFC_ERR_OOM           -2  /* device or host allocation failed */
#define PFC_ERR_HIP           -3  /* a HIP runtime call failed */
#define PFC_ERR_BREAKDOWN     -4  /* non-finite residual or input */
#define PFC_ERR_ADMISSION     -5  /* request does not fit the server's memory budget */
#define PFC_ERR_STATE         -6  /* call not valid in the handle's current state */

enum { PFC_FP64 = 0, PFC_MIXED = 1 };
enum { PFC_INIT_GIVEN = 0, PFC_INIT_CONSISTENT = 1 };
enum { PFC_OP_M = 0, PFC_OP_K = 1 };
enum { PFC_MODEL_PFC2 = 0, PFC_MODEL_PFC1 = 1 };
enum { PFC_GAMMA_SCALE_ROW = 0, PFC_GAMMA_LITERAL = 1 };

typedef struct pfc_mesh pfc_mesh;
typedef struct pfc_instance pfc_instance;
typedef struct pfc_server pfc_server;

/* Solver options.  Fill with pfc_opts_default, then override fields.
 *   precision     PFC_FP64 or PFC_MIXED (float32 inner PCG, float64 FGMRES)
 *   restart       FGMRES restart length m, 1..32 (the paper uses 30)
 *   max_steps     cap on the total number of Arnoldi steps of one solve
 *   outer_tol     relative residual ||b - A^R x||_2 / ||b||_2 to reach (1e-8)
 *   inner_tol     relative residual of every inner PCG solve (1e-3, Table inner_solvers)
 *   inner_maxit   iteration cap of an inner PCG solve (500)
 *   shared_ops    0: store M + delta K and M + sqrt(delta) K per instance;
 *                 1: form them on the fly from the mesh's M and K (less memory,
 *                 more bytes per iteration; useful when many instances share a mesh)
 *   rows_per_thread  rows of the mesh handled per thread in each phase (1..8; 0 means 1)
 *   max_run_steps capacity of per-stage info records of a Rosenbrock run (steps)
 *   ticks_per_graph  solver phases captured per replayed graph (0: 64, or in
 *                 pfc_batch_run the autotuning table's value for the batch)
 *   single_reduction 0: inner PCG in the standard form (two reductions, two
 *                 launches per iteration); 1: the Chronopoulos-Gear form of the
 *                 same iteration (one reduction, one launch per iteration;
 *                 identical iterates in exact arithmetic)
 *   schur_variant 0: Schur complement approximated by S_CH (steps 3.1 and 3.2);
 *                 1: by S_D = M - 2 delta K + delta K M_D^{-1} K, M_D = diag(M)
 *                 (Section 4.1), one PCG solve on the second-ring pattern
 *   sd_iters      iteration count of the S_D solve (20, Table inner_solvers)
 *   model         PFC_MODEL_PFC2 (H^{-1} flow: K_+ = K, F = 0; the default) or
 *                 PFC_MODEL_PFC1 (Wasserstein flow with mobility psi^+ =
 *                 psi - psi_min, Section 2): block (1,0) of A^R becomes
 *                 tau K_+(psi_k), block (1,1) m11 M + tau F(mu_k), with
 *                 K_+(psi)_ij = (psi^+ grad phi_j, grad phi_i) and
 *                 F(mu)_ij = (phi_j grad mu, grad phi_i) (eq. rosenbrock_matrix);
 *                 the stage right-hand side carries -tau K_+(psi_i) mu_i; P_CH is
 *                 built for the time step M0 tau_s with M0 the mean of psi^+
 *                 (constant-mobility approximation, Section 4).  M0 is taken
 *                 from psi_k for a single solve and once from the initial state
 *                 for a Rosenbrock run (the scheme conserves the integral of psi).
 *                 PFC1 needs the element geometry: meshes from pfc_mesh_create_p1.
 *   psi_min       lower bound of the order parameter in the mobility (-1.5)
 *   grid_columns  1 (default): on periodic grid meshes (n = N^dim nodes
 *                 numbered x + N (y + N z), neighbours at most one step away
 *                 per direction) the solver kernel computes the column of each
 *                 stored entry from its row instead of reading it; same
 *                 columns in the same order, so the same results bit for bit.
 *                 0: always read the stored columns.  A launch that serves
 *                 several instances computes the columns only when all of
 *                 them allow it and all their meshes are such grids.
 *   gamma_mode    how the preconditioner meets the factor m11 of block (1,1)
 *                 (the paper derives P for m11 = 1 and uses it unchanged):
 *                 PFC_GAMMA_SCALE_ROW (default): block row 1 of A^R and b is
 *                 multiplied by 1/m11, which gives [tau/m11 K, M, 0], and P_CH
 *                 is built for tau_s = tau/m11; the solution is unchanged and
 *                 the first block column matches the one P was derived for.
 *                 PFC_GAMMA_LITERAL: the unscaled system with P_CH(tau).
 *                 Both coincide for m11 = 1.  Residuals are reported for the
 *                 unscaled system either way.
 *   inner_fixed   iteration counts of the five inner solves (1), (2), (3.1),
 *                 (3.2), (5) of every preconditioner application; 0 (the
 *                 default) runs that solve to inner_tol.  With S_D, entry 2 is
 *                 the S_D solve (overrides sd_iters) and entry 3 is unused.
 *   pcg_steps_per_launch  2 (default): where the launch allows it, the five
 *                 inner solves run two PCG iterations per solver launch in the
 *                 s-step form (basis p, Tp, T^2 p, u, Tu of T = D^{-1} C, one
 *                 reduction of their D-weighted Gram matrix, halo rows staged
 *                 in LDS): same iterates and the same stopping decisions as the
 *                 standard iteration in exact arithmetic, and the same count
 *                 of iterations.  It applies to single_reduction = 1
 *                 instances with grid_columns = 1 and rows_per_thread <= 1:
 *                 on 2D periodic grid meshes of side a multiple of 64 in
 *                 either precision (a workgroup's rows are a block of 64 x 16
 *                 grid points), also in launches that serve many instances
 *                 (whose other instances run one iteration per launch in
 *                 them; the server gives its requests this form where it
 *                 applies); in launches that serve the instance alone, on
 *                 other 2D periodic grid
 *                 meshes in float64 (a workgroup's rows are a range of rows)
 *                 and on 3D periodic grid meshes of side 64 in PFC_MIXED (a
 *                 block of 4 x 4 grid lines).  In PFC_MIXED the inner
 *                 iterations run in float32.  Elsewhere, and with 1, one
 *                 iteration per launch.  Results of the two forms differ by
 *                 rounding: an instance gives the same bits alone and in a
 *                 batch or a served mix with 1, and with 2 in the block form. */
typedef struct pfc_opts {
    int struct_size;
    int precision;
    int restart;
    int max_steps;
    double outer_tol;
    double inner_tol;
    int inner_maxit;
    int shared_ops;
    int rows_per_thread;
    int max_run_steps;
    int ticks_per_graph;
    int single_reduction;
    int schur_variant;
    int sd_iters;
    int model;
    double psi_min;
    int grid_columns;
    int gamma_mode;
    int inner_fixed[5];
    int pcg_steps_per_launch;
} pfc_opts;

/* Result record of one stage solve.
 *   status        PFC_OK / PFC_NOT_CONVERGED / PFC_ERR_BREAKDOWN for this solve
 *   outer_iters   Arnoldi steps (the iteration count of the paper's tables)
 *   cycles        FGMRES cycles (restarts + 1)
 *   inner_applies preconditioner applications
 *   inner_total   PCG iterations summed over all applications and steps
 *   inner_max     largest PCG count seen in each of the five steps (1, 2, 3.1, 3.2, 5)
 *   est_rel_res   last Givens estimate |g_{k}| / ||b_scaled||
 *   true_rel_res  ||b - A^R x||_2 / ||b||_2 recomputed in float64
 *   t_solve       seconds of device time from the solve's first launch to its
 *                 last (the device's constant 100 MHz clock; in a batch or a
 *                 served mix the launches are shared with the other solves) */
typedef struct pfc_solve_info {
    int status;
    int outer_iters;
    int cycles;
    int inner_applies;
    long long inner_total;
    int inner_max[5];
    int reserved;
    double est_rel_res;
    double true_rel_res;
    double t_solve;
} pfc_solve_info;

/* Recorded iteration structure of one FGMRES solve, for replay: the length
 * of each cycle and, for each preconditioner application in order, the five
 * inner PCG iteration counts.  Host memory. */
typedef struct pfc_schedule {
    int n_cycles;
    const int* cycle_len;     /* [n_cycles] */
    int n_applies;
    const int* inner_counts;  /* [5 * n_applies] */
} pfc_schedule;

/* ---- misc --------------------------------------------------------------- */
const char* pfc_status_str(int status);
const char* pfc_last_error(void);
void pfc_opts_default(pfc_opts* opts);
/* Lemma 3: tau* = 27 / (2 (sqrt(a) - 1)(sqrt(a) + 2)^2), a = 1 - 3 r - 9 psibar^2;
 * +infinity when psibar^2 >= -r/3.  Pure host arithmetic. */
double pfc_tau_critical(double r, double psibar);

/* ---- meshes ---------------------------------------------------------------
 * A mesh holds the shared sparsity pattern of M, K and N(psi) (the P1 pattern:
 * every pair of nodes of a common simplex, diagonal included), the values of
 * M and K, and the element lists needed to reassemble N(psi) and the cubic
 * load (psi_h^3, phi_i) in place.
 *
 * pfc_mesh_create_p1: assemble M and K on the GPU from simplices (Section 3):
 *   M_ij = (phi_j, phi_i), K_ij = (grad phi_j, grad phi_i), exact for P1.
 *   dim          2 (triangles) or 3 (tetrahedra)
 *   n            number of nodes
 *   n_elem       number of simplices
 *   elem_nodes   host int32 [n_elem * (dim+1)], node indices in [0, n), distinct per simplex
 *   elem_coords  host float64 [n_elem * (dim+1) * dim], vertex coordinates of
 *                each simplex, unwrapped across periodic boundaries
 *   out          receives the handle
 * Returns PFC_ERR_ARG for out-of-range or repeated nodes, a node that belongs
 * to no simplex, non-finite coordinates, or a degenerate simplex: one whose
 * |det(x_1 - x_0, ..., x_dim - x_0)| is at most 1e-12 times the product of
 * the edge lengths |x_a - x_0|.  All of these are checked on the host before
 * any device call. */
int pfc_mesh_create_p1(int dim, int n, int n_elem, const int32_t* elem_nodes,
                       const double* elem_coords, pfc_mesh** out);

/* pfc_mesh_create_p2: quadratic Lagrange elements (Section 3 with p = 2, the
 * degree of Tables 3-5).  The local basis on a simplex with barycentric
 * coordinates l_0..l_dim is l_a (2 l_a - 1) at the vertices and 4 l_i l_j at
 * the edges; M, K, N(psi) and the cubic load are integrated exactly.
 *   elem_nodes   host int32 [n_elem * q], q = 6 (2D) or 10 (3D): the dim+1
 *                vertex nodes, then the edge nodes of the local vertex pairs
 *                (0,1), (1,2), (0,2) in 2D and (0,1), (1,2), (0,2), (0,3),
 *                (1,3), (2,3) in 3D
 *   elem_coords  host float64 [n_elem * (dim+1) * dim], vertex coordinates
 *                (straight-sided simplices)
 *   n_elem       at most 2^22
 * Other arguments and errors as pfc_mesh_create_p1.  The PFC1 model needs a P1
 * mesh. */
int pfc_mesh_create_p2(int dim, int n, int n_elem, const int32_t* elem_nodes,
                       const double* elem_coords, pfc_mesh** out);

/* pfc_mesh_create_csr: take M and K from the caller in CSR form (host arrays).
 *   row_ptr [n+1], col_idx [nnz]: sorted column indices per row, diagonal
 *   present, pattern structurally symmetric and containing every node pair
 *   of every simplex; M_val, K_val [nnz] float64; elem_nodes as above;
 *   elem_vol [n_elem] simplex measures |T| (used by the reassembly of N and
 *   of the cubic load).  PFC_ERR_ARG on any violation. */
int pfc_mesh_create_csr(int dim, int n, int nnz, const int32_t* row_ptr, const int32_t* col_idx,
                        const double* M_val, const double* K_val, int n_elem,
                        const int32_t* elem_nodes, const double* elem_vol, pfc_mesh** out);

/* pfc_mesh_create_csr_device: the same with every array in device memory
 * (row_ptr, col_idx, M_val, K_val, elem_nodes, elem_vol: device pointers of
 * the sizes above).  The arrays are copied to the host for the validation of
 * pfc_mesh_create_csr (synchronously, on the null stream); PFC_ERR_HIP if a
 * pointer is not readable device memory. */
int pfc_mesh_create_csr_device(int dim, int n, int nnz, const int32_t* row_ptr, const int32_t* col_idx,
                               const double* M_val, const double* K_val, int n_elem,
                               const int32_t* elem_nodes, const double* elem_vol, pfc_mesh** out);

/* Sizes of a mesh; any pointer may be NULL. */
int pfc_mesh_query(const pfc_mesh* mesh, int* dim, int* n, int* nnz, int* n_elem);

/* Side N of a periodic grid mesh whose columns the solver kernel computes from
 * the row (pfc_opts.grid_columns), or 0 for any other mesh.  N: host int. */
int pfc_mesh_grid_side(const pfc_mesh* mesh, int* N);

/* Copy the pattern and the values of M and K out in CSR order (host arrays of
 * n+1, nnz, nnz, nnz entries; any of them may be NULL). */
int pfc_mesh_export_csr(const pfc_mesh* mesh, int32_t* row_ptr, int32_t* col_idx,
                        double* M_val, double* K_val);

void pfc_mesh_destroy(pfc_mesh* mesh);

/* ---- mesh-level operators (device pointers) ------------------------------ */
/* y = M x (which = PFC_OP_M) or y = K x (PFC_OP_K); x, y device float64 [n]. */
int pfc_spmv(const pfc_mesh* mesh, int which, const double* x, double* y, void* stream);
/* Values of N(psi) = -3 (psi_h^2 phi_j, phi_i) in CSR order of the mesh pattern
 * (Section 3, exact quadrature); psi device [n], N_csr device [nnz]. */
int pfc_assemble_N(const pfc_mesh* mesh, const double* psi, double* N_csr, void* stream);
/* Cubic load g_i = (psi_h^3, phi_i) (the psi^3 term of the operator F,
 * Section 3.1); psi, g device [n]. */
int pfc_load_psi3(const pfc_mesh* mesh, const double* psi, double* g, void* stream);

/* ---- instances ------------------------------------------------------------
 * An instance owns all device memory of one solver on one mesh: the FGMRES
 * basis (restart+1 vectors V and restart vectors Z of length 3n, float64),
 * the per-tau operator values, N(psi_k), the Rosenbrock state and the PCG
 * work vectors.  Everything is allocated at creation. */
size_t pfc_instance_footprint(const pfc_mesh* mesh, const pfc_opts* opts);
int pfc_instance_create(pfc_mesh* mesh, const pfc_opts* opts, pfc_instance** out);
void pfc_instance_destroy(pfc_instance* inst);

/* One stage solve, the hot path: A^R x = rhs with A^R built from the mesh's
 * M, K and N(psi_k) reassembled from psi_k, parameters r and tau, and the mass
 * coefficient m11 of block row 1 (1/gamma for Ros3Pw stages, 1 for Euler).
 * FGMRES starts from x = 0.  Block row 1 is divided by m11 before the solve
 * so that P_CH, derived for m11 = 1, is built with tau/m11; the solution is
 * unchanged and convergence is judged on the unscaled system.
 *   psi_k   device float64 [n]
 *   rhs     device float64 [3n]
 *   x       device float64 [3n] (output)
 *   psibar  used only for the tau* check of Lemma 3
 *   replay  NULL, or a host schedule: run exactly that iteration structure
 *           (fixed cycle lengths and inner counts) instead of the tolerances
 *   info    host record (may be NULL)
 * Returns the solve's status (PFC_WARN_TAU_CRITICAL replaces PFC_OK when
 * tau >= tau*(r, psibar)). */
int pfc_solve(pfc_instance* inst, const double* psi_k, double r, double psibar, double tau,
              double m11, const double* rhs, double* x, const pfc_schedule* replay,
              pfc_solve_info* info, void* stream);
/* The same stage solve taking the full step state x_k (device float64 [3n],
 * [mu_k | psi_k | omega_k]): required for PFC_MODEL_PFC1 instances, whose
 * stage matrix also holds K_+(psi_k) and F(mu_k) (eq. rosenbrock_matrix) and
 * whose P_CH uses the mobility mean M0 of psi_k; pfc_solve returns
 * PFC_ERR_ARG for them.  For PFC2 it equals pfc_solve with psi_k = x_k + n. */
int pfc_solve_x(pfc_instance* inst, const double* x_k, double r, double psibar, double tau, double m11,
                const double* rhs, double* x, const pfc_schedule* replay, pfc_solve_info* info, void* stream);

/* After a pfc_solve without replay: copy the recorded inner counts of its
 * preconditioner applications (5 per application, in order) into the host
 * array counts of capacity cap applications; *n_applies receives the count. */
int pfc_last_inner_counts(const pfc_instance* inst, int* counts, int cap, int* n_applies);

/* Launch statistics of the instance's most recent solve or run (for
 * pfc_rosenbrock_adaptive: summed over all its attempted steps): number of
 * solver-kernel launches issued (replayed graphs times launches per graph,
 * including launches that found the instance finished) and number of graph
 * replays.  Host outputs; either may be NULL. */
int pfc_instance_launch_stats(const pfc_instance* inst, long long* launches, long long* graphs);

/* Launch configuration an instance runs with when a launch serves it alone
 * (host outputs; any may be NULL): its team of workgroups, rows per thread,
 * PCG iterations per solver launch (2 where the two-iteration form applies,
 * see pcg_steps_per_launch, else 1) and whether the solver kernel computes the
 * mesh's columns from the row (1) or reads them (0).  In a launch that serves
 * several instances (batches, the server) an instance runs two PCG iterations
 * per launch in the 2D block form and one otherwise (see
 * pcg_steps_per_launch). */
int pfc_instance_config(const pfc_instance* inst, int* team_size, int* rows_per_thread, int* pcg_steps_per_launch,
                        int* grid_columns);

/* n_steps Ros3Pw steps (eqs. rosenbrock, rosenbrock-update; Table
 * rosenbrock_scheme) of the PFC2 system from state = (mu, psi, omega):
 * per step N(psi_k) is reassembled in place, then for i = 1, 2, 3 the stage
 * right-hand side b_i^R is formed and A^R y_i = b_i^R solved, and finally
 * x_{k+1} = x_k + sum m_j y_j.
 *   state     device float64 [3n], in/out
 *   init      PFC_INIT_GIVEN: use state as given; PFC_INIT_CONSISTENT: replace
 *             mu and omega by the values that zero blocks 0 and 2 of F at psi
 *             (M omega = -K psi, M mu = (1+r) M psi - 2 K psi - K omega + g(psi))
 *   replays   NULL, or a host array of 3*n_steps schedules, one per stage solve
 *   per_stage host array of 3*n_steps records (may be NULL)
 * Returns the worst status over all stage solves. */
int pfc_rosenbrock_run(pfc_instance* inst, double* state, double r, double psibar, double tau,
                       int n_steps, int init, const pfc_schedule* replays,
                       pfc_solve_info* per_stage, void* stream);

/* Adaptive Ros3Pw run from t = 0 to t_end (Section 3.1: embedded solution
 * x_hat = x_k + sum mhat_j y_j of Table rosenbrock_scheme, order 2).  After each
 * step, err = RMS over the psi block of (psi_{k+1} - psi_hat) / (atol + rtol
 * max(|psi_k|, |psi_{k+1}|)); the step is accepted if err <= 1 (otherwise the
 * state is restored), and tau <- tau * min(facmax, max(0.2, 0.9 err^(-1/3)))
 * with facmax = 1 for the step after a rejection, 5 otherwise.  A step whose
 * stage solves do not all converge (within the instance's max_steps) is
 * rejected without an error estimate and retried with 0.2 tau.  The last step
 * is shortened to end at t_end.
 *   state       device float64 [3n], in/out
 *   tau0        first trial step; max_attempts caps accepted + rejected steps
 *   taus        host array of capacity max_attempts: accepted step sizes in order
 *   n_accepted, n_rejected  host outputs (n_rejected counts both kinds of rejection)
 *   infos       host array of capacity 3 * max_attempts, or NULL: the records
 *               of the three stage solves of every attempted step (accepted
 *               and rejected, in order)
 * Returns PFC_NOT_CONVERGED if t_end was not reached within max_attempts, a
 * negative code on failure, otherwise the worst status of the accepted steps'
 * stage solves. */
int pfc_rosenbrock_adaptive(pfc_instance* inst, double* state, double r, double psibar, double tau0, double t_end,
                            double rtol, double atol, int max_attempts, int init, double* taus, int* n_accepted,
                            int* n_rejected, pfc_solve_info* infos, void* stream);

/* Operator-level entry points of the hot path (device pointers). */
/* out = A^R y with N(psi_k) reassembled from psi_k; y, out [3n]. */
int pfc_apply_AR(pfc_instance* inst, const double* psi_k, double r, double tau, double m11,
                 const double* y, double* out, void* stream);
/* out = A^R y at the full state x_k [3n] (N(psi_k), and for PFC1 K_+(psi_k)
 * and F(mu_k), reassembled); the form PFC_MODEL_PFC1 instances require. */
int pfc_apply_AR_x(pfc_instance* inst, const double* x_k, double r, double tau, double m11,
                   const double* y, double* out, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid allocation): out = A^R y as
 * pfc_apply_AR, on a PFC2 mesh without an instance.  N(psi_k) is reassembled
 * into a library-owned static device array of PFC_NOALLOC_MAX_ENTRIES float64
 * values (32 MiB; each GPU the library runs on holds its own copy until the
 * process ends) instead of an instance's memory; the call performs no device
 * allocation or free.
 *   mesh      any mesh whose stored pattern has at most PFC_NOALLOC_MAX_ENTRIES
 *             entries (2D 512^2: 1.84M, 3D 64^3: 3.93M); a larger one returns
 *             PFC_ERR_ARG before anything is enqueued
 *   psi_k     device float64 [n]; y, out device float64 [3n]
 * Unlike the other calls it only enqueues its two kernels on `stream` and
 * returns (so it can be captured into a graph); the caller synchronises.
 * The first call on a device resolves the array's address (no allocation);
 * make it outside graph capture.  Every call on a GPU uses that GPU's one
 * array: calls that overlap on one GPU (other streams, other host threads)
 * race on it; calls on one stream are ordered and safe. */
#define PFC_NOALLOC_MAX_ENTRIES (1 << 22)
int pfc_apply_AR_noalloc(const pfc_mesh* mesh, const double* psi_k, double r, double tau, double m11,
                         const double* y, double* out, void* stream);

/* z = P_CH^{-1} v with parameter tau_s (the time step the preconditioner is
 * built for: tau/m11 for PFC2, M0 tau/m11 for PFC1; used as given): the five steps (1), (2), (3.1), (3.2), (4), (5) of Section 4.2 with
 * Jacobi-PCG inner solves.  fixed_counts: NULL (tolerance inner_tol) or host
 * int[5] exact iteration counts; counts_out: host int[5] or NULL. */
int pfc_apply_pch(pfc_instance* inst, double tau_s, const double* v, double* z,
                  const int* fixed_counts, int* counts_out, void* stream);
/* Stage right-hand side b_i^R of stage `stage` (1..3) at step state x_k and
 * earlier stage solutions ys = [y_1 | y_2 | y_3] (device, 3 x 3n; only
 * y_1..y_{stage-1} read): b0 = F0(x_i), b1 = tau F1(x_i) + sum c_ij M y_j^psi,
 * b2 = F2(x_i), x_i = x_k + sum a_ij y_j, with F1(x) = -K mu (PFC2) or
 * -K_+(psi) mu (PFC1, formed element by element at the stage state).  b device [3n]. */
int pfc_stage_rhs(pfc_instance* inst, const double* x_k, const double* ys, int stage,
                  double r, double tau, double* b, void* stream);

/* ---- batches -------------------------------------------------------------
 * Rosenbrock runs of `count` instances (same precision) advanced together:
 * every launch of the solver kernel advances every unfinished instance by one
 * phase, each instance on its own team of workgroups.
 *   insts    host array of instance handles (distinct)
 *   states   host array of device pointers, states[i] float64 [3 n_i]
 *   r, psibar, tau  host arrays [count]
 *   infos    host array of count*3*n_steps records (may be NULL), instance-major */
int pfc_batch_run(pfc_instance* const* insts, int count, double* const* states,
                  const double* r, const double* psibar, const double* tau, int n_steps,
                  int init, pfc_solve_info* infos, void* stream);

/* ---- autotuning -------------------------------------------------------------
 * The launch configuration of the solver kernel (rows per thread, launches per
 * captured graph, PCG iterations per launch (one row per thread), computed or
 * read grid columns, stored or on-the-fly M + c K operators) is chosen by
 * measurement: pfc_autotune times one Rosenbrock step of `count` instances of
 * a mesh on synthetic states (psi = -0.3 + U[-0.01, 0.01] from a counter-based
 * generator, consistent mu and omega, r = -0.35, tau = 0.5) for candidate
 * configurations, coordinate descent from the defaults one knob at a time, and
 * keeps the fastest in a process-wide table.  The table is keyed by (device
 * architecture, dim, n, stored entries per row, precision, count); a lookup
 * for `count` instances takes the entry with the largest tuned count <= count.
 * pfc_batch_run takes its launches per graph from the table when the
 * instances' ticks_per_graph is 0, and a server created with `tuned` takes
 * each request's rows per thread from its mixed-batch entries.  The table is saved to and loaded
 * from a JSON file: {"format": "pfc-tune-1", "entries": [{...}, ...]}. */
typedef struct pfc_tune_entry {
    int struct_size;
    char arch[32];            /* device architecture, e.g. "gfx950" */
    int dim, n, z, precision, count;                 /* key */
    int rows_per_thread, ticks_per_graph, pcg_steps_per_launch, grid_columns, shared_ops;  /* choice */
    double ms_per_step;       /* one Rosenbrock step of all `count` instances with the choice */
    double ms_default;        /* the same with the default options */
    int candidates;           /* configurations timed */
    int from_cache;           /* 1: returned from the table, not measured by this call */
} pfc_tune_entry;

/* Tune (or, unless force, return the table's entry for exactly this count).
 * mesh and precision as for an instance; count >= 1 instances per launch.
 * Allocates and frees `count` instances per candidate; PFC_ERR_OOM if even
 * the default configuration does not fit 80% of the free device memory.
 * out: host record.  Synchronous on `stream`. */
int pfc_autotune(pfc_mesh* mesh, int precision, int count, int force, pfc_tune_entry* out, void* stream);
/* The same for batches that mix several meshes (the server's case): `count`
 * instances dealt round robin over meshes[0..n_meshes-1], only rows per thread
 * searched (the other knobs keep their defaults).  Instances that take the 2D
 * block form at one row per thread keep one row per thread and two PCG
 * iterations per launch, as in the server; the searched value applies to the
 * others.  The entry's key has dim = n = z = 0 ("a mix"), whatever the meshes;
 * tuning another mix replaces it. */
int pfc_autotune_mix(pfc_mesh* const* meshes, int n_meshes, int precision, int count, int force, pfc_tune_entry* out,
                     void* stream);
/* Table entry for `count` instances of a mesh with these sizes (arch: NULL
 * for the current device's); PFC_ERR_STATE if the table has none.  Host only
 * when arch is given. */
int pfc_tune_lookup(const char* arch, int dim, int n, int z, int precision, int count, pfc_tune_entry* out);
/* Merge the entries of a cache file into the table (an entry with the same
 * key and count replaces the table's); PFC_ERR_ARG if the file cannot be read
 * or is not such a cache. */
int pfc_tune_load(const char* path);
/* Write the whole table to `path` (atomically, through a temporary file). */
int pfc_tune_save(const char* path);
void pfc_tune_clear(void);

/* ---- serving --------------------------------------------------------------
 * A server runs a library-owned thread that keeps a set of active requests
 * resident on the GPU and advances them together (continuous batching at the
 * granularity of solver phases).  Requests are admitted when their instance
 * footprint fits into the remaining budget and a slot is free; finished
 * requests are retired and their memory is released.
 *   hbm_budget  bytes of device memory the server may hold for instances
 *   max_slots   maximum number of concurrently active requests
 *   precision   PFC_FP64 or PFC_MIXED
 *   ticks_per_graph  as in pfc_opts (0: default)
 *   rows_per_thread  rows per thread of the request instances, 1..8, or 0
 *               (the default): chosen per request at admission.  A request
 *               that takes the 2D block form of two PCG iterations per launch
 *               at one row per thread (see pcg_steps_per_launch; a server with
 *               more than one slot) gets one; any other request one row per
 *               thread while the active requests and the new one fit into one
 *               round of resident workgroups (CUs x 1024 rows), two beyond.
 *               More rows per thread give each request fewer, longer
 *               workgroups: more throughput when many requests share the GPU,
 *               longer solves when few do.
 *   tuned       1: with rows_per_thread 0, take the rows per thread of the
 *               requests without the block form from the autotuning table's
 *               mixed-batch entry (pfc_autotune_mix, which times its batches
 *               with the same split) for the number of active requests
 *               including it, and use the rule above only where the table
 *               has no such entry; 0: the rule.
 *   n_steps ... Rosenbrock steps per request (set per request) */
typedef struct pfc_server_opts {
    int struct_size;
    int precision;
    size_t hbm_budget;
    int max_slots;
    int ticks_per_graph;
    int rows_per_thread;
    int tuned;
} pfc_server_opts;

typedef struct pfc_result {
    uint64_t req_id;
    int status;
    int n_stages;
    double t_submit;     /* seconds, library clock */
    double t_admit;
    double t_done;
    double* state;       /* host float64 [3n] final state; owned by the caller after poll */
    pfc_solve_info* infos; /* host [n_stages]; owned by the caller after poll */
} pfc_result;

int pfc_server_create(const pfc_server_opts* opts, pfc_server** out);
/* Submit a request: Rosenbrock run of n_steps on `mesh` (kept alive by the
 * caller until the result is polled) from psi0 (host float64 [n]) with
 * consistent initial mu, omega.  Returns PFC_ERR_ADMISSION if the request can
 * never fit the budget. */
int pfc_server_submit(pfc_server* srv, pfc_mesh* mesh, double r, double psibar, double tau,
                      const double* psi0, int n_steps, uint64_t req_id);
/* Collect up to max finished results (non-blocking); *n_out receives the count.
 * The state and infos arrays of each result are malloc'ed; free them with
 * pfc_result_free. */
int pfc_server_poll(pfc_server* srv, pfc_result* out, int max, int* n_out);
void pfc_result_free(pfc_result* res);
/* Block until every submitted request has finished. */
int pfc_server_drain(pfc_server* srv);
double pfc_server_clock(const pfc_server* srv);
void pfc_server_destroy(pfc_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* PFC_H */
