// Internal layout of meshes, instances and the solver state machine.
//
// Device data layout (all arrays in HBM, 256-byte aligned):
//   * the shared P1 pattern of M, K, N is stored as SELL-64: rows are grouped
//     in slices of 64 consecutive rows (one wavefront), each slice padded to
//     its longest row and stored column-major, so entry k of the rows of a
//     slice is one coalesced 64-lane access.  Padded entries of real rows
//     point at the row itself with value 0; rows >= n point at row 0.
//   * value arrays (M, K, N, M + delta K, M + sqrt(delta) K) share that layout;
//   * vectors of the 3x3 block system are [mu | psi | omega], n each.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pfc.h"

#ifndef PFC_WAVES
#define PFC_WAVES 16
#endif
#define PFC_WG (PFC_WAVES * 64)
#define PFC_SLICE 64
#define PFC_MAXM 32
#define PFC_NSTEPS_P 5

// Solver phases.  A phase is the work done by one launch of the solver
// kernel for one instance; the next phase is chosen from the reductions of
// the previous one at the start of the following launch.
enum {
  PH_DONE = 0,
  PH_START,       // job just submitted; no work
  PH_SOLVE_INIT,  // W = b_scaled, X = 0, partials ||b||^2, ||b_s||^2
  PH_RB_BEGIN,    // N(psi_k) reassembled in place
  PH_RB_RHS,      // stage right-hand side b_i, then as SOLVE_INIT
  PH_RB_UPDATE,   // x_{k+1} = x_k + sum m_j y_j
  PH_PCG_SETUP,   // right-hand side of inner solve `kind`, r = rhs, x = 0
  PH_PCG_A,       // p = D^{-1} r + beta p_old, q = C p, partial (p, q)
  PH_PCG_B,       // x += alpha p, r -= alpha q, partials (r, r), (r, D^{-1} r)
  PH_ASPMV,       // w = A_s z_j; Gram partials (w, v_i) i <= j, (v_j, v_k) k < j, (w, w)
  PH_GS_UPDATE,   // w -= sum_i h_i v_i (modified Gram-Schmidt coefficients), partial (w, w)
  PH_UPDATE_X,    // x += Z y
  PH_TRUE_RES,    // r = b - A^R x, partials ||r||^2, ||r_s||^2; W = r_s
  PH_PCH_OUT,     // z_out = P_CH^{-1} v (preconditioner-only job)
  PH_CG_INIT,     // single-reduction PCG: w_0 = C D^{-1} r_0, partials (r,u), (w,u), (r,r)
  PH_CG_ITER,     // single-reduction PCG iteration (one launch per iteration)
  PH_SCG_ITER,    // s-step PCG: two iterations from the Gram matrix, next basis (or x only); its
                  // first basis is formed by PH_PCG_SETUP (right-hand side on the halo, u_0 = D^{-1} b)
};

enum { JOB_NONE = 0, JOB_SOLVE = 1, JOB_RB = 2, JOB_PCH = 3 };

// inner solve kinds: steps (1), (2), (3.1), (3.2), (5) of the P_CH apply,
// then the two mass solves of the consistent initial values
enum { KIND_Y0 = 0, KIND_Y1 = 1, KIND_Z = 2, KIND_X1 = 3, KIND_X2 = 4, KIND_CI_OMEGA = 5, KIND_CI_MU = 6, KIND_SD = 7 };
// step (3) with the diagonal-mass Schur approximation S_D replaces (3.1), (3.2)

// Periodic grid meshes: n = N^dim nodes numbered x + N (y + N z) whose rows
// all have the same length.  The stored entries of a row are its columns in
// ascending order; when the offsets j - i of those columns depend only on
// whether the row lies on the low edge, inside or on the high edge in each
// direction (27 row classes; true for stencils of one step per direction),
// glin[class][k] holds the offset of entry k and the kernel computes the
// column instead of loading it.  Rows past n (padding of the last slice) count
// as row n - 1.  The host checks that this function reproduces every stored
// column before it enables the form.
#define PFC_GRID_W 16
#define PFC_GRID_CLASSES 27
#define PFC_GRID_MAXN (1 << 22)
// floor(v / N) for 0 <= v < 2^22 with inv = float(1/N): (v + 1/2) / N lies at
// least 1/(2N) from an integer, and the two roundings err by less than that
__host__ __device__ __forceinline__ int grid_div(int v, float inv) { return (int)(((float)v + 0.5f) * inv); }
__host__ __device__ __forceinline__ int grid_edge(int v, int N) { return v == 0 ? 0 : (v == N - 1 ? 2 : 1); }
// edge class of row i (in 2D, t = y < N gives z = 0)
__host__ __device__ __forceinline__ int grid_class(int r, int N, float inv) {
  const int t = grid_div(r, inv), x = r - t * N;
  const int z = grid_div(t, inv), y = t - z * N;
  return grid_edge(x, N) + 3 * grid_edge(y, N) + 9 * grid_edge(z, N);
}
__host__ __device__ __forceinline__ int grid_col(int i, int k, int n, int N, float inv, const int* glin) {
  const int r = i < n ? i : n - 1;
  return r + glin[grid_class(r, N, inv) * PFC_GRID_W + k];
}

struct MeshDev {
  int n, dim, n_slices, n_elem;
  long long nnz_sell;
  int uw, pad_uw;         // common width of all slices (structured meshes), 0 if they differ
  int degree, nloc;       // Lagrange degree (1, 2) and nodes per element
  int gN;                 // periodic grid side N (grid_col), or 0
  float gInv;             // float(1 / N)
  int glin[PFC_GRID_CLASSES * PFC_GRID_W];  // column offset of each entry per row class (grid_col)
  // direction of each entry per row class: (dx + 1) + 3 (dy + 1) + 9 (dz + 1), the
  // column's grid step from its row (periodic, each component in -1..1); valid if gdir_ok
  unsigned char gdir[PFC_GRID_CLASSES * PFC_GRID_W];
  int gdir_ok;
  const double* p2_M2;    // P2 reference tables (divided by |T|): M2[a][b],
  const double* p2_D;     //   D[i][j][a][b] = int d_i phi_a d_j phi_b (i, j barycentric),
  const double* p2_C4;    //   C4[a][b][c][d] = int phi_a phi_b phi_c phi_d
  const int* slice_ptr;   // [n_slices+1] entry offset of each slice (multiple of 64)
  const int* col;         // [nnz_sell]
  const double* M;        // [nnz_sell]
  const double* K;
  const float* Mf;
  const float* Kf;
  const double* dinvM;    // [n] 1/diag(M)
  const float* dinvMf;
  const int* sl_el_ptr;   // [nnz_sell+1] element contributions of each stored entry
  const int* sl_el;       // packed (elem << 4) | (a << 2) | b; P2: (elem << 8) | (a << 4) | b
  const int* nd_el_ptr;   // [n+1] simplices containing each node
  const int* nd_el;       // packed (elem << 2) | local index; P2: (elem << 4) | local index
  const int* elem_nodes;  // [n_elem*nloc]
  const double* elem_vol; // [n_elem]
  const double* elem_K;   // [n_elem * k(k+1)/2] |T| grad l_a . grad l_b for a <= b (P1 meshes; else null)
  // second-ring pattern of K M_D^{-1} K (built only for the S_D preconditioner)
  long long w_nnz_sell;
  const int* w_slice_ptr; // [n_slices+1]
  const int* w_col;       // [w_nnz_sell]
  const long long* w_p1pos; // [w_nnz_sell] position of the same entry in the P1 layout, or -1
  const int* w_tri_ptr;   // [w_nnz_sell+1]
  const int* w_tri;       // pairs (e1, e2): P1 positions of (i,k) and (k,j)
};

// Double-buffered scalar state of one instance (written by workgroup 0 of its
// team at the end of every launch into the other buffer).
struct State {
  int phase;
  int job;
  int step, stage;          // Rosenbrock position
  int kind, it, pcur, fuse;  // inner PCG; fuse: this launch also ended the solve of kind fkind
  int j, cycle, total, apply, kcols;
  int status, cur, fkind;
  double rho, bb, alpha, beta_cg;
  double xc0, xc1, xc3;      // its last increment of x over the basis [p, Tp, ., u] (stored the launch after)
  double vscale, bnorm, bnorm_s, est_thresh, w0, est, rel;
  long long t0;             // device clock at the solve's first launch
};

// Single-buffered FGMRES history of the current cycle.  Every entry is
// written once per cycle, by workgroup 0, in a launch after which it is read.
struct Hist {
  double hcol[PFC_MAXM + 1];
  double cs[PFC_MAXM];
  double sn[PFC_MAXM];
  double gpre[PFC_MAXM + 1];
  double gfin[PFC_MAXM];
  double R[PFC_MAXM][PFC_MAXM];   // R[l][c], l <= c
  double L[PFC_MAXM][PFC_MAXM];   // L[i][k] = (v_i, v_k), k < i (the Arnoldi basis' strictly lower Gram)
  int inner_max[PFC_NSTEPS_P];
  int applies;
  long long inner_total;
};

struct InfoDev {
  int status, outer_iters, cycles, inner_applies;
  long long inner_total;
  int inner_max[5];
  int reserved;
  double est_rel_res, true_rel_res;
  double t_solve;  // seconds of the device clock (100 MHz) from the solve's first launch to its last
};

struct InstDev {
  MeshDev m;
  int n, precision, restart, max_steps;
  int inner_maxit, shared_ops, team_size, replay;
  int single_reduction, schur_d;
  int sd_iters, model;          // model: PFC_MODEL_PFC2 / PFC_MODEL_PFC1
  int grid_cols, gamma_mode;    // grid_columns and gamma_mode options
  int inner_fixed[5], pad_if;   // fixed inner iteration counts (0: to inner_tol)
  int sstep, sH;                // two PCG iterations per launch: 0 no, 1 row ranges of a 2D grid (halo sH = N + 1
                                // rows), 2 blocks of a 3D grid of side 64, 3 blocks of a 2D grid (side 64 k)
  double outer_tol, inner_tol, ci_tol;
  // job parameters; tau_p = m0 tau_s is the preconditioner's time step
  // rs: factor of block row 1 in the system FGMRES works on (1/m11 for
  // PFC_GAMMA_SCALE_ROW, 1 for PFC_GAMMA_LITERAL); tau_s = rs tau, m11_s = rs m11
  double r, tau, m11, tau_s, delta, sdelta, rs, m11_s;
  double psi_min, m0, tau_p;
  int job, n_steps, init_mode, max_infos;
  // typed operator arrays (float or double by precision)
  void* Cd; void* Csd; void* dinvCd; void* dinvCsd;
  void* SDv; void* dinvSD;      // S_D values (second-ring layout) and Jacobi diagonal
  double* N;                    // [nnz_sell]
  double* Kp;                   // [nnz_sell] K_+(psi_k) (PFC1)
  double* Fm;                   // [nnz_sell] F(mu_k) (PFC1)
  // float64 vectors
  const double* b_user;         // solve job rhs
  double* x_user;               // solve job solution
  double* b;                    // [3n] stage rhs
  double* xk;                   // [3n] Rosenbrock state
  double* ys;                   // [3][3n] stage solutions
  double* V;                    // [(restart+1)][3n]
  double* Z;                    // [restart][3n]
  double* W;                    // [3n]
  double* pch_out;              // preconditioner-only job output
  double* xbak;                 // [3n] state before an adaptive step attempt
  double* errpart;              // [2 n_slices] per-slice partial sums (embedded error, mobility mean)
  // inner PCG vectors (sized for float64; typed by precision)
  void *r_, *pA, *pB, *q, *y0, *y1, *zt, *x1, *x2;
  void *rB, *wB, *sA, *sB;      // extra buffers of the single-reduction PCG
  double* part;                 // [2][team_size][4] partial sums
  double* gpart;                // [2][team_size][64] Gram partial sums of the orthogonalisation
  // s-step double buffers, indexed by the launch's parity: a launch reads the
  // previous launch's basis and Gram partials from [parity], writes to [1 - parity]
  double* sbas;                 // s-step basis [2][5][n] (p, Tp, T^2 p, u, Tu), or null
  double* spart;                // s-step Gram partial sums [2][team_size][32], or null
  State* st;                    // [2]
  Hist* hist;
  const int* sched_meta;        // replay: per solve {cycle offset, cycles, apply offset, applies}
  const int* sched_cycles;      // replay: cycle lengths
  const int* sched_inner;       // replay: 5 counts per application
  int n_sched_cycles, n_sched_applies;
  int* rec_inner;               // [max_steps * 5] counts of the last solve
  InfoDev* info;                // [max_infos]
};

// One workgroup of a launch: its instance, its rank in the instance's team,
// and the P1 pattern of the instance's mesh for the column staging.
struct TeamEntry {
  int inst, rank, size, uw;
  const int* col;
  int n_slices, pad;
};

// Rosenbrock coefficients of Table rosenbrock_scheme (Ros3Pw, modified form).
#define ROS_GAMMA 0.78867513459481287
#define ROS_A21 2.0
#define ROS_A31 0.633974596215561
#define ROS_A32 0.0
#define ROS_C21 (-2.53589838486225)
#define ROS_C31 (-1.62740473580836)
#define ROS_C32 (-0.274519052838329)
#define ROS_M1 1.63397459621556
#define ROS_M2 0.294228634059948
#define ROS_M3 1.07179676972449
#define ROS_MH1 1.99444650053487
#define ROS_MH2 0.654700538379252
#define ROS_MH3 1.07179676972449
