// The stage solver as a device-resident state machine.
//
// One launch of k_tick advances every active instance by one phase (see
// pfc_internal.h).  A launch first sums the partial reductions that the
// previous launch left behind (every workgroup of a team does this
// redundantly, in fixed order, so all of them take identical decisions), then
// thread 0 of each workgroup applies the transition to a copy of the state in
// LDS, the workgroup executes the work of the new phase, stores its partial
// sums and workgroup 0 of the team writes the new state.  Kernel boundaries
// are the only synchronisation between workgroups: no grid barriers, no
// atomics.  The host captures a fixed number of launches in a graph, replays
// it, and polls a pinned flag written by a small report kernel at the end of
// each replay.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "device.h"
#include "host.h"
#include "solver.h"

namespace pfc {

__device__ __forceinline__ bool phase_partials(int ph) {
  switch (ph) {
    case PH_SOLVE_INIT: case PH_RB_RHS: case PH_PCG_SETUP: case PH_PCG_A: case PH_PCG_B:
    case PH_GS_UPDATE: case PH_TRUE_RES: case PH_CG_INIT: case PH_CG_ITER:
      return true;
    default:
      return false;
  }
}

__device__ __forceinline__ int solve_index(const State& S) { return S.job == JOB_RB ? S.step * 3 + S.stage - 1 : 0; }

// count slot of an inner solve kind in the per-application record (5 slots)
__device__ __forceinline__ int count_slot(int kind) { return kind == KIND_SD ? KIND_Z : kind; }

__device__ __forceinline__ int inner_limit(const InstDev& I, const State& S, bool& fixed, double& tol) {
  if (is_ci(S.kind)) { fixed = false; tol = I.ci_tol; return 2000; }
  tol = I.inner_tol;
  if (I.replay) {
    fixed = true;
    const int idx = solve_index(S);
    const int* meta = I.sched_meta + 4 * idx;
    if (S.apply >= meta[3]) return 0;
    return I.sched_inner[(long long)(meta[2] + S.apply) * 5 + count_slot(S.kind)];
  }
  if (I.inner_fixed[count_slot(S.kind)] > 0) { fixed = true; return I.inner_fixed[count_slot(S.kind)]; }
  if (S.kind == KIND_SD) { fixed = true; return I.sd_iters; }  // Table inner_solvers: fixed count for S_D
  fixed = false;
  return I.inner_maxit;
}

__device__ void finish_solve(State& S, const InstDev& I, bool wr, int status) {
  if (wr) {
    const int idx = solve_index(S);
    if (idx < I.max_infos) {
      InfoDev& f = I.info[idx];
      f.status = status;
      f.outer_iters = S.total;
      f.cycles = S.cycle;
      f.inner_applies = I.hist->applies;
      f.inner_total = I.hist->inner_total;
      for (int k = 0; k < 5; ++k) f.inner_max[k] = I.hist->inner_max[k];
      f.est_rel_res = S.est;
      f.true_rel_res = S.rel;
      f.t_solve = (double)((long long)wall_clock64() - S.t0) * 1e-8;
    }
  }
  if (status < 0) S.status = status;
  else if (status > S.status && S.status >= 0) S.status = status;
  if (S.job == JOB_RB && status >= 0) {
    if (S.stage < 3) { S.stage += 1; S.phase = PH_RB_RHS; }
    else S.phase = PH_RB_UPDATE;
  } else {
    S.phase = PH_DONE;
  }
}

__device__ void begin_solve(State& S, const InstDev& I, bool wr, Red3 red) {
  S.bnorm = sqrt(red.a);
  S.bnorm_s = sqrt(red.b);
  S.total = 0; S.cycle = 0; S.j = 0; S.apply = 0; S.est = 0.0; S.rel = 0.0;
  if (wr) {
    I.hist->applies = 0;
    I.hist->inner_total = 0;
    for (int k = 0; k < 5; ++k) I.hist->inner_max[k] = 0;
  }
  if (!isfinite(S.bnorm)) { finish_solve(S, I, wr, PFC_ERR_BREAKDOWN); return; }
  if (S.bnorm == 0.0) { finish_solve(S, I, wr, PFC_OK); return; }
  if (I.replay && I.sched_meta[4 * solve_index(S) + 1] == 0) { finish_solve(S, I, wr, PFC_OK); return; }
  S.est_thresh = I.gamma_mode == PFC_GAMMA_LITERAL ? I.outer_tol * S.bnorm : I.outer_tol * S.bnorm / fmax(1.0, I.m11);
  if (wr) I.hist->gpre[0] = S.bnorm_s;
  S.vscale = 1.0 / S.bnorm_s;
  S.kind = KIND_Y0;
  S.phase = PH_PCG_SETUP;
}

__device__ void pcg_done(State& S, const InstDev& I, bool wr) {
  if (!is_ci(S.kind) && wr) {
    const int slot = count_slot(S.kind);
    if (S.apply < I.max_steps) {
      I.rec_inner[S.apply * 5 + slot] = S.it;
      if (S.kind == KIND_SD) I.rec_inner[S.apply * 5 + KIND_X1] = 0;
    }
    I.hist->inner_total += S.it;
    if (S.it > I.hist->inner_max[slot]) I.hist->inner_max[slot] = S.it;
  }
  switch (S.kind) {
    case KIND_Y1:
      S.kind = I.schur_d ? KIND_SD : KIND_Z;
      S.phase = PH_PCG_SETUP;
      break;
    case KIND_SD:
      S.kind = KIND_X2;
      S.phase = PH_PCG_SETUP;
      break;
    case KIND_Y0: case KIND_Z: case KIND_X1:
      S.kind += 1;
      S.phase = PH_PCG_SETUP;
      break;
    case KIND_X2:
      if (wr) I.hist->applies += 1;
      S.apply += 1;
      S.phase = (S.job == JOB_PCH) ? PH_PCH_OUT : PH_ASPMV;
      break;
    case KIND_CI_OMEGA:
      S.kind = KIND_CI_MU;
      S.phase = PH_PCG_SETUP;
      break;
    default:  // KIND_CI_MU: consistent initial values done
      S.step = 0;
      S.phase = (I.n_steps > 0) ? PH_RB_BEGIN : PH_DONE;
      break;
  }
}

__device__ void restart_cycle(State& S, const InstDev& I, bool wr, double beta) {
  if (!(beta > 0.0)) { finish_solve(S, I, wr, PFC_OK); return; }
  if (wr) I.hist->gpre[0] = beta;
  S.j = 0;
  S.vscale = 1.0 / beta;
  S.kind = KIND_Y0;
  S.phase = PH_PCG_SETUP;
}

// Givens rotation of column j, cycle control, back substitution.
__device__ void givens(State& S, const InstDev& I, bool wr, double hn2, double* ybuf, double* col) {
  Hist* H = I.hist;
  const int j = S.j;
  const double hn = sqrt(hn2);
  for (int l = 0; l <= j; ++l) col[l] = H->hcol[l];
  col[j + 1] = hn;
  for (int l = 0; l < j; ++l) {
    const double c = H->cs[l], s = H->sn[l];
    const double t = c * col[l] + s * col[l + 1];
    col[l + 1] = -s * col[l] + c * col[l + 1];
    col[l] = t;
  }
  const double d = hypot(col[j], col[j + 1]);
  double cj = 1.0, sj = 0.0;
  if (d != 0.0) { cj = col[j] / d; sj = col[j + 1] / d; }
  col[j] = d;
  const double gj = H->gpre[j];
  const double gfin = cj * gj;
  const double gnext = -sj * gj;
  if (wr) {
    H->cs[j] = cj; H->sn[j] = sj; H->gfin[j] = gfin; H->gpre[j + 1] = gnext;
    for (int l = 0; l <= j; ++l) H->R[l][j] = col[l];
  }
  S.total += 1;
  S.est = fabs(gnext) / S.bnorm_s;
  const bool breakdown = hn <= 1e-14 * S.w0;
  bool done;
  if (I.replay) {
    const int* meta = I.sched_meta + 4 * solve_index(S);
    done = (j + 1 >= I.sched_cycles[meta[0] + S.cycle]);
  } else {
    done = fabs(gnext) <= S.est_thresh || breakdown || S.total >= I.max_steps || j + 1 == I.restart;
  }
  if (!done) {
    S.vscale = 1.0 / hn;
    S.j = j + 1;
    S.kind = KIND_Y0;
    S.phase = PH_PCG_SETUP;
    return;
  }
  const int k = j + 1;
  for (int l = k - 1; l >= 0; --l) {
    double s = (l == j) ? gfin : H->gfin[l];
    for (int c = l + 1; c < k; ++c) s -= ((c == j) ? col[l] : H->R[l][c]) * ybuf[c];
    ybuf[l] = s / ((l == j) ? col[l] : H->R[l][l]);
  }
  S.kcols = k;
  S.phase = PH_UPDATE_X;
}

// The most frequent transition, a single-reduction PCG iteration that is not
// the last of its solve, kept inline next to the launch prologue (the general
// transition below is out of line and its code is fetched only when needed).
// Same decisions and arithmetic as the PH_CG_ITER case of transition().
__device__ __forceinline__ bool cg_iter_continues(State& S, const InstDev& I, Red3 red) {
  if (S.phase != PH_CG_ITER || I.replay || S.kind == KIND_SD || is_ci(S.kind) || I.inner_fixed[count_slot(S.kind)] > 0)
    return false;
  const int it = S.it + 1;
  const double g = red.a, dl = red.b, rr = red.c;
  const double tol = I.inner_tol;
  if (it >= I.inner_maxit || rr <= tol * tol * S.bb || g == 0.0 || !isfinite(rr)) return false;
  S.it = it;
  S.cur ^= 1;
  const double beta = g / S.rho;
  S.alpha = g / (dl - beta * g / S.alpha);
  S.beta_cg = beta;
  S.rho = g;
  return true;
}

// inner solves that may run two iterations per launch: the five P_CH solves on
// the P1 pattern (not S_D, not the consistent-initial-value mass solves)
__device__ __forceinline__ bool scg_kind(int kind) { return kind >= KIND_Y0 && kind <= KIND_X2; }

// s-step PCG: the next two iterations from the Gram sums g of the basis B = [p,
// Tp, T^2 p, u, Tu] (g[0..14]: B^T D B, g[15..24]: D^2-weighted Gram of B[1..4]),
// with the stopping test of the standard iteration after each of them.  coef
// receives the increment of x and the new p and u as combinations of B;
// S.pcur = 1 marks a launch that only adds the increment (the solve ends there).
__device__ __forceinline__ void scg_transition(State& S, const InstDev& I, bool wr, const double* g, double* coef) {
  if (S.phase == PH_SCG_ITER && S.pcur) { pcg_done(S, I, wr); return; }
  const bool first = (S.phase == PH_PCG_SETUP);  // that launch formed the solve's first basis
  S.phase = PH_SCG_ITER;
  // entries (i <= j) of G = B^T D B and of H = B'^T D^2 B' (basis indices 1..4)
  auto G = [&](int i, int j) { return g[ss_tri(i, j, 5)]; };
  auto Hq = [&](int i, int j) { return g[15 + ss_tri(i - 1, j - 1, 4)]; };
  for (int m = 0; m < 15; ++m) coef[m] = 0.0;
  bool fixed; double tol;
  const int lim = inner_limit(I, S, fixed, tol);
  if (first) {
    S.bb = g[25];
    S.it = 0;
    S.pcur = 0;
    if (S.bb == 0.0 || lim == 0) { pcg_done(S, I, wr); return; }  // x_0 = 0 stands
  }
  // first iteration: alpha_0 = <u,u> / <p,Tp>, u_1 = u - alpha_0 Tp
  const double rho0 = G(3, 3);
  const double a0 = rho0 / G(0, 1);
  const double rho1 = G(3, 3) - 2.0 * a0 * G(1, 3) + a0 * a0 * G(1, 1);
  const double rr1 = Hq(3, 3) - 2.0 * a0 * Hq(1, 3) + a0 * a0 * Hq(1, 1);
  coef[0] = a0;
  S.it += 1;
  S.pcur = 1;
  if (S.it >= lim || (!fixed && rr1 <= tol * tol * S.bb) || rho1 == 0.0 || !isfinite(rr1)) return;
  // second: p_1 = u_1 + beta_0 p = b0 e0 - a0 e1 + e3, T p_1 = b0 e1 - a0 e2 + e4
  const double b0 = rho1 / rho0;
  const double ptp = b0 * (b0 * G(0, 1) - a0 * G(0, 2) + G(0, 4)) - a0 * (b0 * G(1, 1) - a0 * G(1, 2) + G(1, 4)) +
                     (b0 * G(1, 3) - a0 * G(2, 3) + G(3, 4));
  const double a1 = rho1 / ptp;
  // u_2 = u_1 - alpha_1 T p_1 = c1 e1 + c2 e2 + e3 + c4 e4
  const double c1 = -a0 - a1 * b0, c2 = a1 * a0, c4 = -a1;
  auto quad = [&](auto M) {
    return c1 * c1 * M(1, 1) + c2 * c2 * M(2, 2) + M(3, 3) + c4 * c4 * M(4, 4) +
           2.0 * (c1 * c2 * M(1, 2) + c1 * M(1, 3) + c1 * c4 * M(1, 4) + c2 * M(2, 3) + c2 * c4 * M(2, 4) + c4 * M(3, 4));
  };
  const double rho2 = quad(G), rr2 = quad(Hq);
  // x += alpha_0 p + alpha_1 p_1
  coef[0] = a0 + a1 * b0;
  coef[1] = -a1 * a0;
  coef[3] = a1;
  S.it += 1;
  if (S.it >= lim || (!fixed && rr2 <= tol * tol * S.bb) || rho2 == 0.0 || !isfinite(rr2)) return;
  // p_2 = u_2 + beta_1 p_1, u_2
  const double b1 = rho2 / rho1;
  coef[5] = b1 * b0; coef[6] = c1 - b1 * a0; coef[7] = c2; coef[8] = 1.0 + b1; coef[9] = c4;
  coef[11] = c1; coef[12] = c2; coef[13] = 1.0; coef[14] = c4;
  S.pcur = 0;
}

// 2D block form: a solve whose last increment this launch adds (S.pcur) ends
// here if the next P_CH step's set-up reads its x as v (steps (1)-(4) to the
// next one, not into S_D): this launch then also forms that set-up from x plus
// the increment on a three-step frame (S.fuse, the kind ending S.fkind), and
// the next launch stores that x (the increment's coefficients kept in S.xc*).
__device__ __forceinline__ void b2_fuse_end(State& S, const InstDev& I, bool wr, const double* coef) {
  S.fuse = 0;
  if (S.phase != PH_SCG_ITER || !S.pcur) return;
  const int k = S.kind;
  if (!(k == KIND_Y0 || k == KIND_Z || k == KIND_X1 || (k == KIND_Y1 && !I.schur_d))) return;
  pcg_done(S, I, wr);
  S.fuse = 1;
  S.fkind = k;
  S.xc0 = coef[0];
  S.xc1 = coef[1];
  S.xc3 = coef[3];
}

// After w = A_s z_j and its Gram sums g (slots as in ph_aspmv; Ls: the rows of
// L stored by earlier steps of the cycle): h solves (I + L) h = c by forward
// substitution, which is modified Gram-Schmidt's sequence of coefficients.
__device__ void gs_coefficients(State& S, const InstDev& I, bool wr, const double* g, const double* Ls, double* h) {
  const int j = S.j;
  for (int i = 0; i <= j; ++i) {
    double s = g[i];
    for (int k = 0; k < i; ++k) s -= (i == j ? g[32 + k] : Ls[i * PFC_MAXM + k]) * h[k];
    h[i] = s;
  }
  if (wr) {
    for (int k = 0; k < j; ++k) I.hist->L[j][k] = g[32 + k];
    for (int i = 0; i <= j; ++i) I.hist->hcol[i] = h[i];
  }
  S.w0 = sqrt(g[32 + j]);
  S.phase = PH_GS_UPDATE;
}

__device__ void transition(State& S, const InstDev& I, bool wr, Red3 red, double* ybuf, double* col, bool ss) {
  switch (S.phase) {
    case PH_START:
      if (S.job == JOB_SOLVE) S.phase = PH_SOLVE_INIT;
      else if (S.job == JOB_PCH) {
        S.j = 0; S.vscale = 1.0; S.kind = KIND_Y0; S.apply = 0; S.phase = PH_PCG_SETUP;
        if (wr) { I.hist->applies = 0; I.hist->inner_total = 0; for (int k = 0; k < 5; ++k) I.hist->inner_max[k] = 0; }
      } else {  // JOB_RB
        S.step = 0;
        if (I.init_mode == PFC_INIT_CONSISTENT) { S.kind = KIND_CI_OMEGA; S.phase = PH_PCG_SETUP; }
        else S.phase = (I.n_steps > 0) ? PH_RB_BEGIN : PH_DONE;
      }
      break;
    case PH_SOLVE_INIT:
    case PH_RB_RHS:
      begin_solve(S, I, wr, red);
      break;
    case PH_RB_BEGIN:
      S.stage = 1;
      S.phase = PH_RB_RHS;
      break;
    case PH_RB_UPDATE:
      S.step += 1;
      S.phase = (S.step < I.n_steps) ? PH_RB_BEGIN : PH_DONE;
      break;
    case PH_PCG_SETUP: {
      S.rho = red.a; S.bb = red.b; S.it = 0; S.pcur = 0; S.cur = 0; S.beta_cg = 0.0;
      bool fixed; double tol;
      const int lim = inner_limit(I, S, fixed, tol);
      if (S.bb == 0.0 || lim == 0) pcg_done(S, I, wr);
      else if (!I.single_reduction) S.phase = PH_PCG_A;
      else S.phase = PH_CG_INIT;
    } break;
    case PH_CG_INIT:
      S.rho = red.a;             // gamma_0 = (r_0, D^{-1} r_0)
      S.alpha = red.a / red.b;   // gamma_0 / (w_0, u_0)
      S.beta_cg = 0.0;
      S.it = 0;
      S.cur = 0;
      S.phase = PH_CG_ITER;
      break;
    case PH_CG_ITER: {
      S.it += 1;
      S.cur ^= 1;
      bool fixed; double tol;
      const int lim = inner_limit(I, S, fixed, tol);
      const double g = red.a, dl = red.b, rr = red.c;
      const bool done = S.it >= lim || (!fixed && rr <= tol * tol * S.bb) || g == 0.0 || !isfinite(rr);
      if (done) pcg_done(S, I, wr);
      else {
        const double beta = g / S.rho;
        S.alpha = g / (dl - beta * g / S.alpha);
        S.beta_cg = beta;
        S.rho = g;
      }
    } break;
    case PH_PCG_A:
      S.alpha = S.rho / red.a;
      S.pcur ^= 1;
      S.phase = PH_PCG_B;
      break;
    case PH_PCG_B: {
      S.it += 1;
      bool fixed; double tol;
      const int lim = inner_limit(I, S, fixed, tol);
      const double rr = red.a, rzn = red.b;
      const bool done = S.it >= lim || (!fixed && rr <= tol * tol * S.bb) || rzn == 0.0 || !isfinite(rr);
      if (done) pcg_done(S, I, wr);
      else { S.beta_cg = rzn / S.rho; S.rho = rzn; S.phase = PH_PCG_A; }
    } break;
    case PH_GS_UPDATE:
      givens(S, I, wr, red.a, ybuf, col);
      break;
    case PH_UPDATE_X:
      S.phase = PH_TRUE_RES;
      break;
    case PH_TRUE_RES: {
      const double rel = sqrt(red.a) / S.bnorm;
      S.rel = rel;
      S.cycle += 1;
      if (!isfinite(rel)) { finish_solve(S, I, wr, PFC_ERR_BREAKDOWN); break; }
      if (I.replay) {
        const int* meta = I.sched_meta + 4 * solve_index(S);
        if (S.cycle < meta[1]) restart_cycle(S, I, wr, sqrt(red.b));
        else finish_solve(S, I, wr, rel <= I.outer_tol ? PFC_OK : PFC_NOT_CONVERGED);
      } else if (rel <= I.outer_tol) {
        finish_solve(S, I, wr, PFC_OK);
      } else if (S.total >= I.max_steps) {
        finish_solve(S, I, wr, PFC_NOT_CONVERGED);
      } else {
        restart_cycle(S, I, wr, sqrt(red.b));
      }
    } break;
    case PH_PCH_OUT:
      S.phase = PH_DONE;
      break;
    case PH_SCG_ITER:  // a two-iteration solve in a launch without that form: refuse, loudly
      finish_solve(S, I, wr, PFC_ERR_STATE);
      break;
    default:
      S.phase = PH_DONE;
      break;
  }
}

#ifdef PFC_TICK_TIMING
// optional instrumentation (separate build only): wall-clock stamps of one workgroup per launch
__device__ unsigned long long* g_trace = nullptr;
__device__ unsigned long long g_trace_n = 0;
__device__ unsigned long long g_trace_cap = 0;
#define PFC_STAMP(v) unsigned long long v = wall_clock64()
#else
#define PFC_STAMP(v)
#endif

// Inner PCG phase PH of the current solve kind, with one call site per
// distinct instantiation: the float64 solves of the consistent initial values
// (every precision), the S_D solve on its unstaged second-ring pattern, and the
// main path.  (Several call sites of one instantiation make the compiler keep
// it out of line, and the out-of-line call costs a scratch spill of the team
// record on every launch.)
template <typename TT, int L, int PH>
__device__ __forceinline__ Red3 pcg_phase_one(const InstDev& I, const State& S, const Team& tm) {
  if constexpr (PH == PH_PCG_SETUP) return ph_pcg_setup<TT, L>(I, S, tm);
  else if constexpr (PH == PH_PCG_A) return ph_pcg_a<TT, L>(I, S, tm);
  else if constexpr (PH == PH_PCG_B) return ph_pcg_b<TT>(I, S, tm);
  else if constexpr (PH == PH_CG_INIT) return ph_cg_init<TT, L>(I, S, tm);
  else return ph_cg_iter<TT, L>(I, S, tm);
}

template <typename T, int COLS, int PH>
__device__ __forceinline__ Red3 pcg_phase(const InstDev& I, const State& S, const Team& tm, bool sd) {
  constexpr bool uses_pattern = (PH != PH_PCG_SETUP && PH != PH_PCG_B);  // the operator's own SpMV
  if constexpr (!std::is_same<T, double>::value) {
    if (is_ci(S.kind)) return pcg_phase_one<double, COLS, PH>(I, S, tm);
  }
  if constexpr (COLS != PFC_COL_MEM && uses_pattern) {
    if (sd) return pcg_phase_one<T, PFC_COL_MEM, PH>(I, S, tm);
  }
  return pcg_phase_one<T, COLS, PH>(I, S, tm);
}

// One solver launch.  SINGLE: the launch serves one instance and receives its
// state and partial-sum buffers and its mesh pattern as kernel arguments
// (preloaded into scalar registers), so the first memory round trip already
// fetches the state.  Otherwise each workgroup looks up its team entry and
// instance descriptor.  COLS: where the P1 columns come from (PFC_COL_*).
// PFC_COL_LDS stages the workgroup's columns in LDS in the same round trip
// (uniform slice width, at most PFC_WAVES slices per workgroup); PFC_COL_GRID
// computes them from the row (periodic grid meshes).  The host picks the
// variant that the launch's meshes allow.
template <typename T, bool SINGLE, int COLS, bool B2>
__global__ __launch_bounds__(PFC_WG) void k_tick(const TeamEntry* __restrict__ teams, const InstDev* __restrict__ insts,
                                                 const State* st_in_arg, State* st_out_arg, const double* part_in_arg,
                                                 double* part_out_arg, int parity, const int* __restrict__ col_arg,
                                                 int uw_arg, int nsl_arg, const double* gram_in_arg) {
  __shared__ State S;
  __shared__ State S0;  // entry state of launches that serve many instances (path choice)
  __shared__ InstDev sI;
  __shared__ Red3 lds4[PFC_WAVES];
  __shared__ double ybuf[PFC_MAXM];
  __shared__ double gcol[PFC_MAXM + 1];
  __shared__ double hbuf[PFC_MAXM];          // Gram-Schmidt coefficients of the current Arnoldi step
  __shared__ double gs_g[PFC_GS_NV];         // Gram sums of the step (after PH_ASPMV)
  __shared__ double gs_L[PFC_MAXM * PFC_MAXM];
  // two PCG iterations per launch on periodic grids: blocks of 2D grids (B2,
  // either precision, launches that serve one or many instances), and in
  // launches that serve one instance row ranges of 2D grids in float64 and
  // blocks of 3D grids of side 64 in float
  constexpr bool SB2 = B2 && COLS == PFC_COL_GRID;
  constexpr bool SS = SINGLE && COLS == PFC_COL_GRID && std::is_same<T, double>::value && !B2;
  constexpr bool SS3 = SINGLE && COLS == PFC_COL_GRID && std::is_same<T, float>::value && !B2;
  constexpr bool SSX = SS || SS3 || SB2;
  __shared__ double ss_g[SSX ? 32 : 1];
  __shared__ double ss_coef[SSX ? 16 : 1];
  PFC_STAMP(t_entry);
  const int tid = threadIdx.x;
  TeamEntry te;
  const InstDev* gI;
  const State* st_in;
  State* st_out;
  const double* part_in;
  double* part_out;
  if (SINGLE) {
    te.inst = 0; te.rank = xcd_rank(blockIdx.x, gridDim.x); te.size = gridDim.x;
    te.uw = uw_arg; te.col = col_arg; te.n_slices = nsl_arg; te.pad = 0;
    gI = insts;
    st_in = st_in_arg; st_out = st_out_arg; part_in = part_in_arg; part_out = part_out_arg;
  } else {
    te = teams[xcd_rank(blockIdx.x, gridDim.x)];
    gI = insts + te.inst;
    st_in = gI->st + parity; st_out = gI->st + (1 - parity);
    part_in = gI->part + (long long)parity * te.size * 4;
    part_out = gI->part + (long long)(1 - parity) * te.size * 4;
  }
  // one round trip: the state record and the instance descriptor (a word per
  // thread, every thread loading at a clamped position), the partial sums of
  // the previous launch and, in single-instance launches of two-iteration
  // solves, the previous launch's Gram partials (gram_in_arg; a launch that
  // runs another phase leaves them unused).  Every load is issued before the
  // first of them is waited for.
  constexpr int NS = (int)(sizeof(State) / 4), ND = (int)(sizeof(InstDev) / 4);
  static_assert(NS <= 64 && ND <= PFC_WG - 64, "state / descriptor too large for the staging threads");
  const int word = tid < 64 ? ((const int*)st_in)[min(tid, NS - 1)] : ((const int*)gI)[min(tid - 64, ND - 1)];
  // the fields that choose a workgroup's path before the transition: thread 0
  // rewrites S in the transition while the other waves may still be reading
  // them, so they come from the state record itself (one instance per launch),
  // or from S0, an LDS copy of the entry state that nothing rewrites
  int ph_in = 0, kind_in = 0, pcur_in = 0, fuse_in = 0;
  if constexpr (SINGLE) {
    ph_in = st_in->phase;
    kind_in = st_in->kind;
    pcur_in = st_in->pcur;
    if constexpr (SB2) fuse_in = st_in->fuse;
  }
  double gpl[SSX ? PFC_SS_GL : 1];
  if constexpr (SSX && SINGLE) ss_gram_prefetch(gram_in_arg, part_in, te.size, gpl);
  // columns of this workgroup's slices: positions [lo, lo + len) of the SELL
  // pattern, issued first and written to LDS once everything has arrived
  int lo = 0, len = 0;
  int cv[PFC_LCOL_W];
  if (COLS == PFC_COL_LDS) {
    const int spw = (te.n_slices + te.size - 1) / te.size;
    const int sbeg = te.rank * spw;
    const int send = min(sbeg + spw, te.n_slices);
    lo = sbeg * 64 * te.uw;
    len = max(send - sbeg, 0) * 64 * te.uw;
#pragma unroll
    for (int q = 0; q < PFC_LCOL_W; ++q) {
      const int idx = tid + q * PFC_WG;
      if (idx < len) cv[q] = te.col[lo + idx];
    }
  }
  Red3 pre = red3(0.0, 0.0, 0.0), pre2 = red3(0.0, 0.0, 0.0);
  if (tid < te.size) { pre.a = part_in[4 * tid]; pre.b = part_in[4 * tid + 1]; pre.c = part_in[4 * tid + 2]; }
  for (int k = tid + PFC_WG; k < te.size; k += PFC_WG) {  // teams of more than PFC_WG workgroups
    pre2.a += part_in[4 * k]; pre2.b += part_in[4 * k + 1]; pre2.c += part_in[4 * k + 2];
  }
  if (tid < NS) {
    ((int*)&S)[tid] = word;
    if constexpr (!SINGLE) ((int*)&S0)[tid] = word;
  } else if (tid >= 64 && tid < 64 + ND) {
    ((int*)&sI)[tid - 64] = word;
  }
  if (COLS == PFC_COL_LDS) {
#pragma unroll
    for (int q = 0; q < PFC_LCOL_W; ++q) {
      const int idx = tid + q * PFC_WG;
      if (idx < len) pfc_lcol[idx] = cv[q];
    }
  }
  pre.a += pre2.a;
  pre.b += pre2.b;
  pre.c += pre2.c;
  pre.a = wave_sum(pre.a);
  pre.b = wave_sum(pre.b);
  pre.c = wave_sum(pre.c);
  if ((tid & 63) == 0) lds4[tid >> 6] = pre;
  __syncthreads();
#ifdef PFC_TICK_TIMING
  const unsigned long long t_ld = wall_clock64();
  unsigned long long t_red = 0;
#endif
  if constexpr (!SINGLE) {
    ph_in = S0.phase;
    kind_in = S0.kind;
    pcur_in = S0.pcur;
    if constexpr (SB2) fuse_in = S0.fuse;
  }
  const InstDev& I = sI;
  const bool writer = (te.rank == 0);
  if (__builtin_expect(ph_in == PH_DONE, 0)) {
    if (writer && tid < NS) ((int*)st_out)[tid] = ((const int*)&S)[tid];
    return;
  }
  // Gram partials of an orthogonalisation (the previous launch formed w = A_s z_j)
  if (__builtin_expect(ph_in == PH_ASPMV, 0))
    gs_gather(I.gpart + (long long)parity * te.size * PFC_GS_NV, te.size, &I.hist->L[0][0], gs_g, gs_L);
  bool scg = false, form = false;
  SsPre ssp;
  S3Pre<float> s3p;
  B2Pre<T> b2p;
  if constexpr (SSX) {
    // launches after a two-iteration launch, or after the set-up that formed the first basis,
    // of an instance whose two-iteration form is this launch's (a launch that serves many
    // instances may hold instances of either form: the others run one iteration per launch)
    form = SB2 ? I.sstep == 3 : (SS ? I.sstep == 1 : I.sstep == 2);
    scg = form && (ph_in == PH_SCG_ITER || (ph_in == PH_PCG_SETUP && scg_kind(kind_in)));
    if (scg && !(ph_in == PH_SCG_ITER && pcur_in)) {
      // the previous launch's Gram partials: loaded in the prologue where the
      // launch serves one instance, else here from the instance's buffer
      const double* gin = SINGLE ? gram_in_arg : I.spart + (long long)parity * te.size * 32;
      if constexpr (!SINGLE) ss_gram_prefetch(gin, gin, te.size, gpl);
      // in flight during the reduction and the transition
      if constexpr (SB2) b2_load<T>(I, te.rank, b2p, parity);
      else if constexpr (SS) ss_load(I, S, ss_rows(I, te.rank, te.size), ssp, parity);
      else s3_load<float>(I, S, te.rank, s3p, parity);
      ss_gram(gin, te.size, gpl, ss_g);
#ifdef PFC_TICK_TIMING
      if (tid == 0) pfc_sst[4] = wall_clock64();
#endif
    }
  }
  if (tid == 0) {
    if (scg) {
      if constexpr (SSX) scg_transition(S, I, writer, ss_g, ss_coef);
      if constexpr (SB2) b2_fuse_end(S, I, writer, ss_coef);
#ifdef PFC_TICK_TIMING
      if constexpr (SSX) pfc_sst[5] = wall_clock64();
#endif
    } else {
      S.fuse = 0;
      Red3 red = red3(0.0, 0.0, 0.0);
      if (phase_partials(S.phase)) {
#pragma unroll
        for (int w = 0; w < PFC_WAVES; ++w) { red.a += lds4[w].a; red.b += lds4[w].b; red.c += lds4[w].c; }
      }
      if (S.phase == PH_ASPMV) gs_coefficients(S, I, writer, gs_g, gs_L, hbuf);
      else if (!cg_iter_continues(S, I, red)) transition(S, I, writer, red, ybuf, gcol, SS && I.sstep);
      if (S.phase == PH_SOLVE_INIT || S.phase == PH_RB_RHS) S.t0 = (long long)wall_clock64();  // a solve starts
    }
  }
  if constexpr (SSX) {
    if (scg) lds_barrier();  // the basis loads issued in the prologue stay in flight
    else __syncthreads();
  } else {
    __syncthreads();
  }
  PFC_STAMP(t_trans);
  // the new state is final: workgroup 0 stores it while the phase runs
  if (writer && tid < NS) ((int*)st_out)[tid] = ((const int*)&S)[tid];
  Team tm{te.rank, te.size, tid >> 6, tid & 63, lo};
  if constexpr (SB2) {
    // the previous launch ended a solve in its set-up: that solve's x on the own rows
    if (__builtin_expect(fuse_in != 0, 0)) {
      const State& Se = SINGLE ? *st_in : S0;
      b2_end_store<T>(I, te.rank, Se.fkind, Se.xc0, Se.xc1, Se.xc3, parity);
    }
  }
  const bool sd = (S.kind == KIND_SD);  // second-ring pattern, never staged
  Red3 acc = red3(0.0, 0.0, 0.0);
  bool fused = false;  // a set-up launch that formed a two-iteration solve's first basis (Gram partials only)
  bool scg_done = false;
  if constexpr (SSX) {
    if (__builtin_expect(S.phase == PH_SCG_ITER, 1)) {  // the common launch, laid out first
      double* gout = I.spart + (long long)(1 - parity) * te.size * 32;
      if constexpr (SB2) ph_scg2b<T>(I, S, tm, ss_coef, false, gout, b2p, parity);
      else if constexpr (SS) ph_scg<COLS>(I, S, tm, ss_coef, false, gout, ss_rows(I, te.rank, te.size), ssp, parity);
      else ph_scg3<float>(I, S, tm, ss_coef, false, gout, s3p, parity);
      scg_done = true;
    }
  }
  if (!scg_done) switch (S.phase) {
    case PH_SOLVE_INIT:
    case PH_RB_RHS: acc = ph_solve_init<COLS>(I, S, tm); break;
    case PH_RB_BEGIN: acc = ph_rb_begin<COLS>(I, tm); break;
    case PH_RB_UPDATE: acc = ph_rb_update(I, tm); break;
    // the mass solves of the consistent initial values run in float64 in every precision
    case PH_PCG_SETUP:
      if constexpr (SSX) {
        if (form && scg_kind(S.kind)) {  // set-up and first basis of a two-iteration solve
          fused = true;
          double* gout = I.spart + (long long)(1 - parity) * te.size * 32;
          if constexpr (SB2) ph_scg2b<T>(I, S, tm, ss_coef, true, gout, b2p, parity);
          else if constexpr (SS) ph_scg<COLS>(I, S, tm, ss_coef, true, gout, ss_rows(I, te.rank, te.size), ssp, parity);
          else ph_scg3<float>(I, S, tm, ss_coef, true, gout, s3p, parity);
          break;
        }
      }
      acc = pcg_phase<T, COLS, PH_PCG_SETUP>(I, S, tm, sd);
      break;
    case PH_PCG_A: acc = pcg_phase<T, COLS, PH_PCG_A>(I, S, tm, sd); break;
    case PH_PCG_B: acc = pcg_phase<T, COLS, PH_PCG_B>(I, S, tm, sd); break;
    case PH_ASPMV: {
      double* gout = I.gpart + (long long)(1 - parity) * te.size * PFC_GS_NV;
      if (I.model == PFC_MODEL_PFC1) ph_aspmv<T, COLS, true>(I, S, tm, gout);
      else ph_aspmv<T, COLS, false>(I, S, tm, gout);
    } break;
    case PH_GS_UPDATE: acc = ph_gs_update(I, S, tm, hbuf); break;
    case PH_UPDATE_X: acc = ph_update_x(I, S, tm, ybuf); break;
    case PH_TRUE_RES:
      acc = I.model == PFC_MODEL_PFC1 ? ph_true_res<COLS, true>(I, S, tm) : ph_true_res<COLS, false>(I, S, tm);
      break;
    case PH_PCH_OUT: acc = ph_pch_out<T>(I, tm); break;
    case PH_CG_INIT: acc = pcg_phase<T, COLS, PH_CG_INIT>(I, S, tm, sd); break;
    case PH_CG_ITER: acc = pcg_phase<T, COLS, PH_CG_ITER>(I, S, tm, sd); break;
    default: break;  // PH_SCG_ITER above
  }
  PFC_STAMP(t_work);
  if (phase_partials(S.phase) && !fused) {
    acc.a = wave_sum(acc.a);
    acc.b = wave_sum(acc.b);
    acc.c = wave_sum(acc.c);
    if ((tid & 63) == 0) lds4[tid >> 6] = acc;
    __syncthreads();
#ifdef PFC_TICK_TIMING
    t_red = wall_clock64();
#endif
    if (tid == 0) {
      Red3 r = red3(0.0, 0.0, 0.0);
#pragma unroll
      for (int w = 0; w < PFC_WAVES; ++w) { r.a += lds4[w].a; r.b += lds4[w].b; r.c += lds4[w].c; }
      double* dst = part_out + (long long)te.rank * 4;
      dst[0] = r.a; dst[1] = r.b; dst[2] = r.c;
    }
  }
#ifdef PFC_TICK_TIMING
  __syncthreads();
  PFC_STAMP(t_exit);
  if (tid == 0 && (te.rank == 0 || te.rank == te.size - 1) && g_trace) {
    const unsigned long long k = atomicAdd(&g_trace_n, 1ULL);
    if (k < g_trace_cap) {
      unsigned long long* r = g_trace + 14 * k;
      r[0] = (unsigned long long)S.phase | ((unsigned long long)te.rank << 8) | ((unsigned long long)S.kind << 40) |
             ((unsigned long long)(S.it & 0xffff) << 48);
      r[1] = t_entry; r[2] = t_ld; r[3] = t_trans; r[4] = t_work; r[5] = t_exit; r[6] = blockIdx.x; r[7] = t_red;
      for (int q = 0; q < 6; ++q) r[8 + q] = (SSX && (fused || S.phase == PH_SCG_ITER)) ? pfc_sst[q] : 0;
    }
  }
#endif
}

#ifdef PFC_TICK_TIMING
extern "C" int pfc_debug_trace(unsigned long long* dev_buf, unsigned long long cap) {
  unsigned long long z = 0;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_trace), &dev_buf, sizeof(dev_buf)) != hipSuccess) return -3;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_trace_cap), &cap, sizeof(cap)) != hipSuccess) return -3;
  if (hipMemcpyToSymbol(HIP_SYMBOL(g_trace_n), &z, sizeof(z)) != hipSuccess) return -3;
  return 0;
}
extern "C" unsigned long long pfc_debug_trace_count(void) {
  unsigned long long n = 0;
  (void)hipMemcpyFromSymbol(&n, HIP_SYMBOL(g_trace_n), sizeof(n));
  return n;
}
#endif

__global__ void k_report(const InstDev* __restrict__ insts, int count, int* __restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) flags[i] = insts[i].st[0].phase;
}

// Per-tau operator values: C_d = M + delta K, C_sd = M + sqrt(delta) K (stored
// unless shared_ops) and their Jacobi diagonals, in the inner precision.
template <typename T>
__global__ void k_prep_ops(InstDev I) {
  const int sl = blockIdx.x * PFC_WAVES + (threadIdx.x >> 6);
  if (sl >= I.m.n_slices) return;
  const int lane = threadIdx.x & 63;
  const int i = sl * 64 + lane;
  const int base = I.m.slice_ptr[sl];
  const int w = (I.m.slice_ptr[sl + 1] - base) >> 6;
  double dd = 0.0, ds = 0.0;
  for (int k = 0; k < w; ++k) {
    const long long e = (long long)base + k * 64 + lane;
    const double cd = I.m.M[e] + I.delta * I.m.K[e];
    const double cs = I.m.M[e] + I.sdelta * I.m.K[e];
    if (!I.shared_ops) {
      ((T*)I.Cd)[e] = T(cd);
      ((T*)I.Csd)[e] = T(cs);
    }
    if (I.m.col[e] == i) { dd += cd; ds += cs; }
  }
  if (i < I.n) {
    ((T*)I.dinvCd)[i] = T(1.0 / dd);
    ((T*)I.dinvCsd)[i] = T(1.0 / ds);
  }
}

// S_D = M - 2 delta K + delta K M_D^{-1} K on the second-ring pattern (Section 4.1)
// and its Jacobi diagonal, in the inner precision.
template <typename T>
__global__ void k_prep_sd(InstDev I) {
  const int sl = blockIdx.x * PFC_WAVES + (threadIdx.x >> 6);
  if (sl >= I.m.n_slices) return;
  const int lane = threadIdx.x & 63;
  const int i = sl * 64 + lane;
  const int base = I.m.w_slice_ptr[sl];
  const int w = (I.m.w_slice_ptr[sl + 1] - base) >> 6;
  double dg = 0.0;
  for (int k = 0; k < w; ++k) {
    const long long e = (long long)base + k * 64 + lane;
    const long long p = I.m.w_p1pos[e];
    double v = p >= 0 ? I.m.M[p] - 2.0 * I.delta * I.m.K[p] : 0.0;
    double acc = 0.0;
    for (int t = I.m.w_tri_ptr[e]; t < I.m.w_tri_ptr[e + 1]; ++t) {
      const int e1 = I.m.w_tri[2 * t], e2 = I.m.w_tri[2 * t + 1];
      acc += I.m.K[e1] * I.m.dinvM[I.m.col[e1]] * I.m.K[e2];
    }
    v += I.delta * acc;
    ((T*)I.SDv)[e] = T(v);
    if (I.m.w_col[e] == i) dg += v;
  }
  if (i < I.n) ((T*)I.dinvSD)[i] = T(1.0 / dg);
}

__global__ void k_assemble_N_sell(InstDev I, const double* __restrict__ psi) {
  const int sl = blockIdx.x * PFC_WAVES + (threadIdx.x >> 6);
  if (sl >= I.m.n_slices) return;
  const int lane = threadIdx.x & 63;
  const int base = I.m.slice_ptr[sl];
  const int w = (I.m.slice_ptr[sl + 1] - base) >> 6;
  for (int k = 0; k < w; ++k) {
    const long long e = (long long)base + k * 64 + lane;
    I.N[e] = -3.0 * entry_Mpsi2(I.m, e, [&](int j) { return psi[j]; });
  }
}

// K_+(psi) and F(mu) of the PFC1 model on the P1 pattern, in place
__global__ void k_assemble_mob(InstDev I, const double* __restrict__ psi, const double* __restrict__ mu) {
  const int sl = blockIdx.x * PFC_WAVES + (threadIdx.x >> 6);
  if (sl >= I.m.n_slices) return;
  const int lane = threadIdx.x & 63;
  const int base = I.m.slice_ptr[sl];
  const int w = (I.m.slice_ptr[sl + 1] - base) >> 6;
  for (int k = 0; k < w; ++k) {
    const long long e = (long long)base + k * 64 + lane;
    I.Kp[e] = entry_Kplus(I.m, e, [&](int j) { return psi[j]; }, I.psi_min);
    I.Fm[e] = entry_F(I.m, e, [&](int j) { return mu[j]; });
  }
}

// per slice: sum of (M psi)_i and of (M 1)_i over its rows (the mobility mean
// M0 = 1^T M psi / 1^T M 1 - psi_min is formed on the host in slice order)
__global__ void k_mass_moments(InstDev I, const double* __restrict__ psi) {
  const int sl = blockIdx.x * PFC_WAVES + (threadIdx.x >> 6);
  if (sl >= I.m.n_slices) return;
  const int lane = threadIdx.x & 63;
  const int base = I.m.slice_ptr[sl];
  const int w = (I.m.slice_ptr[sl + 1] - base) >> 6;
  double a = 0.0, b = 0.0;
  for (int k = 0; k < w; ++k) {
    const long long e = (long long)base + k * 64 + lane;
    a += I.m.M[e] * psi[I.m.col[e]];
    b += I.m.M[e];
  }
  a = wave_sum(a);
  b = wave_sum(b);
  if (lane == 0) { I.errpart[sl] = a; I.errpart[I.m.n_slices + sl] = b; }
}

__global__ void k_apply_AR(InstDev I, const double* __restrict__ y, double* __restrict__ out) {
  const int sl = blockIdx.x * PFC_WAVES + (threadIdx.x >> 6);
  if (sl >= I.m.n_slices) return;
  const int lane = threadIdx.x & 63;
  const int i = sl * 64 + lane;
  const int n = I.n;
  double w0, w1, w2;
  const PatView<PFC_COL_MEM> pv{I.m.slice_ptr, I.m.col, I.m.uw, 0, I.n, 0, 0.0f, nullptr};
  auto yv = [&](int j, double& mu, double& ps, double& om) { mu = y[j]; ps = y[n + j]; om = y[2 * n + j]; };
  if (I.model == PFC_MODEL_PFC1) block_row<PFC_COL_MEM, true>(I, pv, sl, lane, I.tau, I.m11, yv, w0, w1, w2);
  else block_row<PFC_COL_MEM, false>(I, pv, sl, lane, I.tau, I.m11, yv, w0, w1, w2);
  if (i < n) { out[i] = w0; out[n + i] = w1; out[2 * n + i] = w2; }
}

// Embedded error of the step just taken (psi block): per slice the sum of
// ((psi_{k+1} - psi_hat) / (atol + rtol max(|psi_k|, |psi_{k+1}|)))^2 with
// psi_hat = psi_k + sum_j mhat_j y_j^psi (Table rosenbrock_scheme).
__global__ void k_embedded_err(InstDev I, const double* __restrict__ xold, const double* __restrict__ xnew, double rtol,
                               double atol) {
  const int sl = blockIdx.x;
  const int lane = threadIdx.x;
  const int n = I.n;
  const long long n3 = 3LL * n;
  const int i = sl * 64 + lane;
  double e2 = 0.0;
  if (i < n) {
    const double po = xold[n + i], pn = xnew[n + i];
    const double ph = po + ROS_MH1 * I.ys[n + i] + ROS_MH2 * I.ys[n3 + n + i] + ROS_MH3 * I.ys[2 * n3 + n + i];
    const double sc = atol + rtol * fmax(fabs(po), fabs(pn));
    const double e = (pn - ph) / sc;
    e2 = e * e;
  }
  e2 = wave_sum(e2);
  if (lane == 0) I.errpart[sl] = e2;
}

__global__ void k_stage_rhs(InstDev I, int stage, double* __restrict__ b) {
  const int sl = blockIdx.x * PFC_WAVES + (threadIdx.x >> 6);
  if (sl >= I.m.n_slices) return;
  const int lane = threadIdx.x & 63;
  const int i = sl * 64 + lane;
  double b0, b1, b2;
  const PatView<PFC_COL_MEM> pv{I.m.slice_ptr, I.m.col, I.m.uw, 0, I.n, 0, 0.0f, nullptr};
  stage_rhs_row<PFC_COL_MEM>(I, pv, sl, lane, stage, b0, b1, b2);
  if (i < I.n) { b[i] = b0; b[I.n + i] = b1; b[2 * I.n + i] = b2; }
}

// ---- host side ------------------------------------------------------------------

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Halo of the two-iterations-per-launch PCG (N + 1 rows), or 0 where it does not
// apply: float64 single-reduction instances on 2D periodic grids (7 entries per
// row) with computed columns, at most PFC_WAVES slices per workgroup, every
// neighbour within N + 1 rows of its row (mod n), the three LDS arrays within
// PFC_SS_LDS and the halo ranges within the kernel's unrolled passes.
static int sstep_halo(const pfc_mesh* m, const pfc_opts& o, int team_size) {
  const MeshDev& d = m->dev;
  if (o.pcg_steps_per_launch != 2 || o.precision != PFC_FP64 || o.single_reduction != 1 || o.grid_columns != 1) return 0;
  if (d.dim != 2 || d.gN < 3 || d.uw != 7 || team_size < 1) return 0;
  const int spw = (d.n_slices + team_size - 1) / team_size;
  if (spw > PFC_WAVES) return 0;
  const int n = d.n, H = d.gN + 1;
  if (2 * H >= n) return 0;
  for (int c = 0; c < 9; ++c)  // the row classes of a 2D grid
    for (int k = 0; k < d.uw; ++k) {
      int s = d.glin[c * PFC_GRID_W + k];
      s = s > n / 2 ? s - n : (s < -(n / 2) ? s + n : s);
      if (s > H || s < -H) return 0;
    }
  const int rmax = std::min(spw * 64, n);
  if (3 * rmax + 8 * H > PFC_SS_LDS || rmax + 4 * H > PFC_SS_NA * PFC_WG || rmax + 2 * H > PFC_SS_NB * PFC_WG) return 0;
  return H;
}

// Two PCG iterations per launch on blocks of a 3D grid (ph_scg3): float
// (mixed-precision) single-reduction instances on periodic grids of side 64 with
// computed columns and entry directions, one row per thread (a team of 256
// workgroups of 4 x 4 x-lines).
static bool sstep_block3(const pfc_mesh* m, const pfc_opts& o, int team_size) {
  const MeshDev& d = m->dev;
  return o.pcg_steps_per_launch == 2 && o.precision == PFC_MIXED && o.single_reduction == 1 && o.grid_columns == 1 &&
         d.dim == 3 && d.gN == PFC_S3_N && d.uw == 15 && d.gdir_ok && team_size == 256 && d.n_slices == 4096;
}

// Two PCG iterations per launch on blocks of a 2D grid (ph_scg2b): single-
// reduction instances (either precision) on periodic grids whose side is a
// multiple of 64, with computed columns and entry directions, one row per
// thread (a team of N^2 / 1024 workgroups of 64 x 16 rows).
static bool sstep_block2(const pfc_mesh* m, const pfc_opts& o, int team_size) {
  const MeshDev& d = m->dev;
  return o.pcg_steps_per_launch == 2 && o.single_reduction == 1 && o.grid_columns == 1 && d.dim == 2 &&
         d.gN >= 64 && d.gN % 64 == 0 && d.uw == 7 && d.gdir_ok && d.n_slices % PFC_WAVES == 0 &&
         team_size == d.n_slices / PFC_WAVES;
}

bool block_form_applies(const pfc_mesh* m, const pfc_opts& o) {
  pfc_opts o2 = o;
  o2.pcg_steps_per_launch = 2;
  return sstep_block2(m, o2, team_size_for(m->n_slices, o.rows_per_thread));
}

// Carve the instance arena.  With base == nullptr only the size is computed.
size_t carve(InstDev& h, char* base, const pfc_mesh* m, const pfc_opts& o, int team_size) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off += align_up(bytes);
    return p;
  };
  const size_t n = (size_t)m->n, n3 = 3 * n, ns = (size_t)m->nnz_sell;
  const size_t w = o.precision == PFC_MIXED ? 4 : 8;
  const int mr = o.restart;
  if (o.schur_variant == 1) {
    h.SDv = take((size_t)m->dev.w_nnz_sell * w);
    h.dinvSD = take(n * w);
  } else {
    h.SDv = nullptr;
    h.dinvSD = nullptr;
  }
  h.Cd = o.shared_ops ? nullptr : (void*)take(ns * w);
  h.Csd = o.shared_ops ? nullptr : (void*)take(ns * w);
  h.dinvCd = take(n * w);
  h.dinvCsd = take(n * w);
  h.N = (double*)take(ns * 8);
  if (o.model == PFC_MODEL_PFC1) {
    h.Kp = (double*)take(ns * 8);
    h.Fm = (double*)take(ns * 8);
  } else {
    h.Kp = nullptr;
    h.Fm = nullptr;
  }
  h.b = (double*)take(n3 * 8);
  h.xk = (double*)take(n3 * 8);
  h.ys = (double*)take(3 * n3 * 8);
  h.V = (double*)take((size_t)(mr + 1) * n3 * 8);
  h.Z = (double*)take((size_t)mr * n3 * 8);
  h.W = (double*)take(n3 * 8);
  h.r_ = take(n * 8); h.pA = take(n * 8); h.pB = take(n * 8); h.q = take(n * 8);
  h.y0 = take(n * 8); h.y1 = take(n * 8); h.zt = take(n * 8); h.x1 = take(n * 8); h.x2 = take(n * 8);
  h.rB = take(n * 8); h.wB = take(n * 8); h.sA = take(n * 8); h.sB = take(n * 8);
  h.xbak = (double*)take(n3 * 8);
  h.errpart = (double*)take((size_t)m->n_slices * 2 * 8);
  h.part = (double*)take(2 * (size_t)team_size * 4 * sizeof(double));
  h.gpart = (double*)take(2 * (size_t)team_size * PFC_GS_NV * sizeof(double));
  h.sH = sstep_halo(m, o, team_size);
  h.sstep = sstep_block2(m, o, team_size) ? 3 : (h.sH > 0 ? 1 : (sstep_block3(m, o, team_size) ? 2 : 0));
  h.sbas = h.sstep ? (double*)take(10 * n * 8) : nullptr;
  h.spart = h.sstep ? (double*)take(2 * (size_t)team_size * 32 * sizeof(double)) : nullptr;
  h.st = (State*)take(2 * sizeof(State));
  h.hist = (Hist*)take(sizeof(Hist));
  h.rec_inner = (int*)take((size_t)o.max_steps * 5 * sizeof(int));
  h.info = (InfoDev*)take((size_t)3 * o.max_run_steps * sizeof(InfoDev));
  h.max_infos = 3 * o.max_run_steps;
  return off;
}

int team_size_for(int n_slices, int rows_per_thread) {
  int rpt = rows_per_thread;
  if (rpt <= 0) rpt = 1;
  return (n_slices + PFC_WAVES * rpt - 1) / (PFC_WAVES * rpt);
}

static int validate_opts(const pfc_opts* o) {
  if (!o || o->struct_size != (int)sizeof(pfc_opts)) { set_error("pfc_opts: struct_size mismatch"); return PFC_ERR_ARG; }
  if (o->precision != PFC_FP64 && o->precision != PFC_MIXED) { set_error("pfc_opts: bad precision"); return PFC_ERR_ARG; }
  if (o->restart < 1 || o->restart > PFC_MAXM) { set_error("pfc_opts: restart must be in 1..32"); return PFC_ERR_ARG; }
  if (o->max_steps < 1 || o->inner_maxit < 1 || o->max_run_steps < 1) { set_error("pfc_opts: counts must be positive"); return PFC_ERR_ARG; }
  if (!(o->outer_tol > 0.0) || !(o->inner_tol > 0.0) || !(o->inner_tol < 1.0)) { set_error("pfc_opts: tolerances must be in (0,1)"); return PFC_ERR_ARG; }
  if (o->rows_per_thread < 0 || o->rows_per_thread > 8) { set_error("pfc_opts: rows_per_thread must be 0..8"); return PFC_ERR_ARG; }
  if (o->ticks_per_graph < 0 || o->ticks_per_graph > 4096) { set_error("pfc_opts: ticks_per_graph must be 0..4096"); return PFC_ERR_ARG; }
  if (o->single_reduction != 0 && o->single_reduction != 1) { set_error("pfc_opts: single_reduction must be 0 or 1"); return PFC_ERR_ARG; }
  if (o->schur_variant != 0 && o->schur_variant != 1) { set_error("pfc_opts: schur_variant must be 0 (S_CH) or 1 (S_D)"); return PFC_ERR_ARG; }
  if (o->sd_iters < 1 || o->sd_iters > 10000) { set_error("pfc_opts: sd_iters must be in 1..10000"); return PFC_ERR_ARG; }
  if (o->model != PFC_MODEL_PFC2 && o->model != PFC_MODEL_PFC1) { set_error("pfc_opts: bad model"); return PFC_ERR_ARG; }
  if (!std::isfinite(o->psi_min)) { set_error("pfc_opts: psi_min must be finite"); return PFC_ERR_ARG; }
  if (o->grid_columns != 0 && o->grid_columns != 1) { set_error("pfc_opts: grid_columns must be 0 or 1"); return PFC_ERR_ARG; }
  if (o->pcg_steps_per_launch != 1 && o->pcg_steps_per_launch != 2) {
    set_error("pfc_opts: pcg_steps_per_launch must be 1 or 2");
    return PFC_ERR_ARG;
  }
  if (o->gamma_mode != PFC_GAMMA_SCALE_ROW && o->gamma_mode != PFC_GAMMA_LITERAL) {
    set_error("pfc_opts: bad gamma_mode");
    return PFC_ERR_ARG;
  }
  for (int k = 0; k < 5; ++k)
    if (o->inner_fixed[k] < 0 || o->inner_fixed[k] > 100000) {
      set_error("pfc_opts: inner_fixed counts must be in 0..100000");
      return PFC_ERR_ARG;
    }
  return PFC_OK;
}

void fill_info(pfc_solve_info* dst, const InfoDev& s) {
  dst->status = s.status;
  dst->outer_iters = s.outer_iters;
  dst->cycles = s.cycles;
  dst->inner_applies = s.inner_applies;
  dst->inner_total = s.inner_total;
  for (int k = 0; k < 5; ++k) dst->inner_max[k] = s.inner_max[k];
  dst->reserved = 0;
  dst->est_rel_res = s.est_rel_res;
  dst->true_rel_res = s.true_rel_res;
  dst->t_solve = s.t_solve;
}

// The descriptors (h_descs) must be filled before build(): a one-instance
// group bakes that instance's state and partial-sum buffers into the launches.
int Group::build(hipStream_t capture, int precision, int ticks) {
  graph_ticks = ticks;
  for (int i = 0; i < count; ++i)
    if (!h_descs[i].st || !h_descs[i].part || h_descs[i].team_size <= 0) {
      set_error("internal: launch group built before its descriptors were set");
      return PFC_ERR_STATE;
    }
  if (count == 1 && h_descs[0].team_size != n_wg) {
    set_error("internal: team size mismatch");
    return PFC_ERR_STATE;
  }
  // the mesh pattern of every team entry, and whether the launches stage the
  // columns.  They can when every mesh has a uniform slice width <= PFC_LCOL_W
  // and a workgroup owns at most PFC_WAVES slices (the staging buffer holds
  // exactly that).  Staging moves the column stream into the prologue's round
  // trip; it pays where that stream is a large share of a launch's bytes
  // (measured: 3D 64^3 mixed +5.7%, the mixed 2D/3D served mix +6%, 2D 512^2
  // float64 -2%, where the 7 columns are 16% of an iteration's bytes), so
  // float64 runs stage only from 8 columns per row on (3D: 22%).  When every
  // mesh of the launch is a periodic grid (MeshDev::gN), the columns are
  // computed from the row instead and no column stream is read at all
  // (measured against the stored forms: 2D 512^2 float64 +8.7%, 3D 64^3 mixed
  // +17%, the served mix +11%, the batched 128^2 mixed run with 4 rows per
  // thread +5.5%).
  bool lds = true, grid = true;
  for (TeamEntry& t : h_teams) {
    const MeshDev& m = h_descs[t.inst].m;
    t.uw = m.uw;
    t.col = m.col;
    t.n_slices = m.n_slices;
    if (!(m.uw >= 1 && m.uw <= PFC_LCOL_W && (m.n_slices + t.size - 1) / t.size <= PFC_WAVES)) lds = false;
    if (precision == PFC_FP64 && m.uw < 8) lds = false;
    if (!(m.gN > 0 && m.uw >= 1) || !h_descs[t.inst].grid_cols) grid = false;
  }
#ifdef PFC_NO_COLUMN_STAGING
  lds = false;
#endif
  cols = grid ? PFC_COL_GRID : (lds ? PFC_COL_LDS : PFC_COL_MEM);
  PFC_HIP(hipMemcpy(d_teams, h_teams.data(), sizeof(TeamEntry) * h_teams.size(), hipMemcpyHostToDevice));
  const int* pcol = count == 1 ? h_descs[0].m.col : nullptr;
  const int puw = count == 1 ? h_descs[0].m.uw : 0;
  const int pnsl = count == 1 ? h_descs[0].m.n_slices : 0;
  PFC_HIP(hipStreamBeginCapture(capture, hipStreamCaptureModeThreadLocal));
  for (int t = 0; t < ticks; ++t) {
    const int par = t & 1;
    State* sin = nullptr;
    State* sout = nullptr;
    double* pin = nullptr;
    double* pout = nullptr;
    const double* gin = nullptr;
    if (count == 1) {
      sin = h_descs[0].st + par;
      sout = h_descs[0].st + (1 - par);
      pin = h_descs[0].part + (size_t)par * n_wg * 4;
      pout = h_descs[0].part + (size_t)(1 - par) * n_wg * 4;
      if (h_descs[0].spart) gin = h_descs[0].spart + (size_t)par * n_wg * 32;
    }
#define PFC_TICK(TT, SG, LD, BB)                                                                              \
  hipLaunchKernelGGL((k_tick<TT, SG, LD, BB>), dim3(n_wg), dim3(PFC_WG), 0, capture, d_teams, d_descs, sin, sout, pin, \
                     pout, par, pcol, puw, pnsl, gin)
#define PFC_TICK_COLS(TT, SG)                                                  \
  switch (cols) {                                                              \
    case PFC_COL_GRID:                                                         \
      if (b2) { PFC_TICK(TT, SG, PFC_COL_GRID, true); }                        \
      else { PFC_TICK(TT, SG, PFC_COL_GRID, false); }                          \
      break;                                                                   \
    case PFC_COL_LDS: PFC_TICK(TT, SG, PFC_COL_LDS, false); break;             \
    default: PFC_TICK(TT, SG, PFC_COL_MEM, false); break;                      \
  }
    const bool sg = (count == 1);
    // the launches have the 2D block form (ph_scg2b) when some instance takes it;
    // the other instances run one PCG iteration per launch in them
    bool b2 = false;
    for (int i = 0; i < count; ++i) b2 = b2 || h_descs[i].sstep == 3;
    if (precision == PFC_MIXED) {
      if (sg) { PFC_TICK_COLS(float, true); } else { PFC_TICK_COLS(float, false); }
    } else {
      if (sg) { PFC_TICK_COLS(double, true); } else { PFC_TICK_COLS(double, false); }
    }
#undef PFC_TICK_COLS
#undef PFC_TICK
  }
  hipLaunchKernelGGL(k_report, dim3((count + 255) / 256), dim3(256), 0, capture, d_descs, count, d_flags);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(capture, &g);
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  return PFC_OK;
}

int Group::alloc(const std::vector<int>& team_sizes) {
  count = (int)team_sizes.size();
  h_teams.clear();
  for (int i = 0; i < count; ++i)
    for (int r = 0; r < team_sizes[i]; ++r) h_teams.push_back(TeamEntry{i, r, team_sizes[i], 0, nullptr, 0, 0});
  n_wg = (int)h_teams.size();
  PFC_HIP(hipMalloc((void**)&d_teams, sizeof(TeamEntry) * h_teams.size()));
  PFC_HIP(hipMalloc((void**)&d_descs, sizeof(InstDev) * count));
  PFC_HIP(hipHostMalloc((void**)&h_descs, sizeof(InstDev) * count, hipHostMallocDefault));
  PFC_HIP(hipHostMalloc((void**)&h_states, sizeof(State) * count, hipHostMallocDefault));
  PFC_HIP(hipHostMalloc((void**)&h_flags, sizeof(int) * count, hipHostMallocMapped));
  PFC_HIP(hipHostGetDevicePointer((void**)&d_flags, h_flags, 0));
  for (int i = 0; i < count; ++i) h_flags[i] = -1;
  PFC_HIP(hipEventCreateWithFlags(&ev[0], hipEventDisableTiming));
  PFC_HIP(hipEventCreateWithFlags(&ev[1], hipEventDisableTiming));
  return PFC_OK;
}

void Group::release() {
  if (exec) (void)hipGraphExecDestroy(exec);
  if (d_teams) (void)hipFree(d_teams);
  if (d_descs) (void)hipFree(d_descs);
  if (h_descs) (void)hipHostFree(h_descs);
  if (h_states) (void)hipHostFree(h_states);
  if (h_flags) (void)hipHostFree(h_flags);
  if (ev[0]) (void)hipEventDestroy(ev[0]);
  if (ev[1]) (void)hipEventDestroy(ev[1]);
  *this = Group();
}

// Upload descriptors and initial states (stream ordered), then replay the
// graph until every instance reports PH_DONE.
int Group::run(hipStream_t s, const std::vector<State*>& dev_states, double timeout_s) {
  PFC_HIP(hipMemcpyAsync(d_descs, h_descs, sizeof(InstDev) * count, hipMemcpyHostToDevice, s));
  for (int i = 0; i < count; ++i)
    PFC_HIP(hipMemcpyAsync(dev_states[i], h_states + i, sizeof(State), hipMemcpyHostToDevice, s));
  const auto t0 = std::chrono::steady_clock::now();
  PFC_HIP(hipGraphLaunch(exec, s));
  PFC_HIP(hipEventRecord(ev[0], s));
  PFC_HIP(hipGraphLaunch(exec, s));
  PFC_HIP(hipEventRecord(ev[1], s));
  long long k = 0;
  for (;;) {
    PFC_HIP(hipEventSynchronize(ev[k & 1]));
    bool all = true;
    for (int i = 0; i < count; ++i)
      if (((volatile int*)h_flags)[i] != PH_DONE) { all = false; break; }
    if (all) break;
    const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (el > timeout_s) {
      (void)hipStreamSynchronize(s);
      set_error("solver did not finish within the time limit");
      return PFC_ERR_STATE;
    }
    PFC_HIP(hipGraphLaunch(exec, s));
    PFC_HIP(hipEventRecord(ev[k & 1], s));
    ++k;
  }
  graphs_run = k + 2;
  PFC_HIP(hipStreamSynchronize(s));
  return PFC_OK;
}

static int ensure_group(pfc_instance* I) {
  if (I->grp.exec) return PFC_OK;
  int rc = I->grp.alloc(std::vector<int>{I->team_size});
  if (rc) return rc;
  I->grp.h_descs[0] = I->h;
  return I->grp.build(I->capture, I->opts.precision, I->ticks);
}

static int prep_ops(pfc_instance* I, hipStream_t s) {
  const InstDev& h = I->h;
  if (I->ops_tau_s == h.tau_p) return PFC_OK;
  const int nb = slice_blocks(I->mesh->n_slices);
  if (I->opts.precision == PFC_MIXED)
    hipLaunchKernelGGL(k_prep_ops<float>, dim3(nb), dim3(PFC_WG), 0, s, h);
  else
    hipLaunchKernelGGL(k_prep_ops<double>, dim3(nb), dim3(PFC_WG), 0, s, h);
  if (h.schur_d) {
    if (I->opts.precision == PFC_MIXED)
      hipLaunchKernelGGL(k_prep_sd<float>, dim3(nb), dim3(PFC_WG), 0, s, h);
    else
      hipLaunchKernelGGL(k_prep_sd<double>, dim3(nb), dim3(PFC_WG), 0, s, h);
  }
  PFC_HIP(hipGetLastError());
  I->ops_tau_s = h.tau_p;
  return PFC_OK;
}

int prep_ops_public(pfc_instance* I, hipStream_t s) { return prep_ops(I, s); }

// h.m0 (mobility mean, 1 for PFC2) and h.gamma_mode must be current: FGMRES
// sees block row 1 multiplied by rs, and the preconditioner is built for the
// time step tau_p = m0 rs tau
void set_params(InstDev& h, double r, double tau, double m11) {
  h.r = r; h.tau = tau; h.m11 = m11;
  // (row scaling keeps the arithmetic tau / m11 and an exact unit m11_s)
  const bool lit = (h.gamma_mode == PFC_GAMMA_LITERAL);
  h.rs = lit ? 1.0 : 1.0 / m11;
  h.m11_s = lit ? m11 : 1.0;
  h.tau_s = lit ? tau : tau / m11;
  h.tau_p = h.m0 * h.tau_s;
  h.delta = std::sqrt(h.tau_p);
  h.sdelta = std::sqrt(h.delta);
}

// Mobility mean M0 = (1^T M psi)/(1^T M 1) - psi_min of a PFC1 instance from
// psi (device [n]); PFC2 instances keep M0 = 1.
int set_mobility_mean(pfc_instance* I, const double* psi, hipStream_t s) {
  InstDev& h = I->h;
  if (h.model != PFC_MODEL_PFC1) { h.m0 = 1.0; return PFC_OK; }
  const int ns = I->mesh->n_slices;
  hipLaunchKernelGGL(k_mass_moments, dim3(slice_blocks(ns)), dim3(PFC_WG), 0, s, h, psi);
  PFC_HIP(hipGetLastError());
  std::vector<double> part((size_t)2 * ns);
  PFC_HIP(hipMemcpyAsync(part.data(), h.errpart, sizeof(double) * part.size(), hipMemcpyDeviceToHost, s));
  PFC_HIP(hipStreamSynchronize(s));
  double a = 0.0, b = 0.0;
  for (int k = 0; k < ns; ++k) { a += part[k]; b += part[ns + k]; }
  h.m0 = a / b - h.psi_min;
  if (!(h.m0 > 0.0) || !std::isfinite(h.m0)) {
    set_error("PFC1: the mean mobility of the state is not positive (psi below psi_min on average)");
    return PFC_ERR_ARG;
  }
  return PFC_OK;
}

static State initial_state(int job) {
  State s;
  std::memset(&s, 0, sizeof(s));
  s.phase = PH_START;
  s.job = job;
  return s;
}

// Replay schedules: uploaded into a growable device buffer of the instance.
static int upload_schedules(pfc_instance* I, const pfc_schedule* sch, int count, hipStream_t s) {
  std::vector<int> meta(4 * (size_t)count), cyc, inn;
  for (int k = 0; k < count; ++k) {
    const pfc_schedule& q = sch[k];
    if (q.n_cycles < 0 || q.n_applies < 0 || (q.n_cycles && !q.cycle_len) || (q.n_applies && !q.inner_counts)) {
      set_error("pfc_schedule: invalid schedule");
      return PFC_ERR_ARG;
    }
    int steps = 0;
    for (int c = 0; c < q.n_cycles; ++c) {
      if (q.cycle_len[c] < 1 || q.cycle_len[c] > I->opts.restart) {
        set_error("pfc_schedule: cycle length out of range");
        return PFC_ERR_ARG;
      }
      steps += q.cycle_len[c];
    }
    if (steps != q.n_applies || steps > I->opts.max_steps) {
      set_error("pfc_schedule: applications must equal the sum of cycle lengths and fit max_steps");
      return PFC_ERR_ARG;
    }
    meta[4 * k + 0] = (int)cyc.size();
    meta[4 * k + 1] = q.n_cycles;
    meta[4 * k + 2] = (int)(inn.size() / 5);
    meta[4 * k + 3] = q.n_applies;
    cyc.insert(cyc.end(), q.cycle_len, q.cycle_len + q.n_cycles);
    for (int a = 0; a < 5 * q.n_applies; ++a) {
      if (q.inner_counts[a] < 0 || q.inner_counts[a] > 100000) { set_error("pfc_schedule: bad inner count"); return PFC_ERR_ARG; }
      inn.push_back(q.inner_counts[a]);
    }
  }
  if (cyc.empty()) cyc.push_back(0);
  if (inn.empty()) inn.push_back(0);
  const size_t need = sizeof(int) * (meta.size() + cyc.size() + inn.size()) + 1024;
  if (need > I->sched_bytes) {
    if (I->d_sched) (void)hipFree(I->d_sched);
    I->d_sched = nullptr;
    PFC_HIP(hipMalloc((void**)&I->d_sched, need));
    I->sched_bytes = need;
  }
  PFC_HIP(hipStreamSynchronize(s));
  int* p = I->d_sched;
  PFC_HIP(hipMemcpy(p, meta.data(), sizeof(int) * meta.size(), hipMemcpyHostToDevice));
  PFC_HIP(hipMemcpy(p + meta.size(), cyc.data(), sizeof(int) * cyc.size(), hipMemcpyHostToDevice));
  PFC_HIP(hipMemcpy(p + meta.size() + cyc.size(), inn.data(), sizeof(int) * inn.size(), hipMemcpyHostToDevice));
  I->h.sched_meta = p;
  I->h.sched_cycles = p + meta.size();
  I->h.sched_inner = p + meta.size() + cyc.size();
  I->h.replay = 1;
  return PFC_OK;
}

// Scratch of the allocation-free operator apply (pfc_apply_AR_noalloc): the
// values of N(psi_k) on the mesh's stored pattern (PFC_NOALLOC_MAX_ENTRIES,
// include/pfc.h).  Every GPU the library runs
// on holds its own copy of this array, at its own address, until the process
// ends; host code reaches it only through the address resolved per device
// below (the array's name is a host-side stand-in, not a device address).
#define PFC_NOALLOC_MAX_DEVICES 64
static __device__ __align__(256) double scratch[PFC_NOALLOC_MAX_ENTRIES];
static std::mutex g_scratch_mu;
static double* g_scratch_dev[PFC_NOALLOC_MAX_DEVICES] = {};

// Device address of the current device's scratch array, resolved once per
// device (with that device current) and kept.
static int scratch_address(double** out) {
  int d = 0;
  PFC_HIP(hipGetDevice(&d));
  if (d < 0 || d >= PFC_NOALLOC_MAX_DEVICES) {
    set_error("pfc_apply_AR_noalloc: device ordinal beyond the supported " + std::to_string(PFC_NOALLOC_MAX_DEVICES));
    return PFC_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[d]) {
    void* p = nullptr;
    PFC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) { set_error("pfc_apply_AR_noalloc: no device address for the scratch array"); return PFC_ERR_HIP; }
    g_scratch_dev[d] = (double*)p;
  }
  *out = g_scratch_dev[d];
  return PFC_OK;
}

int run_single(pfc_instance* I, hipStream_t s, int job) {
  int rc = ensure_group(I);
  if (rc) return rc;
  I->h.job = job;
  I->grp.h_descs[0] = I->h;
  I->grp.h_states[0] = initial_state(job);
  return I->grp.run(s, std::vector<State*>{I->h.st}, I->timeout_s);
}

}  // namespace pfc

using namespace pfc;

extern "C" {

const char* pfc_status_str(int st) {
  switch (st) {
    case PFC_OK: return "ok";
    case PFC_NOT_CONVERGED: return "not converged";
    case PFC_WARN_TAU_CRITICAL: return "converged; tau at or above the critical time step";
    case PFC_ERR_ARG: return "invalid argument";
    case PFC_ERR_OOM: return "out of memory";
    case PFC_ERR_HIP: return "HIP runtime error";
    case PFC_ERR_BREAKDOWN: return "breakdown: non-finite residual or input";
    case PFC_ERR_ADMISSION: return "request exceeds the memory budget";
    case PFC_ERR_STATE: return "invalid state";
    default: return "unknown status";
  }
}

void pfc_opts_default(pfc_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->struct_size = (int)sizeof(pfc_opts);
  o->precision = PFC_FP64;
  o->restart = 30;
  o->max_steps = 1000;
  o->outer_tol = 1e-8;
  o->inner_tol = 1e-3;
  o->inner_maxit = 500;
  o->shared_ops = 0;
  o->rows_per_thread = 0;
  o->max_run_steps = 256;
  o->ticks_per_graph = 0;
  o->single_reduction = 1;
  o->schur_variant = 0;
  o->sd_iters = 20;
  o->model = PFC_MODEL_PFC2;
  o->psi_min = -1.5;
  o->grid_columns = 1;
  o->pcg_steps_per_launch = 2;
}

double pfc_tau_critical(double r, double psibar) {
  const double a = 1.0 - 3.0 * r - 9.0 * psibar * psibar;
  if (!(a > 1.0)) return INFINITY;
  const double s = std::sqrt(a);
  return 27.0 / (2.0 * (s - 1.0) * (s + 2.0) * (s + 2.0));
}

size_t pfc_instance_footprint(const pfc_mesh* m, const pfc_opts* o) {
  if (!m || validate_opts(o)) return 0;
  // the S_D layout is part of the mesh; build it (once) to know its size
  if (o->schur_variant == 1 && build_second_ring(const_cast<pfc_mesh*>(m))) return 0;
  InstDev h{};
  const int ts = team_size_for(m->n_slices, o->rows_per_thread);
  return carve(h, nullptr, m, *o, ts);
}

int pfc_instance_create(pfc_mesh* m, const pfc_opts* o, pfc_instance** out) {
  if (!m || !out) { set_error("pfc_instance_create: null argument"); return PFC_ERR_ARG; }
  int rc = validate_opts(o);
  if (rc) return rc;
  *out = nullptr;
  if (o->schur_variant == 1 && (rc = build_second_ring(m))) return rc;
  if (o->model == PFC_MODEL_PFC1 && (!m->dev.elem_K || m->degree != 1)) {
    set_error("pfc_instance_create: the PFC1 model needs a P1 mesh with element geometry (pfc_mesh_create_p1)");
    return PFC_ERR_ARG;
  }
  pfc_instance* I = new pfc_instance();
  I->mesh = m;
  I->opts = *o;
  I->team_size = team_size_for(m->n_slices, o->rows_per_thread);
  I->ticks = o->ticks_per_graph > 0 ? o->ticks_per_graph : 64;
  if (const char* t = std::getenv("PFC_TIMEOUT_S")) I->timeout_s = std::atof(t) > 0 ? std::atof(t) : I->timeout_s;
  if (I->ticks & 1) I->ticks += 1;
  InstDev& h = I->h;
  std::memset(&h, 0, sizeof(h));
  const size_t bytes = carve(h, nullptr, m, *o, I->team_size);
  if (hipMalloc((void**)&I->arena, bytes) != hipSuccess) {
    (void)hipGetLastError();
    delete I;
    set_error("pfc_instance_create: device allocation of " + std::to_string(bytes) + " bytes failed");
    return PFC_ERR_OOM;
  }
  I->bytes = bytes;
  carve(h, I->arena, m, *o, I->team_size);
  h.m = m->dev;  // includes the second-ring layout when it was built
  h.n = m->n;
  h.precision = o->precision;
  h.restart = o->restart;
  h.max_steps = o->max_steps;
  h.inner_maxit = o->inner_maxit;
  h.shared_ops = o->shared_ops;
  h.single_reduction = o->single_reduction;
  h.schur_d = o->schur_variant;
  h.sd_iters = o->sd_iters;
  h.model = o->model;
  h.psi_min = o->psi_min;
  h.grid_cols = o->grid_columns;
  h.gamma_mode = o->gamma_mode;
  for (int k = 0; k < 5; ++k) h.inner_fixed[k] = o->inner_fixed[k];
  h.m0 = 1.0;
  h.team_size = I->team_size;
  h.outer_tol = o->outer_tol;
  h.inner_tol = o->inner_tol;
  h.ci_tol = 1e-13;
  if (hipMemset(I->arena, 0, bytes) != hipSuccess || hipStreamCreate(&I->capture) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    pfc_instance_destroy(I);
    set_error("pfc_instance_create: HIP setup failed");
    return PFC_ERR_HIP;
  }
  *out = I;
  return PFC_OK;
}

void pfc_instance_destroy(pfc_instance* I) {
  if (!I) return;
  I->grp.release();
  if (I->capture) (void)hipStreamDestroy(I->capture);
  if (I->d_sched) (void)hipFree(I->d_sched);
  if (I->arena) (void)hipFree(I->arena);
  delete I;
}

// One stage solve at psi_k (and mu_k for the PFC1 mobility matrices).
static int solve_impl(pfc_instance* I, const double* psi_k, const double* mu_k, double r, double psibar, double tau,
                      double m11, const double* rhs, double* x, const pfc_schedule* replay, pfc_solve_info* info,
                      void* stream) {
  if (!I || !psi_k || !rhs || !x || !std::isfinite(r) || !std::isfinite(psibar) || !(tau > 0.0) ||
      !std::isfinite(tau) || !(m11 > 0.0) || !std::isfinite(m11)) {
    set_error("pfc_solve: invalid arguments");
    return PFC_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  InstDev& h = I->h;
  int rc0 = set_mobility_mean(I, psi_k, s);
  if (rc0) return rc0;
  set_params(h, r, tau, m11);
  h.b_user = rhs;
  h.x_user = x;
  h.replay = 0;
  h.n_steps = 0;
  h.init_mode = PFC_INIT_GIVEN;
  if (replay) {
    int rc = upload_schedules(I, replay, 1, s);
    if (rc) return rc;
  }
  int rc = prep_ops(I, s);
  if (rc) return rc;
  hipLaunchKernelGGL(k_assemble_N_sell, dim3(slice_blocks(I->mesh->n_slices)), dim3(PFC_WG), 0, s, h, psi_k);
  if (h.model == PFC_MODEL_PFC1)
    hipLaunchKernelGGL(k_assemble_mob, dim3(slice_blocks(I->mesh->n_slices)), dim3(PFC_WG), 0, s, h, psi_k, mu_k);
  PFC_HIP(hipGetLastError());
  rc = run_single(I, s, JOB_SOLVE);
  h.replay = 0;
  if (rc) return rc;
  InfoDev f;
  PFC_HIP(hipMemcpy(&f, h.info, sizeof(InfoDev), hipMemcpyDeviceToHost));
  I->last_applies = f.inner_applies;
  if (info) fill_info(info, f);
  int st = f.status;
  if (st == PFC_OK && tau >= pfc_tau_critical(r, psibar)) st = PFC_WARN_TAU_CRITICAL;
  return st;
}

int pfc_solve(pfc_instance* I, const double* psi_k, double r, double psibar, double tau, double m11,
              const double* rhs, double* x, const pfc_schedule* replay, pfc_solve_info* info, void* stream) {
  if (I && I->h.model == PFC_MODEL_PFC1) {
    set_error("pfc_solve: a PFC1 instance needs mu_k as well; use pfc_solve_x");
    return PFC_ERR_ARG;
  }
  return solve_impl(I, psi_k, nullptr, r, psibar, tau, m11, rhs, x, replay, info, stream);
}

int pfc_solve_x(pfc_instance* I, const double* x_k, double r, double psibar, double tau, double m11, const double* rhs,
                double* x, const pfc_schedule* replay, pfc_solve_info* info, void* stream) {
  if (!I || !x_k) { set_error("pfc_solve_x: invalid arguments"); return PFC_ERR_ARG; }
  return solve_impl(I, x_k + I->mesh->n, x_k, r, psibar, tau, m11, rhs, x, replay, info, stream);
}

int pfc_instance_launch_stats(const pfc_instance* I, long long* launches, long long* graphs) {
  if (!I) { set_error("pfc_instance_launch_stats: null instance"); return PFC_ERR_ARG; }
  if (graphs) *graphs = I->grp.graphs_run;
  if (launches) *launches = I->grp.graphs_run * (long long)I->grp.graph_ticks;
  return PFC_OK;
}

int pfc_instance_config(const pfc_instance* I, int* team_size, int* rows_per_thread, int* pcg_steps_per_launch,
                        int* grid_columns) {
  if (!I) { set_error("pfc_instance_config: null instance"); return PFC_ERR_ARG; }
  if (team_size) *team_size = I->team_size;
  if (rows_per_thread) *rows_per_thread = I->opts.rows_per_thread > 0 ? I->opts.rows_per_thread : 1;
  if (pcg_steps_per_launch) *pcg_steps_per_launch = I->h.sstep ? 2 : 1;
  if (grid_columns) *grid_columns = (I->h.grid_cols && I->mesh->dev.gN > 0 && I->mesh->dev.uw >= 1) ? 1 : 0;
  return PFC_OK;
}

int pfc_last_inner_counts(const pfc_instance* I, int* counts, int cap, int* n_applies) {
  if (!I || !counts || cap < 0 || !n_applies) { set_error("pfc_last_inner_counts: invalid arguments"); return PFC_ERR_ARG; }
  const int na = std::min(I->last_applies, I->opts.max_steps);
  *n_applies = na;
  const int k = std::min(na, cap);
  if (k > 0) PFC_HIP(hipMemcpy(counts, I->h.rec_inner, sizeof(int) * 5 * k, hipMemcpyDeviceToHost));
  return PFC_OK;
}

int pfc_rosenbrock_run(pfc_instance* I, double* state, double r, double psibar, double tau, int n_steps, int init,
                       const pfc_schedule* replays, pfc_solve_info* per_stage, void* stream) {
  if (!I || !state || !std::isfinite(r) || !std::isfinite(psibar) || !(tau > 0.0) || !std::isfinite(tau) ||
      n_steps < 0 || n_steps > I->opts.max_run_steps || (init != PFC_INIT_GIVEN && init != PFC_INIT_CONSISTENT)) {
    set_error("pfc_rosenbrock_run: invalid arguments (n_steps must be <= max_run_steps)");
    return PFC_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  InstDev& h = I->h;
  // PFC1: the mobility mean of the initial state (conserved by the scheme)
  int rc = set_mobility_mean(I, state + I->mesh->n, s);
  if (rc) return rc;
  set_params(h, r, tau, 1.0 / ROS_GAMMA);
  double* own_xk = h.xk;
  h.xk = state;
  h.replay = 0;
  if (replays) rc = upload_schedules(I, replays, 3 * n_steps, s);
  if (!rc) rc = prep_ops(I, s);
  if (!rc) {
    h.n_steps = n_steps;
    h.init_mode = init;
    rc = run_single(I, s, JOB_RB);
  }
  h.xk = own_xk;
  h.replay = 0;
  if (rc) return rc;
  std::vector<InfoDev> f((size_t)3 * n_steps);
  if (n_steps > 0) PFC_HIP(hipMemcpy(f.data(), h.info, sizeof(InfoDev) * f.size(), hipMemcpyDeviceToHost));
  State fin;
  PFC_HIP(hipMemcpy(&fin, h.st, sizeof(State), hipMemcpyDeviceToHost));
  int worst = PFC_OK;
  for (size_t k = 0; k < f.size(); ++k) {
    if (per_stage) fill_info(per_stage + k, f[k]);
    if (f[k].status < 0) worst = f[k].status;
    else if (worst >= 0 && f[k].status > worst) worst = f[k].status;
  }
  if (fin.status < 0) worst = fin.status;
  if (worst == PFC_OK && tau >= pfc_tau_critical(r, psibar)) worst = PFC_WARN_TAU_CRITICAL;
  return worst;
}

int pfc_rosenbrock_adaptive(pfc_instance* I, double* state, double r, double psibar, double tau0, double t_end,
                            double rtol, double atol, int max_attempts, int init, double* taus, int* n_accepted,
                            int* n_rejected, pfc_solve_info* infos, void* stream) {
  if (!I || !state || !taus || !n_accepted || !n_rejected || !std::isfinite(r) || !std::isfinite(psibar) ||
      !(tau0 > 0.0) || !(t_end > 0.0) || !std::isfinite(t_end) || !(rtol > 0.0) || !(atol > 0.0) || max_attempts < 1 ||
      (init != PFC_INIT_GIVEN && init != PFC_INIT_CONSISTENT)) {
    set_error("pfc_rosenbrock_adaptive: invalid arguments");
    return PFC_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  InstDev& h = I->h;
  const int n = I->mesh->n;
  const int ns = I->mesh->n_slices;
  double* own_xk = h.xk;
  h.xk = state;
  h.replay = 0;
  *n_accepted = 0;
  *n_rejected = 0;
  int rc = set_mobility_mean(I, state + n, s), worst = PFC_OK;
  std::vector<double> part(ns);
  long long graphs = 0;  // launch statistics of the whole call (one run per attempted step)
  if (!rc && init == PFC_INIT_CONSISTENT) {
    set_params(h, r, tau0, 1.0 / ROS_GAMMA);
    h.n_steps = 0;
    h.init_mode = PFC_INIT_CONSISTENT;
    rc = prep_ops(I, s);
    if (!rc) rc = run_single(I, s, JOB_RB);
    graphs += I->grp.graphs_run;
  }
  double t = 0.0, tau = tau0;
  bool after_reject = false;  // the step after a rejection may not grow
  for (int a = 0; !rc && a < max_attempts && t < t_end * (1.0 - 1e-14); ++a) {
    const double step = std::min(tau, t_end - t);
    if (hipMemcpyAsync(h.xbak, state, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess) { rc = PFC_ERR_HIP; break; }
    set_params(h, r, step, 1.0 / ROS_GAMMA);
    h.n_steps = 1;
    h.init_mode = PFC_INIT_GIVEN;
    rc = prep_ops(I, s);
    if (!rc) rc = run_single(I, s, JOB_RB);
    if (rc) break;
    graphs += I->grp.graphs_run;
    State fin;
    if (hipMemcpy(&fin, h.st, sizeof(State), hipMemcpyDeviceToHost) != hipSuccess) { rc = PFC_ERR_HIP; break; }
    if (infos) {  // the three stage solves of this attempt, accepted or not
      InfoDev f[3];
      if (hipMemcpy(f, h.info, sizeof(f), hipMemcpyDeviceToHost) != hipSuccess) { rc = PFC_ERR_HIP; break; }
      for (int k = 0; k < 3; ++k) fill_info(infos + 3 * (size_t)a + k, f[k]);
    }
    if (fin.status < 0) { worst = fin.status; break; }
    if (fin.status == PFC_NOT_CONVERGED) {  // a stage solve missed its tolerance: reject, retry with facmin * step
      *n_rejected += 1;
      if (hipMemcpyAsync(state, h.xbak, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess) { rc = PFC_ERR_HIP; break; }
      tau = step * 0.2;
      after_reject = true;
      continue;
    }
    if (fin.status > worst) worst = fin.status;
    hipLaunchKernelGGL(k_embedded_err, dim3(ns), dim3(64), 0, s, h, h.xbak, state, rtol, atol);
    if (hipGetLastError() != hipSuccess || hipMemcpyAsync(part.data(), h.errpart, sizeof(double) * ns, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) { rc = PFC_ERR_HIP; break; }
    double sum = 0.0;
    for (int k = 0; k < ns; ++k) sum += part[k];
    const double err = std::sqrt(sum / n);
    if (!std::isfinite(err)) { worst = PFC_ERR_BREAKDOWN; break; }
    const double facmax = (err <= 1.0 && after_reject) ? 1.0 : 5.0;
    if (err <= 1.0) {
      t += step;
      taus[*n_accepted] = step;
      *n_accepted += 1;
      after_reject = false;
      if (*n_accepted >= max_attempts) break;
    } else {
      *n_rejected += 1;
      after_reject = true;
      if (hipMemcpyAsync(state, h.xbak, sizeof(double) * 3 * (size_t)n, hipMemcpyDeviceToDevice, s) != hipSuccess) { rc = PFC_ERR_HIP; break; }
    }
    const double fac = err == 0.0 ? facmax : std::min(facmax, std::max(0.2, 0.9 * std::pow(err, -1.0 / 3.0)));
    tau = step * fac;
  }
  if (!rc && hipStreamSynchronize(s) != hipSuccess) rc = PFC_ERR_HIP;
  I->grp.graphs_run = graphs;
  h.xk = own_xk;
  if (rc) return rc;
  if (worst < 0) return worst;
  if (t < t_end * (1.0 - 1e-14)) return PFC_NOT_CONVERGED;
  return worst;
}

static int apply_AR_impl(pfc_instance* I, const double* psi_k, const double* mu_k, double r, double tau, double m11,
                         const double* y, double* out, void* stream) {
  if (!I || !psi_k || !y || !out || !std::isfinite(r) || !std::isfinite(tau) || !std::isfinite(m11)) {
    set_error("pfc_apply_AR: invalid arguments");
    return PFC_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  InstDev h = I->h;
  h.r = r; h.tau = tau; h.m11 = m11;
  const int nb = slice_blocks(I->mesh->n_slices);
  hipLaunchKernelGGL(k_assemble_N_sell, dim3(nb), dim3(PFC_WG), 0, s, h, psi_k);
  if (h.model == PFC_MODEL_PFC1) hipLaunchKernelGGL(k_assemble_mob, dim3(nb), dim3(PFC_WG), 0, s, h, psi_k, mu_k);
  hipLaunchKernelGGL(k_apply_AR, dim3(nb), dim3(PFC_WG), 0, s, h, y, out);
  PFC_HIP(hipGetLastError());
  PFC_HIP(hipStreamSynchronize(s));
  return PFC_OK;
}

int pfc_apply_AR(pfc_instance* I, const double* psi_k, double r, double tau, double m11, const double* y, double* out,
                 void* stream) {
  if (I && I->h.model == PFC_MODEL_PFC1) {
    set_error("pfc_apply_AR: a PFC1 instance needs mu_k as well; use pfc_apply_AR_x");
    return PFC_ERR_ARG;
  }
  return apply_AR_impl(I, psi_k, nullptr, r, tau, m11, y, out, stream);
}

int pfc_apply_AR_x(pfc_instance* I, const double* x_k, double r, double tau, double m11, const double* y, double* out,
                   void* stream) {
  if (!I || !x_k) { set_error("pfc_apply_AR_x: invalid arguments"); return PFC_ERR_ARG; }
  return apply_AR_impl(I, x_k + I->mesh->n, x_k, r, tau, m11, y, out, stream);
}

int pfc_apply_AR_noalloc(const pfc_mesh* m, const double* psi_k, double r, double tau, double m11, const double* y,
                         double* out, void* stream) {
  if (!m || !psi_k || !y || !out || !std::isfinite(r) || !std::isfinite(tau) || !std::isfinite(m11)) {
    set_error("pfc_apply_AR_noalloc: invalid arguments");
    return PFC_ERR_ARG;
  }
  if (m->nnz_sell > PFC_NOALLOC_MAX_ENTRIES) {
    set_error("pfc_apply_AR_noalloc: the mesh stores " + std::to_string(m->nnz_sell) +
              " matrix entries, more than the scratch buffer's " + std::to_string(PFC_NOALLOC_MAX_ENTRIES));
    return PFC_ERR_ARG;
  }
  double* N = nullptr;
  int rc = scratch_address(&N);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  InstDev h;
  std::memset(&h, 0, sizeof(h));
  h.m = m->dev;
  h.n = m->n;
  h.model = PFC_MODEL_PFC2;
  h.r = r; h.tau = tau; h.m11 = m11;
  h.N = N;
  const int nb = slice_blocks(m->n_slices);
  hipLaunchKernelGGL(k_assemble_N_sell, dim3(nb), dim3(PFC_WG), 0, s, h, psi_k);
  hipLaunchKernelGGL(k_apply_AR, dim3(nb), dim3(PFC_WG), 0, s, h, y, out);
  PFC_HIP(hipGetLastError());
  return PFC_OK;
}

int pfc_apply_pch(pfc_instance* I, double tau_s, const double* v, double* z, const int* fixed_counts, int* counts_out,
                  void* stream) {
  if (!I || !v || !z || !(tau_s > 0.0) || !std::isfinite(tau_s)) {
    set_error("pfc_apply_pch: invalid arguments");
    return PFC_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  InstDev& h = I->h;
  h.m0 = 1.0;  // tau_s is the preconditioner's own time step
  set_params(h, 0.0, tau_s, 1.0);
  h.pch_out = z;
  h.replay = 0;
  int rc = PFC_OK;
  if (fixed_counts) {
    int one = 1;
    pfc_schedule q{1, &one, 1, fixed_counts};
    rc = upload_schedules(I, &q, 1, s);
    if (rc) return rc;
  }
  rc = prep_ops(I, s);
  if (rc) return rc;
  PFC_HIP(hipMemcpyAsync(h.W, v, sizeof(double) * 3 * (size_t)h.n, hipMemcpyDeviceToDevice, s));
  rc = run_single(I, s, JOB_PCH);
  h.replay = 0;
  if (rc) return rc;
  if (counts_out) PFC_HIP(hipMemcpy(counts_out, h.rec_inner, sizeof(int) * 5, hipMemcpyDeviceToHost));
  return PFC_OK;
}

int pfc_stage_rhs(pfc_instance* I, const double* x_k, const double* ys, int stage, double r, double tau, double* b,
                  void* stream) {
  if (!I || !x_k || !ys || !b || stage < 1 || stage > 3 || !std::isfinite(r) || !std::isfinite(tau)) {
    set_error("pfc_stage_rhs: invalid arguments");
    return PFC_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  InstDev h = I->h;
  h.r = r; h.tau = tau;
  h.xk = const_cast<double*>(x_k);
  h.ys = const_cast<double*>(ys);
  hipLaunchKernelGGL(k_stage_rhs, dim3(slice_blocks(I->mesh->n_slices)), dim3(PFC_WG), 0, s, h, stage, b);
  PFC_HIP(hipGetLastError());
  PFC_HIP(hipStreamSynchronize(s));
  return PFC_OK;
}

int pfc_batch_run(pfc_instance* const* insts, int count, double* const* states, const double* r, const double* psibar,
                  const double* tau, int n_steps, int init, pfc_solve_info* infos, void* stream) {
  if (!insts || count <= 0 || !states || !r || !psibar || !tau || n_steps < 0 ||
      (init != PFC_INIT_GIVEN && init != PFC_INIT_CONSISTENT)) {
    set_error("pfc_batch_run: invalid arguments");
    return PFC_ERR_ARG;
  }
  const int prec = insts[0] ? insts[0]->opts.precision : -1;
  for (int i = 0; i < count; ++i) {
    if (!insts[i] || !states[i] || insts[i]->opts.precision != prec || n_steps > insts[i]->opts.max_run_steps ||
        !(tau[i] > 0.0) || !std::isfinite(tau[i]) || !std::isfinite(r[i])) {
      set_error("pfc_batch_run: instance " + std::to_string(i) + " invalid (null, mixed precision, or bad parameters)");
      return PFC_ERR_ARG;
    }
  }
  {
    std::vector<const pfc_instance*> sorted(insts, insts + count);
    std::sort(sorted.begin(), sorted.end());
    if (std::adjacent_find(sorted.begin(), sorted.end()) != sorted.end()) {
      set_error("pfc_batch_run: instances must be distinct");
      return PFC_ERR_ARG;
    }
  }
  hipStream_t s = (hipStream_t)stream;
  std::vector<int> ts(count);
  std::vector<State*> sts(count);
  for (int i = 0; i < count; ++i) {
    InstDev& h = insts[i]->h;
    int rcm = set_mobility_mean(insts[i], states[i] + insts[i]->mesh->n, s);
    if (rcm) return rcm;
    set_params(h, r[i], tau[i], 1.0 / ROS_GAMMA);
    h.replay = 0;
    ts[i] = insts[i]->team_size;
    sts[i] = h.st;
    int rc = prep_ops(insts[i], s);
    if (rc) return rc;
  }
  int ticks = insts[0]->ticks;
  if (insts[0]->opts.ticks_per_graph == 0) {  // auto: the autotuning table's value for this batch, if any
    const int tt = tuned_ticks(insts[0]->mesh, prec, count);
    if (tt > 0) ticks = tt + (tt & 1);
  }
  int rc = PFC_OK;
  auto one_pass = [&](int precision, int steps, int initm) -> int {
    Group g;
    int e = g.alloc(ts);
    if (!e) {
      for (int i = 0; i < count; ++i) {
        InstDev h = insts[i]->h;
        h.xk = states[i];
        h.job = JOB_RB;
        h.n_steps = steps;
        h.init_mode = initm;
        g.h_descs[i] = h;
        g.h_states[i] = initial_state(JOB_RB);
      }
      e = g.build(insts[0]->capture, precision, ticks);
    }
    if (!e) e = g.run(s, sts, insts[0]->timeout_s * count);
    g.release();
    return e;
  };
  rc = one_pass(prec, n_steps, init);
  if (rc) return rc;
  int worst = PFC_OK;
  std::vector<InfoDev> f((size_t)3 * n_steps);
  for (int i = 0; i < count; ++i) {
    if (n_steps > 0)
      PFC_HIP(hipMemcpy(f.data(), insts[i]->h.info, sizeof(InfoDev) * f.size(), hipMemcpyDeviceToHost));
    for (size_t k = 0; k < f.size(); ++k) {
      if (infos) fill_info(infos + (size_t)i * f.size() + k, f[k]);
      if (f[k].status < 0) worst = f[k].status;
      else if (worst >= 0 && f[k].status > worst) worst = f[k].status;
    }
  }
  return worst;
}

}  // extern "C"
