// Device functions of the PFC stage solver: the work of every solver phase,
// executed by one team of workgroups over its block of SELL-64 slices.
//
// Each thread owns row i = slice*64 + lane of the node numbering and, in the
// 3x3 block phases, the three entries i, n+i, 2n+i of a block vector.  Dot
// products are accumulated per thread in float64, reduced per wavefront by a
// fixed butterfly (lane 0's result is used), then per workgroup in fixed
// order, and stored as one partial per workgroup; the next launch sums the
// partials in fixed order.  Results are therefore bitwise reproducible and
// independent of what else runs in the same launch.
#pragma once
#include "pfc_internal.h"

namespace pfc {

struct Team {
  int rank, size;   // workgroup rank within the team, team size
  int wave, lane;   // wave within the workgroup, lane
  int lo;           // SELL position of the first staged column (pfc_lcol[0])
};

// Column indices of the P1 pattern for the workgroup's own slices, staged in
// LDS by the launch prologue when every slice of the mesh has the same width
// (at most PFC_LCOL_W) and a workgroup owns at most PFC_WAVES slices.  They are
// loaded in the same memory round trip as the solver state, which takes the
// index load off the critical path of every SpMV in the launch.
#define PFC_LCOL_W 16
#define PFC_LCOL (PFC_WAVES * 64 * PFC_LCOL_W)
__shared__ int pfc_lcol[PFC_LCOL];

// Where a launch takes the columns of the P1 pattern from: memory, the LDS
// staging buffer, or computed from the row (periodic grid meshes, grid_col).
#define PFC_COL_MEM 0
#define PFC_COL_LDS 1
#define PFC_COL_GRID 2

// Slice geometry and columns of a SELL pattern.  L: one of PFC_COL_*; the
// staged and computed forms need a uniform slice width uw.
template <int L>
struct PatView {
  const int* sp;    // slice offsets [n_slices + 1]
  const int* col;   // columns [nnz_sell]
  int uw;           // uniform slice width, or 0
  int lo;           // SELL position of pfc_lcol[0] (L == PFC_COL_LDS)
  int n, gN;        // grid columns (L == PFC_COL_GRID): grid_col with
  float gInv;       //   1/N and the offset table gd
  const int* gd;
  __device__ __forceinline__ int base(int sl) const {
    if constexpr (L != PFC_COL_MEM) return sl * 64 * uw;
    else return uw ? sl * 64 * uw : sp[sl];
  }
  __device__ __forceinline__ int width(int sl) const {
    if constexpr (L != PFC_COL_MEM) return uw;
    else return uw ? uw : ((sp[sl + 1] - sp[sl]) >> 6);
  }
  // column of stored entry e, which belongs to row i (entry e - base(sl) of
  // slice sl = i / 64 sits at position k = (e >> 6) - sl uw of its row)
  __device__ __forceinline__ int at(long long e, int i) const {
    if constexpr (L == PFC_COL_GRID) return grid_col(i, (int)(e >> 6) - (i >> 6) * uw, n, gN, gInv, gd);
    else if constexpr (L == PFC_COL_LDS) return pfc_lcol[(int)(e - lo)];
    else return col[e];
  }
};

template <int L>
__device__ __forceinline__ PatView<L> p1_pat(const InstDev& I, const Team& tm) {
  return PatView<L>{I.m.slice_ptr, I.m.col, I.m.uw, tm.lo, I.n, I.m.gN, I.m.gInv,
                    L == PFC_COL_GRID ? I.m.glin : nullptr};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct Red3 {
  double a, b, c;
};
__device__ __forceinline__ Red3 red3(double a, double b, double c = 0.0) { return Red3{a, b, c}; }

// Sum (a, b, c) over the workgroup; result valid in thread 0.
__device__ __forceinline__ Red3 wg_sum3(Red3 v, Red3* lds4) {
  v.a = wave_sum(v.a);
  v.b = wave_sum(v.b);
  v.c = wave_sum(v.c);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) lds4[wave] = v;
  __syncthreads();
  Red3 r = red3(0.0, 0.0, 0.0);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < PFC_WAVES; ++w) { r.a += lds4[w].a; r.b += lds4[w].b; r.c += lds4[w].c; }
  }
  __syncthreads();
  return r;
}

// Slices handled by this workgroup, cycled over its waves: a contiguous block
// where every slice of the mesh has the same width; where widths differ (P2
// meshes: vertex rows have 19 entries, edge rows 9, numbered in that order) the
// team's slices are dealt round robin (slice rank + size j), so that every
// workgroup, and every SIMD of it, gets its share of the wide slices.
#define PFC_SLICES(I, tm)                                                          \
  const bool _rr = (I).m.uw == 0;                                                  \
  const int _spw = ((I).m.n_slices + (tm).size - 1) / (tm).size;                   \
  const int _sbeg = _rr ? (tm).rank : (tm).rank * _spw;                            \
  const int _send = _rr ? (I).m.n_slices : min(_sbeg + _spw, (I).m.n_slices);      \
  const int _sstep = _rr ? (tm).size * PFC_WAVES : PFC_WAVES;                      \
  for (int sl = _sbeg + (_rr ? (tm).size * (tm).wave : (tm).wave); sl < _send; sl += _sstep)

// Row loops over the entries of a slice: the P1 meshes of this solver have 7
// (2D) or 15 (3D) entries per row, 2D P2 meshes 19 (vertex rows) or 9 (edge
// rows); for those widths the loop is unrolled (fully for 7, in chunks of 5 for
// 15 and of 3 for the P2 widths, to stay within the register budget) so that a
// wave issues the index, value and gather loads of many entries at once.
template <typename F>
__device__ __forceinline__ void for_width(int w, F f) {
  if (w == 7) {
#pragma unroll
    for (int k = 0; k < 7; ++k) f(k);
  } else if (w == 15) {
#pragma unroll 5
    for (int k = 0; k < 15; ++k) f(k);
  } else if (w == 9) {  // P2 edge rows (2D)
#pragma unroll 3
    for (int k = 0; k < 9; ++k) f(k);
  } else if (w == 19) {  // P2 vertex rows (2D)
#pragma unroll 3
    for (int k = 0; k < 19; ++k) f(k);
  } else {
    for (int k = 0; k < w; ++k) f(k);
  }
}

// Stores of phase outputs.  PFC_STORE_POLICY selects the cache policy:
// 0 plain (write-back L2), 1 agent-coherent write-through (sc1), 2 streaming (nt).
// Write-through is the default: every phase output is read by other XCDs in
// the next launch, and writing it through during the kernel shortens the
// cache write-back at the kernel boundary.
#ifndef PFC_STORE_POLICY
#define PFC_STORE_POLICY 1
#endif

// Every phase output and every operand lives in device memory (never LDS).  The
// solver's pointers come from the instance record in LDS, so the compiler cannot
// see that and issues flat accesses, which count against the LDS wait counter as
// well and complete in no guaranteed order: every wait for an LDS access then
// also waits for all memory accesses in flight.  Stores, and the loads of the
// phases that issue loads ahead of their use, therefore name the global address
// space explicitly.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gp(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

template <typename T>
__device__ __forceinline__ void vst(T* p, T v) {
#if PFC_STORE_POLICY == 1
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#elif PFC_STORE_POLICY == 2
  __builtin_nontemporal_store(v, gp(p));
#else
  *gp(p) = v;
#endif
}

// Workgroup placement.  The dispatcher deals the workgroups of a launch to the
// 8 XCDs in turn (workgroup b lands on XCD b mod 8), and each XCD has its own
// L2.  Rows a workgroup gathers from its neighbours' blocks are only reused
// from L2 when those neighbours sit on the same XCD, so the rank (row block)
// of a workgroup is renumbered to give every XCD one contiguous run of ranks:
// XCD x owns ranks [x*q + min(x, r), ...) with q = g / 8, r = g mod 8.  The
// map is a bijection of [0, g) for every g.
#ifndef PFC_XCD_MAP
#define PFC_XCD_MAP 1
#endif
#define PFC_XCDS 8
__device__ __forceinline__ int xcd_rank(int b, int g) {
#if PFC_XCD_MAP
  const int q = g / PFC_XCDS, r = g % PFC_XCDS, x = b % PFC_XCDS;
  return x * q + (x < r ? x : r) + b / PFC_XCDS;
#else
  (void)g;
  return b;
#endif
}

// ---- typed views ----------------------------------------------------------
template <typename T> struct TV;
template <> struct TV<double> {
  __device__ static const double* M(const InstDev& I) { return I.m.M; }
  __device__ static const double* K(const InstDev& I) { return I.m.K; }
  __device__ static const double* dM(const InstDev& I) { return I.m.dinvM; }
};
template <> struct TV<float> {
  __device__ static const float* M(const InstDev& I) { return I.m.Mf; }
  __device__ static const float* K(const InstDev& I) { return I.m.Kf; }
  __device__ static const float* dM(const InstDev& I) { return I.m.dinvMf; }
};

// ---- element integrals (exact for P1, Section 3) ----------------------------
// int_T psi_h^2 lambda_a lambda_b = |T| c_m (1 + [a==b]) [S1^2 + S2 + 2 S1 (pa + pb) + 2 (pa^2 + pb^2 + pa pb)]
// int_T psi_h^3 lambda_a         = |T| c_m [S1^3 + 3 S1 S2 + 2 S3 + 3 pa (S1^2 + S2) + 6 pa^2 S1 + 6 pa^3]
// with S_k = sum over the vertices of psi^k and c_m = m!/(m+4)!.
__device__ __forceinline__ double cm_of(int dim) { return dim == 2 ? (1.0 / 360.0) : (1.0 / 840.0); }

// P2 (Section 3, p = 2; integrands of degree 8, exact through the reference
// table C4[a][b][c][d] = int phi_a phi_b phi_c phi_d / |T|):
//   Mpsi2^T_ab             = |T| sum_{c,d} psi_c psi_d C4[a][b][c][d]
//   int_T psi_h^3 phi_a    = |T| sum_b psi_b sum_{c,d} psi_c psi_d C4[a][b][c][d]
template <int Q, typename PsiF>
__device__ __forceinline__ double entry_Mpsi2_p2(const MeshDev& m, long long e, PsiF psi) {
  double acc = 0.0;
  for (int t = m.sl_el_ptr[e]; t < m.sl_el_ptr[e + 1]; ++t) {
    const int pk = m.sl_el[t];
    const int el = pk >> 8, a = (pk >> 4) & 15, b = pk & 15;
    const int* en = m.elem_nodes + (long long)el * Q;
    double p[Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) p[c] = psi(en[c]);
    const double* C = m.p2_C4 + (a * Q + b) * Q * Q;
    double s = 0.0;
#pragma unroll 1
    for (int c = 0; c < Q; ++c) {  // one row of the table at a time keeps the register use low
      double r = 0.0;
#pragma unroll
      for (int d = 0; d < Q; ++d) r += C[c * Q + d] * p[d];
      s += p[c] * r;
    }
    acc += m.elem_vol[el] * s;
  }
  return acc;
}

template <int Q, typename PsiF>
__device__ __forceinline__ double node_psi3_p2(const MeshDev& m, int i, PsiF psi) {
  double acc = 0.0;
  for (int t = m.nd_el_ptr[i]; t < m.nd_el_ptr[i + 1]; ++t) {
    const int pk = m.nd_el[t];
    const int el = pk >> 4, a = pk & 15;
    const int* en = m.elem_nodes + (long long)el * Q;
    double p[Q];
#pragma unroll
    for (int c = 0; c < Q; ++c) p[c] = psi(en[c]);
    double s = 0.0;
#pragma unroll 1
    for (int b = 0; b < Q; ++b) {
      const double* C = m.p2_C4 + (a * Q + b) * Q * Q;
      double r2 = 0.0;
#pragma unroll 1
      for (int c = 0; c < Q; ++c) {
        double r = 0.0;
#pragma unroll
        for (int d = 0; d < Q; ++d) r += C[c * Q + d] * p[d];
        r2 += p[c] * r;
      }
      s += psi(en[b]) * r2;
    }
    acc += m.elem_vol[el] * s;
  }
  return acc;
}

// The P1 element sums below visit an element list in groups of PFC_EV: the
// loads of a group (list entries, then the elements' nodes, then psi there)
// are issued together instead of one dependent chain per visit, and the
// visits' terms are then added in list order as one visit at a time would.
#define PFC_EV 4  // entry sums
#define PFC_EVN 3  // node sums: psi there is a stage combination (up to three loads)
// psi at the vertices of element el, psi(node) supplied by a functor (p[3] = 0
// on triangles)
template <typename PsiF>
__device__ __forceinline__ void elem_psi4(const MeshDev& m, int el, PsiF psi, double* p) {
  const int k = m.dim + 1;
  const int* en = m.elem_nodes + (long long)el * k;
  const int n0 = en[0], n1 = en[1], n2 = en[2];
  const int n3 = k == 4 ? en[3] : n2;
  p[0] = psi(n0);
  p[1] = psi(n1);
  p[2] = psi(n2);
  p[3] = k == 4 ? psi(n3) : 0.0;
}

template <typename PsiF>
__device__ __forceinline__ double entry_Mpsi2(const MeshDev& m, long long e, PsiF psi) {
  if (m.degree == 2) return m.dim == 2 ? entry_Mpsi2_p2<6>(m, e, psi) : entry_Mpsi2_p2<10>(m, e, psi);
  double acc = 0.0;
  const double cm = cm_of(m.dim);
  const int t0 = m.sl_el_ptr[e], t1 = m.sl_el_ptr[e + 1];
  for (int t = t0; t < t1; t += PFC_EV) {
    int pk[PFC_EV];
#pragma unroll
    for (int u = 0; u < PFC_EV; ++u) pk[u] = m.sl_el[min(t + u, t1 - 1)];
    double p[PFC_EV][4], vol[PFC_EV];
#pragma unroll
    for (int u = 0; u < PFC_EV; ++u) {
      elem_psi4(m, pk[u] >> 4, psi, p[u]);
      vol[u] = m.elem_vol[pk[u] >> 4];
    }
#pragma unroll
    for (int u = 0; u < PFC_EV; ++u) {
      if (t + u >= t1) break;
      const int a = (pk[u] >> 2) & 3, b = pk[u] & 3;
      double S1 = 0.0, S2 = 0.0;
      for (int v = 0; v <= m.dim; ++v) { S1 += p[u][v]; S2 += p[u][v] * p[u][v]; }
      const double pa = p[u][a], pb = p[u][b];
      const double s = S1 * S1 + S2 + 2.0 * S1 * (pa + pb) + 2.0 * (pa * pa + pb * pb + pa * pb);
      acc += vol[u] * cm * (a == b ? 2.0 : 1.0) * s;
    }
  }
  return acc;
}

template <typename PsiF>
__device__ __forceinline__ double node_psi3(const MeshDev& m, int i, PsiF psi) {
  if (m.degree == 2) return m.dim == 2 ? node_psi3_p2<6>(m, i, psi) : node_psi3_p2<10>(m, i, psi);
  double acc = 0.0;
  const double cm = cm_of(m.dim);
  const int t0 = m.nd_el_ptr[i], t1 = m.nd_el_ptr[i + 1];
  for (int t = t0; t < t1; t += PFC_EVN) {
    int pk[PFC_EVN];
#pragma unroll
    for (int u = 0; u < PFC_EVN; ++u) pk[u] = m.nd_el[min(t + u, t1 - 1)];
    double p[PFC_EVN][4], vol[PFC_EVN];
#pragma unroll
    for (int u = 0; u < PFC_EVN; ++u) {
      elem_psi4(m, pk[u] >> 2, psi, p[u]);
      vol[u] = m.elem_vol[pk[u] >> 2];
    }
#pragma unroll
    for (int u = 0; u < PFC_EVN; ++u) {
      if (t + u >= t1) break;
      const int a = pk[u] & 3;
      double S1 = 0.0, S2 = 0.0, S3 = 0.0;
      for (int v = 0; v <= m.dim; ++v) { S1 += p[u][v]; S2 += p[u][v] * p[u][v]; S3 += p[u][v] * p[u][v] * p[u][v]; }
      const double pa = p[u][a];
      const double s = S1 * S1 * S1 + 3.0 * S1 * S2 + 2.0 * S3 + 3.0 * pa * (S1 * S1 + S2) + 6.0 * pa * pa * S1 + 6.0 * pa * pa * pa;
      acc += vol[u] * cm * s;
    }
  }
  return acc;
}

// ---- mobility matrices of the PFC1 model (Section 3) ---------------------------
// P1: grad lambda is constant on a simplex and int_T lambda_c = |T| / (m+1), so
//   K_+(psi)^T_ab = (sum_c psi^+_c / (m+1)) |T| grad l_a . grad l_b
//   F(mu)^T_ab    = (1 / (m+1)) sum_c mu_c |T| grad l_c . grad l_a   (a: test, b: trial)
// with |T| grad l_a . grad l_b read from the element stiffness (upper triangle).
__device__ __forceinline__ double elem_k(const MeshDev& m, int el, int a, int b) {
  const int k = m.dim + 1;
  if (a > b) { const int t = a; a = b; b = t; }
  return m.elem_K[(long long)el * (k * (k + 1) / 2) + a * k - a * (a - 1) / 2 + (b - a)];
}

template <typename PsiF>
__device__ __forceinline__ double entry_Kplus(const MeshDev& m, long long e, PsiF psi, double psi_min) {
  double acc = 0.0;
  const int k = m.dim + 1;
  const double ik = 1.0 / k;
  for (int t = m.sl_el_ptr[e]; t < m.sl_el_ptr[e + 1]; ++t) {
    const int pk = m.sl_el[t];
    const int el = pk >> 4, a = (pk >> 2) & 3, b = pk & 3;
    const int* en = m.elem_nodes + (long long)el * k;
    double s = 0.0;
    for (int c = 0; c < k; ++c) s += psi(en[c]) - psi_min;
    acc += s * ik * elem_k(m, el, a, b);
  }
  return acc;
}

template <typename MuF>
__device__ __forceinline__ double entry_F(const MeshDev& m, long long e, MuF mu) {
  double acc = 0.0;
  const int k = m.dim + 1;
  const double ik = 1.0 / k;
  for (int t = m.sl_el_ptr[e]; t < m.sl_el_ptr[e + 1]; ++t) {
    const int pk = m.sl_el[t];
    const int el = pk >> 4, a = (pk >> 2) & 3;
    const int* en = m.elem_nodes + (long long)el * k;
    double s = 0.0;
    for (int c = 0; c < k; ++c) s += mu(en[c]) * elem_k(m, el, c, a);
    acc += s * ik;
  }
  return acc;
}

// (K_+(psi) mu)_i at node i, element by element (the stage right-hand side
// needs it at the stage state, where no assembled K_+ exists)
template <typename PsiF, typename MuF>
__device__ __forceinline__ double node_Kplus_mu(const MeshDev& m, int i, PsiF psi, MuF mu, double psi_min) {
  double acc = 0.0;
  const int k = m.dim + 1;
  const double ik = 1.0 / k;
  for (int t = m.nd_el_ptr[i]; t < m.nd_el_ptr[i + 1]; ++t) {
    const int pk = m.nd_el[t];
    const int el = pk >> 2, a = pk & 3;
    const int* en = m.elem_nodes + (long long)el * k;
    double sp = 0.0, km = 0.0;
    for (int c = 0; c < k; ++c) {
      const int j = en[c];
      sp += psi(j) - psi_min;
      km += elem_k(m, el, a, c) * mu(j);
    }
    acc += sp * ik * km;
  }
  return acc;
}

// ---- phases ---------------------------------------------------------------
// Every phase returns this thread's contribution to the two partial sums.

// N(psi_k) = -3 Mpsi2 reassembled in place (one value per stored entry).
template <int L>
__device__ __forceinline__ Red3 ph_rb_begin(const InstDev& I, const Team& tm) {
  const int n = I.n;
  const double* xk = I.xk;
  auto psi = [&](int j) { return xk[n + j]; };
  const PatView<L> pv = p1_pat<L>(I, tm);
  PFC_SLICES(I, tm) {
    const int base = pv.base(sl);
    const int w = pv.width(sl);
    const int lane = tm.lane;
    for (int k = 0; k < w; ++k) {
      const long long e = (long long)base + k * 64 + lane;
      I.N[e] = -3.0 * entry_Mpsi2(I.m, e, psi);
      if (I.model == PFC_MODEL_PFC1) {
        I.Kp[e] = entry_Kplus(I.m, e, psi, I.psi_min);
        I.Fm[e] = entry_F(I.m, e, [&](int j) { return xk[j]; });
      }
    }
  }
  return red3(0.0, 0.0);
}

__device__ __forceinline__ double stage_comb(const InstDev& I, int stage, int blk, int j) {
  const long long n3 = 3LL * I.n;
  const long long o = (long long)blk * I.n + j;
  double v = I.xk[o];
  if (stage == 2) v += ROS_A21 * I.ys[o];
  if (stage == 3) v += ROS_A31 * I.ys[o] + ROS_A32 * I.ys[n3 + o];
  return v;
}

// Stage right-hand side at the row of (slice, lane) (Section 3.1): F(x_i) with
// block 1 multiplied by tau, plus sum_j c_ij M y_j^psi on block 1, with the
// stage state x_i = x_k + sum_j a_ij y_j formed on the fly.
template <int L>
__device__ __forceinline__ void stage_rhs_row(const InstDev& I, const PatView<L>& pv, int sl, int lane, int stage,
                                              double& b0, double& b1, double& b2) {
  const int n = I.n;
  const int i = sl * 64 + lane;
  const int base = pv.base(sl);
  const int w = pv.width(sl);
  double sMmu = 0, sMps = 0, sMom = 0, sKmu = 0, sKps = 0, sKom = 0, sMy1 = 0, sMy2 = 0;
  const long long n3 = 3LL * n;
  for (int k = 0; k < w; ++k) {
    const long long e = (long long)base + k * 64 + lane;
    const int j = pv.at(e, i);
    const double Mv = I.m.M[e], Kv = I.m.K[e];
    const double mu = stage_comb(I, stage, 0, j);
    const double ps = stage_comb(I, stage, 1, j);
    const double om = stage_comb(I, stage, 2, j);
    sMmu += Mv * mu; sMps += Mv * ps; sMom += Mv * om;
    sKmu += Kv * mu; sKps += Kv * ps; sKom += Kv * om;
    if (stage >= 2) sMy1 += Mv * I.ys[n + j];
    if (stage >= 3) sMy2 += Mv * I.ys[n3 + n + j];
  }
  double g = 0.0;
  if (i < n) g = node_psi3(I.m, i, [&](int j) { return stage_comb(I, stage, 1, j); });
  b0 = -sMmu + (1.0 + I.r) * sMps - 2.0 * sKps - sKom + g;
  if (I.model == PFC_MODEL_PFC1) {  // -tau K_+(psi_i) mu_i
    double kpm = 0.0;
    if (i < n)
      kpm = node_Kplus_mu(I.m, i, [&](int j) { return stage_comb(I, stage, 1, j); },
                          [&](int j) { return stage_comb(I, stage, 0, j); }, I.psi_min);
    b1 = I.tau * (-kpm);
  } else {
    b1 = I.tau * (-sKmu);
  }
  if (stage == 2) b1 += ROS_C21 * sMy1;
  if (stage == 3) b1 += ROS_C31 * sMy1 + ROS_C32 * sMy2;
  b2 = -sMom - sKps;
}

// Right-hand side of the solve: stage rhs b_i^R for job RB, the caller's rhs
// for job SOLVE.  Writes W = b with block 1 multiplied by rs, X = 0.
template <int L>
__device__ __forceinline__ Red3 ph_solve_init(const InstDev& I, const State& S, const Team& tm) {
  const int n = I.n;
  const bool rb = (S.job == JOB_RB);
  const PatView<L> pv = p1_pat<L>(I, tm);
  double* X = rb ? (I.ys + (long long)(S.stage - 1) * 3 * n) : I.x_user;
  const double im = I.rs;
  double a0 = 0.0, a1 = 0.0;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    double b0 = 0.0, b1 = 0.0, b2 = 0.0;
    if (rb) stage_rhs_row<L>(I, pv, sl, tm.lane, S.stage, b0, b1, b2);
    if (i < n) {
      if (rb) {
        vst(I.b + i, b0); vst(I.b + n + i, b1); vst(I.b + 2 * n + i, b2);
      } else {
        b0 = I.b_user[i]; b1 = I.b_user[n + i]; b2 = I.b_user[2 * n + i];
      }
      const double bs1 = b1 * im;
      vst(I.W + i, b0); vst(I.W + n + i, bs1); vst(I.W + 2 * n + i, b2);
      vst(X + i, 0.0); vst(X + n + i, 0.0); vst(X + 2 * n + i, 0.0);
      a0 += b0 * b0 + b1 * b1 + b2 * b2;
      a1 += b0 * b0 + bs1 * bs1 + b2 * b2;
    }
  }
  return red3(a0, a1);
}

__device__ __forceinline__ Red3 ph_rb_update(const InstDev& I, const Team& tm) {
  const int n = I.n;
  const long long n3 = 3LL * n;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    if (i < n) {
      for (int blk = 0; blk < 3; ++blk) {
        const long long o = (long long)blk * n + i;
        I.xk[o] = I.xk[o] + ROS_M1 * I.ys[o] + ROS_M2 * I.ys[n3 + o] + ROS_M3 * I.ys[2 * n3 + o];
      }
    }
  }
  return red3(0.0, 0.0);
}

// ---- inner PCG --------------------------------------------------------------
template <typename T>
struct PcgOps {
  const T* C;      // stored operator values, or nullptr for M + cK on the fly
  const T* Mv;
  const T* Kv;
  T cK;
  const T* dinv;
  T* x;
  const int* sp;   // slice offsets and columns of the operator's pattern
  const int* colp;
};

__device__ __forceinline__ bool is_ci(int kind) { return kind == KIND_CI_OMEGA || kind == KIND_CI_MU; }

template <typename T>
__device__ __forceinline__ PcgOps<T> pcg_ops(const InstDev& I, int kind) {
  PcgOps<T> o;
  o.Mv = TV<T>::M(I);
  o.Kv = TV<T>::K(I);
  o.cK = T(0);
  o.C = o.Mv;
  o.dinv = TV<T>::dM(I);
  o.x = nullptr;
  o.sp = I.m.slice_ptr;
  o.colp = I.m.col;
  const int n = I.n;
  switch (kind) {
    case KIND_Y0: o.x = (T*)I.y0; break;
    case KIND_Y1:
      o.x = (T*)I.y1;
      o.dinv = (const T*)I.dinvCd;
      if (I.shared_ops) { o.C = nullptr; o.cK = T(I.delta); } else o.C = (const T*)I.Cd;
      break;
    case KIND_Z:
    case KIND_X1:
      o.x = (T*)(kind == KIND_Z ? I.zt : I.x1);
      o.dinv = (const T*)I.dinvCsd;
      if (I.shared_ops) { o.C = nullptr; o.cK = T(I.sdelta); } else o.C = (const T*)I.Csd;
      break;
    case KIND_X2: o.x = (T*)I.x2; break;
    case KIND_SD:
      o.x = (T*)I.x1;
      o.C = (const T*)I.SDv;
      o.dinv = (const T*)I.dinvSD;
      o.sp = I.m.w_slice_ptr;
      o.colp = I.m.w_col;
      break;
    case KIND_CI_OMEGA: o.x = (T*)(I.xk + 2LL * n); break;
    case KIND_CI_MU: o.x = (T*)(I.xk); break;
  }
  return o;
}

// Pattern of the operator of a PCG solve: the P1 pattern (staged columns when
// L) or, for S_D, the second-ring pattern (never staged).
template <int L, typename T>
__device__ __forceinline__ PatView<L> op_pat(const InstDev& I, const PcgOps<T>& o, const Team& tm) {
  // (the S_D pattern is only ever read with L == PFC_COL_MEM)
  return PatView<L>{o.sp, o.colp, o.sp == I.m.slice_ptr ? I.m.uw : 0, tm.lo, I.n, I.m.gN, I.m.gInv,
                    L == PFC_COL_GRID ? I.m.glin : nullptr};
}

template <typename T>
__device__ __forceinline__ T opval(const PcgOps<T>& o, long long e) {
  return o.C ? o.C[e] : (o.Mv[e] + o.cK * o.Kv[e]);
}
template <typename T>
__device__ __forceinline__ T opval_g(const PcgOps<T>& o, long long e) {
  return o.C ? gld(o.C + e) : (gld(o.Mv + e) + o.cK * gld(o.Kv + e));
}

// y_i = (A v)_i for a stored operator A (typed) over the row of thread lane
template <typename T, int L, typename VF>
__device__ __forceinline__ T row_dot(const PatView<L>& pv, int sl, int lane, const T* A, VF v) {
  const int base = pv.base(sl);
  const int w = pv.width(sl);
  T acc = T(0);
  for_width(w, [&](int k) {
    const long long e = (long long)base + k * 64 + lane;
    acc += A[e] * v(pv.at(e, sl * 64 + lane));
  });
  return acc;
}

template <typename T, int L>
__device__ __forceinline__ Red3 ph_pcg_setup(const InstDev& I, const State& S, const Team& tm) {
  const int n = I.n;
  const int kind = S.kind;
  PcgOps<T> o = pcg_ops<T>(I, kind);
  const PatView<L> pv = p1_pat<L>(I, tm);   // every right-hand side is a P1 product
  T* r = (T*)I.r_;
  const long long n3 = 3LL * n;
  double* Vj = I.V + (long long)S.j * n3;
  double* Zj = I.Z + (long long)S.j * n3;
  const T* Mv = o.Mv;
  const T* Kv = o.Kv;
  double a0 = 0.0, a1 = 0.0;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    const int lane = tm.lane;
    double rhs = 0.0;
    switch (kind) {
      case KIND_Y0: {
        if (i < n) {
          const double vs = S.vscale;
          const double v0 = I.W[i] * vs, v1 = I.W[n + i] * vs, v2 = I.W[2 * n + i] * vs;
          vst(Vj + i, v0); vst(Vj + n + i, v1); vst(Vj + 2 * n + i, v2);
          rhs = v0;
        }
      } break;
      case KIND_Y1: {  // (2): b1 - tau K y0
        const T* y0 = (const T*)I.y0;
        const T ky = row_dot<T>(pv, sl, lane, Kv, [&](int j) { return y0[j]; });
        if (i < n) rhs = Vj[n + i] - I.tau_p * (double)ky;
      } break;
      case KIND_SD:   // (3) with S_D: M y1
      case KIND_Z: {  // (3.1): M y1
        const T* y1 = (const T*)I.y1;
        const T my = row_dot<T>(pv, sl, lane, Mv, [&](int j) { return y1[j]; });
        rhs = (double)my;
      } break;
      case KIND_X1: {  // (3.2): M z
        const T* zt = (const T*)I.zt;
        const T mz = row_dot<T>(pv, sl, lane, Mv, [&](int j) { return zt[j]; });
        rhs = (double)mz;
      } break;
      case KIND_X2: {  // (5): b2 - K x1, and (4): x0 = y0 + (y1 - x1)/delta
        const T* x1 = (const T*)I.x1;
        const T kx = row_dot<T>(pv, sl, lane, Kv, [&](int j) { return x1[j]; });
        if (i < n) {
          rhs = Vj[2 * n + i] - (double)kx;
          const double y0i = (double)((const T*)I.y0)[i], y1i = (double)((const T*)I.y1)[i];
          const double x1i = (double)x1[i];
          vst(Zj + i, y0i + (y1i - x1i) / I.delta);
          vst(Zj + n + i, x1i);
        }
      } break;
      case KIND_CI_OMEGA: {  // M omega_0 = -K psi_0
        const double kp = row_dot<double>(pv, sl, lane, I.m.K, [&](int j) { return I.xk[n + j]; });
        rhs = -kp;
      } break;
      case KIND_CI_MU: {  // M mu_0 = (1+r) M psi_0 - 2 K psi_0 - K omega_0 + g(psi_0)
        const int base = pv.base(sl);
        const int w = pv.width(sl);
        double sMp = 0, sKp = 0, sKo = 0;
        for (int k = 0; k < w; ++k) {
          const long long e = (long long)base + k * 64 + lane;
          const int j = pv.at(e, i);
          sMp += I.m.M[e] * I.xk[n + j];
          sKp += I.m.K[e] * I.xk[n + j];
          sKo += I.m.K[e] * I.xk[2 * n + j];
        }
        if (i < n) {
          auto psi = [&](int j) { return I.xk[n + j]; };
          rhs = (1.0 + I.r) * sMp - 2.0 * sKp - sKo + node_psi3(I.m, i, psi);
        }
      } break;
    }
    if (i < n) {
      const T rT = T(rhs);
      vst(r + i, rT);
      vst(o.x + i, T(0));
      const double rd = (double)rT;
      a0 += rd * ((double)o.dinv[i] * rd);
      a1 += rd * rd;
    }
  }
  return red3(a0, a1);
}

// p_j = D^{-1}_j r_j + beta p_old_j, evaluated identically wherever needed
template <typename T>
__device__ __forceinline__ T pval(const T* dinv, const T* r, const T* pold, T beta, bool first, int j) {
  const T z = dinv[j] * r[j];
  return first ? z : (z + beta * pold[j]);
}

template <typename T, int L>
__device__ __forceinline__ Red3 ph_pcg_a(const InstDev& I, const State& S, const Team& tm) {
  const int n = I.n;
  PcgOps<T> o = pcg_ops<T>(I, S.kind);
  const PatView<L> pv = op_pat<L>(I, o, tm);
  const T* r = (const T*)I.r_;
  const T* pold = (const T*)(S.pcur ? I.pB : I.pA);
  T* pnew = (T*)(S.pcur ? I.pA : I.pB);
  T* q = (T*)I.q;
  const bool first = (S.it == 0);
  const T beta = T(S.beta_cg);
  double a0 = 0.0;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    const int base = pv.base(sl);
    const int w = pv.width(sl);
    T acc = T(0);
    for_width(w, [&](int k) {
      const long long e = (long long)base + k * 64 + tm.lane;
      const int j = pv.at(e, i);
      acc += opval(o, e) * pval(o.dinv, r, pold, beta, first, j);
    });
    if (i < n) {
      const T pi = pval(o.dinv, r, pold, beta, first, i);
      vst(pnew + i, pi);
      vst(q + i, acc);
      a0 += (double)pi * (double)acc;
    }
  }
  return red3(a0, 0.0);
}

template <typename T>
__device__ __forceinline__ Red3 ph_pcg_b(const InstDev& I, const State& S, const Team& tm) {
  const int n = I.n;
  PcgOps<T> o = pcg_ops<T>(I, S.kind);
  T* r = (T*)I.r_;
  const T* p = (const T*)(S.pcur ? I.pB : I.pA);
  const T* q = (const T*)I.q;
  const T alpha = T(S.alpha);
  double a0 = 0.0, a1 = 0.0;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    if (i < n) {
      const T xi = o.x[i] + alpha * p[i];
      const T ri = r[i] - alpha * q[i];
      vst(o.x + i, xi);
      vst(r + i, ri);
      const double rd = (double)ri;
      a0 += rd * rd;
      a1 += rd * ((double)o.dinv[i] * rd);
    }
  }
  return red3(a0, a1);
}

// ---- outer block operator ------------------------------------------------------
// (A y)_i for the three block rows at node i:
//   w0 = M mu + (-(1+r) M + 2K + N) psi + K omega
//   w1 = t K mu + s M psi
//   w2 = K psi + M omega
//   PFC1 (MOB): w1 = t K_+ mu + s M psi + t F psi
template <int L, bool MOB, typename YF>
__device__ __forceinline__ void block_row(const InstDev& I, const PatView<L>& pv, int sl, int lane, double t, double s,
                                          YF y, double& w0, double& w1, double& w2) {
  const int base = pv.base(sl);
  const int w = pv.width(sl);
  const double c1 = -(1.0 + I.r);
  w0 = w1 = w2 = 0.0;
  for_width(w, [&](int k) {
    const long long e = (long long)base + k * 64 + lane;
    const int j = pv.at(e, sl * 64 + lane);
    const double Mv = I.m.M[e], Kv = I.m.K[e], Nv = I.N[e];
    double mu, ps, om;
    y(j, mu, ps, om);
    w0 += Mv * mu + (c1 * Mv + 2.0 * Kv + Nv) * ps + Kv * om;
    if constexpr (MOB) w1 += t * I.Kp[e] * mu + s * Mv * ps + t * I.Fm[e] * ps;
    else w1 += t * Kv * mu + s * Mv * ps;
    w2 += Kv * ps + Mv * om;
  });
}

__device__ __forceinline__ Red3 ph_update_x(const InstDev& I, const State& S, const Team& tm, const double* y) {
  const int n = I.n;
  const long long n3 = 3LL * n;
  double* X = (S.job == JOB_RB) ? (I.ys + (long long)(S.stage - 1) * n3) : I.x_user;
  const int kc = S.kcols;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    if (i < n) {
      for (int blk = 0; blk < 3; ++blk) {
        const long long o = (long long)blk * n + i;
        double x = X[o];
        for (int l = 0; l < kc; ++l) x += y[l] * I.Z[(long long)l * n3 + o];
        vst(X + o, x);
      }
    }
  }
  return red3(0.0, 0.0);
}

template <int L, bool MOB>
__device__ __forceinline__ Red3 ph_true_res(const InstDev& I, const State& S, const Team& tm) {
  const int n = I.n;
  const PatView<L> pv = p1_pat<L>(I, tm);
  const long long n3 = 3LL * n;
  const bool rb = (S.job == JOB_RB);
  const double* X = rb ? (I.ys + (long long)(S.stage - 1) * n3) : I.x_user;
  const double* bsrc = rb ? I.b : I.b_user;
  const double im = I.rs;
  double a0 = 0.0, a1 = 0.0;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    double w0, w1, w2;
    block_row<L, MOB>(I, pv, sl, tm.lane, I.tau, I.m11,
              [&](int j, double& mu, double& ps, double& om) { mu = X[j]; ps = X[n + j]; om = X[2 * n + j]; },
              w0, w1, w2);
    if (i < n) {
      const double r0 = bsrc[i] - w0, r1 = bsrc[n + i] - w1, r2 = bsrc[2 * n + i] - w2;
      const double rs1 = r1 * im;
      vst(I.W + i, r0); vst(I.W + n + i, rs1); vst(I.W + 2 * n + i, r2);
      a0 += r0 * r0 + r1 * r1 + r2 * r2;
      a1 += r0 * r0 + rs1 * rs1 + r2 * r2;
    }
  }
  return red3(a0, a1);
}

template <typename T>
__device__ __forceinline__ Red3 ph_pch_out(const InstDev& I, const Team& tm) {
  const int n = I.n;
  const T* x2 = (const T*)I.x2;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    if (i < n) {
      I.pch_out[i] = I.Z[i];
      I.pch_out[n + i] = I.Z[n + i];
      I.pch_out[2 * n + i] = (double)x2[i];
    }
  }
  return red3(0.0, 0.0);
}

// ---- single-reduction Jacobi PCG (Chronopoulos-Gear form) ----------------------
// Same iterates as the standard PCG in exact arithmetic, with the two inner
// products of an iteration taken in one reduction:
//   s_i = w_i + beta_i s_{i-1},  p_i = u_i + beta_i p_{i-1},
//   x_{i+1} = x_i + alpha_i p_i, r_{i+1} = r_i - alpha_i s_i, u = D^{-1} r, w = C u,
//   gamma = (r, u), delta = (w, u), beta_{i+1} = gamma_{i+1}/gamma_i,
//   alpha_{i+1} = gamma_{i+1} / (delta_{i+1} - beta_{i+1} gamma_{i+1} / alpha_i).
// u_{i+1} at gathered neighbours is recomputed from r_i, w_i, s_{i-1}; r, w, s
// are double-buffered, p and x are updated in place by their owners.
template <typename T>
__device__ __forceinline__ T cg_s(const T* wc, const T* so, T beta, bool first, int j) {
  return first ? wc[j] : (wc[j] + beta * so[j]);
}
template <typename T>
__device__ __forceinline__ T cg_unew(const T* dinv, const T* rc, const T* wc, const T* so, T alpha, T beta, bool first,
                                      int j) {
  return dinv[j] * (rc[j] - alpha * cg_s(wc, so, beta, first, j));
}

template <typename T, int L>
__device__ __forceinline__ Red3 ph_cg_init(const InstDev& I, const State& S, const Team& tm) {
  const int n = I.n;
  PcgOps<T> o = pcg_ops<T>(I, S.kind);
  const PatView<L> pv = op_pat<L>(I, o, tm);
  const T* r = (const T*)I.r_;
  T* w = (T*)I.q;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    const int base = pv.base(sl);
    const int wd = pv.width(sl);
    T acc = T(0);
    for_width(wd, [&](int k) {
      const long long e = (long long)base + k * 64 + tm.lane;
      const int j = pv.at(e, i);
      acc += opval(o, e) * (o.dinv[j] * r[j]);
    });
    if (i < n) {
      vst(w + i, acc);
      const T u = o.dinv[i] * r[i];
      a0 += (double)r[i] * (double)u;
      a1 += (double)acc * (double)u;
      a2 += (double)r[i] * (double)r[i];
    }
  }
  return red3(a0, a1, a2);
}

template <typename T, int L>
__device__ __forceinline__ Red3 ph_cg_iter(const InstDev& I, const State& S, const Team& tm) {
  const int n = I.n;
  PcgOps<T> o = pcg_ops<T>(I, S.kind);
  const PatView<L> pv = op_pat<L>(I, o, tm);
  const int c = S.cur;
  const T* rc = (const T*)(c ? I.rB : I.r_);
  T* rn = (T*)(c ? I.r_ : I.rB);
  const T* wc = (const T*)(c ? I.wB : I.q);
  T* wn = (T*)(c ? I.q : I.wB);
  const T* so = (const T*)(c ? I.sB : I.sA);
  T* sn = (T*)(c ? I.sA : I.sB);
  T* p = (T*)I.pA;
  const T alpha = T(S.alpha), beta = T(S.beta_cg);
  const bool first = (S.it == 0);
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    const int base = pv.base(sl);
    const int wd = pv.width(sl);
    T acc = T(0);
    for_width(wd, [&](int k) {
      const long long e = (long long)base + k * 64 + tm.lane;
      const int j = pv.at(e, i);
      acc += opval(o, e) * cg_unew(o.dinv, rc, wc, so, alpha, beta, first, j);
    });
    if (i < n) {
      const T si = cg_s(wc, so, beta, first, i);
      const T uo = o.dinv[i] * rc[i];
      const T pi = first ? uo : (uo + beta * p[i]);
      vst(o.x + i, o.x[i] + alpha * pi);
      const T ri = rc[i] - alpha * si;
      const T ui = cg_unew(o.dinv, rc, wc, so, alpha, beta, first, i);
      vst(sn + i, si);
      vst(p + i, pi);
      vst(rn + i, ri);
      vst(wn + i, acc);
      a0 += (double)ri * (double)ui;
      a1 += (double)acc * (double)ui;
      a2 += (double)ri * (double)ri;
    }
  }
  return red3(a0, a1, a2);
}

// ---- two Jacobi-PCG iterations per launch (s-step form, s = 2) ---------------
// With T = D^{-1} C (D = diag C) the Jacobi PCG is CG for T in the D-weighted
// inner product <a, b> = a^T D b: u = D^{-1} r, (r, u) = <u, u>, (p, C p) =
// <p, T p>, ||r||^2 = u^T D^2 u.  From the basis B = [p, Tp, T^2 p, u, Tu] of a
// launch, the next two iterates are combinations of B whose coefficients follow
// from the Gram matrices G = B^T D B and H = B'^T D^2 B' (B' = [Tp, T^2 p, u,
// Tu]), so one reduction serves two iterations.  A launch forms the new p, u as
// such combinations on its own rows and on the rows two (p) or one (u) stencil
// steps around them, keeps them in LDS, and applies T there: Tp on the rows one
// step around, T^2 p and Tu on its own rows.  The halo is a contiguous range of
// rows (mod n) on 2D periodic grids, whose neighbours lie within N + 1 rows.
#define PFC_SS_LDS 8192
#define PFC_SS_NG 26  // 15 entries of G, 10 of H, and ||b||^2 in the first launch of a solve
#define PFC_SS_NA 4   // passes of a workgroup over the two-step halo (R + 4H <= 4096 rows)
#define PFC_SS_NB 3   // passes over the one-step halo (R + 2H <= 3072 rows); 7 entries per row
__shared__ double pfc_ss[PFC_SS_LDS];
__shared__ double pfc_ssred[64 * 32];
#ifdef PFC_TICK_TIMING
__shared__ unsigned long long pfc_sst[6];  // optional instrumentation (separate build only)
#define PFC_SS_STAMP(k) \
  if (threadIdx.x == 0) pfc_sst[k] = wall_clock64()
#else
#define PFC_SS_STAMP(k)
#endif

// Cross-lane moves of a double through DPP (register to register, no LDS).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Workgroup barrier that orders LDS only: the global loads and stores of the
// two-iterations-per-launch phase are never read back within the launch, so
// loads issued ahead stay in flight across it (a full __syncthreads would wait
// for every outstanding memory operation).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Halving exchange between the lanes of a pair: the lane that keeps the lower
// half returns a + (partner's a), the other b + (partner's b).  Partners: lanes
// l and l ^ 32 (permlane32 swap), rows 2k and 2k + 1 (permlane16 swap), or the
// DPP pairs of CTRL within a row.
__device__ __forceinline__ double ss_pair(unsigned hi, unsigned lo) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <bool ROWS16>
__device__ __forceinline__ double ss_swap(double a, double b, bool upper) {
  const unsigned long long ia = (unsigned long long)__double_as_longlong(a), ib = (unsigned long long)__double_as_longlong(b);
  if constexpr (ROWS16) {
    const auto l = __builtin_amdgcn_permlane16_swap((unsigned)ia, (unsigned)ib, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
    return upper ? b + ss_pair(h[0], l[0]) : a + ss_pair(h[1], l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap((unsigned)ia, (unsigned)ib, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
    return upper ? b + ss_pair(h[0], l[0]) : a + ss_pair(h[1], l[1]);
  }
}
template <int CTRL>
__device__ __forceinline__ double ss_dppx(double a, double b, bool upper) {
  return (upper ? b : a) + dpp_f64<CTRL, 0xf>(upper ? a : b);
}
// Sums of 32 values over the 64 lanes of a wave by recursive halving (32 value
// exchanges in all instead of 6 per value): the total of value idx ends in lanes
// 2m and 2m + 1 with idx = 16 [l >= 32] + 8 [row odd] + 4 [l mod 16 >= 8] +
// 2 [l mod 8 >= 4] + [l & 2].  Returns the total of the lane's idx.
__device__ __forceinline__ double ss_wave_sums32(const double* v, int lane) {
  double w16[16], w8[8], w4[4], w2[2];
#pragma unroll
  for (int k = 0; k < 16; ++k) w16[k] = ss_swap<false>(v[k], v[k + 16], lane >= 32);
#pragma unroll
  for (int k = 0; k < 8; ++k) w8[k] = ss_swap<true>(w16[k], w16[k + 8], (lane >> 4) & 1);
#pragma unroll
  for (int k = 0; k < 4; ++k) w4[k] = ss_dppx<0x140>(w8[k], w8[k + 4], (lane & 15) >= 8);  // row_mirror
#pragma unroll
  for (int k = 0; k < 2; ++k) w2[k] = ss_dppx<0x141>(w4[k], w4[k + 2], (lane & 7) >= 4);   // row_half_mirror
  const double w1 = ss_dppx<0x4e>(w2[0], w2[1], (lane & 2) != 0);                          // quad_perm [2,3,0,1]
  return w1 + dpp_f64<0xb1, 0xf>(w1);                                                      // quad_perm [1,0,3,2]
}
__device__ __forceinline__ int ss_wave_sums32_index(int lane) {
  return (lane >= 32 ? 16 : 0) + (((lane >> 4) & 1) ? 8 : 0) + ((lane & 15) >= 8 ? 4 : 0) + ((lane & 7) >= 4 ? 2 : 0) +
         ((lane & 2) ? 1 : 0);
}

__device__ __forceinline__ int ss_wrap(int g, int n) { return g < 0 ? g + n : (g >= n ? g - n : g); }
// offset j - g of a neighbour as a step within the grid (|step| <= N + 1 < n / 2)
__device__ __forceinline__ int ss_step(int d, int n) { return d > (n >> 1) ? d - n : (d < -(n >> 1) ? d + n : d); }

// upper-triangle index of (i, j), i <= j, in a k x k symmetric matrix
__host__ __device__ __forceinline__ int ss_tri(int i, int j, int k) { return i * k - i * (i - 1) / 2 + (j - i); }

// Rows of a workgroup in the two-iterations-per-launch form: own rows [lo, lo + R)
// (at most PFC_WG), halo H; thread tid's passes over the two-step halo are
// q = tid + c PFC_WG, and its own row (if any) is pass position qo.
struct SsRows {
  int lo, R, H, L1, L2, qo, go;
  bool own;
};
__device__ __forceinline__ SsRows ss_rows(const InstDev& I, int rank, int size) {
  SsRows w;
  const int n = I.n;
  const int spw = (I.m.n_slices + size - 1) / size;
  w.lo = min(rank * spw * 64, n);
  w.R = min(w.lo + spw * 64, n) - w.lo;
  w.H = I.sH;
  w.L1 = w.R + 2 * w.H;
  w.L2 = w.R + 4 * w.H;
  const int tid = threadIdx.x;
  w.qo = 2 * w.H + (((tid - 2 * w.H) % PFC_WG) + PFC_WG) % PFC_WG;
  w.own = w.qo < 2 * w.H + w.R;
  w.go = w.lo + (w.qo - 2 * w.H);
  return w;
}

// Loads of the current basis on the two-step halo (and x on the own row), issued
// before the launch's reductions so that their latency overlaps them.
struct SsPre {
  double bv[PFC_SS_NA][5];
  double xo;
};
__device__ __forceinline__ void ss_load(const InstDev& I, const State& S, const SsRows& w, SsPre& P, int par) {
  const int n = I.n;
  const long long nn = n;
  const int tid = threadIdx.x;
  const double* bin = I.sbas + (long long)par * 5 * nn;  // the basis of the previous launch
#pragma unroll
  for (int c = 0; c < PFC_SS_NA; ++c) {
    const int g = ss_wrap(w.lo - 2 * w.H + min(tid + c * PFC_WG, w.L2 - 1), n);
#pragma unroll
    for (int k = 0; k < 5; ++k) P.bv[c][k] = gld(bin + k * nn + g);
  }
  P.xo = gld(pcg_ops<double>(I, S.kind).x + min(w.go, n - 1));  // used on the own row only
}

// coef: x increment [0..4], new p [5..9], new u [10..14] over B; S.pcur: x only.
// par: the launch's parity (reads basis [par], writes basis [1 - par]).
template <int L>
__device__ __forceinline__ void ph_scg(const InstDev& I, const State& S, const Team& tm, const double* coef, bool init,
                                       double* spart_out, const SsRows& w, SsPre& P, int par) {
  const int n = I.n, H = w.H, R = w.R, L1 = w.L1, L2 = w.L2, lo = w.lo;
  PcgOps<double> o = pcg_ops<double>(I, S.kind);
  const PatView<L> pv = op_pat<L>(I, o, tm);
  const int tid = threadIdx.x;
  const long long nn = n;
  double* bout = I.sbas + (long long)(1 - par) * 5 * nn;
  double bbo = 0.0;  // ||b||^2 over the own rows (first launch of a solve)
  if (init) {
    // the solve's right-hand side b (the set-up of the inner solve, on the own
    // rows and the two-step halo) and u_0 = p_0 = D^{-1} b; x_0 = 0
    const long long n3 = 3 * nn;
    const double* Vj = I.V + (long long)S.j * n3;
    // b = t - s (A v) with, per solve: (1) t = w / ||w||; (2) t = (v_j)_psi, s = tau_p,
    // A v = K y0; (3.1) A v = M y1; (3.2) A v = M z; (5) t = (v_j)_omega, s = 1, A v = K x1
    const int kind = S.kind;
    const double* A = (kind == KIND_Y1 || kind == KIND_X2) ? o.Kv : (kind == KIND_Y0 ? nullptr : o.Mv);
    const double* v = kind == KIND_Y1 ? (const double*)I.y0
                      : kind == KIND_Z ? (const double*)I.y1
                      : kind == KIND_X1 ? (const double*)I.zt
                                        : (const double*)I.x1;
    const double* t = kind == KIND_Y0 ? I.W : (kind == KIND_Y1 ? Vj + nn : (kind == KIND_X2 ? Vj + 2 * nn : nullptr));
    const double ts = kind == KIND_Y0 ? S.vscale : 1.0, sa = kind == KIND_Y1 ? I.tau_p : 1.0;
    double bo = 0.0;
#pragma unroll
    for (int c = 0; c < PFC_SS_NA; ++c) {
      const int g = ss_wrap(lo - 2 * H + min(tid + c * PFC_WG, L2 - 1), n);
      const int base = (g >> 6) * 64 * 7 + (g & 63);
      double d = 0.0;
      if (A) {
#pragma unroll
        for (int k = 0; k < 7; ++k) {
          const long long e = (long long)base + k * 64;
          d += gld(A + e) * gld(v + pv.at(e, g));
        }
      }
      const double tt = t ? gld(t + g) * ts : 0.0;
      const double b = !A ? tt : (t ? tt - sa * d : d);
      P.bv[c][0] = gld(o.dinv + g);
      P.bv[c][1] = b;
      if (tid + c * PFC_WG == w.qo) bo = b;
    }
    if (w.own) {
      const int g = w.go;
      bbo = bo * bo;
      vst(o.x + g, 0.0);
      if (S.kind == KIND_Y0) {  // the Arnoldi vector v_j = w / ||w||
        double* Vw = (double*)Vj;
        vst(Vw + g, bo);
        vst(Vw + nn + g, gld(I.W + nn + g) * S.vscale);
        vst(Vw + 2 * nn + g, gld(I.W + 2 * nn + g) * S.vscale);
      } else if (S.kind == KIND_X2) {  // (4): z_j = (y0 + (y1 - x1) / delta, x1, x2)
        double* Zj = I.Z + (long long)S.j * n3;
        const double y0i = gld((const double*)I.y0 + g), y1i = gld((const double*)I.y1 + g);
        const double x1i = gld((const double*)I.x1 + g);
        vst(Zj + g, y0i + (y1i - x1i) / I.delta);
        vst(Zj + nn + g, x1i);
      }
    }
  }
  if (!init && S.pcur) {  // the solve ends within these two iterations: x only
    if (w.own) {
#pragma unroll
      for (int c = 0; c < PFC_SS_NA; ++c)
        if (tid + c * PFC_WG == w.qo)
          vst(o.x + w.go, P.xo + (coef[0] * P.bv[c][0] + coef[1] * P.bv[c][1] + coef[3] * P.bv[c][3]));
    }
    return;
  }
  double* sp = pfc_ss;     // new p on [lo - 2H, lo + R + 2H)
  double* su = sp + L2;    // new u on [lo - H, lo + R + H)
  double* stp = su + L1;   // T p on [lo - H, lo + R + H)
#pragma unroll
  for (int c = 0; c < PFC_SS_NA; ++c) {
    const int q = tid + c * PFC_WG;
    if (q < L2) {
      const double* b = P.bv[c];
      double pn, un;
      if (init) {
        pn = b[0] * b[1];
        un = pn;
      } else {
        pn = coef[5] * b[0] + coef[6] * b[1] + coef[7] * b[2] + coef[8] * b[3] + coef[9] * b[4];
        un = coef[10] * b[0] + coef[11] * b[1] + coef[12] * b[2] + coef[13] * b[3] + coef[14] * b[4];
      }
      sp[q] = pn;
      if (q >= H && q < H + L1) su[q - H] = un;
      if (q == w.qo && w.own) {
        if (!init) vst(o.x + w.go, P.xo + (coef[0] * b[0] + coef[1] * b[1] + coef[3] * b[3]));
        vst(bout + w.go, pn);
        vst(bout + 3 * nn + w.go, un);
      }
    }
  }
  // operator rows of the one-step halo (at most three passes; the third, if any,
  // holds a few rows of the first wave), in flight across the barrier
  double av[3][7], dv[3];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int g = ss_wrap(lo - H + min(tid + c * PFC_WG, L1 - 1), n);
    const int base = (g >> 6) * 64 * 7 + (g & 63);
#pragma unroll
    for (int k = 0; k < 7; ++k) av[c][k] = opval_g(o, (long long)base + k * 64);
    dv[c] = gld(o.dinv + g);
  }
  if (L1 > 2 * PFC_WG && tid < 64) {
    const int g = ss_wrap(lo - H + min(tid + 2 * PFC_WG, L1 - 1), n);
    const int base = (g >> 6) * 64 * 7 + (g & 63);
#pragma unroll
    for (int k = 0; k < 7; ++k) av[2][k] = opval_g(o, (long long)base + k * 64);
    dv[2] = gld(o.dinv + g);
  }
  lds_barrier();
  PFC_SS_STAMP(0);
  // T p on the one-step halo; T u on the own rows (at most one own row per thread)
  int q1o = -1;
  double tpo = 0.0, tuo = 0.0, dgo = 0.0, dvo = 0.0;
  double ao[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) ao[k] = 0.0;
  auto trow = [&](int q1, const double* a, double di) {
    const int g = ss_wrap(lo - H + q1, n);
    const bool own = q1 >= H && q1 < H + R;
    const int base = (g >> 6) * 64 * 7 + (g & 63);
    double acc = 0.0, acc2 = 0.0, dg = 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const int d = ss_step(pv.at((long long)base + k * 64, g) - g, n);
      acc += a[k] * sp[q1 + H + d];
      dg += d == 0 ? a[k] : 0.0;
    }
    if (own) {
#pragma unroll
      for (int k = 0; k < 7; ++k) acc2 += a[k] * su[q1 + ss_step(pv.at((long long)base + k * 64, g) - g, n)];
    }
    const double tp = di * acc;
    stp[q1] = tp;
    if (own) {
      q1o = q1; tpo = tp; tuo = di * acc2; dgo = dg; dvo = di;
#pragma unroll
      for (int k = 0; k < 7; ++k) ao[k] = a[k];
      vst(bout + nn + g, tpo);
      vst(bout + 4 * nn + g, tuo);
    }
  };
#pragma unroll
  for (int c = 0; c < 2; ++c)
    if (tid + c * PFC_WG < L1) trow(tid + c * PFC_WG, av[c], dv[c]);
  if (tid + 2 * PFC_WG < L1) {  // third pass (at most PFC_SS_NB)
    if (tid < 64) {
      trow(tid + 2 * PFC_WG, av[2], dv[2]);
    } else {
      const int q1 = tid + 2 * PFC_WG;
      const int g = ss_wrap(lo - H + q1, n);
      const int base = (g >> 6) * 64 * 7 + (g & 63);
      double a3[7];
#pragma unroll
      for (int k = 0; k < 7; ++k) a3[k] = opval_g(o, (long long)base + k * 64);
      trow(q1, a3, gld(o.dinv + g));
    }
  }
  lds_barrier();
  PFC_SS_STAMP(1);
  double gp[PFC_SS_NG];
#pragma unroll
  for (int m = 0; m < PFC_SS_NG; ++m) gp[m] = 0.0;
  if (q1o >= 0) {
    const int g = lo + (q1o - H);
    const int base = (g >> 6) * 64 * 7 + (g & 63);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) acc += ao[k] * stp[q1o + ss_step(pv.at((long long)base + k * 64, g) - g, n)];
    const double ttp = dvo * acc;
    vst(bout + 2 * nn + g, ttp);
    const double v[5] = {sp[q1o + H], tpo, ttp, su[q1o], tuo};
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const double di = dgo * v[i];
#pragma unroll
      for (int j = i; j < 5; ++j) gp[ss_tri(i, j, 5)] = di * v[j];
    }
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const double di = dgo * dgo * v[i];
#pragma unroll
      for (int j = i; j < 5; ++j) gp[15 + ss_tri(i - 1, j - 1, 4)] = di * v[j];
    }
  }
  gp[25] = bbo;
  PFC_SS_STAMP(2);
  // workgroup sums, fixed order: over each wave by recursive halving, then over
  // the waves
  const int lane = tid & 63, wave = tid >> 6;
  {
    double v32[32];
#pragma unroll
    for (int m = 0; m < 32; ++m) v32[m] = m < PFC_SS_NG ? gp[m] : 0.0;
    const double tot = ss_wave_sums32(v32, lane);
    const int idx = ss_wave_sums32_index(lane);
    if ((lane & 1) == 0) pfc_ssred[wave * 32 + idx] = tot;
  }
  lds_barrier();
  if (tid < PFC_SS_NG) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < PFC_WAVES; ++w) t += pfc_ssred[w * 32 + tid];
    vst(spart_out + (long long)tm.rank * 32 + tid, t);
  }
  PFC_SS_STAMP(3);
}

// Sum of the Gram partials of a team ([size][32], fixed order) into g[0..25]:
// the first 8 x 32 partials come from loads issued in the launch's prologue,
// before its phase is known, with the state loads (unconditional loads at
// clamped positions, masked in the sum; from fallback[0] where part is null,
// values then unused); teams of more than 256 add the rest here.
#define PFC_SS_GL 8
__device__ __forceinline__ void ss_gram_prefetch(const double* part, const double* fallback, int size, double* pl) {
  const int tid = threadIdx.x, v = tid & 31, grp = tid >> 5;
#pragma unroll
  for (int c = 0; c < PFC_SS_GL; ++c) {
    const int k = min(grp + 32 * c, size - 1);
    pl[c] = gld(part ? part + (long long)k * 32 + min(v, PFC_SS_NG - 1) : fallback);
  }
}
__device__ __forceinline__ void ss_gram(const double* part, int size, const double* pl, double* g) {
  const int tid = threadIdx.x, v = tid & 31, grp = tid >> 5;
  double s = 0.0;
#pragma unroll
  for (int c = 0; c < PFC_SS_GL; ++c) s += (v < PFC_SS_NG && grp + 32 * c < size) ? pl[c] : 0.0;
  if (v < PFC_SS_NG)
    for (int k = grp + 32 * PFC_SS_GL; k < size; k += 32) s += gld(part + (long long)k * 32 + v);
  pfc_ssred[grp * 32 + v] = s;
  lds_barrier();
  // only thread 0 (the transition) reads the totals: the first wave forms them,
  // lane v over groups 0-15 and lane v + 32 over groups 16-31, added across the
  // halves by a permlane32 swap.  Writers and the reader are lanes of that one
  // wave, so a wave barrier between LDS-only fences orders the writes before
  // thread 0's reads (no workgroup barrier needed)
  if (tid < 64) {
    const int half = tid >> 5;
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) t += pfc_ssred[(half * 16 + q) * 32 + v];
    t = ss_swap<false>(t, t, half != 0);
    if (tid < PFC_SS_NG) g[tid] = t;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
  }
}


// ---- two Jacobi-PCG iterations per launch on 3D periodic grids of side 64 -------
// The s-step iteration of ph_scg with a workgroup's rows a block of the grid
// instead of a range of rows: whole x-lines (64 rows, one SELL slice each) at
// y0..y0+3, z0..z0+3, 1024 rows; rank r has y0 = 4 (r mod 16), z0 = 4 (r / 16).
// The two-step frame is the 8 x 8 lines y0-2..y0+5, z0-2..z0+5, the one-step
// frame the 6 x 6 lines y0-1..y0+4, z0-1..z0+4 (periodic in every direction),
// so a row's neighbour in a frame follows from the entry's direction
// (MeshDev::gdir).  Frame positions: q = x + 64 (ly + 8 lz) in the two-step
// frame (4 passes of the workgroup), q1 = x + 64 (ly1 + 6 lz1) in the one-step
// frame (3 passes, the third partial).  New p and u are formed on the frames,
// T p on the one-step frame, and a last pass gives thread t the own row
// x = t mod 64, y0 + (t / 64) mod 4, z0 + t / 256 for T u, T^2 p, the stores and
// the Gram products.  T is the inner precision (float in PFC_MIXED); the Gram
// sums and the coefficients stay float64.
#define PFC_S3_N 64
__device__ __forceinline__ int s3_wrap(int v) { return v & (PFC_S3_N - 1); }
struct S3Geo {
  int y0, z0;
};
__device__ __forceinline__ S3Geo s3_geo(int rank) { return S3Geo{(rank & 15) * 4, (rank >> 4) * 4}; }
__device__ __forceinline__ int s3_row(const S3Geo& G, int x, int yl, int zl) {
  return x + PFC_S3_N * (s3_wrap(G.y0 + yl) + PFC_S3_N * s3_wrap(G.z0 + zl));
}
// row class (grid_class) of the row at block coordinates (x, yl, zl)
__device__ __forceinline__ int s3_class(const S3Geo& G, int x, int yl, int zl) {
  return grid_edge(x, PFC_S3_N) + 3 * grid_edge(s3_wrap(G.y0 + yl), PFC_S3_N) + 9 * grid_edge(s3_wrap(G.z0 + zl), PFC_S3_N);
}
// offset of an entry's neighbour within a frame of f lines per direction:
// (x + dx) mod 64 - x is applied separately
__device__ __forceinline__ int s3_dline(int code, int f) { return PFC_S3_N * ((code / 3) % 3 - 1 + f * (code / 9 - 1)); }
__device__ __forceinline__ int s3_nx(int x, int code) { return s3_wrap(x + code % 3 - 1); }

template <typename T>
struct S3Pre {
  T bv[PFC_SS_NA][5];
};
// the current basis on the two-step frame, issued before the reductions
template <typename T>
__device__ __forceinline__ void s3_load(const InstDev& I, const State& S, int rank, S3Pre<T>& P, int par) {
  const long long nn = I.n;
  const int tid = threadIdx.x;
  const S3Geo G = s3_geo(rank);
  const T* bin = (const T*)I.sbas + (long long)par * 5 * nn;
#pragma unroll
  for (int c = 0; c < PFC_SS_NA; ++c) {
    const int q = tid + c * PFC_WG;
    const int g = s3_row(G, q & 63, ((q >> 6) & 7) - 2, (q >> 9) - 2);
#pragma unroll
    for (int k = 0; k < 5; ++k) P.bv[c][k] = gld(bin + k * nn + g);
  }
}

template <typename T>
__device__ __forceinline__ void ph_scg3(const InstDev& I, const State& S, const Team& tm, const double* coef, bool init,
                                        double* spart_out, S3Pre<T>& P, int par) {
  constexpr int W15 = 15;
  const int n = I.n, tid = threadIdx.x;
  const long long nn = n;
  const S3Geo G = s3_geo(tm.rank);
  PcgOps<T> o = pcg_ops<T>(I, S.kind);
  const PatView<PFC_COL_GRID> pv = op_pat<PFC_COL_GRID>(I, o, tm);
  T* bout = (T*)I.sbas + (long long)(1 - par) * 5 * nn;
  const T* bold = (const T*)I.sbas + (long long)par * 5 * nn;
  const unsigned char* gdir = I.m.gdir;
  T* sp = (T*)pfc_ss;          // new p on the two-step frame [4096]
  T* su = sp + 4096;           // new u on the one-step frame [2304]
  T* stp = su + 2304;          // T p on the one-step frame [2304]
  T* sb = stp + 2304;          // right-hand side on the two-step frame (first launch of a solve) [4096]
  static_assert(12800 * sizeof(T) <= sizeof(pfc_ss), "the frames of ph_scg3 exceed the s-step LDS");
  // own row of this thread
  const int ox = tid & 63, oyl = (tid >> 6) & 3, ozl = tid >> 8;
  const int og = s3_row(G, ox, oyl, ozl);
  if (init) {
    // the solve's right-hand side b on the two-step frame and u_0 = p_0 = D^{-1} b;
    // as ph_scg: b = t - s (A v) by solve kind
    const long long n3 = 3 * nn;
    const double* Vj = I.V + (long long)S.j * n3;
    const int kind = S.kind;
    const T* A = (kind == KIND_Y1 || kind == KIND_X2) ? o.Kv : (kind == KIND_Y0 ? nullptr : o.Mv);
    const T* v = kind == KIND_Y1 ? (const T*)I.y0 : kind == KIND_Z ? (const T*)I.y1 : kind == KIND_X1 ? (const T*)I.zt
                                                                                                      : (const T*)I.x1;
    const double* t = kind == KIND_Y0 ? I.W : (kind == KIND_Y1 ? Vj + nn : (kind == KIND_X2 ? Vj + 2 * nn : nullptr));
    const double ts = kind == KIND_Y0 ? S.vscale : 1.0, sa = kind == KIND_Y1 ? I.tau_p : 1.0;
#pragma unroll
    for (int c = 0; c < PFC_SS_NA; ++c) {
      const int q = tid + c * PFC_WG;
      const int g = s3_row(G, q & 63, ((q >> 6) & 7) - 2, (q >> 9) - 2);
      const int base = (g >> 6) * 64 * W15 + (g & 63);
      T d = T(0);
      if (A) {
#pragma unroll 5
        for (int k = 0; k < W15; ++k) {
          const long long e = (long long)base + k * 64;
          d += gld(A + e) * gld(v + pv.at(e, g));
        }
      }
      const double tt = t ? gld(t + g) * ts : 0.0;
      const double b = !A ? tt : (t ? tt - sa * (double)d : (double)d);
      P.bv[c][0] = gld(o.dinv + g);
      P.bv[c][1] = T(b);
      sb[q] = T(b);
    }
  } else if (S.pcur) {  // the solve ends within these two iterations: x only, on the own row
    const T xo = gld(o.x + og);
    const double p = gld(bold + og), tp = gld(bold + nn + og), u = gld(bold + 3 * nn + og);
    vst(o.x + og, T((double)xo + (coef[0] * p + coef[1] * tp + coef[3] * u)));
    return;
  }
  // operator rows of the one-step frame, issued before the new p and u are
  // formed (whose basis loads they wait for) and in flight across the barrier
  T av[2][W15], dv[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int q1 = tid + c * PFC_WG, t1 = q1 >> 6;
    const int g = s3_row(G, q1 & 63, t1 % 6 - 1, t1 / 6 - 1);
    const int base = (g >> 6) * 64 * W15 + (g & 63);
#pragma unroll
    for (int k = 0; k < W15; ++k) av[c][k] = opval_g(o, (long long)base + k * 64);
    dv[c] = gld(o.dinv + g);
  }
  // new p on the two-step frame, new u on the one-step frame
#pragma unroll
  for (int c = 0; c < PFC_SS_NA; ++c) {
    const int q = tid + c * PFC_WG;
    const T* b = P.bv[c];
    T pn, un;
    if (init) {
      pn = b[0] * b[1];
      un = pn;
    } else {
      pn = T(coef[5] * b[0] + coef[6] * b[1] + coef[7] * b[2] + coef[8] * b[3] + coef[9] * b[4]);
      un = T(coef[10] * b[0] + coef[11] * b[1] + coef[12] * b[2] + coef[13] * b[3] + coef[14] * b[4]);
    }
    sp[q] = pn;
    const int ly = (q >> 6) & 7, lz = q >> 9;
    if (ly >= 1 && ly < 7 && lz >= 1 && lz < 7) su[(q & 63) + 64 * ((ly - 1) + 6 * (lz - 1))] = un;
  }
  lds_barrier();
  // T p on the one-step frame
  auto tprow = [&](int q1, const T* a, T di) {
    const int x = q1 & 63, t1 = q1 >> 6, yl = t1 % 6 - 1, zl = t1 / 6 - 1;
    const unsigned char* gd = gdir + s3_class(G, x, yl, zl) * PFC_GRID_W;
    const int rb = PFC_S3_N * ((yl + 2) + 8 * (zl + 2));
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < W15; ++k) {
      const int code = gd[k];
      acc += a[k] * sp[s3_nx(x, code) + rb + s3_dline(code, 8)];
    }
    stp[q1] = di * acc;
  };
#pragma unroll
  for (int c = 0; c < 2; ++c) tprow(tid + c * PFC_WG, av[c], dv[c]);
  if (tid + 2 * PFC_WG < 2304) {  // the third pass: 256 rows
    const int q1 = tid + 2 * PFC_WG, t1 = q1 >> 6;
    const int g = s3_row(G, q1 & 63, t1 % 6 - 1, t1 / 6 - 1);
    const int base = (g >> 6) * 64 * W15 + (g & 63);
    T a3[W15];
#pragma unroll
    for (int k = 0; k < W15; ++k) a3[k] = opval_g(o, (long long)base + k * 64);
    tprow(q1, a3, gld(o.dinv + g));
  }
  // the own row's operator row (a cache hit: the frame passes read it)
  T ao[W15];
  const int obase = (og >> 6) * 64 * W15 + (og & 63);
#pragma unroll
  for (int k = 0; k < W15; ++k) ao[k] = opval_g(o, (long long)obase + k * 64);
  const T odi = gld(o.dinv + og);
  lds_barrier();
  // own row: T u, T^2 p, the stores and the Gram products
  const unsigned char* gd = gdir + s3_class(G, ox, oyl, ozl) * PFC_GRID_W;
  const int rb1 = PFC_S3_N * ((oyl + 1) + 6 * (ozl + 1));
  T au = T(0), att = T(0), dg = T(0);
#pragma unroll
  for (int k = 0; k < W15; ++k) {
    const int code = gd[k];
    const int i1 = s3_nx(ox, code) + rb1 + s3_dline(code, 6);
    au += ao[k] * su[i1];
    att += ao[k] * stp[i1];
    dg += code == 13 ? ao[k] : T(0);
  }
  const int o2 = ox + PFC_S3_N * ((oyl + 2) + 8 * (ozl + 2)), o1 = ox + rb1;
  const T pn = sp[o2], un = su[o1], tpo = stp[o1], tuo = odi * au, ttp = odi * att;
  double bbo = 0.0;
  if (init) {
    const double bo = (double)sb[o2];
    bbo = bo * bo;
    vst(o.x + og, T(0));
    const long long n3 = 3 * nn;
    if (S.kind == KIND_Y0) {  // the Arnoldi vector v_j = w / ||w||
      double* Vw = I.V + (long long)S.j * n3;
      vst(Vw + og, gld(I.W + og) * S.vscale);
      vst(Vw + nn + og, gld(I.W + nn + og) * S.vscale);
      vst(Vw + 2 * nn + og, gld(I.W + 2 * nn + og) * S.vscale);
    } else if (S.kind == KIND_X2) {  // (4): z_j = (y0 + (y1 - x1) / delta, x1, x2)
      double* Zj = I.Z + (long long)S.j * n3;
      const double y0i = (double)gld((const T*)I.y0 + og), y1i = (double)gld((const T*)I.y1 + og);
      const double x1i = (double)gld((const T*)I.x1 + og);
      vst(Zj + og, y0i + (y1i - x1i) / I.delta);
      vst(Zj + nn + og, x1i);
    }
  } else {
    const T xo = gld(o.x + og);
    const double p = gld(bold + og), tp = gld(bold + nn + og), u = gld(bold + 3 * nn + og);
    vst(o.x + og, T((double)xo + (coef[0] * p + coef[1] * tp + coef[3] * u)));
  }
  vst(bout + og, pn);
  vst(bout + nn + og, tpo);
  vst(bout + 2 * nn + og, ttp);
  vst(bout + 3 * nn + og, un);
  vst(bout + 4 * nn + og, tuo);
  double gp[PFC_SS_NG];
  {
    const double dgo = (double)dg;
    const double v[5] = {(double)pn, (double)tpo, (double)ttp, (double)un, (double)tuo};
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const double di = dgo * v[i];
#pragma unroll
      for (int j = i; j < 5; ++j) gp[ss_tri(i, j, 5)] = di * v[j];
    }
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const double di = dgo * dgo * v[i];
#pragma unroll
      for (int j = i; j < 5; ++j) gp[15 + ss_tri(i - 1, j - 1, 4)] = di * v[j];
    }
  }
  gp[25] = bbo;
  // workgroup sums as ph_scg: each wave by recursive halving, then over the waves
  const int lane = tid & 63, wave = tid >> 6;
  {
    double v32[32];
#pragma unroll
    for (int m = 0; m < 32; ++m) v32[m] = m < PFC_SS_NG ? gp[m] : 0.0;
    const double tot = ss_wave_sums32(v32, lane);
    const int idx = ss_wave_sums32_index(lane);
    if ((lane & 1) == 0) pfc_ssred[wave * 32 + idx] = tot;
  }
  lds_barrier();
  if (tid < PFC_SS_NG) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < PFC_WAVES; ++w) t += pfc_ssred[w * 32 + tid];
    vst(spart_out + (long long)tm.rank * 32 + tid, t);
  }
}

// ---- two Jacobi-PCG iterations per launch on blocks of 2D periodic grids -------
// The iteration of ph_scg3 on a 2D grid of side N, a multiple of 64: rank r
// owns the block of 64 x 16 rows x0 .. x0 + 63, y0 .. y0 + 15 with
// x0 = 64 (r mod N/64), y0 = 16 (r div N/64).  The two-step frame is the
// 68 x 20 rows x0 - 2 .. x0 + 65, y0 - 2 .. y0 + 17, the one-step frame the
// 66 x 18 rows x0 - 1 .. x0 + 64, y0 - 1 .. y0 + 16 (periodic), so a row's
// neighbour in a frame is the row's frame position plus the entry's direction
// (MeshDev::gdir).  Against a range of whole grid lines per workgroup (ph_scg)
// the frames hold 1360 and 1188 rows instead of 3076 and 2050 at N = 512: the
// basis is read, and p and T p are formed, on fewer rows.  Thread t's own row
// is x0 + t mod 64, y0 + t / 64, so a wave's own rows are one SELL slice.
#define PFC_B2_W2 68
#define PFC_B2_N2 (PFC_B2_W2 * 20)  // two-step frame
#define PFC_B2_W1 66
#define PFC_B2_N1 (PFC_B2_W1 * 18)  // one-step frame
#define PFC_B2_W3 70
#define PFC_B2_N3 (PFC_B2_W3 * 22)  // three-step frame (a set-up that also ends the previous solve)
struct B2Geo {
  int x0, y0, N;
};
__device__ __forceinline__ B2Geo b2_geo(int rank, int N) {
  const int bx = N >> 6;
  return B2Geo{(rank % bx) * 64, (rank / bx) * 16, N};
}
__device__ __forceinline__ int b2_wrap(int v, int N) { return v < 0 ? v + N : (v >= N ? v - N : v); }
// row at block coordinates (fx, fy), -2 <= fx < 66, -2 <= fy < 18
__device__ __forceinline__ int b2_row(const B2Geo& G, int fx, int fy) {
  return b2_wrap(G.x0 + fx, G.N) + G.N * b2_wrap(G.y0 + fy, G.N);
}
__device__ __forceinline__ int b2_class(const B2Geo& G, int fx, int fy) {
  return grid_edge(b2_wrap(G.x0 + fx, G.N), G.N) + 3 * grid_edge(b2_wrap(G.y0 + fy, G.N), G.N);
}
// frame offset of an entry's direction code in a frame of width w
__device__ __forceinline__ int b2_doff(int code, int w) { return code % 3 - 1 + w * ((code / 3) % 3 - 1); }

template <typename T>
struct B2Pre {
  T bv[2][5];
};
// the current basis on the two-step frame (the second pass covers 336
// positions; the others load a clamped position), issued before the reductions
template <typename T>
__device__ __forceinline__ void b2_load(const InstDev& I, int rank, B2Pre<T>& P, int par) {
  const long long nn = I.n;
  const int tid = threadIdx.x;
  const B2Geo G = b2_geo(rank, I.m.gN);
  const T* bin = (const T*)I.sbas + (long long)par * 5 * nn;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int q = min(tid + c * PFC_WG, PFC_B2_N2 - 1);
    const int g = b2_row(G, q % PFC_B2_W2 - 2, q / PFC_B2_W2 - 2);
#pragma unroll
    for (int k = 0; k < 5; ++k) P.bv[c][k] = gld(bin + k * nn + g);
  }
}

// The launch after one that ended a solve in its set-up (State::fuse) stores
// that solve's final x on the own rows: x plus the last increment over the
// basis, which is still the other parity's (this launch writes its own rows'
// basis there only afterwards), as the launch that only adds the increment
// would.
template <typename T>
__device__ __forceinline__ void b2_end_store(const InstDev& I, int rank, int kind, double c0, double c1, double c3,
                                             int par) {
  const long long nn = I.n;
  const int tid = threadIdx.x;
  const B2Geo G = b2_geo(rank, I.m.gN);
  const int og = b2_row(G, tid & 63, tid >> 6);
  T* x = pcg_ops<T>(I, kind).x;
  const T* bas = (const T*)I.sbas + (long long)(1 - par) * 5 * nn;
  const T xo = gld(x + og);
  const double p = gld(bas + og), tp = gld(bas + nn + og), u = gld(bas + 3 * nn + og);
  vst(x + og, T((double)xo + (c0 * p + c1 * tp + c3 * u)));
}

template <typename T>
__device__ __forceinline__ void ph_scg2b(const InstDev& I, const State& S, const Team& tm, const double* coef, bool init,
                                         double* spart_out, B2Pre<T>& P, int par) {
  constexpr int W7 = 7;
  const int n = I.n, tid = threadIdx.x;
  const long long nn = n;
  const B2Geo G = b2_geo(tm.rank, I.m.gN);
  PcgOps<T> o = pcg_ops<T>(I, S.kind);
  const PatView<PFC_COL_GRID> pv = op_pat<PFC_COL_GRID>(I, o, tm);
  T* bout = (T*)I.sbas + (long long)(1 - par) * 5 * nn;
  const T* bold = (const T*)I.sbas + (long long)par * 5 * nn;
  const unsigned char* gdir = I.m.gdir;
  T* sp = (T*)pfc_ss;          // new p on the two-step frame
  T* su = sp + PFC_B2_N2;      // new u on the one-step frame
  T* stp = su + PFC_B2_N1;     // T p on the one-step frame
  T* sb = stp + PFC_B2_N1;     // right-hand side on the two-step frame (first launch of a solve)
  T* sv = sb + PFC_B2_N2;      // v on the three-step frame (a set-up that also ends the previous solve)
  static_assert((2 * PFC_B2_N2 + 2 * PFC_B2_N1 + PFC_B2_N3) * sizeof(double) <= sizeof(pfc_ss),
                "the frames of ph_scg2b exceed the s-step LDS");
  const int ox = tid & 63, oy = tid >> 6;
  const int og = b2_row(G, ox, oy);
  if (init) {
    // the solve's right-hand side b on the two-step frame and u_0 = p_0 = D^{-1} b;
    // as ph_scg: b = t - s (A v) by solve kind
    const long long n3 = 3 * nn;
    const double* Vj = I.V + (long long)S.j * n3;
    const int kind = S.kind;
    const T* A = (kind == KIND_Y1 || kind == KIND_X2) ? o.Kv : (kind == KIND_Y0 ? nullptr : o.Mv);
    const T* v = kind == KIND_Y1 ? (const T*)I.y0 : kind == KIND_Z ? (const T*)I.y1 : kind == KIND_X1 ? (const T*)I.zt
                                                                                                      : (const T*)I.x1;
    const double* t = kind == KIND_Y0 ? I.W : (kind == KIND_Y1 ? Vj + nn : (kind == KIND_X2 ? Vj + 2 * nn : nullptr));
    const double ts = kind == KIND_Y0 ? S.vscale : 1.0, sa = kind == KIND_Y1 ? I.tau_p : 1.0;
    const bool fz = S.fuse != 0;
    if (fz) {
      // the previous solve (the P_CH step before, whose x is this solve's v) ends
      // in this launch: its x plus the last increment, formed on the three-step
      // frame; x itself stays unchanged here (other workgroups read it on their
      // halos) and is stored by the next launch (b2_end_store)
      const T* xp = pcg_ops<T>(I, S.fkind).x;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int q3 = tid + c * PFC_WG;
        if (q3 < PFC_B2_N3) {
          const int g = b2_row(G, q3 % PFC_B2_W3 - 3, q3 / PFC_B2_W3 - 3);
          const T xo = gld(xp + g);
          const double p = gld(bold + g), tp = gld(bold + nn + g), u = gld(bold + 3 * nn + g);
          sv[q3] = T((double)xo + (coef[0] * p + coef[1] * tp + coef[3] * u));
        }
      }
      lds_barrier();
    }
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int q = tid + c * PFC_WG, qc = min(q, PFC_B2_N2 - 1);
      const int fx = qc % PFC_B2_W2 - 2, fy = qc / PFC_B2_W2 - 2;
      const int g = b2_row(G, fx, fy);
      const int base = (g >> 6) * 64 * W7 + (g & 63);
      T d = T(0);
      if (A && fz) {
        const unsigned char* gd = gdir + b2_class(G, fx, fy) * PFC_GRID_W;
        const int q3 = (fx + 3) + PFC_B2_W3 * (fy + 3);
#pragma unroll
        for (int k = 0; k < W7; ++k) d += gld(A + (long long)base + k * 64) * sv[q3 + b2_doff(gd[k], PFC_B2_W3)];
      } else if (A) {
#pragma unroll
        for (int k = 0; k < W7; ++k) {
          const long long e = (long long)base + k * 64;
          d += gld(A + e) * gld(v + pv.at(e, g));
        }
      }
      const double tt = t ? gld(t + g) * ts : 0.0;
      const double b = !A ? tt : (t ? tt - sa * (double)d : (double)d);
      P.bv[c][0] = gld(o.dinv + g);
      P.bv[c][1] = T(b);
      if (q < PFC_B2_N2) sb[q] = T(b);
    }
  } else if (S.pcur) {  // the solve ends within these two iterations: x only, on the own row
    const T xo = gld(o.x + og);
    const double p = gld(bold + og), tp = gld(bold + nn + og), u = gld(bold + 3 * nn + og);
    vst(o.x + og, T((double)xo + (coef[0] * p + coef[1] * tp + coef[3] * u)));
    return;
  }
  // operator rows of the one-step frame (the second pass covers 164 rows),
  // issued before the new p and u are formed (whose basis loads they wait for)
  // and in flight across the barrier
  T av[2][W7], dv[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int q1 = min(tid + c * PFC_WG, PFC_B2_N1 - 1);
    const int g = b2_row(G, q1 % PFC_B2_W1 - 1, q1 / PFC_B2_W1 - 1);
    const int base = (g >> 6) * 64 * W7 + (g & 63);
#pragma unroll
    for (int k = 0; k < W7; ++k) av[c][k] = opval_g(o, (long long)base + k * 64);
    dv[c] = gld(o.dinv + g);
  }
  // new p on the two-step frame, new u on the one-step frame
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int q = tid + c * PFC_WG;
    if (q < PFC_B2_N2) {
      const T* b = P.bv[c];
      T pn, un;
      if (init) {
        pn = b[0] * b[1];
        un = pn;
      } else {
        pn = T(coef[5] * b[0] + coef[6] * b[1] + coef[7] * b[2] + coef[8] * b[3] + coef[9] * b[4]);
        un = T(coef[10] * b[0] + coef[11] * b[1] + coef[12] * b[2] + coef[13] * b[3] + coef[14] * b[4]);
      }
      sp[q] = pn;
      const int fx = q % PFC_B2_W2 - 2, fy = q / PFC_B2_W2 - 2;
      if (fx >= -1 && fx < 65 && fy >= -1 && fy < 17) su[(fx + 1) + PFC_B2_W1 * (fy + 1)] = un;
    }
  }
  lds_barrier();
  PFC_SS_STAMP(0);
  // T p on the one-step frame
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int q1 = tid + c * PFC_WG;
    if (q1 < PFC_B2_N1) {
      const int fx = q1 % PFC_B2_W1 - 1, fy = q1 / PFC_B2_W1 - 1;
      const unsigned char* gd = gdir + b2_class(G, fx, fy) * PFC_GRID_W;
      const int q2 = (fx + 2) + PFC_B2_W2 * (fy + 2);
      T acc = T(0);
#pragma unroll
      for (int k = 0; k < W7; ++k) acc += av[c][k] * sp[q2 + b2_doff(gd[k], PFC_B2_W2)];
      stp[q1] = dv[c] * acc;
    }
  }
  // the own row's operator row (a cache hit: the frame pass read it)
  T ao[W7];
  const int obase = (og >> 6) * 64 * W7 + (og & 63);
#pragma unroll
  for (int k = 0; k < W7; ++k) ao[k] = opval_g(o, (long long)obase + k * 64);
  const T odi = gld(o.dinv + og);
  lds_barrier();
  PFC_SS_STAMP(1);
  // own row: T u, T^2 p, the stores and the Gram products
  const unsigned char* gd = gdir + b2_class(G, ox, oy) * PFC_GRID_W;
  const int o1 = (ox + 1) + PFC_B2_W1 * (oy + 1), o2 = (ox + 2) + PFC_B2_W2 * (oy + 2);
  T au = T(0), att = T(0), dg = T(0);
#pragma unroll
  for (int k = 0; k < W7; ++k) {
    const int code = gd[k];
    const int i1 = o1 + b2_doff(code, PFC_B2_W1);
    au += ao[k] * su[i1];
    att += ao[k] * stp[i1];
    dg += code == 13 ? ao[k] : T(0);
  }
  const T pn = sp[o2], un = su[o1], tpo = stp[o1], tuo = odi * au, ttp = odi * att;
  double bbo = 0.0;
  if (init) {
    const double bo = (double)sb[o2];
    bbo = bo * bo;
    vst(o.x + og, T(0));
    const long long n3 = 3 * nn;
    if (S.kind == KIND_Y0) {  // the Arnoldi vector v_j = w / ||w||
      double* Vw = I.V + (long long)S.j * n3;
      vst(Vw + og, gld(I.W + og) * S.vscale);
      vst(Vw + nn + og, gld(I.W + nn + og) * S.vscale);
      vst(Vw + 2 * nn + og, gld(I.W + 2 * nn + og) * S.vscale);
    } else if (S.kind == KIND_X2) {  // (4): z_j = (y0 + (y1 - x1) / delta, x1, x2)
      double* Zj = I.Z + (long long)S.j * n3;
      const double y0i = (double)gld((const T*)I.y0 + og), y1i = (double)gld((const T*)I.y1 + og);
      // x1 (the solve that ends in this launch when it fuses) from the frame
      const double x1i = S.fuse ? (double)sv[(ox + 3) + PFC_B2_W3 * (oy + 3)] : (double)gld((const T*)I.x1 + og);
      vst(Zj + og, y0i + (y1i - x1i) / I.delta);
      vst(Zj + nn + og, x1i);
    }
  } else {
    const T xo = gld(o.x + og);
    const double p = gld(bold + og), tp = gld(bold + nn + og), u = gld(bold + 3 * nn + og);
    vst(o.x + og, T((double)xo + (coef[0] * p + coef[1] * tp + coef[3] * u)));
  }
  vst(bout + og, pn);
  vst(bout + nn + og, tpo);
  vst(bout + 2 * nn + og, ttp);
  vst(bout + 3 * nn + og, un);
  vst(bout + 4 * nn + og, tuo);
  double gp[PFC_SS_NG];
  {
    const double dgo = (double)dg;
    const double v[5] = {(double)pn, (double)tpo, (double)ttp, (double)un, (double)tuo};
#pragma unroll
    for (int i = 0; i < 5; ++i) {
      const double di = dgo * v[i];
#pragma unroll
      for (int j = i; j < 5; ++j) gp[ss_tri(i, j, 5)] = di * v[j];
    }
#pragma unroll
    for (int i = 1; i < 5; ++i) {
      const double di = dgo * dgo * v[i];
#pragma unroll
      for (int j = i; j < 5; ++j) gp[15 + ss_tri(i - 1, j - 1, 4)] = di * v[j];
    }
  }
  gp[25] = bbo;
  PFC_SS_STAMP(2);
  // workgroup sums as ph_scg: each wave by recursive halving, then over the waves
  const int lane = tid & 63, wave = tid >> 6;
  {
    double v32[32];
#pragma unroll
    for (int m = 0; m < 32; ++m) v32[m] = m < PFC_SS_NG ? gp[m] : 0.0;
    const double tot = ss_wave_sums32(v32, lane);
    const int idx = ss_wave_sums32_index(lane);
    if ((lane & 1) == 0) pfc_ssred[wave * 32 + idx] = tot;
  }
  lds_barrier();
  if (tid < PFC_SS_NG) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < PFC_WAVES; ++w) t += pfc_ssred[w * 32 + tid];
    vst(spart_out + (long long)tm.rank * 32 + tid, t);
  }
  PFC_SS_STAMP(3);
}

// ---- orthogonalisation of an Arnoldi step (one reduction) ----------------------
// Modified Gram-Schmidt against v_0..v_j computes h_i = (w - sum_{k<i} h_k v_k,
// v_i) one after the other, which needs j + 1 reductions.  Expanding the inner
// product gives h_i = c_i - sum_{k<i} (v_i, v_k) h_k with c_i = (w, v_i): h
// solves (I + L) h = c, L the strictly lower part of the basis' Gram matrix.
// This equals modified Gram-Schmidt in exact arithmetic for any basis
// (Swirydowicz, Langou, Ananthan, Yang, Thomas, "Low synchronization
// Gram-Schmidt and GMRES algorithms", 2020).  The launch that forms w = A z_j
// therefore also sums c_0..c_j, row j of L ((v_j, v_k), k < j) and (w, w); the
// transition solves for h; the next launch applies w -= sum_i h_i v_i in the
// order of modified Gram-Schmidt and sums (w, w) for h_{j+1,j}.
// Slots of the 64 sums: c_k -> k, (v_j, v_k) -> 32 + k, (w, w) -> 32 + j.
#define PFC_GS_NV 64
__shared__ double pfc_gsred[PFC_WAVES * PFC_GS_NV];

// Sums of 16 values over the 64 lanes of a wave by recursive halving (as
// ss_wave_sums32 for 32): the total of value idx ends in the four lanes of a
// quad, idx = 8 [l >= 32] + 4 [row odd] + 2 [l mod 16 >= 8] + [l mod 8 >= 4].
__device__ __forceinline__ double gs_wave_sums16(const double* v, int lane) {
  double w8[8], w4[4], w2[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) w8[k] = ss_swap<false>(v[k], v[k + 8], lane >= 32);
#pragma unroll
  for (int k = 0; k < 4; ++k) w4[k] = ss_swap<true>(w8[k], w8[k + 4], (lane >> 4) & 1);
#pragma unroll
  for (int k = 0; k < 2; ++k) w2[k] = ss_dppx<0x140>(w4[k], w4[k + 2], (lane & 15) >= 8);  // row_mirror
  double w1 = ss_dppx<0x141>(w2[0], w2[1], (lane & 7) >= 4);                                // row_half_mirror
  w1 += dpp_f64<0x4e, 0xf>(w1);                                                             // quad_perm [2,3,0,1]
  return w1 + dpp_f64<0xb1, 0xf>(w1);                                                       // quad_perm [1,0,3,2]
}
__device__ __forceinline__ int gs_wave_sums16_index(int lane) {
  return (lane >= 32 ? 8 : 0) + (((lane >> 4) & 1) ? 4 : 0) + ((lane & 15) >= 8 ? 2 : 0) + ((lane & 7) >= 4 ? 1 : 0);
}

// w = A_s z_j (the block SpMV of A^R on the scaled system) and the Gram sums
// of the orthogonalisation; the workgroup's 64 sums go to gout[rank * 64 + s].
template <typename T, int L, bool MOB>
__device__ __forceinline__ void ph_aspmv(const InstDev& I, const State& S, const Team& tm, double* gout) {
  const int n = I.n;
  const PatView<L> pv = p1_pat<L>(I, tm);
  const long long n3 = 3LL * n;
  double* Zj = I.Z + (long long)S.j * n3;
  const T* x2 = (const T*)I.x2;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    double w0, w1, w2;
    block_row<L, MOB>(I, pv, sl, tm.lane, I.tau_s, I.m11_s,
              [&](int j, double& mu, double& ps, double& om) { mu = Zj[j]; ps = Zj[n + j]; om = (double)x2[j]; },
              w0, w1, w2);
    if (i < n) {
      vst(I.W + i, w0); vst(I.W + n + i, w1); vst(I.W + 2 * n + i, w2);
      vst(Zj + 2 * n + i, (double)x2[i]);
    }
  }
  // the sums, eight basis vectors at a time; a thread reads back only the rows of
  // w it stored itself
  const int j = S.j;
  const double* Vj = I.V + (long long)j * n3;
  const int lane = tm.lane, wave = tm.wave;
  for (int b = 0; b * 8 <= j; ++b) {
    double v16[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) v16[q] = 0.0;
    PFC_SLICES(I, tm) {
      const int i = sl * 64 + lane;
      if (i < n) {
        double w[3], vj[3];
#pragma unroll
        for (int blk = 0; blk < 3; ++blk) { w[blk] = I.W[blk * n + i]; vj[blk] = gld(Vj + blk * n + i); }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int k = 8 * b + q;
          if (k < j) {
            const double* Vk = I.V + (long long)k * n3;
            double c = 0.0, l = 0.0;
#pragma unroll
            for (int blk = 0; blk < 3; ++blk) {
              const double vk = gld(Vk + blk * n + i);
              c += w[blk] * vk;
              l += vj[blk] * vk;
            }
            v16[q] += c;
            v16[8 + q] += l;
          } else if (k == j) {
            v16[q] += w[0] * vj[0] + w[1] * vj[1] + w[2] * vj[2];
            v16[8 + q] += w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
          }
        }
      }
    }
    const double tot = gs_wave_sums16(v16, lane);
    const int idx = gs_wave_sums16_index(lane);
    if ((lane & 3) == 0) pfc_gsred[wave * PFC_GS_NV + (idx < 8 ? 8 * b + idx : 32 + 8 * b + idx - 8)] = tot;
  }
  __syncthreads();
  const int tid = threadIdx.x;
  if (tid < PFC_GS_NV) {
    const int k = tid & 31;
    double t = 0.0;
    if (k <= j) {
#pragma unroll
      for (int w = 0; w < PFC_WAVES; ++w) t += pfc_gsred[w * PFC_GS_NV + tid];
    }
    vst(gout + (long long)tm.rank * PFC_GS_NV + tid, t);
  }
}

// Sum of the orthogonalisation's Gram partials of a team ([size][64], fixed
// order) into g[0..63] (LDS): thread t sums value t mod 64 over the ranks
// t / 64, t / 64 + 16, ...; the first 64 threads add the 16 group sums.  The
// basis' stored Gram rows L (the Hist record) come to Ls[32 * 32] in the same
// round trip.  Every thread of the workgroup calls this.
static_assert(PFC_WG == PFC_MAXM * PFC_MAXM, "gs_gather loads the stored Gram rows one entry per thread");
#define PFC_GS_U 8  // partials per thread whose loads are issued together
__device__ __forceinline__ void gs_gather(const double* part, int size, const double* Lg, double* g, double* Ls) {
  const int tid = threadIdx.x, v = tid & 63, grp = tid >> 6;
  const double lv = Lg[tid];  // PFC_WG = PFC_MAXM * PFC_MAXM entries, one per thread
  double s = 0.0;
  for (int k0 = grp; k0 < size; k0 += PFC_GS_U * PFC_WAVES) {
    double t[PFC_GS_U];
#pragma unroll
    for (int u = 0; u < PFC_GS_U; ++u) t[u] = part[(long long)min(k0 + u * PFC_WAVES, size - 1) * PFC_GS_NV + v];
#pragma unroll
    for (int u = 0; u < PFC_GS_U; ++u)
      if (k0 + u * PFC_WAVES < size) s += t[u];
  }
  pfc_gsred[grp * PFC_GS_NV + v] = s;
  Ls[tid] = lv;
  __syncthreads();
  if (tid < PFC_GS_NV) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < PFC_WAVES; ++w) t += pfc_gsred[w * PFC_GS_NV + tid];
    g[tid] = t;
  }
  __syncthreads();
}

// w -= sum_{i <= j} h_i v_i in the order of modified Gram-Schmidt; partial (w, w)
__device__ __forceinline__ Red3 ph_gs_update(const InstDev& I, const State& S, const Team& tm, const double* h) {
  const int n = I.n;
  const long long n3 = 3LL * n;
  const int j = S.j;
  double a0 = 0.0;
  PFC_SLICES(I, tm) {
    const int i = sl * 64 + tm.lane;
    if (i < n) {
#pragma unroll
      for (int blk = 0; blk < 3; ++blk) {
        const long long o = (long long)blk * n + i;
        double w = I.W[o];
        for (int k = 0; k <= j; ++k) w -= h[k] * I.V[(long long)k * n3 + o];
        vst(I.W + o, w);
        a0 += w * w;
      }
    }
  }
  return red3(a0, 0.0);
}

}  // namespace pfc
