// Meshes: shared P1 sparsity pattern in SELL-64 layout, GPU assembly of the
// P1 mass and stiffness matrices, element lists for the in-place reassembly
// of N(psi) and the cubic load, and the mesh-level operators of the C ABI.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "device.h"
#include "host.h"

namespace pfc {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
int hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return PFC_ERR_HIP;
}

// ---- kernels ----------------------------------------------------------------

// Volume |T| and barycentric gradients of each simplex from its vertex
// coordinates: with B = [X_1 - X_0, ..., X_m - X_0], grad lambda_a (a >= 1) is
// row a-1 of B^{-1} and grad lambda_0 = -sum of the others.
__global__ void k_elem_geom(int dim, int n_elem, const double* __restrict__ X, double* __restrict__ vol,
                            double* __restrict__ grad, int* __restrict__ bad) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  const int k = dim + 1;
  const double* x = X + (long long)e * k * dim;
  double g[4][3];
  double det;
  if (dim == 2) {
    const double b00 = x[2] - x[0], b10 = x[3] - x[1];   // column 0: X1 - X0
    const double b01 = x[4] - x[0], b11 = x[5] - x[1];   // column 1: X2 - X0
    det = b00 * b11 - b01 * b10;
    const double id = 1.0 / det;
    g[1][0] = b11 * id;  g[1][1] = -b01 * id;
    g[2][0] = -b10 * id; g[2][1] = b00 * id;
    g[0][0] = -(g[1][0] + g[2][0]);
    g[0][1] = -(g[1][1] + g[2][1]);
    vol[e] = fabs(det) * 0.5;
  } else {
    double b[3][3];  // b[r][c] = coordinate r of X_{c+1} - X_0
    for (int c = 0; c < 3; ++c)
      for (int r = 0; r < 3; ++r) b[r][c] = x[(c + 1) * 3 + r] - x[r];
    const double c00 = b[1][1] * b[2][2] - b[1][2] * b[2][1];
    const double c01 = b[1][2] * b[2][0] - b[1][0] * b[2][2];
    const double c02 = b[1][0] * b[2][1] - b[1][1] * b[2][0];
    det = b[0][0] * c00 + b[0][1] * c01 + b[0][2] * c02;
    const double id = 1.0 / det;
    // inverse = adjugate / det; adj[i][j] = cofactor[j][i]
    double inv[3][3];
    inv[0][0] = c00 * id;
    inv[1][0] = c01 * id;
    inv[2][0] = c02 * id;
    inv[0][1] = (b[0][2] * b[2][1] - b[0][1] * b[2][2]) * id;
    inv[1][1] = (b[0][0] * b[2][2] - b[0][2] * b[2][0]) * id;
    inv[2][1] = (b[0][1] * b[2][0] - b[0][0] * b[2][1]) * id;
    inv[0][2] = (b[0][1] * b[1][2] - b[0][2] * b[1][1]) * id;
    inv[1][2] = (b[0][2] * b[1][0] - b[0][0] * b[1][2]) * id;
    inv[2][2] = (b[0][0] * b[1][1] - b[0][1] * b[1][0]) * id;
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) g[a + 1][c] = inv[a][c];
    for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
    vol[e] = fabs(det) / 6.0;
  }
  if (!(det != 0.0) || !isfinite(det)) bad[0] = 1;
  for (int a = 0; a < k; ++a)
    for (int c = 0; c < dim; ++c) grad[((long long)e * k + a) * dim + c] = g[a][c];
}

// M_ij = sum_T |T| (1 + [a==b]) / ((m+1)(m+2)),  K_ij = sum_T |T| grad lambda_a . grad lambda_b,
// gathered per stored entry over its element list (deterministic, no atomics).
__global__ void k_assemble_MK(MeshDev m, const double* __restrict__ grad, double* __restrict__ M,
                              double* __restrict__ K) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nnz_sell) return;
  const int k = m.dim + 1;
  const double cmass = 1.0 / ((m.dim + 1.0) * (m.dim + 2.0));
  double mv = 0.0, kv = 0.0;
  for (int t = m.sl_el_ptr[e]; t < m.sl_el_ptr[e + 1]; ++t) {
    const int pk = m.sl_el[t];
    const int el = pk >> 4, a = (pk >> 2) & 3, b = pk & 3;
    const double v = m.elem_vol[el];
    mv += v * cmass * (a == b ? 2.0 : 1.0);
    double d = 0.0;
    for (int c = 0; c < m.dim; ++c) d += grad[((long long)el * k + a) * m.dim + c] * grad[((long long)el * k + b) * m.dim + c];
    kv += v * d;
  }
  M[e] = mv;
  K[e] = kv;
}

// P2: M_ij = sum_T |T| M2[a][b],  K_ij = sum_T |T| sum_{s,t} (grad l_s . grad l_t) D[s][t][a][b]
// with the reference tables of the quadratic basis (Section 3, p = 2).
__global__ void k_assemble_MK_p2(MeshDev m, const double* __restrict__ grad, double* __restrict__ M,
                                 double* __restrict__ K) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nnz_sell) return;
  const int k = m.dim + 1, q = m.nloc;
  double mv = 0.0, kv = 0.0;
  for (int t = m.sl_el_ptr[e]; t < m.sl_el_ptr[e + 1]; ++t) {
    const int pk = m.sl_el[t];
    const int el = pk >> 8, a = (pk >> 4) & 15, b = pk & 15;
    const double v = m.elem_vol[el];
    mv += v * m.p2_M2[a * q + b];
    double kk = 0.0;
    for (int s = 0; s < k; ++s)
      for (int u = 0; u < k; ++u) {
        double g = 0.0;
        for (int c = 0; c < m.dim; ++c)
          g += grad[((long long)el * k + s) * m.dim + c] * grad[((long long)el * k + u) * m.dim + c];
        kk += g * m.p2_D[((s * k + u) * q + a) * q + b];
      }
    kv += v * kk;
  }
  M[e] = mv;
  K[e] = kv;
}

// Element stiffness |T| grad lambda_a . grad lambda_b, upper triangle a <= b in
// row order (kept for the mobility matrices of the PFC1 model).
__global__ void k_elem_stiff(int dim, int n_elem, const double* __restrict__ vol, const double* __restrict__ grad,
                             double* __restrict__ ek) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_elem) return;
  const int k = dim + 1, kk = k * (k + 1) / 2;
  int q = 0;
  for (int a = 0; a < k; ++a)
    for (int b = a; b < k; ++b) {
      double d = 0.0;
      for (int c = 0; c < dim; ++c) d += grad[((long long)e * k + a) * dim + c] * grad[((long long)e * k + b) * dim + c];
      ek[(long long)e * kk + q++] = vol[e] * d;
    }
}

// float copies of M and K; Jacobi diagonal 1/diag(M) in both precisions
__global__ void k_mesh_derived(MeshDev m, const double* __restrict__ M, const double* __restrict__ K, float* Mf,
                               float* Kf, double* dinvM, float* dinvMf) {
  const int sl = blockIdx.x * PFC_WAVES + (threadIdx.x >> 6);
  if (sl >= m.n_slices) return;
  const int lane = threadIdx.x & 63;
  const int i = sl * 64 + lane;
  const int base = m.slice_ptr[sl];
  const int w = (m.slice_ptr[sl + 1] - base) >> 6;
  double dg = 0.0;
  for (int k = 0; k < w; ++k) {
    const long long e = (long long)base + k * 64 + lane;
    Mf[e] = (float)M[e];
    Kf[e] = (float)K[e];
    if (m.col[e] == i) dg += M[e];
  }
  if (i < m.n) {
    dinvM[i] = 1.0 / dg;
    dinvMf[i] = (float)(1.0 / dg);
  }
}

__global__ void k_spmv(MeshDev m, const double* __restrict__ A, const double* __restrict__ x, double* __restrict__ y) {
  const int sl = blockIdx.x * PFC_WAVES + (threadIdx.x >> 6);
  if (sl >= m.n_slices) return;
  const int lane = threadIdx.x & 63;
  const int i = sl * 64 + lane;
  const int base = m.slice_ptr[sl];
  const int w = (m.slice_ptr[sl + 1] - base) >> 6;
  double acc = 0.0;
  for (int k = 0; k < w; ++k) {
    const long long e = (long long)base + k * 64 + lane;
    acc += A[e] * x[m.col[e]];
  }
  if (i < m.n) y[i] = acc;
}

__global__ void k_assemble_N_csr(MeshDev m, const long long* __restrict__ csr2sell, int nnz,
                                 const double* __restrict__ psi, double* __restrict__ N) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nnz) return;
  N[s] = -3.0 * entry_Mpsi2(m, csr2sell[s], [&](int j) { return psi[j]; });
}

__global__ void k_load_psi3(MeshDev m, const double* __restrict__ psi, double* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m.n) return;
  g[i] = node_psi3(m, i, [&](int j) { return psi[j]; });
}

// ---- host construction ---------------------------------------------------------

template <typename T>
static int upload(T** dst, const T* src, size_t count) {
  *dst = nullptr;
  if (count == 0) count = 1;
  PFC_HIP(hipMalloc((void**)dst, count * sizeof(T)));
  if (src) PFC_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
  return PFC_OK;
}

static void mesh_free(pfc_mesh* m) {
  if (!m) return;
  void* ptrs[] = {m->d_slice_ptr, m->d_col, m->d_M, m->d_K, m->d_Mf, m->d_Kf, m->d_dinvM, m->d_dinvMf,
                  m->d_sl_el_ptr, m->d_sl_el, m->d_nd_el_ptr, m->d_nd_el, m->d_elem_nodes, m->d_vol, m->d_csr2sell,
                  m->d_w_slice_ptr, m->d_w_col, m->d_w_p1pos, m->d_w_tri_ptr, m->d_w_tri, m->d_elemK, m->d_p2tab};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete m;
}

static int check_elements(int k, int n, int n_elem, const int32_t* en) {
  for (long long e = 0; e < n_elem; ++e) {
    for (int a = 0; a < k; ++a) {
      const int v = en[e * k + a];
      if (v < 0 || v >= n) {
        set_error("element " + std::to_string(e) + " has node index out of range");
        return PFC_ERR_ARG;
      }
      for (int b = 0; b < a; ++b)
        if (en[e * k + b] == v) {
          set_error("element " + std::to_string(e) + " repeats a node");
          return PFC_ERR_ARG;
        }
    }
  }
  return PFC_OK;
}

// node -> (element, local index) lists in element order
static void node_elements(int k, int n, int n_elem, const int32_t* en, std::vector<int>& ptr, std::vector<int>& lst) {
  const int bits = k <= 4 ? 2 : 4;
  ptr.assign(n + 1, 0);
  for (long long t = 0; t < (long long)n_elem * k; ++t) ptr[en[t] + 1]++;
  for (int i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
  lst.resize((size_t)n_elem * k);
  std::vector<int> fill(ptr.begin(), ptr.end() - 1);
  for (int e = 0; e < n_elem; ++e)
    for (int a = 0; a < k; ++a) lst[fill[en[(long long)e * k + a]]++] = (e << bits) | a;
}

static int slot_of(const pfc_mesh* m, int row, int col) {
  const int* b = m->col_idx.data() + m->row_ptr[row];
  const int* e = m->col_idx.data() + m->row_ptr[row + 1];
  const int* p = std::lower_bound(b, e, col);
  if (p == e || *p != col) return -1;
  return (int)(p - m->col_idx.data());
}

// SELL-64 layout, element lists per stored entry, uploads.  Requires the CSR
// pattern in m->row_ptr / m->col_idx.
// Whether the columns of the mesh's (sorted) rows follow from grid_col: the
// mesh is a periodic grid of side N (n = N^dim < 2^22, nodes numbered
// x + N (y + N z)), every row has w entries, and rows of one edge class
// (grid_class) have the same column offsets j - i.  The offsets of a class are
// read off its first row; every row, that one included, is then checked entry
// by entry against grid_col.
// Direction of every entry of a grid mesh's rows (for sweeps over blocks of the
// grid): per row class and entry, the step (dx, dy, dz) from the row to the
// column with each component in -1..1 (periodic), read off the class's first
// row and checked on every row.  False if some entry is farther than one step.
static bool detect_grid_dirs(const pfc_mesh* m, int w, int N, std::vector<unsigned char>& gdir) {
  const int n = m->n, dim = m->dim;
  const float inv = 1.0f / (float)N;
  gdir.assign((size_t)PFC_GRID_CLASSES * PFC_GRID_W, 13);  // 13: no step
  std::vector<char> have(PFC_GRID_CLASSES, 0);
  auto coord = [&](int v, int c) { return c == 0 ? v % N : (c == 1 ? (v / N) % N : v / (N * N)); };
  auto step = [&](int a, int b) {  // b - a on the circle of N, or 9 when farther than one step
    int d = b - a;
    if (d > N / 2) d -= N;
    if (d < -(N / 2)) d += N;
    return (d >= -1 && d <= 1) ? d : 9;
  };
  for (int i = 0; i < n; ++i) {
    const int cls = grid_class(i, N, inv);
    const int* col = m->col_idx.data() + m->row_ptr[i];
    for (int k = 0; k < w; ++k) {
      int code = 0, mul = 1;
      for (int c = 0; c < 3; ++c, mul *= 3) {
        const int d = c < dim ? step(coord(i, c), coord(col[k], c)) : 0;
        if (d == 9) return false;
        code += (d + 1) * mul;
      }
      unsigned char& g = gdir[(size_t)cls * PFC_GRID_W + k];
      if (!have[cls]) g = (unsigned char)code;
      else if (g != code) return false;
    }
    have[cls] = 1;
  }
  return true;
}

static bool detect_grid(const pfc_mesh* m, int w, int& gN, std::vector<int>& glin) {
  const int n = m->n, dim = m->dim;
  const int N = (int)std::llround(std::pow((double)n, 1.0 / dim));
  long long p = 1;
  for (int d = 0; d < dim; ++d) p *= N;
  if (p != n || N < 3 || n >= PFC_GRID_MAXN || w < 1 || w > PFC_GRID_W) return false;
  for (int i = 0; i < n; ++i)
    if (m->row_ptr[i + 1] - m->row_ptr[i] != w) return false;
  const float inv = 1.0f / (float)N;
  glin.assign((size_t)PFC_GRID_CLASSES * PFC_GRID_W, 0);
  std::vector<char> have(PFC_GRID_CLASSES, 0);
  for (int i = 0; i < n; ++i) {
    const int cls = grid_class(i, N, inv);
    const int* col = m->col_idx.data() + m->row_ptr[i];
    if (!have[cls]) {
      for (int k = 0; k < w; ++k) glin[(size_t)cls * PFC_GRID_W + k] = col[k] - i;
      have[cls] = 1;
    }
    for (int k = 0; k < w; ++k)
      if (grid_col(i, k, n, N, inv, glin.data()) != col[k]) return false;
  }
  gN = N;
  return true;
}

static int finish_layout(pfc_mesh* m, const int32_t* en, const std::vector<int>& ndp, const std::vector<int>& ndl) {
  const int n = m->n, k = m->nloc;
  const int bits = k <= 4 ? 2 : 4;
  m->n_slices = (n + 63) / 64;
  std::vector<int> sptr(m->n_slices + 1, 0);
  for (int s = 0; s < m->n_slices; ++s) {
    int w = 0;
    for (int l = 0; l < 64; ++l) {
      const int i = s * 64 + l;
      if (i < n) w = std::max(w, m->row_ptr[i + 1] - m->row_ptr[i]);
    }
    const long long nxt = (long long)sptr[s] + 64LL * w;
    if (nxt > 2000000000LL) {
      set_error("mesh too large for 32-bit entry offsets");
      return PFC_ERR_ARG;
    }
    sptr[s + 1] = (int)nxt;
  }
  m->nnz_sell = sptr[m->n_slices];
  // common slice width (structured meshes): lets kernels compute slice offsets
  // and stage a workgroup's columns in LDS
  m->uniform_width = 0;
  if (m->n_slices > 0) {
    const int w0 = (sptr[1] - sptr[0]) / 64;
    bool same = w0 >= 1 && w0 <= PFC_LCOL_W;
    for (int s = 1; same && s < m->n_slices; ++s) same = (sptr[s + 1] - sptr[s]) / 64 == w0;
    if (same) m->uniform_width = w0;
  }
  // periodic grids: the kernels can compute the columns (grid_col)
  int gN = 0;
  std::vector<int> glin;
#ifndef PFC_NO_GRID_COLUMNS
  if (m->uniform_width > 0 && !detect_grid(m, m->uniform_width, gN, glin)) gN = 0;
#endif
  std::vector<int> scol((size_t)m->nnz_sell);
  m->csr2sell.assign(m->nnz, 0);
  for (int s = 0; s < m->n_slices; ++s) {
    const int w = (sptr[s + 1] - sptr[s]) / 64;
    for (int l = 0; l < 64; ++l) {
      const int i = s * 64 + l;
      const int len = i < n ? m->row_ptr[i + 1] - m->row_ptr[i] : 0;
      for (int kk = 0; kk < w; ++kk) {
        const long long pos = (long long)sptr[s] + kk * 64LL + l;
        if (kk < len) {
          scol[pos] = m->col_idx[m->row_ptr[i] + kk];
          m->csr2sell[m->row_ptr[i] + kk] = pos;
        } else {
          scol[pos] = i < n ? i : 0;
        }
      }
    }
  }
  // element contributions of each stored entry, in element order
  std::vector<int> cnt((size_t)m->nnz_sell + 1, 0);
  std::vector<long long> pos_of_pair((size_t)m->n_elem * k * k);
  for (long long e = 0; e < m->n_elem; ++e)
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b) {
        const int s = slot_of(m, en[e * k + a], en[e * k + b]);
        if (s < 0) {
          set_error("element " + std::to_string(e) + " has a node pair missing from the pattern");
          return PFC_ERR_ARG;
        }
        const long long p = m->csr2sell[s];
        pos_of_pair[(e * k + a) * k + b] = p;
        cnt[p + 1]++;
      }
  for (long long p = 0; p < m->nnz_sell; ++p) cnt[p + 1] += cnt[p];
  if ((long long)cnt[m->nnz_sell] != (long long)m->n_elem * k * k) {
    set_error("internal: element list size mismatch");
    return PFC_ERR_STATE;
  }
  std::vector<int> lst((size_t)m->n_elem * k * k);
  std::vector<int> fill(cnt.begin(), cnt.end() - 1);
  for (long long e = 0; e < m->n_elem; ++e)
    for (int a = 0; a < k; ++a)
      for (int b = 0; b < k; ++b)
        lst[fill[pos_of_pair[(e * k + a) * k + b]]++] = (int)((e << (2 * bits)) | (a << bits) | b);
  int rc;
  if ((rc = upload(&m->d_slice_ptr, sptr.data(), sptr.size()))) return rc;
  if ((rc = upload(&m->d_col, scol.data(), scol.size()))) return rc;
  if ((rc = upload(&m->d_sl_el_ptr, cnt.data(), cnt.size()))) return rc;
  if ((rc = upload(&m->d_sl_el, lst.data(), lst.size()))) return rc;
  if ((rc = upload(&m->d_nd_el_ptr, ndp.data(), ndp.size()))) return rc;
  if ((rc = upload(&m->d_nd_el, ndl.data(), ndl.size()))) return rc;
  if ((rc = upload(&m->d_elem_nodes, en, (size_t)m->n_elem * k))) return rc;
  if ((rc = upload(&m->d_csr2sell, m->csr2sell.data(), m->csr2sell.size()))) return rc;
  if ((rc = upload<double>(&m->d_M, nullptr, m->nnz_sell))) return rc;
  if ((rc = upload<double>(&m->d_K, nullptr, m->nnz_sell))) return rc;
  if ((rc = upload<float>(&m->d_Mf, nullptr, m->nnz_sell))) return rc;
  if ((rc = upload<float>(&m->d_Kf, nullptr, m->nnz_sell))) return rc;
  if ((rc = upload<double>(&m->d_dinvM, nullptr, n))) return rc;
  if ((rc = upload<float>(&m->d_dinvMf, nullptr, n))) return rc;
  MeshDev& d = m->dev;
  d.n = n; d.dim = m->dim; d.n_slices = m->n_slices; d.n_elem = m->n_elem; d.nnz_sell = m->nnz_sell;
  d.uw = m->uniform_width;
  d.slice_ptr = m->d_slice_ptr; d.col = m->d_col; d.M = m->d_M; d.K = m->d_K; d.Mf = m->d_Mf; d.Kf = m->d_Kf;
  d.dinvM = m->d_dinvM; d.dinvMf = m->d_dinvMf; d.sl_el_ptr = m->d_sl_el_ptr; d.sl_el = m->d_sl_el;
  d.degree = m->degree; d.nloc = m->nloc;
  d.gN = gN;
  d.gInv = gN ? 1.0f / (float)gN : 0.0f;
  std::memset(d.glin, 0, sizeof(d.glin));
  if (gN) std::memcpy(d.glin, glin.data(), sizeof(d.glin));
  std::vector<unsigned char> gdir;
  d.gdir_ok = gN && detect_grid_dirs(m, m->uniform_width, gN, gdir) ? 1 : 0;
  std::memset(d.gdir, 13, sizeof(d.gdir));
  if (d.gdir_ok) std::memcpy(d.gdir, gdir.data(), sizeof(d.gdir));
  d.nd_el_ptr = m->d_nd_el_ptr; d.nd_el = m->d_nd_el; d.elem_nodes = m->d_elem_nodes; d.elem_vol = m->d_vol;
  return PFC_OK;
}

static int derive(pfc_mesh* m) {
  const int nb = slice_blocks(m->n_slices);
  hipLaunchKernelGGL(k_mesh_derived, dim3(nb), dim3(PFC_WG), 0, 0, m->dev, m->d_M, m->d_K, m->d_Mf, m->d_Kf,
                     m->d_dinvM, m->d_dinvMf);
  PFC_HIP(hipGetLastError());
  PFC_HIP(hipDeviceSynchronize());
  // every diagonal entry of M must be positive
  std::vector<double> dg(m->n);
  PFC_HIP(hipMemcpy(dg.data(), m->d_dinvM, sizeof(double) * m->n, hipMemcpyDeviceToHost));
  for (int i = 0; i < m->n; ++i)
    if (!(dg[i] > 0.0) || !std::isfinite(dg[i])) {
      set_error("mass matrix has a non-positive diagonal entry at row " + std::to_string(i));
      return PFC_ERR_ARG;
    }
  return PFC_OK;
}

// Pattern of K M_D^{-1} K (nodes at graph distance <= 2) in SELL-64 layout,
// with, for each stored entry (i, j), the P1 positions of (i, j) and of the
// pairs (i, k), (k, j) over the common neighbours k.  Symbolic only; the
// values of S_D are formed on the GPU per time step size.
int build_second_ring(pfc_mesh* m) {
  if (m->d_w_slice_ptr) return PFC_OK;
  const int n = m->n;
  // the triples below hold P1 positions as int
  if (m->nnz_sell > 2000000000LL) { set_error("second-ring pattern too large"); return PFC_ERR_ARG; }
  std::vector<int> wrp(n + 1, 0), wcol;
  std::vector<int> buf;
  for (int i = 0; i < n; ++i) {
    buf.clear();
    for (int t = m->row_ptr[i]; t < m->row_ptr[i + 1]; ++t) {
      const int k = m->col_idx[t];
      buf.insert(buf.end(), m->col_idx.begin() + m->row_ptr[k], m->col_idx.begin() + m->row_ptr[k + 1]);
    }
    std::sort(buf.begin(), buf.end());
    buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    wcol.insert(wcol.end(), buf.begin(), buf.end());
    if (wcol.size() > 2000000000ULL) { set_error("second-ring pattern too large"); return PFC_ERR_ARG; }
    wrp[i + 1] = (int)wcol.size();
  }
  const int ns = m->n_slices;
  std::vector<int> sptr(ns + 1, 0);
  for (int sl = 0; sl < ns; ++sl) {
    int w = 0;
    for (int l = 0; l < 64; ++l) {
      const int i = sl * 64 + l;
      if (i < n) w = std::max(w, wrp[i + 1] - wrp[i]);
    }
    const long long nx = (long long)sptr[sl] + 64LL * w;
    if (nx > 2000000000LL) { set_error("second-ring pattern too large"); return PFC_ERR_ARG; }
    sptr[sl + 1] = (int)nx;
  }
  const long long nw = sptr[ns];
  std::vector<int> scol((size_t)nw);
  std::vector<long long> p1pos((size_t)nw, -1);
  std::vector<int> tptr((size_t)nw + 1, 0);
  std::vector<int> tri;
  // first pass: layout; second: triples in entry order
  for (int sl = 0; sl < ns; ++sl) {
    const int w = (sptr[sl + 1] - sptr[sl]) / 64;
    for (int l = 0; l < 64; ++l) {
      const int i = sl * 64 + l;
      const int len = i < n ? wrp[i + 1] - wrp[i] : 0;
      for (int kk = 0; kk < w; ++kk) {
        const long long pos = (long long)sptr[sl] + kk * 64LL + l;
        scol[pos] = kk < len ? wcol[wrp[i] + kk] : (i < n ? i : 0);
      }
    }
  }
  for (int sl = 0; sl < ns; ++sl) {
    const int w = (sptr[sl + 1] - sptr[sl]) / 64;
    for (int kk = 0; kk < w; ++kk)
      for (int l = 0; l < 64; ++l) {
        const long long pos = (long long)sptr[sl] + kk * 64LL + l;
        const int i = sl * 64 + l;
        const int len = i < n ? wrp[i + 1] - wrp[i] : 0;
        if (kk < len) {
          const int j = scol[pos];
          const int sij = slot_of(m, i, j);
          if (sij >= 0) p1pos[pos] = m->csr2sell[sij];
          for (int t = m->row_ptr[i]; t < m->row_ptr[i + 1]; ++t) {
            const int k = m->col_idx[t];
            const int skj = slot_of(m, k, j);
            if (skj < 0) continue;
            tri.push_back((int)m->csr2sell[t]);
            tri.push_back((int)m->csr2sell[skj]);
          }
        }
        if (tri.size() / 2 > 2000000000ULL) { set_error("second-ring pattern too large"); return PFC_ERR_ARG; }
        tptr[pos + 1] = (int)(tri.size() / 2);
      }
  }
  // positions were visited in increasing order, so tptr is a prefix sum over them
  int rc;
  if ((rc = upload(&m->d_w_slice_ptr, sptr.data(), sptr.size()))) return rc;
  if ((rc = upload(&m->d_w_col, scol.data(), scol.size()))) return rc;
  if ((rc = upload(&m->d_w_p1pos, p1pos.data(), p1pos.size()))) return rc;
  if ((rc = upload(&m->d_w_tri_ptr, tptr.data(), tptr.size()))) return rc;
  if ((rc = upload(&m->d_w_tri, tri.data(), tri.size()))) return rc;
  m->dev.w_nnz_sell = nw;
  m->dev.w_slice_ptr = m->d_w_slice_ptr;
  m->dev.w_col = m->d_w_col;
  m->dev.w_p1pos = m->d_w_p1pos;
  m->dev.w_tri_ptr = m->d_w_tri_ptr;
  m->dev.w_tri = m->d_w_tri;
  return PFC_OK;
}

}  // namespace pfc

using namespace pfc;

extern "C" {

const char* pfc_last_error(void) { return g_err.c_str(); }

}  // extern "C"

namespace pfc {

// ---- P2 reference tables ---------------------------------------------------------
// The quadratic Lagrange basis on an m-simplex as polynomials in the
// barycentric coordinates l_0..l_m: vertex a: l_a (2 l_a - 1); edge (i, j):
// 4 l_i l_j, edges in the local order of pfc_mesh_create_p2.  Integrals of
// products follow from int_T prod l^alpha = |T| m! prod(alpha!) / (m + |alpha|)!.
namespace {
using Mono = std::array<int, 4>;
using Poly = std::vector<std::pair<Mono, double>>;

const int kEdges2[3][2] = {{0, 1}, {1, 2}, {0, 2}};
const int kEdges3[6][2] = {{0, 1}, {1, 2}, {0, 2}, {0, 3}, {1, 3}, {2, 3}};

double fact(int k) { double f = 1.0; for (int i = 2; i <= k; ++i) f *= i; return f; }

double integral(const Poly& p, int m) {  // int_T p / |T|
  double s = 0.0;
  for (const auto& t : p) {
    int deg = 0;
    double num = fact(m);
    for (int i = 0; i <= m; ++i) { num *= fact(t.first[i]); deg += t.first[i]; }
    s += t.second * num / fact(m + deg);
  }
  return s;
}

Poly mul(const Poly& a, const Poly& b) {
  Poly r;
  for (const auto& x : a)
    for (const auto& y : b) {
      Mono e;
      for (int i = 0; i < 4; ++i) e[i] = x.first[i] + y.first[i];
      bool found = false;
      for (auto& z : r)
        if (z.first == e) { z.second += x.second * y.second; found = true; break; }
      if (!found) r.push_back({e, x.second * y.second});
    }
  return r;
}

Poly dl(const Poly& a, int i) {  // d / d l_i
  Poly r;
  for (const auto& x : a)
    if (x.first[i] > 0) {
      Mono e = x.first;
      e[i] -= 1;
      r.push_back({e, x.second * x.first[i]});
    }
  return r;
}

std::vector<Poly> p2_basis(int m) {
  std::vector<Poly> B;
  for (int a = 0; a <= m; ++a) {
    Mono sq{0, 0, 0, 0}, li{0, 0, 0, 0};
    sq[a] = 2;
    li[a] = 1;
    B.push_back({{sq, 2.0}, {li, -1.0}});
  }
  const int ne = m == 2 ? 3 : 6;
  for (int k = 0; k < ne; ++k) {
    const int i = m == 2 ? kEdges2[k][0] : kEdges3[k][0];
    const int j = m == 2 ? kEdges2[k][1] : kEdges3[k][1];
    Mono e{0, 0, 0, 0};
    e[i] += 1;
    e[j] += 1;
    B.push_back({{e, 4.0}});
  }
  return B;
}
}  // namespace

// M2 [q*q], D [k*k*q*q], C4 [q^4] concatenated
static std::vector<double> p2_tables(int m) {
  const std::vector<Poly> B = p2_basis(m);
  const int q = (int)B.size(), k = m + 1;
  std::vector<double> t((size_t)q * q + (size_t)k * k * q * q + (size_t)q * q * q * q, 0.0);
  double* M2 = t.data();
  double* D = M2 + q * q;
  double* C4 = D + k * k * q * q;
  std::vector<Poly> P2((size_t)q * q);
  for (int a = 0; a < q; ++a)
    for (int b = 0; b < q; ++b) {
      P2[a * q + b] = mul(B[a], B[b]);
      M2[a * q + b] = integral(P2[a * q + b], m);
    }
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j)
      for (int a = 0; a < q; ++a)
        for (int b = 0; b < q; ++b) D[((i * k + j) * q + a) * q + b] = integral(mul(dl(B[a], i), dl(B[b], j)), m);
  for (int a = 0; a < q; ++a)
    for (int b = a; b < q; ++b)
      for (int c = 0; c < q; ++c)
        for (int d = c; d < q; ++d) {
          const double v = integral(mul(P2[a * q + b], P2[c * q + d]), m);
          C4[((a * q + b) * q + c) * q + d] = C4[((b * q + a) * q + c) * q + d] = v;
          C4[((a * q + b) * q + d) * q + c] = C4[((b * q + a) * q + d) * q + c] = v;
        }
  return t;
}

// Meshes of Lagrange elements of degree 1 or 2 from element nodes and vertex
// coordinates; M and K assembled on the GPU.
static int create_lagrange(const char* who, int dim, int degree, int n, int n_elem, const int32_t* elem_nodes,
                           const double* elem_coords, pfc_mesh** out) {
  const int kv = dim + 1;                                         // vertices per element
  const int k = degree == 1 ? kv : (dim + 1) * (dim + 2) / 2;    // nodes per element
  const int max_elem = degree == 1 ? (1 << 26) : (1 << 22);      // element index fits the packed lists
  if (!out || !elem_nodes || !elem_coords || (dim != 2 && dim != 3) || n <= 0 || n_elem <= 0 || n_elem > max_elem) {
    set_error(std::string(who) + ": invalid arguments");
    return PFC_ERR_ARG;
  }
  *out = nullptr;
  int rc = check_elements(k, n, n_elem, elem_nodes);
  if (rc) return rc;
  for (long long t = 0; t < (long long)n_elem * kv * dim; ++t)
    if (!std::isfinite(elem_coords[t])) {
      set_error(std::string(who) + ": non-finite coordinate");
      return PFC_ERR_ARG;
    }
  // a simplex of (numerically) zero volume has no barycentric gradients:
  // |det(x_1 - x_0, ..., x_m - x_0)| must exceed 1e-12 times the product of
  // its edge lengths from x_0
  for (long long e = 0; e < n_elem; ++e) {
    const double* x = elem_coords + e * kv * dim;
    double J[3][3] = {{0.0}};
    double scale = 1.0;
    for (int a = 1; a <= dim; ++a) {
      double len2 = 0.0;
      for (int d = 0; d < dim; ++d) {
        J[a - 1][d] = x[a * dim + d] - x[d];
        len2 += J[a - 1][d] * J[a - 1][d];
      }
      scale *= std::sqrt(len2);
    }
    const double det = dim == 2 ? J[0][0] * J[1][1] - J[0][1] * J[1][0]
                                : J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                      J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                      J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(std::fabs(det) > 1e-12 * scale)) {
      set_error(std::string(who) + ": element " + std::to_string(e) + " is degenerate (zero volume)");
      return PFC_ERR_ARG;
    }
  }
  pfc_mesh* m = new pfc_mesh();
  m->dim = dim; m->n = n; m->n_elem = n_elem;
  m->degree = degree; m->nloc = k;
  const int bits = k <= 4 ? 2 : 4;
  std::vector<int> ndp, ndl;
  node_elements(k, n, n_elem, elem_nodes, ndp, ndl);
  // pattern: every node pair of a common simplex (diagonal included)
  m->row_ptr.assign(n + 1, 0);
  std::vector<int> cols;
  std::vector<int> rowbuf;
  for (int i = 0; i < n; ++i) {
    rowbuf.clear();
    for (int t = ndp[i]; t < ndp[i + 1]; ++t) {
      const int e = ndl[t] >> bits;
      for (int a = 0; a < k; ++a) rowbuf.push_back(elem_nodes[(long long)e * k + a]);
    }
    if (rowbuf.empty()) rowbuf.push_back(i);
    std::sort(rowbuf.begin(), rowbuf.end());
    rowbuf.erase(std::unique(rowbuf.begin(), rowbuf.end()), rowbuf.end());
    cols.insert(cols.end(), rowbuf.begin(), rowbuf.end());
    if (cols.size() > 2000000000ULL) { mesh_free(m); set_error(std::string(who) + ": pattern too large"); return PFC_ERR_ARG; }
    m->row_ptr[i + 1] = (int)cols.size();
  }
  m->col_idx.swap(cols);
  m->nnz = m->row_ptr[n];
  // isolated nodes would make M singular
  for (int i = 0; i < n; ++i)
    if (ndp[i + 1] == ndp[i]) {
      mesh_free(m);
      set_error(std::string(who) + ": node " + std::to_string(i) + " belongs to no element");
      return PFC_ERR_ARG;
    }
  if ((rc = finish_layout(m, elem_nodes, ndp, ndl))) { mesh_free(m); return rc; }
  if (degree == 2) {
    const std::vector<double> tab = p2_tables(dim);
    if ((rc = upload(&m->d_p2tab, tab.data(), tab.size()))) { mesh_free(m); return rc; }
    m->dev.p2_M2 = m->d_p2tab;
    m->dev.p2_D = m->d_p2tab + k * k;
    m->dev.p2_C4 = m->dev.p2_D + kv * kv * k * k;
  }
  // element geometry and assembly on the GPU
  double* d_X = nullptr;
  double* d_grad = nullptr;
  int* d_bad = nullptr;
  auto fail = [&](int code) {
    if (d_X) (void)hipFree(d_X);
    if (d_grad) (void)hipFree(d_grad);
    if (d_bad) (void)hipFree(d_bad);
    mesh_free(m);
    return code;
  };
  if ((rc = upload(&d_X, elem_coords, (size_t)n_elem * kv * dim))) return fail(rc);
  if ((rc = upload<double>(&d_grad, nullptr, (size_t)n_elem * kv * dim))) return fail(rc);
  if ((rc = upload<double>(&m->d_vol, nullptr, n_elem))) return fail(rc);
  if ((rc = upload<int>(&d_bad, nullptr, 1))) return fail(rc);
  m->dev.elem_vol = m->d_vol;
  if (hipMemset(d_bad, 0, sizeof(int)) != hipSuccess) return fail(hip_fail(hipErrorUnknown, "hipMemset"));
  hipLaunchKernelGGL(k_elem_geom, dim3((n_elem + 255) / 256), dim3(256), 0, 0, dim, n_elem, d_X, m->d_vol, d_grad, d_bad);
  if (degree == 1) {
    hipLaunchKernelGGL(k_assemble_MK, dim3((unsigned)((m->nnz_sell + 255) / 256)), dim3(256), 0, 0, m->dev, d_grad,
                       m->d_M, m->d_K);
    // element stiffness for the mobility matrices of the PFC1 model
    if ((rc = upload<double>(&m->d_elemK, nullptr, (size_t)n_elem * (kv * (kv + 1) / 2)))) return fail(rc);
    m->dev.elem_K = m->d_elemK;
    hipLaunchKernelGGL(k_elem_stiff, dim3((n_elem + 255) / 256), dim3(256), 0, 0, dim, n_elem, m->d_vol, d_grad,
                       m->d_elemK);
  } else {
    hipLaunchKernelGGL(k_assemble_MK_p2, dim3((unsigned)((m->nnz_sell + 255) / 256)), dim3(256), 0, 0, m->dev,
                       d_grad, m->d_M, m->d_K);
  }
  hipError_t he = hipGetLastError();
  if (he == hipSuccess) he = hipDeviceSynchronize();
  if (he != hipSuccess) return fail(hip_fail(he, "element assembly"));
  int bad = 0;
  if (hipMemcpy(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess) return fail(PFC_ERR_HIP);
  if (bad) {
    set_error(std::string(who) + ": degenerate simplex");
    return fail(PFC_ERR_ARG);
  }
  (void)hipFree(d_X); d_X = nullptr;
  (void)hipFree(d_grad); d_grad = nullptr;
  (void)hipFree(d_bad); d_bad = nullptr;
  if ((rc = derive(m))) { mesh_free(m); return rc; }
  *out = m;
  return PFC_OK;
}

}  // namespace pfc

extern "C" {

int pfc_mesh_create_p1(int dim, int n, int n_elem, const int32_t* elem_nodes, const double* elem_coords,
                       pfc_mesh** out) {
  return create_lagrange("pfc_mesh_create_p1", dim, 1, n, n_elem, elem_nodes, elem_coords, out);
}

int pfc_mesh_create_p2(int dim, int n, int n_elem, const int32_t* elem_nodes, const double* elem_coords,
                       pfc_mesh** out) {
  return create_lagrange("pfc_mesh_create_p2", dim, 2, n, n_elem, elem_nodes, elem_coords, out);
}

int pfc_mesh_create_csr(int dim, int n, int nnz, const int32_t* row_ptr, const int32_t* col_idx, const double* M_val,
                        const double* K_val, int n_elem, const int32_t* elem_nodes, const double* elem_vol,
                        pfc_mesh** out) {
  if (!out || !row_ptr || !col_idx || !M_val || !K_val || !elem_nodes || !elem_vol || (dim != 2 && dim != 3) ||
      n <= 0 || nnz <= 0 || n_elem <= 0 || n_elem > (1 << 26)) {
    set_error("pfc_mesh_create_csr: invalid arguments");
    return PFC_ERR_ARG;
  }
  *out = nullptr;
  if (row_ptr[0] != 0 || row_ptr[n] != nnz) {
    set_error("pfc_mesh_create_csr: row_ptr must start at 0 and end at nnz");
    return PFC_ERR_ARG;
  }
  for (int i = 0; i < n; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) {
      set_error("pfc_mesh_create_csr: row_ptr not monotone");
      return PFC_ERR_ARG;
    }
    bool diag = false;
    for (int t = row_ptr[i]; t < row_ptr[i + 1]; ++t) {
      const int c = col_idx[t];
      if (c < 0 || c >= n || (t > row_ptr[i] && c <= col_idx[t - 1])) {
        set_error("pfc_mesh_create_csr: column indices out of range or not strictly increasing in row " +
                  std::to_string(i));
        return PFC_ERR_ARG;
      }
      if (c == i) diag = true;
      if (!std::isfinite(M_val[t]) || !std::isfinite(K_val[t])) {
        set_error("pfc_mesh_create_csr: non-finite matrix value");
        return PFC_ERR_ARG;
      }
    }
    if (!diag) {
      set_error("pfc_mesh_create_csr: missing diagonal in row " + std::to_string(i));
      return PFC_ERR_ARG;
    }
  }
  for (int e = 0; e < n_elem; ++e)
    if (!(elem_vol[e] > 0.0) || !std::isfinite(elem_vol[e])) {
      set_error("pfc_mesh_create_csr: element volumes must be positive");
      return PFC_ERR_ARG;
    }
  int rc = check_elements(dim + 1, n, n_elem, elem_nodes);
  if (rc) return rc;
  pfc_mesh* m = new pfc_mesh();
  m->dim = dim; m->n = n; m->n_elem = n_elem; m->nnz = nnz;
  m->degree = 1; m->nloc = dim + 1;
  m->row_ptr.assign(row_ptr, row_ptr + n + 1);
  m->col_idx.assign(col_idx, col_idx + nnz);
  // structural symmetry
  for (int i = 0; i < n; ++i)
    for (int t = row_ptr[i]; t < row_ptr[i + 1]; ++t)
      if (slot_of(m, col_idx[t], i) < 0) {
        mesh_free(m);
        set_error("pfc_mesh_create_csr: pattern is not structurally symmetric");
        return PFC_ERR_ARG;
      }
  std::vector<int> ndp, ndl;
  node_elements(dim + 1, n, n_elem, elem_nodes, ndp, ndl);
  if ((rc = finish_layout(m, elem_nodes, ndp, ndl))) { mesh_free(m); return rc; }
  std::vector<double> sM((size_t)m->nnz_sell, 0.0), sK((size_t)m->nnz_sell, 0.0);
  for (int t = 0; t < nnz; ++t) {
    sM[m->csr2sell[t]] = M_val[t];
    sK[m->csr2sell[t]] = K_val[t];
  }
  if ((rc = upload(&m->d_vol, elem_vol, n_elem))) { mesh_free(m); return rc; }
  m->dev.elem_vol = m->d_vol;
  if (hipMemcpy(m->d_M, sM.data(), sizeof(double) * sM.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->d_K, sK.data(), sizeof(double) * sK.size(), hipMemcpyHostToDevice) != hipSuccess) {
    mesh_free(m);
    set_error("pfc_mesh_create_csr: upload failed");
    return PFC_ERR_HIP;
  }
  if ((rc = derive(m))) { mesh_free(m); return rc; }
  *out = m;
  return PFC_OK;
}

// The arrays are in device memory: copy them to the host and validate and lay
// them out as pfc_mesh_create_csr does (mesh set-up, once per mesh).
int pfc_mesh_create_csr_device(int dim, int n, int nnz, const int32_t* row_ptr, const int32_t* col_idx,
                               const double* M_val, const double* K_val, int n_elem, const int32_t* elem_nodes,
                               const double* elem_vol, pfc_mesh** out) {
  if (!out || !row_ptr || !col_idx || !M_val || !K_val || !elem_nodes || !elem_vol || (dim != 2 && dim != 3) ||
      n <= 0 || nnz <= 0 || n_elem <= 0 || n_elem > (1 << 26)) {
    set_error("pfc_mesh_create_csr_device: invalid arguments");
    return PFC_ERR_ARG;
  }
  *out = nullptr;
  const void* ptrs[6] = {row_ptr, col_idx, M_val, K_val, elem_nodes, elem_vol};
  for (const void* p : ptrs) {
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess || (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)) {
      (void)hipGetLastError();
      set_error("pfc_mesh_create_csr_device: an array is not in device memory");
      return PFC_ERR_ARG;
    }
  }
  std::vector<int32_t> rp((size_t)n + 1), ci((size_t)nnz), en((size_t)n_elem * (dim + 1));
  std::vector<double> mv((size_t)nnz), kv((size_t)nnz), ev((size_t)n_elem);
  auto get = [](void* dst, const void* src, size_t bytes) {
    return hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost) == hipSuccess;
  };
  if (!get(rp.data(), row_ptr, rp.size() * 4) || !get(ci.data(), col_idx, ci.size() * 4) ||
      !get(mv.data(), M_val, mv.size() * 8) || !get(kv.data(), K_val, kv.size() * 8) ||
      !get(en.data(), elem_nodes, en.size() * 4) || !get(ev.data(), elem_vol, ev.size() * 8)) {
    (void)hipGetLastError();
    set_error("pfc_mesh_create_csr_device: copy from device memory failed");
    return PFC_ERR_HIP;
  }
  return pfc_mesh_create_csr(dim, n, nnz, rp.data(), ci.data(), mv.data(), kv.data(), n_elem, en.data(), ev.data(), out);
}

int pfc_mesh_query(const pfc_mesh* m, int* dim, int* n, int* nnz, int* n_elem) {
  if (!m) { set_error("pfc_mesh_query: null mesh"); return PFC_ERR_ARG; }
  if (dim) *dim = m->dim;
  if (n) *n = m->n;
  if (nnz) *nnz = m->nnz;
  if (n_elem) *n_elem = m->n_elem;
  return PFC_OK;
}

int pfc_mesh_grid_side(const pfc_mesh* m, int* N) {
  if (!m || !N) { set_error("pfc_mesh_grid_side: null argument"); return PFC_ERR_ARG; }
  *N = m->dev.gN;
  return PFC_OK;
}

int pfc_mesh_export_csr(const pfc_mesh* m, int32_t* row_ptr, int32_t* col_idx, double* M_val, double* K_val) {
  if (!m) { set_error("pfc_mesh_export_csr: null mesh"); return PFC_ERR_ARG; }
  if (row_ptr) std::memcpy(row_ptr, m->row_ptr.data(), sizeof(int) * (m->n + 1));
  if (col_idx) std::memcpy(col_idx, m->col_idx.data(), sizeof(int) * m->nnz);
  if (M_val || K_val) {
    std::vector<double> sM((size_t)m->nnz_sell), sK((size_t)m->nnz_sell);
    PFC_HIP(hipMemcpy(sM.data(), m->d_M, sizeof(double) * sM.size(), hipMemcpyDeviceToHost));
    PFC_HIP(hipMemcpy(sK.data(), m->d_K, sizeof(double) * sK.size(), hipMemcpyDeviceToHost));
    for (int t = 0; t < m->nnz; ++t) {
      if (M_val) M_val[t] = sM[m->csr2sell[t]];
      if (K_val) K_val[t] = sK[m->csr2sell[t]];
    }
  }
  return PFC_OK;
}

void pfc_mesh_destroy(pfc_mesh* m) { mesh_free(m); }

int pfc_spmv(const pfc_mesh* m, int which, const double* x, double* y, void* stream) {
  if (!m || !x || !y || (which != PFC_OP_M && which != PFC_OP_K)) {
    set_error("pfc_spmv: invalid arguments");
    return PFC_ERR_ARG;
  }
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_spmv, dim3(slice_blocks(m->n_slices)), dim3(PFC_WG), 0, s, m->dev,
                     which == PFC_OP_M ? m->d_M : m->d_K, x, y);
  PFC_HIP(hipGetLastError());
  PFC_HIP(hipStreamSynchronize(s));
  return PFC_OK;
}

int pfc_assemble_N(const pfc_mesh* m, const double* psi, double* N_csr, void* stream) {
  if (!m || !psi || !N_csr) { set_error("pfc_assemble_N: invalid arguments"); return PFC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_assemble_N_csr, dim3((m->nnz + 255) / 256), dim3(256), 0, s, m->dev, m->d_csr2sell, m->nnz,
                     psi, N_csr);
  PFC_HIP(hipGetLastError());
  PFC_HIP(hipStreamSynchronize(s));
  return PFC_OK;
}

int pfc_load_psi3(const pfc_mesh* m, const double* psi, double* g, void* stream) {
  if (!m || !psi || !g) { set_error("pfc_load_psi3: invalid arguments"); return PFC_ERR_ARG; }
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_load_psi3, dim3((m->n + 255) / 256), dim3(256), 0, s, m->dev, psi, g);
  PFC_HIP(hipGetLastError());
  PFC_HIP(hipStreamSynchronize(s));
  return PFC_OK;
}

}  // extern "C"
