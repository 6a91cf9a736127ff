// Host-side objects behind the C ABI handles.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/pfc.h"
#include "pfc_internal.h"

namespace pfc {

void set_error(const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define PFC_HIP(call)                                   \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return pfc::hip_fail(_e, #call); \
  } while (0)

}  // namespace pfc

struct pfc_mesh {
  int dim = 0, n = 0, nnz = 0, n_elem = 0, n_slices = 0;
  int uniform_width = 0;               // common slice width (1..16), 0 if slices differ
  int degree = 1, nloc = 0;            // Lagrange degree and nodes per element
  double* d_p2tab = nullptr;           // P2 reference tables (M2, D, C4)
  long long nnz_sell = 0;
  std::vector<int> row_ptr, col_idx;   // CSR pattern (host)
  std::vector<long long> csr2sell;     // CSR slot -> SELL position
  // device arrays
  int* d_slice_ptr = nullptr;
  int* d_col = nullptr;
  double* d_M = nullptr;
  double* d_K = nullptr;
  float* d_Mf = nullptr;
  float* d_Kf = nullptr;
  double* d_dinvM = nullptr;
  float* d_dinvMf = nullptr;
  int* d_sl_el_ptr = nullptr;
  int* d_sl_el = nullptr;
  int* d_nd_el_ptr = nullptr;
  int* d_nd_el = nullptr;
  int* d_elem_nodes = nullptr;
  double* d_vol = nullptr;
  long long* d_csr2sell = nullptr;
  double* d_elemK = nullptr;           // element stiffness (P1 meshes), for the PFC1 mobility
  // second-ring pattern for the S_D preconditioner (built on first use)
  int* d_w_slice_ptr = nullptr;
  int* d_w_col = nullptr;
  long long* d_w_p1pos = nullptr;
  int* d_w_tri_ptr = nullptr;
  int* d_w_tri = nullptr;
  MeshDev dev{};
};

namespace pfc {
int build_second_ring(pfc_mesh* m);
}

namespace pfc {
// grid of standalone kernels over the slices of a mesh (one wave per slice)
inline int slice_blocks(int n_slices) { return (n_slices + PFC_WAVES - 1) / PFC_WAVES; }
}  // namespace pfc
