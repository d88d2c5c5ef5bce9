// Host-side precomputation for the HIP solver (runs once per scene, in float64).
//
// Paper: Sec. 3.3 (constant system matrix A = M + h^2 sum w G^T G), Sec. 4.2
// (Theorem 1 and Algorithm 2: L = Cholesky(A), S = L^-1, A^-1 = S^T S, with a
// fill-reducing nested-dissection order), Algorithm 4 (S precomputed once).
//
// Layout decisions (MI355X-first, not from the paper):
//  * nodes are renumbered by geometric nested dissection followed by a postorder
//    of the elimination tree, so every subtree is a contiguous index range
//    [lo_i, i] and row i of S is dense over exactly that range;
//  * S is stored twice in float32: row-skyline (row i over columns [lo4_i, hi4_i),
//    16-byte aligned, zero padded) for the y = S b pass, and column paths
//    (column j over its ancestors j, parent(j), ..., root, in ascending order)
//    for the u = S^T y pass and the Delassus products;
//  * "chains" are maximal runs of consecutive nodes in which each node is the
//    only child of the next one; an ancestor path is a short list of chain runs.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace lg {

struct MeshIn {
  int n = 0, m = 0;
  const double* rest = nullptr;   // [n][3]
  const int32_t* tets = nullptr;  // [m][4]
  const double* init = nullptr;   // [n][3] or null
  const double* vel = nullptr;    // [n][3] or null
  int n_pins = 0;
  const int32_t* pin_nodes = nullptr;
  const int32_t* pin_group = nullptr;
};

struct MaterialIn {
  int model = 1;
  double E = 1e5, nu = 0.3, rho = 1000.0;
  const int32_t* tet_model = nullptr;
  const double* tet_E = nullptr;
  const double* tet_nu = nullptr;
};

struct HostScene {
  int n = 0, m = 0;
  double h = 0.01;
  // caller-order inputs
  std::vector<double> rest, init, vel;      // [n*3]
  std::vector<int32_t> tets;                // [m*4] caller node ids
  // per-tet material and rest data (caller tet order)
  std::vector<int32_t> model;
  std::vector<double> mu, lam, kstiff, vol, Dm_inv;  // Dm_inv rows d1,d2,d3: [m*9]
  std::vector<double> mass;                 // [n] caller order
  std::vector<int32_t> pin_nodes, pin_group;
  std::vector<double> pin_h2w;              // [n_pins]
  // node-level system matrix A_n in caller order (CSR, sorted columns)
  std::vector<int64_t> a_ptr;
  std::vector<int32_t> a_idx;
  std::vector<double> a_val;
  // ordering: perm[orig] = new, iperm[new] = orig
  std::vector<int32_t> perm, iperm;
  std::vector<int32_t> parent, lo, depth;   // new order
  std::vector<int32_t> chain_end;           // [n] last node of the chain containing i
  // S storage (new order)
  std::vector<int64_t> row_ptr;             // [n+1] float offsets, multiples of 4
  std::vector<int32_t> row_lo4;             // [n]   first stored column of row i
  std::vector<float> row_val;
  std::vector<int64_t> col_ptr;             // [n+1]
  std::vector<float> col_val;               // column j: S[j..root path][j], ascending node order
  int64_t nnz_S = 0;                        // sum (depth+1)
  int64_t nnz_L = 0;
  double chol_min_pivot = 0.0;
  // optional float64 dense S for tests (new order, row-major), only when requested
  std::vector<double> S_dense64;
};

// Returns 0 on success, or a negative SIM_E_* code with `err` filled.
int precompute(const MeshIn& mesh, const MaterialIn& mat, double h, double pin_weight_scale,
               bool want_dense_S, HostScene& out, std::string& err);

}  // namespace lg
