// Host-only inspection entry points (lg_host_*) and the thread-local error message.
#include <algorithm>
#include <cstring>
#include <new>

#include "precompute.hpp"
#include "status.hpp"

namespace lg {
namespace {
thread_local std::string g_err;
}
void set_error(const std::string& msg) { g_err = msg; }
const char* last_error() { return g_err.c_str(); }

MeshIn mesh_in(const sim_mesh* m) {
  MeshIn r;
  r.n = m->n_nodes;
  r.m = m->n_tets;
  r.rest = m->rest_xyz;
  r.tets = m->tets;
  r.init = m->init_xyz;
  r.vel = m->init_vel;
  r.n_pins = m->n_pins;
  r.pin_nodes = m->pin_nodes;
  r.pin_group = m->pin_group;
  return r;
}

MaterialIn material_in(const sim_material* m) {
  MaterialIn r;
  r.model = m->model;
  r.E = m->E;
  r.nu = m->nu;
  r.rho = m->rho;
  r.tet_model = m->tet_model;
  r.tet_E = m->tet_E;
  r.tet_nu = m->tet_nu;
  return r;
}
}  // namespace lg

struct lg_host {
  lg::HostScene s;
};

extern "C" {

const char* sim_last_error(void) { return lg::last_error(); }

int lg_host_create(const sim_mesh* mesh, const sim_material* mat, double h, double pin_weight_scale,
                   int32_t want_dense_S, lg_host_t* out) {
  if (!mesh || !mat || !out) {
    lg::set_error("null argument");
    return SIM_E_ARG;
  }
  if (mesh->n_pins > 0 && (!mesh->pin_nodes || !mesh->pin_group)) {
    lg::set_error("pins without arrays");
    return SIM_E_ARG;
  }
  if (want_dense_S && mesh->n_nodes > 4096) {
    lg::set_error("dense S only for n <= 4096");
    return SIM_E_ARG;
  }
  try {
    auto* hs = new lg_host();
    std::string err;
    int rc = lg::precompute(lg::mesh_in(mesh), lg::material_in(mat), h, pin_weight_scale,
                            want_dense_S != 0, hs->s, err);
    if (rc != SIM_OK) {
      delete hs;
      lg::set_error(err);
      return rc;
    }
    *out = hs;
    return SIM_OK;
  } catch (const std::bad_alloc&) {
    lg::set_error("host allocation failed");
    return SIM_E_NOMEM;
  } catch (...) {
    lg::set_error("unexpected host error");
    return SIM_E_ARG;
  }
}

int lg_host_info(lg_host_t hs, int64_t* info) {
  if (!hs || !info) return SIM_E_ARG;
  const auto& s = hs->s;
  int64_t chains = 0;
  for (int i = 0; i < s.n; ++i) chains += (s.chain_end[i] == i);
  info[0] = s.n;
  info[1] = s.m;
  info[2] = s.nnz_S;
  info[3] = s.nnz_L;
  info[4] = s.row_ptr.empty() ? 0 : s.row_ptr.back();
  info[5] = s.depth.empty() ? 0 : *std::max_element(s.depth.begin(), s.depth.end());
  info[6] = chains;
  info[7] = 0;
  return SIM_OK;
}

int lg_host_ordering(lg_host_t hs, int32_t* perm, int32_t* parent) {
  if (!hs) return SIM_E_ARG;
  if (perm) std::copy(hs->s.perm.begin(), hs->s.perm.end(), perm);
  if (parent) std::copy(hs->s.parent.begin(), hs->s.parent.end(), parent);
  return SIM_OK;
}

int lg_host_dense_A(lg_host_t hs, double* A) {
  if (!hs || !A) return SIM_E_ARG;
  const auto& s = hs->s;
  if (s.n > 4096) return SIM_E_ARG;
  std::memset(A, 0, sizeof(double) * (size_t)s.n * s.n);
  for (int o = 0; o < s.n; ++o)
    for (int64_t p = s.a_ptr[o]; p < s.a_ptr[o + 1]; ++p)
      A[(size_t)s.perm[o] * s.n + s.perm[s.a_idx[p]]] = s.a_val[p];
  return SIM_OK;
}

int lg_host_dense_S(lg_host_t hs, double* S) {
  if (!hs || !S || hs->s.S_dense64.empty()) {
    lg::set_error("dense S not requested");
    return SIM_E_ARG;
  }
  std::copy(hs->s.S_dense64.begin(), hs->s.S_dense64.end(), S);
  return SIM_OK;
}

// u = S^T (S b): S b from the row storage, S^T y from the column-path storage.
int lg_host_apply_StS(lg_host_t hs, const double* b, double* u) {
  if (!hs || !b || !u) return SIM_E_ARG;
  const auto& s = hs->s;
  const int n = s.n;
  std::vector<double> y(3 * (size_t)n, 0.0);
  for (int i = 0; i < n; ++i) {
    int64_t base = s.row_ptr[i];
    int len = (int)(s.row_ptr[i + 1] - base);
    for (int k = 0; k < len; ++k) {
      int j = s.row_lo4[i] + k;
      if (j >= n) break;
      double v = s.row_val[base + k];
      for (int c = 0; c < 3; ++c) y[3 * (size_t)i + c] += v * b[3 * (size_t)j + c];
    }
  }
  for (int j = 0; j < n; ++j) {
    double acc[3] = {0, 0, 0};
    int idx = 0;
    for (int i = j; i != -1; i = s.parent[i], ++idx) {
      double v = s.col_val[s.col_ptr[j] + idx];
      for (int c = 0; c < 3; ++c) acc[c] += v * y[3 * (size_t)i + c];
    }
    for (int c = 0; c < 3; ++c) u[3 * (size_t)j + c] = acc[c];
  }
  return SIM_OK;
}

int lg_host_destroy(lg_host_t hs) {
  delete hs;
  return SIM_OK;
}

}  // extern "C"
