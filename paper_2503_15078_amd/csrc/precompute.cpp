// Host-side precomputation: rest quantities, the constant system matrix, the
// nested-dissection + postorder ordering, the float64 Cholesky factor and the
// sparse inverse S = L^-1 (Sec. 3.3, Sec. 4.2 Theorem 1 and Algorithm 2).
#include "precompute.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <functional>
#include <numeric>
#include <thread>

#include "status.hpp"

namespace lg {
namespace {

constexpr int kLeaf = 24;  // nested-dissection leaf size

int worker_count() {
  int hw = (int)std::thread::hardware_concurrency();
  if (const char* s = std::getenv("OMP_NUM_THREADS")) {
    int v = std::atoi(s);
    if (v > 0) hw = std::min(hw > 0 ? hw : v, v);
  }
  return std::max(1, std::min(hw, 32));
}

void parallel_for(int64_t count, int64_t chunk, const std::function<void(int64_t, int64_t)>& body) {
  int nt = worker_count();
  if (nt <= 1 || count <= chunk) {
    body(0, count);
    return;
  }
  std::atomic<int64_t> next{0};
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&]() {
      for (;;) {
        int64_t b = next.fetch_add(chunk);
        if (b >= count) break;
        body(b, std::min(count, b + chunk));
      }
    });
  for (auto& x : th) x.join();
}

// Geometric nested dissection on the node graph of A_n: split the current node set
// at the median coordinate of its longest bounding-box axis, take as separator the
// nodes of the upper half adjacent to the lower half, recurse on both halves and
// number the separator last.
struct ND {
  const std::vector<int64_t>& ptr;
  const std::vector<int32_t>& idx;
  const double* X;
  std::vector<int8_t> side;
  std::vector<int32_t> out;
  ND(const std::vector<int64_t>& p, const std::vector<int32_t>& i, const double* x, int n)
      : ptr(p), idx(i), X(x), side(n, 0) {}

  void run(std::vector<int32_t>& nodes) {
    if ((int)nodes.size() <= kLeaf) {
      out.insert(out.end(), nodes.begin(), nodes.end());
      return;
    }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int v : nodes)
      for (int d = 0; d < 3; ++d) {
        lo[d] = std::min(lo[d], X[3 * v + d]);
        hi[d] = std::max(hi[d], X[3 * v + d]);
      }
    int axes[3] = {0, 1, 2};
    std::sort(axes, axes + 3, [&](int a, int b) { return hi[a] - lo[a] > hi[b] - lo[b]; });
    for (int ai = 0; ai < 3; ++ai) {
      int ax = axes[ai];
      std::vector<double> c(nodes.size());
      for (size_t k = 0; k < nodes.size(); ++k) c[k] = X[3 * nodes[k] + ax];
      std::nth_element(c.begin(), c.begin() + c.size() / 2, c.end());
      double med = c[c.size() / 2];
      std::vector<int32_t> L, R;
      for (int v : nodes) (X[3 * v + ax] < med ? L : R).push_back(v);
      if (L.empty() || R.empty()) continue;
      for (int v : L) side[v] = 1;
      for (int v : R) side[v] = 2;
      std::vector<int32_t> Rr, S;
      for (int v : R) {
        bool touch = false;
        for (int64_t p = ptr[v]; p < ptr[v + 1] && !touch; ++p) touch = side[idx[p]] == 1;
        (touch ? S : Rr).push_back(v);
      }
      for (int v : nodes) side[v] = 0;
      run(L);
      run(Rr);
      out.insert(out.end(), S.begin(), S.end());
      return;
    }
    out.insert(out.end(), nodes.begin(), nodes.end());
  }
};

void inv3(const double* A, double* Ai, double& det) {
  // A row-major 3x3
  double c00 = A[4] * A[8] - A[5] * A[7];
  double c01 = A[5] * A[6] - A[3] * A[8];
  double c02 = A[3] * A[7] - A[4] * A[6];
  det = A[0] * c00 + A[1] * c01 + A[2] * c02;
  double id = 1.0 / det;
  Ai[0] = c00 * id;
  Ai[1] = (A[2] * A[7] - A[1] * A[8]) * id;
  Ai[2] = (A[1] * A[5] - A[2] * A[4]) * id;
  Ai[3] = c01 * id;
  Ai[4] = (A[0] * A[8] - A[2] * A[6]) * id;
  Ai[5] = (A[2] * A[3] - A[0] * A[5]) * id;
  Ai[6] = c02 * id;
  Ai[7] = (A[1] * A[6] - A[0] * A[7]) * id;
  Ai[8] = (A[0] * A[4] - A[1] * A[3]) * id;
}

}  // namespace

int precompute(const MeshIn& mesh, const MaterialIn& mat, double h, double pin_weight_scale,
               bool want_dense_S, HostScene& S, std::string& err) {
  const int n = mesh.n, m = mesh.m;
  if (n <= 0 || m <= 0 || !mesh.rest || !mesh.tets) {
    err = "empty mesh";
    return SIM_E_MESH;
  }
  if (!(h > 0.0) || !std::isfinite(h)) {
    err = "time step must be positive";
    return SIM_E_ARG;
  }
  S.n = n;
  S.m = m;
  S.h = h;
  S.rest.assign(mesh.rest, mesh.rest + 3 * (size_t)n);
  for (double v : S.rest)
    if (!std::isfinite(v)) {
      err = "non-finite rest position";
      return SIM_E_MESH;
    }
  S.init = mesh.init ? std::vector<double>(mesh.init, mesh.init + 3 * (size_t)n) : S.rest;
  S.vel = mesh.vel ? std::vector<double>(mesh.vel, mesh.vel + 3 * (size_t)n) : std::vector<double>(3 * (size_t)n, 0.0);
  for (double v : S.init)
    if (!std::isfinite(v)) {
      err = "non-finite initial position";
      return SIM_E_ARG;
    }
  for (double v : S.vel)
    if (!std::isfinite(v)) {
      err = "non-finite initial velocity";
      return SIM_E_ARG;
    }
  S.tets.assign(mesh.tets, mesh.tets + 4 * (size_t)m);
  std::vector<char> used(n, 0);
  for (int32_t v : S.tets) {
    if (v < 0 || v >= n) {
      err = "tet index out of range";
      return SIM_E_MESH;
    }
    used[v] = 1;
  }
  for (int i = 0; i < n; ++i)
    if (!used[i]) {
      err = "unused node " + std::to_string(i);
      return SIM_E_MESH;
    }

  // ---- rest shape, materials, lumped mass
  S.model.resize(m);
  S.mu.resize(m);
  S.lam.resize(m);
  S.kstiff.resize(m);
  S.vol.resize(m);
  S.Dm_inv.resize(9 * (size_t)m);
  S.mass.assign(n, 0.0);
  if (!(mat.rho > 0.0)) {
    err = "density must be positive";
    return SIM_E_ARG;
  }
  for (int t = 0; t < m; ++t) {
    const int32_t* T = &S.tets[4 * (size_t)t];
    double Dm[9];
    for (int c = 0; c < 3; ++c)
      for (int r = 0; r < 3; ++r) Dm[3 * r + c] = S.rest[3 * T[c + 1] + r] - S.rest[3 * T[0] + r];
    double det;
    inv3(Dm, &S.Dm_inv[9 * (size_t)t], det);
    double V = det / 6.0;
    if (!(V > 0.0)) {
      err = "non-positive volume in tet " + std::to_string(t);
      return SIM_E_MESH;
    }
    S.vol[t] = V;
    int model = mat.tet_model ? mat.tet_model[t] : mat.model;
    double E = mat.tet_E ? mat.tet_E[t] : mat.E;
    double nu = mat.tet_nu ? mat.tet_nu[t] : mat.nu;
    if (model < 0 || model > 3 || !(E > 0.0) || !(nu > -1.0 && nu < 0.5)) {
      err = "bad material in tet " + std::to_string(t);
      return SIM_E_ARG;
    }
    double mu = E / (2.0 * (1.0 + nu));
    double lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
    S.model[t] = model;
    S.mu[t] = mu;
    S.lam[t] = lam;
    S.kstiff[t] = model == 0 ? 2.0 * mu : 2.0 * mu + lam;
    for (int a = 0; a < 4; ++a) S.mass[T[a]] += mat.rho * V / 4.0;
  }

  // ---- node-level system matrix A_n = M + h^2 sum_t w_t [d_a . d_b] (+ pins)
  {
    std::vector<std::vector<std::pair<int32_t, double>>> rows(n);
    for (int t = 0; t < m; ++t) {
      const int32_t* T = &S.tets[4 * (size_t)t];
      const double* Di = &S.Dm_inv[9 * (size_t)t];
      double d[4][3];
      for (int c = 0; c < 3; ++c) {
        d[1][c] = Di[c];
        d[2][c] = Di[3 + c];
        d[3][c] = Di[6 + c];
        d[0][c] = -(d[1][c] + d[2][c] + d[3][c]);
      }
      double s = h * h * S.kstiff[t] * S.vol[t];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
          rows[T[a]].push_back({T[b], s * (d[a][0] * d[b][0] + d[a][1] * d[b][1] + d[a][2] * d[b][2])});
    }
    S.a_ptr.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
      auto& r = rows[i];
      r.push_back({i, S.mass[i]});
      std::sort(r.begin(), r.end(), [](auto& a, auto& b) { return a.first < b.first; });
      int32_t last = -1;
      for (auto& e : r) {
        if (e.first == last) {
          S.a_val.back() += e.second;
        } else {
          S.a_idx.push_back(e.first);
          S.a_val.push_back(e.second);
          last = e.first;
        }
      }
      S.a_ptr[i + 1] = (int64_t)S.a_idx.size();
    }
  }
  // pins: h^2 w_pin = 1e3 * scale * [A_n]_vv before pins
  S.pin_nodes.assign(mesh.pin_nodes, mesh.pin_nodes + mesh.n_pins);
  S.pin_group.assign(mesh.pin_group, mesh.pin_group + mesh.n_pins);
  if (mesh.n_pins > 0 && !(pin_weight_scale > 0.0)) {
    err = "pin weight scale must be positive";
    return SIM_E_ARG;
  }
  {
    std::vector<char> pinned(n, 0);
    S.pin_h2w.resize(mesh.n_pins);
    for (int p = 0; p < mesh.n_pins; ++p) {
      int v = S.pin_nodes[p];
      if (v < 0 || v >= n || pinned[v] || S.pin_group[p] < 0) {
        err = "bad pin entry " + std::to_string(p);
        return SIM_E_ARG;
      }
      pinned[v] = 1;
    }
    for (int p = 0; p < mesh.n_pins; ++p) {
      int v = S.pin_nodes[p];
      for (int64_t q = S.a_ptr[v]; q < S.a_ptr[v + 1]; ++q)
        if (S.a_idx[q] == v) {
          S.pin_h2w[p] = 1e3 * pin_weight_scale * S.a_val[q];
          S.a_val[q] += S.pin_h2w[p];
        }
    }
  }

  // ---- ordering: nested dissection, then a postorder of the elimination tree
  std::vector<int32_t> nd_perm(n), nd_iperm;
  {
    ND nd(S.a_ptr, S.a_idx, S.rest.data(), n);
    std::vector<int32_t> all(n);
    std::iota(all.begin(), all.end(), 0);
    nd.run(all);
    nd_iperm = nd.out;
    for (int k = 0; k < n; ++k) nd_perm[nd_iperm[k]] = k;
  }
  // elimination tree of P A P^T (Liu's algorithm with path compression)
  std::vector<int32_t> par(n, -1), anc(n, -1);
  for (int i = 0; i < n; ++i) {
    int o = nd_iperm[i];
    for (int64_t p = S.a_ptr[o]; p < S.a_ptr[o + 1]; ++p) {
      int k = nd_perm[S.a_idx[p]];
      while (k != -1 && k < i) {
        int nx = anc[k];
        anc[k] = i;
        if (nx == -1) par[k] = i;
        k = nx;
      }
    }
  }
  // postorder (children visited in increasing index)
  std::vector<int32_t> post(n);
  {
    std::vector<int32_t> head(n, -1), next(n, -1);
    for (int j = n - 1; j >= 0; --j)
      if (par[j] != -1) {
        next[j] = head[par[j]];
        head[par[j]] = j;
      }
    int k = 0;
    std::vector<int32_t> stack;
    for (int r = 0; r < n; ++r) {
      if (par[r] != -1) continue;
      stack.push_back(r);
      while (!stack.empty()) {
        int p = stack.back();
        int c = head[p];
        if (c == -1) {
          stack.pop_back();
          post[p] = k++;
        } else {
          head[p] = next[c];
          stack.push_back(c);
        }
      }
    }
  }
  S.perm.resize(n);
  S.iperm.resize(n);
  for (int o = 0; o < n; ++o) {
    S.perm[o] = post[nd_perm[o]];
    S.iperm[S.perm[o]] = o;
  }
  S.parent.assign(n, -1);
  for (int i = 0; i < n; ++i)
    if (par[i] != -1) S.parent[post[i]] = post[par[i]];
  S.lo.resize(n);
  for (int i = 0; i < n; ++i) S.lo[i] = i;
  for (int i = 0; i < n; ++i)
    if (S.parent[i] != -1) S.lo[S.parent[i]] = std::min(S.lo[S.parent[i]], S.lo[i]);
  S.depth.assign(n, 0);
  for (int i = n - 1; i >= 0; --i)
    if (S.parent[i] != -1) S.depth[i] = S.depth[S.parent[i]] + 1;
  {
    std::vector<int32_t> nchild(n, 0);
    for (int i = 0; i < n; ++i)
      if (S.parent[i] != -1) nchild[S.parent[i]]++;
    S.chain_end.resize(n);
    for (int i = n - 1; i >= 0; --i)
      S.chain_end[i] = (i + 1 < n && S.parent[i] == i + 1 && nchild[i + 1] == 1) ? S.chain_end[i + 1] : i;
  }

  // ---- symbolic factorisation: struct(L_j) = lower(A_j) U children structs \ {j}
  std::vector<int64_t> Lp(n + 1, 0);
  std::vector<int32_t> Li;
  {
    std::vector<std::vector<int32_t>> cols(n);
    std::vector<int32_t> mark(n, -1);
    std::vector<int32_t> kids_head(n, -1), kids_next(n, -1);
    for (int j = n - 1; j >= 0; --j)
      if (S.parent[j] != -1) {
        kids_next[j] = kids_head[S.parent[j]];
        kids_head[S.parent[j]] = j;
      }
    for (int j = 0; j < n; ++j) {
      auto& cj = cols[j];
      mark[j] = j;
      int o = S.iperm[j];
      for (int64_t p = S.a_ptr[o]; p < S.a_ptr[o + 1]; ++p) {
        int i = S.perm[S.a_idx[p]];
        if (i > j && mark[i] != j) {
          mark[i] = j;
          cj.push_back(i);
        }
      }
      for (int c = kids_head[j]; c != -1; c = kids_next[c])
        for (int i : cols[c])
          if (i > j && mark[i] != j) {
            mark[i] = j;
            cj.push_back(i);
          }
      std::sort(cj.begin(), cj.end());
      Lp[j + 1] = Lp[j] + 1 + (int64_t)cj.size();
    }
    Li.resize(Lp[n]);
    for (int j = 0; j < n; ++j) {
      Li[Lp[j]] = j;
      std::copy(cols[j].begin(), cols[j].end(), Li.begin() + Lp[j] + 1);
      std::vector<int32_t>().swap(cols[j]);
    }
  }
  S.nnz_L = Lp[n];

  // ---- numeric left-looking Cholesky in float64
  std::vector<double> Lx(Lp[n], 0.0);
  {
    std::vector<double> x(n, 0.0);
    std::vector<int32_t> head(n, -1), nxt(n, -1);
    std::vector<int64_t> pos(n, 0);
    std::vector<int32_t> work;
    double minpiv = 1e300;
    for (int j = 0; j < n; ++j) {
      int o = S.iperm[j];
      for (int64_t p = S.a_ptr[o]; p < S.a_ptr[o + 1]; ++p) {
        int i = S.perm[S.a_idx[p]];
        if (i >= j) x[i] = S.a_val[p];
      }
      work.clear();
      for (int k = head[j]; k != -1; k = nxt[k]) work.push_back(k);
      head[j] = -1;
      for (int k : work) {
        int64_t pk = pos[k];
        double ljk = Lx[pk];
        int64_t end = Lp[k + 1];
        for (int64_t p = pk; p < end; ++p) x[Li[p]] -= Lx[p] * ljk;
        pos[k] = pk + 1;
        if (pk + 1 < end) {
          int r = Li[pk + 1];
          nxt[k] = head[r];
          head[r] = k;
        }
      }
      double d = x[j];
      if (!(d > 0.0) || !std::isfinite(d)) {
        err = "system matrix is not positive definite (pivot " + std::to_string(j) + ")";
        return SIM_E_NOT_SPD;
      }
      double ljj = std::sqrt(d);
      minpiv = std::min(minpiv, ljj);
      Lx[Lp[j]] = ljj;
      x[j] = 0.0;
      for (int64_t p = Lp[j] + 1; p < Lp[j + 1]; ++p) {
        Lx[p] = x[Li[p]] / ljj;
        x[Li[p]] = 0.0;
      }
      if (Lp[j] + 1 < Lp[j + 1]) {
        pos[j] = Lp[j] + 1;
        int r = Li[pos[j]];
        nxt[j] = head[r];
        head[r] = j;
      }
    }
    S.chol_min_pivot = minpiv;
  }

  // ---- S = L^-1, column by column along each ancestor path (Theorem 1)
  S.row_ptr.assign(n + 1, 0);
  S.row_lo4.resize(n);
  for (int i = 0; i < n; ++i) {
    int lo4 = S.lo[i] & ~3;
    int hi4 = (i & ~3) + 4;
    S.row_lo4[i] = lo4;
    S.row_ptr[i + 1] = S.row_ptr[i] + (hi4 - lo4);
  }
  S.col_ptr.assign(n + 1, 0);
  for (int j = 0; j < n; ++j) S.col_ptr[j + 1] = S.col_ptr[j] + S.depth[j] + 1;
  S.nnz_S = S.col_ptr[n];
  S.row_val.assign(S.row_ptr[n], 0.0f);
  S.col_val.assign(S.col_ptr[n], 0.0f);
  if (want_dense_S) S.S_dense64.assign((size_t)n * n, 0.0);
  parallel_for(n, 16, [&](int64_t b, int64_t e) {
    std::vector<double> acc(n, 0.0);
    for (int64_t j = b; j < e; ++j) {
      int64_t cofs = S.col_ptr[j];
      int idx = 0;
      for (int k = (int)j; k != -1; k = S.parent[k], ++idx) {
        double xk = ((k == j ? 1.0 : 0.0) - acc[k]) / Lx[Lp[k]];
        acc[k] = 0.0;
        S.col_val[cofs + idx] = (float)xk;
        S.row_val[S.row_ptr[k] + (j - S.row_lo4[k])] = (float)xk;
        if (want_dense_S) S.S_dense64[(size_t)k * n + j] = xk;
        for (int64_t p = Lp[k] + 1; p < Lp[k + 1]; ++p) acc[Li[p]] += Lx[p] * xk;
      }
    }
  });
  return SIM_OK;
}

}  // namespace lg
