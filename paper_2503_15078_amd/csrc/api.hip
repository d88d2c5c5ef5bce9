// C-ABI of the gfx950 solver: handle creation (precompute + upload), the frame and
// iteration drivers of Algorithm 4, state readback and the parity hooks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <array>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "device.hpp"
#include "precompute.hpp"
#include "status.hpp"

namespace lg {
MeshIn mesh_in(const sim_mesh* m);
MaterialIn material_in(const sim_material* m);
}  // namespace lg

namespace {

constexpr int kSegFloats = 2048;  // S-pass segment length (floats) per wavefront

#define HIPCHK(x)                                                                        \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess) {                                                              \
      lg::set_error(std::string("HIP error: ") + hipGetErrorString(e_) + " at " #x);     \
      return SIM_E_DEVICE;                                                               \
    }                                                                                    \
  } while (0)

struct SceneMeta {
  int n = 0, m = 0;
  int node0 = 0;          // first internal node of the scene
  int caller0 = 0;        // first caller-order node of the scene (batch concatenation)
  int groups0 = 0;        // first global pin group
  int n_groups = 0;
  std::vector<int32_t> perm;  // local caller -> local internal
  double margin = 0.0;
};

}  // namespace

struct lgsim {
  sim_options opt{};
  lg::Dev d{};
  hipStream_t st = nullptr;
  bool own_stream = false;
  // side stream of the frame set-up: the Delassus operator and the warm start run there
  // while the first iteration's local step and S pass run on st (default priority)
  hipStream_t st2 = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  bool setup_forked = false;
  std::vector<void*> allocs;
  std::vector<SceneMeta> scenes;
  std::vector<int32_t> iperm_caller;  // internal node -> caller node (global)
  std::vector<int32_t> perm_caller;   // caller node -> internal node (global)
  std::vector<int32_t> surf_tris;     // [T][3] surface triangles (caller ids) of self contact
  std::vector<lg::ObstacleDev> obst;  // host copy
  std::vector<int> scene_obst0;
  int cr_blocks = 1;
  int* h_pinned = nullptr;            // [8]: n_contacts, overflow, bad[2], convergence flag and count
  int* d_conv = nullptr;              // [2] device convergence flag and iteration count
  hipGraphExec_t cexec = nullptr;     // chunk of iterations of a frame iterated to tolerance
  std::vector<unsigned char> ckey;
  float* h_res = nullptr;             // [NS]
  int iter_c = 0;                     // contact count of the current iterate state
  bool has_model = false;             // learned warm-start parameters uploaded
  bool record_pairs = false;          // compute contact features every frame
  float* d_tgt = nullptr;             // [CMAX][3] scratch of sim_read_training_pairs
  float* d_lam_save = nullptr;        // [3][CMAX] impulses kept across sim_profile_cr
  unsigned long long* d_clock = nullptr;  // wall-clock stamps of sim_profile_cr
  std::vector<unsigned long long> cr_stamps;  // the last stamped launch's stamps, as read back
  unsigned* d_prof_sync = nullptr;    // [SIM_PROFILE_MAX_REPS][kCrSyncWords] CR barrier flags of its launches
  std::vector<int32_t> iter_canon;    // internal contact index -> canonical position
  hipEvent_t ev[8] = {};
  std::vector<hipEvent_t> fev;        // per-frame timing events
  // S-pass segmentation (host copies of the row layout, current segment length)
  std::vector<int64_t> h_row_ptr;
  std::vector<int32_t> h_row_lo4;
  std::vector<int32_t> h_chain_end;
  double* energy_part = nullptr;  // per-block partial sums of sim_lg_energy
  int seg_floats = 0;
  // captured fixed-iteration frame
  hipGraphExec_t gexec = nullptr;
  std::vector<unsigned char> gkey;
  struct Snapshot {
    float *qt = nullptr, *vt = nullptr, *pc_world = nullptr;
    double* t = nullptr;
    int *pc_count = nullptr, *pc_node = nullptr, *pc_obst = nullptr;
  } snap;

  template <class T>
  int alloc(T*& p, size_t count) {
    void* q = nullptr;
    size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;  // never while capturing
    if (st && (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone)) {
      lg::set_error("device allocation during stream capture");
      return SIM_E_STATE;
    }
    if (hipMalloc(&q, bytes) != hipSuccess) {
      lg::set_error("hipMalloc failed (" + std::to_string(bytes) + " bytes)");
      return SIM_E_NOMEM;
    }
    // Zero on the handle's own stream and wait for it: the stream is non-blocking, so a
    // fill on the null stream would be unordered with the uploads that follow on it and
    // could land after them.
    if ((st ? hipMemsetAsync(q, 0, bytes, st) : hipMemset(q, 0, bytes)) != hipSuccess ||
        (st ? hipStreamSynchronize(st) : hipDeviceSynchronize()) != hipSuccess) {
      hipFree(q);
      lg::set_error("hipMemset failed");
      return SIM_E_DEVICE;
    }
    allocs.push_back(q);
    p = static_cast<T*>(q);
    return SIM_OK;
  }
  // release one tracked allocation (nullptr is ignored)
  void release(void* p) {
    if (!p) return;
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i] == p) {
        hipFree(p);
        allocs.erase(allocs.begin() + (long)i);
        return;
      }
  }
  ~lgsim() {
    if (st) hipStreamSynchronize(st);
    if (st2) {
      hipStreamSynchronize(st2);
      hipStreamDestroy(st2);
    }
    if (fork_ev) hipEventDestroy(fork_ev);
    if (join_ev) hipEventDestroy(join_ev);
    if (gexec) hipGraphExecDestroy(gexec);
    if (cexec) hipGraphExecDestroy(cexec);
    for (void* p : allocs) hipFree(p);
    for (auto& e : ev)
      if (e) hipEventDestroy(e);
    for (auto& e : fev) hipEventDestroy(e);
    if (h_pinned) hipHostFree(h_pinned);
    if (h_res) hipHostFree(h_res);
    if (own_stream && st) hipStreamDestroy(st);
  }
};

namespace {

template <class T>
int upload(lgsim* s, T* dst, const T* src, size_t count) {
  if (count == 0) return SIM_OK;
  HIPCHK(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  return SIM_OK;
}

#define TRY(x)                 \
  do {                         \
    int rc_ = (x);             \
    if (rc_ != SIM_OK) return rc_; \
  } while (0)

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    lg::set_error(std::string("kernel launch failed (") + what + "): " + hipGetErrorString(e));
    return SIM_E_DEVICE;
  }
  return SIM_OK;
}

// Upload obstacles of all scenes.
int push_obstacles(lgsim* s) {
  auto& d = s->d;
  if (!s->obst.empty()) TRY(upload(s, d.obst, s->obst.data(), s->obst.size()));
  TRY(upload(s, d.scene_obst0, s->scene_obst0.data(), s->scene_obst0.size()));
  return SIM_OK;
}

// Column groups of the S^T pass: up to col_group consecutive columns of one chain share
// every run of the first column's path except the start of the first run.
int build_col_groups(lgsim* s, int col_group) {
  auto& d = s->d;
  const int N = d.N;
  std::vector<int> j0s, ngs;
  for (int j = 0; j < N;) {
    int ng = 1;
    while (ng < col_group && j + ng < N && s->h_chain_end[j + ng] == s->h_chain_end[j]) ++ng;
    j0s.push_back(j);
    ngs.push_back(ng);
    j += ng;
  }
  HIPCHK(hipStreamSynchronize(s->st));
  s->release(d.stgrp_j0);
  s->release(d.stgrp_ng);
  d.n_stgrp = (int)j0s.size();
  d.col_group = col_group;
  TRY(s->alloc(d.stgrp_j0, j0s.size()));
  TRY(s->alloc(d.stgrp_ng, ngs.size()));
  TRY(upload(s, d.stgrp_j0, j0s.data(), j0s.size()));
  TRY(upload(s, d.stgrp_ng, ngs.data(), ngs.size()));
  HIPCHK(hipStreamSynchronize(s->st));
  return SIM_OK;
}

// Segments of the S pass: consecutive rows stored from the same column quad (at most
// row_group) form a group whose union range [lo4, hi4 of its last row) is cut into
// pieces of at most seg_floats columns, one wavefront each, so each piece of b is loaded
// once for the group; groups of several pieces add their partial sums in a second
// kernel.  Re-run with another length by the autotuner.
int build_segments(lgsim* s, int seg_floats, int row_group) {
  auto& d = s->d;
  const int N = d.N;
  std::vector<int> seg_row, seg_ng, seg_q0, seg_len, seg_col0, long_row, long_seg0, long_nseg, long_ng;
  std::vector<int64_t> seg_off;
  for (int i = 0; i < N;) {
    int ng = 1;
    while (ng < row_group && i + ng < N && s->h_row_lo4[i + ng] == s->h_row_lo4[i]) ++ng;
    // the last row of the group ends last (rows end at their own quad)
    const int64_t len = s->h_row_ptr[i + ng] - s->h_row_ptr[i + ng - 1];
    const int nseg = (int)((len + seg_floats - 1) / seg_floats);
    if (nseg > 1) {
      long_row.push_back(i);
      long_seg0.push_back((int)seg_row.size());
      long_nseg.push_back(nseg);
      long_ng.push_back(ng);
    }
    for (int q = 0; q < nseg; ++q) {
      const int64_t st = (int64_t)q * seg_floats;
      seg_row.push_back(nseg > 1 ? -(i + 1) : i);
      seg_ng.push_back(ng);
      seg_q0.push_back((int)(st / 4));
      seg_off.push_back(s->h_row_ptr[i] + st);
      seg_col0.push_back(s->h_row_lo4[i] + (int)st);
      seg_len.push_back((int)std::min<int64_t>(seg_floats, len - st));
    }
    i += ng;
  }
  HIPCHK(hipStreamSynchronize(s->st));
  for (void* p : {(void*)d.seg_row, (void*)d.seg_ng, (void*)d.seg_q0, (void*)d.seg_len, (void*)d.seg_col0,
                  (void*)d.seg_off, (void*)d.long_row,
                  (void*)d.long_seg0, (void*)d.long_nseg, (void*)d.long_ng, (void*)d.partial})
    s->release(p);
  d.nseg = (int)seg_row.size();
  d.nlong = (int)long_row.size();
  TRY(s->alloc(d.seg_row, d.nseg));
  TRY(s->alloc(d.seg_ng, d.nseg));
  TRY(s->alloc(d.seg_q0, d.nseg));
  TRY(s->alloc(d.seg_len, d.nseg));
  TRY(s->alloc(d.seg_col0, d.nseg));
  TRY(s->alloc(d.seg_off, d.nseg));
  TRY(s->alloc(d.long_row, d.nlong));
  TRY(s->alloc(d.long_seg0, d.nlong));
  TRY(s->alloc(d.long_nseg, d.nlong));
  TRY(s->alloc(d.long_ng, d.nlong));
  d.row_group = row_group;
  TRY(s->alloc(d.partial, 3 * (size_t)row_group * d.nseg));
  TRY(upload(s, d.seg_row, seg_row.data(), seg_row.size()));
  TRY(upload(s, d.seg_ng, seg_ng.data(), seg_ng.size()));
  TRY(upload(s, d.seg_q0, seg_q0.data(), seg_q0.size()));
  TRY(upload(s, d.seg_len, seg_len.data(), seg_len.size()));
  TRY(upload(s, d.seg_col0, seg_col0.data(), seg_col0.size()));
  TRY(upload(s, d.seg_off, seg_off.data(), seg_off.size()));
  TRY(upload(s, d.long_row, long_row.data(), long_row.size()));
  TRY(upload(s, d.long_seg0, long_seg0.data(), long_seg0.size()));
  TRY(upload(s, d.long_nseg, long_nseg.data(), long_nseg.size()));
  TRY(upload(s, d.long_ng, long_ng.data(), long_ng.size()));
  HIPCHK(hipStreamSynchronize(s->st));
  s->seg_floats = seg_floats;
  return SIM_OK;
}

int obstacle_dev(lgsim* s, int k, const sim_obstacle& o, lg::ObstacleDev& od);

// Build one handle from host precomputations of several scenes (concatenated).
// Boundary triangles of a tet mesh (caller ids): the faces that belong to exactly one
// tet, oriented with the normal pointing away from the tet's fourth vertex, sorted by
// their sorted corner triple.
std::vector<int32_t> surface_triangles(const lg::HostScene& h) {
  static const int faces[4][4] = {{1, 2, 3, 0}, {0, 3, 2, 1}, {0, 1, 3, 2}, {0, 2, 1, 3}};
  std::map<std::array<int32_t, 3>, std::pair<int, std::array<int32_t, 3>>> seen;
  const double* X = h.rest.data();
  for (int t = 0; t < h.m; ++t) {
    const int32_t* tv = &h.tets[4 * (size_t)t];
    for (const auto& f : faces) {
      std::array<int32_t, 3> tri = {tv[f[0]], tv[f[1]], tv[f[2]]};
      const int32_t o = tv[f[3]];
      double e1[3], e2[3], r[3];
      for (int c = 0; c < 3; ++c) {
        e1[c] = X[3 * tri[1] + c] - X[3 * tri[0] + c];
        e2[c] = X[3 * tri[2] + c] - X[3 * tri[0] + c];
        r[c] = X[3 * o + c] - X[3 * tri[0] + c];
      }
      const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                            e1[0] * e2[1] - e1[1] * e2[0]};
      if (cr[0] * r[0] + cr[1] * r[1] + cr[2] * r[2] > 0.0) std::swap(tri[1], tri[2]);
      std::array<int32_t, 3> key = tri;
      std::sort(key.begin(), key.end());
      auto& e = seen[key];
      e.first += 1;
      e.second = tri;
    }
  }
  std::vector<int32_t> out;
  for (const auto& kv : seen)
    if (kv.second.first == 1) out.insert(out.end(), kv.second.second.begin(), kv.second.second.end());
  return out;
}

// Device tables of self contact: triangles and surface vertices in internal numbering,
// each vertex's incident triangles (ascending), and the per-frame buffers.
int build_self_contact(lgsim* s, const lg::HostScene& h) {
  auto& d = s->d;
  s->surf_tris = surface_triangles(h);
  const int T = (int)(s->surf_tris.size() / 3);
  std::vector<int32_t> verts(s->surf_tris);
  std::sort(verts.begin(), verts.end());
  verts.erase(std::unique(verts.begin(), verts.end()), verts.end());
  const int NSV = (int)verts.size();
  std::vector<int> tri_v(3 * (size_t)std::max(T, 1), 0), sv(std::max(NSV, 1), 0), vt_ptr(NSV + 1, 0), vt_idx;
  std::vector<int> slot(h.n, -1);
  for (int i = 0; i < NSV; ++i) {
    slot[verts[i]] = i;
    sv[i] = s->perm_caller[verts[i]];
  }
  std::vector<std::vector<int>> inc(NSV);
  for (int t = 0; t < T; ++t)
    for (int a = 0; a < 3; ++a) {
      const int cv = s->surf_tris[3 * (size_t)t + a];
      tri_v[a * (size_t)T + t] = s->perm_caller[cv];
      inc[slot[cv]].push_back(t);
    }
  for (int i = 0; i < NSV; ++i) {
    vt_ptr[i + 1] = vt_ptr[i] + (int)inc[i].size();
    vt_idx.insert(vt_idx.end(), inc[i].begin(), inc[i].end());
  }
  if (vt_idx.empty()) vt_idx.push_back(0);
  d.self_on = 1;
  d.T = T;
  d.NSV = NSV;
  d.self_mu = (float)s->opt.self_mu;
  const size_t CM = d.CMAX;
  TRY(s->alloc(d.tri_v, tri_v.size()));
  TRY(s->alloc(d.sv, sv.size()));
  TRY(s->alloc(d.vt_ptr, vt_ptr.size()));
  TRY(s->alloc(d.vt_idx, vt_idx.size()));
  TRY(s->alloc(d.tri_n, 6 * (size_t)std::max(T, 1)));
  TRY(s->alloc(d.sv_cnt, std::max(NSV, 1)));
  TRY(s->alloc(d.n_obst_c, 1));
  TRY(s->alloc(d.ent_node, 4 * CM));
  TRY(s->alloc(d.ent_w, 4 * CM));
  TRY(s->alloc(d.se_node, 4 * CM));
  TRY(s->alloc(d.se_row, 4 * CM));
  TRY(s->alloc(d.se_w, 4 * CM));
  TRY(s->alloc(d.se_count, 1));
  TRY(s->alloc(d.frange2, 2 * (size_t)d.N));
  TRY(upload(s, d.tri_v, tri_v.data(), tri_v.size()));
  TRY(upload(s, d.sv, sv.data(), sv.size()));
  TRY(upload(s, d.vt_ptr, vt_ptr.data(), vt_ptr.size()));
  TRY(upload(s, d.vt_idx, vt_idx.data(), vt_idx.size()));
  return SIM_OK;
}

int build(lgsim* s, std::vector<lg::HostScene>& hs, const std::vector<std::vector<sim_obstacle>>& obs) {
  auto& d = s->d;
  const int NS = (int)hs.size();
  int N = 0, M = 0, P = 0, G = 0;
  s->scenes.resize(NS);
  for (int k = 0; k < NS; ++k) {
    auto& sm = s->scenes[k];
    sm.n = hs[k].n;
    sm.m = hs[k].m;
    sm.node0 = N;
    sm.caller0 = N;
    sm.perm = hs[k].perm;
    sm.margin = s->opt.contact_margin;
    sm.groups0 = G;
    int ng = 0;
    for (int g : hs[k].pin_group) ng = std::max(ng, g + 1);
    sm.n_groups = ng;
    N += hs[k].n;
    M += hs[k].m;
    P += (int)hs[k].pin_nodes.size();
    G += ng;
  }
  d.N = N;
  d.N4 = ((N + 3) & ~3) + 4;
  d.M = M;
  d.P = P;
  d.G = std::max(G, 1);
  d.NS = NS;
  d.CMAX = std::max(1, s->opt.max_contacts);
  d.KCAP = std::min<int64_t>((int64_t)d.CMAX * lg::kstride(d.CMAX), (int64_t)64 << 20);
  d.h = hs[0].h;
  for (int c = 0; c < 3; ++c) d.g[c] = s->opt.gravity[c];
  d.cr_iters = s->opt.cr_iters;
  d.cr_tol = (float)s->opt.cr_tol;
  d.warm = s->opt.warm;
  d.ncp = s->opt.ncp;
  d.precond = s->opt.precond;
  d.global_step = s->opt.global_step;
  d.lg_form = s->opt.lg_form;
  d.elem_block = lg::kBlock;
  s->perm_caller.resize(N);
  s->iperm_caller.resize(N);
  for (int k = 0; k < NS; ++k)
    for (int o = 0; o < hs[k].n; ++o) {
      int gi = s->scenes[k].node0 + hs[k].perm[o];
      s->perm_caller[s->scenes[k].caller0 + o] = gi;
      s->iperm_caller[gi] = s->scenes[k].caller0 + o;
    }

  // ---- node arrays
  const int N4 = d.N4;
  std::vector<float> qt(3 * (size_t)N4, 0.0f), vt(3 * (size_t)N4, 0.0f), pinw(N, 0.0f), inv_mass(N, 0.0f);
  std::vector<int> node_scene(N, 0);
  for (int k = 0; k < NS; ++k)
    for (int o = 0; o < hs[k].n; ++o) {
      int gi = s->scenes[k].node0 + hs[k].perm[o];
      node_scene[gi] = k;
      inv_mass[gi] = (float)(1.0 / hs[k].mass[o]);
      for (int c = 0; c < 3; ++c) {
        qt[c * (size_t)N4 + gi] = (float)hs[k].init[3 * (size_t)o + c];
        vt[c * (size_t)N4 + gi] = (float)hs[k].vel[3 * (size_t)o + c];
      }
    }
  // pins
  std::vector<int> pin_node(P), pin_group(P);
  std::vector<double> pin_x0(3 * (size_t)std::max(P, 1));
  {
    int p = 0;
    for (int k = 0; k < NS; ++k)
      for (size_t q = 0; q < hs[k].pin_nodes.size(); ++q, ++p) {
        int o = hs[k].pin_nodes[q];
        int gi = s->scenes[k].node0 + hs[k].perm[o];
        pin_node[p] = gi;
        pin_group[p] = s->scenes[k].groups0 + hs[k].pin_group[q];
        pinw[gi] = (float)hs[k].pin_h2w[q];
        for (int c = 0; c < 3; ++c) pin_x0[c * (size_t)P + p] = (double)(float)hs[k].init[3 * (size_t)o + c];
      }
  }
  // tets: internal node indices, sorted per scene by smallest node for locality
  std::vector<int> tidx(4 * (size_t)M);
  std::vector<float> dinv(9 * (size_t)M), hw(M), tmu(M), tlam(M), tk(M);
  std::vector<unsigned char> tmodel(M);
  {
    int t0 = 0;
    for (int k = 0; k < NS; ++k) {
      auto& H = hs[k];
      std::vector<int> order(H.m);
      std::iota(order.begin(), order.end(), 0);
      auto key = [&](int t) {
        int mn = 1 << 30;
        for (int a = 0; a < 4; ++a) mn = std::min(mn, H.perm[H.tets[4 * (size_t)t + a]]);
        return mn;
      };
      std::vector<int> keys(H.m);
      for (int t = 0; t < H.m; ++t) keys[t] = key(t);
      std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return keys[a] < keys[b]; });
      for (int q = 0; q < H.m; ++q) {
        int t = order[q], gt = t0 + q;
        for (int a = 0; a < 4; ++a) tidx[a * (size_t)M + gt] = s->scenes[k].node0 + H.perm[H.tets[4 * (size_t)t + a]];
        for (int e = 0; e < 9; ++e) dinv[e * (size_t)M + gt] = (float)H.Dm_inv[9 * (size_t)t + e];
        hw[gt] = (float)(H.h * H.h * H.kstiff[t] * H.vol[t]);
        tmu[gt] = (float)H.mu[t];
        tlam[gt] = (float)H.lam[t];
        tk[gt] = (float)H.kstiff[t];
        tmodel[gt] = (unsigned char)H.model[t];
      }
      t0 += H.m;
    }
  }
  // node -> (corner, tet) gather lists in increasing (tet, corner) order
  std::vector<int> g_ptr(N + 1, 0), g_slot(4 * (size_t)M);
  for (int t = 0; t < M; ++t)
    for (int a = 0; a < 4; ++a) g_ptr[tidx[a * (size_t)M + t] + 1]++;
  for (int v = 0; v < N; ++v) g_ptr[v + 1] += g_ptr[v];
  {
    std::vector<int> fill(g_ptr.begin(), g_ptr.end() - 1);
    for (int t = 0; t < M; ++t)
      for (int a = 0; a < 4; ++a) g_slot[fill[tidx[a * (size_t)M + t]]++] = 3 * a * M + t;  // fc offset of corner a
  }
  // S: row storage re-padded on global 4-aligned columns, column storage concatenated
  std::vector<int64_t> row_ptr(N + 1, 0), col_ptr(N + 1, 0);
  std::vector<int> row_lo4(N), parent(N), lo(N), depth(N), chain_end(N);
  for (int k = 0; k < NS; ++k) {
    int n0 = s->scenes[k].node0;
    for (int i = 0; i < hs[k].n; ++i) {
      int gi = n0 + i;
      int lo4 = (n0 + hs[k].lo[i]) & ~3;
      int hi4 = (gi & ~3) + 4;
      row_lo4[gi] = lo4;
      row_ptr[gi + 1] = hi4 - lo4;
      col_ptr[gi + 1] = hs[k].col_ptr[i + 1] - hs[k].col_ptr[i];
      parent[gi] = hs[k].parent[i] < 0 ? -1 : n0 + hs[k].parent[i];
      lo[gi] = n0 + hs[k].lo[i];
      depth[gi] = hs[k].depth[i];
      chain_end[gi] = n0 + hs[k].chain_end[i];
    }
  }
  for (int v = 0; v < N; ++v) {
    row_ptr[v + 1] += row_ptr[v];
    col_ptr[v + 1] += col_ptr[v];
  }
  s->h_row_ptr = row_ptr;
  s->h_row_lo4 = row_lo4;

  // ---- allocate
  const size_t NV = 3 * (size_t)N4;
  const int CM = d.CMAX;
  TRY(s->alloc(d.qt, NV));
  TRY(s->alloc(d.vt, NV));
  TRY(s->alloc(d.qp, NV));
  TRY(s->alloc(d.q, NV));
  TRY(s->alloc(d.b, NV));
  TRY(s->alloc(d.y, NV));
  TRY(s->alloc(d.tgt, NV));
  TRY(s->alloc(d.tmp, NV));
  TRY(s->alloc(d.iperm_caller, N));
  TRY(s->alloc(d.pin_w, N));
  TRY(s->alloc(d.inv_mass, N));
  {
    // A_n in internal order (CSR) for the Jacobi global step
    std::vector<int> ap(N + 1, 0), ai;
    std::vector<float> av, adinv(N, 0.0f);
    for (int k = 0; k < NS; ++k)
      for (int o = 0; o < hs[k].n; ++o) ap[s->scenes[k].node0 + hs[k].perm[o] + 1] = (int)(hs[k].a_ptr[o + 1] - hs[k].a_ptr[o]);
    for (int v = 0; v < N; ++v) ap[v + 1] += ap[v];
    ai.resize(ap[N]);
    av.resize(ap[N]);
    for (int k = 0; k < NS; ++k)
      for (int o = 0; o < hs[k].n; ++o) {
        const int gi = s->scenes[k].node0 + hs[k].perm[o];
        int w = ap[gi];
        for (int64_t p = hs[k].a_ptr[o]; p < hs[k].a_ptr[o + 1]; ++p, ++w) {
          const int gj = s->scenes[k].node0 + hs[k].perm[hs[k].a_idx[p]];
          ai[w] = gj;
          av[w] = (float)hs[k].a_val[p];
          if (gj == gi) adinv[gi] = (float)(1.0 / hs[k].a_val[p]);
        }
      }
    TRY(s->alloc(d.a_ptr, N + 1));
    TRY(s->alloc(d.a_idx, ai.size()));
    TRY(s->alloc(d.a_val, av.size()));
    TRY(s->alloc(d.a_dinv, N));
    TRY(upload(s, d.a_ptr, ap.data(), ap.size()));
    TRY(upload(s, d.a_idx, ai.data(), ai.size()));
    TRY(upload(s, d.a_val, av.data(), av.size()));
    TRY(upload(s, d.a_dinv, adinv.data(), adinv.size()));
  }
  TRY(s->alloc(d.node_scene, N));
  TRY(s->alloc(d.g_ptr, N + 1));
  TRY(s->alloc(d.g_slot, 4 * (size_t)M));
  TRY(s->alloc(d.pin_node, P));
  TRY(s->alloc(d.pin_group, P));
  TRY(s->alloc(d.pin_x0, 3 * (size_t)std::max(P, 1)));
  TRY(s->alloc(d.grp, 9 * (size_t)d.G));
  TRY(s->alloc(d.tidx, 4 * (size_t)M));
  TRY(s->alloc(d.dinv, 9 * (size_t)M));
  TRY(s->alloc(d.hw, M));
  TRY(s->alloc(d.tmu, M));
  TRY(s->alloc(d.tlam, M));
  TRY(s->alloc(d.tk, M));
  TRY(s->alloc(d.tmodel, M));
  TRY(s->alloc(d.fc, 12 * (size_t)M));
  TRY(s->alloc(d.dual, s->opt.lg_form == SIM_LG_ADMM ? 9 * (size_t)M : 1));
  TRY(s->alloc(d.row_ptr, N + 1));
  TRY(s->alloc(d.row_lo4, N));
  TRY(s->alloc(d.row_val, (size_t)row_ptr[N]));

  TRY(s->alloc(d.col_ptr, N + 1));
  TRY(s->alloc(d.col_val, (size_t)col_ptr[N]));
  TRY(s->alloc(d.parent, N));
  TRY(s->alloc(d.lo, N));
  TRY(s->alloc(d.depth, N));
  TRY(s->alloc(d.chain_end, N));
  TRY(s->alloc(d.frange, 2 * (size_t)N));
  TRY(s->alloc(d.scene_node0, NS + 1));
  TRY(s->alloc(d.scene_obst0, NS + 1));
  TRY(s->alloc(d.scene_margin, NS));
  TRY(s->alloc(d.ell, NS));
  TRY(s->alloc(d.c_feat, 16 * (size_t)d.CMAX));
  TRY(s->alloc(d.c_comp, d.CMAX));
  TRY(s->alloc(d.mlp_P, lg::kMlpParams));
  TRY(s->alloc(s->d_tgt, 3 * (size_t)d.CMAX));
  TRY(s->alloc(d.obst, (size_t)lg::kMaxObstacles * NS));
  TRY(s->alloc(d.n_contacts, 4));
  TRY(s->alloc(d.overflow, 4));
  TRY(s->alloc(d.cnt, N));
  TRY(s->alloc(d.blk, (N + lg::kBlock - 1) / lg::kBlock + 1));
  TRY(s->alloc(d.c_node, CM));
  TRY(s->alloc(d.c_obst, CM));
  TRY(s->alloc(d.c_scene, CM));
  TRY(s->alloc(d.cC, 9 * (size_t)CM));
  TRY(s->alloc(d.cC64, 9 * (size_t)CM));
  TRY(s->alloc(d.c_dn64, CM));
  TRY(s->alloc(d.c_dn, CM));
  TRY(s->alloc(d.c_df, 2 * (size_t)CM));
  TRY(s->alloc(d.c_mu, CM));
  TRY(s->alloc(d.c_rn, CM));
  TRY(s->alloc(d.c_rf, CM));
  TRY(s->alloc(d.c_gap, CM));
  TRY(s->alloc(d.lam, 3 * (size_t)CM));
  TRY(s->alloc(d.lam_ml, 3 * (size_t)CM));
  TRY(s->alloc(d.wl, 6 * (size_t)CM));
  TRY(s->alloc(d.judge, 2 * (size_t)NS));
  TRY(s->alloc(d.cs_off, NS + 1));
  TRY(s->alloc(d.k_off, NS + 1));
  TRY(s->alloc(d.tile_off, NS + 1));
  TRY(s->alloc(d.K, (size_t)d.KCAP));
  TRY(s->alloc(d.ad, CM));
  TRY(s->alloc(d.pc_count, 4));
  TRY(s->alloc(d.pc_node, CM));
  TRY(s->alloc(d.pc_obst, CM));
  TRY(s->alloc(d.pc_world, 3 * (size_t)CM));
  for (float** p : {&d.Om, &d.Et, &d.hv, &d.X, &d.F})
    TRY(s->alloc(*p, 3 * (size_t)CM));
  // two exchange buffers alternating per barrier, each with up to two 3-vectors
  TRY(s->alloc(d.cr_Z, 2 * 2 * 3 * (size_t)CM));
  TRY(s->alloc(d.cr_prod, (size_t)lg::cr_partial_floats(lg::kCrMaxBlocks, std::max(1, NS))));
  TRY(s->alloc(d.cr_sync, lg::kCrSyncWords));
  TRY(s->alloc(d.t, 1));
  TRY(s->alloc(d.res, NS));
  TRY(s->alloc(d.bad, 4));
  TRY(s->alloc(s->d_conv, 2));

  // ---- upload constants
  std::vector<float> row_val((size_t)row_ptr[N], 0.0f), col_val((size_t)col_ptr[N]);
  for (int k = 0; k < NS; ++k) {
    int n0 = s->scenes[k].node0;
    auto& H = hs[k];
    for (int i = 0; i < H.n; ++i) {
      int gi = n0 + i;
      // true entries are columns [lo_i, i] (local)
      for (int j = H.lo[i]; j <= i; ++j)
        row_val[row_ptr[gi] + (n0 + j - row_lo4[gi])] = H.row_val[H.row_ptr[i] + (j - H.row_lo4[i])];
    }
    std::copy(H.col_val.begin(), H.col_val.end(), col_val.begin() + col_ptr[n0]);
    // release host S copies of this scene
    std::vector<float>().swap(H.row_val);
    std::vector<float>().swap(H.col_val);
  }
  std::vector<int> scene_node0(NS + 1);
  std::vector<double> margins(NS);
  for (int k = 0; k < NS; ++k) {
    scene_node0[k] = s->scenes[k].node0;
    margins[k] = s->scenes[k].margin;
  }
  scene_node0[NS] = N;
  TRY(upload(s, d.qt, qt.data(), qt.size()));
  TRY(upload(s, d.vt, vt.data(), vt.size()));
  TRY(upload(s, d.pin_w, pinw.data(), pinw.size()));
  TRY(upload(s, d.inv_mass, inv_mass.data(), inv_mass.size()));
  TRY(upload(s, d.node_scene, node_scene.data(), node_scene.size()));
  TRY(upload(s, d.iperm_caller, s->iperm_caller.data(), s->iperm_caller.size()));
  TRY(upload(s, d.g_ptr, g_ptr.data(), g_ptr.size()));
  TRY(upload(s, d.g_slot, g_slot.data(), g_slot.size()));
  TRY(upload(s, d.pin_node, pin_node.data(), pin_node.size()));
  TRY(upload(s, d.pin_group, pin_group.data(), pin_group.size()));
  TRY(upload(s, d.pin_x0, pin_x0.data(), pin_x0.size()));
  TRY(upload(s, d.tidx, tidx.data(), tidx.size()));
  TRY(upload(s, d.dinv, dinv.data(), dinv.size()));
  TRY(upload(s, d.hw, hw.data(), hw.size()));
  TRY(upload(s, d.tmu, tmu.data(), tmu.size()));
  TRY(upload(s, d.tlam, tlam.data(), tlam.size()));
  TRY(upload(s, d.tk, tk.data(), tk.size()));
  TRY(upload(s, d.tmodel, tmodel.data(), tmodel.size()));
  TRY(upload(s, d.row_ptr, row_ptr.data(), row_ptr.size()));
  TRY(upload(s, d.row_lo4, row_lo4.data(), row_lo4.size()));
  TRY(upload(s, d.row_val, row_val.data(), row_val.size()));
  TRY(build_segments(s, kSegFloats, 4));
  TRY(upload(s, d.col_ptr, col_ptr.data(), col_ptr.size()));
  TRY(upload(s, d.col_val, col_val.data(), col_val.size()));
  {
    // S^T-pass copy of the columns: each chain run [a, e] of a column's ancestor path is
    // stored from a multiple-of-4 position as the entries of nodes (a & ~3) .. (e | 3),
    // zero outside [a, e], so the pass reads S values and y as aligned float4
    std::vector<int64_t> colp_ptr(N + 1, 0);
    for (int j = 0; j < N; ++j) {
      int64_t tot = 0;
      for (int a = j; a != -1;) {
        const int e = chain_end[a];
        tot += (int64_t)((e | 3) + 1 - (a & ~3));
        a = parent[e];
      }
      colp_ptr[j + 1] = colp_ptr[j] + tot;
    }
    std::vector<float> colp_val((size_t)colp_ptr[N], 0.0f);
    for (int j = 0; j < N; ++j) {
      int64_t t = col_ptr[j], p = colp_ptr[j];
      for (int a = j; a != -1;) {
        const int e = chain_end[a], a4 = a & ~3;
        for (int k = a; k <= e; ++k) colp_val[(size_t)(p + (k - a4))] = col_val[(size_t)(t + (k - a))];
        t += e - a + 1;
        p += (e | 3) + 1 - a4;
        a = parent[e];
      }
    }
    // the runs of every column, so the pass issues its loads without walking the tree
    std::vector<int> run_ptr(N + 1, 0), run_a, run_e;
    for (int j = 0; j < N; ++j) {
      for (int a = j; a != -1;) {
        const int e = chain_end[a];
        run_a.push_back(a);
        run_e.push_back(e);
        a = parent[e];
      }
      run_ptr[j + 1] = (int)run_a.size();
    }
    s->h_chain_end = chain_end;
    TRY(build_col_groups(s, 4));
    TRY(s->alloc(d.run_ptr, N + 1));
    TRY(s->alloc(d.run_a, run_a.size()));
    TRY(s->alloc(d.run_e, run_e.size()));
    TRY(upload(s, d.run_ptr, run_ptr.data(), run_ptr.size()));
    TRY(upload(s, d.run_a, run_a.data(), run_a.size()));
    TRY(upload(s, d.run_e, run_e.data(), run_e.size()));
    TRY(s->alloc(d.colp_ptr, N + 1));
    TRY(s->alloc(d.colp_val, (size_t)colp_ptr[N]));
    TRY(upload(s, d.colp_ptr, colp_ptr.data(), colp_ptr.size()));
    TRY(upload(s, d.colp_val, colp_val.data(), colp_val.size()));
  }
  TRY(upload(s, d.parent, parent.data(), parent.size()));
  TRY(upload(s, d.lo, lo.data(), lo.size()));
  TRY(upload(s, d.depth, depth.data(), depth.size()));
  TRY(upload(s, d.chain_end, chain_end.data(), chain_end.size()));
  TRY(upload(s, d.scene_node0, scene_node0.data(), scene_node0.size()));
  TRY(upload(s, d.scene_margin, margins.data(), margins.size()));
  {
    // mean rest edge length per scene (scale of the learned warm start's features)
    std::vector<double> ell(NS, 0.0);
    for (int k = 0; k < NS; ++k) {
      const auto& H = hs[k];
      static const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
      double sum = 0.0;
      for (int t = 0; t < H.m; ++t)
        for (const auto& e : E) {
          const int a = H.tets[4 * t + e[0]], b = H.tets[4 * t + e[1]];
          double l2 = 0.0;
          for (int q = 0; q < 3; ++q) l2 += (H.rest[3 * a + q] - H.rest[3 * b + q]) * (H.rest[3 * a + q] - H.rest[3 * b + q]);
          sum += std::sqrt(l2);
        }
      ell[k] = H.m > 0 ? sum / (6.0 * H.m) : 1.0;
    }
    TRY(upload(s, d.ell, ell.data(), ell.size()));
  }
  // obstacles
  s->scene_obst0.assign(NS + 1, 0);
  s->obst.clear();
  for (int k = 0; k < NS; ++k) {
    s->scene_obst0[k] = (int)s->obst.size();
    if (k < (int)obs.size())
      for (auto& o : obs[k]) {
        lg::ObstacleDev od{};
        TRY(obstacle_dev(s, k, o, od));
        s->obst.push_back(od);
      }
  }
  s->scene_obst0[NS] = (int)s->obst.size();
  TRY(push_obstacles(s));
  // default pin motion: all groups static
  std::vector<double> grp(9 * (size_t)d.G, 0.0);
  TRY(upload(s, d.grp, grp.data(), grp.size()));
  {
    // enough blocks that each owns at most 256 contacts of the capacity; 64 by default
    // (fastest of 8..128 on 800 contacts: fewer blocks lengthen the per-block matvec,
    // more lengthen the device-wide barrier)
    const int need = (d.CMAX + 255) / 256;
    int want = std::max(64, need);
    if (const char* e = std::getenv("LGSIM_CR_BLOCKS")) want = std::max(need, std::atoi(e));
    s->cr_blocks = std::max(1, std::min(lg::cr_max_blocks(), want));
  }
  int per = (d.CMAX + s->cr_blocks - 1) / s->cr_blocks;
  if (per > 256) {
    lg::set_error("max_contacts too large for the CR launch");
    return SIM_E_ARG;
  }
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&s->h_pinned), 8 * sizeof(int), hipHostMallocDefault));
  HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&s->h_res), std::max(1, NS) * sizeof(float), hipHostMallocDefault));
  for (auto& e : s->ev) HIPCHK(hipEventCreate(&e));
  if (s->opt.self_contact) TRY(build_self_contact(s, hs[0]));
  return SIM_OK;
}

// Device form of an obstacle of scene k; a binding's node (caller order, scene-local) is
// replaced by its internal index, and it carries no friction or surface velocity.
int obstacle_dev(lgsim* s, int k, const sim_obstacle& o, lg::ObstacleDev& od) {
  od.type = o.type;
  od.scene = k;
  std::memcpy(od.geom, o.geom, sizeof(od.geom));
  od.mu = o.mu;
  std::memcpy(od.vel, o.vel, sizeof(od.vel));
  if (o.type == 3) {
    const int node = (int)o.geom[7];
    if (node < 0 || node >= s->scenes[k].n) {
      lg::set_error("binding node out of range");
      return SIM_E_ARG;
    }
    od.geom[7] = (double)s->perm_caller[s->scenes[k].caller0 + node];
    od.mu = 0.0;
    od.vel[0] = od.vel[1] = od.vel[2] = 0.0;
  }
  return SIM_OK;
}

int validate_obstacles(int32_t n, const sim_obstacle* obs) {
  if (n < 0 || n > lg::kMaxObstacles || (n > 0 && !obs)) {
    lg::set_error("bad obstacle count");
    return SIM_E_ARG;
  }
  for (int i = 0; i < n; ++i) {
    const auto& o = obs[i];
    if (o.type < 0 || o.type > 3 || !(o.mu >= 0.0)) {
      lg::set_error("bad obstacle " + std::to_string(i));
      return SIM_E_ARG;
    }
    for (double g : o.geom)
      if (!std::isfinite(g)) {
        lg::set_error("non-finite obstacle geometry");
        return SIM_E_ARG;
      }
    if (o.type == 0 && o.geom[3] * o.geom[3] + o.geom[4] * o.geom[4] + o.geom[5] * o.geom[5] == 0.0) {
      lg::set_error("half-space with zero normal");
      return SIM_E_ARG;
    }
    if (o.type == 3 && (o.geom[3] * o.geom[3] + o.geom[4] * o.geom[4] + o.geom[5] * o.geom[5] == 0.0 ||
                        !(o.geom[6] >= 0.0) || !(o.geom[7] >= 0.0) || o.geom[7] != std::floor(o.geom[7]))) {
      lg::set_error("binding needs a non-zero direction, a compliance >= 0 and a node index");
      return SIM_E_ARG;
    }
    if (o.type == 2 && (!(o.geom[6] > 0.0) || (o.geom[0] == o.geom[3] && o.geom[1] == o.geom[4] && o.geom[2] == o.geom[5]))) {
      lg::set_error("degenerate cylinder");
      return SIM_E_ARG;
    }
  }
  return SIM_OK;
}

// Switched off: a device run that included the Jacobi global step and the objective
// kernel ended in a GPU fault whose cause has not been established.
constexpr bool kJacobiEnabled = false;
constexpr const char* kJacobiOff =
    "the Jacobi global step and the objective kernel are switched off (a run that included them ended in a GPU "
    "fault of unknown cause)";

// The Jacobi global step has no constraint solve: it needs a handle without obstacles.
int check_global_step(lgsim* s) {
  if (s->opt.global_step == SIM_GLOBAL_JACOBI && !kJacobiEnabled) {
    lg::set_error(kJacobiOff);
    return SIM_E_STATE;
  }
  if (s->opt.global_step == SIM_GLOBAL_JACOBI && !s->obst.empty()) {
    lg::set_error("the Jacobi global step is implemented for scenes without obstacles");
    return SIM_E_STATE;
  }
  return SIM_OK;
}

// ---------------------------------------------------------------- drivers
// Frame start (Algorithm 4): predicted state, pin targets, collision detection with
// compaction, Delassus operator and warm start.  No host synchronisation: every kernel
// reads the contact count from device memory and grids are sized by capacity.
// With fork, the steps after detection (Delassus operator, warm start, force ranges) run
// on the side stream; they read only what detection and the predicted state wrote, and
// the first iteration's local step, gather and S pass touch none of their outputs, so the
// two overlap.  join_setup makes the handle's stream wait for them before the contact
// evaluation of the first iteration.
int frame_setup(lgsim* s, bool fork) {
  auto& d = s->d;
  lg::launch_predict(d, s->st);
  lg::launch_pins(d, s->st);
  lg::launch_zero_dual(d, s->st);
  lg::launch_collide(d, s->st);
  hipStream_t cs = s->st;
  if (fork) {
    HIPCHK(hipEventRecord(s->fork_ev, s->st));
    HIPCHK(hipStreamWaitEvent(s->st2, s->fork_ev, 0));
    cs = s->st2;
  }
  lg::launch_delassus(d, cs);
  lg::launch_warm_start(d, cs, 0);
  const bool learned = (s->opt.warm == SIM_WARM_MLP || s->opt.warm == SIM_WARM_MLP_PERSIST) && s->has_model;
  if (s->record_pairs || learned) lg::launch_mlp_features(d, cs);
  if (learned) {
    lg::launch_mlp_warm(d, cs);
    lg::launch_warm_judge(d, cs);
  }
  lg::launch_force_ranges(d, cs);
  if (fork) {
    HIPCHK(hipEventRecord(s->join_ev, s->st2));
    s->setup_forked = true;
  }
  s->iter_c = -1;  // known after the next synchronisation
  return check_launch("frame setup");
}

int join_setup(lgsim* s) {
  if (!s->setup_forked) return SIM_OK;
  s->setup_forked = false;
  HIPCHK(hipStreamWaitEvent(s->st, s->join_ev, 0));
  return SIM_OK;
}

// Timing events of one frame: [0] frame start, [1] setup done, then 6 per iteration,
// then integrate start/end and residual end.
hipEvent_t* frame_event(lgsim* s, int i) {
  while ((int)s->fev.size() <= i) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    s->fev.push_back(e);
  }
  return &s->fev[i];
}

int iteration(lgsim* s, bool timed, int it) {
  auto& d = s->d;
  hipError_t cr_err = hipSuccess;
  const int base = 2 + 6 * it;
  auto rec = [&](int i) {
    if (timed) {
      hipEvent_t* e = frame_event(s, base + i);
      if (e) hipEventRecord(*e, s->st);
    }
  };
  rec(0);
  lg::launch_element(d, s->st);
  lg::launch_gather(d, s->st);
  rec(1);
  if (d.global_step == SIM_GLOBAL_JACOBI) {  // no obstacles (checked by the callers)
    TRY(join_setup(s));
    lg::launch_jacobi_global(d, s->st);
    for (int p = 2; p <= 5; ++p) rec(p);
    return check_launch("iteration");
  }
  lg::launch_spmv_S(d, s->st, d.b, d.y);
  TRY(join_setup(s));
  rec(2);
  if (s->iter_c != 0) {
    lg::launch_contact_prep(d, s->st);
    rec(3);
    cr_err = lg::launch_cr(d, s->st, s->cr_blocks, s->opt.cr_variant);
    lg::launch_apply_forces(d, s->st);
    rec(4);
  } else {
    rec(3);
    rec(4);
  }
  lg::launch_spmv_St(d, s->st, d.y, d.qp, d.q);
  rec(5);
  if (cr_err != hipSuccess) {
    lg::set_error(std::string("CR launch failed: ") + hipGetErrorString(cr_err));
    return SIM_E_DEVICE;
  }
  return check_launch("iteration");
}

// phases: 0 setup, 1 local + gather, 2 S pass, 3 contact evaluation, 4 CR + force
// update, 5 S^T pass, 6 integrate, 7 residual
void collect_times(lgsim* s, int iters, float* ms) {
  auto el = [&](int a, int b) {
    float t = 0.0f;
    if (a < (int)s->fev.size() && b < (int)s->fev.size()) hipEventElapsedTime(&t, s->fev[a], s->fev[b]);
    return t;
  };
  ms[0] += el(0, 1);
  for (int it = 0; it < iters; ++it) {
    int b = 2 + 6 * it;
    for (int p = 0; p < 5; ++p) ms[1 + p] += el(b + p, b + p + 1);
  }
  int e = 2 + 6 * iters;
  ms[6] += el(e, e + 1);
  ms[7] += el(e + 1, e + 2);
}

int read_residual(lgsim* s, double* worst) {
  auto& d = s->d;
  lg::launch_residual(d, s->st);
  HIPCHK(hipMemcpyAsync(s->h_res, d.res, sizeof(float) * d.NS, hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipMemcpyAsync(s->h_pinned, d.n_contacts, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipMemcpyAsync(s->h_pinned + 1, d.overflow, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  double w = 0.0;
  for (int k = 0; k < d.NS; ++k) w = std::max(w, (double)s->h_res[k]);
  *worst = w;
  s->iter_c = s->h_pinned[0];
  return SIM_OK;
}

// Clears a device flag after it was reported.
int clear_flag(lgsim* s, int* dflag) {
  int zero = 0;
  HIPCHK(hipMemcpyAsync(dflag, &zero, sizeof(int), hipMemcpyHostToDevice, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  return SIM_OK;
}

// Integration unless the frame overflowed or produced non-finite positions (then the
// frame is dropped and the state stays at the frame start).
int finish_frame(lgsim* s) {
  auto& d = s->d;
  TRY(join_setup(s));
  lg::launch_check_finite(d, s->st);
  lg::launch_integrate(d, s->st);
  TRY(check_launch("integrate"));
  return SIM_OK;
}

int frame_status(lgsim* s) {
  auto& d = s->d;
  HIPCHK(hipMemcpyAsync(s->h_pinned, d.n_contacts, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipMemcpyAsync(s->h_pinned + 1, d.overflow, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipMemcpyAsync(s->h_pinned + 2, d.bad, 2 * sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  s->iter_c = s->h_pinned[0];
  if (s->h_pinned[3]) {
    TRY(clear_flag(s, d.bad));
    TRY(clear_flag(s, d.bad + 1));
    lg::set_error("constraint solver blocks were not all resident (device busy with other work); frame rolled back");
    return SIM_E_DEVICE;
  }
  if (s->h_pinned[1]) {
    TRY(clear_flag(s, d.overflow));
    lg::set_error("contact capacity exceeded: " + std::to_string(s->h_pinned[0]) + " contacts, max_contacts " +
                  std::to_string(d.CMAX) + " (or Delassus storage full); frame not advanced");
    return SIM_E_CAPACITY;
  }
  if (s->h_pinned[2]) {
    TRY(clear_flag(s, d.bad));
    lg::set_error("non-finite state; frame rolled back");
    return SIM_E_DIVERGED;
  }
  return SIM_OK;
}

int sort_contacts_canonical(lgsim* s, int c, std::vector<int>& node, std::vector<int>& obst,
                            std::vector<int32_t>& order) {
  // order[k] = internal index of the k-th canonical contact
  node.resize(c);
  obst.resize(c);
  HIPCHK(hipMemcpyAsync(node.data(), s->d.c_node, sizeof(int) * c, hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipMemcpyAsync(obst.data(), s->d.c_obst, sizeof(int) * c, hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  order.resize(c);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    int ca = s->iperm_caller[node[a]], cb = s->iperm_caller[node[b]];
    if (ca != cb) return ca < cb;
    return obst[a] < obst[b];
  });
  return SIM_OK;
}

int download_nodes(lgsim* s, const float* dsrc, double* out) {
  auto& d = s->d;
  std::vector<float> buf(3 * (size_t)d.N4);
  HIPCHK(hipMemcpyAsync(buf.data(), dsrc, sizeof(float) * buf.size(), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  for (int gi = 0; gi < d.N; ++gi) {
    int ci = s->iperm_caller[gi];
    for (int c = 0; c < 3; ++c) out[3 * (size_t)ci + c] = buf[c * (size_t)d.N4 + gi];
  }
  return SIM_OK;
}

int upload_nodes(lgsim* s, const double* src, float* ddst) {
  auto& d = s->d;
  std::vector<float> buf(3 * (size_t)d.N4, 0.0f);
  for (int ci = 0; ci < d.N; ++ci) {
    int gi = s->perm_caller[ci];
    for (int c = 0; c < 3; ++c) {
      double v = src[3 * (size_t)ci + c];
      if (!std::isfinite(v)) {
        lg::set_error("non-finite input");
        return SIM_E_ARG;
      }
      buf[c * (size_t)d.N4 + gi] = (float)v;
    }
  }
  return upload(s, ddst, buf.data(), buf.size());
}

int create_common(int32_t count, const sim_mesh* meshes, const sim_material* mats, double h,
                  const sim_options* opt, const std::vector<std::vector<sim_obstacle>>& obs, sim_t* out) {
  if (!meshes || !mats || !out || count <= 0) {
    lg::set_error("null argument");
    return SIM_E_ARG;
  }
  if (count > lg::kMaxScenes) {
    lg::set_error("at most " + std::to_string(lg::kMaxScenes) + " scenes per handle");
    return SIM_E_ARG;
  }
  *out = nullptr;
  lgsim* s = nullptr;
  try {
    s = new lgsim();
  } catch (...) {
    lg::set_error("host allocation failed");
    return SIM_E_NOMEM;
  }
  if (opt) s->opt = *opt;
  else sim_options_default(&s->opt);
  auto fail = [&](int rc) {
    delete s;
    return rc;
  };
  if (s->opt.cr_iters < 0 || s->opt.cr_iters > lg::kMaxCrIters || !(s->opt.cr_tol >= 0.0) ||
      (s->opt.cr_variant != SIM_CR_TEXTBOOK && s->opt.cr_variant != SIM_CR_PIPELINED) ||
      s->opt.max_contacts <= 0 || s->opt.max_iters <= 0 || !(s->opt.ncp_tol > 0.0) ||
      s->opt.warm < 0 || s->opt.warm > SIM_WARM_MLP_PERSIST || !(s->opt.contact_margin >= 0.0) ||
      (s->opt.ncp != SIM_NCP_FB && s->opt.ncp != SIM_NCP_MINMAP) ||
      (s->opt.precond != SIM_PRECOND_DELASSUS && s->opt.precond != SIM_PRECOND_MASS) ||
      (s->opt.global_step != SIM_GLOBAL_DIRECT && s->opt.global_step != SIM_GLOBAL_JACOBI) ||
      (s->opt.lg_form != SIM_LG_PD && s->opt.lg_form != SIM_LG_ADMM) ||
      (s->opt.self_contact != 0 && s->opt.self_contact != 1) || !(s->opt.self_mu >= 0.0)) {
    lg::set_error("bad options");
    return fail(SIM_E_ARG);
  }
  if (s->opt.self_contact && count != 1) {
    lg::set_error("self contact is available for single-scene handles");
    return fail(SIM_E_ARG);
  }
  if (s->opt.self_contact && s->opt.global_step != SIM_GLOBAL_DIRECT) {
    lg::set_error("self contact needs the direct global step");
    return fail(SIM_E_ARG);
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    lg::set_error("no HIP device");
    return fail(SIM_E_DEVICE);
  }
  if (s->opt.hip_stream) {
    s->st = static_cast<hipStream_t>(s->opt.hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess) {
      lg::set_error("stream creation failed");
      return fail(SIM_E_DEVICE);
    }
    s->own_stream = true;
  }
  if (hipStreamCreateWithFlags(&s->st2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&s->join_ev, hipEventDisableTiming) != hipSuccess) {
    lg::set_error("stream creation failed");
    return fail(SIM_E_DEVICE);
  }
  std::vector<lg::HostScene> hs(count);
  try {
    for (int k = 0; k < count; ++k) {
      if (meshes[k].n_pins > 0 && (!meshes[k].pin_nodes || !meshes[k].pin_group)) {
        lg::set_error("pins without arrays");
        return fail(SIM_E_ARG);
      }
      std::string err;
      int rc = lg::precompute(lg::mesh_in(&meshes[k]), lg::material_in(&mats[k]), h, s->opt.pin_weight_scale,
                              false, hs[k], err);
      if (rc != SIM_OK) {
        lg::set_error(count > 1 ? "scene " + std::to_string(k) + ": " + err : err);
        return fail(rc);
      }
    }
    for (auto& o : obs) {
      int rc = validate_obstacles((int)o.size(), o.data());
      if (rc != SIM_OK) return fail(rc);
    }
    int rc = build(s, hs, obs);
    if (rc != SIM_OK) return fail(rc);
  } catch (const std::bad_alloc&) {
    lg::set_error("host allocation failed");
    return fail(SIM_E_NOMEM);
  }
  *out = s;
  return SIM_OK;
}

}  // namespace

extern "C" {

int sim_options_default(sim_options* o) {
  if (!o) return SIM_E_ARG;
  std::memset(o, 0, sizeof(*o));
  o->gravity[2] = -9.81;
  o->pin_weight_scale = 1.0;
  o->contact_margin = 0.0;
  o->cr_iters = 10;
  o->cr_tol = 0.0;
  o->cr_variant = SIM_CR_TEXTBOOK;
  o->graph = 1;
  o->ncp = SIM_NCP_FB;
  o->precond = SIM_PRECOND_DELASSUS;
  o->global_step = SIM_GLOBAL_DIRECT;
  o->lg_form = SIM_LG_PD;
  o->warm = SIM_WARM_PREV;
  o->ncp_tol = 1e-6;
  o->max_iters = 200;
  o->max_contacts = 2048;
  o->hip_stream = nullptr;
  return SIM_OK;
}

int sim_create(const sim_mesh* mesh, const sim_material* mat, double h, const sim_options* opt, sim_t* out) {
  std::vector<std::vector<sim_obstacle>> obs(1);
  return create_common(1, mesh, mat, h, opt, obs, out);
}

int sim_create_batch(int32_t count, const sim_mesh* meshes, const sim_material* mats, const int32_t* n_obstacles,
                     const sim_obstacle* const* obstacles, double h, const sim_options* opt, sim_t* out) {
  if (count <= 0 || !n_obstacles || !obstacles) {
    lg::set_error("bad batch arguments");
    return SIM_E_ARG;
  }
  std::vector<std::vector<sim_obstacle>> obs(count);
  for (int k = 0; k < count; ++k) {
    if (n_obstacles[k] < 0 || (n_obstacles[k] > 0 && !obstacles[k])) {
      lg::set_error("bad obstacle list");
      return SIM_E_ARG;
    }
    obs[k].assign(obstacles[k], obstacles[k] + n_obstacles[k]);
  }
  return create_common(count, meshes, mats, h, opt, obs, out);
}

int sim_batch_info(sim_t s, int32_t* count, int32_t* node_offsets) {
  if (!s) return SIM_E_ARG;
  if (count) *count = (int32_t)s->scenes.size();
  if (node_offsets) {
    for (size_t k = 0; k < s->scenes.size(); ++k) node_offsets[k] = s->scenes[k].caller0;
    node_offsets[s->scenes.size()] = s->d.N;
  }
  return SIM_OK;
}

int sim_set_obstacles(sim_t s, int32_t n, const sim_obstacle* obs) {
  if (!s) {
    lg::set_error("null handle");
    return SIM_E_ARG;
  }
  if (s->scenes.size() != 1) {
    lg::set_error("sim_set_obstacles applies to single-scene handles");
    return SIM_E_STATE;
  }
  TRY(validate_obstacles(n, obs));
  std::vector<lg::ObstacleDev> next;
  for (int i = 0; i < n; ++i) {
    lg::ObstacleDev od{};
    TRY(obstacle_dev(s, 0, obs[i], od));
    next.push_back(od);
  }
  s->obst = next;
  s->scene_obst0 = {0, n};
  return push_obstacles(s);
}

int sim_set_solver(sim_t s, int32_t cr_iters, double cr_tol, int32_t cr_variant) {
  if (!s || cr_iters < 0 || cr_iters > lg::kMaxCrIters || !(cr_tol >= 0.0) ||
      (cr_variant != SIM_CR_TEXTBOOK && cr_variant != SIM_CR_PIPELINED)) {
    lg::set_error("bad solver settings");
    return SIM_E_ARG;
  }
  s->opt.cr_iters = cr_iters;
  s->opt.cr_tol = cr_tol;
  s->opt.cr_variant = cr_variant;
  s->d.cr_iters = cr_iters;
  s->d.cr_tol = (float)cr_tol;
  return SIM_OK;
}

int sim_time_kernel(sim_t s, int32_t which, int32_t reps, float* ms_avg) {
  if (!s || which < 0 || which > 2 || reps <= 0 || !ms_avg) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  if (which == 2 && s->opt.lg_form == SIM_LG_ADMM) {
    lg::set_error("the ADMM-PD local step updates its dual variables: not timed in isolation");
    return SIM_E_STATE;
  }
  auto& d = s->d;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  auto launch = [&]() {
    if (which == 0) lg::launch_spmv_S(d, s->st, d.b, d.tmp);  // reads b, writes scratch
    else if (which == 1) lg::launch_spmv_St(d, s->st, d.y, d.qp, d.tmp);  // reads y and q~, writes scratch
    else lg::launch_element(d, s->st);  // corner forces of the current iterate (same values)
  };
  launch();
  HIPCHK(hipEventRecord(e0, s->st));
  for (int r = 0; r < reps; ++r) launch();
  HIPCHK(hipEventRecord(e1, s->st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  TRY(check_launch("timed kernel"));
  *ms_avg = ms / reps;
  return SIM_OK;
}

int sim_profile_cr(sim_t s, int32_t reps, float* out) {
  if (!s || reps <= 0 || reps > SIM_PROFILE_MAX_REPS || !out) {
    lg::set_error("bad arguments (reps in 1.." + std::to_string(SIM_PROFILE_MAX_REPS) + ")");
    return SIM_E_ARG;
  }
  auto& d = s->d;
  const size_t ncl = 2 + 4 * (size_t)lg::kCrMaxBarriers;
  if (!s->d_lam_save) TRY(s->alloc(s->d_lam_save, 3 * (size_t)d.CMAX));
  if (!s->d_clock) TRY(s->alloc(s->d_clock, ncl));
  const size_t lam_bytes = 3 * (size_t)d.CMAX * sizeof(float);
  HIPCHK(hipMemcpyAsync(s->d_lam_save, d.lam, lam_bytes, hipMemcpyDeviceToDevice, s->st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // Launch durations: `reps` launches back to back between one pair of events (events
  // around every launch would add their own latency), each launch with barrier flags of
  // its own, all zeroed before the first.  A launch adds its increment to lambda only at
  // its end, so repeated launches from one state do the same work.
  const size_t stride = lg::kCrSyncWords;
  if (!s->d_prof_sync) TRY(s->alloc(s->d_prof_sync, stride * SIM_PROFILE_MAX_REPS));
  hipError_t cr_err = hipSuccess;
  float ms_all = 0.0f;
  lg::launch_zero_cr_sync(d, s->st);
  cr_err = lg::launch_cr(d, s->st, s->cr_blocks, s->opt.cr_variant);  // warm-up
  HIPCHK(hipMemsetAsync(s->d_prof_sync, 0, stride * reps * sizeof(unsigned), s->st));
  lg::Dev dr = d;
  HIPCHK(hipEventRecord(e0, s->st));
  for (int r = 0; r < reps && cr_err == hipSuccess; ++r) {
    dr.cr_sync = s->d_prof_sync + stride * r;
    cr_err = lg::launch_cr(dr, s->st, s->cr_blocks, s->opt.cr_variant);
  }
  HIPCHK(hipEventRecord(e1, s->st));
  HIPCHK(hipEventSynchronize(e1));
  HIPCHK(hipEventElapsedTime(&ms_all, e0, e1));
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  HIPCHK(cr_err);
  // one more launch from the saved state with block 0's wall-clock stamps
  lg::Dev dc = d;
  dc.cr_clock = s->d_clock;
  HIPCHK(hipMemcpyAsync(d.lam, s->d_lam_save, lam_bytes, hipMemcpyDeviceToDevice, s->st));
  lg::launch_zero_cr_sync(d, s->st);
  HIPCHK(hipMemsetAsync(s->d_clock, 0, ncl * sizeof(unsigned long long), s->st));
  HIPCHK(lg::launch_cr(dc, s->st, s->cr_blocks, s->opt.cr_variant));
  HIPCHK(hipMemcpyAsync(d.lam, s->d_lam_save, lam_bytes, hipMemcpyDeviceToDevice, s->st));
  std::vector<unsigned long long> clk(ncl);
  HIPCHK(hipMemcpyAsync(clk.data(), s->d_clock, ncl * sizeof(unsigned long long), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  TRY(frame_status(s));
  int dev = 0, khz = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  const double us = khz > 0 ? 1e3 / khz : 0.0;  // microseconds per tick
  int nb = 0;
  double exch = 0.0, wait = 0.0;
  while (nb < lg::kCrMaxBarriers && clk[2 + 4 * nb] != 0) {
    const unsigned long long t_in = clk[2 + 4 * nb], t_out = clk[3 + 4 * nb], t_data = clk[4 + 4 * nb];
    wait += (double)(t_out - t_in) * us;
    exch += (double)((t_data ? t_data : t_out) - t_in) * us;
    ++nb;
  }
  s->cr_stamps.assign(clk.begin(), clk.begin() + 2 + 4 * (size_t)nb);
  out[0] = ms_all / reps;
  out[1] = (float)((double)(clk[1] - clk[0]) * us);
  out[2] = nb ? (float)((double)(clk[2] - clk[0]) * us) : 0.0f;
  out[3] = nb ? (float)(exch / nb) : 0.0f;
  out[4] = nb ? (float)(wait / nb) : 0.0f;
  out[5] = (float)nb;
  return SIM_OK;
}

int sim_read_cr_stamps(sim_t s, uint64_t* out, int32_t cap, int32_t* n) {
  if (!s || !n || cap < 0 || (cap > 0 && !out)) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  const size_t m = std::min(s->cr_stamps.size(), (size_t)cap);
  for (size_t i = 0; i < m; ++i) out[i] = s->cr_stamps[i];
  *n = (int32_t)s->cr_stamps.size();
  return SIM_OK;
}

int sim_set_graph(sim_t s, int32_t on) {
  if (!s) {
    lg::set_error("null handle");
    return SIM_E_ARG;
  }
  s->opt.graph = on != 0;
  return SIM_OK;
}

int sim_get_tuning(sim_t s, sim_tuning* t) {
  if (!s || !t) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  t->cr_blocks = s->cr_blocks;
  t->cr_variant = s->opt.cr_variant;
  t->seg_floats = s->seg_floats;
  t->elem_block = s->d.elem_block;
  t->row_group = s->d.row_group;
  t->col_group = s->d.col_group;
  t->ms_frame = 0.0f;
  return SIM_OK;
}

static bool group_ok(int g) { return g == 1 || g == 2 || g == 4 || g == 8; }

int sim_set_tuning(sim_t s, const sim_tuning* t) {
  if (!s || !t || t->seg_floats < 64 || t->seg_floats % 4 != 0 || t->elem_block < 64 || t->elem_block > lg::kBlock ||
      t->elem_block % lg::kWave != 0 || (t->cr_variant != SIM_CR_TEXTBOOK && t->cr_variant != SIM_CR_PIPELINED) ||
      !group_ok(t->row_group) || !group_ok(t->col_group)) {
    lg::set_error("bad tuning");
    return SIM_E_ARG;
  }
  const int need = (s->d.CMAX + 255) / 256;
  if (t->cr_blocks < need || t->cr_blocks > lg::cr_max_blocks()) {
    lg::set_error("cr_blocks must lie in [" + std::to_string(need) + ", " + std::to_string(lg::cr_max_blocks()) + "]");
    return SIM_E_ARG;
  }
  if (t->seg_floats != s->seg_floats || t->row_group != s->d.row_group)
    TRY(build_segments(s, t->seg_floats, t->row_group));
  if (t->col_group != s->d.col_group) TRY(build_col_groups(s, t->col_group));
  s->cr_blocks = t->cr_blocks;
  s->opt.cr_variant = t->cr_variant;
  s->d.elem_block = t->elem_block;
  return SIM_OK;
}

int sim_autotune(sim_t s, int32_t frames, int32_t iters, int32_t allow_pipelined, sim_tuning* best) {
  if (!s || frames <= 0 || iters <= 0 || !best) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  TRY(sim_save_state(s));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  // time of `frames` frames from the saved state (each frame restarts from it), after one
  // untimed frame that also captures the graph
  auto measure = [&](const sim_tuning& t, float* ms) -> int {
    TRY(sim_set_tuning(s, &t));
    TRY(sim_restore_state(s));
    TRY(sim_step(s, 1, iters, nullptr));
    float total = 0.0f;
    for (int f = 0; f < frames; ++f) {
      TRY(sim_restore_state(s));
      HIPCHK(hipEventRecord(e0, s->st));
      TRY(sim_step(s, 1, iters, nullptr));
      HIPCHK(hipEventRecord(e1, s->st));
      HIPCHK(hipEventSynchronize(e1));
      float m = 0.0f;
      HIPCHK(hipEventElapsedTime(&m, e0, e1));
      total += m;
    }
    *ms = total / frames;
    return SIM_OK;
  };
  sim_tuning cur{};
  TRY(sim_get_tuning(s, &cur));
  float best_ms = 0.0f;
  int rc = measure(cur, &best_ms);
  // S / S^T group sizes and segment length by kernel times, then coordinate search over
  // the element block size and the CR launch by frame times
  auto try_cand = [&](sim_tuning c) -> int {
    float m = 0.0f;
    TRY(measure(c, &m));
    if (m < best_ms) {
      best_ms = m;
      cur = c;
    }
    return SIM_OK;
  };
  // S-pass parameters change only their own kernels: chosen by those kernels' times
  // (back-to-back launches), which are far steadier than whole frames
  if (rc == SIM_OK) {
    float best_s = 0.0f, best_st = 0.0f;
    sim_tuning c = cur;
    for (int g : {1, 2, 4, 8})
      for (int seg : {1024, 2048, 4096}) {
        c.row_group = g;
        c.seg_floats = seg;
        float m = 0.0f;
        if (rc == SIM_OK) rc = sim_set_tuning(s, &c);
        if (rc == SIM_OK) rc = sim_time_kernel(s, 0, 30, &m);
        if (rc == SIM_OK && (best_s == 0.0f || m < best_s)) {
          best_s = m;
          cur.row_group = g;
          cur.seg_floats = seg;
        }
      }
    for (int g : {1, 2, 4, 8}) {
      c = cur;
      c.col_group = g;
      float m = 0.0f;
      if (rc == SIM_OK) rc = sim_set_tuning(s, &c);
      if (rc == SIM_OK) rc = sim_time_kernel(s, 1, 30, &m);
      if (rc == SIM_OK && (best_st == 0.0f || m < best_st)) {
        best_st = m;
        cur.col_group = g;
      }
    }
    if (rc == SIM_OK) rc = measure(cur, &best_ms);
  }
  for (int eb : {64, 128, 256})
    if (rc == SIM_OK && eb != cur.elem_block) {
      sim_tuning c = cur;
      c.elem_block = eb;
      rc = try_cand(c);
    }
  const int need = (s->d.CMAX + 255) / 256, most = lg::cr_max_blocks();
  for (int v = 0; v <= (allow_pipelined ? 1 : 0); ++v)
    for (int g : {16, 32, 48, 64, 96, 128, 192, 256})
      if (rc == SIM_OK && g >= need && g <= most && !(v == cur.cr_variant && g == cur.cr_blocks)) {
        sim_tuning c = cur;
        c.cr_variant = v;
        c.cr_blocks = g;
        rc = try_cand(c);
      }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != SIM_OK) return rc;
  TRY(sim_set_tuning(s, &cur));
  TRY(sim_restore_state(s));
  cur.ms_frame = best_ms;
  *best = cur;
  return SIM_OK;
}

int sim_set_warm_model(sim_t s, const float* params, int32_t n_params) {
  if (!s || !params || n_params != lg::kMlpParams) {
    lg::set_error("sim_set_warm_model: expected " + std::to_string(lg::kMlpParams) + " parameters");
    return SIM_E_ARG;
  }
  TRY(upload(s, s->d.mlp_P, params, (size_t)n_params));
  HIPCHK(hipStreamSynchronize(s->st));
  s->has_model = true;
  return SIM_OK;
}

int sim_set_warm_mode(sim_t s, int32_t warm) {
  if (!s || warm < SIM_WARM_ZERO || warm > SIM_WARM_MLP_PERSIST) {
    lg::set_error("bad warm start mode");
    return SIM_E_ARG;
  }
  s->opt.warm = warm;
  s->d.warm = warm;
  return SIM_OK;
}

int sim_record_training_pairs(sim_t s, int32_t on) {
  if (!s) {
    lg::set_error("null handle");
    return SIM_E_ARG;
  }
  s->record_pairs = on != 0;
  return SIM_OK;
}

int sim_read_training_pairs(sim_t s, int32_t* node, int32_t* obstacle, float* feat, float* target, int32_t cap,
                            int32_t* n) {
  if (!s || !n || cap < 0 || (cap > 0 && (!feat || !target))) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  if (!s->record_pairs && !((s->opt.warm == SIM_WARM_MLP || s->opt.warm == SIM_WARM_MLP_PERSIST) && s->has_model)) {
    lg::set_error("features are not recorded (sim_record_training_pairs)");
    return SIM_E_STATE;
  }
  auto& d = s->d;
  int c = 0;
  HIPCHK(hipMemcpyAsync(&c, d.n_contacts, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  c = std::min(c, d.CMAX);
  *n = c;
  if (c > cap) {
    lg::set_error("capacity too small: " + std::to_string(c) + " contacts");
    return SIM_E_CAPACITY;
  }
  if (c == 0) return SIM_OK;
  std::vector<int> cn, co;
  std::vector<int32_t> order;
  TRY(sort_contacts_canonical(s, c, cn, co, order));
  std::vector<float> f(16 * (size_t)c), t(3 * (size_t)c);
  lg::launch_mlp_targets(d, s->d_tgt, s->st);
  HIPCHK(hipMemcpyAsync(f.data(), d.c_feat, f.size() * sizeof(float), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipMemcpyAsync(t.data(), s->d_tgt, t.size() * sizeof(float), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  for (int k = 0; k < c; ++k) {
    const int j = order[k];
    if (node) node[k] = s->iperm_caller[cn[j]];
    if (obstacle) obstacle[k] = co[j];
    std::memcpy(feat + 16 * (size_t)k, f.data() + 16 * (size_t)j, 16 * sizeof(float));
    std::memcpy(target + 3 * (size_t)k, t.data() + 3 * (size_t)j, 3 * sizeof(float));
  }
  return SIM_OK;
}

int sim_read_warm_judge(sim_t s, float* res, float* lam_learned, int32_t cap, int32_t* n) {
  if (!s || !res || !n || cap < 0 || (cap > 0 && !lam_learned)) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  if (!((s->opt.warm == SIM_WARM_MLP || s->opt.warm == SIM_WARM_MLP_PERSIST) && s->has_model)) {
    lg::set_error("the warm start is not learned: no judge values");
    return SIM_E_STATE;
  }
  auto& d = s->d;
  int c = 0;
  HIPCHK(hipMemcpyAsync(&c, d.n_contacts, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipMemcpyAsync(res, d.judge, 2 * sizeof(float) * d.NS, hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  c = std::min(c, d.CMAX);
  *n = c;
  if (cap == 0 || c == 0) return SIM_OK;
  if (c > cap) {
    lg::set_error("capacity too small: " + std::to_string(c) + " contacts");
    return SIM_E_CAPACITY;
  }
  std::vector<int> cn, co;
  std::vector<int32_t> order;
  TRY(sort_contacts_canonical(s, c, cn, co, order));
  std::vector<float> l(3 * (size_t)d.CMAX);
  HIPCHK(hipMemcpyAsync(l.data(), d.lam_ml, l.size() * sizeof(float), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  for (int k = 0; k < c; ++k)
    for (int q = 0; q < 3; ++q) lam_learned[3 * (size_t)k + q] = l[q * (size_t)d.CMAX + order[k]];
  return SIM_OK;
}

int sim_surface_triangles(sim_t s, int32_t* tris, int32_t cap, int32_t* n) {
  if (!s || !n || cap < 0 || (cap > 0 && !tris)) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  const int T = (int)(s->surf_tris.size() / 3);
  *n = T;
  if (cap == 0) return SIM_OK;
  if (T > cap) {
    lg::set_error("capacity too small: " + std::to_string(T) + " triangles");
    return SIM_E_CAPACITY;
  }
  std::copy(s->surf_tris.begin(), s->surf_tris.end(), tris);
  return SIM_OK;
}

int sim_set_pin_motion(sim_t s, int32_t n_groups, const double* lin, const double* ang, const double* pivot) {
  if (!s || n_groups < 0 || (n_groups > 0 && (!lin || !ang || !pivot))) {
    lg::set_error("bad pin motion arguments");
    return SIM_E_ARG;
  }
  if (s->scenes.size() != 1) {
    lg::set_error("sim_set_pin_motion applies to single-scene handles");
    return SIM_E_STATE;
  }
  if (n_groups < s->scenes[0].n_groups) {
    lg::set_error("pin motion must cover every pin group");
    return SIM_E_ARG;
  }
  std::vector<double> grp(9 * (size_t)s->d.G, 0.0);
  for (int g = 0; g < std::min(n_groups, s->d.G); ++g)
    for (int c = 0; c < 3; ++c) {
      grp[9 * g + c] = lin[3 * g + c];
      grp[9 * g + 3 + c] = ang[3 * g + c];
      grp[9 * g + 6 + c] = pivot[3 * g + c];
    }
  for (double v : grp)
    if (!std::isfinite(v)) {
      lg::set_error("non-finite pin motion");
      return SIM_E_ARG;
    }
  return upload(s, s->d.grp, grp.data(), grp.size());
}

namespace {

// One fixed-iteration frame (setup, iters iterations, integration) replayed from a
// hipGraph captured on the handle's stream; re-captured whenever the device state
// descriptor or a launch setting differs from the captured one.
int frame_by_graph(lgsim* s, int iters) {
  std::vector<unsigned char> key(sizeof(lg::Dev) + 8 * sizeof(int));
  std::memcpy(key.data(), &s->d, sizeof(lg::Dev));
  const int extra[8] = {iters, s->cr_blocks, s->opt.cr_variant, s->opt.warm, (int)s->has_model, (int)s->record_pairs,
                        s->seg_floats, s->d.elem_block};
  std::memcpy(key.data() + sizeof(lg::Dev), extra, sizeof(extra));
  if (!s->gexec || key != s->gkey) {
    if (s->gexec) {
      HIPCHK(hipGraphExecDestroy(s->gexec));
      s->gexec = nullptr;
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
    int rc = frame_setup(s, true);
    for (int k = 0; rc == SIM_OK && k < iters; ++k) rc = iteration(s, false, k);
    if (rc != SIM_OK) (void)join_setup(s);  // no side-stream work left outside the capture
    if (rc == SIM_OK) rc = finish_frame(s);
    hipError_t e = hipStreamEndCapture(s->st, &g);
    if (rc != SIM_OK) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    HIPCHK(e);
    e = hipGraphInstantiate(&s->gexec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    HIPCHK(e);
    s->gkey = key;
  }
  HIPCHK(hipGraphLaunch(s->gexec, s->st));
  s->iter_c = -1;
  return SIM_OK;
}

// Frames iterated to tolerance run their iterations in chunks of kTolChunk, each
// iteration followed by the NCP residual and a convergence check on the device; a chunk is
// replayed from a hipGraph and the host reads the convergence flag once per chunk instead
// of the residual after every iteration.  Iterations after convergence return at once.
constexpr int kTolChunk = 4;

// Points the device descriptor at the convergence flag for the duration of a frame.
struct ConvergenceScope {
  lgsim* s;
  explicit ConvergenceScope(lgsim* s_) : s(s_) {
    s->d.done = s->d_conv;
    s->d.iter_count = s->d_conv + 1;
    s->d.ncp_tol = (float)s->opt.ncp_tol;
    s->d.max_iters = s->opt.max_iters;
  }
  ~ConvergenceScope() {
    s->d.done = nullptr;
    s->d.iter_count = nullptr;
  }
};

int tolerance_chunk(lgsim* s) {
  std::vector<unsigned char> key(sizeof(lg::Dev) + 6 * sizeof(int));
  std::memcpy(key.data(), &s->d, sizeof(lg::Dev));
  const int extra[6] = {kTolChunk, s->cr_blocks, s->opt.cr_variant, s->seg_floats, s->d.elem_block, 1};
  std::memcpy(key.data() + sizeof(lg::Dev), extra, sizeof(extra));
  if (!s->cexec || key != s->ckey) {
    if (s->cexec) {
      HIPCHK(hipGraphExecDestroy(s->cexec));
      s->cexec = nullptr;
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(s->st, hipStreamCaptureModeThreadLocal));
    int rc = SIM_OK;
    for (int k = 0; rc == SIM_OK && k < kTolChunk; ++k) {
      rc = iteration(s, false, k);
      if (rc == SIM_OK) {
        lg::launch_residual(s->d, s->st);
        lg::launch_convergence_check(s->d, s->st);
      }
    }
    hipError_t e = hipStreamEndCapture(s->st, &g);
    if (rc != SIM_OK) {
      if (g) hipGraphDestroy(g);
      return rc;
    }
    HIPCHK(e);
    e = hipGraphInstantiate(&s->cexec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    HIPCHK(e);
    s->ckey = key;
  }
  HIPCHK(hipGraphLaunch(s->cexec, s->st));
  return SIM_OK;
}

// Iterations of one frame until every scene's NCP residual is within ncp_tol, or
// max_iters, or a failure flag; *k = iterations run.  The set-up ran on the one stream.
int iterate_to_tolerance(lgsim* s, int* k) {
  ConvergenceScope scope(s);
  lg::launch_reset_convergence(s->d, s->st);
  while (true) {
    TRY(tolerance_chunk(s));
    HIPCHK(hipMemcpyAsync(s->h_pinned + 4, s->d_conv, 2 * sizeof(int), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    if (s->h_pinned[4] || s->h_pinned[5] >= s->opt.max_iters) break;
  }
  *k = s->h_pinned[5];
  return SIM_OK;
}

}  // namespace

int sim_step(sim_t s, int32_t frames, int32_t iters, sim_stats* stats) {
  if (!s || frames < 0 || iters < 0) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  if ((s->opt.warm == SIM_WARM_MLP || s->opt.warm == SIM_WARM_MLP_PERSIST) && !s->has_model) {
    lg::set_error("learned warm start selected but no model set (sim_set_warm_model)");
    return SIM_E_STATE;
  }
  TRY(check_global_step(s));
  for (int f = 0; f < frames; ++f) {
    const bool timed = stats != nullptr;
    auto t0 = std::chrono::steady_clock::now();
    auto rec = [&](int i) {
      if (timed) {
        hipEvent_t* e = frame_event(s, i);
        if (e) hipEventRecord(*e, s->st);
      }
    };
    if (iters > 0 && s->opt.graph) {
      TRY(frame_by_graph(s, iters));
      int rc = frame_status(s);
      if (rc != SIM_OK) return rc;
      if (timed) {
        lg::launch_residual(s->d, s->st);
        HIPCHK(hipMemcpyAsync(s->h_res, s->d.res, sizeof(float) * s->d.NS, hipMemcpyDeviceToHost, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        double res = 0.0;
        for (int q = 0; q < s->d.NS; ++q) res = std::max(res, (double)s->h_res[q]);
        auto& st = stats[f];
        st.iters_done = iters;
        st.n_contacts = s->iter_c;
        st.ncp_res = res;
        st.ms_frame = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int q = 0; q < 8; ++q) st.ms_phase[q] = 0.0f;  // not resolved inside a graph
      }
      continue;
    }
    if (iters == 0 && s->opt.graph) {  // to tolerance, in replayed chunks
      TRY(frame_setup(s, false));
      int k = 0;
      TRY(iterate_to_tolerance(s, &k));
      TRY(finish_frame(s));
      int rc = frame_status(s);
      if (rc != SIM_OK) return rc;
      if (timed) {
        HIPCHK(hipMemcpyAsync(s->h_res, s->d.res, sizeof(float) * s->d.NS, hipMemcpyDeviceToHost, s->st));
        HIPCHK(hipStreamSynchronize(s->st));
        double res = 0.0;
        for (int q = 0; q < s->d.NS; ++q) res = std::max(res, (double)s->h_res[q]);
        auto& st = stats[f];
        st.iters_done = k;
        st.n_contacts = s->iter_c;
        st.ncp_res = res;
        st.ms_frame = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
        for (int q = 0; q < 8; ++q) st.ms_phase[q] = 0.0f;  // not resolved inside a graph
      }
      continue;
    }
    rec(0);
    TRY(frame_setup(s, !timed));  // the per-phase timing pass keeps one stream
    rec(1);
    int k = 0;
    double res = 0.0;
    bool have_res = false;
    while (true) {
      TRY(iteration(s, timed, k));
      ++k;
      if (iters > 0) {
        if (k >= iters) break;
      } else {
        TRY(read_residual(s, &res));
        have_res = true;
        if (s->h_pinned[1] || res <= s->opt.ncp_tol || k >= s->opt.max_iters) break;
      }
    }
    rec(2 + 6 * k);
    TRY(finish_frame(s));
    rec(3 + 6 * k);
    if (timed && !have_res) {
      lg::launch_residual(s->d, s->st);
      HIPCHK(hipMemcpyAsync(s->h_res, s->d.res, sizeof(float) * s->d.NS, hipMemcpyDeviceToHost, s->st));
    }
    rec(4 + 6 * k);
    int rc = frame_status(s);
    if (rc != SIM_OK) return rc;
    if (timed) {
      if (!have_res) {
        res = 0.0;
        for (int q = 0; q < s->d.NS; ++q) res = std::max(res, (double)s->h_res[q]);
      }
      auto t1 = std::chrono::steady_clock::now();
      auto& st = stats[f];
      float ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      collect_times(s, k, ms);
      st.iters_done = k;
      st.n_contacts = s->iter_c;
      st.ncp_res = res;
      st.ms_frame = std::chrono::duration<float, std::milli>(t1 - t0).count();
      for (int q = 0; q < 8; ++q) st.ms_phase[q] = ms[q];
    }
  }
  HIPCHK(hipStreamSynchronize(s->st));
  return SIM_OK;
}

int sim_read_state(sim_t s, double* xyz, double* vel, sim_contact* contacts, int32_t cap, int32_t* n_contacts) {
  if (!s || cap < 0) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  if (xyz) TRY(download_nodes(s, s->d.qt, xyz));
  if (vel) TRY(download_nodes(s, s->d.vt, vel));
  int c = 0;
  HIPCHK(hipMemcpyAsync(&c, s->d.pc_count, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  if (n_contacts) *n_contacts = c;
  if (contacts && cap > 0 && c > 0) {
    auto& d = s->d;
    const int CM = d.CMAX;
    std::vector<int> node(c), obst(c);
    std::vector<float> C(9 * (size_t)CM), lam(3 * (size_t)CM);
    std::vector<double> gap(c);
    HIPCHK(hipMemcpyAsync(node.data(), d.pc_node, sizeof(int) * c, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(obst.data(), d.pc_obst, sizeof(int) * c, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(C.data(), d.cC, sizeof(float) * C.size(), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(lam.data(), d.lam, sizeof(float) * lam.size(), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipMemcpyAsync(gap.data(), d.c_gap, sizeof(double) * c, hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    std::vector<int> order(c);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
      int ca = s->iperm_caller[node[a]], cb = s->iperm_caller[node[b]];
      if (ca != cb) return ca < cb;
      return obst[a] < obst[b];
    });
    for (int k = 0; k < std::min(c, cap); ++k) {
      int j = order[k];
      auto& o = contacts[k];
      o.node = s->iperm_caller[node[j]];
      o.obstacle = obst[j] < 0 ? obst[j] : obst[j] - s->scene_obst0[s->obst[obst[j]].scene];
      for (int q = 0; q < 9; ++q) o.frame[q] = C[(size_t)q * CM + j];
      for (int q = 0; q < 3; ++q) o.lambda[q] = lam[(size_t)q * CM + j];
      o.gap = gap[j];
    }
  }
  return SIM_OK;
}

int sim_read_state_device(sim_t s, float* d_xyz, void* stream) {
  if (!s || !d_xyz) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  // device-side scatter through the permutation, ordered after the handle's work
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : s->st;
  if (st != s->st) {
    HIPCHK(hipEventRecord(s->ev[7], s->st));
    HIPCHK(hipStreamWaitEvent(st, s->ev[7], 0));
  }
  lg::launch_export_positions(s->d, st, d_xyz);
  return check_launch("export positions");
}

int sim_destroy(sim_t s) {
  delete s;
  return SIM_OK;
}

int sim_save_state(sim_t s) {
  if (!s) return SIM_E_ARG;
  auto& d = s->d;
  auto& b = s->snap;
  const size_t NV = 3 * (size_t)d.N4, CM = d.CMAX;
  if (!b.qt) {
    TRY(s->alloc(b.qt, NV));
    TRY(s->alloc(b.vt, NV));
    TRY(s->alloc(b.t, 1));
    TRY(s->alloc(b.pc_count, 4));
    TRY(s->alloc(b.pc_node, CM));
    TRY(s->alloc(b.pc_obst, CM));
    TRY(s->alloc(b.pc_world, 3 * CM));
  }
  HIPCHK(hipMemcpyAsync(b.qt, d.qt, NV * sizeof(float), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(b.vt, d.vt, NV * sizeof(float), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(b.t, d.t, sizeof(double), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(b.pc_count, d.pc_count, 2 * sizeof(int), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(b.pc_node, d.pc_node, CM * sizeof(int), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(b.pc_obst, d.pc_obst, CM * sizeof(int), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(b.pc_world, d.pc_world, 3 * CM * sizeof(float), hipMemcpyDeviceToDevice, s->st));
  return SIM_OK;
}

int sim_restore_state(sim_t s) {
  if (!s) return SIM_E_ARG;
  auto& d = s->d;
  auto& b = s->snap;
  if (!b.qt) {
    lg::set_error("no saved state");
    return SIM_E_STATE;
  }
  const size_t NV = 3 * (size_t)d.N4, CM = d.CMAX;
  HIPCHK(hipMemcpyAsync(d.qt, b.qt, NV * sizeof(float), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(d.vt, b.vt, NV * sizeof(float), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(d.t, b.t, sizeof(double), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(d.pc_count, b.pc_count, 2 * sizeof(int), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(d.pc_node, b.pc_node, CM * sizeof(int), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(d.pc_obst, b.pc_obst, CM * sizeof(int), hipMemcpyDeviceToDevice, s->st));
  HIPCHK(hipMemcpyAsync(d.pc_world, b.pc_world, 3 * CM * sizeof(float), hipMemcpyDeviceToDevice, s->st));
  return SIM_OK;
}

// ---------------------------------------------------------------- parity hooks
int sim_set_iterate_state(sim_t s, const double* q_t, const double* v_t, const double* q_k, double t, int32_t c,
                          const sim_contact* contacts) {
  if (!s || !q_t || !v_t || c < 0 || (c > 0 && !contacts) || !std::isfinite(t)) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  auto& d = s->d;
  if (c > d.CMAX) {
    lg::set_error("too many contacts");
    return SIM_E_CAPACITY;
  }
  if (s->scenes.size() != 1) {
    lg::set_error("iterate state applies to single-scene handles");
    return SIM_E_STATE;
  }
  TRY(upload_nodes(s, q_t, d.qt));
  TRY(upload_nodes(s, v_t, d.vt));
  TRY(upload(s, d.t, &t, 1));
  lg::launch_predict(d, s->st);
  lg::launch_pins(d, s->st);
  lg::launch_zero_dual(d, s->st);
  TRY(check_launch("predict"));
  if (q_k) {
    TRY(upload_nodes(s, q_k, d.q));
  } else {  // q^0 = q~ (Alg. 4)
    HIPCHK(hipMemcpyAsync(d.q, d.qp, 3 * (size_t)d.N4 * sizeof(float), hipMemcpyDeviceToDevice, s->st));
  }
  // contact list into internal order (internal node, obstacle)
  std::vector<int> order(c);
  std::iota(order.begin(), order.end(), 0);
  const int T = d.self_on ? d.T : 0;
  int n_self = 0;
  for (int k = 0; k < c; ++k) {
    const int o = contacts[k].obstacle;
    if (contacts[k].node < 0 || contacts[k].node >= d.N || o >= (int)s->obst.size() || o < -T) {
      lg::set_error("bad contact entry");
      return SIM_E_ARG;
    }
    n_self += o < 0;
  }
  // single-node contacts in (internal node, obstacle) order, then the self rows
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const bool sa = contacts[a].obstacle < 0, sb = contacts[b].obstacle < 0;
    if (sa != sb) return sb;
    int na = s->perm_caller[contacts[a].node], nb = s->perm_caller[contacts[b].node];
    if (na != nb) return na < nb;
    return contacts[a].obstacle < contacts[b].obstacle;
  });
  std::vector<int> node(c), obst(c), scene(c, 0);
  std::vector<float> lam(3 * (size_t)d.CMAX, 0.0f);
  s->iter_canon.assign(c, 0);
  for (int j = 0; j < c; ++j) {
    const auto& e = contacts[order[j]];
    node[j] = s->perm_caller[e.node];
    obst[j] = e.obstacle;
    for (int q = 0; q < 3; ++q) lam[q * (size_t)d.CMAX + j] = (float)e.lambda[q];
    s->iter_canon[j] = order[j];
  }
  int cc[2] = {c, 0};
  TRY(upload(s, d.n_contacts, cc, 1));
  if (d.self_on) {
    const int c_obst = c - n_self;
    TRY(upload(s, d.n_obst_c, &c_obst, 1));
  }
  TRY(upload(s, d.c_node, node.data(), c));
  TRY(upload(s, d.c_obst, obst.data(), c));
  TRY(upload(s, d.c_scene, scene.data(), c));
  TRY(upload(s, d.lam, lam.data(), lam.size()));
  s->iter_c = c;
  lg::launch_frames_for_list(d, s->st);
  if (c > 0) {
    lg::launch_delassus(d, s->st);
    lg::launch_warm_start(d, s->st, 1);
    lg::launch_force_ranges(d, s->st);
  }
  TRY(check_launch("iterate state"));
  HIPCHK(hipMemcpyAsync(s->h_pinned + 1, d.overflow, sizeof(int), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  if (s->h_pinned[1]) {
    int zero = 0;
    HIPCHK(hipMemcpyAsync(d.overflow, &zero, sizeof(int), hipMemcpyHostToDevice, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    lg::set_error("Delassus storage capacity exceeded");
    return SIM_E_CAPACITY;
  }
  return SIM_OK;
}

int sim_lg_energy(sim_t s, double* energy) {
  if (!s || !energy) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  if (!kJacobiEnabled) {
    lg::set_error(kJacobiOff);
    return SIM_E_STATE;
  }
  auto& d = s->d;
  const int nb = lg::lg_energy_blocks(d);
  if (!s->energy_part) TRY(s->alloc(s->energy_part, nb));
  lg::launch_lg_energy(d, s->st, s->energy_part);
  TRY(check_launch("objective"));
  std::vector<double> part(nb);
  HIPCHK(hipMemcpyAsync(part.data(), s->energy_part, nb * sizeof(double), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  double e = 0.0;
  for (double p : part) e += p;
  *energy = e;
  return SIM_OK;
}

int sim_run_iterations(sim_t s, int32_t k) {
  if (!s || k < 0) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  TRY(check_global_step(s));
  for (int i = 0; i < k; ++i) TRY(iteration(s, false, i));
  TRY(check_launch("iterations"));
  HIPCHK(hipStreamSynchronize(s->st));
  return SIM_OK;
}

int sim_read_iterate(sim_t s, double* q_k, double* lambda) {
  if (!s) return SIM_E_ARG;
  if (q_k) TRY(download_nodes(s, s->d.q, q_k));
  if (lambda && s->iter_c > 0) {
    auto& d = s->d;
    std::vector<float> lam(3 * (size_t)d.CMAX);
    HIPCHK(hipMemcpyAsync(lam.data(), d.lam, sizeof(float) * lam.size(), hipMemcpyDeviceToHost, s->st));
    HIPCHK(hipStreamSynchronize(s->st));
    std::vector<int> node, obst;
    std::vector<int32_t> order;
    TRY(sort_contacts_canonical(s, s->iter_c, node, obst, order));
    for (int k = 0; k < s->iter_c; ++k)
      for (int q = 0; q < 3; ++q) lambda[3 * (size_t)k + q] = lam[(size_t)q * d.CMAX + order[k]];
  }
  return SIM_OK;
}

int sim_global_solve(sim_t s, const double* b, double* u) {
  if (!s || !b || !u) {
    lg::set_error("bad arguments");
    return SIM_E_ARG;
  }
  auto& d = s->d;
  // uses the b / y iteration buffers as scratch
  TRY(upload_nodes(s, b, d.b));
  lg::launch_spmv_S(d, s->st, d.b, d.y);
  lg::launch_spmv_St(d, s->st, d.y, nullptr, d.tmp);
  TRY(check_launch("global solve"));
  return download_nodes(s, d.tmp, u);
}

int sim_debug_rhs(sim_t s, double* rhs) {
  if (!s || !rhs) return SIM_E_ARG;
  auto& d = s->d;
  lg::launch_element(d, s->st);
  lg::launch_gather(d, s->st);
  TRY(check_launch("rhs"));
  return download_nodes(s, d.b, rhs);
}

int sim_debug_delassus(sim_t s, double* K) {
  if (!s || !K) return SIM_E_ARG;
  int c = s->iter_c;
  if (c == 0) return SIM_OK;
  auto& d = s->d;
  const int ks = lg::kstride(c);
  std::vector<float> Kd((size_t)c * ks);
  HIPCHK(hipMemcpyAsync(Kd.data(), d.K, sizeof(float) * Kd.size(), hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  std::vector<int> node, obst;
  std::vector<int32_t> order;
  TRY(sort_contacts_canonical(s, c, node, obst, order));
  for (int a = 0; a < c; ++a)
    for (int b2 = 0; b2 < c; ++b2) K[(size_t)a * c + b2] = Kd[(size_t)order[a] * ks + order[b2]];
  return SIM_OK;
}

}  // extern "C"
