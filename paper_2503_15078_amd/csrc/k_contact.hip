// Contact kernels: collision detection with order-preserving compaction, contact
// frames (App. A), the Delassus block K = B^T S^T S B (Sec. 5.3, W = H S^T S H^T),
// the complementarity preconditioner (Sec. 5.4), the warm start, the per-iteration
// Fischer-Burmeister evaluation (Sec. 5.2, App. B), the Conjugate Residual solve of
// the Schur system (Sec. 5.2, Sec. 6) and the NCP residual.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "lanes.hpp"
#include "path_sums.hpp"

namespace lg {


// ---------------------------------------------------------------- float64 geometry
// Signed distance and outward normal of an obstacle, in float64, with the operation
// order fixed and no contraction, so that contact decisions are reproducible bit for
// bit by any IEEE implementation following the same order.
__device__ void tangents64(const double n[3], double f1[3], double f2[3]) {
#pragma clang fp contract(off)
  double a0 = fabs(n[0]), a1 = fabs(n[1]), a2 = fabs(n[2]);
  int k = 0;
  if (a1 < (k == 0 ? a0 : a1)) k = 1;
  if (a2 < (k == 0 ? a0 : a1)) k = 2;
  double ek[3] = {0.0, 0.0, 0.0};
  ek[k] = 1.0;
  double dot = n[0] * ek[0] + n[1] * ek[1] + n[2] * ek[2];
  double t0 = ek[0] - dot * n[0], t1 = ek[1] - dot * n[1], t2 = ek[2] - dot * n[2];
  double tn = sqrt(t0 * t0 + t1 * t1 + t2 * t2);
  f1[0] = t0 / tn;
  f1[1] = t1 / tn;
  f1[2] = t2 / tn;
  f2[0] = n[1] * f1[2] - n[2] * f1[1];
  f2[1] = n[2] * f1[0] - n[0] * f1[2];
  f2[2] = n[0] * f1[1] - n[1] * f1[0];
}

__device__ double sdf64(const ObstacleDev& ob, const double x[3], double nrm[3]) {
#pragma clang fp contract(off)
  const double* g = ob.geom;
  if (ob.type == 0) {
    double nn = sqrt(g[3] * g[3] + g[4] * g[4] + g[5] * g[5]);
    nrm[0] = g[3] / nn;
    nrm[1] = g[4] / nn;
    nrm[2] = g[5] / nn;
    return nrm[0] * (x[0] - g[0]) + nrm[1] * (x[1] - g[1]) + nrm[2] * (x[2] - g[2]);
  }
  if (ob.type == 1) {
    double r[3] = {x[0] - g[0], x[1] - g[1], x[2] - g[2]};
    double q[3] = {fabs(r[0]) - g[3], fabs(r[1]) - g[4], fabs(r[2]) - g[5]};
    double sg[3] = {r[0] >= 0.0 ? 1.0 : -1.0, r[1] >= 0.0 ? 1.0 : -1.0, r[2] >= 0.0 ? 1.0 : -1.0};
    double o[3] = {q[0] > 0.0 ? q[0] : 0.0, q[1] > 0.0 ? q[1] : 0.0, q[2] > 0.0 ? q[2] : 0.0};
    double out = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
    if (out > 0.0) {
      for (int c = 0; c < 3; ++c) nrm[c] = o[c] * sg[c] / out;
      return out;
    }
    int ax = 0;
    if (q[1] > q[ax]) ax = 1;
    if (q[2] > q[ax]) ax = 2;
    nrm[0] = nrm[1] = nrm[2] = 0.0;
    nrm[ax] = sg[ax];
    return q[ax];
  }
  // capped cylinder
  double e0 = g[3] - g[0], e1 = g[4] - g[1], e2 = g[5] - g[2];
  double L = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
  double u[3] = {e0 / L, e1 / L, e2 / L};
  double r0 = x[0] - g[0], r1 = x[1] - g[1], r2 = x[2] - g[2];
  double t = r0 * u[0] + r1 * u[1] + r2 * u[2];
  double w0 = r0 - t * u[0], w1 = r1 - t * u[1], w2 = r2 - t * u[2];
  double rho = sqrt(w0 * w0 + w1 * w1 + w2 * w2);
  double dr = rho - g[6];
  double da, s[3];
  if (t < 0.0) {
    da = -t;
    s[0] = -u[0];
    s[1] = -u[1];
    s[2] = -u[2];
  } else {
    da = t - L;
    s[0] = u[0];
    s[1] = u[1];
    s[2] = u[2];
  }
  double wh[3];
  if (rho > 0.0) {
    wh[0] = w0 / rho;
    wh[1] = w1 / rho;
    wh[2] = w2 / rho;
  } else {
    double f2[3];
    tangents64(u, wh, f2);
  }
  if (dr > 0.0 && da > 0.0) {
    double out = sqrt(dr * dr + da * da);
    for (int c = 0; c < 3; ++c) nrm[c] = (dr * wh[c] + da * s[c]) / out;
    return out;
  }
  if (dr > 0.0) {
    for (int c = 0; c < 3; ++c) nrm[c] = wh[c];
    return dr;
  }
  if (da > 0.0) {
    for (int c = 0; c < 3; ++c) nrm[c] = s[c];
    return da;
  }
  if (dr > da) {
    for (int c = 0; c < 3; ++c) nrm[c] = wh[c];
    return dr;
  }
  for (int c = 0; c < 3; ++c) nrm[c] = s[c];
  return da;
}

// contact predicate: min(sdf(q_t), sdf(q~)) < margin with q~ = (q_t + h v_t) + (h h) g in float64;
// a binding (type 3) is active for its own node (internal index in geom[7]) at every frame
__device__ bool in_contact(const Dev& d, const ObstacleDev& ob, int v, double margin) {
#pragma clang fp contract(off)
  if (ob.type == 3) return v == (int)ob.geom[7];
  double xt[3], xp[3], nrm[3];
  double hh = d.h * d.h;
  for (int c = 0; c < 3; ++c) {
    xt[c] = (double)d.qt[c * d.N4 + v];
    xp[c] = (xt[c] + d.h * (double)d.vt[c * d.N4 + v]) + hh * d.g[c];
  }
  double dt = sdf64(ob, xt, nrm);
  double dp = sdf64(ob, xp, nrm);
  return (dt < dp ? dt : dp) < margin;
}

// frame rows (n, f1, f2) at q_t, d_n = n . (x_t - sdf n), d_f = f . u^, gap = sdf(x_t)
// (binding, Sec. 3.2 and App. A bilateral items: n = c / |c|, d_b = n . p^, gap n . x_t - d_b,
// no friction, compliance e in c_comp)
__device__ void write_contact_frame(const Dev& d, int j, int v, const ObstacleDev& ob) {
#pragma clang fp contract(off)
  double xt[3], n[3], f1[3], f2[3];
  for (int c = 0; c < 3; ++c) xt[c] = (double)d.qt[c * d.N4 + v];
  double dist;
  double ph[3];
  if (ob.type == 3) {
    const double* g = ob.geom;
    const double cn = sqrt(g[3] * g[3] + g[4] * g[4] + g[5] * g[5]);
    for (int c = 0; c < 3; ++c) {
      n[c] = g[3 + c] / cn;
      ph[c] = g[c];
    }
    dist = (n[0] * xt[0] + n[1] * xt[1] + n[2] * xt[2]) - (n[0] * ph[0] + n[1] * ph[1] + n[2] * ph[2]);
    d.c_comp[j] = (float)g[6];
  } else {
    dist = sdf64(ob, xt, n);
    for (int c = 0; c < 3; ++c) ph[c] = xt[c] - dist * n[c];
    d.c_comp[j] = -1.0f;
  }
  tangents64(n, f1, f2);
  const double* rows[3] = {n, f1, f2};
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      d.cC[(r * 3 + c) * d.CMAX + j] = (float)rows[r][c];
      d.cC64[(r * 3 + c) * d.CMAX + j] = rows[r][c];
    }
  double dn = n[0] * ph[0] + n[1] * ph[1] + n[2] * ph[2];
  d.c_dn[j] = (float)dn;
  d.c_dn64[j] = dn;
  d.c_df[j] = (float)(f1[0] * ob.vel[0] + f1[1] * ob.vel[1] + f1[2] * ob.vel[2]);
  d.c_df[d.CMAX + j] = (float)(f2[0] * ob.vel[0] + f2[1] * ob.vel[1] + f2[2] * ob.vel[2]);
  d.c_mu[j] = ob.type == 3 ? 0.0f : (float)ob.mu;
  d.c_gap[j] = dist;
}

// ---------------------------------------------------------------- detection + compaction
// exclusive prefix of v over a block of 32 * 64 threads at most (wavefront scans by DPP,
// then the wavefront totals), and the block total in *total
__device__ inline int block_excl_scan_i(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave, nw = blockDim.x / kWave;
  const int incl = wave_incl_scan_i(v);
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  int before = 0, all = 0;
  for (int k = 0; k < nw; ++k) {
    const int x = wsum[k];
    if (k < w) before += x;
    all += x;
  }
  *total = all;
  return before + incl - v;
}

__global__ void k_collide_count(Dev d) {
  __shared__ int wsum[kBlock / kWave];
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0;
  if (v < d.N) {
    int s = d.node_scene[v];
    double margin = d.scene_margin[s];
    for (int o = d.scene_obst0[s]; o < d.scene_obst0[s + 1]; ++o) cnt += in_contact(d, d.obst[o], v, margin);
    d.cnt[v] = cnt;
  }
  int total = 0;
  block_excl_scan_i(cnt, wsum, &total);
  if (threadIdx.x == 0) d.blk[blockIdx.x] = total;
}

// single block: exclusive scan of the per-block counts; total -> n_contacts
__global__ void k_collide_scan(Dev d, int nblk) {
  __shared__ int wsum[1024 / kWave];
  int per = (nblk + 1023) / 1024;
  int b0 = threadIdx.x * per, b1 = min(nblk, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += d.blk[b];
  int total = 0;
  int acc = block_excl_scan_i(s, wsum, &total);
  if (threadIdx.x == 0) {
    d.n_contacts[0] = total;
    if (total > d.CMAX) d.overflow[0] = 1;
  }
  for (int b = b0; b < b1; ++b) {
    int x = d.blk[b];
    d.blk[b] = acc;
    acc += x;
  }
}

__global__ void k_collide_write(Dev d) {
  __shared__ int wsum[kBlock / kWave];
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = v < d.N ? d.cnt[v] : 0;
  int total = 0;
  const int excl = block_excl_scan_i(cnt, wsum, &total);
  if (v >= d.N || cnt == 0) return;
  int j = d.blk[blockIdx.x] + excl;
  int s = d.node_scene[v];
  double margin = d.scene_margin[s];
  for (int o = d.scene_obst0[s]; o < d.scene_obst0[s + 1]; ++o) {
    const ObstacleDev& ob = d.obst[o];
    if (!in_contact(d, ob, v, margin)) continue;
    if (j < d.CMAX) {
      d.c_node[j] = v;
      d.c_obst[j] = o;
      d.c_scene[j] = s;
      write_contact_frame(d, j, v, ob);
    }
    ++j;
  }
}

// per-scene contact ranges, Delassus block offsets and tile offsets
// one block: contacts are sorted by scene, so scene s starts at lower_bound(c_scene, s);
// then prefix sums of the per-scene Delassus block sizes and tile counts
__global__ void k_scene_offsets(Dev d) {
  const int c = min(d.n_contacts[0], d.CMAX);
  for (int s = threadIdx.x; s <= d.NS; s += blockDim.x) {
    int lo = 0, hi = c;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (d.c_scene[mid] < s) lo = mid + 1;
      else hi = mid;
    }
    d.cs_off[s] = (s == d.NS) ? c : lo;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t koff = 0;
    int toff = 0;
    for (int s = 0; s < d.NS; ++s) {
      d.k_off[s] = koff;
      d.tile_off[s] = toff;
      int cs = d.cs_off[s + 1] - d.cs_off[s];
      koff += (int64_t)cs * kstride(cs);
      int T = (obst_end(d, s) - d.cs_off[s] + kDelTile - 1) / kDelTile;  // tiles: single-node contacts
      toff += T * (T + 1) / 2;
    }
    d.k_off[d.NS] = koff;
    d.tile_off[d.NS] = toff;
    if (koff > d.KCAP) d.overflow[0] = 1;
  }
}

// ---------------------------------------------------------------- self contact
// Vertex-triangle rows (Sec. 6: H may couple degrees of freedom of one object; App. A
// contact row on the gap n . (x_v - sum_a w_a x_a)).  Float64 from the float32 state,
// contraction off, dot products summed left to right, as the predicate is specified.
__device__ inline void cross3(const double a[3], const double b[3], double o[3]) {
#pragma clang fp contract(off)
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline double dot3(const double a[3], const double b[3]) {
#pragma clang fp contract(off)
  return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}
// node position at q_t (state 0) or at q~ (state 1) in float64
__device__ inline void pos64(const Dev& d, int v, int state, double x[3]) {
#pragma clang fp contract(off)
  const double hh = d.h * d.h;
  for (int c = 0; c < 3; ++c) {
    x[c] = (double)d.qt[c * d.N4 + v];
    if (state) x[c] = (x[c] + d.h * (double)d.vt[c * d.N4 + v]) + hh * d.g[c];
  }
}
// unit normal of triangle t at `state`: cross(xb - xa, xc - xa) / |.|
__device__ inline void tri_normal(const Dev& d, int t, int state, double n[3]) {
#pragma clang fp contract(off)
  double xa[3], xb[3], xc[3], e1[3], e2[3];
  pos64(d, d.tri_v[t], state, xa);
  pos64(d, d.tri_v[d.T + t], state, xb);
  pos64(d, d.tri_v[2 * d.T + t], state, xc);
  for (int c = 0; c < 3; ++c) {
    e1[c] = xb[c] - xa[c];
    e2[c] = xc[c] - xa[c];
  }
  cross3(e1, e2, n);
  const double len = sqrt(dot3(n, n));
  for (int c = 0; c < 3; ++c) n[c] = n[c] / len;
}
// projection of x onto the plane of triangle t (unit normal n) at `state`: weights
// (wa, wb, wc) / tot into w, signed distance returned; false if a weight is negative
__device__ inline bool tri_project(const Dev& d, int t, int state, const double n[3], const double x[3], double w[3],
                                   double* dist) {
#pragma clang fp contract(off)
  double xa[3], xb[3], xc[3], r[3], p[3];
  pos64(d, d.tri_v[t], state, xa);
  pos64(d, d.tri_v[d.T + t], state, xb);
  pos64(d, d.tri_v[2 * d.T + t], state, xc);
  for (int c = 0; c < 3; ++c) r[c] = x[c] - xa[c];
  const double ds = dot3(n, r);
  for (int c = 0; c < 3; ++c) p[c] = x[c] - ds * n[c];
  double u[3], v[3], cr[3], wr[3];
  const double* P[3][2] = {{xb, xc}, {xc, xa}, {xa, xb}};
  for (int k = 0; k < 3; ++k) {
    for (int c = 0; c < 3; ++c) {
      u[c] = P[k][0][c] - p[c];
      v[c] = P[k][1][c] - p[c];
    }
    cross3(u, v, cr);
    wr[k] = dot3(n, cr);
  }
  const double tot = (wr[0] + wr[1]) + wr[2];
  bool inside = true;
  for (int k = 0; k < 3; ++k) {
    w[k] = wr[k] / tot;
    inside = inside && w[k] >= 0.0;
  }
  *dist = ds;
  return inside;
}
// the self-contact predicate of surface vertex index i and triangle t (tri_n ready)
__device__ bool self_pair(const Dev& d, int i, int t, const double vn[3], double w[3], double* dist_t) {
#pragma clang fp contract(off)
  const int v = d.sv[i];
  if (d.tri_v[t] == v || d.tri_v[d.T + t] == v || d.tri_v[2 * d.T + t] == v) return false;
  double n0[3], n1[3];
  for (int c = 0; c < 3; ++c) {
    n0[c] = d.tri_n[c * d.T + t];
    n1[c] = d.tri_n[(3 + c) * d.T + t];
  }
  if (!(dot3(n0, vn) < 0.0)) return false;
  double x[3], w1[3], ds0, ds1;
  pos64(d, v, 0, x);
  if (!tri_project(d, t, 0, n0, x, w, &ds0)) return false;
  pos64(d, v, 1, x);
  if (!tri_project(d, t, 1, n1, x, w1, &ds1)) return false;
  const double margin = d.scene_margin[0];
  *dist_t = ds0;
  return ds0 > -margin && (ds0 < ds1 ? ds0 : ds1) < margin;
}
// sum of the (unnormalised) cross products of the surface triangles of vertex index i at q_t
__device__ void vertex_normal(const Dev& d, int i, double vn[3]) {
#pragma clang fp contract(off)
  vn[0] = vn[1] = vn[2] = 0.0;
  for (int k = d.vt_ptr[i]; k < d.vt_ptr[i + 1]; ++k) {
    const int t = d.vt_idx[k];
    double xa[3], xb[3], xc[3], e1[3], e2[3], cr[3];
    pos64(d, d.tri_v[t], 0, xa);
    pos64(d, d.tri_v[d.T + t], 0, xb);
    pos64(d, d.tri_v[2 * d.T + t], 0, xc);
    for (int c = 0; c < 3; ++c) {
      e1[c] = xb[c] - xa[c];
      e2[c] = xc[c] - xa[c];
    }
    cross3(e1, e2, cr);
    for (int c = 0; c < 3; ++c) vn[c] = vn[c] + cr[c];
  }
}
// row j: vertex v against triangle t, frame and weights at q_t
__device__ void write_self_row(const Dev& d, int j, int v, int t) {
#pragma clang fp contract(off)
  double n[3], f1[3], f2[3], x[3], w[3], dist;
  tri_normal(d, t, 0, n);
  pos64(d, v, 0, x);
  (void)tri_project(d, t, 0, n, x, w, &dist);
  tangents64(n, f1, f2);
  const double* rows[3] = {n, f1, f2};
  const int CM = d.CMAX;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      d.cC[(r * 3 + c) * CM + j] = (float)rows[r][c];
      d.cC64[(r * 3 + c) * CM + j] = rows[r][c];
    }
  d.c_dn[j] = 0.0f;
  d.c_dn64[j] = 0.0;
  d.c_df[j] = 0.0f;
  d.c_df[CM + j] = 0.0f;
  d.c_mu[j] = d.self_mu;
  d.c_gap[j] = dist;
  d.c_comp[j] = -1.0f;
  const int ent[4] = {v, d.tri_v[t], d.tri_v[d.T + t], d.tri_v[2 * d.T + t]};
  const double sg[4] = {1.0, -w[0], -w[1], -w[2]};
  for (int a = 0; a < 4; ++a) {
    d.ent_node[a * CM + j] = ent[a];
    d.ent_w[a * CM + j] = sg[a];
  }
}

__global__ void k_self_tri(Dev d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.T) return;
  for (int state = 0; state < 2; ++state) {
    double n[3];
    tri_normal(d, t, state, n);
    for (int c = 0; c < 3; ++c) d.tri_n[(3 * state + c) * d.T + t] = n[c];
  }
}

__global__ void k_self_count(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.NSV) return;
  double vn[3], w[3], dist;
  vertex_normal(d, i, vn);
  int cnt = 0;
  for (int t = 0; t < d.T; ++t) cnt += self_pair(d, i, t, vn, w, &dist);
  d.sv_cnt[i] = cnt;
}

// single block: exclusive scan of the per-vertex counts into row offsets after the
// obstacle contacts; the total goes to n_contacts
__global__ void k_self_scan(Dev d) {
  __shared__ int part[1024];
  const int per = (d.NSV + 1023) / 1024;
  const int b0 = threadIdx.x * per, b1 = min(d.NSV, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += d.sv_cnt[b];
  part[threadIdx.x] = s;
  __syncthreads();
  const int c0 = d.n_contacts[0];
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int t = 0; t < 1024; ++t) {
      const int x = part[t];
      part[t] = acc;
      acc += x;
    }
    d.n_obst_c[0] = c0;
    d.n_contacts[0] = c0 + acc;
    if (c0 + acc > d.CMAX) d.overflow[0] = 1;
  }
  __syncthreads();
  int acc = c0 + part[threadIdx.x];
  for (int b = b0; b < b1; ++b) {
    const int x = d.sv_cnt[b];
    d.sv_cnt[b] = acc;
    acc += x;
  }
}

__global__ void k_self_write(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.NSV) return;
  double vn[3], w[3], dist;
  vertex_normal(d, i, vn);
  int j = d.sv_cnt[i];
  const int v = d.sv[i];
  for (int t = 0; t < d.T; ++t) {
    if (!self_pair(d, i, t, vn, w, &dist)) continue;
    if (j < d.CMAX) {
      d.c_node[j] = v;
      d.c_obst[j] = -1 - t;
      d.c_scene[j] = 0;
      write_self_row(d, j, v, t);
    }
    ++j;
  }
}

// Self entries (node, row, sign) of the frame's self rows, sorted by (node, row,
// corner) for the force scatter of the global step: each entry's rank is the number of
// entries before it.
__global__ void k_self_entries(Dev d) {
  const int c = min(d.n_contacts[0], d.CMAX), c0 = min(d.n_obst_c[0], c);
  const int E = 4 * (c - c0);
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) d.se_count[0] = E;
  if (e >= E) return;
  const int CM = d.CMAX;
  const int j = c0 + e / 4, a = e % 4;
  const int node = d.ent_node[a * CM + j];
  int rank = 0;
  for (int f = 0; f < E; ++f) {
    const int jf = c0 + f / 4, af = f % 4, nf = d.ent_node[af * CM + jf];
    rank += (nf < node || (nf == node && f < e)) ? 1 : 0;
  }
  d.se_node[rank] = node;
  d.se_row[rank] = j;
  d.se_w[rank] = (float)d.ent_w[a * CM + j];
}

void launch_self_entries(const Dev& d, hipStream_t st) {
  if (!d.self_on) return;
  hipLaunchKernelGGL(k_self_entries, dim3((4 * d.CMAX + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

void launch_collide(const Dev& d, hipStream_t st) {
  int nblk = (d.N + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_collide_count, dim3(nblk), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_collide_scan, dim3(1), dim3(1024), 0, st, d, nblk);
  hipLaunchKernelGGL(k_collide_write, dim3(nblk), dim3(kBlock), 0, st, d);
  if (d.self_on) {
    const int sblk = (d.NSV + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_self_tri, dim3((d.T + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
    hipLaunchKernelGGL(k_self_count, dim3(sblk), dim3(kBlock), 0, st, d);
    hipLaunchKernelGGL(k_self_scan, dim3(1), dim3(1024), 0, st, d);
    hipLaunchKernelGGL(k_self_write, dim3(sblk), dim3(kBlock), 0, st, d);
  }
  hipLaunchKernelGGL(k_scene_offsets, dim3(1), dim3(64), 0, st, d);
}

// frames for a contact list set from the host (parity hook)
__global__ void k_frames_for_list(Dev d) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int c = min(d.n_contacts[0], d.CMAX);
  if (j >= c) return;
  if (d.c_obst[j] < 0) write_self_row(d, j, d.c_node[j], -1 - d.c_obst[j]);
  else write_contact_frame(d, j, d.c_node[j], d.obst[d.c_obst[j]]);
}

void launch_frames_for_list(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_frames_for_list, dim3((d.CMAX + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_scene_offsets, dim3(1), dim3(64), 0, st, d);
}

// ---------------------------------------------------------------- Delassus block
// K_jk = [A_n^-1]_{v_j v_k} = sum over the common ancestors i of v_j and v_k of
// S_{i v_j} S_{i v_k} (Theorem 1: column v of S lives on the ancestor path of v).
// Contacts are sorted by node (a DFS order of the elimination forest), so the
// depth of LCA(v_j, v_k), j < k, is the minimum over adjacent pairs in [j, k).
__global__ void k_adjacent_lca(Dev d) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int c = min(d.n_contacts[0], d.CMAX);
  if (d.self_on) c = min(c, d.n_obst_c[0]);  // self rows follow, unsorted
  if (i >= c - 1) return;
  if (d.c_scene[i] != d.c_scene[i + 1]) {
    d.ad[i] = -1;
    return;
  }
  int u = d.c_node[i], w = d.c_node[i + 1];
  int a = u, lca = -1;
  while (a != -1) {
    int e = d.chain_end[a];
    if (e >= w) {
      lca = a > w ? a : w;
      break;
    }
    a = d.parent[e];
  }
  d.ad[i] = lca < 0 ? -1 : d.depth[lca];
}

// Persistent tiles of kDelTile x kDelTile contact pairs (upper triangle per scene).
// The column paths of both contacts are staged root-aligned in LDS in chunks; a pair
// accumulates only over its common prefix (its common ancestors).
__global__ void __launch_bounds__(kBlock) k_delassus_tiles(Dev d) {
  // rows padded by 4 floats: 16-byte aligned, and the 16 rows of a float4 read start in
  // distinct bank groups
  __shared__ __align__(16) float PJ[kDelTile][kDelChunk + 4];
  __shared__ __align__(16) float PK[kDelTile][kDelChunk + 4];
  __shared__ int LJK[kDelTile][kDelTile];
  __shared__ int sufJ[kDelTile], preK[kDelTile];
  __shared__ int dJ[kDelTile], dK[kDelTile];
  __shared__ int adJ[kDelTile], adK[kDelTile];
  __shared__ int64_t cJ[kDelTile], cK[kDelTile];
  __shared__ int red[kBlock];
  __shared__ int maxL;
  if (d.k_off[d.NS] > d.KCAP) return;  // Delassus storage full (reported as overflow)
  const int total = d.tile_off[d.NS];
  for (int tile = blockIdx.x; tile < total; tile += gridDim.x) {
    // locate scene and (tj, tk) with tj <= tk
    int s = 0;
    while (d.tile_off[s + 1] <= tile) ++s;
    int cs = d.cs_off[s], cnt = d.cs_off[s + 1] - cs;
    const int co = obst_end(d, s) - cs;  // tiles cover the single-node contacts
    int T = (co + kDelTile - 1) / kDelTile;
    int rem = tile - d.tile_off[s], tj = 0;
    while (rem >= T - tj) {
      rem -= T - tj;
      ++tj;
    }
    int tk = tj + rem;
    int J0 = cs + tj * kDelTile, K0 = cs + tk * kDelTile;
    int nJ = min(kDelTile, cs + co - J0), nK = min(kDelTile, cs + co - K0);
    int tid = threadIdx.x;
    // the adjacent-pair depths inside both contact ranges, ad[J0 .. J0+nJ-2] and
    // ad[K0 .. K0+nK-2], staged once (cross-scene pairs as -1); with the column data
    if (tid < kDelTile) {
      const int j = J0 + tid;
      adJ[tid] = tid < nJ - 1 ? max(d.ad[j], -1) : (1 << 30);
      if (tid < nJ) {
        dJ[tid] = d.depth[d.c_node[j]];
        cJ[tid] = d.col_ptr[d.c_node[j]];
      }
    } else if (tid < 2 * kDelTile) {
      const int r = tid - kDelTile, k = K0 + r;
      adK[r] = r < nK - 1 ? max(d.ad[k], -1) : (1 << 30);
      if (r < nK) {
        dK[r] = d.depth[d.c_node[k]];
        cK[r] = d.col_ptr[d.c_node[k]];
      }
    }
    __syncthreads();
    if (tid < kDelTile) {
      if (tid < nJ) {
        int m = 1 << 30;
        for (int q = tid; q < nJ - 1 && tj != tk; ++q) m = min(m, adJ[q]);
        sufJ[tid] = m;  // min ad[j .. J0+nJ-2] (off-diagonal tiles only)
      }
    } else if (tid < 2 * kDelTile) {
      const int r = tid - kDelTile;
      if (r < nK) {
        int m = 1 << 30;
        for (int q = 0; q < r; ++q) m = min(m, adK[q]);
        preK[r] = m;  // min ad[K0 .. k-1]
      }
    }
    // min over the gap ad[J0+nJ-1 .. K0-1] (includes the boundary pair)
    int gm = 1 << 30;
    if (tj != tk)
      for (int q = J0 + nJ - 1 + tid; q < K0; q += kBlock) gm = min(gm, d.ad[q] < 0 ? -1 : d.ad[q]);
    gm = wave_min_i(gm);
    if ((tid & (kWave - 1)) == 0) red[tid / kWave] = gm;
    __syncthreads();
    int gap_min = red[0];
    for (int w = 1; w < kBlock / kWave; ++w) gap_min = min(gap_min, red[w]);
    int lmax = 0;
    for (int p = tid; p < kDelTile * kDelTile; p += kBlock) {
      int a = p / kDelTile, b = p % kDelTile;
      int L = 0;
      if (a < nJ && b < nK) {
        int j = J0 + a, k = K0 + b;
        if (tj == tk) {
          if (k == j) {
            L = dJ[a] + 1;
          } else if (k > j) {
            int m = 1 << 30;
            for (int q = a; q < b; ++q) m = min(m, adJ[q]);  // min ad[j .. k-1]
            L = m + 1;
          }
        } else {
          int m = min(min(sufJ[a], gap_min), preK[b]);
          L = m + 1;
        }
        if (L < 0) L = 0;
      }
      LJK[a][b] = L;
      lmax = max(lmax, L);
    }
    lmax = wave_max_i(lmax);
    __syncthreads();  // every read of red[] above is done
    if ((tid & (kWave - 1)) == 0) red[tid / kWave] = lmax;
    __syncthreads();
    if (tid == 0) {
      int m = red[0];
      for (int w = 1; w < kBlock / kWave; ++w) m = max(m, red[w]);
      maxL = m;
    }
    __syncthreads();
    // each thread: kPP pairs (a, b0 + r) of the tile
    constexpr int kPP = kDelTile * kDelTile / kBlock;
    constexpr int kCols = kDelTile / kPP;
    const int a = tid / kCols, b0 = (tid % kCols) * kPP;
    float acc[kPP];
    for (int r = 0; r < kPP; ++r) acc[r] = 0.0f;
    for (int base = 0; base < maxL; base += kDelChunk) {
      // all loads of the chunk issued before the LDS stores (one memory round trip); the
      // chunk is not prefetched during the previous one's sums, which would keep the rows'
      // path offsets in registers and cost a wavefront per SIMD on large batches
      constexpr int kPer = kDelTile * kDelChunk / kBlock;
      float vj[kPer], vk[kPer];
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int p = tid + u * kBlock, r = p / kDelChunk, q = p % kDelChunk;
        const int depthidx = base + q;  // 0 = root
        vj[u] = (r < nJ && depthidx <= dJ[r]) ? d.col_val[cJ[r] + (dJ[r] - depthidx)] : 0.0f;
        vk[u] = (r < nK && depthidx <= dK[r]) ? d.col_val[cK[r] + (dK[r] - depthidx)] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < kPer; ++u) {
        const int p = tid + u * kBlock, r = p / kDelChunk, q = p % kDelChunk;
        PJ[r][q] = vj[u];
        PK[r][q] = vk[u];
      }
      __syncthreads();
      for (int r = 0; r < kPP; ++r) {
        const int L = LJK[a][b0 + r] - base;
        const int lim = min(L, kDelChunk), lim4 = max(lim, 0) >> 2;
        const float4* pj = reinterpret_cast<const float4*>(&PJ[a][0]);
        const float4* pk = reinterpret_cast<const float4*>(&PK[b0 + r][0]);
        float sacc = 0.0f;
        for (int q = 0; q < lim4; ++q) {
          const float4 x = pj[q], y = pk[q];
          sacc += x.x * y.x + x.y * y.y + x.z * y.z + x.w * y.w;
        }
        for (int q = 4 * lim4; q < lim; ++q) sacc += PJ[a][q] * PK[b0 + r][q];
        acc[r] += sacc;
      }
      __syncthreads();
    }
    const int64_t ko = d.k_off[s];
    for (int r = 0; r < kPP; ++r) {
      int b = b0 + r;
      if (a < nJ && b < nK) {
        int j = J0 + a - cs, k = K0 + b - cs;
        if (tj != tk || k >= j) {
          d.K[ko + (int64_t)j * kstride(cnt) + k] = acc[r];
          d.K[ko + (int64_t)k * kstride(cnt) + j] = acc[r];
        }
      }
    }
    __syncthreads();
  }
}

// [A_n^-1]_(a b) = sum over the common ancestors i of a and b of S_ia S_ib (Theorem 1),
// one wavefront: the common ancestors are the path from LCA(a, b) to the root, found by
// walking up chains from the smaller node (a subtree is the index range [lo_i, i]).
__device__ float ainv_wave(const Dev& d, int a, int b, int lane) {
  if (a > b) {
    const int t = a;
    a = b;
    b = t;
  }
  int lca = a, x = a;
  while (x != -1) {
    const int e = d.chain_end[x];
    if (e >= b) {
      lca = x > b ? x : b;
      break;
    }
    x = d.parent[e];
  }
  if (x == -1) return 0.0f;  // different trees (other scenes): no common ancestor
  const int D = d.depth[lca], da = d.depth[a], db = d.depth[b];
  const float* ca = d.col_val + d.col_ptr[a];
  const float* cb = d.col_val + d.col_ptr[b];
  float acc = 0.0f;
  for (int t = lane; t <= D; t += kWave) acc += ca[da - t] * cb[db - t];
  return wave_sum(acc);
}

// Delassus entries of the self rows: K_jk = sum_e sum_f s_e s_f [A_n^-1]_(n_e n_f) over
// the entries of row j (vertex and triangle corners) and of row k (one node with sign 1
// for a single-node contact), for every self row j and every row k of the frame; one
// wavefront per pair, both K_jk and K_kj written.
__global__ void __launch_bounds__(kBlock) k_self_delassus(Dev d) {
  if (d.k_off[d.NS] > d.KCAP) return;
  const int c = min(d.n_contacts[0], d.CMAX), c0 = min(d.n_obst_c[0], c);
  const int cs = c - c0, CM = d.CMAX, stride = kstride(c);
  const int64_t pairs = (int64_t)cs * c0 + (int64_t)cs * (cs + 1) / 2;
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t waves = (int64_t)gridDim.x * (kBlock / kWave);
  for (int64_t p = (blockIdx.x * (int64_t)kBlock + threadIdx.x) / kWave; p < pairs; p += waves) {
    int j, k;  // j a self row; k < c0 a contact, or a self row k <= j
    if (p < (int64_t)cs * c0) {
      j = c0 + (int)(p / c0);
      k = (int)(p % c0);
    } else {
      int64_t q = p - (int64_t)cs * c0;
      int r = (int)((sqrt(8.0 * (double)q + 1.0) - 1.0) * 0.5);
      while ((int64_t)(r + 1) * (r + 2) / 2 <= q) ++r;
      while ((int64_t)r * (r + 1) / 2 > q) --r;
      j = c0 + r;
      k = c0 + (int)(q - (int64_t)r * (r + 1) / 2);
    }
    j = __builtin_amdgcn_readfirstlane(j);
    k = __builtin_amdgcn_readfirstlane(k);
    const int nk = k < c0 ? 1 : 4;
    float sum = 0.0f;
    for (int a = 0; a < 4; ++a) {
      const int na = d.ent_node[a * CM + j];
      const float sa = (float)d.ent_w[a * CM + j];
      for (int b = 0; b < nk; ++b) {
        const int nb = k < c0 ? d.c_node[k] : d.ent_node[b * CM + k];
        const float sb = k < c0 ? 1.0f : (float)d.ent_w[b * CM + k];
        sum += sa * sb * ainv_wave(d, na, nb, lane);
      }
    }
    if (lane == 0) {
      d.K[d.k_off[0] + (int64_t)j * stride + k] = sum;
      d.K[d.k_off[0] + (int64_t)k * stride + j] = sum;
    }
  }
}

void launch_delassus(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_adjacent_lca, dim3((d.CMAX + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_delassus_tiles, dim3(1024), dim3(kBlock), 0, st, d);
  if (d.self_on) hipLaunchKernelGGL(k_self_delassus, dim3(1024), dim3(kBlock), 0, st, d);
}

// ---------------------------------------------------------------- warm start + r
// r_n = h^2 K_jj, r_f = h K_jj (W_jj of the normal and tangent rows, Sec. 5.4);
// lambda^0: previous frame's world impulse of the same (node, obstacle) re-expressed
// in the new frame, else 0 (keep_lambda: impulses were set by the host).
__global__ void k_warm_start(Dev d, int keep_lambda) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int c = min(d.n_contacts[0], d.CMAX);
  if (j >= c) return;
  int s = d.c_scene[j];
  int cs = d.cs_off[s], cnt = d.cs_off[s + 1] - cs;
  if (d.k_off[d.NS] > d.KCAP) return;
  float* krow = d.K + d.k_off[s] + (int64_t)(j - cs) * kstride(cnt);
  for (int k = cnt; k < kstride(cnt); ++k) krow[k] = 0.0f;  // pads of this row (storage is reused)
  float kjj = krow[j - cs];
  if (d.precond == 1) {  // [H M^-1 H^T]_jj = 1 / m_v; of a self row, sum_e s_e^2 / m_(n_e)
    if (d.c_obst[j] >= 0) {
      kjj = d.inv_mass[d.c_node[j]];
    } else {
      kjj = 0.0f;
      for (int a = 0; a < 4; ++a) {
        const float w = (float)d.ent_w[a * d.CMAX + j];
        kjj += w * w * d.inv_mass[d.ent_node[a * d.CMAX + j]];
      }
    }
  }
  d.c_rn[j] = (float)(d.h * d.h) * kjj;
  d.c_rf[j] = (float)d.h * kjj;
  if (keep_lambda) return;
  float l[3] = {0.0f, 0.0f, 0.0f};
  if (d.warm >= 1) {  // previous frame (also the fallback and an input of the learned start)
    // saved keys: the single-node contacts sorted by (node, obstacle), then self rows
    const int pc = d.pc_count[0], pco = d.pc_count[1];
    int key_n = d.c_node[j], key_o = d.c_obst[j];
    int lo = 0, hi = pco;
    if (key_o >= 0) {
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int mn = d.pc_node[mid], mo = d.pc_obst[mid];
        if (mn < key_n || (mn == key_n && mo < key_o)) lo = mid + 1;
        else hi = mid;
      }
    } else {
      for (lo = pco; lo < pc && !(d.pc_node[lo] == key_n && d.pc_obst[lo] == key_o); ++lo) {
      }
    }
    if (lo < pc && d.pc_node[lo] == key_n && d.pc_obst[lo] == key_o) {
      float w[3] = {d.pc_world[lo], d.pc_world[d.CMAX + lo], d.pc_world[2 * d.CMAX + lo]};
      for (int r = 0; r < 3; ++r)
        l[r] = d.cC[(r * 3 + 0) * d.CMAX + j] * w[0] + d.cC[(r * 3 + 1) * d.CMAX + j] * w[1] +
               d.cC[(r * 3 + 2) * d.CMAX + j] * w[2];
    }
  }
  for (int r = 0; r < 3; ++r) d.lam[r * d.CMAX + j] = l[r];
}

void launch_warm_start(const Dev& d, hipStream_t st, int keep_lambda) {
  hipLaunchKernelGGL(k_warm_start, dim3((d.CMAX + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d, keep_lambda);
}

// ---------------------------------------------------------------- per-iteration contact terms

struct FBTerms {
  float om_n, E_n, phi_n, om_f, E_f, phi_f[2];
};

// App. B, Fischer-Burmeister rows.  Readings: rho_n = 0 takes omega_n = 1 - 1/sqrt2,
// E_n = (1 - 1/sqrt2) r_n; friction rows are inactive (omega_f = 0, E_f = 1) when
// lambda_n <= 0, mu = 0, or the compliance is infinite; 0/0 gives E_f = 0.
__device__ FBTerms fb_terms(float dn, const float vf[2], const float l[3], float rn, float rf, float mu) {
  FBTerms t;
  float rho = sqrtf(dn * dn + rn * rn * l[0] * l[0]);
  t.phi_n = dn + rn * l[0] - rho;
  if (rho > 0.0f) {
    t.om_n = 1.0f - dn / rho;
    t.E_n = (1.0f - rn * l[0] / rho) * rn;
  } else {
    t.om_n = 1.0f - 0.70710678118654752f;
    t.E_n = (1.0f - 0.70710678118654752f) * rn;
  }
  float s = sqrtf(vf[0] * vf[0] + vf[1] * vf[1]);
  float lf = sqrtf(l[1] * l[1] + l[2] * l[2]);
  float gam = mu * l[0] - lf;
  float rhof = sqrtf(s * s + rf * rf * gam * gam);
  float den = s + mu * rf * l[0] - rhof;
  float num = rhof - rf * gam;
  bool active = (l[0] > 0.0f) && (mu > 0.0f) && !(den == 0.0f && num != 0.0f);
  if (active) {
    t.om_f = 1.0f;
    t.E_f = den != 0.0f ? num / den * rf : 0.0f;
  } else {
    t.om_f = 0.0f;
    t.E_f = 1.0f;
  }
  t.phi_f[0] = t.om_f * vf[0] + t.E_f * l[1];
  t.phi_f[1] = t.om_f * vf[1] + t.E_f * l[2];
  return t;
}

// App. B, minimum-map rows.  Normal: phi_n = delta_n (omega_n = 1, E_n = 0) where
// delta_n <= r_n lambda_n, else r_n lambda_n (omega_n = 0, E_n = r_n).  Friction with
// lambda_n > 0 and mu > 0: omega_f = 1, E_f = 0 while |vdot_f| <= r_f (mu lambda_n -
// |lambda_f|) (stick), else E_f = (|vdot_f| - r_f (mu lambda_n - |lambda_f|)) /
// (mu lambda_n) (slide); otherwise inactive (omega_f = 0, E_f = 1) as in the FB rows.
__device__ FBTerms minmap_terms(float dn, const float vf[2], const float l[3], float rn, float rf, float mu) {
  FBTerms t;
  if (dn <= rn * l[0]) {
    t.phi_n = dn;
    t.om_n = 1.0f;
    t.E_n = 0.0f;
  } else {
    t.phi_n = rn * l[0];
    t.om_n = 0.0f;
    t.E_n = rn;
  }
  const float s = sqrtf(vf[0] * vf[0] + vf[1] * vf[1]);
  const float lf = sqrtf(l[1] * l[1] + l[2] * l[2]);
  const float gam = mu * l[0] - lf;
  if (l[0] > 0.0f && mu > 0.0f) {
    t.om_f = 1.0f;
    t.E_f = s > rf * gam ? (s - rf * gam) / (mu * l[0]) : 0.0f;
  } else {
    t.om_f = 0.0f;
    t.E_f = 1.0f;
  }
  t.phi_f[0] = t.om_f * vf[0] + t.E_f * l[1];
  t.phi_f[1] = t.om_f * vf[1] + t.E_f * l[2];
  return t;
}

// One wavefront per contact: u_v = q~_v + (S^T y)_v along the ancestor path of v
// (column_path_sums; the unconstrained solve A^-1 b at the contact node), then Omega, E~, the h vector
// (Sec. 5.2) and X = C^T (Omega lambda) for the W Omega lambda term of J A^-1 g.
__global__ void __launch_bounds__(kBlock) k_contact_prep(Dev d) {
  if (frame_done(d)) return;
  const int j = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  const int c = min(d.n_contacts[0], d.CMAX);
  if (blockIdx.x == 0)  // barrier flags of the CR launch that follows
    for (int k = threadIdx.x; k < 2 * kCrMaxBlocks; k += blockDim.x) d.cr_sync[k * kCrFlagStride] = 0u;
  if (j >= c) return;
  const int CM = d.CMAX;
  // entries of the row: its node with sign 1, or a self row's vertex and triangle corners
  const bool multi = d.self_on && d.c_obst[j] < 0;
  const int ne = multi ? 4 : 1;
  float x[3] = {0.0f, 0.0f, 0.0f}, xt[3] = {0.0f, 0.0f, 0.0f}, du[3] = {0.0f, 0.0f, 0.0f};
  double dn64 = -d.c_dn64[j];
  for (int a = 0; a < ne; ++a) {
    const int v = __builtin_amdgcn_readfirstlane(multi ? d.ent_node[a * CM + j] : d.c_node[j]);
    const double sg = multi ? d.ent_w[a * CM + j] : 1.0;
    float acc[1][3];
    column_path_sums<1>(d, d.y, v, 1, lane, acc);
    const float ax = wave_sum(acc[0][0]), ay = wave_sum(acc[0][1]), az = wave_sum(acc[0][2]);
    float xa[3], xta[3], dua[3];
    for (int q = 0; q < 3; ++q) {
      xa[q] = d.q[q * d.N4 + v];
      xta[q] = d.qt[q * d.N4 + v];
    }
    // u - x^k = (q~ - x^k) + (S^T y)_v: a difference of nearby values, kept small
    dua[0] = (d.qp[v] - xa[0]) + ax;
    dua[1] = (d.qp[d.N4 + v] - xa[1]) + ay;
    dua[2] = (d.qp[2 * d.N4 + v] - xa[2]) + az;
    // delta_n = n . x - d_n in float64 (absolute coordinates, small difference)
    dn64 += sg * (d.cC64[0 * CM + j] * (double)xa[0] + d.cC64[1 * CM + j] * (double)xa[1] +
                  d.cC64[2 * CM + j] * (double)xa[2]);
    const float sf = (float)sg;
    for (int q = 0; q < 3; ++q) {
      x[q] += sf * xa[q];
      xt[q] += sf * xta[q];
      du[q] += sf * dua[q];
    }
  }
  if (lane != 0) return;
  const float h = (float)d.h;
  float C[3][3];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) C[r][q] = d.cC[(r * 3 + q) * CM + j];
  float l[3] = {d.lam[j], d.lam[CM + j], d.lam[2 * CM + j]};
  float dn = (float)dn64;
  float hvf[2];
  for (int r = 0; r < 2; ++r)
    hvf[r] = C[r + 1][0] * (x[0] - xt[0]) + C[r + 1][1] * (x[1] - xt[1]) + C[r + 1][2] * (x[2] - xt[2]) -
             h * d.c_df[r * CM + j];
  float vf[2] = {hvf[0] / h, hvf[1] / h};
  FBTerms f = d.ncp == 1 ? minmap_terms(dn, vf, l, d.c_rn[j], d.c_rf[j], d.c_mu[j])
                         : fb_terms(dn, vf, l, d.c_rn[j], d.c_rf[j], d.c_mu[j]);
  const float comp = d.c_comp[j];
  if (comp >= 0.0f) {  // bilateral row: phi_b = delta_b + e lambda_b; tangent rows inactive
    f.phi_n = dn + comp * l[0];
    f.om_n = 1.0f;
    f.E_n = comp;
    f.om_f = 0.0f;
    f.E_f = 1.0f;
    f.phi_f[0] = l[1];
    f.phi_f[1] = l[2];
  }
  float om[3] = {f.om_n, f.om_f, f.om_f};
  d.Om[j] = om[0];
  d.Om[CM + j] = om[1];
  d.Om[2 * CM + j] = om[2];
  d.Et[j] = f.E_n / (h * h);
  d.Et[CM + j] = f.E_f / h;
  d.Et[2 * CM + j] = f.E_f / h;
  // h_vec - Omega H u = -(phi_n, h phi_f) - Omega C (u - x^k)   (Sec. 5.2, with H q^k cancelled)
  float Cdu[3];
  for (int r = 0; r < 3; ++r) Cdu[r] = C[r][0] * du[0] + C[r][1] * du[1] + C[r][2] * du[2];
  d.hv[j] = -f.phi_n - om[0] * Cdu[0];
  d.hv[CM + j] = -h * f.phi_f[0] - om[1] * Cdu[1];
  d.hv[2 * CM + j] = -h * f.phi_f[1] - om[2] * Cdu[2];
  float ol[3] = {om[0] * l[0], om[1] * l[1], om[2] * l[2]};
  for (int q = 0; q < 3; ++q) d.X[q * CM + j] = C[0][q] * ol[0] + C[1][q] * ol[1] + C[2][q] * ol[2];
}

void launch_contact_prep(const Dev& d, hipStream_t st) {
  int waves_per_block = kBlock / kWave;
  hipLaunchKernelGGL(k_contact_prep, dim3((d.CMAX + waves_per_block - 1) / waves_per_block), dim3(kBlock), 0,
                     st, d);
}

// ---------------------------------------------------------------- NCP residual (metres)
// Residual of contact j with node position x and impulse l (contact frame): |FB(delta_n,
// r_n lambda_n)|, and for lambda_n > 0 h |FB(s, r_f gamma)| and h |vdot_f + s
// lambda_f/|lambda_f||, else h r_f |lambda_f|; a bilateral row takes |delta_b + e
// lambda_b| and its inactive tangent rows.  NaN counts as huge.
// Point of row j in positions `base` ([3][N4] float): its node's position, or for a self
// row the signed sum of its entries x_v - sum_a w_a x_a (float64 normal gap below).
__device__ void row_point(const Dev& d, int j, const float* base, float x[3]) {
  if (d.self_on && d.c_obst[j] < 0) {
    for (int q = 0; q < 3; ++q) x[q] = 0.0f;
    for (int a = 0; a < 4; ++a) {
      const int v = d.ent_node[a * d.CMAX + j];
      const float sg = (float)d.ent_w[a * d.CMAX + j];
      for (int q = 0; q < 3; ++q) x[q] += sg * base[q * d.N4 + v];
    }
    return;
  }
  const int v = d.c_node[j];
  for (int q = 0; q < 3; ++q) x[q] = base[q * d.N4 + v];
}

__device__ float contact_residual(const Dev& d, int j, const float x[3], const float xt[3], const float l[3]) {
  const int CM = d.CMAX;
  const float h = (float)d.h;
  float C[3][3];
  for (int r = 0; r < 3; ++r)
    for (int q = 0; q < 3; ++q) C[r][q] = d.cC[(r * 3 + q) * CM + j];
  float dn = (float)(d.cC64[0 * CM + j] * (double)x[0] + d.cC64[1 * CM + j] * (double)x[1] +
                     d.cC64[2 * CM + j] * (double)x[2] - d.c_dn64[j]);
  float vf[2];
  for (int r = 0; r < 2; ++r)
    vf[r] = (C[r + 1][0] * (x[0] - xt[0]) + C[r + 1][1] * (x[1] - xt[1]) + C[r + 1][2] * (x[2] - xt[2]) -
             h * d.c_df[r * CM + j]) / h;
  float rn = d.c_rn[j], rf = d.c_rf[j], mu = d.c_mu[j];
  float a = rn * l[0];
  float res = fabsf(dn + a - sqrtf(dn * dn + a * a));
  float s = sqrtf(vf[0] * vf[0] + vf[1] * vf[1]);
  float lf = sqrtf(l[1] * l[1] + l[2] * l[2]);
  const float comp = d.c_comp[j];
  if (comp >= 0.0f) {  // bilateral row and its inactive tangent rows
    res = fmaxf(fabsf(dn + comp * l[0]), h * rf * lf);
  } else if (l[0] > 0.0f) {
    float b = rf * (mu * l[0] - lf);
    res = fmaxf(res, h * fabsf(s + b - sqrtf(s * s + b * b)));
    if (lf > 0.0f) {
      float e0 = vf[0] + s * l[1] / lf, e1 = vf[1] + s * l[2] / lf;
      res = fmaxf(res, h * sqrtf(e0 * e0 + e1 * e1));
    }
  } else {
    res = fmaxf(res, h * rf * lf);
  }
  if (!(res == res)) res = 3.0e38f;  // NaN -> huge
  return res;
}

// max over contacts of the residual at the current iterate (q, lambda), per scene
__global__ void k_residual(Dev d) {
  if (frame_done(d)) return;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int c = min(d.n_contacts[0], d.CMAX);
  if (j >= c) return;
  const int CM = d.CMAX;
  float x[3], xt[3], l[3];
  row_point(d, j, d.q, x);
  row_point(d, j, d.qt, xt);
  for (int q = 0; q < 3; ++q) l[q] = d.lam[q * CM + j];
  atomicMax(reinterpret_cast<unsigned int*>(d.res) + d.c_scene[j],
            __float_as_uint(contact_residual(d, j, x, xt, l)));
}

__global__ void k_zero_res(Dev d) {
  if (frame_done(d)) return;
  for (int s = threadIdx.x; s < d.NS; s += blockDim.x) d.res[s] = 0.0f;
}

// After the residual of an iteration of a frame iterated to tolerance: count it and mark
// the frame done once every scene's residual is within the tolerance, the iteration cap
// is reached, or the frame failed (capacity, non-finite state, abandoned CR barrier).
__global__ void k_convergence_check(Dev d) {
  if (threadIdx.x != 0 || *d.done) return;
  const int k = ++d.iter_count[0];
  float w = 0.0f;
  for (int s = 0; s < d.NS; ++s) w = fmaxf(w, d.res[s]);
  if (w <= d.ncp_tol || k >= d.max_iters || d.overflow[0] || d.bad[0] || d.bad[1]) *d.done = 1;
}

__global__ void k_reset_convergence(Dev d) {
  if (threadIdx.x == 0) {
    *d.done = 0;
    *d.iter_count = 0;
  }
}

void launch_reset_convergence(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_reset_convergence, dim3(1), dim3(kWave), 0, st, d);
}

void launch_convergence_check(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_convergence_check, dim3(1), dim3(kWave), 0, st, d);
}

void launch_residual(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_res, dim3(1), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_residual, dim3((d.CMAX + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

// ---------------------------------------------------------------- judge of the learned start
// The paper leaves the frame's start impulse open.  Two candidates exist when the warm
// start is learned: the previous-frame impulse (lambda) and the network's (lam_ml).  Each
// is judged by the NCP residual it leaves in the frame start's linear contact problem:
// positions x_v = q~_v + h^2 sum_k K_jk C_k^T lambda_k (the predicted state moved by the
// impulses through A^-1, Sec. 5.3), velocities from x - q_t.  Per scene, the learned
// candidate is kept only if its largest residual is strictly below the plain one's.

// world impulses C^T lambda of both candidates; judge values zeroed
__global__ void k_warm_world(Dev d) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < 2 * d.NS) d.judge[j] = 0.0f;
  const int c = min(d.n_contacts[0], d.CMAX);
  if (j >= c) return;
  const int CM = d.CMAX;
  for (int q = 0; q < 3; ++q) {
    float wp = 0.0f, wm = 0.0f;
    for (int r = 0; r < 3; ++r) {
      const float cr = d.cC[(r * 3 + q) * CM + j];
      wp += cr * d.lam[r * CM + j];
      wm += cr * d.lam_ml[r * CM + j];
    }
    d.wl[q * CM + j] = wp;
    d.wl[(3 + q) * CM + j] = wm;
  }
}

// one wavefront per contact row j of its scene's Delassus block
__global__ void __launch_bounds__(kBlock) k_warm_judge(Dev d) {
  const int j = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  const int c = min(d.n_contacts[0], d.CMAX);
  if (j >= c || d.k_off[d.NS] > d.KCAP) return;
  const int CM = d.CMAX, sc = d.c_scene[j], cs = d.cs_off[sc], cnt = d.cs_off[sc + 1] - cs;
  const float* krow = d.K + d.k_off[sc] + (int64_t)(j - cs) * kstride(cnt);
  float w[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for (int k = lane; k < cnt; k += kWave) {
    const float kk = krow[k];
    for (int q = 0; q < 6; ++q) w[q] += kk * d.wl[q * CM + cs + k];
  }
  for (int q = 0; q < 6; ++q) w[q] = wave_sum(w[q]);
  if (lane != 0) return;
  const float h2 = (float)(d.h * d.h);
  float xp[3], xm[3], lp[3], lm[3], base[3], xt[3];
  row_point(d, j, d.qp, base);
  row_point(d, j, d.qt, xt);
  for (int q = 0; q < 3; ++q) {
    xp[q] = base[q] + h2 * w[q];
    xm[q] = base[q] + h2 * w[3 + q];
    lp[q] = d.lam[q * CM + j];
    lm[q] = d.lam_ml[q * CM + j];
  }
  unsigned* jd = reinterpret_cast<unsigned*>(d.judge);
  atomicMax(jd + sc, __float_as_uint(contact_residual(d, j, xp, xt, lp)));
  atomicMax(jd + d.NS + sc, __float_as_uint(contact_residual(d, j, xm, xt, lm)));
}

__global__ void k_warm_select(Dev d) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = min(d.n_contacts[0], d.CMAX);
  if (j >= c || d.k_off[d.NS] > d.KCAP) return;
  const int sc = d.c_scene[j], CM = d.CMAX;
  if (d.judge[d.NS + sc] < d.judge[sc])
    for (int q = 0; q < 3; ++q) d.lam[q * CM + j] = d.lam_ml[q * CM + j];
}

void launch_warm_judge(const Dev& d, hipStream_t st) {
  const int blocks = (max(d.CMAX, 2 * d.NS) + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_warm_world, dim3(blocks), dim3(kBlock), 0, st, d);
  const int waves_per_block = kBlock / kWave;
  hipLaunchKernelGGL(k_warm_judge, dim3((d.CMAX + waves_per_block - 1) / waves_per_block), dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_warm_select, dim3((d.CMAX + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

}  // namespace lg
