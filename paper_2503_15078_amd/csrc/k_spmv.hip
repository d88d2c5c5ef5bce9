// The global step as two passes over the sparse inverse (Sec. 4.2, Algorithm 2):
// y = S b over the row-skyline storage and u = S^T y over the column-path storage,
// plus the sparse contact-force update y += S (h^2 H^T Omega lambda) used by the
// constrained global step (Eq. rhs correction, Algorithm 4).
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "lanes.hpp"
#include "path_sums.hpp"

namespace lg {

// One wavefront per segment of a row group.  Row i is stored over columns
// [lo4_i, hi4_i) in 16-byte groups; the rows of a group share lo4, so one float4 of
// each b coordinate serves every row of the group and only the S values are per row.
// Rows end at their own quad (the last row of a group ends last); quads beyond a row's
// end count as zero.  Single-segment groups write y directly; the others write partial
// sums per row.
template <int G>
__global__ void __launch_bounds__(kBlock) k_spmv_S(Dev d, const float* __restrict__ b, float* __restrict__ y) {
  if (frame_done(d)) return;
  const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  if (wave >= d.nseg) return;
  const int r = d.seg_row[wave];
  const int i0 = r >= 0 ? r : -r - 1;
  const int ng = d.seg_ng[wave], q0 = d.seg_q0[wave];
  const int nq = d.seg_len[wave] >> 2;
  const int col0 = d.seg_col0[wave];
  const int64_t off0 = d.seg_off[wave];
  // row i0 + g is stored over quads [lo4 / 4, (i0 + g) / 4 + 1): its length and its
  // offset from row i0 follow from the indices alone
  const int lo4q = (col0 >> 2) - q0;
  const float4* S4[G];
  int n4[G];
  int64_t rel = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int len4 = ((i0 + g) >> 2) + 1 - lo4q;
    n4[g] = g < ng ? min(nq, len4 - q0) : 0;
    S4[g] = reinterpret_cast<const float4*>(d.row_val + off0 + rel);
    rel += 4 * (int64_t)len4;
  }
  const float4* __restrict__ bx = reinterpret_cast<const float4*>(b + col0);
  const float4* __restrict__ by = reinterpret_cast<const float4*>(b + d.N4 + col0);
  const float4* __restrict__ bz = reinterpret_cast<const float4*>(b + 2 * d.N4 + col0);
  float acc[G][3];
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g][0] = acc[g][1] = acc[g][2] = 0.0f;
#pragma unroll(G <= 2 ? 4 : 2)
  for (int q = lane; q < nq; q += kWave) {
    const float4 x = bx[q], yy = by[q], z = bz[q];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (n4[g] > 0) {  // uniform: the row has quads in this segment
        float4 sv;
        if constexpr (G == 1) {  // a lone row spans its whole segment
          sv = S4[g][q];
        } else {
          sv = S4[g][min(q, n4[g] - 1)];
          if (q >= n4[g]) sv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        acc[g][0] += dot4(sv, x);
        acc[g][1] += dot4(sv, yy);
        acc[g][2] += dot4(sv, z);
      }
    }
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (g < ng) {
      const float ax = wave_sum(acc[g][0]), ay = wave_sum(acc[g][1]), az = wave_sum(acc[g][2]);
      if (lane == 0) {
        if (r >= 0) {
          y[i0 + g] = ax;
          y[d.N4 + i0 + g] = ay;
          y[2 * d.N4 + i0 + g] = az;
        } else {
          d.partial[(0 * G + g) * (int64_t)d.nseg + wave] = ax;
          d.partial[(1 * G + g) * (int64_t)d.nseg + wave] = ay;
          d.partial[(2 * G + g) * (int64_t)d.nseg + wave] = az;
        }
      }
    }
  }
}

// Row groups of several segments: y_i = sum of the row's partials, in segment order.
// One thread per (group, coordinate, row of the group); the first eight partials are
// loaded together before the ordered sum.
__global__ void k_spmv_S_finish(Dev d, float* __restrict__ y) {
  if (frame_done(d)) return;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int G = d.row_group;
  if (t >= d.nlong * 3 * G) return;
  const int l = t / (3 * G), c = (t / G) % 3, g = t % G;
  if (g >= d.long_ng[l]) return;
  const int s0 = d.long_seg0[l], ns = d.long_nseg[l], i0 = d.long_row[l];
  const float* p = d.partial + (c * G + g) * (int64_t)d.nseg + s0;
  float v[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) v[k] = k < ns ? p[k] : 0.0f;
  float a = v[0];
#pragma unroll
  for (int k = 1; k < 8; ++k)
    if (k < ns) a += v[k];
  for (int k = 8; k < ns; ++k) a += p[k];
  y[c * d.N4 + i0 + g] = a;
}

void launch_spmv_S(const Dev& d, hipStream_t st, const float* b, float* y) {
  const dim3 grid((d.nseg + kBlock / kWave - 1) / (kBlock / kWave));
  switch (d.row_group) {
    case 1: hipLaunchKernelGGL(k_spmv_S<1>, grid, dim3(kBlock), 0, st, d, b, y); break;
    case 2: hipLaunchKernelGGL(k_spmv_S<2>, grid, dim3(kBlock), 0, st, d, b, y); break;
    case 4: hipLaunchKernelGGL(k_spmv_S<4>, grid, dim3(kBlock), 0, st, d, b, y); break;
    default: hipLaunchKernelGGL(k_spmv_S<8>, grid, dim3(kBlock), 0, st, d, b, y); break;
  }
  if (d.nlong > 0)
    hipLaunchKernelGGL(k_spmv_S_finish, dim3((d.nlong * 3 * d.row_group + kBlock - 1) / kBlock), dim3(kBlock), 0,
                       st, d, y);
}

// One wavefront per group of up to G consecutive columns j0 .. j0 + ng - 1 of one
// chain: u_j = base_j + sum over the ancestors i of j of S_ij y_i (column_path_sums).
template <int G>
__global__ void __launch_bounds__(kBlock) k_spmv_St(Dev d, const float* __restrict__ y,
                                                    const float* __restrict__ base, float* __restrict__ u) {
  if (frame_done(d)) return;
  const int w = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  if (w >= d.n_stgrp) return;
  const int j0 = d.stgrp_j0[w], ng = d.stgrp_ng[w];
  float acc[G][3];
  column_path_sums<G>(d, y, j0, ng, lane, acc);
#pragma unroll
  for (int g = 0; g < G; ++g) {
    if (g < ng) {
      const float ax = wave_sum(acc[g][0]), ay = wave_sum(acc[g][1]), az = wave_sum(acc[g][2]);
      if (lane == 0) {
        const int j = j0 + g;
        u[j] = (base ? base[j] : 0.0f) + ax;
        u[d.N4 + j] = (base ? base[d.N4 + j] : 0.0f) + ay;
        u[2 * d.N4 + j] = (base ? base[2 * d.N4 + j] : 0.0f) + az;
      }
    }
  }
}

void launch_spmv_St(const Dev& d, hipStream_t st, const float* y, const float* base, float* u) {
  const dim3 grid((d.n_stgrp + kBlock / kWave - 1) / (kBlock / kWave));
  switch (d.col_group) {
    case 1: hipLaunchKernelGGL(k_spmv_St<1>, grid, dim3(kBlock), 0, st, d, y, base, u); break;
    case 2: hipLaunchKernelGGL(k_spmv_St<2>, grid, dim3(kBlock), 0, st, d, y, base, u); break;
    case 4: hipLaunchKernelGGL(k_spmv_St<4>, grid, dim3(kBlock), 0, st, d, y, base, u); break;
    default: hipLaunchKernelGGL(k_spmv_St<8>, grid, dim3(kBlock), 0, st, d, y, base, u); break;
  }
}

// y_i += sum over contacts k whose node lies in the subtree [lo_i, i] of row i of
// S_{i,v_k} F_k, with F_k = h^2 C_k^T (Omega_k lambda_k) the world-space contact
// force.  Contacts are sorted by node, so each row sees a contiguous range; one
// wavefront per row, deterministic.
__device__ inline int lower_bound_i(const int* a, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Per frame: the contact range [cb, ce) of every row (contacts are sorted by node), and
// with self contact the range of the sorted self-row entries.
__global__ void k_force_ranges(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.N) return;
  int c = min(d.n_contacts[0], d.CMAX);
  if (d.self_on) {
    c = min(c, d.n_obst_c[0]);
    const int E = d.se_count[0];
    d.frange2[i] = lower_bound_i(d.se_node, E, d.lo[i]);
    d.frange2[d.N + i] = lower_bound_i(d.se_node, E, i + 1);
  }
  d.frange[i] = lower_bound_i(d.c_node, c, d.lo[i]);
  d.frange[d.N + i] = lower_bound_i(d.c_node, c, i + 1);
}

void launch_force_ranges(const Dev& d, hipStream_t st) {
  launch_self_entries(d, st);
  hipLaunchKernelGGL(k_force_ranges, dim3((d.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

// One wavefront per row; rows without contacts in their subtree exit at once.
__global__ void __launch_bounds__(kBlock) k_apply_forces(Dev d) {
  if (frame_done(d)) return;
  const int i = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  if (i >= d.N) return;
  const int cb = __builtin_amdgcn_readfirstlane(d.frange[i]);
  const int ce = __builtin_amdgcn_readfirstlane(d.frange[d.N + i]);
  const int sb = d.self_on ? __builtin_amdgcn_readfirstlane(d.frange2[i]) : 0;
  const int se = d.self_on ? __builtin_amdgcn_readfirstlane(d.frange2[d.N + i]) : 0;
  if (cb >= ce && sb >= se) return;
  const float* row = d.row_val + d.row_ptr[i];
  const int lo4 = d.row_lo4[i];
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
  // four contacts per lane in flight (a row high in the tree holds every contact below it);
  // each lane still adds its contacts in index order
  constexpr int U = 4;
  for (int k0 = cb + lane; k0 < ce; k0 += U * kWave) {
    int node[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * kWave;
      node[u] = k < ce ? d.c_node[k] : lo4;
    }
    float s[U], f[U][3];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = k0 + u * kWave;
      const bool in = k < ce;
      s[u] = in ? row[node[u] - lo4] : 0.0f;
      f[u][0] = in ? d.F[k] : 0.0f;
      f[u][1] = in ? d.F[d.CMAX + k] : 0.0f;
      f[u][2] = in ? d.F[2 * d.CMAX + k] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (k0 + u * kWave < ce) {
        ax += s[u] * f[u][0];
        ay += s[u] * f[u][1];
        az += s[u] * f[u][2];
      }
    }
  }
  for (int k = sb + lane; k < se; k += kWave) {  // entries of self rows: s_e F_row
    const int r = d.se_row[k];
    const float s = row[d.se_node[k] - lo4] * d.se_w[k];
    ax += s * d.F[r];
    ay += s * d.F[d.CMAX + r];
    az += s * d.F[2 * d.CMAX + r];
  }
  ax = wave_sum(ax);
  ay = wave_sum(ay);
  az = wave_sum(az);
  if (lane == 0) {
    d.y[i] += ax;
    d.y[d.N4 + i] += ay;
    d.y[2 * d.N4 + i] += az;
  }
}

void launch_apply_forces(const Dev& d, hipStream_t st) {
  int waves_per_block = kBlock / kWave;
  hipLaunchKernelGGL(k_apply_forces, dim3((d.N + waves_per_block - 1) / waves_per_block), dim3(kBlock), 0, st, d);
}

// Incomplete global step (the baseline of Sec. 7's convergence comparison): one Jacobi
// sweep q <- q + D^-1 (b - A q) from the current iterate.  In the delta form used here
// (b' = b - A q~, dq = q - q~) it reads u = q~ + dq + D^-1 (b' - A dq).  One thread per
// node computes u into tmp; a second kernel copies it to q, so every thread reads the
// old iterate.
__global__ void k_jacobi_global(Dev d) {
  if (frame_done(d)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.N) return;
  const int p0 = d.a_ptr[i], p1 = d.a_ptr[i + 1];
  for (int c = 0; c < 3; ++c) {
    const float* q = d.q + c * d.N4;
    const float* qp = d.qp + c * d.N4;
    float adq = 0.0f;
    for (int p = p0; p < p1; ++p) {
      const int j = d.a_idx[p];
      adq += d.a_val[p] * (q[j] - qp[j]);
    }
    const float dq = q[i] - qp[i];
    d.tmp[c * d.N4 + i] = qp[i] + (dq + (d.b[c * d.N4 + i] - adq) * d.a_dinv[i]);
  }
}

__global__ void k_copy_iterate(Dev d) {
  if (frame_done(d)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.N) return;
  for (int c = 0; c < 3; ++c) d.q[c * d.N4 + i] = d.tmp[c * d.N4 + i];
}

void launch_jacobi_global(const Dev& d, hipStream_t st) {
  const dim3 grid((d.N + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_jacobi_global, grid, dim3(kBlock), 0, st, d);
  hipLaunchKernelGGL(k_copy_iterate, grid, dim3(kBlock), 0, st, d);
}

}  // namespace lg
