// The global step as two passes over the sparse inverse (Sec. 4.2, Algorithm 2):
// y = S b over the row-skyline storage and u = S^T y over the column-path storage,
// plus the sparse contact-force update y += S (h^2 H^T Omega lambda) used by the
// constrained global step (Eq. rhs correction, Algorithm 4).
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace lg {

__device__ inline float wave_sum(float v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// One wavefront per row segment.  Row i is stored over columns [lo4_i, hi4_i) in
// 16-byte groups, so S and the three b coordinates are read as aligned float4.
// Single-segment rows write y directly; segments of long rows write partial sums.
__global__ void __launch_bounds__(kBlock) k_spmv_S(Dev d, const float* __restrict__ b, float* __restrict__ y) {
  const int wave = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  if (wave >= d.nseg) return;
  const int row = d.seg_row[wave];
  const int64_t off = d.seg_off[wave];
  const int col0 = d.seg_col0[wave];
  const int len4 = d.seg_len[wave] >> 2;
  const float4* __restrict__ S4 = reinterpret_cast<const float4*>(d.row_val + off);
  const float4* __restrict__ bx = reinterpret_cast<const float4*>(b + col0);
  const float4* __restrict__ by = reinterpret_cast<const float4*>(b + d.N4 + col0);
  const float4* __restrict__ bz = reinterpret_cast<const float4*>(b + 2 * d.N4 + col0);
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
#pragma unroll 4
  for (int q = lane; q < len4; q += kWave) {
    float4 s = S4[q];
    float4 x = bx[q], yy = by[q], z = bz[q];
    ax += s.x * x.x + s.y * x.y + s.z * x.z + s.w * x.w;
    ay += s.x * yy.x + s.y * yy.y + s.z * yy.z + s.w * yy.w;
    az += s.x * z.x + s.y * z.y + s.z * z.z + s.w * z.w;
  }
  ax = wave_sum(ax);
  ay = wave_sum(ay);
  az = wave_sum(az);
  if (lane == 0) {
    if (row >= 0) {
      y[row] = ax;
      y[d.N4 + row] = ay;
      y[2 * d.N4 + row] = az;
    } else {
      d.partial[wave] = ax;
      d.partial[d.nseg + wave] = ay;
      d.partial[2 * d.nseg + wave] = az;
    }
  }
}

// Rows longer than one segment: y_i = sum of their partials, in segment order.
__global__ void k_spmv_S_finish(Dev d, float* __restrict__ y) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= d.nlong) return;
  int s0 = d.long_seg0[l], ns = d.long_nseg[l], row = d.long_row[l];
  for (int c = 0; c < 3; ++c) {
    float a = 0.0f;
    for (int s = 0; s < ns; ++s) a += d.partial[c * d.nseg + s0 + s];
    y[c * d.N4 + row] = a;
  }
}

void launch_spmv_S(const Dev& d, hipStream_t st, const float* b, float* y) {
  int waves_per_block = kBlock / kWave;
  hipLaunchKernelGGL(k_spmv_S, dim3((d.nseg + waves_per_block - 1) / waves_per_block), dim3(kBlock), 0, st,
                     d, b, y);
  if (d.nlong > 0)
    hipLaunchKernelGGL(k_spmv_S_finish, dim3((d.nlong + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d, y);
}

// One wavefront per column j: u_j = base_j + sum over the ancestors i of j of
// S_ij y_i.  The ancestor path is a list of chain runs [a, e] (precomputed per column,
// read with one vector load and broadcast lane by lane, so no load waits on the tree
// walk); the pass reads the aligned copy of the columns (each run stored from node
// a & ~3, zero-padded to whole 4-node groups), so S values and the three y coordinates
// are loaded as 16-byte vectors.
__global__ void __launch_bounds__(kBlock) k_spmv_St(Dev d, const float* __restrict__ y,
                                                    const float* __restrict__ base, float* __restrict__ u) {
  const int j = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  if (j >= d.N) return;
  const float4* __restrict__ col = reinterpret_cast<const float4*>(d.colp_val + d.colp_ptr[j]);
  const float4* __restrict__ y0 = reinterpret_cast<const float4*>(y);
  const float4* __restrict__ y1 = reinterpret_cast<const float4*>(y + d.N4);
  const float4* __restrict__ y2 = reinterpret_cast<const float4*>(y + 2 * d.N4);
  const int rb = d.run_ptr[j], nr = d.run_ptr[j + 1] - rb;
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
  int t = 0;
  for (int c0 = 0; c0 < nr; c0 += kWave) {
    const int my_a = c0 + lane < nr ? d.run_a[rb + c0 + lane] : 0;
    const int my_e = c0 + lane < nr ? d.run_e[rb + c0 + lane] : 0;
    const int nc = min(kWave, nr - c0);
    for (int r = 0; r < nc; ++r) {
      const int a4 = __builtin_amdgcn_readlane(my_a, r) >> 2;
      const int n4 = (__builtin_amdgcn_readlane(my_e, r) >> 2) + 1 - a4;
#pragma unroll 4
      for (int q = lane; q < n4; q += kWave) {
        const float4 s = col[t + q];
        const float4 x = y0[a4 + q], yy = y1[a4 + q], z = y2[a4 + q];
        ax += s.x * x.x + s.y * x.y + s.z * x.z + s.w * x.w;
        ay += s.x * yy.x + s.y * yy.y + s.z * yy.z + s.w * yy.w;
        az += s.x * z.x + s.y * z.y + s.z * z.z + s.w * z.w;
      }
      t += n4;
    }
  }
  ax = wave_sum(ax);
  ay = wave_sum(ay);
  az = wave_sum(az);
  if (lane == 0) {
    u[j] = (base ? base[j] : 0.0f) + ax;
    u[d.N4 + j] = (base ? base[d.N4 + j] : 0.0f) + ay;
    u[2 * d.N4 + j] = (base ? base[2 * d.N4 + j] : 0.0f) + az;
  }
}

void launch_spmv_St(const Dev& d, hipStream_t st, const float* y, const float* base, float* u) {
  int waves_per_block = kBlock / kWave;
  hipLaunchKernelGGL(k_spmv_St, dim3((d.N + waves_per_block - 1) / waves_per_block), dim3(kBlock), 0, st, d,
                     y, base, u);
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

// Per frame: the contact range [cb, ce) of every row (contacts are sorted by node).
__global__ void k_force_ranges(Dev d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.N) return;
  const int c = min(d.n_contacts[0], d.CMAX);
  d.frange[i] = lower_bound_i(d.c_node, c, d.lo[i]);
  d.frange[d.N + i] = lower_bound_i(d.c_node, c, i + 1);
}

void launch_force_ranges(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_force_ranges, dim3((d.N + kBlock - 1) / kBlock), dim3(kBlock), 0, st, d);
}

// One wavefront per row; rows without contacts in their subtree exit at once.
__global__ void __launch_bounds__(kBlock) k_apply_forces(Dev d) {
  const int i = __builtin_amdgcn_readfirstlane((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int lane = threadIdx.x & (kWave - 1);
  if (i >= d.N) return;
  const int cb = __builtin_amdgcn_readfirstlane(d.frange[i]);
  const int ce = __builtin_amdgcn_readfirstlane(d.frange[d.N + i]);
  if (cb >= ce) return;
  const float* row = d.row_val + d.row_ptr[i];
  const int lo4 = d.row_lo4[i];
  float ax = 0.0f, ay = 0.0f, az = 0.0f;
  for (int k = cb + lane; k < ce; k += kWave) {
    float s = row[d.c_node[k] - lo4];
    ax += s * d.F[k];
    ay += s * d.F[d.CMAX + k];
    az += s * d.F[2 * d.CMAX + k];
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

}  // namespace lg
