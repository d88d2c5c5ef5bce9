// Conjugate Residual solve of the Schur system of the constrained global step
// (Sec. 5.2, Eq. saddle point with the sign of Algorithms 3 and 4; solver per Sec. 6):
//
//   (Omega W Omega + E~) dlambda = (g - Omega h^2 W Omega lambda) / h^2,
//   g = h_vec - Omega H u (delta form, from the contact kernel),
//   W_(j,k) = K_jk C_j C_k^T (Sec. 5.3), E~ = diag(E_n/h^2, E_f/h, E_f/h),
//
// per scene, from dlambda = 0, for at most cr_iters iterations, stopping a scene on
// exact breakdown or, when cr_tol > 0, once |r| <= cr_tol |r_0|; then lambda += dlambda
// and F = h^2 C^T (Omega lambda) for the force update of the global step.  The launch
// ends early when no scene is left running (a decision every block takes from the same
// device counter read after a barrier).
//
// One persistent launch (cooperative, so all blocks are co-resident).  Each block owns a
// contiguous range of contacts; its rows of K, its slices of x, r, p, Ar, Ap and the
// gathered Z = C^T (Omega r) of the scenes it touches live in LDS.  Blocks meet at a
// device-wide barrier (an agent-scope counter) twice per iteration: after publishing
// their slice of Z, and after publishing per-scene partial sums of (r, Ar), (Ar, Ar),
// (Ar, Ap).  (Ap, Ap) of the next step follows by expanding Ap+ = Ar + beta Ap.  Partial
// sums are combined in block order, so results are deterministic.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace lg {

constexpr int kCrKFloats = 20480;   // 80 KB of K rows per block
constexpr int kCrZFloats = 3 * 2048;  // gathered Z of the touched scenes
constexpr int kCrRows = 256;        // max contacts per block
constexpr int kCrSlots = 4;         // partial sums per (block, scene slot)
constexpr int kCrMaxBlocks = 1024;

__device__ inline float wave_sum_cr(float v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Device-wide barrier: the counter is zeroed by the contact kernel that precedes this
// launch; barrier number b waits until all G blocks have arrived b times.
__device__ inline void grid_barrier(unsigned* ctr, unsigned target) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) __builtin_amdgcn_s_sleep(1);
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kBlock) k_cr(Dev d) {
  __shared__ float Ks[kCrKFloats];
  __shared__ float Zs[kCrZFloats];
  __shared__ float vx[3][kCrRows], vr[3][kCrRows], vp[3][kCrRows], vAr[3][kCrRows], vAp[3][kCrRows];
  __shared__ float Cl[9][kCrRows], Oml[3][kCrRows], Etl[3][kCrRows];
  __shared__ float prod[kCrSlots][kCrRows];
  __shared__ float s_rAr[kCrRows], s_ApAp[kCrRows], s_rr[kCrRows], s_rr0[kCrRows], s_sum[kCrSlots][kCrRows];
  __shared__ bool s_live[kCrRows];
  __shared__ bool s_go;
  __shared__ int koffs[kCrRows + 1];
  __shared__ int sl_cs[kCrRows + 1], sl_ce[kCrRows + 1];  // contact range of each touched scene
  __shared__ int bfirst[kCrMaxBlocks];                     // first scene of every block
  const int c = d.k_off[d.NS] > d.KCAP ? 0 : min(d.n_contacts[0], d.CMAX);
  if (c == 0) return;  // uniform across the grid: no block reaches a barrier
  unsigned* ctr = reinterpret_cast<unsigned*>(d.cr_sync);
  const unsigned G = gridDim.x;
  unsigned nbar = 0;
  const int per = (c + (int)G - 1) / (int)G;
  const int j0 = min(c, (int)blockIdx.x * per), j1 = min(c, j0 + per);
  const int R = j1 - j0;
  const int CM = d.CMAX;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const float h2 = (float)(d.h * d.h);
  float* Zg = d.cr_Z;
  float* part = d.cr_prod;  // [G][kCrRows][kCrSlots] partial sums per (block, scene slot)
  // scenes touched by this block: [sfirst, slast]
  const int sfirst = R > 0 ? d.c_scene[j0] : 0;
  const int slast = R > 0 ? d.c_scene[j1 - 1] : -1;
  const int zlo = R > 0 ? d.cs_off[sfirst] : 0;
  const int zhi = R > 0 ? d.cs_off[slast + 1] : 0;
  const bool z_in_lds = 3 * (zhi - zlo) <= kCrZFloats;

  // ---- stage per-contact data and K rows
  if (tid == 0) {
    int o = 0;
    for (int t = 0; t < R; ++t) {
      int s = d.c_scene[j0 + t];
      koffs[t] = o;
      o += d.cs_off[s + 1] - d.cs_off[s];
    }
    koffs[R] = o;
  }
  for (int slot = tid; slot <= slast - sfirst; slot += kBlock) {
    sl_cs[slot] = d.cs_off[sfirst + slot];
    sl_ce[slot] = d.cs_off[sfirst + slot + 1];
  }
  for (int b = tid; b < (int)G; b += kBlock) bfirst[b] = b * per < c ? d.c_scene[b * per] : 0;
  for (int t = tid; t < R; t += kBlock) {
    int j = j0 + t;
    for (int q = 0; q < 9; ++q) Cl[q][t] = d.cC[q * CM + j];
    for (int q = 0; q < 3; ++q) {
      Oml[q][t] = d.Om[q * CM + j];
      Etl[q][t] = d.Et[q * CM + j];
    }
  }
  __syncthreads();
  const bool k_in_lds = koffs[R] <= kCrKFloats;
  if (k_in_lds)
    for (int t = 0; t < R; ++t) {
      int j = j0 + t, s = d.c_scene[j], cs = d.cs_off[s], cnt = d.cs_off[s + 1] - cs;
      const float* src = d.K + d.k_off[s] + (int64_t)(j - cs) * cnt;
      for (int k = tid; k < cnt; k += kBlock) Ks[koffs[t] + k] = src[k];
    }
  __syncthreads();

  // Y_t = sum_k K_jk V_k for every owned row t (one wavefront per row); V is the
  // gathered vector (LDS when it fits, else global), indexed by contact.
  auto matvec_rows = [&](const float* V, int vstride, int vbase, float Y[][kCrRows]) {
    for (int t = wave; t < R; t += kBlock / kWave) {
      int j = j0 + t, s = d.c_scene[j], cs = d.cs_off[s], cnt = d.cs_off[s + 1] - cs;
      const float* Krow = k_in_lds ? Ks + koffs[t] : d.K + d.k_off[s] + (int64_t)(j - cs) * cnt;
      float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
      for (int k = lane; k < cnt; k += kWave) {
        float kv = Krow[k];
        int idx = cs + k - vbase;
        a0 += kv * V[idx];
        a1 += kv * V[vstride + idx];
        a2 += kv * V[2 * vstride + idx];
      }
      a0 = wave_sum_cr(a0);
      a1 = wave_sum_cr(a1);
      a2 = wave_sum_cr(a2);
      if (lane == 0) {
        Y[0][t] = a0;
        Y[1][t] = a1;
        Y[2][t] = a2;
      }
    }
    __syncthreads();
  };
  // gather Z of the touched scenes into LDS after a barrier
  auto gather_Z = [&]() {
    if (z_in_lds) {
      int n = zhi - zlo;
      for (int k = tid; k < n; k += kBlock) {
        Zs[k] = Zg[zlo + k];
        Zs[n + k] = Zg[CM + zlo + k];
        Zs[2 * n + k] = Zg[2 * CM + zlo + k];
      }
    }
    __syncthreads();
  };
  auto matvec_Z = [&](float Y[][kCrRows]) {
    if (z_in_lds) matvec_rows(Zs, zhi - zlo, zlo, Y);
    else matvec_rows(Zg, CM, 0, Y);
  };
  // publish Z_j = C_j^T (Omega_j v_j) for owned contacts
  auto publish_Z = [&](float v[][kCrRows]) {
    for (int t = tid; t < R; t += kBlock) {
      float ov[3] = {Oml[0][t] * v[0][t], Oml[1][t] * v[1][t], Oml[2][t] * v[2][t]};
      for (int q = 0; q < 3; ++q) Zg[q * CM + j0 + t] = Cl[q][t] * ov[0] + Cl[3 + q][t] * ov[1] + Cl[6 + q][t] * ov[2];
    }
  };
  // out = Omega (C Y) + E~ v (row t), in place into Y
  auto applyM = [&](float Y[][kCrRows], float v[][kCrRows]) {
    for (int t = tid; t < R; t += kBlock) {
      float y[3] = {Y[0][t], Y[1][t], Y[2][t]};
      for (int rr = 0; rr < 3; ++rr) {
        float cy = Cl[3 * rr][t] * y[0] + Cl[3 * rr + 1][t] * y[1] + Cl[3 * rr + 2][t] * y[2];
        Y[rr][t] = Oml[rr][t] * cy + Etl[rr][t] * v[rr][t];
      }
    }
    __syncthreads();
  };
  // per-scene partial sums of prod[0..nt) over owned contacts -> global partials
  auto publish_partials = [&](int nt) {
    for (int slot = wave; slot <= slast - sfirst; slot += kBlock / kWave) {
      int t0 = max(sl_cs[slot], j0) - j0, t1 = min(sl_ce[slot], j1) - j0;
      float a[kCrSlots] = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int t = t0 + lane; t < t1; t += kWave)
        for (int q = 0; q < nt; ++q) a[q] += prod[q][t];
      for (int q = 0; q < nt; ++q) {
        float v = wave_sum_cr(a[q]);
        if (lane == 0) part[((int64_t)blockIdx.x * kCrRows + slot) * kCrSlots + q] = v;
      }
    }
  };
  // scene sums: for each touched scene, sum the partials of all blocks holding it, in
  // block order
  auto gather_sums = [&](int nt) {
    for (int slot = wave; slot <= slast - sfirst; slot += kBlock / kWave) {
      int s = sfirst + slot;
      int b0 = sl_cs[slot] / per, b1 = (sl_ce[slot] - 1) / per;
      float a[kCrSlots] = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int b = b0 + lane; b <= b1; b += kWave) {
        const float* pp = part + ((int64_t)b * kCrRows + (s - bfirst[b])) * kCrSlots;
        for (int q = 0; q < nt; ++q) a[q] += pp[q];
      }
      for (int q = 0; q < nt; ++q) {
        float v = wave_sum_cr(a[q]);
        if (lane == 0) {
          int t0 = max(sl_cs[slot], j0) - j0, t1 = min(sl_ce[slot], j1) - j0;
          for (int t = t0; t < t1; ++t) s_sum[q][t] = v;
        }
      }
    }
    __syncthreads();
  };

  // ---- setup: r = (g - Omega h^2 W Omega lambda) / h^2, x = 0
  {
    float(*Y)[kCrRows] = vAr;
    matvec_rows(d.X, CM, 0, Y);  // X = C^T (Omega lambda) from the contact kernel
    for (int t = tid; t < R; t += kBlock) {
      int j = j0 + t;
      float y[3] = {Y[0][t], Y[1][t], Y[2][t]};
      for (int rr = 0; rr < 3; ++rr) {
        float cy = Cl[3 * rr][t] * y[0] + Cl[3 * rr + 1][t] * y[1] + Cl[3 * rr + 2][t] * y[2];
        vx[rr][t] = 0.0f;
        vr[rr][t] = (d.hv[rr * CM + j] - Oml[rr][t] * h2 * cy) / h2;
      }
    }
    __syncthreads();
    publish_Z(vr);
  }
  grid_barrier(ctr, G * ++nbar);
  gather_Z();
  matvec_Z(vAr);
  applyM(vAr, vr);
  for (int t = tid; t < R; t += kBlock) {
    float a = 0.0f, b = 0.0f, e = 0.0f;
    for (int rr = 0; rr < 3; ++rr) {
      vp[rr][t] = vr[rr][t];
      vAp[rr][t] = vAr[rr][t];
      a += vr[rr][t] * vAr[rr][t];
      b += vAr[rr][t] * vAr[rr][t];
      e += vr[rr][t] * vr[rr][t];
    }
    prod[0][t] = a;
    prod[1][t] = b;
    prod[2][t] = e;
  }
  __syncthreads();
  publish_partials(3);
  grid_barrier(ctr, G * ++nbar);
  gather_sums(3);
  for (int t = tid; t < R; t += kBlock) {
    s_rAr[t] = s_sum[0][t];
    s_ApAp[t] = s_sum[1][t];
    s_rr[t] = s_sum[2][t];
    s_rr0[t] = s_sum[2][t];
  }
  __syncthreads();

  const float tol2 = d.cr_tol * d.cr_tol;
  for (int it = 0; it < d.cr_iters; ++it) {
    // a scene is finished after exact breakdown or once |r| <= tol |r0|
    for (int t = tid; t < R; t += kBlock) {
      float rAr = s_rAr[t], ApAp = s_ApAp[t];
      bool live = ApAp != 0.0f && rAr != 0.0f && !(tol2 > 0.0f && s_rr[t] <= tol2 * s_rr0[t]);
      s_live[t] = live;
      if (live) {
        float alpha = rAr / ApAp;
        for (int rr = 0; rr < 3; ++rr) {
          vx[rr][t] += alpha * vp[rr][t];
          vr[rr][t] -= alpha * vAp[rr][t];
        }
      }
    }
    __syncthreads();
    publish_Z(vr);
    // count blocks with a live scene; read after the barrier, so every block takes the
    // same decision to stop
    if (tid == 0) {
      bool any = false;
      for (int t = 0; t < R; ++t) any |= s_live[t];
      if (any) __hip_atomic_fetch_add(d.cr_active + it, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    grid_barrier(ctr, G * ++nbar);
    if (tid == 0) s_go = __hip_atomic_load(d.cr_active + it, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0;
    __syncthreads();
    if (!s_go) break;
    gather_Z();
    matvec_Z(vAr);
    applyM(vAr, vr);
    for (int t = tid; t < R; t += kBlock) {
      float a = 0.0f, b = 0.0f, e = 0.0f, f = 0.0f;
      for (int rr = 0; rr < 3; ++rr) {
        a += vr[rr][t] * vAr[rr][t];
        b += vAr[rr][t] * vAr[rr][t];
        e += vAr[rr][t] * vAp[rr][t];
        f += vr[rr][t] * vr[rr][t];
      }
      prod[0][t] = a;
      prod[1][t] = b;
      prod[2][t] = e;
      prod[3][t] = f;
    }
    __syncthreads();
    publish_partials(4);
    grid_barrier(ctr, G * ++nbar);
    gather_sums(4);
    for (int t = tid; t < R; t += kBlock) {
      if (s_live[t]) {
        float rAr = s_rAr[t], ApAp = s_ApAp[t];
        float rAr_new = s_sum[0][t], ArAr = s_sum[1][t], ArAp = s_sum[2][t];
        float beta = rAr_new / rAr;
        for (int rr = 0; rr < 3; ++rr) {
          vp[rr][t] = vr[rr][t] + beta * vp[rr][t];
          vAp[rr][t] = vAr[rr][t] + beta * vAp[rr][t];
        }
        s_rAr[t] = rAr_new;
        s_ApAp[t] = ArAr + 2.0f * beta * ArAp + beta * beta * ApAp;
        s_rr[t] = s_sum[3][t];
      }
    }
    __syncthreads();
  }
  // lambda += dlambda; F = h^2 C^T (Omega lambda)
  for (int t = tid; t < R; t += kBlock) {
    int j = j0 + t;
    float ol[3];
    for (int rr = 0; rr < 3; ++rr) {
      float l = d.lam[rr * CM + j] + vx[rr][t];
      d.lam[rr * CM + j] = l;
      ol[rr] = Oml[rr][t] * l;
    }
    for (int q = 0; q < 3; ++q) d.F[q * CM + j] = h2 * (Cl[q][t] * ol[0] + Cl[3 + q][t] * ol[1] + Cl[6 + q][t] * ol[2]);
  }
}

int cr_max_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_cr), kBlock, 0) !=
      hipSuccess)
    return 1;
  return max(1, min(cus * max(per, 1), 1024));
}

int cr_partial_floats(int blocks) { return blocks * kCrRows * kCrSlots; }

hipError_t launch_cr(const Dev& d, hipStream_t st, int cr_blocks) {
  Dev dd = d;
  void* args[] = {&dd};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_cr), dim3(cr_blocks), dim3(kBlock), args, 0,
                                    st);
}

}  // namespace lg
