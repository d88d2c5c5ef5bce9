// Conjugate Residual solve of the Schur system of the constrained global step
// (Sec. 5.2, Eq. saddle point with the sign of Algorithms 3 and 4; solver per Sec. 6):
//
//   (Omega W Omega + E~) dlambda = (g - Omega h^2 W Omega lambda) / h^2,
//   g = h_vec - Omega H u (delta form, from the contact kernel),
//   W_(j,k) = K_jk C_j C_k^T (Sec. 5.3), E~ = diag(E_n/h^2, E_f/h, E_f/h),
//
// per scene, from dlambda = 0, for cr_iters iterations (stopping only on exact
// breakdown), then lambda += dlambda and F = h^2 C^T (Omega lambda) for the force
// update of the global step.
//
// One persistent launch (cooperative, so all blocks are co-resident).  Each block owns
// a contiguous range of contacts and keeps their rows of K in LDS when they fit.  The
// blocks meet at a device-wide barrier (an agent-scope counter) twice per iteration:
// once after publishing Z = C^T (Omega r) for the matrix-vector product, once after
// publishing the per-contact terms of (r, Ar), (Ar, Ar) and (Ar, Ap).  (Ap, Ap) for
// the next step follows from those by expanding Ap + = Ar + beta Ap, which saves the
// third reduction of the textbook recurrence.  Scene sums run in a fixed order, so
// the result is deterministic.
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace lg {

constexpr int kCrLdsFloats = 16384;  // 64 KB of K rows per block
constexpr int kCrMaxRows = 256;

__device__ inline float wave_sum_cr(float v) {
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ inline float block_sum_cr(float v, float* red) {
  v = wave_sum_cr(v);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if ((threadIdx.x & (kWave - 1)) == 0) red[w] = v;
  __syncthreads();
  float s = 0.0f;
  for (int q = 0; q < kBlock / kWave; ++q) s += red[q];
  return s;
}

// Device-wide barrier: the counter is zeroed by the contact kernel that precedes this
// launch; barrier number b waits until all G blocks have arrived b+1 times.
__device__ inline void grid_barrier(unsigned* ctr, unsigned target) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) __builtin_amdgcn_s_sleep(1);
  }
  __syncthreads();
}

struct CrRow {
  int j, s, cs, cnt;
  const float* K;  // row of K (LDS or global)
};

__global__ void __launch_bounds__(kBlock) k_cr(Dev d) {
  __shared__ float red[kBlock / kWave];
  __shared__ float Ks[kCrLdsFloats];
  __shared__ float s_rAr[kCrMaxRows], s_ApAp[kCrMaxRows], s_sum[3][kCrMaxRows];
  const int c = d.k_off[d.NS] > d.KCAP ? 0 : min(d.n_contacts[0], d.CMAX);
  if (c == 0) return;  // uniform across the grid: no block reaches a barrier
  unsigned* ctr = reinterpret_cast<unsigned*>(d.cr_sync);
  const unsigned G = gridDim.x;
  unsigned nbar = 0;
  const int per = (c + (int)G - 1) / (int)G;
  const int j0 = min(c, (int)blockIdx.x * per), j1 = min(c, j0 + per);
  const int CM = d.CMAX;
  const float h2 = (float)(d.h * d.h);
  float *x = d.cr_x, *r = d.cr_r, *p = d.cr_p, *Ar = d.cr_Ar, *Ap = d.cr_Ap, *Z = d.cr_Z;
  float* prod = d.cr_prod;  // [3][CMAX]: (r,Ar), (Ar,Ar), (Ar,Ap) per contact

  // stage this block's K rows in LDS when they fit
  int need = 0;
  for (int j = j0; j < j1; ++j) {
    int s = d.c_scene[j];
    need += d.cs_off[s + 1] - d.cs_off[s];
  }
  const bool in_lds = need <= kCrLdsFloats;
  {
    int o = 0;
    for (int j = j0; j < j1; ++j) {
      int s = d.c_scene[j], cs = d.cs_off[s], cnt = d.cs_off[s + 1] - cs;
      const float* src = d.K + d.k_off[s] + (int64_t)(j - cs) * cnt;
      if (in_lds)
        for (int k = threadIdx.x; k < cnt; k += kBlock) Ks[o + k] = src[k];
      o += cnt;
    }
    __syncthreads();
  }
  auto row = [&](int j, int& o) {
    CrRow rw;
    rw.j = j;
    rw.s = d.c_scene[j];
    rw.cs = d.cs_off[rw.s];
    rw.cnt = d.cs_off[rw.s + 1] - rw.cs;
    rw.K = in_lds ? Ks + o : d.K + d.k_off[rw.s] + (int64_t)(j - rw.cs) * rw.cnt;
    o += rw.cnt;
    return rw;
  };
  auto cval = [&](int j, int rr, int q) { return d.cC[(rr * 3 + q) * CM + j]; };
  // Y = sum_k K_jk V_k over the scene (block cooperative)
  auto matvec = [&](const CrRow& rw, const float* V, float Y[3]) {
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    for (int k = threadIdx.x; k < rw.cnt; k += kBlock) {
      float kv = rw.K[k];
      a0 += kv * V[rw.cs + k];
      a1 += kv * V[CM + rw.cs + k];
      a2 += kv * V[2 * CM + rw.cs + k];
    }
    Y[0] = block_sum_cr(a0, red);
    Y[1] = block_sum_cr(a1, red);
    Y[2] = block_sum_cr(a2, red);
  };
  // out = Omega (C_j Y) + E~ v_j
  auto applyM = [&](int j, const float Y[3], const float* v, float out[3]) {
    for (int rr = 0; rr < 3; ++rr) {
      float cy = cval(j, rr, 0) * Y[0] + cval(j, rr, 1) * Y[1] + cval(j, rr, 2) * Y[2];
      out[rr] = d.Om[rr * CM + j] * cy + d.Et[rr * CM + j] * v[rr * CM + j];
    }
  };
  auto setZ = [&](int j, const float* v) {
    float ov[3];
    for (int q = 0; q < 3; ++q) ov[q] = d.Om[q * CM + j] * v[q * CM + j];
    for (int q = 0; q < 3; ++q) Z[q * CM + j] = cval(j, 0, q) * ov[0] + cval(j, 1, q) * ov[1] + cval(j, 2, q) * ov[2];
  };
  // sums of prod[t] over the scene of each owned contact, t < nt (reused across equal scenes)
  auto scene_sums = [&](int nt) {
    int prev = -1;
    for (int j = j0; j < j1; ++j) {
      int s = d.c_scene[j];
      if (s != prev) {
        int cs = d.cs_off[s], ce = d.cs_off[s + 1];
        for (int t = 0; t < nt; ++t) {
          float a = 0.0f;
          for (int k = cs + (int)threadIdx.x; k < ce; k += kBlock) a += prod[t * CM + k];
          float v = block_sum_cr(a, red);
          if (threadIdx.x == 0)
            for (int q = j; q < j1 && d.c_scene[q] == s; ++q) s_sum[t][q - j0] = v;
        }
        prev = s;
      }
    }
    __syncthreads();
  };

  // ---- setup: r = rhs, x = 0
  {
    int o = 0;
    for (int j = j0; j < j1; ++j) {
      CrRow rw = row(j, o);
      float Y[3];
      matvec(rw, d.X, Y);  // X = C^T (Omega lambda): W Omega lambda term
      if (threadIdx.x == 0) {
        for (int rr = 0; rr < 3; ++rr) {
          float cy = cval(j, rr, 0) * Y[0] + cval(j, rr, 1) * Y[1] + cval(j, rr, 2) * Y[2];
          x[rr * CM + j] = 0.0f;
          r[rr * CM + j] = (d.hv[rr * CM + j] - d.Om[rr * CM + j] * h2 * cy) / h2;
        }
        setZ(j, r);
      }
    }
  }
  grid_barrier(ctr, G * ++nbar);
  // Ar = M r, p = r, Ap = Ar; (r, Ar), (Ap, Ap)
  {
    int o = 0;
    for (int j = j0; j < j1; ++j) {
      CrRow rw = row(j, o);
      float Y[3];
      matvec(rw, Z, Y);
      if (threadIdx.x == 0) {
        float out[3], pa = 0.0f, pb = 0.0f;
        applyM(j, Y, r, out);
        for (int rr = 0; rr < 3; ++rr) {
          float rv = r[rr * CM + j];
          Ar[rr * CM + j] = out[rr];
          p[rr * CM + j] = rv;
          Ap[rr * CM + j] = out[rr];
          pa += rv * out[rr];
          pb += out[rr] * out[rr];
        }
        prod[j] = pa;
        prod[CM + j] = pb;
      }
    }
  }
  grid_barrier(ctr, G * ++nbar);
  scene_sums(2);
  if (threadIdx.x == 0)
    for (int j = j0; j < j1; ++j) {
      s_rAr[j - j0] = s_sum[0][j - j0];
      s_ApAp[j - j0] = s_sum[1][j - j0];
    }
  __syncthreads();

  for (int it = 0; it < d.cr_iters; ++it) {
    // x += alpha p, r -= alpha Ap; publish Z = C^T (Omega r)
    if (threadIdx.x == 0)
      for (int j = j0; j < j1; ++j) {
        float rAr = s_rAr[j - j0], ApAp = s_ApAp[j - j0];
        if (ApAp != 0.0f && rAr != 0.0f) {
          float alpha = rAr / ApAp;
          for (int rr = 0; rr < 3; ++rr) {
            x[rr * CM + j] += alpha * p[rr * CM + j];
            r[rr * CM + j] -= alpha * Ap[rr * CM + j];
          }
        }
        setZ(j, r);
      }
    grid_barrier(ctr, G * ++nbar);
    // Ar = M r; per-contact (r, Ar), (Ar, Ar), (Ar, Ap)
    {
      int o = 0;
      for (int j = j0; j < j1; ++j) {
        CrRow rw = row(j, o);
        float Y[3];
        matvec(rw, Z, Y);
        if (threadIdx.x == 0) {
          float out[3], a = 0.0f, b = 0.0f, e = 0.0f;
          applyM(j, Y, r, out);
          for (int rr = 0; rr < 3; ++rr) {
            Ar[rr * CM + j] = out[rr];
            a += r[rr * CM + j] * out[rr];
            b += out[rr] * out[rr];
            e += out[rr] * Ap[rr * CM + j];
          }
          prod[j] = a;
          prod[CM + j] = b;
          prod[2 * CM + j] = e;
        }
      }
    }
    grid_barrier(ctr, G * ++nbar);
    scene_sums(3);
    if (threadIdx.x == 0)
      for (int j = j0; j < j1; ++j) {
        float rAr = s_rAr[j - j0], ApAp = s_ApAp[j - j0];
        if (ApAp != 0.0f && rAr != 0.0f) {  // a scene that broke down keeps its state
          float rAr_new = s_sum[0][j - j0], ArAr = s_sum[1][j - j0], ArAp = s_sum[2][j - j0];
          float beta = rAr_new / rAr;
          for (int rr = 0; rr < 3; ++rr) {
            p[rr * CM + j] = r[rr * CM + j] + beta * p[rr * CM + j];
            Ap[rr * CM + j] = Ar[rr * CM + j] + beta * Ap[rr * CM + j];
          }
          s_rAr[j - j0] = rAr_new;
          s_ApAp[j - j0] = ArAr + 2.0f * beta * ArAp + beta * beta * ApAp;
        }
      }
    __syncthreads();
  }
  // lambda += dlambda; F = h^2 C^T (Omega lambda)
  if (threadIdx.x == 0)
    for (int j = j0; j < j1; ++j) {
      float ol[3];
      for (int rr = 0; rr < 3; ++rr) {
        float l = d.lam[rr * CM + j] + x[rr * CM + j];
        d.lam[rr * CM + j] = l;
        ol[rr] = d.Om[rr * CM + j] * l;
      }
      for (int q = 0; q < 3; ++q)
        d.F[q * CM + j] = h2 * (cval(j, 0, q) * ol[0] + cval(j, 1, q) * ol[1] + cval(j, 2, q) * ol[2]);
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

hipError_t launch_cr(const Dev& d, hipStream_t st, int cr_blocks) {
  Dev dd = d;
  void* args[] = {&dd};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_cr), dim3(cr_blocks), dim3(kBlock), args, 0,
                                    st);
}

}  // namespace lg
