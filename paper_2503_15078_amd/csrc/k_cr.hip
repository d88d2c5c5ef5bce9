// Conjugate Residual solve of the Schur system of the constrained global step
// (Sec. 5.2, Eq. saddle point with the sign of Algorithms 3 and 4; solver per Sec. 6):
//
//   M dlambda = (g - Omega h^2 W Omega lambda) / h^2,   M = Omega W Omega + E~,
//   g = h_vec - Omega H u (delta form, from the contact kernel),
//   W_(j,k) = K_jk C_j C_k^T (Sec. 5.3), E~ = diag(E_n/h^2, E_f/h, E_f/h),
//
// per scene, from dlambda = 0, for at most cr_iters iterations, stopping a scene on
// exact breakdown or, when cr_tol > 0, once |r| <= cr_tol |r_0|; then lambda += dlambda
// and F = h^2 C^T (Omega lambda) for the force update of the global step.
//
// Two forms of CR, the same iterates in exact arithmetic (x, r, p, q = M p, w = M r):
//  - textbook (variant 0): per step, exchange r, compute w = M r, exchange the inner
//    products (r, w), (w, w), (w, q), (r, r); two exchanges between blocks per step.
//  - pipelined (variant 1): also carry z = M q by recurrence and update w -= alpha z,
//    so that the products of the next step, M w~ (for z = M w~ + beta z) and the inner
//    products, need a single exchange.  r is exchanged with it and w is then replaced
//    by the true M r, which keeps the recurrence error to one step (without that
//    replacement float32 CR stalls far from convergence).
// In both, (q, q) of the next step follows by expanding q+ = w + beta q.
//
// One persistent launch.  Its grid never exceeds the number of compute units and its
// LDS allows one block per CU, so on a device that runs nothing else all blocks are
// resident together (kernels on one stream run one after another).  The wait at a
// barrier is bounded: a block that waits too long marks the frame failed (the frame is
// then rolled back and the host reports a device error) and every block leaves.  Each
// block owns a contiguous range of contacts; its rows of K, its slices of the vectors and
// the gathered Z = C^T (Omega v) of the scenes it touches live in LDS, every row and
// every scene's slice padded to a multiple of 4 floats so the products run on float4.  Blocks publish their slices
// of Z and per-scene partial sums, then meet the others at a device-wide barrier (one
// agent-scope arrival flag per block, polled by every block).  Exchange buffers alternate
// with the barrier's parity, since a block may publish step k+1 while another still reads
// step k.  Partial sums are combined in block order, so results are deterministic.  The
// launch ends early when no block has a running scene, a decision every block reads from
// the same flags.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.hpp"
#include "lanes.hpp"

namespace lg {

constexpr int kCrBlock = 512;         // threads per block: eight wavefronts share a CU's LDS
constexpr int kCrKFloats = 20480;     // 80 KB of (padded) K rows per block
constexpr int kCrZFloats = 3 * 2048;  // gathered (padded) Z of the touched scenes
constexpr int kCrRows = 256;          // max contacts per block
constexpr int kCrSlots = 4;           // partial sums per (block, scene slot)
// blocks of at most this many rows keep each row's state in the registers of one lane
constexpr int kCrRegRows = kCrBlock / 16;
constexpr unsigned kCrSpinLimit = 1u << 21;  // polls before a barrier wait is abandoned
// a block's scene slots span at most every scene of the handle
static_assert(kMaxScenes <= kCrRows, "scene slot tables of a CR block");

__device__ inline int pad4(int n) { return (n + 3) & ~3; }
// largest i in [0, n) with a[i] <= e (a ascending, a[0] <= e)
__device__ inline int slot_of(const int* a, int n, int e) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (a[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Device-wide barrier number b (b = 1, 2, ...) by arrival flags, zeroed by the contact
// kernel that precedes the launch.  After the block barrier (which also ORs `live` over
// the block), thread 0 stores 2 b + live into the block's flag of slot b mod 2 with an
// agent-scope release; wave 0 then polls the G flags of that slot, one per lane, with
// relaxed agent-scope loads until each holds barrier b, and acquires.  No block can pass
// barrier b + 1 before every block has arrived there, so the slot of b holds b or b - 2
// until all blocks have arrived at b.  Each block's flag lies on its own 128-byte line, so
// the arrivals are stores to G lines, not G atomic updates of one word.  Returns 1 (some
// block passed live), 0 (none) or -1 (the wait was abandoned; the failure flags are set).
__device__ inline int grid_barrier(unsigned* flags, unsigned b, bool live, int* s_st, int* fail) {
  live = __syncthreads_or(live ? 1 : 0) != 0;
  if (threadIdx.x < kWave) {
    const unsigned G = gridDim.x;
    unsigned* slot = flags + (size_t)(b & 1u) * kCrMaxBlocks * kCrFlagStride;
    if (threadIdx.x == 0)
      __hip_atomic_store(slot + blockIdx.x * kCrFlagStride, 2u * b + (live ? 1u : 0u), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    unsigned polls = 0;
    bool done = false, any = false;
    for (;;) {
      bool ok = true, lv = false;
      for (unsigned k = threadIdx.x; k < G; k += kWave) {
        const unsigned v = __hip_atomic_load(slot + k * kCrFlagStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = ok && (v >> 1) == b;
        lv = lv || (v & 1u) != 0u;
      }
      done = __all(ok);
      any = __any(lv);
      if (done || ++polls >= kCrSpinLimit) break;
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) {
      if (!done) {
        __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);      // frame not valid
        __hip_atomic_store(fail + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // cause: CR barrier
        *s_st = -1;
      } else {
        *s_st = any ? 1 : 0;
      }
    }
  }
  __syncthreads();
  return *s_st;
}

template <int V>
__global__ void __launch_bounds__(kCrBlock) k_cr(Dev d) {
  if (frame_done(d)) return;
  constexpr int NZ = V == 0 ? 1 : 2;  // vectors exchanged per step
  __shared__ __align__(16) float Ks[kCrKFloats];
  __shared__ __align__(16) float Zs[kCrZFloats];
  __shared__ float vx[3][kCrRows], vr[3][kCrRows], vp[3][kCrRows], vw[3][kCrRows], vq[3][kCrRows],
      vn[3][kCrRows];
  __shared__ float vz[V == 0 ? 1 : 3][V == 0 ? 1 : kCrRows], vm[V == 0 ? 1 : 3][V == 0 ? 1 : kCrRows];
  __shared__ float Cl[9][kCrRows], Oml[3][kCrRows], Etl[3][kCrRows];
  __shared__ float prod[kCrSlots][kCrRows];  // per-row products; after a barrier, scene sums
  __shared__ float s_g[kCrRows], s_qq[kCrRows], s_rr[kCrRows], s_rr0[kCrRows];
  __shared__ bool s_live[kCrRows];
  __shared__ int s_st;
  // per touched scene slot: contact range, K offset in global memory, first padded row
  // in Ks, first padded contact in Zs (both prefix sums, with the totals at index nsl)
  __shared__ int sl_cs[kCrRows + 1], sl_ce[kCrRows + 1], sl_koff[kCrRows + 1], sl_kb[kCrRows + 1],
      sl_zb[kCrRows + 1];
  __shared__ int row_slot[kCrRows];
  const int c = d.k_off[d.NS] > d.KCAP ? 0 : min(d.n_contacts[0], d.CMAX);
  if (c == 0) return;  // uniform across the grid: no block reaches a barrier
  // optional wall-clock stamps of block 0 (measurement): [0] start, [1] end, then per
  // barrier b = 1, 2, ...: entry, exit, end of the read of the exchanged data, end of the
  // products with K that follow it
  unsigned long long* clk = (d.cr_clock && blockIdx.x == 0) ? d.cr_clock : nullptr;
  auto stamp = [&](int idx) {
    if (clk && threadIdx.x == 0) clk[idx] = wall_clock64();
  };
  stamp(0);
  unsigned* flags = d.cr_sync;
  int* fail = d.bad;  // [0]: frame invalid, [1]: the CR barrier was abandoned
  const unsigned G = gridDim.x;
  unsigned nbar = 0;
  const int per = (c + (int)G - 1) / (int)G;
  const int j0 = min(c, (int)blockIdx.x * per), j1 = min(c, j0 + per);
  const int R = j1 - j0;
  const int CM = d.CMAX;
  const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
  const float h2 = (float)(d.h * d.h);
  const int64_t part_half = (int64_t)d.NS * G * kCrSlots;  // partials [2][scene][block][slot]
  // scenes touched by this block: [sfirst, sfirst + nsl)
  const int sfirst = R > 0 ? d.c_scene[j0] : 0;
  const int nsl = R > 0 ? d.c_scene[j1 - 1] - sfirst + 1 : 0;

  // ---- stage per-contact data, slot tables and K rows
  for (int sl = tid; sl < nsl; sl += kCrBlock) {
    const int s = sfirst + sl;
    sl_cs[sl] = d.cs_off[s];
    sl_ce[sl] = d.cs_off[s + 1];
    sl_koff[sl] = d.k_off[s];
  }
  for (int t = tid; t < R; t += kCrBlock) {
    int j = j0 + t;
    row_slot[t] = d.c_scene[j] - sfirst;
    if (per > kCrRegRows) {  // else the rows' frames live in registers
      for (int q = 0; q < 9; ++q) Cl[q][t] = d.cC[q * CM + j];
      for (int q = 0; q < 3; ++q) {
        Oml[q][t] = d.Om[q * CM + j];
        Etl[q][t] = d.Et[q * CM + j];
      }
    }
  }
  __syncthreads();
  if (wave == 0) {  // exclusive prefix sums of the padded K rows and Z slices per slot
    int ck = 0, cz = 0;
    for (int base = 0; base < nsl; base += kWave) {
      const int sl = base + lane;
      int nk = 0, nz = 0;
      if (sl < nsl) {
        const int cnt = sl_ce[sl] - sl_cs[sl];
        const int rows = min(sl_ce[sl], j1) - max(sl_cs[sl], j0);
        nk = rows * pad4(cnt);
        nz = pad4(cnt);
      }
      const int vk = wave_incl_scan_i(nk), vz2 = wave_incl_scan_i(nz);
      if (sl < nsl) {
        sl_kb[sl] = ck + vk - nk;
        sl_zb[sl] = cz + vz2 - nz;
      }
      ck += __builtin_amdgcn_readlane(vk, kWave - 1);
      cz += __builtin_amdgcn_readlane(vz2, kWave - 1);
    }
    if (lane == 0) {
      sl_kb[nsl] = ck;
      sl_zb[nsl] = cz;
    }
  }
  __syncthreads();
  const bool k_in_lds = sl_kb[nsl] <= kCrKFloats;
  const int zpad = sl_zb[nsl];
  const bool z_in_lds = 3 * NZ * zpad <= kCrZFloats;
  if (k_in_lds) {
    // Global Delassus rows are stored padded to 4 with zero pads, like Ks: each slot's
    // rows of this block form one contiguous, 16-byte aligned run in both, copied as
    // float4 with eight loads in flight per thread
    const int total4 = sl_kb[nsl] / 4;
    float4* dst = reinterpret_cast<float4*>(Ks);
    for (int base = 0; base < total4; base += 8 * kCrBlock) {
      float4 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e4 = base + tid + u * kCrBlock;
        if (e4 < total4) {
          const int sl = nsl == 1 ? 0 : slot_of(sl_kb, nsl, 4 * e4);
          const int cs = sl_cs[sl], pc = pad4(sl_ce[sl] - cs);
          const int64_t src = sl_koff[sl] + (int64_t)(max(cs, j0) - cs) * pc + (4 * e4 - sl_kb[sl]);
          v[u] = *reinterpret_cast<const float4*>(d.K + src);
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (base + tid + u * kCrBlock < total4) dst[base + tid + u * kCrBlock] = v[u];
    }
  }

  // copy components [0, 3 nv) of the touched scenes' contacts (component q of contact k
  // at Vg[q CM + k]) into Zs, slot by slot at the padded offsets; pads are zero.  No
  // block barrier.
  auto stage = [&](const float* Vg, int nv) {
    if (nsl == 1) {  // one scene: all loads of a round issued before the stores
      const int cs = sl_cs[0], cnt = sl_ce[0] - cs;
      for (int base = 0; base < zpad; base += 4 * kCrBlock) {
        float v[4][6];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = base + tid + u * kCrBlock;
#pragma unroll
          for (int q = 0; q < 6; ++q)
            if (q < 3 * nv) v[u][q] = e < cnt ? Vg[q * CM + cs + e] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = base + tid + u * kCrBlock;
          if (e < zpad)
#pragma unroll
            for (int q = 0; q < 6; ++q)
              if (q < 3 * nv) Zs[q * zpad + e] = v[u][q];
        }
      }
      return;
    }
    // several scenes: four elements per thread, all loads of a round issued before the stores
    for (int base = 0; base < zpad; base += 4 * kCrBlock) {
      float v[4][6];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = base + tid + u * kCrBlock;
        const int sl = e < zpad ? slot_of(sl_zb, nsl, e) : 0;
        const int k = e - sl_zb[sl] + sl_cs[sl];
        const bool ok = e < zpad && k < sl_ce[sl];
#pragma unroll
        for (int q = 0; q < 6; ++q) v[u][q] = (q < 3 * nv && ok) ? Vg[q * CM + k] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = base + tid + u * kCrBlock;
        if (e < zpad)
#pragma unroll
          for (int q = 0; q < 6; ++q)
            if (q < 3 * nv) Zs[q * zpad + e] = v[u][q];
      }
    }
  };
  // Y_v,t = sum_k K_jk V_v,k for every owned row t and nv vectors, 16 lanes per row (32
  // rows per pass); the first lane of each row's group then calls fin(t, Y) with the 3 nv
  // sums of its row.  staged: V in Zs; else V_v,k component q at Vg[(3 v + q) CM + k] in
  // global memory.  K rows and V both in LDS: float4 over the padded columns.
  auto matvec_rows = [&](auto nv, bool staged, const float* Vg, auto fin) {
    constexpr int NV = decltype(nv)::value;
    if (k_in_lds && staged) {
      // Per pass each wavefront takes 4 consecutive rows.  When they belong to one scene
      // (always, for a single scene) the wavefront runs them together: each lane loads a
      // column quad of V once for all 4 rows, and the 4 x 3 NV sums are reduced across the
      // 64 lanes by halving exchanges (each step trades half of a lane's sums with its
      // partner), so lane 16 r ends with row r's sums.  Otherwise each 16-lane group takes
      // one of the rows, with its own slice of V.
      const int grp = tid >> 4, gl = tid & 15;
      for (int base = 0; base < R; base += kCrBlock / 16) {
        const int tw = base + 4 * wave, nr = min(4, R - tw);
        if (nr <= 0) continue;
        const int sl0 = row_slot[tw];
        if (row_slot[tw + nr - 1] == sl0) {  // rows are in contact order, so scenes are contiguous
          constexpr int NQ = 3 * NV;
          const int cs = sl_cs[sl0], pc = pad4(sl_ce[sl0] - cs);
          const float* kb = Ks + sl_kb[sl0] + (j0 + tw - max(cs, j0)) * pc;
          const float* zb = Zs + sl_zb[sl0];
          float a[4][NQ];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int q = 0; q < NQ; ++q) a[r][q] = 0.0f;
          // every row's load issued before any product (a row past the block's last
          // repeats that row; its sums are never used)
          const float4* kr[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) kr[r] = reinterpret_cast<const float4*>(kb + min(r, nr - 1) * pc);
          const int n4 = pc / 4;
          for (int k4 = lane; k4 < n4; k4 += kWave) {
            float4 z[NQ], kv[4];
#pragma unroll
            for (int q = 0; q < NQ; ++q) z[q] = reinterpret_cast<const float4*>(zb + q * zpad)[k4];
#pragma unroll
            for (int r = 0; r < 4; ++r) kv[r] = kr[r][k4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
              for (int q = 0; q < NQ; ++q)
                a[r][q] += kv[r].x * z[q].x + kv[r].y * z[q].y + kv[r].z * z[q].z + kv[r].w * z[q].w;
          }
          // rows (0, 1) stay in lanes 0..31 and rows (2, 3) in lanes 32..63, then the
          // first row of each pair in the even 16-lane rows; the rest within each row
          float w[2][NQ];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int q = 0; q < NQ; ++q) w[i][q] = swap32_add(a[i][q], a[2 + i][q]);
          float u[NQ];
#pragma unroll
          for (int q = 0; q < NQ; ++q) u[q] = row16_sum(swap16_add(w[0][q], w[1][q]));
          const int r = lane >> 4;
          if ((lane & 15) == 0 && r < nr) fin(tw + r, u);
          continue;
        }
        const int t = base + grp;
        if (t >= R) continue;
        const int sl = row_slot[t], cs = sl_cs[sl], pc = pad4(sl_ce[sl] - cs);
        const int rrow = j0 + t - max(cs, j0);
        const float4* K4 = reinterpret_cast<const float4*>(Ks + sl_kb[sl] + rrow * pc);
        const float* zb = Zs + sl_zb[sl];
        float a[3 * NV];
#pragma unroll
        for (int q = 0; q < 3 * NV; ++q) a[q] = 0.0f;
#pragma unroll 2
        for (int k4 = gl; k4 < pc / 4; k4 += 16) {
          const float4 kv = K4[k4];
#pragma unroll
          for (int q = 0; q < 3 * NV; ++q) {
            const float4 z = reinterpret_cast<const float4*>(zb + q * zpad)[k4];
            a[q] += kv.x * z.x + kv.y * z.y + kv.z * z.z + kv.w * z.w;
          }
        }
#pragma unroll
        for (int q = 0; q < 3 * NV; ++q) a[q] = row16_sum(a[q]);
        if (gl == 0) fin(t, a);
      }
      __syncthreads();
      return;
    }
    // K rows from global memory (or unstaged V): 16 lanes per row, 16 rows in flight;
    // rows are padded to 4 with zero pads and 16-byte aligned in both places
    const int grp = tid >> 4, gl = tid & 15;
    for (int t = grp; t < R; t += kCrBlock / 16) {
      const int sl = row_slot[t], cs = sl_cs[sl], cnt = sl_ce[sl] - cs, pc = pad4(cnt);
      const int rrow = j0 + t - max(cs, j0);
      const float4* K4 = reinterpret_cast<const float4*>(k_in_lds ? Ks + sl_kb[sl] + rrow * pc
                                                                  : d.K + sl_koff[sl] + (int64_t)(j0 + t - cs) * pc);
      float a[3 * NV];
#pragma unroll
      for (int q = 0; q < 3 * NV; ++q) a[q] = 0.0f;
      // four quads of K per lane loaded together (fewer round trips per row
      // when K comes from global memory; eight spill to scratch); each lane still adds its
      // quads in column order
      constexpr int U = 4;
      const int n4 = pc / 4;
      for (int base = gl; base < n4; base += 16 * U) {
        float4 kv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k4 = base + 16 * u;
          kv[u] = k4 < n4 ? K4[k4] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int k4 = base + 16 * u;
          const int k = 4 * k4;
#pragma unroll
          for (int q = 0; q < 3 * NV; ++q) {
            if (k4 >= n4) continue;
            float4 z;
            if (staged) {
              z = reinterpret_cast<const float4*>(Zs + q * zpad + sl_zb[sl])[k4];
            } else {  // V beyond the scene's contacts meets a zero pad of K
              const float* vg = Vg + q * CM + cs + k;
              z.x = vg[0];
              z.y = k + 1 < cnt ? vg[1] : 0.0f;
              z.z = k + 2 < cnt ? vg[2] : 0.0f;
              z.w = k + 3 < cnt ? vg[3] : 0.0f;
            }
            a[q] += kv[u].x * z.x + kv[u].y * z.y + kv[u].z * z.z + kv[u].w * z.w;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 3 * NV; ++q) a[q] = row16_sum(a[q]);
      if (gl == 0) fin(t, a);
    }
    __syncthreads();
  };
  // device-wide barrier with the measurement stamps; data_read() stamps the end of the
  // read of what the other blocks published before it
  auto bar = [&](bool live) {
    ++nbar;
    stamp(2 + 4 * (nbar - 1));
    const int r = grid_barrier(flags, nbar, live, &s_st, fail);
    stamp(3 + 4 * (nbar - 1));
    return r;
  };
  auto data_read = [&]() { stamp(4 + 4 * (nbar - 1)); };
  auto products_done = [&]() { stamp(5 + 4 * (nbar - 1)); };
  // K times the first nv vectors of exchange buffer `buf`, staged into Zs when they fit
  auto exch = [&](int buf) { return d.cr_Z + (int64_t)buf * 3 * NZ * CM; };
  auto matvec_Z = [&](auto nv, int buf, auto fin) {
    if (z_in_lds) {
      stage(exch(buf), decltype(nv)::value);
      __syncthreads();
    }
    data_read();
    matvec_rows(nv, z_in_lds, exch(buf), fin);
  };
  // publish Z_j = C_j^T (Omega_j v_j) of owned row t as vector `slot` of buffer `buf`
  auto publish_Z = [&](int buf, int slot, int t, float (*v)[kCrRows]) {
    float* Zg = exch(buf) + 3 * slot * CM;
    float ov[3] = {Oml[0][t] * v[0][t], Oml[1][t] * v[1][t], Oml[2][t] * v[2][t]};
    for (int q = 0; q < 3; ++q) Zg[q * CM + j0 + t] = Cl[q][t] * ov[0] + Cl[3 + q][t] * ov[1] + Cl[6 + q][t] * ov[2];
  };
  // row t of M: out = Omega (C y) + E~ v, with y = (K Z)_t from the matvec
  auto rowM = [&](int t, const float* y, float (*v)[kCrRows], float (*out)[kCrRows]) {
    for (int rr = 0; rr < 3; ++rr) {
      float cy = Cl[3 * rr][t] * y[0] + Cl[3 * rr + 1][t] * y[1] + Cl[3 * rr + 2][t] * y[2];
      out[rr][t] = Oml[rr][t] * cy + Etl[rr][t] * v[rr][t];
    }
  };
  // per-scene partial sums of prod[0..nt) over owned contacts -> buffer `buf`
  auto publish_partials = [&](int buf) {
    constexpr int nt = kCrSlots;
    float* part = d.cr_prod + buf * part_half;
    for (int sl = wave; sl < nsl; sl += kCrBlock / kWave) {
      int t0 = max(sl_cs[sl], j0) - j0, t1 = min(sl_ce[sl], j1) - j0;
      float a[kCrSlots] = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int t = t0 + lane; t < t1; t += kWave)
        for (int q = 0; q < nt; ++q) a[q] += prod[q][t];
      for (int q = 0; q < nt; ++q) {
        float v = wave_sum(a[q]);
        if (lane == 0) part[((int64_t)(sfirst + sl) * G + blockIdx.x) * kCrSlots + q] = v;
      }
    }
  };
  // scene sums into prod[q][t] for every owned row: for each touched scene, the partials
  // of all blocks holding it, added in block order.  With stage_nv > 0, also stage that
  // many vectors of exchange buffer `buf` into Zs, its loads issued together with the
  // first round of partial-sum loads.
  auto gather_sums = [&](int buf, int stage_nv) {
    constexpr int nt = kCrSlots;
    const float* part = d.cr_prod + buf * part_half;
    for (int sl = wave, round = 0; sl < nsl || round == 0; sl += kCrBlock / kWave, ++round) {
      const bool mine = sl < nsl;
      int b0 = 0, b1 = -1;
      if (mine) {
        b0 = sl_cs[sl] / per;
        b1 = (sl_ce[sl] - 1) / per;
      }
      float a[kCrSlots] = {0.0f, 0.0f, 0.0f, 0.0f};
      for (int b = b0 + lane; b <= b1; b += kWave) {
        const float* pp = part + ((int64_t)(sfirst + sl) * G + b) * kCrSlots;
        for (int q = 0; q < nt; ++q) a[q] += pp[q];
      }
      if (round == 0 && stage_nv > 0 && z_in_lds) stage(exch(buf), stage_nv);
      if (!mine) continue;
      const int t0 = max(sl_cs[sl], j0) - j0, t1 = min(sl_ce[sl], j1) - j0;
      for (int q = 0; q < nt; ++q) {
        const float v = wave_sum(a[q]);
        for (int t = t0 + lane; t < t1; t += kWave) prod[q][t] = v;
      }
    }
    __syncthreads();
  };
  // inner products of one step for row t into prod: (r, w), (w, w), (w, q), (r, r)
  auto row_products = [&](int t) {
    float a = 0.0f, b = 0.0f, e = 0.0f, f = 0.0f;
    for (int rr = 0; rr < 3; ++rr) {
      a += vr[rr][t] * vw[rr][t];
      b += vw[rr][t] * vw[rr][t];
      e += vw[rr][t] * vq[rr][t];
      f += vr[rr][t] * vr[rr][t];
    }
    prod[0][t] = a;
    prod[1][t] = b;
    prod[2][t] = e;
    prod[3][t] = f;
  };
  const std::integral_constant<int, 1> one{};
  const std::integral_constant<int, 2> two{};
  const float tol2 = d.cr_tol * d.cr_tol;

  if (per <= kCrRegRows) {
    // ---- every block owns at most 32 rows (uniform over the grid): row t = 4 w + i is
    // owned by lane 16 i of wavefront w, the lane that finishes its products with K, and
    // its state (frame, Omega, E~, the CR vectors and scalars) stays in that lane's
    // registers.  Same arithmetic, exchanges and barriers as the form below.
    const int t = 4 * wave + (lane >> 4);
    const bool own = (lane & 15) == 0 && t < R;
    const int j = j0 + t;
    float C[9], Om[3], Et[3], x[3], r[3], p[3], q[3], w[3];
    float z[3], n[3], m[3];  // pipelined form only
    float g = 0.0f, qq = 0.0f, rr = 0.0f, rr0 = 0.0f;
    bool live = false;
#pragma unroll
    for (int k = 0; k < 3; ++k) x[k] = r[k] = p[k] = q[k] = w[k] = z[k] = n[k] = m[k] = Om[k] = Et[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < 9; ++k) C[k] = 0.0f;
    if (own) {
#pragma unroll
      for (int k = 0; k < 9; ++k) C[k] = d.cC[k * CM + j];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        Om[k] = d.Om[k * CM + j];
        Et[k] = d.Et[k * CM + j];
      }
    }
    // out = Omega (C y) + E~ v
    auto rowM_r = [&](const float* y, const float* v, float* out) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float cy = C[3 * k] * y[0] + C[3 * k + 1] * y[1] + C[3 * k + 2] * y[2];
        out[k] = Om[k] * cy + Et[k] * v[k];
      }
    };
    auto publish_r = [&](int buf, int slot, const float* v) {
      float* Zg = exch(buf) + 3 * slot * CM;
      const float ov[3] = {Om[0] * v[0], Om[1] * v[1], Om[2] * v[2]};
#pragma unroll
      for (int k = 0; k < 3; ++k) Zg[k * CM + j] = C[k] * ov[0] + C[3 + k] * ov[1] + C[6 + k] * ov[2];
    };
    auto products_r = [&]() {  // (r, w), (w, w), (w, q), (r, r)
      float a = 0.0f, b = 0.0f, e = 0.0f, f = 0.0f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        a += r[k] * w[k];
        b += w[k] * w[k];
        e += w[k] * q[k];
        f += r[k] * r[k];
      }
      prod[0][t] = a;
      prod[1][t] = b;
      prod[2][t] = e;
      prod[3][t] = f;
    };

    // setup: r = (g - Omega h^2 W Omega lambda) / h^2, x = 0, w = M r, p = r, q = w
    if (z_in_lds) stage(d.X, 1);
    __syncthreads();
    matvec_rows(one, z_in_lds, d.X, [&](int, const float* a) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float cy = C[3 * k] * a[0] + C[3 * k + 1] * a[1] + C[3 * k + 2] * a[2];
        r[k] = (d.hv[k * CM + j] - Om[k] * h2 * cy) / h2;
      }
      publish_r((nbar + 1) & 1, 0, r);
    });
    if (bar(true) < 0) return;
    matvec_Z(one, nbar & 1, [&](int, const float* a) {
      rowM_r(a, r, w);
#pragma unroll
      for (int k = 0; k < 3; ++k) q[k] = w[k];
      products_r();
      if constexpr (V == 1) publish_r((nbar + 1) & 1, 0, w);
    });
    products_done();
    publish_partials((nbar + 1) & 1);
    if (bar(true) < 0) return;
    gather_sums(nbar & 1, V == 1 ? 1 : 0);
    data_read();
    if (own) {
      g = prod[0][t];
      qq = prod[1][t];
      rr = rr0 = prod[3][t];
#pragma unroll
      for (int k = 0; k < 3; ++k) p[k] = r[k];
    }
    if constexpr (V == 1)  // z = M q = M w
      matvec_rows(one, z_in_lds, exch(nbar & 1), [&](int, const float* a) { rowM_r(a, w, z); });

    for (int it = 0; it < d.cr_iters; ++it) {
      const bool last = it + 1 == d.cr_iters;
      int mine = 0;
      if (own) {
        if (it > 0 && live) {
          const float g_new = prod[0][t], ww = prod[1][t], wq = prod[2][t];
          const float beta = g_new / g;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            p[k] = r[k] + beta * p[k];
            q[k] = w[k] + beta * q[k];
            if constexpr (V == 1) {
              z[k] = n[k] + beta * z[k];
              w[k] = m[k];
            }
          }
          qq = ww + 2.0f * beta * wq + beta * beta * qq;
          g = g_new;
          rr = prod[3][t];
        }
        live = qq != 0.0f && g != 0.0f && !(tol2 > 0.0f && rr <= tol2 * rr0);
        mine = live ? 1 : 0;
        if (live) {
          const float alpha = g / qq;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            x[k] += alpha * p[k];
            r[k] -= alpha * q[k];
            if constexpr (V == 1) w[k] -= alpha * z[k];
          }
        }
        if (!last) {
          if constexpr (V == 0) {
            publish_r((nbar + 1) & 1, 0, r);
          } else {
            products_r();  // with the recurrence w~
            publish_r((nbar + 1) & 1, 0, w);
            publish_r((nbar + 1) & 1, 1, r);
          }
        }
      }
      if (last) break;
      if constexpr (V == 0) {
        const int st = bar(mine != 0);
        if (st < 0) return;
        if (st == 0) break;
        matvec_Z(one, nbar & 1, [&](int, const float* a) {
          rowM_r(a, r, w);  // w = M r
          products_r();
        });
        products_done();
        publish_partials((nbar + 1) & 1);
        if (bar(true) < 0) return;
        gather_sums(nbar & 1, 0);
        data_read();
      } else {
        __syncthreads();  // every row's products before the partial sums
        publish_partials((nbar + 1) & 1);
        const int st = bar(mine != 0);
        if (st < 0) return;
        if (st == 0) break;
        gather_sums(nbar & 1, 2);
        data_read();
        matvec_rows(two, z_in_lds, exch(nbar & 1), [&](int, const float* a) {
          rowM_r(a, w, n);      // n = M w~
          rowM_r(a + 3, r, m);  // true M r
        });
        products_done();
      }
    }
    // lambda += dlambda; F = h^2 C^T (Omega lambda)
    if (own) {
      float ol[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float l = d.lam[k * CM + j] + x[k];
        d.lam[k * CM + j] = l;
        ol[k] = Om[k] * l;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) d.F[k * CM + j] = h2 * (C[k] * ol[0] + C[3 + k] * ol[1] + C[6 + k] * ol[2]);
    }
    stamp(1);
    return;
  }

  // ---- setup: r = (g - Omega h^2 W Omega lambda) / h^2, x = 0, w = M r, p = r, q = w
  // (X = C^T (Omega lambda) from the contact kernel)
  if (z_in_lds) stage(d.X, 1);
  __syncthreads();
  matvec_rows(one, z_in_lds, d.X, [&](int t, const float* a) {
    const int j = j0 + t;
    for (int rr = 0; rr < 3; ++rr) {
      float cy = Cl[3 * rr][t] * a[0] + Cl[3 * rr + 1][t] * a[1] + Cl[3 * rr + 2][t] * a[2];
      vx[rr][t] = 0.0f;
      vr[rr][t] = (d.hv[rr * CM + j] - Oml[rr][t] * h2 * cy) / h2;
    }
    publish_Z((nbar + 1) & 1, 0, t, vr);
  });
  if (bar(true) < 0) return;
  // w = M r, q = w ((w, q) is not used here), the step's products
  matvec_Z(one, nbar & 1, [&](int t, const float* a) {
    rowM(t, a, vr, vw);
    for (int rr = 0; rr < 3; ++rr) vq[rr][t] = vw[rr][t];
    row_products(t);
    if constexpr (V == 1) publish_Z((nbar + 1) & 1, 0, t, vw);
  });
  products_done();
  publish_partials((nbar + 1) & 1);
  if (bar(true) < 0) return;
  gather_sums(nbar & 1, V == 1 ? 1 : 0);
  data_read();
  for (int t = tid; t < R; t += kCrBlock) {
    s_g[t] = prod[0][t];
    s_qq[t] = prod[1][t];
    s_rr[t] = prod[3][t];
    s_rr0[t] = prod[3][t];
    for (int rr = 0; rr < 3; ++rr) vp[rr][t] = vr[rr][t];
  }
  if constexpr (V == 1)  // z = M q = M w
    matvec_rows(one, z_in_lds, exch(nbar & 1), [&](int t, const float* a) { rowM(t, a, vw, vz); });

  // Each step: the previous step's direction update (beta), then this step's update of
  // x and r (alpha) and, unless it is the last, what the exchange needs, all row by row
  // without block barriers; the exchange; the products with K, each row finished (M, the
  // inner products) by the lane that summed it.
  for (int it = 0; it < d.cr_iters; ++it) {
    const bool last = it + 1 == d.cr_iters;
    int mine = 0;
    for (int t = tid; t < R; t += kCrBlock) {
      if (it > 0 && s_live[t]) {
        float g = s_g[t], qq = s_qq[t];
        float g_new = prod[0][t], ww = prod[1][t], wq = prod[2][t];
        float beta = g_new / g;
        for (int rr = 0; rr < 3; ++rr) {
          vp[rr][t] = vr[rr][t] + beta * vp[rr][t];
          vq[rr][t] = vw[rr][t] + beta * vq[rr][t];
          if constexpr (V == 1) {
            vz[rr][t] = vn[rr][t] + beta * vz[rr][t];
            vw[rr][t] = vm[rr][t];
          }
        }
        s_g[t] = g_new;
        s_qq[t] = ww + 2.0f * beta * wq + beta * beta * qq;
        s_rr[t] = prod[3][t];
      }
      // a scene is finished after exact breakdown or once |r| <= tol |r_0|
      float g = s_g[t], qq = s_qq[t];
      bool live = qq != 0.0f && g != 0.0f && !(tol2 > 0.0f && s_rr[t] <= tol2 * s_rr0[t]);
      s_live[t] = live;
      mine |= live ? 1 : 0;
      if (live) {
        float alpha = g / qq;
        for (int rr = 0; rr < 3; ++rr) {
          vx[rr][t] += alpha * vp[rr][t];
          vr[rr][t] -= alpha * vq[rr][t];
          if constexpr (V == 1) vw[rr][t] -= alpha * vz[rr][t];
        }
      }
      if (!last) {
        if constexpr (V == 0) {
          publish_Z((nbar + 1) & 1, 0, t, vr);
        } else {
          row_products(t);  // with the recurrence w~
          publish_Z((nbar + 1) & 1, 0, t, vw);
          publish_Z((nbar + 1) & 1, 1, t, vr);
        }
      }
    }
    if (last) break;
    if constexpr (V == 0) {
      const int st = bar(mine != 0);
      if (st < 0) return;
      if (st == 0) break;
      matvec_Z(one, nbar & 1, [&](int t, const float* a) {
        rowM(t, a, vr, vw);  // w = M r
        row_products(t);
      });
      products_done();
      publish_partials((nbar + 1) & 1);
      if (bar(true) < 0) return;
      gather_sums(nbar & 1, 0);
      data_read();
    } else {
      __syncthreads();  // every row's products before the partial sums
      publish_partials((nbar + 1) & 1);
      const int st = bar(mine != 0);
      if (st < 0) return;
      if (st == 0) break;
      gather_sums(nbar & 1, 2);
      data_read();
      matvec_rows(two, z_in_lds, exch(nbar & 1), [&](int t, const float* a) {
        rowM(t, a, vw, vn);      // n = M w~
        rowM(t, a + 3, vr, vm);  // true M r
      });
      products_done();
    }
  }
  // lambda += dlambda; F = h^2 C^T (Omega lambda)
  for (int t = tid; t < R; t += kCrBlock) {
    int j = j0 + t;
    float ol[3];
    for (int rr = 0; rr < 3; ++rr) {
      float l = d.lam[rr * CM + j] + vx[rr][t];
      d.lam[rr * CM + j] = l;
      ol[rr] = Oml[rr][t] * l;
    }
    for (int q = 0; q < 3; ++q) d.F[q * CM + j] = h2 * (Cl[q][t] * ol[0] + Cl[3 + q][t] * ol[1] + Cl[6 + q][t] * ol[2]);
  }
  stamp(1);
}

int cr_max_blocks() {
  int dev = 0, cus = 0, per = 0, per1 = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(k_cr<0>), kCrBlock, 0) !=
          hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per1, reinterpret_cast<const void*>(k_cr<1>), kCrBlock, 0) !=
          hipSuccess)
    return 1;
  // at most one block per CU is resident (LDS), so the grid must not exceed the CU count
  return max(1, min(cus * max(min(per, per1), 1), min(cus, kCrMaxBlocks)));
}

int64_t cr_partial_floats(int blocks, int scenes) { return 2 * (int64_t)scenes * blocks * kCrSlots; }

__global__ void k_zero_cr_sync(Dev d) {
  for (int k = threadIdx.x; k < 2 * kCrMaxBlocks; k += blockDim.x) d.cr_sync[k * kCrFlagStride] = 0u;
}

void launch_zero_cr_sync(const Dev& d, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_cr_sync, dim3(1), dim3(kBlock), 0, st, d);
}

hipError_t launch_cr(const Dev& d, hipStream_t st, int cr_blocks, int variant) {
  if (cr_blocks < 1 || cr_blocks > kCrMaxBlocks) return hipErrorInvalidValue;  // barrier flag slots
  if (variant == 1) hipLaunchKernelGGL(k_cr<1>, dim3(cr_blocks), dim3(kCrBlock), 0, st, d);
  else hipLaunchKernelGGL(k_cr<0>, dim3(cr_blocks), dim3(kCrBlock), 0, st, d);
  return hipGetLastError();
}

}  // namespace lg
