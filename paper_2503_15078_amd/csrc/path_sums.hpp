// Column path sums of S = L^-1 (Sec. 4.2, Theorem 1: column j of S is nonzero on the
// ancestors of j): sum over the ancestors i of j of S_ij y_i, shared by the S^T pass and
// the contact evaluation.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "lanes.hpp"

namespace lg {

__device__ inline float dot4(const float4& s, const float4& x) {
  return s.x * x.x + s.y * x.y + s.z * x.z + s.w * x.w;
}

// Per-lane partial sums acc[g][c] = sum over this lane's quads of S_ij y_c,i for the
// columns j = j0 + g (g < ng) of one chain, whose ancestor paths are the chain runs
// [a, e] of column j0's path except that column j0 + g starts its first run at its own
// node.  Each column is read from its aligned copy (every run stored from node a & ~3,
// zero-padded to whole 4-node groups), so S values and the three y coordinates are
// 16-byte loads, and one float4 of each y coordinate serves every column of the group.
// The runs are flattened: up to 64 runs are held one per lane with their storage offsets
// (a prefix sum), and each lane takes the storage quad t = c + lane of every pass c; the
// runs that meet a pass's 64 quads are consecutive lanes, found by two ballots, and each
// lane finds the run of its quad by reading their offsets (v_readlane), so every lane
// loads on every pass however short the runs are, without LDS round trips.  The
// caller reduces acc over the wavefront.
template <int G>
__device__ inline void column_path_sums(const Dev& d, const float* __restrict__ y, int j0, int ng, int lane,
                                        float (&acc)[G][3]) {
  const float4* __restrict__ y0 = reinterpret_cast<const float4*>(y);
  const float4* __restrict__ y1 = reinterpret_cast<const float4*>(y + d.N4);
  const float4* __restrict__ y2 = reinterpret_cast<const float4*>(y + 2 * d.N4);
  // column g holds storage quad t of column j0's layout at its own index t - sh[g]: its
  // copy starts ((j0 + g) >> 2) - (j0 >> 2) quads later in the first run, and the runs
  // after the first are the same (quads before its start are zero)
  const float4* col[G];
  int sh[G];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    col[g] = reinterpret_cast<const float4*>(d.colp_val + d.colp_ptr[g < ng ? j0 + g : j0]);
    sh[g] = ((j0 + g) >> 2) - (j0 >> 2);
  }
  const int rb = d.run_ptr[j0], nr = d.run_ptr[j0 + 1] - rb;
#pragma unroll
  for (int g = 0; g < G; ++g) acc[g][0] = acc[g][1] = acc[g][2] = 0.0f;
  int tbase = 0;  // storage quads of the runs before this batch
  for (int c0 = 0; c0 < nr; c0 += kWave) {
    const int nrb = min(kWave, nr - c0);
    int my_a4 = 0, my_n4 = 0;
    if (lane < nrb) {
      my_a4 = d.run_a[rb + c0 + lane] >> 2;
      my_n4 = (d.run_e[rb + c0 + lane] >> 2) + 1 - my_a4;
    }
    const int incl = wave_incl_scan_i(my_n4);
    const int my_t0 = incl - my_n4;     // storage offset of this lane's run within the batch
    const int my_off = my_a4 - my_t0;   // y quad of storage quad t in this run: t + my_off
    const int T = __builtin_amdgcn_readlane(incl, kWave - 1);
#pragma unroll 2
    for (int c = 0; c < T; c += kWave) {
      const int t = c + lane;
      // runs r0 .. r1 meet quads [c, c + 64): r0 the last starting at or before c (run 0
      // starts at 0), r1 the last starting before c + 64
      const unsigned long long le = __ballot(lane < nrb && my_t0 <= c);
      const unsigned long long lt = __ballot(lane < nrb && my_t0 < c + kWave);
      const int r0 = 63 - __clzll(le), r1 = 63 - __clzll(lt);
      int off = __builtin_amdgcn_readlane(my_off, r0);
      for (int k = r0 + 1; k <= r1; ++k)
        if (t >= __builtin_amdgcn_readlane(my_t0, k)) off = __builtin_amdgcn_readlane(my_off, k);
      const int yq = t + off;
      if (t < T) {
        const float4 x = y0[yq], yy = y1[yq], z = y2[yq];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          if (g < ng) {
            const int idx = tbase + t - sh[g];
            float4 sv = col[g][max(idx, 0)];
            if (idx < 0) sv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            acc[g][0] += dot4(sv, x);
            acc[g][1] += dot4(sv, yy);
            acc[g][2] += dot4(sv, z);
          }
        }
      }
    }
    tbase += T;
  }
}

}  // namespace lg
