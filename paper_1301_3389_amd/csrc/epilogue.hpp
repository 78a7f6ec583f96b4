// epilogue.hpp -- pieces shared by the fp32 and 16-bit kernel epilogues:
// deterministic tile reductions and the per-element cost terms.
#pragma once
#include <math.h>

#include "core.hpp"

namespace dna {

// ---------------------------------------------------------------------------
// Deterministic tile reductions of per-lane partials.
// Column form: cp[q][j] holds this lane's partial for column (j, lane&31).
// Row form:    rp[q][i][v] holds this lane's partial for row blk_row(v) of block i.
// `red` is LDS scratch of NQ * max(WGM*BN, WGN*BM) doubles.
// ---------------------------------------------------------------------------
template <class G, int NQ, class OUT>
__device__ __forceinline__ void reduce_cols(double (&cp)[NQ][G::FN], double* red, OUT&& out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % G::WGM, wn = wave / G::WGM;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const double s = cp[q][j] + __shfl_xor(cp[q][j], 32);
      if (lane < 32) red[(q * G::WGM + wm) * G::BN + wn * G::WN + j * 32 + lane] = s;
    }
  __syncthreads();
  for (int c = tid; c < G::BN; c += G::NT) {
    double s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      s[q] = 0.0;
      for (int m = 0; m < G::WGM; ++m) s[q] += red[(q * G::WGM + m) * G::BN + c];
    }
    out(c, s);
  }
  __syncthreads();
}

template <class G, int NQ, class OUT>
__device__ __forceinline__ void reduce_rows(double (&rp)[NQ][G::FM][16], double* red, OUT&& out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % G::WGM, wn = wave / G::WGM;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int i = 0; i < G::FM; ++i) {
      const double y = halfwave_slot_sum(rp[q][i], lane);
      if ((lane & 1) == 0) red[(q * G::WGN + wn) * G::BM + wm * G::WM + i * 32 + slot_row(lane)] = y;
    }
  __syncthreads();
  for (int r = tid; r < G::BM; r += G::NT) {
    double s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      s[q] = 0.0;
      for (int w = 0; w < G::WGN; ++w) s[q] += red[(q * G::WGN + w) * G::BM + r];
    }
    out(r, s);
  }
  __syncthreads();
}

__device__ __forceinline__ double xlogx_over(float v, float z) {
  // v log(v/z) for v > 0, z > 0 (the summand of eq. 1 and steps 9/14); the ratio
  // uses the hardware reciprocal (<= 1 ulp), the logarithm is the accurate one.
  return (double)v * (double)logf(v * __builtin_amdgcn_rcpf(z));
}

// Per-element cost terms with v > 0 and z_DNA, z_MU the two reconstructions
// (z_MU = z_DNA + dZ):
//   s0 += v log(v/z_DNA)          (d_DNA; rows with z_DNA <= 0 flag bit 1)
//   s1 += -v log1p(dZ/z_DNA)      (d_MU - d_DNA; rows where both z > 0)
//   s2 += v log(v/z_MU)           (rows with z_DNA <= 0 < z_MU; bit 2 if z_MU <= 0)
// so that, absent flags, d_MU = s0 + s1 and the margin is s1.
// Branch-free for the common case (both reconstructions positive or v = 0): the
// logarithms take neutral arguments where a term must vanish.  Returns the flag
// bits of this element.
__device__ __forceinline__ int cost_acc(float x, float zN, float dz, double& s0, double& s1, double& s2) {
  const float zM = zN + dz;
  const bool pos = x > 0.f;
  const bool okN = zN > 0.f, okM = zM > 0.f;
  const float izN = __builtin_amdgcn_rcpf(zN);
  const float l0 = logf((pos && okN) ? x * izN : 1.f);
  const float l1 = log1pf((pos && okN && okM) ? dz * izN : 0.f);
  s0 += (double)(x * l0);
  s1 -= (double)(x * l1);
  int fl = 0;
  if (pos && !(okN && okM)) {            // a reconstruction vanished where v > 0
    fl = (okN ? 0 : 1) | (okM ? 0 : 2);
    if (!okN && okM) s2 += xlogx_over(x, zM);
  }
  return fl;
}

}  // namespace dna
