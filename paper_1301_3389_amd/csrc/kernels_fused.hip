// kernels_fused.hip -- one kernel per half-step for the Z pass and the gradient
// products when the rank fits one 64-wide tile (R <= 64): steps 2-5 and 10 of
// Algorithm 1 without the Q / Q-bar round trip through HBM.
//
// H step: a workgroup owns 64 columns t and a range of rows n.  For each
// 64-row sub-tile it forms Z = W H on the matrix cores, turns it into Q and
// Q-bar in LDS (V read once), and accumulates u = W^t Q, u_c = W^t (Q - 1),
// y = (W*W)^t Q-bar over the sub-tile: with all R rows of the gradient in one
// tile, Z is formed exactly once.  W step: the same with a block of 64 rows n
// and a range of columns t.  The outputs are the split partials and V sums
// that the candidate kernels read from the two-kernel path.
#include <math.h>

#include <algorithm>

#include "core.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"

namespace dna {

using GF = Geo<64, 64, GEMM_BK, 2, 2>;     // 64 x 64 tiles, waves 2 x 2 of 32 x 32
constexpr int FP = 64 + 4;                   // LDS row pitch of the 64-wide operand tiles (floats)

// ---------------------------------------------------------------------------
// H step.  Phase 1: Z (64 n x 64 t, K = R) through the tile engine.  Phase 2:
// acc[r][t] += sum over the sub-tile's n of W[n][r] * {Q, Q - 1, W[n][r] Q-bar}.
// LDS: the engine's double buffer (reused for W^t of phase 2), Q and Q-bar.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void k_rgh_H(const float* V, Opnd Wk, Opnd Hm, const float* W, int64_t N,
                                               int64_t T, int64_t R, int64_t nchunk, float* pu, float* puc,
                                               float* py, double* vpart, SumJob fin, int* check) {
  using TZ = Tile<GF, ProdSingle, true, false>;
  static_assert(TZ::LDS_FLOATS >= 64 * FP, "phase-2 W tile must fit in the engine's buffer");
  sum_job(fin);
  __shared__ __align__(16) float lz[TZ::LDS_FLOATS];
  __shared__ __align__(16) float lq[2][64 * FP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % GF::WGM, wn = wave / GF::WGM;
  const int64_t t0 = (int64_t)blockIdx.x * 64, sp = blockIdx.y;
  const int64_t nb0 = sp * nchunk, nb1 = std::min<int64_t>(N, nb0 + nchunk);
  f32x16 acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[c][v] = 0.f;
  double cp[1][GF::FN];
  cp[0][0] = 0.0;
  const int cl = wn * 32 + (lane & 31);           // this lane's column in the tile
  const int64_t col = t0 + cl;
  int bad = 0;
  for (int64_t nb = nb0; nb < nb1; nb += 64) {
    // V at this lane's Z positions and the W rows of phase 2, in flight during phase 1
    float vf[1][1][16];
    TZ::load_frag(vf, V, T, nb, t0, N, T);
    f32x4 wr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int f = tid + i * 256;                // 1024 float4 of the 64 x 64 W sub-tile
      const int n = f / 16, rq = (f % 16) * 4;
      f32x4 x = {0.f, 0.f, 0.f, 0.f};
      if (nb + n < N)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (rq + j < R) x[j] = W[(nb + n) * R + rq + j];
      wr[i] = x;
    }
    TZ tz;
    tz.zero();
    {
      const Opnd A[1] = {Wk};
      const Opnd B[1] = {Hm};
      tz.run(A, B, nb, t0, 0, R, lz);
    }
    // Q and Q-bar into LDS ([n][t]); rows past N and columns past T hold 0
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int rl = wm * 32 + blk_row(v, lane);
      const int64_t row = nb + rl;
      const float x = (row < N && col < T) ? vf[0][0][v] : 0.f;
      const float z = tz.acc[0][0][0][v];
      const float iz = __builtin_amdgcn_rcpf(z);
      const float q = x > 0.f ? x * iz : 0.f;
      bad |= (x > 0.f && !(z > 0.f)) ? 1 : 0;
      lq[0][rl * FP + cl] = q;
      lq[1][rl * FP + cl] = x > 0.f ? q * iz : 0.f;   // padding has z = 0: no 0 * inf
      cp[0][0] += (double)x;
    }
    // W sub-tile for phase 2, [n][r] (the engine's buffer is free after run())
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int f = tid + i * 256;
      const int n = f / 16, rq = (f % 16) * 4;
      *reinterpret_cast<f32x4*>(lz + n * FP + rq) = wr[i];
    }
    __syncthreads();
#pragma unroll 2
    for (int k = 0; k < 64; k += 2) {
      const int kr = k + (lane >> 5);
      const float a = lz[kr * FP + wm * 32 + (lane & 31)];
      const float b0 = lq[0][kr * FP + cl];
      const float b1 = lq[1][kr * FP + cl];
      acc[0] = mfma32(a, b0, acc[0]);
      acc[1] = mfma32(a, b0 - 1.f, acc[1]);
      acc[2] = mfma32(a * a, b1, acc[2]);
    }
    __syncthreads();
  }
  float* out[3] = {pu, puc, py};
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t r = wm * 32 + blk_row(v, lane);
    if (r < R && col < T) {
#pragma unroll
      for (int c = 0; c < 3; ++c) out[c][(sp * R + r) * T + col] = acc[c][v];
    }
  }
  reduce_cols<GF, 1>(cp, reinterpret_cast<double*>(lz), [&](int c, const double (&s)[1]) {
    if (t0 + c < T) vpart[sp * T + t0 + c] = s[0];
  });
  if (check && bad) atomicOr(check, CHK_DOMAIN);
}

// ---------------------------------------------------------------------------
// W step.  Phase 1: Z (64 n x 64 t).  Phase 2: acc[n][r] += sum over the
// sub-tile's t of {Q, Q - 1, Q-bar H[r][t]} H[r][t], with Q stored [t][n] and
// H^t stored [t][r] so that both operands are read along their fast index.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256, 2) void k_rgh_W(const float* V, Opnd Wk, Opnd Hm, const float* H, int64_t N,
                                               int64_t T, int64_t R, int64_t tchunk, float* pu, float* puc,
                                               float* py, double* vpart, SumJob fin, int* check) {
  using TZ = Tile<GF, ProdSingle, true, false>;
  static_assert(TZ::LDS_FLOATS >= 64 * FP, "phase-2 H tile must fit in the engine's buffer");
  sum_job(fin);
  __shared__ __align__(16) float lz[TZ::LDS_FLOATS];
  __shared__ __align__(16) float lq[2][64 * FP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % GF::WGM, wn = wave / GF::WGM;
  const int64_t n0 = (int64_t)blockIdx.x * 64, sp = blockIdx.y;
  const int64_t tb0 = sp * tchunk, tb1 = std::min<int64_t>(T, tb0 + tchunk);
  f32x16 acc[3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[c][v] = 0.f;
  double rp[1][GF::FM][16];
#pragma unroll
  for (int v = 0; v < 16; ++v) rp[0][0][v] = 0.0;
  int bad = 0;
  for (int64_t tb = tb0; tb < tb1; tb += 64) {
    float vf[1][1][16];
    TZ::load_frag(vf, V, T, n0, tb, N, T);
    // H rows for phase 2: 64 r x 64 t, transposed into [t][r] after phase 1
    f32x4 hr[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int f = tid + i * 256;
      const int r = f / 16, tq = (f % 16) * 4;
      f32x4 x = {0.f, 0.f, 0.f, 0.f};
      if (r < R)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (tb + tq + j < T) x[j] = H[(int64_t)r * T + tb + tq + j];
      hr[i] = x;
    }
    TZ tz;
    tz.zero();
    {
      const Opnd A[1] = {Wk};
      const Opnd B[1] = {Hm};
      tz.run(A, B, n0, tb, 0, R, lz);
    }
    const int tl = wn * 32 + (lane & 31);
    const int64_t col = tb + tl;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int rl = wm * 32 + blk_row(v, lane);
      const int64_t row = n0 + rl;
      const float x = (row < N && col < T) ? vf[0][0][v] : 0.f;
      const float z = tz.acc[0][0][0][v];
      const float iz = __builtin_amdgcn_rcpf(z);
      const float q = x > 0.f ? x * iz : 0.f;
      bad |= (x > 0.f && !(z > 0.f)) ? 1 : 0;
      lq[0][tl * FP + rl] = q;
      lq[1][tl * FP + rl] = x > 0.f ? q * iz : 0.f;
      rp[0][0][v] += (double)x;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int f = tid + i * 256;
      const int r = f / 16, tq = (f % 16) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j) lz[(tq + j) * FP + r] = hr[i][j];
    }
    __syncthreads();
#pragma unroll 2
    for (int k = 0; k < 64; k += 2) {
      const int kr = k + (lane >> 5);
      const float a0 = lq[0][kr * FP + wm * 32 + (lane & 31)];
      const float a1 = lq[1][kr * FP + wm * 32 + (lane & 31)];
      const float b = lz[kr * FP + wn * 32 + (lane & 31)];
      acc[0] = mfma32(a0, b, acc[0]);
      acc[1] = mfma32(a0 - 1.f, b, acc[1]);
      acc[2] = mfma32(a1, b * b, acc[2]);
    }
    __syncthreads();
  }
  float* out[3] = {pu, puc, py};
  const int64_t rr = wn * 32 + (lane & 31);       // output column r
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t n = n0 + wm * 32 + blk_row(v, lane);
    if (n < N && rr < R) {
#pragma unroll
      for (int c = 0; c < 3; ++c) out[c][(sp * N + n) * R + rr] = acc[c][v];
    }
  }
  reduce_rows<GF, 1>(rp, reinterpret_cast<double*>(lz), [&](int r, const double (&s)[1]) {
    if (n0 + r < N) vpart[sp * N + n0 + r] = s[0];
  });
  if (check && bad) atomicOr(check, CHK_DOMAIN);
}

hipError_t launch_rgh(int side, const float* V, const float* W, const float* H, int64_t N, int64_t T, int64_t R,
                      int splits, int64_t chunk, float* pu, float* puc, float* py, double* vpart, const SumJob& fin,
                      int* check, hipStream_t s) {
  if (R > 64) return hipErrorInvalidValue;
  const Opnd wk = make_opnd(W, R, N);        // element (n, r) at W[n*R + r]: K-contiguous
  const Opnd hm = make_opnd(H, T, T);        // element (t, r) at H[r*T + t]: MN-contiguous
  if (side == 0) {
    prof_begin("rgh_H", s);
    hipLaunchKernelGGL(k_rgh_H, dim3((unsigned)cdiv(T, 64), (unsigned)splits), dim3(256), 0, s, V, wk, hm, W, N,
                       T, R, chunk, pu, puc, py, vpart, fin, check);
    prof_end("rgh_H", s);
  } else {
    prof_begin("rgh_W", s);
    hipLaunchKernelGGL(k_rgh_W, dim3((unsigned)cdiv(N, 64), (unsigned)splits), dim3(256), 0, s, V, wk, hm, H, N,
                       T, R, chunk, pu, puc, py, vpart, fin, check);
    prof_end("rgh_W", s);
  }
  return hipGetLastError();
}

}  // namespace dna
