// kernels_fused.hip -- one kernel per half-step for the Z pass and the gradient
// products when the rank fits one 64-wide tile (R <= 64): steps 2-5 and 10 of
// Algorithm 1 without the Q / Q-bar round trip through HBM.
//
// H step: a workgroup owns 64 columns t (their H block stays in LDS) and a
// range of rows n.  For each 64-row sub-tile it stages the W rows in LDS, forms
// Z = W H on the matrix cores, turns it into Q and Q-bar in LDS (V read once),
// and accumulates u = W^t Q, u_c = W^t (Q - 1), y = (W*W)^t Q-bar over the
// sub-tile from the same W rows: with all R rows of the gradient in one tile, Z
// is formed exactly once.  W step: the same with a block of 64 rows n (its W
// block stays in LDS) and a range of columns t.  The outputs are the split
// partials and V sums that the candidate kernels read from the two-kernel path.
//
// Every operand tile is 64 x 64 fp32 in LDS with a 68-float row pitch; MFMA
// v_mfma_f32_32x32x2_f32, four waves each owning one 32 x 32 block.  An operand
// whose contraction index runs along the LDS row (read down a column by the
// 32 lanes of a half-wave) is read four k at a time with one 16-byte load, which
// the 68-float pitch keeps free of bank conflicts: the eight k of a group g are
// shared as k = 8g + 4h + m, lane half h, instruction m = 0..3 (kq), and the
// other operand follows the same order.
#include <math.h>

#include <algorithm>

#include "core.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"

namespace dna {

using GF = Geo<64, 64, GEMM_BK, 2, 2>;     // 64 x 64 tiles, waves 2 x 2 of 32 x 32 (reductions)
constexpr int FP = 64 + 4;                   // LDS row pitch (floats)
constexpr int FT = 64 * FP;                  // floats per LDS tile

// Contraction index of lane half (lane >> 5), group g, instruction m; 16-byte LDS read.
__device__ __forceinline__ int kq(int g, int lane, int m) { return 8 * g + 4 * (lane >> 5) + m; }
__device__ __forceinline__ f32x4 ld4(const float* p) { return *reinterpret_cast<const f32x4*>(p); }

// Groups of 8 rank indices the Z contraction runs over: LDS holds zeros past
// rank R in both operands, so stopping at R rounded up to 8 drops only exact
// zero products (the same sums as the full 64-wide tile).
__device__ __forceinline__ int rank_groups(int64_t R) { return (int)std::min<int64_t>(8, (R + 7) / 8); }

// For R <= 32 the gradient products have one 32-row block of rank indices, so
// the wave pair that would own ranks 32..63 takes the second half of each
// sub-tile's contraction for ranks 0..31 instead; at the end it hands its
// partial products through LDS (buf, NA x 2048 floats, free by then) to the
// pair holding the same outputs, which adds them.  `giver` is uniform per wave;
// every thread of the block calls this.
template <int NA>
__device__ __forceinline__ void fold_halves(f32x16 (&acc)[NA], float* buf, bool giver, int pair, int lane) {
  if (giver)
#pragma unroll
    for (int c = 0; c < NA; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) buf[((c * 2 + pair) * 16 + v) * 64 + lane] = acc[c][v];
  __syncthreads();
  if (!giver)
#pragma unroll
    for (int c = 0; c < NA; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[c][v] += buf[((c * 2 + pair) * 16 + v) * 64 + lane];
}

// Load a 64 x 64 block of a row-major fp32 matrix (rows r0.., columns c0..,
// zero outside rows < nr, columns < nc) into registers: four float4 per thread.
__device__ __forceinline__ void fetch_block(const float* X, int64_t ld, int64_t r0, int64_t c0, int64_t nr,
                                            int64_t nc, f32x4 (&x)[4], int tid) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int f = tid + i * 256;
    const int r = f / 16, cq = (f % 16) * 4;
    f32x4 v = {0.f, 0.f, 0.f, 0.f};
    if (r0 + r < nr) {
      const float* p = X + (r0 + r) * ld + c0 + cq;
      if (c0 + cq + 3 < nc && (ld & 3) == 0 && ((reinterpret_cast<uintptr_t>(X) & 15) == 0)) {
        v = *reinterpret_cast<const f32x4*>(p);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (c0 + cq + j < nc) v[j] = p[j];
      }
    }
    x[i] = v;
  }
}
__device__ __forceinline__ void store_block(float* t, const f32x4 (&x)[4], int tid) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int f = tid + i * 256;
    const int r = f / 16, cq = (f % 16) * 4;
    *reinterpret_cast<f32x4*>(t + r * FP + cq) = x[i];
  }
}

// V at this lane's positions of a 32 x 32 block (rows n0.., columns t0..);
// entries outside the matrix read as 0, so the epilogues need no bounds tests.
__device__ __forceinline__ void fetch_v(const float* V, int64_t N, int64_t T, int64_t n0, int64_t t0, int lane,
                                        float (&vf)[16]) {
  const int64_t col = t0 + (lane & 31);
  const bool cok = col < T;
  const int64_t nr = N - n0;                      // rows available from n0
  const int rb = (lane >> 5) * 4;
  const float* p = V + n0 * T + (cok ? col : 0) + rb * T;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int r = (v >> 2) * 8 + (v & 3);         // blk_row(v, lane) - rb
    vf[v] = (cok && r + rb < nr) ? p[(int64_t)r * T] : 0.f;
  }
}

// The same two loads for a block known to lie inside the matrix (no tests).
__device__ __forceinline__ void fetch_block_in(const float* X, int64_t ld, int64_t r0, int64_t c0, f32x4 (&x)[4],
                                               int tid) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int f = tid + i * 256;
    x[i] = *reinterpret_cast<const f32x4*>(X + (r0 + f / 16) * ld + c0 + (f % 16) * 4);
  }
}
__device__ __forceinline__ void fetch_v_in(const float* V, int64_t T, int64_t n0, int64_t t0, int lane,
                                           float (&vf)[16]) {
  const float* p = V + (n0 + (lane >> 5) * 4) * T + t0 + (lane & 31);
#pragma unroll
  for (int v = 0; v < 16; ++v) vf[v] = p[(int64_t)((v >> 2) * 8 + (v & 3)) * T];
}

// ---------------------------------------------------------------------------
// H step.  LDS: lh = H block [r][t] (whole kernel), lw = W rows [n][r],
// lq = Q and Q-bar [n][t] (per sub-tile).
//   phase 1: Z[n][t] = sum_r lw[n][r] lh[r][t]      (wave block n = wm, t = wn)
//   phase 2: acc[r][t] += sum_n lw[n][r] {Q, Q - 1, lw[n][r] Q-bar}[n][t]  (r = wm, t = wn)
// ---------------------------------------------------------------------------
// MODE (both orientations): RGH_DNA forms u, u_c, y and the V sums; RGH_MU the
// MU numerator u alone (no Q-bar tile); RGH_MU_COST also the input state's
// cost sum_{v>0} v log(v/z) per column (row) in place of the V sums, with the
// ratio pass's per-entry arithmetic.
// RGH_DNA_COST: RGH_DNA plus the input state's per-column (row) cost in dpart
// (the damped selection compares the Newton candidate with it).
template <bool CHK, int MODE>
__global__ __launch_bounds__(256, 2) void k_rgh_H(const float* V, const float* W, const float* H, int64_t N,
                                                  int64_t T, int64_t R, int64_t nchunk, float* pu, float* puc,
                                                  float* py, double* vpart, double* dpart, SumJob fin, int* check) {
  constexpr bool DNA = MODE == RGH_DNA || MODE == RGH_DNA_COST;
  constexpr int NA = DNA ? 3 : 1;                 // accumulated products
  constexpr int NQ = MODE == RGH_DNA_COST ? 2 : 1;   // column sums: V (DNA) or cost (MU), and the cost
  __shared__ __align__(16) float lh[FT];
  __shared__ __align__(16) float lw[FT];
  __shared__ __align__(16) float lq[DNA ? 2 : 1][FT];
  sum_job(fin);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave: scalar loop bounds
  const int wm = wave % 2, wn = wave / 2;
  const int kz = 8 * rank_groups(R);
  // phase 2: rank block rb over rows k0 .. k0 + nk of each sub-tile (R <= 32: both pairs on ranks 0..31)
  const bool half = R <= 32;
  const int rb = half ? 0 : wm * 32, k0 = half ? wm * 32 : 0, nk = half ? 32 : 64;
  const int64_t t0 = (int64_t)blockIdx.x * 64, sp = blockIdx.y;
  const int64_t nb0 = sp * nchunk, nb1 = std::min<int64_t>(N, nb0 + nchunk);
  const int cl = wn * 32 + (lane & 31);           // this lane's column t in the tile
  const int64_t col = t0 + cl;
  f32x16 acc[NA];
#pragma unroll
  for (int c = 0; c < NA; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[c][v] = 0.f;
  double cp[NQ][GF::FN];
#pragma unroll
  for (int q = 0; q < NQ; ++q) cp[q][0] = 0.0;
  int bad = 0;
  {
    f32x4 hx[4];
    fetch_block(H, T, 0, t0, R, T, hx, tid);        // rows r < R of H, columns t0..t0+63
    store_block(lh, hx, tid);
  }
  f32x4 wr[4];
  float vf[16];
  fetch_block(W, R, nb0, 0, N, R, wr, tid);
  fetch_v(V, N, T, nb0 + wm * 32, t0 + wn * 32, lane, vf);
  // sub-tiles inside the matrix (all 64 columns t, R = 64, aligned W rows) load without tests
  const bool cols_in = t0 + 64 <= T && R == 64 && (reinterpret_cast<uintptr_t>(W) & 15) == 0;
  for (int64_t nb = nb0; nb < nb1; nb += 64) {
    store_block(lw, wr, tid);
    float vn[16];
    const bool more = nb + 64 < nb1;
    if (more) {                                   // next sub-tile, in flight from here
      if (cols_in && nb + 128 <= N) {
        fetch_block_in(W, R, nb + 64, 0, wr, tid);
        fetch_v_in(V, T, nb + 64 + wm * 32, t0 + wn * 32, lane, vn);
      } else {
        fetch_block(W, R, nb + 64, 0, N, R, wr, tid);
        fetch_v(V, N, T, nb + 64 + wm * 32, t0 + wn * 32, lane, vn);
      }
    }
    __syncthreads();                              // lw (and lh) ready; lq free
    f32x16 z;
#pragma unroll
    for (int v = 0; v < 16; ++v) z[v] = 0.f;
    for (int kb = 0; kb < kz; kb += 8) {          // 4-byte reads: measured faster here than the 16-byte form
#pragma unroll
      for (int k = kb; k < kb + 8; k += 2) {
        const int kr = k + (lane >> 5);
        z = mfma32(lw[(wm * 32 + (lane & 31)) * FP + kr], lh[kr * FP + cl], z);
      }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int rl = wm * 32 + blk_row(v, lane);
      const float x = vf[v];                      // 0 outside the matrix
      const float iz = __builtin_amdgcn_rcpf(z[v]);
      const float q = x > 0.f ? x * iz : 0.f;
      if (CHK) bad |= (x > 0.f && !(z[v] > 0.f)) ? 1 : 0;
      lq[0][rl * FP + cl] = q;
      if constexpr (DNA) {
        lq[1][rl * FP + cl] = x > 0.f ? q * iz : 0.f;   // padding has z = 0: no 0 * inf
        cp[0][0] += (double)x;
        if constexpr (MODE == RGH_DNA_COST) cp[1][0] += (double)(x * log2_hw(x > 0.f ? q : 1.f));
      } else if constexpr (MODE == RGH_MU_COST) {
        cp[0][0] += (double)(x * log2_hw(x > 0.f ? q : 1.f)) * LN2;
      }
    }
    __syncthreads();                              // lq ready
    for (int kb = k0; kb < k0 + nk; kb += 8) {
#pragma unroll
      for (int k = kb; k < kb + 8; k += 2) {
        const int kr = k + (lane >> 5);
        const float a = lw[kr * FP + rb + (lane & 31)];
        const float b0 = lq[0][kr * FP + cl];
        acc[0] = mfma32(a, b0, acc[0]);
        if constexpr (DNA) {
          const float b1 = lq[NA - 2][kr * FP + cl];
          acc[NA - 2] = mfma32(a, b0 - 1.f, acc[NA - 2]);
          acc[NA - 1] = mfma32(a * a, b1, acc[NA - 1]);
        }
      }
    }
    if (more)
#pragma unroll
      for (int v = 0; v < 16; ++v) vf[v] = vn[v];
    __syncthreads();                              // lw and lq free for the next sub-tile
  }
  static_assert(NA * 2048 <= (DNA ? 2 : 1) * FT, "fold buffer");
  if (half) fold_halves<NA>(acc, &lq[0][0], wm == 1, wn, lane);   // the wm = 1 pair holds no rank >= R
  float* out[3] = {pu, puc, py};
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t r = wm * 32 + blk_row(v, lane);
    if (r < R && col < T) {
#pragma unroll
      for (int c = 0; c < NA; ++c) out[c][(sp * R + r) * T + col] = acc[c][v];
    }
  }
  if constexpr (MODE != RGH_MU)                   // V sums (DNA) or input-state costs (MU with cost)
    reduce_cols<GF, NQ>(cp, reinterpret_cast<double*>(lw), [&](int c, const double (&s)[NQ]) {
      if (t0 + c < T) {
        vpart[sp * T + t0 + c] = s[0];
        if constexpr (NQ == 2) dpart[sp * T + t0 + c] = s[NQ - 1] * LN2;
      }
    });
  if (CHK && bad) atomicOr(check, CHK_DOMAIN);
}

// ---------------------------------------------------------------------------
// W step.  LDS: lw = W block [n][r] (whole kernel), lh = H columns [r][t],
// lq = Q and Q-bar [n][t] (per sub-tile).
//   phase 1: Z[n][t] = sum_r lw[n][r] lh[r][t]      (wave block n = wm, t = wn)
//   phase 2: acc[n][r] += sum_t {Q, Q - 1, Q-bar lh[r][t]}[n][t] lh[r][t]  (n = wm, r = wn)
// ---------------------------------------------------------------------------
// CH (DNA modes, R > 32, T >= GH_CHUNK_MIN_K): u_c = sum over the 64-column
// sub-tiles of (sum of q h) - (sum of h), the sub-tile sums of the rows of H
// formed in float64 from the LDS tile; two product chains instead of three
// (the chunked gradient sums of the tiled kernels, chunks of one sub-tile).
template <bool CHK, int MODE, bool CH>
__global__ __launch_bounds__(256, 2) void k_rgh_W(const float* V, const float* W, const float* H, int64_t N,
                                                  int64_t T, int64_t R, int64_t tchunk, float* pu, float* puc,
                                                  float* py, double* vpart, double* dpart, SumJob fin, int* check) {
  constexpr bool DNA = MODE == RGH_DNA || MODE == RGH_DNA_COST;
  static_assert(!CH || DNA, "the chunked sums are a DNA form");
  constexpr int NA = DNA ? (CH ? 2 : 3) : 1;
  constexpr int NQ = MODE == RGH_DNA_COST ? 2 : 1;
  __shared__ __align__(16) float lw[FT];
  __shared__ __align__(16) float lh[FT];
  __shared__ __align__(16) float lq[DNA ? 2 : 1][FT];
  __shared__ float csk[CH ? 64 : 1];
  sum_job(fin);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave: scalar loop bounds
  const int wm = wave % 2, wn = wave / 2;
  const int gz = rank_groups(R);
  // phase 2: rank block rb over column groups g0 .. g0 + ng (R <= 32: both pairs on ranks 0..31)
  const bool half = R <= 32;
  const int rb = half ? 0 : wn * 32, g0 = half ? wn * 4 : 0, ng = half ? 4 : 8;
  const int64_t n0 = (int64_t)blockIdx.x * 64, sp = blockIdx.y;
  const int64_t tb0 = sp * tchunk, tb1 = std::min<int64_t>(T, tb0 + tchunk);
  const int tl = wn * 32 + (lane & 31);           // this lane's column in the Z block / r in phase 2
  f32x16 acc[NA];
#pragma unroll
  for (int c = 0; c < NA; ++c)
#pragma unroll
    for (int v = 0; v < 16; ++v) acc[c][v] = 0.f;
  float ur[CH ? 16 : 1], ucr[CH ? 16 : 1];
#pragma unroll
  for (int v = 0; v < (CH ? 16 : 1); ++v) ur[v] = ucr[v] = 0.f;
  double rp[NQ][GF::FM][16];
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int v = 0; v < 16; ++v) rp[q][0][v] = 0.0;
  int bad = 0;
  {
    f32x4 wx[4];
    fetch_block(W, R, n0, 0, N, R, wx, tid);        // rows n0..n0+63 of W, columns r < R
    store_block(lw, wx, tid);
  }
  f32x4 hr[4];
  float vf[16];
  fetch_block(H, T, 0, tb0, R, T, hr, tid);
  fetch_v(V, N, T, n0 + wm * 32, tb0 + wn * 32, lane, vf);
  // sub-tiles inside the matrix (all 64 rows n, R = 64, aligned H rows) load without tests
  const bool rows_in = n0 + 64 <= N && R == 64 && (T & 3) == 0 && (reinterpret_cast<uintptr_t>(H) & 15) == 0;
  for (int64_t tb = tb0; tb < tb1; tb += 64) {
    store_block(lh, hr, tid);
    const bool more = tb + 64 < tb1;
    float vn[16];
    if (more) {                                   // next sub-tile, in flight from here
      if (rows_in && tb + 128 <= T) {
        fetch_block_in(H, T, 0, tb + 64, hr, tid);
        fetch_v_in(V, T, n0 + wm * 32, tb + 64 + wn * 32, lane, vn);
      } else {
        fetch_block(H, T, 0, tb + 64, R, T, hr, tid);
        fetch_v(V, N, T, n0 + wm * 32, tb + 64 + wn * 32, lane, vn);
      }
    }
    __syncthreads();
    f32x16 z;
#pragma unroll
    for (int v = 0; v < 16; ++v) z[v] = 0.f;
    {
      const float* pa = lw + (wm * 32 + (lane & 31)) * FP + 4 * (lane >> 5);
#pragma unroll 2
      for (int g = 0; g < gz; ++g) {
        const f32x4 a4 = ld4(pa + 8 * g);
#pragma unroll
        for (int m = 0; m < 4; ++m) z = mfma32(a4[m], lh[kq(g, lane, m) * FP + tl], z);
      }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int rl = wm * 32 + blk_row(v, lane);
      const float x = vf[v];                      // 0 outside the matrix
      const float iz = __builtin_amdgcn_rcpf(z[v]);
      const float q = x > 0.f ? x * iz : 0.f;
      if (CHK) bad |= (x > 0.f && !(z[v] > 0.f)) ? 1 : 0;
      lq[0][rl * FP + tl] = q;
      if constexpr (DNA) {
        lq[1][rl * FP + tl] = x > 0.f ? q * iz : 0.f;
        rp[0][0][v] += (double)x;
        if constexpr (MODE == RGH_DNA_COST) rp[1][0][v] += (double)(x * log2_hw(x > 0.f ? q : 1.f));
      } else if constexpr (MODE == RGH_MU_COST) {
        rp[0][0][v] += (double)(x * log2_hw(x > 0.f ? q : 1.f)) * LN2;
      }
    }
    if constexpr (CH) {   // sum over this sub-tile's 64 columns of each row r of H (zeros past T and R)
      const int r = tid >> 2, qd = tid & 3;
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const f32x4 h4 = ld4(lh + r * FP + 16 * qd + 4 * j);
        a += ((double)h4[0] + (double)h4[1]) + ((double)h4[2] + (double)h4[3]);
      }
      a += __shfl_xor(a, 1);
      a += __shfl_xor(a, 2);
      if (qd == 0) csk[r] = (float)a;
    }
    __syncthreads();
    {
      const int o = (wm * 32 + (lane & 31)) * FP + 4 * (lane >> 5);
      const float* pb = lh + (rb + (lane & 31)) * FP + 4 * (lane >> 5);   // H[r][t]
#pragma unroll 2
      for (int g = g0; g < g0 + ng; ++g) {
        const f32x4 a0 = ld4(lq[0] + o + 8 * g);
        const f32x4 b = ld4(pb + 8 * g);
        if constexpr (DNA) {
          const f32x4 a1 = ld4(lq[1] + o + 8 * g);
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            acc[0] = mfma32(a0[m], b[m], acc[0]);
            if constexpr (!CH) acc[1] = mfma32(a0[m] - 1.f, b[m], acc[1]);
            acc[NA - 1] = mfma32(a1[m], b[m] * b[m], acc[NA - 1]);
          }
        } else {
#pragma unroll
          for (int m = 0; m < 4; ++m) acc[0] = mfma32(a0[m], b[m], acc[0]);
        }
      }
    }
    if constexpr (CH) {   // this sub-tile's sum of q h, into u and (less the H sums) into u_c
      const float cr = csk[tl];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float x = acc[0][v];
        ur[v] += x;
        ucr[v] += x - cr;
        acc[0][v] = 0.f;
      }
    }
    if (more)
#pragma unroll
      for (int v = 0; v < 16; ++v) vf[v] = vn[v];
    __syncthreads();
  }
  static_assert(NA * 2048 <= (DNA ? 2 : 1) * FT, "fold buffer");
  if (half) fold_halves<NA>(acc, &lq[0][0], wn == 1, wm, lane);   // the wn = 1 pair holds no rank >= R
  float* out[3] = {pu, puc, py};
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int64_t n = n0 + wm * 32 + blk_row(v, lane);
    if (n < N && tl < R) {
      if constexpr (CH) {
        out[0][(sp * N + n) * R + tl] = ur[v];
        out[1][(sp * N + n) * R + tl] = ucr[v];
        out[2][(sp * N + n) * R + tl] = acc[1][v];
      } else {
#pragma unroll
        for (int c = 0; c < NA; ++c) out[c][(sp * N + n) * R + tl] = acc[c][v];
      }
    }
  }
  if constexpr (MODE != RGH_MU)
    reduce_rows<GF, NQ>(rp, reinterpret_cast<double*>(lw), [&](int r, const double (&s)[NQ]) {
      if (n0 + r < N) {
        vpart[sp * N + n0 + r] = s[0];
        if constexpr (NQ == 2) dpart[sp * N + n0 + r] = s[NQ - 1] * LN2;
      }
    });
  if (CHK && bad) atomicOr(check, CHK_DOMAIN);
}

// ---------------------------------------------------------------------------
// Candidate costs (steps 7-9, 12-14) for R <= 64, the candidates' block
// resident in LDS.  acc 0 = z_DNA, acc 1 = dZ = z_MU - z_DNA; cost terms as in
// cost_acc (base-2 units, scaled by LN2 on output).
//
// H orientation: a workgroup owns 64 columns t (H_DNA and H_MU - H_DNA blocks,
// [r][t]) and a range of rows n (W rows streamed, [n][r]); each lane keeps
// float64 column partials over the whole range.  Partials: part[q][sp][t].
// ---------------------------------------------------------------------------
// NO (newton only, the damped selection): z_DNA alone, the cost terms of
// d_DNA only (the margin and MU slots of the partials are written as zero).
template <bool NO, bool S0>
__global__ __launch_bounds__(256, 2) void k_costf_H(const float* V, const float* W, const float* Xmu,
                                                    const float* Xn, int64_t N, int64_t T, int64_t R,
                                                    int64_t nchunk, double* part, int* fpart) {
  __shared__ __align__(16) float ln[FT];
  __shared__ __align__(16) float ld[FT];
  __shared__ __align__(16) float lw[FT];
  __shared__ int fl_s[64];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave: scalar loop bounds
  const int wm = wave % 2, wn = wave / 2;
  const int gz = rank_groups(R);
  const int64_t t0 = (int64_t)blockIdx.x * 64, sp = blockIdx.y;
  const int64_t nb0 = sp * nchunk, nb1 = std::min<int64_t>(N, nb0 + nchunk);
  const int cl = wn * 32 + (lane & 31);
  const int64_t col = t0 + cl;
  if (tid < 64) fl_s[tid] = 0;
  {
    f32x4 a[4], b[4];
    fetch_block(Xn, T, 0, t0, R, T, a, tid);
    store_block(ln, a, tid);
    if (!NO) {
      fetch_block(Xmu, T, 0, t0, R, T, b, tid);
#pragma unroll
      for (int i = 0; i < 4; ++i) b[i] -= a[i];
      store_block(ld, b, tid);
    }
  }
  double cp[3][GF::FN];
  cp[0][0] = cp[1][0] = cp[2][0] = 0.0;
  int fl = 0;
  f32x4 wr[4];
  float vf[16];
  fetch_block(W, R, nb0, 0, N, R, wr, tid);
  fetch_v(V, N, T, nb0 + wm * 32, t0 + wn * 32, lane, vf);
  // sub-tiles inside the matrix (all 64 columns t, R = 64, aligned W rows) load without tests
  const bool cols_in = t0 + 64 <= T && R == 64 && (reinterpret_cast<uintptr_t>(W) & 15) == 0;
  for (int64_t nb = nb0; nb < nb1; nb += 64) {
    store_block(lw, wr, tid);
    float vn[16];
    const bool more = nb + 64 < nb1;
    if (more) {                                   // next sub-tile, in flight from here
      if (cols_in && nb + 128 <= N) {
        fetch_block_in(W, R, nb + 64, 0, wr, tid);
        fetch_v_in(V, T, nb + 64 + wm * 32, t0 + wn * 32, lane, vn);
      } else {
        fetch_block(W, R, nb + 64, 0, N, R, wr, tid);
        fetch_v(V, N, T, nb + 64 + wm * 32, t0 + wn * 32, lane, vn);
      }
    }
    __syncthreads();
    f32x16 zn, dz;
#pragma unroll
    for (int v = 0; v < 16; ++v) zn[v] = dz[v] = 0.f;
    {
      const float* pa = lw + (wm * 32 + (lane & 31)) * FP + 4 * (lane >> 5);
#pragma unroll 2
      for (int g = 0; g < gz; ++g) {
        const f32x4 a4 = ld4(pa + 8 * g);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const int kk = kq(g, lane, m) * FP + cl;
          zn = mfma32(a4[m], ln[kk], zn);
          if (!NO) dz = mfma32(a4[m], ld[kk], dz);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float x = vf[v];                      // 0 outside the matrix
      if (NO) fl |= cost_acc_newton(x, zn[v], cp[0][0]);
      else fl |= cost_acc<S0>(x, zn[v], dz[v], cp[0][0], cp[1][0], cp[2][0]);
    }
    if (more)
#pragma unroll
      for (int v = 0; v < 16; ++v) vf[v] = vn[v];
    __syncthreads();
  }
  if (fl) atomicOr(&fl_s[cl], fl);
  const int64_t stride = (int64_t)gridDim.y * T;
  reduce_cols<GF, 3>(cp, reinterpret_cast<double*>(lw), [&](int c, const double (&s)[3]) {
    if (t0 + c < T) {
      part[sp * T + t0 + c] = s[0] * LN2;
      part[stride + sp * T + t0 + c] = s[1] * LN2;
      part[2 * stride + sp * T + t0 + c] = s[2] * LN2;
      fpart[sp * T + t0 + c] = fl_s[c];
    }
  });
}

// W orientation: a workgroup owns 64 rows n (W_DNA and W_MU - W_DNA blocks,
// [n][r]) and a range of columns t (H streamed, [r][t]).  Row partials of each
// sub-tile are reduced across the half-wave at once (halfwave_slot_sum) and
// kept per lane in float64.  Partials: part[q][sp][n].
template <bool NO, bool S0>
__global__ __launch_bounds__(256, 2) void k_costf_W(const float* V, const float* H, const float* Xmu,
                                                    const float* Xn, int64_t N, int64_t T, int64_t R,
                                                    int64_t tchunk, double* part, int* fpart) {
  __shared__ __align__(16) float ln[FT];
  __shared__ __align__(16) float ld[FT];
  __shared__ __align__(16) float lh[FT];
  __shared__ int fl_s[64];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform per wave: scalar loop bounds
  const int wm = wave % 2, wn = wave / 2;
  const int gz = rank_groups(R);
  const int64_t n0 = (int64_t)blockIdx.x * 64, sp = blockIdx.y;
  const int64_t tb0 = sp * tchunk, tb1 = std::min<int64_t>(T, tb0 + tchunk);
  const int tl = wn * 32 + (lane & 31);
  if (tid < 64) fl_s[tid] = 0;
  {
    f32x4 a[4], b[4];
    fetch_block(Xn, R, n0, 0, N, R, a, tid);
    store_block(ln, a, tid);
    if (!NO) {
      fetch_block(Xmu, R, n0, 0, N, R, b, tid);
#pragma unroll
      for (int i = 0; i < 4; ++i) b[i] -= a[i];
      store_block(ld, b, tid);
    }
  }
  double rs[3] = {0.0, 0.0, 0.0};                 // this lane's slot of the row partials
  int flr[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) flr[v] = 0;
  // d_DNA and margin terms of up to CW_GROUP sub-tiles add up per element in
  // float32 before one float64 half-wave reduction
  constexpr int CW_GROUP = 4;
  float a0[16], a1[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) a0[v] = a1[v] = 0.f;
  int ng = 0;
  f32x4 hr[4];
  float vf[16];
  fetch_block(H, T, 0, tb0, R, T, hr, tid);
  fetch_v(V, N, T, n0 + wm * 32, tb0 + wn * 32, lane, vf);
  // sub-tiles inside the matrix (all 64 rows n, R = 64, aligned H rows) load without tests
  const bool rows_in = n0 + 64 <= N && R == 64 && (T & 3) == 0 && (reinterpret_cast<uintptr_t>(H) & 15) == 0;
  for (int64_t tb = tb0; tb < tb1; tb += 64) {
    store_block(lh, hr, tid);
    float vn[16];
    const bool more = tb + 64 < tb1;
    if (more) {                                   // next sub-tile, in flight from here
      if (rows_in && tb + 128 <= T) {
        fetch_block_in(H, T, 0, tb + 64, hr, tid);
        fetch_v_in(V, T, n0 + wm * 32, tb + 64 + wn * 32, lane, vn);
      } else {
        fetch_block(H, T, 0, tb + 64, R, T, hr, tid);
        fetch_v(V, N, T, n0 + wm * 32, tb + 64 + wn * 32, lane, vn);
      }
    }
    __syncthreads();
    f32x16 zn, dz;
#pragma unroll
    for (int v = 0; v < 16; ++v) zn[v] = dz[v] = 0.f;
    {
      const int o = (wm * 32 + (lane & 31)) * FP + 4 * (lane >> 5);
#pragma unroll 2
      for (int g = 0; g < gz; ++g) {
        const f32x4 an = ld4(ln + o + 8 * g);
        const f32x4 ad = NO ? an : ld4(ld + o + 8 * g);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const float b = lh[kq(g, lane, m) * FP + tl];
          zn = mfma32(an[m], b, zn);
          if (!NO) dz = mfma32(ad[m], b, dz);
        }
      }
    }
    double s2[16];
    int fsub = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      s2[v] = 0.0;
      const float x = vf[v];                      // 0 outside the matrix
      const int f = NO ? cost_acc_newton_f(x, zn[v], a0[v]) : cost_acc_f<S0>(x, zn[v], dz[v], a0[v], a1[v], s2[v]);
      flr[v] |= f;
      fsub |= f;
    }
    if (__any(fsub)) rs[2] += halfwave_slot_sum(s2, lane);   // s2 is 0 unless an element flagged
    if (++ng == CW_GROUP || !more) {
      double s0[16], s1[16];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        s0[v] = (double)a0[v];
        s1[v] = (double)a1[v];
        a0[v] = a1[v] = 0.f;
      }
      if (NO || S0) rs[0] += halfwave_slot_sum(s0, lane);
      rs[1] += halfwave_slot_sum(s1, lane);
      ng = 0;
    }
    if (more)
#pragma unroll
      for (int v = 0; v < 16; ++v) vf[v] = vn[v];
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 16; ++v)
    if (flr[v]) atomicOr(&fl_s[wm * 32 + blk_row(v, lane)], flr[v]);
  // the two waves along t hold partials of the same rows: add them in LDS
  double* red = reinterpret_cast<double*>(lh);
  if ((lane & 1) == 0) {
    const int r = wm * 32 + slot_row(lane);
#pragma unroll
    for (int q = 0; q < 3; ++q) red[(q * 2 + wn) * 64 + r] = rs[q];
  }
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.y * N;
  if (tid < 64 && n0 + tid < N) {
#pragma unroll
    for (int q = 0; q < 3; ++q)
      part[q * stride + sp * N + n0 + tid] = (red[(q * 2) * 64 + tid] + red[(q * 2 + 1) * 64 + tid]) * LN2;
    fpart[sp * N + n0 + tid] = fl_s[tid];
  }
}

hipError_t launch_costf(int side, const float* V, const float* F, const float* Xmu, const float* Xn, int64_t N,
                        int64_t T, int64_t R, int splits, int64_t chunk, double* part, int* fpart, hipStream_t s,
                        bool newton_only, bool s0) {
  if (R > FUSED_MAX_R) return hipErrorInvalidValue;
  if (side == 0) {
    prof_begin("costf_H", s);
    const dim3 grid((unsigned)cdiv(T, 64), (unsigned)splits);
    auto k = newton_only ? k_costf_H<true, true> : (s0 ? k_costf_H<false, true> : k_costf_H<false, false>);
    hipLaunchKernelGGL(k, grid, dim3(256), 0, s, V, F, Xmu, Xn, N, T, R, chunk, part, fpart);
    prof_end("costf_H", s);
  } else {
    prof_begin("costf_W", s);
    const dim3 grid((unsigned)cdiv(N, 64), (unsigned)splits);
    auto k = newton_only ? k_costf_W<true, true> : (s0 ? k_costf_W<false, true> : k_costf_W<false, false>);
    hipLaunchKernelGGL(k, grid, dim3(256), 0, s, V, F, Xmu, Xn, N, T, R, chunk, part, fpart);
    prof_end("costf_W", s);
  }
  return hipGetLastError();
}

template <int MODE>
static void launch_rgh_mode(int side, const float* V, const float* W, const float* H, int64_t N, int64_t T,
                            int64_t R, int splits, int64_t chunk, float* pu, float* puc, float* py, double* vpart,
                            double* dpart, const SumJob& fin, int* check, hipStream_t s) {
  if (side == 0) {
    const dim3 grid((unsigned)cdiv(T, 64), (unsigned)splits);
    if (check)
      hipLaunchKernelGGL((k_rgh_H<true, MODE>), grid, dim3(256), 0, s, V, W, H, N, T, R, chunk, pu, puc, py, vpart,
                         dpart, fin, check);
    else
      hipLaunchKernelGGL((k_rgh_H<false, MODE>), grid, dim3(256), 0, s, V, W, H, N, T, R, chunk, pu, puc, py, vpart,
                         dpart, fin, check);
  } else {
    const dim3 grid((unsigned)cdiv(N, 64), (unsigned)splits);
    // the chunked u_c for the plain DNA mode (the cost-carrying mode of the damped
    // selection has no registers to spare for it)
    constexpr bool PLAIN = MODE == RGH_DNA;
    const bool ch = PLAIN && R > 32 && T >= GH_CHUNK_MIN_K;   // chunk = one 64-column sub-tile
    static_assert(GH_CHUNK == 64, "the chunks of k_rgh_W are its sub-tiles");
    auto k = check ? (ch ? k_rgh_W<true, MODE, PLAIN> : k_rgh_W<true, MODE, false>)
                   : (ch ? k_rgh_W<false, MODE, PLAIN> : k_rgh_W<false, MODE, false>);
    hipLaunchKernelGGL(k, grid, dim3(256), 0, s, V, W, H, N, T, R, chunk, pu, puc, py, vpart, dpart, fin, check);
  }
}

hipError_t launch_rgh(int side, const float* V, const float* W, const float* H, int64_t N, int64_t T, int64_t R,
                      int splits, int64_t chunk, float* pu, float* puc, float* py, double* vpart, const SumJob& fin,
                      int* check, hipStream_t s, int mode, double* dpart) {
  if (R > FUSED_MAX_R) return hipErrorInvalidValue;
  if (mode == RGH_DNA_COST && !dpart) return hipErrorInvalidValue;
  const bool dna = mode == RGH_DNA || mode == RGH_DNA_COST;
  const char* name = dna ? (side == 0 ? "rgh_H" : "rgh_W") : (side == 0 ? "rgh_mu_H" : "rgh_mu_W");
  prof_begin(name, s);
  if (mode == RGH_DNA)
    launch_rgh_mode<RGH_DNA>(side, V, W, H, N, T, R, splits, chunk, pu, puc, py, vpart, dpart, fin, check, s);
  else if (mode == RGH_DNA_COST)
    launch_rgh_mode<RGH_DNA_COST>(side, V, W, H, N, T, R, splits, chunk, pu, puc, py, vpart, dpart, fin, check, s);
  else if (mode == RGH_MU)
    launch_rgh_mode<RGH_MU>(side, V, W, H, N, T, R, splits, chunk, pu, puc, py, vpart, dpart, fin, check, s);
  else
    launch_rgh_mode<RGH_MU_COST>(side, V, W, H, N, T, R, splits, chunk, pu, puc, py, vpart, dpart, fin, check, s);
  prof_end(name, s);
  return hipGetLastError();
}

}  // namespace dna
