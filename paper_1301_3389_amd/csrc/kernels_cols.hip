// kernels_cols.hip -- the whole DNA H half-step (Algorithm 1 steps 2-15) in one
// kernel, for R <= 64 and many columns.
//
// Given W the columns of H are independent problems (Sec. 2): a workgroup that
// owns a block of 16 columns t and runs over all N rows holds the complete
// gradient sums and the complete candidate costs of its columns.  It needs no
// split partials in HBM, no second kernel for the candidates and none for the
// choice; V is read twice (once per pass), W streams through LDS from L2.
//
// W rows and V go from global memory straight into LDS (global_load_lds)
// through a ring of three stages, two sub-tiles ahead of the one being
// computed, so the loads of a sub-tile have two sub-tiles of products to land.
// A stage holds the 64 x 64 W rows (16-byte chunks swizzled by row, which keeps
// both read patterns below free of bank conflicts) and the four V values of
// every lane at that lane's own slots.
//
// Pass 1, per sub-tile of 64 rows n: Z = W H on the matrix cores (each wave 16
// rows x 16 columns, v_mfma_f32_16x16x4_f32), Q = V/Z and Q-bar = Q/Z in
// registers, and u = W^t Q, u_c = W^t (Q - 1), y = (W*W)^t Q-bar accumulated
// from those registers: in the 16x16x4 layout a lane holds Z at rows 4g + v of
// its wave's block, which are exactly the contraction indices it supplies to
// the gradient products (lane group g, instruction v), so Q never leaves the
// registers.  After the last sub-tile the four waves' partial sums are added in
// a fixed order and the candidates (eq. 7, 11, 14, 15, 17 and the rescaling of
// eq. 10) are formed in LDS.
//
// Pass 2, over the same sub-tiles: z_DNA = W X_DNA and dZ = W (X_MU - X_DNA),
// the cost terms of steps 7-9 and 12-14 (float64 column sums); then the choice
// of step 15 per column, H overwritten with the chosen columns, and the partial
// row sums of the new block (16 columns) for the normalisation of step 16.
#include <math.h>

#include <algorithm>
#include <type_traits>

#include "core.hpp"
#include "core16.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"

namespace dna {

constexpr int HC_TB = (int)HCOLS_TB;   // columns per workgroup
constexpr int HC_SUB = 64;             // rows per sub-tile
constexpr int HC_XP = HC_TB + 1;       // LDS row pitch of the candidate tiles (floats)
constexpr int HC_STAGES = 3;
constexpr int HC_WST = 64 * 64;        // floats of the W rows of a stage
constexpr int HC_VST = 4 * 256;        // floats of the V values of a stage

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Instruction-group order for the scheduler (sched_group_barrier masks): a
// wave issues its instructions in order, so vector-ALU work placed between its
// matrix instructions runs while the matrix core is busy instead of after it.
constexpr int SG_VALU = 0x002, SG_MFMA = 0x008, SG_DSR = 0x100;
template <int NM, int NV>
__device__ __forceinline__ void interleave_mfma_valu() {
#pragma unroll
  for (int k = 0; k < NM; ++k) {
    __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
    __builtin_amdgcn_sched_group_barrier(SG_VALU, NV, 0);
  }
}

// Sum over the four lane groups (lanes j, j + 16, j + 32, j + 48) in a fixed
// order; every lane of the four ends with the same value.
__device__ __forceinline__ double group4_sum(double x) {
  x += __shfl_xor(x, 16);
  return x + __shfl_xor(x, 32);
}

// DMA of one piece per lane (16 or 4 bytes) from a buffer descriptor into LDS
// at dst + lane * size; reads past the descriptor's range return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const float* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)std::min<int64_t>(bytes, 0x7fffffff), 0x00020000);
}
template <int SIZE>
__device__ __forceinline__ void buf_to_lds(__amdgpu_buffer_rsrc_t r, float* dst, uint32_t off) {
  auto* d = (__attribute__((address_space(3))) void*)dst;
  if constexpr (SIZE == 16) __builtin_amdgcn_raw_ptr_buffer_load_lds(r, d, 16, off, 0, 0, 0);
  else __builtin_amdgcn_raw_ptr_buffer_load_lds(r, d, 4, off, 0, 0, 0);
}

// Float offset of W row n (0..63 in the sub-tile), rank column c in a stage:
// the 16-byte chunk c / 4 of row n sits at chunk position (c / 4) ^ (n % 16).
__device__ __forceinline__ int wsw(int n, int c) { return n * 64 + (((c >> 2) ^ (n & 15)) << 2) + (c & 3); }

// W16: R % 4 == 0 and 16-byte aligned W, the rows go in 16-byte pieces (four
// per thread and stage); otherwise in 4-byte pieces (sixteen).  Rows past N
// read as zero (the descriptor range); rank columns past R hold the next row's
// finite entries, which meet zero operands (H and the candidates past R); V of
// padding columns is a valid column's, masked where used.
template <int RB, bool CHK, bool W16, bool DS>
__global__ __launch_bounds__(256, 2) void k_hstep_cols(HColsArgs a) {
  constexpr int WLOADS = W16 ? 4 : 16, LOADS = WLOADS + 4;   // DMA instructions per thread and stage
  static_assert(2 * LOADS <= 63, "vmcnt holds at most 63 outstanding operations");
  __shared__ __align__(16) float ring[HC_STAGES][HC_WST + HC_VST];
  __shared__ __align__(16) float lx[3][64 * HC_XP];       // X_DNA, X_MU - X_DNA, X_MU  [r][t]
  __shared__ float cs[64];                                // c_r = (W^t 1)_r + lambda
  __shared__ double dred[16][HC_TB];                      // per row group / per wave column partials
  __shared__ double col3[3][4][HC_TB];                    // per wave cost partials
  __shared__ double fac[HC_TB];
  __shared__ int flw[HC_TB];
  __shared__ int pick[HC_TB];

  const int64_t N = a.N, T = a.T, R = a.R;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int j = lane & 15, g = lane >> 4;
  // column block: consecutive blocks on one XCD (they share the 128-byte lines of V)
  const int64_t nblk = gridDim.x, b = blockIdx.x;
  const int64_t q8 = nblk / 8, rem = nblk % 8, xx = b % 8, ss = b / 8;
  const int64_t blk = (xx < rem ? xx * (q8 + 1) : rem * (q8 + 1) + (xx - rem) * q8) + ss;
  const int64_t t0 = blk * HC_TB, col = t0 + j;
  const bool cok = col < T;
  const int64_t colc = cok ? col : T - 1;      // a valid column for the loads of padding lanes

  // sub-tiles 0 and 1 of pass 1 go first: the loads below overlap them.
  // The DMA reads through buffer descriptors whose range ends with the matrix:
  // rows past N read as zero.  Per-lane byte offsets are fixed for the kernel;
  // a sub-tile moves only the descriptor base (scalar work).
  const int64_t ns = (N + HC_SUB - 1) / HC_SUB;
  constexpr int WK = W16 ? 4 : 16;
  uint32_t woff[WK], voff[4];
#pragma unroll
  for (int k = 0; k < WK; ++k) {
    if constexpr (W16) {
      const int row = 4 * (4 * k + w) + (lane >> 4);   // 1 KiB block 4k + w: rows 4 blk .. 4 blk + 3
      woff[k] = (uint32_t)((row * R + 4 * ((lane & 15) ^ (row & 15))) * 4);
    } else {
      const int row = 16 * w + k;                      // one 256-byte row per instruction
      woff[k] = (uint32_t)((row * R + ((((lane >> 2) ^ (row & 15)) << 2) + (lane & 3))) * 4);
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) voff[v] = (uint32_t)(((16 * w + 4 * g + v) * T + colc) * 4);
  auto issue = [&](int64_t nb, auto stc) {
    float* base = ring[decltype(stc)::value];
    const auto rw = buf_rsrc(a.W + nb * R, (N - nb) * R * 4);
    const auto rv = buf_rsrc(a.V + nb * T, (N - nb) * T * 4);
#pragma unroll
    for (int k = 0; k < WK; ++k)
      buf_to_lds<W16 ? 16 : 4>(rw, base + (W16 ? (4 * k + w) * 256 : (16 * w + k) * 64), woff[k]);
#pragma unroll
    for (int v = 0; v < 4; ++v) buf_to_lds<4>(rv, base + HC_WST + v * 256 + 64 * w, voff[v]);
  };
  using S0 = std::integral_constant<int, 0>;
  using S1 = std::integral_constant<int, 1>;
  using S2 = std::integral_constant<int, 2>;
  // sub-tiles 0 and 1 of a pass (call after the last reads of stages 0 and 1)
  auto prime = [&]() {
    issue(0, S0{});
    if (ns > 1) issue(HC_SUB, S1{});
  };
  prime();

  // this thread's entries of H for the candidates: rows rq + 16i, column tc
  const int tt = tid & 15, rq = tid >> 4;
  const int64_t tc = t0 + tt, tcc = tc < T ? tc : T - 1;
  float hx[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) hx[i] = a.H[std::min<int64_t>(rq + 16 * i, R - 1) * T + tcc];

  if (tid < 64) {                                 // c_r, summed as the factor-sum job does
    float c = 0.f;
    if (tid < R) {
      double tot = 0.0;
#pragma unroll 8
      for (int p = 0; p < a.cj.nparts; ++p) tot += a.cj.part[(int64_t)p * R + tid];
      c = (float)(tot + a.cj.reg);
      if (CHK && blk == 0 && !(tot > 0.0)) atomicOr(a.check, CHK_DOMAIN);
    }
    cs[tid] = c;
  }
  if (tid < HC_TB) flw[tid] = 0;

  // B operand of Z: H[16q + 4g + m][col] (zero past R and past T)
  f32x4 hb[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int r = 16 * q + 4 * g + m;
      const float h = a.H[std::min<int64_t>(r, R - 1) * T + colc];
      hb[q][m] = (cok && r < R) ? h : 0.f;
    }

  // V of sub-tile nb at this lane's positions (rows nb + 16w + 4g + v, column
  // col), zero outside the matrix
  auto vload = [&](int st, int64_t nb, float (&x)[4]) {
    const int64_t n0 = nb + 16 * w + 4 * g;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float y = ring[st][HC_WST + v * 256 + tid];
      x[v] = (cok && n0 + v < N) ? y : 0.f;
    }
  };
  // the pass over the sub-tiles: wait for sub-tile i (one younger stage may
  // stay in flight), barrier, DMA of sub-tile i + 2 into the stage sub-tile
  // i - 1 used, products of sub-tile i
  // The loop runs three sub-tiles per trip so that every stage index (and with
  // it every LDS address) is a compile-time constant.
  auto run = [&](auto&& compute) {
    auto step = [&](auto stc, int64_t i) {
      constexpr int ST = decltype(stc)::value;
      asm volatile("" ::: "memory");
      if (i + 1 < ns) __builtin_amdgcn_s_waitcnt(vmcnt_imm(LOADS));
      else __builtin_amdgcn_s_waitcnt(vmcnt_imm(0));
      asm volatile("s_barrier" ::: "memory");
      if (i + 2 < ns) issue((i + 2) * HC_SUB, std::integral_constant<int, (ST + 2) % HC_STAGES>{});
      float vf[4];
      vload(ST, i * HC_SUB, vf);
      compute(ring[ST], i * HC_SUB, vf);
    };
    for (int64_t i = 0; i < ns; i += HC_STAGES) {
      step(S0{}, i);
      if (i + 1 < ns) step(S1{}, i + 1);
      if (i + 2 < ns) step(S2{}, i + 2);
    }
    __syncthreads();                              // the ring may be reused
  };

  // ---------------- pass 1: gradient sums ----------------
  f32x4 acc[3][RB];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int q = 0; q < RB; ++q) acc[c][q] = f32x4{0.f, 0.f, 0.f, 0.f};
  double vs = 0.0;
  int bad = 0;
  // Software pipeline: step i issues the Z products of sub-tile i, then the
  // gradient products of sub-tile i - 1 (its W operands and Q values kept in
  // registers), while the epilogue of sub-tile i runs on the vector ALU.  The
  // first step's "previous" operands are zero and add nothing.
  float wp[4][RB], qvp[4], qcp[4], qbp[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    qvp[v] = qcp[v] = qbp[v] = 0.f;
#pragma unroll
    for (int q = 0; q < RB; ++q) wp[v][q] = 0.f;
  }
  // u, u_c, y: contraction over the rows n = 16w + 4g' + v of this wave
  auto grad = [&]() {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        acc[0][q] = mfma16(wp[v][q], qvp[v], acc[0][q]);
        acc[1][q] = mfma16(wp[v][q], qcp[v], acc[1][q]);
        acc[2][q] = mfma16(wp[v][q] * wp[v][q], qbp[v], acc[2][q]);
      }
  };
  run([&](const float* L, int64_t nb, const float (&vf)[4]) {
    float wn[4][RB];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int q = 0; q < RB; ++q) wn[v][q] = L[wsw(16 * w + 4 * g + v, 16 * q + j)];
    // Z at rows 16w + 4g + v, column col; contraction r = 16q + 4g' + m
    f32x4 z0 = {0.f, 0.f, 0.f, 0.f}, z1 = z0;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const f32x4 a4 = *reinterpret_cast<const f32x4*>(L + wsw(16 * w + j, 16 * q + 4 * g));
      z0 = mfma16(a4[0], hb[q][0], z0);
      z1 = mfma16(a4[1], hb[q][1], z1);
      z0 = mfma16(a4[2], hb[q][2], z0);
      z1 = mfma16(a4[3], hb[q][3], z1);
    }
    grad();
    const int64_t n0 = nb + 16 * w + 4 * g;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const float x = vf[v], z = z0[v] + z1[v];   // x = 0 outside the matrix
      const float iz = __builtin_amdgcn_rcpf(z);
      const float q = x > 0.f ? x * iz : 0.f;
      qvp[v] = q;
      qcp[v] = n0 + v < N ? q - 1.f : 0.f;        // rows past N hold repeated W rows
      qbp[v] = x > 0.f ? q * iz : 0.f;
      if (CHK) bad |= (x > 0.f && !(z > 0.f)) ? 1 : 0;
      vs += (double)x;
#pragma unroll
      for (int q2 = 0; q2 < RB; ++q2) wp[v][q2] = wn[v][q2];
    }
    // the Z products with the operand reads, then the gradient products with
    // the epilogue between them
#pragma unroll
    for (int k = 0; k < 4 * RB; ++k) {
      __builtin_amdgcn_sched_group_barrier(SG_MFMA, 1, 0);
      __builtin_amdgcn_sched_group_barrier(SG_DSR, 1, 0);
    }
    interleave_mfma_valu<12 * RB, 2>();
  });
  grad();                                         // the last sub-tile

  // ---------------- candidates ----------------
  // the four waves' partial sums, added in wave order: thread (tt, r = rq + 16i)
  float gs[3][4];
  {
    float* red = ring[2];                         // 4 waves x 64 x 16 floats per product
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int q = 0; q < RB; ++q)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[(w * 64 + 16 * q + 4 * g + v) * HC_TB + j] = acc[c][q][v];
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = rq + 16 * i;
        float s = 0.f;
        if (r < 16 * RB)
#pragma unroll
          for (int ww = 0; ww < 4; ++ww) s += red[(ww * 64 + r) * HC_TB + tt];
        gs[c][i] = s;
      }
      __syncthreads();
    }
  }
  // column sums of V over all rows (lane groups, then waves, in a fixed order)
  {
    const double s = group4_sum(vs);
    if (g == 0) dred[w][j] = s;
  }
  float keep[4];
  double den = 0.0;
  const float reg = (float)a.cj.reg;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = rq + 16 * i;
    float xm = 0.f;
    keep[i] = 0.f;
    if (r < R && tc < T) {
      const Cand k = candidate(hx[i], gs[0][i], gs[1][i], gs[2][i], cs[r], a.eps, a.alpha, reg);
      xm = k.mu;
      keep[i] = k.newton;
      den += (double)cs[r] * (double)k.newton;
    }
    lx[2][r * HC_XP + tt] = xm;
  }
  if (!a.xmu_out) prime();                        // pass 2, sub-tiles 0 and 1, in flight from here
  __syncthreads();                                // dred[0..3] (V sums) complete
  double vcol = 0.0;
  if (tid < HC_TB) vcol = (dred[0][tid] + dred[1][tid]) + (dred[2][tid] + dred[3][tid]);
  __syncthreads();
  dred[rq][tt] = den;
  __syncthreads();
  if (tid < HC_TB) {                              // eq. (10): the Newton column rescaled to sum v
    double d = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) d += dred[k][tid];
    fac[tid] = d > 0.0 ? vcol / d : 1.0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = rq + 16 * i;
    float xn = 0.f;
    if (r < R && tc < T) xn = fmaxf((float)((double)keep[i] * fac[tt]), VALUE_FLOOR);
    lx[0][r * HC_XP + tt] = xn;
    lx[1][r * HC_XP + tt] = lx[2][r * HC_XP + tt] - xn;
  }
  if (a.xmu_out) {                                // the candidates alone (steps 2-6, 10-11)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int r = rq + 16 * i;
      if (r < R && tc < T) {
        a.xmu_out[(int64_t)r * T + tc] = lx[2][r * HC_XP + tt];
        a.xn_out[(int64_t)r * T + tc] = lx[0][r * HC_XP + tt];
      }
    }
    return;
  }
  __syncthreads();                                // the candidate tiles are complete

  // ---------------- pass 2: candidate costs ----------------
  f32x4 xb[RB], db[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int r = 16 * q + 4 * g + m;
      xb[q][m] = lx[0][r * HC_XP + j];
      db[q][m] = lx[1][r * HC_XP + j];
    }
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  int fl = 0;
  // the cost terms of sub-tile i - 1 run on the vector ALU behind the products
  // of sub-tile i (the first step's "previous" entries have v = 0: no terms);
  // per sub-tile float sums, added to the float64 sums
  float zp[4], dp[4], vp[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) zp[v] = dp[v] = vp[v] = 0.f;
  auto costs = [&]() {
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int v = 0; v < 4; ++v) fl |= cost_acc_f<DS>(vp[v], zp[v], dp[v], a0, a1, s2);
    if (DS) s0 += (double)a0;
    s1 += (double)a1;
  };
  run([&](const float* L, int64_t nb, const float (&vf)[4]) {
    f32x4 zn0 = {0.f, 0.f, 0.f, 0.f}, zn1 = zn0, dz0 = zn0, dz1 = zn0;
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      const f32x4 a4 = *reinterpret_cast<const f32x4*>(L + wsw(16 * w + j, 16 * q + 4 * g));
      zn0 = mfma16(a4[0], xb[q][0], zn0);
      dz0 = mfma16(a4[0], db[q][0], dz0);
      zn1 = mfma16(a4[1], xb[q][1], zn1);
      dz1 = mfma16(a4[1], db[q][1], dz1);
      zn0 = mfma16(a4[2], xb[q][2], zn0);
      dz0 = mfma16(a4[2], db[q][2], dz0);
      zn1 = mfma16(a4[3], xb[q][3], zn1);
      dz1 = mfma16(a4[3], db[q][3], dz1);
    }
    costs();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      zp[v] = zn0[v] + zn1[v];
      dp[v] = dz0[v] + dz1[v];
      vp[v] = vf[v];
    }
    interleave_mfma_valu<8 * RB, 4>();             // the products with the previous sub-tile's cost terms
  });
  costs();                                        // the last sub-tile

  // ---------------- choice (step 15), H, row sums ----------------
  {
    const double a0 = DS ? group4_sum(s0) : 0.0, a1 = group4_sum(s1), a2 = group4_sum(s2);
    if (g == 0) {
      col3[0][w][j] = a0;
      col3[1][w][j] = a1;
      col3[2][w][j] = a2;
    }
    if (fl) atomicOr(&flw[j], fl);
  }
  __syncthreads();
  if (tid < HC_TB && t0 + tid < T) {
    double q3[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      q3[k] = ((col3[k][0][tid] + col3[k][1][tid]) + (col3[k][2][tid] + col3[k][3][tid])) * LN2;
    double ds, mg;
    const bool nw = decide(q3[0], q3[1], q3[2], flw[tid], ds, mg);
    const int64_t t = t0 + tid;
    if (a.mask) a.mask[t] = nw ? 1 : 0;
    if (a.dsel) a.dsel[t] = ds;
    if (a.margin) a.margin[t] = mg;
    pick[tid] = nw ? 1 : 0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = rq + 16 * i;
    double hs = 0.0;
    if (r < R && tc < T) {
      const float h = pick[tt] ? lx[0][r * HC_XP + tt] : lx[2][r * HC_XP + tt];
      a.H[(int64_t)r * T + tc] = h;
      hs = (double)h;
    }
    // row sum over the block's 16 columns: lanes tt = 0..15 of this row group
#pragma unroll
    for (int k = 1; k < 16; k <<= 1) hs += __shfl_xor(hs, k);
    if (tt == 0 && r < R) a.emit[blk * R + r] = hs;
  }
  if (CHK && bad) atomicOr(a.check, CHK_DOMAIN);
}

hipError_t launch_hstep_cols(const HColsArgs& a, hipStream_t s) {
  if (a.R < 1 || a.R > 64) return hipErrorInvalidValue;
  const dim3 grid((unsigned)hcols_blocks(a.T));
  const int rb = (int)((a.R + 15) / 16);
  prof_begin("hstep_cols", s);
  const bool w16 = a.R % 4 == 0 && (reinterpret_cast<uintptr_t>(a.W) & 15) == 0;
  // modes: no check and no cost wanted (the choice reads the margin and the
  // flags only), the kept cost wanted, checked (with the cost)
  typedef void (*Kern)(HColsArgs);
  static const Kern table[3][4][2] = {
      {{&k_hstep_cols<1, false, false, false>, &k_hstep_cols<1, false, true, false>},
       {&k_hstep_cols<2, false, false, false>, &k_hstep_cols<2, false, true, false>},
       {&k_hstep_cols<3, false, false, false>, &k_hstep_cols<3, false, true, false>},
       {&k_hstep_cols<4, false, false, false>, &k_hstep_cols<4, false, true, false>}},
      {{&k_hstep_cols<1, false, false, true>, &k_hstep_cols<1, false, true, true>},
       {&k_hstep_cols<2, false, false, true>, &k_hstep_cols<2, false, true, true>},
       {&k_hstep_cols<3, false, false, true>, &k_hstep_cols<3, false, true, true>},
       {&k_hstep_cols<4, false, false, true>, &k_hstep_cols<4, false, true, true>}},
      {{&k_hstep_cols<1, true, false, true>, &k_hstep_cols<1, true, true, true>},
       {&k_hstep_cols<2, true, false, true>, &k_hstep_cols<2, true, true, true>},
       {&k_hstep_cols<3, true, false, true>, &k_hstep_cols<3, true, true, true>},
       {&k_hstep_cols<4, true, false, true>, &k_hstep_cols<4, true, true, true>}}};
  const int mode = a.check ? 2 : (a.dsel ? 1 : 0);
  const Kern k = table[mode][rb - 1][w16 ? 1 : 0];
  hipLaunchKernelGGL(k, grid, dim3(256), 0, s, a);
  prof_end("hstep_cols", s);
  return hipGetLastError();
}

}  // namespace dna
