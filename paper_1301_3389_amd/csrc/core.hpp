// core.hpp -- MFMA tile machinery shared by every libdna kernel (gfx950).
//
// A workgroup computes a BM x BN tile of one or more products C_i += A_a * B_b
// with K-tiles staged through LDS (double buffered, register prefetch of the
// next K-tile while the current one feeds the matrix cores).  FP32 operands use
// v_mfma_f32_32x32x2_f32 on 32x32 blocks; a wave owns WM x WN = (FM*32) x (FN*32).
//
// Operands are logical MN x K matrices in global memory, either K-contiguous
// ("K-major": element (mn,k) at p[mn*ld + k]) or MN-contiguous (p[k*ld + mn]).
// Both are staged into LDS as [k][mn] rows so that the 32 lanes of a fragment
// read consecutive words.  An operand may carry a second pointer p2: the staged
// value is then p - p2 (used for the candidate difference H_MU - H_DNA).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dna {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct Opnd {
  const float* p;
  const float* p2;   // nullptr, or subtract this operand (same layout and ld)
  int64_t ld;
  int64_t mn_end;    // valid extent along MN
  int vec;           // 1 if 16-byte vector loads are legal (ld % 4 == 0, 16B aligned)
};

__host__ __device__ inline Opnd make_opnd(const float* p, int64_t ld, int64_t mn_end,
                                          const float* p2 = nullptr) {
  Opnd o;
  o.p = p;
  o.p2 = p2;
  o.ld = ld;
  o.mn_end = mn_end;
  bool al = ((reinterpret_cast<uintptr_t>(p) & 15) == 0) && (ld % 4 == 0);
  if (p2) al = al && ((reinterpret_cast<uintptr_t>(p2) & 15) == 0);
  o.vec = al ? 1 : 0;
  return o;
}

template <int BM_, int BN_, int BK_, int WGM_, int WGN_>
struct Geo {
  static constexpr int BM = BM_, BN = BN_, BK = BK_;
  static constexpr int WGM = WGM_, WGN = WGN_;
  static constexpr int WAVES = WGM * WGN;
  static constexpr int NT = 64 * WAVES;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int FM = WM / 32, FN = WN / 32;
  static constexpr int LDA = BM + 4, LDB = BN + 4;   // LDS row pitch (floats)
  static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be a multiple of 32");
  static_assert(BK % 4 == 0, "BK must be a multiple of 4");
};

// Fetch 4 consecutive elements along the contiguous dimension, zero outside.
template <bool KMAJ>
__device__ __forceinline__ f32x4 fetch4(const Opnd& o, int64_t mn, int64_t k, int64_t k_end) {
  f32x4 r = {0.f, 0.f, 0.f, 0.f};
  if (KMAJ) {
    if (mn >= o.mn_end) return r;
    const int64_t base = mn * o.ld + k;
    if (o.vec && k + 3 < k_end) {
      r = *reinterpret_cast<const f32x4*>(o.p + base);
      if (o.p2) r -= *reinterpret_cast<const f32x4*>(o.p2 + base);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (k + j < k_end) r[j] = o.p[base + j] - (o.p2 ? o.p2[base + j] : 0.f);
    }
  } else {
    if (k >= k_end) return r;
    const int64_t base = k * o.ld + mn;
    if (o.vec && mn + 3 < o.mn_end) {
      r = *reinterpret_cast<const f32x4*>(o.p + base);
      if (o.p2) r -= *reinterpret_cast<const f32x4*>(o.p2 + base);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        if (mn + j < o.mn_end) r[j] = o.p[base + j] - (o.p2 ? o.p2[base + j] : 0.f);
    }
  }
  return r;
}

// Register stage of one MN x BK operand tile (MN = BM or BN).  A DIFF stage
// may hold a difference operand (Opnd::p2 set): its unchecked loads keep both
// terms in registers and subtract them when the stage is stored, so that no
// load result is consumed before the stage's LDS store.
template <int MN, int BK, int NT, bool KMAJ, bool DIFF = false>
struct Stage {
  static constexpr int NV = MN * BK / 4;
  static constexpr int PT = (NV + NT - 1) / NT;
  f32x4 r[PT];
  f32x4 r2[DIFF ? PT : 1];

  // Element offset of this thread's i-th vector from the tile origin (mn0, k0).
  __device__ __forceinline__ static int64_t offset(int f, int64_t ld) {
    if (KMAJ) return (int64_t)(f / (BK / 4)) * ld + (f % (BK / 4)) * 4;
    return (int64_t)(f / (MN / 4)) * ld + (f % (MN / 4)) * 4;
  }

  // Bounds-checked loads (any tile, any alignment).
  __device__ __forceinline__ void load(const Opnd& o, int64_t mn0, int64_t k0, int64_t k_end, int tid) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int f = tid + i * NT;
      if (NV % NT != 0 && f >= NV) break;
      if (KMAJ) {
        const int row = f / (BK / 4), kq = (f % (BK / 4)) * 4;
        r[i] = fetch4<true>(o, mn0 + row, k0 + kq, k_end);
      } else {
        const int kr = f / (MN / 4), mq = (f % (MN / 4)) * 4;
        r[i] = fetch4<false>(o, mn0 + mq, k0 + kr, k_end);
      }
      if (DIFF) r2[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }

  // Unchecked 16-byte loads: the caller has established that the whole tile
  // lies inside the operand and that o.vec holds.
  __device__ __forceinline__ void load_fast(const Opnd& o, int64_t mn0, int64_t k0, int tid) {
    const int64_t origin = KMAJ ? mn0 * o.ld + k0 : k0 * o.ld + mn0;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int f = tid + i * NT;
      if (NV % NT != 0 && f >= NV) break;
      r[i] = *reinterpret_cast<const f32x4*>(o.p + origin + offset(f, o.ld));
    }
    if (DIFF) {
      if (o.p2) {
#pragma unroll
        for (int i = 0; i < PT; ++i) {
          const int f = tid + i * NT;
          if (NV % NT != 0 && f >= NV) break;
          r2[i] = *reinterpret_cast<const f32x4*>(o.p2 + origin + offset(f, o.ld));
        }
      } else {
#pragma unroll
        for (int i = 0; i < PT; ++i) r2[i] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }

  __device__ __forceinline__ void store(float* lds, int tid) const {
    constexpr int LD = MN + 4;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int f = tid + i * NT;
      if (NV % NT != 0 && f >= NV) break;
      const f32x4 x = DIFF ? r[i] - r2[i] : r[i];
      if (KMAJ) {
        const int row = f / (BK / 4), kq = (f % (BK / 4)) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) lds[(kq + j) * LD + row] = x[j];
      } else {
        const int kr = f / (MN / 4), mq = (f % (MN / 4)) * 4;
        *reinterpret_cast<f32x4*>(lds + kr * LD + mq) = x;
      }
    }
  }
};

// Product lists may mark their A (B) operands as possible difference operands
// with a static member DIFF_A (DIFF_B) = true.
template <class PR, class = void>
struct DiffA {
  static constexpr bool v = false;
};
template <class PR>
struct DiffA<PR, decltype(void(PR::DIFF_A))> {
  static constexpr bool v = PR::DIFF_A;
};
template <class PR, class = void>
struct DiffB {
  static constexpr bool v = false;
};
template <class PR>
struct DiffB<PR, decltype(void(PR::DIFF_B))> {
  static constexpr bool v = PR::DIFF_B;
};

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Output coordinate of accumulator register v of a 32x32 block for this lane.
__device__ __forceinline__ int blk_row(int v, int lane) { return (v >> 2) * 8 + (lane >> 5) * 4 + (v & 3); }
__device__ __forceinline__ int blk_col(int lane) { return lane & 31; }

// The tile engine.  PR (product list) provides:
//   static constexpr int NA, NB, NC;
//   static __device__ void mma(const float (&a)[NA], const float (&b)[NB], f32x16 (&c)[NC]);
template <class G, class PR, bool AK, bool BKM>
struct Tile {
  static constexpr int NA = PR::NA, NB = PR::NB, NC = PR::NC;
  static constexpr int BUF = (NA * G::LDA + NB * G::LDB) * G::BK;  // floats per buffer
  static constexpr int LDS_FLOATS = 2 * BUF;

  f32x16 acc[G::FM][G::FN][NC];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int j = 0; j < G::FN; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int v = 0; v < 16; ++v) acc[i][j][c][v] = 0.f;
  }

  // One K tile: every fragment of the tile is read from LDS first (all reads in
  // flight together, one wait), then the MFMA chains run back to back.
  __device__ __forceinline__ void compute(const float* lds) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % G::WGM, wn = wave / G::WGM;
    const float* la = lds;
    const float* lb = lds + NA * G::LDA * G::BK;
    constexpr int KP = G::BK / 2;
    float af[KP][G::FM][NA], bf[KP][G::FN][NB];
#pragma unroll
    for (int kp = 0; kp < KP; ++kp) {
      const int kr = 2 * kp + (lane >> 5);
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int a = 0; a < NA; ++a)
          af[kp][i][a] = la[a * G::LDA * G::BK + kr * G::LDA + wm * G::WM + i * 32 + (lane & 31)];
#pragma unroll
      for (int j = 0; j < G::FN; ++j)
#pragma unroll
        for (int b = 0; b < NB; ++b)
          bf[kp][j][b] = lb[b * G::LDB * G::BK + kr * G::LDB + wn * G::WN + j * 32 + (lane & 31)];
    }
#pragma unroll
    for (int kp = 0; kp < KP; ++kp)
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j) PR::mma(af[kp][i], bf[kp][j], acc[i][j]);
  }

  typedef Stage<G::BM, G::BK, G::NT, AK, DiffA<PR>::v> SA;
  typedef Stage<G::BN, G::BK, G::NT, BKM, DiffB<PR>::v> SB;

  // Whether the tile's MN ranges lie inside every operand and all of them take
  // 16-byte loads: then every K tile but a ragged last one loads unchecked.
  __device__ __forceinline__ static bool interior(const Opnd (&A)[NA], const Opnd (&B)[NB], int64_t m0, int64_t n0) {
    bool ok = true;
#pragma unroll
    for (int a = 0; a < NA; ++a) ok = ok && A[a].vec && m0 + G::BM <= A[a].mn_end && (DiffA<PR>::v || !A[a].p2);
#pragma unroll
    for (int b = 0; b < NB; ++b) ok = ok && B[b].vec && n0 + G::BN <= B[b].mn_end && (DiffB<PR>::v || !B[b].p2);
    return ok;
  }

  __device__ __forceinline__ static void load_stage(SA (&sa)[NA], SB (&sb)[NB], const Opnd (&A)[NA],
                                                    const Opnd (&B)[NB], int64_t m0, int64_t n0, int64_t k,
                                                    int64_t k_end, bool inner, int tid) {
    if (inner && k + G::BK <= k_end) {
#pragma unroll
      for (int a = 0; a < NA; ++a) sa[a].load_fast(A[a], m0, k, tid);
#pragma unroll
      for (int b = 0; b < NB; ++b) sb[b].load_fast(B[b], n0, k, tid);
    } else {
#pragma unroll
      for (int a = 0; a < NA; ++a) sa[a].load(A[a], m0, k, k_end, tid);
#pragma unroll
      for (int b = 0; b < NB; ++b) sb[b].load(B[b], n0, k, k_end, tid);
    }
  }

  __device__ __forceinline__ static void store_stage(const SA (&sa)[NA], const SB (&sb)[NB], float* buf, int tid) {
#pragma unroll
    for (int a = 0; a < NA; ++a) sa[a].store(buf + a * G::LDA * G::BK, tid);
#pragma unroll
    for (int b = 0; b < NB; ++b) sb[b].store(buf + NA * G::LDA * G::BK + b * G::LDB * G::BK, tid);
  }

  // Accumulate over k in [k_begin, k_end).  lds must hold LDS_FLOATS floats.
  __device__ __forceinline__ void run(const Opnd (&A)[NA], const Opnd (&B)[NB], int64_t m0, int64_t n0,
                                      int64_t k_begin, int64_t k_end, float* lds) {
    run_flush(A, B, m0, n0, k_begin, k_end, lds, 1 << 30, [](int) {});
  }

  // run() with a hook: after every `tiles_per_chunk` K-tiles of this range (and
  // after the last one) flush(c) is called with the chunk's index c = 0, 1, ...
  // counted from k_begin, while the next K-tile's loads are in flight.
  template <class FL>
  __device__ __forceinline__ void run_flush(const Opnd (&A)[NA], const Opnd (&B)[NB], int64_t m0, int64_t n0,
                                            int64_t k_begin, int64_t k_end, float* lds, int tiles_per_chunk,
                                            FL&& flush) {
    const int tid = threadIdx.x;
    const int64_t nk = (k_end - k_begin + G::BK - 1) / G::BK;
    if (nk <= 0) return;
    const bool inner = interior(A, B, m0, n0);
    SA sa[NA];
    SB sb[NB];
    load_stage(sa, sb, A, B, m0, n0, k_begin, k_end, inner, tid);
    store_stage(sa, sb, lds, tid);
    __syncthreads();
    int in_chunk = 0, chunk = 0;
    for (int64_t kt = 0; kt < nk; ++kt) {
      const bool more = kt + 1 < nk;
      if (more) load_stage(sa, sb, A, B, m0, n0, k_begin + (kt + 1) * G::BK, k_end, inner, tid);
      compute(lds + (kt & 1) * BUF);
      if (++in_chunk == tiles_per_chunk || !more) {
        flush(chunk);
        ++chunk;
        in_chunk = 0;
      }
      if (more) store_stage(sa, sb, lds + ((kt + 1) & 1) * BUF, tid);
      __syncthreads();
    }
  }

  // Load X[row][col] (row-major, leading dimension ld) at this lane's accumulator
  // positions.  Indices are clamped into the matrix so that every load is issued
  // unconditionally (and early, before the K loop); callers ignore the clamped
  // entries.
  __device__ __forceinline__ static void load_frag(float (&out)[G::FM][G::FN][16], const float* X, int64_t ld,
                                                   int64_t m0, int64_t n0, int64_t M, int64_t Ncols) {
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = min(col_of(n0, j), Ncols - 1);
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = min(row_of(m0, i, v), M - 1);
          out[i][j][v] = X[row * ld + col];
        }
    }
  }

  // Global (row, col) of accumulator element (i, j, v) for this thread.
  __device__ __forceinline__ static int64_t row_of(int64_t m0, int i, int v) {
    const int tid = threadIdx.x, lane = tid & 63, wm = (tid >> 6) % G::WGM;
    return m0 + wm * G::WM + i * 32 + blk_row(v, lane);
  }
  __device__ __forceinline__ static int64_t col_of(int64_t n0, int j) {
    const int tid = threadIdx.x, lane = tid & 63, wn = (tid >> 6) / G::WGM;
    return n0 + wn * G::WN + j * 32 + blk_col(lane);
  }
};

// ---- product lists -------------------------------------------------------

struct ProdSingle {  // C0 += A0 B0
  static constexpr int NA = 1, NB = 1, NC = 1;
  __device__ __forceinline__ static void mma(const float (&a)[1], const float (&b)[1], f32x16 (&c)[1]) {
    c[0] = mfma32(a[0], b[0], c[0]);
  }
};
struct ProdDualB_SqA {  // C0 += A B0, C1 += (A*A) B1   (W^t Q and (W*W)^t Q-bar)
  static constexpr int NA = 1, NB = 2, NC = 2;
  __device__ __forceinline__ static void mma(const float (&a)[1], const float (&b)[2], f32x16 (&c)[2]) {
    c[0] = mfma32(a[0], b[0], c[0]);
    c[1] = mfma32(a[0] * a[0], b[1], c[1]);
  }
};
struct ProdDualA_SqB {  // C0 += A0 B, C1 += A1 (B*B)   (Q H^t and Q-bar (H*H)^t)
  static constexpr int NA = 2, NB = 1, NC = 2;
  __device__ __forceinline__ static void mma(const float (&a)[2], const float (&b)[1], f32x16 (&c)[2]) {
    c[0] = mfma32(a[0], b[0], c[0]);
    c[1] = mfma32(a[1], b[0] * b[0], c[1]);
  }
};
// Gradient / Hessian numerators with both forms of the gradient sum:
//   C0 += w q          (u,  relative accuracy of the MU gain u/c)
//   C1 += w (q - 1)    (u_c = u - c, absolute accuracy of A = u_c/c near 0)
//   C2 += w^2 q-bar    (y)
// Zero-filled padding contributes nothing: w = 0 there.
struct ProdGH3_H {  // A = W^t (shared), B0 = Q, B1 = Q-bar
  static constexpr int NA = 1, NB = 2, NC = 3;
  __device__ __forceinline__ static void mma(const float (&a)[1], const float (&b)[2], f32x16 (&c)[3]) {
    c[0] = mfma32(a[0], b[0], c[0]);
    c[1] = mfma32(a[0], b[0] - 1.f, c[1]);
    c[2] = mfma32(a[0] * a[0], b[1], c[2]);
  }
};
struct ProdGH3_W {  // A0 = Q, A1 = Q-bar, B = H^t (shared)
  static constexpr int NA = 2, NB = 1, NC = 3;
  __device__ __forceinline__ static void mma(const float (&a)[2], const float (&b)[1], f32x16 (&c)[3]) {
    c[0] = mfma32(a[0], b[0], c[0]);
    c[1] = mfma32(a[0] - 1.f, b[0], c[1]);
    c[2] = mfma32(a[1], b[0] * b[0], c[2]);
  }
};

struct ProdDualB {  // C0 += A B0, C1 += A B1   (B1 may be a difference operand)
  static constexpr int NA = 1, NB = 2, NC = 2;
  static constexpr bool DIFF_B = true;
  __device__ __forceinline__ static void mma(const float (&a)[1], const float (&b)[2], f32x16 (&c)[2]) {
    c[0] = mfma32(a[0], b[0], c[0]);
    c[1] = mfma32(a[0], b[1], c[1]);
  }
};
struct ProdDualA {  // C0 += A0 B, C1 += A1 B   (A1 may be a difference operand)
  static constexpr int NA = 2, NB = 1, NC = 2;
  static constexpr bool DIFF_A = true;
  __device__ __forceinline__ static void mma(const float (&a)[2], const float (&b)[1], f32x16 (&c)[2]) {
    c[0] = mfma32(a[0], b[0], c[0]);
    c[1] = mfma32(a[1], b[0], c[1]);
  }
};

// ---- deterministic reductions over a tile --------------------------------

// Sum over the 32 lanes of each half-wave for 16 per-lane slots (one value per
// row of a 32x32 accumulator block), by halving exchanges.  On return lane l
// holds the full 32-lane sum of slot ((l >> 1) & 15); lanes l and l^1 agree.
__device__ __forceinline__ double halfwave_slot_sum(double (&x)[16], int lane) {
  double y8[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const bool hi = lane & 16;
    const double send = hi ? x[j] : x[j + 8];
    const double keep = hi ? x[j + 8] : x[j];
    y8[j] = keep + __shfl_xor(send, 16);
  }
  double y4[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const bool hi = lane & 8;
    const double send = hi ? y8[j] : y8[j + 4];
    const double keep = hi ? y8[j + 4] : y8[j];
    y4[j] = keep + __shfl_xor(send, 8);
  }
  double y2[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const bool hi = lane & 4;
    const double send = hi ? y4[j] : y4[j + 2];
    const double keep = hi ? y4[j + 2] : y4[j];
    y2[j] = keep + __shfl_xor(send, 4);
  }
  const bool hi = lane & 2;
  const double send = hi ? y2[0] : y2[1];
  const double keep = hi ? y2[1] : y2[0];
  double y = keep + __shfl_xor(send, 2);
  return y + __shfl_xor(y, 1);
}

// Slot s of halfwave_slot_sum corresponds to block row blk_row(s, lane).
__device__ __forceinline__ int slot_row(int lane) {
  const int s = (lane >> 1) & 15;
  return (s >> 2) * 8 + (lane >> 5) * 4 + (s & 3);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}
__device__ __forceinline__ float wave_sumf(float x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m);
  return x;
}
__device__ __forceinline__ int wave_or(int x) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) x |= __shfl_xor(x, m);
  return x;
}

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// Remap the dispatch order so that every XCD receives one contiguous range of
// the logical tile order (x fastest): tiles that are neighbours along x -- and
// share an operand block -- then run on the same XCD at the same time.
struct Tile3 {
  int64_t x, y, z;
};
__device__ __forceinline__ Tile3 xcd_tile() {
  const int64_t gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const int64_t total = gx * gy * gz;
  const int64_t b = (int64_t)blockIdx.x + gx * ((int64_t)blockIdx.y + gy * (int64_t)blockIdx.z);
  const int64_t q = total / 8, rem = total % 8, x = b % 8, s = b / 8;
  const int64_t L = (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + s;
  Tile3 t;
  t.x = L % gx;
  t.y = (L / gx) % gy;
  t.z = L / (gx * gy);
  return t;
}

// The same XCD ranges over a grouped logical order: the x-y plane of tiles is cut
// into bands of GY rows (y) and inside a band y runs fastest.  A window of
// consecutive tiles then covers about as many x as y blocks, so the operand
// blocks of both sides are each read once by the tiles that share them on an
// XCD, whichever side is the larger one.  A grid of fewer than two workgroups
// per CU keeps the dispatch order: its operands stay in the caches anyway, and
// there the remap measured slower.
template <int GY>
__device__ __forceinline__ Tile3 xcd_tile_grouped() {
  const int64_t gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
  const int64_t plane = gx * gy, total = plane * gz;
  if (total < 512) return Tile3{(int64_t)blockIdx.x, (int64_t)blockIdx.y, (int64_t)blockIdx.z};
  const int64_t b = (int64_t)blockIdx.x + gx * ((int64_t)blockIdx.y + gy * (int64_t)blockIdx.z);
  const int64_t q = total / 8, rem = total % 8, x = b % 8, s = b / 8;
  const int64_t L = (x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q) + s;
  const int64_t l = L % plane, band = l / (GY * gx), y0 = band * GY;
  const int64_t h = gy - y0 < GY ? gy - y0 : GY, o = l - band * GY * gx;
  Tile3 t;
  t.y = y0 + o % h;
  t.x = o / h;
  t.z = L / plane;
  return t;
}

}  // namespace dna
