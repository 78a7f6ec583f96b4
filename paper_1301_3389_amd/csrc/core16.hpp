// core16.hpp -- 16-bit operand tile engine (bf16 / fp16 MFMA, fp32 accumulate).
//
// v_mfma_f32_32x32x16_{bf16,f16}: lane l supplies 8 consecutive k (k = 8*(l/32)
// + 0..7) of row (l % 32) of A and of column (l % 32) of B; the 32x32 fp32
// result has the same register layout as the fp32 MFMA (blk_row / blk_col).
// Tiles live in LDS K-major, [mn][BK + 8] elements, so a fragment is one 16-byte
// LDS read per lane.  Global operands are fp32 or 16-bit, K- or MN-contiguous;
// staging converts to 16-bit after an optional transform in fp32:
//   XF_ID: x          XF_SQ: x*x          XF_P1: x + a (a per MN index, default 1)
//   XF_LO: x - round16(x), the low part of a two-term split x = hi + lo
// after optional power-of-two scales, per K index (exactly compensated between
// the two operands of a product) or per MN index (folded out of the result).
#pragma once
#include "core.hpp"

namespace dna {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

template <typename TE>
struct MF;
template <>
struct MF<__bf16> {
  typedef bf16x8 v8;
  typedef bf16x4 v4;
  __device__ __forceinline__ static f32x16 mma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct MF<_Float16> {
  typedef f16x8 v8;
  typedef f16x4 v4;
  __device__ __forceinline__ static f32x16 mma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

enum Xform { XF_ID = 0, XF_SQ = 1, XF_P1 = 2, XF_LO = 3 };

// A global operand for the 16-bit engine.  `p` holds fp32 or 16-bit elements
// (the stage's SRC type); `p2` (same type and layout) is subtracted when set.
// `sk` / `smn`: optional scale vectors indexed by K / by MN (nullptr = 1); the
// staged value is x * sk[k] * smn[mn] (each squared under XF_SQ).
struct Op16 {
  const void* p;
  const void* p2;
  int64_t ld;
  int64_t mn_end;
  const float* sk;
  const float* smn;
  const float* addmn;   // XF_P1 adds addmn[mn] (nullptr: 1)
  int vec;
};

template <typename SRC>
__host__ inline Op16 make_op16(const SRC* p, int64_t ld, int64_t mn_end, const SRC* p2 = nullptr,
                               const float* sk = nullptr, const float* smn = nullptr,
                               const float* addmn = nullptr) {
  Op16 o;
  o.p = p;
  o.p2 = p2;
  o.ld = ld;
  o.mn_end = mn_end;
  o.sk = sk;
  o.smn = smn;
  o.addmn = addmn;
  const uintptr_t al = 16;
  const int per16 = 16 / (int)sizeof(SRC);          // elements per 16 bytes
  bool v = (reinterpret_cast<uintptr_t>(p) % al == 0) && (ld % per16 == 0);
  if (p2) v = v && (reinterpret_cast<uintptr_t>(p2) % al == 0);
  o.vec = v ? 1 : 0;
  return o;
}

template <int BM_, int BN_, int BK_, int WGM_, int WGN_>
struct Geo16 {
  static constexpr int BM = BM_, BN = BN_, BK = BK_;
  static constexpr int WGM = WGM_, WGN = WGN_;
  static constexpr int WAVES = WGM * WGN;
  static constexpr int NT = 64 * WAVES;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int FM = WM / 32, FN = WN / 32;
  static constexpr int PITCH = BK + 8;              // LDS row pitch in elements
  static_assert(BK % 16 == 0, "BK must be a multiple of the MFMA K (16)");
  static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be a multiple of 32");
};

template <typename SRC>
__device__ __forceinline__ float ld1(const void* p, int64_t i) {
  return (float)(reinterpret_cast<const SRC*>(p)[i]);
}

// Stage of one MN x BK operand tile.
//   K-major source: a unit is 8 consecutive k at one mn (one 16-byte LDS store).
//   MN-major source: a unit is 8 k x 4 mn (four 16-byte LDS stores after an
//   in-register transpose).
template <int MN, int BK, int NT, typename SRC, typename TE, bool KMAJ, int XF = XF_ID>
struct Stage16 {
  static constexpr int NU = KMAJ ? MN * BK / 8 : MN * BK / 32;
  static constexpr int PT = (NU + NT - 1) / NT;
  static constexpr int PITCH = BK + 8;
  float r[PT][KMAJ ? 8 : 32];

  __device__ __forceinline__ void load(const Op16& o, int64_t mn0, int64_t k0, int64_t k_end, int tid) {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int f = tid + i * NT;
      if (NU % NT != 0 && f >= NU) break;
      if (KMAJ) {
        const int row = f / (BK / 8), kq = (f % (BK / 8)) * 8;
        const int64_t mn = mn0 + row, k = k0 + kq;
#pragma unroll
        for (int j = 0; j < 8; ++j) r[i][j] = 0.f;
        if (mn < o.mn_end) {
          const int64_t base = mn * o.ld + k;
          if (o.vec && k + 7 < k_end) {
            if (sizeof(SRC) == 4) {
              const f32x4 a = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.p) + base);
              const f32x4 b = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.p) + base + 4);
#pragma unroll
              for (int j = 0; j < 4; ++j) { r[i][j] = a[j]; r[i][j + 4] = b[j]; }
              if (o.p2) {
                const f32x4 c = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.p2) + base);
                const f32x4 d = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.p2) + base + 4);
#pragma unroll
                for (int j = 0; j < 4; ++j) { r[i][j] -= c[j]; r[i][j + 4] -= d[j]; }
              }
            } else {
              typedef typename MF<TE>::v8 V8;
              const V8 a = *reinterpret_cast<const V8*>(reinterpret_cast<const TE*>(o.p) + base);
#pragma unroll
              for (int j = 0; j < 8; ++j) r[i][j] = (float)a[j];
            }
          } else {
#pragma unroll
            for (int j = 0; j < 8; ++j)
              if (k + j < k_end) r[i][j] = ld1<SRC>(o.p, base + j) - (o.p2 ? ld1<SRC>(o.p2, base + j) : 0.f);
          }
        }
      } else {
        const int mq = (f % (MN / 4)) * 4, kb = (f / (MN / 4)) * 8;
        const int64_t mn = mn0 + mq;
#pragma unroll
        for (int j = 0; j < 32; ++j) r[i][j] = 0.f;
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
          const int64_t k = k0 + kb + kk;
          if (k >= k_end) continue;
          const int64_t base = k * o.ld + mn;
          if (o.vec && mn + 3 < o.mn_end) {
            if (sizeof(SRC) == 4) {
              f32x4 a = *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.p) + base);
              if (o.p2) a -= *reinterpret_cast<const f32x4*>(reinterpret_cast<const float*>(o.p2) + base);
#pragma unroll
              for (int j = 0; j < 4; ++j) r[i][j * 8 + kk] = a[j];
            } else {
              typedef typename MF<TE>::v4 V4;
              const V4 a = *reinterpret_cast<const V4*>(reinterpret_cast<const TE*>(o.p) + base);
#pragma unroll
              for (int j = 0; j < 4; ++j) r[i][j * 8 + kk] = (float)a[j];
            }
          } else {
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (mn + j < o.mn_end)
                r[i][j * 8 + kk] = ld1<SRC>(o.p, base + j) - (o.p2 ? ld1<SRC>(o.p2, base + j) : 0.f);
          }
        }
      }
    }
  }

  // Apply scales and the transform, convert, and write to LDS.
  template <int X>
  __device__ __forceinline__ float finish(float x, const Op16& o, int64_t mn, int64_t k, int64_t k_end) const {
    float s = 1.f;
    if (o.smn && mn < o.mn_end) s = o.smn[mn];
    if (o.sk) s *= (k < k_end) ? o.sk[k] : 0.f;
    x *= s;
    if (X == XF_SQ) return x * x;
    if (X == XF_P1) return x + ((o.addmn && mn < o.mn_end) ? o.addmn[mn] : 1.f);
    if (X == XF_LO) return x - (float)(TE)x;
    return x;
  }

  template <int X = XF>
  __device__ __forceinline__ void store(TE* lds, const Op16& o, int64_t mn0, int64_t k0, int64_t k_end,
                                        int tid) const {
    typedef typename MF<TE>::v8 V8;
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int f = tid + i * NT;
      if (NU % NT != 0 && f >= NU) break;
      if (KMAJ) {
        const int row = f / (BK / 8), kq = (f % (BK / 8)) * 8;
        V8 v;
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (TE)finish<X>(r[i][j], o, mn0 + row, k0 + kq + j, k_end);
        *reinterpret_cast<V8*>(lds + row * PITCH + kq) = v;
      } else {
        const int mq = (f % (MN / 4)) * 4, kb = (f / (MN / 4)) * 8;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          V8 v;
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) v[kk] = (TE)finish<X>(r[i][j * 8 + kk], o, mn0 + mq + j, k0 + kb + kk, k_end);
          *reinterpret_cast<V8*>(lds + (mq + j) * PITCH + kb) = v;
        }
      }
    }
  }
};

// Fragment of a K-major LDS tile: 8 consecutive k of row `row` at k-step kk16.
template <typename TE>
__device__ __forceinline__ typename MF<TE>::v8 frag16(const TE* tile, int pitch, int row, int kk16, int lane) {
  typedef typename MF<TE>::v8 V8;
  return *reinterpret_cast<const V8*>(tile + row * pitch + kk16 * 16 + 8 * (lane >> 5));
}

// The K loop shared by every 16-bit kernel.  The policy P provides
//   NC, LDS_ELEMS (elements of TE for one staged K-tile),
//   load(k0, k_end, tid), store(lds, k0, k_end, tid)  -- all of its operands,
//   compute(lds, acc, lane, wm, wn)                   -- one staged K-tile.
// LDS holds one K-tile; the next one is prefetched into registers while the
// current one feeds the matrix cores.
template <class G, class P, typename TE>
__device__ __forceinline__ void run16(P& pol, f32x16 (&acc)[G::FM][G::FN][P::NC], int64_t k_begin,
                                      int64_t k_end, TE* lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % G::WGM, wn = wave / G::WGM;
  const int64_t nk = (k_end - k_begin + G::BK - 1) / G::BK;
  if (nk <= 0) return;
  pol.load(k_begin, k_end, tid);
  pol.store(lds, k_begin, k_end, tid);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const bool more = kt + 1 < nk;
    const int64_t kn = k_begin + (kt + 1) * G::BK;
    if (more) pol.load(kn, k_end, tid);
    pol.compute(lds, acc, lane, wm, wn);
    __syncthreads();
    if (more) {
      pol.store(lds, kn, k_end, tid);
      __syncthreads();
    }
  }
}

template <class G>
__device__ __forceinline__ int64_t row16(int64_t m0, int i, int v) {
  const int tid = threadIdx.x, lane = tid & 63, wm = (tid >> 6) % G::WGM;
  return m0 + wm * G::WM + i * 32 + blk_row(v, lane);
}
template <class G>
__device__ __forceinline__ int64_t col16(int64_t n0, int j) {
  const int tid = threadIdx.x, lane = tid & 63, wn = (tid >> 6) / G::WGM;
  return n0 + wn * G::WN + j * 32 + blk_col(lane);
}

template <class G, int NC>
__device__ __forceinline__ void zero16(f32x16 (&acc)[G::FM][G::FN][NC]) {
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[i][j][c][v] = 0.f;
}

}  // namespace dna
