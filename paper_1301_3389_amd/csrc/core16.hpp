// core16.hpp -- 16-bit operand GEMM engine (bf16 / fp16 MFMA, fp32 accumulate).
//
// Every operand is a zero-padded, K-contiguous 16-bit matrix prepared by a
// conversion pass: element (mn, k) at p[mn * ld + k], with the MN extent padded
// to the tile size and K padded to a multiple of BK.  The K loop therefore has
// no bounds tests, no transforms and no scalar fallbacks: 16-byte global loads
// into registers, 16-byte LDS stores, one 16-byte LDS read per lane and
// fragment.
//
// v_mfma_f32_32x32x16_{bf16,f16}: lane l supplies 8 consecutive k (k = 8*(l/32)
// + 0..7) of row (l % 32) of A and of column (l % 32) of B; the 32x32 fp32
// result has the register layout of the fp32 MFMA (blk_row / blk_col).
#pragma once
#include "core.hpp"

namespace dna {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

template <typename TE>
struct MF;
template <>
struct MF<__bf16> {
  typedef bf16x8 v8;
  __device__ __forceinline__ static f32x16 mma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct MF<_Float16> {
  typedef f16x8 v8;
  __device__ __forceinline__ static f32x16 mma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// BM x BN tile, BK = 32, four waves in a 2 x 2 grid, wave tile (BM/2) x (BN/2).
template <int BM_, int BN_>
struct G16 {
  static constexpr int BM = BM_, BN = BN_, BK = 32;
  static constexpr int WGM = 2, WGN = 2, WAVES = 4, NT = 256;
  static constexpr int WM = BM / WGM, WN = BN / WGN;
  static constexpr int FM = WM / 32, FN = WN / 32;
  static constexpr int PITCH = BK + 8;               // LDS row pitch in elements (80 bytes)
  static constexpr int TA = BM * PITCH, TB = BN * PITCH;
  static_assert(WM % 32 == 0 && WN % 32 == 0, "wave tile must be a multiple of 32");
};

// A padded 16-bit operand (element (mn, k) at p[mn * ld + k]).
struct Mat16 {
  const void* p;
  int64_t ld;
};

// Registers of one MN x BK tile in flight: 16-byte chunks of 8 k-values.
template <int MN, int BK, int NT>
struct Ld16 {
  static constexpr int CPR = BK / 8;
  static constexpr int CH = MN * CPR;
  static_assert(CH % NT == 0, "tile chunks must divide among the threads");
  static constexpr int PT = CH / NT;
  static constexpr int PITCH = BK + 8;
  u32x4 r[PT];

  __device__ __forceinline__ void load(const Mat16& m, int64_t mn0, int64_t k0, int tid) {
    const uint16_t* p = reinterpret_cast<const uint16_t*>(m.p);
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int f = tid + i * NT;
      const int row = f / CPR, kq = (f % CPR) * 8;
      r[i] = *reinterpret_cast<const u32x4*>(p + (mn0 + row) * m.ld + k0 + kq);
    }
  }
  __device__ __forceinline__ void store(uint16_t* lds, int tid) const {
#pragma unroll
    for (int i = 0; i < PT; ++i) {
      const int f = tid + i * NT;
      const int row = f / CPR, kq = (f % CPR) * 8;
      *reinterpret_cast<u32x4*>(lds + row * PITCH + kq) = r[i];
    }
  }
};

// Product list: product c adds A operand aof(c) times B operand bof(c) into
// accumulator cof(c).  NACC accumulators in all.
template <int NA_, int NB_, int NC_, int NACC_, int A0, int B0, int C0, int A1 = 0, int B1 = 0, int C1 = 0,
          int A2 = 0, int B2 = 0, int C2 = 0>
struct Prods {
  static constexpr int NA = NA_, NB = NB_, NC = NC_, NACC = NACC_;
  __device__ __forceinline__ static constexpr int aof(int c) { return c == 0 ? A0 : (c == 1 ? A1 : A2); }
  __device__ __forceinline__ static constexpr int bof(int c) { return c == 0 ? B0 : (c == 1 ? B1 : B2); }
  __device__ __forceinline__ static constexpr int cof(int c) { return c == 0 ? C0 : (c == 1 ? C1 : C2); }
};

// The K loop over k in [k0, k1), (k1 - k0) a multiple of BK.  LDS holds two
// buffers of NA A tiles and NB B tiles (uint16_t elements, LDS_ELEMS in all);
// the next K tile is loaded into registers while the current one feeds the
// matrix cores, one barrier per K tile.
template <class G, typename TE, class PR>
struct Gemm16 {
  static constexpr int NA = PR::NA, NB = PR::NB, NC = PR::NC, NACC = PR::NACC;
  static constexpr int BUF = NA * G::TA + NB * G::TB;
  static constexpr int LDS_ELEMS = 2 * BUF;
  typedef typename MF<TE>::v8 V8;

  __device__ __forceinline__ static void compute(const uint16_t* buf, f32x16 (&acc)[G::FM][G::FN][NACC], int lane,
                                                 int wm, int wn) {
#pragma unroll
    for (int kk = 0; kk < G::BK / 16; ++kk) {
      const int ko = kk * 16 + 8 * (lane >> 5);
      V8 af[NA][G::FM], bf[NB][G::FN];
#pragma unroll
      for (int x = 0; x < NA; ++x)
#pragma unroll
        for (int i = 0; i < G::FM; ++i)
          af[x][i] = *reinterpret_cast<const V8*>(buf + x * G::TA + (wm * G::WM + i * 32 + (lane & 31)) * G::PITCH + ko);
#pragma unroll
      for (int y = 0; y < NB; ++y)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
          bf[y][j] = *reinterpret_cast<const V8*>(buf + NA * G::TA + y * G::TB +
                                                  (wn * G::WN + j * 32 + (lane & 31)) * G::PITCH + ko);
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
#pragma unroll
          for (int c = 0; c < NC; ++c)
            acc[i][j][PR::cof(c)] = MF<TE>::mma(af[PR::aof(c)][i], bf[PR::bof(c)][j], acc[i][j][PR::cof(c)]);
    }
  }

  __device__ __forceinline__ static void run(const Mat16 (&A)[NA], const Mat16 (&B)[NB], int64_t m0, int64_t n0,
                                             int64_t k0, int64_t k1, uint16_t* lds,
                                             f32x16 (&acc)[G::FM][G::FN][NACC]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % G::WGM, wn = wave / G::WGM;
    const int64_t nk = (k1 - k0) / G::BK;
    if (nk <= 0) return;
    Ld16<G::BM, G::BK, G::NT> la[NA];
    Ld16<G::BN, G::BK, G::NT> lb[NB];
#pragma unroll
    for (int x = 0; x < NA; ++x) la[x].load(A[x], m0, k0, tid);
#pragma unroll
    for (int y = 0; y < NB; ++y) lb[y].load(B[y], n0, k0, tid);
#pragma unroll
    for (int x = 0; x < NA; ++x) la[x].store(lds + x * G::TA, tid);
#pragma unroll
    for (int y = 0; y < NB; ++y) lb[y].store(lds + NA * G::TA + y * G::TB, tid);
    __syncthreads();
    for (int64_t kt = 0; kt < nk; ++kt) {
      const bool more = kt + 1 < nk;
      if (more) {
        const int64_t kn = k0 + (kt + 1) * G::BK;
#pragma unroll
        for (int x = 0; x < NA; ++x) la[x].load(A[x], m0, kn, tid);
#pragma unroll
        for (int y = 0; y < NB; ++y) lb[y].load(B[y], n0, kn, tid);
      }
      compute(lds + (kt & 1) * BUF, acc, lane, wm, wn);
      if (more) {
        uint16_t* nb = lds + ((kt + 1) & 1) * BUF;
#pragma unroll
        for (int x = 0; x < NA; ++x) la[x].store(nb + x * G::TA, tid);
#pragma unroll
        for (int y = 0; y < NB; ++y) lb[y].store(nb + NA * G::TA + y * G::TB, tid);
      }
      __syncthreads();
    }
  }
};

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
