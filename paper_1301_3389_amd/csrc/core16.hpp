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

// s_waitcnt immediate that waits until at most n vector-memory operations of
// this wave are outstanding (gfx9 encoding: vmcnt in bits 3:0 and 15:14;
// expcnt and lgkmcnt left at their no-wait maxima).
__host__ __device__ constexpr int vmcnt_imm(int n) { return (n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8); }

// The K loop over k in [k0, k1), (k1 - k0) a multiple of BK = 32.
//
// Operand tiles go from global memory straight into LDS (global_load_lds, 16
// bytes per lane) through STAGES ring buffers, so that STAGES - 1 K tiles are
// in flight while one feeds the matrix cores; one barrier per K tile.  A tile is
// MN rows of 64 bytes (32 k-values); the 16-byte chunk cq of row r sits at
// chunk position cq ^ ((r >> 2) & 3) of that row, which makes the 16-lane
// passes of the fragment reads hit 64 distinct banks.  The DMA writes 64
// consecutive chunks per wave instruction, so each lane fetches the global
// chunk that belongs at its position.
template <class G, typename TE, class PR, int STAGES>
struct Gemm16 {
  static constexpr int NA = PR::NA, NB = PR::NB, NC = PR::NC, NACC = PR::NACC;
  static_assert(G::BK == 32, "tile rows are 64 bytes");
  static constexpr int TAB = G::BM * 64, TBB = G::BN * 64;          // bytes per A / B tile
  static constexpr int STAGE_BYTES = NA * TAB + NB * TBB;
  static constexpr int LDS_BYTES = STAGES * STAGE_BYTES;
  static constexpr int LOADS = NA * (G::BM / 64) + NB * (G::BN / 64); // DMA instructions per thread and stage
  typedef typename MF<TE>::v8 V8;

  template <int MN>
  __device__ __forceinline__ static void issue(const Mat16& m, int64_t mn0, int64_t k0, char* tile, int tid) {
    const int wave = tid >> 6, lane = tid & 63;
    const char* base = reinterpret_cast<const char*>(m.p);
#pragma unroll
    for (int i = 0; i < MN / 64; ++i) {
      const int b = i * 4 + wave;                 // 1 KiB block of the tile written by this instruction
      const int p = b * 64 + lane;                // chunk position in the tile
      const int r = p >> 2, cq = (p & 3) ^ ((r >> 2) & 3);
      const char* g = base + ((mn0 + r) * m.ld + k0 + cq * 8) * 2;
      __builtin_amdgcn_global_load_lds((void*)g, (__attribute__((address_space(3))) void*)(tile + b * 1024), 16, 0, 0);
    }
  }

  __device__ __forceinline__ static void issue_stage(const Mat16 (&A)[NA], const Mat16 (&B)[NB], int64_t m0, int64_t n0,
                                                     int64_t k, char* st, int tid) {
#pragma unroll
    for (int x = 0; x < NA; ++x) issue<G::BM>(A[x], m0, k, st + x * TAB, tid);
#pragma unroll
    for (int y = 0; y < NB; ++y) issue<G::BN>(B[y], n0, k, st + NA * TAB + y * TBB, tid);
  }

  __device__ __forceinline__ static V8 frag(const char* tile, int row, int cq) {
    return *reinterpret_cast<const V8*>(tile + row * 64 + ((cq ^ ((row >> 2) & 3)) << 4));
  }

  __device__ __forceinline__ static void compute(const char* st, f32x16 (&acc)[G::FM][G::FN][NACC], int lane, int wm,
                                                 int wn) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      const int cq = 2 * kk + (lane >> 5);
      V8 af[NA][G::FM], bf[NB][G::FN];
#pragma unroll
      for (int x = 0; x < NA; ++x)
#pragma unroll
        for (int i = 0; i < G::FM; ++i) af[x][i] = frag(st + x * TAB, wm * G::WM + i * 32 + (lane & 31), cq);
#pragma unroll
      for (int y = 0; y < NB; ++y)
#pragma unroll
        for (int j = 0; j < G::FN; ++j) bf[y][j] = frag(st + NA * TAB + y * TBB, wn * G::WN + j * 32 + (lane & 31), cq);
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
#pragma unroll
          for (int c = 0; c < NC; ++c)
            acc[i][j][PR::cof(c)] = MF<TE>::mma(af[PR::aof(c)][i], bf[PR::bof(c)][j], acc[i][j][PR::cof(c)]);
    }
  }

  // Wait for this thread's DMA of the oldest outstanding stage (N younger
  // stages may stay in flight), then make every thread's data visible.
  template <int N>
  __device__ __forceinline__ static void wait_stage() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(vmcnt_imm(N * LOADS));
    asm volatile("s_barrier" ::: "memory");
  }

  __device__ __forceinline__ static void run(const Mat16 (&A)[NA], const Mat16 (&B)[NB], int64_t m0, int64_t n0,
                                             int64_t k0, int64_t k1, char* lds,
                                             f32x16 (&acc)[G::FM][G::FN][NACC]) {
    static_assert(STAGES >= 2 && STAGES <= 4, "2 to 4 stages");
    static_assert((STAGES - 1) * LOADS <= 63, "vmcnt holds at most 63 outstanding operations");
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave % G::WGM, wn = wave / G::WGM;
    const int64_t nk = (k1 - k0) / G::BK;
    if (nk <= 0) return;
    // all earlier LDS use of the block (a previous epilogue) is finished
    __syncthreads();
#pragma unroll
    for (int s = 0; s < STAGES - 1; ++s)
      if (s < nk) issue_stage(A, B, m0, n0, k0 + s * G::BK, lds + s * STAGE_BYTES, tid);
    for (int64_t kt = 0; kt < nk; ++kt) {
      // stages issued so far: min(kt + STAGES - 2, nk - 1); younger than kt: that minus kt
      const int64_t younger = std::min<int64_t>(STAGES - 2, nk - 1 - kt);
      if (younger >= 2) wait_stage<2>();
      else if (younger == 1) wait_stage<1>();
      else wait_stage<0>();
      const int64_t kn = kt + STAGES - 1;
      if (kn < nk) issue_stage(A, B, m0, n0, k0 + kn * G::BK, lds + (kn % STAGES) * STAGE_BYTES, tid);
      compute(lds + (kt % STAGES) * STAGE_BYTES, acc, lane, wm, wn);
    }
    // the epilogue may reuse the LDS: every wave is done with its last stage
    __syncthreads();
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
