// kernels_16.hpp -- launch interface of the 16-bit precision-form kernels.
#pragma once
#include "kernels.hpp"

namespace dna {

// Workgroups of the 16-bit gradient products resident per CU (sizes their split-K).
constexpr int GH16_WG_PER_CU = 2;

// Padded extents of the 16-bit operands: N and T to the 128-wide tiles, R to
// the 32-deep K tile where it is contracted and to 128 where it is a tile
// dimension.
struct Dims16 {
  int64_t Np, Tp, Rk, Rm;
};
inline Dims16 dims16(int64_t N, int64_t T, int64_t R) {
  return Dims16{cdiv(N, 128) * 128, cdiv(T, 128) * 128, cdiv(R, 32) * 32, cdiv(R, 128) * 128};
}

// Workspace pieces of the 16-bit path (all 16-bit buffers zero-padded):
//   fa_hi, fa_lo  Np x Rk   W (hi / lo parts of a two-term split)
//   fb_hi, fb_lo  Tp x Rk   H^t
//   g0, g1        Rm x max(Np, Tp)   W^t, (W*W)^t (H step) or H, H*H (W step)
//   x0, x1        max(Np, Tp) x Rk   candidate operands of the cost pass
//   q3            3 x Np x Tp        Q, Q - 1, Q-bar (H step: transposed)
//   bits, rs, irs, irs2, qs, iqs     fp16 scales (Rm + 3 max(N, T) words,
//                                    3 Rm floats, 2 x 3 max(N, T) floats)
struct Scratch16 {
  void* fa_hi; void* fa_lo; void* fb_hi; void* fb_lo;
  void* g0; void* g1; void* x0; void* x1; void* q3;
  unsigned* bits;
  float* rs; float* irs; float* irs2; float* qs; float* iqs;
};
size_t scratch16_bytes(int64_t N, int64_t T, int64_t R);
Scratch16 scratch16_carve(void* base, int64_t N, int64_t T, int64_t R);

// Steps 2-5 and 10 with 16-bit products (gemm 1: bf16, 2: fp16): conversion of
// the factors, the Z pass (16-bit Q, Q - 1, Q-bar and the V sums, the folded
// second level of the factor sum), and the gradient products (fp32 split
// partials of u, u_c, y for the fp32 candidate kernels).  vpart holds
// cdiv(N, 128) (H step) or cdiv(T, 128) (W step) tiles of V sums.
hipError_t launch_ratio_gh16(int gemm, int side, const float* V, const float* W, const float* H, int64_t N,
                             int64_t T, int64_t R, const Scratch16& S, int splits, int64_t kchunk, float* pu,
                             float* puc, float* py, double* vpart, int* check, const SumJob& fin,
                             hipStream_t s, bool qmax_given = false);

// Steps 7-9, 12-14 with 16-bit reconstruction products (float64 cost sums);
// partials over cdiv(N, 128) (H step) or cdiv(T, 128) (W step) tiles.
hipError_t launch_cost16(int gemm, int side, const float* V, const float* F, const float* Xmu, const float* Xn,
                         int64_t N, int64_t T, int64_t R, const Scratch16& S, double* part, int* fpart,
                         hipStream_t s, bool s0 = true, bool qmax_next = false);

}  // namespace dna
