// kernels_16.hpp -- launch interface of the 16-bit precision-form kernels.
#pragma once
#include "kernels.hpp"

namespace dna {

// Workspace pieces of the 16-bit path.  q16 holds Q and Q - 1 (2 N T elements
// of 16 bits), qb16 holds Q-bar; bits / rs / irs / irs2 / qs / iqs are the fp16
// scale buffers (R + 3 max(N, T) words, 3 R floats, 2 x 3 max(N, T) floats).
struct Scratch16 {
  void* q16;
  void* qb16;
  unsigned* bits;
  float* rs;
  float* irs;
  float* irs2;
  float* qs;
  float* iqs;
};

// Steps 2-5 and 10 with 16-bit products (gemm 1: bf16, 2: fp16): the Z pass
// writes 16-bit Q, Q - 1, Q-bar and the V sums; the gradient products write the
// fp32 split partials of u, u_c, y that the fp32 candidate kernels consume.
hipError_t launch_ratio_gh16(int gemm, int side, const float* V, const float* W, const float* H, int64_t N,
                             int64_t T, int64_t R, const Scratch16& S, int splits, int64_t kchunk, float* pu,
                             float* puc, float* py, double* vpart, int* check, const SumJob& fin,
                             hipStream_t s);

// Steps 7-9, 12-14 with 16-bit reconstruction products (float64 cost sums).
hipError_t launch_cost16(int gemm, int side, const float* V, const float* F, const float* Xmu, const float* Xn,
                         int64_t N, int64_t T, int64_t R, const Scratch16& S, double* part, int* fpart,
                         hipStream_t s);

}  // namespace dna
