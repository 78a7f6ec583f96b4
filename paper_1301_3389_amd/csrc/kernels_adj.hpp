// kernels_adj.hpp -- internal launch interface of the adjoint kernels.
#pragma once
#include "kernels.hpp"

namespace dna {

constexpr int WB_BM = 64;   // W-gradient products: rows (n) per tile
constexpr int WB_BN = 64;   //                      columns (r) per tile

hipError_t launch_cand_bwd_H(const float* H, const float* pu, const float* puc, const float* py, int splits, const float* c,
                             const double* vpart, int tiles_m, int64_t T, int64_t R, float eps, float alpha,
                             const uint8_t* sel, const float* G, float* Ubar, float* Ybar, float* Hd,
                             float* Cbar, float* sbar, hipStream_t s);
hipError_t launch_zbar(const float* V, const float* Z, const float* W, const float* Ubar, const float* Ybar,
                       const float* sbar, int64_t N, int64_t T, int64_t R, float* Zbar, float* dV, int accumulate,
                       hipStream_t s);
hipError_t launch_dh_final(const float* Hd, const float* pu, int splits, int64_t R, int64_t T, float* Gout,
                           hipStream_t s);
hipError_t launch_wbar(const float* Q, const float* Zbar, const float* Qb, const float* Ubar, const float* H,
                       const float* Ybar, int64_t N, int64_t T, int64_t R, int splits, int64_t kchunk, float* p0,
                       float* p1, hipStream_t s);
hipError_t launch_dw_final(const float* W, const float* p0, const float* p1, int splits, const double* cbar,
                           int64_t N, int64_t R, float* dW, int accumulate, hipStream_t s);
hipError_t launch_copy(const float* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_fill(float* dst, float value, int64_t n, hipStream_t s);

}  // namespace dna
