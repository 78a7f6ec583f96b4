// kernels_sparse.hpp -- launch interface of the sparse-V kernels.
#pragma once
#include "kernels.hpp"

namespace dna {

// Device view of a sparse V (the fields of dna_sparse_v, see dna.h): CSR and CSC
// orders of the same nonzeros and their segments of at most SP_SEG entries.
struct SpV {
  int64_t nnz;
  const int32_t* col_idx;     // [nnz] CSR: column of each entry
  const float* val;           // [nnz] CSR: value of each entry
  const int32_t* row_of;      // [nnz] CSR: row of each entry
  const int32_t* csc_row;     // [nnz] CSC: row of each entry
  const int32_t* csc_col;     // [nnz] CSC: column of each entry
  const int32_t* csc_pos;     // [nnz] CSC: CSR position of each entry
  int64_t nseg_r, nseg_c;
  const int32_t* segr_start;  // [nseg_r + 1] CSR position where each row segment starts (last: nnz)
  const int32_t* segr_ptr;    // [N + 1] first row segment of each row
  const int32_t* segc_start;  // [nseg_c + 1] CSC position where each column segment starts
  const int32_t* segc_ptr;    // [T + 1] first column segment of each column
};
constexpr int SP_SEG = 64;     // entries per segment at most (one per lane in the cost kernels)
constexpr int64_t SP_MAX_R = 256;

hipError_t launch_sp_transpose(const float* X, float* Y, int64_t R, int64_t T, hipStream_t s);
// z, q, q-bar at the nonzeros (CSR order), W (N x R) and H^t (T x R).
hipError_t launch_sp_zq(const SpV& v, const float* W, const float* Ht, int64_t N, int64_t T, int64_t R, float* q,
                        float* qb, int* check, const SumJob& fin, hipStream_t s);
// q, q-bar from a carried reconstruction (zc = z_DNA, dzc = z_MU - z_DNA at the
// nonzeros, CSR order; mask[key == 0 ? t : n] = 1 where the Newton candidate
// was kept).
hipError_t launch_sp_qz(const SpV& v, const float* zc, const float* dzc, const uint8_t* mask, int key, int64_t N,
                        int64_t T, float* q, float* qb, int* check, const SumJob& fin, hipStream_t s);
// Gradient sums (side 0: F = W, CSC segments, outputs [r][t]; side 1: F = H^t,
// CSR segments, outputs [n][r]) in the layout of the dense split partials with
// one split, and the V sums per column / row.  c64: the factor sums (c or g).
// gp: 4 x nseg x R floats, vseg: nseg doubles.  mu_only: the MU numerator u
// alone (puc, py, vpart untouched).  R > SP_MAX_R: hipErrorInvalidValue.
hipError_t launch_sp_grad(int side, bool mu_only, const SpV& v, const float* F, const float* q, const float* qb,
                          const double* c64, int64_t N, int64_t T, int64_t R, float* gp, double* vseg, float* pu,
                          float* puc, float* py, double* vpart, hipStream_t s);
// Candidate costs (side 0: F = W, X rows = candidates^t (T x R); side 1: F = H^t,
// X rows = candidates (N x R)); Xd = X_MU - X_DNA in the same layout as Xn.
// cseg: 3 x nseg doubles, fseg: nseg ints; part/fpart in the dense cost layout
// with one tile.  zc, dzc (nnz floats each, or nullptr): z_DNA and z_MU - z_DNA
// at the nonzeros in CSR order, for launch_sp_qz.
hipError_t launch_sp_cost(int side, const SpV& v, const float* F, const float* Xn, const float* Xd, int64_t N,
                          int64_t T, int64_t R, double* cseg, int* fseg, double* part, int* fpart, hipStream_t s,
                          float* zc = nullptr, float* dzc = nullptr);
hipError_t launch_sp_diff(const float* Xmu, const float* Xn, float* D, int64_t n, hipStream_t s);
// KL of eq. 1; kseg: nseg_r doubles; c, g: float64 column sums of W and row sums of H.
hipError_t launch_sp_kl(const SpV& v, const float* W, const float* Ht, int64_t N, int64_t T, int64_t R,
                        double* kseg, const double* c, const double* g, double* out, hipStream_t s);

}  // namespace dna
