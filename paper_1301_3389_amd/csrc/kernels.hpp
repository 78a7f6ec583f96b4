// kernels.hpp -- internal (C++) launch interface between the C ABI layer and
// the HIP kernels.  Nothing here is exported from libdna.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dna {

// Kernel timing hooks (implemented by the ABI layer).
void prof_begin(const char* name, hipStream_t s);
void prof_end(const char* name, hipStream_t s);

// Bits of the device check word (checked mode).
enum CheckBits { CHK_DOMAIN = 1, CHK_NONFINITE = 2 };

// Tile sizes the host uses to size partial-sum buffers.
constexpr int ZT_BM = 128;   // rows (n) per tile of the adjoint Z-type products
constexpr int ZT_BN = 128;   // columns (t) per tile of the adjoint Z-type products
constexpr int RT_BM = 128;   // ratio pass (Z = W H + Q / Q-bar epilogue): rows (n) per tile
constexpr int RT_BN = 64;    //                                            columns (t) per tile
constexpr int CH_BM = 128;   // H-orientation cost pass: rows (n) per tile (column partials)
constexpr int CH_BN = 64;
constexpr int CW_BM = 64;    // W-orientation cost pass: rows (n) per tile
constexpr int CW_BN = 128;   //                          columns (t) per tile (row partials)
constexpr int GH_BM = 64;    // H orientation gradient GEMM: rows (r) per tile
constexpr int GH_BN = 128;   //                              columns (t) per tile
constexpr int GW_BM = 128;   // W orientation gradient GEMM: rows (n) per tile
constexpr int GW_BN = 64;    //                              columns (r) per tile
constexpr int GEMM_BK = 16;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Rows per tile of the fp32 ratio pass and of the H-orientation cost pass:
// 128, or 64 where 128-row tiles would give fewer than two workgroups per CU
// (the partial sums of both passes then come in cdiv(N, 64) row tiles).
inline int ratio_tile_rows(int64_t N, int64_t T) { return cdiv(N, RT_BM) * cdiv(T, RT_BN) < 512 ? 64 : RT_BM; }
inline int cost_h_tile_rows(int64_t N, int64_t T) { return cdiv(N, CH_BM) * cdiv(T, CH_BN) < 512 ? 64 : CH_BM; }

// Every updated factor entry is kept at or above the smallest positive normal
// float32 (2^-126).  In exact arithmetic no update sends a positive entry to 0
// (the eps floor bounds the shrink per step), but float32 underflows an entry
// that keeps shrinking and 0 is a fixed point of every update; the floor keeps
// such entries able to grow back.
constexpr float VALUE_FLOOR = 1.17549435e-38f;

// What the ratio pass (Z = W H and its epilogue) produces.
enum RatioMode {
  RM_H = 0,        // Q, Q-bar, column sums of V         (DNA H step)
  RM_W = 1,        // Q, Q-bar, row sums of V            (DNA W step)
  RM_MU_H = 2,     // Q only                              (MU H step)
  RM_MU_H_COST = 3,// Q, per-column cost of the input
  RM_MU_W = 4,     // Q only                              (MU W step)
  RM_MU_W_COST = 5,// Q, per-row cost of the input
  RM_KL = 6,       // per-tile sums of the eq. (1) terms only
  RM_ADJ = 7,      // Q, Q-bar, Z and column sums of V      (adjoint recompute)
  RM_H_CARRY = 8,  // RM_H with Z read from the preceding W step's cost pass
  RM_W_CARRY = 9   // RM_W with Z read from the preceding H step's cost pass
};

// Z of the candidate each row (RM_H_CARRY: the preceding W step chose per row
// n) or column (RM_W_CARRY: per column t) kept, from that step's cost pass:
// z = zd + (sel == 0 ? dz : 0), zd = Z_DNA, dz = Z_MU - Z_DNA (Algorithm 1
// steps 15 and 28 carry Z; the normalisations between leave W H unchanged).
struct ZCarry {
  const float* zd = nullptr;
  const float* dz = nullptr;
  const uint8_t* sel = nullptr;
};

// Second level of a column / row sum of a factor (see launch_colsum_part): the
// parts are added in a fixed order into s64 / s32 (either may be nullptr), and
// a sum <= 0 sets CHK_DOMAIN in *check (if not nullptr).  s32 receives the sum
// plus `reg` (the eq. 2 weight of the half-step that divides by it: lambda for
// c = W^t 1, rho for g = H 1); s64 the sum alone.  A kernel that receives a
// SumJob with part != nullptr performs it on the side, before its own work.
struct SumJob {
  const double* part = nullptr;
  int nparts = 0;
  int64_t R = 0;
  double* s64 = nullptr;
  float* s32 = nullptr;
  int* check = nullptr;
  double reg = 0.0;
};

struct RatioArgs {
  const float* V; const float* W; const float* H;
  int64_t N, T, R;
  float* Q; float* Qb;
  double* vpart;      // [tiles_m][T] (column sums) or [tiles_n][N] (row sums)
  double* cpart;      // cost partials, same layouts; RM_KL: [tiles]
  int* check;         // nullptr unless checked
  float* Z;           // RM_ADJ only: Z = W H
  SumJob fin;         // folded second level of the preceding factor sum (part = nullptr: none)
  ZCarry carry;       // RM_H_CARRY / RM_W_CARRY only
};
hipError_t launch_ratio(RatioMode mode, const RatioArgs& a, hipStream_t s);

// Gradient / Hessian numerators, split over the contraction index.
//   H orientation: pu[sp][r][t] = sum_{n in split} w_nr q_nt, py with w^2, q-bar
//   W orientation: pu[sp][n][r] = sum_{t in split} q_nt h_rt, py with q-bar, h^2
// With Qb == nullptr only pu is written (MU).  Otherwise, with cs == nullptr,
// u_c = sum w (q - 1) is a third product over q - 1; with cs (the fixed
// factor's chunk sums, launch_chunk_sums: cdiv(K, GH_CHUNK) x (R rounded up to
// 64) floats) it is formed from the chunk sums of
// w q (GH_CHUNK contraction indices each) less cs, two products instead of
// three, and kchunk must be a multiple of GH_CHUNK.  The chunk form carries
// about 2^-24 u sqrt(GH_CHUNK / K) of rounding in u_c, the direct one
// 2^-24 times the partial sums of w (q - 1), which stay small near a fixed
// point; the chunk form is used for contractions of at least GH_CHUNK_MIN_K
// indices.  See the candidate kernels for which form of the gain is used where.
constexpr int64_t GH_CHUNK = 64;
constexpr int64_t GH_CHUNK_MIN_K = 2048;
hipError_t launch_chunk_sums(int side, const float* F, int64_t N, int64_t T, int64_t R, float* cs, hipStream_t s);
hipError_t launch_gh_H(const float* W, const float* Q, const float* Qb, const float* cs, int64_t N, int64_t T,
                       int64_t R, int splits, int64_t kchunk, float* pu, float* puc, float* py,
                       hipStream_t s);
hipError_t launch_gh_W(const float* Q, const float* Qb, const float* H, const float* cs, int64_t N, int64_t T,
                       int64_t R, int splits, int64_t kchunk, float* pu, float* puc, float* py,
                       hipStream_t s);

// Block layout of the H-orientation candidate kernel (columns per block, row
// groups), which its adjoint repeats so that every sum over r rounds alike.
struct CandLayout {
  int cols, rg;
};
inline CandLayout cand_layout(int64_t T, int64_t R) {
  if (R <= 128) return {32, 32};
  // 1024-thread blocks run two per CU: only where the blocks fill those rounds
  // to at least 85%
  const int64_t b = cdiv(T, 32);
  if (R <= 512 && b >= 256 && b * 100 >= cdiv(b, 512) * 512 * 85) return {32, 32};
  if (cdiv(T, 32) >= 512) return {32, 8};
  return {8, 32};
}

// Adds the `splits` partials of u, u_c, y (each splits x n floats) into split 0,
// in split order.
hipError_t launch_fold_splits(float* pu, float* puc, float* py, int splits, int64_t n, hipStream_t s);
// Candidates (MU and renormalised Newton) from the split partials.  c (g) holds
// the factor sums plus reg, the eq. 2 weight of this half-step (lambda / rho).
hipError_t launch_cand_H(const float* H, const float* pu, const float* puc, const float* py, int splits,
                         const float* c, const double* vpart, int tiles_m, int64_t T, int64_t R,
                         float eps, float alpha, float reg, float* Xmu, float* Xn, float* Aout, float* Bout,
                         hipStream_t s);
hipError_t launch_cand_W(const float* W, const float* pu, const float* puc, const float* py, int splits,
                         const float* g, const double* vpart, int tiles_n, int64_t N, int64_t R,
                         float eps, float alpha, float reg, float* Xmu, float* Xn, float* Aout, float* Bout,
                         hipStream_t s);

// Fused candidate reconstruction + log + reduction (costs of both candidates).
//   part: [3][tiles][L] float64 (sum_N, margin, MU-only rows), fpart: [tiles][L] int
// With zd / dz (N x T, row-major) the kernels also store z_DNA and dZ there.
// s0 = false: the sum_N partials are written as 0 (the choice needs only the
// margin and the flags; the kept candidate's cost is then not available).
hipError_t launch_cost_H(const float* V, const float* W, const float* Xmu, const float* Xn,
                         int64_t N, int64_t T, int64_t R, double* part, int* fpart, hipStream_t s,
                         float* zd = nullptr, float* dz = nullptr, bool s0 = true);
hipError_t launch_cost_W(const float* V, const float* H, const float* Xmu, const float* Xn,
                         int64_t N, int64_t T, int64_t R, double* part, int* fpart, hipStream_t s,
                         float* zd = nullptr, float* dz = nullptr, bool s0 = true);

// Selection and write-back.
// The damped selection's inputs (dpart == nullptr: Algorithm 1's rule).  With
// them the selection reads the current factor from the output buffer before
// overwriting it (Xout must hold the input state).
struct Damp {
  const double* dpart = nullptr;   // input-state cost parts, dtiles x L
  int dtiles = 0;
  const double* vpart = nullptr;   // data sum parts, vtiles x L
  int vtiles = 0;
  const double* c64 = nullptr;     // c = W^t 1 (H step) / g = H 1 (W step), float64
  double reg = 0.0;                // lambda (H step) / rho (W step)
};
hipError_t launch_select_H(const float* Xmu, const float* Xn, float* Hout, const double* part,
                           const int* fpart, int tiles_m, int64_t T, int64_t R, uint8_t* mask,
                           double* dsel, double* margin, hipStream_t s, const Damp& dp = Damp{});
// With `emit`, also the float64 column sums of the new W over each block's
// rows: emit[p * R + r] for the select_w_parts(tiles_n, N) blocks p.
hipError_t launch_select_W(const float* Xmu, const float* Xn, float* Wout, const double* part,
                           const int* fpart, int tiles_n, int64_t N, int64_t R, uint8_t* mask,
                           double* dsel, double* margin, hipStream_t s, const Damp& dp = Damp{},
                           double* emit = nullptr);
int select_w_parts(int tiles_n, int64_t N);

// MU update from split partials (+ optional cost finalisation).
hipError_t launch_mu_H(float* H, const float* pu, int splits, const float* c, int64_t T, int64_t R,
                       const double* cpart, int tiles_m, double* d_out, hipStream_t s);
hipError_t launch_mu_W(float* W, const float* pu, int splits, const float* g, int64_t N, int64_t R,
                       const double* cpart, int tiles_n, double* d_out, hipStream_t s);

// Column sums of W (R values) / row sums of H (R values) in two fixed-order
// levels: the part kernels write float64 partials to `part` (at most SUM_PARTS *
// R doubles) and return, in `job`, the second level (nparts, R; the caller sets
// s64 / s32 / check), to be folded into a later kernel or run by
// launch_sum_final.
constexpr int SUM_PARTS = 32;
hipError_t launch_colsum_part(const float* W, int64_t N, int64_t R, double* part, SumJob& job, hipStream_t s);
hipError_t launch_rowsum_part(const float* H, int64_t T, int64_t R, double* part, SumJob& job, hipStream_t s);
hipError_t launch_sum_final(const SumJob& job, hipStream_t s);
// Steps 1 / 29 (side 0, f = column sums of W: W[:,r] /= f_r, H[r,:] *= f_r) and
// step 16 (side 1, f = row sums of H: H[r,:] /= f_r, W[:,r] *= f_r), with the
// second level of the sums (job) done per tile.  With `emit` non-null the
// kernel also writes the first level of the sums of the factor it normalised
// (side 0: column sums of the new W, cdiv(N, 64) parts; side 1: row sums of
// the new H, cdiv(T, SC_TCHUNK) parts) and returns their second level in
// `emitted`, for the half-step that follows.
constexpr int SC_TCHUNK = 2048;
// out[0] += rho sum C + lambda sum G from the parts of C = W^t 1, G = H 1.
hipError_t launch_penalty(const SumJob& cj, const SumJob& gj, double rho, double lam, double* out, hipStream_t s);
int64_t scale_emit_parts(int side, int64_t N, int64_t T);
// `other`, wj, wo: the balanced form (see k_scale); other.part == nullptr: the
// unit-sum form.
hipError_t launch_scale(int side, float* W, float* H, int64_t N, int64_t T, int64_t R, const SumJob& job,
                        double* emit, SumJob* emitted, hipStream_t s, const SumJob& other = SumJob{},
                        double wj = 0.0, double wo = 0.0);

// Steps 2-5 and 10 in one kernel per half-step when R <= 64 (side 0: H step,
// rows n split into `splits` chunks of `chunk`; side 1: W step, columns t split
// likewise): the split partials of u, u_c, y and the per-split V sums, as the
// ratio + gradient kernel pair writes them.  R > 64: hipErrorInvalidValue.
// mode RGH_MU: the MU numerator u alone (puc, py, vpart untouched); RGH_MU_COST:
// u and, in vpart, the per-column (side 0) / per-row (side 1) cost
// sum_{v>0} v log(v/z) of the input state, natural log.
constexpr int64_t FUSED_MAX_R = 64;
// RGH_DNA_COST: RGH_DNA and, in dpart (same layout as vpart), the input
// state's per-column (row) cost, natural log (the damped selection).
constexpr int RGH_DNA = 0, RGH_MU = 1, RGH_MU_COST = 2, RGH_DNA_COST = 3;
hipError_t launch_rgh(int side, const float* V, const float* W, const float* H, int64_t N, int64_t T, int64_t R,
                      int splits, int64_t chunk, float* pu, float* puc, float* py, double* vpart, const SumJob& fin,
                      int* check, hipStream_t s, int mode = RGH_DNA, double* dpart = nullptr);

// Steps 7-9, 12-14 for R <= 64 with the candidates' block resident in LDS:
// cost partials over `splits` chunks of rows n (side 0) or columns t (side 1),
// in the layout of launch_cost_H / launch_cost_W with tiles = splits.
// newton_only: the damped selection's pass, the Newton candidate's cost alone
// (one product; the margin and MU slots of the partials are zero).  s0 = false
// (both candidates): the sum_N partials are written as 0, as in launch_cost_H.
hipError_t launch_costf(int side, const float* V, const float* F, const float* Xmu, const float* Xn, int64_t N,
                        int64_t T, int64_t R, int splits, int64_t chunk, double* part, int* fpart, hipStream_t s,
                        bool newton_only = false, bool s0 = true);

// The whole H half-step (steps 2-15) for R <= 64 in one kernel, a workgroup per
// block of HCOLS_TB columns running over all N rows (kernels_cols.hip): H is
// overwritten with the chosen columns; emit[block][r] (cdiv(T, HCOLS_TB) x R
// doubles) receives the partial row sums of the new H; mask / dsel / margin as
// launch_select_H (nullptr: not written).  cj: first-level parts of W^t 1,
// cj.reg = lambda.  With xmu_out (and xn_out) set, the kernel stops after the
// candidates and writes them there (R x T each) instead: H, emit and the
// selection outputs are left alone.  Used where T gives every compute unit
// column blocks of its own (T >= HCOLS_MIN_T).
constexpr int64_t HCOLS_TB = 16;
constexpr int64_t HCOLS_MIN_T = 4096;
constexpr int64_t HCOLS_MAX_T = int64_t(1) << 23;   // 32-bit byte offsets within a 64-row sub-tile
struct HColsArgs {
  const float* V; const float* W; float* H;
  int64_t N, T, R;
  SumJob cj;
  float eps, alpha;
  uint8_t* mask; double* dsel; double* margin;
  double* emit;
  int* check;
  float* xmu_out = nullptr;
  float* xn_out = nullptr;
};
inline int64_t hcols_blocks(int64_t T) { return cdiv(T, HCOLS_TB); }
hipError_t launch_hstep_cols(const HColsArgs& a, hipStream_t s);

hipError_t launch_kl_final(const double* cpart, int ntiles, double* out, hipStream_t s);

// Checked mode: negative or non-finite entries in a buffer.
hipError_t launch_check(const float* X, int64_t n, int* check, hipStream_t s);

}  // namespace dna
