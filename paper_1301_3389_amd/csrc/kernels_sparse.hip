// kernels_sparse.hip -- DNA half-steps for a sparse V (the sparse data matrices
// of Sec. 4.2), float32 products, float64 cost sums.
//
// Only the nonzeros of V enter Q, Q-bar and the costs (end of Sec. 3), so every
// O(NRT) product of the dense path becomes O(nnz R) work:
//   k_sp_zq        z = W[n,:] . H[:,t] at each nonzero (one thread per nonzero,
//                  CSR order), q = v/z, q-bar = q/z            (steps 2-3, 10)
//   k_sp_grad_H    per column segment of the CSC order: the partial sums over
//                  its nonzeros of W q, W (q - 1), W and (W*W) q-bar, one lane
//                  per r                                         (steps 4-5, 10)
//   k_sp_comb_H    per column t: the segment partials in order, then
//                  u_c = sum_nz W (q - 1) - sum_{v = 0} W, the last term as
//                  c - sum_nz W in float64 (zeros of V contribute q = 0)
//   k_sp_cost_H    per column segment, one lane per nonzero: z_DNA and
//                  dZ = W (H_MU - H_DNA) at that entry, the cost terms of the
//                  dense path, wave sums in float64                 (steps 7-9, 12-14)
// and the W half-step mirrors them over the CSR row segments with H^t rows.
// The candidate, selection and normalisation kernels of the dense path serve
// unchanged (one "split", one cost tile).  Segments hold at most SP_SEG
// nonzeros of one row (column), so a few long rows of a skewed matrix do not
// serialise the launch; they are added back in a fixed order.
#include <math.h>

#include <algorithm>

#include "core.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"
#include "kernels_sparse.hpp"

namespace dna {

// a . b over R floats (rows of row-major matrices), vector loads when both rows
// are 16-byte aligned.
__device__ __forceinline__ float dot_rows(const float* __restrict__ a, const float* __restrict__ b, int64_t R,
                                          bool vec) {
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  int64_t r = 0;
  if (vec) {
    for (; r + 4 <= R; r += 4) {
      const f32x4 x = *reinterpret_cast<const f32x4*>(a + r);
      const f32x4 y = *reinterpret_cast<const f32x4*>(b + r);
      s0 = fmaf(x[0], y[0], s0);
      s1 = fmaf(x[1], y[1], s1);
      s2 = fmaf(x[2], y[2], s2);
      s3 = fmaf(x[3], y[3], s3);
    }
  }
  for (; r < R; ++r) s0 = fmaf(a[r], b[r], s0);
  return (s0 + s1) + (s2 + s3);
}

__device__ __forceinline__ bool rows_aligned(const void* a, const void* b, int64_t R) {
  return (R & 3) == 0 && ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0;
}

// Indices read from the caller's arrays are clamped into range, so a malformed
// structure gives wrong numbers, never an out-of-bounds access.
__device__ __forceinline__ int64_t clampi(int64_t i, int64_t n) { return (i >= 0 && i < n) ? i : 0; }
// A range [a, b) read from a segment table, clamped into [0, n].
__device__ __forceinline__ void clamp_range(int64_t& a, int64_t& b, int64_t n) {
  a = std::min<int64_t>(std::max<int64_t>(a, 0), n);
  b = std::min<int64_t>(std::max<int64_t>(b, a), n);
}

// ---------------------------------------------------------------------------
// Transpose of an R x T row-major matrix into T x R (H^t rows for the gathers).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sp_transpose(const float* __restrict__ X, float* __restrict__ Y, int64_t R,
                                                      int64_t T) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const int64_t t0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t r = r0 + ty + 8 * k, t = t0 + tx;
    tile[ty + 8 * k][tx] = (r < R && t < T) ? X[r * T + t] : 0.f;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int64_t t = t0 + ty + 8 * k, r = r0 + tx;
    if (r < R && t < T) Y[t * R + r] = tile[tx][ty + 8 * k];
  }
}

hipError_t launch_sp_transpose(const float* X, float* Y, int64_t R, int64_t T, hipStream_t s) {
  prof_begin("sp_transpose", s);
  hipLaunchKernelGGL(k_sp_transpose, dim3((unsigned)cdiv(T, 32), (unsigned)cdiv(R, 32)), dim3(256), 0, s, X, Y, R, T);
  prof_end("sp_transpose", s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// z, q, q-bar at every nonzero (CSR order).  `fin` folds the second level of a
// factor sum into this launch (as the dense ratio pass does).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sp_zq(SpV v, const float* __restrict__ W, const float* __restrict__ Ht,
                                               int64_t N, int64_t T, int64_t R, float* __restrict__ q,
                                               float* __restrict__ qb, int* check, SumJob fin) {
  sum_job(fin);
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int bad = 0;
  if (j < v.nnz) {
    const int64_t n = clampi(v.row_of[j], N), t = clampi(v.col_idx[j], T);
    const float* a = W + n * R;
    const float* b = Ht + t * R;
    const float z = dot_rows(a, b, R, rows_aligned(a, b, R));
    const float x = v.val[j];
    const bool pos = x > 0.f;
    const float iz = __builtin_amdgcn_rcpf(z);
    const float qq = pos ? x * iz : 0.f;
    q[j] = qq;
    qb[j] = pos ? qq * iz : 0.f;
    bad = (pos && !(z > 0.f)) ? 1 : 0;
  }
  bad = wave_or(bad);
  if (check && bad && (threadIdx.x & 63) == 0) atomicOr(check, CHK_DOMAIN);
}

hipError_t launch_sp_zq(const SpV& v, const float* W, const float* Ht, int64_t N, int64_t T, int64_t R, float* q,
                        float* qb, int* check, const SumJob& fin, hipStream_t s) {
  prof_begin("sp_zq", s);
  hipLaunchKernelGGL(k_sp_zq, dim3((unsigned)std::max<int64_t>(1, cdiv(v.nnz, 256))), dim3(256), 0, s, v, W, Ht, N, T,
                     R, q, qb, check, fin);
  prof_end("sp_zq", s);
  return hipGetLastError();
}

// q, q-bar at every nonzero from the reconstruction the preceding half-step's
// cost pass left (Algorithm 1 carries Z from steps 15 / 28; the normalisation
// between the half-steps leaves W H unchanged): z = z_DNA where that selection
// kept the Newton candidate, z_DNA + dZ where it kept MU.  key 0: the mask is
// per column t (after an H step), key 1: per row n (after a W step).
__global__ __launch_bounds__(256) void k_sp_qz(SpV v, const float* __restrict__ zc, const float* __restrict__ dzc,
                                               const uint8_t* __restrict__ mask, int key, int64_t N, int64_t T,
                                               float* __restrict__ q, float* __restrict__ qb, int* check, SumJob fin) {
  sum_job(fin);
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int bad = 0;
  if (j < v.nnz) {
    const int64_t g = key == 0 ? clampi(v.col_idx[j], T) : clampi(v.row_of[j], N);
    const float zN = zc[j];
    const float z = mask[g] ? zN : zN + dzc[j];
    const float x = v.val[j];
    const bool pos = x > 0.f;
    const float iz = __builtin_amdgcn_rcpf(z);
    const float qq = pos ? x * iz : 0.f;
    q[j] = qq;
    qb[j] = pos ? qq * iz : 0.f;
    bad = (pos && !(z > 0.f)) ? 1 : 0;
  }
  bad = wave_or(bad);
  if (check && bad && (threadIdx.x & 63) == 0) atomicOr(check, CHK_DOMAIN);
}

hipError_t launch_sp_qz(const SpV& v, const float* zc, const float* dzc, const uint8_t* mask, int key, int64_t N,
                        int64_t T, float* q, float* qb, int* check, const SumJob& fin, hipStream_t s) {
  prof_begin("sp_qz", s);
  hipLaunchKernelGGL(k_sp_qz, dim3((unsigned)std::max<int64_t>(1, cdiv(v.nnz, 256))), dim3(256), 0, s, v, zc, dzc,
                     mask, key, N, T, q, qb, check, fin);
  prof_end("sp_qz", s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gradient sums.  One wave per segment, lane r (+64 k, k < KR); segment partials
// gp[4][seg][R] = (F q, F (q - 1), F, (F*F) q-bar) and the V sum of the segment.
//   SIDE 0 (H step): segments of the CSC order, F = W[n, :] of each entry's row.
//   SIDE 1 (W step): segments of the CSR order, F = H^t[t, :] of each entry's column.
// ---------------------------------------------------------------------------
// A segment of more than SG_DIRECT entries first copies its factor rows into
// LDS (pitch P floats: R rounded up to 4, or 64 per chunk of 64 ranks), all
// loads issued before any is used, 16 bytes per lane when the rows are 16-byte
// aligned; a shorter one reads each row in the loop.  The sums are formed in
// the same order either way.
constexpr int SG_DIRECT = 16;

template <int SIDE, int KR, bool MU>
__global__ __launch_bounds__(64) void k_sp_grad(SpV v, const float* __restrict__ F, const float* __restrict__ q,
                                                const float* __restrict__ qb, int64_t N, int64_t T, int64_t R,
                                                float* __restrict__ gp, double* __restrict__ vseg) {
  extern __shared__ float sgr[];                  // 64 entries x P rank values
  const int lane = threadIdx.x;
  const int64_t sg = blockIdx.x;
  const int64_t nseg = SIDE == 0 ? v.nseg_c : v.nseg_r;
  if (sg >= nseg) return;
  const int32_t* start = SIDE == 0 ? v.segc_start : v.segr_start;
  int64_t i0 = start[sg], i1 = start[sg + 1];
  clamp_range(i0, i1, v.nnz);
  const int cnt = (int)std::min<int64_t>(i1 - i0, SP_SEG);
  const int64_t nF = SIDE == 0 ? N : T;
  // lane l loads entry i0 + l of the segment (its factor row, q, q-bar, v) at
  // once; the loop then broadcasts one entry at a time from its lane
  int rowl = 0;
  float ql = 0.f, qbl = 0.f;
  double vl = 0.0;
  if (lane < cnt) {
    const int64_t i = i0 + lane;
    const int64_t p = SIDE == 0 ? clampi(v.csc_pos[i], v.nnz) : i;
    rowl = (int)clampi(SIDE == 0 ? v.csc_row[i] : v.col_idx[i], nF);
    ql = q[p];
    if (!MU) {
      qbl = qb[p];
      vl = (double)v.val[p];
    }
  }
  float u[KR], uc[KR], fs[KR], y[KR];
#pragma unroll
  for (int k = 0; k < KR; ++k) u[k] = uc[k] = fs[k] = y[k] = 0.f;
  const int P = KR == 1 ? (int)((R + 3) & ~3) : 64;
  const bool vec = (R & 3) == 0 && (reinterpret_cast<uintptr_t>(F) & 15) == 0;
  const bool staged = cnt > SG_DIRECT;
#pragma unroll
  for (int k = 0; k < KR; ++k) {                  // ranks 64 k .. 64 k + rw
    const int64_t rb = 64 * k;
    const int rw = (int)std::min<int64_t>(64, R - rb);
    if (rw <= 0) break;
    // entry j's value of this lane's rank (f), added to the four sums in entry order
    auto add = [&](int j, float f) {
      const float qq = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, ql), j));
      const float qbb =
          MU ? 0.f : __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, qbl), j));
      u[k] = fmaf(f, qq, u[k]);
      if (!MU) {
        uc[k] = fmaf(f, qq - 1.f, uc[k]);
        fs[k] += f;
        y[k] = fmaf(f * f, qbb, y[k]);
      }
    };
    if (!staged) {
#pragma unroll 8
      for (int j = 0; j < cnt; ++j) {
        const int64_t re = __builtin_amdgcn_readlane(rowl, j);
        add(j, lane < rw ? F[re * R + rb + lane] : 0.f);
      }
      continue;
    }
    if (k > 0) __syncthreads();                   // the previous chunk's reads are done
    if (vec) {
#pragma unroll
      for (int j = 0; j < 16; ++j) {              // entry e = d / 16, float4 c = d % 16
        const int d = j * 64 + lane, e = d >> 4, c = d & 15;
        const int re = __shfl(rowl, e);
        if (e < cnt && 4 * c < rw)
          *reinterpret_cast<f32x4*>(sgr + e * P + 4 * c) =
              *reinterpret_cast<const f32x4*>(F + (int64_t)re * R + rb + 4 * c);
      }
    } else {
      for (int j = 0; j < cnt; ++j) {
        const int64_t re = __builtin_amdgcn_readlane(rowl, j);
        if (lane < rw) sgr[j * P + lane] = F[re * R + rb + lane];
      }
    }
    __syncthreads();
#pragma unroll 8
    for (int j = 0; j < cnt; ++j) add(j, lane < rw ? sgr[j * P + lane] : 0.f);
  }
  const int64_t stride = nseg * R;
#pragma unroll
  for (int k = 0; k < KR; ++k) {
    const int64_t r = lane + 64 * k;
    if (r < R) {
      gp[sg * R + r] = u[k];
      if (!MU) {
        gp[stride + sg * R + r] = uc[k];
        gp[2 * stride + sg * R + r] = fs[k];
        gp[3 * stride + sg * R + r] = y[k];
      }
    }
  }
  if (!MU) {
    const double vs = wave_sum(vl);
    if (lane == 0) vseg[sg] = vs;
  }
}

// Per column t (SIDE 0) / row n (SIDE 1): the segment partials in order, written
// in the layout of the dense split partials with one split (SIDE 0: [r][t],
// SIDE 1: [n][r]) and the V sums as one tile; u_c adds the entries where v = 0
// (q = 0, so q - 1 = -1): minus (c_r - sum_nz F_r), formed in float64.
template <int SIDE, bool MU>
__global__ __launch_bounds__(256) void k_sp_comb(SpV v, const float* __restrict__ gp, const double* __restrict__ vseg,
                                                 const double* __restrict__ c64, int64_t N, int64_t T, int64_t R,
                                                 float* __restrict__ pu, float* __restrict__ puc,
                                                 float* __restrict__ py, double* __restrict__ vpart) {
  const int lane = threadIdx.x & 63;
  const int64_t o = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);   // column t / row n
  const int64_t no = SIDE == 0 ? T : N;
  if (o >= no) return;
  const int32_t* segp = SIDE == 0 ? v.segc_ptr : v.segr_ptr;
  const int64_t nseg = SIDE == 0 ? v.nseg_c : v.nseg_r;
  int64_t s0 = segp[o], s1 = segp[o + 1];
  clamp_range(s0, s1, nseg);
  const int64_t stride = nseg * R;
  for (int64_t r = lane; r < R; r += 64) {
    float u = 0.f, uc = 0.f, fs = 0.f, y = 0.f;
    for (int64_t sg = s0; sg < s1; ++sg) {
      u += gp[sg * R + r];
      if (!MU) {
        uc += gp[stride + sg * R + r];
        fs += gp[2 * stride + sg * R + r];
        y += gp[3 * stride + sg * R + r];
      }
    }
    const int64_t idx = SIDE == 0 ? r * T + o : o * R + r;
    pu[idx] = u;
    if (!MU) {
      puc[idx] = (float)((double)uc - (c64[r] - (double)fs));
      py[idx] = y;
    }
  }
  if (!MU && lane == 0) {
    double vs = 0.0;
    for (int64_t sg = s0; sg < s1; ++sg) vs += vseg[sg];
    vpart[o] = vs;
  }
}

template <int SIDE, bool MU>
static hipError_t grad_launch(const SpV& v, const float* F, const float* q, const float* qb, const double* c64,
                              int64_t N, int64_t T, int64_t R, float* gp, double* vseg, float* pu, float* puc,
                              float* py, double* vpart, hipStream_t s) {
  const int64_t nseg = SIDE == 0 ? v.nseg_c : v.nseg_r;
  const dim3 grid((unsigned)std::max<int64_t>(1, nseg));      // a workgroup (one wave) per segment
  const size_t lds = (size_t)64 * (R <= 64 ? ((R + 3) & ~int64_t(3)) : 64) * sizeof(float);
  const char* gname = SIDE == 0 ? (MU ? "sp_grad_mu_H" : "sp_grad_H") : (MU ? "sp_grad_mu_W" : "sp_grad_W");
  prof_begin(gname, s);
  if (R <= 64)
    hipLaunchKernelGGL((k_sp_grad<SIDE, 1, MU>), grid, dim3(64), lds, s, v, F, q, qb, N, T, R, gp, vseg);
  else if (R <= 128)
    hipLaunchKernelGGL((k_sp_grad<SIDE, 2, MU>), grid, dim3(64), lds, s, v, F, q, qb, N, T, R, gp, vseg);
  else
    hipLaunchKernelGGL((k_sp_grad<SIDE, 4, MU>), grid, dim3(64), lds, s, v, F, q, qb, N, T, R, gp, vseg);
  prof_end(gname, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t no = SIDE == 0 ? T : N;
  const char* cname = SIDE == 0 ? "sp_comb_H" : "sp_comb_W";
  prof_begin(cname, s);
  hipLaunchKernelGGL((k_sp_comb<SIDE, MU>), dim3((unsigned)cdiv(no, 4)), dim3(256), 0, s, v, gp, vseg, c64, N, T, R,
                     pu, puc, py, vpart);
  prof_end(cname, s);
  return hipGetLastError();
}

hipError_t launch_sp_grad(int side, bool mu_only, const SpV& v, const float* F, const float* q, const float* qb,
                          const double* c64, int64_t N, int64_t T, int64_t R, float* gp, double* vseg, float* pu,
                          float* puc, float* py, double* vpart, hipStream_t s) {
  if (R > SP_MAX_R) return hipErrorInvalidValue;
  if (side == 0)
    return mu_only ? grad_launch<0, true>(v, F, q, qb, c64, N, T, R, gp, vseg, pu, puc, py, vpart, s)
                   : grad_launch<0, false>(v, F, q, qb, c64, N, T, R, gp, vseg, pu, puc, py, vpart, s);
  return mu_only ? grad_launch<1, true>(v, F, q, qb, c64, N, T, R, gp, vseg, pu, puc, py, vpart, s)
                 : grad_launch<1, false>(v, F, q, qb, c64, N, T, R, gp, vseg, pu, puc, py, vpart, s);
}

// ---------------------------------------------------------------------------
// Candidate costs.  One wave per segment, one lane per nonzero (segments hold
// at most 64): z_DNA = F_row . X_DNA and dZ = F_row . (X_MU - X_DNA) at the
// entry, the dense path's cost terms (cost_acc), then wave sums in float64 and
// the OR of the flags -> cseg[3][seg], fseg[seg].
//   SIDE 0: CSC segments, F_row = W[n, :], X rows = candidates^t[t, :] (T x R).
//   SIDE 1: CSR segments, F_row = H^t[t, :], X rows = candidates[n, :] (N x R).
// ---------------------------------------------------------------------------
// The gathered factor rows pass through LDS SC_RC floats at a time: the wave
// reads its (at most 64) rows with contiguous loads, eight lanes per 32-float
// row chunk, instead of each lane walking its own row with loads that hit 64
// different rows per instruction; each lane then forms its dot products from
// LDS (row pitch SC_RC + 1: conflict-free column reads) in dot_rows' order,
// so the sums are those of dot_rows.
constexpr int SC_RC = 32, SC_PITCH = SC_RC + 1;

template <int SIDE>
__global__ __launch_bounds__(64) void k_sp_cost(SpV v, const float* __restrict__ F, const float* __restrict__ Xn,
                                                const float* __restrict__ Xd, int64_t N, int64_t T, int64_t R,
                                                double* __restrict__ cseg, int* __restrict__ fseg,
                                                float* __restrict__ zc, float* __restrict__ dzc) {
  __shared__ float st[64 * SC_PITCH];
  __shared__ float sx[2 * SC_RC];
  const int lane = threadIdx.x;
  const int64_t sg = blockIdx.x;
  const int64_t nseg = SIDE == 0 ? v.nseg_c : v.nseg_r;
  if (sg >= nseg) return;                         // the whole workgroup (one wave)
  const int32_t* start = SIDE == 0 ? v.segc_start : v.segr_start;
  int64_t i0 = start[sg], i1 = start[sg + 1];
  clamp_range(i0, i1, v.nnz);
  const int cnt = (int)std::min<int64_t>(64, i1 - i0);
  const int64_t i = i0 + lane;
  const bool act = lane < cnt;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  int fl = 0;
  // every entry of a segment lies in one column (SIDE 0) / row (SIDE 1): that
  // index is uniform, so its candidate rows are read once for the wave
  const int64_t own = i0 < i1 ? (SIDE == 0 ? v.csc_col[i0] : v.row_of[i0]) : 0;
  const int64_t fixed = clampi(__builtin_amdgcn_readfirstlane((int)own), SIDE == 0 ? T : N);
  int64_t p = 0;
  int gi = 0;                                     // this lane's gathered row (n or t)
  if (act) {
    if (SIDE == 0) {
      p = clampi(v.csc_pos[i], v.nnz);
      gi = (int)clampi(v.csc_row[i], N);
    } else {
      p = i;
      gi = (int)clampi(v.col_idx[i], T);
    }
  }
  const float* xn = Xn + fixed * R;
  const float* xd = Xd + fixed * R;
  const bool vec = (R & 3) == 0 &&
                   ((reinterpret_cast<uintptr_t>(F) | reinterpret_cast<uintptr_t>(Xn) |
                     reinterpret_cast<uintptr_t>(Xd)) & 15) == 0;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;   // z_DNA partials (dot_rows' four)
  float b0 = 0.f, b1 = 0.f, b2 = 0.f, b3 = 0.f;   // dZ partials
  for (int64_t c0 = 0; c0 < R; c0 += SC_RC) {
    const int rc = (int)std::min<int64_t>(SC_RC, R - c0);
    __syncthreads();                              // the previous chunk's reads are done
    if (lane < SC_RC) {
      if (lane < rc) sx[lane] = xn[c0 + lane];
    } else if (lane - SC_RC < rc) {
      sx[lane] = xd[c0 + lane - SC_RC];
    }
    if (vec) {
#pragma unroll
      for (int j = 0; j < SC_RC / 4; ++j) {       // row e = q / 8, float4 k = q % 8
        const int q = j * 64 + lane, e = q >> 3, k = q & 7;
        const int ge = __shfl(gi, e);
        if (e < cnt && 4 * k < rc) {
          const f32x4 x = *reinterpret_cast<const f32x4*>(F + (int64_t)ge * R + c0 + 4 * k);
#pragma unroll
          for (int m = 0; m < 4; ++m) st[e * SC_PITCH + 4 * k + m] = x[m];
        }
      }
    } else {
#pragma unroll 8
      for (int j = 0; j < SC_RC; ++j) {           // row e = q / 32, float r = q % 32
        const int q = j * 64 + lane, e = q >> 5, r = q & 31;
        const int ge = __shfl(gi, e);
        if (e < cnt && r < rc) st[e * SC_PITCH + r] = F[(int64_t)ge * R + c0 + r];
      }
    }
    __syncthreads();
    if (act) {
      const float* f = st + lane * SC_PITCH;
      if (vec) {                                  // rc is a multiple of 4 here
        for (int r = 0; r < rc; r += 4) {
          a0 = fmaf(f[r], sx[r], a0);
          a1 = fmaf(f[r + 1], sx[r + 1], a1);
          a2 = fmaf(f[r + 2], sx[r + 2], a2);
          a3 = fmaf(f[r + 3], sx[r + 3], a3);
          b0 = fmaf(f[r], sx[SC_RC + r], b0);
          b1 = fmaf(f[r + 1], sx[SC_RC + r + 1], b1);
          b2 = fmaf(f[r + 2], sx[SC_RC + r + 2], b2);
          b3 = fmaf(f[r + 3], sx[SC_RC + r + 3], b3);
        }
      } else {
        for (int r = 0; r < rc; ++r) {
          a0 = fmaf(f[r], sx[r], a0);
          b0 = fmaf(f[r], sx[SC_RC + r], b0);
        }
      }
    }
  }
  if (act) {
    const float zN = (a0 + a1) + (a2 + a3);
    const float dz = (b0 + b1) + (b2 + b3);
    fl = cost_acc(v.val[p], zN, dz, s0, s1, s2);
    if (zc) {                                    // carried to the next half-step (CSR order)
      zc[p] = zN;
      dzc[p] = dz;
    }
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  fl = wave_or(fl);
  if (lane == 0) {
    cseg[sg] = s0 * LN2;
    cseg[nseg + sg] = s1 * LN2;
    cseg[2 * nseg + sg] = s2 * LN2;
    fseg[sg] = fl;
  }
}

// Per column (row): the segment sums in order, in the dense cost pass's part
// layout with one tile: part[q][o], fpart[o].
template <int SIDE>
__global__ __launch_bounds__(256) void k_sp_cost_comb(SpV v, const double* __restrict__ cseg,
                                                      const int* __restrict__ fseg, int64_t no,
                                                      double* __restrict__ part, int* __restrict__ fpart) {
  const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (o >= no) return;
  const int32_t* segp = SIDE == 0 ? v.segc_ptr : v.segr_ptr;
  const int64_t nseg = SIDE == 0 ? v.nseg_c : v.nseg_r;
  double a = 0.0, b = 0.0, c = 0.0;
  int fl = 0;
  int64_t s0 = segp[o], s1 = segp[o + 1];
  clamp_range(s0, s1, nseg);
  for (int64_t sg = s0; sg < s1; ++sg) {
    a += cseg[sg];
    b += cseg[nseg + sg];
    c += cseg[2 * nseg + sg];
    fl |= fseg[sg];
  }
  part[o] = a;
  part[no + o] = b;
  part[2 * no + o] = c;
  fpart[o] = fl;
}

hipError_t launch_sp_cost(int side, const SpV& v, const float* F, const float* Xn, const float* Xd, int64_t N,
                          int64_t T, int64_t R, double* cseg, int* fseg, double* part, int* fpart, hipStream_t s,
                          float* zc, float* dzc) {
  const int64_t nseg = side == 0 ? v.nseg_c : v.nseg_r;
  const dim3 grid((unsigned)std::max<int64_t>(1, nseg));      // a workgroup (one wave) per segment
  prof_begin(side == 0 ? "sp_cost_H" : "sp_cost_W", s);
  if (side == 0)
    hipLaunchKernelGGL(k_sp_cost<0>, grid, dim3(64), 0, s, v, F, Xn, Xd, N, T, R, cseg, fseg, zc, dzc);
  else
    hipLaunchKernelGGL(k_sp_cost<1>, grid, dim3(64), 0, s, v, F, Xn, Xd, N, T, R, cseg, fseg, zc, dzc);
  prof_end(side == 0 ? "sp_cost_H" : "sp_cost_W", s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t no = side == 0 ? T : N;
  prof_begin(side == 0 ? "sp_cost_comb_H" : "sp_cost_comb_W", s);
  if (side == 0)
    hipLaunchKernelGGL(k_sp_cost_comb<0>, dim3((unsigned)cdiv(no, 256)), dim3(256), 0, s, v, cseg, fseg, no, part,
                       fpart);
  else
    hipLaunchKernelGGL(k_sp_cost_comb<1>, dim3((unsigned)cdiv(no, 256)), dim3(256), 0, s, v, cseg, fseg, no, part,
                       fpart);
  prof_end(side == 0 ? "sp_cost_comb_H" : "sp_cost_comb_W", s);
  return hipGetLastError();
}

// X_MU - X_DNA (elementwise, n elements), the second operand of the dZ product.
__global__ __launch_bounds__(256) void k_sp_diff(const float* __restrict__ a, const float* __restrict__ b,
                                                 float* __restrict__ d, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) d[e] = a[e] - b[e];
}

hipError_t launch_sp_diff(const float* Xmu, const float* Xn, float* D, int64_t n, hipStream_t s) {
  prof_begin("sp_diff", s);
  hipLaunchKernelGGL(k_sp_diff, dim3((unsigned)std::min<int64_t>(cdiv(n, 256), 4096)), dim3(256), 0, s, Xmu, Xn, D,
                     n);
  prof_end("sp_diff", s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// KL cost (eq. 1) of a sparse V: sum_nz v log(v/z) - sum v + sum z, with
// sum z = sum_r c_r (H 1)_r.  Per CSR segment (one lane per nonzero) the float64
// sum of v log(v/z) - v; the final kernel adds the segments in order and the
// closed-form sum of Z.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sp_kl_seg(SpV v, const float* __restrict__ W, const float* __restrict__ Ht,
                                                   int64_t N, int64_t T, int64_t R, double* __restrict__ kseg) {
  const int lane = threadIdx.x & 63;
  const int64_t sg = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (sg >= v.nseg_r) return;
  int64_t i0 = v.segr_start[sg], i1 = v.segr_start[sg + 1];
  clamp_range(i0, i1, v.nnz);
  const int64_t i = i0 + lane;
  double term = 0.0;
  if (i < i1) {
    const int64_t n = clampi(v.row_of[i], N), t = clampi(v.col_idx[i], T);
    const float* a = W + n * R;
    const float* b = Ht + t * R;
    const float z = dot_rows(a, b, R, rows_aligned(a, b, R));
    const float x = v.val[i];
    if (x > 0.f) term = (double)(x * log2_hw(x * __builtin_amdgcn_rcpf(z))) * LN2 - (double)x;
  }
  term = wave_sum(term);
  if (lane == 0) kseg[sg] = term;
}

// One block: segments in a fixed order (256 strided lanes, then a fixed tree),
// plus sum_r c_r g_r from the float64 factor sums.
__global__ __launch_bounds__(256) void k_sp_kl_final(const double* __restrict__ kseg, int64_t nseg,
                                                     const double* __restrict__ c, const double* __restrict__ g,
                                                     int64_t R, double* __restrict__ out) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int64_t k = tid; k < nseg; k += 256) s += kseg[k];
  for (int64_t r = tid; r < R; r += 256) s += c[r] * g[r];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_sp_kl(const SpV& v, const float* W, const float* Ht, int64_t N, int64_t T, int64_t R,
                        double* kseg, const double* c, const double* g, double* out, hipStream_t s) {
  prof_begin("sp_kl", s);
  hipLaunchKernelGGL(k_sp_kl_seg, dim3((unsigned)std::max<int64_t>(1, cdiv(v.nseg_r, 4))), dim3(256), 0, s, v, W, Ht,
                     N, T, R, kseg);
  hipLaunchKernelGGL(k_sp_kl_final, dim3(1), dim3(256), 0, s, kseg, v.nseg_r, c, g, R, out);
  prof_end("sp_kl", s);
  return hipGetLastError();
}

}  // namespace dna
