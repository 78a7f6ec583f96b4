// kernels_fwd.hip -- forward HIP kernels of one DNA / MU half-step (gfx950).
//
// H half-step (Algorithm 1 steps 4-15), kernel by kernel:
//   k_ratio     Z = W H tile on MFMA (K = R); epilogue Q = V/Z, Q-bar = V/Z^2,
//               column sums of V.  Z never leaves registers.
//   k_gh_H      [A-numerator, B-numerator] = [W, W*W]^t [Q, Q-bar] on MFMA, the
//               W tile staged once and squared in registers; split over N.
//   k_cand_H    A (eq. 7), B (eq. 14), MU candidate (eq. 11), Newton candidate
//               (eq. 15/17 with floor and ceiling) and its renormalisation (eq. 10).
//   k_cost_H    Z_DNA = W H_DNA and dZ = W (H_MU - H_DNA) on MFMA with two
//               accumulators; epilogue v log(v/z_DNA) and -v log1p(dZ/z_DNA),
//               column sums in float64 (steps 7-9, 12-14).
//   k_select_H  per column: d_DNA < d_MU ? Newton : MU (step 15), write H.
// The W half-step runs the same stages in the transposed orientation
// (contractions over T, per-row reductions).
#include <math.h>

#include <algorithm>

#include "core.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"

namespace dna {

using GR = Geo<RT_BM, RT_BN, GEMM_BK, 2, 2>;   // ratio pass, M = N, N = T, K = R
using GCH = Geo<CH_BM, CH_BN, GEMM_BK, 2, 2>;  // H-orientation cost (column reductions)
using GCW = Geo<CW_BM, CW_BN, GEMM_BK, 2, 2>;  // W-orientation cost (row reductions)
using GH = Geo<GH_BM, GH_BN, GEMM_BK, 2, 2>;   // H orientation gradient, M = R, N = T, K = N
using GW = Geo<GW_BM, GW_BN, GEMM_BK, 2, 2>;   // W orientation gradient, M = N, N = R, K = T
using GS = Geo<64, 64, GEMM_BK, 2, 2>;         // either gradient orientation when the grid is small
// Below this many workgroups the gradient products switch to 64 x 64 tiles, so
// that small problems still put two workgroups (eight waves) on every CU.
constexpr int64_t GH_SMALL_GRID = 512;

// ---------------------------------------------------------------------------
// k_ratio: Z = W H (MFMA, K = R) and its epilogue.
// ---------------------------------------------------------------------------
struct RatioKArgs {
  const float* V;
  Opnd W, H;
  int64_t N, T, R;
  float* Q; float* Qb;
  double* vpart; double* cpart;
  int* check;
  float* Z;
  SumJob fin;
  ZCarry carry;
};

template <int MODE, class GZ>
__global__ __launch_bounds__(GZ::NT) void k_ratio(RatioKArgs a) {
  using TL = Tile<GZ, ProdSingle, true, false>;
  __shared__ __align__(16) float lds[TL::LDS_FLOATS];
  // dispatch order: the Q, Q-bar (and Z) writes of the resident tiles then
  // cover whole rows; the XCD remaps measured slower here
  const Tile3 tl{(int64_t)blockIdx.x, (int64_t)blockIdx.y, 0};
  const int64_t m0 = tl.y * GZ::BM, n0 = tl.x * GZ::BN;
  constexpr bool CARRY = MODE == RM_H_CARRY || MODE == RM_W_CARRY;
  sum_job(a.fin);
  float vf[GZ::FM][GZ::FN][16];
  TL::load_frag(vf, a.V, a.T, m0, n0, a.N, a.T);     // in flight during the K loop
  TL t;
  t.zero();
  if constexpr (CARRY) {
    // Z of the kept candidates: z_DNA, plus dZ where MU was kept (per row n
    // after a W step, per column t after an H step)
    float zf[GZ::FM][GZ::FN][16], df[GZ::FM][GZ::FN][16];
    TL::load_frag(zf, a.carry.zd, a.T, m0, n0, a.N, a.T);
    TL::load_frag(df, a.carry.dz, a.T, m0, n0, a.N, a.T);
#pragma unroll
    for (int i = 0; i < GZ::FM; ++i)
#pragma unroll
      for (int j = 0; j < GZ::FN; ++j) {
        const int64_t col = min(TL::col_of(n0, j), a.T - 1);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = min(TL::row_of(m0, i, v), a.N - 1);
          const bool mu = (MODE == RM_H_CARRY ? a.carry.sel[row] : a.carry.sel[col]) == 0;
          t.acc[i][j][0][v] = mu ? zf[i][j][v] + df[i][j][v] : zf[i][j][v];
        }
      }
  } else {
    const Opnd A[1] = {a.W};
    const Opnd B[1] = {a.H};
    t.run(A, B, m0, n0, 0, a.R, lds);
  }
  constexpr bool WANT_Q = MODE != RM_KL;
  constexpr bool WANT_QB = MODE == RM_H || MODE == RM_W || MODE == RM_ADJ || CARRY;
  constexpr bool WANT_Z = MODE == RM_ADJ;
  constexpr bool COLS = MODE == RM_H || MODE == RM_MU_H_COST || MODE == RM_ADJ || MODE == RM_H_CARRY;
  constexpr bool ROWS = MODE == RM_W || MODE == RM_MU_W_COST || MODE == RM_W_CARRY;
  constexpr bool COST = MODE == RM_MU_H_COST || MODE == RM_MU_W_COST;
  const int64_t N = a.N, T = a.T;
  double cp[1][GZ::FN];
  double rp[1][GZ::FM][16];
  double klsum = 0.0;
#pragma unroll
  for (int j = 0; j < GZ::FN; ++j) cp[0][j] = 0.0;
#pragma unroll
  for (int i = 0; i < GZ::FM; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) rp[0][i][v] = 0.0;
  int bad = 0;
#pragma unroll
  for (int i = 0; i < GZ::FM; ++i)
#pragma unroll
    for (int j = 0; j < GZ::FN; ++j) {
      const int64_t col = TL::col_of(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = TL::row_of(m0, i, v);
        if (row < N && col < T) {
          const float x = vf[i][j][v];
          const float z = t.acc[i][j][0][v];
          const bool pos = x > 0.f;
          const float iz = __builtin_amdgcn_rcpf(z);
          const float q = pos ? x * iz : 0.f;
          const float qb = pos ? q * iz : 0.f;
          bad |= (pos && !(z > 0.f)) ? 1 : 0;
          double term = 0.0;
          if (COST || MODE == RM_KL) term = (double)(x * log2_hw(pos ? q : 1.f)) * LN2;
          if (WANT_Q) a.Q[row * T + col] = q;
          if (WANT_QB) a.Qb[row * T + col] = qb;
          if (WANT_Z) a.Z[row * T + col] = z;
          if (MODE == RM_KL) klsum += term - (double)x + (double)z;
          const double val = COST ? term : (double)x;
          if (COLS) cp[0][j] += val;
          if (ROWS) rp[0][i][v] += val;
        }
      }
    }
  if (a.check && bad) atomicOr(a.check, CHK_DOMAIN);
  double* red = reinterpret_cast<double*>(lds);
  if (COLS) {
    double* dst = COST ? a.cpart : a.vpart;
    reduce_cols<GZ, 1>(cp, red, [&](int c, const double (&s)[1]) {
      if (n0 + c < T) dst[tl.y * T + n0 + c] = s[0];
    });
  }
  if (ROWS) {
    double* dst = COST ? a.cpart : a.vpart;
    reduce_rows<GZ, 1>(rp, red, [&](int r, const double (&s)[1]) {
      if (m0 + r < N) dst[tl.x * N + m0 + r] = s[0];
    });
  }
  if (MODE == RM_KL) {
    const int tid = threadIdx.x;
    const double w = wave_sum(klsum);
    if ((tid & 63) == 0) red[tid >> 6] = w;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int k = 0; k < GZ::WAVES; ++k) s += red[k];
      a.cpart[tl.y * gridDim.x + tl.x] = s;
    }
  }
}

hipError_t launch_ratio(RatioMode mode, const RatioArgs& a, hipStream_t s) {
  RatioKArgs k;
  k.V = a.V;
  k.W = make_opnd(a.W, a.R, a.N);
  k.H = make_opnd(a.H, a.T, a.T);
  k.N = a.N; k.T = a.T; k.R = a.R;
  k.Q = a.Q; k.Qb = a.Qb; k.vpart = a.vpart; k.cpart = a.cpart; k.check = a.check; k.Z = a.Z;
  k.fin = a.fin;
  k.carry = a.carry;
  if ((mode == RM_H_CARRY || mode == RM_W_CARRY) && (!a.carry.zd || !a.carry.dz || !a.carry.sel))
    return hipErrorInvalidValue;
  const bool small = ratio_tile_rows(a.N, a.T) == GS::BM;
  static_assert(GS::BN == GR::BN, "both ratio geometries tile T alike");
  dim3 grid((unsigned)cdiv(a.T, GR::BN), (unsigned)cdiv(a.N, small ? GS::BM : GR::BM));
  const char* nm = "ratio";
#define DNA_RATIO_CASE(M, NAME)                                                           \
  case M:                                                                                  \
    nm = NAME;                                                                             \
    prof_begin(nm, s);                                                                     \
    if (small) hipLaunchKernelGGL((k_ratio<M, GS>), grid, dim3(GS::NT), 0, s, k);         \
    else hipLaunchKernelGGL((k_ratio<M, GR>), grid, dim3(GR::NT), 0, s, k);               \
    break;
  switch (mode) {
    DNA_RATIO_CASE(RM_H, "ratio_H")
    DNA_RATIO_CASE(RM_W, "ratio_W")
    DNA_RATIO_CASE(RM_MU_H, "ratio_mu_H")
    DNA_RATIO_CASE(RM_MU_H_COST, "ratio_mu_H_cost")
    DNA_RATIO_CASE(RM_MU_W, "ratio_mu_W")
    DNA_RATIO_CASE(RM_MU_W_COST, "ratio_mu_W_cost")
    DNA_RATIO_CASE(RM_KL, "kl_terms")
    DNA_RATIO_CASE(RM_ADJ, "ratio_adj")
    DNA_RATIO_CASE(RM_H_CARRY, "ratio_H")
    DNA_RATIO_CASE(RM_W_CARRY, "ratio_W")
    default: return hipErrorInvalidValue;
  }
#undef DNA_RATIO_CASE
  prof_end(nm, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gradient / Hessian numerators.
// ---------------------------------------------------------------------------
// Outputs of the gradient kernels: split partials of u, u_c (= u - c) and y.
struct GHOut {
  float* p[3];
};

template <class G, class PR>
__global__ __launch_bounds__(G::NT) void k_gh_H(Opnd Wt, Opnd Q, Opnd Qb, int64_t N, int64_t T,
                                                 int64_t R, int64_t kchunk, GHOut out) {
  using TL = Tile<G, PR, false, false>;
  __shared__ __align__(16) float lds[TL::LDS_FLOATS];
  const Tile3 tl = xcd_tile_grouped<8>();
  const int64_t m0 = tl.y * G::BM, n0 = tl.x * G::BN;
  const int64_t sp = tl.z;
  const int64_t k0 = sp * kchunk, k1 = min(N, k0 + kchunk);
  TL t;
  t.zero();
  {
    const Opnd A[PR::NA] = {Wt};
    Opnd B[PR::NB];
    B[0] = Q;
    if constexpr (PR::NB > 1) B[PR::NB - 1] = Qb;
    t.run(A, B, m0, n0, k0, k1, lds);
  }
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = TL::col_of(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = TL::row_of(m0, i, v);
        if (row < R && col < T) {
#pragma unroll
          for (int c = 0; c < PR::NC; ++c) out.p[c][(sp * R + row) * T + col] = t.acc[i][j][c][v];
        }
      }
    }
}

// The DNA gradient products with two MFMA chains instead of three: the
// contraction runs in chunks of GH_CHUNK indices; each chunk's sum of w q is
// added to the plain sum u and, less the chunk's sum of the fixed factor
// (cs[chunk][r]), to the centred sum u_c = sum w (q - 1).  Each chunk sum
// carries float32 rounding of its own size only, so u keeps the MU gain's
// relative accuracy and u_c the absolute accuracy of A near 0, as a separate
// product over q - 1 would.
template <class G>
__global__ __launch_bounds__(G::NT, 2) void k_gh2_H(Opnd Wt, Opnd Q, Opnd Qb, const float* __restrict__ cs, int64_t N,
                                                  int64_t T, int64_t R, int64_t kchunk, GHOut out) {
  using TL = Tile<G, ProdDualB_SqA, false, false>;     // acc 0: w q, acc 1: w^2 q-bar
  __shared__ __align__(16) float lds[TL::LDS_FLOATS];
  const Tile3 tl = xcd_tile_grouped<8>();
  const int64_t m0 = tl.y * G::BM, n0 = tl.x * G::BN;
  const int64_t sp = tl.z;
  const int64_t k0 = sp * kchunk, k1 = min(N, k0 + kchunk);
  const int64_t c0 = k0 / GH_CHUNK;
  TL t;
  t.zero();
  float ur[G::FM][G::FN][16], ucr[G::FM][G::FN][16];
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) ur[i][j][v] = ucr[i][j][v] = 0.f;
  {
    const Opnd A[1] = {Wt};
    const Opnd B[2] = {Q, Qb};
    // this lane's chunk sums (table rows padded to a multiple of 64 ranks with
    // zeros), four rows per 16-byte load, one chunk ahead of their use
    const int64_t Rp = (R + 63) / 64 * 64;
    const int64_t nchunks = (k1 - k0 + GH_CHUNK - 1) / GH_CHUNK;
    const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) % G::WGM;
    const float* csb = cs + c0 * Rp + m0 + wm * G::WM + (lane >> 5) * 4;
    f32x4 cc[G::FM][4];
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int g = 0; g < 4; ++g) cc[i][g] = *reinterpret_cast<const f32x4*>(csb + i * 32 + g * 8);
    t.run_flush(A, B, m0, n0, k0, k1, lds, GH_CHUNK / G::BK, [&](int c) {
      const float* nx = csb + min<int64_t>(c + 1, nchunks - 1) * Rp;
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
#pragma unroll
          for (int j = 0; j < G::FN; ++j) {
            const float x = t.acc[i][j][0][v];
            ur[i][j][v] += x;
            ucr[i][j][v] += x - cc[i][v >> 2][v & 3];
            t.acc[i][j][0][v] = 0.f;
          }
        }
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int g = 0; g < 4; ++g) cc[i][g] = *reinterpret_cast<const f32x4*>(nx + i * 32 + g * 8);
    });
  }
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = TL::col_of(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = TL::row_of(m0, i, v);
        if (row < R && col < T) {
          const int64_t e = (sp * R + row) * T + col;
          out.p[0][e] = ur[i][j][v];
          out.p[1][e] = ucr[i][j][v];
          out.p[2][e] = t.acc[i][j][1][v];
        }
      }
    }
}

template <class G>
__global__ __launch_bounds__(G::NT, 2) void k_gh2_W(Opnd Q, Opnd Qb, Opnd Ht, const float* __restrict__ cs, int64_t N,
                                                  int64_t T, int64_t R, int64_t kchunk, GHOut out) {
  using TL = Tile<G, ProdDualA_SqB, true, true>;       // acc 0: q h, acc 1: q-bar h^2
  __shared__ __align__(16) float lds[TL::LDS_FLOATS];
  const Tile3 tl = xcd_tile_grouped<8>();
  const int64_t m0 = tl.y * G::BM, n0 = tl.x * G::BN;
  const int64_t sp = tl.z;
  const int64_t k0 = sp * kchunk, k1 = min(T, k0 + kchunk);
  const int64_t c0 = k0 / GH_CHUNK;
  TL t;
  t.zero();
  float ur[G::FM][G::FN][16], ucr[G::FM][G::FN][16];
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) ur[i][j][v] = ucr[i][j][v] = 0.f;
  {
    const Opnd A[2] = {Q, Qb};
    const Opnd B[1] = {Ht};
    const int64_t Rp = (R + 63) / 64 * 64;
    const int64_t nchunks = (k1 - k0 + GH_CHUNK - 1) / GH_CHUNK;
    const float* csb = cs + c0 * Rp + TL::col_of(n0, 0);
    float cc[G::FN];
#pragma unroll
    for (int j = 0; j < G::FN; ++j) cc[j] = csb[j * 32];
    t.run_flush(A, B, m0, n0, k0, k1, lds, GH_CHUNK / G::BK, [&](int c) {
      const float* nx = csb + min<int64_t>(c + 1, nchunks - 1) * Rp;
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
#pragma unroll
        for (int i = 0; i < G::FM; ++i)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const float x = t.acc[i][j][0][v];
            ur[i][j][v] += x;
            ucr[i][j][v] += x - cc[j];
            t.acc[i][j][0][v] = 0.f;
          }
        cc[j] = nx[j * 32];
      }
    });
  }
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = TL::col_of(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = TL::row_of(m0, i, v);
        if (row < N && col < R) {
          const int64_t e = (sp * N + row) * R + col;
          out.p[0][e] = ur[i][j][v];
          out.p[1][e] = ucr[i][j][v];
          out.p[2][e] = t.acc[i][j][1][v];
        }
      }
    }
}

// cs[c][r] = float32 of the float64 sum of W[n][r] over the rows n of chunk c
// (GH_CHUNK rows; side 0), or of H[r][t] over the columns t of chunk c (side 1);
// rows r of the table padded to Rp = R rounded up to 64 with zeros.
__global__ __launch_bounds__(256) void k_chunk_sums_W(const float* __restrict__ W, int64_t N, int64_t R, int64_t Rp,
                                                      float* __restrict__ cs) {
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x, c = blockIdx.y;
  if (r >= Rp) return;
  double s = 0.0;
  if (r < R) {
    const int64_t n1 = min(N, (c + 1) * GH_CHUNK);
    for (int64_t n = c * GH_CHUNK; n < n1; ++n) s += (double)W[n * R + r];
  }
  cs[c * Rp + r] = (float)s;
}

__global__ __launch_bounds__(256) void k_chunk_sums_H(const float* __restrict__ H, int64_t T, int64_t R, int64_t Rp,
                                                      int64_t nchunks, float* __restrict__ cs) {
  // GH_CHUNK lanes (a half-wave or a wave) per (chunk, r): a value per lane,
  // then a fixed-order sum
  static_assert(GH_CHUNK == 32 || GH_CHUNK == 64, "a chunk is a half-wave or a wave");
  const int lane = threadIdx.x & (GH_CHUNK - 1);
  const int64_t item = (int64_t)blockIdx.x * (256 / GH_CHUNK) + threadIdx.x / GH_CHUNK;
  const bool ok = item < nchunks * Rp;
  const int64_t r = ok ? item / nchunks : 0, c = ok ? item % nchunks : 0;
  const int64_t t = c * GH_CHUNK + lane;
  double s = (ok && r < R && t < T) ? (double)H[r * T + t] : 0.0;
#pragma unroll
  for (int m = GH_CHUNK / 2; m >= 1; m >>= 1) s += __shfl_xor(s, m);
  if (ok && lane == 0) cs[c * Rp + r] = (float)s;
}

hipError_t launch_chunk_sums(int side, const float* F, int64_t N, int64_t T, int64_t R, float* cs, hipStream_t s) {
  const int64_t Rp = cdiv(R, 64) * 64;
  prof_begin("chunk_sums", s);
  if (side == 0) {
    hipLaunchKernelGGL(k_chunk_sums_W, dim3((unsigned)cdiv(Rp, 256), (unsigned)cdiv(N, GH_CHUNK)), dim3(256), 0, s,
                       F, N, R, Rp, cs);
  } else {
    const int64_t nc = cdiv(T, GH_CHUNK);
    hipLaunchKernelGGL(k_chunk_sums_H, dim3((unsigned)cdiv(nc * Rp, 256 / GH_CHUNK)), dim3(256), 0, s, F, T, R, Rp,
                       nc, cs);
  }
  prof_end("chunk_sums", s);
  return hipGetLastError();
}

hipError_t launch_gh_H(const float* W, const float* Q, const float* Qb, const float* cs, int64_t N, int64_t T,
                       int64_t R, int splits, int64_t kchunk, float* pu, float* puc, float* py,
                       hipStream_t s) {
  const bool small = cdiv(T, GH::BN) * cdiv(R, GH::BM) * splits < GH_SMALL_GRID;
  dim3 grid((unsigned)cdiv(T, GH::BN), (unsigned)cdiv(R, GH::BM), (unsigned)splits);
  if (small) grid = dim3((unsigned)cdiv(T, GS::BN), (unsigned)cdiv(R, GS::BM), (unsigned)splits);
  const Opnd wt = make_opnd(W, R, R);     // element (r, n) at W[n*R + r]: MN-contiguous
  const Opnd q = make_opnd(Q, T, T);      // element (t, n) at Q[n*T + t]: MN-contiguous
  GHOut out = {{pu, puc, py}};
  if (Qb && cs) {
    if (kchunk % GH_CHUNK != 0) return hipErrorInvalidValue;
    const Opnd qb = make_opnd(Qb, T, T);
    prof_begin("gh_H", s);
    if (small) hipLaunchKernelGGL((k_gh2_H<GS>), grid, dim3(GS::NT), 0, s, wt, q, qb, cs, N, T, R, kchunk, out);
    else hipLaunchKernelGGL((k_gh2_H<GH>), grid, dim3(GH::NT), 0, s, wt, q, qb, cs, N, T, R, kchunk, out);
    prof_end("gh_H", s);
  } else if (Qb) {
    const Opnd qb = make_opnd(Qb, T, T);
    prof_begin("gh_H", s);
    if (small) hipLaunchKernelGGL((k_gh_H<GS, ProdGH3_H>), grid, dim3(GS::NT), 0, s, wt, q, qb, N, T, R, kchunk, out);
    else hipLaunchKernelGGL((k_gh_H<GH, ProdGH3_H>), grid, dim3(GH::NT), 0, s, wt, q, qb, N, T, R, kchunk, out);
    prof_end("gh_H", s);
  } else {
    prof_begin("gh_mu_H", s);
    if (small) hipLaunchKernelGGL((k_gh_H<GS, ProdSingle>), grid, dim3(GS::NT), 0, s, wt, q, q, N, T, R, kchunk, out);
    else hipLaunchKernelGGL((k_gh_H<GH, ProdSingle>), grid, dim3(GH::NT), 0, s, wt, q, q, N, T, R, kchunk, out);
    prof_end("gh_mu_H", s);
  }
  return hipGetLastError();
}

template <class G, class PR>
__global__ __launch_bounds__(G::NT) void k_gh_W(Opnd Q, Opnd Qb, Opnd Ht, int64_t N, int64_t T,
                                                 int64_t R, int64_t kchunk, GHOut out) {
  using TL = Tile<G, PR, true, true>;
  __shared__ __align__(16) float lds[TL::LDS_FLOATS];
  const Tile3 tl = xcd_tile_grouped<8>();
  const int64_t m0 = tl.y * G::BM, n0 = tl.x * G::BN;
  const int64_t sp = tl.z;
  const int64_t k0 = sp * kchunk, k1 = min(T, k0 + kchunk);
  TL t;
  t.zero();
  {
    Opnd A[PR::NA];
    A[0] = Q;
    if constexpr (PR::NA > 1) A[PR::NA - 1] = Qb;
    const Opnd B[PR::NB] = {Ht};
    t.run(A, B, m0, n0, k0, k1, lds);
  }
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = TL::col_of(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = TL::row_of(m0, i, v);
        if (row < N && col < R) {
#pragma unroll
          for (int c = 0; c < PR::NC; ++c) out.p[c][(sp * N + row) * R + col] = t.acc[i][j][c][v];
        }
      }
    }
}

hipError_t launch_gh_W(const float* Q, const float* Qb, const float* H, const float* cs, int64_t N, int64_t T,
                       int64_t R, int splits, int64_t kchunk, float* pu, float* puc, float* py,
                       hipStream_t s) {
  const bool small = cdiv(R, GW::BN) * cdiv(N, GW::BM) * splits < GH_SMALL_GRID;
  dim3 grid((unsigned)cdiv(R, GW::BN), (unsigned)cdiv(N, GW::BM), (unsigned)splits);
  if (small) grid = dim3((unsigned)cdiv(R, GS::BN), (unsigned)cdiv(N, GS::BM), (unsigned)splits);
  const Opnd q = make_opnd(Q, T, N);      // element (n, t) at Q[n*T + t]: K-contiguous
  const Opnd ht = make_opnd(H, T, R);     // element (r, t) at H[r*T + t]: K-contiguous
  GHOut out = {{pu, puc, py}};
  if (Qb && cs) {
    if (kchunk % GH_CHUNK != 0) return hipErrorInvalidValue;
    const Opnd qb = make_opnd(Qb, T, N);
    prof_begin("gh_W", s);
    if (small) hipLaunchKernelGGL((k_gh2_W<GS>), grid, dim3(GS::NT), 0, s, q, qb, ht, cs, N, T, R, kchunk, out);
    else hipLaunchKernelGGL((k_gh2_W<GW>), grid, dim3(GW::NT), 0, s, q, qb, ht, cs, N, T, R, kchunk, out);
    prof_end("gh_W", s);
  } else if (Qb) {
    const Opnd qb = make_opnd(Qb, T, N);
    prof_begin("gh_W", s);
    if (small) hipLaunchKernelGGL((k_gh_W<GS, ProdGH3_W>), grid, dim3(GS::NT), 0, s, q, qb, ht, N, T, R, kchunk, out);
    else hipLaunchKernelGGL((k_gh_W<GW, ProdGH3_W>), grid, dim3(GW::NT), 0, s, q, qb, ht, N, T, R, kchunk, out);
    prof_end("gh_W", s);
  } else {
    prof_begin("gh_mu_W", s);
    if (small) hipLaunchKernelGGL((k_gh_W<GS, ProdSingle>), grid, dim3(GS::NT), 0, s, q, q, ht, N, T, R, kchunk, out);
    else hipLaunchKernelGGL((k_gh_W<GW, ProdSingle>), grid, dim3(GW::NT), 0, s, q, q, ht, N, T, R, kchunk, out);
    prof_end("gh_mu_W", s);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Candidates.
// ---------------------------------------------------------------------------
// CAND_COLS columns per block, RG row groups; renormalisation eq. (10) per
// column through a fixed-order LDS reduction.  With RPT > 0 (R <= RPT * RG)
// each thread keeps its RPT Newton values in registers between the two passes
// and issues the loads of all its rows for one split together; RPT = 0 is the
// general form for any R.
constexpr int CAND_COLS = 32, CAND_RG = 256 / CAND_COLS;

template <int RPT, int RG, int COLS = CAND_COLS>
__global__ __launch_bounds__(COLS * RG) void k_cand_H(
    const float* __restrict__ H, const float* __restrict__ pu, const float* __restrict__ puc,
    const float* __restrict__ py, int splits, const float* __restrict__ c, const double* __restrict__ vpart,
    int tiles_m, int64_t T, int64_t R, float eps, float alpha, float reg, float* __restrict__ Xmu,
    float* __restrict__ Xn,
    float* __restrict__ Aout, float* __restrict__ Bout) {
  __shared__ double red[RG][COLS];
  __shared__ double fac[COLS];
  const int tid = threadIdx.x, cl = tid % COLS, rg = tid / COLS;
  const int64_t t = (int64_t)blockIdx.x * COLS + cl;
  const bool ok = t < T;
  double den = 0.0;
  constexpr int KEEP = RPT > 0 ? RPT : 1;
  float keep[KEEP];
  if (ok) {
    if constexpr (RPT > 0) {
      // rows in groups of CH (the sums of a group in flight together); the
      // Newton values stay in registers until the renormalisation
      constexpr int CH = RPT < 4 ? RPT : 4;
#pragma unroll
      for (int i0 = 0; i0 < RPT; i0 += CH) {
        float u[CH], uc[CH], y[CH];
#pragma unroll
        for (int i = 0; i < CH; ++i) u[i] = uc[i] = y[i] = 0.f;
        constexpr int SPU = CH <= 2 ? 8 : (CH <= 8 ? 2 : 1);   // loads in flight: 3 x CH x SPU
#pragma unroll SPU
        for (int sp = 0; sp < splits; ++sp) {
          const int64_t o = (int64_t)sp * R * T + t;
#pragma unroll
          for (int i = 0; i < CH; ++i) {
            const int64_t r = rg + (i0 + i) * RG;
            if (r < R) {
              u[i] += pu[o + r * T];
              uc[i] += puc[o + r * T];
              y[i] += py[o + r * T];
            }
          }
        }
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const int64_t r = rg + (i0 + i) * RG;
          keep[i0 + i] = 0.f;
          if (r < R) {
            const Cand k = candidate(H[r * T + t], u[i], uc[i], y[i], c[r], eps, alpha, reg);
            Xmu[r * T + t] = k.mu;
            keep[i0 + i] = k.newton;
            if (Aout) Aout[r * T + t] = k.A;
            if (Bout) Bout[r * T + t] = k.B;
            den += (double)c[r] * (double)k.newton;
          }
        }
      }
    } else {
#pragma unroll 4
      for (int64_t r = rg; r < R; r += RG) {
        float u = 0.f, uc = 0.f, y = 0.f;
#pragma unroll 4
        for (int sp = 0; sp < splits; ++sp) {
          u += pu[(sp * R + r) * T + t];
          uc += puc[(sp * R + r) * T + t];
          y += py[(sp * R + r) * T + t];
        }
        const Cand k = candidate(H[r * T + t], u, uc, y, c[r], eps, alpha, reg);
        Xmu[r * T + t] = k.mu;
        Xn[r * T + t] = k.newton;
        if (Aout) Aout[r * T + t] = k.A;
        if (Bout) Bout[r * T + t] = k.B;
        den += (double)c[r] * (double)k.newton;
      }
    }
  }
  red[rg][cl] = den;
  __syncthreads();
  if (rg == 0 && ok) {
    double d = 0.0;
    for (int k = 0; k < RG; ++k) d += red[k][cl];
    double s = 0.0;
#pragma unroll 8
    for (int m = 0; m < tiles_m; ++m) s += vpart[(int64_t)m * T + t];
    fac[cl] = d > 0.0 ? s / d : 1.0;
  }
  __syncthreads();
  if (ok) {
    const double f = fac[cl];
    if constexpr (RPT > 0) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int64_t r = rg + i * RG;
        if (r < R) Xn[r * T + t] = fmaxf((float)((double)keep[i] * f), VALUE_FLOOR);
      }
    } else {
#pragma unroll 4
      for (int64_t r = rg; r < R; r += RG)
        Xn[r * T + t] = fmaxf((float)((double)Xn[r * T + t] * f), VALUE_FLOOR);
    }
  }
}

// The split partials of u, u_c, y added into split 0 in split order, a thread
// per entry (what k_cand_H adds per entry, so its result is unchanged); for
// many splits over few columns, where k_cand_H's few workgroups would add
// them one after another.
__global__ __launch_bounds__(256) void k_fold_splits(float* __restrict__ pu, float* __restrict__ puc,
                                                     float* __restrict__ py, int splits, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  float u = 0.f, uc = 0.f, y = 0.f;
#pragma unroll 8
  for (int sp = 0; sp < splits; ++sp) {
    u += pu[sp * n + e];
    uc += puc[sp * n + e];
    y += py[sp * n + e];
  }
  pu[e] = u;
  puc[e] = uc;
  py[e] = y;
}

hipError_t launch_fold_splits(float* pu, float* puc, float* py, int splits, int64_t n, hipStream_t s) {
  prof_begin("fold_splits", s);
  hipLaunchKernelGGL(k_fold_splits, dim3((unsigned)std::max<int64_t>(1, cdiv(n, 256))), dim3(256), 0, s, pu, puc, py,
                     splits, n);
  prof_end("fold_splits", s);
  return hipGetLastError();
}

hipError_t launch_cand_H(const float* H, const float* pu, const float* puc, const float* py, int splits, const float* c,
                         const double* vpart, int tiles_m, int64_t T, int64_t R, float eps, float alpha, float reg,
                         float* Xmu, float* Xn, float* Aout, float* Bout, hipStream_t s) {
  prof_begin("cand_H", s);
  // for R <= 128 (and R <= 512 where T gives at least 256 blocks), 32 row
  // groups (1024 threads) give every CU 16 waves of independent loads and keep
  // each thread's Newton values in registers until the renormalisation; larger
  // R takes the general loop, with 32 columns x 8 row groups per block, or
  // 8 x 32 where that would leave fewer than 512 blocks
  const CandLayout lay = cand_layout(T, R);
  const dim3 grid((unsigned)cdiv(T, lay.cols));
  constexpr int RG = 32;
  if (R <= 2 * RG)
    hipLaunchKernelGGL((k_cand_H<2, RG>), grid, dim3(CAND_COLS * RG), 0, s, H, pu, puc, py, splits, c, vpart,
                       tiles_m, T, R, eps, alpha, reg, Xmu, Xn, Aout, Bout);
  else if (R <= 4 * RG)
    hipLaunchKernelGGL((k_cand_H<4, RG>), grid, dim3(CAND_COLS * RG), 0, s, H, pu, puc, py, splits, c, vpart,
                       tiles_m, T, R, eps, alpha, reg, Xmu, Xn, Aout, Bout);
  else if (lay.rg == RG && R <= 16 * RG)
    hipLaunchKernelGGL((k_cand_H<16, RG>), grid, dim3(CAND_COLS * RG), 0, s, H, pu, puc, py, splits, c, vpart,
                       tiles_m, T, R, eps, alpha, reg, Xmu, Xn, Aout, Bout);
  else if (lay.cols == CAND_COLS)
    hipLaunchKernelGGL((k_cand_H<0, CAND_RG>), grid, dim3(CAND_COLS * CAND_RG), 0, s, H, pu, puc, py, splits, c,
                       vpart, tiles_m, T, R, eps, alpha, reg, Xmu, Xn, Aout, Bout);
  else
    hipLaunchKernelGGL((k_cand_H<0, 32, 8>), grid, dim3(8 * 32), 0, s, H, pu, puc, py, splits, c, vpart, tiles_m, T,
                       R, eps, alpha, reg, Xmu, Xn, Aout, Bout);
  prof_end("cand_H", s);
  return hipGetLastError();
}

// One block per row n of W: the four waves each add a quarter of the splits
// (lane = r, RPW values of r per lane, RPW = 0 for the general form), the
// quarters are added in LDS in fixed order, then wave 0 forms the candidates.
template <int RPW>
__global__ __launch_bounds__(256) void k_cand_W(const float* __restrict__ W, const float* __restrict__ pu,
                                                const float* __restrict__ puc, const float* __restrict__ py,
                                                int splits, const float* __restrict__ g,
                                                const double* __restrict__ vpart, int tiles_n, int64_t N, int64_t R,
                                                float eps, float alpha, float reg, float* __restrict__ Xmu,
                                                float* __restrict__ Xn, float* __restrict__ Aout,
                                                float* __restrict__ Bout) {
  constexpr int NR = RPW > 0 ? RPW : 1;
  __shared__ float red[3][4][64 * NR];
  __shared__ double vs[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = blockIdx.x;
  if constexpr (RPW == 0) {
    // general form: wave 0 alone, lanes stride over r
    if (wave != 0) return;
    double den = 0.0;
    for (int64_t r = lane; r < R; r += 64) {
      float u = 0.f, uc = 0.f, y = 0.f;
#pragma unroll 4
      for (int sp = 0; sp < splits; ++sp) {
        u += pu[(sp * N + n) * R + r];
        uc += puc[(sp * N + n) * R + r];
        y += py[(sp * N + n) * R + r];
      }
      const Cand k = candidate(W[n * R + r], u, uc, y, g[r], eps, alpha, reg);
      Xmu[n * R + r] = k.mu;
      Xn[n * R + r] = k.newton;
      if (Aout) Aout[n * R + r] = k.A;
      if (Bout) Bout[n * R + r] = k.B;
      den += (double)g[r] * (double)k.newton;
    }
    double s = 0.0;
    for (int64_t m = lane; m < tiles_n; m += 64) s += vpart[m * N + n];
    den = __shfl(wave_sum(den), 0);
    s = __shfl(wave_sum(s), 0);
    const double f = den > 0.0 ? s / den : 1.0;
    for (int64_t r = lane; r < R; r += 64)
      Xn[n * R + r] = fmaxf((float)((double)Xn[n * R + r] * f), VALUE_FLOOR);
  } else {
    float u[RPW], uc[RPW], y[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) u[i] = uc[i] = y[i] = 0.f;
#pragma unroll 4
    for (int sp = wave; sp < splits; sp += 4) {
      const int64_t o = ((int64_t)sp * N + n) * R;
#pragma unroll
      for (int i = 0; i < RPW; ++i) {
        const int64_t r = lane + 64 * i;
        if (r < R) {
          u[i] += pu[o + r];
          uc[i] += puc[o + r];
          y[i] += py[o + r];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      red[0][wave][i * 64 + lane] = u[i];
      red[1][wave][i * 64 + lane] = uc[i];
      red[2][wave][i * 64 + lane] = y[i];
    }
    {  // the V row sum, one part per lane of wave 1
      double s = 0.0;
      if (wave == 1)
        for (int64_t m = lane; m < tiles_n; m += 64) s += vpart[m * N + n];
      s = wave_sum(s);
      if (wave == 1 && lane == 0) vs[0] = s;
    }
    __syncthreads();
    if (wave != 0) return;
    double den = 0.0;
    float keep[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int64_t r = lane + 64 * i;
      keep[i] = 0.f;
      if (r < R) {
        const int e = i * 64 + lane;
        const float uu = (red[0][0][e] + red[0][1][e]) + (red[0][2][e] + red[0][3][e]);
        const float ucc = (red[1][0][e] + red[1][1][e]) + (red[1][2][e] + red[1][3][e]);
        const float yy = (red[2][0][e] + red[2][1][e]) + (red[2][2][e] + red[2][3][e]);
        const Cand k = candidate(W[n * R + r], uu, ucc, yy, g[r], eps, alpha, reg);
        Xmu[n * R + r] = k.mu;
        keep[i] = k.newton;
        if (Aout) Aout[n * R + r] = k.A;
        if (Bout) Bout[n * R + r] = k.B;
        den += (double)g[r] * (double)k.newton;
      }
    }
    den = __shfl(wave_sum(den), 0);
    const double s = vs[0];
    const double f = den > 0.0 ? s / den : 1.0;
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int64_t r = lane + 64 * i;
      if (r < R) Xn[n * R + r] = fmaxf((float)((double)keep[i] * f), VALUE_FLOOR);
    }
  }
}

// Few splits (at most 4, e.g. the sparse path's one): a wave per row, four rows
// per block.  The split sums are added in the four-wave form's order
// ((s0 + s1) + (s2 + s3)), so the results equal k_cand_W's bit for bit.
template <int RPW>
__global__ __launch_bounds__(256) void k_cand_W_rows(const float* __restrict__ W, const float* __restrict__ pu,
                                                     const float* __restrict__ puc, const float* __restrict__ py,
                                                     int splits, const float* __restrict__ g,
                                                     const double* __restrict__ vpart, int tiles_n, int64_t N,
                                                     int64_t R, float eps, float alpha, float reg,
                                                     float* __restrict__ Xmu, float* __restrict__ Xn,
                                                     float* __restrict__ Aout, float* __restrict__ Bout) {
  const int lane = threadIdx.x & 63;
  const int64_t n = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= N) return;
  double den = 0.0;
  float keep[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int64_t r = lane + 64 * i;
    keep[i] = 0.f;
    if (r < R) {
      float u[4], uc[4], y[4];
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        u[w] = uc[w] = y[w] = 0.f;
        if (w < splits) {
          const int64_t o = ((int64_t)w * N + n) * R + r;
          u[w] += pu[o];
          uc[w] += puc[o];
          y[w] += py[o];
        }
      }
      const float uu = (u[0] + u[1]) + (u[2] + u[3]);
      const float ucc = (uc[0] + uc[1]) + (uc[2] + uc[3]);
      const float yy = (y[0] + y[1]) + (y[2] + y[3]);
      const Cand k = candidate(W[n * R + r], uu, ucc, yy, g[r], eps, alpha, reg);
      Xmu[n * R + r] = k.mu;
      keep[i] = k.newton;
      if (Aout) Aout[n * R + r] = k.A;
      if (Bout) Bout[n * R + r] = k.B;
      den += (double)g[r] * (double)k.newton;
    }
  }
  double s = 0.0;
  for (int64_t m = lane; m < tiles_n; m += 64) s += vpart[m * N + n];
  s = wave_sum(s);
  den = __shfl(wave_sum(den), 0);
  const double f = den > 0.0 ? s / den : 1.0;
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int64_t r = lane + 64 * i;
    if (r < R) Xn[n * R + r] = fmaxf((float)((double)keep[i] * f), VALUE_FLOOR);
  }
}

hipError_t launch_cand_W(const float* W, const float* pu, const float* puc, const float* py, int splits, const float* g,
                         const double* vpart, int tiles_n, int64_t N, int64_t R, float eps, float alpha, float reg,
                         float* Xmu, float* Xn, float* Aout, float* Bout, hipStream_t s) {
  prof_begin("cand_W", s);
  const dim3 grid((unsigned)N);
  if (splits <= 4 && R <= 128) {
    const dim3 g4((unsigned)cdiv(N, 4));
    if (R <= 64)
      hipLaunchKernelGGL(k_cand_W_rows<1>, g4, dim3(256), 0, s, W, pu, puc, py, splits, g, vpart, tiles_n, N, R,
                         eps, alpha, reg, Xmu, Xn, Aout, Bout);
    else
      hipLaunchKernelGGL(k_cand_W_rows<2>, g4, dim3(256), 0, s, W, pu, puc, py, splits, g, vpart, tiles_n, N, R,
                         eps, alpha, reg, Xmu, Xn, Aout, Bout);
  } else if (R <= 64)
    hipLaunchKernelGGL(k_cand_W<1>, grid, dim3(256), 0, s, W, pu, puc, py, splits, g, vpart, tiles_n, N, R, eps,
                       alpha, reg, Xmu, Xn, Aout, Bout);
  else if (R <= 128)
    hipLaunchKernelGGL(k_cand_W<2>, grid, dim3(256), 0, s, W, pu, puc, py, splits, g, vpart, tiles_n, N, R, eps,
                       alpha, reg, Xmu, Xn, Aout, Bout);
  else
    hipLaunchKernelGGL(k_cand_W<0>, grid, dim3(256), 0, s, W, pu, puc, py, splits, g, vpart, tiles_n, N, R, eps,
                       alpha, reg, Xmu, Xn, Aout, Bout);
  prof_end("cand_W", s);
  return hipGetLastError();
}

// z_DNA and dZ of a finished cost tile to zd / dz (both N x T, row-major).
template <class TL, class G>
__device__ __forceinline__ void store_recon(const TL& t, int64_t m0, int64_t n0, int64_t N, int64_t T, float* zd,
                                            float* dz) {
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = TL::col_of(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = TL::row_of(m0, i, v);
        if (row < N && col < T) {
          zd[row * T + col] = t.acc[i][j][0][v];
          dz[row * T + col] = t.acc[i][j][1][v];
        }
      }
    }
}

template <bool S0, class GZ>
__global__ __launch_bounds__(GZ::NT) void k_cost_H(const float* V, Opnd W, Opnd Hn, Opnd Hd, int64_t N,
                                                     int64_t T, int64_t R, double* part, int* fpart, float* zd,
                                                     float* dz) {
  using TL = Tile<GZ, ProdDualB, true, false>;
  __shared__ __align__(16) float lds[TL::LDS_FLOATS];
  __shared__ int fl_s[GZ::BN];
  const Tile3 tl = xcd_tile_grouped<8>();
  const int64_t m0 = tl.y * GZ::BM, n0 = tl.x * GZ::BN;
  const int tid = threadIdx.x;
  for (int c = tid; c < GZ::BN; c += GZ::NT) fl_s[c] = 0;
  float vf[GZ::FM][GZ::FN][16];
  TL::load_frag(vf, V, T, m0, n0, N, T);
  TL t;
  t.zero();
  {
    const Opnd A[1] = {W};
    const Opnd B[2] = {Hn, Hd};
    t.run(A, B, m0, n0, 0, R, lds);
  }
  if (zd) store_recon<TL, GZ>(t, m0, n0, N, T, zd, dz);
  const int64_t base = tl.y * T, stride = (int64_t)gridDim.y * T;
  cost_cols<GZ, S0>(vf, t.acc, m0, n0, N, T, reinterpret_cast<double*>(lds), fl_s, part, fpart, base, stride);
}

hipError_t launch_cost_H(const float* V, const float* W, const float* Xmu, const float* Xn, int64_t N,
                         int64_t T, int64_t R, double* part, int* fpart, hipStream_t s, float* zd, float* dz,
                         bool s0) {
  const bool small = cost_h_tile_rows(N, T) == GS::BM;
  static_assert(GS::BN == GCH::BN, "both cost geometries tile T alike");
  dim3 grid((unsigned)cdiv(T, GCH::BN), (unsigned)cdiv(N, small ? GS::BM : GCH::BM));
  const Opnd w = make_opnd(W, R, N);
  const Opnd hn = make_opnd(Xn, T, T);
  const Opnd hd = make_opnd(Xmu, T, T, Xn);
  prof_begin("cost_H", s);
  auto k = small ? (s0 ? k_cost_H<true, GS> : k_cost_H<false, GS>) : (s0 ? k_cost_H<true, GCH> : k_cost_H<false, GCH>);
  hipLaunchKernelGGL(k, grid, dim3(256), 0, s, V, w, hn, hd, N, T, R, part, fpart, zd, dz);
  prof_end("cost_H", s);
  return hipGetLastError();
}

template <bool S0>
__global__ __launch_bounds__(GCW::NT, 2) void k_cost_W(const float* V, Opnd Wn, Opnd Wd, Opnd H, int64_t N,
                                                     int64_t T, int64_t R, double* part, int* fpart, float* zd,
                                                     float* dz) {
  using TL = Tile<GCW, ProdDualA, true, false>;
  __shared__ __align__(16) float lds[TL::LDS_FLOATS];
  __shared__ int fl_s[GCW::BM];
  const Tile3 tl = xcd_tile_grouped<8>();
  const int64_t m0 = tl.y * GCW::BM, n0 = tl.x * GCW::BN;
  const int tid = threadIdx.x;
  for (int r = tid; r < GCW::BM; r += GCW::NT) fl_s[r] = 0;
  float vf[GCW::FM][GCW::FN][16];
  TL::load_frag(vf, V, T, m0, n0, N, T);
  TL t;
  t.zero();
  {
    const Opnd A[2] = {Wn, Wd};
    const Opnd B[1] = {H};
    t.run(A, B, m0, n0, 0, R, lds);
  }
  if (zd) store_recon<TL, GCW>(t, m0, n0, N, T, zd, dz);
  const int64_t base = tl.x * N, stride = (int64_t)gridDim.x * N;
  cost_rows<GCW, S0>(vf, t.acc, m0, n0, N, T, reinterpret_cast<double*>(lds), fl_s, part, fpart, base, stride);
}

hipError_t launch_cost_W(const float* V, const float* H, const float* Xmu, const float* Xn, int64_t N,
                         int64_t T, int64_t R, double* part, int* fpart, hipStream_t s, float* zd, float* dz,
                         bool s0) {
  dim3 grid((unsigned)cdiv(T, GCW::BN), (unsigned)cdiv(N, GCW::BM));
  const Opnd wn = make_opnd(Xn, R, N);
  const Opnd wd = make_opnd(Xmu, R, N, Xn);
  const Opnd h = make_opnd(H, T, T);
  prof_begin("cost_W", s);
  if (s0) hipLaunchKernelGGL(k_cost_W<true>, grid, dim3(GCW::NT), 0, s, V, wn, wd, h, N, T, R, part, fpart, zd, dz);
  else hipLaunchKernelGGL(k_cost_W<false>, grid, dim3(GCW::NT), 0, s, V, wn, wd, h, N, T, R, part, fpart, zd, dz);
  prof_end("cost_W", s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Selection (steps 15 and 28).
// ---------------------------------------------------------------------------
// The damped selection (dp.dpart != nullptr): the Newton candidate is kept iff
// its column (row) objective of eq. (5), d_DNA (Sigma c x = Sigma v by eq. 10),
// is not above the current state's, d_cur + Sigma_r c_r x_r - Sigma v; the
// margin is their difference and d_sel is NaN where MU is kept uncosted.
__device__ __forceinline__ bool decide_damped(double dN, int fl, double dcur, double cx, double sv, double& dsel,
                                              double& margin) {
  const bool finite = (fl & 1) == 0;
  margin = finite ? (dcur + cx - sv) - dN : -INFINITY;
  const bool newton = finite && margin >= 0.0;
  dsel = newton ? dN : NAN;
  return newton;
}

// Per-column (row) inputs of the damped rule, each summed in a fixed order:
// the input state's cost parts (dtiles of them), the data sum parts (vtiles)
// and Sigma_r (c_r + reg) x_r of the current factor entries.
__device__ __forceinline__ void damp_sums(const Damp& dp, int64_t L, int64_t idx, double& dcur, double& sv) {
  dcur = 0.0;
  sv = 0.0;
  for (int m = 0; m < dp.dtiles; ++m) dcur += dp.dpart[(int64_t)m * L + idx];
  for (int m = 0; m < dp.vtiles; ++m) sv += dp.vpart[(int64_t)m * L + idx];
}


__global__ __launch_bounds__(256) void k_select_H(const float* __restrict__ Xmu, const float* __restrict__ Xn,
                                                  float* __restrict__ Hout,
                                                  const double* part, const int* fpart, int tiles,
                                                  int64_t T, int64_t R, uint8_t* mask, double* dsel,
                                                  double* margin, Damp dp) {
  // CAND_COLS columns per block: row group 0 decides, every row group copies.
  __shared__ int pick[CAND_COLS];
  const int tid = threadIdx.x, cl = tid % CAND_COLS, rg = tid / CAND_COLS;
  const int64_t t = (int64_t)blockIdx.x * CAND_COLS + cl;
  const bool ok = t < T;
  if (rg == 0 && ok) {
    const int64_t stride = (int64_t)tiles * T;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    int fl = 0;
#pragma unroll 8
    for (int m = 0; m < tiles; ++m) {
      const int64_t o = (int64_t)m * T + t;
      q0 += part[o];
      q1 += part[stride + o];
      q2 += part[2 * stride + o];
      fl |= fpart[o];
    }
    double ds, mg;
    bool nw;
    if (dp.dpart) {                      // Hout still holds the current H
      double dcur, sv, cx = 0.0;
      damp_sums(dp, T, t, dcur, sv);
      for (int64_t r = 0; r < R; ++r) cx += (dp.c64[r] + dp.reg) * (double)Hout[r * T + t];
      nw = decide_damped(q0, fl, dcur, cx, sv, ds, mg);
    } else {
      nw = decide(q0, q1, q2, fl, ds, mg);
    }
    if (mask) mask[t] = nw ? 1 : 0;
    if (dsel) dsel[t] = ds;
    if (margin) margin[t] = mg;
    pick[cl] = nw ? 1 : 0;
  }
  __syncthreads();
  if (!ok) return;
  const float* src = pick[cl] ? Xn : Xmu;
#pragma unroll 8
  for (int64_t r = rg; r < R; r += CAND_RG) Hout[r * T + t] = src[r * T + t];
}

// Many tile partials over few columns: a wave per column (four per block), the
// lanes add the partials, then the wave copies the chosen column (a strided
// copy, so only for few columns: SEL_MANY_COLS).
constexpr int SEL_MANY = 16;
constexpr int64_t SEL_MANY_COLS = 4096;
__global__ __launch_bounds__(256) void k_select_H_cols(const float* __restrict__ Xmu, const float* __restrict__ Xn,
                                                       float* __restrict__ Hout,
                                                       const double* part, const int* fpart, int tiles,
                                                       int64_t T, int64_t R, uint8_t* mask, double* dsel,
                                                       double* margin, Damp dp) {
  const int lane = threadIdx.x & 63;
  const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= T) return;
  const int64_t stride = (int64_t)tiles * T;
  double q0 = 0.0, q1 = 0.0, q2 = 0.0;
  int fl = 0;
  for (int64_t m = lane; m < tiles; m += 64) {
    const int64_t o = m * T + t;
    q0 += part[o];
    q1 += part[stride + o];
    q2 += part[2 * stride + o];
    fl |= fpart[o];
  }
  q0 = __shfl(wave_sum(q0), 0);
  q1 = __shfl(wave_sum(q1), 0);
  q2 = __shfl(wave_sum(q2), 0);
  fl = wave_or(fl);
  double ds, mg;
  bool nw;
  if (dp.dpart) {                        // Hout still holds the current H
    double cx = 0.0;
    for (int64_t r = lane; r < R; r += 64) cx += (dp.c64[r] + dp.reg) * (double)Hout[r * T + t];
    cx = __shfl(wave_sum(cx), 0);
    double dcur, sv;
    damp_sums(dp, T, t, dcur, sv);
    nw = decide_damped(q0, fl, dcur, cx, sv, ds, mg);
  } else {
    nw = decide(q0, q1, q2, fl, ds, mg);
  }
  if (lane == 0) {
    if (mask) mask[t] = nw ? 1 : 0;
    if (dsel) dsel[t] = ds;
    if (margin) margin[t] = mg;
  }
  const float* src = nw ? Xn : Xmu;
  for (int64_t r = lane; r < R; r += 64) Hout[r * T + t] = src[r * T + t];
}

hipError_t launch_select_H(const float* Xmu, const float* Xn, float* Hout, const double* part,
                           const int* fpart, int tiles_m, int64_t T, int64_t R, uint8_t* mask,
                           double* dsel, double* margin, hipStream_t s, const Damp& dp) {
  prof_begin("select_H", s);
  if (tiles_m > SEL_MANY && T <= SEL_MANY_COLS)
    hipLaunchKernelGGL(k_select_H_cols, dim3((unsigned)cdiv(T, 4)), dim3(256), 0, s, Xmu, Xn, Hout, part, fpart,
                       tiles_m, T, R, mask, dsel, margin, dp);
  else
    hipLaunchKernelGGL(k_select_H, dim3((unsigned)cdiv(T, CAND_COLS)), dim3(256), 0, s, Xmu, Xn, Hout, part, fpart,
                       tiles_m, T, R, mask, dsel, margin, dp);
  prof_end("select_H", s);
  return hipGetLastError();
}

// The column sums over a block's four rows of the new W: wave w holds row
// w's entries (`row`, nullptr for a row past N), lane r of every 64-column
// chunk; the four rows are added in order through LDS.  Every wave of the block
// calls this (it has barriers).
__device__ __forceinline__ void select_w_emit(const float* row, int64_t R, int wave, int lane, double* emit) {
  __shared__ double cs[4][64];
  for (int64_t r0 = 0; r0 < R; r0 += 64) {
    const int64_t r = r0 + lane;
    cs[wave][lane] = (row && r < R) ? (double)row[r] : 0.0;
    __syncthreads();
    if (wave == 0 && r < R) emit[(int64_t)blockIdx.x * R + r] = ((cs[0][lane] + cs[1][lane]) + cs[2][lane]) + cs[3][lane];
    __syncthreads();
  }
}

// A wave per row (four rows per block): the lanes add the tile partials.
// With `emit`, the block also writes the float64 sums over its rows of each
// column r of the new W (emit[block * R + r]; parts for the normalisation).
__global__ __launch_bounds__(256) void k_select_W(const float* __restrict__ Xmu, const float* __restrict__ Xn,
                                                  float* __restrict__ Wout,
                                                  const double* part, const int* fpart, int tiles,
                                                  int64_t N, int64_t R, uint8_t* mask, double* dsel,
                                                  double* margin, Damp dp, double* emit) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * 4 + wave;
  if (n >= N) {
    if (emit) select_w_emit(nullptr, R, wave, lane, emit);
    return;
  }
  const int64_t stride = (int64_t)tiles * N;
  double q0 = 0.0, q1 = 0.0, q2 = 0.0;
  int fl = 0;
  for (int64_t m = lane; m < tiles; m += 64) {
    const int64_t o = m * N + n;
    q0 += part[o];
    q1 += part[stride + o];
    q2 += part[2 * stride + o];
    fl |= fpart[o];
  }
  q0 = __shfl(wave_sum(q0), 0);
  q1 = __shfl(wave_sum(q1), 0);
  q2 = __shfl(wave_sum(q2), 0);
  fl = wave_or(fl);
  double ds, mg;
  bool nw;
  if (dp.dpart) {                        // Wout still holds the current W
    double cx = 0.0;
    for (int64_t r = lane; r < R; r += 64) cx += (dp.c64[r] + dp.reg) * (double)Wout[n * R + r];
    cx = __shfl(wave_sum(cx), 0);
    double dcur, sv;
    damp_sums(dp, N, n, dcur, sv);
    nw = decide_damped(q0, fl, dcur, cx, sv, ds, mg);
  } else {
    nw = decide(q0, q1, q2, fl, ds, mg);
  }
  if (lane == 0) {
    if (mask) mask[n] = nw ? 1 : 0;
    if (dsel) dsel[n] = ds;
    if (margin) margin[n] = mg;
  }
  const float* src = nw ? Xn : Xmu;
  for (int64_t r = lane; r < R; r += 64) Wout[n * R + r] = src[n * R + r];
  if (emit) select_w_emit(src + n * R, R, wave, lane, emit);
}

// Few tile partials (at most SEL_FEW, e.g. the sparse path's one): SEL_ROWS
// rows per block, one thread per row adds its partials in order and decides;
// then each wave copies every fourth of the block's rows.
constexpr int SEL_ROWS = 64, SEL_FEW = 4;
__global__ __launch_bounds__(256) void k_select_W_rows(const float* __restrict__ Xmu, const float* __restrict__ Xn,
                                                       float* __restrict__ Wout,
                                                       const double* part, const int* fpart, int tiles,
                                                       int64_t N, int64_t R, uint8_t* mask, double* dsel,
                                                       double* margin, Damp dp, double* emit) {
  __shared__ int pick[SEL_ROWS];
  __shared__ double cs[4][64];
  const int tid = threadIdx.x;
  const int64_t n0 = (int64_t)blockIdx.x * SEL_ROWS;
  if (tid < SEL_ROWS && n0 + tid < N) {
    const int64_t n = n0 + tid;
    const int64_t stride = (int64_t)tiles * N;
    double q0 = 0.0, q1 = 0.0, q2 = 0.0;
    int fl = 0;
#pragma unroll 4
    for (int m = 0; m < tiles; ++m) {
      const int64_t o = (int64_t)m * N + n;
      q0 += part[o];
      q1 += part[stride + o];
      q2 += part[2 * stride + o];
      fl |= fpart[o];
    }
    double ds, mg;
    bool nw;
    if (dp.dpart) {                      // Wout still holds the current W
      double dcur, sv, cx = 0.0;
      damp_sums(dp, N, n, dcur, sv);
      for (int64_t r = 0; r < R; ++r) cx += (dp.c64[r] + dp.reg) * (double)Wout[n * R + r];
      nw = decide_damped(q0, fl, dcur, cx, sv, ds, mg);
    } else {
      nw = decide(q0, q1, q2, fl, ds, mg);
    }
    if (mask) mask[n] = nw ? 1 : 0;
    if (dsel) dsel[n] = ds;
    if (margin) margin[n] = mg;
    pick[tid] = nw ? 1 : 0;
  }
  __syncthreads();
  const int64_t rows = std::min<int64_t>(SEL_ROWS, N - n0);
  const int lane = tid & 63, wave = tid >> 6;
  for (int64_t nl = wave; nl < rows; nl += 4) {
    const int64_t o = (n0 + nl) * R;
    const float* src = pick[nl] ? Xn : Xmu;
    for (int64_t r = lane; r < R; r += 64) Wout[o + r] = src[o + r];
  }
  if (emit) {   // column sums over the block's rows: each wave every fourth row, then the four waves in order
    for (int64_t r0 = 0; r0 < R; r0 += 64) {
      const int64_t r = r0 + lane;
      double a = 0.0;
      if (r < R)
        for (int64_t nl = wave; nl < rows; nl += 4) a += (double)(pick[nl] ? Xn : Xmu)[(n0 + nl) * R + r];
      cs[wave][lane] = a;
      __syncthreads();
      if (wave == 0 && r < R) emit[(int64_t)blockIdx.x * R + r] = ((cs[0][lane] + cs[1][lane]) + cs[2][lane]) + cs[3][lane];
      __syncthreads();
    }
  }
}

int select_w_parts(int tiles_n, int64_t N) { return (int)(tiles_n <= SEL_FEW ? cdiv(N, SEL_ROWS) : cdiv(N, 4)); }

hipError_t launch_select_W(const float* Xmu, const float* Xn, float* Wout, const double* part,
                           const int* fpart, int tiles_n, int64_t N, int64_t R, uint8_t* mask,
                           double* dsel, double* margin, hipStream_t s, const Damp& dp, double* emit) {
  prof_begin("select_W", s);
  if (tiles_n <= SEL_FEW)
    hipLaunchKernelGGL(k_select_W_rows, dim3((unsigned)cdiv(N, SEL_ROWS)), dim3(256), 0, s, Xmu, Xn, Wout, part,
                       fpart, tiles_n, N, R, mask, dsel, margin, dp, emit);
  else
    hipLaunchKernelGGL(k_select_W, dim3((unsigned)cdiv(N, 4)), dim3(256), 0, s, Xmu, Xn, Wout, part, fpart,
                       tiles_n, N, R, mask, dsel, margin, dp, emit);
  prof_end("select_W", s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// MU updates (eq. 11): X <- X * numerator / scale.
// ---------------------------------------------------------------------------
// A thread per entry (r, t): 64 columns x 4 rows per block, rows over the
// grid's y; the split sums are unrolled so their loads overlap (order kept).
__global__ __launch_bounds__(256) void k_mu_H(float* H, const float* pu, int splits, const float* c,
                                              int64_t T, int64_t R, const double* cpart, int tiles,
                                              double* d_out) {
  const int tid = threadIdx.x, cl = tid & 63, rg = tid >> 6;
  const int64_t t = (int64_t)blockIdx.x * 64 + cl;
  const int64_t r = (int64_t)blockIdx.y * 4 + rg;
  if (t >= T) return;
  if (r < R) {
    float u = 0.f;
#pragma unroll 8
    for (int sp = 0; sp < splits; ++sp) u += pu[(sp * R + r) * T + t];
    H[r * T + t] = fmaxf(H[r * T + t] * (u / c[r]), VALUE_FLOOR);     // eq. (11): h (W^t q)_r / c_r
  }
  if (d_out && blockIdx.y == 0 && rg == 0) {
    double s = 0.0;
#pragma unroll 8
    for (int m = 0; m < tiles; ++m) s += cpart[(int64_t)m * T + t];
    d_out[t] = s;
  }
}

hipError_t launch_mu_H(float* H, const float* pu, int splits, const float* c, int64_t T, int64_t R,
                       const double* cpart, int tiles_m, double* d_out, hipStream_t s) {
  prof_begin("mu_H", s);
  hipLaunchKernelGGL(k_mu_H, dim3((unsigned)cdiv(T, 64), (unsigned)cdiv(R, 4)), dim3(256), 0, s, H, pu, splits, c,
                     T, R, cpart, tiles_m, d_out);
  prof_end("mu_H", s);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_mu_W(float* W, const float* pu, int splits, const float* g,
                                              int64_t N, int64_t R, const double* cpart, int tiles,
                                              double* d_out) {
  const int lane = threadIdx.x & 63;
  const int64_t n = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (n >= N) return;
  for (int64_t r = lane; r < R; r += 64) {
    float u = 0.f;
#pragma unroll 8
    for (int sp = 0; sp < splits; ++sp) u += pu[(sp * N + n) * R + r];
    W[n * R + r] = fmaxf(W[n * R + r] * (u / g[r]), VALUE_FLOOR);
  }
  if (d_out) {
    double s = 0.0;
    for (int64_t m = lane; m < tiles; m += 64) s += cpart[m * N + n];
    s = wave_sum(s);
    if (lane == 0) d_out[n] = s;
  }
}

hipError_t launch_mu_W(float* W, const float* pu, int splits, const float* g, int64_t N, int64_t R,
                       const double* cpart, int tiles_n, double* d_out, hipStream_t s) {
  prof_begin("mu_W", s);
  hipLaunchKernelGGL(k_mu_W, dim3((unsigned)cdiv(N, 4)), dim3(256), 0, s, W, pu, splits, g, N, R, cpart,
                     tiles_n, d_out);
  prof_end("mu_W", s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Normalisation (steps 1, 16, 29) and the column / row sums they need.
// ---------------------------------------------------------------------------
// Column sums of W (N x R) and row sums of H (R x T), each in two fixed-order
// levels: `nparts` blocks per column / row write partial float64 sums to
// part[p][r]; the second level adds the parts in order (sum_job).
// 64 columns x CS_RG row groups per block (tall W with few parts keeps more
// loads in flight per block); the row groups are added in a fixed tree.
constexpr int CS_RG = 16;
__global__ __launch_bounds__(64 * CS_RG) void k_colsum_part(const float* W, int64_t N, int64_t R, int64_t rows,
                                                           double* part) {
  __shared__ double red[CS_RG][64];
  const int tid = threadIdx.x, cl = tid & 63, rg = tid >> 6;
  const int64_t r = (int64_t)blockIdx.x * 64 + cl;
  const int64_t p = blockIdx.y;
  const int64_t n1 = std::min<int64_t>(N, (p + 1) * rows);
  double s = 0.0;
  if (r < R) {
#pragma unroll 8
    for (int64_t n = p * rows + rg; n < n1; n += CS_RG) s += (double)W[n * R + r];
  }
  red[rg][cl] = s;
  __syncthreads();
#pragma unroll
  for (int h = CS_RG / 2; h >= 1; h >>= 1) {
    if (rg < h) red[rg][cl] += red[rg + h][cl];
    __syncthreads();
  }
  if (rg == 0 && r < R) part[p * R + r] = red[0][cl];
}

__global__ __launch_bounds__(256) void k_rowsum_part(const float* H, int64_t T, int64_t R, int64_t cols,
                                                     double* part) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  const int64_t p = blockIdx.x, r = blockIdx.y;
  const int64_t t1 = std::min<int64_t>(T, (p + 1) * cols);
  double s = 0.0;
#pragma unroll 8
  for (int64_t t = p * cols + tid; t < t1; t += 256) s += (double)H[r * T + t];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) part[p * R + r] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_sum_final(SumJob j) { sum_job(j); }

hipError_t launch_colsum_part(const float* W, int64_t N, int64_t R, double* part, SumJob& job, hipStream_t s) {
  const int64_t nparts = std::min<int64_t>(SUM_PARTS, cdiv(N, 64));
  const int64_t rows = cdiv(N, nparts);
  prof_begin("colsum_W", s);
  hipLaunchKernelGGL(k_colsum_part, dim3((unsigned)cdiv(R, 64), (unsigned)nparts), dim3(64 * CS_RG), 0, s, W, N,
                     R, rows, part);
  prof_end("colsum_W", s);
  job = SumJob{part, (int)nparts, R, nullptr, nullptr, nullptr};
  return hipGetLastError();
}

hipError_t launch_rowsum_part(const float* H, int64_t T, int64_t R, double* part, SumJob& job, hipStream_t s) {
  const int64_t nparts = std::min<int64_t>(SUM_PARTS, cdiv(T, 2048));
  const int64_t cols = cdiv(T, nparts);
  prof_begin("rowsum_H", s);
  hipLaunchKernelGGL(k_rowsum_part, dim3((unsigned)nparts, (unsigned)R), dim3(256), 0, s, H, T, R, cols, part);
  prof_end("rowsum_H", s);
  job = SumJob{part, (int)nparts, R, nullptr, nullptr, nullptr};
  return hipGetLastError();
}

hipError_t launch_sum_final(const SumJob& job, hipStream_t s) {
  prof_begin("sum_final", s);
  hipLaunchKernelGGL(k_sum_final, dim3((unsigned)cdiv(job.R, 256)), dim3(256), 0, s, job);
  prof_end("sum_final", s);
  return hipGetLastError();
}

// Normalisation with the second level of the sums done per tile: blocks
// [0, wtiles) scale (4096 / WR) x WR tiles of W (WR columns r, each block
// summing the parts of its WR factors, 256 / WR lanes per column); the
// remaining blocks scale a chunk of one row r of H (SC_TCHUNK entries, or the
// whole row where the parts are so many that every chunk re-reading all of
// them would cost more than the row: then HP = 32 entries per lane and
// piece).  WR = 64 serves
// few parts; with many (the W selection leaves one per four rows of W) the
// part sums of 64-column tiles become long dependent chains, and WR = 16 cuts
// them to a quarter.  Every block loads its factor entries before it adds the
// parts, so the two latencies overlap.  Multiplying by the float64 reciprocal
// of f rounds like dividing except in double-rounding ties.  With `emit`, the
// blocks of the normalised factor (W tiles for side 0, H chunks for side 1)
// also write the float64 sum of the values they stored (an unchanged column /
// row where f is not positive): emit[tile * R + r].
//
// With `o.part` (the balanced normalisation of eq. 2, both weights positive)
// the other factor's sums come in `o` and f becomes sqrt(w_j * S_j / (w_o * S_o))
// (S: the two sums, w: their eq. 2 weights; side 0: S_j = C with rho, S_o = G
// with lambda; side 1 the reverse), so W column r is multiplied by
// sqrt(lambda G_r / (rho C_r)) either way; a sum that is not positive leaves
// the column / row unscaled and sets CHK_DOMAIN.
constexpr int SC_MANY_PARTS = 128;   // above this many parts the 16-column W tiles
__device__ __forceinline__ double balance_factor(double sj, double so, double wj, double wo, int* check) {
  if (sj > 0.0 && so > 0.0) return sqrt((wj * sj) / (wo * so));
  if (check) atomicOr(check, CHK_DOMAIN);
  return 0.0;
}

// Sum of x over the lanes of a wave with equal lane % WR, in a fixed order
// (every such lane ends with the same value: the pairings are symmetric).
template <int WR>
__device__ __forceinline__ double lane_group_sum(double x) {
  if constexpr (WR <= 16) x += __shfl_xor(x, 16);
  if constexpr (WR <= 32) x += __shfl_xor(x, 32);
  return x;
}

template <int WR, int HP>
__global__ __launch_bounds__(256) void k_scale(int side, float* __restrict__ W, float* __restrict__ H, int64_t N,
                                               int64_t T, int64_t R, SumJob j, SumJob o, double wj, double wo,
                                               int64_t rtiles, int64_t wtiles, int64_t tchunks, int64_t tspan,
                                               double* __restrict__ emit) {
  constexpr int WG = 256 / WR, WN = 4096 / WR, WPER = WN / WG;   // lane groups, tile rows, rows per lane
  static_assert(WR == 16 || WR == 32 || WR == 64, "16, 32 or 64 columns per W tile");
  __shared__ double fs[WR];
  __shared__ double red[4][WR];
  __shared__ double red2[4][WR];
  const int tid = threadIdx.x, wave = tid >> 6;
  const int64_t b = blockIdx.x;
  if (b < wtiles) {
    const int64_t rt = b % rtiles, nt = b / rtiles;
    const int rr = tid % WR, g = tid / WR;
    const int64_t r = rt * WR + rr;
    const int64_t nb = nt * WN + g;
    float w[WPER];
#pragma unroll
    for (int k = 0; k < WPER; ++k) {
      const int64_t n = nb + WG * k;
      w[k] = (n < N && r < R) ? W[n * R + r] : 0.f;
    }
    {  // WG groups of WR lanes add every WG-th part, then the groups are added
      double f = 0.0, f2 = 0.0;
      if (r < R) {
#pragma unroll 8
        for (int p = g; p < j.nparts; p += WG) f += j.part[(int64_t)p * R + r];
        if (o.part)
#pragma unroll 8
          for (int p = g; p < o.nparts; p += WG) f2 += o.part[(int64_t)p * R + r];
      }
      f = lane_group_sum<WR>(f);
      f2 = lane_group_sum<WR>(f2);
      if ((tid & 63) < WR) {
        red[wave][rr] = f;
        red2[wave][rr] = f2;
      }
    }
    __syncthreads();
    if (tid < WR) {
      double f = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
      const bool in = rt * WR + tid < R;
      if (o.part) {
        const double f2 = (red2[0][tid] + red2[1][tid]) + (red2[2][tid] + red2[3][tid]);
        f = in ? balance_factor(f, f2, wj, wo, j.check) : 0.0;
      } else if (j.check && in && !(f > 0.0)) {
        atomicOr(j.check, CHK_DOMAIN);
      }
      fs[tid] = f;
    }
    __syncthreads();
    const double f = fs[rr];
    const bool sc = r < R && f > 0.0;
    const double m = side == 0 ? 1.0 / f : f;
    double cs = 0.0;
#pragma unroll
    for (int k = 0; k < WPER; ++k) {
      const int64_t n = nb + WG * k;
      const float x = sc ? (float)((double)w[k] * m) : w[k];
      if (sc && n < N) W[n * R + r] = x;
      cs += (double)x;                            // 0 outside the matrix
    }
    if (emit && side == 0) {                      // column sums of this tile of the new W
      cs = lane_group_sum<WR>(cs);
      if ((tid & 63) < WR) red[wave][rr] = cs;
      __syncthreads();
      if (tid < WR && rt * WR + tid < R)
        emit[nt * R + rt * WR + tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
    }
  } else {
    const int64_t hb = b - wtiles;
    const int64_t r = hb / tchunks, ch = hb % tchunks;
    const int64_t tb = ch * tspan, te = std::min<int64_t>(T, tb + tspan);   // pieces of 256 HP entries
    float h[HP];
#pragma unroll
    for (int k = 0; k < HP; ++k) {
      const int64_t t = tb + tid + 256 * k;
      h[k] = t < te ? H[r * T + t] : 0.f;
    }
    if (tid < 64) {  // one wave: a lane per part, fixed-order butterfly
      double f = tid < j.nparts ? j.part[(int64_t)tid * R + r] : 0.0;
#pragma unroll 8
      for (int p = tid + 64; p < j.nparts; p += 64) f += j.part[(int64_t)p * R + r];
      f = wave_sum(f);
      if (o.part) {
        double f2 = tid < o.nparts ? o.part[(int64_t)tid * R + r] : 0.0;
        for (int p = tid + 64; p < o.nparts; p += 64) f2 += o.part[(int64_t)p * R + r];
        f2 = wave_sum(f2);
        if (tid == 0) f = balance_factor(f, f2, wj, wo, nullptr);   // the W tiles report
      }
      if (tid == 0) fs[0] = f;
    }
    __syncthreads();
    const double f = fs[0];
    const bool sc = f > 0.0;
    const double m = side == 0 ? f : 1.0 / f;
    double rs = 0.0;
    for (int64_t t0 = tb; t0 < te; t0 += 256 * HP) {
      if (t0 != tb)
#pragma unroll
        for (int k = 0; k < HP; ++k) {
          const int64_t t = t0 + tid + 256 * k;
          h[k] = t < te ? H[r * T + t] : 0.f;
        }
#pragma unroll
      for (int k = 0; k < HP; ++k) {
        const int64_t t = t0 + tid + 256 * k;
        const float x = sc ? (float)((double)h[k] * m) : h[k];
        if (sc && t < te) H[r * T + t] = x;
        rs += (double)x;                          // 0 outside the matrix
      }
    }
    if (emit && side == 1) {                      // row sum of this chunk of the new H
      rs = wave_sum(rs);
      if ((tid & 63) == 0) red[0][tid >> 6] = rs;
      __syncthreads();
      if (tid == 0) emit[ch * R + r] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    }
  }
}

// out[0] += rho sum_r C_r + lambda sum_r G_r (the penalty of eq. 2), C and G
// finished from their parts; one block, fixed-order reduction.
__global__ __launch_bounds__(256) void k_penalty(SumJob cj, SumJob gj, double rho, double lam, double* out) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int64_t r = tid; r < cj.R; r += 256) {
    double C = 0.0, G = 0.0;
    for (int p = 0; p < cj.nparts; ++p) C += cj.part[(int64_t)p * cj.R + r];
    for (int p = 0; p < gj.nparts; ++p) G += gj.part[(int64_t)p * gj.R + r];
    acc += rho * C + lam * G;
  }
  acc = wave_sum(acc);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid == 0) out[0] += (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_penalty(const SumJob& cj, const SumJob& gj, double rho, double lam, double* out, hipStream_t s) {
  prof_begin("penalty", s);
  hipLaunchKernelGGL(k_penalty, dim3(1), dim3(256), 0, s, cj, gj, rho, lam, out);
  prof_end("penalty", s);
  return hipGetLastError();
}

// The most parts any normalisation emits (the 64-column W tiles emit the most).
int64_t scale_emit_parts(int side, int64_t N, int64_t T) {
  return side == 0 ? cdiv(N, 64) : cdiv(T, SC_TCHUNK);
}

hipError_t launch_scale(int side, float* W, float* H, int64_t N, int64_t T, int64_t R, const SumJob& job,
                        double* emit, SumJob* emitted, hipStream_t s, const SumJob& other, double wj, double wo) {
  const int64_t np = std::max(job.nparts, other.part ? other.nparts : 0);
  const bool many = np > SC_MANY_PARTS;
  const int wr = many ? 16 : 64, wn = 4096 / wr;
  const int64_t rtiles = cdiv(R, wr), wtiles = rtiles * cdiv(N, wn);
  // every chunk of an H row reads all of the row's parts (8 bytes each, a
  // sector apart): fewer chunks where those reads would pass about 32 MiB
  const int64_t cap = std::max<int64_t>(1, (int64_t(1) << 25) / std::max<int64_t>(1, R * np * 64));
  const int64_t want = std::min(cdiv(T, SC_TCHUNK), cap);
  const int64_t tspan = cdiv(cdiv(T, want), SC_TCHUNK) * SC_TCHUNK, tchunks = cdiv(T, tspan);
  const bool longrow = tspan > SC_TCHUNK;
  const int64_t blocks = wtiles + R * tchunks;
  typedef void (*Kern)(int, float*, float*, int64_t, int64_t, int64_t, SumJob, SumJob, double, double, int64_t,
                       int64_t, int64_t, int64_t, double*);
  const Kern k = many ? (longrow ? k_scale<16, 32> : k_scale<16, SC_TCHUNK / 256>)
                      : (longrow ? k_scale<64, 32> : k_scale<64, SC_TCHUNK / 256>);
  prof_begin("scale", s);
  hipLaunchKernelGGL(k, dim3((unsigned)blocks), dim3(256), 0, s, side, W, H, N, T, R, job, other, wj, wo, rtiles,
                     wtiles, tchunks, tspan, emit);
  prof_end("scale", s);
  if (emit && emitted)
    *emitted = SumJob{emit, (int)(side == 0 ? cdiv(N, wn) : tchunks), R, nullptr, nullptr, nullptr};
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_kl_final(const double* cpart, int ntiles, double* out) {
  __shared__ double red[4];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int k = tid; k < ntiles; k += 256) s += cpart[k];
  s = wave_sum(s);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_kl_final(const double* cpart, int ntiles, double* out, hipStream_t s) {
  prof_begin("kl_final", s);
  hipLaunchKernelGGL(k_kl_final, dim3(1), dim3(256), 0, s, cpart, ntiles, out);
  prof_end("kl_final", s);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_check(const float* X, int64_t n, int* check) {
  int fl = 0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const float x = X[e];
    if (!isfinite(x)) fl |= CHK_NONFINITE;
    else if (x < 0.f) fl |= CHK_DOMAIN;
  }
  fl = wave_or(fl);
  if ((threadIdx.x & 63) == 0 && fl) atomicOr(check, fl);
}

hipError_t launch_check(const float* X, int64_t n, int* check, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<int64_t>(cdiv(n, 256), 4096);
  prof_begin("check", s);
  hipLaunchKernelGGL(k_check, dim3(blocks), dim3(256), 0, s, X, n, check);
  prof_end("check", s);
  return hipGetLastError();
}

}  // namespace dna
