// kernels_16.hip -- the precision form: the five products of a DNA half-step
// (Z, the gradient/Hessian pair, the two candidate reconstructions) with bf16 or
// fp16 MFMA operands and fp32 accumulation; Q, Q - 1 and Q-bar handed between
// kernels in 16-bit.  Candidates, costs (float64 sums) and selection are the
// fp32 path's.  fp16 needs power-of-two scales to stay in range:
//   * rank scales: W columns scaled to max 1 (and H rows by the inverse) inside
//     the Z-type products, where they cancel exactly; in the gradient products
//     the scale of W^t (H^t) is folded out of the result;
//   * Q, Q - 1, Q-bar scaled per column (H step) / per row (W step) so that each
//     column's (row's) maximum is 2^13, from a max pass over the same Z tiles,
//     and folded out of the gradient sums.
// bf16 keeps fp32's exponent range and uses no scales.
#include <math.h>

#include <algorithm>

#include "core16.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"
#include "kernels_16.hpp"

namespace dna {

constexpr int BK16 = 32;
using G16R = Geo16<RT_BM, RT_BN, BK16, 2, 2>;    // ratio / max pass: M = N, N = T, K = R
using G16CH = Geo16<CH_BM, CH_BN, BK16, 2, 2>;   // H-orientation cost
using G16CW = Geo16<CW_BM, CW_BN, BK16, 2, 2>;   // W-orientation cost
using G16H = Geo16<GH_BM, GH_BN, BK16, 2, 2>;    // H-orientation gradient: M = R, N = T, K = N
using G16W = Geo16<GW_BM, GW_BN, BK16, 2, 2>;    // W-orientation gradient: M = N, N = R, K = T

// ---------------------------------------------------------------------------
// Policies: which global sources are staged into which LDS tiles, and the
// products formed from them.
// ---------------------------------------------------------------------------

// Z-type products (K = R).  A sources are K-major fp32 (W or W candidates), B
// sources MN-major fp32 (H or H candidates).  NA_ x NB_ sources; products:
//   NA = NB = 1: C0 = A0 B0
//   NA = 1, NB = 2: C0 = A0 B0, C1 = A0 B1
//   NA = 2, NB = 1: C0 = A0 B0, C1 = A1 B0
// SPLIT (NA = NB = 1 only): bit 0 stages B as hi + lo 16-bit parts, bit 1 does
// the same for A, and the product adds the cross terms A_hi B_lo / A_lo B_hi, so
// that the split operand enters with about twice the 16-bit precision.
template <class G, typename TE, int NA_, int NB_, int SPLIT = 0>
struct PolZ {
  static_assert(SPLIT == 0 || (NA_ == 1 && NB_ == 1), "split operands only in the single product");
  static constexpr bool SA = (SPLIT & 2) != 0, SB = (SPLIT & 1) != 0;
  static constexpr int NC = (NA_ > NB_) ? NA_ : NB_;
  static constexpr int TA = G::BM * G::PITCH, TB = G::BN * G::PITCH;
  static constexpr int LA = NA_ + (SA ? 1 : 0), LB = NB_ + (SB ? 1 : 0);   // LDS tiles per side
  static constexpr int LDS_ELEMS = LA * TA + LB * TB;
  typedef typename MF<TE>::v8 V8;
  Stage16<G::BM, G::BK, G::NT, float, TE, true> sa[NA_];
  Stage16<G::BN, G::BK, G::NT, float, TE, false> sb[NB_];
  Op16 A[NA_], B[NB_];
  int64_t m0, n0;

  __device__ __forceinline__ void load(int64_t k0, int64_t k_end, int tid) {
#pragma unroll
    for (int a = 0; a < NA_; ++a) sa[a].load(A[a], m0, k0, k_end, tid);
#pragma unroll
    for (int b = 0; b < NB_; ++b) sb[b].load(B[b], n0, k0, k_end, tid);
  }
  __device__ __forceinline__ void store(TE* lds, int64_t k0, int64_t k_end, int tid) {
#pragma unroll
    for (int a = 0; a < NA_; ++a) sa[a].template store<XF_ID>(lds + a * TA, A[a], m0, k0, k_end, tid);
    if (SA) sa[0].template store<XF_LO>(lds + NA_ * TA, A[0], m0, k0, k_end, tid);
#pragma unroll
    for (int b = 0; b < NB_; ++b) sb[b].template store<XF_ID>(lds + LA * TA + b * TB, B[b], n0, k0, k_end, tid);
    if (SB) sb[0].template store<XF_LO>(lds + LA * TA + NB_ * TB, B[0], n0, k0, k_end, tid);
  }
  __device__ __forceinline__ void compute(const TE* lds, f32x16 (&acc)[G::FM][G::FN][NC], int lane, int wm, int wn) {
#pragma unroll
    for (int kk = 0; kk < G::BK / 16; ++kk) {
      V8 a[LA][G::FM], b[LB][G::FN];
#pragma unroll
      for (int x = 0; x < LA; ++x)
#pragma unroll
        for (int i = 0; i < G::FM; ++i)
          a[x][i] = frag16<TE>(lds + x * TA, G::PITCH, wm * G::WM + i * 32 + (lane & 31), kk, lane);
#pragma unroll
      for (int y = 0; y < LB; ++y)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
          b[y][j] = frag16<TE>(lds + LA * TA + y * TB, G::PITCH, wn * G::WN + j * 32 + (lane & 31), kk, lane);
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j) {
          if (SPLIT) {
            // small cross terms first, then the hi x hi product
            if (SB) acc[i][j][0] = MF<TE>::mma(a[0][i], b[1][j], acc[i][j][0]);
            if (SA) acc[i][j][0] = MF<TE>::mma(a[1][i], b[0][j], acc[i][j][0]);
            acc[i][j][0] = MF<TE>::mma(a[0][i], b[0][j], acc[i][j][0]);
          } else {
#pragma unroll
            for (int c = 0; c < NC; ++c)
              acc[i][j][c] = MF<TE>::mma(a[NA_ > 1 ? c : 0][i], b[NB_ > 1 ? c : 0][j], acc[i][j][c]);
          }
        }
    }
  }
};

// H-orientation gradient (M = R, N = T, K = N).  Sources: W (fp32, element
// (r, n) MN-contiguous) staged as w and w^2; Q, Q - 1, Q-bar (16-bit, element
// (t, n) MN-contiguous).  C0 = W^t Q (u), C1 = W^t (Q - 1) (u_c), C2 = (W*W)^t Q-bar (y).
template <class G, typename TE>
struct PolGH_H {
  static constexpr int NC = 3;
  static constexpr int TA = G::BM * G::PITCH, TB = G::BN * G::PITCH;
  static constexpr int LDS_ELEMS = 2 * TA + 3 * TB;
  typedef typename MF<TE>::v8 V8;
  Stage16<G::BM, G::BK, G::NT, float, TE, false> sw;
  Stage16<G::BN, G::BK, G::NT, TE, TE, false> sq[3];
  Op16 W, Q[3];
  int64_t m0, n0;

  __device__ __forceinline__ void load(int64_t k0, int64_t k_end, int tid) {
    sw.load(W, m0, k0, k_end, tid);
#pragma unroll
    for (int x = 0; x < 3; ++x) sq[x].load(Q[x], n0, k0, k_end, tid);
  }
  __device__ __forceinline__ void store(TE* lds, int64_t k0, int64_t k_end, int tid) {
    sw.template store<XF_ID>(lds, W, m0, k0, k_end, tid);
    sw.template store<XF_SQ>(lds + TA, W, m0, k0, k_end, tid);
#pragma unroll
    for (int x = 0; x < 3; ++x) sq[x].template store<XF_ID>(lds + 2 * TA + x * TB, Q[x], n0, k0, k_end, tid);
  }
  __device__ __forceinline__ void compute(const TE* lds, f32x16 (&acc)[G::FM][G::FN][NC], int lane, int wm, int wn) {
#pragma unroll
    for (int kk = 0; kk < G::BK / 16; ++kk) {
      V8 a[2][G::FM], b[3][G::FN];
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int i = 0; i < G::FM; ++i)
          a[x][i] = frag16<TE>(lds + x * TA, G::PITCH, wm * G::WM + i * 32 + (lane & 31), kk, lane);
#pragma unroll
      for (int y = 0; y < 3; ++y)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
          b[y][j] = frag16<TE>(lds + 2 * TA + y * TB, G::PITCH, wn * G::WN + j * 32 + (lane & 31), kk, lane);
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j) {
          acc[i][j][0] = MF<TE>::mma(a[0][i], b[0][j], acc[i][j][0]);
          acc[i][j][1] = MF<TE>::mma(a[0][i], b[1][j], acc[i][j][1]);
          acc[i][j][2] = MF<TE>::mma(a[1][i], b[2][j], acc[i][j][2]);
        }
    }
  }
};

// W-orientation gradient (M = N, N = R, K = T).  Sources: Q, Q - 1, Q-bar (16-bit,
// element (n, t) K-contiguous); H (fp32, element (r, t) K-contiguous) staged as h
// and h^2.  C0 = Q H^t (u), C1 = (Q - 1) H^t (u_c), C2 = Q-bar (H*H)^t (y).
template <class G, typename TE>
struct PolGH_W {
  static constexpr int NC = 3;
  static constexpr int TA = G::BM * G::PITCH, TB = G::BN * G::PITCH;
  static constexpr int LDS_ELEMS = 3 * TA + 2 * TB;
  typedef typename MF<TE>::v8 V8;
  Stage16<G::BM, G::BK, G::NT, TE, TE, true> sq[3];
  Stage16<G::BN, G::BK, G::NT, float, TE, true> sh;
  Op16 Q[3], H;
  int64_t m0, n0;

  __device__ __forceinline__ void load(int64_t k0, int64_t k_end, int tid) {
#pragma unroll
    for (int x = 0; x < 3; ++x) sq[x].load(Q[x], m0, k0, k_end, tid);
    sh.load(H, n0, k0, k_end, tid);
  }
  __device__ __forceinline__ void store(TE* lds, int64_t k0, int64_t k_end, int tid) {
#pragma unroll
    for (int x = 0; x < 3; ++x) sq[x].template store<XF_ID>(lds + x * TA, Q[x], m0, k0, k_end, tid);
    sh.template store<XF_ID>(lds + 3 * TA, H, n0, k0, k_end, tid);
    sh.template store<XF_SQ>(lds + 3 * TA + TB, H, n0, k0, k_end, tid);
  }
  __device__ __forceinline__ void compute(const TE* lds, f32x16 (&acc)[G::FM][G::FN][NC], int lane, int wm, int wn) {
#pragma unroll
    for (int kk = 0; kk < G::BK / 16; ++kk) {
      V8 a[3][G::FM], b[2][G::FN];
#pragma unroll
      for (int x = 0; x < 3; ++x)
#pragma unroll
        for (int i = 0; i < G::FM; ++i)
          a[x][i] = frag16<TE>(lds + x * TA, G::PITCH, wm * G::WM + i * 32 + (lane & 31), kk, lane);
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int j = 0; j < G::FN; ++j)
          b[y][j] = frag16<TE>(lds + 3 * TA + y * TB, G::PITCH, wn * G::WN + j * 32 + (lane & 31), kk, lane);
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int j = 0; j < G::FN; ++j) {
          acc[i][j][0] = MF<TE>::mma(a[0][i], b[0][j], acc[i][j][0]);
          acc[i][j][1] = MF<TE>::mma(a[1][i], b[0][j], acc[i][j][1]);
          acc[i][j][2] = MF<TE>::mma(a[2][i], b[1][j], acc[i][j][2]);
        }
    }
  }
};

// ---------------------------------------------------------------------------
// Ratio pass (and its max-only variant for the fp16 scales).
// ---------------------------------------------------------------------------
struct Ratio16Args {
  const float* V;
  Op16 W, H;
  int64_t N, T, R;
  void* Q; void* Qc; void* Qb;      // 16-bit outputs (element type of the instantiation)
  double* vpart;
  const float* qs[3];               // output scales of Q, Q - 1, Q-bar (nullptr = 1)
  unsigned* qmax[3];                // max pass: float bits of max |.| per column / row
  int* check;
  SumJob fin;                       // folded second level of the factor sum (not in the max pass)
};

// SIDE 0: H step (column sums of V, scales per column t); SIDE 1: W step (rows n).
// SPLIT as in PolZ: the factor being updated (H in the H step, W in the W step)
// must enter Z with more than 16-bit precision -- otherwise the gradient is
// taken at a point a relative 16-bit rounding away from the one the step is
// applied to, an error that does not shrink as the fit converges.
template <typename TE, int SIDE, bool MAXONLY, int SPLIT>
__global__ __launch_bounds__(G16R::NT) void k_ratio16(Ratio16Args a) {
  using G = G16R;
  typedef PolZ<G, TE, 1, 1, SPLIT> P;
  __shared__ __align__(16) TE lds[P::LDS_ELEMS > 4 * G::BM * 8 ? P::LDS_ELEMS : 4 * G::BM * 8];
  const int64_t m0 = (int64_t)blockIdx.y * G::BM, n0 = (int64_t)blockIdx.x * G::BN;
  if (!MAXONLY) sum_job(a.fin);
  float vf[G::FM][G::FN][16];
#pragma unroll
  for (int j = 0; j < G::FN; ++j) {
    const int64_t col = std::min<int64_t>(col16<G>(n0, j), a.T - 1);
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) vf[i][j][v] = a.V[std::min<int64_t>(row16<G>(m0, i, v), a.N - 1) * a.T + col];
  }
  f32x16 acc[G::FM][G::FN][1];
  zero16<G, 1>(acc);
  P pol;
  pol.A[0] = a.W;
  pol.B[0] = a.H;
  pol.m0 = m0;
  pol.n0 = n0;
  run16<G, P, TE>(pol, acc, 0, a.R, lds);
  const int64_t N = a.N, T = a.T;
  double cp[1][G::FN];
  double rp[1][G::FM][16];
#pragma unroll
  for (int j = 0; j < G::FN; ++j) cp[0][j] = 0.0;
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) rp[0][i][v] = 0.0;
  float mx[3][G::FN] = {};        // max pass, SIDE 0: per column of this lane
  int bad = 0;
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = col16<G>(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row16<G>(m0, i, v);
        if (row < N && col < T) {
          const float x = vf[i][j][v];
          const float z = acc[i][j][0][v];
          const bool pos = x > 0.f;
          const float iz = __builtin_amdgcn_rcpf(z);
          const float q = pos ? x * iz : 0.f;
          const float qc = pos ? (x - z) * iz : -1.f;
          const float qb = pos ? q * iz : 0.f;
          bad |= (pos && !(z > 0.f)) ? 1 : 0;
          if (MAXONLY) {
            if (SIDE == 0) {
              mx[0][j] = fmaxf(mx[0][j], q);
              mx[1][j] = fmaxf(mx[1][j], fabsf(qc));
              mx[2][j] = fmaxf(mx[2][j], qb);
            } else {
              atomicMax(a.qmax[0] + row, __float_as_uint(q));
              atomicMax(a.qmax[1] + row, __float_as_uint(fabsf(qc)));
              atomicMax(a.qmax[2] + row, __float_as_uint(qb));
            }
          } else {
            const int64_t si = SIDE == 0 ? col : row;
            const float s0 = a.qs[0] ? a.qs[0][si] : 1.f;
            const float s1 = a.qs[1] ? a.qs[1][si] : 1.f;
            const float s2 = a.qs[2] ? a.qs[2][si] : 1.f;
            reinterpret_cast<TE*>(a.Q)[row * T + col] = (TE)(q * s0);
            reinterpret_cast<TE*>(a.Qc)[row * T + col] = (TE)(qc * s1);
            reinterpret_cast<TE*>(a.Qb)[row * T + col] = (TE)(qb * s2);
            if (SIDE == 0) cp[0][j] += (double)x;
            else rp[0][i][v] += (double)x;
          }
        }
      }
    }
  if (a.check && bad) atomicOr(a.check, CHK_DOMAIN);
  if (MAXONLY) {
    if (SIDE == 0) {
      const int lane = threadIdx.x & 63;
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
        const int64_t col = col16<G>(n0, j);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const float m = fmaxf(mx[k][j], __shfl_xor(mx[k][j], 32));
          if (lane < 32 && col < T) atomicMax(a.qmax[k] + col, __float_as_uint(m));
        }
      }
    }
    return;
  }
  double* red = reinterpret_cast<double*>(lds);
  if (SIDE == 0) {
    reduce_cols<G, 1>(cp, red, [&](int c, const double (&s)[1]) {
      if (n0 + c < T) a.vpart[(int64_t)blockIdx.y * T + n0 + c] = s[0];
    });
  } else {
    reduce_rows<G, 1>(rp, red, [&](int r, const double (&s)[1]) {
      if (m0 + r < N) a.vpart[(int64_t)blockIdx.x * N + m0 + r] = s[0];
    });
  }
}

// ---------------------------------------------------------------------------
// Gradient / Hessian numerators (split over the contraction, scales folded out).
// ---------------------------------------------------------------------------
// Scale folds of the three outputs (u, u_c, y): per output row and per output
// column (nullptr = 1).
struct Fold {
  const float* r[3];
  const float* c[3];
};

template <typename TE>
__global__ __launch_bounds__(G16H::NT) void k_gh16_H(Op16 W, Op16 Q, Op16 Qc, Op16 Qb, int64_t N, int64_t T,
                                                     int64_t R, int64_t kchunk, float* pu, float* puc, float* py,
                                                     Fold f) {
  using G = G16H;
  typedef PolGH_H<G, TE> P;
  __shared__ __align__(16) TE lds[P::LDS_ELEMS];
  const int64_t m0 = (int64_t)blockIdx.y * G::BM, n0 = (int64_t)blockIdx.x * G::BN;
  const int64_t sp = blockIdx.z;
  const int64_t k0 = sp * kchunk, k1 = std::min<int64_t>(N, k0 + kchunk);
  f32x16 acc[G::FM][G::FN][3];
  zero16<G, 3>(acc);
  P pol;
  pol.W = W;
  pol.Q[0] = Qc;     // tile B0: Q - 1
  pol.Q[1] = Q;      // tile B1: Q
  pol.Q[2] = Qb;     // tile B2: Q-bar
  pol.m0 = m0;
  pol.n0 = n0;
  run16<G, P, TE>(pol, acc, k0, k1, lds);
  float* out[3] = {pu, puc, py};
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = col16<G>(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row16<G>(m0, i, v);
        if (row < R && col < T) {
          const int64_t e = (sp * R + row) * T + col;
          const int src[3] = {1, 0, 2};          // u = W^t Q, u_c = W^t (Q - 1), y
#pragma unroll
          for (int c = 0; c < 3; ++c)
            out[c][e] = acc[i][j][src[c]][v] * (f.r[c] ? f.r[c][row] : 1.f) * (f.c[c] ? f.c[c][col] : 1.f);
        }
      }
    }
}

template <typename TE>
__global__ __launch_bounds__(G16W::NT) void k_gh16_W(Op16 Q, Op16 Qc, Op16 Qb, Op16 H, int64_t N, int64_t T,
                                                     int64_t R, int64_t kchunk, float* pu, float* puc, float* py,
                                                     Fold f) {
  using G = G16W;
  typedef PolGH_W<G, TE> P;
  __shared__ __align__(16) TE lds[P::LDS_ELEMS];
  const int64_t m0 = (int64_t)blockIdx.y * G::BM, n0 = (int64_t)blockIdx.x * G::BN;
  const int64_t sp = blockIdx.z;
  const int64_t k0 = sp * kchunk, k1 = std::min<int64_t>(T, k0 + kchunk);
  f32x16 acc[G::FM][G::FN][3];
  zero16<G, 3>(acc);
  P pol;
  pol.Q[0] = Q;      // tile A0: Q
  pol.Q[1] = Qc;     // tile A1: Q - 1
  pol.Q[2] = Qb;     // tile A2: Q-bar
  pol.H = H;
  pol.m0 = m0;
  pol.n0 = n0;
  run16<G, P, TE>(pol, acc, k0, k1, lds);
  float* out[3] = {pu, puc, py};
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = col16<G>(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row16<G>(m0, i, v);
        if (row < N && col < R) {
          const int64_t e = (sp * N + row) * R + col;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            out[c][e] = acc[i][j][c][v] * (f.r[c] ? f.r[c][row] : 1.f) * (f.c[c] ? f.c[c][col] : 1.f);
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Candidate costs (as the fp32 kernels, with 16-bit reconstruction products).
// ---------------------------------------------------------------------------
template <typename TE>
__global__ __launch_bounds__(G16CH::NT) void k_cost16_H(const float* V, Op16 W, Op16 Hn, Op16 Hd, int64_t N,
                                                        int64_t T, int64_t R, double* part, int* fpart) {
  using G = G16CH;
  typedef PolZ<G, TE, 1, 2> P;
  __shared__ __align__(16) TE lds[P::LDS_ELEMS > 12 * G::BN * 4 ? P::LDS_ELEMS : 12 * G::BN * 4];
  __shared__ int fl_s[G::BN];
  const int64_t m0 = (int64_t)blockIdx.y * G::BM, n0 = (int64_t)blockIdx.x * G::BN;
  const int tid = threadIdx.x;
  for (int c = tid; c < G::BN; c += G::NT) fl_s[c] = 0;
  float vf[G::FM][G::FN][16];
#pragma unroll
  for (int j = 0; j < G::FN; ++j) {
    const int64_t col = std::min<int64_t>(col16<G>(n0, j), T - 1);
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) vf[i][j][v] = V[std::min<int64_t>(row16<G>(m0, i, v), N - 1) * T + col];
  }
  f32x16 acc[G::FM][G::FN][2];
  zero16<G, 2>(acc);
  P pol;
  pol.A[0] = W;
  pol.B[0] = Hn;
  pol.B[1] = Hd;
  pol.m0 = m0;
  pol.n0 = n0;
  run16<G, P, TE>(pol, acc, 0, R, lds);
  const int64_t base = (int64_t)blockIdx.y * T, stride = (int64_t)gridDim.y * T;
  cost_cols<G>(vf, acc, m0, n0, N, T, reinterpret_cast<double*>(lds), fl_s, part, fpart, base, stride);
}

template <typename TE>
__global__ __launch_bounds__(G16CW::NT) void k_cost16_W(const float* V, Op16 Wn, Op16 Wd, Op16 H, int64_t N,
                                                        int64_t T, int64_t R, double* part, int* fpart) {
  using G = G16CW;
  typedef PolZ<G, TE, 2, 1> P;
  __shared__ __align__(16) TE lds[P::LDS_ELEMS > 12 * G::BM * 4 ? P::LDS_ELEMS : 12 * G::BM * 4];
  __shared__ int fl_s[G::BM];
  const int64_t m0 = (int64_t)blockIdx.y * G::BM, n0 = (int64_t)blockIdx.x * G::BN;
  const int tid = threadIdx.x;
  for (int r = tid; r < G::BM; r += G::NT) fl_s[r] = 0;
  float vf[G::FM][G::FN][16];
#pragma unroll
  for (int j = 0; j < G::FN; ++j) {
    const int64_t col = std::min<int64_t>(col16<G>(n0, j), T - 1);
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) vf[i][j][v] = V[std::min<int64_t>(row16<G>(m0, i, v), N - 1) * T + col];
  }
  f32x16 acc[G::FM][G::FN][2];
  zero16<G, 2>(acc);
  P pol;
  pol.A[0] = Wn;
  pol.A[1] = Wd;
  pol.B[0] = H;
  pol.m0 = m0;
  pol.n0 = n0;
  run16<G, P, TE>(pol, acc, 0, R, lds);
  const int64_t base = (int64_t)blockIdx.x * N, stride = (int64_t)gridDim.x * N;
  cost_rows<G>(vf, acc, m0, n0, N, T, reinterpret_cast<double*>(lds), fl_s, part, fpart, base, stride);
}

// ---------------------------------------------------------------------------
// Scales for fp16.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_zero_u32(unsigned* p, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) p[e] = 0u;
}

// max over n of W[n][r] (column maxima) into bits[r]
__global__ __launch_bounds__(256) void k_colmax_W(const float* W, int64_t N, int64_t R, int64_t rows, unsigned* bits) {
  __shared__ float red[4][64];
  const int tid = threadIdx.x, cl = tid & 63, rg = tid >> 6;
  const int64_t r = (int64_t)blockIdx.x * 64 + cl, p = blockIdx.y;
  const int64_t n1 = std::min<int64_t>(N, (p + 1) * rows);
  float m = 0.f;
  if (r < R)
    for (int64_t n = p * rows + rg; n < n1; n += 4) m = fmaxf(m, W[n * R + r]);
  red[rg][cl] = m;
  __syncthreads();
  if (rg == 0 && r < R)
    atomicMax(bits + r, __float_as_uint(fmaxf(fmaxf(red[0][cl], red[1][cl]), fmaxf(red[2][cl], red[3][cl]))));
}

// max over t of H[r][t] (row maxima) into bits[r]
__global__ __launch_bounds__(256) void k_rowmax_H(const float* H, int64_t T, int64_t R, int64_t cols, unsigned* bits) {
  const int tid = threadIdx.x;
  const int64_t p = blockIdx.x, r = blockIdx.y;
  const int64_t t1 = std::min<int64_t>(T, (p + 1) * cols);
  float m = 0.f;
  for (int64_t t = p * cols + tid; t < t1; t += 256) m = fmaxf(m, H[r * T + t]);
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) m = fmaxf(m, __shfl_xor(m, k));
  if ((tid & 63) == 0) atomicMax(bits + r, __float_as_uint(m));
}

// s = 2^(top - ceil(log2 max)), is = 1/s, is2 = 1/s^2 (max <= 0: 1).
__global__ __launch_bounds__(256) void k_scales(const unsigned* bits, int64_t n, int top, float* s, float* is,
                                                float* is2) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const float m = __uint_as_float(bits[e]);
    int ex = 0;
    if (m > 0.f && isfinite(m)) {
      frexpf(m, &ex);                 // m = f * 2^ex, f in [0.5, 1): 2^ex >= m
      ex = top - ex;
      ex = std::max(-100, std::min(100, ex));
    }
    const float sc = ldexpf(1.f, ex);
    s[e] = sc;
    if (is) is[e] = 1.f / sc;
    if (is2) is2[e] = 1.f / (sc * sc);
  }
}

static unsigned grid1(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(cdiv(n, 256), 4096)); }

// Rank scales for fp16: H step -> from the column maxima of W, W step -> from the
// row maxima of H; rs = 2^-ceil(log2 max) (max scaled to at most 1).
static void rank_scales(int side, const float* W, const float* H, int64_t N, int64_t T, int64_t R,
                        const Scratch16& S, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(grid1(R)), dim3(256), 0, s, S.bits, R);
  if (side == 0) {
    const int64_t parts = std::min<int64_t>(SUM_PARTS, cdiv(N, 64));
    hipLaunchKernelGGL(k_colmax_W, dim3((unsigned)cdiv(R, 64), (unsigned)parts), dim3(256), 0, s, W, N, R,
                       cdiv(N, parts), S.bits);
  } else {
    const int64_t parts = std::min<int64_t>(SUM_PARTS, cdiv(T, 2048));
    hipLaunchKernelGGL(k_rowmax_H, dim3((unsigned)parts, (unsigned)R), dim3(256), 0, s, H, T, R, cdiv(T, parts),
                       S.bits);
  }
  hipLaunchKernelGGL(k_scales, dim3(grid1(R)), dim3(256), 0, s, S.bits, R, 0, S.rs, S.irs, S.irs2);
}

template <typename TE>
static hipError_t ratio_gh16(int side, const float* V, const float* W, const float* H, int64_t N, int64_t T,
                             int64_t R, const Scratch16& S, bool scaled, int splits, int64_t kchunk, float* pu,
                             float* puc, float* py, double* vpart, int* check, const SumJob& fin,
                             hipStream_t s) {
  TE* Qp = reinterpret_cast<TE*>(S.q16);
  TE* Qc = Qp + N * T;
  TE* Qb = reinterpret_cast<TE*>(S.qb16);
  const int64_t L = side == 0 ? T : N;     // index range of the Q scales
  const float* rs = nullptr;
  const float* irs = nullptr;
  const float* irs2 = nullptr;
  const float* qs[3] = {nullptr, nullptr, nullptr};
  const float* iqs[3] = {nullptr, nullptr, nullptr};
  if (scaled) {
    rank_scales(side, W, H, N, T, R, S, s);
    rs = S.rs; irs = S.irs; irs2 = S.irs2;
  }
  // Z-type product: the rank scales cancel between W and H
  const Op16 w = make_op16<float>(W, R, N, nullptr, side == 0 ? rs : irs);
  const Op16 h = make_op16<float>(H, T, T, nullptr, side == 0 ? irs : rs);
  Ratio16Args ra;
  ra.V = V; ra.W = w; ra.H = h; ra.N = N; ra.T = T; ra.R = R;
  ra.Q = Qp; ra.Qc = Qc; ra.Qb = Qb; ra.vpart = vpart; ra.check = check; ra.fin = fin;
  for (int k = 0; k < 3; ++k) { ra.qs[k] = nullptr; ra.qmax[k] = nullptr; }
  dim3 rgrid((unsigned)cdiv(T, G16R::BN), (unsigned)cdiv(N, G16R::BM));
  if (scaled) {
    unsigned* qbits = S.bits + R;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid1(3 * L)), dim3(256), 0, s, qbits, 3 * L);
    for (int k = 0; k < 3; ++k) ra.qmax[k] = qbits + k * L;
    // the scales only need the maxima to a few bits: unsplit product
    prof_begin("qmax16", s);
    if (side == 0) hipLaunchKernelGGL((k_ratio16<TE, 0, true, 0>), rgrid, dim3(G16R::NT), 0, s, ra);
    else hipLaunchKernelGGL((k_ratio16<TE, 1, true, 0>), rgrid, dim3(G16R::NT), 0, s, ra);
    prof_end("qmax16", s);
    for (int k = 0; k < 3; ++k) {
      hipLaunchKernelGGL(k_scales, dim3(grid1(L)), dim3(256), 0, s, qbits + k * L, L, 13, S.qs + k * L,
                         S.iqs + k * L, (float*)nullptr);
      qs[k] = S.qs + k * L;
      iqs[k] = S.iqs + k * L;
    }
  }
  for (int k = 0; k < 3; ++k) ra.qs[k] = qs[k];
  // bf16: both factors split (its 8-bit significand in the fixed factor also
  // biases the fit); fp16: the updated factor only
  prof_begin(side == 0 ? "ratio16_H" : "ratio16_W", s);
  if (scaled) {
    if (side == 0) hipLaunchKernelGGL((k_ratio16<TE, 0, false, 1>), rgrid, dim3(G16R::NT), 0, s, ra);
    else hipLaunchKernelGGL((k_ratio16<TE, 1, false, 2>), rgrid, dim3(G16R::NT), 0, s, ra);
  } else {
    if (side == 0) hipLaunchKernelGGL((k_ratio16<TE, 0, false, 3>), rgrid, dim3(G16R::NT), 0, s, ra);
    else hipLaunchKernelGGL((k_ratio16<TE, 1, false, 3>), rgrid, dim3(G16R::NT), 0, s, ra);
  }
  prof_end(side == 0 ? "ratio16_H" : "ratio16_W", s);
  Fold f;
  if (side == 0) {          // rows r carry the W^t scale, columns t the Q scales
    const float* rr[3] = {irs, irs, irs2};
    for (int k = 0; k < 3; ++k) { f.r[k] = rr[k]; f.c[k] = iqs[k]; }
    const Op16 wt = make_op16<float>(W, R, R, nullptr, nullptr, rs);
    const Op16 q = make_op16<TE>(Qp, T, T), qc = make_op16<TE>(Qc, T, T), qb = make_op16<TE>(Qb, T, T);
    dim3 grid((unsigned)cdiv(T, G16H::BN), (unsigned)cdiv(R, G16H::BM), (unsigned)splits);
    prof_begin("gh16_H", s);
    hipLaunchKernelGGL(k_gh16_H<TE>, grid, dim3(G16H::NT), 0, s, wt, q, qc, qb, N, T, R, kchunk, pu, puc, py, f);
    prof_end("gh16_H", s);
  } else {                  // rows n carry the Q scales, columns r the H^t scale
    const float* cc[3] = {irs, irs, irs2};
    for (int k = 0; k < 3; ++k) { f.r[k] = iqs[k]; f.c[k] = cc[k]; }
    const Op16 q = make_op16<TE>(Qp, T, N), qc = make_op16<TE>(Qc, T, N), qb = make_op16<TE>(Qb, T, N);
    const Op16 ht = make_op16<float>(H, T, R, nullptr, nullptr, rs);
    dim3 grid((unsigned)cdiv(R, G16W::BN), (unsigned)cdiv(N, G16W::BM), (unsigned)splits);
    prof_begin("gh16_W", s);
    hipLaunchKernelGGL(k_gh16_W<TE>, grid, dim3(G16W::NT), 0, s, q, qc, qb, ht, N, T, R, kchunk, pu, puc, py, f);
    prof_end("gh16_W", s);
  }
  return hipGetLastError();
}

template <typename TE>
static hipError_t cost16(int side, const float* V, const float* F, const float* Xmu, const float* Xn, int64_t N,
                         int64_t T, int64_t R, const Scratch16& S, bool scaled, double* part, int* fpart,
                         hipStream_t s) {
  const float* rs = nullptr;
  const float* irs = nullptr;
  if (scaled) {
    if (side == 0) rank_scales(0, F, nullptr, N, T, R, S, s);
    else rank_scales(1, nullptr, F, N, T, R, S, s);
    rs = S.rs;
    irs = S.irs;
  }
  if (side == 0) {
    const Op16 w = make_op16<float>(F, R, N, nullptr, rs);
    const Op16 hn = make_op16<float>(Xn, T, T, nullptr, irs);
    const Op16 hd = make_op16<float>(Xmu, T, T, Xn, irs);
    dim3 grid((unsigned)cdiv(T, G16CH::BN), (unsigned)cdiv(N, G16CH::BM));
    prof_begin("cost16_H", s);
    hipLaunchKernelGGL(k_cost16_H<TE>, grid, dim3(G16CH::NT), 0, s, V, w, hn, hd, N, T, R, part, fpart);
    prof_end("cost16_H", s);
  } else {
    const Op16 wn = make_op16<float>(Xn, R, N, nullptr, irs);
    const Op16 wd = make_op16<float>(Xmu, R, N, Xn, irs);
    const Op16 h = make_op16<float>(F, T, T, nullptr, rs);
    dim3 grid((unsigned)cdiv(T, G16CW::BN), (unsigned)cdiv(N, G16CW::BM));
    prof_begin("cost16_W", s);
    hipLaunchKernelGGL(k_cost16_W<TE>, grid, dim3(G16CW::NT), 0, s, V, wn, wd, h, N, T, R, part, fpart);
    prof_end("cost16_W", s);
  }
  return hipGetLastError();
}

hipError_t launch_ratio_gh16(int gemm, int side, const float* V, const float* W, const float* H, int64_t N,
                             int64_t T, int64_t R, const Scratch16& S, int splits, int64_t kchunk, float* pu,
                             float* puc, float* py, double* vpart, int* check, const SumJob& fin,
                             hipStream_t s) {
  if (gemm == 1)
    return ratio_gh16<__bf16>(side, V, W, H, N, T, R, S, false, splits, kchunk, pu, puc, py, vpart, check, fin, s);
  return ratio_gh16<_Float16>(side, V, W, H, N, T, R, S, true, splits, kchunk, pu, puc, py, vpart, check, fin, s);
}

hipError_t launch_cost16(int gemm, int side, const float* V, const float* F, const float* Xmu, const float* Xn,
                         int64_t N, int64_t T, int64_t R, const Scratch16& S, double* part, int* fpart,
                         hipStream_t s) {
  if (gemm == 1) return cost16<__bf16>(side, V, F, Xmu, Xn, N, T, R, S, false, part, fpart, s);
  return cost16<_Float16>(side, V, F, Xmu, Xn, N, T, R, S, true, part, fpart, s);
}

}  // namespace dna
