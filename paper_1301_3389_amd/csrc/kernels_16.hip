// kernels_16.hip -- the precision form: the products of a DNA half-step (Z, the
// gradient/Hessian sums, the two candidate reconstructions) with bf16 or fp16
// MFMA operands and fp32 accumulation.  Candidates, costs (float64 sums) and
// selection are the fp32 path's.
//
// Each half-step first converts its fp32 factors into zero-padded, K-contiguous
// 16-bit operands (k_conv16), so that every product runs the bounds-free engine
// of core16.hpp.  The Z pass writes Q, Q - 1 and Q-bar in 16 bits, laid out for
// the gradient products (contraction index contiguous); it and the cost pass
// compute the W step's tiles transposed, (t, n), so that both orientations
// keep per-column partials.
//
// The factor being updated (H in the H step, W in the W step) enters Z as a
// two-term split hi + lo (BF16: both factors): with a single rounding the
// gradient would be taken a relative 16-bit rounding away from the point the
// step is applied to, an error that does not shrink as the fit converges.
//
// fp16 needs power-of-two scales to stay in range:
//   * rank scales: W columns scaled to max 1 (H rows by the inverse) where they
//     cancel in the Z-type products; in the gradient products the scale of the
//     fixed factor is folded out of the result;
//   * Q, Q - 1, Q-bar scaled per column (H step) / per row (W step) so that each
//     column's (row's) maximum lies in [2^12, 2^13), from a max pass over the
//     same Z tiles, and folded out of the gradient sums.
// bf16 keeps fp32's exponent range and uses no scales.
#include <math.h>

#include <algorithm>

#include "core16.hpp"
#include "epilogue.hpp"
#include "kernels.hpp"
#include "kernels_16.hpp"

namespace dna {

using G128 = G16<128, 128>;
using GGH = G128;   // tiles of the gradient products

// ---------------------------------------------------------------------------
// Workspace.
// ---------------------------------------------------------------------------
struct Off16 {
  size_t fa_hi, fa_lo, fb_hi, fb_lo, g0, g1, x0, x1, q3, bits, rs, irs, irs2, qs, iqs, total;
};

static Off16 offsets16(int64_t N, int64_t T, int64_t R) {
  const Dims16 d = dims16(N, T, R);
  const size_t mx = (size_t)std::max(d.Np, d.Tp);
  Off16 o;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t p = off; off = (off + bytes + 255) & ~size_t(255); return p; };
  o.fa_hi = take((size_t)d.Np * d.Rk * 2);
  o.fa_lo = take((size_t)d.Np * d.Rk * 2);
  o.fb_hi = take((size_t)d.Tp * d.Rk * 2);
  o.fb_lo = take((size_t)d.Tp * d.Rk * 2);
  o.g0 = take((size_t)d.Rm * mx * 2);
  o.g1 = take((size_t)d.Rm * mx * 2);
  o.x0 = take(mx * d.Rk * 2);
  o.x1 = take(mx * d.Rk * 2);
  o.q3 = take((size_t)3 * d.Np * d.Tp * 2);
  o.bits = take(((size_t)d.Rm + 3 * mx) * 4);
  o.rs = take((size_t)d.Rm * 4);
  o.irs = take((size_t)d.Rm * 4);
  o.irs2 = take((size_t)d.Rm * 4);
  o.qs = take(3 * mx * 4);
  o.iqs = take(3 * mx * 4);
  o.total = off;
  return o;
}

size_t scratch16_bytes(int64_t N, int64_t T, int64_t R) { return offsets16(N, T, R).total; }

Scratch16 scratch16_carve(void* base, int64_t N, int64_t T, int64_t R) {
  const Off16 o = offsets16(N, T, R);
  char* b = static_cast<char*>(base);
  Scratch16 S;
  S.fa_hi = b + o.fa_hi; S.fa_lo = b + o.fa_lo; S.fb_hi = b + o.fb_hi; S.fb_lo = b + o.fb_lo;
  S.g0 = b + o.g0; S.g1 = b + o.g1; S.x0 = b + o.x0; S.x1 = b + o.x1; S.q3 = b + o.q3;
  S.bits = reinterpret_cast<unsigned*>(b + o.bits);
  S.rs = reinterpret_cast<float*>(b + o.rs);
  S.irs = reinterpret_cast<float*>(b + o.irs);
  S.irs2 = reinterpret_cast<float*>(b + o.irs2);
  S.qs = reinterpret_cast<float*>(b + o.qs);
  S.iqs = reinterpret_cast<float*>(b + o.iqs);
  return S;
}

// ---------------------------------------------------------------------------
// Conversion: dst (Dr x Dc, leading dimension ldd, 16-bit) from an fp32 source
// (Sr x Sc, leading dimension lds), transposed or not; zero outside the source.
//   x = (src - src2) * sr[source row] * sc[source column]   (nullptr: 0 / 1)
//   out0 = round16(x);  out1 = round16(x - out0) (MODE1 = 1) or round16(x * x) (2)
// 64 x 64 tiles through LDS so that both sides are read / written along rows.
// ---------------------------------------------------------------------------
struct ConvArgs {
  const float* src; const float* src2;
  int64_t Sr, Sc, lds;
  const float* sr; const float* sc;
  void* out0; void* out1;
  int mode1;
  int64_t Dr, Dc, ldd;
};

template <typename TE, bool TR>
__global__ __launch_bounds__(256) void k_conv16(ConvArgs a) {
  __shared__ float t[64][65];
  const int tid = threadIdx.x;
  const int64_t d0 = (int64_t)blockIdx.y * 64, e0 = (int64_t)blockIdx.x * 64;   // dest rows / cols
  // source tile: rows / cols of the source covered by this dest tile
  const int64_t s0 = TR ? e0 : d0, c0 = TR ? d0 : e0;
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int rr = idx / 64, cc = idx % 64;
    const int64_t r = s0 + rr, c = c0 + cc;
    float x = 0.f;
    if (r < a.Sr && c < a.Sc) {
      x = a.src[r * a.lds + c];
      if (a.src2) x -= a.src2[r * a.lds + c];
      if (a.sr) x *= a.sr[r];
      if (a.sc) x *= a.sc[c];
    }
    t[rr][cc] = x;
  }
  __syncthreads();
  TE* o0 = reinterpret_cast<TE*>(a.out0);
  TE* o1 = reinterpret_cast<TE*>(a.out1);
  for (int idx = tid; idx < 64 * 64; idx += 256) {
    const int dr = idx / 64, dc = idx % 64;
    const int64_t r = d0 + dr, c = e0 + dc;
    if (r >= a.Dr || c >= a.Dc) continue;
    const float x = TR ? t[dc][dr] : t[dr][dc];
    const TE h = (TE)x;
    o0[r * a.ldd + c] = h;
    if (o1) o1[r * a.ldd + c] = (TE)(a.mode1 == 1 ? x - (float)h : x * x);
  }
}

template <typename TE>
static void conv16(const ConvArgs& a, bool tr, hipStream_t s) {
  dim3 grid((unsigned)cdiv(a.Dc, 64), (unsigned)cdiv(a.Dr, 64));
  if (tr) hipLaunchKernelGGL((k_conv16<TE, true>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_conv16<TE, false>), grid, dim3(256), 0, s, a);
}

// ---------------------------------------------------------------------------
// Z pass: Z = W H from the converted operands; epilogue Q = v/z, Q - 1 =
// (v - z)/z, Q-bar = q/z (zero where v = 0, except Q - 1 = -1; zero in the
// padding), optional per-column / per-row scales, 16-bit output through LDS
// (SIDE 0: transposed, [t][n]; SIDE 1: [n][t], both with leading dimension of
// the padded extent), plus V column (SIDE 0) / row (SIDE 1) sums.
// MAXONLY: only the maxima of |Q|, |Q - 1|, Q-bar per column / row (fp16 scales).
// ---------------------------------------------------------------------------
struct Ratio16Args {
  const float* V;
  Mat16 A[2], B[2];
  int64_t N, T, Rk, Np, Tp;
  void* q3;                         // 3 x Np x Tp, 16-bit
  double* vpart;
  const float* qs[3];               // output scales of Q, Q - 1, Q-bar (nullptr = 1)
  unsigned* qmax[3];                // max pass: float bits of max |.| per column / row
  int* check;
  SumJob fin;                       // folded second level of the factor sum (not in the max pass)
};

template <int SPLIT> struct ZProds;
template <> struct ZProds<0> { typedef Prods<1, 1, 1, 1, 0, 0, 0> P; };
template <> struct ZProds<1> { typedef Prods<1, 2, 2, 1, 0, 1, 0, 0, 0, 0> P; };          // B split
template <> struct ZProds<3> { typedef Prods<2, 2, 3, 1, 1, 0, 0, 0, 1, 0, 0, 0, 0> P; }; // both

constexpr int OUT_PITCH = 128 + 8;   // LDS pitch of the 128 x 128 output staging tiles
constexpr int OUT_TILE = 128 * OUT_PITCH;                  // elements of one staging tile
constexpr int RATIO_OUT_BYTES = 2 * OUT_TILE * 2;          // Q and Q - 1 staged together, Q-bar after

// The Z pass runs two workgroups per CU (a 2-stage ring, 64 KiB of LDS, at most
// 256 registers per lane): one workgroup's epilogue and V loads overlap the
// other's products.
// The gradient products likewise: a 2-stage ring (80 KiB) and two workgroups
// per CU (GH16_WG_PER_CU), all accumulators in registers.
// The cost passes keep per-column partials of their tiles (a light epilogue)
// and fit two waves per SIMD with a 2-stage ring: one workgroup's epilogue then
// overlaps another's products.  Both read V after the products.
constexpr int RATIO_STAGES = 2, GH_STAGES = 2, COST_STAGES = 2;

template <typename TE, int SPLIT>
using ZEng = Gemm16<G128, TE, typename ZProds<SPLIT>::P, RATIO_STAGES>;

// V of this lane's accumulator positions of the tile at (m0, n0), after the
// products: a buffer descriptor from the tile's first entry to the end of V
// (rows past N read as zero; columns past T, masked by the callers, read the
// next row), a per-lane offset and a uniform one per (i, j, v).
template <class G>
__device__ __forceinline__ void load_v16(const float* V, int64_t N, int64_t T, int64_t m0, int64_t n0,
                                         float (&vf)[G::FM][G::FN][16]) {
  // the wave index made uniform, so that the per-slot offsets are scalars
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % G::WGM, wn = wave / G::WGM;
  const float* base = V + m0 * T + n0;
  const int64_t bytes = (N * T - (m0 * T + n0)) * 4;
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)std::min<int64_t>(bytes, 0x7fffffff), 0x00020000);
  const int voff = (int)(((lane >> 5) * 4 * T + (lane & 31)) * 4);
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t ru = wm * G::WM + i * 32 + (v >> 2) * 8 + (v & 3), cu = wn * G::WN + j * 32;
        vf[i][j][v] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, (int)((ru * T + cu) * 4), 0));
      }
}

// The same for a transposed tile: tile rows are columns t of V (from m0), tile
// columns are rows n (from n0), v(n, t) = V[n * T + t].  Rows n past N read as
// zero; entries past T read the next row n and are masked by the callers.  The
// four accumulator slots 4g .. 4g + 3 of a lane are four consecutive t of one
// row n: one 16-byte load where the rows of V are 16-byte aligned (V itself
// and T % 4 == 0).
template <class G>
__device__ __forceinline__ void load_v16t(const float* V, int64_t N, int64_t T, int64_t m0, int64_t n0,
                                          float (&vf)[G::FM][G::FN][16]) {
  // the wave index made uniform, so that the per-slot offsets are scalars
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave % G::WGM, wn = wave / G::WGM;
  const float* base = V + n0 * T + m0;
  const int64_t bytes = (N * T - (n0 * T + m0)) * 4;
  const __amdgpu_buffer_rsrc_t r =
      __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)std::min<int64_t>(bytes, 0x7fffffff), 0x00020000);
  const int voff = (int)(((lane & 31) * T + (lane >> 5) * 4) * 4);
  if ((T & 3) == 0 && (reinterpret_cast<uintptr_t>(V) & 15) == 0) {
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int j = 0; j < G::FN; ++j)
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
          const int64_t ru = wm * G::WM + i * 32 + gq * 8, cu = wn * G::WN + j * 32;
          const u32x4 x = __builtin_amdgcn_raw_buffer_load_b128(r, voff, (int)((cu * T + ru) * 4), 0);
#pragma unroll
          for (int u = 0; u < 4; ++u) {   // element to a scalar first: a bit cast of x[u] itself reads x[0]
            const unsigned e = x[u];
            vf[i][j][4 * gq + u] = __uint_as_float(e);
          }
        }
  } else {
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int j = 0; j < G::FN; ++j)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t ru = wm * G::WM + i * 32 + (v >> 2) * 8 + (v & 3), cu = wn * G::WN + j * 32;
          vf[i][j][v] =
              __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, (int)((cu * T + ru) * 4), 0));
        }
  }
}

// The Z pass.  H step (SIDE 0): tile (n, t) = W H, A = W, B = H^t.  W step
// (SIDE 1): the transposed tile (t, n) = H^t W^t, A = H^t, B = W, so that in
// both the per-column quantities (V sums, Q scales and maxima) belong to the
// index the gradient products do not contract over, and the outputs (Q^t,
// (Q - 1)^t, Q-bar^t for the H step; Q, Q - 1, Q-bar for the W step) are the
// tile transposed.  Grid x walks t in both (consecutive tiles read adjacent
// blocks of the same rows of V).
template <typename TE, int SIDE, bool MAXONLY, int SPLIT>
__global__ __launch_bounds__(256, 2) void k_ratio16(Ratio16Args a) {
  using G = G128;
  typedef typename ZProds<SPLIT>::P PR;
  typedef ZEng<TE, SPLIT> E;
  // launched with at least RATIO_OUT_BYTES of dynamic LDS (the staging tiles)
  extern __shared__ __align__(16) char lds_dyn[];
  char* lds = lds_dyn;
  const Tile3 tl = xcd_tile();
  // tile row block rt (rows from m0), column block (columns from n0)
  const int64_t rt = SIDE == 0 ? tl.y : tl.x, ct = SIDE == 0 ? tl.x : tl.y;
  const int64_t m0 = rt * G::BM, n0 = ct * G::BN;
  const int64_t N = a.N, T = a.T;
  const int64_t ME = SIDE == 0 ? N : T, CE = SIDE == 0 ? T : N;   // extents of tile rows / columns
  if (!MAXONLY) sum_job(a.fin);
  f32x16 acc[G::FM][G::FN][1];
  zero16<G, 1>(acc);
  {
    Mat16 A[PR::NA], B[PR::NB];
#pragma unroll
    for (int x = 0; x < PR::NA; ++x) A[x] = a.A[x];
#pragma unroll
    for (int y = 0; y < PR::NB; ++y) B[y] = a.B[y];
    E::run(A, B, m0, n0, 0, a.Rk, lds, acc);
  }
  float vf[G::FM][G::FN][16];
  if (SIDE == 0) load_v16<G>(a.V, N, T, m0, n0, vf);
  else load_v16t<G>(a.V, N, T, m0, n0, vf);
  const int lane = threadIdx.x & 63;
  if (MAXONLY) {   // per-column maxima of Q, |Q - 1|, Q-bar
    float mx[3][G::FN] = {};
    int bad = 0;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
        const int64_t col = col16<G>(n0, j);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = row16<G>(m0, i, v);
          if (row < ME && col < CE) {
            const float x = vf[i][j][v], z = acc[i][j][0][v];
            const bool pos = x > 0.f;
            const float iz = __builtin_amdgcn_rcpf(z);
            const float q = pos ? x * iz : 0.f;
            const float qc = pos ? (x - z) * iz : -1.f;
            const float qb = pos ? q * iz : 0.f;
            bad |= (pos && !(z > 0.f)) ? 1 : 0;
            mx[0][j] = fmaxf(mx[0][j], q);
            mx[1][j] = fmaxf(mx[1][j], fabsf(qc));
            mx[2][j] = fmaxf(mx[2][j], qb);
          }
        }
      }
    if (a.check && bad) atomicOr(a.check, CHK_DOMAIN);
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = col16<G>(n0, j);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float m = fmaxf(mx[k][j], __shfl_xor(mx[k][j], 32));
        if (lane < 32 && col < CE) atomicMax(a.qmax[k] + col, __float_as_uint(m));
      }
    }
    return;
  }
  // V sums of this tile's columns (column sums of V in the H step, row sums in
  // the W step): vpart[rt * CE + column]
  {
    double* red = reinterpret_cast<double*>(lds);
    double cp[1][G::FN];
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      cp[0][j] = 0.0;
      const int64_t col = col16<G>(n0, j);
#pragma unroll
      for (int i = 0; i < G::FM; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v)
          if (row16<G>(m0, i, v) < ME && col < CE) cp[0][j] += (double)vf[i][j][v];
    }
    reduce_cols<G, 1>(cp, red, [&](int c, const double (&s)[1]) {
      if (n0 + c < CE) a.vpart[rt * CE + n0 + c] = s[0];
    });
  }
  // The outputs through LDS staging tiles: Q and Q - 1 in a first round, Q-bar
  // (recomputed from the same z and v) in a second.  The staging tiles are the
  // tile transposed ([column][row]); the four consecutive rows a lane holds per
  // group of four accumulator slots are adjacent: one 8-byte store.
  TE* st = reinterpret_cast<TE*>(lds);
  int bad = 0;
  const int64_t ld = SIDE == 0 ? a.Np : a.Tp;
#pragma unroll
  for (int round = 0; round < 2; ++round) {
    const int nout = round == 0 ? 2 : 1;
    __syncthreads();                              // the staging tiles are free
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
        const int64_t col = col16<G>(n0, j);
        const int cl = (int)(col - n0);
        float sc[2];
#pragma unroll
        for (int o = 0; o < 2; ++o) {
          const int k = round == 0 ? o : 2;
          sc[o] = (a.qs[k] && col < CE) ? a.qs[k][col] : 1.f;
        }
#pragma unroll
        for (int gq = 0; gq < 4; ++gq) {
          TE out[2][4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int v = 4 * gq + u;
            const int64_t row = row16<G>(m0, i, v);
            float o0 = 0.f, o1 = 0.f;
            if (row < ME && col < CE) {
              const float x = vf[i][j][v], z = acc[i][j][0][v];
              const bool pos = x > 0.f;
              const float iz = __builtin_amdgcn_rcpf(z);
              const float q = pos ? x * iz : 0.f;
              if (round == 0) {
                o0 = q * sc[0];
                o1 = (pos ? (x - z) * iz : -1.f) * sc[1];
                bad |= (pos && !(z > 0.f)) ? 1 : 0;
              } else {
                o0 = (pos ? q * iz : 0.f) * sc[0];
              }
            }
            out[0][u] = (TE)o0;
            out[1][u] = (TE)o1;
          }
          const int rl0 = (int)(row16<G>(m0, i, 4 * gq) - m0);    // rows rl0 .. rl0 + 3
#pragma unroll
          for (int o = 0; o < 2; ++o) {
            if (o >= nout) continue;
            TE* t = st + o * OUT_TILE;
            typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
            u32x2 w;
            w[0] = (unsigned)__builtin_bit_cast(uint16_t, out[o][0]) |
                   ((unsigned)__builtin_bit_cast(uint16_t, out[o][1]) << 16);
            w[1] = (unsigned)__builtin_bit_cast(uint16_t, out[o][2]) |
                   ((unsigned)__builtin_bit_cast(uint16_t, out[o][3]) << 16);
            *reinterpret_cast<u32x2*>(t + cl * OUT_PITCH + rl0) = w;
          }
        }
      }
    __syncthreads();
    // copy out: nout tiles of 128 output rows (tile columns) of 128 elements,
    // 16-byte chunks
    const uint16_t* src = reinterpret_cast<const uint16_t*>(st);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int f = threadIdx.x + k * 256;
      const int o = f / 2048, rr = (f % 2048) / 16, ch = (f % 16) * 8;
      if (o >= nout) continue;
      const int ko = round == 0 ? o : 2;
      uint16_t* dst = reinterpret_cast<uint16_t*>(a.q3) + (int64_t)ko * a.Np * a.Tp;
      *reinterpret_cast<u32x4*>(dst + (n0 + rr) * ld + m0 + ch) =
          *reinterpret_cast<const u32x4*>(src + o * OUT_TILE + rr * OUT_PITCH + ch);
    }
  }
  if (a.check && bad) atomicOr(a.check, CHK_DOMAIN);
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

// Operand table of a product kernel (A operands first, then B operands).
struct Ops16 {
  Mat16 m[5];
};

// H orientation: M = R (rows r), N = T (cols t), K = N.  A = {W^t, (W*W)^t},
// B = {Q^t, (Q - 1)^t, Q-bar^t}:  u = A0 B0, u_c = A0 B1, y = A1 B2.
typedef Prods<2, 3, 3, 3, 0, 0, 0, 0, 1, 1, 1, 2, 2> GHH_P;
// W orientation: M = N (rows n), N = R (cols r), K = T.  A = {Q, Q - 1, Q-bar},
// B = {H, H*H}:  u = A0 B0, u_c = A1 B0, y = A2 B1.
typedef Prods<3, 2, 3, 3, 0, 0, 0, 1, 0, 1, 2, 1, 2> GHW_P;

template <typename TE, int SIDE>
__global__ __launch_bounds__(256, GH16_WG_PER_CU) void k_gh16(Ops16 ops, int64_t M, int64_t Ncol,
                                              int64_t K32, int64_t kchunk, float* pu, float* puc, float* py,
                                              Fold f) {
  using G = GGH;
  typedef typename std::conditional<SIDE == 0, GHH_P, GHW_P>::type PR;
  typedef Gemm16<G, TE, PR, GH_STAGES> E;
  extern __shared__ __align__(16) char lds_dyn[];
  // grid x walks the tiles that share the large operand block: SIDE 0 (r-blocks,
  // t-blocks) share Q^t, SIDE 1 (r-blocks, n-blocks) share Q
  const Tile3 tl = xcd_tile();
  const int64_t m0 = (SIDE == 0 ? tl.x : tl.y) * G::BM, n0 = (SIDE == 0 ? tl.y : tl.x) * G::BN;
  const int64_t sp = tl.z;
  const int64_t k0 = sp * kchunk, k1 = std::min<int64_t>(K32, k0 + kchunk);
  f32x16 acc[G::FM][G::FN][3];
  zero16<G, 3>(acc);
  {
    Mat16 A[PR::NA], B[PR::NB];
#pragma unroll
    for (int x = 0; x < PR::NA; ++x) A[x] = ops.m[x];
#pragma unroll
    for (int y = 0; y < PR::NB; ++y) B[y] = ops.m[PR::NA + y];
    E::run(A, B, m0, n0, k0, k1, lds_dyn, acc);
  }
  float* out[3] = {pu, puc, py};
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const int64_t col = col16<G>(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = row16<G>(m0, i, v);
        if (row < M && col < Ncol) {
          const int64_t e = (sp * M + row) * Ncol + col;
#pragma unroll
          for (int c = 0; c < 3; ++c)
            out[c][e] = acc[i][j][c][v] * (f.r[c] ? f.r[c][row] : 1.f) * (f.c[c] ? f.c[c][col] : 1.f);
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Candidate costs (epilogues shared with the fp32 kernels), 16-bit products,
// A = the fixed factor, B = {X_DNA, X_MU - X_DNA}; acc 0 = z_DNA, acc 1 = dZ.
// H orientation: A = W, B = the candidates' transposes, tile (n, t), one
// partial per column t.  W orientation: the tile transposed, A = H^t, B = the
// candidates, tile (t, n), so that its partials (one per row n of W) are again
// per tile column and both orientations share the column epilogue.
// ---------------------------------------------------------------------------
typedef Prods<1, 2, 2, 2, 0, 0, 0, 0, 1, 1> CH_P;

// FP16 inside dna_iterate: bounds of the next half-step's Q, |Q - 1| and Q-bar
// maxima per tile row (H step: rows n, for the W step's Q scales; W step: rows
// t, for the H step's), taken element by element over both candidates'
// reconstructions z_DNA and z_DNA + dZ, one of which the selection keeps for
// each column of H (H step) or row of W (W step), so that the bound holds
// whatever it picks (the normalisation after it changes Z only by rounding;
// the scales are powers of two).  They
// replace the next Z pass's maxima pass.  The 32 lanes of a half-wave hold the
// same 16 rows: a halving exchange leaves one lane per row, which adds it to
// the row's maximum with an atomic.  (Per-tile stores reduced by the next Z
// pass instead of the atomics measured slower.)
template <class G>
__device__ __forceinline__ void row_qmax(const float (&vf)[G::FM][G::FN][16], const f32x16 (&acc)[G::FM][G::FN][2],
                                         int64_t m0, int64_t n0, int64_t ME, int64_t CE, unsigned* qmax,
                                         int64_t L) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int hv = 0; hv < 2; ++hv) {   // row slots 8 hv .. 8 hv + 7 (eight at a time: registers)
      float x[3][8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[0][e] = x[1][e] = x[2][e] = 0.f;
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
        const int64_t col = col16<G>(n0, j);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int v = 8 * hv + e;
          if (row16<G>(m0, i, v) < ME && col < CE) {
            // q = v/z is largest at the smaller positive z, and so is v/z^2;
            // |q - 1| is largest at one of the two (a candidate whose z is not
            // positive is left out: its z reads as infinity, q as 0)
            const float xv = vf[i][j][v];
            float z1 = acc[i][j][0][v], z2 = acc[i][j][0][v] + acc[i][j][1][v];
            // opaque copies: the cost epilogue's reciprocals of the same z are
            // not kept live until here (they would not fit the registers)
            asm volatile("" : "+v"(z1), "+v"(z2));
            const float inf = __builtin_inff();
            const float za = z1 > 0.f ? z1 : inf, zb = z2 > 0.f ? z2 : inf;
            const float zlo = fminf(za, zb), zhi = fmaxf(za, zb) < inf ? fmaxf(za, zb) : zlo;
            const float rlo = __builtin_amdgcn_rcpf(zlo), rhi = __builtin_amdgcn_rcpf(zhi);
            const float qlo = xv * rlo, qhi = xv * rhi;
            x[0][e] = fmaxf(x[0][e], qlo);
            x[1][e] = fmaxf(x[1][e], fmaxf(fabsf(qlo - 1.f), fabsf(qhi - 1.f)));
            x[2][e] = fmaxf(x[2][e], qlo * rlo);
          }
        }
      }
      // halving exchange deciding on lane bits 3, 2, 1 (lane c keeps slot
      // (c >> 1) & 7), with partners that flip the deciding bit and keep the
      // higher ones: the row mirror (c ^ 15), the half-row mirror (c ^ 7), then
      // c ^ 2; c ^ 1 and c ^ 16 complete the half-wave (DPP moves, one shuffle)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int h = 4; h >= 1; h >>= 1) {
          const bool up = (lane & (2 * h)) != 0;
#pragma unroll
          for (int e = 0; e < h; ++e) {
            const float send = up ? x[k][e] : x[k][e + h];
            const float keep = up ? x[k][e + h] : x[k][e];
            const int si = __float_as_int(send);
            const int got = h == 4 ? __builtin_amdgcn_mov_dpp(si, 0x140, 0xF, 0xF, false)    // row mirror
                          : h == 2 ? __builtin_amdgcn_mov_dpp(si, 0x141, 0xF, 0xF, false)    // half-row mirror
                                   : __builtin_amdgcn_mov_dpp(si, 0x4E, 0xF, 0xF, false);    // quad [2,3,0,1]
            x[k][e] = fmaxf(keep, __int_as_float(got));
          }
        }
        float m = fmaxf(x[k][0], __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x[k][0]), 0xB1, 0xF, 0xF,
                                                                           false)));   // quad [1,0,3,2]
        m = fmaxf(m, __shfl_xor(m, 16));
        const int64_t row = row16<G>(m0, i, 8 * hv + ((lane >> 1) & 7));
        if ((lane & 17) == 0 && row < ME && m > 0.f) atomicMax(qmax + k * L + row, __float_as_uint(m));
      }
    }
}

template <typename TE, int SIDE, bool S0, bool QM>
__global__ __launch_bounds__(256, 2) void k_cost16(const float* V, Ops16 ops, int64_t N, int64_t T, int64_t Rk,
                                                   double* part, int* fpart, unsigned* qmax) {
  using G = G128;
  typedef CH_P PR;
  typedef Gemm16<G, TE, PR, COST_STAGES> E;
  extern __shared__ __align__(16) char lds_dyn[];
  __shared__ int fl_s[128];
  const Tile3 tl = xcd_tile();
  // tile row block rt, column block ct; grid x walks t in both orientations
  const int64_t rt = SIDE == 0 ? tl.y : tl.x, ct = SIDE == 0 ? tl.x : tl.y;
  const int64_t m0 = rt * G::BM, n0 = ct * G::BN;
  const int tid = threadIdx.x;
  if (tid < 128) fl_s[tid] = 0;
  f32x16 acc[G::FM][G::FN][2];
  zero16<G, 2>(acc);
  {
    Mat16 A[PR::NA], B[PR::NB];
#pragma unroll
    for (int x = 0; x < PR::NA; ++x) A[x] = ops.m[x];
#pragma unroll
    for (int y = 0; y < PR::NB; ++y) B[y] = ops.m[PR::NA + y];
    E::run(A, B, m0, n0, 0, Rk, lds_dyn, acc);
  }
  float vf[G::FM][G::FN][16];
  if (SIDE == 0) load_v16<G>(V, N, T, m0, n0, vf);
  else load_v16t<G>(V, N, T, m0, n0, vf);
  double* red = reinterpret_cast<double*>(lds_dyn);
  // extents of the tile rows and columns; partials part[q * stride + base + column]
  const int64_t M = SIDE == 0 ? N : T, C = SIDE == 0 ? T : N;
  const int64_t base = rt * C, stride = (int64_t)(SIDE == 0 ? gridDim.y : gridDim.x) * C;
  cost_cols<G, S0>(vf, acc, m0, n0, M, C, red, fl_s, part, fpart, base, stride);
  if (QM) row_qmax<G>(vf, acc, m0, n0, M, C, qmax, M);
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
// row maxima of H; rs = 2^-ceil(log2 max) (max scaled into [1/2, 1)).
static void rank_scales(int side, const float* W, const float* H, int64_t N, int64_t T, int64_t R,
                        const Scratch16& S, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_u32, dim3(grid1(R)), dim3(256), 0, s, S.bits, R);
  if (side == 0) {
    const int64_t parts = std::min<int64_t>(256, cdiv(N, 64));
    hipLaunchKernelGGL(k_colmax_W, dim3((unsigned)cdiv(R, 64), (unsigned)parts), dim3(256), 0, s, W, N, R,
                       cdiv(N, parts), S.bits);
  } else {
    const int64_t parts = std::min<int64_t>(256, cdiv(T, 2048));
    hipLaunchKernelGGL(k_rowmax_H, dim3((unsigned)parts, (unsigned)R), dim3(256), 0, s, H, T, R, cdiv(T, parts),
                       S.bits);
  }
  hipLaunchKernelGGL(k_scales, dim3(grid1(R)), dim3(256), 0, s, S.bits, R, 0, S.rs, S.irs, S.irs2);
}

// Dynamic LDS above the default 64 KiB needs the attribute once per kernel.
template <typename F>
static void lds_attr(F* fn, size_t bytes) {
  if (bytes > 65536) (void)hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <typename K>
static void launch_ratio_k(K* fn, int lds_bytes, dim3 grid, const Ratio16Args& ra, hipStream_t s) {
  const size_t lb = (size_t)std::max(lds_bytes, RATIO_OUT_BYTES);
  lds_attr(fn, lb);
  hipLaunchKernelGGL(fn, grid, dim3(256), lb, s, ra);
}

template <typename TE>
static hipError_t ratio_gh16(int side, const float* V, const float* W, const float* H, int64_t N, int64_t T,
                             int64_t R, const Scratch16& S, bool scaled, int splits, int64_t kchunk, float* pu,
                             float* puc, float* py, double* vpart, int* check, const SumJob& fin,
                             hipStream_t s, bool qmax_given) {
  const Dims16 d = dims16(N, T, R);
  const float* rs = nullptr;
  const float* irs = nullptr;
  const float* irs2 = nullptr;
  if (scaled) {
    rank_scales(side, W, H, N, T, R, S, s);
    rs = S.rs; irs = S.irs; irs2 = S.irs2;
  }
  // bf16: both factors split; fp16: the updated factor only
  const int split = scaled ? (side == 0 ? 1 : 2) : 3;
  const bool split_a = (split & 2) != 0, split_b = (split & 1) != 0;
  // Z operands: A = W (Np x Rk), B = H^t (Tp x Rk); the rank scales cancel
  prof_begin(side == 0 ? "conv16_H" : "conv16_W", s);
  conv16<TE>(ConvArgs{W, nullptr, N, R, R, nullptr, side == 0 ? rs : irs, S.fa_hi, split_a ? S.fa_lo : nullptr,
                      1, d.Np, d.Rk, d.Rk}, false, s);
  conv16<TE>(ConvArgs{H, nullptr, R, T, T, side == 0 ? irs : rs, nullptr, S.fb_hi, split_b ? S.fb_lo : nullptr,
                      1, d.Tp, d.Rk, d.Rk}, true, s);
  // gradient operands of the fixed factor: W^t, (W*W)^t (H step) or H, H*H (W step)
  if (side == 0)
    conv16<TE>(ConvArgs{W, nullptr, N, R, R, nullptr, rs, S.g0, S.g1, 2, d.Rm, d.Np, d.Np}, true, s);
  else
    conv16<TE>(ConvArgs{H, nullptr, R, T, T, rs, nullptr, S.g0, S.g1, 2, d.Rm, d.Tp, d.Tp}, false, s);
  prof_end(side == 0 ? "conv16_H" : "conv16_W", s);

  // H step: tile (n, t), A = W, B = H^t; W step: tile (t, n), A = H^t, B = W
  const Mat16 wm[2] = {Mat16{S.fa_hi, d.Rk}, Mat16{split_a ? S.fa_lo : S.fa_hi, d.Rk}};
  const Mat16 hm[2] = {Mat16{S.fb_hi, d.Rk}, Mat16{split_b ? S.fb_lo : S.fb_hi, d.Rk}};
  Ratio16Args ra;
  ra.V = V;
  for (int k = 0; k < 2; ++k) {
    ra.A[k] = side == 0 ? wm[k] : hm[k];
    ra.B[k] = side == 0 ? hm[k] : wm[k];
  }
  ra.N = N; ra.T = T; ra.Rk = d.Rk; ra.Np = d.Np; ra.Tp = d.Tp;
  ra.q3 = S.q3; ra.vpart = vpart; ra.check = check; ra.fin = fin;
  for (int k = 0; k < 3; ++k) { ra.qs[k] = nullptr; ra.qmax[k] = nullptr; }
  const dim3 rgrid((unsigned)(d.Tp / 128), (unsigned)(d.Np / 128));
  const int64_t L = side == 0 ? T : N;     // index range of the Q scales
  const float* iqs[3] = {nullptr, nullptr, nullptr};
  if (scaled) {
    unsigned* qbits = S.bits + d.Rm;
    if (!qmax_given) {   // else the preceding cost pass left bounds of them there
      hipLaunchKernelGGL(k_zero_u32, dim3(grid1(3 * L)), dim3(256), 0, s, qbits, 3 * L);
      for (int k = 0; k < 3; ++k) ra.qmax[k] = qbits + k * L;
      // the scales only need the maxima to a few bits: unsplit product
      prof_begin("qmax16", s);
      if (side == 0) launch_ratio_k(k_ratio16<TE, 0, true, 0>, ZEng<TE, 0>::LDS_BYTES, rgrid, ra, s);
      else launch_ratio_k(k_ratio16<TE, 1, true, 0>, ZEng<TE, 0>::LDS_BYTES, rgrid, ra, s);
      prof_end("qmax16", s);
      for (int k = 0; k < 3; ++k) ra.qmax[k] = nullptr;
    }
    for (int k = 0; k < 3; ++k) {
      hipLaunchKernelGGL(k_scales, dim3(grid1(L)), dim3(256), 0, s, qbits + k * L, L, 13, S.qs + k * L,
                         S.iqs + k * L, (float*)nullptr);
      ra.qs[k] = S.qs + k * L;
      iqs[k] = S.iqs + k * L;
    }
  }
  prof_begin(side == 0 ? "ratio16_H" : "ratio16_W", s);
  if (side == 0) {
    if (split == 1) launch_ratio_k(k_ratio16<TE, 0, false, 1>, ZEng<TE, 1>::LDS_BYTES, rgrid, ra, s);
    else launch_ratio_k(k_ratio16<TE, 0, false, 3>, ZEng<TE, 3>::LDS_BYTES, rgrid, ra, s);
  } else {           // the operands swapped: W (split in FP16) is now the B operand
    if (split == 2) launch_ratio_k(k_ratio16<TE, 1, false, 1>, ZEng<TE, 1>::LDS_BYTES, rgrid, ra, s);
    else launch_ratio_k(k_ratio16<TE, 1, false, 3>, ZEng<TE, 3>::LDS_BYTES, rgrid, ra, s);
  }
  prof_end(side == 0 ? "ratio16_H" : "ratio16_W", s);

  // gradient products
  const int64_t npt = d.Np * d.Tp;
  const uint16_t* q = reinterpret_cast<const uint16_t*>(S.q3);
  Fold f;
  Ops16 ops;
  int64_t M, Ncol, K32;
  dim3 grid;
  if (side == 0) {   // rows r carry the W^t scale, columns t the Q scales
    const float* rr[3] = {irs, irs, irs2};
    for (int k = 0; k < 3; ++k) { f.r[k] = rr[k]; f.c[k] = iqs[k]; }
    ops.m[0] = Mat16{S.g0, d.Np}; ops.m[1] = Mat16{S.g1, d.Np};
    for (int k = 0; k < 3; ++k) ops.m[2 + k] = Mat16{q + k * npt, d.Np};
    M = R; Ncol = T; K32 = cdiv(N, 32) * 32;
    grid = dim3((unsigned)(d.Rm / GGH::BM), (unsigned)(d.Tp / GGH::BN), (unsigned)splits);
  } else {           // rows n carry the Q scales, columns r the H scale
    const float* cc[3] = {irs, irs, irs2};
    for (int k = 0; k < 3; ++k) { f.r[k] = iqs[k]; f.c[k] = cc[k]; }
    for (int k = 0; k < 3; ++k) ops.m[k] = Mat16{q + k * npt, d.Tp};
    ops.m[3] = Mat16{S.g0, d.Tp}; ops.m[4] = Mat16{S.g1, d.Tp};
    M = N; Ncol = R; K32 = cdiv(T, 32) * 32;
    grid = dim3((unsigned)(d.Rm / GGH::BN), (unsigned)(d.Np / GGH::BM), (unsigned)splits);
  }
  const size_t lb = (size_t)std::max(Gemm16<GGH, TE, GHH_P, GH_STAGES>::LDS_BYTES,
                                     Gemm16<GGH, TE, GHW_P, GH_STAGES>::LDS_BYTES);
  prof_begin(side == 0 ? "gh16_H" : "gh16_W", s);
  if (side == 0) {
    lds_attr(k_gh16<TE, 0>, lb);
    hipLaunchKernelGGL((k_gh16<TE, 0>), grid, dim3(256), lb, s, ops, M, Ncol, K32, kchunk, pu, puc, py, f);
  } else {
    lds_attr(k_gh16<TE, 1>, lb);
    hipLaunchKernelGGL((k_gh16<TE, 1>), grid, dim3(256), lb, s, ops, M, Ncol, K32, kchunk, pu, puc, py, f);
  }
  prof_end(side == 0 ? "gh16_H" : "gh16_W", s);
  return hipGetLastError();
}

template <typename TE>
static hipError_t cost16(int side, const float* V, const float* F, const float* Xmu, const float* Xn, int64_t N,
                         int64_t T, int64_t R, const Scratch16& S, bool scaled, double* part, int* fpart,
                         hipStream_t s, bool s0, bool qmax_next) {
  const Dims16 d = dims16(N, T, R);
  const float* rs = nullptr;
  const float* irs = nullptr;
  if (scaled) {
    if (side == 0) rank_scales(0, F, nullptr, N, T, R, S, s);
    else rank_scales(1, nullptr, F, N, T, R, S, s);
    rs = S.rs;
    irs = S.irs;
  }
  Ops16 ops;
  prof_begin(side == 0 ? "conv16c_H" : "conv16c_W", s);
  if (side == 0) {   // A = W (scaled rs), B = X^t (scaled irs)
    conv16<TE>(ConvArgs{F, nullptr, N, R, R, nullptr, rs, S.fa_hi, nullptr, 0, d.Np, d.Rk, d.Rk}, false, s);
    conv16<TE>(ConvArgs{Xn, nullptr, R, T, T, irs, nullptr, S.x0, nullptr, 0, d.Tp, d.Rk, d.Rk}, true, s);
    conv16<TE>(ConvArgs{Xmu, Xn, R, T, T, irs, nullptr, S.x1, nullptr, 0, d.Tp, d.Rk, d.Rk}, true, s);
    ops.m[0] = Mat16{S.fa_hi, d.Rk}; ops.m[1] = Mat16{S.x0, d.Rk}; ops.m[2] = Mat16{S.x1, d.Rk};
  } else {           // A = H^t (scaled rs), B = X (scaled irs): the transposed tile
    conv16<TE>(ConvArgs{Xn, nullptr, N, R, R, nullptr, irs, S.x0, nullptr, 0, d.Np, d.Rk, d.Rk}, false, s);
    conv16<TE>(ConvArgs{Xmu, Xn, N, R, R, nullptr, irs, S.x1, nullptr, 0, d.Np, d.Rk, d.Rk}, false, s);
    conv16<TE>(ConvArgs{F, nullptr, R, T, T, rs, nullptr, S.fb_hi, nullptr, 0, d.Tp, d.Rk, d.Rk}, true, s);
    ops.m[0] = Mat16{S.fb_hi, d.Rk}; ops.m[1] = Mat16{S.x0, d.Rk}; ops.m[2] = Mat16{S.x1, d.Rk};
  }
  prof_end(side == 0 ? "conv16c_H" : "conv16c_W", s);
  const dim3 grid((unsigned)(d.Tp / 128), (unsigned)(d.Np / 128));
  const size_t lb = (size_t)Gemm16<G128, TE, CH_P, COST_STAGES>::LDS_BYTES;
  // maxima for the next half-step's Q scales: per n after the H step, per t after the W step
  unsigned* qmax = nullptr;
  if (scaled && qmax_next) {
    const int64_t L = side == 0 ? N : T;
    qmax = S.bits + d.Rm;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid1(3 * L)), dim3(256), 0, s, qmax, 3 * L);
  }
  prof_begin(side == 0 ? "cost16_H" : "cost16_W", s);
  typedef void (*Kern)(const float*, Ops16, int64_t, int64_t, int64_t, double*, int*, unsigned*);
  Kern k;
  if (side == 0)
    k = qmax ? (s0 ? k_cost16<TE, 0, true, true> : k_cost16<TE, 0, false, true>)
             : (s0 ? k_cost16<TE, 0, true, false> : k_cost16<TE, 0, false, false>);
  else
    k = qmax ? (s0 ? k_cost16<TE, 1, true, true> : k_cost16<TE, 1, false, true>)
             : (s0 ? k_cost16<TE, 1, true, false> : k_cost16<TE, 1, false, false>);
  lds_attr(k, lb);
  hipLaunchKernelGGL(k, grid, dim3(256), lb, s, V, ops, N, T, d.Rk, part, fpart, qmax);
  prof_end(side == 0 ? "cost16_H" : "cost16_W", s);
  return hipGetLastError();
}

hipError_t launch_ratio_gh16(int gemm, int side, const float* V, const float* W, const float* H, int64_t N,
                             int64_t T, int64_t R, const Scratch16& S, int splits, int64_t kchunk, float* pu,
                             float* puc, float* py, double* vpart, int* check, const SumJob& fin,
                             hipStream_t s, bool qmax_given) {
  // the Z pass addresses V with 32-bit byte offsets of up to 128 rows
  if (T >= (int64_t(1) << 22)) return hipErrorInvalidValue;
  if (gemm == 1)
    return ratio_gh16<__bf16>(side, V, W, H, N, T, R, S, false, splits, kchunk, pu, puc, py, vpart, check, fin, s,
                              false);
  return ratio_gh16<_Float16>(side, V, W, H, N, T, R, S, true, splits, kchunk, pu, puc, py, vpart, check, fin, s,
                              qmax_given);
}

hipError_t launch_cost16(int gemm, int side, const float* V, const float* F, const float* Xmu, const float* Xn,
                         int64_t N, int64_t T, int64_t R, const Scratch16& S, double* part, int* fpart,
                         hipStream_t s, bool s0, bool qmax_next) {
  if (T >= (int64_t(1) << 22)) return hipErrorInvalidValue;   // 32-bit offsets into V, as the Z pass
  if (gemm == 1) return cost16<__bf16>(side, V, F, Xmu, Xn, N, T, R, S, false, part, fpart, s, s0, false);
  return cost16<_Float16>(side, V, F, Xmu, Xn, N, T, R, S, true, part, fpart, s, s0, qmax_next);
}

}  // namespace dna
