// epilogue.hpp -- pieces shared by the fp32 and 16-bit kernel epilogues:
// deterministic tile reductions and the per-element cost terms.
#pragma once
#include <math.h>

#include "core.hpp"
#include "kernels.hpp"

namespace dna {

// ---------------------------------------------------------------------------
// Second level of a factor sum (struct SumJob), spread over every block of the
// grid that carries it: r-th sum = parts added in order p = 0, 1, ...
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sum_job(const SumJob& j) {
  if (!j.part) return;
  const int64_t nb = (int64_t)gridDim.x * gridDim.y * gridDim.z;
  const int64_t lin = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
  for (int64_t r = lin * blockDim.x + threadIdx.x; r < j.R; r += nb * blockDim.x) {
    double tot = 0.0;
#pragma unroll 8
    for (int p = 0; p < j.nparts; ++p) tot += j.part[(int64_t)p * j.R + r];
    if (j.s64) j.s64[r] = tot;
    if (j.s32) j.s32[r] = (float)(tot + j.reg);
    if (j.check && !(tot > 0.0)) atomicOr(j.check, CHK_DOMAIN);
  }
}

// ---------------------------------------------------------------------------
// Deterministic tile reductions of per-lane partials.
// Column form: cp[q][j] holds this lane's partial for column (j, lane&31).
// Row form:    rp[q][i][v] holds this lane's partial for row blk_row(v) of block i.
// `red` is LDS scratch of NQ * max(WGM*BN, WGN*BM) doubles.
// ---------------------------------------------------------------------------
template <class G, int NQ, class OUT>
__device__ __forceinline__ void reduce_cols(double (&cp)[NQ][G::FN], double* red, OUT&& out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % G::WGM, wn = wave / G::WGM;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      const double s = cp[q][j] + __shfl_xor(cp[q][j], 32);
      if (lane < 32) red[(q * G::WGM + wm) * G::BN + wn * G::WN + j * 32 + lane] = s;
    }
  __syncthreads();
  for (int c = tid; c < G::BN; c += G::NT) {
    double s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      s[q] = 0.0;
      for (int m = 0; m < G::WGM; ++m) s[q] += red[(q * G::WGM + m) * G::BN + c];
    }
    out(c, s);
  }
  __syncthreads();
}

template <class G, int NQ, class OUT>
__device__ __forceinline__ void reduce_rows(double (&rp)[NQ][G::FM][16], double* red, OUT&& out) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % G::WGM, wn = wave / G::WGM;
#pragma unroll
  for (int q = 0; q < NQ; ++q)
#pragma unroll
    for (int i = 0; i < G::FM; ++i) {
      const double y = halfwave_slot_sum(rp[q][i], lane);
      if ((lane & 1) == 0) red[(q * G::WGN + wn) * G::BM + wm * G::WM + i * 32 + slot_row(lane)] = y;
    }
  __syncthreads();
  for (int r = tid; r < G::BM; r += G::NT) {
    double s[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      s[q] = 0.0;
      for (int w = 0; w < G::WGN; ++w) s[q] += red[(q * G::WGN + w) * G::BM + r];
    }
    out(r, s);
  }
  __syncthreads();
}

// The cost terms use the hardware base-2 logarithm (v_log_f32, within 1 ulp
// over the whole float range, including arguments near 1) and are summed in
// base-2 units; LN2 converts a finished sum to natural units.
constexpr double LN2 = 0.69314718055994530942;

__device__ __forceinline__ float log2_hw(float x) { return __builtin_amdgcn_logf(x); }

// log2(1 + u) for u > -1, accurate for small |u|: with w = 1 + u rounded,
// log2(w) * u / (w - 1) cancels the rounding of w to first order (Goldberg's
// log1p construction); w == 1 takes the first series term.
// u is clamped to FLT_MAX (an overflowed ratio still gives a finite, huge term).
// Both forms are evaluated and one is selected, so the code has no branch.
__device__ __forceinline__ float log2_1p(float u) {
  u = fminf(u, 3.402823466e38f);
  const float w = 1.f + u;
  const float d = w - 1.f;
  const float general = log2_hw(w) * (u * __builtin_amdgcn_rcpf(d));
  const float series = u * 1.44269504088896341f;
  return (d == 0.f) ? series : general;
}

// log2(z_MU / z_DNA) for z_DNA, z_MU > 0 given u = dZ / z_DNA: the log1p form
// while the ratio is near 1; below 1/2 the ratio itself, formed as z_MU / z_DNA
// (1 + u would lose its relative precision, or fall to or below zero through
// rounding, when z_MU is far smaller than z_DNA).
// The direct form is evaluated only when some lane of the wave needs it (a
// wave-uniform branch): z_MU below half of z_DNA is rare, and the logarithm
// costs a quarter-rate instruction per element.
__device__ __forceinline__ float log2_ratio(float u, float zM, float izN) {
  const float near1 = log2_1p(fmaxf(u, -0.5f));
  const bool low = u < -0.5f;
  if (__any(low)) return low ? log2_hw(zM * izN) : near1;
  return near1;
}

__device__ __forceinline__ double xlog2x_over(float v, float z) {
  // v log2(v/z) for v > 0, z > 0 (the summand of eq. 1 and steps 9/14, base 2)
  return (double)(v * log2_hw(v * __builtin_amdgcn_rcpf(z)));
}

// Per-element cost terms, in base-2 units, with v > 0 and z_DNA, z_MU the two
// reconstructions (z_MU = z_DNA + dZ):
//   s0 += v log2(v/z_DNA)         (d_DNA; rows with z_DNA <= 0 flag bit 1)
//   s1 += -v log2(1 + dZ/z_DNA)   (d_MU - d_DNA; rows where both z > 0)
//   s2 += v log2(v/z_MU)          (rows with z_DNA <= 0 < z_MU; bit 2 if z_MU <= 0)
// so that, absent flags, d_MU = s0 + s1 and the margin is s1.
// Branch-free for the common case (both reconstructions positive or v = 0): the
// logarithms take neutral arguments where a term must vanish.  Returns the flag
// bits of this element.
// The choice (decide) reads s1 and the flags only; s0 is the kept candidate's
// cost, so callers that want no cost pass S0 = false and s0 stays untouched.
template <bool S0 = true>
__device__ __forceinline__ int cost_acc(float x, float zN, float dz, double& s0, double& s1, double& s2) {
  const float zM = zN + dz;
  const bool pos = x > 0.f;
  const bool okN = zN > 0.f, okM = zM > 0.f;
  const float izN = __builtin_amdgcn_rcpf(zN);
  if (S0) s0 += (double)(x * log2_hw((pos && okN) ? x * izN : 1.f));
  const bool both = pos && okN && okM;
  const float l1 = log2_ratio(both ? dz * izN : 0.f, both ? zM : 1.f, both ? izN : 1.f);
  s1 -= (double)(x * l1);
  int fl = 0;
  if (pos && !(okN && okM)) {            // a reconstruction vanished where v > 0
    fl = (okN ? 0 : 1) | (okM ? 0 : 2);
    if (!okN && okM) s2 += xlog2x_over(x, zM);
  }
  return fl;
}

// cost_acc with the first two terms added to float32 accumulators (a caller
// that flushes them to float64 every few elements).
template <bool S0 = true>
__device__ __forceinline__ int cost_acc_f(float x, float zN, float dz, float& a0, float& a1, double& s2) {
  const float zM = zN + dz;
  const bool pos = x > 0.f;
  const bool okN = zN > 0.f, okM = zM > 0.f;
  const float izN = __builtin_amdgcn_rcpf(zN);
  if (S0) a0 += x * log2_hw((pos && okN) ? x * izN : 1.f);
  const bool both = pos && okN && okM;
  const float l1 = log2_ratio(both ? dz * izN : 0.f, both ? zM : 1.f, both ? izN : 1.f);
  a1 -= x * l1;
  int fl = 0;
  if (pos && !(okN && okM)) {
    fl = (okN ? 0 : 1) | (okM ? 0 : 2);
    if (!okN && okM) s2 += xlog2x_over(x, zM);
  }
  return fl;
}

// ---------------------------------------------------------------------------
// The Newton candidate's term alone (damped selection): s0 += v log2(v/z_DNA);
// returns flag bit 1 where z_DNA <= 0 at v > 0.
__device__ __forceinline__ int cost_acc_newton(float x, float zN, double& s0) {
  const bool pos = x > 0.f, okN = zN > 0.f;
  s0 += (double)(x * log2_hw((pos && okN) ? x * __builtin_amdgcn_rcpf(zN) : 1.f));
  return (pos && !okN) ? 1 : 0;
}
__device__ __forceinline__ int cost_acc_newton_f(float x, float zN, float& a0) {
  const bool pos = x > 0.f, okN = zN > 0.f;
  a0 += x * log2_hw((pos && okN) ? x * __builtin_amdgcn_rcpf(zN) : 1.f);
  return (pos && !okN) ? 1 : 0;
}

// Epilogues of the candidate-cost passes (steps 7-9, 12-14), shared by the fp32
// and 16-bit kernels.  acc[..][0] holds z_DNA, acc[..][1] holds dZ = z_MU - z_DNA
// at this lane's accumulator positions; vf holds v there.  Partials (natural
// log units) go to part[q * stride + base + index], q = 0, 1, 2 for s0, s1, s2,
// and the OR of the flags to fpart[base + index].
// ---------------------------------------------------------------------------
template <class G>
__device__ __forceinline__ int64_t epi_row(int64_t m0, int i, int v) {
  const int tid = threadIdx.x, lane = tid & 63, wm = (tid >> 6) % G::WGM;
  return m0 + wm * G::WM + i * 32 + blk_row(v, lane);
}
template <class G>
__device__ __forceinline__ int64_t epi_col(int64_t n0, int j) {
  const int tid = threadIdx.x, lane = tid & 63, wn = (tid >> 6) / G::WGM;
  return n0 + wn * G::WN + j * 32 + blk_col(lane);
}

// Column form (H orientation: one partial per column t of the tile).
template <class G, bool S0, int NC>
__device__ __forceinline__ void cost_cols_acc(const float (&vf)[G::FM][G::FN][16],
                                              const f32x16 (&acc)[G::FM][G::FN][NC], int64_t m0, int64_t n0,
                                              int64_t N, int64_t T, double (&cp)[3][G::FN], int* fl_s) {
#pragma unroll
  for (int j = 0; j < G::FN; ++j) {
    const int64_t col = epi_col<G>(n0, j);
    int fl = 0;
#pragma unroll
    for (int i = 0; i < G::FM; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const float x = (epi_row<G>(m0, i, v) < N && col < T) ? vf[i][j][v] : 0.f;
        fl |= cost_acc<S0>(x, acc[i][j][0][v], acc[i][j][1][v], cp[0][j], cp[1][j], cp[2][j]);
      }
    if (fl) atomicOr(&fl_s[col - n0], fl);
  }
}

// With S0 = false the s0 partials are written as 0 (no cost wanted).
template <class G, bool S0 = true, int NC>
__device__ __forceinline__ void cost_cols(const float (&vf)[G::FM][G::FN][16],
                                          const f32x16 (&acc)[G::FM][G::FN][NC], int64_t m0, int64_t n0,
                                          int64_t N, int64_t T, double* red, int* fl_s, double* part, int* fpart,
                                          int64_t base, int64_t stride) {
  double cp[3][G::FN];
#pragma unroll
  for (int j = 0; j < G::FN; ++j) cp[0][j] = cp[1][j] = cp[2][j] = 0.0;
  cost_cols_acc<G, S0>(vf, acc, m0, n0, N, T, cp, fl_s);
  if (S0) {
    reduce_cols<G, 3>(cp, red, [&](int c, const double (&s)[3]) {
      if (n0 + c < T) {
        part[base + n0 + c] = s[0] * LN2;
        part[stride + base + n0 + c] = s[1] * LN2;
        part[2 * stride + base + n0 + c] = s[2] * LN2;
        fpart[base + n0 + c] = fl_s[c];
      }
    });
  } else {
    double c2[2][G::FN];
#pragma unroll
    for (int j = 0; j < G::FN; ++j) {
      c2[0][j] = cp[1][j];
      c2[1][j] = cp[2][j];
    }
    reduce_cols<G, 2>(c2, red, [&](int c, const double (&s)[2]) {
      if (n0 + c < T) {
        part[base + n0 + c] = 0.0;
        part[stride + base + n0 + c] = s[0] * LN2;
        part[2 * stride + base + n0 + c] = s[1] * LN2;
        fpart[base + n0 + c] = fl_s[c];
      }
    });
  }
}

// Row form (W orientation: one partial per row n of the tile).
template <class G, bool S0, int NC>
__device__ __forceinline__ void cost_rows_acc(const float (&vf)[G::FM][G::FN][16],
                                              const f32x16 (&acc)[G::FM][G::FN][NC], int64_t m0, int64_t n0,
                                              int64_t N, int64_t T, double (&rp)[3][G::FM][16], int* fl_s) {
#pragma unroll
  for (int i = 0; i < G::FM; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int64_t row = epi_row<G>(m0, i, v);
      int fl = 0;
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
        const float x = (row < N && epi_col<G>(n0, j) < T) ? vf[i][j][v] : 0.f;
        fl |= cost_acc<S0>(x, acc[i][j][0][v], acc[i][j][1][v], rp[0][i][v], rp[1][i][v], rp[2][i][v]);
      }
      if (fl) atomicOr(&fl_s[row - m0], fl);
    }
}

// The partials of one row block i at a time (the sums, their order and the
// LDS layout of reduce_rows, with a third of the float64 registers live).
// With S0 = false the s0 partials are written as 0 (no cost wanted).
template <class G, bool S0 = true, int NC>
__device__ __forceinline__ void cost_rows(const float (&vf)[G::FM][G::FN][16],
                                          const f32x16 (&acc)[G::FM][G::FN][NC], int64_t m0, int64_t n0,
                                          int64_t N, int64_t T, double* red, int* fl_s, double* part, int* fpart,
                                          int64_t base, int64_t stride) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % G::WGM, wn = wave / G::WGM;
#pragma unroll
  for (int i = 0; i < G::FM; ++i) {
    double rp[3][16];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      rp[0][v] = rp[1][v] = rp[2][v] = 0.0;
      const int64_t row = epi_row<G>(m0, i, v);
      int fl = 0;
#pragma unroll
      for (int j = 0; j < G::FN; ++j) {
        const float x = (row < N && epi_col<G>(n0, j) < T) ? vf[i][j][v] : 0.f;
        fl |= cost_acc<S0>(x, acc[i][j][0][v], acc[i][j][1][v], rp[0][v], rp[1][v], rp[2][v]);
      }
      if (fl) atomicOr(&fl_s[row - m0], fl);
    }
#pragma unroll
    for (int q = S0 ? 0 : 1; q < 3; ++q) {
      const double y = halfwave_slot_sum(rp[q], lane);
      if ((lane & 1) == 0) red[(q * G::WGN + wn) * G::BM + wm * G::WM + i * 32 + slot_row(lane)] = y;
    }
  }
  __syncthreads();
  for (int r = tid; r < G::BM; r += G::NT) {
    double s[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      s[q] = 0.0;
      if (q > 0 || S0)
        for (int w = 0; w < G::WGN; ++w) s[q] += red[(q * G::WGN + w) * G::BM + r];
    }
    if (m0 + r < N) {
      part[base + m0 + r] = s[0] * LN2;
      part[stride + base + m0 + r] = s[1] * LN2;
      part[2 * stride + base + m0 + r] = s[2] * LN2;
      fpart[base + m0 + r] = fl_s[r];
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Candidates (eq. 7, 11, 14, 15, 17) of one coordinate.
// ---------------------------------------------------------------------------
struct Cand {
  float mu, newton, A, B;
};

// MU gain g = u/c and A = g - 1 (eq. 7) from the two forms of the gradient sum,
// c = (F^t 1)_r + reg (reg: the eq. 2 weight, lambda or rho): where g < 1/2 the
// plain sum u = (F^t q)_r carries g to float32 relative accuracy; elsewhere the
// centred sum u_c = (F^t (q - 1))_r = u - (c - reg) carries A = (u_c - reg)/c to
// float32 accuracy near its zero (near-stationary coordinates, where the Newton
// step divides by b).
__device__ __forceinline__ void gain(float u, float uc, float c, float reg, float& g, float& A) {
  const float gp = u / c;
  if (gp < 0.5f) {
    g = gp;
    A = gp - 1.f;
  } else {
    A = (uc - reg) / c;
    g = 1.f + A;
  }
}

// One coordinate: numerators u, u_c, y = ((F*F)^t q-bar)_r, scale c_r (which
// includes reg).
__device__ __forceinline__ Cand candidate(float x, float u, float uc, float y, float c, float eps, float alpha,
                                          float reg) {
  Cand o;
  float g;
  gain(u, uc, c, reg, g, o.A);      // eq. (7)
  o.B = y / c;                      // eq. (14)
  o.mu = fmaxf(x * g, VALUE_FLOOR); // eq. (11), kept a positive normal float
  if (o.A < 0.f) {                  // eq. (15), gain floored at eps
    const float xb = x * o.B;
    o.newton = x * fmaxf(xb / (xb - o.A), eps);
  } else {                          // eq. (17), step capped at alpha x
    const float step = (o.B > 0.f) ? o.A / o.B : (o.A > 0.f ? INFINITY : 0.f);
    o.newton = x + fminf(step, alpha * x);
  }
  return o;
}

// ---------------------------------------------------------------------------
// The choice of step 15 (28) from a column's (row's) cost sums: q0 = d_DNA,
// q1 = d_MU - d_DNA, q2 = the terms where only z_MU is positive, fl the flags.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool decide(double q0, double q1, double q2, int fl, double& dsel, double& margin) {
  const double dN = (fl & 1) ? INFINITY : q0;
  const double dM = (fl & 2) ? INFINITY : q0 + q1 + q2;
  bool newton;
  if (fl == 0) {
    newton = q1 > 0.0;        // d_DNA < d_MU, decided on the directly computed difference
    margin = q1;
  } else {
    newton = dN < dM;
    margin = dM - dN;
  }
  dsel = newton ? dN : dM;
  return newton;
}

}  // namespace dna
