// kernels_adj.hip -- adjoint (vector-Jacobian product) of one DNA H-update with W
// fixed, for the differentiable unrolled H-solve.
//
// Forward of one update, per column t (Algorithm 1 steps 4-15):
//   z = W h, q = v/z, qb = v/z^2, c = W^t 1, s = sum_n v_n,
//   u = W^t q, y = (W*W)^t qb, A = u/c - 1 (eq. 7), B = y/c (eq. 14),
//   MU:     h'_r = h_r u_r / c_r                                  (eq. 11)
// (A and the MU gain are evaluated exactly as in the forward kernels, from the
// plain and the centred gradient sums, so every branch repeats.)
//   Newton: p_r = eq. (15) / eq. (17) branch with floor and cap,
//           h'_r = kappa p_r, kappa = s / sum_l c_l p_l           (eq. 10)
// The selection of each column is frozen at its forward value and each entry is
// differentiated along the branch it took.  Given G = dL/dh', the kernels form
//   ubar = dL/du, ybar = dL/dy, hd = direct dL/dh, cbar (per entry), sbar = dL/ds
// (k_cand_bwd_H), then qbar = W ubar, qbbar = (W*W) ybar on MFMA with the
// epilogue zbar = -(qbar q + 2 qbbar qb)/z and vbar = qbar/z + qbbar/z^2 + sbar
// (k_zbar), then dL/dh = hd + W^t zbar (split GEMM + k_dh_final) and
// dL/dW += Q ubar^t + zbar H^t + 2 W * (Qb ybar^t) + cbar (k_wbar + k_dw_final).
#include <math.h>

#include <algorithm>

#include "core.hpp"
#include "kernels_adj.hpp"

namespace dna {

using GZB = Geo<ZT_BM, ZT_BN, GEMM_BK, 2, 2>;   // zbar products, M = N, N = T, K = R
using GWB = Geo<WB_BM, WB_BN, GEMM_BK, 2, 2>;   // W-gradient products, M = N, N = R, K = T

struct Deriv {
  float p;              // Newton candidate before renormalisation
  float dh, dA, dB;     // partial derivatives of p
};

// Newton candidate and its partials along the active branch (same arithmetic as
// the forward candidate so that every branch decision repeats exactly).
__device__ __forceinline__ Deriv newton_deriv(float x, float A, float B, float eps, float alpha) {
  Deriv d;
  if (A < 0.f) {
    const float xb = x * B;
    const float den = xb - A;
    const float g = xb / den;
    if (g < eps) {                                   // floored gain
      d.p = x * eps;
      d.dh = eps; d.dA = 0.f; d.dB = 0.f;
    } else {
      d.p = x * g;
      d.dh = g * (xb - 2.f * A) / den;               // x B (x B - 2A) / den^2
      d.dA = x * g / den;                            // x^2 B / den^2
      d.dB = -x * x * A / (den * den);
    }
  } else {
    const float step = (B > 0.f) ? A / B : (A > 0.f ? INFINITY : 0.f);
    if (step > alpha * x) {                          // capped step
      d.p = x * (1.f + alpha);
      d.dh = 1.f + alpha; d.dA = 0.f; d.dB = 0.f;
    } else {
      d.p = x + step;
      d.dh = 1.f;
      d.dA = (B > 0.f) ? 1.f / B : 0.f;
      d.dB = (B > 0.f) ? -step / B : 0.f;
    }
  }
  return d;
}

// MU gain and A from the plain and centred sums, as in the forward candidates.
__device__ __forceinline__ void gain_bwd(float u, float uc, float c, float& g, float& A) {
  const float gp = u / c;
  if (gp < 0.5f) {
    g = gp;
    A = gp - 1.f;
  } else {
    A = uc / c;
    g = 1.f + A;
  }
}

// Per-column adjoint of one H-update.  Block: COLS columns x RG row groups, the
// forward candidate kernel's layout for the same T and R (cand_layout), so
// every sum over r rounds identically.
// Newton columns take three passes over r: D = sum c p (-> kappa), then the
// clamp-aware sum of G p (-> beta), then the per-entry adjoints.  An entry held
// at the value floor in the forward pass is a constant and carries no gradient.

struct Sums {
  float u, uc, y;
};

__device__ __forceinline__ Sums split_sums(const float* pu, const float* puc, const float* py, int splits,
                                           int64_t R, int64_t T, int64_t r, int64_t t) {
  Sums s = {0.f, 0.f, 0.f};
  for (int sp = 0; sp < splits; ++sp) {
    s.u += pu[(sp * R + r) * T + t];
    s.uc += puc[(sp * R + r) * T + t];
    s.y += py[(sp * R + r) * T + t];
  }
  return s;
}

// One entry (r, t) of the per-column adjoint (pass 3 of k_cand_bwd_H), with G
// at (r, t) given.
__device__ __forceinline__ void cand_bwd_entry(const float* pu, const float* puc, const float* py, int splits,
                                               int64_t R, int64_t T, int64_t r, int64_t t, const float* c,
                                               const float* H, float gr, float eps, float alpha, bool newton,
                                               bool renorm, double kappa, double beta, float* Ubar, float* Ybar,
                                               float* Hd, float* Cbar) {
  {
    const Sums q = split_sums(pu, puc, py, splits, R, T, r, t);
    const float cr = c[r], x = H[r * T + t];
    float g, A;
    gain_bwd(q.u, q.uc, cr, g, A);
    float ub, yb, hd, cb;
    if (newton) {
      const Deriv d = newton_deriv(x, A, q.y / cr, eps, alpha);
      const bool clamped = (float)((double)d.p * kappa) < VALUE_FLOOR;
      const double gt = clamped ? 0.0 : (double)gr;
      const float pbar = renorm ? (float)(kappa * (gt - (double)cr * beta)) : (float)gt;
      const float Ab = pbar * d.dA, Bb = pbar * d.dB;
      hd = pbar * d.dh;
      ub = Ab / cr;
      yb = Bb / cr;
      cb = -(Ab * q.u + Bb * q.y) / (cr * cr) - (renorm ? (float)(kappa * beta * (double)d.p) : 0.f);
    } else if (x * g < VALUE_FLOOR) {      // MU output held at the floor
      hd = ub = yb = cb = 0.f;
    } else {
      hd = gr * g;
      ub = gr * x / cr;
      yb = 0.f;
      cb = -gr * x * q.u / (cr * cr);
    }
    Ubar[r * T + t] = ub;
    Ybar[r * T + t] = yb;
    Hd[r * T + t] = hd;
    Cbar[r * T + t] = cb;
  }
}

template <int BW_COLS, int BW_RG>
__global__ __launch_bounds__(BW_COLS * BW_RG) void k_cand_bwd_H(const float* H, const float* pu, const float* puc, const float* py, int splits,
                                                    const float* c, const double* vpart, int tiles_m, int64_t T,
                                                    int64_t R, float eps, float alpha, const uint8_t* sel,
                                                    const float* G, float* Ubar, float* Ybar, float* Hd,
                                                    float* Cbar, float* sbar) {
  __shared__ double red[BW_RG][BW_COLS];
  __shared__ double kap[BW_COLS], bet[BW_COLS];
  const int tid = threadIdx.x, cl = tid % BW_COLS, rg = tid / BW_COLS;
  const int64_t t = (int64_t)blockIdx.x * BW_COLS + cl;
  const bool ok = t < T;
  const bool newton = ok && sel[t] != 0;
  // pass 1: D = sum_r c_r p_r (the renormalisation denominator of eq. 10).
  // With at most CI rows per thread, p and G stay in registers from pass to
  // pass (pass 2 then reads only G, pass 3 not G); the sums are the same.
  constexpr int CI = 32;
  const bool cache = (R + BW_RG - 1) / BW_RG <= CI;
  float pc[CI], gc[CI];
  double D = 0.0;
  if (newton) {
    if (cache) {
#pragma unroll
      for (int i = 0; i < CI; ++i) {
        const int64_t r = rg + (int64_t)i * BW_RG;
        pc[i] = 0.f;
        if (r < R) {
          const Sums q = split_sums(pu, puc, py, splits, R, T, r, t);
          const float cr = c[r];
          float g, A;
          gain_bwd(q.u, q.uc, cr, g, A);
          pc[i] = newton_deriv(H[r * T + t], A, q.y / cr, eps, alpha).p;
          D += (double)cr * (double)pc[i];
        }
      }
    } else {
      for (int64_t r = rg; r < R; r += BW_RG) {
        const Sums q = split_sums(pu, puc, py, splits, R, T, r, t);
        const float cr = c[r];
        float g, A;
        gain_bwd(q.u, q.uc, cr, g, A);
        D += (double)cr * (double)newton_deriv(H[r * T + t], A, q.y / cr, eps, alpha).p;
      }
    }
  }
  red[rg][cl] = D;
  __syncthreads();
  if (rg == 0) {
    double d = 0.0, kappa = 1.0;
    if (newton) {
      for (int k = 0; k < BW_RG; ++k) d += red[k][cl];
      if (d > 0.0) {
        double s = 0.0;
        for (int m = 0; m < tiles_m; ++m) s += vpart[(int64_t)m * T + t];
        kappa = s / d;
      }
    }
    kap[cl] = kappa;
    bet[cl] = d;          // keeps D for pass 2
  }
  __syncthreads();
  const double kappa = kap[cl], Dsum = bet[cl];
  // pass 2: beta = sum over unclamped r of G_r p_r / D
  double GP = 0.0;
  if (newton && Dsum > 0.0) {
    if (cache) {
#pragma unroll
      for (int i = 0; i < CI; ++i) {
        const int64_t r = rg + (int64_t)i * BW_RG;
        if (r < R) {
          gc[i] = G[r * T + t];
          if (!((float)((double)pc[i] * kappa) < VALUE_FLOOR)) GP += (double)gc[i] * (double)pc[i];
        }
      }
    } else {
      for (int64_t r = rg; r < R; r += BW_RG) {
        const Sums q = split_sums(pu, puc, py, splits, R, T, r, t);
        const float cr = c[r];
        float g, A;
        gain_bwd(q.u, q.uc, cr, g, A);
        const float p = newton_deriv(H[r * T + t], A, q.y / cr, eps, alpha).p;
        if (!((float)((double)p * kappa) < VALUE_FLOOR)) GP += (double)G[r * T + t] * (double)p;
      }
    }
  }
  __syncthreads();
  red[rg][cl] = GP;
  __syncthreads();
  if (rg == 0) {
    double b = 0.0;
    if (newton && Dsum > 0.0) {
      for (int k = 0; k < BW_RG; ++k) b += red[k][cl];
      b /= Dsum;
    }
    bet[cl] = b;
  }
  __syncthreads();
  if (!ok) return;
  const double beta = bet[cl];
  const bool renorm = newton && Dsum > 0.0;
  if (rg == 0) sbar[t] = renorm ? (float)beta : 0.f;
  // pass 3: per-entry adjoints
  const bool gcached = cache && newton && Dsum > 0.0;
#pragma unroll
  for (int i = 0; i < CI; ++i) {
    const int64_t r = rg + (int64_t)i * BW_RG;
    if (cache && r < R) cand_bwd_entry(pu, puc, py, splits, R, T, r, t, c, H, gcached ? gc[i] : G[r * T + t], eps,
                                       alpha, newton, renorm, kappa, beta, Ubar, Ybar, Hd, Cbar);
  }
  if (!cache)
    for (int64_t r = rg; r < R; r += BW_RG)
      cand_bwd_entry(pu, puc, py, splits, R, T, r, t, c, H, G[r * T + t], eps, alpha, newton, renorm, kappa, beta,
                     Ubar, Ybar, Hd, Cbar);
}

hipError_t launch_cand_bwd_H(const float* H, const float* pu, const float* puc, const float* py, int splits, const float* c,
                             const double* vpart, int tiles_m, int64_t T, int64_t R, float eps, float alpha,
                             const uint8_t* sel, const float* G, float* Ubar, float* Ybar, float* Hd,
                             float* Cbar, float* sbar, hipStream_t s) {
  prof_begin("cand_bwd_H", s);
  const CandLayout lay = cand_layout(T, R);
  if (lay.cols == 32 && lay.rg == 32)
    hipLaunchKernelGGL((k_cand_bwd_H<32, 32>), dim3((unsigned)cdiv(T, 32)), dim3(1024), 0, s, H, pu, puc, py, splits,
                       c, vpart, tiles_m, T, R, eps, alpha, sel, G, Ubar, Ybar, Hd, Cbar, sbar);
  else if (lay.cols == 32)
    hipLaunchKernelGGL((k_cand_bwd_H<32, 8>), dim3((unsigned)cdiv(T, 32)), dim3(256), 0, s, H, pu, puc, py, splits,
                       c, vpart, tiles_m, T, R, eps, alpha, sel, G, Ubar, Ybar, Hd, Cbar, sbar);
  else
    hipLaunchKernelGGL((k_cand_bwd_H<8, 32>), dim3((unsigned)cdiv(T, 8)), dim3(256), 0, s, H, pu, puc, py, splits,
                       c, vpart, tiles_m, T, R, eps, alpha, sel, G, Ubar, Ybar, Hd, Cbar, sbar);
  prof_end("cand_bwd_H", s);
  return hipGetLastError();
}

// qbar = W ubar, qbbar = (W*W) ybar (MFMA, K = R) and the pointwise chain rule
// through q = v/z, qb = v/z^2.
template <class GZB>
__global__ __launch_bounds__(GZB::NT) void k_zbar(const float* V, const float* Z, Opnd W, Opnd Ub, Opnd Yb,
                                                  const float* sbar, int64_t N, int64_t T, int64_t R,
                                                  float* Zbar, float* dV, int accumulate) {
  using TL = Tile<GZB, ProdDualB_SqA, true, false>;
  __shared__ __align__(16) float lds[TL::LDS_FLOATS];
  const Tile3 tl = xcd_tile_grouped<8>();
  const int64_t m0 = tl.y * GZB::BM, n0 = tl.x * GZB::BN;
  TL t;
  t.zero();
  {
    const Opnd A[1] = {W};
    const Opnd B[2] = {Ub, Yb};
    t.run(A, B, m0, n0, 0, R, lds);
  }
#pragma unroll
  for (int i = 0; i < GZB::FM; ++i)
#pragma unroll
    for (int j = 0; j < GZB::FN; ++j) {
      const int64_t col = TL::col_of(n0, j);
      if (col >= T) continue;
      const float sb = sbar[col];
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = TL::row_of(m0, i, v);
        if (row < N) {
          const int64_t e = row * T + col;
          const float x = V[e], z = Z[e];
          const float qbar = t.acc[i][j][0][v], qbbar = t.acc[i][j][1][v];
          const float iz = 1.f / z;
          const float q = x * iz, qb = q * iz;
          Zbar[e] = -(qbar * q + 2.f * qbbar * qb) * iz;
          const float vb = qbar * iz + qbbar * iz * iz + sb;
          dV[e] = accumulate ? dV[e] + vb : vb;
        }
      }
    }
}

hipError_t launch_zbar(const float* V, const float* Z, const float* W, const float* Ubar, const float* Ybar,
                       const float* sbar, int64_t N, int64_t T, int64_t R, float* Zbar, float* dV, int accumulate,
                       hipStream_t s) {
  const Opnd w = make_opnd(W, R, N);
  const Opnd ub = make_opnd(Ubar, T, T);
  const Opnd yb = make_opnd(Ybar, T, T);
  prof_begin("zbar", s);
  // fewer 128 x 128 tiles than two per CU: 64 x 64 tiles (elementwise outputs,
  // the same sums per entry)
  if (cdiv(T, GZB::BN) * cdiv(N, GZB::BM) < 512) {
    using GS = Geo<64, 64, GEMM_BK, 2, 2>;
    dim3 grid((unsigned)cdiv(T, GS::BN), (unsigned)cdiv(N, GS::BM));
    hipLaunchKernelGGL(k_zbar<GS>, grid, dim3(GS::NT), 0, s, V, Z, w, ub, yb, sbar, N, T, R, Zbar, dV, accumulate);
  } else {
    dim3 grid((unsigned)cdiv(T, GZB::BN), (unsigned)cdiv(N, GZB::BM));
    hipLaunchKernelGGL(k_zbar<GZB>, grid, dim3(GZB::NT), 0, s, V, Z, w, ub, yb, sbar, N, T, R, Zbar, dV, accumulate);
  }
  prof_end("zbar", s);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_dh_final(const float* Hd, const float* pu, int splits, int64_t RT,
                                                  float* Gout) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < RT; e += (int64_t)gridDim.x * 256) {
    float acc = 0.f;
    for (int sp = 0; sp < splits; ++sp) acc += pu[sp * RT + e];
    Gout[e] = Hd[e] + acc;
  }
}

hipError_t launch_dh_final(const float* Hd, const float* pu, int splits, int64_t R, int64_t T, float* Gout,
                           hipStream_t s) {
  const int64_t RT = R * T;
  const unsigned blocks = (unsigned)std::min<int64_t>(cdiv(RT, 256), 8192);
  prof_begin("dh_final", s);
  hipLaunchKernelGGL(k_dh_final, dim3(blocks), dim3(256), 0, s, Hd, pu, splits, RT, Gout);
  prof_end("dh_final", s);
  return hipGetLastError();
}

// W-gradient products: C0 = Q ubar^t + zbar H^t, C1 = Qb ybar^t (contraction over T).
struct ProdWbar {
  static constexpr int NA = 3, NB = 3, NC = 2;
  __device__ __forceinline__ static void mma(const float (&a)[3], const float (&b)[3], f32x16 (&c)[2]) {
    c[0] = mfma32(a[0], b[0], c[0]);
    c[0] = mfma32(a[1], b[1], c[0]);
    c[1] = mfma32(a[2], b[2], c[1]);
  }
};

__global__ __launch_bounds__(GWB::NT) void k_wbar(Opnd Q, Opnd Zb, Opnd Qb, Opnd Ub, Opnd H, Opnd Yb, int64_t N,
                                                  int64_t T, int64_t R, int64_t kchunk, float* p0, float* p1) {
  using TL = Tile<GWB, ProdWbar, true, true>;
  __shared__ __align__(16) float lds[TL::LDS_FLOATS];
  const Tile3 tl = xcd_tile_grouped<8>();
  const int64_t m0 = tl.y * GWB::BM, n0 = tl.x * GWB::BN;
  const int64_t sp = tl.z;
  const int64_t k0 = sp * kchunk, k1 = std::min<int64_t>(T, k0 + kchunk);
  TL t;
  t.zero();
  {
    const Opnd A[3] = {Q, Zb, Qb};
    const Opnd B[3] = {Ub, H, Yb};
    t.run(A, B, m0, n0, k0, k1, lds);
  }
  float* d0 = p0 + sp * N * R;
  float* d1 = p1 + sp * N * R;
#pragma unroll
  for (int i = 0; i < GWB::FM; ++i)
#pragma unroll
    for (int j = 0; j < GWB::FN; ++j) {
      const int64_t col = TL::col_of(n0, j);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int64_t row = TL::row_of(m0, i, v);
        if (row < N && col < R) {
          d0[row * R + col] = t.acc[i][j][0][v];
          d1[row * R + col] = t.acc[i][j][1][v];
        }
      }
    }
}

hipError_t launch_wbar(const float* Q, const float* Zbar, const float* Qb, const float* Ubar, const float* H,
                       const float* Ybar, int64_t N, int64_t T, int64_t R, int splits, int64_t kchunk, float* p0,
                       float* p1, hipStream_t s) {
  dim3 grid((unsigned)cdiv(R, GWB::BN), (unsigned)cdiv(N, GWB::BM), (unsigned)splits);
  const Opnd q = make_opnd(Q, T, N), zb = make_opnd(Zbar, T, N), qb = make_opnd(Qb, T, N);
  const Opnd ub = make_opnd(Ubar, T, R), h = make_opnd(H, T, R), yb = make_opnd(Ybar, T, R);
  prof_begin("wbar", s);
  hipLaunchKernelGGL(k_wbar, grid, dim3(GWB::NT), 0, s, q, zb, qb, ub, h, yb, N, T, R, kchunk, p0, p1);
  prof_end("wbar", s);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_dw_final(const float* W, const float* p0, const float* p1, int splits,
                                                  const double* cbar, int64_t N, int64_t R, float* dW,
                                                  int accumulate) {
  const int64_t NR = N * R;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < NR; e += (int64_t)gridDim.x * 256) {
    float a0 = 0.f, a1 = 0.f;
    for (int sp = 0; sp < splits; ++sp) {
      a0 += p0[sp * NR + e];
      a1 += p1[sp * NR + e];
    }
    const float g = a0 + 2.f * W[e] * a1 + (float)cbar[e % R];
    dW[e] = accumulate ? dW[e] + g : g;
  }
}

hipError_t launch_dw_final(const float* W, const float* p0, const float* p1, int splits, const double* cbar,
                           int64_t N, int64_t R, float* dW, int accumulate, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<int64_t>(cdiv(N * R, 256), 8192);
  prof_begin("dw_final", s);
  hipLaunchKernelGGL(k_dw_final, dim3(blocks), dim3(256), 0, s, W, p0, p1, splits, cbar, N, R, dW, accumulate);
  prof_end("dw_final", s);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_copy(const float* src, float* dst, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = src[e];
}

hipError_t launch_copy(const float* src, float* dst, int64_t n, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<int64_t>(cdiv(n, 256), 8192);
  prof_begin("copy", s);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, src, dst, n);
  prof_end("copy", s);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill(float* dst, float value, int64_t n) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) dst[e] = value;
}

hipError_t launch_fill(float* dst, float value, int64_t n, hipStream_t s) {
  const unsigned blocks = (unsigned)std::min<int64_t>(cdiv(n, 256), 8192);
  prof_begin("fill", s);
  hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, dst, value, n);
  prof_end("fill", s);
  return hipGetLastError();
}

}  // namespace dna
