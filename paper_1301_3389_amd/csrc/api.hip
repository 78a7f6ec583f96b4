// api.hip -- the C ABI of libdna (declared in include/dna.h): argument checks,
// workspace carving and the kernel sequence of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dna.h"
#include "kernels.hpp"
#include "kernels_16.hpp"
#include "kernels_adj.hpp"
#include "kernels_sparse.hpp"

namespace dna {

// ---------------------------------------------------------------------------
// Error text and kernel timing.
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";

static dna_status fail(dna_status s, const char* msg) {
  std::snprintf(g_err, sizeof(g_err), "%s", msg);
  return s;
}
static dna_status hip_fail(hipError_t e, const char* where) {
  std::snprintf(g_err, sizeof(g_err), "%s: %s", where, hipGetErrorString(e));
  return DNA_EHIP;
}

struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
static std::mutex g_prof_mu;
static bool g_prof = false;
static std::vector<ProfRec> g_pending;
static std::vector<hipEvent_t> g_pool;
static std::map<std::string, std::pair<int64_t, double>> g_stats;
static std::vector<std::string> g_names;   // stable storage for returned names

static hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void prof_begin(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof) return;
  hipEvent_t a = take_event();
  if (!a) return;
  hipEventRecord(a, s);
  g_pending.push_back({name, a, nullptr});
}

void prof_end(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_prof || g_pending.empty() || g_pending.back().b != nullptr) return;
  hipEvent_t b = take_event();
  if (!b) return;
  hipEventRecord(b, s);
  g_pending.back().b = b;
  (void)name;
}

// ---------------------------------------------------------------------------
// Workspace layout (one layout serves every forward entry point).
// ---------------------------------------------------------------------------
constexpr int64_t MIN_KCHUNK = 256;    // never split the contraction finer than this

struct Split {
  int splits;
  int64_t kchunk;
};

// Split-K for a product of base_tiles output tiles of which `slots` workgroups
// run at once (CUs x workgroups per CU): the split whose rounds of resident
// workgroups, each worth one chunk (plus a fixed epilogue of about 64
// contraction indices), take the least time; ties go to fewer splits (less
// partial traffic).  Chunks are multiples of `align` and at least MIN_KCHUNK
// long.  A tile count just above a multiple of `slots` would otherwise run a
// nearly empty last round.
static Split wave_split(int64_t K, int64_t base_tiles, int64_t slots, int64_t align) {
  const int64_t base = std::max<int64_t>(1, base_tiles);
  const int64_t max_sp = std::min<int64_t>(1024, std::max<int64_t>(1, K / MIN_KCHUNK));
  Split best{1, std::max<int64_t>(1, cdiv(K, align)) * align};
  if (K <= 0) return best;
  int64_t best_cost = INT64_MAX;
  for (int64_t sp = 1; sp <= max_sp; ++sp) {
    const int64_t kchunk = cdiv(cdiv(K, sp), align) * align;
    const int64_t real = cdiv(K, kchunk);
    if (real != sp) continue;
    const int64_t cost = cdiv(base * real, slots) * (kchunk + 64);
    if (cost < best_cost) {
      best_cost = cost;
      best.splits = (int)real;
      best.kchunk = kchunk;
    }
  }
  return best;
}

// Chunks of the fused kernels along the contraction (multiples of 64), aiming
// at two workgroups per CU.
static Split fused_split(int64_t K, int64_t base_tiles) {
  int64_t sp = std::max<int64_t>(1, cdiv(2 * 256, std::max<int64_t>(1, base_tiles)));
  sp = std::min<int64_t>(sp, cdiv(K, 64));
  Split s;
  s.kchunk = cdiv(cdiv(K, sp), 64) * 64;
  s.splits = (int)cdiv(K, s.kchunk);
  return s;
}

// Chunks for a fused kernel of which `per_cu` workgroups fit on a CU: all
// workgroups resident at once, and the busiest CU's work (workgroups per CU x
// 64-row sub-tiles per workgroup) as small as possible; on a tie, more
// workgroups.
static Split balanced_split(int64_t K, int64_t base_tiles, int64_t per_cu) {
  const int64_t k64 = std::max<int64_t>(1, cdiv(K, 64)), base = std::max<int64_t>(1, base_tiles);
  int64_t best_per = k64, best_load = INT64_MAX;
  for (int64_t sp = 1; sp <= k64; ++sp) {
    const int64_t per = cdiv(k64, sp);                    // sub-tiles per workgroup
    const int64_t wgs = base * cdiv(k64, per);
    const int64_t on_cu = cdiv(wgs, 256);
    if (on_cu > per_cu && sp > 1) break;                  // wgs only grows with sp
    if (on_cu * per <= best_load) {
      best_load = on_cu * per;
      best_per = per;
    }
  }
  Split s;
  s.kchunk = best_per * 64;
  s.splits = (int)cdiv(K, s.kchunk);
  return s;
}

struct Layout {
  Split sh, sw;              // split-K of the fp32 gradient products (H / W orientation)
  Split sh16, sw16;          // the same for the 16-bit products (128 x 128 tiles)
  Split shf, swf;            // row / column chunks of the fused kernels (R <= FUSED_MAX_R)
  Split chf;                 // row chunks of the fused H-orientation cost pass (three workgroups per CU fit)
  int rt_m, rt_n;            // ratio-pass tiles along N and along T
  int ch_m, cw_n;            // cost-pass tiles along N (H orientation) / T (W orientation)
  size_t q, qb, pu, puc, py, xmu, xn, c32, c64, sump, sump2, sume, vpart, dpart, cpart, fpart, s16, cs, zd, dz, selm,
      check, total;
};

static size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

// Q and Q-bar (N x T fp32 each) are carved only where a kernel reads them: Q
// for the tiled fp32 products (DNA and MU) when R > FUSED_MAX_R, Q-bar for the
// tiled fp32 DNA products, and both for the unrolled adjoint (`adj`).  The
// 16-bit forms keep their 16-bit Q, Q - 1 and Q-bar in their own scratch.
static Layout make_layout(int64_t N, int64_t T, int64_t R, bool with16, bool adj = false) {
  Layout L;
  // the fp32 gradient products run two workgroups per CU
  L.sh = wave_split(N, cdiv(T, GH_BN) * cdiv(R, GH_BM), 2 * 256, GH_CHUNK);
  L.sw = wave_split(T, cdiv(R, GW_BN) * cdiv(N, GW_BM), 2 * 256, GH_CHUNK);
  L.sh16 = wave_split(N, cdiv(T, 128) * cdiv(R, 128), GH16_WG_PER_CU * 256, 32);
  L.sw16 = wave_split(T, cdiv(R, 128) * cdiv(N, 128), GH16_WG_PER_CU * 256, 32);
  L.shf = fused_split(N, cdiv(T, 64));
  L.swf = fused_split(T, cdiv(N, 64));
  L.chf = balanced_split(N, cdiv(T, 64), 3);
  L.rt_m = (int)cdiv(N, ratio_tile_rows(N, T));
  L.rt_n = (int)cdiv(T, RT_BN);
  L.ch_m = (int)cdiv(N, cost_h_tile_rows(N, T));
  L.cw_n = (int)cdiv(T, CW_BN);
  const size_t nt = (size_t)N * T, fac = (size_t)std::max(R * T, N * R);
  const int64_t sph = std::max({L.sh.splits, L.sh16.splits, L.shf.splits});
  const int64_t spw = std::max({L.sw.splits, L.sw16.splits, L.swf.splits});
  const size_t psplit = (size_t)std::max<int64_t>(sph * R * T, spw * N * R);
  const size_t red = (size_t)std::max({(int64_t)L.rt_m * T, (int64_t)L.rt_n * N, (int64_t)L.ch_m * T,
                                       (int64_t)L.cw_n * N, sph * T, (int64_t)L.chf.splits * T, spw * N});
  const size_t klt = (size_t)L.rt_m * L.rt_n;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  const bool tiled = R > FUSED_MAX_R;
  L.q = take((adj || tiled) ? nt * 4 : 0);
  L.qb = take((adj || (tiled && !with16)) ? nt * 4 : 0);
  L.pu = take(psplit * 4);
  L.puc = take(psplit * 4);
  L.py = take(psplit * 4);
  L.xmu = take(fac * 4);
  L.xn = take(fac * 4);
  L.c32 = take((size_t)R * 4);
  L.c64 = take((size_t)R * 8);
  L.sump = take((size_t)SUM_PARTS * R * 8);
  L.sump2 = take((size_t)SUM_PARTS * R * 8);          // the other factor's parts (eq. 2 normalisation, penalty)
  // sums emitted by the normalisation for the next half-step (dna_iterate)
  L.sume = take((size_t)std::max(scale_emit_parts(0, N, T), scale_emit_parts(1, N, T)) * R * 8);
  L.vpart = take(red * 8);
  L.dpart = take(R <= FUSED_MAX_R ? red * 8 : 0);     // input-state costs of the damped selection
  L.cpart = take(std::max(3 * red, klt) * 8);
  L.fpart = take(red * 4);
  L.s16 = take(with16 ? scratch16_bytes(N, T, R) : 0);
  // chunk sums of the fixed factor for the tiled fp32 gradient products
  L.cs = take((adj || (tiled && !with16)) ? (size_t)std::max(cdiv(N, GH_CHUNK), cdiv(T, GH_CHUNK)) * cdiv(R, 64) * 64 * 4
                                           : 0);
  // Z_DNA, dZ and the selection a cost pass leaves for the next ratio pass (dna_iterate, tiled fp32)
  const bool carry = tiled && !with16 && !adj;
  L.zd = take(carry ? nt * 4 : 0);
  L.dz = take(carry ? nt * 4 : 0);
  L.selm = take(carry ? (size_t)std::max(N, T) : 0);
  L.check = take(16);
  L.total = off;
  return L;
}

// The adjoint needs the forward layout plus Z, Z-bar, the per-entry adjoint
// quantities, two ping-pong H-gradients and the W-gradient split partials.
struct AdjLayout {
  Layout base;
  Split swb;
  size_t z, zbar, ubar, ybar, hd, cbar, g0, g1, sbar, cbar64, wp0, wp1, total;
};

static AdjLayout make_adj_layout(int64_t N, int64_t T, int64_t R) {
  AdjLayout A;
  A.base = make_layout(N, T, R, false, true);
  A.swb = wave_split(T, cdiv(R, WB_BN) * cdiv(N, WB_BM), 3 * 256, 32);   // three k_wbar workgroups fit a CU
  size_t off = A.base.total;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  const size_t nt = (size_t)N * T, rt = (size_t)R * T, nr = (size_t)N * R;
  A.z = take(nt * 4);
  A.zbar = take(nt * 4);
  A.ubar = take(rt * 4);
  A.ybar = take(rt * 4);
  A.hd = take(rt * 4);
  A.cbar = take(rt * 4);
  A.g0 = take(rt * 4);
  A.g1 = take(rt * 4);
  A.sbar = take((size_t)T * 4);
  A.cbar64 = take((size_t)R * 8);
  A.wp0 = take((size_t)A.swb.splits * nr * 4);
  A.wp1 = take((size_t)A.swb.splits * nr * 4);
  A.total = off;
  return A;
}

template <class T>
static T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// ---------------------------------------------------------------------------
// Argument checks.
// ---------------------------------------------------------------------------
static dna_status check_opts(const dna_opts* o) {
  if (!o) return fail(DNA_EINVAL, "opts is NULL");
  if (!(o->eps >= 0.f && o->eps <= 1.f)) return fail(DNA_EINVAL, "eps must lie in [0, 1]");
  if (!(o->alpha > 0.f) || !std::isfinite(o->alpha)) return fail(DNA_EINVAL, "alpha must be finite and > 0");
  if (o->gemm < DNA_GEMM_FP32 || o->gemm > DNA_GEMM_FP16) return fail(DNA_EINVAL, "unknown gemm type");
  if (!(o->rho >= 0.f) || !std::isfinite(o->rho) || !(o->lambda >= 0.f) || !std::isfinite(o->lambda))
    return fail(DNA_EINVAL, "rho and lambda must be finite and >= 0");
  if (o->select != DNA_SELECT_BOTH && o->select != DNA_SELECT_NEWTON_FIRST)
    return fail(DNA_EINVAL, "unknown selection rule");
  return DNA_OK;
}

// The damped selection runs on the fused fp32 path (R <= FUSED_MAX_R).
static dna_status check_select(const dna_opts* o, int64_t R) {
  if (o->select == DNA_SELECT_NEWTON_FIRST && (o->gemm != DNA_GEMM_FP32 || R > FUSED_MAX_R))
    return fail(DNA_EUNSUPPORTED, "DNA_SELECT_NEWTON_FIRST runs with FP32 products and R <= 64 only");
  return DNA_OK;
}
static dna_status check_select_both(const dna_opts* o) {
  if (o->select != DNA_SELECT_BOTH) return fail(DNA_EUNSUPPORTED, "this call supports DNA_SELECT_BOTH only");
  return DNA_OK;
}

static dna_status check_dims(int64_t N, int64_t T, int64_t R) {
  if (N <= 0 || T <= 0 || R <= 0) return fail(DNA_EINVAL, "N, T and R must be positive");
  if (cdiv(N, CW_BM) > 65535 || cdiv(R, GH_BM) > 65535)
    return fail(DNA_EUNSUPPORTED, "N or R exceeds the launch grid limit");
  if ((double)N * (double)T > 4.0e9 || (double)N * (double)R > 4.0e9 || (double)R * (double)T > 4.0e9)
    return fail(DNA_EUNSUPPORTED, "matrix too large (more than 4e9 entries)");
  return DNA_OK;
}

static dna_status check_aux(const void* aux, size_t aux_bytes, size_t need) {
  if (aux_bytes < need) return fail(DNA_EWORKSPACE, "kept-sums buffer smaller than dna_unrolled_aux_bytes()");
  if ((reinterpret_cast<uintptr_t>(aux) & 255) != 0) return fail(DNA_EINVAL, "kept-sums buffer must be 256-byte aligned");
  return DNA_OK;
}

static dna_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (!ws) return fail(DNA_EINVAL, "workspace is NULL");
  if (ws_bytes < need) return fail(DNA_EWORKSPACE, "workspace smaller than dna_workspace_bytes()");
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0) return fail(DNA_EINVAL, "workspace must be 256-byte aligned");
  return DNA_OK;
}

#define DNA_TRY(expr)                              \
  do {                                             \
    dna_status _s = (expr);                        \
    if (_s != DNA_OK) return _s;                   \
  } while (0)
#define DNA_HIP(expr, where)                       \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

__global__ void k_zero_int(int* p) { *p = 0; }

// Checked mode: clear the flag word and scan the inputs.
static dna_status checked_begin(int* chk, const float* const* bufs, const int64_t* sizes, int nb,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, s, chk);
  DNA_HIP(hipGetLastError(), "check flag reset");
  for (int i = 0; i < nb; ++i) DNA_HIP(launch_check(bufs[i], sizes[i], chk, s), "input check");
  return DNA_OK;
}

static dna_status checked_end(int* chk, hipStream_t s) {
  int h = 0;
  DNA_HIP(hipMemcpyAsync(&h, chk, sizeof(int), hipMemcpyDeviceToHost, s), "check flag read-back");
  DNA_HIP(hipStreamSynchronize(s), "checked-mode synchronise");
  if (h & CHK_NONFINITE) return fail(DNA_ENONFINITE, "non-finite entry in an input");
  if (h & CHK_DOMAIN) return fail(DNA_EDOMAIN, "negative entry, zero W column / H row sum, or z = 0 where v > 0");
  return DNA_OK;
}

// ---------------------------------------------------------------------------
// Shared stages.
// The 16-bit path's operands, 16-bit Q, Q - 1, Q-bar and scale buffers.
static Scratch16 scratch16(void* ws, const Layout& L, int64_t N, int64_t T, int64_t R) {
  return scratch16_carve(at<char>(ws, L.s16), N, T, R);
}

// ---------------------------------------------------------------------------
// side 0: candidates for H (R x T) given W;  side 1: candidates for W (N x R) given H.
// `pre`, if given, holds the first level of c (side 0) / g (side 1) already
// written by the preceding normalisation; otherwise a sum kernel writes it.
// `carry`: inside dna_iterate on the tiled fp32 path, Z of the current state is
// taken from the preceding half-step's cost pass (Algorithm 1 steps 15, 28)
// instead of being formed again from W H.
// Where the H step of the tiled fp32 path (R > 64) leaves Z, Q, Q-bar, the
// split partials of u, u_c, y and the V column sums, for an adjoint that reads
// them instead of recomputing them (the unrolled forward's kept sums).
struct AuxOut {
  float* Z;
  float* Q;
  float* Qb;
  float* pu;
  float* puc;
  float* py;
  double* vpart;
};

static dna_status run_candidates(int side, const float* V, const float* W, const float* H, int64_t N,
                                 int64_t T, int64_t R, const dna_opts* o, const Layout& L, void* ws,
                                 float* Xmu, float* Xn, float* Aout, float* Bout, int* chk, hipStream_t s,
                                 const SumJob* pre = nullptr, bool carry = false, const AuxOut* aux = nullptr,
                                 bool qmax16 = false) {
  const bool keep_sums = aux && side == 0 && o->gemm == DNA_GEMM_FP32 && R > FUSED_MAX_R && !carry;
  float* Q = keep_sums ? aux->Q : at<float>(ws, L.q);
  float* Qb = keep_sums ? aux->Qb : at<float>(ws, L.qb);
  float* pu = keep_sums ? aux->pu : at<float>(ws, L.pu);
  float* puc = keep_sums ? aux->puc : at<float>(ws, L.puc);
  float* py = keep_sums ? aux->py : at<float>(ws, L.py);
  float* c32 = at<float>(ws, L.c32);
  double* c64 = at<double>(ws, L.c64);
  double* vpart = keep_sums ? aux->vpart : at<double>(ws, L.vpart);
  RatioArgs ra{V, W, H, N, T, R, Q, Qb, vpart, nullptr, chk, keep_sums ? aux->Z : nullptr};
  if (carry) {
    ra.carry.zd = at<float>(ws, L.zd);
    ra.carry.dz = at<float>(ws, L.dz);
    ra.carry.sel = at<uint8_t>(ws, L.selm);
  }
  const bool p16 = o->gemm != DNA_GEMM_FP32;
  const Scratch16 S = scratch16(ws, L, N, T, R);
  SumJob job;
  if (side == 0) {
    if (pre) job = *pre;
    else DNA_HIP(launch_colsum_part(W, N, R, at<double>(ws, L.sump), job, s), "colsum_W");
    job.s64 = c64; job.s32 = c32; job.check = chk; job.reg = o->lambda;
    ra.fin = job;                                   // c = W^t 1 (+ lambda) finished inside the ratio pass
    const bool fused = !p16 && R <= FUSED_MAX_R;
    if (p16) {
      DNA_HIP(launch_ratio_gh16(o->gemm, 0, V, W, H, N, T, R, S, L.sh16.splits, L.sh16.kchunk, pu, puc, py,
                                vpart, chk, job, s, qmax16), "ratio_gh16_H");
    } else if (fused) {
      const bool damp = o->select == DNA_SELECT_NEWTON_FIRST;
      DNA_HIP(launch_rgh(0, V, W, H, N, T, R, L.shf.splits, L.shf.kchunk, pu, puc, py, vpart, job, chk, s,
                         damp ? RGH_DNA_COST : RGH_DNA, damp ? at<double>(ws, L.dpart) : nullptr), "rgh_H");
    } else {
      float* cs = at<float>(ws, L.cs);
      DNA_HIP(launch_ratio(carry ? RM_H_CARRY : (keep_sums ? RM_ADJ : RM_H), ra, s), "ratio_H");
      if (N >= GH_CHUNK_MIN_K) DNA_HIP(launch_chunk_sums(0, W, N, T, R, cs, s), "chunk_sums_W");
      DNA_HIP(launch_gh_H(W, Q, Qb, N >= GH_CHUNK_MIN_K ? cs : nullptr, N, T, R, L.sh.splits, L.sh.kchunk, pu, puc,
                          py, s), "gh_H");
    }
    // the 16-bit Z pass tiles N by 128
    int sp = p16 ? L.sh16.splits : (fused ? L.shf.splits : L.sh.splits);
    const int tiles = p16 ? (int)cdiv(N, 128) : (fused ? L.shf.splits : L.rt_m);
    if (sp > 8 && T < 256 * 32) {                   // few column blocks, many splits: fold them first
      DNA_HIP(launch_fold_splits(pu, puc, py, sp, R * T, s), "fold_splits");
      sp = 1;
    }
    DNA_HIP(launch_cand_H(H, pu, puc, py, sp, c32, vpart, tiles, T, R, o->eps, o->alpha,
                          o->lambda, Xmu, Xn, Aout, Bout, s), "cand_H");
  } else {
    if (pre) job = *pre;
    else DNA_HIP(launch_rowsum_part(H, T, R, at<double>(ws, L.sump), job, s), "rowsum_H");
    job.s64 = c64; job.s32 = c32; job.check = chk; job.reg = o->rho;
    ra.fin = job;                                   // g = H 1 (+ rho) finished inside the ratio pass
    const bool fused = !p16 && R <= FUSED_MAX_R;
    if (p16) {
      DNA_HIP(launch_ratio_gh16(o->gemm, 1, V, W, H, N, T, R, S, L.sw16.splits, L.sw16.kchunk, pu, puc, py,
                                vpart, chk, job, s, qmax16), "ratio_gh16_W");
    } else if (fused) {
      const bool damp = o->select == DNA_SELECT_NEWTON_FIRST;
      DNA_HIP(launch_rgh(1, V, W, H, N, T, R, L.swf.splits, L.swf.kchunk, pu, puc, py, vpart, job, chk, s,
                         damp ? RGH_DNA_COST : RGH_DNA, damp ? at<double>(ws, L.dpart) : nullptr), "rgh_W");
    } else {
      float* cs = at<float>(ws, L.cs);
      DNA_HIP(launch_ratio(carry ? RM_W_CARRY : RM_W, ra, s), "ratio_W");
      if (T >= GH_CHUNK_MIN_K) DNA_HIP(launch_chunk_sums(1, H, N, T, R, cs, s), "chunk_sums_H");
      DNA_HIP(launch_gh_W(Q, Qb, H, T >= GH_CHUNK_MIN_K ? cs : nullptr, N, T, R, L.sw.splits, L.sw.kchunk, pu, puc,
                          py, s), "gh_W");
    }
    // the 16-bit Z pass tiles T by 128, the fp32 one by RT_BN
    const int sp = p16 ? L.sw16.splits : (fused ? L.swf.splits : L.sw.splits);
    const int tiles = p16 ? (int)cdiv(T, 128) : (fused ? L.swf.splits : L.rt_n);
    DNA_HIP(launch_cand_W(W, pu, puc, py, sp, c32, vpart, tiles, N, R, o->eps, o->alpha, o->rho, Xmu, Xn, Aout,
                          Bout, s), "cand_W");
  }
  return DNA_OK;
}

// `keep`: the cost pass also stores Z_DNA and dZ, and the selection is written to
// the workspace mask when the caller wants none, for the next half-step's
// carried Z (tiled fp32 path only).
// `fresh` (W step): the selection also leaves the first level of the column
// sums of the new W (in the pu buffer, whose split partials the candidates have
// consumed) for the normalisation that follows.
// `qmax16` (FP16): the cost pass also leaves bounds of the next half-step's Q
// maxima, which that half-step's Z pass then takes instead of a maxima pass.
static dna_status run_select(int side, const float* V, const float* F, const float* Xmu, const float* Xn,
                             float* Xout, int64_t N, int64_t T, int64_t R, const dna_opts* o, const Layout& L,
                             void* ws, uint8_t* mask, double* dsel, double* margin, hipStream_t s,
                             bool keep = false, SumJob* fresh = nullptr, bool qmax16 = false) {
  double* emit = fresh ? at<double>(ws, L.pu) : nullptr;
  float* zd = keep ? at<float>(ws, L.zd) : nullptr;
  float* dz = keep ? at<float>(ws, L.dz) : nullptr;
  // the choice reads the margin and the flags only; the kept candidate's cost
  // (the sum_N partials) is formed only when the caller asks for d_sel
  const bool s0 = dsel != nullptr;
  if (keep) mask = at<uint8_t>(ws, L.selm);
  double* cpart = at<double>(ws, L.cpart);
  int* fpart = at<int>(ws, L.fpart);
  if (o->gemm != DNA_GEMM_FP32) {
    DNA_HIP(launch_cost16(o->gemm, side, V, F, Xmu, Xn, N, T, R, scratch16(ws, L, N, T, R), cpart, fpart, s, s0,
                          qmax16), "cost16");
    if (side == 0)
      DNA_HIP(launch_select_H(Xmu, Xn, Xout, cpart, fpart, (int)cdiv(N, 128), T, R, mask, dsel, margin, s),
              "select_H");   // the 16-bit cost pass tiles N by 128
    else {
      DNA_HIP(launch_select_W(Xmu, Xn, Xout, cpart, fpart, (int)cdiv(T, 128), N, R, mask, dsel, margin, s, Damp{},
                              emit), "select_W");
      if (fresh) *fresh = SumJob{emit, select_w_parts((int)cdiv(T, 128), N), R};
    }
    return DNA_OK;
  }
  const bool fused = R <= FUSED_MAX_R;   // candidates' block resident in LDS
  // the damped selection: the Newton candidate's cost against the input
  // state's (its cost parts from the fused ratio pass; Xout holds that state)
  const bool damp = o->select == DNA_SELECT_NEWTON_FIRST;
  Damp dp;
  if (damp) {
    dp.dpart = at<double>(ws, L.dpart);
    dp.vpart = at<double>(ws, L.vpart);
    dp.dtiles = dp.vtiles = side == 0 ? L.shf.splits : L.swf.splits;
    dp.c64 = at<double>(ws, L.c64);
    dp.reg = side == 0 ? o->lambda : o->rho;
  }
  if (side == 0) {
    if (fused)
      DNA_HIP(launch_costf(0, V, F, Xmu, Xn, N, T, R, L.chf.splits, L.chf.kchunk, cpart, fpart, s, damp, s0),
              "costf_H");
    else
      DNA_HIP(launch_cost_H(V, F, Xmu, Xn, N, T, R, cpart, fpart, s, zd, dz, s0), "cost_H");
    DNA_HIP(launch_select_H(Xmu, Xn, Xout, cpart, fpart, fused ? L.chf.splits : L.ch_m, T, R, mask, dsel, margin,
                            s, dp), "select_H");
  } else {
    if (fused)
      DNA_HIP(launch_costf(1, V, F, Xmu, Xn, N, T, R, L.swf.splits, L.swf.kchunk, cpart, fpart, s, damp, s0),
              "costf_W");
    else
      DNA_HIP(launch_cost_W(V, F, Xmu, Xn, N, T, R, cpart, fpart, s, zd, dz, s0), "cost_W");
    const int tiles = fused ? L.swf.splits : L.cw_n;
    DNA_HIP(launch_select_W(Xmu, Xn, Xout, cpart, fpart, tiles, N, R, mask, dsel, margin, s, dp, emit),
            "select_W");
    if (fresh) *fresh = SumJob{emit, select_w_parts(tiles, N), R};
  }
  return DNA_OK;
}

struct Common {
  Layout L;
  int* chk;
  hipStream_t s;
};

static dna_status prologue(const float* V, const float* W, const float* H, int64_t N, int64_t T, int64_t R,
                           const dna_opts* o, void* ws, size_t ws_bytes, void* stream, Common& c) {
  DNA_TRY(check_dims(N, T, R));
  DNA_TRY(check_opts(o));
  c.L = make_layout(N, T, R, o->gemm != DNA_GEMM_FP32);
  DNA_TRY(check_ws(ws, ws_bytes, c.L.total));
  c.s = static_cast<hipStream_t>(stream);
  c.chk = o->checked ? at<int>(ws, c.L.check) : nullptr;
  if (c.chk) {
    const float* bufs[3] = {W, H, V};
    const int64_t sizes[3] = {N * R, R * T, N * T};
    DNA_TRY(checked_begin(c.chk, bufs, sizes, V ? 3 : 2, c.s));
  }
  return DNA_OK;
}

static dna_status epilogue(const Common& c) {
  if (c.chk) return checked_end(c.chk, c.s);
  return DNA_OK;
}

// Algorithm 1 steps 1, 16, 29 under the eq. 2 weights: the form `side` names
// when rho = lambda = 0 or both are positive (then the balanced scale, whose
// factors either form applies), else the unit sums of the unpenalised factor
// (W columns when only lambda > 0, H rows when only rho > 0).
static int norm_side(const dna_opts* o, int side) {
  const bool r = o->rho > 0.f, l = o->lambda > 0.f;
  if (r != l) return l ? 0 : 1;
  return side;
}

// One normalisation.  sump / sump2: SUM_PARTS x R doubles each.
// With `emit`, the scale kernel also leaves the first level of the sums of the
// factor of side norm_side(o, side) in `emitted` (W column sums for 0, H row
// sums for 1).
static dna_status run_normalize(int side, float* W, float* H, int64_t N, int64_t T, int64_t R, const dna_opts* o,
                                double* sump, double* sump2, int* chk, hipStream_t s, double* emit,
                                SumJob* emitted, const SumJob* fresh = nullptr) {
  const int es = norm_side(o, side);
  SumJob cj, gj;
  // `fresh`: first-level sums of the factor the half-step just wrote (H row
  // sums after an H step, side 1), left by that step's kernel
  const bool fh = fresh && side == 1, fw = fresh && side == 0;
  if (o->rho > 0.f && o->lambda > 0.f) {          // balanced: the scale kernel takes both factors' sums
    if (fw) cj = *fresh;
    else DNA_HIP(launch_colsum_part(W, N, R, sump, cj, s), "colsum_W");
    if (fh) gj = *fresh;
    else DNA_HIP(launch_rowsum_part(H, T, R, sump2, gj, s), "rowsum_H");
    SumJob& mine = es == 0 ? cj : gj;
    mine.check = chk;
    DNA_HIP(launch_scale(es, W, H, N, T, R, mine, emit, emitted, s, es == 0 ? gj : cj,
                         es == 0 ? o->rho : o->lambda, es == 0 ? o->lambda : o->rho), "scale");
    return DNA_OK;
  }
  SumJob& job = es == 0 ? cj : gj;
  if (es == 0 && fw) job = *fresh;
  else if (es == 1 && fh) job = *fresh;
  else if (es == 0) DNA_HIP(launch_colsum_part(W, N, R, sump, job, s), "colsum_W");
  else DNA_HIP(launch_rowsum_part(H, T, R, sump, job, s), "rowsum_H");
  job.check = chk;
  DNA_HIP(launch_scale(es, W, H, N, T, R, job, emit, emitted, s), "scale");
  return DNA_OK;
}

// Adds rho sum w + lambda sum h to out[0] when either weight is positive.
static dna_status add_penalty(const float* W, const float* H, int64_t N, int64_t T, int64_t R, const dna_opts* o,
                              double* sump, double* sump2, double* out, hipStream_t s) {
  if (!(o->rho > 0.f) && !(o->lambda > 0.f)) return DNA_OK;
  SumJob cj, gj;
  DNA_HIP(launch_colsum_part(W, N, R, sump, cj, s), "colsum_W");
  DNA_HIP(launch_rowsum_part(H, T, R, sump2, gj, s), "rowsum_H");
  DNA_HIP(launch_penalty(cj, gj, o->rho, o->lambda, out, s), "penalty");
  return DNA_OK;
}

}  // namespace dna

using namespace dna;

// ---------------------------------------------------------------------------
// Exported entry points.
// ---------------------------------------------------------------------------
extern "C" {

void dna_default_opts(dna_opts* o) {
  if (!o) return;
  o->eps = 0.01f;
  o->alpha = 4.0f;
  o->gemm = DNA_GEMM_FP32;
  o->checked = 0;
  o->rho = 0.f;
  o->lambda = 0.f;
  o->select = DNA_SELECT_BOTH;
}

size_t dna_workspace_bytes(int64_t N, int64_t T, int64_t R, const dna_opts* o) {
  if (N <= 0 || T <= 0 || R <= 0) return 0;
  return make_layout(N, T, R, o && o->gemm != DNA_GEMM_FP32).total;
}

dna_status dna_normalize(int side, float* W, float* H, int64_t N, int64_t T, int64_t R, const dna_opts* o,
                         void* ws, size_t ws_bytes, void* stream) {
  if (!W || !H) return fail(DNA_EINVAL, "W or H is NULL");
  if (side != 0 && side != 1) return fail(DNA_EINVAL, "side must be 0 or 1");
  Common c;
  DNA_TRY(prologue(nullptr, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  DNA_TRY(run_normalize(side, W, H, N, T, R, o, at<double>(ws, c.L.sump), at<double>(ws, c.L.sump2), c.chk, c.s,
                        nullptr, nullptr));
  return epilogue(c);
}

// The H half-step as one kernel (R <= 64, float32 products, the selection of
// Algorithm 1, T >= HCOLS_MIN_T): candidates, costs and choice per block of
// columns, no split partials.  `fresh` receives the partial row sums of the new
// H (in the pu buffer, which the next W step overwrites only after the
// normalisation has read them).
static bool hcols_path(const dna_opts* o, int64_t T, int64_t R) {
  return o->gemm == DNA_GEMM_FP32 && R <= FUSED_MAX_R && o->select == DNA_SELECT_BOTH && T >= HCOLS_MIN_T &&
         T <= HCOLS_MAX_T;
}

static dna_status run_hstep_cols(const float* V, const float* W, float* H, int64_t N, int64_t T, int64_t R,
                                 const dna_opts* o, const Common& c, void* ws, const SumJob* pre, uint8_t* mask,
                                 double* dsel, double* margin, SumJob* fresh) {
  SumJob job;
  if (pre) job = *pre;
  else DNA_HIP(launch_colsum_part(W, N, R, at<double>(ws, c.L.sump), job, c.s), "colsum_W");
  job.reg = o->lambda;
  const HColsArgs a{V, W, H, N, T, R, job, o->eps, o->alpha, mask, dsel, margin, at<double>(ws, c.L.pu), c.chk};
  DNA_HIP(launch_hstep_cols(a, c.s), "hstep_cols");
  if (fresh) *fresh = SumJob{a.emit, (int)hcols_blocks(T), R};
  return DNA_OK;
}

dna_status dna_update_H(const float* V, const float* W, float* H, int64_t N, int64_t T, int64_t R,
                        const dna_opts* o, void* ws, size_t ws_bytes, uint8_t* chose_newton, double* d_sel,
                        double* margin, void* stream) {
  if (!V || !W || !H) return fail(DNA_EINVAL, "V, W or H is NULL");
  Common c;
  DNA_TRY(check_opts(o));
  DNA_TRY(check_select(o, R));   // before anything is enqueued
  DNA_TRY(prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  if (hcols_path(o, T, R)) {
    DNA_TRY(run_hstep_cols(V, W, H, N, T, R, o, c, ws, nullptr, chose_newton, d_sel, margin, nullptr));
    return epilogue(c);
  }
  float* Xmu = at<float>(ws, c.L.xmu);
  float* Xn = at<float>(ws, c.L.xn);
  DNA_TRY(run_candidates(0, V, W, H, N, T, R, o, c.L, ws, Xmu, Xn, nullptr, nullptr, c.chk, c.s));
  DNA_TRY(run_select(0, V, W, Xmu, Xn, H, N, T, R, o, c.L, ws, chose_newton, d_sel, margin, c.s));
  return epilogue(c);
}

dna_status dna_update_W(const float* V, float* W, const float* H, int64_t N, int64_t T, int64_t R,
                        const dna_opts* o, void* ws, size_t ws_bytes, uint8_t* chose_newton, double* d_sel,
                        double* margin, void* stream) {
  if (!V || !W || !H) return fail(DNA_EINVAL, "V, W or H is NULL");
  Common c;
  DNA_TRY(check_opts(o));
  DNA_TRY(check_select(o, R));   // before anything is enqueued
  DNA_TRY(prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  float* Xmu = at<float>(ws, c.L.xmu);
  float* Xn = at<float>(ws, c.L.xn);
  DNA_TRY(run_candidates(1, V, W, H, N, T, R, o, c.L, ws, Xmu, Xn, nullptr, nullptr, c.chk, c.s));
  DNA_TRY(run_select(1, V, H, Xmu, Xn, W, N, T, R, o, c.L, ws, chose_newton, d_sel, margin, c.s));
  return epilogue(c);
}

// Normalisation inside dna_iterate: the scale kernel emits the first level of
// the sums of the factor it normalised; they are the next half-step's c (g)
// when that factor is W (H), i.e. unless one eq. 2 weight alone is positive
// and fixes the other factor's scale.
static dna_status iterate_normalize(int side, float* W, float* H, int64_t N, int64_t T, int64_t R,
                                    const dna_opts* o, const Common& c, void* ws, SumJob& next, bool& valid,
                                    const SumJob* fresh = nullptr) {
  DNA_TRY(run_normalize(side, W, H, N, T, R, o, at<double>(ws, c.L.sump), at<double>(ws, c.L.sump2), c.chk, c.s,
                        at<double>(ws, c.L.sume), &next, fresh));
  valid = norm_side(o, side) == side;
  return DNA_OK;
}

dna_status dna_iterate(const float* V, float* W, float* H, int64_t N, int64_t T, int64_t R, int iters,
                       const dna_opts* o, void* ws, size_t ws_bytes, void* stream) {
  if (!V || !W || !H) return fail(DNA_EINVAL, "V, W or H is NULL");
  if (iters < 0) return fail(DNA_EINVAL, "iters must be >= 0");
  Common c;
  DNA_TRY(check_opts(o));
  DNA_TRY(check_select(o, R));   // before anything is enqueued
  DNA_TRY(prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  float* Xmu = at<float>(ws, c.L.xmu);
  float* Xn = at<float>(ws, c.L.xn);
  SumJob next;
  bool have = false;                                // `next` holds c for the coming H step
  // tiled fp32 path: each cost pass leaves Z of both candidates and the choice
  // for the next half-step's ratio pass (Algorithm 1 steps 15, 28)
  const bool keep = o->gemm == DNA_GEMM_FP32 && R > FUSED_MAX_R;
  bool zin = false;                                 // Z of the current state is in the workspace
  const bool cols = hcols_path(o, T, R);
  // FP16: each cost pass bounds the next Z pass's Q maxima (the first has none)
  const bool qm = o->gemm == DNA_GEMM_FP16;
  for (int it = 0; it < iters; ++it) {
    if (cols) {
      SumJob fresh;
      DNA_TRY(run_hstep_cols(V, W, H, N, T, R, o, c, ws, have ? &next : nullptr, nullptr, nullptr, nullptr, &fresh));
      DNA_TRY(iterate_normalize(1, W, H, N, T, R, o, c, ws, next, have, &fresh));  // step 16; next = g
    } else {
      DNA_TRY(run_candidates(0, V, W, H, N, T, R, o, c.L, ws, Xmu, Xn, nullptr, nullptr, c.chk, c.s,
                             have ? &next : nullptr, zin, nullptr, qm && it > 0));
      DNA_TRY(run_select(0, V, W, Xmu, Xn, H, N, T, R, o, c.L, ws, nullptr, nullptr, nullptr, c.s, keep, nullptr,
                         qm));
      DNA_TRY(iterate_normalize(1, W, H, N, T, R, o, c, ws, next, have));  // step 16; next = g
    }
    DNA_TRY(run_candidates(1, V, W, H, N, T, R, o, c.L, ws, Xmu, Xn, nullptr, nullptr, c.chk, c.s,
                           have ? &next : nullptr, keep, nullptr, qm));
    SumJob freshW;
    DNA_TRY(run_select(1, V, H, Xmu, Xn, W, N, T, R, o, c.L, ws, nullptr, nullptr, nullptr, c.s, keep, &freshW,
                       qm && it + 1 < iters));
    DNA_TRY(iterate_normalize(0, W, H, N, T, R, o, c, ws, next, have, &freshW));  // step 29; next = c
    zin = keep;
  }
  return epilogue(c);
}

// ---------------------------------------------------------------------------
// dna_iterate_noalloc: dna_iterate on a scratch array the library owns, for
// callers that cannot allocate device memory.  The array is a file-scope
// device variable: every GPU the library runs on holds its own copy, at its own
// address, from code-object load until the process ends.  In host code its name
// is a host-side stand-in, not a device address; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current, and is
// the only form of the array host code passes anywhere.  No kernel needs the
// workspace to start at any particular content, so nothing is cleared.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[DNA_NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

static dna_status scratch_address(void** out) {
  int dev = -1;
  DNA_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(DNA_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    DNA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!p) return fail(DNA_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return DNA_OK;
}

// One MU half-step (eq. 11) on the prologue's state; with_cost writes the input
// state's per-column (row) cost to d_out.
static dna_status run_mu(int side, const float* V, float* W, float* H, int64_t N, int64_t T, int64_t R,
                         int with_cost, double* d_out, const dna_opts* o, const Common& c, void* ws) {
  const Layout& L = c.L;
  float* Q = at<float>(ws, L.q);
  float* pu = at<float>(ws, L.pu);
  float* c32 = at<float>(ws, L.c32);
  double* cpart = at<double>(ws, L.cpart);
  RatioArgs ra{V, W, H, N, T, R, Q, nullptr, nullptr, cpart, c.chk, nullptr};
  const bool fused = R <= FUSED_MAX_R;            // Z, Q and u in one pass, Q never stored
  const int mode = with_cost ? RGH_MU_COST : RGH_MU;
  SumJob job;
  if (side == 0) {
    DNA_HIP(launch_colsum_part(W, N, R, at<double>(ws, L.sump), job, c.s), "colsum_W");
    job.s32 = c32; job.check = c.chk; job.reg = o->lambda;
    if (fused) {
      DNA_HIP(launch_rgh(0, V, W, H, N, T, R, L.shf.splits, L.shf.kchunk, pu, nullptr, nullptr, cpart, job, c.chk,
                         c.s, mode), "rgh_mu_H");
      DNA_HIP(launch_mu_H(H, pu, L.shf.splits, c32, T, R, cpart, L.shf.splits, with_cost ? d_out : nullptr, c.s),
              "mu_H");
      return DNA_OK;
    }
    ra.fin = job;
    DNA_HIP(launch_ratio(with_cost ? RM_MU_H_COST : RM_MU_H, ra, c.s), "ratio_mu_H");
    DNA_HIP(launch_gh_H(W, Q, nullptr, nullptr, N, T, R, L.sh.splits, L.sh.kchunk, pu, nullptr, nullptr, c.s),
            "gh_mu_H");
    DNA_HIP(launch_mu_H(H, pu, L.sh.splits, c32, T, R, cpart, L.rt_m, with_cost ? d_out : nullptr, c.s), "mu_H");
  } else {
    DNA_HIP(launch_rowsum_part(H, T, R, at<double>(ws, L.sump), job, c.s), "rowsum_H");
    job.s32 = c32; job.check = c.chk; job.reg = o->rho;
    if (fused) {
      DNA_HIP(launch_rgh(1, V, W, H, N, T, R, L.swf.splits, L.swf.kchunk, pu, nullptr, nullptr, cpart, job, c.chk,
                         c.s, mode), "rgh_mu_W");
      DNA_HIP(launch_mu_W(W, pu, L.swf.splits, c32, N, R, cpart, L.swf.splits, with_cost ? d_out : nullptr, c.s),
              "mu_W");
      return DNA_OK;
    }
    ra.fin = job;
    DNA_HIP(launch_ratio(with_cost ? RM_MU_W_COST : RM_MU_W, ra, c.s), "ratio_mu_W");
    DNA_HIP(launch_gh_W(Q, nullptr, H, nullptr, N, T, R, L.sw.splits, L.sw.kchunk, pu, nullptr, nullptr, c.s),
            "gh_mu_W");
    DNA_HIP(launch_mu_W(W, pu, L.sw.splits, c32, N, R, cpart, L.rt_n, with_cost ? d_out : nullptr, c.s), "mu_W");
  }
  return DNA_OK;
}

dna_status dna_iterate_noalloc(const float* V, float* W, float* H, int64_t N, int64_t T, int64_t R, int iters,
                               const dna_opts* o, void* stream) {
  if (!V || !W || !H) return fail(DNA_EINVAL, "V, W or H is NULL");
  if (iters < 0) return fail(DNA_EINVAL, "iters must be >= 0");
  DNA_TRY(check_dims(N, T, R));
  DNA_TRY(check_opts(o));
  const size_t need = make_layout(N, T, R, o->gemm != DNA_GEMM_FP32).total;
  if (need > DNA_NOALLOC_SCRATCH_BYTES) {
    std::snprintf(g_err, sizeof(g_err),
                  "dna_iterate_noalloc: this problem needs %zu bytes of workspace, more than the %zu-byte scratch "
                  "array; call dna_iterate with a workspace instead", need, (size_t)DNA_NOALLOC_SCRATCH_BYTES);
    return DNA_EUNSUPPORTED;
  }
  void* ws = nullptr;
  DNA_TRY(scratch_address(&ws));
  return dna_iterate(V, W, H, N, T, R, iters, o, ws, DNA_NOALLOC_SCRATCH_BYTES, stream);
}

dna_status mu_update(int side, const float* V, float* W, float* H, int64_t N, int64_t T, int64_t R,
                     int with_cost, double* d_out, const dna_opts* o, void* ws, size_t ws_bytes, void* stream) {
  if (!V || !W || !H) return fail(DNA_EINVAL, "V, W or H is NULL");
  if (side != 0 && side != 1) return fail(DNA_EINVAL, "side must be 0 or 1");
  if (with_cost && !d_out) return fail(DNA_EINVAL, "with_cost requires d_out");
  Common c;
  DNA_TRY(prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  DNA_TRY(run_mu(side, V, W, H, N, T, R, with_cost, d_out, o, c, ws));
  return epilogue(c);
}

dna_status mu_iterate(const float* V, float* W, float* H, int64_t N, int64_t T, int64_t R, int iters,
                      int with_cost, const dna_opts* o, void* ws, size_t ws_bytes, void* stream) {
  if (!V || !W || !H) return fail(DNA_EINVAL, "V, W or H is NULL");
  if (iters < 0) return fail(DNA_EINVAL, "iters must be >= 0");
  Common c;
  DNA_TRY(prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  double* dcost = at<double>(ws, c.L.vpart);        // the with-cost outputs, not returned
  double* sp = at<double>(ws, c.L.sump);
  double* sp2 = at<double>(ws, c.L.sump2);
  for (int it = 0; it < iters; ++it) {
    DNA_TRY(run_mu(0, V, W, H, N, T, R, with_cost, dcost, o, c, ws));
    DNA_TRY(run_normalize(1, W, H, N, T, R, o, sp, sp2, c.chk, c.s, nullptr, nullptr));   // step 16
    DNA_TRY(run_mu(1, V, W, H, N, T, R, with_cost, dcost, o, c, ws));
    DNA_TRY(run_normalize(0, W, H, N, T, R, o, sp, sp2, c.chk, c.s, nullptr, nullptr));   // step 29
  }
  return epilogue(c);
}

dna_status kl_cost(const float* V, const float* W, const float* H, int64_t N, int64_t T, int64_t R,
                   const dna_opts* o, void* ws, size_t ws_bytes, double* out, void* stream) {
  if (!V || !W || !H || !out) return fail(DNA_EINVAL, "V, W, H or out is NULL");
  Common c;
  DNA_TRY(prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  double* cpart = at<double>(ws, c.L.cpart);
  RatioArgs ra{V, W, H, N, T, R, nullptr, nullptr, nullptr, cpart, c.chk, nullptr};
  DNA_HIP(launch_ratio(RM_KL, ra, c.s), "kl_terms");
  DNA_HIP(launch_kl_final(cpart, c.L.rt_m * c.L.rt_n, out, c.s), "kl_final");
  DNA_TRY(add_penalty(W, H, N, T, R, o, at<double>(ws, c.L.sump), at<double>(ws, c.L.sump2), out, c.s));
  return epilogue(c);
}

dna_status dna_gradient_hessian(int side, const float* V, const float* W, const float* H, int64_t N, int64_t T,
                                int64_t R, const dna_opts* o, float* A_out, float* B_out, void* ws,
                                size_t ws_bytes, void* stream) {
  if (!V || !W || !H || !A_out || !B_out) return fail(DNA_EINVAL, "NULL argument");
  if (side != 0 && side != 1) return fail(DNA_EINVAL, "side must be 0 or 1");
  Common c;
  DNA_TRY(prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  float* Xmu = at<float>(ws, c.L.xmu);
  float* Xn = at<float>(ws, c.L.xn);
  DNA_TRY(run_candidates(side, V, W, H, N, T, R, o, c.L, ws, Xmu, Xn, A_out, B_out, c.chk, c.s));
  return epilogue(c);
}

dna_status dna_candidates(int side, const float* V, const float* W, const float* H, int64_t N, int64_t T,
                          int64_t R, const dna_opts* o, float* X_mu, float* X_newton, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!V || !W || !H || !X_mu || !X_newton) return fail(DNA_EINVAL, "NULL argument");
  if (side != 0 && side != 1) return fail(DNA_EINVAL, "side must be 0 or 1");
  Common c;
  DNA_TRY(prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  if (side == 0 && hcols_path(o, T, R)) {          // the candidates the one-kernel H step forms
    SumJob job;
    DNA_HIP(launch_colsum_part(W, N, R, at<double>(ws, c.L.sump), job, c.s), "colsum_W");
    job.reg = o->lambda;
    HColsArgs a{V, W, const_cast<float*>(H), N, T, R, job, o->eps, o->alpha, nullptr, nullptr, nullptr,
                at<double>(ws, c.L.pu), c.chk};
    a.xmu_out = X_mu;
    a.xn_out = X_newton;
    DNA_HIP(launch_hstep_cols(a, c.s), "hstep_cols");
    return epilogue(c);
  }
  DNA_TRY(run_candidates(side, V, W, H, N, T, R, o, c.L, ws, X_mu, X_newton, nullptr, nullptr, c.chk, c.s));
  return epilogue(c);
}

dna_status dna_select(int side, const float* V, const float* F, const float* X_mu, const float* X_newton,
                      float* X_out, int64_t N, int64_t T, int64_t R, const dna_opts* o, uint8_t* chose_newton,
                      double* d_sel, double* margin, void* ws, size_t ws_bytes, void* stream) {
  if (!V || !F || !X_mu || !X_newton || !X_out) return fail(DNA_EINVAL, "NULL argument");
  if (side != 0 && side != 1) return fail(DNA_EINVAL, "side must be 0 or 1");
  Common c;
  DNA_TRY(check_dims(N, T, R));
  DNA_TRY(check_opts(o));
  DNA_TRY(check_select_both(o));
  c.L = make_layout(N, T, R, o->gemm != DNA_GEMM_FP32);
  DNA_TRY(check_ws(ws, ws_bytes, c.L.total));
  c.s = static_cast<hipStream_t>(stream);
  c.chk = nullptr;
  DNA_TRY(run_select(side, V, F, X_mu, X_newton, X_out, N, T, R, o, c.L, ws, chose_newton, d_sel, margin, c.s));
  return DNA_OK;
}

size_t dna_unrolled_workspace_bytes(int64_t N, int64_t T, int64_t R, const dna_opts* o) {
  (void)o;
  if (N <= 0 || T <= 0 || R <= 0) return 0;
  return make_adj_layout(N, T, R).total;
}

// The kept sums of the unrolled forward: per update k, Z, Q, Q-bar (N x T
// each) and the split partials of u, u_c, y (splits x R x T each), then the V
// column sums of the ratio pass (the same for every k).  Only the tiled fp32
// path (R > 64) keeps them; with R <= 64 the adjoint recomputes (fused, cheap).
struct AuxLayout {
  size_t z, q, qb, pu, puc, py, step, vpart, total;
};

static AuxLayout make_aux_layout(int64_t N, int64_t T, int64_t R, int K) {
  AuxLayout X{};
  if (R <= FUSED_MAX_R || K <= 0) return X;
  const Layout L = make_adj_layout(N, T, R).base;
  const size_t nt = align_up((size_t)N * T * 4), part = align_up((size_t)L.sh.splits * R * T * 4);
  X.z = 0;
  X.q = nt;
  X.qb = 2 * nt;
  X.pu = 3 * nt;
  X.puc = 3 * nt + part;
  X.py = 3 * nt + 2 * part;
  X.step = 3 * nt + 3 * part;
  X.vpart = X.step * (size_t)K;
  X.total = X.vpart + align_up((size_t)L.rt_m * T * 8);
  return X;
}

static AuxOut aux_at(void* aux, const AuxLayout& X, int k) {
  char* b = static_cast<char*>(aux) + X.step * (size_t)k;
  return AuxOut{reinterpret_cast<float*>(b + X.z), reinterpret_cast<float*>(b + X.q),
                reinterpret_cast<float*>(b + X.qb), reinterpret_cast<float*>(b + X.pu),
                reinterpret_cast<float*>(b + X.puc), reinterpret_cast<float*>(b + X.py),
                reinterpret_cast<double*>(static_cast<char*>(aux) + X.vpart)};
}

size_t dna_unrolled_aux_bytes(int64_t N, int64_t T, int64_t R, int K, const dna_opts* o) {
  (void)o;
  if (N <= 0 || T <= 0 || R <= 0 || K <= 0) return 0;
  return make_aux_layout(N, T, R, K).total;
}

static dna_status unrolled_fwd(const float* V, const float* W, const float* H_init, int K, int64_t N, int64_t T,
                               int64_t R, const dna_opts* o, float* H_ckpt, uint8_t* sel_ckpt, void* ws,
                               size_t ws_bytes, void* aux, size_t aux_bytes, void* stream) {
  if (!V || !W || !H_init || !H_ckpt || (K > 0 && !sel_ckpt)) return fail(DNA_EINVAL, "NULL argument");
  if (K < 0) return fail(DNA_EINVAL, "K must be >= 0");
  DNA_TRY(check_dims(N, T, R));
  DNA_TRY(check_opts(o));
  DNA_TRY(check_select_both(o));
  if (o->gemm != DNA_GEMM_FP32) return fail(DNA_EUNSUPPORTED, "the unrolled adjoint runs in fp32 only");
  if (o->lambda != 0.f) return fail(DNA_EUNSUPPORTED, "the unrolled adjoint has no lambda terms");
  const AdjLayout A = make_adj_layout(N, T, R);
  DNA_TRY(check_ws(ws, ws_bytes, A.total));
  const AuxLayout X = make_aux_layout(N, T, R, K);
  const bool keep = aux != nullptr && X.total > 0;
  if (keep) DNA_TRY(check_aux(aux, aux_bytes, X.total));
  hipStream_t s = static_cast<hipStream_t>(stream);
  int* chk = o->checked ? at<int>(ws, A.base.check) : nullptr;
  if (chk) {
    const float* bufs[3] = {W, H_init, V};
    const int64_t sizes[3] = {N * R, R * T, N * T};
    DNA_TRY(checked_begin(chk, bufs, sizes, 3, s));
  }
  const int64_t RT = R * T;
  DNA_HIP(launch_copy(H_init, H_ckpt, RT, s), "copy");
  float* Xmu = at<float>(ws, A.base.xmu);
  float* Xn = at<float>(ws, A.base.xn);
  for (int k = 0; k < K; ++k) {
    const float* Hk = H_ckpt + (int64_t)k * RT;
    float* Hk1 = H_ckpt + (int64_t)(k + 1) * RT;
    const AuxOut ax = keep ? aux_at(aux, X, k) : AuxOut{};
    DNA_TRY(run_candidates(0, V, W, Hk, N, T, R, o, A.base, ws, Xmu, Xn, nullptr, nullptr, chk, s, nullptr, false,
                           keep ? &ax : nullptr));
    DNA_TRY(run_select(0, V, W, Xmu, Xn, Hk1, N, T, R, o, A.base, ws, sel_ckpt + (int64_t)k * T, nullptr, nullptr, s));
  }
  if (chk) return checked_end(chk, s);
  return DNA_OK;
}

dna_status dna_unrolled_H_fwd(const float* V, const float* W, const float* H_init, int K, int64_t N, int64_t T,
                              int64_t R, const dna_opts* o, float* H_ckpt, uint8_t* sel_ckpt, void* ws,
                              size_t ws_bytes, void* stream) {
  return unrolled_fwd(V, W, H_init, K, N, T, R, o, H_ckpt, sel_ckpt, ws, ws_bytes, nullptr, 0, stream);
}

dna_status dna_unrolled_H_fwd_aux(const float* V, const float* W, const float* H_init, int K, int64_t N, int64_t T,
                                  int64_t R, const dna_opts* o, float* H_ckpt, uint8_t* sel_ckpt, void* ws,
                                  size_t ws_bytes, void* aux, size_t aux_bytes, void* stream) {
  return unrolled_fwd(V, W, H_init, K, N, T, R, o, H_ckpt, sel_ckpt, ws, ws_bytes, aux, aux_bytes, stream);
}

static dna_status unrolled_bwd(const float* V, const float* W, const float* H_ckpt, const uint8_t* sel_ckpt, int K,
                               int64_t N, int64_t T, int64_t R, const float* dH_K, float* dW, float* dV,
                               float* dH_init, const dna_opts* o, void* ws, size_t ws_bytes, const void* aux,
                               size_t aux_bytes, void* stream) {
  if (!V || !W || !H_ckpt || !dH_K || !dW || !dV || (K > 0 && !sel_ckpt)) return fail(DNA_EINVAL, "NULL argument");
  if (K < 0) return fail(DNA_EINVAL, "K must be >= 0");
  DNA_TRY(check_dims(N, T, R));
  DNA_TRY(check_opts(o));
  DNA_TRY(check_select_both(o));
  if (o->gemm != DNA_GEMM_FP32) return fail(DNA_EUNSUPPORTED, "the unrolled adjoint runs in fp32 only");
  if (o->lambda != 0.f) return fail(DNA_EUNSUPPORTED, "the unrolled adjoint has no lambda terms");
  const AdjLayout A = make_adj_layout(N, T, R);
  DNA_TRY(check_ws(ws, ws_bytes, A.total));
  const AuxLayout X = make_aux_layout(N, T, R, K);
  const bool kept = aux != nullptr && X.total > 0;
  if (kept) DNA_TRY(check_aux(aux, aux_bytes, X.total));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Layout& L = A.base;
  const int64_t RT = R * T;
  if (K == 0) {
    DNA_HIP(launch_fill(dW, 0.f, N * R, s), "fill");
    DNA_HIP(launch_fill(dV, 0.f, N * T, s), "fill");
    if (dH_init) DNA_HIP(launch_copy(dH_K, dH_init, RT, s), "copy");
    return DNA_OK;
  }
  float* wpu = at<float>(ws, L.pu);
  float* c32 = at<float>(ws, L.c32);
  float* Zbar = at<float>(ws, A.zbar);
  float* Ub = at<float>(ws, A.ubar);
  float* Yb = at<float>(ws, A.ybar);
  float* Hd = at<float>(ws, A.hd);
  float* Cb = at<float>(ws, A.cbar);
  float* G[2] = {at<float>(ws, A.g0), at<float>(ws, A.g1)};
  float* sbar = at<float>(ws, A.sbar);
  double* cbar64 = at<double>(ws, A.cbar64);
  float* p0 = at<float>(ws, A.wp0);
  float* p1 = at<float>(ws, A.wp1);
  float* cs = at<float>(ws, L.cs);
  {
    SumJob job;
    DNA_HIP(launch_colsum_part(W, N, R, at<double>(ws, L.sump), job, s), "colsum_W");
    job.s32 = c32;
    DNA_HIP(launch_sum_final(job, s), "sum_final");
    if (!kept && R > FUSED_MAX_R && N >= GH_CHUNK_MIN_K) DNA_HIP(launch_chunk_sums(0, W, N, T, R, cs, s), "chunk_sums_W");
  }
  const float* Gin = dH_K;
  for (int k = K - 1; k >= 0; --k) {
    const float* Hk = H_ckpt + (int64_t)k * RT;
    const int acc = k != K - 1;
    float* Gout = (k == 0) ? dH_init : G[k & 1];
    // Z, Q, Q-bar, u, u_c, y and the V sums of the forward's update k: kept
    // by the forward, or recomputed on the product path and split the
    // forward's run_candidates took, so that every branch of the candidate
    // arithmetic (gain form, floor, cap, value floor) repeats bit for bit
    float *Z, *Q, *Qb, *pu, *puc, *py;
    double* vpart;
    int sp = L.sh.splits, vtiles = L.rt_m;
    if (kept) {
      const AuxOut ax = aux_at(const_cast<void*>(aux), X, k);
      Z = ax.Z; Q = ax.Q; Qb = ax.Qb; pu = ax.pu; puc = ax.puc; py = ax.py; vpart = ax.vpart;
      if (sp > 8 && T < 256 * 32) sp = 1;              // the forward folded them into split 0
    } else {
      Z = at<float>(ws, A.z); Q = at<float>(ws, L.q); Qb = at<float>(ws, L.qb);
      pu = wpu; puc = at<float>(ws, L.puc); py = at<float>(ws, L.py); vpart = at<double>(ws, L.vpart);
      RatioArgs ra{V, W, Hk, N, T, R, Q, Qb, vpart, nullptr, nullptr, Z};
      DNA_HIP(launch_ratio(RM_ADJ, ra, s), "ratio_adj");
      if (R <= FUSED_MAX_R) {
        DNA_HIP(launch_rgh(0, V, W, Hk, N, T, R, L.shf.splits, L.shf.kchunk, pu, puc, py, vpart, SumJob{}, nullptr,
                           s), "rgh_H");
        sp = L.shf.splits;
        vtiles = L.shf.splits;
      } else {
        DNA_HIP(launch_gh_H(W, Q, Qb, N >= GH_CHUNK_MIN_K ? cs : nullptr, N, T, R, L.sh.splits, L.sh.kchunk, pu,
                            puc, py, s), "gh_H");
      }
      if (sp > 8 && T < 256 * 32) {
        DNA_HIP(launch_fold_splits(pu, puc, py, sp, R * T, s), "fold_splits");
        sp = 1;
      }
    }
    DNA_HIP(launch_cand_bwd_H(Hk, pu, puc, py, sp, c32, vpart, vtiles, T, R, o->eps, o->alpha,
                              sel_ckpt + (int64_t)k * T, Gin, Ub, Yb, Hd, Cb, sbar, s), "cand_bwd_H");
    DNA_HIP(launch_zbar(V, Z, W, Ub, Yb, sbar, N, T, R, Zbar, dV, acc, s), "zbar");
    {
      SumJob job;
      DNA_HIP(launch_rowsum_part(Cb, T, R, at<double>(ws, L.sump), job, s), "rowsum cbar");
      job.s64 = cbar64;
      DNA_HIP(launch_sum_final(job, s), "sum_final cbar");
    }
    DNA_HIP(launch_wbar(Q, Zbar, Qb, Ub, Hk, Yb, N, T, R, A.swb.splits, A.swb.kchunk, p0, p1, s), "wbar");
    DNA_HIP(launch_dw_final(W, p0, p1, A.swb.splits, cbar64, N, R, dW, acc, s), "dw_final");
    if (Gout) {
      DNA_HIP(launch_gh_H(W, Zbar, nullptr, nullptr, N, T, R, L.sh.splits, L.sh.kchunk, wpu, nullptr, nullptr, s),
              "gh_zbar");
      DNA_HIP(launch_dh_final(Hd, wpu, L.sh.splits, R, T, Gout, s), "dh_final");
    }
    Gin = Gout;
  }
  return DNA_OK;
}

dna_status dna_unrolled_H_bwd(const float* V, const float* W, const float* H_ckpt, const uint8_t* sel_ckpt, int K,
                              int64_t N, int64_t T, int64_t R, const float* dH_K, float* dW, float* dV,
                              float* dH_init, const dna_opts* o, void* ws, size_t ws_bytes, void* stream) {
  return unrolled_bwd(V, W, H_ckpt, sel_ckpt, K, N, T, R, dH_K, dW, dV, dH_init, o, ws, ws_bytes, nullptr, 0,
                      stream);
}

dna_status dna_unrolled_H_bwd_aux(const float* V, const float* W, const float* H_ckpt, const uint8_t* sel_ckpt,
                                  int K, int64_t N, int64_t T, int64_t R, const float* dH_K, float* dW, float* dV,
                                  float* dH_init, const dna_opts* o, void* ws, size_t ws_bytes, const void* aux,
                                  size_t aux_bytes, void* stream) {
  return unrolled_bwd(V, W, H_ckpt, sel_ckpt, K, N, T, R, dH_K, dW, dV, dH_init, o, ws, ws_bytes, aux, aux_bytes,
                      stream);
}

// ---------------------------------------------------------------------------
// Sparse V.
// ---------------------------------------------------------------------------
struct SpLayout {
  int64_t nseg;
  size_t ht, q, qb, gp, vseg, pu, puc, py, xmu, xn, xd, xnt, xdt, c32, c64, g64, sump, sump2, sume, vpart, cseg,
      fseg, part, fpart, zc, dzc, smask, check, total;
};

static SpLayout make_sp_layout(int64_t N, int64_t T, int64_t R, const dna_sparse_v* V) {
  SpLayout L;
  L.nseg = std::max<int64_t>({V->nseg_r, V->nseg_c, 1});
  const size_t fac = (size_t)std::max(R * T, N * R), mx = (size_t)std::max(N, T), nnz = (size_t)V->nnz;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  L.ht = take((size_t)T * R * 4);
  L.q = take(nnz * 4);
  L.qb = take(nnz * 4);
  L.gp = take(4 * (size_t)L.nseg * R * 4);
  L.vseg = take((size_t)L.nseg * 8);
  L.pu = take(fac * 4);
  L.puc = take(fac * 4);
  L.py = take(fac * 4);
  L.xmu = take(fac * 4);
  L.xn = take(fac * 4);
  L.xd = take(fac * 4);
  L.xnt = take((size_t)R * T * 4);
  L.xdt = take((size_t)R * T * 4);
  L.c32 = take((size_t)R * 4);
  L.c64 = take((size_t)R * 8);
  L.g64 = take((size_t)R * 8);
  L.sump = take((size_t)SUM_PARTS * R * 8);
  L.sump2 = take((size_t)SUM_PARTS * R * 8);
  L.sume = take((size_t)std::max(scale_emit_parts(0, N, T), scale_emit_parts(1, N, T)) * R * 8);
  L.vpart = take(mx * 8);
  L.cseg = take(3 * (size_t)L.nseg * 8);
  L.fseg = take((size_t)L.nseg * 4);
  L.part = take(3 * mx * 8);
  L.fpart = take(mx * 4);
  // the reconstruction a half-step's cost pass leaves for the next one
  L.zc = take(nnz * 4);
  L.dzc = take(nnz * 4);
  L.smask = take(mx);
  L.check = take(16);
  L.total = off;
  return L;
}

static dna_status check_sparse(const dna_sparse_v* V, int64_t N, int64_t T, int64_t R, const dna_opts* o) {
  if (!V) return fail(DNA_EINVAL, "sparse V is NULL");
  DNA_TRY(check_dims(N, T, R));
  DNA_TRY(check_opts(o));
  DNA_TRY(check_select_both(o));
  if (o->gemm != DNA_GEMM_FP32) return fail(DNA_EUNSUPPORTED, "sparse V supports FP32 products only");
  if (R > SP_MAX_R) return fail(DNA_EUNSUPPORTED, "sparse V supports R <= 256");
  if (V->nnz < 0 || V->nnz >= ((int64_t)1 << 31)) return fail(DNA_EINVAL, "nnz must lie in [0, 2^31)");
  if (V->nseg_r < 0 || V->nseg_c < 0 || V->nseg_r > V->nnz || V->nseg_c > V->nnz)
    return fail(DNA_EINVAL, "segment counts must lie in [0, nnz]");
  if (!V->segr_start || !V->segr_ptr || !V->segc_start || !V->segc_ptr)
    return fail(DNA_EINVAL, "segment tables must not be NULL");
  if (V->nnz > 0 && (!V->col_idx || !V->val || !V->row_of || !V->csc_row || !V->csc_col || !V->csc_pos))
    return fail(DNA_EINVAL, "an index or value array is NULL");
  return DNA_OK;
}

static SpV sp_view(const dna_sparse_v* V) {
  return SpV{V->nnz, V->col_idx, V->val, V->row_of, V->csc_row, V->csc_col, V->csc_pos, V->nseg_r, V->nseg_c,
             V->segr_start, V->segr_ptr, V->segc_start, V->segc_ptr};
}

struct SpCommon {
  SpLayout L;
  int* chk;
  hipStream_t s;
};

static dna_status sp_prologue(const dna_sparse_v* V, const float* W, const float* H, int64_t N, int64_t T, int64_t R,
                              const dna_opts* o, void* ws, size_t ws_bytes, void* stream, SpCommon& c) {
  DNA_TRY(check_sparse(V, N, T, R, o));
  c.L = make_sp_layout(N, T, R, V);
  DNA_TRY(check_ws(ws, ws_bytes, c.L.total));
  c.s = static_cast<hipStream_t>(stream);
  c.chk = o->checked ? at<int>(ws, c.L.check) : nullptr;
  if (c.chk) {
    const float* bufs[3] = {W, H, V->val};
    const int64_t sizes[3] = {N * R, R * T, V->nnz};
    DNA_TRY(checked_begin(c.chk, bufs, sizes, V->nnz > 0 ? 3 : 2, c.s));
  }
  return DNA_OK;
}

static dna_status sp_epilogue(const SpCommon& c) {
  if (c.chk) return checked_end(c.chk, c.s);
  return DNA_OK;
}

// One sparse half-step: side 0 updates H (R x T) given W, side 1 updates W.
// `pre`, if given, holds the first level of c (side 0) / g (side 1) already
// written by the preceding normalisation.  carry_in >= 0: the preceding
// half-step (of side carry_in) left its reconstruction at the nonzeros and its
// selection mask in the workspace, and Q, Q-bar come from them instead of new
// dot products; carry_out: leave this step's for the next one.
static dna_status sp_half_step(int side, const dna_sparse_v* V, float* W, float* H, int64_t N, int64_t T, int64_t R,
                               const dna_opts* o, const SpCommon& c, void* ws, uint8_t* mask, double* dsel,
                               double* margin, const SumJob* pre = nullptr, int carry_in = -1,
                               bool carry_out = false) {
  const SpLayout& L = c.L;
  const SpV v = sp_view(V);
  float* Ht = at<float>(ws, L.ht);
  float* q = at<float>(ws, L.q);
  float* qb = at<float>(ws, L.qb);
  float* pu = at<float>(ws, L.pu);
  float* puc = at<float>(ws, L.puc);
  float* py = at<float>(ws, L.py);
  float* Xmu = at<float>(ws, L.xmu);
  float* Xn = at<float>(ws, L.xn);
  float* Xd = at<float>(ws, L.xd);
  float* c32 = at<float>(ws, L.c32);
  double* c64 = at<double>(ws, L.c64);
  double* vpart = at<double>(ws, L.vpart);
  double* part = at<double>(ws, L.part);
  int* fpart = at<int>(ws, L.fpart);
  if (side == 1 || carry_in < 0)                    // H^t: the W step's factor rows and the fresh Z
    DNA_HIP(launch_sp_transpose(H, Ht, R, T, c.s), "sp_transpose H");
  SumJob job;
  if (pre) job = *pre;
  else if (side == 0) DNA_HIP(launch_colsum_part(W, N, R, at<double>(ws, L.sump), job, c.s), "colsum_W");
  else DNA_HIP(launch_rowsum_part(H, T, R, at<double>(ws, L.sump), job, c.s), "rowsum_H");
  job.s64 = c64; job.s32 = c32; job.check = c.chk;  // c = W^t 1 (side 0) or g = H 1 (side 1)
  job.reg = side == 0 ? o->lambda : o->rho;         // c32 = c + lambda or g + rho; c64 without
  float* zc = at<float>(ws, L.zc);
  float* dzc = at<float>(ws, L.dzc);
  uint8_t* smask = at<uint8_t>(ws, L.smask);
  if (carry_in >= 0)
    DNA_HIP(launch_sp_qz(v, zc, dzc, smask, carry_in, N, T, q, qb, c.chk, job, c.s), "sp_qz");
  else
    DNA_HIP(launch_sp_zq(v, W, Ht, N, T, R, q, qb, c.chk, job, c.s), "sp_zq");
  if (carry_out && !mask) mask = smask;
  float* zo = carry_out ? zc : nullptr;
  float* dzo = carry_out ? dzc : nullptr;
  DNA_HIP(launch_sp_grad(side, false, v, side == 0 ? W : Ht, q, qb, c64, N, T, R, at<float>(ws, L.gp),
                         at<double>(ws, L.vseg), pu, puc, py, vpart, c.s), "sp_grad");
  if (side == 0) {
    DNA_HIP(launch_cand_H(H, pu, puc, py, 1, c32, vpart, 1, T, R, o->eps, o->alpha, o->lambda, Xmu, Xn, nullptr,
                          nullptr, c.s), "cand_H");
    DNA_HIP(launch_sp_diff(Xmu, Xn, Xd, R * T, c.s), "sp_diff");
    float* XnT = at<float>(ws, L.xnt);
    float* XdT = at<float>(ws, L.xdt);
    DNA_HIP(launch_sp_transpose(Xn, XnT, R, T, c.s), "sp_transpose X_DNA");
    DNA_HIP(launch_sp_transpose(Xd, XdT, R, T, c.s), "sp_transpose X_MU - X_DNA");
    DNA_HIP(launch_sp_cost(0, v, W, XnT, XdT, N, T, R, at<double>(ws, L.cseg), at<int>(ws, L.fseg), part, fpart,
                           c.s, zo, dzo), "sp_cost_H");
    DNA_HIP(launch_select_H(Xmu, Xn, H, part, fpart, 1, T, R, mask, dsel, margin, c.s), "select_H");
  } else {
    DNA_HIP(launch_cand_W(W, pu, puc, py, 1, c32, vpart, 1, N, R, o->eps, o->alpha, o->rho, Xmu, Xn, nullptr,
                          nullptr, c.s), "cand_W");
    DNA_HIP(launch_sp_diff(Xmu, Xn, Xd, N * R, c.s), "sp_diff");
    DNA_HIP(launch_sp_cost(1, v, Ht, Xn, Xd, N, T, R, at<double>(ws, L.cseg), at<int>(ws, L.fseg), part, fpart,
                           c.s, zo, dzo), "sp_cost_W");
    DNA_HIP(launch_select_W(Xmu, Xn, W, part, fpart, 1, N, R, mask, dsel, margin, c.s), "select_W");
  }
  return DNA_OK;
}

size_t dna_sparse_workspace_bytes(int64_t N, int64_t T, int64_t R, const dna_sparse_v* V, const dna_opts* o) {
  if (!V || !o || N <= 0 || T <= 0 || R <= 0 || V->nnz < 0) return 0;
  return make_sp_layout(N, T, R, V).total;
}

dna_status dna_sparse_update_H(const dna_sparse_v* V, const float* W, float* H, int64_t N, int64_t T, int64_t R,
                               const dna_opts* o, void* ws, size_t ws_bytes, uint8_t* chose_newton,
                               double* d_sel, double* margin, void* stream) {
  if (!W || !H) return fail(DNA_EINVAL, "W or H is NULL");
  SpCommon c;
  DNA_TRY(sp_prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  DNA_TRY(sp_half_step(0, V, const_cast<float*>(W), H, N, T, R, o, c, ws, chose_newton, d_sel, margin));
  return sp_epilogue(c);
}

dna_status dna_sparse_update_W(const dna_sparse_v* V, float* W, const float* H, int64_t N, int64_t T, int64_t R,
                               const dna_opts* o, void* ws, size_t ws_bytes, uint8_t* chose_newton,
                               double* d_sel, double* margin, void* stream) {
  if (!W || !H) return fail(DNA_EINVAL, "W or H is NULL");
  SpCommon c;
  DNA_TRY(sp_prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  DNA_TRY(sp_half_step(1, V, W, const_cast<float*>(H), N, T, R, o, c, ws, chose_newton, d_sel, margin));
  return sp_epilogue(c);
}

dna_status dna_sparse_kl_cost(const dna_sparse_v* V, const float* W, const float* H, int64_t N, int64_t T, int64_t R,
                              const dna_opts* o, void* ws, size_t ws_bytes, double* out, void* stream) {
  if (!W || !H || !out) return fail(DNA_EINVAL, "W, H or out is NULL");
  SpCommon c;
  DNA_TRY(sp_prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  const SpLayout& L = c.L;
  float* Ht = at<float>(ws, L.ht);
  double* sp = at<double>(ws, L.sump);
  DNA_HIP(launch_sp_transpose(H, Ht, R, T, c.s), "sp_transpose H");
  SumJob job;
  DNA_HIP(launch_colsum_part(W, N, R, sp, job, c.s), "colsum_W");
  job.s64 = at<double>(ws, L.c64);
  DNA_HIP(launch_sum_final(job, c.s), "sum_final c");
  DNA_HIP(launch_rowsum_part(H, T, R, sp, job, c.s), "rowsum_H");
  job.s64 = at<double>(ws, L.g64);
  DNA_HIP(launch_sum_final(job, c.s), "sum_final g");
  DNA_HIP(launch_sp_kl(sp_view(V), W, Ht, N, T, R, at<double>(ws, L.cseg), at<double>(ws, L.c64),
                       at<double>(ws, L.g64), out, c.s), "sp_kl");
  if (o->rho > 0.f || o->lambda > 0.f)
    DNA_HIP(launch_penalty(SumJob{at<double>(ws, L.c64), 1, R}, SumJob{at<double>(ws, L.g64), 1, R}, o->rho,
                           o->lambda, out, c.s), "penalty");
  return sp_epilogue(c);
}

// One sparse MU half-step on the prologue's state.
static dna_status sp_run_mu(int side, const dna_sparse_v* V, float* W, float* H, int64_t N, int64_t T, int64_t R,
                            const dna_opts* o, const SpCommon& c, void* ws) {
  const SpLayout& L = c.L;
  const SpV v = sp_view(V);
  float* Ht = at<float>(ws, L.ht);
  float* q = at<float>(ws, L.q);
  float* pu = at<float>(ws, L.pu);
  float* c32 = at<float>(ws, L.c32);
  double* c64 = at<double>(ws, L.c64);
  DNA_HIP(launch_sp_transpose(H, Ht, R, T, c.s), "sp_transpose H");
  SumJob job;
  if (side == 0) DNA_HIP(launch_colsum_part(W, N, R, at<double>(ws, L.sump), job, c.s), "colsum_W");
  else DNA_HIP(launch_rowsum_part(H, T, R, at<double>(ws, L.sump), job, c.s), "rowsum_H");
  job.s64 = c64; job.s32 = c32; job.check = c.chk; job.reg = side == 0 ? o->lambda : o->rho;
  DNA_HIP(launch_sp_zq(v, W, Ht, N, T, R, q, at<float>(ws, L.qb), c.chk, job, c.s), "sp_zq");
  DNA_HIP(launch_sp_grad(side, true, v, side == 0 ? W : Ht, q, nullptr, c64, N, T, R, at<float>(ws, L.gp),
                         nullptr, pu, nullptr, nullptr, nullptr, c.s), "sp_grad_mu");
  if (side == 0) DNA_HIP(launch_mu_H(H, pu, 1, c32, T, R, nullptr, 1, nullptr, c.s), "mu_H");
  else DNA_HIP(launch_mu_W(W, pu, 1, c32, N, R, nullptr, 1, nullptr, c.s), "mu_W");
  return DNA_OK;
}

dna_status dna_sparse_mu_update(int side, const dna_sparse_v* V, float* W, float* H, int64_t N, int64_t T,
                                int64_t R, const dna_opts* o, void* ws, size_t ws_bytes, void* stream) {
  if (!W || !H) return fail(DNA_EINVAL, "W or H is NULL");
  if (side != 0 && side != 1) return fail(DNA_EINVAL, "side must be 0 or 1");
  SpCommon c;
  DNA_TRY(sp_prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  DNA_TRY(sp_run_mu(side, V, W, H, N, T, R, o, c, ws));
  return sp_epilogue(c);
}

dna_status dna_sparse_mu_iterate(const dna_sparse_v* V, float* W, float* H, int64_t N, int64_t T, int64_t R,
                                 int iters, const dna_opts* o, void* ws, size_t ws_bytes, void* stream) {
  if (!W || !H) return fail(DNA_EINVAL, "W or H is NULL");
  if (iters < 0) return fail(DNA_EINVAL, "iters must be >= 0");
  SpCommon c;
  DNA_TRY(sp_prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  double* sp = at<double>(ws, c.L.sump);
  double* sp2 = at<double>(ws, c.L.sump2);
  for (int it = 0; it < iters; ++it) {
    DNA_TRY(sp_run_mu(0, V, W, H, N, T, R, o, c, ws));
    DNA_TRY(run_normalize(1, W, H, N, T, R, o, sp, sp2, c.chk, c.s, nullptr, nullptr));   // step 16
    DNA_TRY(sp_run_mu(1, V, W, H, N, T, R, o, c, ws));
    DNA_TRY(run_normalize(0, W, H, N, T, R, o, sp, sp2, c.chk, c.s, nullptr, nullptr));   // step 29
  }
  return sp_epilogue(c);
}

dna_status dna_sparse_iterate(const dna_sparse_v* V, float* W, float* H, int64_t N, int64_t T, int64_t R, int iters,
                              const dna_opts* o, void* ws, size_t ws_bytes, void* stream) {
  if (!W || !H) return fail(DNA_EINVAL, "W or H is NULL");
  if (iters < 0) return fail(DNA_EINVAL, "iters must be >= 0");
  SpCommon c;
  DNA_TRY(sp_prologue(V, W, H, N, T, R, o, ws, ws_bytes, stream, c));
  double* sp = at<double>(ws, c.L.sump);
  double* sp2 = at<double>(ws, c.L.sump2);
  double* se = at<double>(ws, c.L.sume);
  SumJob next;                                      // sums emitted by a normalisation (as in dna_iterate)
  bool have = false;
  for (int it = 0; it < iters; ++it) {                // Z carried from each selection to the next half-step
    DNA_TRY(sp_half_step(0, V, W, H, N, T, R, o, c, ws, nullptr, nullptr, nullptr, have ? &next : nullptr,
                         it > 0 ? 1 : -1, true));
    DNA_TRY(run_normalize(1, W, H, N, T, R, o, sp, sp2, c.chk, c.s, se, &next));           // step 16
    have = norm_side(o, 1) == 1;
    DNA_TRY(sp_half_step(1, V, W, H, N, T, R, o, c, ws, nullptr, nullptr, nullptr, have ? &next : nullptr, 0,
                         it + 1 < iters));
    DNA_TRY(run_normalize(0, W, H, N, T, R, o, sp, sp2, c.chk, c.s, se, &next));           // step 29
    have = norm_side(o, 0) == 0;
  }
  return sp_epilogue(c);
}

const char* dna_status_string(dna_status s) {
  switch (s) {
    case DNA_OK: return "DNA_OK";
    case DNA_EINVAL: return "DNA_EINVAL: invalid argument";
    case DNA_EWORKSPACE: return "DNA_EWORKSPACE: workspace too small";
    case DNA_EDOMAIN: return "DNA_EDOMAIN: input outside the domain of the method";
    case DNA_ENONFINITE: return "DNA_ENONFINITE: non-finite input";
    case DNA_EHIP: return "DNA_EHIP: HIP runtime error";
    case DNA_EUNSUPPORTED: return "DNA_EUNSUPPORTED: not supported by this library";
  }
  return "unknown dna_status";
}

const char* dna_last_error(void) { return g_err; }

void dna_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof = on != 0;
}

void dna_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_pending) {
    hipEventSynchronize(r.b ? r.b : r.a);
    g_pool.push_back(r.a);
    if (r.b) g_pool.push_back(r.b);
  }
  g_pending.clear();
  g_stats.clear();
}

int dna_profile_read(dna_kernel_stat* out, int max_entries) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_pending) {
    float ms = 0.f;
    if (r.b && hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& e = g_stats[r.name];
      e.first += 1;
      e.second += ms;
    }
    g_pool.push_back(r.a);
    if (r.b) g_pool.push_back(r.b);
  }
  g_pending.clear();
  g_names.clear();
  for (auto& kv : g_stats) g_names.push_back(kv.first);
  int i = 0;
  for (auto& kv : g_stats) {
    if (out && i < max_entries) {
      out[i].name = g_names[i].c_str();
      out[i].launches = kv.second.first;
      out[i].total_ms = kv.second.second;
    }
    ++i;
  }
  return (int)g_stats.size();
}

const char* dna_build_info(void) {
  return "libdna gfx950 fp32-mfma32x32x2"
#ifdef DNA_BUILD_FLAGS
         " " DNA_BUILD_FLAGS
#endif
      ;
}

}  // extern "C"
