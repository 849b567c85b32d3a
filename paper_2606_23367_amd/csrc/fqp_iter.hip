// ADMM iteration kernels for the batched factor-model QP (gfx950).
//
// Splitting (project's choice; the paper's engine is closed, Sec. "Claim
// Boundary"): x carries the smooth risk/return part of Eq. 1 plus the budget,
// z carries every separable term (box, exclusion, L1 turnover, piecewise-
// linear tax) and the turnover cap, and y = A x carries the exposure bands:
//
//   x-step   (gamma Sigma + rho I + rho_b A^T A) x = mu + rho(z - u)
//            + rho_b A^T (y - v) + nu 1,   1^T x = 1
//   relax    xh = alpha x + (1 - alpha) z
//   z-step   z = prox_{psi/rho}(xh + u)  with the cap multiplier lam
//   duals    u += xh - z;   band block: OSQP-style relaxation on A x
//
// Sigma = B diag(f) B^T + diag(d) and the one-hot A^T A are both low rank,
// so with B~ = [B | A^T] and Delta = gamma d + rho the x-step is a Woodbury
// solve in the (k+G)-dimensional factor space:
//
//   t = B~^T Delta^-1 r,  s0 = 1^T Delta^-1 r,
//   nu = (1 - s0 + q^T t) / sigma1,  p = K^-1 (t + nu c),
//   x = Delta^-1 (r + nu 1 - B~ p),
//   K = F~^-1 + B~^T Delta^-1 B~,  c = B~^T Delta^-1 1,  q = K^-1 c,
//   sigma1 = 1^T Delta^-1 1 - c^T q.
//
// The ADMM state kept per (account, asset) is v = xh + u.  With z = prox(v)
// and r = mu + rho (z - u) the update of v splits into a part every row
// computes alone and the back-projection,
//   v' = alpha x + (1 - alpha) z + u = w + alpha Delta^-1 (nu - (B~ p)_i),
//   w  = v + alpha (Delta^-1 r - z),
// so one iteration is four launches (below): PROX, per account, finds the
// exact turnover-cap multiplier lam* of v (a safeguarded Newton search on
// the piecewise-linear turnover) and writes R' = r / Delta and w for every
// row -- the only pass that reads the row data (masks, holdings, tax
// records); CONTRACT contracts R' with B~ (MFMA) into per-row-tile partials
// of t = B~^T R'; a small per-account kernel reduces the partials and solves
// in factor space (nu, p); PROJECT streams w and applies the back-projection
// B~ p (MFMA), writing the new v.
#include <algorithm>

#include <hip/hip_ext.h>

#include "fqp_common.h"
#include "fqp_kernels.h"
#include "../../include/fqp.h"

namespace fqp {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// ---------------------------------------------------------------------------
// universe packing:  B~ = [B | onehot(group) | H^T | 1 | 0]
// (the halfspace rows enter the x-update as further low-rank directions,
// exactly as the one-hot band rows do)
// ---------------------------------------------------------------------------
__global__ void build_bt_kernel(int n, int k, int G, int H, int kp, const float* B,
                                const int32_t* group, const float* half, float* Bt) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t total = (size_t)n * kp;
  if (e >= total) return;
  int i = (int)(e / kp), j = (int)(e % kp);
  float v = 0.f;
  if (j < k) v = B[(size_t)i * k + j];
  else if (j < k + G) v = (group[i] == j - k) ? 1.f : 0.f;
  else if (j < k + G + H) v = half[(size_t)(j - k - G) * n + i];
  else if (j == k + G + H) v = 1.f;
  Bt[e] = v;
}

// partial Gram  sum_i B~_ij B~_il / Delta_i  over a chunk of rows, for
// j, l <= kg (kg = k + G; index kg is the ones column), float64.  Grid:
// x = row chunk, y = tile of 8192 matrix entries (32 per thread).
__global__ __launch_bounds__(256) void gram_partial_kernel(
    int n, int kp, int kg, int rows_per_blk, const float* Bt, const float* d,
    double gamma, double rho, double* part) {
  extern __shared__ float sB[];               // [64][kp]
  const int nk = kg + 1;
  const int ne = nk * nk;
  const int e0 = blockIdx.y * 8192;
  const int r_begin = blockIdx.x * rows_per_blk;
  const int r_end = min(n, r_begin + rows_per_blk);
  double acc[32];
  int jj[32], ll[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) {
    acc[c] = 0.0;
    int e = e0 + threadIdx.x + 256 * c;
    jj[c] = (e < ne) ? e / nk : 0;
    ll[c] = (e < ne) ? e % nk : 0;
  }
  for (int r0 = r_begin; r0 < r_end; r0 += 64) {
    __syncthreads();
    int rows = min(64, r_end - r0);
    for (int e = threadIdx.x; e < rows * kp; e += blockDim.x)
      sB[e] = Bt[(size_t)r0 * kp + e];
    __syncthreads();
    for (int rr = 0; rr < rows; ++rr) {
      const double idl = 1.0 / (gamma * (double)d[r0 + rr] + rho);
      const float* row = sB + rr * kp;
#pragma unroll
      for (int c = 0; c < 32; ++c)
        acc[c] += (double)row[jj[c]] * (double)row[ll[c]] * idl;
    }
  }
#pragma unroll
  for (int c = 0; c < 32; ++c) {
    int e = e0 + threadIdx.x + 256 * c;
    if (e < ne) part[(size_t)blockIdx.x * ne + e] = acc[c];
  }
}

// the Gram matrix: the row-block partials summed in block order, one entry
// per thread (Gm = the first (kg + 1)^2 doubles of Kw)
__global__ __launch_bounds__(256) void gram_reduce_kernel(int ne, int nparts, const double* part,
                                                          double* Gm) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= ne) return;
  double s = 0.0;
  int p = 0;
  for (; p + 8 <= nparts; p += 8) {
    double b[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) b[u] = part[(size_t)(p + u) * ne + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += b[u];
  }
  for (; p < nparts; ++p) s += part[(size_t)p * ne + e];
  Gm[e] = s;
}

// add F~^-1 to the Gram matrix, invert, border vectors.  One workgroup of
// 16 waves per class, everything in float64.  kg <= kKfLds: K is inverted by
// Gauss-Jordan elimination with the matrix held in registers (a wave owns
// rows, its lanes two columns each); wider blocks are factored (Cholesky)
// and inverted by triangular sweeps in the global scratch Kw
constexpr int kKfLds = 96;
constexpr int kKfRows = kKfLds / 16;     // rows per wave of the in-register inversion (16 waves)

__global__ __launch_bounds__(1024) void kfactor_kernel(int k, int G, int kp, int nparts,
                               const double* part, const float* f,
                               double gamma, double rho_b, double* Kw,
                               float* Kinv_out, float* c_out, float* q_out,
                               float* sig_out, float* mbg_out) {
  extern __shared__ double kf_smem[];
  const int kg = k + G, nk = kg + 1, ne = nk * nk;
  const bool in_lds = kg <= kKfLds;
  double* Gm = Kw;                   // [nk][nk]
  // [kg][kg]: K, then (wide blocks) its Cholesky factor
  double* L = in_lds ? kf_smem : Kw + ne;
  double* X = in_lds ? kf_smem : L + kg * kg;             // [kg][kg] K^-1
  // LDS after X (in-register path) or from its start (wide blocks): the
  // border column c with its last entry (c_kg = 1^T Delta^-1 1), then q
  double* cv = in_lds ? kf_smem + kg * kg + 4 * kg : kf_smem;   // [kg + 1]
  double* qs = cv + kg + 1;                                     // [kg]
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);
  // (Gm holds the sum of the row-block partials: gram_reduce_kernel)
  (void)part;
  (void)nparts;
  for (int j = threadIdx.x; j <= kg; j += blockDim.x) cv[j] = Gm[j * nk + kg];
  auto k_entry = [&](int j, int l) {
    double v = Gm[j * nk + l];
    if (j == l) v += (j < k) ? 1.0 / (gamma * (double)f[j]) : 1.0 / rho_b;
    return v;
  };
  if (in_lds) {
    // K^-1 by Gauss-Jordan elimination in place: K is symmetric positive
    // definite, so every pivot is positive and no row exchange is needed.
    // Step p scales row p by 1 / K_pp (its own entry becomes 1 / K_pp) and
    // removes column p from every other row.  Thread (wave w, lane) keeps
    // entries (w + 16 t, lane) and (w + 16 t, lane + 64) in registers for
    // the whole elimination; a step exchanges only row p and column p,
    // through a pair of LDS buffers used alternately, so one barrier per
    // step orders the writes of step p + 1 after every read of step p - 1.
    double* rbuf = kf_smem + kg * kg;        // [2][kg] row p before scaling
    double* cbuf = rbuf + 2 * kg;            // [2][kg] column p before the step
    // every load is issued before any is used (indices clamped into the
    // matrix, out-of-range entries set to zero afterwards)
    const int c0 = min(lane, kg - 1), c1 = min(lane + 64, kg - 1);
    const double fd0 = c0 < k ? (double)f[c0] : 1.0, fd1 = c1 < k ? (double)f[c1] : 1.0;
    double x0[kKfRows], x1[kKfRows];
#pragma unroll
    for (int t = 0; t < kKfRows; ++t) {
      const int i = min(wv + nw * t, kg - 1);
      x0[t] = Gm[i * nk + c0];
      x1[t] = Gm[i * nk + c1];
    }
    const double dg0 = c0 < k ? 1.0 / (gamma * fd0) : 1.0 / rho_b;
    const double dg1 = c1 < k ? 1.0 / (gamma * fd1) : 1.0 / rho_b;
#pragma unroll
    for (int t = 0; t < kKfRows; ++t) {
      const int i = wv + nw * t;
      x0[t] = (i < kg && lane < kg) ? x0[t] + (i == lane ? dg0 : 0.0) : 0.0;
      x1[t] = (i < kg && lane + 64 < kg) ? x1[t] + (i == lane + 64 ? dg1 : 0.0) : 0.0;
    }
    for (int p = 0; p < kg; ++p) {
      double* rb = rbuf + (p & 1) * kg;
      double* cb = cbuf + (p & 1) * kg;
      const int pl = p & 63;
      const bool phi = p >= 64;
#pragma unroll
      for (int t = 0; t < kKfRows; ++t) {
        const int i = wv + nw * t;
        if (i == p) {
          if (lane < kg) rb[lane] = x0[t];
          if (lane + 64 < kg) rb[lane + 64] = x1[t];
        }
        if (i < kg && lane == pl) cb[i] = phi ? x1[t] : x0[t];
      }
      __syncthreads();
      // all of this step's LDS reads at once (clamped indices)
      const double piv = rb[p], a0 = rb[c0], a1 = rb[c1];
      double cr[kKfRows];
#pragma unroll
      for (int t = 0; t < kKfRows; ++t) cr[t] = cb[min(wv + nw * t, kg - 1)];
      const double ip = 1.0 / piv;
      const double r0 = lane < kg ? (lane == p ? 1.0 : a0) * ip : 0.0;
      const double r1 = lane + 64 < kg ? (lane + 64 == p ? 1.0 : a1) * ip : 0.0;
#pragma unroll
      for (int t = 0; t < kKfRows; ++t) {
        const int i = wv + nw * t;
        const double c = (i < kg && i != p) ? cr[t] : 0.0;
        x0[t] = (i == p) ? r0 : ((lane == p) ? 0.0 : x0[t]) - c * r0;
        x1[t] = (i == p) ? r1 : ((lane + 64 == p) ? 0.0 : x1[t]) - c * r1;
      }
    }
#pragma unroll
    for (int t = 0; t < kKfRows; ++t) {
      const int i = wv + nw * t;
      if (i < kg && lane < kg) X[i * kg + lane] = x0[t];
      if (i < kg && lane + 64 < kg) X[i * kg + lane + 64] = x1[t];
    }
    __syncthreads();
  } else {
  for (int e = threadIdx.x; e < kg * kg; e += blockDim.x) L[e] = k_entry(e / kg, e % kg);
  __syncthreads();
  // right-looking Cholesky, lower triangle of L
  for (int j = 0; j < kg; ++j) {
    if (threadIdx.x == 0) L[j * kg + j] = sqrt(fmax(L[j * kg + j], 1e-300));
    __syncthreads();
    double djj = L[j * kg + j];
    for (int i = j + 1 + threadIdx.x; i < kg; i += blockDim.x)
      L[i * kg + j] /= djj;
    __syncthreads();
    for (int e = threadIdx.x; e < (kg - j - 1) * (kg - j - 1); e += blockDim.x) {
      int i = j + 1 + e / (kg - j - 1), l = j + 1 + e % (kg - j - 1);
      if (l <= i) L[i * kg + l] -= L[i * kg + j] * L[l * kg + j];
    }
    __syncthreads();
  }
  // inverse: L L^T X = I
  for (int e = threadIdx.x; e < kg * kg; e += blockDim.x) X[e] = (e / kg == e % kg) ? 1.0 : 0.0;
  __syncthreads();
  {
  // right-looking forward and backward sweeps, every thread updating a
  // slice of the trailing block at each step
  for (int j = 0; j < kg; ++j) {
    const double djj = L[j * kg + j];
    for (int c = threadIdx.x; c < kg; c += blockDim.x) X[j * kg + c] /= djj;
    __syncthreads();
    for (int e = threadIdx.x; e < (kg - j - 1) * kg; e += blockDim.x) {
      const int i = j + 1 + e / kg, c = e % kg;
      X[i * kg + c] -= L[i * kg + j] * X[j * kg + c];
    }
    __syncthreads();
  }
  for (int j = kg - 1; j >= 0; --j) {
    const double djj = L[j * kg + j];
    for (int c = threadIdx.x; c < kg; c += blockDim.x) X[j * kg + c] /= djj;
    __syncthreads();
    for (int e = threadIdx.x; e < j * kg; e += blockDim.x) {
      const int i = e / kg, c = e % kg;
      X[i * kg + c] -= L[j * kg + i] * X[j * kg + c];
    }
    __syncthreads();
  }
  }
  }
  // q = K^-1 c, a wave per row; sigma1 = 1^T Delta^-1 1 - c^T q
  for (int j = wv; j < kg; j += nw) {
    double s = 0.0;
    for (int l = lane; l < kg; l += 64) s += X[j * kg + l] * cv[l];
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) qs[j] = s;
  }
  __syncthreads();
  if (wv == 0) {
    double s = 0.0;
    for (int l = lane; l < kg; l += 64) s += cv[l] * qs[l];
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (lane == 0) sig_out[0] = (float)(cv[kg] - s);
  }
  for (int e = threadIdx.x; e < kp * kp; e += blockDim.x) {
    int j = e / kp, l = e % kp;
    Kinv_out[e] = (j < kg && l < kg) ? (float)X[j * kg + l] : 0.f;
  }
  for (int j = threadIdx.x; j < kp; j += blockDim.x) {
    c_out[j] = (j < kg) ? (float)cv[j] : 0.f;
    q_out[j] = (j < kg) ? (float)qs[j] : 0.f;
  }
  for (int e = threadIdx.x; e < kp * G; e += blockDim.x) {
    int j = e / G, g = e % G;
    mbg_out[e] = (j < kg) ? (float)Gm[j * nk + (k + g)] : 0.f;
  }
}

// ---------------------------------------------------------------------------
// the fused passes
//
// The ADMM state kept in HBM is v = xh + u per (account, asset).  One
// iteration is
//   PROX      lam* of v (per account, exact); z = prox(v; lam*), u = v - z,
//             r = mu + rho (z - u); R' = r / Delta and
//             w = v + alpha (R' - z) written
//   CONTRACT  t = B~^T R' (MFMA), per row tile
//   k-solve   nu, p from t (factor space)
//   PROJECT   v <- w + alpha Delta^-1 (nu - B~ p)   (MFMA)
// ---------------------------------------------------------------------------
enum PassMode { MODE_CONTRACT = 0, MODE_PROJECT = 1 };

struct RowInfo {
  float lb, ub, w0;
  bool taxed;
  TaxLots t;
};

__device__ __forceinline__ float prox_row(const RowInfo& ri, float v, float th, float irho,
                                          bool* at_kink) {
  float zn;
  if (ri.taxed) {
    zn = prox_taxed(v, ri.w0, th, irho, ri.t, ri.lb, ri.ub);
    if (at_kink)
      *at_kink = (zn == ri.w0) || (zn == ri.w0 - ri.t.b1) || (zn == ri.w0 - ri.t.b2) ||
                 (zn == ri.w0 - ri.t.b3) || zn <= ri.lb || zn >= ri.ub;
  } else {
    zn = prox_plain(v, ri.w0, th, ri.lb, ri.ub);
    if (at_kink) *at_kink = (zn == ri.w0) || zn <= ri.lb || zn >= ri.ub;
  }
  return zn;
}

// box, w0 and tax lots of (account a, row) from its eligibility word, its
// holding word and the holding prefix word (already loaded) and the
// account's first record hptr: one more dependent load, only for held rows
template <typename Args>
__device__ __forceinline__ RowInfo row_info_w(const Args& A, size_t off, int row, float lbp,
                                              float ubp, uint32_t ew, uint32_t hw, int hpre,
                                              int hptr) {
  RowInfo ri;
  const int b = row & 31;
  const bool el = (ew >> b) & 1u;
  asset_box(A, off, el, lbp, ubp, ri.lb, ri.ub);
  ri.w0 = 0.f;
  ri.taxed = false;
  if ((hw >> b) & 1u) {
    const int idx = hptr + hpre + popc_below(hw, b);
    const float4 r0 = A.hold_rec[2 * idx], r1 = A.hold_rec[2 * idx + 1];
    ri.w0 = r0.x;
    ri.taxed = r0.y > 0.f;
    ri.t.b1 = r0.y; ri.t.b2 = r0.z; ri.t.b3 = r0.w;
    ri.t.s0 = r1.x; ri.t.s1 = r1.y; ri.t.s2 = r1.z; ri.t.s3 = r1.w;
  }
  return ri;
}

template <typename Args>
__device__ __forceinline__ RowInfo row_info(const Args& A, int a, int row, float lbp, float ubp) {
  const size_t wi = (size_t)a * A.W + (row >> 5);
  const uint32_t ew = A.elig ? A.elig[wi] : 0xffffffffu;
  return row_info_w(A, (size_t)a * A.n + row, row, lbp, ubp, ew, A.hold[wi], A.hold_pre[wi],
                    A.hold_ptr[a]);
}

template <int NCH, int MODE>
__global__ __launch_bounds__(256, 2) void iter_kernel(IterArgs A) {
  constexpr int kp = NCH * 32;
  constexpr int BS = kp + 1;            // LDS row stride (odd: no conflicts)
  extern __shared__ float smem[];
  float* Bs = smem;                     // [128][BS]
  // mode-specific region: PROJECT keeps p (32 x BS) and a [4][32] max
  // reduction, CONTRACT the per-wave transposes of R' ([4][32][33])
  constexpr int kXs = (MODE == MODE_PROJECT) ? kTM * BS + kWaves * kTM : kWaves * 32 * 33;
  float* Xs = Bs + kRowsPerChunk * BS;
  float* Ps = Xs;                       // PROJECT: [32][BS]
  float* Rt = Xs;                       // CONTRACT: [4][32][33]
  // per tile account: {rho, 1/rho, gamma, (kappa + lam)/rho}, {lb, ub, nu, alpha}
  float4* Acc = reinterpret_cast<float4*>(Xs + kXs);   // [32][2]
  int* Aid = (int*)(Acc + 2 * kTM);     // [32]
  int* Hp = Aid + kTM;                  // [32] first held record of each account
  int* Ao = Hp + kTM;                   // [32] a * n (element offset of the account)
  int* Wo = Ao + kTM;                   // [32] a * W (bitmask word offset)

  const int m_act = *A.m_act;
  const TileMap tm = tile_map(m_act, A.n, gridDim.x * gridDim.y,
                              blockIdx.y * gridDim.x + blockIdx.x);
  if (!tm.active) return;
  const int slot0 = tm.tile * kTM;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int l32 = lane & 31, hi = lane >> 5;
  const int n = A.n;

  if (tid < kTM) {
    int s = slot0 + tid;
    const int a = (s < m_act) ? A.act[s] : -1;
    Aid[tid] = a;
    Hp[tid] = (a >= 0) ? A.hold_ptr[a] : 0;
    Ao[tid] = (a >= 0) ? a * n : 0;        // m n < 2^31 (checked by the runtime)
    Wo[tid] = (a >= 0) ? a * A.W : 0;
    float4 q0 = make_float4(1.f, 1.f, 0.f, 0.f), q1 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (a >= 0) {
      const float* p = A.par + (size_t)a * kNPar;
      const float rho = p[P_RHO], irho = 1.f / rho;
      q0 = make_float4(rho, irho, p[P_GAMMA], (p[P_KAPPA] + p[P_LAM]) * irho);
      q1 = make_float4(p[P_LB], p[P_UB], p[P_NU], p[P_ALPHA]);
    }
    Acc[2 * tid] = q0;
    Acc[2 * tid + 1] = q1;
  }
  __syncthreads();
  if (MODE == MODE_PROJECT) {
    for (int e = tid; e < kTM * kp; e += 256) {
      int j = e / kp, c = e % kp;
      int a = Aid[j];
      Ps[j * BS + c] = (a >= 0) ? A.pp[(size_t)a * kp + c] : 0.f;
    }
  }

  floatx16 T[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) T[c][r] = 0.f;
  float* Rw = Rt + w * 32 * 33;
  const int row_begin = tm.row_begin;

  for (int ch = 0; ch < tm.chunks; ++ch) {
    const int r0 = row_begin + ch * kRowsPerChunk;
    if (r0 >= n) break;
    __syncthreads();
    for (int e = tid; e < kRowsPerChunk * (kp / 4); e += 256) {
      int rr = e / (kp / 4), c4 = e % (kp / 4);
      int row = r0 + rr;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (row < n) v = reinterpret_cast<const float4*>(A.Bt + (size_t)row * kp)[c4];
      float* dst = Bs + rr * BS + 4 * c4;
      dst[0] = v.x; dst[1] = v.y; dst[2] = v.z; dst[3] = v.w;
    }
    __syncthreads();

    const int row = r0 + 32 * w + l32;
    const bool row_ok = row < n;
    const float d_i = row_ok ? A.d[row] : 1.f;

    floatx16 X;
#pragma unroll
    for (int r = 0; r < 16; ++r) X[r] = 0.f;
    if (MODE == MODE_PROJECT) {
      const float* pa = Ps + l32 * BS + hi;
      const float* pb = Bs + (32 * w + l32) * BS + hi;
#pragma unroll 8
      for (int s = 0; s < kp / 2; ++s)
        X = __builtin_amdgcn_mfma_f32_32x32x2f32(pa[2 * s], pb[2 * s], X, 0, 0, 0);
    }

    if (MODE == MODE_PROJECT) {
      // v' = w + alpha Delta^-1 (nu - (B~ p)_i), w from the CONTRACT pass
      float w_r[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = 8 * (r >> 2) + 4 * hi + (r & 3);
        w_r[r] = (Aid[m] >= 0 && row_ok) ? A.zs[(unsigned)(Ao[m] + row)] : 0.f;
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int m = 8 * (r >> 2) + 4 * hi + (r & 3);
        if (Aid[m] >= 0 && row_ok) {
          const float4 q0 = Acc[2 * m], q1 = Acc[2 * m + 1];
          const float iDelta = __builtin_amdgcn_rcpf(q0.z * d_i + q0.x);
          A.v[(unsigned)(Ao[m] + row)] = w_r[r] + q1.w * iDelta * (q1.z - X[r]);
        }
      }
      continue;
    }

    // R' = r / Delta of the lane's 16 (account, row) elements, from the
    // PROX pass, through a per-wave LDS transpose into the MFMA A operand
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = 8 * (r >> 2) + 4 * hi + (r & 3);
      const int a = Aid[m];
      Rw[m * 33 + l32] = (a >= 0 && row_ok) ? A.rp[(size_t)a * A.npad + row] : 0.f;
    }
    if (MODE == MODE_CONTRACT) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      const float* ra = Rw + l32 * 33 + hi;
      const float* rb = Bs + (32 * w + hi) * BS + l32;
#pragma unroll 4
      for (int s = 0; s < 16; ++s) {
        const float av = ra[2 * s];
#pragma unroll
        for (int c = 0; c < NCH; ++c)
          T[c] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, rb[(2 * s) * BS + 32 * c], T[c], 0, 0, 0);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }

  const size_t M = A.m_total;
  if (MODE == MODE_PROJECT) return;

  __syncthreads();                       // all waves done with Bs / Rt
  float* red = Bs;                       // [4][32][kp]
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = 8 * (r >> 2) + 4 * hi + (r & 3);
      red[(w * kTM + m) * kp + 32 * c + l32] = T[c][r];
    }
  __syncthreads();
  for (int e = tid; e < kTM * kp; e += 256) {
    const int m = e / kp, c = e % kp;
    const int a = Aid[m];
    if (a < 0) continue;
    float s = red[(0 * kTM + m) * kp + c] + red[(1 * kTM + m) * kp + c] +
              red[(2 * kTM + m) * kp + c] + red[(3 * kTM + m) * kp + c];
    A.part[((size_t)tm.rt * M + a) * kp + c] = s;
  }
}

// ---------------------------------------------------------------------------
// the same two passes with the contractions on bf16 MFMA (32x32x16)
//
// Every float32 operand x enters as the pair hi = bf16(x), lo = bf16(x - hi)
// and each product as hi*hi + hi*lo + lo*hi with float32 accumulation: the
// dropped lo*lo term and the rounding of lo leave a relative error of about
// 2^-16 per product, against 2^-24 for the float32 MFMA, at an eighth of the
// matrix-core time.  B~ is split once per solve into row-major (PROJECT) and
// column-major (CONTRACT) copies whose rows are padded with zeros to a whole
// number of chunks, so that the operands come straight from global memory
// (no LDS staging, no workgroup barrier inside the row loop).
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ void split_bf16(float x, __bf16& h, __bf16& l) {
  h = (__bf16)x;
  l = (__bf16)(x - (float)h);
}

template <int NCH, int MODE>
constexpr int bf_lds_floats() {
  // CONTRACT: the cross-wave reduction of the partial sums [4][32][kp];
  // PROJECT: the split p of the tile (hi, lo) [2][32][kp + 8] bf16 (after
  // 4 x 32 unused floats)
  return (MODE == MODE_CONTRACT) ? kWaves * kTM * NCH * 32
                                 : kWaves * kTM + kTM * (NCH * 32 + 8);
}

template <int NCH, int MODE>
__global__ __launch_bounds__(256, 3) void iter_kernel_bf(IterArgs A) {
  constexpr int kp = NCH * 32;
  constexpr int KS = kp / 16;            // K steps of the PROJECT product
  constexpr int kX = bf_lds_floats<NCH, MODE>();
  extern __shared__ float smem[];
  float* Xs = smem;
  float4* Acc = reinterpret_cast<float4*>(Xs + kX);    // [32] PROJECT constants (room for [32][2])
  int* Aid = (int*)(Acc + 2 * kTM);     // [32]
  int* Ao = Aid + kTM;                  // [32] a * n

  const int m_act = *A.m_act;
  const TileMap tm = tile_map(m_act, A.n, gridDim.x * gridDim.y,
                              blockIdx.y * gridDim.x + blockIdx.x);
  if (!tm.active) return;
  const int slot0 = tm.tile * kTM;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int l32 = lane & 31, hi = lane >> 5;
  const int n = A.n;
  const __bf16* bh = reinterpret_cast<const __bf16*>(A.bt_hi);
  const __bf16* bl = reinterpret_cast<const __bf16*>(A.bt_lo);
  const __bf16* bth = reinterpret_cast<const __bf16*>(A.btt_hi);
  const __bf16* btl = reinterpret_cast<const __bf16*>(A.btt_lo);

  if (tid < kTM) {
    int s = slot0 + tid;
    const int a = (s < m_act) ? A.act[s] : -1;
    Aid[tid] = a;
    Ao[tid] = (a >= 0) ? a * n : 0;        // m n < 2^31 (checked by the runtime)
    // PROJECT: {rho, gamma, nu, alpha} of the account
    float4 q = make_float4(1.f, 0.f, 0.f, 0.f);
    if (MODE == MODE_PROJECT && a >= 0) {
      const float* p = A.par + (size_t)a * kNPar;
      q = make_float4(p[P_RHO], p[P_GAMMA], p[P_NU], p[P_ALPHA]);
    }
    Acc[tid] = q;
  }
  __syncthreads();

  // PROJECT: the A operand (p of the tile's accounts), split once per
  // workgroup into LDS: PsH / PsL [32][kp + 8] bf16 (16-byte aligned rows)
  constexpr int PS = kp + 8;
  __bf16* PsH = reinterpret_cast<__bf16*>(Xs + kWaves * kTM);
  __bf16* PsL = PsH + kTM * PS;
  if (MODE == MODE_PROJECT) {
    for (int e = tid; e < kTM * kp; e += 256) {
      const int j = e / kp, c = e % kp;
      const int a = Aid[j];
      const float x = (a >= 0) ? A.pp[(size_t)a * kp + c] : 0.f;
      __bf16 h, l;
      split_bf16(x, h, l);
      PsH[j * PS + c] = h;
      PsL[j * PS + c] = l;
    }
    __syncthreads();
  }

  floatx16 T[NCH];
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) T[c][r] = 0.f;
  const int row_begin = tm.row_begin;
  // PROJECT: the lane's 16 accounts (MFMA output rows m = 8 (r / 4) + 4 hi +
  // r % 4): offset a n of each, -1 for an empty slot of the tile
  int ao[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int m = 8 * (r >> 2) + 4 * hi + (r & 3);
    ao[r] = (MODE == MODE_PROJECT && Aid[m] >= 0) ? Ao[m] : -1;
  }

  for (int ch = 0; ch < tm.chunks; ++ch) {
    const int r0 = row_begin + ch * kRowsPerChunk;
    if (r0 >= n) break;
    const int row_base = r0 + 32 * w;     // < npad: rows are padded to whole chunks
    const int row = row_base + l32;
    const bool row_ok = row < n;

    if (MODE == MODE_PROJECT) {
      // w of this iterate comes from the PROX pass: no row data, no returns
      // and no old state needed here.  Every load of the chunk is issued
      // before the first is used (an empty slot reads element 0 and drops
      // it), so that the chunk costs one memory round trip.
      const float d_i = row_ok ? A.d[row] : 1.f;
      float w_r[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const bool ok = ao[r] >= 0 && row_ok;
        w_r[r] = A.zs[ok ? (unsigned)(ao[r] + row) : 0u];
      }
      // the wave's 32 rows x 16 columns per K step in MFMA operand order: 1 KB
      const size_t ob = (size_t)(row_base >> 5) * KS * 512 + (size_t)(hi * 32 + l32) * 8;
      bf16x8 bH[KS], bL[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        bH[s] = *reinterpret_cast<const bf16x8*>(bh + ob + (size_t)s * 512);
        bL[s] = *reinterpret_cast<const bf16x8*>(bl + ob + (size_t)s * 512);
      }
      // (keeps the scheduler from sinking the loads towards their uses)
      __builtin_amdgcn_sched_barrier(0);
      floatx16 X;
#pragma unroll
      for (int r = 0; r < 16; ++r) X[r] = 0.f;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const bf16x8 pH = *reinterpret_cast<const bf16x8*>(PsH + l32 * PS + 16 * s + 8 * hi);
        const bf16x8 pL = *reinterpret_cast<const bf16x8*>(PsL + l32 * PS + 16 * s + 8 * hi);
        X = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pH, bH[s], X, 0, 0, 0);
        X = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pH, bL[s], X, 0, 0, 0);
        X = __builtin_amdgcn_mfma_f32_32x32x16_bf16(pL, bH[s], X, 0, 0, 0);
      }
      // v' = w + alpha Delta^-1 (nu - (B~ p)_i), four accounts' constants
      // read together
#pragma unroll
      for (int g4 = 0; g4 < 4; ++g4) {
        float4 q[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) q[j] = Acc[8 * g4 + 4 * hi + j];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int r = 4 * g4 + j;
          if (ao[r] >= 0 && row_ok) {
            const float iDelta = __builtin_amdgcn_rcpf(q[j].y * d_i + q[j].x);
            A.v[(unsigned)(ao[r] + row)] = w_r[r] + q[j].w * iDelta * (q[j].z - X[r]);
          }
        }
      }
    } else if (row_base < n) {            // uniform per wave
      // A operand straight from R' (PROX pass): lane l32 takes account
      // Aid[l32], rows row_base + 16 s + 8 hi .. + 8 (the rows past n of the
      // last chunk are masked: R' is not written there).  Both K steps' R'
      // and B~ operands are loaded before any is used: one memory round
      // trip per chunk.
      const int am = Aid[l32];
      float4 x[2][2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int rb = row_base + 16 * s + 8 * hi;
        // (an empty slot of the tile reads account 0's rows and drops them)
        const float4* src =
            reinterpret_cast<const float4*>(A.rp + (size_t)(am >= 0 ? am : 0) * A.npad + rb);
        x[s][0] = src[0];
        x[s][1] = src[1];
      }
      // 16 rows x 32 columns per K step and column block in MFMA operand
      // order: 1 KB
      bf16x8 bH[2][NCH], bL[2][NCH];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          const size_t o = ((size_t)((row_base >> 4) + s) * NCH + c) * 512 +
                           (size_t)(hi * 32 + l32) * 8;
          bH[s][c] = *reinterpret_cast<const bf16x8*>(bth + o);
          bL[s][c] = *reinterpret_cast<const bf16x8*>(btl + o);
        }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int rb = row_base + 16 * s + 8 * hi;
        float rv[8] = {x[s][0].x, x[s][0].y, x[s][0].z, x[s][0].w,
                       x[s][1].x, x[s][1].y, x[s][1].z, x[s][1].w};
#pragma unroll
        for (int j = 0; j < 8; ++j) rv[j] = (am >= 0 && rb + j < n) ? rv[j] : 0.f;
        bf16x8 aH, aL;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 h, l;
          split_bf16(rv[j], h, l);
          aH[j] = h;
          aL[j] = l;
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          T[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aH, bH[s][c], T[c], 0, 0, 0);
          T[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aH, bL[s][c], T[c], 0, 0, 0);
          T[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aL, bH[s][c], T[c], 0, 0, 0);
        }
      }
    }
  }

  const size_t M = A.m_total;
  if (MODE == MODE_PROJECT) return;

  __syncthreads();                       // all waves done with their transposes
  float* red = Xs;                       // [4][32][kp]
#pragma unroll
  for (int c = 0; c < NCH; ++c)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int m = 8 * (r >> 2) + 4 * hi + (r & 3);
      red[(w * kTM + m) * kp + 32 * c + l32] = T[c][r];
    }
  __syncthreads();
  for (int e = tid; e < kTM * kp; e += 256) {
    const int m = e / kp, c = e % kp;
    const int a = Aid[m];
    if (a < 0) continue;
    float s = red[(0 * kTM + m) * kp + c] + red[(1 * kTM + m) * kp + c] +
              red[(2 * kTM + m) * kp + c] + red[(3 * kTM + m) * kp + c];
    A.part[((size_t)tm.rt * M + a) * kp + c] = s;
  }
}

// hi/lo bf16 copies of B~ (rows n..npad-1 zero), each in the operand order
// of one pass's MFMA, so that a wave's operand load is 1 KB of contiguous
// memory (64 lanes x 8 bf16) instead of 16 bytes from each of 32 rows or
// columns:
//   bh / bl (PROJECT, B operand: lane = row, 8 consecutive columns):
//     [npad / 32 row blocks][kp / 16 column steps][hi][l32 = row][8 columns]
//   bth / btl (CONTRACT, B operand: lane = column, 8 consecutive rows):
//     [npad / 16 row steps][kp / 32 column blocks][hi][l32 = column][8 rows]
__global__ void split_bt_kernel(int n, int npad, int kp, const float* Bt, uint16_t* bh,
                                uint16_t* bl, uint16_t* bth, uint16_t* btl) {
  const size_t total = (size_t)npad * kp;
  const int ks = kp >> 4, nch = kp >> 5;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / kp), col = (int)(e % kp);
    const float x = row < n ? Bt[e] : 0.f;
    __bf16 h, l;
    split_bf16(x, h, l);
    const uint16_t hb = __builtin_bit_cast(uint16_t, h), lb = __builtin_bit_cast(uint16_t, l);
    const size_t ep = (((size_t)(row >> 5) * ks + (col >> 4)) * 64 + ((col >> 3) & 1) * 32 +
                       (row & 31)) * 8 + (col & 7);
    const size_t ec = (((size_t)(row >> 4) * nch + (col >> 5)) * 64 + ((row >> 3) & 1) * 32 +
                       (col & 31)) * 8 + (row & 7);
    bh[ep] = hb;
    bl[ep] = lb;
    bth[ec] = hb;
    btl[ec] = lb;
  }
}

// ---------------------------------------------------------------------------
// PROX: the per-account pass of an iteration (one workgroup per account)
//
// 1. The exact turnover-cap multiplier lam* of the current v (accounts with
//    a finite cap): turnover(lam) = sum_i |prox_i(v_i; lam) - w0_i| is
//    piecewise linear and non-increasing in lam, with slope -(number of
//    coordinates strictly inside a linear piece)/rho.  lam* = 0 when
//    turnover(0) <= tau, else the root of turnover(lam) = tau, found by
//    Newton steps from the previous lam* inside a bracket that every
//    evaluation tightens (bisection when a step leaves it).
// 2. For every row, z = prox(v; lam*), u = v - z, r = mu + rho (z - u) and
//    the two streams the rest of the iteration needs: R' = r / Delta (the
//    CONTRACT pass contracts it with B~) and w = v + alpha (R' - z) (the
//    PROJECT pass adds the back-projection to it).  With zmode the pass
//    writes z instead (the input of the polish).
// The row data (masks, holdings, tax records) is read here only: the
// CONTRACT pass is a plain contraction of R'.
// ---------------------------------------------------------------------------
constexpr int kCapT = 1024;             // 16 waves per account: latency-bound passes
constexpr int kCapQ = 16;               // rows per thread kept in registers (n <= 16384)
constexpr int kCapH = 2 * kCapT;        // held rows kept in registers (two per thread)
// the resident layout is compiled for 4, 8, 10, 12 and 16 rows per thread, the
// smallest that holds the book taken: registers beyond the book's rows would
// push the kernel past the 64 registers a lane may use with two accounts per
// compute unit

// one safeguarded Newton step on turnover(lam) = tau from the summed
// turnover gt and free count nft at lam; updates the bracket [lo, hi_b], the
// best multiplier known to be feasible and returns the next multiplier
__device__ __forceinline__ float cap_step(float gt, float nft, float tau, float rho, float lam,
                                          float& lo, float& hi_b, float& best_feas,
                                          bool& done) {
  const float tol = 1e-6f * fmaxf(tau, 1e-6f);
  if (gt <= tau) { hi_b = lam; best_feas = lam; } else { lo = lam; }
  done = fabsf(gt - tau) <= tol || (lam == 0.f && gt <= tau);
  float nl = lam;
  if (!done) {
    nl = (nft > 0.f) ? lam + rho * (gt - tau) / nft : NAN;
    if (gt <= tau && !(nl > 0.f) && lo == 0.f && lam > 0.f) {
      nl = 0.f;                        // try the unconstrained multiplier
    } else if (!(nl > lo && nl < hi_b)) {
      nl = isfinite(hi_b) ? 0.5f * (lo + hi_b) : fmaxf(2.f * lam, lam + 1e-4f);
    }
    if (isfinite(hi_b) && hi_b - lo <= 1e-6f * hi_b && lo > 0.f) { done = true; nl = hi_b; }
  }
  return fmaxf(nl, 0.f);
}

// the multiplier the search hands on: never one whose turnover is known to
// exceed tau
__device__ __forceinline__ float cap_result(float lam, bool done, float best_feas) {
  return (!done && isfinite(best_feas)) ? best_feas : lam;
}

// the account's rows as seen by the output phase: base pointers the whole
// workgroup shares, so that a row is addressed by its 32-bit index
struct ProxRows {
  const float* mu;   // mu (or mu') of the account
  float* w;          // w (zmode: z) of the account
  float* rp;         // R' of the account
};

__device__ __forceinline__ ProxRows prox_rows(const IterArgs& A, int a) {
  ProxRows o;
  o.mu = A.mu + (size_t)a * A.n;
  o.w = A.zs + (size_t)a * A.n;
  o.rp = A.rp + (size_t)a * A.npad;
  return o;
}

// the row's outputs from v and its z (zmode: z itself)
__device__ __forceinline__ void prox_out(const ProxRows& o, int zmode, int i, float v, float z,
                                         float d_i, float rho, float gam, float alpha) {
  if (zmode) {
    o.w[i] = z;
    return;
  }
  const float iDelta = __builtin_amdgcn_rcpf(gam * d_i + rho);
  const float u = v - z;
  const float Rp = (o.mu[i] + rho * (z - u)) * iDelta;
  o.rp[i] = Rp;
  o.w[i] = v + alpha * (Rp - z);
}

// Resident layout (n <= kCapQ * kCapT, at most kCapH held rows in every
// account of the book, one box per account; the host picks the layout per
// solve): one pass loads the account; rows that are not held keep v in a
// register (an excluded row has the box [0, 0], so z = 0 for every
// multiplier); held row j moves to LDS, and thread j keeps the first kCapT
// held rows' tax records in registers (records past that are re-read from
// the cache at each evaluation); every evaluation then runs on registers and
// LDS, and every thread takes the same Newton step from the same sums (one
// barrier per evaluation, double-buffered sums).
template <int Q>
__global__ __launch_bounds__(kCapT, 8) void prox_kernel(IterArgs A, int zmode) {
  __shared__ float s_g[2][kCapT / 64], s_n[2][kCapT / 64];
  __shared__ float s_hv[kCapH];
  __shared__ int s_hrow[kCapH];          // row of held record j, sign bit: excluded
  // the account's eligibility, holding and prefix words (one per 32 rows)
  __shared__ uint32_t s_ew[kCapQ * kCapT / 32], s_hw[kCapQ * kCapT / 32];
  __shared__ int s_hp[kCapQ * kCapT / 32];
  __shared__ float4 s_rec[2 * kCapT];    // tax records of the first kCapT held rows
  __shared__ float s_hz[kCapH];          // z of held record j at the final multiplier
  const int slot = blockIdx.x;
  if (slot >= *A.m_act) return;
  const int a = A.act[slot];
  float* par = A.par_rw + (size_t)a * kNPar;
  const float tau = par[P_TAU];
  const bool capped = isfinite(tau);
  const int tid = threadIdx.x, n = A.n, wv = tid >> 6;
  const float rho = par[P_RHO], irho = 1.f / rho, kap = par[P_KAPPA];
  const float lbp = par[P_LB], ubp = par[P_UB];
  float lam = capped ? par[P_LAM] : 0.f;
  const int hptr = A.hold_ptr[a];
  const int H = A.hold_ptr[a + 1] - hptr;
  float lo = 0.f, hi_b = INFINITY, best_feas = INFINITY;
  bool done = !capped;
  // a zero lower bound (every long-only account): the soft threshold and
  // the box reduce to min(max(v - th, 0), ub), the same value bit for bit
  const bool lb0 = lbp == 0.f;

  const float* va = A.v + (size_t)a * n;
  const size_t wa = (size_t)a * A.W;
  float vr[Q];
  // bit q: slot q is an eligible, unheld row inside the book (box [lb, ub]);
  // a held row lives in LDS and with thread j (its slot here holds 0)
  unsigned box_bits = 0u;
  // every load of the account issued before any is used: the words go to
  // LDS (one load per word, not one per row), v to registers
  {
    const int nw = (n + 31) >> 5;                // <= kCapT
    if (tid < nw) {
      s_ew[tid] = A.elig ? A.elig[wa + tid] : 0xffffffffu;
      s_hw[tid] = A.hold[wa + tid];
      s_hp[tid] = A.hold_pre[wa + tid];
    }
    if (tid < H) {
      s_rec[2 * tid] = A.hold_rec[2 * (hptr + tid)];
      s_rec[2 * tid + 1] = A.hold_rec[2 * (hptr + tid) + 1];
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = q * kCapT + tid;
      vr[q] = i < n ? va[i] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int i = q * kCapT + tid;
      const int wi = min(i, n - 1) >> 5;
      const int b = i & 31;
      const uint32_t hw = s_hw[wi];
      const bool el = i < n && ((s_ew[wi] >> b) & 1u);
      const bool held = i < n && ((hw >> b) & 1u);
      if (held) {
        const int j = s_hp[wi] + popc_below(hw, b);
        s_hv[j] = vr[q];
        s_hrow[j] = el ? i : ~i;
      }
      vr[q] = held ? 0.f : vr[q];
      box_bits |= (el && !held) ? (1u << q) : 0u;
    }
  }
  __syncthreads();
  // held row j: v from LDS, its tax record from LDS (j < kCapT) or from the
  // cache (j >= kCapT: the second held row of thread j - kCapT)
  const float hv = tid < H ? s_hv[tid] : 0.f;
  auto held_row = [&](int j, RowInfo& ri) {
    float4 r0, r1;
    if (j < kCapT) {
      r0 = s_rec[2 * j];
      r1 = s_rec[2 * j + 1];
    } else {
      r0 = A.hold_rec[2 * (hptr + j)];
      r1 = A.hold_rec[2 * (hptr + j) + 1];
    }
    const bool el = s_hrow[j] >= 0;
    ri.lb = el ? lbp : 0.f;
    ri.ub = el ? ubp : 0.f;
    ri.w0 = r0.x;
    ri.taxed = r0.y > 0.f;
    ri.t.b1 = r0.y; ri.t.b2 = r0.z; ri.t.b3 = r0.w;
    ri.t.s0 = r1.x; ri.t.s1 = r1.y; ri.t.s2 = r1.z; ri.t.s3 = r1.w;
  };
  for (int it = 0; it < 48 && !done; ++it) {          // done is uniform
    const float th = (kap + lam) * irho;
    float g = 0.f, nf = 0.f;
    if (lb0) {                             // uniform: z = min(max(v - th, 0), ub)
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (q * kCapT < n) {               // uniform
          const bool in_box = (box_bits >> q) & 1u;
          const float z = in_box ? fminf(fmaxf(vr[q] - th, 0.f), ubp) : 0.f;
          g += z;
          nf += (z > 0.f && z < ubp) ? 1.f : 0.f;
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        if (q * kCapT < n) {               // uniform
          const bool in_box = (box_bits >> q) & 1u;
          float z = fminf(vr[q] + th, fmaxf(0.f, vr[q] - th));
          z = in_box ? fminf(fmaxf(z, lbp), ubp) : 0.f;
          g += fabsf(z);
          nf += (in_box && z != 0.f && z > lbp && z < ubp) ? 1.f : 0.f;
        }
      }
    }
    if (tid < H) {
      RowInfo ri;
      held_row(tid, ri);
      bool kink;
      const float z = prox_row(ri, hv, th, irho, &kink);
      g += fabsf(z - ri.w0);
      nf += kink ? 0.f : 1.f;
    }
    if (H > kCapT && tid + kCapT < H) {          // uniform test first
      RowInfo ri;
      held_row(tid + kCapT, ri);
      bool kink;
      const float z = prox_row(ri, s_hv[tid + kCapT], th, irho, &kink);
      g += fabsf(z - ri.w0);
      nf += kink ? 0.f : 1.f;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      g += __shfl_xor(g, o, 64);
      nf += __shfl_xor(nf, o, 64);
    }
    const int buf = it & 1;
    if ((tid & 63) == 0) { s_g[buf][wv] = g; s_n[buf][wv] = nf; }
    __syncthreads();
    float gt = 0.f, nft = 0.f;
#pragma unroll
    for (int q = 0; q < kCapT / 64; ++q) { gt += s_g[buf][q]; nft += s_n[buf][q]; }
    lam = cap_step(gt, nft, tau, rho, lam, lo, hi_b, best_feas, done);
  }
  if (capped) {
    lam = cap_result(lam, done, best_feas);      // the same in every thread
    if (tid == 0) par[P_LAM] = lam;
  }
  // ---- the row outputs at lam* -------------------------------------------
  // (gamma and alpha read only now: registers are short during the search)
  const float gam = par[P_GAMMA], alpha = par[P_ALPHA];
  const float th = (kap + lam) * irho;
  const ProxRows o = prox_rows(A, a);
  // held rows first: their z goes to LDS, so that every row's outputs are
  // written below in row order (whole lines, not one word apart from the
  // rest of its line)
  if (tid < H) {
    RowInfo ri;
    held_row(tid, ri);
    s_hz[tid] = prox_row(ri, hv, th, irho, nullptr);
  }
  if (H > kCapT && tid + kCapT < H) {
    RowInfo ri;
    held_row(tid + kCapT, ri);
    s_hz[tid + kCapT] = prox_row(ri, s_hv[tid + kCapT], th, irho, nullptr);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int i = q * kCapT + tid;
    if (q * kCapT < n && i < n) {
      // (the row class comes from the LDS words again: box_bits would have
      // to live through the search in a register)
      const uint32_t hw = s_hw[i >> 5];
      const int b = i & 31;
      float v = vr[q], z;
      if ((hw >> b) & 1u) {
        const int j = s_hp[i >> 5] + popc_below(hw, b);
        v = s_hv[j];
        z = s_hz[j];
      } else {
        const bool in_box = (s_ew[i >> 5] >> b) & 1u;
        if (lb0) {
          z = in_box ? fminf(fmaxf(vr[q] - th, 0.f), ubp) : 0.f;
        } else {
          z = fminf(vr[q] + th, fmaxf(0.f, vr[q] - th));
          z = in_box ? fminf(fmaxf(z, lbp), ubp) : 0.f;
        }
      }
      prox_out(o, zmode, i, v, z, A.d[i], rho, gam, alpha);
    }
    // one row's loads at a time: issuing all of them ahead would not fit in
    // the registers two accounts per compute unit leave
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Streaming layout (any size, per-asset bounds): each evaluation re-reads
// the account; a last pass writes the row outputs.
__global__ __launch_bounds__(kCapT) void prox_stream_kernel(IterArgs A, int zmode) {
  __shared__ float s_g[2][kCapT / 64], s_n[2][kCapT / 64];
  __shared__ float s_lam;
  __shared__ int s_done;
  const int slot = blockIdx.x;
  if (slot >= *A.m_act) return;
  const int a = A.act[slot];
  float* par = A.par_rw + (size_t)a * kNPar;
  const float tau = par[P_TAU];
  const bool capped = isfinite(tau);
  const int tid = threadIdx.x, n = A.n, wv = tid >> 6;
  const float rho = par[P_RHO], irho = 1.f / rho, kap = par[P_KAPPA];
  const float lbp = par[P_LB], ubp = par[P_UB];
  const float gam = par[P_GAMMA], alpha = par[P_ALPHA];
  float lam = capped ? par[P_LAM] : 0.f;
  const int hptr = A.hold_ptr[a];
  float lo = 0.f, hi_b = INFINITY, best_feas = INFINITY;
  bool done = !capped;

  if (tid == 0) s_done = 0;
  for (int it = 0; it < 48 && !done; ++it) {          // done is uniform
    const float th = (kap + lam) * irho;
    float g = 0.f, nf = 0.f;
    // groups of 8 rows per thread: every load of a group is issued before
    // the group is evaluated
    for (int i0 = 0; i0 < n; i0 += 8 * kCapT) {
      float vr[8];
      uint32_t ew[8], hw[8];
      int hp[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + q * kCapT + tid;
        vr[q] = 0.f; ew[q] = 0u; hw[q] = 0u; hp[q] = 0;
        if (i < n) {
          const size_t wi = (size_t)a * A.W + (i >> 5);
          vr[q] = A.v[(size_t)a * n + i];
          ew[q] = A.elig ? A.elig[wi] : 0xffffffffu;
          hw[q] = A.hold[wi];
          hp[q] = A.hold_pre[wi];
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int i = i0 + q * kCapT + tid;
        if (i < n) {
          const RowInfo ri = row_info_w(A, (size_t)a * n + i, i, lbp, ubp, ew[q], hw[q], hp[q],
                                        hptr);
          bool kink;
          const float z = prox_row(ri, vr[q], th, irho, &kink);
          g += fabsf(z - ri.w0);
          nf += kink ? 0.f : 1.f;
        }
      }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      g += __shfl_xor(g, o, 64);
      nf += __shfl_xor(nf, o, 64);
    }
    if ((tid & 63) == 0) { s_g[0][wv] = g; s_n[0][wv] = nf; }
    __syncthreads();
    if (tid == 0) {
      float gt = 0.f, nft = 0.f;
      for (int q = 0; q < kCapT / 64; ++q) { gt += s_g[0][q]; nft += s_n[0][q]; }
      bool dn;
      s_lam = cap_step(gt, nft, tau, rho, lam, lo, hi_b, best_feas, dn);
      s_done = dn ? 1 : 0;
      // tid 0 carries the bracket: the hand-on multiplier, ready when done
      if (dn || it == 47) s_lam = cap_result(s_lam, dn, best_feas);
    }
    __syncthreads();
    lam = s_lam;
    done = s_done != 0;
    __syncthreads();
  }
  if (capped && tid == 0) par[P_LAM] = lam;
  // ---- the row outputs at lam* -------------------------------------------
  const float th = (kap + lam) * irho;
  const ProxRows o = prox_rows(A, a);
  for (int i0 = 0; i0 < n; i0 += 8 * kCapT) {
    float vr[8];
    uint32_t ew[8], hw[8];
    int hp[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + q * kCapT + tid;
      vr[q] = 0.f; ew[q] = 0u; hw[q] = 0u; hp[q] = 0;
      if (i < n) {
        const size_t wi = (size_t)a * A.W + (i >> 5);
        vr[q] = A.v[(size_t)a * n + i];
        ew[q] = A.elig ? A.elig[wi] : 0xffffffffu;
        hw[q] = A.hold[wi];
        hp[q] = A.hold_pre[wi];
      }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = i0 + q * kCapT + tid;
      if (i < n) {
        const RowInfo ri = row_info_w(A, (size_t)a * n + i, i, lbp, ubp, ew[q], hw[q], hp[q],
                                      hptr);
        const float z = prox_row(ri, vr[q], th, irho, nullptr);
        prox_out(o, zmode, i, vr[q], z, A.d[i], rho, gam, alpha);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// per-account factor-space solve
// ---------------------------------------------------------------------------
// threads per account: at kp = 96, five threads per factor column, so that
// each thread's partial sums (up to 79 row tiles) and K^-1 rows come in one
// batch of loads each
constexpr int kKsT = 512;
__global__ __launch_bounds__(kKsT) void ksolve_kernel(KArgs A) {
  __shared__ double t[kMaxKp], rhs[kMaxKp], red[kKsT], redq[kKsT / 64];
  __shared__ float tsp[kKsT];                // split partial sums
  __shared__ float pprime[kMaxKp];
  const int slot = blockIdx.x;
  if (slot >= *A.m_act) return;
  const int a = A.act[slot];
  const int tid = threadIdx.x;
  const int kp = A.kp, k = A.k, G = A.G, kg = k + G;
  const size_t M = A.m_total;
  const int n_rt = tile_map(*A.m_act, A.n, A.nblk, 0).n_rt;
  float* par = A.par + (size_t)a * kNPar;
  // (one class: no dependent load of the account's class before K^-1)
  const int cls = A.ncls == 1 ? 0 : (int)par[P_CLASS];
  const float* Kinv = A.Kinv + (size_t)cls * kp * kp;
  const float* cv = A.cvec + (size_t)cls * kp;
  const float* qv = A.qvec + (size_t)cls * kp;
  const float sig1 = A.sig1[cls];
  const float rhob = par[P_RHOB];
  // this thread's entry of q (kg <= kMaxKp <= kKsT: one each), loaded with
  // the partials rather than on the way to nu
  static_assert(kMaxKp <= kKsT, "one factor column per thread");
  const float qvj = tid < kg ? qv[tid] : 0.f;

  // nsp threads per factor column split the row tiles (and below the
  // K^-1 rows), so that more independent loads are in flight.  Each thread
  // issues its first batch of 16 partials, then its first 16 entries of
  // K^-1 (used after the reduction), before any of them is waited on.
  const int nsp = kp <= kKsT ? kKsT / kp : 1;
  const int jq = tid % kp, qq = tid / kp;
  float kb[16];
  if (tid < nsp * kp) {
    float buf[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int rt = qq + u * nsp;
      buf[u] = rt < n_rt ? A.part[((size_t)rt * M + a) * kp + jq] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int l = qq + u * nsp;
      kb[u] = (jq < kg && l < kg) ? Kinv[l * kp + jq] : 0.f;
    }
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < 16; ++u) s += buf[u];
    // batches of 16 loads issued before any is added
    for (int r0 = qq + 16 * nsp; r0 < n_rt; r0 += 16 * nsp) {
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int rt = r0 + u * nsp;
        buf[u] = rt < n_rt ? A.part[((size_t)rt * M + a) * kp + jq] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) s += buf[u];
    }
    tsp[tid] = s;
  }
  __syncthreads();
  for (int j = tid; j < kp; j += kKsT) {
    float s = 0.f;
    for (int q = 0; q < nsp; ++q) s += tsp[q * kp + j];
    t[j] = s;
  }
  __syncthreads();
  // band terms: t += (K - F~^-1)[:, G] rho_b (zb - vb);  s0 += c_G . same
  double s0 = t[kg];
  if (G > 0) {
    const float* mbg = A.mbg + (size_t)cls * kp * G;
    const float* zb = A.zb + (size_t)a * G;
    const float* vb = A.vb + (size_t)a * G;
    for (int j = tid; j < kg; j += kKsT) {
      double s = 0.0;
      for (int g = 0; g < G; ++g) s += (double)mbg[j * G + g] * rhob * ((double)zb[g] - vb[g]);
      rhs[j] = s;
    }
    __syncthreads();
    double cs = 0.0;
    for (int g = 0; g < G; ++g) cs += (double)cv[k + g] * rhob * ((double)zb[g] - vb[g]);
    s0 += cs;
    for (int j = tid; j < kg; j += kKsT) t[j] += rhs[j];
    __syncthreads();
  }
  // p = K^-1 (t + nu c) = K^-1 t + nu q (q = K^-1 c): the product with t
  // does not wait for nu = (1 - s0 + q^T t) / sigma1, and both reductions
  // share one LDS step
  if (tid < nsp * kp) {
    const int j = jq, q = qq;
    double s = 0.0;
    if (j < kg) {
      // K^-1 is symmetric: column j (consecutive j -> consecutive words);
      // the first batch was loaded at the start, later ones here in
      // batches of 16 loads issued before any is used
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int l = q + u * nsp;
        if (l < kg) s += (double)kb[u] * t[l];
      }
      for (int l0 = q + 16 * nsp; l0 < kg; l0 += 16 * nsp) {
        float buf[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int l = l0 + u * nsp;
          buf[u] = l < kg ? Kinv[l * kp + j] : 0.f;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int l = l0 + u * nsp;
          if (l < kg) s += (double)buf[u] * t[l];
        }
      }
    }
    red[tid] = s;
  }
  double part = tid < kg ? (double)qvj * t[tid] : 0.0;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
  if ((tid & 63) == 0) redq[tid >> 6] = part;
  __syncthreads();
  double qt = 0.0;                       // the same order in every thread
  for (int q = 0; q < kKsT / 64; ++q) qt += redq[q];
  const double nu = (1.0 - s0 + qt) / (double)sig1;
  // back-projection coefficients: band directions carry -rho_b (zb - vb)
  float* pp = A.pp + (size_t)a * kp;
  if (tid < kp) {                        // kp <= kKsT: column tid (whose q entry it holds)
    double s = 0.0;
    for (int q = 0; q < nsp; ++q) s += red[q * kp + tid];
    const float pj = (float)(s + nu * (double)qvj);
    pprime[tid] = pj;
    float v = 0.f;
    if (tid < k) v = pj;
    else if (tid < kg) v = pj - rhob * (A.zb[(size_t)a * G + (tid - k)] - A.vb[(size_t)a * G + (tid - k)]);
    pp[tid] = v;
  }
  if (G > 0) __syncthreads();            // the band block reads pprime
  // band ADMM block:  A x = p'_G / rho_b
  if (G > 0 && tid < G) {
    const int g = tid;
    const float alpha = par[P_ALPHA];
    float* zb = A.zb + (size_t)a * G;
    float* vb = A.vb + (size_t)a * G;
    const float ax = pprime[k + g] / rhob;
    const float zh = alpha * ax + (1.f - alpha) * zb[g];
    float zn = zh + vb[g];
    zn = fminf(fmaxf(zn, A.blo[(size_t)a * G + g]), A.bhi[(size_t)a * G + g]);
    vb[g] = vb[g] + zh - zn;
    zb[g] = zn;
  }
  if (tid == 0) {
    par[P_NU] = (float)nu;
    A.iters[a] += 1;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// LDS of one workgroup (mirrors the layout at the top of iter_kernel); the
// two passes need different regions, which keeps each under half a CU's
// LDS so that two workgroups share a CU
template <int NCH, int MODE>
static size_t iter_smem() {
  constexpr int kp = NCH * 32, BS = kp + 1;
  constexpr int kXs = (MODE == MODE_PROJECT) ? kTM * BS + kWaves * kTM : kWaves * 32 * 33;
  return sizeof(float) * ((size_t)kRowsPerChunk * BS + kXs + 8 * kTM) + 4 * sizeof(int) * kTM;
}

template <int NCH, int MODE>
static size_t iter_smem_bf() {
  return sizeof(float) * ((size_t)bf_lds_floats<NCH, MODE>() + 8 * kTM) + 4 * sizeof(int) * kTM;
}

// with events the launch goes through hipExtLaunchKernelGGL, which stamps
// them at the kernel's own start and end
template <typename K>
static void launch_timed(K kernel, dim3 grid, size_t smem, hipStream_t st, hipEvent_t ev0,
                         hipEvent_t ev1, const IterArgs& A) {
  if (ev0 || ev1)
    hipExtLaunchKernelGGL(kernel, grid, dim3(256), (std::uint32_t)smem, st, ev0, ev1, 0u, A);
  else
    hipLaunchKernelGGL(kernel, grid, dim3(256), smem, st, A);
}

template <int NCH>
static hipError_t launch_iter_t(const IterArgs& A, int mode, int prec, dim3 grid,
                                hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (prec == FQP_PREC_BF16X3 && NCH * 32 <= kMaxKpBf) {
    constexpr int NB = NCH * 32 <= kMaxKpBf ? NCH : 1;   // instantiate narrow widths only
    if (mode == MODE_CONTRACT)
      launch_timed(iter_kernel_bf<NB, MODE_CONTRACT>, grid, iter_smem_bf<NB, MODE_CONTRACT>(),
                   st, ev0, ev1, A);
    else
      launch_timed(iter_kernel_bf<NB, MODE_PROJECT>, grid, iter_smem_bf<NB, MODE_PROJECT>(),
                   st, ev0, ev1, A);
    return hipGetLastError();
  }
  if (mode == MODE_CONTRACT)
    launch_timed(iter_kernel<NCH, MODE_CONTRACT>, grid, iter_smem<NCH, MODE_CONTRACT>(), st,
                 ev0, ev1, A);
  else
    launch_timed(iter_kernel<NCH, MODE_PROJECT>, grid, iter_smem<NCH, MODE_PROJECT>(), st,
                 ev0, ev1, A);
  return hipGetLastError();
}

hipError_t configure_iter_kernels() {
  hipError_t e = hipSuccess;
#define FQP_CFG(N)                                                                     \
  e = hipFuncSetAttribute((const void*)iter_kernel<N, MODE_CONTRACT>,                  \
                          hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                          (int)iter_smem<N, MODE_CONTRACT>());                         \
  if (e != hipSuccess) return e;                                                       \
  e = hipFuncSetAttribute((const void*)iter_kernel<N, MODE_PROJECT>,                   \
                          hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                          (int)iter_smem<N, MODE_PROJECT>());                          \
  if (e != hipSuccess) return e;                                                       \
  e = hipFuncSetAttribute((const void*)iter_kernel_bf<(N * 32 <= kMaxKpBf ? N : 1), MODE_CONTRACT>, \
                          hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                          (int)iter_smem_bf<(N * 32 <= kMaxKpBf ? N : 1), MODE_CONTRACT>()); \
  if (e != hipSuccess) return e;
  FQP_CFG(1) FQP_CFG(2) FQP_CFG(3) FQP_CFG(4) FQP_CFG(5) FQP_CFG(6)
#undef FQP_CFG
  e = hipFuncSetAttribute((const void*)kfactor_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)(2 * sizeof(double) * kKfLds * kKfLds));
  if (e != hipSuccess) return e;
  return e;
}

template <int NCH>
static int iter_blocks_per_cu_t(int prec, int mode) {
  int nb = 0;
  hipError_t e;
  if (prec == FQP_PREC_BF16X3 && NCH * 32 <= kMaxKpBf) {
    constexpr int NB = NCH * 32 <= kMaxKpBf ? NCH : 1;
    e = (mode == MODE_CONTRACT)
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &nb, (const void*)iter_kernel_bf<NB, MODE_CONTRACT>, 256,
                  iter_smem_bf<NB, MODE_CONTRACT>())
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &nb, (const void*)iter_kernel_bf<NB, MODE_PROJECT>, 256,
                  iter_smem_bf<NB, MODE_PROJECT>());
  } else {
    e = (mode == MODE_CONTRACT)
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &nb, (const void*)iter_kernel<NCH, MODE_CONTRACT>, 256,
                  iter_smem<NCH, MODE_CONTRACT>())
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(
                  &nb, (const void*)iter_kernel<NCH, MODE_PROJECT>, 256,
                  iter_smem<NCH, MODE_PROJECT>());
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

int iter_blocks_per_cu(int kp, int prec, int mode) {
  switch (kp / 32) {
    case 1: return iter_blocks_per_cu_t<1>(prec, mode);
    case 2: return iter_blocks_per_cu_t<2>(prec, mode);
    case 3: return iter_blocks_per_cu_t<3>(prec, mode);
    case 4: return iter_blocks_per_cu_t<4>(prec, mode);
    case 5: return iter_blocks_per_cu_t<5>(prec, mode);
    case 6: return iter_blocks_per_cu_t<6>(prec, mode);
    default: return 0;
  }
}

hipError_t launch_iter(const IterArgs& A, int kp, int mode, int prec, dim3 grid,
                       hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  switch (kp / 32) {
    case 1: return launch_iter_t<1>(A, mode, prec, grid, st, ev0, ev1);
    case 2: return launch_iter_t<2>(A, mode, prec, grid, st, ev0, ev1);
    case 3: return launch_iter_t<3>(A, mode, prec, grid, st, ev0, ev1);
    case 4: return launch_iter_t<4>(A, mode, prec, grid, st, ev0, ev1);
    case 5: return launch_iter_t<5>(A, mode, prec, grid, st, ev0, ev1);
    case 6: return launch_iter_t<6>(A, mode, prec, grid, st, ev0, ev1);
    default: return hipErrorInvalidValue;
  }
}

bool cap_resident_fits(int n, int max_held) {
  return n <= kCapQ * kCapT && max_held <= kCapH;
}
// (the resident layout keeps one box per account; books with per-asset
// bounds take the streaming layout)

template <typename K>
static void launch_prox_t(K kernel, int m_total, const IterArgs& A, int zmode, hipStream_t st,
                          hipEvent_t ev0, hipEvent_t ev1) {
  if (ev0 || ev1)
    hipExtLaunchKernelGGL(kernel, dim3(m_total), dim3(kCapT), 0u, st, ev0, ev1, 0u, A, zmode);
  else
    hipLaunchKernelGGL(kernel, dim3(m_total), dim3(kCapT), 0, st, A, zmode);
}

hipError_t launch_prox(const IterArgs& A, int m_total, bool resident, int zmode,
                       hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const int q = (A.n + kCapT - 1) / kCapT;
  if (resident && q <= 4) launch_prox_t(prox_kernel<4>, m_total, A, zmode, st, ev0, ev1);
  else if (resident && q <= 8) launch_prox_t(prox_kernel<8>, m_total, A, zmode, st, ev0, ev1);
  else if (resident && q <= 10) launch_prox_t(prox_kernel<10>, m_total, A, zmode, st, ev0, ev1);
  else if (resident && q <= 12) launch_prox_t(prox_kernel<12>, m_total, A, zmode, st, ev0, ev1);
  else if (resident) launch_prox_t(prox_kernel<16>, m_total, A, zmode, st, ev0, ev1);
  else launch_prox_t(prox_stream_kernel, m_total, A, zmode, st, ev0, ev1);
  return hipGetLastError();
}

hipError_t launch_ksolve(const KArgs& A, int m_total, hipStream_t st) {
  hipLaunchKernelGGL(ksolve_kernel, dim3(m_total), dim3(kKsT), 0, st, A);
  return hipGetLastError();
}

hipError_t launch_split_bt(int n, int npad, int kp, const float* Bt, uint16_t* bh, uint16_t* bl,
                           uint16_t* bth, uint16_t* btl, hipStream_t st) {
  const size_t total = (size_t)npad * kp;
  const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 8192);
  hipLaunchKernelGGL(split_bt_kernel, dim3(blocks), dim3(256), 0, st, n, npad, kp, Bt, bh, bl,
                     bth, btl);
  return hipGetLastError();
}

hipError_t launch_build_bt(int n, int k, int G, int H, int kp, const float* B,
                           const int32_t* group, const float* half, float* Bt, hipStream_t st) {
  size_t total = (size_t)n * kp;
  hipLaunchKernelGGL(build_bt_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     n, k, G, H, kp, B, group, half, Bt);
  return hipGetLastError();
}

hipError_t launch_gram(int n, int kp, int kg, int nparts, int rows_per_blk, const float* Bt,
                       const float* d, double gamma, double rho, double* part, hipStream_t st) {
  const int ne = (kg + 1) * (kg + 1);
  hipLaunchKernelGGL(gram_partial_kernel, dim3(nparts, (ne + 8191) / 8192), dim3(256),
                     64 * kp * sizeof(float), st, n, kp, kg, rows_per_blk, Bt, d, gamma, rho,
                     part);
  return hipGetLastError();
}

hipError_t launch_kfactor(int k, int G, int kp, int nparts, const double* part, const float* f,
                          double gamma, double rho_b, double* Kw, float* Kinv, float* c,
                          float* q, float* sig, float* mbg, hipStream_t st) {
  const int kg = k + G;
  // LDS: K^-1, the row and column buffers, c and q (wide blocks: c and q)
  const size_t smem = sizeof(double) * (kg <= kKfLds ? (size_t)kg * kg + 6 * kg + 8 : 2 * kg + 8);
  const int ne = (kg + 1) * (kg + 1);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((ne + 255) / 256), dim3(256), 0, st, ne, nparts,
                     part, Kw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kfactor_kernel, dim3(1), dim3(1024), smem, st, k, G, kp, nparts, part, f,
                     gamma, rho_b, Kw, Kinv, c, q, sig, mbg);
  return hipGetLastError();
}

}  // namespace fqp
