// Float64 polish and certification on the GPU (gfx950).
//
// At the optimum of the build's Eq. 1 instance every eligible coordinate
// either sits at a bound or at a kink of its piecewise-linear trade cost
// ("fixed") or inside one linear piece ("free", known slope).  Given that
// pattern and which bands / cap bind, the optimum solves one equality-
// constrained QP in float64:
//
//   gamma Sigma_FF w_F + C_F^T eta = mu_F - slope_F - gamma Sigma_FX w_X
//   C_F w_F = h      (budget, binding bands, binding cap)
//
// H = gamma Sigma_FF = gamma (B_F diag(f) B_F^T + D_F) is inverted through
// the factor space: H^-1 = (D^-1 - D^-1 B_F Kf^-1 B_F^T D^-1)/gamma with
// Kf = diag(f)^-1 + B_F^T D_F^-1 B_F (k x k, Cholesky in LDS), and the
// multipliers eta come from the Schur complement S = C H^-1 C^T.  When the
// free set does not pin every multiplier (S singular) the ADMM estimates are
// corrected by the minimum-norm step, as the fixed coordinates then decide.
//
// The certification kernel recomputes the external diagnostics of Sec.
// "External Diagnostics" in float64 (budget, box, exposure and turnover
// residuals; nonsmooth stationarity against the subdifferential of the
// trade cost and the normal cone of the box; complementarity of bands and
// cap).  A pattern that fails is refined primal-dual active-set style:
// free coordinates that left their piece are fixed at the crossed point,
// fixed coordinates whose stationarity is violated move into the adjacent
// piece, and bands / cap are switched on when violated or off when their
// multiplier has the wrong sign.
#include <climits>

#include "fqp_common.h"
#include "fqp_kernels.h"
#include "../../include/fqp.h"

namespace fqp {

enum PState {
  PS_CAP = 0, PS_NF, PS_NX, PS_NC, PS_DONE, PS_ROUNDS,
  PS_BACT0, PS_BACT1, PS_BUP0, PS_BUP1, PS_STALL, PS_ND, PS_SIG, kNPState
};
static_assert(kNPState <= kPStateStride, "polish bookkeeping does not fit");

constexpr double kSnap = 1e-10;
constexpr int kSmallF = 64;               // free sets solved in row space
constexpr int kMaxNull = 8;
// one workgroup of 16 waves per account: the row passes are latency bound
constexpr int kPT = 1024;                 // polish_solve
constexpr int kPTC = 1024;                // polish_check
constexpr int kPW = kPT / 64;             // most waves of either

// The points, kinks and slopes of one asset's line, as scalar fields: a
// run-time index goes through the select chains below, never through an
// array, so that the structure stays in registers (an indexed array would
// live in scratch memory, one memory round trip per access).
struct Geom {
  int np;            // points on the asset's line: bounds and inner kinks
  int nk;            // kinks of the trade cost (w0 last when present)
  double p0, p1, p2, p3, p4, p5;       // the points (ascending)
  float f0, f1, f2, f3, f4, f5;        // the same points as the float32 prox evaluates them
  double k0, k1, k2, k3;               // kinks (ascending)
  double s0, s1, s2, s3, s4;           // slope of the trade cost on each side of the kinks
  double w0;
  __device__ __forceinline__ double pt(int i) const {
    return i <= 0 ? p0 : i == 1 ? p1 : i == 2 ? p2 : i == 3 ? p3 : i == 4 ? p4 : p5;
  }
  __device__ __forceinline__ float ptf(int i) const {
    return i <= 0 ? f0 : i == 1 ? f1 : i == 2 ? f2 : i == 3 ? f3 : i == 4 ? f4 : f5;
  }
  __device__ __forceinline__ double kink(int i) const {
    return i <= 0 ? k0 : i == 1 ? k1 : i == 2 ? k2 : k3;
  }
  __device__ __forceinline__ double ks(int i) const {
    return i <= 0 ? s0 : i == 1 ? s1 : i == 2 ? s2 : i == 3 ? s3 : s4;
  }
  // point i <- (x, xf) when `on` (i in 1..5)
  __device__ __forceinline__ void put(int i, bool on, double x, float xf) {
    p1 = (on && i == 1) ? x : p1; f1 = (on && i == 1) ? xf : f1;
    p2 = (on && i == 2) ? x : p2; f2 = (on && i == 2) ? xf : f2;
    p3 = (on && i == 3) ? x : p3; f3 = (on && i == 3) ? xf : f3;
    p4 = (on && i == 4) ? x : p4; f4 = (on && i == 4) ? xf : f4;
    p5 = (on && i == 5) ? x : p5; f5 = (on && i == 5) ? xf : f5;
  }
};

// eligibility, w0 and lot data of (account, row): the bitmask words, then
// one dependent load of the packed record for a held row
struct RowData {
  bool el;
  bool taxed;
  float w0;
  float lb, ub;      // box of the asset ([0, 0] when excluded)
  float b1, b2, b3, s0, s1, s2, s3;
};

// lbf / ubf: the account's scalar bounds (used without per-asset bounds)
__device__ __forceinline__ RowData row_data(const PolishArgs& A, int a, int i, float lbf,
                                            float ubf) {
  RowData r;
  const int wd = i >> 5, b = i & 31;
  const size_t wi = (size_t)a * A.W + wd;
  r.el = A.elig == nullptr || ((A.elig[wi] >> b) & 1u);
  asset_box(A, (size_t)a * A.n + i, r.el, lbf, ubf, r.lb, r.ub);
  const uint32_t hw = A.hold[wi];
  r.w0 = 0.f;
  r.taxed = false;
  r.b1 = r.b2 = r.b3 = r.s0 = r.s1 = r.s2 = r.s3 = 0.f;
  if ((hw >> b) & 1u) {
    const int idx = A.hold_ptr[a] + A.hold_pre[wi] + popc_below(hw, b);
    const float4 r0 = A.hold_rec[2 * idx], r1 = A.hold_rec[2 * idx + 1];
    r.w0 = r0.x;
    r.taxed = r0.y > 0.f;
    r.b1 = r0.y; r.b2 = r0.z; r.b3 = r0.w;
    r.s0 = r1.x; r.s1 = r1.y; r.s2 = r1.z; r.s3 = r1.w;
  }
  return r;
}

__device__ __forceinline__ void make_geom(Geom& g, float kap, bool phi, const RowData& r) {
  const float w0f = r.w0;
  const double lb = r.lb, ub = r.ub;
  g.w0 = w0f;
  // every field is written on every path (selects, not branches)
  const bool tx = phi && r.taxed, pl = phi && !r.taxed;
  const double kd = kap;
  g.nk = tx ? 4 : (pl ? 1 : 0);
  const float kf0 = tx ? w0f - r.b3 : w0f, kf1 = tx ? w0f - r.b2 : 0.f;
  const float kf2 = tx ? w0f - r.b1 : 0.f, kf3 = tx ? w0f : 0.f;
  g.k0 = tx ? (double)w0f - r.b3 : (double)w0f;
  g.k1 = tx ? (double)w0f - r.b2 : 0.0;
  g.k2 = tx ? (double)w0f - r.b1 : 0.0;
  g.k3 = tx ? (double)w0f : 0.0;
  g.s0 = tx ? -(kd + r.s3) : (pl ? -kd : 0.0);
  g.s1 = tx ? -(kd + r.s2) : (pl ? kd : 0.0);
  g.s2 = tx ? -(kd + r.s1) : 0.0;
  g.s3 = tx ? -(kd + r.s0) : 0.0;
  g.s4 = tx ? kd : 0.0;
  // points: lb, the kinks strictly inside (lb, ub) (ascending), ub
  g.np = 1;
  g.p0 = lb; g.f0 = r.lb;
  g.p1 = g.p2 = g.p3 = g.p4 = g.p5 = 0.0;
  g.f1 = g.f2 = g.f3 = g.f4 = g.f5 = 0.f;
  const bool in0 = g.nk > 0 && g.k0 > lb && g.k0 < ub;
  g.put(g.np, in0, g.k0, kf0); g.np += in0 ? 1 : 0;
  const bool in1 = g.nk > 1 && g.k1 > lb && g.k1 < ub;
  g.put(g.np, in1, g.k1, kf1); g.np += in1 ? 1 : 0;
  const bool in2 = g.nk > 2 && g.k2 > lb && g.k2 < ub;
  g.put(g.np, in2, g.k2, kf2); g.np += in2 ? 1 : 0;
  const bool in3 = g.nk > 3 && g.k3 > lb && g.k3 < ub;
  g.put(g.np, in3, g.k3, kf3); g.np += in3 ? 1 : 0;
  const bool top = ub > lb;
  g.put(g.np, top, ub, r.ub); g.np += top ? 1 : 0;
}

// number of kinks below x (the kinks ascend)
__device__ __forceinline__ int kinks_below(const Geom& g, double x) {
  return (g.nk > 0 && g.k0 < x ? 1 : 0) + (g.nk > 1 && g.k1 < x ? 1 : 0) +
         (g.nk > 2 && g.k2 < x ? 1 : 0) + (g.nk > 3 && g.k3 < x ? 1 : 0);
}

// slope of the trade cost (without cap) on the piece between points q, q+1
__device__ __forceinline__ void piece_slope(const Geom& g, int q, double& slope, double& sgn) {
  const double mid = 0.5 * (g.pt(q) + g.pt(q + 1));
  slope = g.ks(kinks_below(g, mid));
  sgn = (mid > g.w0) ? 1.0 : -1.0;
}

// subdifferential interval of phi + lam |. - w0| + N_box at x (with snap)
__device__ __forceinline__ void subdiff(const Geom& g, double x, double lam, double lb,
                                        double ub, double& lo, double& hi, double& snap) {
  snap = 0.0;
  // the first kink within kSnap of x, or -1
  const int at = (g.nk > 0 && fabs(x - g.k0) <= kSnap) ? 0
               : (g.nk > 1 && fabs(x - g.k1) <= kSnap) ? 1
               : (g.nk > 2 && fabs(x - g.k2) <= kSnap) ? 2
               : (g.nk > 3 && fabs(x - g.k3) <= kSnap) ? 3 : -1;
  if (at >= 0) {
    lo = g.ks(at) + ((at < g.nk) ? -lam : lam);
    hi = g.ks(at + 1) + ((at + 1 < g.nk) ? -lam : lam);
    snap = fabs(x - g.kink(at));
  } else {
    const int s = kinks_below(g, x);
    lo = hi = g.ks(s) + ((s < g.nk) ? -lam : lam);
  }
  if (g.nk == 0) lo = hi = 0.0;
  if (x <= lb + kSnap) { lo = -INFINITY; snap = fmax(snap, fmax(x - lb, 0.0)); }
  if (x >= ub - kSnap) { hi = INFINITY; snap = fmax(snap, fmax(ub - x, 0.0)); }
}

// sale-side tax of selling s >= 0 from lots with breakpoints b1 < b2 < b3
// and slopes t0..t3 (the last slope continues past b3)
__device__ __forceinline__ double lot_tax(double s, const RowData& r) {
  const double b1 = r.b1, b2 = r.b2, b3 = r.b3;
  double tc = r.s0 * fmin(s, b1);
  tc += (s > b1) ? r.s1 * (fmin(s, b2) - b1) : 0.0;
  tc += (s > b2) ? r.s2 * (fmin(s, b3) - b2) : 0.0;
  tc += (s > b3) ? r.s3 * (s - b3) : 0.0;
  return tc;
}


size_t polish_wk_stride(int k, int G) {
  const size_t ncol = (size_t)G + 3;
  // Waug, Y (k x ncol), CV (ncol^2), S (ncol^2), yX, Fy, sol (k), h, eta, eta0
  // (ncol), misc 16
  return 2 * (size_t)k * ncol + 2 * ncol * ncol + 3 * (size_t)k + 3 * ncol +
         (size_t)kMaxNull * ncol + (size_t)k + (size_t)G + 1 + 16;
}

struct Wk {
  double *Waug, *Y, *CV, *S, *yX, *Fy, *sol, *h, *eta, *eta0, *nul, *yF, *gsum, *misc;
};
__device__ __forceinline__ Wk wk_of(const PolishArgs& A, int a) {
  Wk w;
  const int k = A.k;
  const size_t ncol = (size_t)A.G + 3;
  double* p = A.wk + (size_t)a * A.wk_stride;
  w.Waug = p; p += (size_t)k * ncol;
  w.Y = p; p += (size_t)k * ncol;
  w.CV = p; p += ncol * ncol;
  w.S = p; p += ncol * ncol;
  w.yX = p; p += k;
  w.Fy = p; p += k;
  w.sol = p; p += k;
  w.h = p; p += ncol;
  w.eta = p; p += ncol;
  w.eta0 = p; p += ncol;
  w.nul = p; p += (size_t)kMaxNull * ncol;   // [kMaxNull][ncol] null directions
  w.yF = p; p += k;                            // F B^T w of the polished w
  w.gsum = p; p += (size_t)A.G + 1;            // group sums of the polished w
  w.misc = p;
  return w;
}

__device__ __forceinline__ bool band_active(const int* ps, int g) {
  return g < 32 ? ((ps[PS_BACT0] >> g) & 1) : ((ps[PS_BACT1] >> (g - 32)) & 1);
}
__device__ __forceinline__ bool band_upper(const int* ps, int g) {
  return g < 32 ? ((ps[PS_BUP0] >> g) & 1) : ((ps[PS_BUP1] >> (g - 32)) & 1);
}
__device__ __forceinline__ void set_band(int* ps, int g, bool act, bool up) {
  const int w = g < 32 ? 0 : 1, b = g & 31;
  int* pa = ps + PS_BACT0 + w;
  int* pu = ps + PS_BUP0 + w;
  *pa = act ? (*pa | (1 << b)) : (*pa & ~(1 << b));
  *pu = up ? (*pu | (1 << b)) : (*pu & ~(1 << b));
}

// block reductions: wave shuffles, then one partial per wave
template <typename T>
__device__ T bsum(T v, T* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  T r = sh[0];
  const int nw = (int)(blockDim.x >> 6);
  for (int q = 1; q < nw; ++q) r += sh[q];
  return r;
}
template <typename T>
__device__ T bmax(T v, T* sh) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  T r = sh[0];
  const int nw = (int)(blockDim.x >> 6);
  for (int q = 1; q < nw; ++q) r = fmax(r, sh[q]);
  return r;
}

// Sums over a list of rows (LDS-staged, 64 rows at a time):
//   ys[j] += sum_t B[i_t][j] w[i_t]   (thread j < k)
//   gs[g] += sum_t (row g at i_t) w[i_t]   (thread g < G: band rows by
//            label, halfspace rows from the columns k + g of B~)
// Entries are list[t] (rev = 0) or list[n - 1 - t] (rev = 1), t < cnt.
__device__ void list_sums(const PolishArgs& A, const int32_t* list, int n, int cnt, int rev,
                          const double* w, float* sB, double* sw, int* si, double& ys,
                          double& gs) {
  const int k = A.k, G = A.G, tid = threadIdx.x;
  for (int c0 = 0; c0 < cnt; c0 += 64) {
    const int rows = min(64, cnt - c0);
    __syncthreads();
    if (tid < rows) {
      const int i = rev ? list[n - 1 - (c0 + tid)] : list[c0 + tid];
      si[tid] = i;
      sw[tid] = w[i];
    }
    __syncthreads();
    for (int e = tid; e < rows * k; e += (int)blockDim.x) {
      const int rr = e / k, j = e % k;
      sB[rr * (k + 1) + j] = A.Bt[(size_t)si[rr] * A.kp + j];
    }
    __syncthreads();
    if (tid < k)
      for (int rr = 0; rr < rows; ++rr) ys += (double)sB[rr * (k + 1) + tid] * sw[rr];
    if (tid < A.Gl)
      for (int rr = 0; rr < rows; ++rr) gs += (A.group[si[rr]] == tid) ? sw[rr] : 0.0;
    else if (tid < G)             // halfspace rows: the columns k + tid of B~
      for (int rr = 0; rr < rows; ++rr)
        gs += (double)A.Bt[(size_t)si[rr] * A.kp + k + tid] * sw[rr];
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// polish_solve: classify (first round), lists, reduced KKT solve, w
// ---------------------------------------------------------------------------
// Row-space solve of a small free set (nF <= kSmallF): with the free rows'
// constraint coefficients V_r = [1, band coefficients, sgn_r | rhs_r] and
// H = gamma Sigma_FF = gamma (B_F diag(f) B_F^T + diag(d_F)), it forms H,
// factors it (Cholesky by one wave), solves X = H^-1 V and writes the Schur
// block S = V_C^T X = C H^-1 [C^T | rhs] the factor-space path forms by
// Woodbury.  It also adds sum_F sgn_r w0_r to the cap's right-hand side.
// Returns X ([nF][ncol], LDS) for the free-row values.
__device__ double* small_free_solve(const PolishArgs& A, int a, int nF, const int32_t* flist,
                                    const int8_t* code, const int* ps, int nc, int ncol,
                                    int cap_on, double gam, float lbf, float ubf, float kap,
                                    bool phi, const Wk& wk, double* sm, double* shd) {
  const int k = A.k, G = A.G, tid = threadIdx.x, n = A.n;
  double* Hs = sm;                                   // [nF][nF]
  double* Vs = Hs + kSmallF * kSmallF;               // [nF][ncol]
  double* Xs = Vs + kSmallF * ncol;                  // [nF][ncol]
  double* fs = Xs + kSmallF * ncol;                  // [k]
  float* Bs = reinterpret_cast<float*>(fs + k);      // [nF][k]
  // stage the free rows' B, f and the constraint / rhs rows
  for (int e = tid; e < nF * k; e += kPT) {
    const int r = e / k, j = e % k;
    Bs[e] = A.Bt[(size_t)flist[r] * A.kp + j];
  }
  for (int j = tid; j < k; j += kPT) fs[j] = (double)A.f[j];
  double sgn_w0 = 0.0;
  for (int r = tid; r < nF; r += kPT) {
    const int i = flist[r];
    RowData rd = row_data(A, a, i, lbf, ubf);
    Geom g;
    make_geom(g, kap, phi, rd);
    double slope, sgn;
    piece_slope(g, code[i] >> 1, slope, sgn);
    double cross = 0.0;
    for (int j = 0; j < k; ++j) cross += (double)A.Bt[(size_t)i * A.kp + j] * wk.Fy[j];
    double* v = Vs + r * ncol;
    v[0] = 1.0;
    int col = 1;
    for (int gg = 0; gg < G; ++gg) {
      if (!band_active(ps, gg)) continue;
      v[col++] = row_coef(A, i, gg);
    }
    if (cap_on) v[col++] = sgn;
    v[col] = mu_at(A, (size_t)a * n + i) - slope - gam * cross;
    sgn_w0 += sgn * (double)rd.w0;
  }
  sgn_w0 = bsum<double>(sgn_w0, shd);            // (synchronises the staging)
  if (tid == 0 && cap_on) wk.h[nc - 1] += sgn_w0;
  // H, lower triangle
  for (int e = tid; e < nF * nF; e += kPT) {
    const int r = e / nF, c = e % nF;
    if (c > r) continue;
    const float* br = Bs + r * k;
    const float* bc = Bs + c * k;
    double h = 0.0;
    for (int j = 0; j < k; ++j) h += (double)br[j] * fs[j] * (double)bc[j];
    if (r == c) h += (double)A.d[flist[r]];
    Hs[e] = gam * h;
  }
  for (int e = tid; e < nF * ncol; e += kPT) Xs[e] = Vs[e];
  __syncthreads();
  // Cholesky by wave 0: lane i keeps row i; column j is scaled, then each
  // lane updates its own row of the trailing block (LDS accesses of one
  // wave complete in order; the fences keep the compiler from moving them)
  if (tid < 64) {
    const int i = tid;
    for (int j = 0; j < nF; ++j) {
      const double djj = sqrt(fmax(Hs[j * nF + j], 1e-300));
      double lij = 0.0;
      if (i > j && i < nF) {
        lij = Hs[i * nF + j] / djj;
        Hs[i * nF + j] = lij;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (i == j) Hs[j * nF + j] = djj;
      if (i > j && i < nF) {
        for (int l = j + 1; l <= i; ++l) Hs[i * nF + l] -= lij * Hs[l * nF + j];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  __syncthreads();
  chol_solve_cols(Hs, nF, Xs, ncol);               // X = H^-1 V (ends synchronised)
  // S = V_C^T X
  for (int e = tid; e < nc * ncol; e += kPT) {
    const int p = e / ncol, q = e % ncol;
    double s = 0.0;
    for (int r = 0; r < nF; ++r) s += Vs[r * ncol + p] * Xs[r * ncol + q];
    wk.S[p * ncol + q] = s;
  }
  return Xs;
}

__global__ __launch_bounds__(kPT) void polish_solve_kernel(PolishArgs A) {
  extern __shared__ double smem_d[];
  const int k = A.k, G = A.G, n = A.n;
  double* Kf = smem_d;                      // [k][k]
  // the Kf region also stages 64 float B rows before Kf is built
  const int kfsz = max(k * k, (64 * (k + 1) + 1) / 2);
  double* stg = Kf + kfsz;                  // staging: 16 rows x (k + 4)
  __shared__ double shd[kPW];
  __shared__ unsigned s_sig[kPW];
  __shared__ int s_cnt[2], s_same;
  const int slot = blockIdx.x;
  if (slot >= *A.m_act) return;
  const int a = A.act[slot];
  const int tid = threadIdx.x;
  int* ps = A.pstate + (size_t)a * kPStateStride;
  const float* par = A.par + (size_t)a * kNPar;
  const float lbf = par[P_LB], ubf = par[P_UB], kap = par[P_KAPPA], tauf = par[P_TAU];
  const double gam = par[P_GAMMA];
  const bool phi = (kap > 0.f) || isfinite(tauf) || (par[P_HASTAX] != 0.f);
  Wk wk = wk_of(A, a);
  int8_t* code = A.code + (size_t)a * n;
  int32_t* flist = A.flist + (size_t)a * n;         // free rows from the front
  double* w = A.wout + (size_t)a * n;

  if (A.first_round) {
    if (tid == 0) {
      ps[PS_CAP] = isfinite(tauf) && par[P_LAM] > 0.f;
      ps[PS_DONE] = 0;
      ps[PS_ROUNDS] = 0;
      ps[PS_STALL] = 0;
      ps[PS_BACT0] = ps[PS_BACT1] = ps[PS_BUP0] = ps[PS_BUP1] = 0;
      double* mult = A.mult + (size_t)a * (2 + G);
      mult[0] = par[P_NU];
      mult[1] = fmax((double)par[P_LAM], 0.0);
      for (int g = 0; g < G; ++g) {
        const float zb = A.zb[(size_t)a * G + g];
        const float lo = A.blo[(size_t)a * G + g], hi = A.bhi[(size_t)a * G + g];
        if (zb >= hi) set_band(ps, g, true, true);
        else if (zb <= lo) set_band(ps, g, true, false);
        mult[2 + g] = (double)par[P_RHOB] * (double)A.vb[(size_t)a * G + g];
      }
    }
    __syncthreads();
  } else if (ps[PS_DONE] || ps[PS_STALL]) {
    return;
  }
  const int cap_on = ps[PS_CAP];

  // ---- one pass over the rows: (first round) the pattern of the iterate,
  // fixed values, the free list from the front of flist and the nonzero
  // fixed list from its back (wave ballots + a per-wave prefix), the
  // budget and turnover sums of the fixed rows
  __shared__ int s_wc[2][kPW][2];
  if (tid == 0) { s_cnt[0] = 0; s_cnt[1] = 0; }
  __syncthreads();
  unsigned sig = 0u;                          // signature of the pattern
  double sx = 0.0, sturn = 0.0;
  {
    const int lane = tid & 63, wv = tid >> 6;
    int it = 0;
    for (int base = 0; base < n; base += kPT, ++it) {
      const int i = base + tid;
      int isfree = 0, isnz = 0;
      if (i < n) {
        int c;
        Geom g;
        RowData r;
        bool have = false;
        if (A.first_round) {
          r = row_data(A, a, i, lbf, ubf);
          make_geom(g, kap, phi, r);
          have = true;
          const float z = A.z[(size_t)a * n + i];
          // at point j (the float32 value the prox lands on), else inside
          // the piece above the inner points below z (the points ascend)
          c = (z == g.f0) ? 0 : (g.np > 1 && z == g.f1) ? 2 : (g.np > 2 && z == g.f2) ? 4
            : (g.np > 3 && z == g.f3) ? 6 : (g.np > 4 && z == g.f4) ? 8
            : (g.np > 5 && z == g.f5) ? 10 : -1;
          if (c < 0) {
            const double zd = z;
            const int q = (g.np > 2 && zd > g.p1 ? 1 : 0) + (g.np > 3 && zd > g.p2 ? 1 : 0) +
                          (g.np > 4 && zd > g.p3 ? 1 : 0) + (g.np > 5 && zd > g.p4 ? 1 : 0);
            c = (g.np == 1) ? 0 : 2 * q + 1;
            if (g.np > 1 && zd <= g.p0) c = 0;
            if (g.np > 1 && zd >= g.pt(g.np - 1)) c = 2 * (g.np - 1);
          }
          code[i] = (int8_t)c;
          sig += (unsigned)(c + 1) * ((unsigned)i * 2654435761u + 1u);
        } else {
          c = code[i];
        }
        if (c & 1) {
          isfree = 1;
          w[i] = 0.0;
        } else {
          if (!have) {
            r = row_data(A, a, i, lbf, ubf);
            make_geom(g, kap, phi, r);
          }
          const double v = g.pt(c >> 1);
          w[i] = v;
          isnz = (v != 0.0);
          sx += v;
          sturn += fabs(v - (double)r.w0);
        }
      }
      const unsigned long long mf = __ballot(isfree), mn = __ballot(isnz);
      const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
      const int par_ = it & 1;
      if (lane == 0) { s_wc[par_][wv][0] = __popcll(mf); s_wc[par_][wv][1] = __popcll(mn); }
      __syncthreads();
      int pf = __popcll(mf & below), pn = __popcll(mn & below), tf = 0, tn = 0;
      for (int q = 0; q < kPW; ++q) {
        if (q < wv) { pf += s_wc[par_][q][0]; pn += s_wc[par_][q][1]; }
        tf += s_wc[par_][q][0];
        tn += s_wc[par_][q][1];
      }
      const int c0 = s_cnt[0], c1 = s_cnt[1];
      if (isfree) flist[c0 + pf] = i;
      if (isnz) flist[n - 1 - (c1 + pn)] = i;
      __syncthreads();
      if (tid == 0) { s_cnt[0] = c0 + tf; s_cnt[1] = c1 + tn; }
    }
    __syncthreads();
  }
  if (A.first_round) {
    sig = bsum<unsigned>(sig, s_sig);
    if (tid == 0) {
      sig += (unsigned)ps[PS_CAP] * 97u + (unsigned)ps[PS_BACT0] * 31u + (unsigned)ps[PS_BACT1] * 7u +
             (unsigned)ps[PS_BUP0] * 5u + (unsigned)ps[PS_BUP1] * 3u;
      s_same = (unsigned)ps[PS_SIG] == sig;
      ps[PS_SIG] = (int)sig;
    }
  }
  sx = bsum<double>(sx, shd);
  sturn = bsum<double>(sturn, shd);
  const int nF = s_cnt[0], nX = s_cnt[1];
  // a pattern with many free coordinates belongs to an iterate that is far
  // from the optimum's vertex structure: skip the (costly) solve for now
  if ((A.nf_gate > 0 && nF > A.nf_gate) ||
      // a larger free set is solved only when the iterate shows the same
      // pattern at two consecutive checks
      (A.first_round && A.nf_small > 0 && nF > A.nf_small && !s_same)) {
    if (tid == 0) { ps[PS_STALL] = 1; ps[PS_NF] = nF; atomicAdd(A.pcount + 1, 1); }
    return;
  }
  if (tid == 0) atomicAdd(A.pcount, 1);

  // ---- fixed contributions ----------------------------------------------
  // yX = B_X^T w_X, budget / band / cap sums of the fixed rows
  __shared__ double s_gfix[kMaxG];
  {
    double ys = 0.0, gs = 0.0;
    float* sB = reinterpret_cast<float*>(Kf);          // Kf is not built yet
    double* swv = stg;
    int* siv = reinterpret_cast<int*>(stg + 64);
    list_sums(A, flist, n, nX, 1, w, sB, swv, siv, ys, gs);
    if (tid < k) { wk.yX[tid] = ys; wk.Fy[tid] = ys * (double)A.f[tid]; }
    if (tid < G) s_gfix[tid] = gs;
  }
  // active constraint columns: 0 budget, bands (active order), cap
  int nb = 0;
  for (int g = 0; g < G; ++g) nb += band_active(ps, g) ? 1 : 0;
  const int nc = 1 + nb + (cap_on ? 1 : 0);
  const int ncol = nc + 1;                      // + rhs column
  {
    if (tid == 0) {
      wk.h[0] = 1.0 - sx;
      int col = 1;
      for (int g = 0; g < G; ++g) {
        if (!band_active(ps, g)) continue;
        const double bnd = band_upper(ps, g) ? A.bhi[(size_t)a * G + g] : A.blo[(size_t)a * G + g];
        wk.h[col] = bnd - s_gfix[g];
        ++col;
      }
      if (cap_on) wk.h[col] = (double)tauf - sturn;   // + sum_F sgn w0 added below
      ps[PS_NF] = nF;
      ps[PS_NX] = nX;
      ps[PS_NC] = nc;
    }
  }
  __syncthreads();

  // A free set of at most kSmallF rows is solved in row space (its
  // gamma Sigma_FF is at most 64 x 64: one wave factors it); a larger one
  // through the factor space below.
  const bool small = nF <= kSmallF;
  double* Xs = nullptr;                   // small path: H^-1 [C | rhs] (LDS)
  if (small) {
    Xs = small_free_solve(A, a, nF, flist, code, ps, nc, ncol, cap_on, gam, lbf, ubf, kap,
                          phi, wk, smem_d, shd);
  } else {
  // ---- Kf = diag(1/f) + sum_F b b^T / d  (lower triangle, LDS) -----------
  // one 4 x 4 register tile of the lower triangle per thread; staged rows
  // are zero-padded to a multiple of 4 columns, 1/d_i follows them
  for (int e = tid; e < k * k; e += kPT) Kf[e] = 0.0;
  const int kt = (k + 3) >> 2;
  const int SR = 16, SS = 4 * kt + 4;
  {
    double acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;
    const int ntile = kt * (kt + 1) / 2;
    const bool own = tid < ntile;
    int tj = 0, tl = 0;
    if (own) {
      int j = (int)((sqrt(8.0 * tid + 1.0) - 1.0) * 0.5);
      while ((j + 1) * (j + 2) / 2 <= tid) ++j;
      while (j * (j + 1) / 2 > tid) --j;
      tj = j;
      tl = tid - j * (j + 1) / 2;
    }
    for (int f0 = 0; f0 < nF; f0 += SR) {
      const int rows = min(SR, nF - f0);
      __syncthreads();
      for (int e = tid; e < rows * 4 * kt; e += kPT) {
        const int rr = e / (4 * kt), j = e % (4 * kt);
        const int i = flist[f0 + rr];
        stg[rr * SS + j] = (j < k) ? (double)A.Bt[(size_t)i * A.kp + j] : 0.0;
      }
      for (int rr = tid; rr < rows; rr += kPT) stg[rr * SS + 4 * kt] = 1.0 / (double)A.d[flist[f0 + rr]];
      __syncthreads();
      if (own) {
        for (int rr = 0; rr < rows; ++rr) {
          const double* b = stg + rr * SS;
          const double id = b[4 * kt];
          double bj[4], bl[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) { bj[q] = b[4 * tj + q] * id; bl[q] = b[4 * tl + q]; }
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[q * 4 + r] += bj[q] * bl[r];
        }
      }
    }
    if (own) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = 4 * tj + q, l = 4 * tl + r;
          if (j < k && l <= j) {
            double v = acc[q * 4 + r];
            if (j == l) v += 1.0 / (double)A.f[j];
            Kf[j * k + l] = v;
          }
        }
    }
  }
  __syncthreads();

  // ---- Waug = sum_F b V^T / d,  CV = sum_F V V^T / d  ---------------------
  // V_i = [1, band indicators (active order), sgn_i (cap), rhs_i],
  // rhs_i = mu_i - slope_i - gamma b_i . F yX.  With X_i = [b_i | V_i] both
  // blocks are X^T D^-1 V: one 4 x 4 register tile per thread.
  double sgn_w0 = 0.0;
  {
    const int kx = k + ncol;
    const int xt = (kx + 3) >> 2, vt = (ncol + 3) >> 2;
    const int CS = 4 * xt + 4;                // 1/d_i at index 4 xt
    const bool own = tid < xt * vt;
    const int tj = own ? tid / vt : 0, tl = own ? tid % vt : 0;
    double acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;
    for (int f0 = 0; f0 < nF; f0 += SR) {
      const int rows = min(SR, nF - f0);
      __syncthreads();
      for (int e = tid; e < rows * 4 * xt; e += kPT) {
        const int rr = e / (4 * xt), j = e % (4 * xt);
        const int i = flist[f0 + rr];
        stg[rr * CS + j] = (j < k) ? (double)A.Bt[(size_t)i * A.kp + j] : 0.0;
      }
      __syncthreads();
      if (tid < rows) {
        const int rr = tid;
        const int i = flist[f0 + rr];
        RowData r = row_data(A, a, i, lbf, ubf);
        Geom g;
        make_geom(g, kap, phi, r);
        double slope, sgn;
        piece_slope(g, code[i] >> 1, slope, sgn);
        double* x = stg + rr * CS;
        double cross = 0.0;
        for (int j = 0; j < k; ++j) cross += x[j] * wk.Fy[j];
        double* v = x + k;
        v[0] = 1.0;
        int col = 1;
        for (int gg = 0; gg < G; ++gg) {
          if (!band_active(ps, gg)) continue;
          v[col++] = row_coef(A, i, gg);
        }
        if (cap_on) v[col++] = sgn;
        v[col] = mu_at(A, (size_t)a * n + i) - slope - gam * cross;
        x[4 * xt] = 1.0 / (double)A.d[i];
        sgn_w0 += sgn * (double)r.w0;
      }
      __syncthreads();
      if (own) {
        for (int rr = 0; rr < rows; ++rr) {
          const double* x = stg + rr * CS;
          const double id = x[4 * xt];
          double xl[4], vr[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            xl[q] = x[4 * tj + q] * id;
            vr[q] = (4 * tl + q < ncol) ? x[k + 4 * tl + q] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[q * 4 + r] += xl[q] * vr[r];
        }
      }
    }
    if (own) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int j = 4 * tj + q, l = 4 * tl + r;
          if (j >= kx || l >= ncol) continue;
          if (j < k) wk.Waug[j * ncol + l] = acc[q * 4 + r];
          else wk.CV[(j - k) * ncol + l] = acc[q * 4 + r];
        }
    }
  }
  sgn_w0 = bsum<double>(sgn_w0, shd);
  if (tid == 0 && cap_on) wk.h[nc - 1] += sgn_w0;
  __syncthreads();

  // ---- Cholesky of Kf (lower, in LDS) -------------------------------------
  for (int j = 0; j < k; ++j) {
    // every thread takes the pivot itself; thread 0 stores it after the
    // barrier that ends this step's reads of the unscaled diagonal
    const double djj = sqrt(fmax(Kf[j * k + j], 1e-300));
    for (int i = j + 1 + tid; i < k; i += kPT) Kf[i * k + j] /= djj;
    __syncthreads();
    if (tid == 0) Kf[j * k + j] = djj;
    const int m = k - j - 1;
    for (int e = tid; e < m * m; e += kPT) {
      const int i = j + 1 + e / m, l = j + 1 + e % m;
      if (l <= i) Kf[i * k + l] -= Kf[i * k + j] * Kf[l * k + j];
    }
    __syncthreads();
  }
  // ---- Y = Kf^-1 Waug -------------------------------------------------------
  for (int e = tid; e < k * ncol; e += kPT) wk.Y[e] = wk.Waug[e];
  __syncthreads();
  chol_solve_cols(Kf, k, wk.Y, ncol);
  // ---- Schur system on the constraint columns ------------------------------
  // gamma * C H^-1 V = CV[C, V] - Waug[:, C]^T Y[:, V]
  for (int e = tid; e < nc * ncol; e += kPT) {
    const int p = e / ncol, q = e % ncol;
    double s = wk.CV[p * ncol + q];
    for (int j = 0; j < k; ++j) s -= wk.Waug[j * ncol + p] * wk.Y[j * ncol + q];
    wk.S[p * ncol + q] = s / gam;
  }
  }                                       // factor-space path
  __syncthreads();
  if (tid == 0) {
    // eta0 from the ADMM iterate: -nu, band duals, lam_cap
    // eta0: multipliers of the previous pattern (first pattern: ADMM's)
    double* e0 = wk.eta0;
    const double* m0 = A.mult + (size_t)a * (2 + G);
    e0[0] = -m0[0];
    int col = 1;
    for (int g = 0; g < G; ++g) {
      if (!band_active(ps, g)) continue;
      e0[col++] = m0[2 + g];
    }
    if (cap_on) e0[col++] = fmax(m0[1], 0.0);
    // S eta = C H^-1 rhs - h with S = C H^-1 C^T (PSD).  Pivoted Cholesky
    // finds rank r; the pivot components are solved for, the others keep
    // eta0, and the null directions of S (the multipliers the free rows do
    // not pin) are stored for the certification step.
    double* Sm = wk.CV;                  // CV is consumed: nc x nc factor
    double* rr = wk.eta;
    int perm[kMaxG + 3];
    double dmax = 0.0;
    for (int p = 0; p < nc; ++p) {
      perm[p] = p;
      dmax = fmax(dmax, wk.S[p * ncol + p]);
      for (int q = 0; q < nc; ++q) Sm[p * nc + q] = wk.S[p * ncol + q];
    }
    const double ptol = 1e-12 * dmax;
    int rank = 0;
    for (int j = 0; j < nc; ++j) {
      int best = j;
      for (int p = j + 1; p < nc; ++p)
        if (Sm[p * nc + p] > Sm[best * nc + best]) best = p;
      if (!(Sm[best * nc + best] > ptol)) break;
      if (best != j) {
        for (int q = 0; q < nc; ++q) { double t = Sm[j * nc + q]; Sm[j * nc + q] = Sm[best * nc + q]; Sm[best * nc + q] = t; }
        for (int q = 0; q < nc; ++q) { double t = Sm[q * nc + j]; Sm[q * nc + j] = Sm[q * nc + best]; Sm[q * nc + best] = t; }
        int t = perm[j]; perm[j] = perm[best]; perm[best] = t;
      }
      const double djj = sqrt(Sm[j * nc + j]);
      Sm[j * nc + j] = djj;
      for (int i = j + 1; i < nc; ++i) Sm[i * nc + j] /= djj;
      for (int i = j + 1; i < nc; ++i)
        for (int l = j + 1; l <= i; ++l) {
          Sm[i * nc + l] -= Sm[i * nc + j] * Sm[l * nc + j];
          Sm[l * nc + i] = Sm[i * nc + l];
        }
      ++rank;
    }
    // right-hand side on the pivot rows, null components from eta0
    double x[kMaxG + 3];
    for (int j = 0; j < nc; ++j) x[j] = (j >= rank) ? e0[perm[j]] : 0.0;
    for (int j = 0; j < rank; ++j) {
      const int pj = perm[j];
      double t = wk.S[pj * ncol + nc] - wk.h[pj];
      for (int q = rank; q < nc; ++q) t -= wk.S[pj * ncol + perm[q]] * x[q];
      x[j] = t;
    }
    for (int i = 0; i < rank; ++i) {
      double t = x[i];
      for (int l = 0; l < i; ++l) t -= Sm[i * nc + l] * x[l];
      x[i] = t / Sm[i * nc + i];
    }
    for (int i = rank - 1; i >= 0; --i) {
      double t = x[i];
      for (int l = i + 1; l < rank; ++l) t -= Sm[l * nc + i] * x[l];
      x[i] = t / Sm[i * nc + i];
    }
    for (int j = 0; j < nc; ++j) rr[perm[j]] = x[j];
    // null directions: v_piv = -L11^-T L21^T e_t, v_t = 1
    const int nd = min(nc - rank, kMaxNull);
    for (int t = 0; t < nd; ++t) {
      double v[kMaxG + 3];
      for (int j = 0; j < nc; ++j) v[j] = 0.0;
      v[rank + t] = 1.0;
      for (int i = rank - 1; i >= 0; --i) {
        double u = -Sm[(rank + t) * nc + i];
        for (int l = i + 1; l < rank; ++l) u -= Sm[l * nc + i] * v[l];
        v[i] = u / Sm[i * nc + i];
      }
      // rows of the null block have the workspace's full column stride
      for (int j = 0; j < nc; ++j) wk.nul[t * (G + 3) + perm[j]] = v[j];
    }
    ps[PS_ND] = nd;
    // multipliers in the build's convention
    double* mult = A.mult + (size_t)a * (2 + G);
    mult[0] = -rr[0];
    col = 1;
    for (int g = 0; g < G; ++g) {
      if (band_active(ps, g)) mult[2 + g] = rr[col++];
      else mult[2 + g] = 0.0;
    }
    mult[1] = cap_on ? rr[col] : 0.0;
  }
  __syncthreads();
  if (small) {
    // w_F = H^-1 (rhs - C^T eta) = X[:, rhs] - X[:, C] eta
    for (int t = tid; t < nF; t += kPT) {
      double v = Xs[t * ncol + nc];
      for (int p = 0; p < nc; ++p) v -= Xs[t * ncol + p] * wk.eta[p];
      w[flist[t]] = v;
    }
  } else {
  // sol = Y[:, rhs] - Y[:, C] eta
  for (int j = tid; j < k; j += kPT) {
    double s = wk.Y[j * ncol + nc];
    for (int p = 0; p < nc; ++p) s -= wk.Y[j * ncol + p] * wk.eta[p];
    wk.sol[j] = s;
  }
  __syncthreads();
  // ---- free rows: w_i = (rhs_i - C_i^T eta - b_i . sol) / (gamma d_i) ----
  for (int t = tid; t < nF; t += kPT) {
    const int i = flist[t];
    RowData r = row_data(A, a, i, lbf, ubf);
    Geom g;
    make_geom(g, kap, phi, r);
    double slope, sgn;
    piece_slope(g, code[i] >> 1, slope, sgn);
    double cross = 0.0, bs = 0.0;
    for (int j = 0; j < k; ++j) {
      const double b = (double)A.Bt[(size_t)i * A.kp + j];
      cross += b * wk.Fy[j];
      bs += b * wk.sol[j];
    }
    const double rhs = mu_at(A, (size_t)a * n + i) - slope - gam * cross;
    double ct = wk.eta[0];
    int col = 1;
    for (int gg = 0; gg < G; ++gg) {
      if (!band_active(ps, gg)) continue;
      ct += row_coef(A, i, gg) * wk.eta[col];
      ++col;
    }
    if (cap_on) ct += sgn * wk.eta[col];
    w[i] = (rhs - ct - bs) / (gam * (double)A.d[i]);
  }
  }                                       // factor-space path
  // ---- y = F B^T w and the row sums of the polished w (nonzero rows), for
  // the gradient base and the certification: the fixed rows' parts from
  // above plus the free rows' --------------------------------------------
  __syncthreads();
  {
    double ys = 0.0, gs = 0.0;
    float* sB = reinterpret_cast<float*>(Kf);          // the solve is done with it
    double* swv = stg;
    int* siv = reinterpret_cast<int*>(stg + 64);
    list_sums(A, flist, n, nF, 0, w, sB, swv, siv, ys, gs);
    if (tid < k) wk.yF[tid] = (wk.yX[tid] + ys) * (double)A.f[tid];
    if (tid < G) wk.gsum[tid] = s_gfix[tid] + gs;
  }
}

// ---------------------------------------------------------------------------
// polish_gbase: gb_i = gamma (Sigma w)_i - mu_i for every row, spread over
// (row block, account) workgroups; per block: max |gamma Sigma w|, max |mu|,
// turnover and a non-finite flag
// ---------------------------------------------------------------------------
constexpr int kGbRows = 256;              // rows per gbase workgroup (one per thread)
constexpr int kGbAcc = 16;                // accounts per gbase workgroup

// g_i = gamma (d_i w_i + b_i . y) - mu_i for kGbRows rows x kGbAcc accounts:
// each thread streams its row of B once (four columns at a time) against
// the accounts' y vectors (LDS broadcasts), so the universe block is read
// once per 16 accounts; per-(account, row block) maxima / sums go to gpart
__global__ __launch_bounds__(256) void polish_gbase_kernel(PolishArgs A, int final_pass) {
  __shared__ double s_y[kGbAcc][kMaxK + 4];
  __shared__ int s_a[kGbAcc];
  __shared__ double s_gam[kGbAcc];
  __shared__ double s_red[4][kGbAcc][4];
  const int k = A.k, n = A.n, tid = threadIdx.x;
  const int m_act = *A.m_act;
  const int g0 = blockIdx.y * kGbAcc;
  if (g0 >= m_act) return;
  if (tid < kGbAcc) {
    int a = -1;
    if (g0 + tid < m_act) {
      const int aa = A.act[g0 + tid];
      const int* ps = A.pstate + (size_t)aa * kPStateStride;
      if (!(ps[PS_DONE] || (ps[PS_STALL] && !final_pass))) a = aa;
    }
    s_a[tid] = a;
    s_gam[tid] = a >= 0 ? (double)A.par[(size_t)a * kNPar + P_GAMMA] : 0.0;
  }
  __syncthreads();
  const int k4 = (k + 3) & ~3;                 // <= kp: whole float4 of each row
  for (int e = tid; e < kGbAcc * k4; e += 256) {
    const int q = e / k4, j = e % k4;
    const int a = s_a[q];
    s_y[q][j] = (a >= 0 && j < k) ? wk_of(A, a).yF[j] : 0.0;
  }
  __syncthreads();
  const int i = blockIdx.x * kGbRows + tid;
  const bool row_ok = i < n;
  double sig[kGbAcc];
#pragma unroll
  for (int q = 0; q < kGbAcc; ++q) sig[q] = 0.0;
  if (row_ok) {
    const float4* brow = reinterpret_cast<const float4*>(A.Bt + (size_t)i * A.kp);
    for (int j4 = 0; j4 < k4 / 4; ++j4) {
      const float4 b = brow[j4];
      const double b0 = b.x, b1 = b.y, b2 = b.z, b3 = b.w;
#pragma unroll
      for (int q = 0; q < kGbAcc; ++q) {
        const double* y = &s_y[q][4 * j4];
        sig[q] += b0 * y[0] + b1 * y[1] + b2 * y[2] + b3 * y[3];
      }
    }
  }
  const double di = row_ok ? (double)A.d[i] : 0.0;
  const int wv = tid >> 6;
#pragma unroll
  for (int q = 0; q < kGbAcc; ++q) {
    const int a = s_a[q];
    if (a < 0) continue;                       // uniform
    double gmax = 0.0, mumax = 0.0, turn = 0.0, bad = 0.0;
    if (row_ok) {
      const double wi = A.wout[(size_t)a * n + i];
      const double sg = sig[q] + di * wi;
      const double mui = mu_at(A, (size_t)a * n + i);
      const double v = s_gam[q] * sg - mui;
      A.gbase[(size_t)a * n + i] = v;
      gmax = fabs(s_gam[q] * sg);
      mumax = fabs(mui);
      turn = fabs(wi - (double)row_data(A, a, i, 0.f, 0.f).w0);
      if (!isfinite(v) || !isfinite(wi)) bad = 1.0;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
      gmax = fmax(gmax, __shfl_xor(gmax, o, 64));
      mumax = fmax(mumax, __shfl_xor(mumax, o, 64));
      turn += __shfl_xor(turn, o, 64);
      bad = fmax(bad, __shfl_xor(bad, o, 64));
    }
    if ((tid & 63) == 0) {
      s_red[wv][q][0] = gmax; s_red[wv][q][1] = mumax;
      s_red[wv][q][2] = turn; s_red[wv][q][3] = bad;
    }
  }
  __syncthreads();
  if (tid < 4 * kGbAcc) {
    const int q = tid >> 2, c = tid & 3;
    const int a = s_a[q];
    if (a >= 0) {
      double v = s_red[0][q][c];
      for (int w = 1; w < 4; ++w) v = (c == 2) ? v + s_red[w][q][c] : fmax(v, s_red[w][q][c]);
      A.gpart[((size_t)a * A.n_rb + blockIdx.x) * 4 + c] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// polish_check: external diagnostics in float64 and refinement
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPTC) void polish_check_kernel(PolishArgs A, fqp_result R,
                                                          int final_pass) {
  __shared__ double shd[kPW];
  __shared__ double s_gs[kMaxG];
  const int k = A.k, G = A.G, n = A.n;
  const int slot = blockIdx.x;
  if (slot >= *A.m_act) return;
  const int a = A.act[slot];
  const int tid = threadIdx.x;
  int* ps = A.pstate + (size_t)a * kPStateStride;
  if (ps[PS_DONE] || (ps[PS_STALL] && !final_pass)) return;
  __shared__ int s_changed;
  if (tid == 0) s_changed = 0;
  const float* par = A.par + (size_t)a * kNPar;
  const float lbf = par[P_LB], ubf = par[P_UB], kap = par[P_KAPPA], tauf = par[P_TAU];
  const double gam = par[P_GAMMA];
  const bool phi = (kap > 0.f) || isfinite(tauf) || (par[P_HASTAX] != 0.f);
  int changed = 0;
  int8_t* code_r = A.code + (size_t)a * n;
  int8_t* code = A.code_next + (size_t)a * n;    // proposals
  const int32_t* flist = A.flist + (size_t)a * n;
  const double* w = A.wout + (size_t)a * n;
  double* gmult = A.mult + (size_t)a * (2 + G);
  __shared__ double mult[2 + kMaxG];
  for (int q = tid; q < 2 + G; q += kPTC) mult[q] = gmult[q];
  const int nF = ps[PS_NF], nX = ps[PS_NX];
  double* gb = A.gbase + (size_t)a * n;
  __shared__ int s_bad, s_done;
  if (tid == 0) { s_bad = 0; s_done = 0; }

  // row sums (from the solve) and the reductions of polish_gbase
  __syncthreads();                        // flags above are initialised
  const Wk wkc = wk_of(A, a);
  for (int g = tid; g < G; g += kPTC) s_gs[g] = wkc.gsum[g];
  double gmax = 0.0, mumax = 0.0, turn0 = 0.0;
  int bad = 0;
  for (int rb = tid; rb < A.n_rb; rb += kPTC) {
    const double* gp = A.gpart + ((size_t)a * A.n_rb + rb) * 4;
    gmax = fmax(gmax, gp[0]);
    mumax = fmax(mumax, gp[1]);
    turn0 += gp[2];
    if (gp[3] != 0.0) bad = 1;
  }
  if (bad) atomicOr(&s_bad, 1);
  gmax = bmax<double>(gmax, shd);
  mumax = bmax<double>(mumax, shd);
  turn0 = bsum<double>(turn0, shd);
  const double scale = fmax(fmax(gmax, mumax), 1e-12);

  // ---- multipliers the free rows leave open -----------------------------
  // Along a stored null direction v of the free-row equations the free rows
  // stay stationary, and every fixed row's stationarity interval becomes a
  // pair of linear inequalities in the step s.  The step aims at zeroing
  // the multiplier of an active constraint that is not tight (its row was
  // dependent, so the solve could not enforce it); otherwise it stays
  // nearest to 0.  When a fixed row blocks that target, the row is the
  // one to release (dual active-set step): it is proposed below.
  __shared__ int s_block;                 // row * 16 + proposed code, or -1
  __shared__ int s_key[2];
  __shared__ double s_st;
  if (tid == 0) s_block = -1;
  {
    const int nd = ps[PS_ND];
    const int nc = ps[PS_NC];
    const int ncol = G + 3;
    const double* nul = wk_of(A, a).nul;
    const double thr = 0.01 * A.eps_comp * scale;
    // (a second sweep only matters when directions interact: nd > 1)
    for (int sweep = 0; sweep < (nd > 1 ? 2 : 1) && nd > 0; ++sweep) {
      for (int q = 0; q < nd; ++q) {
        const double* nv = nul + q * ncol;
        // column of each multiplier inside eta = (-nu, bands..., lam_cap)
        const double n0 = nv[0];
        const double ncap = ps[PS_CAP] ? nv[nc - 1] : 0.0;
        const double lamc = mult[1];
        double Lo = -INFINITY, Up = INFINITY;
        int loKey = INT_MAX, upKey = INT_MAX;
        for (int i = tid; i < n; i += kPTC) {
          const int c = code_r[i];
          if (c & 1) continue;
          RowData r = row_data(A, a, i, lbf, ubf);
          if (!r.el) continue;
          Geom g;
          make_geom(g, kap, phi, r);
          const double lb = r.lb, ub = r.ub;
          double nb = 0.0, lg = 0.0;
          if (G) {
            lg = rows_dot(A, i, mult + 2);
            int col = 1;
            for (int g2 = 0; g2 < G; ++g2) {
              if (!band_active(ps, g2)) continue;
              nb += row_coef(A, i, g2) * nv[col];
              ++col;
            }
          }
          const double T = -(gb[i] - mult[0] + lg);
          const double al = n0 + nb;
          const int j = c >> 1;
          // leaving the interval at its lower end: the row wants to go down
          const int keyL = (j > 0) ? i * 16 + 2 * (j - 1) + 1 : INT_MAX;
          const int keyU = (j + 1 < g.np) ? i * 16 + 2 * j + 1 : INT_MAX;
          double lo0, hi0, lo1, hi1, sn;
          subdiff(g, w[i], 0.0, lb, ub, lo0, hi0, sn);
          subdiff(g, w[i], 1.0, lb, ub, lo1, hi1, sn);
          // a coefficient that cancels to rounding level (a fixed row whose
          // interval moves with the free rows along v: the degenerate case
          // of free rows that all trade one way) puts no bound on the step;
          // taken at face value it would allow a step of 1/rounding
          if (isfinite(lo0)) {           // lo0 + s_lo (lamc + s ncap) <= T - al s
            const double slo = lo1 - lo0;
            const double aa = al + slo * ncap, bb = T - lo0 - slo * lamc;
            const double tz = 1e-12 * (fabs(al) + fabs(slo * ncap));
            if (aa > tz) { const double u = bb / aa; if (u < Up) { Up = u; upKey = keyL; } }
            else if (aa < -tz) { const double u = bb / aa; if (u > Lo) { Lo = u; loKey = keyL; } }
          }
          if (isfinite(hi0)) {           // T - al s <= hi0 + s_hi (lamc + s ncap)
            const double shi = hi1 - hi0;
            const double aa = -(al + shi * ncap), bb = hi0 + shi * lamc - T;
            const double tz = 1e-12 * (fabs(al) + fabs(shi * ncap));
            if (aa > tz) { const double u = bb / aa; if (u < Up) { Up = u; upKey = keyU; } }
            else if (aa < -tz) { const double u = bb / aa; if (u > Lo) { Lo = u; loKey = keyU; } }
          }
        }
        const double Lb = bmax<double>(Lo, shd);
        const double Ub = -bmax<double>(-Up, shd);
        if (tid == 0) { s_key[0] = INT_MAX; s_key[1] = INT_MAX; }
        __syncthreads();
        if (Lo == Lb && isfinite(Lb)) atomicMin(&s_key[0], loKey);
        if (Up == Ub && isfinite(Ub)) atomicMin(&s_key[1], upKey);
        __syncthreads();
        if (tid == 0) {
          Lo = Lb; Up = Ub;
          int kLo = s_key[0], kUp = s_key[1];
          // targets along this direction, by priority: (1) an active
          // constraint the solve could not enforce (dependent row) and that
          // is violated: push its multiplier outward until a fixed row
          // blocks, and release that row; (2) an active constraint that is
          // slack: zero its multiplier (complementarity)
          double tgt = 0.0, best = 0.0, worst = 0.0;
          bool has_tgt = false;
          const double vtol = 0.1 * A.eps_prim;
          if (ps[PS_CAP]) {              // lam_cap + s ncap >= 0
            if (ncap > 1e-12) { const double u = -lamc / ncap; if (u > Lo) { Lo = u; kLo = INT_MAX; } }
            else if (ncap < -1e-12) { const double u = -lamc / ncap; if (u < Up) { Up = u; kUp = INT_MAX; } }
            const double sl = (double)tauf - turn0;
            if (fabs(ncap) > 1e-12) {
              if (sl < -vtol && -sl > worst) {
                worst = -sl; tgt = (ncap > 0.0) ? INFINITY : -INFINITY; has_tgt = true;
              } else if (worst == 0.0) {
                const double v = fabs(lamc) * fmax(sl, 0.0);
                if (v > thr && v > best) { best = v; tgt = -lamc / ncap; has_tgt = true; }
              }
            }
          }
          int col = 1;
          for (int gg = 0; gg < G; ++gg) {
            if (!band_active(ps, gg)) continue;
            const double nbv = nv[col++];
            const double cur = mult[2 + gg];
            const bool up = band_upper(ps, gg);
            // upper band: lam >= 0 ; lower band: lam <= 0
            const double sgn_req = up ? 1.0 : -1.0;
            const double aa = sgn_req * nbv, bb = sgn_req * cur;   // bb + s aa >= 0
            if (aa > 1e-12) { const double u = -bb / aa; if (u > Lo) { Lo = u; kLo = INT_MAX; } }
            else if (aa < -1e-12) { const double u = -bb / aa; if (u < Up) { Up = u; kUp = INT_MAX; } }
            if (fabs(nbv) <= 1e-12) continue;
            const double sl = up ? (double)A.bhi[(size_t)a * G + gg] - s_gs[gg]
                                 : s_gs[gg] - (double)A.blo[(size_t)a * G + gg];
            if (sl < -vtol && -sl > worst) {
              worst = -sl; tgt = (aa > 0.0) ? INFINITY : -INFINITY; has_tgt = true;
            } else if (worst == 0.0) {
              const double v = fabs(cur) * fmax(sl, 0.0);
              if (v > thr && v > best) { best = v; tgt = -cur / nbv; has_tgt = true; }
            }
          }
          double st;
          if (Lo <= Up) {
            st = fmin(fmax(tgt, Lo), Up);
            if (has_tgt) {
              const int key = (tgt < Lo) ? kLo : (tgt > Up) ? kUp : INT_MAX;
              if (key != INT_MAX && s_block < 0) s_block = key;
            } else if (isfinite(Lo) && isfinite(Up)) {
              st += 1e-3 * (0.5 * (Lo + Up) - st);
            }
          } else {
            st = 0.5 * (Lo + Up);
          }
          if (!isfinite(st)) st = 0.0;
          // eta += st * v  ->  nu -= st v0, bands += st v_b, lam_cap += st v_cap
          mult[0] -= st * n0;
          col = 1;
          for (int gg = 0; gg < G; ++gg)
            if (band_active(ps, gg)) mult[2 + gg] += st * nv[col++];
          if (ps[PS_CAP]) mult[1] += st * ncap;
          s_st = st;
        }
        __syncthreads();
      }
    }
  }
  const double nu = mult[0], lam = mult[1];

  double sw = 0.0, turn = 0.0, dmax = 0.0, box = 0.0, snapm = 0.0, obj = 0.0;
  for (int i = tid; i < n; i += kPTC) {
    RowData r = row_data(A, a, i, lbf, ubf);
    Geom g;
    make_geom(g, kap, phi, r);
    const double lb = r.lb, ub = r.ub;
    const double wi = w[i];
    const double mui = mu_at(A, (size_t)a * n + i);
    const double sig = (gb[i] + mui) / gam;
    double gi = gb[i] - nu;
    if (G) gi += rows_dot(A, i, mult + 2);
    double lo, hi, snap;
    subdiff(g, wi, lam, lb, ub, lo, hi, snap);
    const double t = -gi;
    const double dist = fmax(fmax(lo - t, t - hi), 0.0);
    sw += wi;
    turn += fabs(wi - g.w0);
    dmax = fmax(dmax, dist);
    if (!isfinite(dist)) bad = 1;
    box = fmax(box, fmax(lb - wi, wi - ub));
    snapm = fmax(snapm, snap);
    // objective: (gamma/2) w.Sigma w - mu w + trade cost
    double tc = (double)kap * fabs(wi - g.w0);
    if (r.taxed && wi < g.w0) tc += lot_tax(g.w0 - wi, r);
    obj += 0.5 * gam * wi * sig - mui * wi + tc;
    // refinement proposal (applied only if the pattern fails)
    const int c = code_r[i];
    code[i] = (int8_t)c;
    if (g.np > 1) {
      const double tolm = A.eps_dual * 0.1;
      if (c & 1) {
        const int q = c >> 1;
        if (wi > g.pt(q + 1)) { code[i] = (int8_t)(2 * (q + 1)); ++changed; }
        else if (wi < g.pt(q)) { code[i] = (int8_t)(2 * q); ++changed; }
      } else {
        // move off a point when -g lies outside its subdifferential
        const int j = c >> 1;
        double l2, h2, sn2;
        subdiff(g, g.pt(j), lam, lb, ub, l2, h2, sn2);
        const double sc = fmax(fabs(mui), 1e-12);
        if (t > h2 + tolm * sc && j + 1 < g.np) { code[i] = (int8_t)(2 * j + 1); ++changed; }
        else if (t < l2 - tolm * sc && j > 0) { code[i] = (int8_t)(2 * (j - 1) + 1); ++changed; }
      }
    }
  }
  if (changed) atomicAdd(&s_changed, changed);
  if (bad) atomicOr(&s_bad, 1);
  sw = bsum<double>(sw, shd);
  turn = bsum<double>(turn, shd);
  obj = bsum<double>(obj, shd);
  dmax = bmax<double>(dmax, shd);
  box = bmax<double>(box, shd);
  snapm = bmax<double>(snapm, shd);

  if (tid == 0) {
    // comp: the largest |multiplier| x slack; gap: their sum, the duality
    // gap the multipliers leave (with stationarity and feasibility exact,
    // f(w) - f* <= gap)
    double rexp = 0.0, comp = 0.0, gap = 0.0;
    for (int g = 0; g < G; ++g) {
      const double lo = A.blo[(size_t)a * G + g], hi = A.bhi[(size_t)a * G + g];
      rexp = fmax(rexp, fmax(lo - s_gs[g], s_gs[g] - hi));
      const double lg = mult[2 + g];
      if (lg != 0.0) {              // (a one-sided row's other slack is infinite)
        const double slack = (lg > 0.0) ? hi - s_gs[g] : s_gs[g] - lo;
        comp = fmax(comp, fabs(lg) * fabs(slack));
        gap += fabs(lg) * fabs(slack);
      }
    }
    const double tau = tauf;
    double rturn = 0.0;
    if (isfinite(tauf)) {
      rturn = fmax(turn - tau, 0.0);
      comp = fmax(comp, fmax(lam, 0.0) * fabs(tau - turn));
      gap += fmax(lam, 0.0) * fabs(tau - turn);
    } else {
      comp = fmax(comp, fabs(lam));
    }
    const double obj_full = obj + (A.obj_const ? A.obj_const[a] : 0.0);
    const double r_prim = fmax(fmax(fabs(sw - 1.0), fmax(box, 0.0)), fmax(rexp, rturn)) + snapm;
    const double r_dual = fmax(dmax, fmax(-lam, 0.0)) / scale;
    const double r_comp = comp / scale;
    const bool finite = !s_bad && isfinite(sw) && isfinite(obj) && isfinite(nu) &&
                        isfinite(lam) && isfinite(r_prim) && isfinite(r_dual) &&
                        isfinite(r_comp);
    // the certificate also bounds the relative objective error: the gap
    // against |f| (when |f| is below the gradient scale, as a benchmark term
    // can make it, r_comp <= eps alone does not)
    const bool ok = finite && r_prim <= A.eps_prim && r_dual <= A.eps_dual &&
                    r_comp <= A.eps_comp && gap <= A.eps_comp * fmax(fabs(obj_full), 1e-12);
    for (int q = 0; q < 2 + G; ++q) gmult[q] = mult[q];
    ps[PS_ROUNDS] += 1;
    // keep the diagnostics of the latest pattern in the result arrays
    if (ok || final_pass) {
      if (R.r_prim) R.r_prim[a] = r_prim;
      if (R.r_dual) R.r_dual[a] = r_dual;
      if (R.r_comp) R.r_comp[a] = r_comp;
      // (the benchmark's constant (gamma/2) w_b^T Sigma w_b completes Eq. 1)
      if (R.obj) R.obj[a] = obj_full;
      if (R.nu) R.nu[a] = nu;
      if (R.lam_cap) R.lam_cap[a] = lam;
    }
    s_done = ok ? 1 : 0;
    if (ok) {
      ps[PS_DONE] = 1;
      R.status[a] = FQP_SOLVED;
    } else if (final_pass) {
      // the paper's quality gates (Sec. "Quality Gates and Failure
      // Vocabulary"): budget <= 1e-4 and bound violation <= 1e-6
      const bool gates = fabs(sw - 1.0) <= 1e-4 && box <= 1e-6 && rexp <= 1e-6 && rturn <= 1e-6;
      R.status[a] = gates ? FQP_FEASIBLE_UNCERTIFIED : FQP_MAX_ITER;
    } else {
      // bands / cap refinement
      int nchg = s_changed;
      if (s_block >= 0) {                // release the row that blocks
        code[s_block >> 4] = (int8_t)(s_block & 15);
        ++nchg;
      }
      for (int g = 0; g < G; ++g) {
        const double lo = A.blo[(size_t)a * G + g], hi = A.bhi[(size_t)a * G + g];
        const bool act = band_active(ps, g), up = band_upper(ps, g);
        const double lg = mult[2 + g];
        if (act && ((up && lg < 0.0) || (!up && lg > 0.0))) { set_band(ps, g, false, false); ++nchg; }
        else if (!act && s_gs[g] > hi + 0.1 * A.eps_prim) { set_band(ps, g, true, true); ++nchg; }
        else if (!act && s_gs[g] < lo - 0.1 * A.eps_prim) { set_band(ps, g, true, false); ++nchg; }
      }
      if (isfinite(tauf)) {
        if (ps[PS_CAP] && lam < 0.0) { ps[PS_CAP] = 0; ++nchg; }
        else if (!ps[PS_CAP] && turn > tau + 0.1 * A.eps_prim) { ps[PS_CAP] = 1; ++nchg; }
      }
      // no proposal: further rounds on this iterate cannot help; many
      // proposals: the iterate is still far from its final pattern, and the
      // next block of iterations is a cheaper way to get closer
      if (nchg == 0 || nchg > A.max_prop) ps[PS_STALL] = 1;
    }
  }
  __syncthreads();
  if (final_pass || s_done) {
    if (R.lam_band && G) {
      for (int g = tid; g < G; g += kPTC) R.lam_band[(size_t)a * G + g] = mult[2 + g];
    }
  } else {
    // the pattern failed: adopt the proposals for the next round
    for (int i = tid; i < n; i += kPTC) code_r[i] = code[i];
  }
}

static size_t polish_smem(int k, int G) {
  // Kf (k^2 doubles) and a staging region; the Kf region first holds 64
  // staged B rows (64 (k + 1) floats) and the staging region 64 weights +
  // 64 indices
  const size_t a = sizeof(double) * ((size_t)k * k);
  const size_t b = sizeof(float) * 64 * (size_t)(k + 1);
  // staging: 16 rows of [b | V | pad | 1/d]
  const size_t rest = sizeof(double) * 16 * (size_t)(4 * ((k + kMaxG + 3 + 3) / 4) + 4);
  const size_t factor = (a > b ? a : b) + (rest > 64 * 12 ? rest : 64 * 12);
  // row-space path: H, V, X, f (doubles) and the free rows of B (floats)
  const size_t ncol = (size_t)G + 3;
  const size_t rows = sizeof(double) * (kSmallF * kSmallF + 2 * kSmallF * ncol + (size_t)k) +
                      sizeof(float) * kSmallF * (size_t)k;
  return factor > rows ? factor : rows;
}

hipError_t launch_polish_solve(const PolishArgs& A, hipStream_t st) {
  const size_t smem = polish_smem(A.k, A.G);
  hipError_t e = hipFuncSetAttribute((const void*)polish_solve_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(polish_solve_kernel, dim3(A.m_total), dim3(kPT), smem, st, A);
  return hipGetLastError();
}

hipError_t launch_polish_check_r(const PolishArgs& A, const fqp_result& R, int final_pass,
                                 hipStream_t st) {
  hipLaunchKernelGGL(polish_gbase_kernel, dim3(A.n_rb, (A.m_total + kGbAcc - 1) / kGbAcc),
                     dim3(256), 0, st, A, final_pass);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(polish_check_kernel, dim3(A.m_total), dim3(kPTC), 0, st, A, R, final_pass);
  return hipGetLastError();
}

int polish_row_blocks(int n) { return (n + kGbRows - 1) / kGbRows; }

// The accounts of the active list still refining their pattern (neither
// certified nor stalled in this pass), in list order: the later rounds of a
// pass run on this list, so that their grids (the gradient base above all,
// which works on groups of accounts) cover only those accounts.
__global__ __launch_bounds__(1024) void polish_list_kernel(const int* m_act, const int* act,
                                                           const int32_t* pstate, int* pact,
                                                           int* pm_act) {
  __shared__ int s_wc[16];
  __shared__ int s_base;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m = *m_act;
  if (tid == 0) s_base = 0;
  __syncthreads();
  for (int b0 = 0; b0 < m; b0 += 1024) {
    const int slot = b0 + tid;
    int keep = 0, a = -1;
    if (slot < m) {
      a = act[slot];
      const int32_t* ps = pstate + (size_t)a * kPStateStride;
      keep = !(ps[PS_DONE] || ps[PS_STALL]);
    }
    const unsigned long long mk = __ballot(keep);
    if (lane == 0) s_wc[wv] = __popcll(mk);
    __syncthreads();
    int off = s_base + __popcll(mk & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
    for (int q = 0; q < wv; ++q) off += s_wc[q];
    if (keep) pact[off] = a;
    __syncthreads();
    if (tid == 0) {
      int t = 0;
      for (int q = 0; q < 16; ++q) t += s_wc[q];
      s_base += t;
    }
    __syncthreads();
  }
  if (tid == 0) *pm_act = s_base;
}

hipError_t launch_polish_list(const int* m_act, const int* act, const int32_t* pstate, int* pact,
                              int* pm_act, hipStream_t st) {
  hipLaunchKernelGGL(polish_list_kernel, dim3(1), dim3(1024), 0, st, m_act, act, pstate, pact,
                     pm_act);
  return hipGetLastError();
}

}  // namespace fqp
