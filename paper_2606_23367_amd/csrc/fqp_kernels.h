// Kernel argument blocks and launchers (internal to libfqp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fqp_common.h"

namespace fqp {

struct IterArgs {
  int n, W;                  // assets, bitmask words per account
  int m_total;               // accounts in the book (partials are indexed by id)
  const int* m_act;          // device: number of active accounts
  const int* act;            // device: active account ids [m_act]
  const float* Bt;           // [n][kp]
  const float* d;            // [n]
  const float* mu;           // [m][n]
  float* v;                  // [m][n]  ADMM state v = xh + u
  const uint32_t* elig;      // [m][W] or null
  const uint32_t* hold;      // [m][W]
  const int32_t* hold_pre;   // [m][W]
  const int32_t* hold_ptr;   // [m+1]
  const float* hold_w0;      // [nnz_h]
  const int32_t* hold_tax;   // [nnz_h]
  const float* tax_brk;      // [nnz_t][3]
  const float* tax_slope;    // [nnz_t][4]
  const float4* hold_rec;    // [nnz_h][2]: {w0, b1, b2, b3}, {s0, s1, s2, s3}; b1 < 0: no lots
  int npad;                  // rows of the bf16 copies of B~ (n padded to whole chunks)
  const uint16_t* bt_hi;     // npad x kp bf16 hi part of B~, PROJECT operand order
  const uint16_t* bt_lo;     // its lo part
  const uint16_t* btt_hi;    // npad x kp bf16 hi part of B~, CONTRACT operand order
  const uint16_t* btt_lo;    // its lo part
  const float* pp;           // [m][kp]
  const float* par;          // [m][kNPar]
  float* par_rw;             // same array, written by the cap kernel
  float* part;               // [row tiles][m][kp] (at most one per 128-row chunk)
  const float* lbv;          // [m][n] per-asset bounds, or null (the
  const float* ubv;          //   account's scalars P_LB / P_UB)
  float* zs;                 // [m][n] w = v + alpha (Delta^-1 r - z) of the
                             // current iterate: PROX writes it, PROJECT adds
                             // the back-projection; before a polish it holds
                             // z = prox(v; lam*) instead (PROX in z mode)
  float* rp;                 // [m][npad] R' = r / Delta of the current iterate
                             // (PROX writes rows < n, CONTRACT reads it)
};

struct KArgs {
  int kp, k, G, n, nblk, m_total;    // nblk: workgroups of the CONTRACT pass
  int nblk_p;                        // workgroups of the PROJECT pass
  int ncls;                          // gamma classes (1: no per-account class lookup)
  const int* m_act;
  const int* act;
  const float* part;
  float* par;                // [m][kNPar]
  float* pp;                 // [m][kp]
  const float* Kinv;         // [ncls][kp][kp]
  const float* cvec;         // [ncls][kp]
  const float* qvec;         // [ncls][kp]
  const float* sig1;         // [ncls]
  const float* mbg;          // [ncls][kp][G]
  float* zb;                 // [m][G]
  float* vb;                 // [m][G]
  const float* blo;          // [m][G]
  const float* bhi;          // [m][G]
  int* iters;                // [m]
};

// Work split of the two iteration passes for the current number of active
// accounts: the grid's workgroups are spread over the active 32-account
// tiles, and each tile's rows are cut into as many row tiles as it gets
// workgroups (whole 128-row chunks), so a short active list still fills the
// chip.  The k-space solve uses the same split to find the partials.
struct TileMap {
  int tile, rt, n_rt, chunks, row_begin;
  bool active;
};
__device__ __forceinline__ TileMap tile_map(int m_act, int n, int nblk, int lin) {
  const int tiles = (m_act + kTM - 1) / kTM;
  const int total_chunks = (n + kRowsPerChunk - 1) / kRowsPerChunk;
  int r = tiles > 0 ? nblk / tiles : 1;
  r = r < 1 ? 1 : (r > total_chunks ? total_chunks : r);
  const int cpt = (total_chunks + r - 1) / r;        // chunks per row tile
  TileMap t;
  t.n_rt = (total_chunks + cpt - 1) / cpt;
  t.chunks = cpt;
  t.tile = lin / t.n_rt;
  t.rt = lin % t.n_rt;
  t.row_begin = t.rt * cpt * kRowsPerChunk;
  t.active = t.tile < tiles;
  return t;
}

hipError_t configure_iter_kernels();
// workgroups of one iteration pass (mode) resident on one compute unit at
// once; 0 if the runtime cannot tell
int iter_blocks_per_cu(int kp, int prec, int mode);
// ev0 / ev1 (optional): events stamped at the start and the end of the
// kernel's own execution (not of the queue around it)
hipError_t launch_iter(const IterArgs& A, int kp, int mode, int prec, dim3 grid,
                       hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_split_bt(int n, int npad, int kp, const float* Bt, uint16_t* bh, uint16_t* bl,
                           uint16_t* bth, uint16_t* btl, hipStream_t st);
// the per-account PROX pass (cap multiplier, then R' and w; zmode: z): the
// register-resident layout needs n <= 16384, at most 2048 held rows in
// every account and no per-asset bounds
bool cap_resident_fits(int n, int max_held);
hipError_t launch_prox(const IterArgs& A, int m_total, bool resident, int zmode,
                       hipStream_t st, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_ksolve(const KArgs& A, int m_total, hipStream_t st);
hipError_t launch_build_bt(int n, int k, int G, int H, int kp, const float* B,
                           const int32_t* group, const float* half, float* Bt, hipStream_t st);
hipError_t launch_gram(int n, int kp, int kg, int nparts, int rows_per_blk, const float* Bt,
                       const float* d, double gamma, double rho, double* part, hipStream_t st);
hipError_t launch_kfactor(int k, int G, int kp, int nparts, const double* part, const float* f,
                          double gamma, double rho_b, double* Kw, float* Kinv, float* c,
                          float* q, float* sig, float* mbg, hipStream_t st);

// ---- packing / validation -------------------------------------------------
struct PackArgs {
  int n, W, m, G;            // G: constraint rows (bands, then halfspaces)
  int Gl;                    // band rows (finite bounds required)
  const float* lbv;          // [m][n] per-asset bounds or null
  const float* ubv;
  const float* eta;          // [m] or null
  const float* mu;
  const float* w0;
  const float* lb;
  const float* ub;
  const uint32_t* elig;
  const float* gamma;
  const float* kappa;
  const float* tau;
  const float* blo;
  const float* bhi;
  const int32_t* tax_ptr;
  const int32_t* tax_asset;
  const float* tax_brk;
  const float* tax_slope;
  // outputs
  uint32_t* hold;
  int32_t* hold_pre;
  int32_t* hold_cnt;        // [m]
  int32_t* hold_ptr;        // [m+2]: prefix [m+1], then the largest count
  float* hold_w0;
  int32_t* hold_tax;
  int32_t* status;          // [m]
  float* par;               // [m][kNPar]
  // pinned host memory (device address) or null: the total of held names
  // and the most held names of one account, stored by the scan
  int32_t* host_counts;
};
hipError_t launch_pack_count(const PackArgs& A, hipStream_t st);
hipError_t launch_pack_scan(const PackArgs& A, hipStream_t st);
hipError_t launch_pack_fill(const PackArgs& A, hipStream_t st);
hipError_t launch_pack_rec(const PackArgs& A, float4* rec, int total, hipStream_t st);

// ---- polish / certification (float64) -------------------------------------
// ints of polish bookkeeping per account
constexpr int kPStateStride = 16;

struct PolishArgs {
  int n, k, G, kp, W, m_total;  // G: constraint rows, bands then halfspaces
  int Gl;                    // band rows, one-hot by label; rows Gl..G-1 are
                             // the halfspace columns k + Gl.. of B~
  const float* lbv;          // [m][n] per-asset bounds or null
  const float* ubv;
  const double* obj_const;   // [m] (gamma/2) w_b^T Sigma w_b, or null
  const double* mu64;        // [m][n] mu' = eta mu + gamma Sigma w_b in float64
                             // (with a benchmark or eta; mu holds it in float32)
  const int* m_act;
  const int* act;
  const float* Bt;           // [n][kp] (first k columns = B)
  const float* f;            // [k]
  const float* d;            // [n]
  const int32_t* group;      // [n] or null
  const float* mu;           // [m][n]
  const float* z;            // [m][n]  ADMM iterate
  const uint32_t* elig;
  const uint32_t* hold;
  const int32_t* hold_pre;
  const float4* hold_rec;    // [nnz_h][2] packed held records (as IterArgs)
  const int32_t* hold_ptr;
  const float* hold_w0;
  const int32_t* hold_tax;
  const float* tax_brk;
  const float* tax_slope;
  const float* par;          // [m][kNPar]
  const float* zb;           // [m][G] ADMM band state
  const float* vb;           // [m][G] ADMM band scaled duals
  const float* blo;
  const float* bhi;
  int8_t* code;              // [m][n] active-set codes
  int8_t* code_next;         // [m][n] refinement proposals
  int32_t* flist;            // [m][n] free list
  double* wk;                // [m][wk_stride] per-account scratch
  size_t wk_stride;
  double* wout;              // [m][n] polished weights (caller output)
  double* gbase;             // [m][n] gamma (Sigma w)_i - mu_i of the pattern
  double* mult;              // [m][2 + G] nu, lam_cap, lam_band
  int32_t* pstate;           // [m][kPStateStride] polish bookkeeping
  double eps_prim, eps_dual, eps_comp;
  int first_round;           // classify from z when nonzero
  int nf_gate;               // skip patterns with more free rows (0: never)
  int nf_small;              // larger free sets wait for a repeated pattern
  int* pcount;               // [2] reduced solves formed, attempts gated
  int max_prop;              // a failed pattern with more proposals stops refining
  int n_rb;                  // row blocks of the gradient-base pass
  double* gpart;             // [m][n_rb][4] its per-block reductions
  int n_sb;                  // row blocks of the other row passes
  int32_t* fseg;             // [m][n] per-block free / nonzero fixed rows
  double* rpart;             // [m][n_sb][polish_rpart_stride] pattern partials
  double* spart;             // [m][n_sb][4] null-direction sweep partials
  double* cpart;             // [m][n_sb][8] diagnostic partials
};
hipError_t launch_polish_solve(const PolishArgs& A, hipStream_t st);
// pact / pm_act: the accounts of act / m_act that neither certified nor stalled;
// host_count (pinned host memory, device address, or null) also receives the count
hipError_t launch_polish_list(const int* m_act, const int* act, const int32_t* pstate, int* pact,
                              int* pm_act, int* host_count, hipStream_t st);
size_t polish_wk_stride(int k, int G);
int polish_row_blocks(int n);
int polish_pass_blocks(int n);
int polish_rpart_stride(int k, int G);

// ---- KKT adjoint (float64) ---------------------------------------------------
struct AdjArgs {
  int n, k, G, kp, m;        // G: constraint rows (as PolishArgs)
  int Gl;
  const float* wb;           // [m][n] benchmark weights or null
  const float* eta;          // [m] return scale or null
  const double* ywb;         // [m][k] B^T w_b (with wb)
  const float* Bt;
  const float* f;
  const float* d;
  const int32_t* group;
  const float* w0in;         // [m][n] caller's w0
  const float* par;
  const int32_t* status;     // [m] statuses of the last solve
  const int32_t* pstate;
  const int32_t* flist;
  const int8_t* code;
  const double* w;           // [m][n] weights of the last solve
  const double* dLdw;        // [m][n]
  double* dmu;               // [m][n] out
  double* dB;                // [n][k] out
  double* yvw;               // [m][2k] scratch
  double* wk;
  size_t wk_stride;
};
hipError_t launch_adjoint(const AdjArgs& A, hipStream_t st);

// ---- the rest of Eq. 1 -------------------------------------------------------
// box of (account a, asset i) of an eligible asset: the per-asset bounds
// when the book has them, else the account's scalars (excluded: [0, 0])
template <typename Args>
__device__ __forceinline__ void asset_box(const Args& A, size_t off, bool el, float lbp,
                                          float ubp, float& lb, float& ub) {
  if (!el) { lb = 0.f; ub = 0.f; return; }
  lb = A.lbv ? A.lbv[off] : lbp;
  ub = A.ubv ? A.ubv[off] : ubp;
}

// the linear term of the polish and certificate: mu' in float64 when the
// book has a benchmark term, else the caller's mu
__device__ __forceinline__ double mu_at(const PolishArgs& A, size_t off) {
  return A.mu64 ? A.mu64[off] : (double)A.mu[off];
}

// coefficient of constraint row g at asset i: band rows (g < Gl) are
// one-hot by label, halfspace rows are the columns k + g of B~
template <typename Args>
__device__ __forceinline__ double row_coef(const Args& A, int i, int g) {
  return g < A.Gl ? (A.group[i] == g ? 1.0 : 0.0) : (double)A.Bt[(size_t)i * A.kp + A.k + g];
}

// sum_g (row g at asset i) x[g] over every constraint row
template <typename Args>
__device__ __forceinline__ double rows_dot(const Args& A, int i, const double* x) {
  double s = A.Gl ? x[A.group[i]] : 0.0;
  for (int g = A.Gl; g < A.G; ++g) s += (double)A.Bt[(size_t)i * A.kp + A.k + g] * x[g];
  return s;
}

// mu' = eta mu + gamma Sigma w_b and (gamma/2) w_b^T Sigma w_b per account
// (the benchmark term of Eq. 1 expanded)
hipError_t launch_benchmark_prep(int m, int n, int k, const float* B, const float* f,
                                 const float* d, const float* mu, const float* wb,
                                 const float* eta, const float* gamma, double* ywb,
                                 double* part, float* mu_out, double* mu64_out,
                                 double* obj_const, hipStream_t st);
int benchmark_row_blocks(int n);
// the band bounds then the halfspace bounds, [m][G + H]
hipError_t launch_concat_rows(int m, int G, int H, const float* blo, const float* bhi,
                              const float* hlo, const float* hhi, float* lo, float* hi,
                              hipStream_t st);

}  // namespace fqp
