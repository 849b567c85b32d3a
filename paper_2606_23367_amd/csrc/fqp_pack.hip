// Book packing and per-account input validation (gfx950).
//
// Held assets (w0 != 0) are stored sparsely: a bitmask per account
// ([m][W] words, bit i%32 of word i/32), a per-word prefix count, and one
// record per held asset (w0 and the index of its tax lots, or -1).  The
// fused iteration reads one broadcast word per 32 assets and gathers the
// record only for held assets, so untraded names cost no w0 traffic.
//
// Validation follows the problem class of Eq. 1 (Sec. "Benchmark Problem
// Class"): the program must be convex (non-negative, non-decreasing lot
// slopes; increasing breakpoints; eta >= 0) and feasible.  Box + budget
// feasibility is sum_elig lb_i <= 1 <= sum_elig ub_i; the least turnover of
// any feasible portfolio is sum_i |w0_i - clip_i(w0_i)| + |1 - sum_i
// clip_i(w0_i)| (clip to the asset's box, 0 for excluded names), so a
// smaller cap is infeasible.  Band rows need finite bounds lo <= hi; a
// halfspace row may leave one side infinite.  (Feasibility of the bands and
// halfspaces themselves is not proven here: an account whose rows cannot
// be met ends uncertified.)
#include "fqp_common.h"
#include "fqp_kernels.h"
#include "../../include/fqp.h"

namespace fqp {

__device__ __forceinline__ bool is_elig(const uint32_t* elig, int W, int a, int i) {
  return elig == nullptr || ((elig[(size_t)a * W + (i >> 5)] >> (i & 31)) & 1u);
}

template <typename T>
__device__ T block_reduce_sum(T v, T* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = blockDim.x / 2; o >= 1; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  T r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void pack_count_kernel(PackArgs A) {
  __shared__ double shd[256];
  __shared__ int shi[256];
  const int a = blockIdx.x;
  const int n = A.n, W = A.W;
  const float lb = A.lb[a], ub = A.ub[a];
  int held = 0, bad = 0, bad_box = 0;
  double sum_clip = 0.0, dist = 0.0, sum_lb = 0.0, sum_ub = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const size_t off = (size_t)a * n + i;
    const float mu = A.mu[off];
    const float w0 = A.w0[off];
    if (!isfinite(mu) || !isfinite(w0)) bad = 1;
    if (w0 != 0.f) ++held;
    const bool el = is_elig(A.elig, W, a, i);
    float lf, uf;
    asset_box(A, off, el, lb, ub, lf, uf);
    if (!(lf <= uf) || !isfinite(lf) || !isfinite(uf)) bad_box = 1;
    const double l = lf, u = uf;
    sum_lb += l;
    sum_ub += u;
    const double c = fmin(fmax((double)w0, l), u);
    sum_clip += c;
    dist += fabs((double)w0 - c);
  }
  held = block_reduce_sum<int>(held, shi);
  bad = block_reduce_sum<int>(bad, shi);
  bad_box = block_reduce_sum<int>(bad_box, shi);
  sum_clip = block_reduce_sum<double>(sum_clip, shd);
  dist = block_reduce_sum<double>(dist, shd);
  sum_lb = block_reduce_sum<double>(sum_lb, shd);
  sum_ub = block_reduce_sum<double>(sum_ub, shd);

  // lot data of this account
  int bad_tax = 0;
  if (A.tax_ptr) {
    const int s = A.tax_ptr[a], e = A.tax_ptr[a + 1];
    if (e < s) bad_tax = 1;
    for (int j = s + threadIdx.x; j < e; j += 256) {
      const int i = A.tax_asset[j];
      if (i < 0 || i >= n) { bad_tax = 1; continue; }
      if (j > s && A.tax_asset[j - 1] >= i) bad_tax = 1;
      if (!(A.w0[(size_t)a * n + i] > 0.f)) bad_tax = 1;
      const float b1 = A.tax_brk[3 * j], b2 = A.tax_brk[3 * j + 1], b3 = A.tax_brk[3 * j + 2];
      const float s0 = A.tax_slope[4 * j], s1 = A.tax_slope[4 * j + 1];
      const float s2 = A.tax_slope[4 * j + 2], s3 = A.tax_slope[4 * j + 3];
      if (!(b1 > 0.f && b2 > b1 && b3 > b2 && isfinite(b3))) bad_tax = 1;
      if (!(s0 >= 0.f && s1 >= s0 && s2 >= s1 && s3 >= s2 && isfinite(s3))) bad_tax = 1;
    }
  }
  bad_tax = block_reduce_sum<int>(bad_tax, shi);
  int bad_band = 0;
  if (A.blo) {
    for (int g = threadIdx.x; g < A.G; g += 256) {
      const float lo = A.blo[(size_t)a * A.G + g], hi = A.bhi[(size_t)a * A.G + g];
      if (!(lo <= hi) || lo == INFINITY || hi == -INFINITY) bad_band = 1;
      if (g < A.Gl && (!isfinite(lo) || !isfinite(hi))) bad_band = 1;
    }
  }
  bad_band = block_reduce_sum<int>(bad_band, shi);

  if (threadIdx.x == 0) {
    A.hold_cnt[a] = held;
    const float gam = A.gamma[a], kap = A.kappa[a], tau = A.tau[a];
    const float eta = A.eta ? A.eta[a] : 1.f;
    int st = FQP_SOLVED;   // tentatively "to be solved"
    if (bad) st = FQP_NUMERICAL_ERROR;
    else if (!(lb <= ub) || !isfinite(lb) || !isfinite(ub) || !(gam > 0.f) || !isfinite(gam) ||
             !(kap >= 0.f) || !isfinite(kap) || !(tau >= 0.f) || bad_tax || bad_band ||
             bad_box || !(eta >= 0.f) || !isfinite(eta))
      st = FQP_INVALID_INPUT;
    else if (sum_ub < 1.0 - 1e-7 || sum_lb > 1.0 + 1e-7)
      st = FQP_PRIMAL_INFEASIBLE;
    else if (isfinite(tau)) {
      const double tau_min = dist + fabs(1.0 - sum_clip);
      if ((double)tau < tau_min * (1.0 - 1e-7) - 1e-9) st = FQP_PRIMAL_INFEASIBLE;
    }
    A.status[a] = (st == FQP_SOLVED) ? -1 : st;   // -1: valid, not yet solved
  }
}

__global__ void pack_scan_kernel(PackArgs A) {
  // exclusive scan of hold_cnt into hold_ptr (single workgroup); the total
  // goes to hold_ptr[m], the largest count of one account to hold_ptr[m + 1]
  __shared__ int carry, most;
  __shared__ int sh[256];
  if (threadIdx.x == 0) {
    carry = 0;
    most = 0;
  }
  __syncthreads();
  int mx = 0;
  for (int base = 0; base < A.m; base += 256) {
    const int i = base + threadIdx.x;
    const int v = (i < A.m) ? A.hold_cnt[i] : 0;
    mx = max(mx, v);
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      int t = (threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < A.m) A.hold_ptr[i] = carry + sh[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 255) carry += sh[255];
    __syncthreads();
  }
  atomicMax(&most, mx);
  __syncthreads();
  if (threadIdx.x == 0) {
    A.hold_ptr[A.m] = carry;
    A.hold_ptr[A.m + 1] = most;
    if (A.host_counts) {
      A.host_counts[0] = carry;
      A.host_counts[1] = most;
    }
  }
}

__global__ __launch_bounds__(256) void pack_fill_kernel(PackArgs A) {
  __shared__ int sh[256];
  __shared__ int carry;
  __shared__ uint32_t s_bits[256];
  const int a = blockIdx.x;
  const int n = A.n, W = A.W;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int base_rec = A.hold_ptr[a];
  const int t0 = A.tax_ptr ? A.tax_ptr[a] : 0;
  const int t1 = A.tax_ptr ? A.tax_ptr[a + 1] : 0;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int wb = 0; wb < W; wb += 256) {
    // the holding words wb .. wb + 255: their rows read coalesced, one per
    // thread and step, each wave's 64 rows turned into two words by a ballot
#pragma unroll 8
    for (int s = 0; s < 32; ++s) {
      const int i = 32 * wb + 256 * s + threadIdx.x;
      const bool h = i < n && A.w0[(size_t)a * n + i] != 0.f;
      const unsigned long long mk = __ballot(h);
      if (lane == 0) {
        const int wr = 8 * s + 2 * wv;           // (256 s + 64 wv) / 32
        s_bits[wr] = (uint32_t)mk;
        s_bits[wr + 1] = (uint32_t)(mk >> 32);
      }
    }
    __syncthreads();
    const int wd = wb + threadIdx.x;
    const uint32_t bits = (wd < W) ? s_bits[threadIdx.x] : 0u;
    const int pc = __popc(bits);
    sh[threadIdx.x] = pc;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      int t = (threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    const int pre = carry + sh[threadIdx.x] - pc;
    if (wd < W) {
      A.hold[(size_t)a * W + wd] = bits;
      A.hold_pre[(size_t)a * W + wd] = pre;
      int r = 0;
      for (int b = 0; b < 32; ++b) {
        if (!((bits >> b) & 1u)) continue;
        const int i = 32 * wd + b;
        const int idx = base_rec + pre + r;
        ++r;
        A.hold_w0[idx] = A.w0[(size_t)a * n + i];
        A.hold_tax[idx] = -1;                    // set below for a taxed name
      }
    }
    __syncthreads();
    if (threadIdx.x == 255) carry += sh[255];
    __syncthreads();
  }
  // every lot entry points its name's record at itself: the record index is
  // the name's rank among the held rows, from the word and prefix written
  // above.  An entry off the book or on a name not held (an account the
  // count pass already marked invalid) writes nothing, so it cannot reach
  // another account's records.
  __threadfence_block();
  __syncthreads();
  for (int j = t0 + threadIdx.x; j < t1; j += 256) {
    const int i = A.tax_asset[j];
    if (i < 0 || i >= n) continue;
    const size_t wi = (size_t)a * W + (i >> 5);
    const uint32_t hw = A.hold[wi];
    if (!((hw >> (i & 31)) & 1u)) continue;
    A.hold_tax[base_rec + A.hold_pre[wi] + __popc(hw & ((1u << (i & 31)) - 1u))] = j;
  }
}

// held-asset records in the layout the iteration kernels read: two float4
// per record, w0 and the lot data side by side (one dependent load level)
__global__ void pack_rec_kernel(PackArgs A, float4* rec, int total) {
  for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += gridDim.x * blockDim.x) {
    const float w0 = A.hold_w0[idx];
    const int ti = A.hold_tax[idx];
    if (ti >= 0) {
      rec[2 * idx] = make_float4(w0, A.tax_brk[3 * ti], A.tax_brk[3 * ti + 1], A.tax_brk[3 * ti + 2]);
      rec[2 * idx + 1] = make_float4(A.tax_slope[4 * ti], A.tax_slope[4 * ti + 1],
                                     A.tax_slope[4 * ti + 2], A.tax_slope[4 * ti + 3]);
    } else {
      rec[2 * idx] = make_float4(w0, -1.f, 0.f, 0.f);
      rec[2 * idx + 1] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
}

hipError_t launch_pack_rec(const PackArgs& A, float4* rec, int total, hipStream_t st) {
  if (total <= 0) return hipSuccess;
  const int blocks = (total + 255) / 256 < 4096 ? (total + 255) / 256 : 4096;
  hipLaunchKernelGGL(pack_rec_kernel, dim3(blocks), dim3(256), 0, st, A, rec, total);
  return hipGetLastError();
}

hipError_t launch_pack_count(const PackArgs& A, hipStream_t st) {
  hipLaunchKernelGGL(pack_count_kernel, dim3(A.m), dim3(256), 0, st, A);
  return hipGetLastError();
}
hipError_t launch_pack_scan(const PackArgs& A, hipStream_t st) {
  hipLaunchKernelGGL(pack_scan_kernel, dim3(1), dim3(256), 0, st, A);
  return hipGetLastError();
}
hipError_t launch_pack_fill(const PackArgs& A, hipStream_t st) {
  hipLaunchKernelGGL(pack_fill_kernel, dim3(A.m), dim3(256), 0, st, A);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the benchmark term of Eq. 1: (gamma/2)(w - w_b)^T Sigma (w - w_b) - eta mu^T w
// = (gamma/2) w^T Sigma w - mu'^T w + (gamma/2) w_b^T Sigma w_b with
// mu' = eta mu + gamma Sigma w_b.  Float64 throughout; mu' is stored in
// float32 for the iterations and in float64 for the polish and the
// certificate, the constant in float64.
// ---------------------------------------------------------------------------
constexpr int kBpRows = 256;     // rows per workgroup of the row passes

// part[a][blk][j] = sum over the block's rows of B_ij w_b,i  (j < k)
__global__ __launch_bounds__(256) void bench_bt_kernel(int n, int k, const float* B,
                                                       const float* wb, double* part) {
  __shared__ double s_w[kBpRows];
  const int a = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
  const int r0 = blk * kBpRows;
  const int i0 = r0 + tid;
  s_w[tid] = (i0 < n && wb) ? (double)wb[(size_t)a * n + i0] : 0.0;
  __syncthreads();
  const int rows = min(kBpRows, n - r0);
  // thread j < k walks the block's rows (consecutive j: consecutive words)
  for (int j = tid; j < k; j += 256) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += (double)B[(size_t)(r0 + r) * k + j] * s_w[r];
    part[((size_t)a * gridDim.x + blk) * k + j] = s;
  }
}

// y = B^T w_b (fixed order over the blocks), then per row
// mu'_i = eta mu_i + gamma (b_i . (f * y) + d_i w_b,i) and the block's part
// of w_b^T (gamma Sigma w_b)
__global__ __launch_bounds__(256) void bench_mu_kernel(int n, int k, int nblk, const float* B,
                                                       const float* f, const float* d,
                                                       const float* mu, const float* wb,
                                                       const float* eta, const float* gamma,
                                                       const double* part, double* ywb,
                                                       float* mu_out, double* mu64_out,
                                                       double* cpart) {
  __shared__ double s_fy[kMaxK];
  __shared__ double s_red[4];
  const int a = blockIdx.y, blk = blockIdx.x, tid = threadIdx.x;
  const double gam = gamma[a];
  const double et = eta ? (double)eta[a] : 1.0;
  for (int j = tid; j < k; j += 256) {
    double y = 0.0;
    if (wb)
      for (int b = 0; b < nblk; ++b) y += part[((size_t)a * nblk + b) * k + j];
    s_fy[j] = (double)f[j] * y;
    if (blk == 0 && wb) ywb[(size_t)a * k + j] = y;
  }
  __syncthreads();
  const int i = blk * kBpRows + tid;
  double c = 0.0;
  if (i < n) {
    const size_t off = (size_t)a * n + i;
    double sw = 0.0;
    if (wb) {
      for (int j = 0; j < k; ++j) sw += (double)B[(size_t)i * k + j] * s_fy[j];
      sw += (double)d[i] * (double)wb[off];
    }
    const double mu_eff = et * (double)mu[off] + gam * sw;
    mu_out[off] = (float)mu_eff;
    mu64_out[off] = mu_eff;
    if (wb) c = 0.5 * gam * (double)wb[off] * sw;
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((tid & 63) == 0) s_red[tid >> 6] = c;
  __syncthreads();
  if (tid == 0) cpart[(size_t)a * nblk + blk] = s_red[0] + s_red[1] + s_red[2] + s_red[3];
}

__global__ void bench_const_kernel(int m, int nblk, const double* cpart, double* obj_const) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= m) return;
  double c = 0.0;
  for (int b = 0; b < nblk; ++b) c += cpart[(size_t)a * nblk + b];
  obj_const[a] = c;
}

int benchmark_row_blocks(int n) { return (n + kBpRows - 1) / kBpRows; }

// part: [m][nblk][k] + [m][nblk] doubles of scratch
hipError_t launch_benchmark_prep(int m, int n, int k, const float* B, const float* f,
                                 const float* d, const float* mu, const float* wb,
                                 const float* eta, const float* gamma, double* ywb,
                                 double* part, float* mu_out, double* mu64_out,
                                 double* obj_const, hipStream_t st) {
  const int nblk = benchmark_row_blocks(n);
  double* cpart = part + (size_t)m * nblk * k;
  if (wb) {
    hipLaunchKernelGGL(bench_bt_kernel, dim3(nblk, m), dim3(256), 0, st, n, k, B, wb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(bench_mu_kernel, dim3(nblk, m), dim3(256), 0, st, n, k, nblk, B, f, d, mu,
                     wb, eta, gamma, part, ywb, mu_out, mu64_out, cpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bench_const_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, nblk, cpart,
                     obj_const);
  return hipGetLastError();
}

__global__ void concat_rows_kernel(int m, int G, int H, const float* blo, const float* bhi,
                                   const float* hlo, const float* hhi, float* lo, float* hi) {
  const int R = G + H;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)m * R) return;
  const int a = (int)(e / R), g = (int)(e % R);
  if (g < G) {
    lo[e] = blo[(size_t)a * G + g];
    hi[e] = bhi[(size_t)a * G + g];
  } else {
    lo[e] = hlo[(size_t)a * H + g - G];
    hi[e] = hhi[(size_t)a * H + g - G];
  }
}

hipError_t launch_concat_rows(int m, int G, int H, const float* blo, const float* bhi,
                              const float* hlo, const float* hhi, float* lo, float* hi,
                              hipStream_t st) {
  const size_t total = (size_t)m * (G + H);
  hipLaunchKernelGGL(concat_rows_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st,
                     m, G, H, blo, bhi, hlo, hhi, lo, hi);
  return hipGetLastError();
}

}  // namespace fqp
