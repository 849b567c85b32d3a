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
// slopes; increasing breakpoints) and feasible.  Box + budget feasibility is
// n_elig lb <= 1 <= n_elig ub; the least turnover of any feasible portfolio
// is sum_i |w0_i - clip_i(w0_i)| + |1 - sum_i clip_i(w0_i)| (clip to the
// account's box, 0 for excluded names), so a smaller cap is infeasible.
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
  int held = 0, bad = 0, nel = 0;
  double sum_clip = 0.0, dist = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const float mu = A.mu[(size_t)a * n + i];
    const float w0 = A.w0[(size_t)a * n + i];
    if (!isfinite(mu) || !isfinite(w0)) bad = 1;
    if (w0 != 0.f) ++held;
    const bool el = is_elig(A.elig, W, a, i);
    nel += el ? 1 : 0;
    const double l = el ? lb : 0.0, u = el ? ub : 0.0;
    const double c = fmin(fmax((double)w0, l), u);
    sum_clip += c;
    dist += fabs((double)w0 - c);
  }
  held = block_reduce_sum<int>(held, shi);
  bad = block_reduce_sum<int>(bad, shi);
  nel = block_reduce_sum<int>(nel, shi);
  sum_clip = block_reduce_sum<double>(sum_clip, shd);
  dist = block_reduce_sum<double>(dist, shd);

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
      if (!(lo <= hi) || !isfinite(lo) || !isfinite(hi)) bad_band = 1;
    }
  }
  bad_band = block_reduce_sum<int>(bad_band, shi);

  if (threadIdx.x == 0) {
    A.hold_cnt[a] = held;
    const float gam = A.gamma[a], kap = A.kappa[a], tau = A.tau[a];
    int st = FQP_SOLVED;   // tentatively "to be solved"
    if (bad) st = FQP_NUMERICAL_ERROR;
    else if (!(lb <= ub) || !isfinite(lb) || !isfinite(ub) || !(gam > 0.f) || !isfinite(gam) ||
             !(kap >= 0.f) || !isfinite(kap) || !(tau >= 0.f) || bad_tax || bad_band)
      st = FQP_INVALID_INPUT;
    else if ((double)nel * ub < 1.0 - 1e-7 || (double)nel * lb > 1.0 + 1e-7)
      st = FQP_PRIMAL_INFEASIBLE;
    else if (isfinite(tau)) {
      const double tau_min = dist + fabs(1.0 - sum_clip);
      if ((double)tau < tau_min * (1.0 - 1e-7) - 1e-9) st = FQP_PRIMAL_INFEASIBLE;
    }
    A.status[a] = (st == FQP_SOLVED) ? -1 : st;   // -1: valid, not yet solved
  }
}

__global__ void pack_scan_kernel(PackArgs A) {
  // exclusive scan of hold_cnt into hold_ptr (single workgroup)
  __shared__ int carry;
  __shared__ int sh[256];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < A.m; base += 256) {
    const int i = base + threadIdx.x;
    const int v = (i < A.m) ? A.hold_cnt[i] : 0;
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
  if (threadIdx.x == 0) A.hold_ptr[A.m] = carry;
}

__global__ __launch_bounds__(256) void pack_fill_kernel(PackArgs A) {
  __shared__ int sh[256];
  __shared__ int carry;
  const int a = blockIdx.x;
  const int n = A.n, W = A.W;
  const int base_rec = A.hold_ptr[a];
  const int t0 = A.tax_ptr ? A.tax_ptr[a] : 0;
  const int t1 = A.tax_ptr ? A.tax_ptr[a + 1] : 0;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int wb = 0; wb < W; wb += 256) {
    const int wd = wb + threadIdx.x;
    uint32_t bits = 0;
    if (wd < W) {
      for (int b = 0; b < 32; ++b) {
        const int i = 32 * wd + b;
        if (i < n && A.w0[(size_t)a * n + i] != 0.f) bits |= (1u << b);
      }
    }
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
        // binary search of asset i among the account's lot entries
        int lo = t0, hi = t1 - 1, found = -1;
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          const int v = A.tax_asset[mid];
          if (v == i) { found = mid; break; }
          if (v < i) lo = mid + 1; else hi = mid - 1;
        }
        A.hold_tax[idx] = found;
      }
    }
    __syncthreads();
    if (threadIdx.x == 255) carry += sh[255];
    __syncthreads();
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

}  // namespace fqp
