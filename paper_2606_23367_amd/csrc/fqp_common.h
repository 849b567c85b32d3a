// Device-side layout shared by the fqp kernels (gfx950).
//
// Book state lives in HBM as account-major float32 arrays [m][n] (an
// account's row of assets is contiguous), so a wavefront half reading 32
// consecutive assets of one account issues one 128-byte line.  The factor
// block B~ = [B | A^T | 1 | 0-pad] is float32 [n][kp] with kp a multiple of
// 32: B (k columns), one one-hot column per exposure group (bands enter the
// x-update as extra low-rank directions), one column of ones (its
// contraction gives 1^T Delta^-1 r for the budget border), zero padding.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fqp {

constexpr int kTM = 32;        // accounts per workgroup tile (MFMA M)
constexpr int kWaves = 4;      // waves per workgroup
constexpr int kRowsPerChunk = 32 * kWaves;  // rows per chunk (MFMA N x waves)
constexpr int kMaxKp = 192;    // padded factor width limit
constexpr int kMaxK = 128;     // factor limit (polish keeps K_F in LDS)
constexpr int kMaxG = 64;      // exposure groups limit
constexpr int kMaxKpBf = 96;   // widest factor block of the bf16-split passes
                               // (their B~ and p operands stay in registers)

// per-account float parameters, [m][kNPar]
enum AccPar {
  P_GAMMA = 0, P_RHO, P_KAPPA, P_LAM, P_NU, P_LB, P_UB, P_TAU,
  P_ALPHA, P_RHOB, P_CLASS, P_HASTAX, kNPar = 12
};

// ---------------------------------------------------------------------------
// separable proximal step of phi_i + lam|. - w0| + box  (float32)
//
// For a convex piecewise-linear g with kinks c_1 < ... < c_m and slopes
// s_0 < ... < s_m, argmin_z g(z) + (rho/2)(z - v)^2 is
//   min(v - s_0/rho, max(c_1, min(v - s_1/rho, max(c_2, ... max(c_m,
//       v - s_m/rho)))))
// and adding the box [lb, ub] clips the result (1-D convexity).
// ---------------------------------------------------------------------------
struct TaxLots {
  float b1, b2, b3;        // cumulative sale breakpoints
  float s0, s1, s2, s3;    // lot slopes (non-decreasing)
};

__device__ __forceinline__ float prox_plain(float v, float w0, float th,
                                            float lb, float ub) {
  // kink at w0 with slopes -th*rho, +th*rho (th = (kappa+lam)/rho)
  float z = fminf(v + th, fmaxf(w0, v - th));
  return fminf(fmaxf(z, lb), ub);
}

__device__ __forceinline__ float prox_taxed(float v, float w0, float th,
                                            float irho, const TaxLots& t,
                                            float lb, float ub) {
  // kinks w0-b3 < w0-b2 < w0-b1 < w0; slopes (times 1/rho):
  //   -(th + s3/rho), -(th + s2/rho), -(th + s1/rho), -(th + s0/rho), +th
  float acc = v - th;
  acc = fmaxf(w0, acc);
  acc = fminf(v + th + t.s0 * irho, acc);
  acc = fmaxf(w0 - t.b1, acc);
  acc = fminf(v + th + t.s1 * irho, acc);
  acc = fmaxf(w0 - t.b2, acc);
  acc = fminf(v + th + t.s2 * irho, acc);
  acc = fmaxf(w0 - t.b3, acc);
  acc = fminf(v + th + t.s3 * irho, acc);
  return fminf(fmaxf(acc, lb), ub);
}

__device__ __forceinline__ int popc_below(uint32_t word, int bit) {
  return __popc(word & ((1u << bit) - 1u));
}

// Y <- L^-T L^-1 Y for the k x ncol matrix Y (row-major, any memory), L
// lower (k <= 128).  Columns are independent: wave q solves columns q,
// q + nwaves, ... with lane i holding rows i and i + 64, so the substitution
// runs on shuffles without workgroup barriers.  Ends with a barrier.
__device__ inline void chol_solve_cols(const double* L, int k, double* Y, int ncol) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);
  for (int c = wv; c < ncol; c += nw) {
    double y0 = (lane < k) ? Y[lane * ncol + c] : 0.0;
    double y1 = (lane + 64 < k) ? Y[(lane + 64) * ncol + c] : 0.0;
    for (int j = 0; j < k; ++j) {              // L z = y
      const double yj = (j < 64) ? __shfl(y0, j, 64) : __shfl(y1, j - 64, 64);
      const double zj = yj / L[j * k + j];
      if (j < 64) {
        if (lane == j) y0 = zj;
        else if (lane > j && lane < k) y0 -= L[lane * k + j] * zj;
      } else if (lane == j - 64) {
        y1 = zj;
      }
      if (lane + 64 > j && lane + 64 < k) y1 -= L[(lane + 64) * k + j] * zj;
    }
    for (int j = k - 1; j >= 0; --j) {         // L^T x = z
      const double zj = (j < 64) ? __shfl(y0, j, 64) : __shfl(y1, j - 64, 64);
      const double xj = zj / L[j * k + j];
      if (j < 64) {
        if (lane == j) y0 = xj;
        else if (lane < j) y0 -= L[j * k + lane] * xj;
      } else {
        if (lane == j - 64) y1 = xj;
        else if (lane + 64 < j) y1 -= L[j * k + lane + 64] * xj;
        y0 -= L[j * k + lane] * xj;            // every row i < 64 <= j
      }
    }
    if (lane < k) Y[lane * ncol + c] = y0;
    if (lane + 64 < k) Y[(lane + 64) * ncol + c] = y1;
  }
  __syncthreads();
}

}  // namespace fqp
