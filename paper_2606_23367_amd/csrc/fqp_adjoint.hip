// KKT adjoint of the certified solutions (gfx950, float64).
//
// For a certified account the optimum of the build's Eq. 1 instance solves
// the reduced equality system of its active pattern (fixed coordinates at
// bounds / kinks, free coordinates F inside linear pieces, binding budget /
// bands / cap rows C_F):
//
//   gamma Sigma_FF w_F + C_F^T eta = mu_F - slope_F - gamma Sigma_FX w_X,
//   C_F w_F = h.
//
// Differentiating, for a loss L with gradient c = dL/dw the adjoint solves
//   [gamma Sigma_FF  C_F^T; C_F  0] [v; xi] = [c_F; 0],   v = 0 off F,
// and then  dL/dmu = eta v  and  dL/dB = -sum_a gamma_a (v_a (F B^T e_a)^T +
// e_a (F B^T v_a)^T)  with e = w - w_b (Sigma e changes by dB F B^T e +
// B F dB^T e; the halfspace rows are data of their own).  The constraint
// rows C_F are the budget, the binding band and halfspace rows and the cap.
// The solve reuses the polish's factor-space structure: Kf = diag(f)^-1 +
// B_F^T D_F^-1 B_F in LDS, Schur complement on the constraint rows.
#include "fqp_common.h"
#include "fqp_kernels.h"
#include "../../include/fqp.h"

namespace fqp {

enum PStateA { PA_CAP = 0, PA_NF, PA_NX, PA_NC, PA_DONE, PA_ROUNDS, PA_BACT0, PA_BACT1 };

__device__ __forceinline__ bool band_on(const int* ps, int g) {
  return g < 32 ? ((ps[PA_BACT0] >> g) & 1) : ((ps[PA_BACT1] >> (g - 32)) & 1);
}

// one workgroup per account: v (= dL/dmu) and the factor vectors F B^T w,
// F B^T v used by the dL/dB product
__global__ __launch_bounds__(256) void adjoint_solve_kernel(AdjArgs A) {
  extern __shared__ double smem_d[];
  const int k = A.k, G = A.G, n = A.n;
  double* Kf = smem_d;                      // [k][k]
  double* stg = Kf + k * k;                 // 16 x (k + 4)
  const int a = blockIdx.x;
  const int tid = threadIdx.x;
  double* v = A.dmu + (size_t)a * n;
  if (A.status[a] != FQP_SOLVED) {
    for (int i = tid; i < n; i += 256) v[i] = 0.0;
    for (int j = tid; j < 2 * k; j += 256) A.yvw[(size_t)a * 2 * k + j] = 0.0;
    return;
  }
  const int* ps = A.pstate + (size_t)a * kPStateStride;
  const int nF = ps[PA_NF], nX = ps[PA_NX];
  const int cap_on = ps[PA_CAP];
  const int32_t* flist = A.flist + (size_t)a * n;
  const int8_t* code = A.code + (size_t)a * n;
  const double gam = A.par[(size_t)a * kNPar + P_GAMMA];
  const double* c = A.dLdw + (size_t)a * n;
  const double* w = A.w + (size_t)a * n;
  int nb = 0;
  for (int g = 0; g < G; ++g) nb += band_on(ps, g) ? 1 : 0;
  const int nc = 1 + nb + (cap_on ? 1 : 0);
  const int ncol = nc + 1;
  double* Waug = A.wk + (size_t)a * A.wk_stride;
  double* Y = Waug + (size_t)k * (G + 3);
  double* CV = Y + (size_t)k * (G + 3);
  double* S = CV + (size_t)(G + 3) * (G + 3);
  double* sol = S + (size_t)(G + 3) * (G + 3);
  double* xi = sol + k;

  for (int i = tid; i < n; i += 256) v[i] = 0.0;
  // ---- Kf (lower triangle) -------------------------------------------------
  const int ntri = k * (k + 1) / 2;
  const int SR = 16, SS = k + 4;
  {
    double acc[33];
    int ej[33], el_[33];
#pragma unroll
    for (int q = 0; q < 33; ++q) {
      acc[q] = 0.0;
      const int e = tid + 256 * q;
      int j = (int)((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
      while ((j + 1) * (j + 2) / 2 <= e) ++j;
      while (j * (j + 1) / 2 > e) --j;
      ej[q] = (e < ntri) ? j : 0;
      el_[q] = (e < ntri) ? e - j * (j + 1) / 2 : 0;
    }
    for (int f0 = 0; f0 < nF; f0 += SR) {
      const int rows = min(SR, nF - f0);
      __syncthreads();
      for (int e = tid; e < rows * k; e += 256) {
        const int rr = e / k, j = e % k;
        stg[rr * SS + j] = (double)A.Bt[(size_t)flist[f0 + rr] * A.kp + j];
      }
      for (int rr = tid; rr < rows; rr += 256) stg[rr * SS + k] = 1.0 / (double)A.d[flist[f0 + rr]];
      __syncthreads();
      for (int rr = 0; rr < rows; ++rr) {
        const double* b = stg + rr * SS;
#pragma unroll
        for (int q = 0; q < 33; ++q) acc[q] += b[ej[q]] * b[el_[q]] * b[k];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 33; ++q) {
      const int e = tid + 256 * q;
      if (e < ntri) {
        double val = acc[q];
        if (ej[q] == el_[q]) val += 1.0 / (double)A.f[ej[q]];
        Kf[ej[q] * k + el_[q]] = val;
      }
    }
  }
  // ---- Waug = sum_F b V^T / d, CV = sum_F V V^T / d, V = [C_i, c_i] ------
  {
    const int nW = k * ncol, ne2 = nW + ncol * ncol;
    double acc[48];
#pragma unroll
    for (int q = 0; q < 48; ++q) acc[q] = 0.0;
    double* vst = stg + SR * SS;
    for (int f0 = 0; f0 < nF; f0 += SR) {
      const int rows = min(SR, nF - f0);
      __syncthreads();
      for (int e = tid; e < rows * k; e += 256) {
        const int rr = e / k, j = e % k;
        stg[rr * SS + j] = (double)A.Bt[(size_t)flist[f0 + rr] * A.kp + j];
      }
      if (tid < rows) {
        const int i = flist[f0 + tid];
        double* vv = vst + tid * ncol;
        vv[0] = 1.0;
        int col = 1;
        for (int g = 0; g < G; ++g) {
          if (!band_on(ps, g)) continue;
          vv[col++] = row_coef(A, i, g);
        }
        if (cap_on) {
          // side of w0 of the piece the free coordinate lies in
          const double w0 = A.w0in[(size_t)a * n + i];
          vv[col++] = (w[i] > w0) ? 1.0 : -1.0;
        }
        vv[col] = c[i];
        stg[tid * SS + k] = 1.0 / (double)A.d[i];
      }
      __syncthreads();
      for (int rr = 0; rr < rows; ++rr) {
        const double* b = stg + rr * SS;
        const double* vv = vst + rr * ncol;
#pragma unroll
        for (int q = 0; q < 48; ++q) {
          const int e = tid + 256 * q;
          if (e < nW) acc[q] += b[e / ncol] * vv[e % ncol] * b[k];
          else if (e < ne2) {
            const int r2 = e - nW;
            acc[q] += vv[r2 / ncol] * vv[r2 % ncol] * b[k];
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 48; ++q) {
      const int e = tid + 256 * q;
      if (e < nW) Waug[e] = acc[q];
      else if (e < ne2) CV[e - nW] = acc[q];
    }
  }
  __syncthreads();
  // ---- Cholesky of Kf ------------------------------------------------------
  for (int j = 0; j < k; ++j) {
    if (tid == 0) Kf[j * k + j] = sqrt(fmax(Kf[j * k + j], 1e-300));
    __syncthreads();
    const double djj = Kf[j * k + j];
    for (int i = j + 1 + tid; i < k; i += 256) Kf[i * k + j] /= djj;
    __syncthreads();
    const int mm = k - j - 1;
    for (int e = tid; e < mm * mm; e += 256) {
      const int i = j + 1 + e / mm, l = j + 1 + e % mm;
      if (l <= i) Kf[i * k + l] -= Kf[i * k + j] * Kf[l * k + j];
    }
    __syncthreads();
  }
  for (int e = tid; e < k * ncol; e += 256) Y[e] = Waug[e];
  __syncthreads();
  chol_solve_cols(Kf, k, Y, ncol);
  for (int e = tid; e < nc * ncol; e += 256) {
    const int p = e / ncol, q = e % ncol;
    double s = CV[p * ncol + q];
    for (int j = 0; j < k; ++j) s -= Waug[j * ncol + p] * Y[j * ncol + q];
    S[p * ncol + q] = s / gam;
  }
  __syncthreads();
  if (tid == 0) {
    // S xi = C H^-1 c (h = 0), S PSD: pivoted Cholesky, the components the
    // free rows do not pin are set to 0 (they do not change v)
    double* Sm = CV;
    int perm[kMaxG + 3];
    double dmax = 0.0;
    for (int p = 0; p < nc; ++p) {
      perm[p] = p;
      dmax = fmax(dmax, S[p * ncol + p]);
      for (int q = 0; q < nc; ++q) Sm[p * nc + q] = S[p * ncol + q];
    }
    int rank = 0;
    for (int j = 0; j < nc; ++j) {
      int best = j;
      for (int p = j + 1; p < nc; ++p)
        if (Sm[p * nc + p] > Sm[best * nc + best]) best = p;
      if (!(Sm[best * nc + best] > 1e-12 * dmax)) break;
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
    double x[kMaxG + 3];
    for (int j = 0; j < nc; ++j) x[j] = (j < rank) ? S[perm[j] * ncol + nc] : 0.0;
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
    for (int j = 0; j < nc; ++j) xi[perm[j]] = x[j];
  }
  __syncthreads();
  for (int j = tid; j < k; j += 256) {
    double s = Y[j * ncol + nc];
    for (int p = 0; p < nc; ++p) s -= Y[j * ncol + p] * xi[p];
    sol[j] = s;
  }
  __syncthreads();
  for (int t = tid; t < nF; t += 256) {
    const int i = flist[t];
    double ct = xi[0];
    int col = 1;
    for (int g = 0; g < G; ++g) {
      if (!band_on(ps, g)) continue;
      ct += row_coef(A, i, g) * xi[col];
      ++col;
    }
    if (cap_on) ct += ((w[i] > (double)A.w0in[(size_t)a * n + i]) ? 1.0 : -1.0) * xi[col];
    double bs = 0.0;
    for (int j = 0; j < k; ++j) bs += (double)A.Bt[(size_t)i * A.kp + j] * sol[j];
    v[i] = (c[i] - ct - bs) / (gam * (double)A.d[i]);
  }
  __syncthreads();
  // ---- F B^T w (free + nonzero fixed rows) and F B^T v (free rows) -----------
  for (int j = tid; j < k; j += 256) {
    double sw = 0.0, sv = 0.0;
    for (int t = 0; t < nF; ++t) {
      const int i = flist[t];
      const double b = (double)A.Bt[(size_t)i * A.kp + j];
      sw += b * w[i];
      sv += b * v[i];
    }
    for (int t = 0; t < nX; ++t) {
      const int i = flist[n - 1 - t];
      sw += (double)A.Bt[(size_t)i * A.kp + j] * w[i];
    }
    if (A.wb) sw -= A.ywb[(size_t)a * k + j];                         // e = w - w_b
    A.yvw[(size_t)a * 2 * k + j] = gam * (double)A.f[j] * sw;        // gamma F B^T e
    A.yvw[(size_t)a * 2 * k + k + j] = gam * (double)A.f[j] * sv;    // gamma F B^T v
  }
  (void)code;
}

// dL/dB[i][j] = -sum_a ( v_a,i (gamma F B^T w_a)_j + w_a,i (gamma F B^T v_a)_j )
// grid: row tiles of 64; accounts looped in a fixed order (deterministic)
__global__ __launch_bounds__(256) void adjoint_db_kernel(AdjArgs A) {
  __shared__ double sv[64], sw[64];
  const int k = A.k, n = A.n;
  const int r0 = blockIdx.x * 64;
  const int tid = threadIdx.x;
  // each thread owns entries e = tid + 256 q of the 64 x k tile
  double acc[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) acc[q] = 0.0;
  for (int a = 0; a < A.m; ++a) {
    if (A.status[a] != FQP_SOLVED) continue;
    __syncthreads();
    if (tid < 64) {
      const int i = r0 + tid;
      sv[tid] = (i < n) ? A.dmu[(size_t)a * n + i] : 0.0;
      sw[tid] = (i < n) ? A.w[(size_t)a * n + i] - (A.wb ? (double)A.wb[(size_t)a * n + i] : 0.0)
                        : 0.0;
    }
    __syncthreads();
    const double* y = A.yvw + (size_t)a * 2 * k;
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int e = tid + 256 * q;
      if (e < 64 * k) {
        const int rr = e / k, j = e % k;
        acc[q] += sv[rr] * y[j] + sw[rr] * y[k + j];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const int e = tid + 256 * q;
    if (e < 64 * k) {
      const int rr = e / k, j = e % k;
      if (r0 + rr < n) A.dB[(size_t)(r0 + rr) * k + j] = -acc[q];
    }
  }
}

// dL/dmu = eta dL/dmu' (mu' = eta mu + gamma Sigma w_b), after dL/dB used v
__global__ void adjoint_eta_kernel(AdjArgs A) {
  const size_t total = (size_t)A.m * A.n;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x)
    A.dmu[e] *= (double)A.eta[e / A.n];
}

hipError_t launch_adjoint(const AdjArgs& A, hipStream_t st) {
  const size_t smem = sizeof(double) * ((size_t)A.k * A.k + 16 * (size_t)(A.k + 4) +
                                        16 * (size_t)(kMaxG + 3));
  hipError_t e = hipFuncSetAttribute((const void*)adjoint_solve_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adjoint_solve_kernel, dim3(A.m), dim3(256), smem, st, A);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adjoint_db_kernel, dim3((A.n + 63) / 64), dim3(256), 0, st, A);
  e = hipGetLastError();
  if (e != hipSuccess || !A.eta) return e;
  hipLaunchKernelGGL(adjoint_eta_kernel, dim3(1024), dim3(256), 0, st, A);
  return hipGetLastError();
}

}  // namespace fqp
