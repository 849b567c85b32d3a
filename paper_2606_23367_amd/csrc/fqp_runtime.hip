// Host runtime of libfqp: handle, workspace, setup, the iteration / polish
// schedule, and the C-ABI declared in include/fqp.h.
//
// Schedule of one fqp_solve_batch call (all on the caller's stream):
//   pack   universe block B~, per-account validation and held-asset records
//   setup  one factor-space Cholesky/inverse per distinct (gamma, rho) class
//   init   z = u = 0, contraction of mu for the first x-step
//   loop   blocks of `check_every` iterations [prox, contract, k-solve,
//          project] (captured
//          once in a hipGraph and replayed), then float64 polish and
//          certification rounds on every active account, then compaction
//          of the active list; the host reads the number still active
//   final  one last polish + diagnostics pass for accounts not certified
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fqp_common.h"
#include "fqp_kernels.h"
#include "../../include/fqp.h"

namespace fqp {
hipError_t launch_polish_check_r(const PolishArgs& A, const fqp_result& R, int final_pass,
                                 hipStream_t st);

// ---------------------------------------------------------------------------
// small bookkeeping kernels
// ---------------------------------------------------------------------------
__global__ void init_accounts_kernel(int m, int G, const int* cls, const float* rho_cls,
                                     const float* gamma, const float* kappa, const float* lb,
                                     const float* ub, const float* tau, const int32_t* tax_ptr,
                                     float alpha, float rho_b, float* par, float* zb, float* vb,
                                     const float* blo, const float* bhi, int* iters,
                                     int32_t* pstate, int npstate, int warm,
                                     const float* wz, const float* wv, const float* wl,
                                     const int32_t* st_in, int32_t* st_out) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= m) return;
  // statuses of the validation pass reach the caller's array only here,
  // after every workspace request of the call has succeeded
  st_out[a] = st_in[a];
  float* p = par + (size_t)a * kNPar;
  const int c = cls[a];
  p[P_GAMMA] = gamma[a];
  p[P_RHO] = rho_cls[c];
  p[P_KAPPA] = kappa[a];
  // a warm start keeps the last cap multiplier and band state when finite
  // (from the caller's state block when given, else from the handle)
  if (wl) p[P_LAM] = wl[a];
  if (!warm || !(isfinite(p[P_LAM]) && p[P_LAM] >= 0.f)) p[P_LAM] = 0.f;
  p[P_NU] = 0.f;
  p[P_LB] = lb[a];
  p[P_UB] = ub[a];
  p[P_TAU] = tau[a];
  p[P_ALPHA] = alpha;
  p[P_RHOB] = rho_b;
  p[P_CLASS] = (float)c;
  p[P_HASTAX] = (tax_ptr && tax_ptr[a + 1] > tax_ptr[a]) ? 1.f : 0.f;
  for (int g = 0; g < G; ++g) {
    const size_t e = (size_t)a * G + g;
    if (wz) { zb[e] = wz[e]; vb[e] = wv[e]; }
    if (warm && isfinite(zb[e]) && isfinite(vb[e])) continue;
    zb[e] = fminf(fmaxf(0.f, blo[e]), bhi[e]);
    vb[e] = 0.f;
  }
  iters[a] = 0;
  for (int q = 0; q < npstate; ++q) pstate[(size_t)a * npstate + q] = 0;
}

// the ADMM state of a finished solve for the caller: v, band state, lam
__global__ void export_state_kernel(int m, int n, int G, const float* v, const float* zb,
                                    const float* vb, const float* par, float* out) {
  const size_t mn = (size_t)m * n;
  const size_t total = mn + 2 * (size_t)m * G + m;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    float x;
    if (e < mn) x = v[e];
    else if (e < mn + (size_t)m * G) x = zb[e - mn];
    else if (e < mn + 2 * (size_t)m * G) x = vb[e - mn - (size_t)m * G];
    else x = par[(e - mn - 2 * (size_t)m * G) * kNPar + P_LAM];
    out[e] = x;
  }
}

// warm start: a non-finite entry of the kept state (an account that failed
// last time) restarts from 0
__global__ void sanitize_state_kernel(size_t count, float* v) {
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (size_t)gridDim.x * blockDim.x)
    if (!isfinite(v[e])) v[e] = 0.f;
}

// active list = accounts whose status is still -1 (valid, not certified)
// (host_count: pinned host memory that also receives the count, or null)
__global__ void compact_kernel(int m, const int32_t* status, int* act, int* m_act,
                               int* host_count) {
  __shared__ int sh[256];
  __shared__ int carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < m; base += 256) {
    const int a = base + threadIdx.x;
    const int v = (a < m && status[a] == -1) ? 1 : 0;
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
      int t = (threadIdx.x >= o) ? sh[threadIdx.x - o] : 0;
      __syncthreads();
      sh[threadIdx.x] += t;
      __syncthreads();
    }
    if (v) act[carry + sh[threadIdx.x] - 1] = a;
    __syncthreads();
    if (threadIdx.x == 255) carry += sh[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *m_act = carry;
    if (host_count) *host_count = carry;
  }
}

// the call's counters for the host, stored into pinned host memory (out:
// certified accounts, account-iterations, polish solves, gated polish
// attempts); one workgroup, so the host needs no copy of status or iters
__global__ __launch_bounds__(256) void solve_stats_kernel(int m, const int32_t* status,
                                                          const int* iters, const int32_t* pcount,
                                                          long long* out) {
  __shared__ long long s_c[4], s_i[4];
  long long c = 0, it = 0;
  for (int a = threadIdx.x; a < m; a += 256) {
    c += status[a] == FQP_SOLVED ? 1 : 0;
    it += iters[a];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    c += __shfl_xor(c, o, 64);
    it += __shfl_xor(it, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_c[threadIdx.x >> 6] = c;
    s_i[threadIdx.x >> 6] = it;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
    out[1] = s_i[0] + s_i[1] + s_i[2] + s_i[3];
    out[2] = pcount[0];
    out[3] = pcount[1];
  }
}

// outputs of accounts that never ran (invalid / infeasible input)
__global__ void finalize_kernel(int m, int n, const int32_t* status, const int* iters_dev,
                                fqp_result R) {
  const int a = blockIdx.x;
  const int st = status[a];
  if (threadIdx.x == 0 && R.iters) R.iters[a] = iters_dev[a];
  if (st == FQP_SOLVED || st == FQP_FEASIBLE_UNCERTIFIED || st == FQP_MAX_ITER ||
      st == FQP_TIME_LIMIT)
    return;
  for (int i = threadIdx.x; i < n; i += blockDim.x) R.w[(size_t)a * n + i] = 0.0;
  if (threadIdx.x == 0) {
    if (R.r_prim) R.r_prim[a] = NAN;
    if (R.r_dual) R.r_dual[a] = NAN;
    if (R.r_comp) R.r_comp[a] = NAN;
    if (R.obj) R.obj[a] = NAN;
    if (R.nu) R.nu[a] = 0.0;
    if (R.lam_cap) R.lam_cap[a] = 0.0;
  }
}

__global__ void mark_time_limit_kernel(int m, int32_t* status) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a < m && status[a] == FQP_MAX_ITER) status[a] = FQP_TIME_LIMIT;
}

}  // namespace fqp

using namespace fqp;

// ---------------------------------------------------------------------------
// statically allocated scratch of fqp_adjoint_batch_noalloc
//
// The adjoint's only workspace is the factor vectors gamma F B^T w and
// gamma F B^T v of every account ([m][2k] float64).  The no-allocation
// entry point takes them from this array instead: every device the library
// runs on holds its own copy until the process ends.  Host code never uses
// the array's name as an address: the device address comes from
// hipGetSymbolAddress, taken once per device in fqp_create with that device
// current.
// ---------------------------------------------------------------------------
static constexpr size_t kNoAllocDoubles = (size_t)1 << 18;   // 2 MiB per device
static __device__ __align__(256) double scratch[kNoAllocDoubles];

static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_ptr;   // indexed by device

// device address of `scratch` on `device`, which must be current
static hipError_t scratch_address(int device, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// everything a captured block of iterations depends on: a later call whose
// key is byte-identical replays the same executable graph
struct GraphKey {
  IterArgs ia;
  KArgs ka;
  unsigned gx, gy, gpx, gpy;
  int m, kp, precision, count, cap_resident;
};

struct fqp_handle {
  int device = 0;
  int n_cu = 0;                   // compute units of the device
  double* scratch = nullptr;      // this device's copy of the static scratch
  hipStream_t stream = nullptr;   // the handle's own stream (capturable)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_t[4] = {nullptr, nullptr, nullptr, nullptr};   // phase timing
  // polish rounds: refining-account counts read back behind the launches
  hipEvent_t ev_r[4] = {nullptr, nullptr, nullptr, nullptr};
  // [8] pinned host memory: [0, 4) round counts, [4, 6) held names, [6]
  // valid accounts at set-up, [7] accounts left after a certification pass;
  // kernels store the counts there themselves (no copy launch)
  int32_t* hcount = nullptr;
  int32_t* hcount_dev = nullptr;  // the same memory, as the device addresses it
  // [4] pinned host memory: certified accounts, account-iterations, polish
  // solves, gated polish attempts of the last call (solve_stats_kernel)
  long long* hstat = nullptr;
  long long* hstat_dev = nullptr;
  hipEvent_t ev_pack = nullptr;   // set-up counts (held names, valid accounts) are in hcount
  // pinned host staging of the class tables: gamma [m], then the rho of
  // each class [m at most] and the class of each account [m]; grown on demand
  float* hstage = nullptr;
  size_t hstage_n = 0;            // accounts it holds
  std::string err;
  fqp_stats stats{};
  std::map<std::string, DevBuf> bufs;
  size_t total_bytes = 0;
  bool configured = false;
  // debug hook of the current call: the workspace request with this number
  // (1-based) fails as a device allocation failure would
  int fail_at = 0, requests = 0;
  // context of the last successful solve, for fqp_adjoint_batch
  bool have_last = false;
  // shape of the last completed solve, whose ADMM state a warm start reuses
  bool warm_ok = false;
  int warm_m = 0, warm_n = 0, warm_G = 0;
  // certification passes of the last solve: iterations before, end time
  std::vector<int32_t> pass_iter;
  std::vector<double> pass_ms;
  AdjArgs last{};
  // executable graph of one block of iterations, kept across calls
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  GraphKey gkey;
  bool have_graph = false;

  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    have_graph = false;
  }

  template <typename T>
  T* get(const char* name, size_t count, fqp_error* e) {
    ++requests;
    if (fail_at > 0 && requests == fail_at) {
      *e = FQP_ERR_ALLOC;
      err = std::string("workspace allocation failed (debug_fail_alloc): ") + name;
      return nullptr;
    }
    DevBuf& b = bufs[name];
    const size_t need = count * sizeof(T) + 256;
    if (b.bytes < need) {
      // a captured graph may point into the buffer being replaced
      drop_graph();
      if (b.p) { (void)hipFree(b.p); total_bytes -= b.bytes; }
      b.p = nullptr;
      b.bytes = 0;
      if (hipMalloc(&b.p, need) != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        *e = FQP_ERR_ALLOC;
        err = std::string("workspace allocation failed: ") + name;
        return nullptr;
      }
      b.bytes = need;
      total_bytes += need;
    }
    return static_cast<T*>(b.p);
  }
};

extern "C" {

void fqp_default_settings(fqp_settings* s) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->eps_prim = 1e-6;
  s->eps_dual = 1e-6;
  s->eps_comp = 1e-6;
  s->max_iter = 4000;
  s->check_every = 50;
  s->rho = 0.f;
  s->rho_band = 0.f;
  s->alpha = 1.6f;
  s->polish_rounds = 16;
  s->use_graph = 1;
  s->profile = 0;
  s->time_limit_ms = 0.0;
  s->precision = FQP_PREC_BF16X3;
  s->first_check = 0;
  s->warm_start = 0;
  s->debug_fail_alloc = 0;
  s->tile_rows = 0;
}

const char* fqp_error_string(int e) {
  switch (e) {
    case FQP_OK: return "ok";
    case FQP_ERR_INVALID_ARG: return "invalid argument";
    case FQP_ERR_ALLOC: return "device allocation failed";
    case FQP_ERR_HIP: return "HIP runtime error";
    case FQP_ERR_UNSUPPORTED: return "unsupported problem size";
    default: return "unknown error";
  }
}

const char* fqp_status_string(int s) {
  switch (s) {
    case FQP_SOLVED: return "certified";
    case FQP_FEASIBLE_UNCERTIFIED: return "feasible / non-certified";
    case FQP_MAX_ITER: return "iteration cap, no accepted feasible return";
    case FQP_TIME_LIMIT: return "timeout";
    case FQP_PRIMAL_INFEASIBLE: return "primal infeasible";
    case FQP_INVALID_INPUT: return "invalid input";
    case FQP_NUMERICAL_ERROR: return "allocation / numerical failure";
    default: return "unknown status";
  }
}

const char* fqp_last_error(const fqp_handle* h) { return h ? h->err.c_str() : "null handle"; }

fqp_error fqp_create(fqp_handle** h, int device) {
  if (!h) return FQP_ERR_INVALID_ARG;
  *h = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return FQP_ERR_INVALID_ARG;
  }
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    return FQP_ERR_HIP;
  }
  double* scr = nullptr;
  if (scratch_address(device, &scr) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipSetDevice(cur);
    return FQP_ERR_HIP;
  }
  fqp_handle* hh = new fqp_handle();
  hh->device = device;
  hh->scratch = scr;
  if (hipDeviceGetAttribute(&hh->n_cu, hipDeviceAttributeMultiprocessorCount, device) !=
      hipSuccess) {
    (void)hipGetLastError();
    hh->n_cu = 0;
  }
  // default priority, non-blocking with respect to the legacy stream
  bool ok = hipStreamCreateWithFlags(&hh->stream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&hh->ev_in, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&hh->ev_out, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&hh->ev_pack, hipEventDisableTiming) == hipSuccess;
  for (int q = 0; q < 4 && ok; ++q) ok = hipEventCreate(&hh->ev_t[q]) == hipSuccess;
  for (int q = 0; q < 4 && ok; ++q)
    ok = hipEventCreateWithFlags(&hh->ev_r[q], hipEventDisableTiming) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&hh->hcount, 8 * sizeof(int32_t), hipHostMallocDefault) ==
                 hipSuccess;
  ok = ok && hipHostGetDevicePointer((void**)&hh->hcount_dev, hh->hcount, 0) == hipSuccess;
  ok = ok && hipHostMalloc((void**)&hh->hstat, 4 * sizeof(long long), hipHostMallocDefault) ==
                 hipSuccess;
  ok = ok && hipHostGetDevicePointer((void**)&hh->hstat_dev, hh->hstat, 0) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (hh->stream) (void)hipStreamDestroy(hh->stream);
    if (hh->ev_in) (void)hipEventDestroy(hh->ev_in);
    if (hh->ev_out) (void)hipEventDestroy(hh->ev_out);
    if (hh->ev_pack) (void)hipEventDestroy(hh->ev_pack);
    for (int q = 0; q < 4; ++q) {
      if (hh->ev_t[q]) (void)hipEventDestroy(hh->ev_t[q]);
      if (hh->ev_r[q]) (void)hipEventDestroy(hh->ev_r[q]);
    }
    if (hh->hcount) (void)hipHostFree(hh->hcount);
    if (hh->hstat) (void)hipHostFree(hh->hstat);
    delete hh;
    (void)hipSetDevice(cur);
    return FQP_ERR_HIP;
  }
  (void)hipSetDevice(cur);
  *h = hh;
  return FQP_OK;
}

void fqp_destroy(fqp_handle* h) {
  if (!h) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  h->drop_graph();
  for (auto& kv : h->bufs)
    if (kv.second.p) (void)hipFree(kv.second.p);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  if (h->ev_in) (void)hipEventDestroy(h->ev_in);
  if (h->ev_out) (void)hipEventDestroy(h->ev_out);
  if (h->ev_pack) (void)hipEventDestroy(h->ev_pack);
  for (int q = 0; q < 4; ++q) {
    if (h->ev_t[q]) (void)hipEventDestroy(h->ev_t[q]);
    if (h->ev_r[q]) (void)hipEventDestroy(h->ev_r[q]);
  }
  if (h->hcount) (void)hipHostFree(h->hcount);
  if (h->hstat) (void)hipHostFree(h->hstat);
  if (h->hstage) (void)hipHostFree(h->hstage);
  (void)hipSetDevice(cur);
  delete h;
}

fqp_error fqp_get_stats(const fqp_handle* h, fqp_stats* out) {
  if (!h || !out) return FQP_ERR_INVALID_ARG;
  *out = h->stats;
  return FQP_OK;
}

fqp_error fqp_get_pass_times(const fqp_handle* h, int32_t* iter, double* ms, int32_t cap,
                             int32_t* count) {
  if (!h || !count || (cap > 0 && (!iter || !ms))) return FQP_ERR_INVALID_ARG;
  const int np = (int)h->pass_iter.size();
  for (int p = 0; p < np && p < cap; ++p) {
    iter[p] = h->pass_iter[p];
    ms[p] = h->pass_ms[p];
  }
  *count = np;
  return FQP_OK;
}

}  // extern "C"

#define HIP_CHECK(x)                                                              \
  do {                                                                            \
    hipError_t _e = (x);                                                          \
    if (_e != hipSuccess) {                                                       \
      h->err = std::string("HIP error at " #x ": ") + hipGetErrorString(_e);       \
      return FQP_ERR_HIP;                                                         \
    }                                                                             \
  } while (0)

#define WS(var, T, name, count)                                                   \
  T* var = h->get<T>(name, (size_t)(count), &e);                                  \
  if (!var) return e;

static float auto_rho(const fqp_settings* S) { return S->rho > 0.f ? S->rho : 5.0f; }

extern "C" fqp_error fqp_solve_batch(fqp_handle* h, const fqp_universe* U, const fqp_book* P,
                                     const fqp_settings* S_in, fqp_result* R, void* stream_v) {
  if (!h) return FQP_ERR_INVALID_ARG;
  h->err.clear();
  h->stats = fqp_stats{};
  h->pass_iter.clear();
  h->pass_ms.clear();
  auto t_start = std::chrono::steady_clock::now();
  auto ms_since_start = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
        .count();
  };
  h->have_last = false;
  if (!U || !P || !R) { h->err = "null universe/book/result"; return FQP_ERR_INVALID_ARG; }
  fqp_settings S;
  if (S_in) S = *S_in; else fqp_default_settings(&S);
  h->fail_at = S.debug_fail_alloc;
  h->requests = 0;
  // constraint rows with two-sided bounds: the Gl one-hot band rows, then
  // the H policy halfspace rows; both join the factor block B~
  const int n = U->n, k = U->k, Gl = U->n_groups, H = U->n_half, m = P->m;
  const int G = Gl + H;
  if (n < 1 || k < 1 || m < 1 || Gl < 0 || H < 0) {
    h->err = "non-positive size";
    return FQP_ERR_INVALID_ARG;
  }
  // a caller's state block, or the state the handle kept from its last
  // solve of the same shape; a solve that fails part-way leaves no state
  const bool warm_kept = S.warm_start && h->warm_ok && h->warm_m == m && h->warm_n == n &&
                         h->warm_G == G;
  const bool warm_given = S.warm_start && P->warm_state != nullptr;
  const bool warm = warm_kept || warm_given;
  h->warm_ok = false;
  if (!U->B || !U->f || !U->d || !P->mu || !P->w0 || !P->lb || !P->ub || !P->gamma ||
      !P->kappa || !P->tau || !R->w || !R->status) {
    h->err = "required pointer is null";
    return FQP_ERR_INVALID_ARG;
  }
  if (Gl > 0 && (!U->group || !P->band_lo || !P->band_hi)) {
    h->err = "n_groups > 0 needs group labels and band bounds";
    return FQP_ERR_INVALID_ARG;
  }
  if (H > 0 && (!U->half || !P->half_lo || !P->half_hi)) {
    h->err = "n_half > 0 needs the halfspace rows and their bounds";
    return FQP_ERR_INVALID_ARG;
  }
  if ((P->lb_asset == nullptr) != (P->ub_asset == nullptr)) {
    h->err = "per-asset bounds need both lb_asset and ub_asset";
    return FQP_ERR_INVALID_ARG;
  }
  if (P->tax_ptr && (!P->tax_asset || !P->tax_brk || !P->tax_slope)) {
    h->err = "tax_ptr given without lot arrays";
    return FQP_ERR_INVALID_ARG;
  }
  if (S.max_iter < 1 || S.check_every < 1 || !(S.alpha > 0.f && S.alpha < 2.f) ||
      S.polish_rounds < 1 || (S.precision != FQP_PREC_FP32 && S.precision != FQP_PREC_BF16X3) ||
      S.tile_rows < 0 || S.debug_fail_alloc < 0) {
    h->err = "invalid settings";
    return FQP_ERR_INVALID_ARG;
  }
  const int kg = k + (G > 0 ? G : 0);
  const int kp = ((kg + 1 + 31) / 32) * 32;
  if ((size_t)m * (size_t)n >= ((size_t)1 << 31)) {
    h->err = "book of 2^31 or more (account, asset) entries: split it into several calls";
    return FQP_ERR_UNSUPPORTED;
  }
  if (k > kMaxK || G > kMaxG || kp > kMaxKp) {
    h->err = "factor count / constraint rows (n_groups + n_half) beyond the library limits";
    return FQP_ERR_UNSUPPORTED;
  }
  {
    const long ncol = G + 3;
    if ((long)k * ncol + ncol * ncol > 48L * 256) {
      h->err = "factors x groups beyond the polish limits";
      return FQP_ERR_UNSUPPORTED;
    }
  }
  hipStream_t caller = static_cast<hipStream_t>(stream_v);
  int prev_dev = 0;
  (void)hipGetDevice(&prev_dev);
  HIP_CHECK(hipSetDevice(h->device));
  struct Restore {
    int d;
    ~Restore() { (void)hipSetDevice(d); }
  } restore{prev_dev};
  // all work runs on the handle's stream, ordered after the caller's prior
  // work; the caller's stream waits for it at the end
  hipStream_t st = h->stream;
  HIP_CHECK(hipEventRecord(h->ev_in, caller));
  HIP_CHECK(hipStreamWaitEvent(st, h->ev_in, 0));
  struct Fence {
    fqp_handle* h;
    hipStream_t caller;
    ~Fence() {
      if (hipEventRecord(h->ev_out, h->stream) == hipSuccess)
        (void)hipStreamWaitEvent(caller, h->ev_out, 0);
    }
  } fence{h, caller};
  fqp_error e = FQP_OK;
  if (!h->configured) {
    HIP_CHECK(configure_iter_kernels());
    h->configured = true;
  }
  const int W = (n + 31) / 32;
  HIP_CHECK(hipEventRecord(h->ev_t[0], st));         // start of the device lane

  // ---- classes: distinct gamma values share one factor-space factorisation
  // (through pinned staging, so that the copies back to the device later
  // on are asynchronous; the previous call's copies out of it are complete
  // once the stream has drained here)
  if (h->hstage_n < (size_t)m) {
    HIP_CHECK(hipStreamSynchronize(st));
    if (h->hstage) (void)hipHostFree(h->hstage);
    h->hstage = nullptr;
    h->hstage_n = 0;
    HIP_CHECK(hipHostMalloc((void**)&h->hstage, 3 * sizeof(float) * (size_t)m,
                            hipHostMallocDefault));
    h->hstage_n = (size_t)m;
  }
  const float* gam_h = h->hstage;
  float* rho_stage = h->hstage + m;
  int* cls_h = reinterpret_cast<int*>(h->hstage + 2 * (size_t)m);
  HIP_CHECK(hipMemcpyAsync(h->hstage, P->gamma, sizeof(float) * m, hipMemcpyDeviceToHost, st));
  HIP_CHECK(hipStreamSynchronize(st));
  std::vector<float> cls_gamma;
  {
    std::map<float, int> seen;
    for (int a = 0; a < m; ++a) {
      float g = gam_h[a];
      if (!(g > 0.f) || !std::isfinite(g)) g = 1.f;   // invalid: flagged by pack
      auto it = seen.find(g);
      if (it == seen.end()) {
        int id = (int)cls_gamma.size();
        seen[g] = id;
        cls_gamma.push_back(g);
        cls_h[a] = id;
      } else {
        cls_h[a] = it->second;
      }
    }
  }
  const int ncls = (int)cls_gamma.size();
  const float rho = auto_rho(&S);
  const float rho_b = S.rho_band > 0.f ? S.rho_band : rho;
  std::vector<float> rho_cls(ncls, rho);

  // ---- workspace ----------------------------------------------------------
  // Every request comes before the first write to the caller's outputs: a
  // failed allocation returns FQP_ERR_ALLOC with the outputs untouched.
  WS(Bt, float, "Bt", (size_t)n * kp);
  const int gram_rows = 32;          // row blocks of the Gram partials: 313 at n = 10,000
  const int nparts = (n + gram_rows - 1) / gram_rows;
  WS(gpart, double, "gram_part", (size_t)nparts * (kg + 1) * (kg + 1));
  const size_t kw_stride = (size_t)(kg + 1) * (kg + 1) + 2 * (size_t)kg * kg + kg + 16;
  WS(Kw, double, "kwork", kw_stride * ncls);
  WS(Kinv, float, "Kinv", (size_t)ncls * kp * kp);
  WS(cvec, float, "cvec", (size_t)ncls * kp);
  WS(qvec, float, "qvec", (size_t)ncls * kp);
  WS(sig1, float, "sig1", (size_t)ncls);
  WS(mbg, float, "mbg", (size_t)ncls * kp * (G > 0 ? G : 1));
  WS(rho_d, float, "rho_cls", (size_t)ncls);
  WS(cls_d, int, "cls", (size_t)m);
  WS(v, float, "v", (size_t)m * n);
  WS(z, float, "z", (size_t)m * n);
  WS(hold, uint32_t, "hold", (size_t)m * W);
  WS(hold_pre, int32_t, "hold_pre", (size_t)m * W);
  WS(hold_cnt, int32_t, "hold_cnt", (size_t)m);
  WS(hold_ptr, int32_t, "hold_ptr", (size_t)m + 2);
  WS(hold_w0, float, "hold_w0", (size_t)m * n);
  WS(hold_tax, int32_t, "hold_tax", (size_t)m * n);
  WS(st_in, int32_t, "status_in", (size_t)m);
  WS(par, float, "par", (size_t)m * kNPar);
  WS(pp, float, "pp", (size_t)m * kp);
  WS(zb, float, "zb", (size_t)m * (G > 0 ? G : 1));
  WS(vb, float, "vb", (size_t)m * (G > 0 ? G : 1));
  WS(iters, int, "iters", (size_t)m);
  WS(act, int, "act", (size_t)m);
  WS(m_act, int, "m_act", 1);
  WS(code, int8_t, "code", (size_t)m * n);
  WS(code_next, int8_t, "code_next", (size_t)m * n);
  WS(flist, int32_t, "flist", (size_t)m * n);
  const size_t wks = polish_wk_stride(k, G);
  WS(wk, double, "polish_wk", (size_t)m * wks);
  WS(mult, double, "mult", (size_t)m * (2 + G));
  WS(gbase, double, "gbase", (size_t)m * n);
  WS(pact, int, "polish_act", (size_t)m);
  WS(pm_act, int, "polish_m_act", 1);
  WS(pstate, int32_t, "pstate", (size_t)m * kPStateStride);
  WS(pcount, int32_t, "pcount", 2);
  const int n_rb = polish_row_blocks(n);
  WS(gpart_p, double, "polish_gpart", (size_t)m * n_rb * 4);
  const int n_sb = polish_pass_blocks(n);
  WS(fseg, int32_t, "polish_fseg", (size_t)m * n);
  WS(rpart, double, "polish_rpart", (size_t)m * n_sb * polish_rpart_stride(k, G));
  WS(spart, double, "polish_spart", (size_t)m * n_sb * 4);
  WS(cpart, double, "polish_cpart", (size_t)m * n_sb * 8);
  // the rest of Eq. 1: bounds of every constraint row [m][G] (bands, then
  // halfspaces); mu' = eta mu + gamma Sigma w_b and the constant of the
  // benchmark term when the book has a benchmark or a return scale
  const bool concat_rows = Gl > 0 && H > 0;
  WS(rlo_ws, float, "row_lo", concat_rows ? (size_t)m * G : 1);
  WS(rhi_ws, float, "row_hi", concat_rows ? (size_t)m * G : 1);
  const float* rlo = concat_rows ? rlo_ws : (Gl ? P->band_lo : (H ? P->half_lo : nullptr));
  const float* rhi = concat_rows ? rhi_ws : (Gl ? P->band_hi : (H ? P->half_hi : nullptr));
  const bool bench = P->wb != nullptr || P->eta != nullptr;
  const int nbb = benchmark_row_blocks(n);
  WS(mu_b, float, "mu_eff", bench ? (size_t)m * n : 1);
  WS(mu_b64, double, "mu_eff64", bench ? (size_t)m * n : 1);
  WS(obj_c, double, "obj_const", bench ? (size_t)m : 1);
  WS(ywb, double, "ywb", P->wb ? (size_t)m * k : 1);
  WS(bpart, double, "bench_part", P->wb ? (size_t)m * nbb * (k + 1) : (size_t)m * nbb);
  const float* mu_use = bench ? mu_b : P->mu;

  // iteration geometry, per pass: (row tiles x account tiles) workgroups, as
  // many as the compute units hold at once (one round: a partial second
  // round of workgroups would double the pass), else ~1024; tile_rows
  // fixes the rows of a workgroup instead (whole 128-row chunks)
  const int acc_tiles = (m + kTM - 1) / kTM;
  auto row_tiles = [&](int mode) {
    int chunks;
    if (S.tile_rows > 0) {
      chunks = S.tile_rows;
    } else {
      const int per_cu = iter_blocks_per_cu(kp, S.precision, mode);
      const int slots = (per_cu > 0 && h->n_cu > 0) ? per_cu * h->n_cu : 1024;
      const int target_rt = std::max(1, slots / acc_tiles);
      chunks = (n + kRowsPerChunk * target_rt - 1) / (kRowsPerChunk * target_rt);
    }
    chunks = std::max(1, std::min(chunks, 64));
    const int rows_per_wg = chunks * kRowsPerChunk;
    return (n + rows_per_wg - 1) / rows_per_wg;            // at the full batch
  };
  const int n_rt = row_tiles(0), n_rt_p = row_tiles(1);
  const int max_rt = (n + kRowsPerChunk - 1) / kRowsPerChunk;   // short active lists
  WS(part, float, "part", (size_t)max_rt * m * kp);
  // R' = r / Delta of every (account, row), rows padded to whole chunks
  const int npad_r = ((n + kRowsPerChunk - 1) / kRowsPerChunk) * kRowsPerChunk;
  WS(rprime, float, "rprime", (size_t)m * npad_r);
  // bf16 hi/lo copies of B~ for the split-precision contractions
  const int npad = ((n + kRowsPerChunk - 1) / kRowsPerChunk) * kRowsPerChunk;
  const bool split = S.precision == FQP_PREC_BF16X3 && kp <= kMaxKpBf;
  const size_t nbf = split ? (size_t)npad * kp : 1;
  WS(bt_hi, uint16_t, "bt_hi", nbf);
  WS(bt_lo, uint16_t, "bt_lo", nbf);
  WS(btt_hi, uint16_t, "btt_hi", nbf);
  WS(btt_lo, uint16_t, "btt_lo", nbf);

  // ---- universe ------------------------------------------------------------
  std::copy(rho_cls.begin(), rho_cls.end(), rho_stage);
  HIP_CHECK(hipMemcpyAsync(rho_d, rho_stage, sizeof(float) * ncls, hipMemcpyHostToDevice, st));
  HIP_CHECK(hipMemcpyAsync(cls_d, cls_h, sizeof(int) * m, hipMemcpyHostToDevice, st));
  HIP_CHECK(launch_build_bt(n, k, Gl, H, kp, U->B, U->group, U->half, Bt, st));
  if (concat_rows)
    HIP_CHECK(launch_concat_rows(m, Gl, H, P->band_lo, P->band_hi, P->half_lo, P->half_hi,
                                 rlo_ws, rhi_ws, st));
  if (bench)
    HIP_CHECK(launch_benchmark_prep(m, n, k, U->B, U->f, U->d, P->mu, P->wb, P->eta, P->gamma,
                                    ywb, bpart, mu_b, mu_b64, obj_c, st));

  // ---- book: validation and held records (workspace only) ----------------
  PackArgs pk{};
  pk.n = n; pk.W = W; pk.m = m; pk.G = G; pk.Gl = Gl;
  pk.lbv = P->lb_asset; pk.ubv = P->ub_asset; pk.eta = P->eta;
  pk.mu = mu_use; pk.w0 = P->w0; pk.lb = P->lb; pk.ub = P->ub; pk.elig = P->eligible;
  pk.gamma = P->gamma; pk.kappa = P->kappa; pk.tau = P->tau;
  pk.blo = rlo; pk.bhi = rhi;
  pk.tax_ptr = P->tax_ptr; pk.tax_asset = P->tax_asset; pk.tax_brk = P->tax_brk;
  pk.tax_slope = P->tax_slope;
  pk.hold = hold; pk.hold_pre = hold_pre; pk.hold_cnt = hold_cnt; pk.hold_ptr = hold_ptr;
  pk.hold_w0 = hold_w0; pk.hold_tax = hold_tax; pk.status = st_in; pk.par = par;
  pk.host_counts = h->hcount_dev + 4;
  HIP_CHECK(launch_pack_count(pk, st));
  HIP_CHECK(launch_pack_scan(pk, st));
  HIP_CHECK(launch_pack_fill(pk, st));
  // the held-asset records are sized by the packed count, the PROX layout
  // by the most held names of any account: both counts come back to pinned
  // memory while the factor-space set-up below runs
  HIP_CHECK(hipEventRecord(h->ev_pack, st));

  // ---- universe: bf16 copies of B~ and the factor-space blocks per class
  if (split) HIP_CHECK(launch_split_bt(n, npad, kp, Bt, bt_hi, bt_lo, btt_hi, btt_lo, st));
  for (int c = 0; c < ncls; ++c) {
    HIP_CHECK(launch_gram(n, kp, kg, nparts, gram_rows, Bt, U->d, cls_gamma[c], rho_cls[c], gpart, st));
    HIP_CHECK(launch_kfactor(k, G, kp, nparts, gpart, U->f, cls_gamma[c], rho_b,
                             Kw + kw_stride * c, Kinv + (size_t)c * kp * kp, cvec + (size_t)c * kp,
                             qvec + (size_t)c * kp, sig1 + c, mbg + (size_t)c * kp * (G > 0 ? G : 1),
                             st));
  }
  HIP_CHECK(hipEventSynchronize(h->ev_pack));
  const int n_held = h->hcount[4], max_held = h->hcount[5];
  const bool cap_resident = cap_resident_fits(n, max_held) && P->lb_asset == nullptr;
  WS(hold_rec, float4, "hold_rec", 2 * (size_t)std::max(n_held, 1));
  HIP_CHECK(launch_pack_rec(pk, hold_rec, n_held, st));
  h->stats.workspace_bytes = h->total_bytes;
  h->stats.workspace_requests = h->requests;

  // ---- first writes to the caller's outputs --------------------------------
  const float* ws_v = warm_given ? P->warm_state : nullptr;
  const float* ws_z = warm_given ? P->warm_state + (size_t)m * n : nullptr;
  const float* ws_vb = warm_given ? ws_z + (size_t)m * G : nullptr;
  const float* ws_l = warm_given ? ws_vb + (size_t)m * G : nullptr;
  hipLaunchKernelGGL(init_accounts_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, G, cls_d,
                     rho_d, P->gamma, P->kappa, P->lb, P->ub, P->tau, P->tax_ptr, S.alpha, rho_b,
                     par, zb, vb, rlo, rhi, iters, pstate, kPStateStride,
                     warm ? 1 : 0, G ? ws_z : nullptr, G ? ws_vb : nullptr, ws_l, st_in,
                     R->status);
  HIP_CHECK(hipGetLastError());
  if (warm) {
    if (warm_given)
      HIP_CHECK(hipMemcpyAsync(v, ws_v, sizeof(float) * (size_t)m * n, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(sanitize_state_kernel, dim3(1024), dim3(256), 0, st, (size_t)m * n, v);
    HIP_CHECK(hipGetLastError());
  } else {
    HIP_CHECK(hipMemsetAsync(v, 0, sizeof(float) * (size_t)m * n, st));
  }
  hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(256), 0, st, m, R->status, act, m_act,
                     h->hcount_dev + 6);
  HIP_CHECK(hipGetLastError());

  IterArgs ia;
  std::memset(&ia, 0, sizeof(ia));       // byte-comparable (graph key)
  ia.n = n; ia.W = W;
  ia.m_total = m; ia.m_act = m_act; ia.act = act; ia.Bt = Bt; ia.d = U->d; ia.mu = mu_use;
  ia.lbv = P->lb_asset; ia.ubv = P->ub_asset;
  ia.v = v; ia.elig = P->eligible; ia.hold = hold; ia.hold_pre = hold_pre;
  ia.hold_ptr = hold_ptr; ia.hold_w0 = hold_w0; ia.hold_tax = hold_tax;
  ia.tax_brk = P->tax_brk; ia.tax_slope = P->tax_slope; ia.pp = pp; ia.par = par;
  ia.par_rw = par;
  ia.part = part; ia.zs = z; ia.rp = rprime;
  ia.npad = npad; ia.bt_hi = bt_hi; ia.bt_lo = bt_lo; ia.btt_hi = btt_hi; ia.btt_lo = btt_lo;
  ia.hold_rec = hold_rec;
  KArgs ka;
  std::memset(&ka, 0, sizeof(ka));
  ka.kp = kp; ka.k = k; ka.G = G; ka.n = n; ka.nblk = n_rt * acc_tiles; ka.m_total = m;
  ka.nblk_p = n_rt_p * acc_tiles;
  ka.ncls = ncls;
  ka.m_act = m_act; ka.act = act;
  ka.part = part; ka.par = par; ka.pp = pp; ka.Kinv = Kinv; ka.cvec = cvec;
  ka.qvec = qvec; ka.sig1 = sig1; ka.mbg = mbg; ka.zb = zb; ka.vb = vb;
  ka.blo = rlo; ka.bhi = rhi;
  ka.iters = iters;
  PolishArgs pa{};
  pa.n = n; pa.k = k; pa.G = G; pa.Gl = Gl; pa.kp = kp; pa.W = W; pa.m_total = m;
  pa.m_act = m_act;
  pa.act = act; pa.Bt = Bt; pa.f = U->f; pa.d = U->d; pa.group = Gl ? U->group : nullptr;
  pa.lbv = P->lb_asset; pa.ubv = P->ub_asset; pa.obj_const = bench ? obj_c : nullptr;
  pa.mu64 = bench ? mu_b64 : nullptr;
  pa.mu = mu_use; pa.z = z; pa.elig = P->eligible; pa.hold = hold; pa.hold_pre = hold_pre;
  pa.hold_ptr = hold_ptr; pa.hold_w0 = hold_w0; pa.hold_tax = hold_tax;
  pa.tax_brk = P->tax_brk; pa.tax_slope = P->tax_slope; pa.par = par; pa.zb = zb; pa.vb = vb;
  pa.blo = rlo; pa.bhi = rhi;
  pa.code = code; pa.code_next = code_next; pa.flist = flist; pa.wk = wk; pa.wk_stride = wks; pa.wout = R->w;
  pa.mult = mult; pa.pstate = pstate; pa.gbase = gbase; pa.pcount = pcount;
  pa.n_rb = n_rb; pa.gpart = gpart_p;
  pa.n_sb = n_sb; pa.fseg = fseg; pa.rpart = rpart; pa.spart = spart; pa.cpart = cpart;
  pa.hold_rec = hold_rec;
  HIP_CHECK(hipMemsetAsync(pcount, 0, 2 * sizeof(int32_t), st));
  pa.eps_prim = S.eps_prim; pa.eps_dual = S.eps_dual; pa.eps_comp = S.eps_comp;
  HIP_CHECK(hipEventRecord(h->ev_t[1], st));         // end of setup

  std::vector<hipEvent_t> evs;
  if (S.profile) {
    evs.resize(6 * S.check_every);      // PROJECT pairs, CONTRACT pairs, PROX pairs
    for (auto& ev : evs) HIP_CHECK(hipEventCreate(&ev));
  }
  struct EvGuard {
    std::vector<hipEvent_t>* v;
    ~EvGuard() { for (auto& ev : *v) (void)hipEventDestroy(ev); }
  } evguard{&evs};
  const dim3 igrid(n_rt, acc_tiles), igrid_p(n_rt_p, acc_tiles);
  // one ADMM iteration: prox (cap multiplier, R', w), contract,
  // factor-space solve, project
  auto launch_iteration = [&](int c) -> hipError_t {
    // profiling: events stamped by the pass kernels' own start and end
    const int cb = 2 * S.check_every, xb = 4 * S.check_every;
    hipError_t e0 = (S.profile & 4) ? launch_prox(ia, m, cap_resident, 0, st, evs[xb + 2 * c],
                                                  evs[xb + 2 * c + 1])
                                    : launch_prox(ia, m, cap_resident, 0, st);
    if (e0 != hipSuccess) return e0;
    e0 = (S.profile & 2) ? launch_iter(ia, kp, 0, S.precision, igrid, st, evs[cb + 2 * c],
                                       evs[cb + 2 * c + 1])
                         : launch_iter(ia, kp, 0, S.precision, igrid, st);
    if (e0 != hipSuccess) return e0;
    e0 = launch_ksolve(ka, m, st);
    if (e0 != hipSuccess) return e0;
    e0 = (S.profile & 1) ? launch_iter(ia, kp, 1, S.precision, igrid_p, st, evs[2 * c],
                                       evs[2 * c + 1])
                         : launch_iter(ia, kp, 1, S.precision, igrid_p, st);
    return e0;
  };

  // ---- iteration blocks -------------------------------------------------------
  // A whole block of check_every iterations is one captured graph, kept by
  // the handle: a later call with the same arguments replays it
  const bool use_graph = S.use_graph && !S.profile;
  GraphKey key;
  std::memset(&key, 0, sizeof(key));
  key.ia = ia; key.ka = ka;
  key.gx = igrid.x; key.gy = igrid.y; key.gpx = igrid_p.x; key.gpy = igrid_p.y;
  key.m = m; key.kp = kp; key.precision = S.precision; key.count = S.check_every;
  key.cap_resident = cap_resident ? 1 : 0;

  // graph_reused reports a call that captured nothing: every block replayed
  // the graph kept from an earlier call
  bool captured = false, replayed = false;
  auto run_block = [&](int count) -> fqp_error {
    if (use_graph && count == S.check_every) {
      if (h->have_graph && std::memcmp(&h->gkey, &key, sizeof(key)) == 0) {
        replayed = true;
      } else {
        captured = true;
        h->drop_graph();
        HIP_CHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int c = 0; c < count; ++c) {
          hipError_t e1 = launch_iteration(c);
          if (e1 != hipSuccess) {
            hipGraph_t tmp = nullptr;
            (void)hipStreamEndCapture(st, &tmp);
            if (tmp) (void)hipGraphDestroy(tmp);
            h->err = "launch failed during graph capture";
            return FQP_ERR_HIP;
          }
        }
        HIP_CHECK(hipStreamEndCapture(st, &h->graph));
        HIP_CHECK(hipGraphInstantiate(&h->gexec, h->graph, nullptr, nullptr, 0));
        h->gkey = key;
        h->have_graph = true;
      }
      HIP_CHECK(hipGraphLaunch(h->gexec, st));
    } else {
      for (int c = 0; c < count; ++c) HIP_CHECK(launch_iteration(c));
      if (S.profile) {
        HIP_CHECK(hipStreamSynchronize(st));
        const int cb = 2 * S.check_every;
        for (int c = 0; c < count; ++c) {
          float ms = 0.f;
          if (S.profile & 1) {
            HIP_CHECK(hipEventElapsedTime(&ms, evs[2 * c], evs[2 * c + 1]));
            h->stats.iter_kernel_ms += ms;
          }
          if (S.profile & 2) {
            HIP_CHECK(hipEventElapsedTime(&ms, evs[cb + 2 * c], evs[cb + 2 * c + 1]));
            h->stats.contract_kernel_ms += ms;
          }
          if (S.profile & 4) {
            const int xb = 4 * S.check_every;
            HIP_CHECK(hipEventElapsedTime(&ms, evs[xb + 2 * c], evs[xb + 2 * c + 1]));
            h->stats.prox_kernel_ms += ms;
          }
        }
      }
    }
    h->stats.iter_launches += count;
    return FQP_OK;
  };

  // device-lane phases: ev_t[1] marks the start of the current stretch of
  // iterations, ev_t[2] its end, ev_t[3] the end of the certification pass
  auto add_elapsed = [&](double& acc, hipEvent_t a0, hipEvent_t a1) -> fqp_error {
    float ms = 0.f;
    HIP_CHECK(hipEventElapsedTime(&ms, a0, a1));
    acc += ms;
    return FQP_OK;
  };
  int done_iters = 0;
  // the number of valid accounts comes back to pinned memory while the
  // first block of iterations runs (its passes skip every workgroup when
  // no account is valid): the host does not wait for the set-up to drain
  HIP_CHECK(hipEventRecord(h->ev_pack, st));
  bool count_known = false;
  int active = 1;
  auto first_count = [&]() -> fqp_error {
    HIP_CHECK(hipEventSynchronize(h->ev_pack));
    count_known = true;
    active = h->hcount[6];
    return add_elapsed(h->stats.phase_ms[0], h->ev_t[0], h->ev_t[1]);
  };
  bool timed_out = false;
  while (active > 0 && done_iters < S.max_iter) {
    const int count = std::min(S.check_every, S.max_iter - done_iters);
    fqp_error be = run_block(count);
    if (be != FQP_OK) return be;
    if (!count_known) {
      if ((e = first_count()) != FQP_OK) return e;
      if (active == 0) break;           // that block ran on an empty list
    }
    done_iters += count;
    // no pass before first_check (blocks stay whole, so graph replays too)
    if (done_iters < S.first_check && done_iters < S.max_iter) continue;
    HIP_CHECK(hipEventRecord(h->ev_t[2], st));
    // polish + certification rounds on z = prox(v; lam*)
    HIP_CHECK(launch_prox(ia, m, cap_resident, 1, st));   // z = prox(v; lam*)
    pa.nf_gate = std::max(4 * k + 64, n / 8 + 4 * k);
    pa.nf_small = 2 * k + 32;
    pa.max_prop = 16;
    for (int r = 0; r < S.polish_rounds; ++r) {
      pa.first_round = (r == 0);
      // later rounds: only the accounts still refining; the list kernel also
      // stores their count to pinned host memory, and the host stops
      // launching rounds once the count of the round before this one (read
      // without stalling the device, which still has this round queued)
      // shows none left
      PolishArgs pr = pa;
      if (r > 0) {
        HIP_CHECK(launch_polish_list(m_act, act, pstate, pact, pm_act, h->hcount_dev + (r & 3),
                                     st));
        pr.act = pact;
        pr.m_act = pm_act;
        HIP_CHECK(hipEventRecord(h->ev_r[r & 3], st));
      }
      HIP_CHECK(launch_polish_solve(pr, st));
      HIP_CHECK(launch_polish_check_r(pr, *R, 0, st));
      h->stats.polish_calls += 1;
      if (r >= 2) {
        HIP_CHECK(hipEventSynchronize(h->ev_r[(r - 1) & 3]));
        if (h->hcount[(r - 1) & 3] == 0) break;
      }
    }
    hipLaunchKernelGGL(compact_kernel, dim3(1), dim3(256), 0, st, m, R->status, act, m_act,
                       h->hcount_dev + 7);
    HIP_CHECK(hipGetLastError());
    HIP_CHECK(hipEventRecord(h->ev_t[3], st));
    HIP_CHECK(hipStreamSynchronize(st));
    active = h->hcount[7];
    if ((e = add_elapsed(h->stats.phase_ms[1], h->ev_t[1], h->ev_t[2])) != FQP_OK) return e;
    if ((e = add_elapsed(h->stats.phase_ms[2], h->ev_t[2], h->ev_t[3])) != FQP_OK) return e;
    std::swap(h->ev_t[1], h->ev_t[3]);             // the next stretch starts here
    h->pass_iter.push_back(done_iters);
    h->pass_ms.push_back(ms_since_start());
    if (S.time_limit_ms > 0.0 && ms_since_start() > S.time_limit_ms) {
      timed_out = true;
      break;
    }
  }
  if (!count_known && (e = first_count()) != FQP_OK) return e;   // no block ran
  if (active > 0) {
    // last pattern from the current iterate, diagnostics, final statuses
    HIP_CHECK(launch_prox(ia, m, cap_resident, 1, st));   // z = prox(v; lam*)
    pa.first_round = 1;
    pa.nf_gate = 0;
    pa.nf_small = 0;
    pa.max_prop = 1 << 30;
    HIP_CHECK(launch_polish_solve(pa, st));
    HIP_CHECK(launch_polish_check_r(pa, *R, 1, st));
    if (timed_out) {
      hipLaunchKernelGGL(mark_time_limit_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m,
                         R->status);
      HIP_CHECK(hipGetLastError());
    }
  }
  hipLaunchKernelGGL(finalize_kernel, dim3(m), dim3(256), 0, st, m, n, R->status, iters, *R);
  HIP_CHECK(hipGetLastError());
  if (R->state) {
    const size_t total = (size_t)m * n + 2 * (size_t)m * G + m;
    const unsigned blocks = (unsigned)std::min<size_t>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(export_state_kernel, dim3(blocks), dim3(256), 0, st, m, n, G, v, zb, vb,
                       par, R->state);
    HIP_CHECK(hipGetLastError());
  }
  HIP_CHECK(hipEventRecord(h->ev_t[2], st));
  // count solved accounts and account-iterations (stored into pinned host
  // memory by one small kernel: no copy of status or iters)
  hipLaunchKernelGGL(solve_stats_kernel, dim3(1), dim3(256), 0, st, m, R->status, iters, pcount,
                     h->hstat_dev);
  HIP_CHECK(hipGetLastError());
  HIP_CHECK(hipStreamSynchronize(st));
  if ((e = add_elapsed(h->stats.phase_ms[3], h->ev_t[1], h->ev_t[2])) != FQP_OK) return e;
  h->stats.n_solved += (int32_t)h->hstat[0];
  h->stats.account_iters += (double)h->hstat[1];
  h->stats.iterations = done_iters;
  h->stats.graph_reused = (replayed && !captured) ? 1 : 0;
  h->stats.polish_solves = (int32_t)h->hstat[2];
  h->stats.polish_gated = (int32_t)h->hstat[3];
  {
    AdjArgs& L = h->last;
    L = AdjArgs{};
    L.n = n; L.k = k; L.G = G; L.Gl = Gl; L.kp = kp; L.m = m;
    L.Bt = Bt; L.f = U->f; L.d = U->d; L.group = Gl ? U->group : nullptr; L.w0in = P->w0;
    L.wb = P->wb; L.eta = P->eta; L.ywb = P->wb ? ywb : nullptr;
    L.par = par; L.status = R->status; L.pstate = pstate; L.flist = flist; L.code = code;
    L.w = R->w; L.wk = wk; L.wk_stride = wks;
    h->have_last = true;
  }
  h->warm_ok = true;
  h->warm_m = m; h->warm_n = n; h->warm_G = G;
  h->stats.total_ms = ms_since_start();
  return FQP_OK;
}

// the adjoint of the last solve; `scr` (a device array of at least m * 2k
// doubles) replaces the workspace request when given
static fqp_error adjoint_common(fqp_handle* h, const double* dL_dw, double* dL_dmu,
                                double* dL_dB, void* stream_v, double* scr) {
  if (!h) return FQP_ERR_INVALID_ARG;
  if (!h->have_last) { h->err = "no solve to differentiate"; return FQP_ERR_INVALID_ARG; }
  if (!dL_dw || !dL_dmu || !dL_dB) { h->err = "null gradient pointer"; return FQP_ERR_INVALID_ARG; }
  int prev_dev = 0;
  (void)hipGetDevice(&prev_dev);
  HIP_CHECK(hipSetDevice(h->device));
  struct Restore {
    int d;
    ~Restore() { (void)hipSetDevice(d); }
  } restore{prev_dev};
  hipStream_t caller = static_cast<hipStream_t>(stream_v);
  hipStream_t st = h->stream;
  fqp_error e = FQP_OK;
  AdjArgs A = h->last;
  if (scr) {
    A.yvw = scr;
  } else {
    WS(yvw, double, "adj_yvw", (size_t)A.m * 2 * A.k);
    A.yvw = yvw;
  }
  HIP_CHECK(hipEventRecord(h->ev_in, caller));
  HIP_CHECK(hipStreamWaitEvent(st, h->ev_in, 0));
  A.dLdw = dL_dw;
  A.dmu = dL_dmu;
  A.dB = dL_dB;
  HIP_CHECK(launch_adjoint(A, st));
  HIP_CHECK(hipEventRecord(h->ev_out, st));
  HIP_CHECK(hipStreamWaitEvent(caller, h->ev_out, 0));
  return FQP_OK;
}

extern "C" fqp_error fqp_adjoint_batch(fqp_handle* h, const double* dL_dw, double* dL_dmu,
                                       double* dL_dB, void* stream_v) {
  return adjoint_common(h, dL_dw, dL_dmu, dL_dB, stream_v, nullptr);
}

extern "C" fqp_error fqp_adjoint_batch_noalloc(fqp_handle* h, const double* dL_dw,
                                               double* dL_dmu, double* dL_dB, void* stream_v) {
  if (!h) return FQP_ERR_INVALID_ARG;
  if (!h->scratch) { h->err = "no static scratch on this device"; return FQP_ERR_HIP; }
  if (h->have_last && (size_t)h->last.m * 2 * (size_t)h->last.k > kNoAllocDoubles) {
    h->err = "fqp_adjoint_batch_noalloc: m * 2k = " +
             std::to_string((size_t)h->last.m * 2 * (size_t)h->last.k) +
             " float64 values exceed the static scratch of " + std::to_string(kNoAllocDoubles) +
             " (use fqp_adjoint_batch)";
    return FQP_ERR_UNSUPPORTED;
  }
  return adjoint_common(h, dL_dw, dL_dmu, dL_dB, stream_v, h->scratch);
}
