// MBAR (Shirts & Chodera 2008), named in section "Simulation protocol" as the
// estimator of each segment's free energy.  The free energies f solve
//   f_i = -ln sum_n exp(-u_in) / sum_k N_k exp(f_k - u_kn),
// the stationary point of the convex function
//   F(f) = sum_n logden_n(f) - sum_i N_i f_i,  logden_n = LSE_k(ln N_k + f_k - u_kn),
// with gradient g_i = N_i (sum_n W_in - 1) and Hessian
//   H_ij = delta_ij N_i sum_n W_in - N_i N_j sum_n W_in W_jn,
// W_in = exp(f_i - u_in - logden_n).  Newton steps on the sampled states
// (gauge: the first sampled state is held fixed), with a backtracking line
// search on F while steps are large (a change of F below its rounding level
// counts as no increase), and a self-consistent step
// f_i <- f_i - ln sum_n W_in when the Newton system is singular.  Unsampled
// states follow from the converged denominators.  Converged when the
// self-consistent update at the current iterate (the fixed-point iteration's
// own change, relative to the gauge state) or a full Newton step is within
// tol * max(1, max|f|); final gauge f_0 = 0.
//
// Device work per evaluation (FP64, fixed summation order, so the result is
// independent of launch timing): logden per sample with per-block objective
// partials, the weight matrix W [K][N], per-chunk partial sums of W rows and
// of the 16x16 tiles of W W^T, and a fixed-order reduction over chunks.  The
// K x K Newton system is solved on the host.
#include <cmath>
#include <mutex>
#include <vector>

#include "felis_internal.h"

namespace felis {
namespace {

constexpr int kChunk = 4096;      // samples per partial-sum chunk
constexpr int kTile = 16;         // Hessian tile edge
constexpr int kStage = 64;        // samples staged in LDS per tile step

inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

struct MbarWork {
  double* logden;   // [N]
  double* fpart;    // [ceil(N/256)] block sums of logden
  double* W;        // [K][N]
  double* gpart;    // [nch][K]
  double* hpart;    // [nch][K][K]
  double* G;        // [K] sum_n W_in
  double* H;        // [K][K] sum_n W_in W_jn
  double* f;        // [K]
  double* logN;     // [K] (-inf for N_k = 0)
};

MbarWork carve(void* work, int K, long long N) {
  const long long nch = (N + kChunk - 1) / kChunk, nb = (N + 255) / 256;
  char* p = (char*)work;
  MbarWork w;
  w.logden = (double*)p; p += al256(N * 8);
  w.fpart = (double*)p; p += al256(nb * 8);
  w.W = (double*)p; p += al256((size_t)K * N * 8);
  w.gpart = (double*)p; p += al256((size_t)nch * K * 8);
  w.hpart = (double*)p; p += al256((size_t)nch * K * K * 8);
  w.G = (double*)p; p += al256((size_t)K * 8);
  w.H = (double*)p; p += al256((size_t)K * K * 8);
  w.f = (double*)p; p += al256((size_t)K * 8);
  w.logN = (double*)p; p += al256((size_t)K * 8);
  return w;
}

// thread per sample: logden_n; block sums of logden (objective)
__global__ __launch_bounds__(256) void k_logden(const double* __restrict__ u, MbarWork w, int K, long long N) {
  __shared__ double s_b[512];
  __shared__ double red[256];
  for (int k = threadIdx.x; k < K; k += blockDim.x) s_b[k] = w.logN[k] + w.f[k];
  __syncthreads();
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double ld = 0.0;
  if (n < N) {
    double m = -INFINITY;
    for (int k = 0; k < K; ++k) m = fmax(m, s_b[k] - u[(long long)k * N + n]);
    double s = 0.0;
    for (int k = 0; k < K; ++k) s += exp(s_b[k] - u[(long long)k * N + n] - m);
    ld = m + log(s);
    w.logden[n] = ld;
  }
  red[threadIdx.x] = ld;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) w.fpart[blockIdx.x] = red[0];
}

// thread per (i, n): W_in
__global__ __launch_bounds__(256) void k_weights(const double* __restrict__ u, MbarWork w, int K, long long N) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)K * N) return;
  const int i = (int)(t / N);
  const long long n = t - (long long)i * N;
  w.W[t] = exp(w.f[i] - u[t] - w.logden[n]);
}

// block (chunk, tile i, tile j): partial sums over the chunk of W_in W_jn for a
// 16x16 tile (thread = one (i, j)); tiles on the diagonal also sum W_in
__global__ __launch_bounds__(256) void k_gram(MbarWork w, int K, long long N, int ntile) {
  const int per = ntile * ntile;
  const int c = blockIdx.x / per;
  const int tt = blockIdx.x - c * per;
  const int ti = tt / ntile, tj = tt - ti * ntile;
  const int a = threadIdx.x / kTile, b = threadIdx.x % kTile;
  const int i = ti * kTile + a, j = tj * kTile + b;
  const long long n0 = (long long)c * kChunk, n1 = min(N, n0 + kChunk);
  __shared__ double si[kTile][kStage + 1], sj[kTile][kStage + 1];
  double acc = 0.0, gs = 0.0;
  for (long long s0 = n0; s0 < n1; s0 += kStage) {
    const int len = (int)min((long long)kStage, n1 - s0);
    for (int e = threadIdx.x; e < kTile * kStage; e += blockDim.x) {
      const int r = e / kStage, q = e % kStage;
      const int ri = ti * kTile + r, rj = tj * kTile + r;
      si[r][q] = (q < len && ri < K) ? w.W[(long long)ri * N + s0 + q] : 0.0;
      sj[r][q] = (q < len && rj < K) ? w.W[(long long)rj * N + s0 + q] : 0.0;
    }
    __syncthreads();
    for (int q = 0; q < len; ++q) acc += si[a][q] * sj[b][q];
    if (ti == tj && b == 0)
      for (int q = 0; q < len; ++q) gs += si[a][q];
    __syncthreads();
  }
  if (i < K && j < K) w.hpart[((long long)c * K + i) * K + j] = acc;
  if (ti == tj && b == 0 && i < K) w.gpart[(long long)c * K + i] = gs;
}

// thread per (i, j): fixed-order sum over chunks
__global__ __launch_bounds__(256) void k_reduce(MbarWork w, int K, int nch) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= K * K) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += w.hpart[(long long)c * K * K + t];
  w.H[t] = s;
  if (t < K) {
    double g = 0.0;
    for (int c = 0; c < nch; ++c) g += w.gpart[(long long)c * K + t];
    w.G[t] = g;
  }
}

struct Eval {
  double F;                      // objective
  std::vector<double> G, H;      // sum_n W_in, sum_n W_in W_jn
};

// Upload f, run the device passes, bring back what the host step needs.
int evaluate(hipStream_t s, const double* u, const MbarWork& w, int K, long long N, const std::vector<double>& f,
             const std::vector<double>& Nk, bool full, Eval& ev) {
  const long long nb = (N + 255) / 256;
  const int nch = (int)((N + kChunk - 1) / kChunk);
  const int ntile = (K + kTile - 1) / kTile;
  if (hipMemcpyAsync(w.f, f.data(), sizeof(double) * K, hipMemcpyHostToDevice, s) != hipSuccess) return FELIS_E_DEVICE;
  hipLaunchKernelGGL(k_logden, dim3((unsigned)nb), dim3(256), 0, s, u, w, K, N);
  std::vector<double> fp(nb);
  if (full) {
    hipLaunchKernelGGL(k_weights, dim3((unsigned)(((long long)K * N + 255) / 256)), dim3(256), 0, s, u, w, K, N);
    hipLaunchKernelGGL(k_gram, dim3((unsigned)(nch * ntile * ntile)), dim3(256), 0, s, w, K, N, ntile);
    hipLaunchKernelGGL(k_reduce, dim3((unsigned)((K * K + 255) / 256)), dim3(256), 0, s, w, K, nch);
    ev.G.resize(K);
    ev.H.resize((size_t)K * K);
    if (hipMemcpyAsync(ev.G.data(), w.G, sizeof(double) * K, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(ev.H.data(), w.H, sizeof(double) * K * K, hipMemcpyDeviceToHost, s) != hipSuccess)
      return FELIS_E_DEVICE;
  }
  if (hipMemcpyAsync(fp.data(), w.fpart, sizeof(double) * nb, hipMemcpyDeviceToHost, s) != hipSuccess)
    return FELIS_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return FELIS_E_DEVICE;
  double F = 0.0;
  for (long long b = 0; b < nb; ++b) F += fp[b];
  for (int i = 0; i < K; ++i)
    if (Nk[i] > 0) F -= Nk[i] * f[i];
  ev.F = F;
  return FELIS_OK;
}

// Solve A x = b (m x m, row-major, overwritten) by Gaussian elimination with
// partial pivoting; false if a pivot vanishes or the result is not finite.
bool solve(std::vector<double>& A, std::vector<double>& b, int m) {
  double scale = 0.0;
  for (double v : A) scale = std::fmax(scale, std::fabs(v));
  if (!(scale > 0.0)) return m == 0;
  for (int k = 0; k < m; ++k) {
    int p = k;
    for (int r = k + 1; r < m; ++r)
      if (std::fabs(A[(size_t)r * m + k]) > std::fabs(A[(size_t)p * m + k])) p = r;
    if (!(std::fabs(A[(size_t)p * m + k]) > 1e-14 * scale)) return false;
    if (p != k) {
      for (int c = 0; c < m; ++c) std::swap(A[(size_t)k * m + c], A[(size_t)p * m + c]);
      std::swap(b[k], b[p]);
    }
    for (int r = k + 1; r < m; ++r) {
      const double l = A[(size_t)r * m + k] / A[(size_t)k * m + k];
      if (l == 0.0) continue;
      for (int c = k; c < m; ++c) A[(size_t)r * m + c] -= l * A[(size_t)k * m + c];
      b[r] -= l * b[k];
    }
  }
  for (int k = m - 1; k >= 0; --k) {
    double v = b[k];
    for (int c = k + 1; c < m; ++c) v -= A[(size_t)k * m + c] * b[c];
    b[k] = v / A[(size_t)k * m + k];
    if (!std::isfinite(b[k])) return false;
  }
  return true;
}

}  // namespace

size_t mbar_work_bytes(int K, long long N) {
  const long long nch = (N + kChunk - 1) / kChunk, nb = (N + 255) / 256;
  return al256(N * 8) + al256(nb * 8) + al256((size_t)K * N * 8) + al256((size_t)nch * K * 8) +
         al256((size_t)nch * K * K * 8) + al256((size_t)K * 8) + al256((size_t)K * K * 8) + 2 * al256((size_t)K * 8);
}

int launch_mbar(hipStream_t s, const double* u, const int* N_k, int K, long long N, double tol, int max_iter,
                double* f_out, int* iters, void* work, size_t work_bytes) {
  if (K < 2 || K > 512 || N < 1 || !u || !N_k || !f_out || !work || !(tol > 0) || max_iter < 1)
    return FELIS_E_INVAL;
  if (work_bytes < mbar_work_bytes(K, N)) return FELIS_E_INVAL;
  long long tot = 0;
  for (int k = 0; k < K; ++k) {
    if (N_k[k] < 0) return FELIS_E_INVAL;
    tot += N_k[k];
  }
  if (tot != N) return FELIS_E_INVAL;
  MbarWork w = carve(work, K, N);
  std::vector<double> Nk(K), logN(K);
  std::vector<int> idx;                 // sampled states other than the gauge state
  int ref = -1;
  for (int k = 0; k < K; ++k) {
    Nk[k] = N_k[k];
    logN[k] = N_k[k] > 0 ? std::log((double)N_k[k]) : -INFINITY;
    if (N_k[k] > 0) {
      if (ref < 0) ref = k;
      else idx.push_back(k);
    }
  }
  if (hipMemcpyAsync(w.logN, logN.data(), sizeof(double) * K, hipMemcpyHostToDevice, s) != hipSuccess)
    return FELIS_E_DEVICE;
  const int m = (int)idx.size();
  std::vector<double> f(K, 0.0), step(K), ftry(K);
  Eval ev, trial;
  bool done = false;
  int it = 0;
  while (it < max_iter) {
    int rc = evaluate(s, u, w, K, N, f, Nk, true, ev);
    if (rc) return rc;
    ++it;
    // the self-consistent update at this iterate, -ln(sum_n W_in) relative
    // to the gauge state: the change of f the fixed-point iteration would
    // make, which is the stopping rule's quantity
    double fscale = 1.0;
    for (int k = 0; k < K; ++k) fscale = std::fmax(fscale, std::fabs(f[k]));
    if (ev.G[ref] > 0.0) {
      double sc = 0.0;
      bool finite = true;
      for (int r = 0; r < m; ++r) {
        const double d = std::log(ev.G[idx[r]]) - std::log(ev.G[ref]);
        finite = finite && std::isfinite(d);
        sc = std::fmax(sc, std::fabs(d));
      }
      if (finite && sc <= tol * fscale) { done = true; break; }
    }
    // gradient of F on the free states and the Newton system H d = -g
    std::vector<double> A((size_t)m * m), b(m);
    for (int r = 0; r < m; ++r) {
      const int i = idx[r];
      b[r] = -Nk[i] * (ev.G[i] - 1.0);
      for (int c = 0; c < m; ++c) {
        const int j = idx[c];
        A[(size_t)r * m + c] = (i == j ? Nk[i] * ev.G[i] : 0.0) - Nk[i] * Nk[j] * ev.H[(size_t)i * K + j];
      }
    }
    std::vector<double> g(b);            // -gradient
    std::fill(step.begin(), step.end(), 0.0);
    bool newton = solve(A, b, m);
    double slope = 0.0;                  // g . d (negative for a descent direction)
    if (newton) {
      for (int r = 0; r < m; ++r) { step[idx[r]] = b[r]; slope -= g[r] * b[r]; }
      newton = slope < 0.0 || m == 0;
    }
    if (!newton) {                       // self-consistent step
      std::fill(step.begin(), step.end(), 0.0);
      if (ev.G[ref] > 0.0)
        for (int r = 0; r < m; ++r) step[idx[r]] = -std::log(ev.G[idx[r]]) + std::log(ev.G[ref]);
    }
    double smax = 0.0;
    for (int k = 0; k < K; ++k) {
      if (!std::isfinite(step[k])) return FELIS_E_NOCONV;
      smax = std::fmax(smax, std::fabs(step[k]));
    }
    double t = 1.0;
    if (newton && smax > 1e-3) {         // backtracking on F while the step is large
      // F is a sum over every sample: a change below its rounding level
      // (far from the optimum's curvature along flat directions) is no increase
      double fabs_sum = std::fabs(ev.F);
      for (int k = 0; k < K; ++k) fabs_sum += Nk[k] * std::fabs(f[k]);
      const double f_round = 1e-12 * fabs_sum;
      bool ok = false;
      for (int ls = 0; ls < 30 && !ok; ++ls) {
        for (int k = 0; k < K; ++k) ftry[k] = f[k] + t * step[k];
        rc = evaluate(s, u, w, K, N, ftry, Nk, false, trial);
        if (rc) return rc;
        ok = trial.F <= ev.F + 1e-4 * t * slope + f_round;
        if (!ok) t *= 0.5;
      }
      if (!ok) {                         // no decrease found: self-consistent step instead
        t = 1.0;
        smax = 0.0;
        std::fill(step.begin(), step.end(), 0.0);
        if (ev.G[ref] > 0.0)
          for (int r = 0; r < m; ++r) {
            step[idx[r]] = -std::log(ev.G[idx[r]]) + std::log(ev.G[ref]);
            smax = std::fmax(smax, std::fabs(step[idx[r]]));
          }
      }
    }
    double fmaxv = 0.0;
    for (int k = 0; k < K; ++k) {
      f[k] += t * step[k];
      fmaxv = std::fmax(fmaxv, std::fabs(f[k]));
    }
    // or converged when the full (undamped) step is within the tolerance: a
    // step the line search cut short says nothing about the distance left
    if (t == 1.0 && smax <= tol * std::fmax(1.0, fmaxv)) { done = true; break; }
  }
  // unsampled states from the final denominators, then the gauge f_0 = 0
  int rc = evaluate(s, u, w, K, N, f, Nk, true, ev);
  if (rc) return rc;
  for (int k = 0; k < K; ++k)
    if (Nk[k] == 0) f[k] -= std::log(ev.G[k]);
  const double f0 = f[0];
  for (int k = 0; k < K; ++k) f_out[k] = f[k] - f0;
  if (iters) *iters = it;
  for (int k = 0; k < K; ++k)
    if (!std::isfinite(f_out[k])) return FELIS_E_NOCONV;
  return done ? FELIS_OK : FELIS_E_NOCONV;
}

// ---- allocation-free MBAR
//
// Workspace in a file-scope device array, for callers that cannot allocate
// device memory.  Host code never passes `scratch` itself to a kernel (in
// host code the name is a stand-in, not a device address): its device
// address is looked up once per device with hipGetSymbolAddress at context
// creation and kept in g_scratch[device].  Every region of the workspace is
// written by a kernel before any kernel reads it, so nothing needs clearing
// between calls; calls that overlap on one device share the array and race.

static __device__ __align__(256) unsigned char scratch[kMbarStaticBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};
}  // namespace

int mbar_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return FELIS_E_INVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return FELIS_OK;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return FELIS_E_DEVICE;
  g_scratch[device] = p;
  return FELIS_OK;
}

int launch_mbar_noalloc(int device, hipStream_t s, const double* u, const int* N_k, int K, long long N, double tol,
                        int max_iter, double* f_out, int* iters) {
  if (K < 2 || K > 512 || N < 1) return FELIS_E_INVAL;
  if (mbar_work_bytes(K, N) > kMbarStaticBytes) return FELIS_E_CAPACITY;
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device >= 0 && device < kMaxDevices) p = g_scratch[device];
  }
  if (!p) return FELIS_E_DEVICE;
  return launch_mbar(s, u, N_k, K, N, tol, max_iter, f_out, iters, p, kMbarStaticBytes);
}

}  // namespace felis
