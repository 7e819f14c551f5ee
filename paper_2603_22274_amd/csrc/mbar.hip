// MBAR (Shirts & Chodera 2008), named in section "Simulation protocol" as the
// estimator of each segment's free energy.  FP64 self-consistent iteration in
// log-sum-exp form on u[K][N]:
//   logden_n = LSE_k (ln N_k + f_k - u_kn)
//   f_i <- f_i - ln sum_n exp(f_i - u_in - logden_n)     (terms <= 1/N_i)
// then the gauge f_0 = 0; converged when max|df| <= tol max(1, max|f|).
// Each iteration: one pass computing logden (thread per sample), one pass of
// fixed-order partial sums per (state, chunk), one single-block update; the
// result is independent of launch timing.  After convergence the kernels do
// nothing, so iterations can be queued in batches between host checks.
#include "felis_internal.h"

namespace felis {
namespace {

constexpr int kChunk = 4096;

struct MbarWork {
  double* logden;   // [N]
  double* part;     // [K][nch]
  double* f;        // [K]
  double* logN;     // [K] (-inf for N_k = 0)
  int* state;       // [0] done, [1] iterations
};

__global__ __launch_bounds__(256) void k_logden(const double* __restrict__ u, MbarWork w, int K, long long N,
                                                int max_iter) {
  if (w.state[0] || w.state[1] >= max_iter) return;
  __shared__ double s_b[512];
  for (int k = threadIdx.x; k < K; k += blockDim.x) s_b[k] = w.logN[k] + w.f[k];
  __syncthreads();
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  double m = -INFINITY;
  for (int k = 0; k < K; ++k) m = fmax(m, s_b[k] - u[(long long)k * N + n]);
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += exp(s_b[k] - u[(long long)k * N + n] - m);
  w.logden[n] = m + log(s);
}

// block (i, chunk): sum_n exp(f_i - u_in - logden_n) over the chunk
__global__ __launch_bounds__(256) void k_partial(const double* __restrict__ u, MbarWork w, int K, long long N,
                                                 int nch, int max_iter) {
  if (w.state[0] || w.state[1] >= max_iter) return;
  const int i = blockIdx.x / nch, c = blockIdx.x - (blockIdx.x / nch) * nch;
  const double fi = w.f[i];
  const long long n0 = (long long)c * kChunk, n1 = min(N, n0 + kChunk);
  double s = 0.0;
  for (long long n = n0 + threadIdx.x; n < n1; n += blockDim.x)
    s += exp(fi - u[(long long)i * N + n] - w.logden[n]);
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) w.part[(long long)i * nch + c] = red[0];
}

__global__ __launch_bounds__(256) void k_update(MbarWork w, int K, int nch, double tol, int max_iter) {
  if (w.state[0] || w.state[1] >= max_iter) return;
  __shared__ double fn[512];
  for (int i = threadIdx.x; i < K; i += blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += w.part[(long long)i * nch + c];
    fn[i] = w.f[i] - log(s);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double g0 = fn[0];
    double delta = 0.0, fmaxv = 0.0;
    for (int i = 0; i < K; ++i) {
      const double v = fn[i] - g0;
      delta = fmax(delta, fabs(v - w.f[i]));
      fmaxv = fmax(fmaxv, fabs(v));
      w.f[i] = v;
    }
    w.state[1] += 1;
    if (delta <= tol * fmax(1.0, fmaxv)) w.state[0] = 1;
  }
}

__global__ void k_init(MbarWork w, const double* logN, int K) {
  const int i = threadIdx.x;
  if (i < K) { w.f[i] = 0.0; w.logN[i] = logN[i]; }
  if (i == 0) { w.state[0] = 0; w.state[1] = 0; }
}

MbarWork carve(void* work, int K, long long N, int nch) {
  char* p = (char*)work;
  MbarWork w;
  w.logden = (double*)p; p += ((N * 8 + 255) / 256) * 256;
  w.part = (double*)p; p += (((long long)K * nch * 8 + 255) / 256) * 256;
  w.f = (double*)p; p += 4096;
  w.logN = (double*)p; p += 4096;
  w.state = (int*)p;
  return w;
}

}  // namespace

size_t mbar_work_bytes(int K, long long N) {
  const int nch = (int)((N + kChunk - 1) / kChunk);
  return ((N * 8 + 255) / 256) * 256 + (((long long)K * nch * 8 + 255) / 256) * 256 + 4096 * 2 + 256;
}

int launch_mbar(hipStream_t s, const double* u, const int* N_k, int K, long long N, double tol, int max_iter,
                double* f_out, int* iters, void* work, size_t work_bytes) {
  if (K < 2 || K > 512 || N < 1 || !u || !N_k || !f_out || !work) return FELIS_E_INVAL;
  if (work_bytes < mbar_work_bytes(K, N)) return FELIS_E_INVAL;
  long long tot = 0;
  for (int k = 0; k < K; ++k) {
    if (N_k[k] < 0) return FELIS_E_INVAL;
    tot += N_k[k];
  }
  if (tot != N) return FELIS_E_INVAL;
  const int nch = (int)((N + kChunk - 1) / kChunk);
  MbarWork w = carve(work, K, N, nch);
  // ln N_k is staged through the partial-sum buffer before k_init copies it
  double logN[512];
  for (int k = 0; k < K; ++k) logN[k] = N_k[k] > 0 ? log((double)N_k[k]) : -INFINITY;
  if (hipMemcpyAsync(w.part, logN, sizeof(double) * K, hipMemcpyHostToDevice, s) != hipSuccess) return FELIS_E_DEVICE;
  hipLaunchKernelGGL(k_init, dim3(1), dim3(512), 0, s, w, (const double*)w.part, K);
  if (hipStreamSynchronize(s) != hipSuccess) return FELIS_E_DEVICE;
  const int per = 25;
  int state[2] = {0, 0};
  while (true) {
    for (int it = 0; it < per; ++it) {
      hipLaunchKernelGGL(k_logden, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, u, w, K, N, max_iter);
      hipLaunchKernelGGL(k_partial, dim3((unsigned)(K * nch)), dim3(256), 0, s, u, w, K, N, nch, max_iter);
      hipLaunchKernelGGL(k_update, dim3(1), dim3(256), 0, s, w, K, nch, tol, max_iter);
    }
    if (hipMemcpyAsync(state, w.state, sizeof(state), hipMemcpyDeviceToHost, s) != hipSuccess) return FELIS_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) return FELIS_E_DEVICE;
    if (state[0] || state[1] >= max_iter) break;
  }
  if (hipMemcpyAsync(f_out, w.f, sizeof(double) * K, hipMemcpyDeviceToHost, s) != hipSuccess) return FELIS_E_DEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return FELIS_E_DEVICE;
  if (iters) *iters = state[1];
  return state[0] ? FELIS_OK : FELIS_E_NOCONV;
}

}  // namespace felis
