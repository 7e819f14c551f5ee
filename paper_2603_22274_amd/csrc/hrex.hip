// Hamiltonian replica exchange among the windows of one leg (simulation
// details: exchanges among the windows on one GPU every 5 ps).  Replicas keep
// their coordinates, velocities, noise streams and neighbour lists; an
// accepted swap exchanges the states two replicas hold, i.e. their lambda
// rows.  Scheme: neighbouring states, pairs (0,1), (2,3), ... on even attempts
// and (1,2), (3,4), ... on odd ones; the swap of states s and s+1 held by
// replicas i and j changes the total reduced potential by
//   D = u[s][j] + u[s+1][i] - u[s][i] - u[s+1][j]   (FP64, in this order)
// and is taken when D <= 0 or U < exp(-D) (Metropolis).  U: Philox4x32-10 on
// counter (s, 0x48524558, attempt_lo, attempt_hi), key (seed_lo, seed_hi),
// U = ((w0 >> 5) 2^26 + (w1 >> 6)) 2^-53.
#include "felis_internal.h"

namespace felis {
namespace {

constexpr unsigned kTagHrex = 0x48524558u;

__device__ __forceinline__ double hrex_uniform(unsigned long long seed, long long attempt, int s) {
  unsigned c[4] = {(unsigned)s, kTagHrex, (unsigned)((unsigned long long)attempt & 0xffffffffull),
                   (unsigned)((unsigned long long)attempt >> 32)};
  philox(c, (unsigned)(seed & 0xffffffffull), (unsigned)(seed >> 32));
  return ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6)) * 0x1.0p-53;
}

// one workgroup; W <= kMaxHrex replicas, so the disjoint pairs of one sweep
// take one thread each
__global__ __launch_bounds__(kMaxHrex) void k_hrex(const LegDev* legs, const double* __restrict__ u,
                                                   long long ustride, long long attempt, unsigned long long seed,
                                                   int* accepted) {
  const LegDev& g = legs[0];
  const int W = g.W, lane = threadIdx.x;
  __shared__ int s_state[kMaxHrex], s_rep[kMaxHrex];
  if (lane < W) {
    const int st = g.rstate[lane];
    s_state[lane] = st;
    s_rep[st] = lane;
  }
  __syncthreads();
  const int s = (int)(attempt & 1) + 2 * lane;
  bool acc = false;
  if (s + 1 < W) {
    const int i = s_rep[s], j = s_rep[s + 1];
    const double* us = u + (size_t)s * ustride;
    const double* us1 = us + ustride;
    const double d = us[j] + us1[i] - us[i] - us1[j];
    acc = d <= 0.0 || hrex_uniform(seed, attempt, s) < exp(-d);
    if (acc) { s_state[i] = s + 1; s_state[j] = s; }     // pairs of a sweep touch distinct replicas
  }
  const int n_acc = __syncthreads_count(acc);
  if (lane < W) {
    const int st = s_state[lane];
    g.rstate[lane] = st;
    for (int c = 0; c < 4; ++c) g.lam[4 * lane + c] = g.lamS[4 * st + c];
  }
  if (lane == 0 && accepted) *accepted = n_acc;
}

}  // namespace

void launch_hrex(hipStream_t s, const LegDev* d, const LegHost& h, const double* u, long long u_stride,
                 long long attempt, unsigned long long seed, int* accepted) {
  (void)h;
  hipLaunchKernelGGL(k_hrex, dim3(1), dim3(kMaxHrex), 0, s, d, u, u_stride, attempt, seed, accepted);
}

}  // namespace felis
