// Random-hyperplane rounding of the relaxed solution (Goemans and
// Williamson, cited in the paper's Section 1.1 as the rounding that made
// semidefinite relaxations of max-cut practical): for a Gaussian vector g,
//   x = sign(V diag(sqrt(lambda)) g)  in {-1, +1}^n     (x_i = +1 when the sum is >= 0),
// the vertex signs of a hyperplane through the origin cutting the vectors
// of the factorisation X = (V sqrt(Lambda)) (V sqrt(Lambda))^T.  The value of a
// trial is <C, x x^T> (for the max-cut relaxation C = -L/4 it is minus the
// weight of the cut).  The Gaussian vectors are inputs (the caller draws them).
#pragma once

#include "common.hpp"

namespace proxsdp {

constexpr int ROUND_MAX_TRIALS = 64;
constexpr int ROUND_BLOCKS = 256;

// x[i * trials + t] for i < n, t < trials; one thread per (i, t).
__global__ __launch_bounds__(256) void k_round_signs(const double* __restrict__ V, int r,
                                                     const double* __restrict__ lam,
                                                     const double* __restrict__ g, int trials,
                                                     int n, signed char* __restrict__ x) {
  const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gid >= (int64_t)n * trials) return;
  const int i = (int)(gid / trials), t = (int)(gid - (gid / trials) * trials);
  double s = 0.0;
  for (int q = 0; q < r; ++q) s += V[(int64_t)i * KMAX + q] * sqrt(fmax(lam[q], 0.0)) * g[t * r + q];
  x[gid] = s >= 0.0 ? 1 : -1;
}

// Per-block partials of <C, x_t x_t^T> = sum over the pattern entries e = (a, b),
// a <= b, of w_e C_e x_a x_b (w_e = 2 off the diagonal): lane t of every wave
// accumulates trial t over the wave's entries, then the waves are summed in
// a fixed order.  part: ROUND_BLOCKS x ROUND_MAX_TRIALS.
__global__ __launch_bounds__(256) void k_round_values(DevProblem dp, const signed char* __restrict__ x,
                                                      int trials, double* __restrict__ part) {
  __shared__ double acc_w[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double acc = 0.0;
  if (lane < trials) {
    for (int e = blockIdx.x * 4 + wave; e < dp.n_pat; e += gridDim.x * 4) {
      const double c = dp.pat_c[e];
      if (c == 0.0) continue;
      const int a = dp.pat_a[e], b = dp.pat_b[e];
      const double w = (a == b) ? 1.0 : 2.0;
      acc += w * c * (double)x[(int64_t)a * trials + lane] * (double)x[(int64_t)b * trials + lane];
    }
  }
  acc_w[wave][lane] = acc;
  __syncthreads();
  if (threadIdx.x < 64)
    part[(int64_t)blockIdx.x * ROUND_MAX_TRIALS + threadIdx.x] =
        (acc_w[0][threadIdx.x] + acc_w[1][threadIdx.x]) + (acc_w[2][threadIdx.x] + acc_w[3][threadIdx.x]);
}

// out[t] = sum over the blocks of part[b][t], in block order.
__global__ void k_round_reduce(const double* __restrict__ part, int nblocks, int trials,
                               double* __restrict__ out) {
  const int t = threadIdx.x;
  if (t >= trials) return;
  double s = 0.0;
  for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * ROUND_MAX_TRIALS + t];
  out[t] = s;
}

}  // namespace proxsdp
