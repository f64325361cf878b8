// Dense kernels over the n x n iterate and the n x k subspace blocks.
//
// block_partial_f64   Z = W B for symmetric W (the product that dominates the
//                     partial eigensolve of the truncated projection, Section
//                     3.1).  FP64 MFMA tiles; each W element is read once per
//                     pass; the contraction is split over row chunks.
// reduce_gram         sums the chunk partials (+ optional Chebyshev step) and
//                     forms per-slice Gram partials [B^T B, B^T Z, Z^T Z].
// rowwise             V = B S (Ritz vectors), next basis Bn = Z MZ + B MB, and
//                     per-slice partials of V^T V, V^T Vold, u^T V.
// write_w             fused write of W+ = V diag(lambda+) V^T + sum_q gamma_q u_q u_q^T
//                     + D, with D the sparse -alpha C + alpha M*(y) (Algorithm 1
//                     primal-step input, Section 2.3.3 trace resolvent).
#pragma once

#include "common.hpp"

namespace proxsdp {

typedef double d4 __attribute__((ext_vector_type(4)));

// Workgroup: 4 waves x 16 columns; rows [j0, j0 + R) of W.
// MFMA f64 16x16x4 operands (lane l):
//   A[m][kk]  with m = l % 16, kk = l / 16  := B[j + kk][c0 + m]
//   Bop[kk][n] with kk = l / 16, n = l % 16 := W[j + kk][col]
// D[c][i] accumulates sum_j B[j][c] W[j][i] = (W B)[i][c] since W = W^T.
// Result lane l, register v holds D[m = l/16 + 4 v][n = l % 16].
template <int KB, bool PADDED>
__global__ __launch_bounds__(256) void k_block_partial_f64(
    const double* __restrict__ W, int64_t ld, int n, const double* __restrict__ B, int ldk,
    double* __restrict__ part, int rows_per_chunk, int npad) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + wave * 16 + (lane & 15);
  const int chunk = blockIdx.y;
  const int j0 = chunk * rows_per_chunk;
  const int j1 = min(j0 + rows_per_chunk, npad);
  const int lrow = lane >> 4;
  d4 acc[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) acc[kb] = d4{0.0, 0.0, 0.0, 0.0};

  for (int j = j0; j < j1; j += 64) {
    double w[16];
    double a[16][KB];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int row = j + 4 * u + lrow;
      if (PADDED)
        w[u] = W[(int64_t)row * ld + col];
      else
        w[u] = (row < n && col < n) ? W[(int64_t)row * ld + col] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int row = j + 4 * u + lrow;
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) a[u][kb] = B[(int64_t)row * ldk + kb * 16 + (lane & 15)];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        acc[kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][kb], w[u], acc[kb], 0, 0, 0);
    }
  }
  double* out = part + (int64_t)chunk * npad * ldk + (int64_t)col * ldk;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) out[kb * 16 + lrow + 4 * v] = acc[kb][v];
  }
}

// Sums partials into Z, optional Chebyshev step, Gram partials per slice.
//   cheb 0: Z = W B;   1: Z = (W B - c B) / e;   2: Z = 2 (W B - c B) / e - Bprev
__global__ __launch_bounds__(256) void k_reduce_gram(const double* __restrict__ part, int nchunks,
                                                     double* __restrict__ Z,
                                                     const double* __restrict__ B,
                                                     const double* __restrict__ Bprev, int npad,
                                                     int k, double* __restrict__ gram_part,
                                                     int cheb, double cc, double ce, int grams) {
  extern __shared__ double sm[];
  double* sB = sm;
  double* sZ = sm + SLICE * k;
  const int s = blockIdx.x;
  const int64_t base = (int64_t)s * SLICE * k;
  const int cnt = SLICE * k;
  const int64_t cstride = (int64_t)npad * k;
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    const int64_t off = base + t;
    double z = 0.0;
    for (int c = 0; c < nchunks; ++c) z += part[c * cstride + off];
    const double b = B[off];
    if (cheb == 1)
      z = (z - cc * b) / ce;
    else if (cheb == 2)
      z = 2.0 * (z - cc * b) / ce - Bprev[off];
    Z[off] = z;
    sZ[t] = z;
    sB[t] = b;
  }
  if (!grams) return;
  __syncthreads();
  const int kk = k * k;
  double* out = gram_part + (int64_t)s * 3 * kk;
  for (int t = threadIdx.x; t < 3 * kk; t += blockDim.x) {
    const int which = t / kk;
    const int e = t - which * kk;
    const int a = e / k, b = e - a * k;
    const double* X = (which == 2) ? sZ : sB;
    const double* Y = (which == 0) ? sB : sZ;
    double acc = 0.0;
#pragma unroll 8
    for (int i = 0; i < SLICE; ++i) acc += X[i * k + a] * Y[i * k + b];
    out[t] = acc;
  }
}

// Per slice of SLICE rows:
//   Vs = B S[:, :r], ZS = Z S[:, :r]  (Ritz vectors and W times them)
//   residual partials ||ZS_c - theta_c Vs_c||^2 over the slice -> fac_part[FAC_RES + c]
//   V = Vs (row stride KMAX)                                  if V
//   Bn = Z MZ + B MB (row stride k)                           if Bn
//   factor partials [V^T V | V^T Vold | u_q^T V]              if V
__global__ __launch_bounds__(256) void k_rowwise(const double* __restrict__ B,
                                                 const double* __restrict__ Z,
                                                 const double* __restrict__ small, int k,
                                                 double* __restrict__ V, int r,
                                                 const double* __restrict__ Vold, int r_old,
                                                 double* __restrict__ Bn, int n_r1,
                                                 const double* __restrict__ r1_u, int npad,
                                                 double* __restrict__ fac_part) {
  extern __shared__ double sm[];
  double* sB = sm;
  double* sZ = sB + SLICE * k;
  double* sV = sZ + SLICE * k;
  double* sZS = sV + SLICE * r;
  const int s = blockIdx.x;
  const int i0 = s * SLICE;
  const int64_t base = (int64_t)i0 * k;
  for (int t = threadIdx.x; t < SLICE * k; t += blockDim.x) {
    sB[t] = B[base + t];
    sZ[t] = Z[base + t];
  }
  __syncthreads();
  const double* S = small + SL::S;
  const double* MZ = small + SL::MZ;
  const double* MB = small + SL::MB;
  for (int t = threadIdx.x; t < SLICE * r; t += blockDim.x) {
    const int i = t / r, c = t - (t / r) * r;
    double acc = 0.0, accz = 0.0;
    for (int q = 0; q < k; ++q) {
      const double sq = S[q * KMAX + c];
      acc += sB[i * k + q] * sq;
      accz += sZ[i * k + q] * sq;
    }
    sV[t] = acc;
    sZS[t] = accz;
    if (V) V[(int64_t)(i0 + i) * KMAX + c] = acc;
  }
  if (Bn) {
    for (int t = threadIdx.x; t < SLICE * k; t += blockDim.x) {
      const int i = t / k, c = t - (t / k) * k;
      double acc = 0.0;
      for (int q = 0; q < k; ++q)
        acc += sZ[i * k + q] * MZ[q * KMAX + c] + sB[i * k + q] * MB[q * KMAX + c];
      Bn[base + t] = acc;
    }
  }
  __syncthreads();
  double* out = fac_part + (int64_t)s * FAC_STRIDE;
  const double* theta = small + SL::THETA;
  for (int c = threadIdx.x; c < r; c += blockDim.x) {
    const double th = theta[c];
    double acc = 0.0;
    for (int i = 0; i < SLICE; ++i) {
      const double d = sZS[i * r + c] - th * sV[i * r + c];
      acc += d * d;
    }
    out[FAC_RES + c] = acc;
  }
  if (!V) return;
  const int n1 = r * r, n2 = r * r_old, n3 = n_r1 * r;
  for (int t = threadIdx.x; t < n1 + n2 + n3; t += blockDim.x) {
    double acc = 0.0;
    if (t < n1) {
      const int a = t / r, b = t - (t / r) * r;
      for (int i = 0; i < SLICE; ++i) acc += sV[i * r + a] * sV[i * r + b];
    } else if (t < n1 + n2) {
      const int e = t - n1;
      const int a = e / r_old, b = e - (e / r_old) * r_old;
      for (int i = 0; i < SLICE; ++i) acc += sV[i * r + a] * Vold[(int64_t)(i0 + i) * KMAX + b];
    } else {
      const int e = t - n1 - n2;
      const int q = e / r, a = e - (e / r) * r;
      for (int i = 0; i < SLICE; ++i) acc += r1_u[(int64_t)q * npad + i0 + i] * sV[i * r + a];
    }
    out[t] = acc;
  }
}

// Fills rows < n of an npad x ldk block (columns [c0, c1)) with uniform(-1, 1)
// values from a counter-based hash (splitmix64 finaliser) of (seed, row, col);
// rows >= n get 0.  Columns < c0 are copied from `src` when src != null.
__device__ inline double hash_uniform(uint64_t seed, uint64_t row, uint64_t col) {
  uint64_t z = seed * 0x9E3779B97F4A7C15ull + row * 0xBF58476D1CE4E5B9ull + col * 0x94D049BB133111EBull;
  z ^= z >> 30;
  z *= 0xBF58476D1CE4E5B9ull;
  z ^= z >> 27;
  z *= 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

__global__ void k_fill_basis(double* __restrict__ B, int ldk, const double* __restrict__ src,
                             int ld_src, int c0, int n, int npad, uint32_t seed) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= (int64_t)npad * ldk) return;
  const int i = (int)(t / ldk), c = (int)(t - (int64_t)(t / ldk) * ldk);
  double v;
  if (i >= n)
    v = 0.0;
  else if (c < c0 && src)
    v = src[(int64_t)i * ld_src + c];
  else
    v = hash_uniform(seed, i, c);
  B[t] = v;
}

__global__ void k_zero(double* __restrict__ x, int64_t count) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) x[t] = 0.0;
}

// Dense write, one workgroup per 64 x 64 tile (rows a0.., cols b0..):
//   W[a][b] = sum_t lam_t V[a][t] V[b][t] + sum_q gamma_q u_q[a] u_q[b] + D(a, b)
// gamma_q = alpha sigma_q y[row_q].  The tile is assembled in LDS, the sparse
// items of the tile are added, then rows are stored contiguously.
// Workgroups beyond the tile grid run `finalize` (see sparse.hpp).
struct FinArgs {
  const double* fac_part;
  int nslices;
  int r, r_old;
  int lam_new, lam_old;    // offsets in small
  int x2_new, x2_old;      // scalar slots in small
  const double* row_part;
  int nrow_blocks;
  const double* pat_part;
  int npat_blocks;
  IterRecord* ring;
  int ring_slot;
};

__device__ void finalize_iteration(const FinArgs& f, double* small, const DevProblem& dp,
                                   const double* y, const double* y_old, double* red);

__global__ __launch_bounds__(256) void k_write_w(double* __restrict__ W, int64_t ld, int n,
                                                 const double* __restrict__ V, int ldv, int r,
                                                 double* __restrict__ small, int lam_off,
                                                 DevProblem dp, const double* __restrict__ y,
                                                 const double* __restrict__ y_old,
                                                 const double* __restrict__ dval, int sparse,
                                                 int rank1, int has_fin, FinArgs fin,
                                                 int tiles_side) {
  extern __shared__ double sm[];
  const int ntiles = tiles_side * tiles_side;
  if ((int)blockIdx.x >= ntiles) {
    if (has_fin) finalize_iteration(fin, small, dp, y, y_old, sm);
    return;
  }
  const int I = blockIdx.x / tiles_side;
  const int J = blockIdx.x - I * tiles_side;
  const int a0 = I * TILE, b0 = J * TILE;
  const int nq = rank1 ? dp.n_r1 : 0;
  const int rr = r + nq;
  double* sT = sm;                          // 64 x 65
  double* sVa = sT + TILE * (TILE + 1);     // 64 x rr
  double* sVb = sVa + TILE * (rr > 0 ? rr : 1);
  const double* lam = small + lam_off;
  const double alpha = small[SL::SC + S_ALPHA];
  for (int t = threadIdx.x; t < TILE * rr; t += blockDim.x) {
    const int i = t / rr, q = t - (t / rr) * rr;
    double va = 0.0, vb = 0.0;
    if (q < r) {
      if (a0 + i < n) va = V[(int64_t)(a0 + i) * ldv + q];
      if (b0 + i < n) vb = V[(int64_t)(b0 + i) * ldv + q] * lam[q];
    } else {
      const int u = q - r;
      const double gamma = alpha * dp.r1_sigma[u] * y[dp.r1_row[u]];
      va = dp.r1_u[(int64_t)u * dp.npad + a0 + i];
      vb = dp.r1_u[(int64_t)u * dp.npad + b0 + i] * gamma;
    }
    sVa[t] = va;
    sVb[t] = vb;
  }
  __syncthreads();
  const int c = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  for (int q = 0; q < TILE / 4; ++q) {
    const int a = w + 4 * q;
    double acc = 0.0;
    for (int t = 0; t < rr; ++t) acc += sVa[a * rr + t] * sVb[c * rr + t];
    sT[a * (TILE + 1) + c] = acc;
  }
  if (sparse) {
    __syncthreads();
    const int t0 = dp.tile_ptr[blockIdx.x], t1 = dp.tile_ptr[blockIdx.x + 1];
    for (int t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
      const int it = dp.tile_item[t];
      sT[(it >> 8) * (TILE + 1) + (it & 255)] += dval[dp.tile_e[t]];
    }
  }
  __syncthreads();
  for (int q = 0; q < TILE / 4; ++q) {
    const int a = w + 4 * q;
    const int ga = a0 + a, gb = b0 + c;
    if (ga < n && gb < n) W[(int64_t)ga * ld + gb] = sT[a * (TILE + 1) + c];
    else if (ga < n + TILE && gb < ld) {
      // padding inside the caller-visible region stays zero for internal buffers
    }
  }
}

// Gershgorin lower bound of a dense symmetric S: per row, S_aa - sum_{b != a} |S_ab|.
// One wave per row; partial minima per workgroup.
__global__ __launch_bounds__(256) void k_gersh_dense(const double* __restrict__ S, int64_t ld,
                                                     int n, double* __restrict__ part) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double best = 1e308;
  for (int a = blockIdx.x * 4 + wave; a < n; a += gridDim.x * 4) {
    double s = 0.0;
    for (int b = lane; b < n; b += 64) s += fabs(S[(int64_t)a * ld + b]);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    const double d = S[(int64_t)a * ld + a];
    const double lo = d - (s - fabs(d));
    best = fmin(best, lo);
  }
  if (lane == 0) red[wave] = best;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

}  // namespace proxsdp
