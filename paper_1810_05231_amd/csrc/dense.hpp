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

// Workgroup: 4 waves x 16 columns; rows [j0, j0 + R) of W, 64 rows per step.
// The step's 64 x k block of the basis is staged once per workgroup in LDS
// (the four waves share it).  The next step's basis block is loaded into
// registers when the current step's MFMAs start, and each W entry of the next
// step as soon as the products that use the register holding the current one
// are issued (122 VGPRs, no AGPRs: 4 waves per SIMD at k = 64; without the
// waves-per-EU bound the compiler chose 164 VGPRs + 32 AGPRs, 2 waves per
// SIMD).  Measured at n = 5000,
// k = 64: 68.8 us against 79.1 us for per-wave basis loads from L2, and 74.6 us
// when the next step's W entries load all at once into a second set of
// registers (3 waves per SIMD); identical results.
// MFMA f64 16x16x4 operands (lane l):
//   A[m][kk]  with m = l % 16, kk = l / 16  := B[j + kk][c0 + m]
//   Bop[kk][n] with kk = l / 16, n = l % 16 := W[j + kk][col]
// D[c][i] accumulates sum_j B[j][c] W[j][i] = (W B)[i][c] since W = W^T.
// Result lane l, register v holds D[m = l/16 + 4 v][n = l % 16].
template <int KB, bool PADDED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_block_partial_f64(
    const double* __restrict__ W, int64_t ld, int n, const double* __restrict__ B, int ldk,
    double* __restrict__ part, int rows_per_chunk, int npad) {
  constexpr int K = KB * 16;
  // rows one apart sit 32 banks apart: a half-wave's 64-bit reads are conflict-free
  constexpr int LDB = (K % 32 == 16) ? K : K + 16;
  constexpr int NQ = K / 8;   // 16-byte pieces of the 64 x K basis block (ldk == K) per thread
  __shared__ double sB[64 * LDB];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  // XCD-aware order: workgroup L of the launch runs on XCD L % 8, so the
  // (column block, chunk) items are dealt in chunk-major order in contiguous
  // ranges per XCD, and each XCD's L2 holds the basis rows of two chunks, not
  // all of them (a permutation of the work: any dispatch order is correct).
  // n = 5000, k = 64: HBM reads 228.0 -> 209.6 MB per launch (204.5 MB of W),
  // 71.0 -> 70.6 us.
  const int ncols = gridDim.x;
  const int T = ncols * gridDim.y;
  const int L = blockIdx.x + ncols * blockIdx.y;
  const int xcd = L & 7, slot = L >> 3;
  int start = 0;   // items dealt to the XCDs before this one
  for (int q = 0; q < xcd; ++q) start += (T - q + 7) >> 3;
  const int item = start + slot;
  const int chunk = item / ncols;
  const int col = (item - chunk * ncols) * 64 + wave * 16 + (lane & 15);
  const int j0 = chunk * rows_per_chunk;
  const int j1 = min(j0 + rows_per_chunk, npad);
  const int lrow = lane >> 4;
  d4 acc[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) acc[kb] = d4{0.0, 0.0, 0.0, 0.0};
  // entry (row, col) of W, zero outside n x n when W is not padded
  auto w_at = [&](int row) -> double {
    if (PADDED) return W[(int64_t)row * ld + col];
    return (row < n && col < n) ? W[(int64_t)row * ld + col] : 0.0;
  };
  double w[16];
  typedef double dd2 __attribute__((ext_vector_type(2)));
  dd2 bq[NQ];
  if (j0 < j1) {
#pragma unroll
    for (int u = 0; u < 16; ++u) w[u] = w_at(j0 + 4 * u + lrow);
    const dd2* src = reinterpret_cast<const dd2*>(B + (int64_t)j0 * ldk);
#pragma unroll
    for (int x = 0; x < NQ; ++x) bq[x] = src[threadIdx.x + 256 * x];
  }
  for (int j = j0; j < j1; j += 64) {
    __syncthreads();   // every wave is done with the previous block
#pragma unroll
    for (int x = 0; x < NQ; ++x) {
      const int e = 2 * (threadIdx.x + 256 * x);
      const int rr = e / K, cc = e - (e / K) * K;
      *reinterpret_cast<dd2*>(&sB[rr * LDB + cc]) = bq[x];
    }
    __syncthreads();
    const bool more = j + 64 < j1;
    if (more) {
      const dd2* src = reinterpret_cast<const dd2*>(B + (int64_t)(j + 64) * ldk);
#pragma unroll
      for (int x = 0; x < NQ; ++x) bq[x] = src[threadIdx.x + 256 * x];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        acc[kb] = __builtin_amdgcn_mfma_f64_16x16x4f64(sB[(4 * u + lrow) * LDB + kb * 16 + (lane & 15)],
                                                       w[u], acc[kb], 0, 0, 0);
      // w[u] is free once its products are issued: load the next step's entry
      if (more) w[u] = w_at(j + 64 + 4 * u + lrow);
    }
  }
  double* out = part + (int64_t)chunk * npad * ldk + (int64_t)col * ldk;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) out[kb * 16 + lrow + 4 * v] = acc[kb][v];
  }
}

// FP32 form of the pass for W stored in single precision (precision form):
// W and the basis entries are FP32 operands of MFMA f32 16x16x4 (FP32
// accumulation over the rows of one chunk); the chunk partials are written in
// FP64 and summed in FP64 by k_reduce_gram.  Operand layout as in the FP64
// kernel; the FP32 accumulator holds D[4 (l / 16) + v][l % 16].  The 64 x k
// block of the basis for each 64-row step is converted and staged once per
// workgroup in LDS (measured 2.4x faster at k = 64 than per-wave loads).
typedef float f4 __attribute__((ext_vector_type(4)));
template <int KB>
__global__ __launch_bounds__(256) void k_block_partial_f32(
    const float* __restrict__ W, int64_t ld, const float* __restrict__ Bf, int ldk,
    double* __restrict__ part, int rows_per_chunk, int npad) {
  constexpr int K = KB * 16;
  constexpr int LDB = K + 1;
  __shared__ float sB[64 * LDB];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = blockIdx.x * 64 + wave * 16 + (lane & 15);
  const int chunk = blockIdx.y;
  const int j0 = chunk * rows_per_chunk;
  const int j1 = min(j0 + rows_per_chunk, npad);
  const int lrow = lane >> 4;
  f4 acc[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) acc[kb] = f4{0.f, 0.f, 0.f, 0.f};
  for (int j = j0; j < j1; j += 64) {
    float w[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) w[u] = W[(int64_t)(j + 4 * u + lrow) * ld + col];
    // the step's 64 x K basis block (FP32, contiguous): K / 16 float4 per thread
    float4 bq[K / 16];
#pragma unroll
    for (int x = 0; x < K / 16; ++x)
      bq[x] = reinterpret_cast<const float4*>(Bf + (int64_t)j * ldk)[threadIdx.x + 256 * x];
    __syncthreads();
#pragma unroll
    for (int x = 0; x < K / 16; ++x) {
      const int t = 4 * (threadIdx.x + 256 * x);
      const int rr = t / K, cc = t - (t / K) * K;
      sB[rr * LDB + cc] = bq[x].x;
      sB[rr * LDB + cc + 1] = bq[x].y;
      sB[rr * LDB + cc + 2] = bq[x].z;
      sB[rr * LDB + cc + 3] = bq[x].w;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        acc[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(sB[(4 * u + lrow) * LDB + kb * 16 + (lane & 15)],
                                                       w[u], acc[kb], 0, 0, 0);
    }
  }
  double* out = part + (int64_t)chunk * npad * ldk + (int64_t)col * ldk;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) out[kb * 16 + 4 * lrow + v] = (double)acc[kb][v];
  }
}

// Chebyshev step on an exactly applied product Z = W B (precision form, when
// the low-precision pass is not accurate enough for the current target):
//   mode 1: Bn = (Z - c B) / e;   mode 2: Bn = 2 (Z - c B) / e - Bprev
// c, e are read from the device (centre and half-width of the last
// Rayleigh-Ritz step).
__global__ __launch_bounds__(256) void k_cheb_combine(const double* __restrict__ Z,
                                                      const double* __restrict__ B,
                                                      const double* __restrict__ Bprev,
                                                      double* __restrict__ Bn, int64_t count,
                                                      int mode, const double* __restrict__ filt) {
  const double cc = filt[0], ce = filt[1];
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count;
       t += (int64_t)gridDim.x * blockDim.x) {
    const double z = (Z[t] - cc * B[t]) / ce;
    Bn[t] = (mode == 2) ? 2.0 * z - Bprev[t] : z;
  }
}

// Round to nearest even of an FP64 value to bfloat16 (through FP32, itself
// round to nearest even); NaN stays a quiet NaN.
__device__ __forceinline__ unsigned short to_bf16_rne(double x) {
  const float f = (float)x;
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

template <typename T>
__device__ __forceinline__ T store_cast(double x);
template <>
__device__ __forceinline__ double store_cast<double>(double x) { return x; }
template <>
__device__ __forceinline__ float store_cast<float>(double x) { return (float)x; }
template <>
__device__ __forceinline__ unsigned short store_cast<unsigned short>(double x) { return to_bf16_rne(x); }

// BF16 form of the pass (precision form with W stored in bfloat16): MFMA
// f32 16x16x32 bf16 with FP32 accumulation.  D[c][i] = sum_j B[j][c] W[j][i];
// the W operand of lane l is W[i0 + l % 16][j + 8 (l / 16) .. + 7] (a 16-byte
// row load, W being symmetric) and the basis operand the same eight rows of
// column c from a transposed BF16 copy of the step's 64 x k basis block staged
// in LDS.  The accumulator holds D[4 (l / 16) + v][l % 16].
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
template <int KB>
__global__ __launch_bounds__(256) void k_block_partial_bf16(
    const unsigned short* __restrict__ W, int64_t ld, const unsigned short* __restrict__ Bt, int ldk,
    double* __restrict__ part, int rows_per_chunk, int npad) {
  constexpr int K = KB * 16;
  constexpr int LDT = 64 + 8;   // staged row stride (bf16), 16-byte aligned rows
  __shared__ __attribute__((aligned(16))) unsigned short sBt[K * LDT];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int m = lane & 15, q = lane >> 4;
  const int i = blockIdx.x * 64 + wave * 16 + m;
  const int chunk = blockIdx.y;
  const int j0 = chunk * rows_per_chunk;
  const int j1 = min(j0 + rows_per_chunk, npad);
  f4 acc[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) acc[kb] = f4{0.f, 0.f, 0.f, 0.f};
  const unsigned short* wrow = W + (int64_t)i * ld;
  for (int j = j0; j < j1; j += 64) {
    uint4 wv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) wv[h] = *reinterpret_cast<const uint4*>(wrow + j + 32 * h + 8 * q);
    // the step's K x 64 block of the transposed BF16 basis: 8 pieces of 16
    // bytes per basis column, K / 32 pieces per thread
    constexpr int NP = (K * 8 + 255) / 256;
    uint4 bp[NP];
#pragma unroll
    for (int x = 0; x < NP; ++x) {
      const int c = threadIdx.x + 256 * x;
      if (c < K * 8)
        bp[x] = *reinterpret_cast<const uint4*>(Bt + (int64_t)(c >> 3) * npad + j + 8 * (c & 7));
    }
    __syncthreads();
#pragma unroll
    for (int x = 0; x < NP; ++x) {
      const int c = threadIdx.x + 256 * x;
      if (c < K * 8) *reinterpret_cast<uint4*>(&sBt[(c >> 3) * LDT + 8 * (c & 7)]) = bp[x];
    }
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const bf8 bw = __builtin_bit_cast(bf8, wv[h]);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
        const uint4 av = *reinterpret_cast<const uint4*>(&sBt[(kb * 16 + m) * LDT + 32 * h + 8 * q]);
        acc[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, av), bw, acc[kb],
                                                          0, 0, 0);
      }
    }
  }
  double* out = part + (int64_t)chunk * npad * ldk + (int64_t)i * ldk;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int v = 0; v < 4; ++v) out[kb * 16 + 4 * q + v] = (double)acc[kb][v];
  }
}

// Gram partials of one SLICE-row block on MFMA f64 16x16x4:
//   out[0] = X^T X, out[1] = X^T Y, out[2] = Y^T Y  (k x k each, row-major),
// X, Y: SLICE x k in LDS (row stride k).  Output blocks of 16 x 16 are dealt
// to the waves; operands  A[m][kk] = P[i0 + kk][a0 + m], B[kk][n] = Q[i0 + kk][b0 + n].
__device__ inline void gram_blocks_mfma(const double* X, const double* Y, int k, double* out) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int kb = k / 16;
  const int nblk = 3 * kb * kb;
  const int m = lane & 15, kq = lane >> 4;
  for (int blk = wave; blk < nblk; blk += nw) {
    const int which = blk / (kb * kb);
    const int rem = blk - which * kb * kb;
    const int a0 = (rem / kb) * 16, b0 = (rem - (rem / kb) * kb) * 16;
    const double* Pm = (which == 2) ? Y : X;
    const double* Qm = (which == 0) ? X : Y;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
    for (int i0 = 0; i0 < SLICE; i0 += 4) {
      const double a = Pm[(i0 + kq) * k + a0 + m];
      const double b = Qm[(i0 + kq) * k + b0 + m];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    double* o = out + (int64_t)which * k * k;
#pragma unroll
    for (int v = 0; v < 4; ++v) o[(a0 + kq + 4 * v) * k + b0 + m] = acc[v];
  }
}

// Sums partials into Z, optional Chebyshev step, Gram partials per slice.
//   cheb 0: Z = W B;   1: Z = (W B - c B) / e;   2: Z = 2 (W B - c B) / e - Bprev
// Z == nullptr: Z is not stored (Gram partials of a product that already exists).
__global__ __launch_bounds__(1024) void k_reduce_gram(const double* __restrict__ part, int nchunks,
                                                     double* __restrict__ Z,
                                                     const double* __restrict__ B,
                                                     const double* __restrict__ Bprev, int npad,
                                                     int k, double* __restrict__ gram_part,
                                                     int cheb, double cc, double ce, int grams,
                                                     const double* __restrict__ filt) {
  extern __shared__ double sm[];
  if (filt) {  // filter centre and half-width of the last Rayleigh-Ritz step (device)
    cc = filt[0];
    ce = filt[1];
  }
  double* sB = sm;
  double* sZ = sm + SLICE * k;
  const int s = blockIdx.x;
  const int64_t base = (int64_t)s * SLICE * k;
  const int cnt = SLICE * k;
  const int64_t cstride = (int64_t)npad * k;
  // pairs of elements (16-byte loads), RG_PAIRS per thread of the 1024; the
  // chunk partials of all of a thread's pairs are loaded RG_BATCH chunks at a
  // time before any is added (one memory latency per batch, not per pair), and
  // each element is summed in chunk order.  The 16 waves also share the Gram
  // blocks (one slice per workgroup leaves most CUs idle, so a workgroup of
  // 1024 threads: the n = 5000 solve's 7,000 calls took 14 ms less in all)
  constexpr int RG_PAIRS = SLICE * KMAX / 2 / 1024, RG_BATCH = 5;
  int tt[RG_PAIRS];
  double2 z[RG_PAIRS], b[RG_PAIRS], bp[RG_PAIRS];
#pragma unroll
  for (int j = 0; j < RG_PAIRS; ++j) {
    tt[j] = 2 * ((int)threadIdx.x + j * (int)blockDim.x);
    z[j] = make_double2(0.0, 0.0);
    const bool in = tt[j] < cnt;
    b[j] = in ? *reinterpret_cast<const double2*>(B + base + tt[j]) : make_double2(0.0, 0.0);
    bp[j] = (in && cheb == 2) ? *reinterpret_cast<const double2*>(Bprev + base + tt[j])
                              : make_double2(0.0, 0.0);
  }
  for (int c = 0; c < nchunks; c += RG_BATCH) {
    double2 v[RG_BATCH][RG_PAIRS];
#pragma unroll
    for (int u = 0; u < RG_BATCH; ++u)
#pragma unroll
      for (int j = 0; j < RG_PAIRS; ++j)
        v[u][j] = (c + u < nchunks && tt[j] < cnt)
                      ? *reinterpret_cast<const double2*>(part + (c + u) * cstride + base + tt[j])
                      : make_double2(0.0, 0.0);
#pragma unroll
    for (int u = 0; u < RG_BATCH; ++u)
#pragma unroll
      for (int j = 0; j < RG_PAIRS; ++j)
        if (c + u < nchunks) {
          z[j].x += v[u][j].x;
          z[j].y += v[u][j].y;
        }
  }
#pragma unroll
  for (int j = 0; j < RG_PAIRS; ++j) {
    const int t = tt[j];
    if (t >= cnt) continue;
    if (cheb == 1) {
      z[j].x = (z[j].x - cc * b[j].x) / ce;
      z[j].y = (z[j].y - cc * b[j].y) / ce;
    } else if (cheb == 2) {
      z[j].x = 2.0 * (z[j].x - cc * b[j].x) / ce - bp[j].x;
      z[j].y = 2.0 * (z[j].y - cc * b[j].y) / ce - bp[j].y;
    }
    if (Z) *reinterpret_cast<double2*>(Z + base + t) = z[j];
    sZ[t] = z[j].x;
    sZ[t + 1] = z[j].y;
    sB[t] = b[j].x;
    sB[t + 1] = b[j].y;
  }
  if (!grams) return;
  __syncthreads();
  gram_blocks_mfma(sB, sZ, k, gram_part + (int64_t)s * 3 * k * k);
}

// Per slice of SLICE rows (all products on MFMA f64 16x16x4), in three kinds of
// workgroup (blockIdx.y) that run side by side:
//   0 factors    Vs = B S[:, :rp] (rp = r rounded to 16); V = Vs[:, :r] (row
//                stride KMAX); partials of [V^T V | V^T Vold | u_q^T V]   (if V)
//   1 basis      Bn = Z MZ + B MB (row stride k)                          (if Bn)
//   2 residuals  Vs and ZS = Z S[:, :rp]; partials ||ZS_c - theta_c Vs_c||^2
//                -> fac_part[FAC_RES + c], c < r
// (Vs is formed by kinds 0 and 2 alike, by the same code.)
// LDS: B, Z with row stride k + 1 and Vs, ZS with row stride rp + 1 (odd
// strides keep the 16 lanes of an MFMA operand column on distinct banks).
// Operand columns of the small matrices (S, MZ, MB) are loaded from global
// memory once per wave and column block: with 8 waves and at most 4 column
// blocks every job of a wave shares one.
__device__ inline void load_small_col(const double* Sg, int ldS, int col0, int k,
                                      double (&bq)[KMAX / 4]) {
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int q = 0; q < KMAX / 4; ++q) bq[q] = (4 * q < k) ? Sg[(4 * q + kq) * ldS + col0 + m] : 0.0;
}

__device__ inline d4 mfma_rows_times_cols(const double* Xl, int ldx, int row0,
                                          const double (&bq)[KMAX / 4], int k, d4 acc) {
  // acc[m][n] += sum_q Xl[row0 + m][q] * S[q][col0 + n], S's column block in bq
  const int lane = threadIdx.x & 63;
  const int m = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int q = 0; q < KMAX / 4; ++q) {
    if (4 * q < k) {
      const double a = Xl[(row0 + m) * ldx + 4 * q + kq];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bq[q], acc, 0, 0, 0);
    }
  }
  return acc;
}

__global__ __launch_bounds__(512) void k_rowwise(const double* __restrict__ B,
                                                 const double* __restrict__ Z,
                                                 const double* __restrict__ small, int k,
                                                 double* __restrict__ V, int r,
                                                 const double* __restrict__ Vold, int r_old,
                                                 double* __restrict__ Bn, int n_r1,
                                                 const double* __restrict__ r1_u, int npad,
                                                 double* __restrict__ fac_part) {
  extern __shared__ double sm[];
  const int rp = (r + 15) & ~15;
  const int ldk = k + 1, ldr = rp + 1;
  double* sB = sm;                   // SLICE x ldk
  double* sZ = sB + SLICE * ldk;     // SLICE x ldk
  double* sV = sZ + SLICE * ldk;     // SLICE x ldr
  double* sZS = sV + SLICE * ldr;    // SLICE x ldr
  double* sU = sZS + SLICE * ldr;    // n_r1 x SLICE: rank-one vectors on the slice
  const int s = blockIdx.x;
  const int kind = blockIdx.y;
  if ((kind == 0 && !V) || (kind == 1 && !Bn)) return;
  const bool needZ = kind != 0;
  const int i0 = s * SLICE;
  const int64_t base = (int64_t)i0 * k;
  {
    // all loads of the slice in flight together (blockDim.x = 512)
    constexpr int PER = SLICE * KMAX / 512;
    const int cnt = SLICE * k;
    double vb[PER], vz[PER];
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int t = threadIdx.x + j * 512;
      vb[j] = t < cnt ? B[base + t] : 0.0;
      vz[j] = (needZ && t < cnt) ? Z[base + t] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int t = threadIdx.x + j * 512;
      if (t < cnt) {
        const int i = t / k, c = t - (t / k) * k;
        sB[i * ldk + c] = vb[j];
        if (needZ) sZ[i * ldk + c] = vz[j];
      }
    }
  }
  if (kind == 0)
    for (int t = threadIdx.x; t < n_r1 * SLICE; t += blockDim.x)
      sU[t] = r1_u[(int64_t)(t / SLICE) * npad + i0 + (t % SLICE)];
  __syncthreads();
  const double* S = small + SL::S;
  const double* MZ = small + SL::MZ;
  const double* MB = small + SL::MB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int rb = rp / 16, kb = k / 16;
  double bq[KMAX / 4], bq2[KMAX / 4];
  int cached = -1;
  if (kind == 1) {
    // jobs: Bn blocks (4 x kb)
    for (int job = wave; job < 4 * kb; job += nw) {
      const int row0 = (job / kb) * 16, col0 = (job - (job / kb) * kb) * 16;
      if (col0 != cached) {
        load_small_col(MZ, KMAX, col0, k, bq);
        load_small_col(MB, KMAX, col0, k, bq2);
        cached = col0;
      }
      d4 acc = d4{0.0, 0.0, 0.0, 0.0};
      acc = mfma_rows_times_cols(sZ, ldk, row0, bq, k, acc);
      acc = mfma_rows_times_cols(sB, ldk, row0, bq2, k, acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + kq + 4 * v, col = col0 + m;
        Bn[base + (int64_t)row * k + col] = acc[v];
      }
    }
    return;
  }
  // jobs: [Vs blocks: 4 x rb] (+ [ZS blocks: 4 x rb] for the residuals)
  const int nV = 4 * rb;
  const int njobs = kind == 2 ? 2 * nV : nV;
  for (int job = wave; job < njobs; job += nw) {
    const bool isZ = job >= nV;
    const int jb = isZ ? job - nV : job;
    const int row0 = (jb / rb) * 16, col0 = (jb - (jb / rb) * rb) * 16;
    if (col0 != cached) {
      load_small_col(S, KMAX, col0, k, bq);
      cached = col0;
    }
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    acc = mfma_rows_times_cols(isZ ? sZ : sB, ldk, row0, bq, k, acc);
    double* dst = isZ ? sZS : sV;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = row0 + kq + 4 * v, col = col0 + m;
      dst[row * ldr + col] = acc[v];
      if (kind == 0 && col < r) V[(int64_t)(i0 + row) * KMAX + col] = acc[v];
    }
  }
  __syncthreads();
  double* out = fac_part + (int64_t)s * FAC_STRIDE;
  if (kind == 2) {
    const double* theta = small + SL::THETA;
    // residual norms: eight lanes per column, SLICE / 8 rows each, combined by
    // a fixed butterfly
    for (int c0 = 0; c0 < r; c0 += (int)blockDim.x / 8) {
      const int c = c0 + (int)(threadIdx.x >> 3), part = threadIdx.x & 7;
      const int cc = c < r ? c : 0;
      const double th = theta[cc];
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < SLICE / 8; ++j) {
        const int i = part * (SLICE / 8) + j;
        const double d = sZS[i * ldr + cc] - th * sV[i * ldr + cc];
        acc += d * d;
      }
      acc += __shfl_xor(acc, 1);
      acc += __shfl_xor(acc, 2);
      acc += __shfl_xor(acc, 4);
      if (c < r && part == 0) out[FAC_RES + c] = acc;
    }
    return;
  }
  // factor Grams on MFMA: V^T V (rb x rb blocks) and V^T Vold (rb x rob blocks)
  const int rop = (r_old + 15) & ~15;
  const int rob = rop / 16;
  const int n1 = r * r;
  int cached_old = -1;
  double bo[SLICE / 4];
  for (int job = wave; job < rb * rb + rb * rob; job += nw) {
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    const bool old = job >= rb * rb;
    const int jb = old ? job - rb * rb : job;
    const int nbk = old ? rob : rb;
    const int a0 = (jb / nbk) * 16, b0 = (jb - (jb / nbk) * nbk) * 16;
    if (old) {
      if (b0 != cached_old) {
        const bool in = b0 + m < r_old;
#pragma unroll
        for (int q = 0; q < SLICE / 4; ++q)
          bo[q] = in ? Vold[(int64_t)(i0 + 4 * q + kq) * KMAX + b0 + m] : 0.0;
        cached_old = b0;
      }
#pragma unroll
      for (int q = 0; q < SLICE / 4; ++q) {
        const double a = sV[(4 * q + kq) * ldr + a0 + m];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bo[q], acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < SLICE / 4; ++q) {
        const double a = sV[(4 * q + kq) * ldr + a0 + m];
        const double bv = sV[(4 * q + kq) * ldr + b0 + m];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ra = a0 + kq + 4 * v, cb = b0 + m;
      if (!old) {
        if (ra < r && cb < r) out[ra * r + cb] = acc[v];
      } else {
        if (ra < r && cb < r_old) out[n1 + ra * r_old + cb] = acc[v];
      }
    }
  }
  const int n2 = r * r_old;
  for (int t = threadIdx.x; t < n_r1 * r; t += blockDim.x) {
    const int q = t / r, a = t - (t / r) * r;
    double acc = 0.0;
    for (int i = 0; i < SLICE; ++i) acc += sU[q * SLICE + i] * sV[i * ldr + a];
    out[n1 + n2 + t] = acc;
  }
}

// ------------------------------------------------------ implicit operator
// The iterate W = X - alpha (C - M*(y)) is low rank plus sparse:
//   W = V diag(lam) V^T + D + sum_q gamma_q u_q u_q^T,
// with X = V diag(lam) V^T the current factors, D = -alpha C + alpha M*(y) on the
// sparsity pattern (the values the dense write adds) and gamma_q = alpha sigma_q y_q.
// Z = W B is applied exactly in FP64 without the dense matrix:
//   k_vtb            per-slice partials of V^T B (r x k) and u_q^T B (MFMA)
//   k_sum_vb         slice sums, scaled by lambda_t and gamma_q
//   k_implicit_rows  Z_i = V_i M + sum_q u_q[i] M_q + sum_{e in row i} D_e B_other(e)
// and the Rayleigh-Ritz Gram partials come from k_reduce_gram on Z.
__device__ inline int last_positive(const double* lam, int r) {
  // number of leading factor columns that can contribute: the index after
  // the last positive lambda (r <= KMAX, one lane per column)
  const int ln = threadIdx.x & 63;
  const unsigned long long pos = __ballot(ln < r && lam[ln < r ? ln : 0] > 0.0);
  return pos ? 64 - __clzll((long long)pos) : 0;
}

__global__ __launch_bounds__(256) void k_vtb(const double* __restrict__ V, int r,
                                             const double* __restrict__ lam,
                                             const double* __restrict__ B, int k, int n_r1,
                                             const double* __restrict__ r1_u, int npad,
                                             double* __restrict__ vb_part) {
  const int s = blockIdx.x;
  const int i0 = s * SLICE;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  // columns after the last positive lambda are zero in X; their rows of
  // V^T B are never read (k_sum_vb and k_implicit_rows stop there too)
  r = last_positive(lam, r);
  const int rb = (r + 15) / 16, kb = k / 16;
  double* out = vb_part + (int64_t)s * VB_STRIDE;
  for (int blk = wave; blk < rb * kb; blk += nw) {
    const int a0 = (blk / kb) * 16, b0 = (blk - (blk / kb) * kb) * 16;
    d4 acc = d4{0.0, 0.0, 0.0, 0.0};
    // all operands of the block's 16 MFMAs are loaded before the first one
    double av[SLICE / 4], bv[SLICE / 4];
#pragma unroll
    for (int q = 0; q < SLICE / 4; ++q) {
      const int row = i0 + 4 * q + kq;
      av[q] = (a0 + m < r) ? V[(int64_t)row * KMAX + a0 + m] : 0.0;
      bv[q] = B[(int64_t)row * k + b0 + m];
    }
#pragma unroll
    for (int q = 0; q < SLICE / 4; ++q)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ra = a0 + kq + 4 * v;
      if (ra < r) out[ra * KMAX + b0 + m] = acc[v];
    }
  }
  for (int t = threadIdx.x; t < n_r1 * k; t += blockDim.x) {
    const int q = t / k, c = t - (t / k) * k;
    double acc = 0.0;
    for (int i = 0; i < SLICE; ++i) acc += r1_u[(int64_t)q * npad + i0 + i] * B[(int64_t)(i0 + i) * k + c];
    out[KMAX * KMAX + q * KMAX + c] = acc;
  }
}

// Slice sums of the V^T B and u^T B partials, scaled for the apply:
//   small[VB + t KMAX + c]          = lambda_t (V^T B)_tc          (t < r)
//   small[VB + KMAX^2 + q KMAX + c] = gamma_q (u_q^T B)_c,  gamma_q = alpha sigma_q y_row(q)
// SVB_LANES lanes per value, each summing every SVB_LANES-th slice with the
// loads of a batch in flight together, combined by a fixed butterfly.
constexpr int SVB_LANES = 8, SVB_BATCH = 10;
__global__ __launch_bounds__(256) void k_sum_vb(const double* __restrict__ vb_part, int nslices,
                                                int r, int k, DevProblem dp,
                                                const double* __restrict__ y, int lam_off,
                                                double* __restrict__ small) {
  r = last_positive(small + lam_off, r);
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = g / SVB_LANES, part = g % SVB_LANES;
  const int n1 = r * k;
  if (t >= n1 + dp.n_r1 * k) return;   // whole groups of SVB_LANES lanes
  int src;
  double sc;
  if (t < n1) {
    const int a = t / k;
    src = a * KMAX + (t - a * k);
    sc = small[lam_off + a];
  } else {
    const int q = (t - n1) / k;
    src = KMAX * KMAX + q * KMAX + (t - n1 - q * k);
    sc = small[SL::SC + S_ALPHA] * dp.r1_sigma[q] * y[dp.r1_row[q]];
  }
  double acc = 0.0;
  for (int s0 = part; s0 < nslices; s0 += SVB_LANES * SVB_BATCH) {
    double v[SVB_BATCH];
#pragma unroll
    for (int u = 0; u < SVB_BATCH; ++u) {
      const int s = s0 + u * SVB_LANES;
      v[u] = s < nslices ? vb_part[(int64_t)s * VB_STRIDE + src] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < SVB_BATCH; ++u) acc += v[u];
  }
#pragma unroll
  for (int o = 1; o < SVB_LANES; o <<= 1) acc += __shfl_xor(acc, o);
  if (part == 0) small[SL::VB + src] = sc * acc;
}

// Z = W B applied exactly (rows of the precision form's Rayleigh-Ritz pass):
//   Z_i = sum_t V_it M_t + sum_q u_q[i] M_q + sum_{e in row i} D_e B_other(e)
// with M from k_sum_vb.  A workgroup covers 4 rows, a thread one column.
__global__ __launch_bounds__(256) void k_implicit_rows(DevProblem dp, const double* __restrict__ V,
                                                       int r, int lam_off,
                                                       const double* __restrict__ small,
                                                       const double* __restrict__ dval,
                                                       const double* __restrict__ B, int k,
                                                       double* __restrict__ Z) {
  // one wave per row i (lane c = column c of Z); the row's pattern entries are
  // fetched by the lanes together and broadcast one by one, so that their
  // basis rows are read back to back instead of after a chain of index loads
  const int c = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= dp.npad) return;   // whole waves
  r = last_positive(small + lam_off, r);
  double acc = 0.0;
  if (i < dp.n) {
    if (c < k) {
      const double* M = small + SL::VB;
      // the row of V in one coalesced load, its entries broadcast from lanes;
      // the rows of M loaded 16 at a time before they are used
      const double vv = V[(int64_t)i * KMAX + c];
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      for (int t0 = 0; t0 < r; t0 += 16) {
        double mv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) mv[u] = (t0 + u < r) ? M[(t0 + u) * KMAX + c] : 0.0;
#pragma unroll
        for (int u = 0; u < 16; u += 4) {
          const double x0 = (t0 + u < r) ? __shfl(vv, t0 + u) : 0.0;
          const double x1 = (t0 + u + 1 < r) ? __shfl(vv, t0 + u + 1) : 0.0;
          const double x2 = (t0 + u + 2 < r) ? __shfl(vv, t0 + u + 2) : 0.0;
          const double x3 = (t0 + u + 3 < r) ? __shfl(vv, t0 + u + 3) : 0.0;
          a0 += x0 * mv[u];
          a1 += x1 * mv[u + 1];
          a2 += x2 * mv[u + 2];
          a3 += x3 * mv[u + 3];
        }
      }
      acc = (a0 + a1) + (a2 + a3);
      for (int q = 0; q < dp.n_r1; ++q)
        acc += dp.r1_u[(int64_t)q * dp.npad + i] * M[KMAX * KMAX + q * KMAX + c];
    }
    const int s0 = dp.sym_ptr[i], s1 = dp.sym_ptr[i + 1];
    for (int base = s0; base < s1; base += 64) {
      const int s = base + c;
      int other = 0;
      double dv = 0.0;
      if (s < s1) {
        other = dp.slot_other[s];
        dv = dval[dp.sym_e[s]];
      }
      const int cnt = min(64, s1 - base);
#pragma unroll 8
      for (int j = 0; j < cnt; ++j) {
        const int oj = __shfl(other, j);
        const double dj = __shfl(dv, j);
        if (c < k) acc += dj * B[(int64_t)oj * k + c];
      }
    }
  }
  if (c < k) Z[(int64_t)i * k + c] = acc;
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

// Low-precision copies of the basis block for the precision form's passes,
// made once per pass (the pass workgroups then stage 2 or 4 bytes per entry
// instead of converting 8-byte entries themselves):
//   FP32: Bf[i][c] = (float) B[i][c]            (same layout, row stride k)
//   BF16: Bt[c][i] = bf16_rne(B[i][c])          (transposed, row stride npad)
__global__ __launch_bounds__(256) void k_basis_f32(const double* __restrict__ B, int64_t count,
                                                   float* __restrict__ Bf) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < count) Bf[t] = (float)B[t];
}
__global__ __launch_bounds__(256) void k_basis_bf16t(const double* __restrict__ B, int k, int npad,
                                                     unsigned short* __restrict__ Bt) {
  __shared__ unsigned short s[64 * (KMAX + 2)];
  const int i0 = blockIdx.x * 64;
  for (int t = threadIdx.x; t < 64 * k; t += blockDim.x) {
    const int ii = t / k, c = t - (t / k) * k;
    s[ii * (KMAX + 2) + c] = to_bf16_rne(B[(int64_t)(i0 + ii) * k + c]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 64 * k; t += blockDim.x) {
    const int c = t >> 6, ii = t & 63;
    Bt[(int64_t)c * npad + i0 + ii] = s[ii * (KMAX + 2) + c];
  }
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

// The finalising workgroup's code would raise the register count to 98 (four
// workgroups per CU); capped at five waves per SIMD, the LDS limit, without spills.
template <typename OutT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_write_w(OutT* __restrict__ W, int64_t ld, int n,
                                                 const double* __restrict__ V, int ldv, int r,
                                                 double* __restrict__ small, int lam_off,
                                                 DevProblem dp, const double* __restrict__ y,
                                                 const double* __restrict__ y_old,
                                                 const double* __restrict__ dval, int sparse,
                                                 int rank1, int has_fin, FinArgs fin,
                                                 int tiles_side) {
  extern __shared__ double sm[];
  const int T = tiles_side;
  // block 0 finalises the iteration (scheduled first, so that it overlaps the tiles)
  if (has_fin && blockIdx.x == 0) {
    finalize_iteration(fin, small, dp, y, y_old, sm);
    return;
  }
  // block -> tile pair (I, J), I <= J, row-major over the upper triangle of tiles
  const int idx = (int)blockIdx.x - (has_fin ? 1 : 0);
  auto first = [&](int i) { return i * T - (i * (i - 1)) / 2; };
  const double tt = 2.0 * T + 1.0;
  int I = (int)((tt - sqrt(fmax(tt * tt - 8.0 * idx, 0.0))) * 0.5);
  I = max(0, min(I, T - 1));
  while (I + 1 < T && first(I + 1) <= idx) ++I;
  while (I > 0 && first(I) > idx) --I;
  const int J = I + (idx - first(I));
  const int tile_id = I * T + J;
  const int a0 = I * TILE, b0 = J * TILE;
  const double* lam = small + lam_off;
  // The tile's pattern items are fetched first and their values gathered
  // while the factor rows load and the products run (one item per thread; a
  // longer list is finished after the products): the chain tile range ->
  // item -> value would otherwise stall every workgroup for three memory
  // latencies between its products and its stores.
  int p0 = 0, p1 = 0;
  if (sparse) {
    p0 = dp.tile_ptr[tile_id];
    p1 = dp.tile_ptr[tile_id + 1];
  }
  int my_item = -1, my_e = 0;
  if (sparse && p0 + (int)threadIdx.x < p1) {
    my_item = dp.tile_item[p0 + threadIdx.x];
    my_e = dp.tile_e[p0 + threadIdx.x];
  }
  // factor columns after the last positive lambda add nothing to the tile
  r = last_positive(lam, r);
  const int nq = rank1 ? dp.n_r1 : 0;
  const int rr = r + nq;
  // LDS: first the scaled factor rows of the column block (64 x rr, odd row
  // stride, rr <= KMAX + MAX_R1), staged once for the four waves with
  // coalesced loads; then, in the same memory, the 64 x 64 output tile,
  // unpadded with its columns permuted per row (element (a, c) at column
  // c ^ a), so that both a row and a column of it are read without bank
  // conflicts and the block needs 32 KB (five workgroups per CU) at rr < 64.
  const int LDVB = rr | 1;   // odd, >= rr (columns >= rr are never read)
  auto tix = [](int a, int c) { return a * TILE + (c ^ a); };
  double* sVb = sm;
  double* sT = sm;
  const double alpha = small[SL::SC + S_ALPHA];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  // lane q of a wave holds column q (and q + 64) of a row: factor columns
  // scaled by lambda_q, then the rank-one terms scaled by
  // gamma_u = alpha sigma_u y_u
  double my_val = 0.0;
  for (int half = 0; half < 2; ++half) {
    const int q = lane + 64 * half;
    if (half == 1 && rr <= 64) break;
    double sc = 0.0;
    const double* uu = nullptr;
    if (q < r) {
      sc = lam[q];
    } else if (q < rr) {
      const int u = q - r;
      sc = alpha * dp.r1_sigma[u] * y[dp.r1_row[u]];
      uu = dp.r1_u + (int64_t)u * dp.npad;
    }
    if (q < LDVB) {
      double v[TILE / 4];
#pragma unroll
      for (int i = 0; i < TILE / 4; ++i) {
        const int gb = b0 + w + 4 * i;
        v[i] = 0.0;
        if (q < r) v[i] = V[(int64_t)gb * ldv + q];
        else if (q < rr) v[i] = uu[gb];
      }
      if (half == 0 && my_item >= 0) my_val = dval[my_e];
#pragma unroll
      for (int i = 0; i < TILE / 4; ++i) sVb[(w + 4 * i) * LDVB + q] = v[i] * sc;
    } else if (half == 0 && my_item >= 0) {
      my_val = dval[my_e];
    }
  }
  __syncthreads();
  // low-rank part on MFMA f64 16x16x4: wave w owns rows [16w, 16w + 16) of the
  // tile; A from the factor rows of the row block (16 contraction indices per
  // batch, loads issued before the MFMAs), B from the staged block:
  //   A[m][q] = Vrow(a0 + 16w + m)[q],  B[q][c] = s_q Vrow(b0 + 16nb + c)[q]
  {
    d4 acc[4];
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) acc[nb] = d4{0.0, 0.0, 0.0, 0.0};
    const int m = lane & 15, kq = lane >> 4;
    const int arow = a0 + 16 * w + m;
    for (int t0 = 0; t0 < rr; t0 += 16) {
      double av[4];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int q = t0 + 4 * s4 + kq;
        if (q < r) av[s4] = V[(int64_t)arow * ldv + q];
        else if (q < rr) av[s4] = dp.r1_u[(int64_t)(q - r) * dp.npad + arow];
        else av[s4] = 0.0;
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int q = t0 + 4 * s4 + kq;
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
          const double bv = (q < rr) ? sVb[(16 * nb + m) * LDVB + q] : 0.0;
          acc[nb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s4], bv, acc[nb], 0, 0, 0);
        }
      }
    }
    __syncthreads();   // every wave is done with the staged rows
    // result lane l, register v: row l/16 + 4 v, column l % 16
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
        sT[tix(16 * w + kq + 4 * v, 16 * nb + m)] = acc[nb][v];
    }
  }
  if (sparse) {
    __syncthreads();
    // every item of the tile pair is a distinct (row, column) of the tile
    if (my_item >= 0) sT[tix(my_item >> 8, my_item & 255)] += my_val;
    for (int t = p0 + (int)blockDim.x + (int)threadIdx.x; t < p1; t += blockDim.x) {
      const int it = dp.tile_item[t];
      sT[tix(it >> 8, it & 255)] += dval[dp.tile_e[t]];
    }
  }
  __syncthreads();
  // tile (I, J) row by row, then its transpose into tile (J, I): W is symmetric
  // (V diag(lam) V^T, the rank-one terms and the mirrored pattern all are).
  // Non-temporal stores: the store stream then leaves the factor rows that the
  // other tiles read in L2 (n = 5000, FP64: 79.7 -> 73.2 us per write, the next
  // pass 69.2 -> 71.1 us as less of W is still cached, 30 ms less per solve).
  const int c = lane;
  for (int q = 0; q < TILE / 4; ++q) {
    const int a = w + 4 * q;
    const int ga = a0 + a, gb = b0 + c;
    if (ga < n && gb < n) __builtin_nontemporal_store(store_cast<OutT>(sT[tix(a, c)]), &W[(int64_t)ga * ld + gb]);
  }
  if (I != J) {
    for (int q = 0; q < TILE / 4; ++q) {
      const int b = w + 4 * q;
      const int gb = b0 + b, ga = a0 + c;
      if (gb < n && ga < n) __builtin_nontemporal_store(store_cast<OutT>(sT[tix(c, b)]), &W[(int64_t)gb * ld + ga]);
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
