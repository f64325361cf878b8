// Single-workgroup kernels for the small dense problems of the partial
// eigensolve (Rayleigh-Ritz on the k x k projected matrix) and for the exact
// eigendecomposition used by PD-SDP at small n (Section 2.3.2).
//
// Eigensolver: cyclic two-sided Jacobi with the round-robin (tournament)
// ordering, so that k/2 disjoint rotations are applied per round in
// parallel; LDS resident.  Rotation angle from the 2x2 symmetric Schur
// decomposition (Golub and Van Loan, Algorithm 8.4.1).
#pragma once

#include "common.hpp"

namespace proxsdp {

// Index of the partner pairs in round `rnd` of a kk-player round robin
// (kk even): player 0 stays, the others rotate.
__device__ __forceinline__ int rr_player(int pos, int rnd, int kk) {
  if (pos == 0) return 0;
  return ((pos - 1 + rnd) % (kk - 1)) + 1;
}

// Symmetric eigendecomposition of A (k x k, LDS, stride lda) in place: on exit
// the diagonal holds the eigenvalues and U (LDS, stride ldu) the eigenvectors
// (columns).  Each round applies the k/2 disjoint rotations of the
// round-robin ordering; the two-sided update is done per 2 x 2 block
// (J_i^T A_ij J_j), so a round needs two barriers.  Sweeps stop when the
// off-diagonal norm is below 1e-15 of the diagonal norm.
// `cs` is LDS scratch of 3 (KMAX/2 + 1) doubles; `red` of 2 doubles.
// Returns the number of sweeps.
//
// `threshold` (for nearly diagonal input): a pair is rotated only if its
// off-diagonal entry exceeds tol_off ||diag||_2 / k, and a round with no such
// pair skips its update (one barrier instead of two).
// `imp` (optional, threshold mode): only pairs with imp[p] or imp[q] set are
// rotated and counted in the off-diagonal test.
__device__ __forceinline__ int jacobi_eig(double* A, int lda, double* U, int ldu, int k, double* cs, int* flag,
                          int max_sweeps, double tol_off = 1e-15, bool threshold = false,
                          const int* imp = nullptr) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int t = tid; t < (k << 6); t += nt) {
    const int i = t >> 6, j = t & 63;
    if (j < k) U[i * ldu + j] = (i == j) ? 1.0 : 0.0;
  }
  const int kk = (k & 1) ? k + 1 : k;
  const int np = kk / 2;
  double* cc = cs;
  double* ss = cs + np;
  int* pp = reinterpret_cast<int*>(cs + 2 * np);
  int* qq = pp + np;
  int sweeps = 0;
  __shared__ double offw[2 * 16];   // per-wave partial sums (fixed-order reduction)
  __shared__ int anyrot[2];
  if (tid == 0) { anyrot[0] = 1; anyrot[1] = 1; }
  const int nw = nt >> 6;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    // convergence test on the off-diagonal mass
    if (tid == 0) *flag = 0;
    __syncthreads();
    double off = 0.0, dg = 0.0;
    for (int t = tid; t < (k << 6); t += nt) {
      const int i = t >> 6, j = t & 63;
      if (j >= k) continue;
      const double v = A[i * lda + j];
      if (i == j) dg += v * v;
      else if (!imp || imp[i] || imp[j]) off += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      dg += __shfl_xor(dg, o);
    }
    if ((tid & 63) == 0) {
      offw[2 * (tid >> 6)] = off;
      offw[2 * (tid >> 6) + 1] = dg;
    }
    __syncthreads();
    off = 0.0;
    dg = 0.0;
    for (int w = 0; w < nw; ++w) {
      off += offw[2 * w];
      dg += offw[2 * w + 1];
    }
    if (!(off > tol_off * tol_off * dg) || !(off > 1e-300)) break;
    const double pair_thr = threshold ? tol_off * sqrt(dg) / k : 0.0;
    for (int rnd = 0; rnd < kk - 1; ++rnd) {
      if (threshold && tid == 0) anyrot[(rnd + 1) & 1] = 0;
      for (int i = tid; i < np; i += nt) {
        int p = rr_player(i, rnd, kk), q = rr_player(kk - 1 - i, rnd, kk);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < k && (!imp || imp[p] || imp[q])) {
          const double app = A[p * lda + p], aqq = A[q * lda + q], apq = A[p * lda + q];
          const double thr = fmax(1e-18 * sqrt(fabs(app * aqq)), pair_thr) + 1e-300;
          if (fabs(apq) > thr) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
            if (threshold) anyrot[rnd & 1] = 1;
          }
        }
        cc[i] = c; ss[i] = s; pp[i] = p; qq[i] = (q < k) ? q : -1;
      }
      __syncthreads();
      if (threshold && anyrot[rnd & 1] == 0) continue;
      // A <- J^T A J blockwise; U <- U J.  A thread keeps one row pair (its
      // rotation in registers) and handles column pairs / rows in batches of
      // four: all loads, then the arithmetic, then all stores, so the LDS
      // latency is paid once per batch.
      {
        const int groups = nt / np;
        const int bi = tid % np, g0 = tid / np;
        if (g0 < groups) {
          const int pi = pp[bi], qi = qq[bi];
          const double ci = cc[bi], si = ss[bi];
          for (int b0 = g0; b0 < np; b0 += 4 * groups) {
            double a[4], b[4], c_[4], d[4], cj[4], sj[4];
            int pj[4], qj[4];
            bool on[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int bj = b0 + u * groups;
              on[u] = bj < np;
              const int bjj = on[u] ? bj : bi;
              pj[u] = pp[bjj];
              qj[u] = qq[bjj];
              cj[u] = cc[bjj];
              sj[u] = ss[bjj];
              on[u] = on[u] && !(si == 0.0 && sj[u] == 0.0);
              a[u] = A[pi * lda + pj[u]];
              b[u] = (qj[u] >= 0) ? A[pi * lda + qj[u]] : 0.0;
              c_[u] = (qi >= 0) ? A[qi * lda + pj[u]] : 0.0;
              d[u] = (qi >= 0 && qj[u] >= 0) ? A[qi * lda + qj[u]] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              if (!on[u]) continue;
              const double a1 = ci * a[u] - si * c_[u], b1 = ci * b[u] - si * d[u];
              const double c1 = si * a[u] + ci * c_[u], d1 = si * b[u] + ci * d[u];
              A[pi * lda + pj[u]] = cj[u] * a1 - sj[u] * b1;
              if (qj[u] >= 0) A[pi * lda + qj[u]] = sj[u] * a1 + cj[u] * b1;
              if (qi >= 0) A[qi * lda + pj[u]] = cj[u] * c1 - sj[u] * d1;
              if (qi >= 0 && qj[u] >= 0) A[qi * lda + qj[u]] = sj[u] * c1 + cj[u] * d1;
            }
          }
          if (qi >= 0 && si != 0.0) {
            for (int r0 = g0; r0 < k; r0 += 4 * groups) {
              double up[4], uq[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int r = r0 + u * groups;
                up[u] = (r < k) ? U[r * ldu + pi] : 0.0;
                uq[u] = (r < k) ? U[r * ldu + qi] : 0.0;
              }
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const int r = r0 + u * groups;
                if (r < k) {
                  U[r * ldu + pi] = ci * up[u] - si * uq[u];
                  U[r * ldu + qi] = si * up[u] + ci * uq[u];
                }
              }
            }
          }
        }
      }
      __syncthreads();
    }
    ++sweeps;
  }
  __syncthreads();
  return sweeps;
}

// FP64 reciprocal and reciprocal square root: the hardware estimates refined
// by two Newton steps each (x <- x (2 - a x), y <- y (3 - a y^2) / 2).
__device__ __forceinline__ double rcp_refined(double a) {
  double x = __builtin_amdgcn_rcp(a);
  double e = fma(-a, x, 1.0);
  x = fma(x, e, x);
  e = fma(-a, x, 1.0);
  return fma(x, e, x);
}
__device__ __forceinline__ double rsq_refined(double a) {
  double y = __builtin_amdgcn_rsq(a);
  double r = fma(-a * y, y, 1.0);
  y = fma(0.5 * y, r, y);
  r = fma(-a * y, y, 1.0);
  return fma(0.5 * y, r, y);
}

// Rotation of the 2 x 2 symmetric Schur decomposition of (app, apq; apq, aqq)
// (Golub and Van Loan, Algorithm 8.4.1; the tangent of jacobi_eig's rotation,
// t = sign(d) e / (|d| + sqrt(d^2 + e^2)), d = aqq - app, e = 2 apq, up to
// rounding; c = 1, s = 0 below the negligible level) without IEEE divisions
// or square roots: d and e are scaled by 1 / max(|d|, |e|) so that
// d^2 + e^2 lies in [1, 2], and c = (1 + t^2)^(-1/2) is refined to full
// precision, so c^2 + s^2 = 1 to rounding.
__device__ __forceinline__ void jacobi_rotation_fast(double app, double aqq, double apq, double& c,
                                                     double& s) {
  c = 1.0;
  s = 0.0;
  if (apq * apq > 1e-36 * fabs(app * aqq) && fabs(apq) > 1e-300) {
    const double d = aqq - app, e = 2.0 * apq;
    const double im = rcp_refined(fmax(fabs(d), fabs(e)));
    const double dn = d * im, en = e * im;
    const double q = fma(dn, dn, en * en);
    const double hq = q * rsq_refined(q);
    double t = en * rcp_refined(fabs(dn) + hq);
    if (dn < 0.0) t = -t;
    c = rsq_refined(fma(t, t, 1.0));
    s = t * c;
  }
}

// Cyclic Jacobi as jacobi_eig without threshold (same orderings, rotations
// and stopping rule, k even), with A alternating between two LDS buffers A0
// and A1: each round reads one and writes the other, and every thread forms
// the rotations it applies from the round's input, so a round needs one
// barrier.  Thread (bi, g) applies the rotation of row pair bi to the 2 x 2
// blocks (bi, bj) for bj = g, g + groups, ... and to rows g, g + groups, ...
// of U.  Returns the number of sweeps; *out is the buffer holding the result.
__device__ __forceinline__ int jacobi_eig_db(double* A0, double* A1, int lda, double* U, int ldu,
                                             int k, int max_sweeps, double tol_off, double* red,
                                             double** out) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int t = tid; t < (k << 6); t += nt) {
    const int i = t >> 6, j = t & 63;
    if (j < k) U[i * ldu + j] = (i == j) ? 1.0 : 0.0;
  }
  const int np = k / 2, km1 = k - 1;
  const int groups = nt / np;
  const int bi = tid % np, g0 = tid / np;
  const int nw = nt >> 6;
  // every thread forms the rotation of its own row pair bi; the rotation of
  // column pair bj comes from the lane of the same wave whose row pair is bj
  // (np <= 32 < 64: every wave holds all of them), not recomputed
  const int wbase = (tid - (tid & 63)) % np;   // row pair of the wave's lane 0
  const int nbj = (np + groups - 1) / groups;   // same count for every thread
  double* Ain = A0;
  double* Aout = A1;
  auto player = [&](int pos, int rnd) {
    if (pos == 0) return 0;
    int v = pos - 1 + rnd;
    if (v >= km1) v -= km1;
    return v + 1;
  };
  int sweeps = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    __syncthreads();
    double off = 0.0, dg = 0.0;
    for (int t = tid; t < (k << 6); t += nt) {
      const int i = t >> 6, j = t & 63;
      if (j >= k) continue;
      const double v = Ain[i * lda + j];
      if (i == j)
        dg += v * v;
      else
        off += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      dg += __shfl_xor(dg, o);
    }
    if ((tid & 63) == 0) {
      red[2 * (tid >> 6)] = off;
      red[2 * (tid >> 6) + 1] = dg;
    }
    __syncthreads();
    off = 0.0;
    dg = 0.0;
    for (int w = 0; w < nw; ++w) {
      off += red[2 * w];
      dg += red[2 * w + 1];
    }
    if (!(off > tol_off * tol_off * dg) || !(off > 1e-300)) break;
    for (int rnd = 0; rnd < km1; ++rnd) {
      int pi = player(bi, rnd), qi = player(k - 1 - bi, rnd);
      if (pi > qi) { const int t = pi; pi = qi; qi = t; }
      double ci, si;
      jacobi_rotation_fast(Ain[pi * lda + pi], Ain[qi * lda + qi], Ain[pi * lda + qi], ci, si);
      for (int x = 0; x < nbj; ++x) {
        const int bj = g0 + x * groups;
        int src = (bj < np ? bj : 0) - wbase;
        if (src < 0) src += np;
        const double cj = __shfl(ci, src), sj = __shfl(si, src);
        if (g0 < groups && bj < np) {
          int pj = player(bj, rnd), qj = player(k - 1 - bj, rnd);
          if (pj > qj) { const int t = pj; pj = qj; qj = t; }
          const double a = Ain[pi * lda + pj], b = Ain[pi * lda + qj];
          const double c_ = Ain[qi * lda + pj], d = Ain[qi * lda + qj];
          const double a1 = ci * a - si * c_, b1 = ci * b - si * d;
          const double c1 = si * a + ci * c_, d1 = si * b + ci * d;
          Aout[pi * lda + pj] = cj * a1 - sj * b1;
          Aout[pi * lda + qj] = sj * a1 + cj * b1;
          Aout[qi * lda + pj] = cj * c1 - sj * d1;
          Aout[qi * lda + qj] = sj * c1 + cj * d1;
        }
      }
      if (g0 < groups && si != 0.0) {
        for (int r0 = g0; r0 < k; r0 += groups) {
          const double up = U[r0 * ldu + pi], uq = U[r0 * ldu + qi];
          U[r0 * ldu + pi] = ci * up - si * uq;
          U[r0 * ldu + qi] = si * up + ci * uq;
        }
      }
      __syncthreads();
      double* t = Ain;
      Ain = Aout;
      Aout = t;
    }
    ++sweeps;
  }
  __syncthreads();
  *out = Ain;
  return sweeps;
}

// Sorts eigenvalues (diagonal of A) decreasingly: writes values to `vals`
// and the permutation to `perm`.  Rank sort: thread i counts the entries that
// precede it (larger, or equal with a smaller index), k <= KMAX.
__device__ __forceinline__ void sort_desc(const double* A, int lda, int k, double* vals, int* perm) {
  // identity first, so that a non-finite value (flagged elsewhere) can only
  // leave a valid index behind
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    vals[i] = A[i * lda + i];
    perm[i] = i;
  }
  __syncthreads();
  // eight lanes per entry, each counting over every eighth competitor
  for (int i0 = 0; i0 < k; i0 += (int)blockDim.x / 8) {
    const int i = i0 + (int)(threadIdx.x >> 3), part = threadIdx.x & 7;
    const int ii = i < k ? i : k - 1;
    const double v = A[ii * lda + ii];
    int rank = 0;
    for (int j = part; j < k; j += 8) {
      const double u = A[j * lda + j];
      rank += (u > v) || (u == v && j < ii);
    }
    rank += __shfl_xor(rank, 1);
    rank += __shfl_xor(rank, 2);
    rank += __shfl_xor(rank, 4);
    if (i < k && part == 0 && rank < k) {
      vals[rank] = v;
      perm[rank] = i;
    }
  }
  __syncthreads();
}

// One 16 x 16 tile of op(A) B on FP64 MFMA 16x16x4, KQ = k / 4.  All operand
// loads are issued before the MFMA chain.  Result element v of a lane is row
// a0 + 4 (lane / 16) + ... see the callers: row a0 + kq + 4 v, column b0 + m.
template <int KQ>
__device__ __forceinline__ d4 tile_mm(const double* A, int lda, bool ta, const double* B, int ldb,
                                      int a0, int b0, int m, int kq) {
  double av[KQ], bv[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    av[q] = ta ? A[(4 * q + kq) * lda + a0 + m] : A[(a0 + m) * lda + 4 * q + kq];
    bv[q] = B[(4 * q + kq) * ldb + b0 + m];
  }
  d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < KQ; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
  return acc;
}

template <int KQ>
__device__ __forceinline__ void lds_mm_k(double* C, int ldc, const double* A, int lda, bool ta,
                                         const double* B, int ldb, bool sym) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  constexpr int kb = KQ / 4;
  constexpr int ntiles = kb * kb;
  for (int blk = wave; blk < ntiles; blk += nw) {
    const int ta_ = blk / kb, tb_ = blk - (blk / kb) * kb;
    if (sym && ta_ > tb_) continue;
    const int a0 = ta_ * 16, b0 = tb_ * 16;
    const d4 acc = tile_mm<KQ>(A, lda, ta, B, ldb, a0, b0, m, kq);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      C[(a0 + kq + 4 * v) * ldc + b0 + m] = acc[v];
      if (sym && ta_ != tb_) C[(b0 + m) * ldc + a0 + kq + 4 * v] = acc[v];
    }
  }
}

// C = op(A) B for k x k matrices in LDS (k in {16, 32, 48, 64}) on FP64 MFMA,
// op(A) = A^T when `ta`; `sym`: the product is known to be symmetric, only
// the upper tiles are computed and mirrored.  Output tiles are spread over
// the waves.  C must not alias A or B; the caller synchronises afterwards.
__device__ __forceinline__ void lds_mm(double* C, int ldc, const double* A, int lda, bool ta,
                                       const double* B, int ldb, int k, bool sym = false) {
  switch (k) {
    case 16: lds_mm_k<4>(C, ldc, A, lda, ta, B, ldb, sym); break;
    case 32: lds_mm_k<8>(C, ldc, A, lda, ta, B, ldb, sym); break;
    case 48: lds_mm_k<12>(C, ldc, A, lda, ta, B, ldb, sym); break;
    default: lds_mm_k<16>(C, ldc, A, lda, ta, B, ldb, sym); break;
  }
}

// Out = D X F[:, perm] (perm == nullptr: identity; d == nullptr: D = I) with X
// k x k in global memory (row stride ldx) and F in LDS.  A wave owns whole
// 16-row strips and loads its strip of X before any store, so Out may be X
// itself.
__device__ __forceinline__ void strip_mm(double* Out, int ldo, const double* X, int ldx,
                                         const double* F, int ldf, const int* perm,
                                         const double* d, int k) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int m = lane & 15, kq = lane >> 4, kb = k / 16, ks = k / 4;
  for (int a0 = wave * 16; a0 < k; a0 += nw * 16) {
    double xa[KMAX / 4];
#pragma unroll
    for (int q = 0; q < KMAX / 4; ++q) xa[q] = (q < ks) ? X[(a0 + m) * ldx + 4 * q + kq] : 0.0;
    d4 acc[KMAX / 16];
#pragma unroll
    for (int b = 0; b < KMAX / 16; ++b) {
      acc[b] = d4{0.0, 0.0, 0.0, 0.0};
      if (b < kb) {
        const int col = perm ? perm[b * 16 + m] : b * 16 + m;
        double fv[KMAX / 4];
#pragma unroll
        for (int q = 0; q < KMAX / 4; ++q) fv[q] = (q < ks) ? F[(4 * q + kq) * ldf + col] : 0.0;
#pragma unroll
        for (int q = 0; q < KMAX / 4; ++q)
          if (q < ks) acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[q], fv[q], acc[b], 0, 0, 0);
      }
    }
#pragma unroll
    for (int b = 0; b < KMAX / 16; ++b) {
      if (b < kb) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = a0 + kq + 4 * v;
          Out[row * ldo + b * 16 + m] = (d ? d[row] : 1.0) * acc[b][v];
        }
      }
    }
  }
}

// For every entry (i, j) of a k x k matrix, load(i, j, v) fills NV values
// (global loads) and store(i, j, v) consumes them; each thread issues the
// loads of four entries before it stores any, so a copy from global memory
// into LDS waits for memory once per four entries instead of once per entry.
template <int NV, class LoadF, class StoreF>
__device__ __forceinline__ void kk_batched(int k, LoadF load, StoreF store) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int kk = k * k;
  for (int t0 = tid; t0 < kk; t0 += 4 * nt) {
    double v[4][NV];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * nt;
      if (t < kk) {
        const int i = t / k, j = t - (t / k) * k;
        load(i, j, v[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int t = t0 + u * nt;
      if (t < kk) {
        const int i = t / k, j = t - (t / k) * k;
        store(i, j, v[u]);
      }
    }
  }
}

// Threads of k_small_rr (eight waves; the Newton step below assumes it).
constexpr int RR_THREADS = 512;

// One Newton step's products, in place:  G <- F^T G F,  S <- F^T S F,  X <- X F
// (k x k in LDS, row stride ld, k = 4 KQ), eight waves.  Wave w < 2 kb owns
// column block b of G (w even) or S (w odd), b = kb - 1 - w / 2: it forms the
// column block (M F)[:, b] in registers, whose MFMA output layout is already
// the B-operand layout of the second product, and then the blocks a <= b of
// F^T (M F) (the rest by symmetry).  The kb^2 tiles of X F go to the waves
// from the last one down.  Everything is read before the first barrier and
// written after it; the second barrier publishes the per-wave partial sums of
// ||I - G||_F^2 and of the important off-diagonal S entries, returned in
// aR and aS (fixed summation order).
template <int KQ>
__device__ __forceinline__ void newton_products(double* G, double* S, const double* F, double* X,
                                                int ld, const int* imp, double* red, double& aR,
                                                double& aS) {
  constexpr int kb = KQ / 4;
  constexpr int NW = RR_THREADS / 64;
  constexpr int XT = (kb * kb + NW - 1) / NW;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const bool mjob = wave < 2 * kb;
  const bool isS = wave & 1;
  const int b = kb - 1 - (wave >> 1);
  double* M = isS ? S : G;
  d4 res[kb];
  d4 xres[XT];
  if (mjob) {
    // (M F)[:, b]: the F operand column block is shared by the kb tiles
    double bv[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) bv[q] = F[(4 * q + kq) * ld + b * 16 + m];
    d4 tcol[kb];
#pragma unroll
    for (int a = 0; a < kb; ++a) {
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < KQ; ++q)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(M[(a * 16 + m) * ld + 4 * q + kq], bv[q], acc, 0, 0, 0);
      tcol[a] = acc;
    }
    // F^T (M F)[:, b]: lane value v of tile a is row 16 a + kq + 4 v of the
    // column block, i.e. the B operand of k-step q = 4 a + v
#pragma unroll
    for (int a = 0; a < kb; ++a) {
      if (a > b) continue;
      d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < KQ; ++q)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(F[(4 * q + kq) * ld + a * 16 + m], tcol[q >> 2][q & 3],
                                                   acc, 0, 0, 0);
      res[a] = acc;
    }
  }
#pragma unroll
  for (int x = 0; x < XT; ++x) {
    const int t = NW - 1 - wave + x * NW;
    if (t < kb * kb) xres[x] = tile_mm<KQ>(X, ld, false, F, ld, (t / kb) * 16, (t % kb) * 16, m, kq);
  }
  __syncthreads();
  double pr = 0.0, ps = 0.0;
  if (mjob) {
#pragma unroll
    for (int a = 0; a < kb; ++a) {
      if (a > b) continue;
      const double wgt = (a != b) ? 2.0 : 1.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = a * 16 + kq + 4 * v, col = b * 16 + m;
        const double val = res[a][v];
        M[row * ld + col] = val;
        if (a != b) M[col * ld + row] = val;
        if (!isS) {
          const double rij = ((row == col) ? 1.0 : 0.0) - val;
          pr += wgt * rij * rij;
        } else if (row != col && (imp[row] || imp[col])) {
          ps += wgt * val * val;
        }
      }
    }
  }
#pragma unroll
  for (int x = 0; x < XT; ++x) {
    const int t = NW - 1 - wave + x * NW;
    if (t < kb * kb) {
      const int a0 = (t / kb) * 16, b0 = (t % kb) * 16;
#pragma unroll
      for (int v = 0; v < 4; ++v) X[(a0 + kq + 4 * v) * ld + b0 + m] = xres[x][v];
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    pr += __shfl_xor(pr, o);
    ps += __shfl_xor(ps, o);
  }
  if (lane == 0) {
    red[2 * wave] = pr;
    red[2 * wave + 1] = ps;
  }
  __syncthreads();
  aR = 0.0;
  aS = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    aR += red[2 * w];
    aS += red[2 * w + 1];
  }
}

// Deterministic workgroup reduction of (sum a, sum b, max(c, 0)); every thread
// gets the result.  `red` is LDS scratch of 3 * (blockDim / 64) doubles.
__device__ __forceinline__ void block_sum2_max1(double& a, double& b, double& c, double* red) {
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
    c = fmax(c, __shfl_xor(c, o));
  }
  const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[3 * wave] = a;
    red[3 * wave + 1] = b;
    red[3 * wave + 2] = c;
  }
  __syncthreads();
  a = 0.0; b = 0.0; c = 0.0;
  for (int w = 0; w < nw; ++w) {
    a += red[3 * w];
    b += red[3 * w + 1];
    c = fmax(c, red[3 * w + 2]);
  }
}

// Rayleigh-Ritz on span(B) from the reduced Grams G = B^T B, T = B^T W B,
// P = (W B)^T (W B): the pencil T s = theta G s.
//
// Newton path (nearly converged basis, the usual case with warm starts): the
// basis coefficients X (start: the column equilibration D) are refined by the
// quadratically convergent update of Ogita and Aishima (2018), generalised to
// the G inner product: with R = I - X^T G X, S = X^T T X and
// mu_i = S_ii / (1 - R_ii),
//   E_ij = (S_ij + mu_j R_ij) / (mu_j - mu_i)   (separated pairs),
//   E_ij = R_ij / 2                             (otherwise and on i = j),
//   X <- X (I + E),
// with matrix products only (MFMA).  The update is applied to the pairs that
// touch an important index (a positive value among the r largest) whose gap
// exceeds delta = 2 (||off(S)|| + max|mu| ||R||) and whose coupling is weak
// (|E_ij| <= 0.1); the unwanted tail is only re-orthonormalised (its dense
// near-degenerate spectrum makes Newton steps there erratic).  The result is
// accepted if X^T G X is within 1e-12 of I, the important couplings are below
// 1e-4 max|mu| and a Gershgorin bound of the tail block shows that no tail
// eigenvalue exceeds max(mu_(r), 0); threshold Jacobi on the important pairs
// finishes.  Otherwise the Cholesky path is taken.
//
// Cholesky path: generalised problem through a Cholesky factor of the
// column-equilibrated G (one CholeskyQR step folded into RR), cyclic Jacobi on
// L^{-1} T L^{-T}, back substitution.
//
// Writes (small): S (k x k, V = B S with V^T V = I), THETA (decreasing), RES
// (relative Ritz residuals ||W v - theta v|| / max|theta|), lambda_+ of the r
// kept pairs at lam_off, S_LAMR/S_LAMR1/S_MAXRES/S_NORMW, and the next-basis
// coefficients MZ, MB of the degree-one Chebyshev filter
//   Bn_i = (W - c I) v_i / ||(W - c I) v_i||,  c = (lo + theta_k) / 2,
// where lo = small[S_GERSH] bounds the spectrum from below (filter != 0;
// filter == 0 gives Bn_i = W v_i / ||W v_i||).
// k is a multiple of 16 (<= KMAX).  Loops over k x k entries use the index
// map t -> (t >> 6, t & 63) (no integer division).  LDS: 4 k x (k + 1)
// matrices + vectors.
// Dot product of length n over LDS with four independent accumulators
// (keeps several LDS loads in flight).
__device__ __forceinline__ double lds_dot(const double* a, int sa, const double* b, int sb, int n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = 0;
  for (; j + 3 < n; j += 4) {
    s0 += a[(j + 0) * sa] * b[(j + 0) * sb];
    s1 += a[(j + 1) * sa] * b[(j + 1) * sb];
    s2 += a[(j + 2) * sa] * b[(j + 2) * sb];
    s3 += a[(j + 3) * sa] * b[(j + 3) * sb];
  }
  for (; j < n; ++j) s0 += a[j * sa] * b[j * sb];
  return (s0 + s1) + (s2 + s3);
}

// Scratch doubles of k_small_rr's reductions: 3 per wave (up to 16 waves) and
// one slot (the last) for the r-th largest value.
constexpr int RR_RED = 3 * 16 + 1;

// LDS doubles of k_small_rr for subspace width k.
__host__ __device__ inline size_t small_rr_lds_doubles(int k) {
  return 4 * (size_t)k * (k + 1) + 4 * KMAX + 3 * (KMAX / 2 + 1) + RR_RED;
}

#define RR_FOR_KK(t, i, j)                              \
  for (int t = tid; t < (k << 6); t += nt)              \
    if (const int j = t & 63, i = t >> 6; j < k)

// KQN = k / 4 (the kernel is instantiated per subspace width).
template <int KQN>
__global__ __launch_bounds__(RR_THREADS) void k_small_rr(double* __restrict__ small, int k, int r,
                                                  int lam_off, int filter, double jac_tol,
                                                  int oa_steps) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ld = k + 1;           // odd LDS row stride: column walks hit distinct banks
  double* B0 = sm;                // four k x ld matrices
  double* B1 = B0 + k * ld;
  double* B2 = B1 + k * ld;
  double* B3 = B2 + k * ld;
  double* d = B3 + k * ld;        // KMAX
  double* vals = d + KMAX;        // KMAX
  double* inv = vals + KMAX;      // KMAX
  double* mu = inv + KMAX;        // KMAX
  double* cs = mu + KMAX;         // 3 * (KMAX/2 + 1)
  double* red = cs + 3 * (KMAX / 2 + 1);   // RR_RED
  double* mu_r = red + RR_RED - 1;          // r-th largest mu (Newton path)
  int* perm = reinterpret_cast<int*>(red + RR_RED);
  int* flag = perm + KMAX;  // [0] dropped count, [1] jacobi
  int* imp = flag + 4;      // KMAX: pair importance on the Newton path
  const double* G = small + SL::GG;
  const double* T = small + SL::TG;
  const double* P = small + SL::PG;
  double* Sg = small + SL::S;     // coefficients (global, row stride KMAX)
  // 1. equilibrate: d_i = 1/sqrt(G_ii)
  for (int t = tid; t < k; t += nt) {
    const double g = G[t * k + t];
    d[t] = (g > 0.0) ? 1.0 / sqrt(g) : 1.0;
  }
  if (tid == 0) { flag[0] = 0; flag[1] = 0; }
  // phase clock (constant-rate counter, 100 MHz): start, Newton steps done,
  // Cholesky path done, projected matrix diagonalised, coefficients out
  unsigned long long tph[5];
  tph[0] = wall_clock64();
  __syncthreads();
  int sweeps = 0, path = -1;
  int why = 0;   // Cholesky path taken because: 1 G not orthonormal, 2 kept couplings, 3 tail bound
  int nsteps = 0;   // Newton steps taken
  double* Sbuf;   // sorted Ritz coefficients (k x ld)
  double* Pbuf;   // P (k x ld)
  double* Ybuf;   // P S (k x ld)
  // ---------------------------------------------------------- Newton path
  bool newton_ok = false;
  if (oa_steps > 0) {
    double* Gc = B0;
    double* Sc = B1;
    double* F = B2;
    double* Xc = B3;   // accumulated coefficients X (G-orthonormalising, diagonalising)
    kk_batched<4>(k,
        [&](int i, int j, double* v) {
          v[0] = G[i * k + j];
          v[1] = G[j * k + i];
          v[2] = T[i * k + j];
          v[3] = T[j * k + i];
        },
        [&](int i, int j, const double* v) {
          Gc[i * ld + j] = 0.5 * (v[0] + v[1]) * d[i] * d[j];
          Sc[i * ld + j] = 0.5 * (v[2] + v[3]) * d[i] * d[j];
          Xc[i * ld + j] = (i == j) ? 1.0 : 0.0;
        });
    __syncthreads();
    double offR = 1.0, offS = 1.0, smax = 1.0;
    // important pairs: those touching a positive value among the r largest.
    // Ranked once here from the starting values and once more for the
    // acceptance test (the steps keep the set).
    auto rank_important = [&]() {
      // eight lanes per value, each counting over every eighth competitor
      for (int t0 = 0; t0 < k; t0 += nt / 8) {
        const int t = t0 + (tid >> 3), part = tid & 7;
        const int tt = t < k ? t : k - 1;
        const double v = mu[tt];
        int rank = 0;
        for (int j = part; j < k; j += 8) rank += (mu[j] > v) || (mu[j] == v && j < tt);
        rank += __shfl_xor(rank, 1);
        rank += __shfl_xor(rank, 2);
        rank += __shfl_xor(rank, 4);
        if (t < k && part == 0) {
          imp[t] = (rank < r && v > 0.0) ? 1 : 0;
          if (rank == (r < k ? r : k) - 1) *mu_r = v;   // r-th largest
        }
      }
      __syncthreads();
    };
    for (int t = tid; t < k; t += nt) mu[t] = Sc[t * ld + t] / Gc[t * ld + t];
    __syncthreads();
    rank_important();
    // statistics of the starting matrices; later steps form them in the
    // epilogue of their products
    double aR = 0.0, aS = 0.0, mx = 0.0;
    RR_FOR_KK(t, i, j) {
      const double rij = ((i == j) ? 1.0 : 0.0) - Gc[i * ld + j];
      aR += rij * rij;
      if (i == j)
        mx = fmax(mx, fabs(mu[i]));
      else if (imp[i] || imp[j])
        aS += Sc[i * ld + j] * Sc[i * ld + j];
    }
    block_sum2_max1(aR, aS, mx, red);
    // G-orthonormality is needed to a level tied to the eigen-accuracy
    // target (it bounds the error of the factors), not to the last ulp; a
    // stagnating defect below 1e-12 is taken as converged as well.
    const double rtol = fmax(1e-13, 1e-3 * jac_tol);
    double offR_prev = 1.0, offS_prev = 1e308;
    int st = 0;
    for (;; ++st) {
      offR = sqrt(aR);
      offS = sqrt(aS);
      smax = fmax(mx, 1e-300);
      const bool rdone = offR <= rtol || (offR <= 1e-12 && offR > 0.25 * offR_prev);
      const bool conv = rdone && offS <= fmax(jac_tol, 1e-15) * smax;
      // couplings that no longer shrink (pairs too close for the Newton update)
      // within the acceptance level are left to the Jacobi rotations
      const bool stall = rdone && offS <= 1e-4 * smax && offS > 0.5 * offS_prev;
      if (conv || stall || st == oa_steps || !(offR < 0.5) || !isfinite(offS) || !isfinite(smax))
        break;
      offR_prev = offR;
      offS_prev = offS;
      const double delta = 2.0 * (offS + smax * offR);
      RR_FOR_KK(t, i, j) {
        const double rij = ((i == j) ? 1.0 : 0.0) - Gc[i * ld + j];
        double e = 0.5 * rij;
        const double gap = mu[j] - mu[i];
        const double num = Sc[i * ld + j] + mu[j] * rij;
        if (i != j && (imp[i] || imp[j]) && fabs(gap) > delta && fabs(num) <= 0.1 * fabs(gap))
          e = num / gap;
        F[i * ld + j] = ((i == j) ? 1.0 : 0.0) + e;
      }
      __syncthreads();
      newton_products<KQN>(Gc, Sc, F, Xc, ld, imp, red, aR, aS);
      // Rayleigh quotients of the new pairs; every wave forms max |mu| itself
      {
        const int lane = tid & 63;
        double v = 0.0;
        if (lane < k) {
          v = Sc[lane * ld + lane] / Gc[lane * ld + lane];
          if (tid < k) mu[lane] = v;
        }
        double a = fabs(v);
        for (int o = 32; o > 0; o >>= 1) a = fmax(a, __shfl_xor(a, o));
        mx = a;
      }
      __syncthreads();
    }
    newton_ok = offR <= fmax(1e-12, rtol) && offS <= 1e-4 * smax;
    if (!newton_ok) why = (offR <= fmax(1e-12, rtol)) ? 2 : 1;
    if (newton_ok) {
      // re-rank on the final values; the kept couplings are re-measured on
      // that set, and the unwanted tail, not diagonalised, may hide an
      // eigenvalue above the kept ones: Gershgorin bound of the tail block,
      // accepted only if no tail eigenvalue can exceed max(mu_(r), 0).
      rank_important();
      double aS = 0.0, z1 = 0.0, gb = 0.0;
      RR_FOR_KK(t, i, j) {
        if (i != j && (imp[i] || imp[j])) aS += Sc[i * ld + j] * Sc[i * ld + j];
      }
      for (int i0 = 0; i0 < k; i0 += nt / 8) {
        const int i = i0 + (tid >> 3), part = tid & 7;
        const int ii = i < k ? i : k - 1;
        double rad = 0.0;
        for (int j = part; j < k; j += 8)
          if (j != ii && !imp[j]) rad += fabs(Sc[ii * ld + j]);
        rad += __shfl_xor(rad, 1);
        rad += __shfl_xor(rad, 2);
        rad += __shfl_xor(rad, 4);
        if (i < k && part == 0 && !imp[i]) gb = fmax(gb, mu[i] + rad);
      }
      const double thr = fmax(*mu_r, 0.0);
      block_sum2_max1(aS, z1, gb, red);   // sum over the kept pairs, max(gb, 0) over the tail
      newton_ok = gb <= thr && sqrt(aS) <= 1e-4 * smax;
      if (!newton_ok) why = (gb <= thr) ? 2 : 3;
    }
    if (newton_ok) path = st;
    nsteps = st;
  }
  tph[1] = wall_clock64();
  // -------------------------------------------------------- Cholesky path
  if (!newton_ok) {
    double* L = B0;
    double* M = B1;
    double* U = B2;
    kk_batched<4>(k,
        [&](int i, int j, double* v) {
          v[0] = G[i * k + j];
          v[1] = G[j * k + i];
          v[2] = T[i * k + j];
          v[3] = T[j * k + i];
        },
        [&](int i, int j, const double* v) {
          const double tij = 0.5 * (v[2] + v[3]);
          const double gij = 0.5 * (v[0] + v[1]);
          L[i * ld + j] = gij * d[i] * d[j] + ((i == j) ? 1e-15 * k : 0.0);
          M[i * ld + j] = tij * d[i] * d[j];
        });
    __syncthreads();
    // Cholesky of the equilibrated G (lower, in L).  A column whose pivot
    // falls below 1e-14 (numerically dependent on the previous ones) is
    // dropped: L_jj = 1 with a zero sub-column, so its orthogonalised
    // direction is the tiny remainder and its Ritz value is ~0.
    {
      const int c = tid & 63, ty = tid >> 6, nty = nt >> 6;
      for (int j = 0; j < k; ++j) {
        const double piv = L[j * ld + j];
        const bool dropped = !(piv > 1e-14);
        const double ljj = dropped ? 1.0 : sqrt(piv);
        const double rl = 1.0 / ljj;
        for (int i = j + 1 + tid; i < k; i += nt) L[i * ld + j] = dropped ? 0.0 : L[i * ld + j] * rl;
        __syncthreads();
        if (tid == 0) {
          L[j * ld + j] = ljj;
          if (dropped) flag[0] += 1;
        }
        // trailing update of the lower triangle: lane c owns column c, the
        // waves split the rows i >= c
        if (c > j && c < k) {
          const double lcj = L[c * ld + j];
          for (int i = c + ty; i < k; i += nty) L[i * ld + c] -= L[i * ld + j] * lcj;
        }
        __syncthreads();
      }
    }
    // Tt = L^{-1} M L^{-T}: U = L^{-1} M column by column, then M = L^{-1} U^T.
    // Four lanes per column share each dot product (shuffle reduction).
    {
      const int c = tid >> 2, part = tid & 3;
      if (c < k) {
        for (int i = 0; i < k; ++i) {
          double sacc = 0.0;
          for (int j = part; j < i; j += 4) sacc += L[i * ld + j] * U[j * ld + c];
          sacc += __shfl_xor(sacc, 1);
          sacc += __shfl_xor(sacc, 2);
          const double v = (M[i * ld + c] - sacc) / L[i * ld + i];
          if (part == 0) U[i * ld + c] = v;
        }
      }
      __syncthreads();
      if (c < k) {
        for (int i = 0; i < k; ++i) {
          double sacc = 0.0;
          for (int j = part; j < i; j += 4) sacc += L[i * ld + j] * M[j * ld + c];
          sacc += __shfl_xor(sacc, 1);
          sacc += __shfl_xor(sacc, 2);
          const double v = (U[c * ld + i] - sacc) / L[i * ld + i];
          if (part == 0) M[i * ld + c] = v;
        }
      }
    }
    __syncthreads();
  }
  tph[2] = wall_clock64();
  // symmetrise the projected matrix (B1)
  RR_FOR_KK(t, i, j) {
    if (i < j) {
      const double v = 0.5 * (B1[i * ld + j] + B1[j * ld + i]);
      B1[i * ld + j] = v;
      B1[j * ld + i] = v;
    }
  }
  __syncthreads();
  // eigendecomposition of the projected matrix (B1, nearly diagonal on the
  // Newton path), eigenvectors in B2
  double* Aeig = B1;
  if (newton_ok)
    sweeps = jacobi_eig(B1, ld, B2, ld, k, cs, flag + 1, 40, jac_tol, true, imp);
  else   // B3 (free on this path) is the second buffer
    sweeps = jacobi_eig_db(B1, B3, ld, B2, ld, k, 40, jac_tol, red, &Aeig);
  sort_desc(Aeig, ld, k, vals, perm);
  tph[3] = wall_clock64();
  if (newton_ok) {
    // coefficients D X U[:, perm] into B0 (X^T G X is no longer needed)
    strip_mm(B0, ld, B3, ld, B2, ld, perm, d, k);
    __syncthreads();
    Sbuf = B0;
    Pbuf = B1;
    Ybuf = B3;
  } else {
    double* L = B0;
    double* M = B1;
    double* U = B2;
    // S = D L^{-T} U_sorted: back substitution per column into M (sorted
    // column order)
    {
      const int c = tid >> 2, part = tid & 3;
      if (c < k) {
        const int pc = perm[c];
        for (int i = k - 1; i >= 0; --i) {
          double sacc = 0.0;
          for (int j = i + 1 + part; j < k; j += 4) sacc += L[j * ld + i] * M[j * ld + c];
          sacc += __shfl_xor(sacc, 1);
          sacc += __shfl_xor(sacc, 2);
          const double v = (U[i * ld + pc] - sacc) / L[i * ld + i];
          if (part == 0) M[i * ld + c] = v;
        }
      }
    }
    __syncthreads();
    RR_FOR_KK(t, i, c) M[i * ld + c] *= d[i];
    __syncthreads();
    Sbuf = M;
    Pbuf = U;
    Ybuf = L;
  }
  // coefficients out; P into Pbuf for the residual product
  kk_batched<2>(k,
      [&](int i, int c, double* v) {
        v[0] = P[i * k + c];
        v[1] = P[c * k + i];
      },
      [&](int i, int c, const double* v) {
        Sg[i * KMAX + c] = Sbuf[i * ld + c];
        Pbuf[i * ld + c] = 0.5 * (v[0] + v[1]);
      });
  __syncthreads();
  // Y = P S (MFMA), then s_c^T P s_c = ||W v_c||^2.
  lds_mm(Ybuf, ld, Pbuf, ld, false, Sbuf, ld, k);
  __syncthreads();
  double* theta = small + SL::THETA;
  double* res = small + SL::RES;
  double scale = fmax(fabs(vals[0]), fabs(vals[k - 1]));
  if (!(scale > 0.0)) scale = 1.0;
  const double thk = vals[k - 1];
  double fc = 0.0, fe = 1.0;
  if (filter) {
    double lo = small[SL::SC + S_GERSH];
    if (!(lo < thk)) lo = thk - 0.5 * (vals[0] - thk) - 1e-300;
    fc = 0.5 * (lo + thk);
    fe = fmax(0.5 * (thk - lo), 1e-300);
    // A spectrum of zero width (e.g. W = 0 before the first step of a problem
    // with C = 0) gives no direction to amplify, and the predicted norms
    // below would underflow: use the neutral filter W + I, which keeps the
    // basis (and is harmless for the Chebyshev passes).
    if (!(vals[0] - lo > 1e-200)) {
      fc = -1.0;
      fe = 1.0;
    }
  }
  const double gam = filter ? fmax(fabs(vals[0] - fc), fe) : scale;
  double resc = 0.0;   // column tid's residual (k <= 64: wave 0 holds them all)
  for (int c = tid; c < k; c += nt) {
    const double sps = lds_dot(Sbuf + c, ld, Ybuf + c, ld, k);
    const double th = vals[c];
    theta[c] = th;
    resc = sqrt(fmax(sps - th * th, 0.0)) / scale;
    res[c] = resc;
    // column scale of the next basis: the predicted norm ||(W - cI) v|| (with
    // v^T W v = theta), floored at 1e-7 of the filter's largest amplification
    // (the prediction cancels below that level) so that no column is blown up
    // by rounding noise.
    const double nrm2 = filter ? (sps - 2.0 * fc * th + fc * fc) : sps;
    inv[c] = 1.0 / fmax(sqrt(fmax(nrm2, 0.0)), 1e-7 * gam);
  }
  __syncthreads();
  RR_FOR_KK(t, i, c) {
    const double sv = Sbuf[i * ld + c] * inv[c];
    small[SL::MZ + i * KMAX + c] = sv;
    small[SL::MB + i * KMAX + c] = -fc * sv;
  }
  if (tid < 64) {
    // wave 0, lane c = column c
    const int c = tid;
    const int rk = r < k ? r : k;
    // leading positive values among the r kept (values sorted decreasingly)
    const unsigned long long stop = __ballot(c < rk && !(vals[c < k ? c : 0] > 0.0));
    const int npos = stop ? (__ffsll((long long)stop) - 1) : rk;
    const int nchk = npos > 0 ? npos : (rk > 0 ? 1 : 0);
    double mr = (c < nchk) ? resc : 0.0;
    for (int o = 32; o > 0; o >>= 1) mr = fmax(mr, __shfl_xor(mr, o));
    if (c < rk) small[lam_off + c] = fmax(vals[c], 0.0);
    const bool bad = __ballot(c < k && !isfinite(vals[c < k ? c : 0])) != 0ull;
    if (c == 0) {
      double* sc = small + SL::SC;
      sc[S_MAXRES] = mr;
      sc[S_LAMR] = vals[rk - 1];
      sc[S_LAMR1] = (rk < k) ? vals[rk] : __builtin_nan("");
      sc[S_NORMW] = scale;
      sc[S_NPOS] = (double)npos;
      sc[S_FILTX1] = filter ? (vals[0] - fc) / fe : 0.0;
      sc[S_CHOLFIX] = (double)flag[0];
      sc[S_FILTC] = fc;
      sc[S_FILTE] = fe;
      sc[S_SWEEPS] = (double)sweeps;
      sc[S_RRPATH] = (double)path;
      sc[S_RRCHOL] += (path < 0) ? 1.0 : 0.0;
      if (why > 0) sc[S_RRWHY1 + why - 1] += 1.0;
      sc[S_RRSTEPS] += (double)nsteps;
      sc[S_RRCAP] += (nsteps >= oa_steps && oa_steps > 0) ? 1.0 : 0.0;
      if (newton_ok) sc[S_RRJSW] += (double)sweeps;
      tph[4] = wall_clock64();
      for (int ph = 0; ph < 4; ++ph) sc[S_RRT0 + ph] += 1e-8 * (double)(tph[ph + 1] - tph[ph]);
      sc[S_RRCOUNT] += 1.0;
      if (bad) sc[S_NONFINITE] = fmax(sc[S_NONFINITE], 1.0);
    }
  }
}
#undef RR_FOR_KK

// Sums the per-slice Gram partials [B^T B, B^T Z, Z^T Z] into the GG/TG/PG
// slots of `small`: SG_LANES lanes per entry, each summing every SG_LANES-th
// slice with SG_BATCH loads in flight, combined by a fixed butterfly (fixed
// summation order).
constexpr int SG_LANES = 8, SG_BATCH = 10;
__global__ __launch_bounds__(256) void k_sum_grams(const double* __restrict__ gram_part,
                                                   int nslices, int k, double* __restrict__ small) {
  const int kk = k * k;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = g / SG_LANES, part = g % SG_LANES;
  double acc = 0.0;
  if (t < 3 * kk) {
    for (int s0 = part; s0 < nslices; s0 += SG_LANES * SG_BATCH) {
      double v[SG_BATCH];
#pragma unroll
      for (int u = 0; u < SG_BATCH; ++u) {
        const int s = s0 + u * SG_LANES;
        v[u] = s < nslices ? gram_part[(int64_t)s * 3 * kk + t] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < SG_BATCH; ++u) acc += v[u];
    }
  }
#pragma unroll
  for (int o = 1; o < SG_LANES; o <<= 1) acc += __shfl_xor(acc, o);
  if (t < 3 * kk && part == 0) {
    const int which = t / kk;
    small[SL::GG + which * SL::kk + (t - which * kk)] = acc;
  }
}

// Exact eigendecomposition of the n x n W (n <= KMAX) in one workgroup; the
// top r eigenpairs become the factors (V row stride KMAX, lambda_+ at
// lam_off), and the factor partials of the single slice are formed as in
// k_rowwise (nslices = 1 downstream).
__global__ __launch_bounds__(1024) void k_full_eig(const double* __restrict__ W, int64_t ldw, int n,
                                                   double* __restrict__ V, int r,
                                                   const double* __restrict__ Vold, int r_old,
                                                   double* __restrict__ small, int lam_off,
                                                   int n_r1, const double* __restrict__ r1_u,
                                                   int npad, double* __restrict__ fac_part) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ld = n + 1;            // odd LDS stride
  double* A = sm;                  // n x ld
  double* U = A + n * ld;          // n x ld
  double* vals = U + n * ld;       // n
  double* cs = vals + n;           // 2 (n/2 + 1) + ints
  int* perm = reinterpret_cast<int*>(cs + 3 * (KMAX / 2 + 1));
  int* flag = perm + KMAX;
  for (int t = tid; t < n * n; t += nt) {
    const int i = t / n, j = t - (t / n) * n;
    A[i * (n + 1) + j] = 0.5 * (W[(int64_t)i * ldw + j] + W[(int64_t)j * ldw + i]);
  }
  __syncthreads();
  const int sweeps = jacobi_eig(A, ld, U, ld, n, cs, flag, 60);
  sort_desc(A, ld, n, vals, perm);
  // factors
  for (int t = tid; t < n * r; t += nt) {
    const int i = t / r, c = t - (t / r) * r;
    V[(int64_t)i * KMAX + c] = U[i * ld + perm[c]];
  }
  double* theta = small + SL::THETA;
  for (int c = tid; c < n; c += nt) {
    theta[c] = vals[c];
    small[SL::RES + c] = 0.0;
  }
  if (tid == 0) {
    for (int c = 0; c < r; ++c) small[lam_off + c] = fmax(vals[c], 0.0);
    double* sc = small + SL::SC;
    sc[S_MAXRES] = 0.0;
    sc[S_LAMR] = vals[r - 1];
    sc[S_LAMR1] = (r < n) ? vals[r] : __builtin_nan("");
    sc[S_NORMW] = fmax(fabs(vals[0]), fabs(vals[n - 1]));
    sc[S_SWEEPS] = (double)sweeps;
    bool bad = false;
    for (int c = 0; c < n; ++c) bad |= !isfinite(vals[c]);
    if (bad) sc[S_NONFINITE] = fmax(sc[S_NONFINITE], 2.0);
  }
  __syncthreads();
  // factor partials (single slice)
  const int n1 = r * r, n2 = r * r_old, n3 = n_r1 * r;
  for (int t = tid; t < n1 + n2 + n3; t += nt) {
    double acc = 0.0;
    if (t < n1) {
      const int a = t / r, b = t - (t / r) * r;
      for (int i = 0; i < n; ++i) acc += U[i * ld + perm[a]] * U[i * ld + perm[b]];
    } else if (t < n1 + n2) {
      const int e = t - n1;
      const int a = e / r_old, b = e - (e / r_old) * r_old;
      for (int i = 0; i < n; ++i) acc += U[i * ld + perm[a]] * Vold[(int64_t)i * KMAX + b];
    } else {
      const int e = t - n1 - n2;
      const int q = e / r, a = e - (e / r) * r;
      for (int i = 0; i < n; ++i) acc += r1_u[(int64_t)q * npad + i] * U[i * ld + perm[a]];
    }
    fac_part[t] = acc;
  }
  for (int c = tid; c < r; c += nt) fac_part[FAC_RES + c] = 0.0;
}

// True relative Ritz residuals ||W v_c - theta_c v_c|| / max|theta| of the r kept
// pairs from the row-wise partials; writes RES[c] and S_MAXRES (one workgroup).
__global__ void k_reduce_res(const double* __restrict__ fac_part, int nslices, int r,
                             double* __restrict__ small) {
  __shared__ double red[256];
  double worst = 0.0;
  const double scale = fmax(small[SL::SC + S_NORMW], 1e-300);
  const double* theta = small + SL::THETA;
  // leading positive values (one ballot of the first wave, shared through LDS)
  __shared__ int npos_s;
  if (threadIdx.x < 64) {
    const int ln = threadIdx.x;
    const unsigned long long stop = __ballot(ln < r && !(theta[ln < r ? ln : 0] > 0.0));
    if (ln == 0) npos_s = stop ? (__ffsll((long long)stop) - 1) : r;
  }
  __syncthreads();
  const int npos = npos_s;
  const int nchk = npos > 0 ? npos : (r > 0 ? 1 : 0);
  for (int c = threadIdx.x; c < r; c += blockDim.x) {
    double acc = 0.0;
    for (int s = 0; s < nslices; ++s) acc += fac_part[(int64_t)s * FAC_STRIDE + FAC_RES + c];
    const double rel = sqrt(acc) / scale;
    small[SL::RES + c] = rel;
    if (c < nchk) worst = fmax(worst, rel);
  }
  red[threadIdx.x] = worst;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) small[SL::SC + S_MAXRES] = red[0];
}

// Lower spectral bound for the filter from an unshifted block: the block has
// converged towards the largest-magnitude eigenvalues, so -1.05 max|theta|
// bounds the spectrum from below; the rigorous bound in S_GERSH is kept if larger.
__global__ void k_set_lower_bound(double* __restrict__ small) {
  if (threadIdx.x == 0) {
    double* sc = small + SL::SC;
    const double est = -1.05 * sc[S_NORMW];
    sc[S_GERSH] = fmax(sc[S_GERSH], est);
  }
}

// Reduces Gershgorin partial minima into small[S_GERSH] (one workgroup).
__global__ void k_reduce_min(const double* __restrict__ part, int cnt, double* __restrict__ small,
                             int slot) {
  __shared__ double red[256];
  double b = 1e308;
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) b = fmin(b, part[t]);
  red[threadIdx.x] = b;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) small[SL::SC + slot] = red[0];
}

}  // namespace proxsdp
