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
__device__ inline int rr_player(int pos, int rnd, int kk) {
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
__device__ int jacobi_eig(double* A, int lda, double* U, int ldu, int k, double* cs, int* flag,
                          int max_sweeps, double tol_off = 1e-15) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int t = tid; t < k * k; t += nt) {
    const int i = t / k, j = t - (t / k) * k;
    U[i * ldu + j] = (i == j) ? 1.0 : 0.0;
  }
  const int kk = (k & 1) ? k + 1 : k;
  const int np = kk / 2;
  double* cc = cs;
  double* ss = cs + np;
  int* pp = reinterpret_cast<int*>(cs + 2 * np);
  int* qq = pp + np;
  int sweeps = 0;
  __shared__ double offd[2];
  for (int sw = 0; sw < max_sweeps; ++sw) {
    // convergence test on the off-diagonal mass
    if (tid == 0) { offd[0] = 0.0; offd[1] = 0.0; *flag = 0; }
    __syncthreads();
    double off = 0.0, dg = 0.0;
    for (int t = tid; t < k * k; t += nt) {
      const int i = t / k, j = t - (t / k) * k;
      const double v = A[i * lda + j];
      if (i == j) dg += v * v; else off += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      dg += __shfl_xor(dg, o);
    }
    if ((tid & 63) == 0) {
      atomicAdd(&offd[0], off);
      atomicAdd(&offd[1], dg);
    }
    __syncthreads();
    if (!(offd[0] > tol_off * tol_off * offd[1]) || !(offd[0] > 1e-300)) break;
    for (int rnd = 0; rnd < kk - 1; ++rnd) {
      for (int i = tid; i < np; i += nt) {
        int p = rr_player(i, rnd, kk), q = rr_player(kk - 1 - i, rnd, kk);
        if (p > q) { const int t = p; p = q; q = t; }
        double c = 1.0, s = 0.0;
        if (q < k) {
          const double app = A[p * lda + p], aqq = A[q * lda + q], apq = A[p * lda + q];
          const double thr = 1e-18 * sqrt(fabs(app * aqq)) + 1e-300;
          if (fabs(apq) > thr) {
            const double th = (aqq - app) / (2.0 * apq);
            const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        cc[i] = c; ss[i] = s; pp[i] = p; qq[i] = (q < k) ? q : -1;
      }
      __syncthreads();
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

// Sorts eigenvalues (diagonal of A) decreasingly: writes values to `vals`
// and the permutation to `perm`.  Rank sort: thread i counts the entries that
// precede it (larger, or equal with a smaller index), k <= KMAX.
__device__ void sort_desc(const double* A, int lda, int k, double* vals, int* perm) {
  // identity first, so that a non-finite value (flagged elsewhere) can only
  // leave a valid index behind
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    vals[i] = A[i * lda + i];
    perm[i] = i;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += blockDim.x) {
    const double v = A[i * lda + i];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double u = A[j * lda + j];
      rank += (u > v) || (u == v && j < i);
    }
    if (rank < k) {
      vals[rank] = v;
      perm[rank] = i;
    }
  }
  __syncthreads();
}

// Rayleigh-Ritz on span(B) from the reduced Grams G = B^T B, T = B^T W B,
// P = (W B)^T (W B).  Generalised problem T s = theta G s through a Cholesky
// factor of the column-equilibrated G (one CholeskyQR step folded into RR).
// Writes (small): S (k x k, V = B S with V^T V = I), THETA (decreasing), RES
// (relative Ritz residuals ||W v - theta v|| / max|theta|), lambda_+ of the r
// kept pairs at lam_off, S_LAMR/S_LAMR1/S_MAXRES/S_NORMW, and the next-basis
// coefficients MZ, MB of the degree-one Chebyshev filter
//   Bn_i = (W - c I) v_i / ||(W - c I) v_i||,  c = (lo + theta_k) / 2,
// where lo = small[S_GERSH] bounds the spectrum from below (filter != 0;
// filter == 0 gives Bn_i = W v_i / ||W v_i||).
// LDS: 3 k x k matrices (L, Tt, U) + vectors.
// Dot product of length n over LDS with four independent accumulators
// (keeps several LDS loads in flight).
__device__ inline double lds_dot(const double* a, int sa, const double* b, int sb, int n) {
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

__global__ __launch_bounds__(256) void k_small_rr(double* __restrict__ small, int k, int r,
                                                  int lam_off, int filter, double jac_tol) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x, nt = blockDim.x;
  const int kk = k * k;
  const int ld = k + 1;           // odd LDS row stride: column walks hit distinct banks
  double* L = sm;                 // k x ld
  double* M = L + k * ld;         // k x ld
  double* U = M + k * ld;         // k x ld
  double* d = U + k * ld;         // KMAX
  double* vals = d + KMAX;        // KMAX
  double* inv = vals + KMAX;      // KMAX
  double* cs = inv + KMAX;        // 3 * (KMAX/2 + 1)
  int* perm = reinterpret_cast<int*>(cs + 3 * (KMAX / 2 + 1));
  int* flag = perm + KMAX;  // [0] dropped count, [1] jacobi
  const double* G = small + SL::GG;
  const double* T = small + SL::TG;
  const double* P = small + SL::PG;
  // 1. equilibrate: d_i = 1/sqrt(G_ii); L = D G D (+ shift), M = D T D (symmetrised)
  for (int t = tid; t < k; t += nt) {
    const double g = G[t * k + t];
    d[t] = (g > 0.0) ? 1.0 / sqrt(g) : 1.0;
  }
  if (tid == 0) { flag[0] = 0; flag[1] = 0; }
  __syncthreads();
  for (int t = tid; t < kk; t += nt) {
    const int i = t / k, j = t - (t / k) * k;
    const double tij = 0.5 * (T[i * k + j] + T[j * k + i]);
    const double gij = 0.5 * (G[i * k + j] + G[j * k + i]);
    L[i * ld + j] = gij * d[i] * d[j] + ((i == j) ? 1e-15 * k : 0.0);
    M[i * ld + j] = tij * d[i] * d[j];
  }
  __syncthreads();
  // 2. Cholesky of the equilibrated G (lower, in L).  A column whose pivot
  //    falls below 1e-14 (numerically dependent on the previous ones) is
  //    dropped: L_jj = 1 with a zero sub-column, so its orthogonalised
  //    direction is the tiny remainder and its Ritz value is ~0.
  for (int j = 0; j < k; ++j) {
    const double piv = L[j * ld + j];
    const bool dropped = !(piv > 1e-14);
    const double ljj = dropped ? 1.0 : sqrt(piv);
    for (int i = j + 1 + tid; i < k; i += nt) L[i * ld + j] = dropped ? 0.0 : L[i * ld + j] / ljj;
    __syncthreads();
    if (tid == 0) {
      L[j * ld + j] = ljj;
      if (dropped) flag[0] += 1;
    }
    // trailing update of the lower triangle (i >= c > j), four entries per batch
    const int rem = k - 1 - j;
    for (int t0 = tid; t0 < rem * rem; t0 += 4 * nt) {
      double lij[4], lcj[4], lic[4];
      int pos[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + u * nt;
        const int i = j + 1 + t / rem, c = j + 1 + (t - (t / rem) * rem);
        const bool on = t < rem * rem && c <= i;
        pos[u] = on ? i * ld + c : -1;
        lij[u] = on ? L[i * ld + j] : 0.0;
        lcj[u] = on ? L[c * ld + j] : 0.0;
        lic[u] = on ? L[i * ld + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (pos[u] >= 0) L[pos[u]] = lic[u] - lij[u] * lcj[u];
    }
    __syncthreads();
  }
  // 3. Tt = L^{-1} M L^{-T}: U = L^{-1} M column by column, then M = L^{-1} U^T.
  //    Four lanes per column share each dot product (shuffle reduction).
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
  for (int t = tid; t < kk; t += nt) {
    const int i = t / k, j = t - (t / k) * k;
    if (i < j) {
      const double v = 0.5 * (M[i * ld + j] + M[j * ld + i]);
      M[i * ld + j] = v;
      M[j * ld + i] = v;
    }
  }
  __syncthreads();
  // 4. eigendecomposition of Tt
  const int sweeps = jacobi_eig(M, ld, U, ld, k, cs, flag + 1, 40, jac_tol);
  sort_desc(M, ld, k, vals, perm);
  // 5. S = D L^{-T} U_sorted: back substitution per column (into L's upper
  //    part is not possible: write into M, sorted column order)
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
  double* S = small + SL::S;
  for (int t = tid; t < kk; t += nt) {
    const int i = t / k, c = t - (t / k) * k;
    const double v = d[i] * M[i * ld + c];
    M[i * ld + c] = v;             // M now holds S
    S[i * KMAX + c] = v;
  }
  // P into U (LDS) for the residual product
  for (int t = tid; t < kk; t += nt) {
    const int i = t / k, j = t - (t / k) * k;
    U[i * ld + j] = 0.5 * (P[i * k + j] + P[j * k + i]);
  }
  __syncthreads();
  // 6. Y = P S (into L) on MFMA f64 16x16x4, then s_c^T P s_c = ||W v_c||^2.
  {
    typedef double d4v __attribute__((ext_vector_type(4)));
    const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    const int m = lane & 15, kq = lane >> 4, kb = k / 16;
    for (int blk = wave; blk < kb * kb; blk += nw) {
      const int a0 = (blk / kb) * 16, b0 = (blk - (blk / kb) * kb) * 16;
      d4v acc = {0.0, 0.0, 0.0, 0.0};
      for (int q0 = 0; q0 < k; q0 += 4) {
        const double av = U[(a0 + m) * ld + q0 + kq];
        const double bv = M[(q0 + kq) * ld + b0 + m];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) L[(a0 + kq + 4 * v) * ld + b0 + m] = acc[v];
    }
  }
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
  }
  const double gam = filter ? fmax(fabs(vals[0] - fc), fe) : scale;
  for (int c = tid; c < k; c += nt) {
    const double sps = lds_dot(M + c, ld, L + c, ld, k);
    const double th = vals[c];
    theta[c] = th;
    res[c] = sqrt(fmax(sps - th * th, 0.0)) / scale;
    // column scale of the next basis: the predicted norm ||(W - cI) v|| (with
    // v^T W v = theta), floored at 1e-7 of the filter's largest amplification
    // (the prediction cancels below that level) so that no column is blown up
    // by rounding noise.
    const double nrm2 = filter ? (sps - 2.0 * fc * th + fc * fc) : sps;
    inv[c] = 1.0 / fmax(sqrt(fmax(nrm2, 0.0)), 1e-7 * gam);
  }
  __syncthreads();
  for (int t = tid; t < kk; t += nt) {
    const int i = t / k, c = t - (t / k) * k;
    const double sv = M[i * ld + c] * inv[c];
    small[SL::MZ + i * KMAX + c] = sv;
    small[SL::MB + i * KMAX + c] = -fc * sv;
  }
  if (tid == 0) {
    double mr = 0.0;
    const int rk = r < k ? r : k;
    int npos = 0;
    while (npos < rk && vals[npos] > 0.0) ++npos;
    const int nchk = npos > 0 ? npos : (rk > 0 ? 1 : 0);
    for (int c = 0; c < nchk; ++c) mr = fmax(mr, res[c]);
    for (int c = 0; c < rk; ++c) small[lam_off + c] = fmax(vals[c], 0.0);
    double* sc = small + SL::SC;
    sc[S_MAXRES] = mr;
    sc[S_LAMR] = vals[rk - 1];
    sc[S_LAMR1] = (rk < k) ? vals[rk] : __builtin_nan("");
    sc[S_NORMW] = scale;
    sc[S_CHOLFIX] = (double)flag[0];
    sc[S_FILTC] = fc;
    sc[S_FILTE] = fe;
    sc[S_SWEEPS] = (double)sweeps;
    bool bad = false;
    for (int c = 0; c < k; ++c) bad |= !isfinite(vals[c]);
    if (bad) sc[S_NONFINITE] = fmax(sc[S_NONFINITE], 1.0);
  }
}

// Sums the per-slice Gram partials [B^T B, B^T Z, Z^T Z] into the GG/TG/PG
// slots of `small` (one thread per entry, fixed summation order).
__global__ __launch_bounds__(256) void k_sum_grams(const double* __restrict__ gram_part,
                                                   int nslices, int k, double* __restrict__ small) {
  const int kk = k * k;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 3 * kk) return;
  double acc = 0.0;
#pragma unroll 8
  for (int s = 0; s < nslices; ++s) acc += gram_part[(int64_t)s * 3 * kk + t];
  const int which = t / kk;
  small[SL::GG + which * SL::kk + (t - which * kk)] = acc;
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
  int npos = 0;
  while (npos < r && theta[npos] > 0.0) ++npos;
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
