// Sparse kernels of the PDHG step.
//
// gather_dual  M(X+) from the factors X+ = V diag(lambda+) V^T, then the
//              dual step of Algorithm 1 in the Section 1.3 sign:
//                u = y + alpha (rhs - (2 M(X+) - M(X)))
//                y+ = u (equality rows),  y+ = min(0, u) (inequality rows)
//              (box resolvent of Section 2.3.1 through the Moreau identity),
//              and per-block sums for the dual residual of Section 2.2.
// pattern      values D_e = -alpha C_e + alpha M*(y+)_e on the sparsity
//              pattern (consumed by the dense write), the Gershgorin lower
//              bound of D and the sparse part of ||M*(y+ - y)||_F^2.
// finalize     combines the partial sums into eps_primal, eps_dual (Section
//              2.2), the objective and the iteration record.
#pragma once

#include "common.hpp"

namespace proxsdp {

__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = (blockDim.x + 63) >> 6;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// Sums of N values over the workgroup with one pair of barriers (each value
// in the same order as block_sum: wave butterfly, then the waves in order).
template <int N>
__device__ inline void block_sum_many(double* v, double* red) {
#pragma unroll
  for (int j = 0; j < N; ++j)
    for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_xor(v[j], o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < N; ++j) red[wave * N + j] = v[j];
  __syncthreads();
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w * N + j];
    v[j] = s;
  }
}

// Minima of two values over the workgroup with one pair of barriers.
__device__ inline void block_min2(double& a, double& b, double* red) {
  for (int o = 32; o > 0; o >>= 1) {
    a = fmin(a, __shfl_xor(a, o));
    b = fmin(b, __shfl_xor(b, o));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) {
    red[2 * wave] = a;
    red[2 * wave + 1] = b;
  }
  __syncthreads();
  a = 1e308;
  b = 1e308;
  for (int w = 0; w < nw; ++w) {
    a = fmin(a, red[2 * w]);
    b = fmin(b, red[2 * w + 1]);
  }
}

__device__ inline double block_min(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 1e308;
  const int nw = (blockDim.x + 63) >> 6;
  for (int w = 0; w < nw; ++w) s = fmin(s, red[w]);
  return s;
}

__global__ __launch_bounds__(256) void k_gather_dual(DevProblem dp, const double* __restrict__ V,
                                                     int r, double* __restrict__ small,
                                                     int lam_off, const double* __restrict__ fac_part,
                                                     int nslices, int r_old,
                                                     double* __restrict__ y,
                                                     double* __restrict__ y_old,
                                                     double* __restrict__ MX,
                                                     double* __restrict__ MX_old,
                                                     double* __restrict__ row_part) {
  __shared__ double red[16 * (1 + MAX_R1)];
  // reduce the factor partials over the slices for the finalisation:
  // [V^T V (r x r) | V^T Vold (r x r_old)] -> small[FR ..], residuals -> small[FR + FAC_RES ..]
  // (FR_LANES lanes per value, each summing every FR_LANES-th slice with
  // FR_BATCH loads in flight, then a fixed butterfly)
  {
    constexpr int FR_LANES = 8, FR_BATCH = 10;
    const int nfac = r * r + r * r_old;
    const int gsz = gridDim.x * blockDim.x;
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < (nfac + r) * FR_LANES; g += gsz) {
      const int t = g / FR_LANES, part = g % FR_LANES;
      const int src = (t < nfac) ? t : FAC_RES + (t - nfac);
      double acc = 0.0;
      for (int s0 = part; s0 < nslices; s0 += FR_LANES * FR_BATCH) {
        double v[FR_BATCH];
#pragma unroll
        for (int u = 0; u < FR_BATCH; ++u) {
          const int s = s0 + u * FR_LANES;
          v[u] = s < nslices ? fac_part[(int64_t)s * FAC_STRIDE + src] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < FR_BATCH; ++u) acc += v[u];
      }
#pragma unroll
      for (int o = 1; o < FR_LANES; o <<= 1) acc += __shfl_xor(acc, o);
      if (part == 0) small[SL::FR + src] = acc;
    }
  }
  const double* lam = small + lam_off;
  const double alpha = small[SL::SC + S_ALPHA];
  // ROW_LANES threads per row: each sums the factor columns t = sub (mod
  // ROW_LANES) of every entry of the row, then a shuffle reduction
  const int sub = threadIdx.x % ROW_LANES;
  const int i = blockIdx.x * ROWS_PER_BLOCK + threadIdx.x / ROW_LANES;
  double ed2 = 0.0, cross = 0.0, dobj = 0.0, bad = 0.0, ymx = 0.0;
  double mx = 0.0;
  // the row's old values, loaded with its entries
  const bool row_in = i < dp.rows;
  const double mx0 = row_in ? MX[i] : 0.0;
  const double y0 = row_in ? y[i] : 0.0;
  const double rhs_i = row_in ? dp.rhs[i] : 0.0;
  if (i < dp.rows) {
    for (int e = dp.row_ptr[i]; e < dp.row_ptr[i + 1]; ++e) {
      const double* va = V + (int64_t)dp.row_a[e] * KMAX;
      const double* vb = V + (int64_t)dp.row_b[e] * KMAX;
      double acc = 0.0;
      for (int t = sub; t < r; t += ROW_LANES) acc += lam[t] * va[t] * vb[t];
      mx += dp.row_w[e] * acc;
    }
    const int q = dp.row_r1[i];
    if (q >= 0) {
      // sigma_q u_q^T X+ u_q = sigma_q sum_t lam_t (u_q^T v_t)^2
      const int off = r * r + r * r_old + q * r;
      double acc = 0.0;
      for (int t = sub; t < r; t += ROW_LANES) {
        double uv = 0.0;
        for (int s = 0; s < nslices; ++s) uv += fac_part[(int64_t)s * FAC_STRIDE + off + t];
        acc += lam[t] * uv * uv;
      }
      mx += dp.r1_sigma[q] * acc;
    }
  }
  for (int o = ROW_LANES / 2; o > 0; o >>= 1) mx += __shfl_xor(mx, o);
  if (i < dp.rows && sub == 0) {
    double u = y0 + alpha * (rhs_i - (2.0 * mx - mx0));
    if (i >= dp.m) u = fmin(u, 0.0);
    const double dy = u - y0, dmx = mx - mx0;
    const double rd = dy / alpha + dmx;
    ed2 = rd * rd;
    cross = dmx * dy;
    dobj = rhs_i * u;
    ymx = y0 * mx;   // <y, M(X+)> with the y that built the projected matrix
    if (!isfinite(u) || !isfinite(mx)) bad = 1.0;
    y_old[i] = y0;
    y[i] = u;
    MX_old[i] = mx0;
    MX[i] = mx;
  }
  {
    double v[5] = {ed2, cross, dobj, bad, ymx};
    block_sum_many<5>(v, red);
    ed2 = v[0]; cross = v[1]; dobj = v[2]; bad = v[3]; ymx = v[4];
  }
  if (threadIdx.x == 0) {
    double* o = row_part + (int64_t)blockIdx.x * ROW_PART;
    o[0] = ed2; o[1] = cross; o[2] = dobj; o[3] = bad; o[4] = ymx;
  }
}

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// One wave per row a of the symmetric pattern (rows strided over the grid);
// lanes split the row's entries.
__global__ __launch_bounds__(256) void k_pattern(DevProblem dp, const double* __restrict__ y,
                                                 const double* __restrict__ y_old,
                                                 const double* __restrict__ small,
                                                 double* __restrict__ dval,
                                                 double* __restrict__ pat_part) {
  __shared__ double red[16 * (1 + MAX_R1)];
  const double alpha = small[SL::SC + S_ALPHA];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double lo = 1e308, lo2 = 1e308, mdy2 = 0.0;
  double crossq[MAX_R1];
  for (int q = 0; q < MAX_R1; ++q) crossq[q] = 0.0;
  for (int a = blockIdx.x * 4 + wave; a < dp.n; a += gridDim.x * 4) {
    double center = 0.0, radius = 0.0, center2 = 0.0, radius2 = 0.0;
    const int s0 = dp.sym_ptr[a], s1 = dp.sym_ptr[a + 1];
    for (int s = s0 + lane; s < s1; s += 64) {
      // the slot's copies of its entry's data: one contiguous read per field
      const int e = dp.sym_e[s];
      const int other = dp.slot_other[s];
      const int i0 = dp.slot_row0[s];
      const int t1 = dp.slot_t1[s];
      const double v0 = dp.slot_val0[s];
      const double cv = dp.slot_c[s];
      double my = 0.0, md = 0.0;
      if (i0 >= 0) {
        const double yi = y[i0];
        my += alpha * yi * v0;
        md += (yi - y_old[i0]) * v0;
        for (int t = dp.slot_t0[s] + 1; t < t1; ++t) {
          const int i = dp.pat_row[t];
          const double v = dp.pat_val[t];
          const double yt = y[i];
          my += alpha * yt * v;
          md += (yt - y_old[i]) * v;
        }
      }
      const double dv = -alpha * cv + my;
      const bool diag = other == a;
      if (diag) {
        center += dv;
        center2 += my;
      } else {
        radius += fabs(dv);
        radius2 += fabs(my);
      }
      if (a <= other) {  // owner of the entry (its smaller index)
        dval[e] = dv;
        const double w = diag ? 1.0 : 2.0;
        mdy2 += w * md * md;
        for (int q = 0; q < dp.n_r1; ++q)
          crossq[q] += w * md * dp.r1_u[(int64_t)q * dp.npad + a] * dp.r1_u[(int64_t)q * dp.npad + other];
      }
    }
    center = wave_sum(center);
    radius = wave_sum(radius);
    center2 = wave_sum(center2);
    radius2 = wave_sum(radius2);
    lo = fmin(lo, center - radius);
    lo2 = fmin(lo2, center2 - radius2);
  }
  block_min2(lo, lo2, red);
  {
    double v[1 + MAX_R1];
    v[0] = mdy2;
    for (int q = 0; q < MAX_R1; ++q) v[1 + q] = crossq[q];
    block_sum_many<1 + MAX_R1>(v, red);
    mdy2 = v[0];
    for (int q = 0; q < MAX_R1; ++q) crossq[q] = v[1 + q];
  }
  if (threadIdx.x == 0) {
    double* o = pat_part + (int64_t)blockIdx.x * PAT_PART;
    o[0] = lo; o[1] = mdy2; o[2] = lo2; o[3] = 0.0;
    for (int q = 0; q < MAX_R1; ++q) o[4 + q] = crossq[q];
  }
}

// Number of leading positive values of v[0 .. r) (r <= 64), from one ballot
// of the wave (every wave of the caller computes it).
__device__ inline int leading_positive(const double* v, int r) {
  const int ln = threadIdx.x & 63;
  const unsigned long long stop = __ballot(ln < r && !(v[ln < r ? ln : 0] > 0.0));
  return stop ? (__ffsll((long long)stop) - 1) : r;
}

// Runs in one workgroup (the extra block of the dense write).
//   ||X+ - X||^2 = ||X+||^2 + ||X||^2 - 2 <X+, X> from the factor Grams,
//   eps_p^2 = ||dX||^2 / alpha^2 + (2/alpha) <M(dX), dy> + ||M*(dy)||^2,
//   eps_d^2 = sum (dy/alpha + M(dX))^2     (Section 2.2, sign of Section 1.3).
// The objective <C, X+> comes from the projected matrix W = X - alpha (C -
// M*(y)): X+ = V diag(lambda) V^T with v_t^T W v_t = theta_t (Rayleigh-Ritz,
// or the exact eigenpairs), so <W, X+> = sum_t lambda_t theta_t and
//   <C, X+> = (<X, X+> + alpha <y, M(X+)> - sum_t lambda_t theta_t) / alpha,
// with <X, X+> from the factor Grams and <y, M(X+)> from the dual step.
__device__ void finalize_iteration(const FinArgs& f, double* small, const DevProblem& dp,
                                   const double* y, const double* y_old, double* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const double* lam = small + f.lam_new;
  const double* lam0 = small + f.lam_old;
  const int r = f.r, r0 = f.r_old;
  double x2 = 0.0, x01 = 0.0;
  const double* fr = small + SL::FR;   // slice sums formed by the dual-step kernel
  // both iterates' lambdas in LDS after the reduction scratch (`red` holds at
  // least 32 KB); the factor Gram entries are loaded FB at a time per thread
  double* lam_s = red + 16 * (9 + MAX_R1);
  double* lam0_s = lam_s + KMAX;
  for (int t = tid; t < 2 * KMAX; t += nt) {
    if (t < KMAX) lam_s[t] = t < r ? lam[t] : 0.0;
    else lam0_s[t - KMAX] = (t - KMAX < r0) ? lam0[t - KMAX] : 0.0;
  }
  __syncthreads();
  {
    constexpr int FB = 8;
    const int nf = r * r + r * r0;
    for (int t0 = tid; t0 < nf; t0 += FB * nt) {
      double g[FB];
#pragma unroll
      for (int u = 0; u < FB; ++u) {
        const int t = t0 + u * nt;
        g[u] = t < nf ? fr[t] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < FB; ++u) {
        const int t = t0 + u * nt;
        if (t >= nf) continue;
        if (t < r * r) {
          const int a = t / r, b = t - (t / r) * r;
          x2 += lam_s[a] * lam_s[b] * g[u] * g[u];
        } else {
          const int e = t - r * r;
          const int a = e / r0, b = e - (e / r0) * r0;
          x01 += lam_s[a] * lam0_s[b] * g[u] * g[u];
        }
      }
    }
  }
  // block partials of the dual step and of the pattern kernel, PB blocks per
  // thread loaded before any is added
  constexpr int PB = 4;
  double ed2 = 0.0, cross = 0.0, dobj = 0.0, bad = 0.0, ymx = 0.0;
  for (int b0 = tid; b0 < f.nrow_blocks; b0 += PB * nt) {
    double o[PB][ROW_PART];
#pragma unroll
    for (int u = 0; u < PB; ++u)
#pragma unroll
      for (int j = 0; j < ROW_PART; ++j)
        o[u][j] = (b0 + u * nt < f.nrow_blocks) ? f.row_part[(int64_t)(b0 + u * nt) * ROW_PART + j] : 0.0;
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      ed2 += o[u][0]; cross += o[u][1]; dobj += o[u][2]; bad += o[u][3]; ymx += o[u][4];
    }
  }
  double lo = 1e308, lo2 = 1e308, mdy2 = 0.0, lth = 0.0;
  double cq[MAX_R1];
  for (int q = 0; q < MAX_R1; ++q) cq[q] = 0.0;
  for (int b0 = tid; b0 < f.npat_blocks; b0 += PB * nt) {
    double o[PB][PAT_PART];
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      const bool in = b0 + u * nt < f.npat_blocks;
#pragma unroll
      for (int j = 0; j < PAT_PART; ++j)
        o[u][j] = in ? f.pat_part[(int64_t)(b0 + u * nt) * PAT_PART + j] : ((j == 0 || j == 2) ? 1e308 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < PB; ++u) {
      lo = fmin(lo, o[u][0]); mdy2 += o[u][1]; lo2 = fmin(lo2, o[u][2]);
      for (int q = 0; q < MAX_R1; ++q) cq[q] += o[u][4 + q];
    }
  }
  for (int t = tid; t < r; t += nt) lth += lam_s[t] * small[SL::THETA + t];
  {
    double v[9 + MAX_R1] = {x2, x01, ed2, cross, dobj, bad, ymx, lth, mdy2};
    for (int q = 0; q < MAX_R1; ++q) v[9 + q] = cq[q];
    block_sum_many<9 + MAX_R1>(v, red);
    x2 = v[0]; x01 = v[1]; ed2 = v[2]; cross = v[3]; dobj = v[4]; bad = v[5];
    ymx = v[6]; lth = v[7]; mdy2 = v[8];
    for (int q = 0; q < MAX_R1; ++q) cq[q] = v[9 + q];
  }
  block_min2(lo, lo2, red);
  // true Ritz residuals of the kept pairs (row-wise partials of the final round)
  double worst = 0.0;
  {
    const double scale = fmax(small[SL::SC + S_NORMW], 1e-300);
    const int npos = leading_positive(small + SL::THETA, r);
    const int nchk = npos > 0 ? npos : (r > 0 ? 1 : 0);
    for (int c = tid; c < nchk; c += nt) worst = fmax(worst, sqrt(fr[FAC_RES + c]) / scale);
    for (int o = 32; o > 0; o >>= 1) worst = fmax(worst, __shfl_xor(worst, o));
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = worst;
    __syncthreads();
    const int nw = (nt + 63) >> 6;
    for (int w = 0; w < nw; ++w) worst = fmax(worst, red[w]);
  }
  if (tid == 0) {
    double* sc = small + SL::SC;
    // every scalar this tail reads, loaded before its first store
    const double alpha = sc[S_ALPHA];
    const double x2old = sc[f.x2_old];
    const double lam_r = sc[S_LAMR], lam_r1 = sc[S_LAMR1], normw = sc[S_NORMW];
    const double npos_rr = sc[S_NPOS], filt_x1 = sc[S_FILTX1], nonfinite = sc[S_NONFINITE];
    const double iter = sc[S_ITER];
    sc[S_MAXRES] = worst;
    const double dx2 = fmax(x2 + x2old - 2.0 * x01, 0.0);
    // rank-one part of M*(dy)
    double my2 = mdy2;
    double gamma_lo = 0.0;
    for (int q = 0; q < dp.n_r1; ++q) {
      const int rq = dp.r1_row[q];
      const double dyq = y[rq] - y_old[rq];
      my2 += 2.0 * dp.r1_sigma[q] * dyq * cq[q];
      for (int q2 = 0; q2 < dp.n_r1; ++q2) {
        const int rq2 = dp.r1_row[q2];
        my2 += dp.r1_sigma[q] * dp.r1_sigma[q2] * dyq * (y[rq2] - y_old[rq2]) *
               dp.r1_gram[q * MAX_R1 + q2];
      }
      gamma_lo += fmin(0.0, alpha * dp.r1_sigma[q] * y[rq] * dp.r1_norm2[q]);
    }
    const double ep2 = dx2 / (alpha * alpha) + 2.0 * cross / alpha + my2;
    const double eps_p = sqrt(fmax(ep2, 0.0));
    const double eps_d = sqrt(fmax(ed2, 0.0));
    const double obj = (x01 + alpha * ymx - lth) / alpha;
    sc[f.x2_new] = x2;
    sc[S_EPSP] = eps_p;
    sc[S_EPSD] = eps_d;
    sc[S_OBJ] = obj;
    sc[S_DOBJ] = dobj;
    sc[S_DX2] = dx2;
    // lower bound of lambda_min(W) (X+ is PSD): Gershgorin of D, or Weyl with
    // lambda_max(C) <= ||C||_F and Gershgorin of alpha M*(y) -- the second is
    // far tighter for a dense C
    sc[S_GERSH] = fmax(lo, -alpha * dp.norm_c + lo2) + gamma_lo;
    double nf = nonfinite;
    if (bad > 0.0) nf = fmax(nf, 3.0);
    if (!isfinite(eps_p) || !isfinite(eps_d)) nf = fmax(nf, 4.0);
    if (nf != nonfinite) sc[S_NONFINITE] = nf;
    IterRecord rec;
    rec.eps_p = eps_p;
    rec.eps_d = eps_d;
    rec.obj = obj;
    rec.dual_obj = dobj;
    rec.lambda_r = lam_r;
    rec.lambda_r1 = lam_r1;
    rec.maxres = worst;
    rec.normw = normw;
    rec.npos = npos_rr;
    rec.filt_x1 = filt_x1;
    // ring slot: given (set-up record) or the device iteration counter, so
    // that a captured round of iterations can be replayed
    int slot = f.ring_slot;
    if (slot < 0) {
      slot = (int)iter % RING;
      sc[S_ITER] = iter + 1.0;
    }
    f.ring[slot] = rec;
  }
}

}  // namespace proxsdp
