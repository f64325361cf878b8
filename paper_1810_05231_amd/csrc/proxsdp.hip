// libproxsdp: host side of the C interface declared in include/proxsdp.h.
//
// One process drives one GPU.  The host validates and preprocesses the
// problem once (create), then enqueues the per-iteration kernel schedule on
// the caller's stream and only synchronises at control checks (every
// `check_every` iterations), where it applies the rank control of
// Algorithm 2 (Section 3.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <tuple>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include "../../include/proxsdp.h"
#include "common.hpp"
#include "dense.hpp"
#include "rounding.hpp"
#include "small.hpp"
#include "sparse.hpp"

using namespace proxsdp;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_OK(expr)                                                                 \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(PROXSDP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline int roundup(int x, int m) { return (x + m - 1) / m * m; }
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// --------------------------------------------------------------- preprocessing
struct Host {
  int n = 0, npad = 0, m = 0, p = 0, rows = 0;
  std::vector<int> pat_a, pat_b;
  std::vector<double> pat_c;
  std::vector<int> pat_rptr, pat_row;
  std::vector<double> pat_val;
  std::vector<int> row_ptr, row_a, row_b;
  std::vector<double> row_w;
  std::vector<int> sym_ptr, sym_e;
  std::vector<int> slot_other, slot_t0, slot_t1, slot_row0;
  std::vector<double> slot_c, slot_val0;
  std::vector<int> tile_ptr, tile_item, tile_e;
  int n_r1 = 0;
  std::vector<int> r1_row;
  std::vector<double> r1_sigma, r1_u, r1_norm2, r1_gram;
  std::vector<int> row_r1;
  std::vector<double> rhs, scale;
  double norm_c = 0, norm_rhs = 0, norm_m = 0;
};

bool finite_all(const double* v, int64_t cnt) {
  for (int64_t i = 0; i < cnt; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

int validate(const proxsdp_problem* pb, const proxsdp_options* o) {
  if (!pb) return fail(PROXSDP_ERR_INVALID, "problem is NULL");
  if (pb->n < 1) return fail(PROXSDP_ERR_INVALID, "n must be >= 1");
  if (pb->m < 0 || pb->p < 0) return fail(PROXSDP_ERR_INVALID, "m and p must be >= 0");
  if (pb->m + pb->p < 1) return fail(PROXSDP_ERR_INVALID, "at least one constraint row required");
  if (pb->nnz_c < 0 || pb->nnz_a < 0 || pb->n_r1 < 0)
    return fail(PROXSDP_ERR_INVALID, "negative count");
  if (pb->nnz_c > 0 && (!pb->c_i || !pb->c_j || !pb->c_v))
    return fail(PROXSDP_ERR_INVALID, "C arrays are NULL");
  if (pb->nnz_a > 0 && (!pb->a_row || !pb->a_i || !pb->a_j || !pb->a_v))
    return fail(PROXSDP_ERR_INVALID, "constraint arrays are NULL");
  if (pb->m > 0 && !pb->b) return fail(PROXSDP_ERR_INVALID, "b is NULL");
  if (pb->p > 0 && !pb->h) return fail(PROXSDP_ERR_INVALID, "h is NULL");
  if (pb->n_r1 > MAX_R1)
    return fail(PROXSDP_ERR_UNSUPPORTED, "at most " + std::to_string(MAX_R1) + " rank-one terms");
  if (pb->n_r1 > 0 && (!pb->r1_row || !pb->r1_sigma || !pb->r1_u))
    return fail(PROXSDP_ERR_INVALID, "rank-one arrays are NULL");
  const int n = pb->n, rows = pb->m + pb->p;
  for (int64_t t = 0; t < pb->nnz_c; ++t) {
    const int i = pb->c_i[t], j = pb->c_j[t];
    if (i < 0 || j < 0 || i >= n || j >= n) return fail(PROXSDP_ERR_INVALID, "C index out of range");
    if (i > j) return fail(PROXSDP_ERR_INVALID, "C entry below the diagonal (need i <= j)");
  }
  for (int64_t t = 0; t < pb->nnz_a; ++t) {
    const int r = pb->a_row[t], i = pb->a_i[t], j = pb->a_j[t];
    if (r < 0 || r >= rows) return fail(PROXSDP_ERR_INVALID, "constraint row out of range");
    if (i < 0 || j < 0 || i >= n || j >= n)
      return fail(PROXSDP_ERR_INVALID, "constraint index out of range");
    if (i > j) return fail(PROXSDP_ERR_INVALID, "constraint entry below the diagonal (need i <= j)");
  }
  if (!finite_all(pb->c_v, pb->nnz_c) || !finite_all(pb->a_v, pb->nnz_a) ||
      !finite_all(pb->b, pb->m) || !finite_all(pb->h, pb->p))
    return fail(PROXSDP_ERR_INVALID, "non-finite problem data");
  std::vector<int> seen(rows, 0);
  for (int q = 0; q < pb->n_r1; ++q) {
    const int r = pb->r1_row[q];
    if (r < 0 || r >= rows) return fail(PROXSDP_ERR_INVALID, "rank-one row out of range");
    if (seen[r]++) return fail(PROXSDP_ERR_UNSUPPORTED, "at most one rank-one term per row");
    if (!std::isfinite(pb->r1_sigma[q]) || !finite_all(pb->r1_u + (int64_t)q * n, n))
      return fail(PROXSDP_ERR_INVALID, "non-finite rank-one data");
  }
  if (o) {
    if (!(o->tol > 0)) return fail(PROXSDP_ERR_INVALID, "tol must be > 0");
    if (o->check_every < 1 || o->window < o->check_every || o->window % o->check_every)
      return fail(PROXSDP_ERR_INVALID, "window must be a positive multiple of check_every");
    if (o->precision != PROXSDP_FP64 && o->precision != PROXSDP_FP32 && o->precision != PROXSDP_BF16 &&
        o->precision != PROXSDP_IMPLICIT)
      return fail(PROXSDP_ERR_INVALID,
                  "precision must be PROXSDP_FP64, PROXSDP_FP32, PROXSDP_BF16 or PROXSDP_IMPLICIT");
    if (o->alpha < 0) return fail(PROXSDP_ERR_INVALID, "alpha must be >= 0");
    if (o->full_eig && pb->n > KMAX)
      return fail(PROXSDP_ERR_UNSUPPORTED, "full_eig needs n <= " + std::to_string(KMAX));
    if (!(o->eig_rel > 0)) return fail(PROXSDP_ERR_INVALID, "eig_rel must be > 0");
    if (o->block && (o->block < 0 || o->block % 16 || o->block > KMAX))
      return fail(PROXSDP_ERR_INVALID, "block must be a multiple of 16 and <= 64");
    if (o->rank_test != PROXSDP_RANK_TEST_LAMBDA_R && o->rank_test != PROXSDP_RANK_TEST_LAMBDA_R_PLUS_1)
      return fail(PROXSDP_ERR_INVALID, "rank_test must be PROXSDP_RANK_TEST_LAMBDA_R or _PLUS_1");
  }
  return PROXSDP_OK;
}

// K y for the Gram operator K = M M* of the (scaled) rows, on the host.
struct GramOp {
  const Host& h;
  explicit GramOp(const Host& hh) : h(hh) {}
  void apply(const std::vector<double>& y, std::vector<double>& out) const {
    const int npat = (int)h.pat_a.size();
    std::vector<double> s(npat, 0.0);
    for (int e = 0; e < npat; ++e) {
      double acc = 0.0;
      for (int t = h.pat_rptr[e]; t < h.pat_rptr[e + 1]; ++t) acc += y[h.pat_row[t]] * h.pat_val[t];
      s[e] = acc;
    }
    std::vector<double> cq(h.n_r1);
    for (int q = 0; q < h.n_r1; ++q) cq[q] = h.r1_sigma[q] * y[h.r1_row[q]];
    const int np = h.npad;
    out.assign(h.rows, 0.0);
    // Sparse-sparse part through entry ids: iterate entries once.
    for (int e = 0; e < npat; ++e) {
      const double w = (h.pat_a[e] == h.pat_b[e]) ? 1.0 : 2.0;
      double rank1 = 0.0;
      for (int q = 0; q < h.n_r1; ++q)
        rank1 += cq[q] * h.r1_u[(size_t)q * np + h.pat_a[e]] * h.r1_u[(size_t)q * np + h.pat_b[e]];
      for (int t = h.pat_rptr[e]; t < h.pat_rptr[e + 1]; ++t)
        out[h.pat_row[t]] += w * h.pat_val[t] * (s[e] + rank1);
    }
    for (int q = 0; q < h.n_r1; ++q) {
      double acc = 0.0;
      for (int e = 0; e < npat; ++e) {
        const double w = (h.pat_a[e] == h.pat_b[e]) ? 1.0 : 2.0;
        acc += w * s[e] * h.r1_u[(size_t)q * np + h.pat_a[e]] * h.r1_u[(size_t)q * np + h.pat_b[e]];
      }
      for (int q2 = 0; q2 < h.n_r1; ++q2) acc += cq[q2] * h.r1_gram[q * MAX_R1 + q2];
      out[h.r1_row[q]] += h.r1_sigma[q] * acc;
    }
  }
};

// Largest eigenvalue of a symmetric tridiagonal matrix by bisection (Sturm count).
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int k = (int)a.size();
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_greater = [&](double x) {
    int c = 0;
    double d = 1.0;
    for (int i = 0; i < k; ++i) {
      const double bb = (i > 0) ? b[i - 1] * b[i - 1] : 0.0;
      d = (a[i] - x) - ((i > 0) ? bb / d : 0.0);
      if (d == 0.0) d = -1e-300;
      if (d > 0) ++c;
    }
    return c;  // number of eigenvalues > x
  };
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_greater(mid) > 0) lo = mid; else hi = mid;
    if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(hi))) break;
  }
  return hi;
}

// ||M||_2 = sqrt(lambda_max(K)) by Lanczos on K (no reorthogonalisation: the
// extreme Ritz value is unaffected by the loss of orthogonality).
double op_norm(const Host& h) {
  GramOp K(h);
  const int rows = h.rows;
  std::vector<double> v(rows), w, vprev(rows, 0.0);
  for (int i = 0; i < rows; ++i) v[i] = 1.0 + 0.5 * std::sin(1.0 + 0.37 * i);
  double nv = 0;
  for (double x : v) nv += x * x;
  nv = std::sqrt(nv);
  for (double& x : v) x /= nv;
  std::vector<double> al, be;
  double beta = 0.0, last = 0.0;
  const int steps = std::min(rows, 120);
  for (int it = 0; it < steps; ++it) {
    K.apply(v, w);
    double a = 0;
    for (int i = 0; i < rows; ++i) a += w[i] * v[i];
    for (int i = 0; i < rows; ++i) w[i] -= a * v[i] + beta * vprev[i];
    double b = 0;
    for (double x : w) b += x * x;
    b = std::sqrt(b);
    al.push_back(a);
    const double est = tridiag_max_eig(al, be);
    if (it > 5 && std::fabs(est - last) <= 1e-14 * std::fabs(est)) { last = est; break; }
    last = est;
    if (b <= 1e-14 * std::fabs(est)) break;
    be.push_back(b);
    vprev = v;
    for (int i = 0; i < rows; ++i) v[i] = w[i] / b;
    beta = b;
  }
  return std::sqrt(std::max(last, 0.0));
}

int preprocess(const proxsdp_problem* pb, int row_scaling, Host& h) {
  const int n = pb->n;
  h.n = n;
  h.npad = roundup(n, TILE);
  h.m = pb->m;
  h.p = pb->p;
  h.rows = pb->m + pb->p;
  // pattern keys
  struct Trip { int64_t key; int row; double v; };
  std::vector<Trip> ct(pb->nnz_c), at(pb->nnz_a);
  for (int64_t t = 0; t < pb->nnz_c; ++t)
    ct[t] = {(int64_t)pb->c_i[t] * n + pb->c_j[t], -1, pb->c_v[t]};
  for (int64_t t = 0; t < pb->nnz_a; ++t)
    at[t] = {(int64_t)pb->a_i[t] * n + pb->a_j[t], pb->a_row[t], pb->a_v[t]};
  std::vector<int64_t> keys;
  keys.reserve(ct.size() + at.size());
  for (auto& t : ct) keys.push_back(t.key);
  for (auto& t : at) keys.push_back(t.key);
  std::sort(keys.begin(), keys.end());
  keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
  const int npat = (int)keys.size();
  auto eid = [&](int64_t key) {
    return (int)(std::lower_bound(keys.begin(), keys.end(), key) - keys.begin());
  };
  h.pat_a.resize(npat);
  h.pat_b.resize(npat);
  h.pat_c.assign(npat, 0.0);
  for (int e = 0; e < npat; ++e) {
    h.pat_a[e] = (int)(keys[e] / n);
    h.pat_b[e] = (int)(keys[e] % n);
  }
  for (auto& t : ct) h.pat_c[eid(t.key)] += t.v;
  // (row, entry, v) merged
  struct RE { int row, e; double v; };
  std::vector<RE> re(at.size());
  for (size_t t = 0; t < at.size(); ++t) re[t] = {at[t].row, eid(at[t].key), at[t].v};
  std::sort(re.begin(), re.end(), [](const RE& x, const RE& y) {
    return x.row != y.row ? x.row < y.row : x.e < y.e;
  });
  std::vector<RE> mr;
  for (auto& x : re) {
    if (!mr.empty() && mr.back().row == x.row && mr.back().e == x.e) mr.back().v += x.v;
    else mr.push_back(x);
  }
  // rank-one terms
  h.n_r1 = pb->n_r1;
  h.r1_row.assign(pb->r1_row, pb->r1_row + h.n_r1);
  h.r1_sigma.assign(pb->r1_sigma, pb->r1_sigma + h.n_r1);
  h.r1_u.assign((size_t)std::max(h.n_r1, 1) * h.npad, 0.0);
  for (int q = 0; q < h.n_r1; ++q)
    for (int i = 0; i < n; ++i) h.r1_u[(size_t)q * h.npad + i] = pb->r1_u[(size_t)q * n + i];
  h.row_r1.assign(h.rows, -1);
  for (int q = 0; q < h.n_r1; ++q) h.row_r1[h.r1_row[q]] = q;
  // row norms ||M_i||_F
  h.scale.assign(h.rows, 0.0);
  std::vector<double> nrm2(h.rows, 0.0);
  for (auto& x : mr) {
    const double w = (h.pat_a[x.e] == h.pat_b[x.e]) ? 1.0 : 2.0;
    nrm2[x.row] += w * x.v * x.v;
  }
  h.r1_norm2.assign(MAX_R1, 0.0);
  for (int q = 0; q < h.n_r1; ++q) {
    double s = 0;
    for (int i = 0; i < n; ++i) s += h.r1_u[(size_t)q * h.npad + i] * h.r1_u[(size_t)q * h.npad + i];
    h.r1_norm2[q] = s;
    const int row = h.r1_row[q];
    const double sg = h.r1_sigma[q];
    double crossv = 0.0;
    for (auto& x : mr) {
      if (x.row != row) continue;
      const double w = (h.pat_a[x.e] == h.pat_b[x.e]) ? 1.0 : 2.0;
      crossv += w * x.v * h.r1_u[(size_t)q * h.npad + h.pat_a[x.e]] *
                h.r1_u[(size_t)q * h.npad + h.pat_b[x.e]];
    }
    nrm2[row] += 2.0 * sg * crossv + sg * sg * s * s;
  }
  for (int i = 0; i < h.rows; ++i) {
    if (!(nrm2[i] > 0.0)) return fail(PROXSDP_ERR_INVALID, "constraint row " + std::to_string(i) + " is zero");
    h.scale[i] = row_scaling ? std::sqrt(nrm2[i]) : 1.0;
  }
  for (auto& x : mr) x.v /= h.scale[x.row];
  for (int q = 0; q < h.n_r1; ++q) h.r1_sigma[q] /= h.scale[h.r1_row[q]];
  h.r1_gram.assign(MAX_R1 * MAX_R1, 0.0);
  for (int q = 0; q < h.n_r1; ++q)
    for (int q2 = 0; q2 < h.n_r1; ++q2) {
      double s = 0;
      for (int i = 0; i < n; ++i) s += h.r1_u[(size_t)q * h.npad + i] * h.r1_u[(size_t)q2 * h.npad + i];
      h.r1_gram[q * MAX_R1 + q2] = s * s;
    }
  h.rhs.resize(h.rows);
  for (int i = 0; i < h.m; ++i) h.rhs[i] = pb->b[i] / h.scale[i];
  for (int i = 0; i < h.p; ++i) h.rhs[h.m + i] = pb->h[i] / h.scale[h.m + i];
  // row -> entries
  h.row_ptr.assign(h.rows + 1, 0);
  for (auto& x : mr) h.row_ptr[x.row + 1]++;
  for (int i = 0; i < h.rows; ++i) h.row_ptr[i + 1] += h.row_ptr[i];
  h.row_a.resize(mr.size());
  h.row_b.resize(mr.size());
  h.row_w.resize(mr.size());
  for (size_t t = 0; t < mr.size(); ++t) {
    const int e = mr[t].e;
    h.row_a[t] = h.pat_a[e];
    h.row_b[t] = h.pat_b[e];
    h.row_w[t] = mr[t].v * ((h.pat_a[e] == h.pat_b[e]) ? 1.0 : 2.0);
  }
  // entry -> rows
  h.pat_rptr.assign(npat + 1, 0);
  for (auto& x : mr) h.pat_rptr[x.e + 1]++;
  for (int e = 0; e < npat; ++e) h.pat_rptr[e + 1] += h.pat_rptr[e];
  h.pat_row.resize(mr.size());
  h.pat_val.resize(mr.size());
  {
    std::vector<int> fill(h.pat_rptr.begin(), h.pat_rptr.end() - 1);
    for (auto& x : mr) {
      const int pos = fill[x.e]++;
      h.pat_row[pos] = x.row;
      h.pat_val[pos] = x.v;
    }
  }
  // symmetric rows of the pattern
  h.sym_ptr.assign(n + 1, 0);
  for (int e = 0; e < npat; ++e) {
    h.sym_ptr[h.pat_a[e] + 1]++;
    if (h.pat_a[e] != h.pat_b[e]) h.sym_ptr[h.pat_b[e] + 1]++;
  }
  for (int i = 0; i < n; ++i) h.sym_ptr[i + 1] += h.sym_ptr[i];
  h.sym_e.resize(h.sym_ptr[n]);
  {
    std::vector<int> fill(h.sym_ptr.begin(), h.sym_ptr.end() - 1);
    for (int e = 0; e < npat; ++e) {
      h.sym_e[fill[h.pat_a[e]]++] = e;
      if (h.pat_a[e] != h.pat_b[e]) h.sym_e[fill[h.pat_b[e]]++] = e;
    }
  }
  // per-slot copies of what the pattern kernels read for an entry (its other
  // index, C value, row range and first row), so that a row's slots are read
  // contiguously instead of through the entry index
  {
    const size_t ns = h.sym_e.size();
    h.slot_other.resize(ns);
    h.slot_t0.resize(ns);
    h.slot_t1.resize(ns);
    h.slot_row0.resize(ns);
    h.slot_c.resize(ns);
    h.slot_val0.resize(ns);
    for (int a = 0; a < n; ++a)
      for (int sl = h.sym_ptr[a]; sl < h.sym_ptr[a + 1]; ++sl) {
        const int e = h.sym_e[sl];
        h.slot_other[sl] = (h.pat_a[e] == a) ? h.pat_b[e] : h.pat_a[e];
        h.slot_c[sl] = h.pat_c[e];
        h.slot_t0[sl] = h.pat_rptr[e];
        h.slot_t1[sl] = h.pat_rptr[e + 1];
        const bool any = h.pat_rptr[e + 1] > h.pat_rptr[e];
        h.slot_row0[sl] = any ? h.pat_row[h.pat_rptr[e]] : -1;
        h.slot_val0[sl] = any ? h.pat_val[h.pat_rptr[e]] : 0.0;
      }
  }
  // tile lists of the mirrored pattern
  const int ts = h.npad / TILE;
  h.tile_ptr.assign((size_t)ts * ts + 1, 0);
  auto tile_of = [&](int a, int b) { return (a / TILE) * ts + (b / TILE); };
  for (int e = 0; e < npat; ++e) {
    h.tile_ptr[tile_of(h.pat_a[e], h.pat_b[e]) + 1]++;
    if (h.pat_a[e] != h.pat_b[e]) h.tile_ptr[tile_of(h.pat_b[e], h.pat_a[e]) + 1]++;
  }
  for (size_t t = 0; t + 1 < h.tile_ptr.size(); ++t) h.tile_ptr[t + 1] += h.tile_ptr[t];
  h.tile_item.resize(h.tile_ptr.back());
  h.tile_e.resize(h.tile_ptr.back());
  {
    std::vector<int> fill(h.tile_ptr.begin(), h.tile_ptr.end() - 1);
    auto put = [&](int a, int b, int e) {
      const int pos = fill[tile_of(a, b)]++;
      h.tile_item[pos] = ((a % TILE) << 8) | (b % TILE);
      h.tile_e[pos] = e;
    };
    for (int e = 0; e < npat; ++e) {
      put(h.pat_a[e], h.pat_b[e], e);
      if (h.pat_a[e] != h.pat_b[e]) put(h.pat_b[e], h.pat_a[e], e);
    }
  }
  // norms
  double nc = 0;
  for (int e = 0; e < npat; ++e) {
    const double w = (h.pat_a[e] == h.pat_b[e]) ? 1.0 : 2.0;
    nc += w * h.pat_c[e] * h.pat_c[e];
  }
  h.norm_c = std::sqrt(nc);
  double nr = 0;
  for (double v : h.rhs) nr += v * v;
  h.norm_rhs = std::sqrt(nr);
  h.norm_m = op_norm(h);
  if (!(h.norm_m > 0)) return fail(PROXSDP_ERR_INVALID, "constraint operator is zero");
  return PROXSDP_OK;
}

// ------------------------------------------------------------- workspace
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* b) : base(static_cast<char*>(b)) {}
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align256(off + std::max<size_t>(count, 1) * sizeof(T));
    return p;
  }
};

int k_for_r(int r) {
  int k = roundup(r + std::max(8, (r + 1) / 2), 16);
  return std::min(k, KMAX);
}

struct Chunking {
  int rows_per_chunk, nchunks;
};

// Row chunks of the dense pass: about 704 workgroups in total, ~2.75 per CU
// of the 256 (measured at n = 5000, k = 64 with 7 / 9 / 12 chunks: 93 / 86 /
// 90 us; the Gram reduction of the partials grows by ~1 us per chunk).
Chunking chunking(int npad) {
  const int cols = npad / 64;
  const int steps = npad / 64;
  const int c = std::min(std::max(1, (704 + cols / 2) / cols), steps);
  const int R = ((steps + c - 1) / c) * 64;
  return {R, (npad + R - 1) / R};
}

}  // namespace

// ------------------------------------------------------------------ handle
struct proxsdp_handle {
  hipStream_t st = nullptr;
  proxsdp_options opt{};
  Host h;
  DevProblem dp{};
  int n = 0, npad = 0, rows = 0;
  bool full = false;      // exact eigendecomposition path (n <= KMAX)
  int k_cap = 16, r_cap = 1;
  int k = 16, r = 1, r_old = 0;
  Chunking ch{};
  int nsl = 1, nrow_blocks = 1, npat_blocks = 1;
  // device buffers
  int prec = PROXSDP_FP64;   // storage of W: FP64 (plain form), FP32 or BF16 (precision form)
  int wbytes = 8;            // bytes per stored element of W
  float* Bl = nullptr;       // FP32 / BF16 copy of the basis block (precision form)
  double* W = nullptr;       // FP64 W (plain form and the exact small-n path)
  void* Wl = nullptr;        // FP32 / BF16 W (precision form)
  double* vb_part = nullptr; // per-slice partials of V^T B, u^T B (implicit operator)
  bool w_fresh = false;      // precision form: the low-precision W matches the current iterate
  double* B[3] = {nullptr, nullptr, nullptr};
  int bcur = 0;
  double* Z = nullptr;
  double* part = nullptr;
  double* gram_part = nullptr;
  double* small = nullptr;
  double* V[2] = {nullptr, nullptr};
  double* fac_part = nullptr;
  double *y = nullptr, *y_old = nullptr, *MX = nullptr, *MX_old = nullptr;
  double *row_part = nullptr, *pat_part = nullptr, *dval = nullptr;
  IterRecord* ring = nullptr;
  double* round_g = nullptr;        // hyperplane rounding: Gaussian vectors (trials x r)
  signed char* round_x = nullptr;   //   signs (n x trials)
  double* round_part = nullptr;     //   per-block partial values
  double* round_val = nullptr;      //   values <C, x x^T> per trial
  // control
  int iters = 0, passes = 0, rank_updates = 0;
  int m_rounds = 2;
  double eta = 1e-3;       // current relative Ritz residual target
  int status = PROXSDP_STATUS_RUNNING;
  std::vector<double> hist;
  std::vector<int> path_it, path_r, path_why;
  double eps_lambda = 0;
  double rank_value = std::nan("");   // last confirmed rank-test value (upper estimate)
  int verify_steps = 0;               // exact-step convergence checks taken
  int verify_unconverged = 0;         // of those, checks whose eigensolve missed its bound
  int width_changes = 0;
  int cheb_max = 2;                   // largest pass count of one filtered Rayleigh-Ritz step
  double verify_q = 1.0;              // last failed check: exact / reported residual
  int strict_rounds = 200;            // round budget of the strict schedule
  double strict_abs = 0.0;            // > 0: the strict rounds stop on the step error bound
  bool strict_converged = false;      // the last strict eigensolve met its target
  double eig_rel_user = 0.2;          // eig_rel as created (the checks may lower it)
  // Algorithm 2's intermediate feasible solutions X_[r] (host copies)
  struct Saved {
    int iter = 0, r = 0;
    std::vector<double> V, lam, y;
  };
  std::vector<Saved> saved;
  double time_s = 0;
  proxsdp_info last{};
  size_t ws_need = 0;
  // captured rounds of check_every iterations (opt.graphs)
  struct GraphEntry {
    hipGraph_t g = nullptr;
    hipGraphExec_t ex = nullptr;
    int end_bcur = 0, d_passes = 0;
    bool end_wfresh = false;
  };
  std::map<std::tuple<int, int, int, int, int, int, int, int, int, int64_t>, GraphEntry> graphs;
  // optional kernel timing (benchmarks)
  bool prof = false;
  std::vector<hipEvent_t> ev_pass, ev_write;   // start/stop pairs
  std::vector<int> prof_k, prof_r;             // subspace width / rank of each timed launch
  int n_pass = 0, n_write = 0;
  hipEvent_t round_ev = nullptr;   // end of the last round launched by step_many
  // pinned host copy of a control check's records (+ the non-finite flag), so
  // that the check's device-to-host copy is a plain DMA
  IterRecord* host_rec = nullptr;
  int host_rec_cap = 0;
  ~proxsdp_handle() {
    if (host_rec) (void)hipHostFree(host_rec);
    if (round_ev) (void)hipEventDestroy(round_ev);
    for (auto& kv : graphs) {
      if (kv.second.ex) (void)hipGraphExecDestroy(kv.second.ex);
      if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
    }
    for (auto e : ev_pass) (void)hipEventDestroy(e);
    for (auto e : ev_write) (void)hipEventDestroy(e);
  }
};

constexpr int PROF_MAX = 8192;

static void prof_mark(proxsdp_handle* H, std::vector<hipEvent_t>& pool, int& cnt, bool start) {
  if (!H->prof) return;
  const int idx = 2 * cnt + (start ? 0 : 1);
  if (cnt >= PROF_MAX || idx >= (int)pool.size()) return;
  (void)hipEventRecord(pool[idx], H->st);
  if (start) {
    if (&pool == &H->ev_pass) H->prof_k.push_back(H->k);
    else H->prof_r.push_back(H->full ? H->r : std::min(H->r, H->k));
  }
  if (!start) ++cnt;
}

// Number of Ritz pairs kept as factors: the target rank r of Algorithm 2
// within the subspace width k (k >= r whenever the width is automatic; a
// fixed `block` caps r at k).
static int rf(const proxsdp_handle* H) { return H->full ? H->r : std::min(H->r, H->k); }

static size_t carve(proxsdp_handle* H, void* ws) {
  const int npad = H->npad;
  Carver c(ws);
  const Host& h = H->h;
  if (H->prec == PROXSDP_FP64) {
    H->W = c.take<double>((size_t)npad * npad);
    H->Wl = nullptr;
  } else if (H->prec == PROXSDP_IMPLICIT) {
    H->W = nullptr;   // no dense iterate: every pass applies W through the factors
    H->Wl = nullptr;
  } else {
    H->W = nullptr;
    H->Wl = c.take<char>((size_t)npad * npad * H->wbytes);
  }
  // low-precision copy of the basis block (precision form's dense passes)
  H->Bl = (H->prec == PROXSDP_FP32 || H->prec == PROXSDP_BF16)
              ? c.take<float>((size_t)npad * H->k_cap) : nullptr;
  H->vb_part = c.take<double>((size_t)std::max(H->nsl, 1) * VB_STRIDE);
  H->B[0] = c.take<double>((size_t)npad * H->k_cap);
  H->B[1] = c.take<double>((size_t)npad * H->k_cap);
  H->B[2] = c.take<double>((size_t)npad * H->k_cap);
  H->Z = c.take<double>((size_t)npad * H->k_cap);
  // split-K partials of the dense passes (none without a dense iterate)
  H->part = H->prec == PROXSDP_IMPLICIT ? nullptr
                                        : c.take<double>((size_t)H->ch.nchunks * npad * H->k_cap);
  H->gram_part = c.take<double>((size_t)H->nsl * 3 * H->k_cap * H->k_cap);
  H->small = c.take<double>(SL::TOTAL);
  H->V[0] = c.take<double>((size_t)npad * KMAX);
  H->V[1] = c.take<double>((size_t)npad * KMAX);
  H->fac_part = c.take<double>((size_t)std::max(H->nsl, 1) * FAC_STRIDE);
  H->y = c.take<double>(H->rows);
  H->y_old = c.take<double>(H->rows);
  H->MX = c.take<double>(H->rows);
  H->MX_old = c.take<double>(H->rows);
  H->row_part = c.take<double>((size_t)H->nrow_blocks * ROW_PART);
  H->pat_part = c.take<double>((size_t)H->npat_blocks * PAT_PART);
  H->dval = c.take<double>(h.pat_a.size());
  H->ring = c.take<IterRecord>(RING);
  H->round_g = c.take<double>((size_t)ROUND_MAX_TRIALS * KMAX);
  H->round_x = c.take<signed char>((size_t)npad * ROUND_MAX_TRIALS);
  H->round_part = c.take<double>((size_t)ROUND_BLOCKS * ROUND_MAX_TRIALS);
  H->round_val = c.take<double>(ROUND_MAX_TRIALS);
  // problem data
  DevProblem& d = H->dp;
  d.pat_a = c.take<int>(h.pat_a.size());
  d.pat_b = c.take<int>(h.pat_b.size());
  d.pat_c = c.take<double>(h.pat_c.size());
  d.pat_rptr = c.take<int>(h.pat_rptr.size());
  d.pat_row = c.take<int>(h.pat_row.size());
  d.pat_val = c.take<double>(h.pat_val.size());
  d.row_ptr = c.take<int>(h.row_ptr.size());
  d.row_a = c.take<int>(h.row_a.size());
  d.row_b = c.take<int>(h.row_b.size());
  d.row_w = c.take<double>(h.row_w.size());
  d.sym_ptr = c.take<int>(h.sym_ptr.size());
  d.sym_e = c.take<int>(h.sym_e.size());
  d.slot_other = c.take<int>(h.slot_other.size());
  d.slot_t0 = c.take<int>(h.slot_t0.size());
  d.slot_t1 = c.take<int>(h.slot_t1.size());
  d.slot_row0 = c.take<int>(h.slot_row0.size());
  d.slot_c = c.take<double>(h.slot_c.size());
  d.slot_val0 = c.take<double>(h.slot_val0.size());
  d.tile_ptr = c.take<int>(h.tile_ptr.size());
  d.tile_item = c.take<int>(h.tile_item.size());
  d.tile_e = c.take<int>(h.tile_e.size());
  d.r1_u = c.take<double>(h.r1_u.size());
  d.row_r1 = c.take<int>(h.row_r1.size());
  d.rhs = c.take<double>(h.rhs.size());
  return c.off + 256;
}

static void setup_dims(proxsdp_handle* H) {
  const Host& h = H->h;
  H->n = h.n;
  H->npad = h.npad;
  H->rows = h.rows;
  H->full = H->opt.full_eig || h.n <= KMAX;
  // the exact small-n path reads W in FP64
  H->prec = H->full ? PROXSDP_FP64 : H->opt.precision;
  H->wbytes = H->prec == PROXSDP_FP64 ? 8
             : (H->prec == PROXSDP_FP32 ? 4 : (H->prec == PROXSDP_BF16 ? 2 : 0));
  if (H->full) {
    H->r_cap = h.n;
    H->k_cap = 16;
  } else {
    // Algorithm 2 doubles r up to n; the partial path holds at most KMAX Ritz
    // pairs, so r stops at KMAX (KMAX - 16 with the lambda_{r+1} test, which
    // needs a Ritz value beyond r).  A fixed subspace width caps r at k (k - 1).
    const bool plus1 = H->opt.rank_test == PROXSDP_RANK_TEST_LAMBDA_R_PLUS_1;
    const int rmax_auto = plus1 ? KMAX - 16 : KMAX;
    H->r_cap = std::min(h.n, H->opt.r_max > 0 ? std::min(H->opt.r_max, rmax_auto) : rmax_auto);
    if (H->opt.block) H->r_cap = std::min(H->r_cap, H->opt.block - (plus1 ? 1 : 0));
    H->k_cap = H->opt.block ? H->opt.block : k_for_r(H->r_cap);
    H->k_cap = std::max(H->k_cap, 16);
  }
  if (H->opt.full_eig)
    H->r = h.n;
  else
    H->r = std::min(std::max(H->opt.r0, 1), H->r_cap);
  H->k = H->full ? 16 : (H->opt.block ? H->opt.block : k_for_r(H->r));
  H->ch = chunking(h.npad);
  H->nsl = n_slices(h.npad);
  H->nrow_blocks = (h.rows + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
  H->npat_blocks = std::min(4096, (h.n + 3) / 4);
}

static void fill_dev_problem(proxsdp_handle* H) {
  const Host& h = H->h;
  DevProblem& d = H->dp;
  d.n = h.n;
  d.npad = h.npad;
  d.rows = h.rows;
  d.m = h.m;
  d.p = h.p;
  d.n_pat = (int)h.pat_a.size();
  d.tiles_side = h.npad / TILE;
  d.n_r1 = h.n_r1;
  d.norm_c = h.norm_c;
  for (int q = 0; q < MAX_R1; ++q) {
    d.r1_row[q] = q < h.n_r1 ? h.r1_row[q] : 0;
    d.r1_sigma[q] = q < h.n_r1 ? h.r1_sigma[q] : 0.0;
    d.r1_norm2[q] = h.r1_norm2[q];
  }
  for (int t = 0; t < MAX_R1 * MAX_R1; ++t) d.r1_gram[t] = h.r1_gram[t];
}

template <class T>
static int up(const T* dst, const std::vector<T>& src, hipStream_t st) {
  if (src.empty()) return PROXSDP_OK;
  HIP_OK(hipMemcpyAsync(const_cast<T*>(dst), src.data(), src.size() * sizeof(T),
                        hipMemcpyHostToDevice, st));
  return PROXSDP_OK;
}

static void zero(double* x, size_t count, hipStream_t st) {
  if (!count) return;
  const int64_t c = (int64_t)count;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)((c + 255) / 256)), dim3(256), 0, st, x, c);
}

// Raises the dynamic LDS limit of the kernels that need more than 64 KB to
// 160 KB minus the kernel's static LDS.
static int set_lds_one(const void* fn) {
  hipFuncAttributes at{};
  HIP_OK(hipFuncGetAttributes(&at, fn));
  const int total = 160 * 1024;
  const int dyn = total - (int)at.sharedSizeBytes;
  HIP_OK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, dyn));
  return PROXSDP_OK;
}

static int set_lds_limits() {
  static bool done = false;
  if (done) return PROXSDP_OK;
  int rc;
  if ((rc = set_lds_one((const void*)k_reduce_gram))) return rc;
  if ((rc = set_lds_one((const void*)k_small_rr<4>))) return rc;
  if ((rc = set_lds_one((const void*)k_small_rr<8>))) return rc;
  if ((rc = set_lds_one((const void*)k_small_rr<12>))) return rc;
  if ((rc = set_lds_one((const void*)k_small_rr<16>))) return rc;
  if ((rc = set_lds_one((const void*)k_rowwise))) return rc;
  if ((rc = set_lds_one((const void*)k_full_eig))) return rc;
  if ((rc = set_lds_one((const void*)k_write_w<double>))) return rc;
  if ((rc = set_lds_one((const void*)k_write_w<float>))) return rc;
  if ((rc = set_lds_one((const void*)k_write_w<unsigned short>))) return rc;
  done = true;
  return PROXSDP_OK;
}

// ----------------------------------------------------------- launch helpers
static void launch_block(const double* W, int64_t ld, int n, int npad, const double* B, int k,
                         double* part, const Chunking& ch, bool padded, hipStream_t st) {
  dim3 grid(npad / 64, ch.nchunks);
#define BP(KB)                                                                                   \
  if (padded)                                                                                    \
    hipLaunchKernelGGL((k_block_partial_f64<KB, true>), grid, dim3(256), 0, st, W, ld, n, B, k, \
                       part, ch.rows_per_chunk, npad);                                           \
  else                                                                                           \
    hipLaunchKernelGGL((k_block_partial_f64<KB, false>), grid, dim3(256), 0, st, W, ld, n, B, k, \
                       part, ch.rows_per_chunk, npad);
  switch (k / 16) {
    case 1: BP(1); break;
    case 2: BP(2); break;
    case 3: BP(3); break;
    case 4: BP(4); break;
    default: break;
  }
#undef BP
}

static void launch_reduce(const double* part, int nchunks, double* Z, const double* B,
                          const double* Bprev, int npad, int k, double* gram_part, int cheb,
                          double cc, double ce, bool grams, hipStream_t st,
                          const double* filt = nullptr) {
  const size_t lds = 2 * (size_t)SLICE * k * sizeof(double);
  hipLaunchKernelGGL(k_reduce_gram, dim3(n_slices(npad)), dim3(1024), lds, st, part, nchunks, Z, B,
                     Bprev, npad, k, gram_part, cheb, cc, ce, grams ? 1 : 0, filt);
}


// jac_tol: relative off-diagonal level at which the Jacobi sweeps stop.
// oa_steps: largest number of Newton refinement steps before the Cholesky path.
static void launch_rr(const double* gram_part, int nsl, double* small, int k, int r, int lam_off,
                      int filter, double jac_tol, hipStream_t st, int oa_steps = 10) {
  const int kk = k * k;
  hipLaunchKernelGGL(k_sum_grams, dim3((SG_LANES * 3 * kk + 255) / 256), dim3(256), 0, st, gram_part, nsl, k,
                     small);
  const size_t lds = small_rr_lds_doubles(k) * sizeof(double) + (2 * KMAX + 4) * sizeof(int);
#define RR_LAUNCH(KQ)                                                                    \
  hipLaunchKernelGGL(k_small_rr<KQ>, dim3(1), dim3(RR_THREADS), lds, st, small, k, r, lam_off, \
                     filter, jac_tol, oa_steps)
  switch (k) {
    case 16: RR_LAUNCH(4); break;
    case 32: RR_LAUNCH(8); break;
    case 48: RR_LAUNCH(12); break;
    default: RR_LAUNCH(16); break;
  }
#undef RR_LAUNCH
}

static void launch_rowwise(proxsdp_handle* H, const double* B, double* V, int r, const double* Vold,
                           int r_old, double* Bn, hipStream_t st) {
  const int rp = (r + 15) & ~15;
  const size_t lds = (2 * (size_t)SLICE * (H->k + 1) + 2 * (size_t)SLICE * (rp + 1) +
                      (size_t)MAX_R1 * SLICE) * sizeof(double);
  hipLaunchKernelGGL(k_rowwise, dim3(H->nsl, 3), dim3(512), lds, st, B, H->Z, H->small, H->k, V, r,
                     Vold, r_old, Bn, H->dp.n_r1, H->dp.r1_u, H->npad, H->fac_part);
}

static void launch_full(proxsdp_handle* H, double* V, int r, const double* Vold, int r_old,
                        int lam_off) {
  const int n = H->n;
  const size_t lds = (2 * (size_t)n * (n + 1) + n + 3 * (KMAX / 2 + 1)) * sizeof(double) +
                     (KMAX + 4) * sizeof(int);
  hipLaunchKernelGGL(k_full_eig, dim3(1), dim3(1024), lds, H->st, H->W, (int64_t)H->npad, n, V, r,
                     Vold, r_old, H->small, lam_off, H->dp.n_r1, H->dp.r1_u, H->npad, H->fac_part);
}

static int lam_slot(int parity) { return SL::LAM + parity * KMAX; }

// Dense write of V diag(lambda+) V^T (+ rank-one terms, + the sparse part) into
// Wout, stored as `out_prec` (FP64 for outputs, the handle's storage for W).
static void launch_write(proxsdp_handle* H, void* Wout, int out_prec, int64_t ld, const double* V,
                         int r, int lam_off, bool sparse, bool rank1, const FinArgs* fin,
                         bool tiles = true) {
  const int ts = H->npad / TILE;
  // staged factor block (TILE x (rr + 1)), reused for the TILE x TILE output tile
  const int rr = r + (rank1 ? H->dp.n_r1 : 0);
  const size_t lds = (size_t)TILE * std::max(rr + 1, TILE) * sizeof(double);
  FinArgs f{};
  if (fin) f = *fin;
  if (!tiles && !fin) return;
  const dim3 grid((tiles ? ts * (ts + 1) / 2 : 0) + (fin ? 1 : 0));
#define WR(T)                                                                                   \
  hipLaunchKernelGGL(k_write_w<T>, grid, dim3(256), lds, H->st, static_cast<T*>(Wout), ld, H->n, \
                     V, KMAX, r, H->small, lam_off, H->dp, H->y, H->y_old, H->dval,             \
                     sparse ? 1 : 0, rank1 ? 1 : 0, fin ? 1 : 0, f, ts)
  if (out_prec == PROXSDP_FP32)
    WR(float);
  else if (out_prec == PROXSDP_BF16)
    WR(unsigned short);
  else
    WR(double);
#undef WR
}

// Z = W B for the current iterate through the precision form's dense W
// (FP32 storage: FP32 MFMA; summed in FP64 by the reduction).
static void launch_block_lowp(proxsdp_handle* H, const double* B, double* part) {
  dim3 grid(H->npad / 64, H->ch.nchunks);
  const int64_t cnt = (int64_t)H->npad * H->k;
  if (H->prec == PROXSDP_BF16) {
    const unsigned short* Wb = static_cast<const unsigned short*>(H->Wl);
    unsigned short* Bt = reinterpret_cast<unsigned short*>(H->Bl);
    hipLaunchKernelGGL(k_basis_bf16t, dim3(H->npad / 64), dim3(256), 0, H->st, B, H->k, H->npad, Bt);
#define BB(KB) hipLaunchKernelGGL((k_block_partial_bf16<KB>), grid, dim3(256), 0, H->st, Wb, (int64_t)H->npad, Bt, H->k, part, H->ch.rows_per_chunk, H->npad)
    switch (H->k / 16) {
      case 1: BB(1); break;
      case 2: BB(2); break;
      case 3: BB(3); break;
      default: BB(4); break;
    }
#undef BB
    return;
  }
  const float* Wf = static_cast<const float*>(H->Wl);
  hipLaunchKernelGGL(k_basis_f32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, H->st, B, cnt, H->Bl);
#define BF(KB) hipLaunchKernelGGL((k_block_partial_f32<KB>), grid, dim3(256), 0, H->st, Wf, (int64_t)H->npad, H->Bl, H->k, part, H->ch.rows_per_chunk, H->npad)
  switch (H->k / 16) {
    case 1: BF(1); break;
    case 2: BF(2); break;
    case 3: BF(3); break;
    default: BF(4); break;
  }
#undef BF
}

// Z = W B applied exactly in FP64 from the factors of the current X, the
// sparse part D and the rank-one terms (never reads the dense W), with the
// per-slice Gram partials [B^T B, B^T Z, Z^T Z] for Rayleigh-Ritz.
static void launch_implicit(proxsdp_handle* H, const double* B, double* Z, bool grams = true) {
  hipStream_t st = H->st;
  const int pp = 1 - (H->iters & 1);       // factors of the current X
  const int r = H->r_old;
  const int k = H->k;
  hipLaunchKernelGGL(k_vtb, dim3(H->nsl), dim3(256), 0, st, H->V[pp], r, H->small + lam_slot(pp), B,
                     k, H->dp.n_r1, H->dp.r1_u, H->npad, H->vb_part);
  const int cnt = (r + H->dp.n_r1) * k;
  if (cnt > 0)
    hipLaunchKernelGGL(k_sum_vb, dim3((SVB_LANES * cnt + 255) / 256), dim3(256), 0, st, H->vb_part, H->nsl, r,
                       k, H->dp, H->y, lam_slot(pp), H->small);
  hipLaunchKernelGGL(k_implicit_rows, dim3(H->npad / 4), dim3(256), 0, st, H->dp, H->V[pp], r,
                     lam_slot(pp), H->small, H->dval, B, k, Z);
  // Gram partials [B^T B, B^T Z, Z^T Z] per slice (a one-chunk reduction of Z)
  if (grams) launch_reduce(Z, 1, nullptr, B, nullptr, H->npad, k, H->gram_part, 0, 0.0, 1.0, true, st);
}


// Precision form: the low-precision W is written only when a dense filter
// pass needs it (from the factors of the current X, the sparse part and the
// rank-one terms, as the fused write at the end of an iteration would).
static void ensure_w_fresh(proxsdp_handle* H) {
  if (H->prec == PROXSDP_FP64 || H->prec == PROXSDP_IMPLICIT || H->w_fresh) return;
  const int pp = 1 - (H->iters & 1);
  const int r = H->r_old;
  prof_mark(H, H->ev_write, H->n_write, true);
  launch_write(H, H->Wl, H->prec, H->npad, H->V[pp], r, lam_slot(pp), true, true, nullptr);
  prof_mark(H, H->ev_write, H->n_write, false);
  H->w_fresh = true;
}

// BF16 filter passes are used only while the eigen-accuracy target is looser
// than the BF16 rounding level of W; exact passes (implicit operator) after.
constexpr double BF16_ETA_FLOOR = 1e-2;

// Reduces the residual partials of the last row-wise call and reads the
// largest relative Ritz residual of the kept pairs (synchronises).
static int true_maxres(proxsdp_handle* H, int r, double* out) {
  hipLaunchKernelGGL(k_reduce_res, dim3(1), dim3(256), 0, H->st, H->fac_part, H->nsl, r, H->small);
  HIP_OK(hipMemcpyAsync(out, H->small + SL::SC + S_MAXRES, sizeof(double), hipMemcpyDeviceToHost, H->st));
  HIP_OK(hipStreamSynchronize(H->st));
  return PROXSDP_OK;
}
// Error bound of the step's projection from the last round's Ritz pairs:
// with residuals rho_t = ||W v_t - theta_t v_t|| of the kept pairs, W differs
// by about 2 ||R|| from a matrix whose eigenpairs they are, and the PSD
// projection is 1-Lipschitz; a kept pair with theta_t < rho_t moves X by at most
// about theta_t whatever its vector.  Returns sqrt(sum_t min(rho_t, theta_t)^2)
// over the kept positive pairs (absolute units; synchronises).
static int step_error(proxsdp_handle* H, int r, double* out) {
  hipLaunchKernelGGL(k_reduce_res, dim3(1), dim3(256), 0, H->st, H->fac_part, H->nsl, r, H->small);
  double th[KMAX], rel[KMAX], scale = 0;
  HIP_OK(hipMemcpyAsync(th, H->small + SL::THETA, r * sizeof(double), hipMemcpyDeviceToHost, H->st));
  HIP_OK(hipMemcpyAsync(rel, H->small + SL::RES, r * sizeof(double), hipMemcpyDeviceToHost, H->st));
  HIP_OK(hipMemcpyAsync(&scale, H->small + SL::SC + S_NORMW, sizeof(double), hipMemcpyDeviceToHost, H->st));
  HIP_OK(hipStreamSynchronize(H->st));
  double e2 = 0;
  for (int t = 0; t < r && th[t] > 0.0; ++t) {
    const double e = std::min(rel[t] * scale, th[t]);
    e2 += e * e;
  }
  *out = std::isfinite(e2) ? std::sqrt(e2) : INFINITY;
  return PROXSDP_OK;
}

static int x2_slot(int parity) { return SL::SC + S_X2 + parity; }

// Eigensolver rounds on the current W with the current basis.  `final_round`
// forms the factors V[par] and the partials; other rounds only update the basis.
// Jacobi stopping level of the Rayleigh-Ritz step for the current accuracy
// target, rounded down to a half decade (so that a captured round stays valid
// while the target drifts within it).
static double jacobi_tol(const proxsdp_handle* H) {
  if (H->opt.eig_strict) return 1e-15;
  double t = std::max(1e-15, std::min(1e-6, 0.01 * H->eta));
  const double q = std::floor(std::log10(t) * 2.0) / 2.0;
  return std::max(1e-15, std::pow(10.0, q));
}

static void eig_round(proxsdp_handle* H, int par, bool final_round) {
  hipStream_t st = H->st;
  const double* Bc = H->B[H->bcur];
  const int nb = (H->bcur + 1) % 3;
  double* Bn = H->B[nb];
  if (H->prec == PROXSDP_FP64) {
    prof_mark(H, H->ev_pass, H->n_pass, true);
    launch_block(H->W, H->npad, H->n, H->npad, Bc, H->k, H->part, H->ch, true, st);
    prof_mark(H, H->ev_pass, H->n_pass, false);
    launch_reduce(H->part, H->ch.nchunks, H->Z, Bc, nullptr, H->npad, H->k, H->gram_part, 0, 0.0,
                  1.0, true, st);
  } else {
    launch_implicit(H, Bc, H->Z);
  }
  launch_rr(H->gram_part, H->nsl, H->small, H->k, rf(H), lam_slot(par), 1, jacobi_tol(H), st);
  if (final_round)
    launch_rowwise(H, Bc, H->V[par], rf(H), H->V[1 - par], H->r_old, Bn, st);
  else
    launch_rowwise(H, Bc, nullptr, rf(H), nullptr, 0, Bn, st);
  H->bcur = nb;
  H->passes += 1;
}

// One iteration's partial eigensolve with m dense passes: m - 1 Chebyshev
// filter passes (T_j((W - cI)/e) applied to the current basis by the
// three-term recurrence, fused into the reduction of each pass; c, e from the
// last Rayleigh-Ritz step) and one pass followed by Rayleigh-Ritz, the Ritz
// factors V[par] and the next basis (degree-one filter of the Ritz vectors).
static void eig_iteration(proxsdp_handle* H, int par, int m, bool final_round = true) {
  hipStream_t st = H->st;
  const double* filt = H->small + SL::SC + S_FILTC;
  int prev = -1, cur = H->bcur;
  for (int j = 0; j < m - 1; ++j) {
    int nxt = 0;
    while (nxt == cur || nxt == prev) ++nxt;
    if (H->prec == PROXSDP_IMPLICIT || (H->prec == PROXSDP_BF16 && H->eta < BF16_ETA_FLOOR)) {
      // exact filter pass: Z = W B from the factors, then the Chebyshev step
      launch_implicit(H, H->B[cur], H->Z, false);
      launch_reduce(H->Z, 1, H->B[nxt], H->B[cur], prev >= 0 ? H->B[prev] : nullptr, H->npad,
                    H->k, H->gram_part, prev >= 0 ? 2 : 1, 0.0, 1.0, false, st, filt);
    } else {
      ensure_w_fresh(H);
      prof_mark(H, H->ev_pass, H->n_pass, true);
      if (H->prec == PROXSDP_FP64)
        launch_block(H->W, H->npad, H->n, H->npad, H->B[cur], H->k, H->part, H->ch, true, st);
      else
        launch_block_lowp(H, H->B[cur], H->part);
      prof_mark(H, H->ev_pass, H->n_pass, false);
      launch_reduce(H->part, H->ch.nchunks, H->B[nxt], H->B[cur], prev >= 0 ? H->B[prev] : nullptr,
                    H->npad, H->k, H->gram_part, prev >= 0 ? 2 : 1, 0.0, 1.0, false, st, filt);
    }
    prev = cur;
    cur = nxt;
    H->passes += 1;
  }
  int nb = 0;
  while (nb == cur) ++nb;
  if (H->prec == PROXSDP_FP64) {
    prof_mark(H, H->ev_pass, H->n_pass, true);
    launch_block(H->W, H->npad, H->n, H->npad, H->B[cur], H->k, H->part, H->ch, true, st);
    prof_mark(H, H->ev_pass, H->n_pass, false);
    launch_reduce(H->part, H->ch.nchunks, H->Z, H->B[cur], nullptr, H->npad, H->k, H->gram_part, 0,
                  0.0, 1.0, true, st);
  } else {
    // precision form: the Rayleigh-Ritz pass applies W exactly (FP64 refinement)
    launch_implicit(H, H->B[cur], H->Z);
  }
  launch_rr(H->gram_part, H->nsl, H->small, H->k, rf(H), lam_slot(par), 1, jacobi_tol(H), st);
  if (final_round)
    launch_rowwise(H, H->B[cur], H->V[par], rf(H), H->V[1 - par], H->r_old, H->B[nb], st);
  else
    launch_rowwise(H, H->B[cur], nullptr, rf(H), nullptr, 0, H->B[nb], st);
  H->bcur = nb;
  H->passes += 1;
}

static void pattern_and_write(proxsdp_handle* H, int par, int ring_slot) {
  hipStream_t st = H->st;
  hipLaunchKernelGGL(k_pattern, dim3(H->npat_blocks), dim3(256), 0, st, H->dp, H->y, H->y_old,
                     H->small, H->dval, H->pat_part);
  FinArgs f{};
  f.fac_part = H->fac_part;
  f.nslices = H->full ? 1 : H->nsl;
  f.r = rf(H);
  f.r_old = H->r_old;
  f.lam_new = lam_slot(par);
  f.lam_old = lam_slot(1 - par);
  f.x2_new = S_X2 + par;
  f.x2_old = S_X2 + (1 - par);
  f.row_part = H->row_part;
  f.nrow_blocks = H->nrow_blocks;
  f.pat_part = H->pat_part;
  f.npat_blocks = H->npat_blocks;
  f.ring = H->ring;
  f.ring_slot = ring_slot;
  if (H->prec == PROXSDP_FP64) {
    prof_mark(H, H->ev_write, H->n_write, true);
    launch_write(H, H->W, H->prec, H->npad, H->V[par], rf(H), lam_slot(par), true, true, &f);
    prof_mark(H, H->ev_write, H->n_write, false);
  } else {
    // precision form: finalise only; the low-precision W is written when a
    // dense filter pass needs it
    launch_write(H, H->Wl, H->prec, H->npad, H->V[par], rf(H), lam_slot(par), true, true, &f, false);
    H->w_fresh = false;
  }
}

// One PDHG iteration (Algorithm 1 / Algorithm 2 inner loop).
static void iterate_once(proxsdp_handle* H) {
  hipStream_t st = H->st;
  const int par = H->iters & 1;
  // primal step: factors of aproj(W, r)
  if (H->full) {
    launch_full(H, H->V[par], H->r, H->V[1 - par], H->r_old, lam_slot(par));
    H->passes += 1;
  } else if (H->opt.eig_strict) {
    // rounds until the kept Ritz pairs meet eig_tol, then one final round
    const double target = H->opt.eig_tol;
    H->strict_converged = false;
    for (int rd = 0; rd < H->strict_rounds; ++rd) {
      double mr = 1.0;
      if (H->strict_abs > 0) {
        // exact-step check: Chebyshev-filtered rounds (the degree the
        // spectrum allows, see cheb_max)
        eig_iteration(H, par, std::min(H->cheb_max, H->opt.max_passes), false);
        // exact-step check: the projection's error bound against its target
        if (step_error(H, rf(H), &mr)) break;
        if (mr <= H->strict_abs) {
          H->strict_converged = true;
          break;
        }
        continue;
      }
      eig_round(H, par, false);
      if (true_maxres(H, rf(H), &mr)) break;
      if (mr <= target) {
        H->strict_converged = true;
        break;
      }
    }
    eig_round(H, par, true);
  } else {
    // Chebyshev filter passes without Rayleigh-Ritz up to the degree that
    // keeps the basis well conditioned (cheb_max); further passes as full
    // rounds (pass, Rayleigh-Ritz, next basis)
    const int mc = std::min(H->m_rounds, H->cheb_max);
    for (int rd = 0; rd < H->m_rounds - mc; ++rd) eig_round(H, par, false);
    eig_iteration(H, par, mc);
  }
  // dual step
  hipLaunchKernelGGL(k_gather_dual, dim3(H->nrow_blocks), dim3(ROW_LANES * ROWS_PER_BLOCK), 0, st, H->dp, H->V[par],
                     rf(H), H->small, lam_slot(par), H->fac_part, H->full ? 1 : H->nsl, H->r_old,
                     H->y, H->y_old, H->MX, H->MX_old, H->row_part);
  // next W, residuals
  pattern_and_write(H, par, -1);   // ring slot from the device iteration counter
  H->r_old = rf(H);
  H->iters += 1;
}

// Enqueues `count` iterations.  With opt.graphs, a round that starts at a
// control check and spans check_every iterations is captured once per
// configuration and replayed afterwards (same kernels, same arguments: every
// quantity that varies between rounds of one configuration is read on the
// device).
static int run_round(proxsdp_handle* H, int count) {
  // the legacy null stream cannot be captured: graphs need the handle on a
  // stream of its own
  const bool graphable = H->opt.graphs && H->st != nullptr && !H->opt.eig_strict && !H->prof &&
                         !H->full && count == H->opt.check_every &&
                         H->iters % H->opt.check_every == 0 && (H->opt.check_every % 2) == 0;
  if (!graphable) {
    for (int t = 0; t < count; ++t) iterate_once(H);
    return PROXSDP_OK;
  }
  const bool lowp = H->prec == PROXSDP_BF16 && H->eta < BF16_ETA_FLOOR;
  double jt = jacobi_tol(H);
  int64_t jbits;
  std::memcpy(&jbits, &jt, sizeof(jbits));
  const auto key = std::make_tuple(H->bcur, H->r, H->r_old, H->k, H->m_rounds * 256 + H->cheb_max,
                                   H->prec, (int)H->w_fresh, (int)lowp, count, jbits);
  auto it = H->graphs.find(key);
  if (it == H->graphs.end()) {
    proxsdp_handle::GraphEntry e{};
    const int bcur0 = H->bcur, passes0 = H->passes, iters0 = H->iters, rold0 = H->r_old;
    const bool wf0 = H->w_fresh;
    if (hipStreamBeginCapture(H->st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
      (void)hipGetLastError();   // capture refused: clear the error, launch directly
      H->opt.graphs = 0;
      for (int t = 0; t < count; ++t) iterate_once(H);
      return PROXSDP_OK;
    }
    for (int t = 0; t < count; ++t) iterate_once(H);
    const hipError_t ce = hipStreamEndCapture(H->st, &e.g);
    e.end_bcur = H->bcur;
    e.d_passes = H->passes - passes0;
    e.end_wfresh = H->w_fresh;
    // nothing ran yet: restore the host state, then replay below
    H->bcur = bcur0;
    H->passes = passes0;
    H->iters = iters0;
    H->r_old = rold0;
    H->w_fresh = wf0;
    if (ce != hipSuccess) return fail(PROXSDP_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
    HIP_OK(hipGraphInstantiate(&e.ex, e.g, nullptr, nullptr, 0));
    it = H->graphs.emplace(key, e).first;
  }
  HIP_OK(hipGraphLaunch(it->second.ex, H->st));
  H->iters += count;
  H->passes += it->second.d_passes;
  H->bcur = it->second.end_bcur;
  H->w_fresh = it->second.end_wfresh;
  H->r_old = rf(H);
  return PROXSDP_OK;
}

// Re-layout of the basis block with a new subspace width: the leading
// columns (the Ritz directions of the largest values) are kept, new ones are
// random.
static void set_width(proxsdp_handle* H, int k_new) {
  if (k_new == H->k) return;
  const int64_t cnt = (int64_t)H->npad * k_new;
  const int nb = (H->bcur + 1) % 3;
  H->width_changes += 1;
  hipLaunchKernelGGL(k_fill_basis, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, H->st,
                     H->B[nb], k_new, H->B[H->bcur], H->k, std::min(H->k, k_new), H->n,
                     H->npad, (uint32_t)(H->opt.seed * 7919 + H->rank_updates + 131 * H->width_changes));
  H->bcur = nb;
  H->k = k_new;
}

static void set_rank(proxsdp_handle* H, int r_new, int why) {
  if (r_new == H->r) return;
  H->r = r_new;
  H->rank_updates += 1;
  H->path_it.push_back(H->iters);
  H->path_r.push_back(r_new);
  H->path_why.push_back(why);
  if (H->full) return;
  set_width(H, H->opt.block ? H->opt.block : k_for_r(r_new));
}

static int read_records(proxsdp_handle* H, int first_iter, int count, std::vector<IterRecord>& out) {
  out.resize(count);
  int done = 0;
  while (done < count) {
    const int slot = (first_iter + done) % RING;
    const int len = std::min(count - done, RING - slot);
    HIP_OK(hipMemcpyAsync(&out[done], H->ring + slot, len * sizeof(IterRecord),
                          hipMemcpyDeviceToHost, H->st));
    done += len;
  }
  return PROXSDP_OK;
}

static int fill_info(proxsdp_handle* H, const IterRecord& rec, double nonfinite) {
  proxsdp_info& I = H->last;
  I.status = H->status;
  I.iters = H->iters;
  I.r = H->r;
  I.k = H->full ? H->n : H->k;
  I.rank_updates = H->rank_updates;
  I.passes = H->passes;
  I.lambda_r = rec.lambda_r;
  I.lambda_r1 = rec.lambda_r1;
  I.eps_p = rec.eps_p;
  I.eps_d = rec.eps_d;
  I.rho_p = rec.eps_p / (1.0 + H->h.norm_c);
  I.rho_d = rec.eps_d / (1.0 + H->h.norm_rhs);
  I.obj = rec.obj;
  I.dual_obj = rec.dual_obj;
  I.alpha = H->opt.alpha;
  I.norm_M = H->h.norm_m;
  I.ritz_res = rec.maxres;
  I.time_s = H->time_s;
  I.gap = std::fabs(rec.obj - rec.dual_obj) / (1.0 + std::fabs(rec.obj) + std::fabs(rec.dual_obj));
  I.rank_value = H->rank_value;
  I.saved = (int32_t)H->saved.size();
  I.verify_steps = H->verify_steps;
  (void)nonfinite;
  return PROXSDP_OK;
}

// Rank test of Algorithm 2 on a confirmed subspace.  Rounds of the partial
// eigensolve (dense pass or exact apply, Rayleigh-Ritz on the Cholesky path,
// which resolves every Ritz value, next basis) on the current W, in batches of
// eight; after each batch the true Ritz residuals ||W u_c - theta_c u_c|| of
// the columns up to r + 1 are formed from the same pass.  A Ritz value is a
// lower bound of the eigenvalue of the same index (interlacing), and the
// residual norm bounds the distance to an eigenvalue, so the test is decided
// on the pair (theta, theta + ||res||) of the tested index: it fails when even
// theta is above the threshold, passes when theta + ||res|| is below it, and
// another batch runs while it is undecided (at most four).  Overwrites only
// data the next iteration recomputes (and improves the basis).
enum RankVerdict { RANK_PASS = 0, RANK_FAIL = 1, RANK_UNDECIDED = 2 };

static int rank_probe(proxsdp_handle* H, double thr, int* verdict, double* ub_out) {
  hipStream_t st = H->st;
  const int slot = H->iters & 1;   // lambda slot the next iteration overwrites
  const bool plus1 = H->opt.rank_test == PROXSDP_RANK_TEST_LAMBDA_R_PLUS_1;
  const int want = plus1 ? H->r : H->r - 1;   // 0-based index Algorithm 2's test reads
  // A block narrower than that index tests its last value instead:
  // lambda_want <= lambda_idx, so an upper estimate of lambda_idx below the
  // threshold passes the test, but a large theta_idx says nothing about
  // lambda_want.
  const int idx = std::min(want, H->k - 1);
  const bool exact_index = idx == want;
  const int ncol = idx + 1;
  const int per_batch = 8, batches = 4;
  *verdict = RANK_UNDECIDED;
  for (int b = 0; b < batches && *verdict == RANK_UNDECIDED; ++b) {
    for (int rd = 0; rd < per_batch; ++rd) {
      const bool last = rd == per_batch - 1;
      const double* Bc = H->B[H->bcur];
      if (H->prec == PROXSDP_FP64) {
        launch_block(H->W, H->npad, H->n, H->npad, Bc, H->k, H->part, H->ch, true, st);
        launch_reduce(H->part, H->ch.nchunks, H->Z, Bc, nullptr, H->npad, H->k, H->gram_part, 0,
                      0.0, 1.0, true, st);
      } else {
        launch_implicit(H, Bc, H->Z);
      }
      launch_rr(H->gram_part, H->nsl, H->small, H->k, rf(H), lam_slot(slot), 1, 1e-15, st,
                last ? 0 : 10);
      const int nb = (H->bcur + 1) % 3;
      // the last round of a batch also forms the true residuals of columns < ncol
      launch_rowwise(H, Bc, nullptr, last ? ncol : rf(H), nullptr, 0, H->B[nb], st);
      H->bcur = nb;
      H->passes += 1;
    }
    hipLaunchKernelGGL(k_reduce_res, dim3(1), dim3(256), 0, st, H->fac_part, H->nsl, ncol, H->small);
    double th = 0, rel = 0, scale = 0;
    HIP_OK(hipMemcpyAsync(&th, H->small + SL::THETA + idx, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&rel, H->small + SL::RES + idx, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(&scale, H->small + SL::SC + S_NORMW, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    const double ub = th + rel * std::max(scale, 1e-300);
    *ub_out = ub;
    if (!std::isfinite(ub)) break;
    if (std::max(ub, 0.0) <= thr) *verdict = RANK_PASS;
    else if (std::max(th, 0.0) > thr) {
      if (exact_index) *verdict = RANK_FAIL;
      else break;   // more positive values than the block holds: undecided
    }
  }
  return PROXSDP_OK;
}

// One PDHG iteration whose partial eigensolve runs until the kept Ritz pairs
// are converged (the eig_strict schedule), i.e. the exact step of Algorithm 1
// from the current (X, y) once the rank test has shown that r covers every
// positive eigenvalue.  Its residuals are those of an exact step, which is
// what decides convergence (Section 2.2: the fixed point of the exact
// iteration is the KKT point); the adaptive-accuracy iterations before it
// only report residuals of their own inexact steps.  The eigen error only
// has to be small against the step: an error delta in X moves eps_p by about
// delta / alpha and eps_d by at most ||M|| delta = 0.95 delta / alpha, so the
// rounds run until the projection's error bound (step_error) is below 10% of
// what the stopping rule allows either residual,
//   0.1 alpha tol min(1 + ||C||_F, (1 + ||[b; h]||) / 0.95),
// within 1000 rounds (strict_converged says whether it got there).  *out gets
// its record.
static int verify_step(proxsdp_handle* H, const IterRecord& last, IterRecord* out) {
  const int strict = H->opt.eig_strict;
  H->opt.eig_strict = 1;
  (void)last;
  const double scale = std::min(1.0 + H->h.norm_c, (1.0 + H->h.norm_rhs) / 0.95);
  H->strict_abs = std::max(0.1 * H->opt.alpha * H->opt.tol * scale, 1e-300);
  H->strict_rounds = 1000;
  iterate_once(H);
  H->opt.eig_strict = strict;
  H->strict_abs = 0.0;
  H->strict_rounds = 200;
  std::vector<IterRecord> recs;
  int rc = read_records(H, H->iters - 1, 1, recs);
  if (rc) return rc;
  HIP_OK(hipStreamSynchronize(H->st));
  *out = recs[0];
  H->verify_steps += 1;
  return PROXSDP_OK;
}

// Host copy of the current iterate as Algorithm 2's intermediate X_[r].
static int save_intermediate(proxsdp_handle* H) {
  proxsdp_handle::Saved sv;
  sv.iter = H->iters;
  int32_t r = 0;
  int rc = proxsdp_get_factors(H, nullptr, nullptr, &r);
  if (rc) return rc;
  sv.r = r;
  sv.V.assign((size_t)H->n * std::max(r, 1), 0.0);
  sv.lam.assign(std::max(r, 1), 0.0);
  sv.y.assign(H->rows, 0.0);
  rc = proxsdp_get_factors(H, sv.V.data(), sv.lam.data(), &r);
  if (rc) return rc;
  rc = proxsdp_get_solution(H, nullptr, sv.y.data(), 0);
  if (rc) return rc;
  H->saved.push_back(std::move(sv));
  return PROXSDP_OK;
}

// Control check after iteration H->iters (a multiple of check_every).
static int control(proxsdp_handle* H) {
  const int ce = H->opt.check_every;
  if (H->host_rec_cap < ce + 1) {
    if (H->host_rec) HIP_OK(hipHostFree(H->host_rec));
    H->host_rec = nullptr;
    H->host_rec_cap = 0;
    HIP_OK(hipHostMalloc((void**)&H->host_rec, (size_t)(ce + 1) * sizeof(IterRecord), hipHostMallocDefault));
    H->host_rec_cap = ce + 1;
  }
  {
    int done = 0;
    const int first = H->iters - ce;
    while (done < ce) {
      const int slot = ((first + done) % RING + RING) % RING;
      const int len = std::min(ce - done, RING - slot);
      HIP_OK(hipMemcpyAsync(H->host_rec + done, H->ring + slot, len * sizeof(IterRecord),
                            hipMemcpyDeviceToHost, H->st));
      done += len;
    }
  }
  double* nf_host = reinterpret_cast<double*>(H->host_rec + ce);
  HIP_OK(hipMemcpyAsync(nf_host, H->small + SL::SC + S_NONFINITE, sizeof(double),
                        hipMemcpyDeviceToHost, H->st));
  HIP_OK(hipStreamSynchronize(H->st));
  const std::vector<IterRecord> recs(H->host_rec, H->host_rec + ce);
  const double nonfinite = *nf_host;
  int rc = 0;
  const IterRecord& rec = recs.back();
  const double rho_p = rec.eps_p / (1.0 + H->h.norm_c);
  const double rho_d = rec.eps_d / (1.0 + H->h.norm_rhs);
  const double comb = rec.eps_p + rec.eps_d;
  const int L = H->opt.window / ce;
  if (nonfinite != 0.0 || !std::isfinite(comb)) {
    H->status = PROXSDP_STATUS_NUMERICAL;
  } else if (std::max(rho_p, rho_d) <= H->opt.tol / H->verify_q) {
    // (verify_q > 1 after an exact-step check found the reported residuals
    // that much below the exact ones: wait until they are low enough to pass.)
    // Algorithm 2: converged residuals stop the solve only if the rank test
    // (n - r) max(lambda, 0) <= eps_lambda passes; otherwise X_[r] is kept and
    // r doubles (at the cap the solve stops with a status saying so).
    const int n = H->n;
    const bool plus1 = H->opt.rank_test == PROXSDP_RANK_TEST_LAMBDA_R_PLUS_1;
    int verdict = RANK_PASS;
    if (H->r < n) {
      const double thr = H->eps_lambda / (double)(n - H->r);
      if (H->full) {
        const double lam_t = plus1 ? rec.lambda_r1 : rec.lambda_r;   // exact eigenvalues
        verdict = std::max(lam_t, 0.0) <= thr ? RANK_PASS : RANK_FAIL;
      } else if (!plus1 && rf(H) == H->r && std::max(rec.lambda_r, 0.0) > thr) {
        // a positive r-th Ritz value is kept, hence resolved, and bounds
        // lambda_r from below: the test fails without confirmation
        verdict = RANK_FAIL;
      } else {
        double ub = 0;
        const int rc2 = rank_probe(H, thr, &verdict, &ub);
        if (rc2) return rc2;
        H->rank_value = ub;
      }
    }
    if (verdict == RANK_PASS && !H->full && !H->opt.eig_strict) {
      // the residuals above are those of an inexact step: decide on an exact one
      IterRecord vr{};
      const int rc4 = verify_step(H, rec, &vr);
      if (rc4) return rc4;
      if (!H->strict_converged) {
        // the exact step could not be formed within the round budget: no
        // convergence claim now; after three such checks, none at all
        if (++H->verify_unconverged >= 3) {
          H->status = PROXSDP_STATUS_EIG_NOT_CONVERGED;
          fill_info(H, vr, nonfinite);
          return PROXSDP_OK;
        }
      }
      const double vp = vr.eps_p / (1.0 + H->h.norm_c), vd = vr.eps_d / (1.0 + H->h.norm_rhs);
      if (H->strict_converged && std::max(vp, vd) <= H->opt.tol && std::isfinite(vp + vd)) {
        H->status = PROXSDP_STATUS_CONVERGED;
        fill_info(H, vr, nonfinite);
        return PROXSDP_OK;
      }
      // The exact step's residual q times the inexact one's: the excess q - 1
      // is the bias of the reported residuals, which scales with the eigen
      // error allowed per step (eig_rel).  Bring it down to about 0.1 (no
      // change for a residual that only sat on the threshold); iterate on.
      const double q = std::max(vp, vd) / std::max(std::max(rho_p, rho_d), 1e-300);
      if (q > 1.1)
        H->opt.eig_rel = std::max(H->opt.eig_rel * std::min(1.0, 0.1 / (q - 1.0)), 1e-3);
      if (std::isfinite(q)) H->verify_q = std::max(H->verify_q, 1.02 * q);
      H->hist.push_back(vr.eps_p + vr.eps_d);
    } else if (verdict == RANK_PASS) {
      H->status = PROXSDP_STATUS_CONVERGED;
    } else {
      const int rc3 = save_intermediate(H);
      if (rc3) return rc3;
      if (H->r >= H->r_cap) {
        H->status = verdict == RANK_FAIL ? PROXSDP_STATUS_RANK_LIMIT
                                         : PROXSDP_STATUS_EIG_NOT_CONVERGED;
      } else {
        set_rank(H, std::min(2 * H->r, H->r_cap), verdict == RANK_FAIL ? 1 : 3);
        H->hist.clear();
      }
    }
  } else {
    H->hist.push_back(comb);
    if (H->r < H->r_cap && (int)H->hist.size() > L &&
        H->hist.back() >= H->hist[H->hist.size() - 1 - L]) {
      set_rank(H, std::min(2 * H->r, H->r_cap), 2);
      H->hist.clear();
    }
  }
  // accuracy schedule of the partial eigensolve (summable errors, Section
  // 3.2): an eigen error delta in X moves eps_p by about delta / alpha, so the
  // absolute Ritz residual of the kept pairs is held below
  //   eig_rel * alpha * eps_p   (floor: eig_tol * max|theta|),
  // i.e. a fixed fraction of the current primal step.  The target is tied to
  // the iteration's own scale, not to ||W|| (a target relative to ||W|| is
  // far too loose for problems with C = 0, such as sensor localisation).
  if (!H->full) {
    double worst = 0, normw = 0;
    for (auto& x : recs) {
      worst = std::max(worst, x.maxres * x.normw);
      normw = std::max(normw, x.normw);
    }
    const double eta_abs =
        std::max(H->opt.eig_tol * normw, H->opt.eig_rel * H->opt.alpha * rec.eps_p);
    H->eta = normw > 0 ? eta_abs / normw : H->opt.eig_tol;
    if (worst > eta_abs && H->m_rounds < H->opt.max_passes) H->m_rounds += 1;
    else if (worst < 0.05 * eta_abs && H->m_rounds > 1) H->m_rounds -= 1;
    // Filter degree: with x1 = (theta_1 - c) / e the top Ritz value in the
    // filter's variable, a degree-d Chebyshev polynomial amplifies the top of
    // the wanted spectrum by up to T_d(x1) against its lower edge (x = 1);
    // degrees with T_d(x1) <= 100 keep the basis well conditioned for the
    // Rayleigh-Ritz step (higher ones collapse it onto the dominant vectors).
    // A wide spectrum (x1 near 1, e.g. a dense C) gets many filter passes per
    // step, a narrow one a single pass.
    double x1 = 1.0;
    for (auto& x : recs) x1 = std::max(x1, x.filt_x1);
    const double d = x1 > 1.0 + 1e-12 ? std::acosh(100.0) / std::acosh(x1) : 1e9;
    H->cheb_max = (int)std::max(2.0, std::min((double)H->opt.max_passes, 1.0 + std::floor(d)));
  }
  fill_info(H, rec, nonfinite);
  return PROXSDP_OK;
}

static int warm_start(proxsdp_handle* H, const double* src = nullptr, int nsrc = 0) {
  // subspace for the first projection: the first nsrc columns from src
  // (factor layout, row stride KMAX), the others random; rounds until the
  // kept Ritz pairs are accurate to 1e-3 (relative) or 60 rounds.
  if (H->full) return PROXSDP_OK;
  const int64_t cnt = (int64_t)H->npad * H->k;
  hipLaunchKernelGGL(k_fill_basis, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, H->st,
                     H->B[H->bcur], H->k, src, KMAX, src ? std::min(nsrc, H->k) : 0, H->n, H->npad,
                     (uint32_t)H->opt.seed);
  for (int rd = 0; rd < 60; ++rd) {
    eig_round(H, 0, false);
    if (rd % 4 == 3) {
      double mr = 1;
      const int rc = true_maxres(H, rf(H), &mr);
      if (rc) return rc;
      if (mr <= 1e-3) break;
    }
  }
  return PROXSDP_OK;
}

// Zeroes the iteration state (device buffers, scalars, control history) and
// sets the working rank r0; X0 = 0, y0 = 0 until the caller writes more.
static int reset_buffers(proxsdp_handle* H) {
  hipStream_t st = H->st;
  if (H->prec == PROXSDP_FP64)
    zero(H->W, (size_t)H->npad * H->npad, st);
  else if (H->Wl)
    zero(static_cast<double*>(H->Wl), (size_t)H->npad * H->npad * H->wbytes / 8, st);
  zero(H->B[0], (size_t)H->npad * H->k_cap, st);
  zero(H->B[1], (size_t)H->npad * H->k_cap, st);
  zero(H->B[2], (size_t)H->npad * H->k_cap, st);
  zero(H->Z, (size_t)H->npad * H->k_cap, st);
  zero(H->small, SL::TOTAL, st);
  zero(H->V[0], (size_t)H->npad * KMAX, st);
  zero(H->V[1], (size_t)H->npad * KMAX, st);
  zero(H->fac_part, (size_t)std::max(H->nsl, 1) * FAC_STRIDE, st);
  zero(H->y, H->rows, st);
  zero(H->y_old, H->rows, st);
  zero(H->MX, H->rows, st);
  zero(H->MX_old, H->rows, st);
  zero(H->row_part, (size_t)H->nrow_blocks * ROW_PART, st);
  zero(H->pat_part, (size_t)H->npat_blocks * PAT_PART, st);
  std::vector<double> sc(S_COUNT, 0.0);
  sc[S_ALPHA] = H->opt.alpha;
  HIP_OK(hipMemcpyAsync(H->small + SL::SC, sc.data(), sc.size() * sizeof(double),
                        hipMemcpyHostToDevice, st));
  H->iters = 0;
  H->passes = 0;
  H->rank_updates = 0;
  H->m_rounds = 2;
  H->eta = 1e-3;
  H->status = PROXSDP_STATUS_RUNNING;
  H->hist.clear();
  H->path_it.clear();
  H->path_r.clear();
  H->path_why.clear();
  H->saved.clear();
  H->rank_value = std::nan("");
  H->verify_steps = 0;
  H->verify_unconverged = 0;
  H->width_changes = 0;
  H->cheb_max = 2;
  H->verify_q = 1.0;
  H->opt.eig_rel = H->eig_rel_user;
  H->time_s = 0;
  H->last = proxsdp_info{};
  H->bcur = 0;
  H->r_old = 0;
  H->r = H->opt.full_eig ? H->n : std::min(std::max(H->opt.r0, 1), H->r_cap);
  H->k = H->full ? 16 : (H->opt.block ? H->opt.block : k_for_r(H->r));
  return PROXSDP_OK;
}

static int init_state(proxsdp_handle* H) {
  hipStream_t st = H->st;
  int rc = reset_buffers(H);
  if (rc) return rc;
  // W0 = X0 - alpha (C - M*(y0)) = -alpha C
  const int r_save = H->r;
  H->r = 0;
  pattern_and_write(H, 1, RING - 1);
  H->r = r_save;
  const double zero_flag = 0.0;
  HIP_OK(hipMemcpyAsync(H->small + SL::SC + S_NONFINITE, &zero_flag, sizeof(double),
                        hipMemcpyHostToDevice, st));
  rc = warm_start(H);
  if (rc) return rc;
  HIP_OK(hipStreamSynchronize(st));
  return PROXSDP_OK;
}

// ======================================================================== API
extern "C" {

int proxsdp_default_options(proxsdp_options* o) {
  if (!o) return fail(PROXSDP_ERR_INVALID, "options is NULL");
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-4;
  o->eps_lambda = -1.0;
  o->alpha = 0.0;
  o->window = 50;
  o->check_every = 10;
  o->r0 = 1;
  o->r_max = 0;
  o->full_eig = 0;
  o->precision = PROXSDP_FP64;
  o->max_iters = 200000;
  o->time_limit_s = 1200.0;
  o->row_scaling = 1;
  o->block = 0;
  o->eig_tol = 1e-10;
  o->max_passes = 8;
  o->seed = 1;
  o->eig_strict = 0;
  o->eig_rel = 0.2;
  o->rank_test = PROXSDP_RANK_TEST_LAMBDA_R;
  return PROXSDP_OK;
}

int proxsdp_workspace_size(const proxsdp_problem* pb, const proxsdp_options* opt, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(PROXSDP_ERR_INVALID, "bytes is NULL");
  proxsdp_options o;
  if (opt) o = *opt; else proxsdp_default_options(&o);
  int rc = validate(pb, &o);
  if (rc) return rc;
  proxsdp_handle H;
  H.opt = o;
  rc = preprocess(pb, o.row_scaling, H.h);
  if (rc) return rc;
  setup_dims(&H);
  *bytes = carve(&H, nullptr);
  return PROXSDP_OK;
}

int proxsdp_create(const proxsdp_problem* pb, const proxsdp_options* opt, void* ws, size_t ws_bytes,
                   void* stream, proxsdp_handle** out) {
  g_err.clear();
  if (!out) return fail(PROXSDP_ERR_INVALID, "out is NULL");
  *out = nullptr;
  proxsdp_options o;
  if (opt) o = *opt; else proxsdp_default_options(&o);
  int rc = validate(pb, &o);
  if (rc) return rc;
  if (!ws) return fail(PROXSDP_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PROXSDP_ERR_WORKSPACE, "workspace not 256-byte aligned");
  auto* H = new proxsdp_handle();
  H->opt = o;
  H->st = static_cast<hipStream_t>(stream);
  rc = preprocess(pb, o.row_scaling, H->h);
  if (rc) { delete H; return rc; }
  setup_dims(H);
  const size_t need = carve(H, nullptr);
  if (ws_bytes < need) {
    delete H;
    return fail(PROXSDP_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  }
  carve(H, ws);
  fill_dev_problem(H);
  if ((rc = set_lds_limits())) { delete H; return rc; }
  const Host& h = H->h;
  H->opt.alpha = (o.alpha > 0) ? o.alpha : 0.95 / h.norm_m;
  H->eps_lambda = (o.eps_lambda >= 0) ? o.eps_lambda : o.tol;
  H->eig_rel_user = o.eig_rel;
  hipStream_t st = H->st;
  const DevProblem& d = H->dp;
#define UP(dst, src) if ((rc = up(dst, src, st))) { delete H; return rc; }
  UP(d.pat_a, h.pat_a); UP(d.pat_b, h.pat_b); UP(d.pat_c, h.pat_c);
  UP(d.pat_rptr, h.pat_rptr); UP(d.pat_row, h.pat_row); UP(d.pat_val, h.pat_val);
  UP(d.row_ptr, h.row_ptr); UP(d.row_a, h.row_a); UP(d.row_b, h.row_b); UP(d.row_w, h.row_w);
  UP(d.sym_ptr, h.sym_ptr); UP(d.sym_e, h.sym_e);
  UP(d.slot_other, h.slot_other); UP(d.slot_t0, h.slot_t0); UP(d.slot_t1, h.slot_t1);
  UP(d.slot_row0, h.slot_row0); UP(d.slot_c, h.slot_c); UP(d.slot_val0, h.slot_val0);
  UP(d.tile_ptr, h.tile_ptr); UP(d.tile_item, h.tile_item); UP(d.tile_e, h.tile_e);
  UP(d.r1_u, h.r1_u); UP(d.row_r1, h.row_r1); UP(d.rhs, h.rhs);
#undef UP
  if (hipHostMalloc((void**)&H->host_rec, (size_t)(H->opt.check_every + 1) * sizeof(IterRecord),
                    hipHostMallocDefault) != hipSuccess) {
    H->host_rec = nullptr;
    delete H;
    return fail(PROXSDP_ERR_HIP, "pinned host buffer for the control checks");
  }
  H->host_rec_cap = H->opt.check_every + 1;
  if ((rc = init_state(H))) { delete H; return rc; }
  H->ws_need = need;
  H->status = PROXSDP_STATUS_RUNNING;
  *out = H;
  return PROXSDP_OK;
}

int proxsdp_step(proxsdp_handle* H, int32_t n_iters, proxsdp_info* info) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  if (n_iters < 0) return fail(PROXSDP_ERR_INVALID, "n_iters < 0");
  auto t_last = std::chrono::steady_clock::now();
  auto tick = [&]() {
    const auto now = std::chrono::steady_clock::now();
    H->time_s += std::chrono::duration<double>(now - t_last).count();
    t_last = now;
  };
  int done = 0;
  while (done < n_iters && H->status == PROXSDP_STATUS_RUNNING) {
    const int ce = H->opt.check_every;
    const int chunk = std::min(ce - H->iters % ce, n_iters - done);
    const int rc0 = run_round(H, chunk);
    if (rc0) return rc0;
    done += chunk;
    if (H->iters % H->opt.check_every == 0) {
      const int rc = control(H);  // synchronises the stream
      if (rc) return rc;
      tick();
      H->last.time_s = H->time_s;
      if (H->status == PROXSDP_STATUS_RUNNING && H->iters >= H->opt.max_iters)
        H->status = PROXSDP_STATUS_MAX_ITERS;
      if (H->status == PROXSDP_STATUS_RUNNING && H->opt.time_limit_s > 0 &&
          H->time_s > H->opt.time_limit_s)
        H->status = PROXSDP_STATUS_TIME_LIMIT;
      H->last.status = H->status;
    }
  }
  if (info) {
    HIP_OK(hipStreamSynchronize(H->st));
    if (H->iters > 0 && H->iters % H->opt.check_every != 0) {
      std::vector<IterRecord> recs;
      int rc = read_records(H, H->iters - 1, 1, recs);
      if (rc) return rc;
      HIP_OK(hipStreamSynchronize(H->st));
      fill_info(H, recs.back(), 0.0);
    }
    tick();
    H->last.status = H->status;
    H->last.time_s = H->time_s;
    *info = H->last;
  } else {
    tick();
  }
  return PROXSDP_OK;
}

int proxsdp_step_many(proxsdp_handle** hs, int32_t count, int32_t n_iters, int32_t flags,
                      proxsdp_info* infos) {
  g_err.clear();
  if (count < 0 || (count > 0 && !hs)) return fail(PROXSDP_ERR_INVALID, "bad handle array");
  if (n_iters < 0) return fail(PROXSDP_ERR_INVALID, "n_iters < 0");
  for (int i = 0; i < count; ++i)
    if (!hs[i]) return fail(PROXSDP_ERR_INVALID, "handle " + std::to_string(i) + " is NULL");
  for (int i = 0; i < count; ++i)
    if (!hs[i]->round_ev) HIP_OK(hipEventCreateWithFlags(&hs[i]->round_ev, hipEventDisableTiming));
  std::vector<int> remaining(count, n_iters);
  std::vector<char> in_flight(count, 0);
  std::vector<std::chrono::steady_clock::time_point> t_start(count);
  bool stop = false;
  for (;;) {
    // launch the next round of every idle running handle (each on its own stream)
    if (!stop) {
      for (int i = 0; i < count; ++i) {
        proxsdp_handle* H = hs[i];
        if (in_flight[i] || H->status != PROXSDP_STATUS_RUNNING || remaining[i] <= 0) continue;
        const int ce = H->opt.check_every;
        const int chunk = std::min(ce - H->iters % ce, remaining[i]);
        t_start[i] = std::chrono::steady_clock::now();
        const int rc = run_round(H, chunk);
        if (rc) return rc;
        HIP_OK(hipEventRecord(H->round_ev, H->st));
        remaining[i] -= chunk;
        in_flight[i] = 1;
      }
    }
    bool any_in_flight = false;
    // completed rounds: control check at once, independently of the others
    for (int i = 0; i < count; ++i) {
      if (!in_flight[i]) continue;
      proxsdp_handle* H = hs[i];
      const hipError_t q = hipEventQuery(H->round_ev);
      if (q == hipErrorNotReady) {
        any_in_flight = true;
        continue;
      }
      if (q != hipSuccess) return fail(PROXSDP_ERR_HIP, std::string("round event: ") + hipGetErrorString(q));
      in_flight[i] = 0;
      H->time_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start[i]).count();
      if (H->iters % H->opt.check_every == 0) {
        const int rc = control(H);
        if (rc) return rc;
        if (H->status == PROXSDP_STATUS_RUNNING && H->iters >= H->opt.max_iters)
          H->status = PROXSDP_STATUS_MAX_ITERS;
        if (H->status == PROXSDP_STATUS_RUNNING && H->opt.time_limit_s > 0 &&
            H->time_s > H->opt.time_limit_s)
          H->status = PROXSDP_STATUS_TIME_LIMIT;
        H->last.status = H->status;
        H->last.time_s = H->time_s;
        if (H->status != PROXSDP_STATUS_RUNNING && (flags & PROXSDP_STEP_UNTIL_ANY_STOPS)) stop = true;
      }
    }
    bool more = false;
    if (!stop)
      for (int i = 0; i < count; ++i)
        more |= hs[i]->status == PROXSDP_STATUS_RUNNING && remaining[i] > 0 && !in_flight[i];
    if (!any_in_flight && !more) break;
  }
  for (int i = 0; i < count; ++i) {
    proxsdp_handle* H = hs[i];
    HIP_OK(hipStreamSynchronize(H->st));
    if (infos) {
      if (H->iters > 0 && H->iters % H->opt.check_every != 0) {
        std::vector<IterRecord> recs;
        const int rc = read_records(H, H->iters - 1, 1, recs);
        if (rc) return rc;
        HIP_OK(hipStreamSynchronize(H->st));
        fill_info(H, recs.back(), 0.0);
      }
      H->last.status = H->status;
      H->last.time_s = H->time_s;
      infos[i] = H->last;
    }
  }
  return PROXSDP_OK;
}

int proxsdp_solve(proxsdp_handle* H, proxsdp_info* info) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  while (H->status == PROXSDP_STATUS_RUNNING) {
    const int rc = proxsdp_step(H, H->opt.check_every, nullptr);
    if (rc) return rc;
  }
  HIP_OK(hipStreamSynchronize(H->st));
  if (info) {
    H->last.status = H->status;
    H->last.time_s = H->time_s;
    *info = H->last;
  }
  return PROXSDP_OK;
}

int proxsdp_get_factors(proxsdp_handle* H, double* V, double* lambda, int32_t* r_out) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  const int par = (H->iters - 1) & 1;
  const int r = H->r_old;
  if (r_out) *r_out = r;
  if (r == 0) return PROXSDP_OK;
  if (V) {
    std::vector<double> tmp((size_t)H->n * KMAX);
    HIP_OK(hipMemcpyAsync(tmp.data(), H->V[par], tmp.size() * sizeof(double), hipMemcpyDeviceToHost, H->st));
    HIP_OK(hipStreamSynchronize(H->st));
    for (int i = 0; i < H->n; ++i)
      for (int t = 0; t < r; ++t) V[(size_t)i * r + t] = tmp[(size_t)i * KMAX + t];
  }
  if (lambda) {
    HIP_OK(hipMemcpyAsync(lambda, H->small + lam_slot(par), r * sizeof(double), hipMemcpyDeviceToHost, H->st));
    HIP_OK(hipStreamSynchronize(H->st));
  }
  return PROXSDP_OK;
}

int proxsdp_set_state(proxsdp_handle* H, int32_t r, const double* V, const double* lambda,
                      const double* y) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  const int n = H->n;
  const Host& h = H->h;
  const int rmax = std::min(H->opt.full_eig ? n : H->r_cap, KMAX);
  if (r < 0 || r > rmax)
    return fail(PROXSDP_ERR_INVALID, "r must be in [0, " + std::to_string(rmax) + "]");
  if (r > 0 && (!V || !lambda)) return fail(PROXSDP_ERR_INVALID, "V and lambda are required for r > 0");
  for (int t = 0; t < r; ++t)
    if (!(lambda[t] >= 0.0) || !std::isfinite(lambda[t]))
      return fail(PROXSDP_ERR_INVALID, "lambda must be finite and >= 0 (X is PSD)");
  for (size_t t = 0; t < (size_t)n * r; ++t)
    if (!std::isfinite(V[t])) return fail(PROXSDP_ERR_INVALID, "V has a non-finite entry");
  if (y)
    for (int i = 0; i < H->rows; ++i) {
      if (!std::isfinite(y[i])) return fail(PROXSDP_ERR_INVALID, "y has a non-finite entry");
      if (i >= h.m && y[i] > 0.0)
        return fail(PROXSDP_ERR_INVALID, "inequality duals must be <= 0 (Section 1.3 sign)");
    }
  int rc = reset_buffers(H);
  if (rc) return rc;
  hipStream_t st = H->st;
  // factors of X0 into the slot of iteration -1 (parity 1)
  std::vector<double> Vp((size_t)H->npad * KMAX, 0.0);
  for (int i = 0; i < n; ++i)
    for (int t = 0; t < r; ++t) Vp[(size_t)i * KMAX + t] = V[(size_t)i * r + t];
  std::vector<double> lam(r);
  for (int t = 0; t < r; ++t) lam[t] = lambda[t];
  // y0 in the scaled rows, M(X0) (the dual step's previous M(X)), ||X0||_F^2
  std::vector<double> ys(H->rows, 0.0), mx(H->rows, 0.0);
  for (int i = 0; i < H->rows; ++i) ys[i] = y ? y[i] * h.scale[i] : 0.0;
  auto xab = [&](int a, int b) {
    double acc = 0.0;
    for (int t = 0; t < r; ++t) acc += lam[t] * V[(size_t)a * r + t] * V[(size_t)b * r + t];
    return acc;
  };
  std::vector<double> uv((size_t)std::max(h.n_r1, 1) * std::max(r, 1), 0.0);
  for (int q = 0; q < h.n_r1; ++q)
    for (int t = 0; t < r; ++t) {
      double acc = 0.0;
      for (int i = 0; i < n; ++i) acc += h.r1_u[(size_t)q * h.npad + i] * V[(size_t)i * r + t];
      uv[(size_t)q * r + t] = acc;
    }
  for (int i = 0; i < H->rows; ++i) {
    double acc = 0.0;
    for (int e = h.row_ptr[i]; e < h.row_ptr[i + 1]; ++e) acc += h.row_w[e] * xab(h.row_a[e], h.row_b[e]);
    const int q = h.row_r1[i];
    if (q >= 0) {
      double a1 = 0.0;
      for (int t = 0; t < r; ++t) a1 += lam[t] * uv[(size_t)q * r + t] * uv[(size_t)q * r + t];
      acc += h.r1_sigma[q] * a1;
    }
    mx[i] = acc;
  }
  double sc2[2] = {0.0, 0.0};   // ||X0||_F^2, cleared non-finite flag
  for (int a = 0; a < r; ++a)
    for (int b = 0; b < r; ++b) {
      double g = 0.0;
      for (int i = 0; i < n; ++i) g += V[(size_t)i * r + a] * V[(size_t)i * r + b];
      sc2[0] += lam[a] * lam[b] * g * g;
    }
  HIP_OK(hipMemcpyAsync(H->V[1], Vp.data(), Vp.size() * sizeof(double), hipMemcpyHostToDevice, st));
  if (r > 0)
    HIP_OK(hipMemcpyAsync(H->small + lam_slot(1), lam.data(), r * sizeof(double),
                          hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(H->y, ys.data(), ys.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(H->y_old, ys.data(), ys.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(H->MX, mx.data(), mx.size() * sizeof(double), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(H->MX_old, mx.data(), mx.size() * sizeof(double), hipMemcpyHostToDevice, st));
  // W0 = X0 - alpha (C - M*(y0)) from the factors (its record is not used);
  // the finalisation it runs overwrites ||X||^2 of parity 1, set afterwards
  H->r_old = r;
  const int r_work = H->opt.full_eig ? n : std::max(H->r, std::min(std::max(r, 1), H->r_cap));
  H->k = H->full ? 16 : (H->opt.block ? H->opt.block : k_for_r(r_work));   // k >= r
  H->r = r;
  pattern_and_write(H, 1, RING - 1);
  H->r = r_work;
  HIP_OK(hipMemcpyAsync(H->small + SL::SC + S_X2 + 1, &sc2[0], sizeof(double), hipMemcpyHostToDevice, st));
  HIP_OK(hipMemcpyAsync(H->small + SL::SC + S_NONFINITE, &sc2[1], sizeof(double), hipMemcpyHostToDevice, st));
  // Ritz basis: the given factors first
  rc = warm_start(H, H->V[1], r);
  if (rc) return rc;
  HIP_OK(hipStreamSynchronize(st));   // the host buffers above end here
  return PROXSDP_OK;
}

int proxsdp_saved_count(proxsdp_handle* H, int32_t* count) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  if (count) *count = (int32_t)H->saved.size();
  return PROXSDP_OK;
}

int proxsdp_get_saved(proxsdp_handle* H, int32_t idx, double* V, double* lambda, double* y,
                      int32_t* r_out, int32_t* iter_out) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  if (idx < 0 || idx >= (int)H->saved.size())
    return fail(PROXSDP_ERR_INVALID, "saved index out of range");
  const proxsdp_handle::Saved& sv = H->saved[idx];
  if (r_out) *r_out = sv.r;
  if (iter_out) *iter_out = sv.iter;
  if (V && sv.r > 0) std::memcpy(V, sv.V.data(), (size_t)H->n * sv.r * sizeof(double));
  if (lambda && sv.r > 0) std::memcpy(lambda, sv.lam.data(), (size_t)sv.r * sizeof(double));
  if (y) std::memcpy(y, sv.y.data(), (size_t)H->rows * sizeof(double));
  return PROXSDP_OK;
}

int proxsdp_round_hyperplane(proxsdp_handle* H, int32_t trials, const double* g, double* values,
                             int8_t* x_best, int32_t* best) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  if (trials < 1 || trials > ROUND_MAX_TRIALS)
    return fail(PROXSDP_ERR_INVALID, "trials must be in [1, " + std::to_string(ROUND_MAX_TRIALS) + "]");
  const int r = H->r_old;
  if (r > 0 && !g) return fail(PROXSDP_ERR_INVALID, "g is NULL");
  if (g)
    for (int64_t t = 0; t < (int64_t)trials * r; ++t)
      if (!std::isfinite(g[t])) return fail(PROXSDP_ERR_INVALID, "g has a non-finite entry");
  hipStream_t st = H->st;
  const int par = (H->iters - 1) & 1;
  const int n = H->n;
  if (r > 0)
    HIP_OK(hipMemcpyAsync(H->round_g, g, (size_t)trials * r * sizeof(double), hipMemcpyHostToDevice, st));
  const int64_t cnt = (int64_t)n * trials;
  hipLaunchKernelGGL(k_round_signs, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, H->V[par], r,
                     H->small + lam_slot(par), H->round_g, trials, n, H->round_x);
  hipLaunchKernelGGL(k_round_values, dim3(ROUND_BLOCKS), dim3(256), 0, st, H->dp, H->round_x, trials,
                     H->round_part);
  hipLaunchKernelGGL(k_round_reduce, dim3(1), dim3(64), 0, st, H->round_part, ROUND_BLOCKS, trials,
                     H->round_val);
  std::vector<double> val(trials);
  HIP_OK(hipMemcpyAsync(val.data(), H->round_val, trials * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  int b = 0;
  for (int t = 1; t < trials; ++t)
    if (val[t] < val[b]) b = t;
  if (values) std::memcpy(values, val.data(), trials * sizeof(double));
  if (best) *best = b;
  if (x_best) {
    std::vector<signed char> xs((size_t)n * trials);
    HIP_OK(hipMemcpyAsync(xs.data(), H->round_x, xs.size(), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) x_best[i] = xs[(size_t)i * trials + b];
  }
  return PROXSDP_OK;
}

int proxsdp_get_state(proxsdp_handle* H, double* V, double* lambda, double* y, int32_t* r_out) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  int rc = proxsdp_get_factors(H, V, lambda, r_out);
  if (rc) return rc;
  if (y) return proxsdp_get_solution(H, nullptr, y, 0);
  return PROXSDP_OK;
}

int proxsdp_get_solution(proxsdp_handle* H, double* X, double* y, int32_t on_device) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  const int n = H->n;
  if (y) {
    std::vector<double> ys(H->rows);
    HIP_OK(hipMemcpyAsync(ys.data(), H->y, H->rows * sizeof(double), hipMemcpyDeviceToHost, H->st));
    HIP_OK(hipStreamSynchronize(H->st));
    for (int i = 0; i < H->rows; ++i) ys[i] /= H->h.scale[i];
    if (on_device)
      HIP_OK(hipMemcpyAsync(y, ys.data(), H->rows * sizeof(double), hipMemcpyHostToDevice, H->st));
    else
      std::memcpy(y, ys.data(), H->rows * sizeof(double));
  }
  if (X) {
    const int par = (H->iters - 1) & 1;
    const int r = H->r_old;
    if (on_device) {
      launch_write(H, X, PROXSDP_FP64, n, H->V[par], r, lam_slot(par), false, false, nullptr);
    } else {
      std::vector<double> V((size_t)n * std::max(r, 1)), lam(std::max(r, 1));
      int32_t rr = 0;
      const int rc = proxsdp_get_factors(H, V.data(), lam.data(), &rr);
      if (rc) return rc;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          double acc = 0;
          for (int t = 0; t < rr; ++t) acc += lam[t] * V[(size_t)i * rr + t] * V[(size_t)j * rr + t];
          X[(size_t)i * n + j] = acc;
        }
    }
  }
  HIP_OK(hipStreamSynchronize(H->st));
  return PROXSDP_OK;
}

// --------------------------------------------------------- projection only
// Context of one stateless projection: the solver's buffers with an empty
// constraint set.
// ---------------------------------------- exact projection for n > KMAX
// proj(S) of Section 2.3.2 through a full symmetric eigendecomposition
// (rocSOLVER dsyevd, divide and conquer) and P = U+ U+^T with U+ the
// eigenvectors of the positive eigenvalues scaled by sqrt(lambda) (rocBLAS
// dgemm).  This is the PD-SDP projection the truncated one is compared with;
// rocBLAS / rocSOLVER get their scratch from the caller's workspace.
struct FullEig {
  rocblas_handle h = nullptr;
  int dev = -1;
};
static FullEig g_fulleig;

static int fulleig_handle(rocblas_handle* out) {
  int dev = 0;
  HIP_OK(hipGetDevice(&dev));
  if (!g_fulleig.h || g_fulleig.dev != dev) {
    if (g_fulleig.h) rocblas_destroy_handle(g_fulleig.h);
    g_fulleig.h = nullptr;
    if (rocblas_create_handle(&g_fulleig.h) != rocblas_status_success)
      return fail(PROXSDP_ERR_HIP, "rocblas_create_handle failed");
    g_fulleig.dev = dev;
  }
  *out = g_fulleig.h;
  return PROXSDP_OK;
}

// Scratch of rocSOLVER dsyevd + rocBLAS dgemm for size n (bytes).
static int fulleig_scratch(int n, size_t* bytes) {
  rocblas_handle h;
  int rc = fulleig_handle(&h);
  if (rc) return rc;
  if (rocblas_start_device_memory_size_query(h) != rocblas_status_success)
    return fail(PROXSDP_ERR_HIP, "rocblas size query failed");
  rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, nullptr, n, nullptr, nullptr,
                   nullptr);
  const double one = 1.0, zero = 0.0;
  rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one, nullptr, n,
                nullptr, n, &zero, nullptr, n);
  size_t sz = 0;
  if (rocblas_stop_device_memory_size_query(h, &sz) != rocblas_status_success)
    return fail(PROXSDP_ERR_HIP, "rocblas size query failed");
  *bytes = sz;
  return PROXSDP_OK;
}

// Eigenvector rows scaled by sqrt(max(lambda, 0)): A holds the eigenvectors
// as rows (dsyevd's column-major columns), D the eigenvalues.
__global__ __launch_bounds__(256) void k_scale_evec_rows(const double* __restrict__ A,
                                                         const double* __restrict__ D, int n,
                                                         double* __restrict__ U) {
  const int64_t cnt = (int64_t)n * n;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < cnt;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / n);
    const double lam = D[j];
    U[t] = lam > 0.0 ? sqrt(lam) * A[t] : 0.0;
  }
}

struct FullLayout {
  double *A, *U, *D, *E;
  int* info;
  void* rb;
  size_t rb_bytes;
};

static size_t full_layout(int n, size_t rb_bytes, void* ws, FullLayout* L) {
  Carver c(ws);
  L->A = c.take<double>((size_t)n * n);
  L->U = c.take<double>((size_t)n * n);
  L->D = c.take<double>(n);
  L->E = c.take<double>(n);
  L->info = c.take<int>(4);
  L->rb = c.take<char>(std::max<size_t>(rb_bytes, 256));
  L->rb_bytes = std::max<size_t>(rb_bytes, 256);
  return c.off + 256;
}

static int project_full_large(const double* S, int n, int64_t lds, double tol_unused, double* P,
                              int64_t ldp, double* evals, double* evecs, int32_t* rank_out,
                              void* ws, size_t ws_bytes, hipStream_t st) {
  (void)tol_unused;
  size_t rb = 0;
  int rc = fulleig_scratch(n, &rb);
  if (rc) return rc;
  FullLayout L{};
  const size_t need = full_layout(n, rb, nullptr, &L);
  if (ws_bytes < need) return fail(PROXSDP_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  full_layout(n, rb, ws, &L);
  rocblas_handle h;
  if ((rc = fulleig_handle(&h))) return rc;
  if (rocblas_set_stream(h, st) != rocblas_status_success)
    return fail(PROXSDP_ERR_HIP, "rocblas_set_stream failed");
  if (rocblas_set_workspace(h, L.rb, L.rb_bytes) != rocblas_status_success)
    return fail(PROXSDP_ERR_HIP, "rocblas_set_workspace failed");
  HIP_OK(hipMemcpy2DAsync(L.A, (size_t)n * sizeof(double), S, (size_t)lds * sizeof(double),
                          (size_t)n * sizeof(double), n, hipMemcpyDeviceToDevice, st));
  if (rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, L.A, n, L.D, L.E, L.info) !=
      rocblas_status_success)
    return fail(PROXSDP_ERR_HIP, "rocsolver_dsyevd failed");
  const int64_t cnt = (int64_t)n * n;
  hipLaunchKernelGGL(k_scale_evec_rows, dim3((unsigned)std::min<int64_t>((cnt + 255) / 256, 4096)),
                     dim3(256), 0, st, L.A, L.D, n, L.U);
  if (P) {
    // column-major view: U^T has the scaled eigenvectors as columns; P = U^T U
    const double one = 1.0, zero = 0.0;
    if (rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_transpose, n, n, n, &one, L.U, n,
                      L.U, n, &zero, P, (rocblas_int)ldp) != rocblas_status_success)
      return fail(PROXSDP_ERR_HIP, "rocblas_dgemm failed");
  }
  std::vector<double> D(n);
  int info = 0;
  HIP_OK(hipMemcpyAsync(D.data(), L.D, n * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_OK(hipMemcpyAsync(&info, L.info, sizeof(int), hipMemcpyDeviceToHost, st));
  if (evecs) {
    std::vector<double> A((size_t)n * n);
    HIP_OK(hipMemcpyAsync(A.data(), L.A, A.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (int t = 0; t < n; ++t) {
      const int j = n - 1 - t;   // descending
      for (int i = 0; i < n; ++i) evecs[(size_t)i * n + t] = A[(size_t)j * n + i];
    }
  }
  HIP_OK(hipStreamSynchronize(st));
  if (info != 0) return fail(PROXSDP_ERR_HIP, "dsyevd did not converge (info " + std::to_string(info) + ")");
  int pos = 0;
  for (int t = 0; t < n; ++t) {
    if (evals) evals[t] = D[n - 1 - t];
    pos += D[n - 1 - t] > 0.0;
  }
  if (rank_out) *rank_out = pos;
  return PROXSDP_OK;
}

static size_t project_layout(proxsdp_handle* H, int n, int r, void* ws, double** gpart) {
  H->n = n;
  H->npad = roundup(n, TILE);
  H->rows = 0;
  H->full = (n <= KMAX);
  H->r = r;
  H->k = H->full ? 16 : k_for_r(r);
  H->k_cap = H->k;
  H->ch = chunking(H->npad);
  H->nsl = n_slices(H->npad);
  Carver c(ws);
  const int npad = H->npad;
  H->B[0] = c.take<double>((size_t)npad * H->k);
  H->B[1] = c.take<double>((size_t)npad * H->k);
  H->Z = c.take<double>((size_t)npad * H->k);
  H->part = c.take<double>((size_t)H->ch.nchunks * npad * H->k);
  H->gram_part = c.take<double>((size_t)H->nsl * 3 * H->k * H->k);
  H->small = c.take<double>(SL::TOTAL);
  H->V[0] = c.take<double>((size_t)npad * KMAX);
  H->V[1] = H->V[0];
  H->fac_part = c.take<double>((size_t)std::max(H->nsl, 1) * FAC_STRIDE);
  *gpart = c.take<double>(256);
  return c.off + 256;
}

int proxsdp_project_workspace_size(int32_t n, int32_t r, int32_t precision, size_t* bytes) {
  g_err.clear();
  if (!bytes) return fail(PROXSDP_ERR_INVALID, "bytes is NULL");
  if (n < 1) return fail(PROXSDP_ERR_INVALID, "n must be >= 1");
  if (r < 0) return fail(PROXSDP_ERR_INVALID, "r must be >= 0");
  if (precision != PROXSDP_FP64) return fail(PROXSDP_ERR_UNSUPPORTED, "only PROXSDP_FP64 is built");
  const int re = (r == 0 || r >= n) ? n : r;
  if (n > KMAX && re == n) {   // exact projection through rocSOLVER
    size_t rb = 0;
    const int rc = fulleig_scratch(n, &rb);
    if (rc) return rc;
    FullLayout L{};
    *bytes = full_layout(n, rb, nullptr, &L);
    return PROXSDP_OK;
  }
  if (n > KMAX && re > 48)
    return fail(PROXSDP_ERR_UNSUPPORTED, "for n > 64 the target rank must be <= 48 (or 0 / n for the exact projection)");
  proxsdp_handle H;
  double* g = nullptr;
  *bytes = project_layout(&H, n, re, nullptr, &g);
  return PROXSDP_OK;
}

// aproj / proj of a device matrix for the paths that need no library routine
// (one-workgroup Jacobi for n <= KMAX, partial eigensolve otherwise), with the
// device memory at `ws` (project_layout bytes, 256-byte aligned).
static int project_core(const double* Sd, int n, int64_t lds, int re, double tol, double* P,
                        int64_t ldp, double* evals, double* evecs, int32_t* rank_out, void* ws,
                        hipStream_t st) {
  int rc = 0;
  proxsdp_handle H;
  H.st = st;
  double* gpart = nullptr;
  project_layout(&H, n, re, ws, &gpart);
  H.dp.n = n;
  H.dp.npad = H.npad;
  H.dp.tiles_side = H.npad / TILE;
  zero(H.small, SL::TOTAL, st);
  zero(H.V[0], (size_t)H.npad * KMAX, st);
  const int lam_off = lam_slot(0);
  if (H.full) {
    const size_t lds_b = (2 * (size_t)n * (n + 1) + n + 3 * (KMAX / 2 + 1)) * sizeof(double) + (KMAX + 4) * sizeof(int);
    hipLaunchKernelGGL(k_full_eig, dim3(1), dim3(1024), lds_b, st, Sd, lds, n, H.V[0], re, H.V[0], 0,
                       H.small, lam_off, 0, (const double*)nullptr, H.npad, H.fac_part);
  } else {
    const int k = H.k;
    const int64_t cnt = (int64_t)H.npad * k;
    hipLaunchKernelGGL(k_fill_basis, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, H.B[0], k,
                       (const double*)nullptr, 0, 0, n, H.npad, 12345u);
    H.bcur = 0;
    const int gblocks = std::min(256, (n + 3) / 4);
    hipLaunchKernelGGL(k_gersh_dense, dim3(gblocks), dim3(256), 0, st, Sd, lds, n, gpart);
    hipLaunchKernelGGL(k_reduce_min, dim3(1), dim3(256), 0, st, gpart, gblocks, H.small, (int)S_GERSH);
    bool ok = false;
    const int max_rounds = 600;
    for (int rd = 0; rd < max_rounds; ++rd) {
      const double* Bc = H.B[H.bcur];
      double* Bn = H.B[1 - H.bcur];
      launch_block(Sd, lds, n, H.npad, Bc, k, H.part, H.ch, false, st);
      launch_reduce(H.part, H.ch.nchunks, H.Z, Bc, nullptr, H.npad, k, H.gram_part, 0, 0.0, 1.0, true, st);
      const int n_unshifted = 6;
      launch_rr(H.gram_part, H.nsl, H.small, k, re, lam_off, rd >= n_unshifted ? 1 : 0, 1e-15, st,
                0);
      if (rd == n_unshifted - 1) hipLaunchKernelGGL(k_set_lower_bound, dim3(1), dim3(64), 0, st, H.small);
      launch_rowwise(&H, Bc, H.V[0], re, H.V[0], 0, Bn, st);
      const bool check = (rd % 4 == 3) || rd == max_rounds - 1;
      if (check) {
        double mr = 1.0;
        if ((rc = true_maxres(&H, re, &mr))) return rc;
        if (mr <= tol) { ok = true; break; }
      }
      H.bcur = 1 - H.bcur;
    }
    if (!ok) {
      HIP_OK(hipStreamSynchronize(st));
      return fail(PROXSDP_ERR_UNSUPPORTED, "partial eigensolve did not reach tol within the pass budget");
    }
  }
  if (P) launch_write(&H, P, PROXSDP_FP64, ldp, H.V[0], re, lam_off, false, false, nullptr);
  std::vector<double> theta(std::max(re, 1));
  HIP_OK(hipMemcpyAsync(theta.data(), H.small + SL::THETA, re * sizeof(double), hipMemcpyDeviceToHost, st));
  if (evecs) {
    std::vector<double> tmp((size_t)n * KMAX);
    HIP_OK(hipMemcpyAsync(tmp.data(), H.V[0], tmp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i)
      for (int t = 0; t < re; ++t) evecs[(size_t)i * re + t] = tmp[(size_t)i * KMAX + t];
  }
  HIP_OK(hipStreamSynchronize(st));
  if (evals) std::memcpy(evals, theta.data(), re * sizeof(double));
  if (rank_out) {
    int c = 0;
    for (int t = 0; t < re; ++t) c += theta[t] > 0.0;
    *rank_out = c;
  }
  return PROXSDP_OK;
}

int proxsdp_project_psd(const void* S, int32_t n, int64_t lds, int32_t r, int32_t precision,
                        double tol, void* P, int64_t ldp, double* evals, double* evecs,
                        int32_t* rank_out, void* ws, size_t ws_bytes, void* stream) {
  g_err.clear();
  if (!S) return fail(PROXSDP_ERR_INVALID, "S is NULL");
  if (n < 1 || lds < n) return fail(PROXSDP_ERR_INVALID, "need n >= 1 and lds >= n");
  if (P && ldp < n) return fail(PROXSDP_ERR_INVALID, "ldp < n");
  size_t need = 0;
  int rc = proxsdp_project_workspace_size(n, r, precision, &need);
  if (rc) return rc;
  if (!ws) return fail(PROXSDP_ERR_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % 256) return fail(PROXSDP_ERR_WORKSPACE, "workspace not 256-byte aligned");
  if (ws_bytes < need) return fail(PROXSDP_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  if ((rc = set_lds_limits())) return rc;
  if (!(tol > 0)) tol = 1e-12;
  const int re = (r == 0 || r >= n) ? n : r;
  if (n > KMAX && re == n)
    return project_full_large(static_cast<const double*>(S), n, lds, tol, static_cast<double*>(P), ldp,
                              evals, evecs, rank_out, ws, ws_bytes, static_cast<hipStream_t>(stream));
  return project_core(static_cast<const double*>(S), n, lds, re, tol, static_cast<double*>(P), ldp,
                      evals, evecs, rank_out, ws, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------ allocation-free projection
// Device memory of proxsdp_project_psd_noalloc: one file-scope array, which
// every GPU the library runs on holds (its own copy) until the process ends.
// Host code must not pass `scratch` itself to a kernel (that is a host-side
// stand-in, not a device address): its device address is looked up once per
// device with hipGetSymbolAddress and kept in g_scratch_dev.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(32) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

static int scratch_address(void** out) {
  int dev = -1;
  HIP_OK(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(PROXSDP_ERR_UNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PROXSDP_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PROXSDP_OK;
}

int proxsdp_project_psd_noalloc(const void* S, int32_t n, int64_t lds, int32_t r, int32_t precision,
                                double tol, void* P, int64_t ldp, double* evals, double* evecs,
                                int32_t* rank_out, void* stream) {
  g_err.clear();
  if (!S) return fail(PROXSDP_ERR_INVALID, "S is NULL");
  if (n < 1 || lds < n) return fail(PROXSDP_ERR_INVALID, "need n >= 1 and lds >= n");
  if (P && ldp < n) return fail(PROXSDP_ERR_INVALID, "ldp < n");
  const int re = (r == 0 || r >= n) ? n : r;
  if (r >= 0 && n > KMAX && re == n)
    return fail(PROXSDP_ERR_UNSUPPORTED,
                "the exact projection for n > 64 goes through rocSOLVER, which allocates; "
                "use proxsdp_project_psd");
  size_t need = 0;
  int rc = proxsdp_project_workspace_size(n, r, precision, &need);
  if (rc) return rc;
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(PROXSDP_ERR_WORKSPACE, "needs " + std::to_string(need) +
                " bytes of scratch; the static scratch holds " +
                std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes (use proxsdp_project_psd)");
  if ((rc = set_lds_limits())) return rc;
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  if (!(tol > 0)) tol = 1e-12;
  return project_core(static_cast<const double*>(S), n, lds, re, tol, static_cast<double*>(P), ldp,
                      evals, evecs, rank_out, ws, static_cast<hipStream_t>(stream));
}

int proxsdp_reset(proxsdp_handle* H) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  return init_state(H);
}

int proxsdp_profile_enable(proxsdp_handle* H, int32_t enable) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  if (enable) {
    while ((int)H->ev_pass.size() < 2 * PROF_MAX) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      H->ev_pass.push_back(e);
    }
    while ((int)H->ev_write.size() < 2 * PROF_MAX) {
      hipEvent_t e;
      HIP_OK(hipEventCreate(&e));
      H->ev_write.push_back(e);
    }
  }
  H->prof = enable != 0;
  H->n_pass = 0;
  H->n_write = 0;
  H->prof_k.clear();
  H->prof_r.clear();
  return PROXSDP_OK;
}

int proxsdp_profile_totals(proxsdp_handle* H, double* out, int32_t count) {
  g_err.clear();
  if (!H || !out) return fail(PROXSDP_ERR_INVALID, "handle or out is NULL");
  HIP_OK(hipStreamSynchronize(H->st));
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const double np2 = (double)H->npad * H->npad, n2 = (double)H->n * H->n;
  const int ts = H->npad / TILE;
  const double pair_cells = (double)ts * (ts + 1) / 2 * TILE * TILE;
  for (int i = 0; i < H->n_pass; ++i) {
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, H->ev_pass[2 * i], H->ev_pass[2 * i + 1]));
    v[0] += ms;
    v[2] += 2.0 * np2 * (i < (int)H->prof_k.size() ? H->prof_k[i] : H->k);
    v[3] += (double)H->wbytes * np2;
  }
  for (int i = 0; i < H->n_write; ++i) {
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, H->ev_write[2 * i], H->ev_write[2 * i + 1]));
    v[4] += ms;
    v[6] += 2.0 * pair_cells * (i < (int)H->prof_r.size() ? H->prof_r[i] : H->r);
    v[7] += (double)H->wbytes * n2;
  }
  v[1] = H->n_pass;
  v[5] = H->n_write;
  for (int i = 0; i < count && i < 8; ++i) out[i] = v[i];
  H->prof = false;
  return PROXSDP_OK;
}

int proxsdp_profile_read(proxsdp_handle* H, double* pass_ms, int32_t* pass_count, double* write_ms,
                         int32_t* write_count) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  HIP_OK(hipStreamSynchronize(H->st));
  double tp = 0, tw = 0;
  for (int i = 0; i < H->n_pass; ++i) {
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, H->ev_pass[2 * i], H->ev_pass[2 * i + 1]));
    tp += ms;
  }
  for (int i = 0; i < H->n_write; ++i) {
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, H->ev_write[2 * i], H->ev_write[2 * i + 1]));
    tw += ms;
  }
  if (pass_ms) *pass_ms = tp;
  if (pass_count) *pass_count = H->n_pass;
  if (write_ms) *write_ms = tw;
  if (write_count) *write_count = H->n_write;
  H->prof = false;
  return PROXSDP_OK;
}

int proxsdp_rank_path(proxsdp_handle* H, int32_t* iters, int32_t* ranks, int32_t* reasons,
                      int32_t cap, int32_t* count) {
  g_err.clear();
  if (!H) return fail(PROXSDP_ERR_INVALID, "handle is NULL");
  const int n = (int)H->path_it.size();
  if (count) *count = n;
  for (int i = 0; i < n && i < cap; ++i) {
    if (iters) iters[i] = H->path_it[i];
    if (ranks) ranks[i] = H->path_r[i];
    if (reasons) reasons[i] = H->path_why[i];
  }
  return PROXSDP_OK;
}

int proxsdp_debug_scalars(proxsdp_handle* H, double* out, int32_t count) {
  g_err.clear();
  if (!H || !out) return fail(PROXSDP_ERR_INVALID, "NULL argument");
  const int c1 = std::min<int>(count, 64);
  if (c1 > 0)
    HIP_OK(hipMemcpyAsync(out, H->small + SL::SC, c1 * sizeof(double), hipMemcpyDeviceToHost, H->st));
  if (count > 64) {
    const int c2 = std::min<int>(count - 64, KMAX);
    HIP_OK(hipMemcpyAsync(out + 64, H->small + SL::THETA, c2 * sizeof(double), hipMemcpyDeviceToHost, H->st));
  }
  HIP_OK(hipStreamSynchronize(H->st));
  return PROXSDP_OK;
}

void proxsdp_destroy(proxsdp_handle* H) { delete H; }

const char* proxsdp_last_error(void) { return g_err.c_str(); }

const char* proxsdp_version(void) { return "proxsdp-mi355x 0.1 (gfx950, FP64)"; }

}  // extern "C"
