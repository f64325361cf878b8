// Host-side validation and preprocessing of libproxsdp (duplicate summing,
// row scaling, sparsity pattern and tile buckets, ||M||_2) exercised through
// proxsdp_workspace_size, which makes no HIP call: built with AddressSanitizer
// and UndefinedBehaviorSanitizer on the host code only, it runs without a GPU.
// Valid problems of several sizes (1 ... 300, ragged against the 64-wide
// tiles), kinds (diagonal rows, a rank-one row, inequality rows) and storage
// precisions must be accepted; malformed ones must be refused.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>
#include "proxsdp.h"

struct Prob {
  int n, m, p;
  std::vector<int32_t> ci, cj, ar, ai, aj, r1row;
  std::vector<double> cv, av, b, h, r1s, r1u;
  proxsdp_problem view() {
    proxsdp_problem q{};
    q.n = n; q.m = m; q.p = p;
    q.nnz_c = (int64_t)ci.size(); q.c_i = ci.data(); q.c_j = cj.data(); q.c_v = cv.data();
    q.nnz_a = (int64_t)ar.size(); q.a_row = ar.data(); q.a_i = ai.data(); q.a_j = aj.data(); q.a_v = av.data();
    q.n_r1 = (int32_t)r1row.size(); q.r1_row = r1row.data(); q.r1_sigma = r1s.data(); q.r1_u = r1u.data();
    q.b = b.data(); q.h = h.data();
    return q;
  }
};

static Prob graph(int n, double pe, unsigned seed, bool equip, bool dup) {
  std::mt19937 g(seed);
  std::uniform_real_distribution<double> U(0, 1);
  Prob P{}; P.n = n; P.m = n + (equip ? 1 : 0); P.p = 0;
  std::vector<double> deg(n, 0);
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (U(g) < pe) {
        P.ci.push_back(i); P.cj.push_back(j); P.cv.push_back(equip ? -1.0 : 0.25);
        if (dup) { P.ci.push_back(i); P.cj.push_back(j); P.cv.push_back(0.0); }
        deg[i] += 1; deg[j] += 1;
      }
  for (int i = 0; i < n; ++i) { P.ci.push_back(i); P.cj.push_back(i); P.cv.push_back(equip ? deg[i] : -deg[i] / 4); }
  for (int i = 0; i < n; ++i) { P.ar.push_back(i); P.ai.push_back(i); P.aj.push_back(i); P.av.push_back(1.0); P.b.push_back(1.0); }
  if (equip) { P.r1row.push_back(n); P.r1s.push_back(1.0); P.r1u.assign(n, 1.0); P.b.push_back(0.0); }
  return P;
}

static Prob with_ineq(int n, unsigned seed) {
  Prob P = graph(n, 0.1, seed, false, false);
  std::mt19937 g(seed + 7);
  std::uniform_int_distribution<int> I(0, n - 1);
  for (int t = 0; t < 3 * n; ++t) {
    int a = I(g), c = I(g);
    if (a == c) continue;
    if (a > c) std::swap(a, c);
    const int row = P.m + P.p;
    P.ar.push_back(row); P.ai.push_back(a); P.aj.push_back(a); P.av.push_back(1.0);
    P.ar.push_back(row); P.ai.push_back(c); P.aj.push_back(c); P.av.push_back(1.0);
    P.ar.push_back(row); P.ai.push_back(a); P.aj.push_back(c); P.av.push_back(-1.0);
    P.h.push_back(0.5);
    P.p += 1;
  }
  return P;
}

static int ws(Prob& P, int prec, int full) {
  proxsdp_options o; proxsdp_default_options(&o);
  o.precision = prec; o.full_eig = full;
  proxsdp_problem q = P.view();
  size_t bytes = 0;
  const int rc = proxsdp_workspace_size(&q, &o, &bytes);
  return rc == 0 ? (bytes > 0 ? 0 : -99) : rc;
}

int main() {
  int bad = 0;
  for (int n : {1, 2, 17, 50, 64, 65, 130, 300}) {
    for (int kind = 0; kind < 3; ++kind) {
      Prob P = kind == 2 ? with_ineq(n, n) : graph(n, 0.2, n, kind == 1, n % 2 == 0);
      for (int prec = 0; prec < 3; ++prec) {
        const int rc = ws(P, prec, 0);
        if (rc) { printf("n=%d kind=%d prec=%d rc=%d %s\n", n, kind, prec, rc, proxsdp_last_error()); ++bad; }
      }
      if (n <= 64) { const int rc = ws(P, 0, 1); if (rc) { printf("full n=%d rc=%d\n", n, rc); ++bad; } }
    }
  }
  // empty problem pieces
  { Prob P{}; P.n = 5; P.m = 0; P.p = 0; const int rc = ws(P, 0, 0); printf("empty problem: rc=%d %s\n", rc, proxsdp_last_error()); }
  // invalid inputs must be refused
  { Prob P = graph(10, 0.3, 1, false, false); P.ci[0] = 5; P.cj[0] = 2; if (ws(P, 0, 0) != PROXSDP_ERR_INVALID) { printf("i>j not refused\n"); ++bad; } }
  { Prob P = graph(10, 0.3, 1, false, false); P.ai[0] = 10; if (ws(P, 0, 0) != PROXSDP_ERR_INVALID) { printf("range not refused\n"); ++bad; } }
  { Prob P = graph(10, 0.3, 1, false, false); P.av[0] = NAN; if (ws(P, 0, 0) != PROXSDP_ERR_INVALID) { printf("nan not refused\n"); ++bad; } }
  { Prob P = graph(10, 0.3, 1, false, false); P.ar[0] = 99; if (ws(P, 0, 0) != PROXSDP_ERR_INVALID) { printf("row not refused\n"); ++bad; } }
  printf("%s (%d problems)\n", bad ? "FAILURES" : "all ok", bad);
  return bad ? 1 : 0;
}
