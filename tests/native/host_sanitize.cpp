// Host-side setup and closed-loop code run under AddressSanitizer and
// UndefinedBehaviorSanitizer: the factor products of App. B (sys_factor),
// the single-branch dual preconditioner of Sec. IV-D, the plant step of the
// flow model (Sec. V) and the closed-loop KPIs of Sec. V-B, on small random
// systems of several shapes, and their error paths.  No GPU is touched.
// Built and run by tests/test_host_sanitizers.py; prints "ok" and exits 0
// when every check holds.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "smpc_host.h"

namespace smpc {
// the library's error recorder lives with the device code; here the code is
// all a caller sees
int set_error(int code, const char*, ...) { return code; }
}  // namespace smpc

namespace {

int g_fails = 0;
#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      ++g_fails;                                                          \
    }                                                                     \
  } while (0)

double max_abs(const std::vector<double>& v) {
  double m = 0.0;
  for (double a : v) m = std::fmax(m, std::fabs(a));
  return m;
}

// A random system: sparse B, full-row-rank E, SPD Wu (diagonal plus a small
// symmetric coupling), A the identity or a random contraction.
void make_sys(std::mt19937_64& g, int nx, int nu, int nd, int ne, bool ident, smpc_sys& s) {
  std::uniform_real_distribution<double> U(-1.0, 1.0), P(0.5, 2.0);
  std::bernoulli_distribution keep(0.3);
  s.nx = nx, s.nu = nu, s.nd = nd, s.ne = ne;
  s.A.assign((size_t)nx * nx, 0.0);
  for (int i = 0; i < nx; ++i)
    for (int j = 0; j < nx; ++j) s.A[(size_t)i * nx + j] = ident ? (i == j ? 1.0 : 0.0) : 0.3 * U(g) / nx;
  s.B.assign((size_t)nx * nu, 0.0);
  for (auto& b : s.B) b = keep(g) ? U(g) : 0.0;
  s.Gd.assign((size_t)nx * nd, 0.0);
  for (auto& v : s.Gd) v = U(g);
  s.E.assign((size_t)ne * nu, 0.0);
  for (auto& v : s.E) v = U(g);
  s.Ed.assign((size_t)ne * nd, 0.0);
  for (auto& v : s.Ed) v = U(g);
  s.Wu.assign((size_t)nu * nu, 0.0);
  for (int i = 0; i < nu; ++i) {
    s.Wu[(size_t)i * nu + i] = P(g) + 1.0;
    for (int j = 0; j < i; ++j) {
      const double c = 0.05 * U(g) / nu;
      s.Wu[(size_t)i * nu + j] = s.Wu[(size_t)j * nu + i] = c;
    }
  }
  s.umin.assign(nu, 0.0);
  s.umax.assign(nu, 1.0);
  s.xmin.assign(nx, 0.0);
  s.xmax.assign(nx, 10.0);
  s.xs.assign(nx, 2.0);
  s.alpha1.assign(nu, 0.0);
  for (auto& a : s.alpha1) a = P(g);
}

// sys_factor: P = L (L' Wu L)^{-1} L' and uhat = Mu d satisfy E P = 0,
// P Wu P = P, E Mu + Ed = 0; the CSR copies hold exactly B's and A's
// nonzeros; the preconditioner is finite and positive.
void check_factor(std::mt19937_64& g, int nx, int nu, int nd, int ne, bool ident) {
  smpc_sys s;
  make_sys(g, nx, nu, nd, ne, ident, s);
  CHECK(smpc::sys_factor(&s) == SMPC_OK);
  const double tol = 1e-10 * (1.0 + max_abs(s.P));
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j) CHECK(s.P[(size_t)i * nu + j] == s.P[(size_t)j * nu + i]);
  for (int r = 0; r < ne; ++r)
    for (int j = 0; j < nu; ++j) {
      double acc = 0.0;
      for (int k = 0; k < nu; ++k) acc += s.E[(size_t)r * nu + k] * s.P[(size_t)k * nu + j];
      CHECK(std::fabs(acc) <= tol);
    }
  std::vector<double> wp((size_t)nu * nu, 0.0);
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j)
      for (int k = 0; k < nu; ++k) wp[(size_t)i * nu + j] += s.Wu[(size_t)i * nu + k] * s.P[(size_t)k * nu + j];
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j) {
      double acc = 0.0;
      for (int k = 0; k < nu; ++k) acc += s.P[(size_t)i * nu + k] * wp[(size_t)k * nu + j];
      CHECK(std::fabs(acc - s.P[(size_t)i * nu + j]) <= tol);
    }
  for (int r = 0; r < ne; ++r)
    for (int c = 0; c < nd; ++c) {
      double acc = s.Ed[(size_t)r * nd + c];
      for (int k = 0; k < nu; ++k) acc += s.E[(size_t)r * nu + k] * s.Mu[(size_t)k * nd + c];
      CHECK(std::fabs(acc) <= 1e-10 * (1.0 + max_abs(s.Mu)));
    }
  int nnz = 0;
  for (double b : s.B) nnz += b != 0.0;
  CHECK((int)s.Bc.v.size() == nnz && (int)s.Btc.v.size() == nnz);
  CHECK((int)s.Bc.rp.size() == nx + 1 && (int)s.Btc.rp.size() == nu + 1);
  for (int i = 0; i < nx; ++i)
    for (int q = s.Bc.rp[i]; q < s.Bc.rp[i + 1]; ++q) CHECK(s.B[(size_t)i * nu + s.Bc.ci[q]] == s.Bc.v[q]);
  for (int j = 0; j < nu; ++j)
    for (int q = s.Btc.rp[j]; q < s.Btc.rp[j + 1]; ++q) CHECK(s.B[(size_t)s.Btc.ci[q] * nu + j] == s.Btc.v[q]);
  CHECK(s.a_identity == (ident ? 1 : 0));
  for (int N : {1, 2, 7}) {
    std::vector<double> diag;
    smpc::single_branch_precond(&s, N, diag);
    CHECK((int)diag.size() == 3 * N);
    for (double d : diag) CHECK(std::isfinite(d) && d >= 0.0);
    for (int n = 1; n < N; ++n) CHECK(diag[(size_t)n * 3 + 2] > diag[(size_t)(n - 1) * 3 + 2]);
  }
}

void check_factor_errors(std::mt19937_64& g) {
  {
    smpc_sys s;
    make_sys(g, 4, 6, 2, 2, true, s);
    s.Wu[1] += 0.5;  // not symmetric
    CHECK(smpc::sys_factor(&s) == SMPC_ENOTSPD);
  }
  {
    smpc_sys s;
    make_sys(g, 4, 6, 2, 2, true, s);
    s.Wu[(size_t)2 * 6 + 2] = -1.0;  // not positive definite
    CHECK(smpc::sys_factor(&s) == SMPC_ENOTSPD);
  }
  {
    smpc_sys s;
    make_sys(g, 4, 6, 2, 3, true, s);
    for (int k = 0; k < 6; ++k) s.E[(size_t)2 * 6 + k] = s.E[k];  // two equal rows
    CHECK(smpc::sys_factor(&s) == SMPC_ERANK);
  }
}

void check_loop(std::mt19937_64& g) {
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  smpc_sys s;
  make_sys(g, 5, 7, 3, 2, false, s);
  std::vector<double> x(5), u(7), d(3), xn(5);
  for (auto& v : x) v = U(g);
  for (auto& v : u) v = U(g);
  for (auto& v : d) v = U(g);
  CHECK(smpc_plant_step(&s, x.data(), u.data(), d.data(), xn.data()) == SMPC_OK);
  for (int i = 0; i < 5; ++i) {
    double acc = 0.0;
    for (int j = 0; j < 5; ++j) acc += s.A[(size_t)i * 5 + j] * x[j];
    for (int j = 0; j < 7; ++j) acc += s.B[(size_t)i * 7 + j] * u[j];
    for (int j = 0; j < 3; ++j) acc += s.Gd[(size_t)i * 3 + j] * d[j];
    CHECK(std::fabs(acc - xn[i]) <= 1e-14);
  }
  std::vector<double> bad = u;
  bad[3] = NAN;
  CHECK(smpc_plant_step(&s, x.data(), bad.data(), d.data(), xn.data()) == SMPC_ENAN);
  CHECK(smpc_plant_step(&s, nullptr, u.data(), d.data(), xn.data()) == SMPC_EINVAL);
  for (int Hs : {1, 3}) {
    std::vector<double> uu((size_t)Hs * 7), xx((size_t)Hs * 5), a2((size_t)Hs * 7), up(7);
    for (auto& v : uu) v = U(g);
    for (auto& v : xx) v = 3.0 * U(g);
    for (auto& v : a2) v = U(g) + 1.0;
    for (auto& v : up) v = U(g);
    smpc_kpi k{};
    CHECK(smpc_closed_loop_kpi(&s, Hs, uu.data(), xx.data(), a2.data(), up.data(), &k) == SMPC_OK);
    CHECK(std::isfinite(k.E) && std::isfinite(k.dU) && k.S >= 0.0 && k.R > 0.0);
    CHECK(smpc_closed_loop_kpi(&s, Hs, uu.data(), xx.data(), nullptr, up.data(), &k) == SMPC_OK);
  }
  smpc_kpi k{};
  CHECK(smpc_closed_loop_kpi(&s, 0, u.data(), x.data(), nullptr, u.data(), &k) == SMPC_EINVAL);
}

}  // namespace

int main() {
  std::mt19937_64 g(20260412);
  for (bool ident : {true, false}) {
    check_factor(g, 5, 7, 3, 2, ident);
    check_factor(g, 63, 114, 88, 17, ident);  // the network's dimensions
    check_factor(g, 1, 1, 1, 0, ident);       // no coupling
    check_factor(g, 3, 4, 2, 3, ident);       // one free input direction
  }
  check_factor_errors(g);
  check_loop(g);
  if (g_fails) {
    std::fprintf(stderr, "%d checks failed\n", g_fails);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
