// Float64 host setup: the tree-independent factor products (App. B) and the
// single-branch dual preconditioner (Sec. IV-D).  Plain loops; run once per
// system.  (The per-node cost update of App. A runs on the device,
// smpc_data.hip.)
//
// Input-space form of the factor step.  App. A writes u = L v + uhat with L a
// basis of ker E and eliminates the coupling; App. B then needs
// Lambda = -(L' Wu L)^{-1}, Phi = Lambda Bbar', Psi = Lambda L'.  Every use of
// these in the solve step is of the form L Lambda L' r, so the library keeps
// only the nu x nu matrix
//     P = L (L' Wu L)^{-1} L' = Wu^{-1} - Wu^{-1} E' (E Wu^{-1} E')^{-1} E Wu^{-1},
// which does not depend on the basis L and is computed here from two
// Cholesky factorisations (of Wu and of E Wu^{-1} E').  The particular
// solution is the minimum-norm one, uhat = -E' (E E')^{-1} Ed d.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "smpc_host.h"

namespace smpc {

bool cholesky(std::vector<double>& a, int n) {
  double dmax = 0.0;
  for (int i = 0; i < n; ++i) dmax = std::fmax(dmax, std::fabs(a[(size_t)i * n + i]));
  const double tiny = 1e-13 * (dmax > 0 ? dmax : 1.0);
  for (int j = 0; j < n; ++j) {
    double s = a[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= a[(size_t)j * n + k] * a[(size_t)j * n + k];
    if (!(s > tiny)) return false;
    const double d = std::sqrt(s);
    a[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = a[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= a[(size_t)i * n + k] * a[(size_t)j * n + k];
      a[(size_t)i * n + j] = t / d;
    }
    for (int i = 0; i < j; ++i) a[(size_t)i * n + j] = 0.0;
  }
  return true;
}

void chol_solve(const std::vector<double>& l, int n, double* b) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= l[(size_t)i * n + k] * b[k];
    b[i] = s / l[(size_t)i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int k = i + 1; k < n; ++k) s -= l[(size_t)k * n + i] * b[k];
    b[i] = s / l[(size_t)i * n + i];
  }
}

Csr dense_to_csr(const double* a, int rows, int cols) {
  Csr c;
  c.rp.assign(rows + 1, 0);
  for (int i = 0; i < rows; ++i) {
    for (int j = 0; j < cols; ++j) {
      const double v = a[(size_t)i * cols + j];
      if (v != 0.0) {
        c.ci.push_back(j);
        c.v.push_back(v);
      }
    }
    c.rp[i + 1] = (int32_t)c.ci.size();
  }
  return c;
}

Csr dense_to_csr_transposed(const double* a, int rows, int cols) {
  std::vector<double> t((size_t)rows * cols);
  for (int i = 0; i < rows; ++i)
    for (int j = 0; j < cols; ++j) t[(size_t)j * rows + i] = a[(size_t)i * cols + j];
  return dense_to_csr(t.data(), cols, rows);
}

int sys_factor(smpc_sys* s) {
  const int nu = s->nu, ne = s->ne, nd = s->nd;
  // Wu symmetric positive definite
  double wmax = 0.0;
  for (double v : s->Wu) wmax = std::fmax(wmax, std::fabs(v));
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < i; ++j)
      if (std::fabs(s->Wu[(size_t)i * nu + j] - s->Wu[(size_t)j * nu + i]) > 1e-12 * wmax)
        return set_error(SMPC_ENOTSPD, "Wu is not symmetric (entry %d,%d)", i, j);
  std::vector<double> lw = s->Wu;
  if (!cholesky(lw, nu)) return set_error(SMPC_ENOTSPD, "Wu is not positive definite");
  // Winv = Wu^{-1}
  std::vector<double> winv((size_t)nu * nu, 0.0), col(nu);
  for (int j = 0; j < nu; ++j) {
    std::fill(col.begin(), col.end(), 0.0);
    col[j] = 1.0;
    chol_solve(lw, nu, col.data());
    for (int i = 0; i < nu; ++i) winv[(size_t)i * nu + j] = col[i];
  }
  s->P = winv;
  s->Mu.assign((size_t)nu * nd, 0.0);
  if (ne > 0) {
    // G = Winv E'  (nu x ne),  S = E G  (ne x ne)
    std::vector<double> G((size_t)nu * ne, 0.0), S((size_t)ne * ne, 0.0);
    for (int i = 0; i < nu; ++i)
      for (int r = 0; r < ne; ++r) {
        double acc = 0.0;
        for (int k = 0; k < nu; ++k) acc += winv[(size_t)i * nu + k] * s->E[(size_t)r * nu + k];
        G[(size_t)i * ne + r] = acc;
      }
    for (int a = 0; a < ne; ++a)
      for (int b = 0; b < ne; ++b) {
        double acc = 0.0;
        for (int k = 0; k < nu; ++k) acc += s->E[(size_t)a * nu + k] * G[(size_t)k * ne + b];
        S[(size_t)a * ne + b] = acc;
      }
    std::vector<double> ls = S;
    if (!cholesky(ls, ne)) return set_error(SMPC_ERANK, "E does not have full row rank");
    // P = Winv - G S^{-1} G'
    std::vector<double> sg((size_t)ne * nu);  // S^{-1} G'
    std::vector<double> tmp(ne);
    for (int i = 0; i < nu; ++i) {
      for (int r = 0; r < ne; ++r) tmp[r] = G[(size_t)i * ne + r];
      chol_solve(ls, ne, tmp.data());
      for (int r = 0; r < ne; ++r) sg[(size_t)r * nu + i] = tmp[r];
    }
    for (int i = 0; i < nu; ++i)
      for (int j = 0; j < nu; ++j) {
        double acc = 0.0;
        for (int r = 0; r < ne; ++r) acc += G[(size_t)i * ne + r] * sg[(size_t)r * nu + j];
        s->P[(size_t)i * nu + j] -= acc;
      }
    // Mu = -E' (E E')^{-1} Ed
    std::vector<double> EE((size_t)ne * ne, 0.0);
    for (int a = 0; a < ne; ++a)
      for (int b = 0; b < ne; ++b) {
        double acc = 0.0;
        for (int k = 0; k < nu; ++k) acc += s->E[(size_t)a * nu + k] * s->E[(size_t)b * nu + k];
        EE[(size_t)a * ne + b] = acc;
      }
    if (!cholesky(EE, ne)) return set_error(SMPC_ERANK, "E does not have full row rank");
    std::vector<double> colr(ne);
    for (int c = 0; c < nd; ++c) {
      for (int r = 0; r < ne; ++r) colr[r] = s->Ed[(size_t)r * nd + c];
      chol_solve(EE, ne, colr.data());
      for (int i = 0; i < nu; ++i) {
        double acc = 0.0;
        for (int r = 0; r < ne; ++r) acc += s->E[(size_t)r * nu + i] * colr[r];
        s->Mu[(size_t)i * nd + c] = -acc;
      }
    }
  }
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < i; ++j) {
      const double m = 0.5 * (s->P[(size_t)i * nu + j] + s->P[(size_t)j * nu + i]);
      s->P[(size_t)i * nu + j] = m;
      s->P[(size_t)j * nu + i] = m;
    }
  s->Bc = dense_to_csr(s->B.data(), s->nx, nu);
  s->Btc = dense_to_csr_transposed(s->B.data(), s->nx, nu);
  s->Ac = dense_to_csr(s->A.data(), s->nx, s->nx);
  s->Atc = dense_to_csr_transposed(s->A.data(), s->nx, s->nx);
  int ident = 1;
  for (int i = 0; i < s->nx && ident; ++i)
    for (int j = 0; j < s->nx; ++j)
      if (s->A[(size_t)i * s->nx + j] != (i == j ? 1.0 : 0.0)) {
        ident = 0;
        break;
      }
  s->a_identity = ident;
  return SMPC_OK;
}

// Diagonal of the dual Hessian for one branch of the tree (a chain of N
// nodes with probability one), averaged per dual block (Sec. IV-D).  On a
// chain, z_lin(w) minimises sum_k dv_k' Rbar dv_k + <w, G v>; the Hessian in
// v is 2 (T kron Rbar) with T^{-1}_{kl} = min(k, l) + 1, so the dual Hessian
// is (1/2) G (T^{-1} kron Rbar^{-1}) G'.  Its diagonal entries are
//   psi block, node n, input c:  (n + 1) P_cc / 2
//   state blocks, node n, tank c:
//       (1/2) sum_{m, m' <= n} (n + 1 - max(m, m')) (W_m P W_{m'}')_cc,
//   W_m = A^m B.
// diag is N x 3 (sigma, zeta, psi block means).
void single_branch_precond(const smpc_sys* s, int N, std::vector<double>& diag) {
  const int nx = s->nx, nu = s->nu;
  diag.assign((size_t)N * 3, 0.0);
  double pmean = 0.0;
  for (int c = 0; c < nu; ++c) pmean += s->P[(size_t)c * nu + c];
  pmean /= nu;
  // W_m = A^m B and V_m = W_m P for m < N
  std::vector<std::vector<double>> W(N), V(N);
  W[0] = s->B;
  for (int m = 1; m < N; ++m) {
    W[m].assign((size_t)nx * nu, 0.0);
    for (int i = 0; i < nx; ++i)
      for (int k = 0; k < nx; ++k) {
        const double a = s->A[(size_t)i * nx + k];
        if (a == 0.0) continue;
        for (int j = 0; j < nu; ++j) W[m][(size_t)i * nu + j] += a * W[m - 1][(size_t)k * nu + j];
      }
  }
  for (int m = 0; m < N; ++m) {
    V[m].assign((size_t)nx * nu, 0.0);
    for (int i = 0; i < nx; ++i)
      for (int k = 0; k < nu; ++k) {
        const double w = W[m][(size_t)i * nu + k];
        if (w == 0.0) continue;
        for (int j = 0; j < nu; ++j) V[m][(size_t)i * nu + j] += w * s->P[(size_t)k * nu + j];
      }
  }
  // C[m][m'] = mean_c (V_m W_{m'}')_cc
  std::vector<double> C((size_t)N * N, 0.0);
  for (int m = 0; m < N; ++m)
    for (int mp = 0; mp < N; ++mp) {
      double acc = 0.0;
      for (int c = 0; c < nx; ++c)
        for (int j = 0; j < nu; ++j) acc += V[m][(size_t)c * nu + j] * W[mp][(size_t)c * nu + j];
      C[(size_t)m * N + mp] = acc / nx;
    }
  for (int n = 0; n < N; ++n) {
    double xs = 0.0;
    for (int m = 0; m <= n; ++m)
      for (int mp = 0; mp <= n; ++mp) xs += (double)(n + 1 - (m > mp ? m : mp)) * C[(size_t)m * N + mp];
    diag[(size_t)n * 3 + 0] = 0.5 * xs;
    diag[(size_t)n * 3 + 1] = 0.5 * xs;
    diag[(size_t)n * 3 + 2] = 0.5 * (n + 1) * pmean;
  }
}

}  // namespace smpc
