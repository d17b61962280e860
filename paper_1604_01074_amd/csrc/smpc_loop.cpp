// Closed loop of Alg. 2 around the solver: the plant step of the flow model
// (Sec. II, eq. model) and the performance indicators of Sec. V-B over a
// simulated run.  Float64 host code: one matrix-vector product per step and
// sums over the run, outside the iteration.
#include <cmath>
#include <vector>

#include "smpc_host.h"

using namespace smpc;

extern "C" {

int smpc_plant_step(smpc_sys* s, const double* x, const double* u, const double* d, double* x_next) {
  if (!s || !x || !u || !x_next || (s->nd > 0 && !d)) return set_error(SMPC_EINVAL, "NULL argument");
  const int nx = s->nx, nu = s->nu, nd = s->nd;
  for (int i = 0; i < nx; ++i)
    if (!std::isfinite(x[i])) return set_error(SMPC_ENAN, "NaN or Inf in x");
  for (int j = 0; j < nu; ++j)
    if (!std::isfinite(u[j])) return set_error(SMPC_ENAN, "NaN or Inf in u");
  for (int j = 0; j < nd; ++j)
    if (!std::isfinite(d[j])) return set_error(SMPC_ENAN, "NaN or Inf in d");
  std::vector<double> out(nx);
  for (int i = 0; i < nx; ++i) {
    double acc = 0.0;
    for (int j = 0; j < nx; ++j) acc += s->A[(size_t)i * nx + j] * x[j];
    for (int j = 0; j < nu; ++j) acc += s->B[(size_t)i * nu + j] * u[j];
    for (int j = 0; j < nd; ++j) acc += s->Gd[(size_t)i * nd + j] * d[j];
    out[i] = acc;
  }
  for (int i = 0; i < nx; ++i) {
    if (!std::isfinite(out[i])) return set_error(SMPC_ENAN, "NaN or Inf in the next state");
    x_next[i] = out[i];
  }
  return SMPC_OK;
}

int smpc_closed_loop_kpi(smpc_sys* s, int Hs, const double* u, const double* x, const double* alpha2,
                         const double* u_prev, smpc_kpi* out) {
  if (!s || !u || !x || !u_prev || !out) return set_error(SMPC_EINVAL, "NULL argument");
  if (Hs < 1) return set_error(SMPC_EINVAL, "Hs must be >= 1");
  const int nx = s->nx, nu = s->nu;
  double e = 0.0, du = 0.0, sf = 0.0, vol = 0.0, xs1 = 0.0;
  for (int k = 0; k < Hs; ++k) {
    const double* uk = u + (size_t)k * nu;
    const double* up = k == 0 ? u_prev : u + (size_t)(k - 1) * nu;
    const double* a2 = alpha2 ? alpha2 + (size_t)k * nu : nullptr;
    const double* xk = x + (size_t)k * nx;
    for (int j = 0; j < nu; ++j) {
      e += (s->alpha1[j] + (a2 ? a2[j] : 0.0)) * std::fabs(uk[j]);
      const double dj = uk[j] - up[j];
      du += dj * dj;
    }
    for (int i = 0; i < nx; ++i) {
      const double below = s->xs[i] - xk[i];
      if (below > 0.0) sf += below;
      vol += std::fabs(xk[i]);
    }
  }
  for (int i = 0; i < nx; ++i) xs1 += std::fabs(s->xs[i]);
  out->E = e / Hs;
  out->dU = du / Hs;
  out->S = sf;
  out->R = vol > 0.0 ? xs1 / (vol / Hs) * 100.0 : HUGE_VAL;
  return SMPC_OK;
}

}  // extern "C"
