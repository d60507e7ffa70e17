// Host side of the latsum C ABI: error state, argument checks, the
// quadrature table (Sec. 2.1) and master-grid sizing.
#include <cmath>
#include <cstring>

#include "ls_common.hpp"

namespace ls {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

ls_status check_lattice(const ls_lattice* lat, Lat* out) {
  LS_REQUIRE(lat != nullptr, "lattice descriptor is null");
  LS_REQUIRE(lat->n >= 1, "n must be >= 1 (got %d)", lat->n);
  LS_REQUIRE(std::isfinite(lat->b) && lat->b > 0.0, "b must be finite and > 0");
  LS_REQUIRE(lat->periodic == 0 || lat->periodic == 1, "periodic must be 0 or 1");
  out->n = lat->n;
  out->b = lat->b;
  out->h = lat->b / lat->n;
  out->periodic = lat->periodic;
  for (int l = 0; l < 3; ++l) {
    LS_REQUIRE(lat->L[l] >= 1, "L[%d] must be >= 1 (got %d)", l, lat->L[l]);
    out->L[l] = lat->L[l];
    const long long N = lat->periodic ? (long long)lat->n : (long long)lat->L[l] * lat->n;
    LS_REQUIRE(N <= (1LL << 26), "grid too large on axis %d", l);
    out->N[l] = (int)N;
    // box: k = 0..L-1; periodic: -p..p (L = 2p+1) or -L/2..L/2-1
    out->kmin[l] = lat->periodic ? -(lat->L[l] / 2) : 0;
  }
  return LS_OK;
}

ls_status check_quad(const ls_quad* quad, double h, QuadArg* out) {
  LS_REQUIRE(quad != nullptr && quad->t != nullptr && quad->w != nullptr, "quadrature is null");
  LS_REQUIRE(quad->R >= 1, "quadrature rank must be >= 1");
  if (quad->R > kMaxR) {
    set_error("quadrature rank %d exceeds the supported %d", quad->R, kMaxR);
    return LS_EUNSUPPORTED;
  }
  out->R = quad->R;
  for (int q = 0; q < quad->R; ++q) {
    LS_REQUIRE(std::isfinite(quad->t[q]), "t[%d] must be finite", q);
    LS_REQUIRE(std::isfinite(quad->w[q]), "w[%d] must be finite", q);
    // only t^2 enters the Gaussians (rule U has nodes of both signs)
    out->tau[q] = std::fabs(quad->t[q]) * h;
    out->w[q] = quad->w[q];
  }
  return LS_OK;
}

int master_halfwidth(const Lat& L) {
  int X = 0;
  for (int l = 0; l < 3; ++l) {
    // offsets j = g - p - k n, g in [0, N), p in [0, n), k in images:
    // j in [-(n-1) - kmax n, (N-1) - kmin n]; need -X <= j < X
    const int kmax = L.periodic ? (L.L[l] % 2 ? L.L[l] / 2 : L.L[l] / 2 - 1) : L.L[l] - 1;
    const long long lo = -(long long)(L.n - 1) - (long long)kmax * L.n;
    const long long hi = (long long)(L.N[l] - 1) - (long long)L.kmin[l] * L.n + 1;
    const long long need = (-lo > hi) ? -lo : hi;
    if (need > X) X = (int)need;
  }
  return X;
}

ls_status launch_status(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error("%s: %s", what, hipGetErrorString(e));
    return LS_EHIP;
  }
  return LS_OK;
}

}  // namespace ls

extern "C" {

const char* ls_version(void) { return "latsum 0.1 (gfx950)"; }

const char* ls_last_error(void) { return ls::g_err; }

ls_status ls_quadrature(int32_t rule, int32_t M, double C0, double s, double* t, double* w,
                        int32_t capacity, int32_t* R) {
  ls::clear_error();
  LS_REQUIRE(t != nullptr && w != nullptr && R != nullptr, "null output pointer");
  LS_REQUIRE(M >= 2, "M must be >= 2 (got %d)", M);
  LS_REQUIRE(std::isfinite(C0) && C0 > 0.0, "C0 must be finite and > 0");
  const double hM = C0 * std::log((double)M) / (double)M;
  const double inv_sqrt_pi = 0.56418958354775628695;
  if (rule == LS_RULE_U) {
    const int n = 2 * M + 1;
    LS_REQUIRE(capacity >= n, "capacity %d < %d terms", capacity, n);
    for (int k = -M; k <= M; ++k) {
      t[k + M] = k * hM;
      w[k + M] = hM * inv_sqrt_pi;
    }
    *R = n;
    return LS_OK;
  }
  if (rule == LS_RULE_S) {
    LS_REQUIRE(std::isfinite(s) && s > 0.0, "s must be finite and > 0");
    const int n = M + 1;
    LS_REQUIRE(capacity >= n, "capacity %d < %d terms", capacity, n);
    for (int q = 0; q <= M; ++q) {
      t[q] = s * std::sinh(q * hM);
      w[q] = (q == 0 ? 1.0 : 2.0) * s * hM * std::cosh(q * hM) * inv_sqrt_pi;
    }
    *R = n;
    return LS_OK;
  }
  ls::set_error("unknown quadrature rule %d", rule);
  return LS_EINVAL;
}

ls_status ls_master_halfwidth(const ls_lattice* lat, int32_t* X) {
  ls::clear_error();
  LS_REQUIRE(X != nullptr, "null output pointer");
  ls::Lat L;
  ls_status st = ls::check_lattice(lat, &L);
  if (st != LS_OK) return st;
  *X = ls::master_halfwidth(L);
  return LS_OK;
}

}  // extern "C"
