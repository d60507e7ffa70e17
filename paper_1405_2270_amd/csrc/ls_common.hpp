// Shared host/device helpers of the latsum library (internal header).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdint>
#include <cstdio>

#include "latsum.h"
#include "ls_erfc_fit.hpp"

namespace ls {

// Largest quadrature rank handled; the node table travels as a kernel
// argument (no device allocation).
constexpr int kMaxR = 160;
// word 3 of a raw buffer resource on gfx9-family chips (32-bit data format);
// loads past the resource's byte count return 0
constexpr int kBufferFlags = 0x00020000;
// Largest density rank in the Gram kernels (per-lane accumulators).
constexpr int kMaxRho = 16;

struct QuadArg {
  int R;
  double tau[kMaxR];  // t_q * h: nodes in inverse cells
  double w[kMaxR];
};

struct Lat {
  int n;
  int L[3];
  int N[3];         // cells per axis of the summation grid
  int kmin[3];      // first image index per axis
  double b, h;
  int periodic;
};

// thread-local error text
void set_error(const char* fmt, ...);
void clear_error();

ls_status check_lattice(const ls_lattice* lat, Lat* out);
ls_status check_quad(const ls_quad* quad, double h, QuadArg* out);
int master_halfwidth(const Lat& L);
ls_status launch_status(const char* what);
// rmax[l K + r] = max_x |f_l[r][x]| (one workgroup per rank and axis)
ls_status launch_rank_max(const double* f0, const double* f1, const double* f2, int K, int len0,
                          int len1, int len2, double* rmax, hipStream_t stream);

// Workspaces are 256-byte aligned (as hipMalloc returns): kernels read them
// with 16-byte vector loads at 256-byte aligned offsets.
inline bool ws_aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255) == 0; }

#define LS_REQUIRE(cond, ...)            \
  do {                                   \
    if (!(cond)) {                       \
      ::ls::set_error(__VA_ARGS__);      \
      return LS_EINVAL;                  \
    }                                    \
  } while (0)

// ---------------------------------------------------------------------------
// Cell integrals in grid units (cell size 1), FP64.
// ---------------------------------------------------------------------------

// Integral of exp(-tau^2 y^2) over [y0, y0 + 1].
//
// With u = tau*y, a = tau*(y0 + 1/2) and c = tau/2 the integral is
// (1/tau) * integral over [a - c, a + c] of exp(-u^2) du. Two evaluations:
//  * nearly flat integrand (tau <= 0.35 and |a| tau <= 0.25, hermite_cell):
//    expand around the cell centre, exp(-(a+s)^2) = exp(-a^2) exp(-2as - s^2),
//    whose even part in s has the Hermite series sum_m H_2m(a) s^2m/(2m)!, so
//    integral = exp(-a^2) * sum_m H_2m(a) c^2m / (2m+1)!   (up to 8 terms);
//    this avoids the cancelling difference of two nearly equal erf values.
//  * otherwise the erfc difference on the tail side (or the erf sum across
//    the origin); there erfc(far)/erfc(near) <= ~0.6, so nothing cancels.
// Entries whose near edge is beyond |u| = 27 are below 1e-318 and return 0.
// erfc is erfc_fit (ls_erfc_fit.hpp, relative error about 1e-15); erf(v) is
// taken as 1 - erfc(v): a cell across the origin outside the series range
// has tau > 0.35, so its erf sum is at least erf(0.35) ~ 0.38 and the
// roundings of 1 - erfc add only about 1e-16 relative to it.
__device__ __forceinline__ bool hermite_cell(double tau, double y0) {
  const double a = 0.5 * (tau * y0 + tau * (y0 + 1.0));
  return tau <= 0.35 && fabs(a) * tau <= 0.25;
}

// ea (nullable) receives exp(-a^2), the factor the series multiplies.
__device__ __forceinline__ double hermite_series(double tau, double y0, double* ea) {
  const double a = 0.5 * (tau * y0 + tau * (y0 + 1.0));
  const double c = 0.5 * tau;
  const double c2 = c * c;
  // Terms kept (m < mt): by Indritz's inequality |H_n(x)| <= 1.0865
  // (2^n n!)^(1/2) e^(x^2/2), term m of exp(-a^2) * sum is at most
  // 1.0865 2^m c^2m / ((2m)!^(1/2) (2m+1)), and these fall by more than 2c^2
  // from one m to the next; mt is the first m where that bound is below 1e-17
  // (of the largest cell of the row, about 1 in these units: c <= 0.175 here).
  const int mt = c < 8.66e-5 ? 2 : c < 2.45e-3 ? 3 : c < 0.0134 ? 4 : c < 0.0378 ? 5
               : c < 0.0766 ? 6 : c < 0.1279 ? 7 : 8;
  const double two_a = 2.0 * fabs(a);
  // H_0 = 1, H_1 = 2a, H_{k+1} = 2a H_k - 2k H_{k-1}
  double hkm1 = 1.0, hk = two_a;
  double sum = 1.0, cp = 1.0;
  const double inv_fact[8] = {1.0,
                              1.0 / 6.0,
                              1.0 / 120.0,
                              1.0 / 5040.0,
                              1.0 / 362880.0,
                              1.0 / 39916800.0,
                              1.0 / 6227020800.0,
                              1.0 / 1307674368000.0};
#pragma unroll
  for (int m = 1; m < 8; ++m) {
    if (m >= mt) break;
    // advance twice: k = 2m-1 -> 2m
    double h2 = two_a * hk - 2.0 * (2 * m - 1) * hkm1;  // H_{2m}
    double h3 = two_a * h2 - 2.0 * (2 * m) * hk;        // H_{2m+1}
    hkm1 = h2;
    hk = h3;
    cp *= c2;
    sum = fma(h2 * cp, inv_fact[m], sum);
  }
  const double e = exp(-a * a);
  if (ea) *ea = e;
  return e * sum;
}
__device__ __forceinline__ double hermite_series(double tau, double y0) {
  return hermite_series(tau, y0, nullptr);
}

__device__ __forceinline__ double cell_integral(double tau, double y0) {
  if (tau == 0.0) return 1.0;
  if (hermite_cell(tau, y0)) return hermite_series(tau, y0);
  const double u0 = tau * y0;
  const double u1 = tau * (y0 + 1.0);
  const double k = 0.88622692545275801365 / tau;  // sqrt(pi)/(2 tau)
  if (u0 >= 0.0) {
    if (u0 > 27.0) return 0.0;
    return k * (erfc_fit(u0) - (u1 > 27.0 ? 0.0 : erfc_fit(u1)));
  }
  if (u1 <= 0.0) {
    if (u1 < -27.0) return 0.0;
    return k * (erfc_fit(-u1) - (u0 < -27.0 ? 0.0 : erfc_fit(-u0)));
  }
  return k * ((1.0 - (u1 > 27.0 ? 0.0 : erfc_fit(u1))) + (1.0 - (u0 < -27.0 ? 0.0 : erfc_fit(-u0))));
}

// Shared edges. Outside the series range a cell integral is a fixed
// combination of E(y) = erfc(tau |y|) at its two edges (difference on one
// side of the origin, 2 - E - E across it), so a thread that covers
// consecutive cells y0 = j - delta evaluates each edge once: edge j, between
// cells j-1 and j, at y = j - delta, only where one of the two cells needs it.
__device__ __forceinline__ bool edge_needed(double tau, int j, double delta) {
  return !hermite_cell(tau, (double)(j - 1) - delta) || !hermite_cell(tau, (double)j - delta);
}

__device__ __forceinline__ double edge_value(double tau, double y) {
  const double u = fabs(tau * y);
  return u > 27.0 ? 0.0 : erfc_fit(u);
}
// The same edge value and the Gaussian G(y) = exp(-tau^2 y^2) there (0 beyond
// |tau y| = 27, where it is below 1e-316).
__device__ __forceinline__ double edge_value(double tau, double y, double* gauss) {
  const double u = fabs(tau * y);
  if (u > 27.0) {
    *gauss = 0.0;
    return 0.0;
  }
  return erfc_fit(u, gauss);
}

// Integral over cell [y0, y0 + 1] from its edge values eL = E(y0), eR = E(y0 + 1);
// k = sqrt(pi) / (2 tau) (cell_half_norm), which callers may compute once per node.
__device__ __forceinline__ double cell_half_norm(double tau) { return 0.88622692545275801365 / tau; }
__device__ __forceinline__ double cell_from_edges(double tau, double y0, double eL, double eR,
                                                  double k) {
  if (tau == 0.0) return 1.0;
  if (hermite_cell(tau, y0)) return hermite_series(tau, y0);
  if (y0 >= 0.0) return k * (eL - eR);
  if (y0 + 1.0 <= 0.0) return k * (eR - eL);
  return k * ((1.0 - eL) + (1.0 - eR));
}
__device__ __forceinline__ double cell_from_edges(double tau, double y0, double eL, double eR) {
  return cell_from_edges(tau, y0, eL, eR, cell_half_norm(tau));
}

// A raw buffer resource over `bytes` bytes at p, both uniform across the
// workgroup (taken through readfirstlane, so that the compiler keeps the
// resource in scalar registers): loads take a 32-bit lane offset and read 0
// past the end.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t uniform_rsrc(const void* p, int bytes) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((unsigned long long)hi << 32) | lo),
                                           (short)0, __builtin_amdgcn_readfirstlane(bytes),
                                           kBufferFlags);
}

// sinh(x) for |x| <= 1/4 (Taylor series to x^11: truncation below 1e-17 relative)
__device__ __forceinline__ double sinh_small(double x) {
  const double x2 = x * x;
  double p = 1.0 / 39916800.0;
  p = fma(p, x2, 1.0 / 362880.0);
  p = fma(p, x2, 1.0 / 5040.0);
  p = fma(p, x2, 1.0 / 120.0);
  p = fma(p, x2, 1.0 / 6.0);
  p = fma(p, x2, 1.0);
  return x * p;
}

// Value and derivative of one cell together (the derivative as
// cell_derivative defines it), sharing their Gaussian factor:
//  * series cells (hermite_cell): with a = tau (y0 + 1/2) and c = tau / 2,
//    G(y0) - G(y1) = exp(-(a - c)^2) - exp(-(a + c)^2)
//                  = 2 exp(-a^2) exp(-c^2) sinh(2 a c),
//    exp(-a^2) from the series and |2 a c| = |a| tau <= 1/4; ec = exp(-c^2);
//  * other cells: from the edge values eL, eR and edge Gaussians gL, gR:
//    gL - gR where the two differ by a factor of 2 or more, else the larger
//    one times expm1 of the exponent difference tau^2 (2 y0 + 1), which does
//    not cancel.
// k = cell_half_norm(tau). Returns the value's integral; *deriv gets the derivative.
__device__ __forceinline__ double cell_value_deriv(double tau, double y0, double eL, double eR,
                                                   double gL, double gR, double k, double ec,
                                                   double* deriv) {
  if (tau == 0.0) {
    *deriv = 0.0;
    return 1.0;
  }
  if (hermite_cell(tau, y0)) {
    double ea;
    const double v = hermite_series(tau, y0, &ea);
    const double a = 0.5 * (tau * y0 + tau * (y0 + 1.0));
    *deriv = 2.0 * ea * ec * sinh_small(a * tau);
    return v;
  }
  const double x = tau * tau * (2.0 * y0 + 1.0);
  if (fabs(x) >= 0.6931471805599453)
    *deriv = gL - gR;
  else if (fabs(y0) <= fabs(y0 + 1.0))
    *deriv = -gL * expm1(-x);
  else
    *deriv = gR * expm1(x);
  if (y0 >= 0.0) return k * (eL - eR);
  if (y0 + 1.0 <= 0.0) return k * (eR - eL);
  return k * ((1.0 - eL) + (1.0 - eR));
}

// d/da of the integral of exp(-t^2 (x - a)^2) over a cell, in grid units:
// exp(-tau^2 y0^2) - exp(-tau^2 y1^2) with y1 = y0 + 1, written as the
// larger exponential times expm1 of the exponent difference
// (y1^2 - y0^2 = 2 y0 + 1), which does not cancel.
__device__ __forceinline__ double cell_derivative(double tau, double y0) {
  const double y1 = y0 + 1.0;
  const double t2 = tau * tau;
  const double dsq = 2.0 * y0 + 1.0;
  if (fabs(y0) <= fabs(y1)) {
    const double e = t2 * y0 * y0;
    if (e > 745.0) return 0.0;
    return -exp(-e) * expm1(-t2 * dsq);
  }
  const double e = t2 * y1 * y1;
  if (e > 745.0) return 0.0;
  return exp(-e) * expm1(t2 * dsq);
}

// Cells whose offset from the charge satisfies |y| > support_halfwidth(tau)
// (grid units) have |tau*y| > 28 at both edges: cell_integral and
// cell_derivative return exactly 0 there, so loops may skip them.
__device__ __forceinline__ double support_halfwidth(double tau) {
  return tau > 0.0 ? 28.0 / tau + 2.0 : 1e300;
}

// Node index p and offset delta of a coordinate, (a + b/2)/h = p + delta.
// p = floor((a + b/2)/h) clamped to [0, n-1], so every memory index derived
// from p stays inside its buffer for any input (a NaN position gives NaN
// results, never an out-of-range access). The geometry stays exact after the
// clamp: cell offsets are j - delta with j = g - p - k n, and only the split
// between p and delta moves (delta = 1 when rounding puts a + b/2 at b).
__device__ __forceinline__ void node_offset(double a, double b, double h, int n, int* p,
                                            double* delta) {
  const double s = (a + 0.5 * b) / h;
  double f = floor(s);
  f = fmin(fmax(f, 0.0), (double)(n - 1));  // fmax/fmin map NaN to the other operand
  *p = (int)f;
  *delta = s - f;
}

}  // namespace ls
