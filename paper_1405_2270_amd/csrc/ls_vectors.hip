// Kernel vectors (Sec. 2.1, eqs. C_nD_0, galten_int, master_pot) and their
// assembly over the lattice (Theorem 3.1 / eq. EwaldTensorM0, Lemma 3.2).
//
// Data layout in HBM
//   masters  [M0*3][R][2X]  FP64, entry j + X = cell integral of master cell j
//   factors  f_l [M0*R][N_l] FP64, r = nu*R + q, vector-contiguous
//
// Box assembly from masters (HBM-bound). For output g = rho + m n (residue
// rho in [0, n), block m in [0, L)) the lattice sum over k = 0..L-1 is
//   v[rho + m n] = sum_{d = m-L+1}^{m} beta[d],  beta[d] = master[rho - p + d n],
// a window of length L sliding over the 2L-1 values of one residue class.
// Every window is a suffix of the left half (d < 0) plus a prefix of the
// right half (d >= 0), so one lane per residue computes the left suffix sums
// once (held in registers), then streams the outputs with a running prefix
// sum: each master entry is read once, each output written once, and all
// partial sums add like-signed terms only (no subtraction).
#include "ls_common.hpp"

namespace ls {

// ---------------------------------------------------------------------------
// masters
// ---------------------------------------------------------------------------
// A wave covers 63 consecutive master cells: lane i evaluates the left edge
// of cell base + i and takes the right edge from lane i + 1, so each edge's
// erfc is computed once (lane 63 only supplies an edge).
constexpr int kMasterCellsPerWave = 63;

__global__ __launch_bounds__(256) void k_masters(const double* __restrict__ pos, QuadArg qa,
                                                  double b, double h, int n, int X, int deriv,
                                                  double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int wave = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int jj = wave * kMasterCellsPerWave + lane;  // master cell (edge for lane 63)
  // q slowest: the widest Gaussians (the most cells to evaluate) go first
  const int q = blockIdx.z;
  const int c = blockIdx.y;  // nu*3 + l
  int p;
  double delta;
  node_offset(pos[c], b, h, n, &p, &delta);
  const double tau = qa.tau[q];
  const double y0 = (double)(jj - X) - delta;
  // a wave whose cells all lie beyond the support (exactly 0 in every branch
  // of the cell integral and its derivative) stores the zeros at once
  if (__all(fabs(y0) > support_halfwidth(tau))) {
    if (lane < kMasterCellsPerWave && jj < 2 * X)
      out[((size_t)c * qa.R + q) * (size_t)(2 * X) + jj] = 0.0;
    return;
  }
  double v;
  if (deriv) {
    v = cell_derivative(tau, y0);
  } else {
    const double e = edge_needed(tau, jj - X, delta) ? edge_value(tau, y0) : 0.0;
    const double eR = __shfl_down(e, 1, 64);
    v = h * cell_from_edges(tau, y0, e, eR);
  }
  if (lane < kMasterCellsPerWave && jj < 2 * X)
    out[((size_t)c * qa.R + q) * (size_t)(2 * X) + jj] = v;
}

// ---------------------------------------------------------------------------
// box assembly from masters: one lane per residue class, LMAX >= L
// ---------------------------------------------------------------------------
template <int LMAX>
__global__ __launch_bounds__(256) void k_assemble_box(const double* __restrict__ masters,
                                                       const double* __restrict__ pos,
                                                       const double* __restrict__ Z, QuadArg qa,
                                                       int n,
                                                       int L0, int L1, int L2, double b, double h,
                                                       int X, double* __restrict__ f0,
                                                       double* __restrict__ f1,
                                                       double* __restrict__ f2,
                                                       double* __restrict__ coef) {
  const int R = qa.R;
  const int rho = blockIdx.x * 64 + (threadIdx.x & 63);
  const int q = blockIdx.y * 4 + (threadIdx.x >> 6);
  const int c = blockIdx.z;
  if (rho >= n || q >= R) return;
  const int nu = c / 3, l = c - 3 * (c / 3);
  if (coef != nullptr && rho == 0 && l == 0) coef[nu * R + q] = Z[nu] * qa.w[q];
  const int L = (l == 0) ? L0 : (l == 1 ? L1 : L2);
  const size_t N = (size_t)L * n;
  int p;
  double delta;
  node_offset(pos[c], b, h, n, &p, &delta);
  // beta[d] = mrow[d * n], d in [-(L-1), L-1]
  const double* mrow = masters + ((size_t)c * R + q) * (size_t)(2 * X) + X + rho - p;
  double* out = ((l == 0) ? f0 : (l == 1 ? f1 : f2)) + ((size_t)nu * R + q) * N + rho;
  // suf[e] = sum_{i=e}^{L-2} beta[i - (L-1)] for e in [0, L-2]
  double suf[LMAX > 1 ? LMAX - 1 : 1];
  const double* left = mrow - (ptrdiff_t)(L - 1) * n;
  double acc = 0.0;
#pragma unroll
  for (int e = LMAX - 2; e >= 0; --e) {
    if (e <= L - 2) acc += left[(ptrdiff_t)e * n];
    suf[e] = acc;
  }
  double pre = 0.0;
#pragma unroll
  for (int m = 0; m < LMAX; ++m) {
    if (m < L) {
      pre += mrow[(ptrdiff_t)m * n];
      const double s = (m <= L - 2) ? suf[m] : 0.0;
      out[(ptrdiff_t)m * n] = s + pre;
    }
  }
}

// ---------------------------------------------------------------------------
// box assembly with the master window in LDS (kernel vectors fused in)
// ---------------------------------------------------------------------------
// One workgroup per (atom, axis, q) vector. The master cells the vector
// needs, j in [-p - (L-1) n, N - p), are generated into LDS exactly as
// k_masters generates them (shared edges across the lanes of a wave; cells
// beyond the Gaussian's support are exact zeros and not evaluated), then the
// residue-class sums of k_assemble_box run on them: beta[d] of residue rho is
// window entry rho + (d + L - 1) n, the same values added in the same order,
// so the factors equal the stored-masters assembly's bit for bit, without the
// masters' round trip through HBM. The lanes split each residue's L outputs
// into `parts` runs (the prefix sum of a later run first re-adds the earlier
// terms in the same order). Optionally the row maximum max_g |f_l[r][g]|
// goes to rowmax[l K + r].
constexpr int kWindowCells = 8192;  // LDS window: (2L - 1) n <= 8192 cells (64 KB)
// 512 lanes per vector (four waves per SIMD, as the window's 64 KB of LDS
// and 120 registers allow) and runs of at most 8 outputs per lane: 42 us on
// the headline workload, against 45 us with runs of 32, 48-54 us with 256
// lanes or the cell constants hoisted out of the generation loop, 52-70 us
// with 1024 lanes (one workgroup per CU: generation and stores no longer
// overlap; forcing 64 registers spills), and 54 us for the two launches
// through stored masters
#ifndef LS_ASM_THREADS
#define LS_ASM_THREADS 512
#endif
#ifndef LS_ASM_RUN
#define LS_ASM_RUN 8
#endif
#ifndef LS_ASM_MINW
#define LS_ASM_MINW 1
#endif
constexpr int kAsmThreads = LS_ASM_THREADS;
constexpr int kAsmRun = LS_ASM_RUN;  // outputs per lane and residue (suffix registers)

template <int RUN, int BS>
__global__ __launch_bounds__(BS, LS_ASM_MINW) void k_assemble_box_lds(const double* __restrict__ pos,
                                                          const double* __restrict__ Z,
                                                          QuadArg qa, int n, int L0, int L1,
                                                          int L2, double b, double h, int deriv,
                                                          double* __restrict__ f0,
                                                          double* __restrict__ f1,
                                                          double* __restrict__ f2,
                                                          double* __restrict__ coef,
                                                          double* __restrict__ rowmax) {
  constexpr int NW = BS / 64;
  __shared__ double ms[kWindowCells];
  __shared__ double red[NW];
  const int R = qa.R;
  // (atom, axis) fastest: the widest Gaussians (smallest q, the most cells to
  // generate) are dispatched first and the cheap narrow ones fill the tail
  const int q = blockIdx.y;
  const int c = blockIdx.x;
  const int nu = c / 3, l = c - 3 * (c / 3);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (coef != nullptr && tid == 0 && l == 0) coef[nu * R + q] = Z[nu] * qa.w[q];
  const int L = (l == 0) ? L0 : (l == 1 ? L1 : L2);
  const int N = L * n;
  const int W = (2 * L - 1) * n;
  int p;
  double delta;
  node_offset(pos[c], b, h, n, &p, &delta);
  const double tau = qa.tau[q];
  const int jlo = -p - (L - 1) * n;
  // cells whose offset exceeds the support half-width are exactly 0
  const double hw = support_halfwidth(tau);
  const int js = (int)fmax((double)jlo, floor(delta - hw) - 1.0);
  const int je = (int)fmin((double)(jlo + W), ceil(delta + hw) + 2.0);
#pragma unroll 1
  for (int i = tid; i < W; i += BS) {
    const int j = jlo + i;
    if (j < js || j >= je) ms[i] = 0.0;
  }
  // the support: 63 cells per wave and step, lane i's left edge shared with
  // lane i - 1 as its right edge
#pragma unroll 1
  for (int base = js + wave * kMasterCellsPerWave; base < je; base += NW * kMasterCellsPerWave) {
    const int j = base + lane;
    // tau and delta re-enter each iteration as opaque register values, so the
    // compiler cannot hoist the cell integral's tau-dependent constants out of
    // the loop (that kept them all live and doubled the registers per lane)
    double tq = tau, dq = delta;
    asm volatile("" : "+v"(tq), "+v"(dq));
    const double y0 = (double)j - dq;
    double v;
    if (deriv) {
      v = cell_derivative(tq, y0);
    } else {
      const double e = edge_needed(tq, j, dq) ? edge_value(tq, y0) : 0.0;
      const double eR = __shfl_down(e, 1, 64);
      v = h * cell_from_edges(tq, y0, e, eR);
    }
    if (lane < kMasterCellsPerWave && j < je) ms[j - jlo] = v;
  }
  __syncthreads();
  double* out = ((l == 0) ? f0 : (l == 1 ? f1 : f2)) + ((size_t)nu * R + q) * (size_t)N;
  // lanes per residue: `parts` runs of at most RUN outputs (RUN a compile-time
  // bound, so a run's suffix sums stay in RUN registers)
  int parts = 1;
  while ((L + parts - 1) / parts > RUN) parts *= 2;
  while (parts * 2 * n <= BS && parts * 2 <= L) parts *= 2;
  const int run = (L + parts - 1) / parts;
  double vmax = 0.0;
  for (int t0 = 0; t0 < n * parts; t0 += BS) {
    const int t = t0 + tid;
    if (t < n * parts) {
      const int rho = t % n, part = t / n;
      const int m0 = part * run, m1 = min(L, m0 + run);
      const double* beta = ms + rho;  // beta(d) = beta[(d + L - 1) n]
      // suf(e) = sum_{i=e}^{L-2} beta(i - (L-1)), accumulated from i = L-2
      // downwards (the terms above this run first), so every suffix sum adds
      // the same terms in the same order as the stored-masters assembly
      double acc = 0.0;
      for (int e = L - 2; e >= m1; --e) acc += beta[e * n];
      double suf[RUN];
#pragma unroll
      for (int u = RUN - 1; u >= 0; --u) {
        const int e = m0 + u;
        if (e < m1 && e <= L - 2) acc += beta[e * n];
        suf[u] = acc;
      }
      // prefix over the outputs before this run, in order
      double pre = 0.0;
      for (int m = 0; m < m0; ++m) pre += beta[(m + L - 1) * n];
#pragma unroll
      for (int u = 0; u < RUN; ++u) {
        const int m = m0 + u;
        if (m < m1) {
          pre += beta[(m + L - 1) * n];
          const double s = (m <= L - 2) ? suf[u] : 0.0;
          const double v = s + pre;
          out[(size_t)m * n + rho] = v;
          vmax = fmax(vmax, fabs(v));
        }
      }
    }
  }
  if (rowmax != nullptr) {
    for (int o = 32; o > 0; o >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, o, 64));
    if (lane == 0) red[wave] = vmax;
    __syncthreads();
    if (tid == 0) {
      double mx = red[0];
      for (int w = 1; w < NW; ++w) mx = fmax(mx, red[w]);
      const size_t K = (size_t)(gridDim.x / 3) * R;
      rowmax[(size_t)l * K + nu * R + q] = mx;
    }
  }
}

// Box assembly from masters for any L: one lane per output, L reads.
__global__ __launch_bounds__(256) void k_assemble_box_direct(const double* __restrict__ masters,
                                                              const double* __restrict__ pos,
                                                              const double* __restrict__ Z,
                                                              QuadArg qa, int n, int L0, int L1,
                                                              int L2,
                                                              double b, double h, int X,
                                                              double* __restrict__ f0,
                                                              double* __restrict__ f1,
                                                              double* __restrict__ f2,
                                                              double* __restrict__ coef) {
  const int R = qa.R;
  const int q = blockIdx.y;
  const int c = blockIdx.z;
  const int nu = c / 3, l = c - 3 * (c / 3);
  const int L = (l == 0) ? L0 : (l == 1 ? L1 : L2);
  const int N = L * n;
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= N) return;
  if (coef != nullptr && g == 0 && l == 0) coef[nu * R + q] = Z[nu] * qa.w[q];
  int p;
  double delta;
  node_offset(pos[c], b, h, n, &p, &delta);
  const double* m = masters + ((size_t)c * R + q) * (size_t)(2 * X) + X;
  // ascending k: d = m_blk - k; sum in order of increasing k
  double acc = 0.0;
  for (int k = 0; k < L; ++k) acc += m[g - p - k * n];
  double* out = ((l == 0) ? f0 : (l == 1 ? f1 : f2)) + ((size_t)nu * R + q) * (size_t)N;
  out[g] = acc;
}

// Assembly with every cell integral generated in registers (periodic cell,
// or box without stored masters): one lane per output, one integral per image.
__global__ __launch_bounds__(256) void k_assemble_fused(const double* __restrict__ pos, QuadArg qa,
                                                         Lat lat, int deriv, double* __restrict__ f0,
                                                         double* __restrict__ f1,
                                                         double* __restrict__ f2,
                                                         const double* __restrict__ Z,
                                                         double* __restrict__ coef) {
  // q slowest: the widest Gaussians (the most images in reach) go first
  const int q = blockIdx.z;
  const int c = blockIdx.y;
  const int nu = c / 3, l = c - 3 * (c / 3);
  const int N = lat.N[l];
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (g >= N) return;
  if (coef != nullptr && g == 0 && l == 0) coef[nu * qa.R + q] = Z[nu] * qa.w[q];
  int p;
  double delta;
  node_offset(pos[c], lat.b, lat.h, lat.n, &p, &delta);
  const double tau = qa.tau[q];
  int k0 = lat.kmin[l], k1 = lat.kmin[l] + lat.L[l];
  // images whose cell lies beyond the Gaussian's support contribute exactly 0:
  // |g - p - k n - delta| <= hw  <=>  k in [(g - p - delta - hw)/n, (g - p - delta + hw)/n]
  const double hw = support_halfwidth(tau);
  const double base = (double)(g - p) - delta;
  k0 = (int)fmax((double)k0, floor((base - hw) / lat.n));
  k1 = (int)fmin((double)k1, ceil((base + hw) / lat.n) + 1.0);
  double acc = 0.0;
  for (int k = k0; k < k1; ++k) {
    const double y0 = (double)(g - p - k * lat.n) - delta;
    acc += deriv ? cell_derivative(tau, y0) : cell_integral(tau, y0);
  }
  double* out = ((l == 0) ? f0 : (l == 1 ? f1 : f2)) + ((size_t)nu * qa.R + q) * (size_t)N;
  out[g] = deriv ? acc : lat.h * acc;
}

// Non-equidistant tensor lattice (Sec. 3.1, remark after eq. EwaldTensorM0):
// the lattice coordinates of each axis are arbitrary (units of the cell), so
// every image has its own sub-cell offset and no master vector is shared;
// each cell integral is generated in registers, one lane per output cell.
// The coordinates of the axis pass through LDS 256 at a time, split into an
// integer part and a fraction, so the cell offset
//   y0 = (g - p - I_k) - (delta + phi_k)
// takes its lattice-size part as an exact integer (the rounding of y0 stays
// at the level of the charge's own sub-cell offset). Coordinates beyond
// +-1e9 cells are clamped there (exact zeros on any grid this library takes);
// a non-finite coordinate gives NaN outputs. Memory indices depend on g and
// k only.
struct TLat {
  int n;
  double b, h;
  int N[3];
  int L[3];
  const double* s[3];
};

__global__ __launch_bounds__(256) void k_assemble_tensor(const double* __restrict__ pos,
                                                          QuadArg qa, TLat tl, int deriv,
                                                          double* __restrict__ f0,
                                                          double* __restrict__ f1,
                                                          double* __restrict__ f2,
                                                          const double* __restrict__ Z,
                                                          double* __restrict__ coef) {
  __shared__ int sI[256];
  __shared__ double sF[256];
  // q slowest: the widest Gaussians (the most images in reach) go first
  const int q = blockIdx.z;
  const int c = blockIdx.y;
  const int nu = c / 3, l = c - 3 * (c / 3);
  const int N = tl.N[l];
  if ((int)blockIdx.x * 256 >= N) return;  // whole workgroup beyond this axis
  const int g = blockIdx.x * 256 + threadIdx.x;
  if (coef != nullptr && g == 0 && l == 0) coef[nu * qa.R + q] = Z[nu] * qa.w[q];
  int p;
  double delta;
  node_offset(pos[c], tl.b, tl.h, tl.n, &p, &delta);
  const double tau = qa.tau[q];
  const double hw = support_halfwidth(tau);
  const double* s = tl.s[l];
  const int L = tl.L[l];
  double acc = 0.0;
  for (int k0 = 0; k0 < L; k0 += 256) {
    __syncthreads();
    if (k0 + (int)threadIdx.x < L) {
      const double v = s[k0 + threadIdx.x];
      if (v == v && fabs(v) <= 1e300) {
        const double fl = floor(fmin(fmax(v, -1e9), 1e9));
        sI[threadIdx.x] = (int)fl;
        sF[threadIdx.x] = fmin(fmax(v, -1e9), 1e9) - fl;
      } else {
        sI[threadIdx.x] = 0;
        sF[threadIdx.x] = __builtin_nan("");
      }
    }
    __syncthreads();
    const int kn = min(256, L - k0);
    if (g < N) {
      for (int j = 0; j < kn; ++j) {
        const double y0 = (double)(g - p - sI[j]) - (delta + sF[j]);
        if (y0 > hw || y0 < -hw) continue;  // the whole cell beyond the support: exactly 0
        acc += deriv ? cell_derivative(tau, y0) : cell_integral(tau, y0);
      }
    }
  }
  if (g < N) {
    double* out = ((l == 0) ? f0 : (l == 1 ? f1 : f2)) + ((size_t)nu * qa.R + q) * (size_t)N;
    out[g] = deriv ? acc : tl.h * acc;
  }
}

}  // namespace ls

using namespace ls;

extern "C" ls_status ls_kernel_vectors(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                                       const double* pos_dev, int32_t X, int32_t derivative,
                                       double* masters_dev, hipStream_t stream) {
  clear_error();
  Lat L;
  ls_status st = check_lattice(lat, &L);
  if (st != LS_OK) return st;
  QuadArg qa;
  st = check_quad(quad, L.h, &qa);
  if (st != LS_OK) return st;
  LS_REQUIRE(M0 >= 1 && M0 <= 20000, "M0 must be in [1, 20000] (got %d)", M0);
  LS_REQUIRE(pos_dev != nullptr && masters_dev != nullptr, "null device pointer");
  LS_REQUIRE(X == master_halfwidth(L), "X = %d does not match the lattice (%d)", X,
             master_halfwidth(L));
  const int waves = (2 * X + kMasterCellsPerWave - 1) / kMasterCellsPerWave;
  dim3 grid((waves + 3) / 4, 3 * M0, qa.R);
  hipLaunchKernelGGL(k_masters, grid, dim3(256), 0, stream, pos_dev, qa, L.b, L.h, L.n, X,
                     derivative ? 1 : 0, masters_dev);
  return launch_status("ls_kernel_vectors");
}

extern "C" ls_status ls_assemble(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                                 const double* pos_dev, const double* Z_dev,
                                 const double* masters_dev, int32_t X, int32_t derivative,
                                 double* f0_dev, double* f1_dev, double* f2_dev, double* coef_dev,
                                 double* rowmax_dev, hipStream_t stream) {
  clear_error();
  Lat L;
  ls_status st = check_lattice(lat, &L);
  if (st != LS_OK) return st;
  QuadArg qa;
  st = check_quad(quad, L.h, &qa);
  if (st != LS_OK) return st;
  LS_REQUIRE(M0 >= 1 && M0 <= 20000, "M0 must be in [1, 20000] (got %d)", M0);
  LS_REQUIRE(pos_dev != nullptr && f0_dev != nullptr && f1_dev != nullptr && f2_dev != nullptr,
             "null device pointer");
  LS_REQUIRE(derivative || (Z_dev != nullptr && coef_dev != nullptr),
             "Z and coef are required for value vectors");
  LS_REQUIRE(!(L.periodic && masters_dev != nullptr),
             "the periodic cell generates its cell integrals in registers; pass masters = NULL");
  if (masters_dev != nullptr)
    LS_REQUIRE(X == master_halfwidth(L), "X = %d does not match the lattice (%d)", X,
               master_halfwidth(L));
  // the coefficients coef[nu R + q] = Z[nu] w[q] are written by the assembly
  // kernel itself (value vectors only)
  double* coef = derivative ? nullptr : coef_dev;
  const int Lmax = std::max(L.L[0], std::max(L.L[1], L.L[2]));
  bool rowmax_done = false;
  if (masters_dev == nullptr && !L.periodic && Lmax <= 64 &&
      (long long)(2 * Lmax - 1) * L.n <= kWindowCells) {
    // box: master window in LDS, kernel vectors and assembly in one launch
    dim3 grid(3 * M0, qa.R);
hipLaunchKernelGGL((k_assemble_box_lds<kAsmRun, kAsmThreads>), grid, dim3(kAsmThreads), 0, stream,
                       pos_dev, Z_dev, qa, L.n, L.L[0], L.L[1], L.L[2], L.b, L.h,
                       derivative ? 1 : 0, f0_dev, f1_dev, f2_dev, coef, rowmax_dev);
    rowmax_done = true;
  } else if (masters_dev == nullptr) {
    const int Nmax = L.N[0] > L.N[1] ? (L.N[0] > L.N[2] ? L.N[0] : L.N[2])
                                     : (L.N[1] > L.N[2] ? L.N[1] : L.N[2]);
    dim3 grid((Nmax + 255) / 256, 3 * M0, qa.R);
    hipLaunchKernelGGL(k_assemble_fused, grid, dim3(256), 0, stream, pos_dev, qa, L,
                       derivative ? 1 : 0, f0_dev, f1_dev, f2_dev, Z_dev, coef);
  } else {
    dim3 grid((L.n + 63) / 64, (qa.R + 3) / 4, 3 * M0);
#define LS_ASM(LM)                                                                            \
  hipLaunchKernelGGL(k_assemble_box<LM>, grid, dim3(256), 0, stream, masters_dev, pos_dev,    \
                     Z_dev, qa, L.n, L.L[0], L.L[1], L.L[2], L.b, L.h, X, f0_dev, f1_dev, f2_dev,  \
                     coef)
    if (Lmax <= 8)
      LS_ASM(8);
    else if (Lmax <= 16)
      LS_ASM(16);
    else if (Lmax <= 32)
      LS_ASM(32);
    else if (Lmax <= 64)
      LS_ASM(64);
    else {
      const int Nmax = Lmax * L.n;
      dim3 g2((Nmax + 255) / 256, qa.R, 3 * M0);
      hipLaunchKernelGGL(k_assemble_box_direct, g2, dim3(256), 0, stream, masters_dev, pos_dev,
                         Z_dev, qa, L.n, L.L[0], L.L[1], L.L[2], L.b, L.h, X, f0_dev, f1_dev,
                         f2_dev, coef);
    }
#undef LS_ASM
  }
  st = launch_status("ls_assemble");
  if (st != LS_OK || rowmax_dev == nullptr || rowmax_done) return st;
  return launch_rank_max(f0_dev, f1_dev, f2_dev, M0 * qa.R, L.N[0], L.N[1], L.N[2], rowmax_dev,
                         stream);
}

extern "C" ls_status ls_assemble_tensor(const ls_tensor_lattice* tlat, const ls_quad* quad,
                                        int32_t M0, const double* pos_dev, const double* Z_dev,
                                        int32_t derivative, double* f0_dev, double* f1_dev,
                                        double* f2_dev, double* coef_dev, hipStream_t stream) {
  clear_error();
  LS_REQUIRE(tlat != nullptr, "tensor lattice descriptor is null");
  LS_REQUIRE(tlat->n >= 1, "n must be >= 1 (got %d)", tlat->n);
  LS_REQUIRE(std::isfinite(tlat->b) && tlat->b > 0.0, "b must be finite and > 0");
  TLat tl;
  tl.n = tlat->n;
  tl.b = tlat->b;
  tl.h = tlat->b / tlat->n;
  int Nmax = 0;
  for (int l = 0; l < 3; ++l) {
    LS_REQUIRE(tlat->N[l] >= 1 && tlat->N[l] <= (1 << 26), "N[%d] must be in [1, 2^26] (got %d)",
               l, tlat->N[l]);
    LS_REQUIRE(tlat->L[l] >= 1 && tlat->L[l] <= (1 << 24), "L[%d] must be in [1, 2^24] (got %d)",
               l, tlat->L[l]);
    LS_REQUIRE(tlat->s[l] != nullptr, "lattice coordinates of axis %d are null", l);
    tl.N[l] = tlat->N[l];
    tl.L[l] = tlat->L[l];
    tl.s[l] = tlat->s[l];
    Nmax = std::max(Nmax, tl.N[l]);
  }
  QuadArg qa;
  ls_status st = check_quad(quad, tl.h, &qa);
  if (st != LS_OK) return st;
  LS_REQUIRE(M0 >= 1 && M0 <= 20000, "M0 must be in [1, 20000] (got %d)", M0);
  LS_REQUIRE(pos_dev != nullptr && f0_dev != nullptr && f1_dev != nullptr && f2_dev != nullptr,
             "null device pointer");
  LS_REQUIRE(derivative || (Z_dev != nullptr && coef_dev != nullptr),
             "Z and coef are required for value vectors");
  dim3 grid((Nmax + 255) / 256, 3 * M0, qa.R);
  hipLaunchKernelGGL(k_assemble_tensor, grid, dim3(256), 0, stream, pos_dev, qa, tl,
                     derivative ? 1 : 0, f0_dev, f1_dev, f2_dev, Z_dev,
                     derivative ? nullptr : coef_dev);
  return launch_status("ls_assemble_tensor");
}
