// Energy as a canonical scalar product (Appendix, eq. scal) and forces on the
// unit-cell atoms by the adjoint of the assembled vectors.
//
// Energy from factors (HBM-bound): G_l[r][s] = <f_l[r], rho_l[s]> streams each
// factor row once through the matrix cores (density rows from L2), then
// E = sum_r coef[r] sum_s d[s] prod_l G_l[r][s] in one workgroup.
//
// Forces without factors: with Phi_l[s][i] = sum_k rho_l[s][i + k n] (the
// density folded back over the lattice shifts, the transpose of the shift
// sum), each Gram entry of an atom's assembled vector is a master-length dot
// product <m_q, Phi_l[s](. + p)>, for the value masters and for their position
// derivatives alike. One workgroup per (atom, axis, q) generates both master
// vectors in registers and contracts them with Phi, so neither masters nor
// factors touch HBM.
//
// All cross-lane reductions are fixed-order trees (bitwise reproducible).
#include <mutex>

#include "ls_common.hpp"

namespace ls {

template <typename T>
__device__ __forceinline__ double block_sum256(T v, double* sh) {
  // deterministic: lanes write, tree in LDS
  const int tid = threadIdx.x;
  sh[tid] = (double)v;
  __syncthreads();
#pragma unroll
  for (int s = 128; s > 0; s >>= 1) {
    if (tid < s) sh[tid] += sh[tid + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Grams G_l = f_l rho_l^T on MFMA, read as G_l^T (Krho x K) = rho_l (Krho x N)
// times f_l^T (N x K): one wave per 16 factor rows and cell chunk, density
// rows as the A operand (rows s, zero beyond Krho), factor rows as B (columns
// r). Lane l loads four consecutive cells c0 + 4(l/16) + j of its row r0 + l%16
// and of density row l%16, one 32-byte run per row, and issues one MFMA per j
// (its k index l/16 then stands for cell c0 + 4(l/16) + j): each factor row is
// read once from HBM in whole 128-byte lines (two 16-byte loads per lane when
// the rows are 16-byte aligned). The cells are split into kGramChunks chunks;
// the partial Grams are summed in a fixed order.
constexpr int kGramChunks = 64;
typedef double gram_d4_t __attribute__((ext_vector_type(4)));
typedef float gram_f4_t __attribute__((ext_vector_type(4)));

template <typename T>
struct GramMma;
template <>
struct GramMma<double> {
  typedef gram_d4_t acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return (lane >> 4) + 4 * v; }
};
template <>
struct GramMma<float> {
  typedef gram_f4_t acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int drow(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <typename T>
__global__ __launch_bounds__(256) void k_gram_mfma(const double* __restrict__ f0,
                                                    const double* __restrict__ f1,
                                                    const double* __restrict__ f2,
                                                    const double* __restrict__ D0,
                                                    const double* __restrict__ D1,
                                                    const double* __restrict__ D2, int K, int Krho,
                                                    int N0, int N1, int N2, int chunk,
                                                    double* __restrict__ part) {
  typedef GramMma<T> G;
  const int lane = threadIdx.x & 63;
  const int r0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  const int q = blockIdx.y;
  const int l = blockIdx.z;
  if (r0 >= K) return;
  const double* f = (l == 0 ? f0 : (l == 1 ? f1 : f2));
  const double* D = (l == 0 ? D0 : (l == 1 ? D1 : D2));
  const int N = (l == 0 ? N0 : (l == 1 ? N1 : N2));
  const int c_beg = q * chunk;
  const int c_end = min(N, c_beg + chunk);
  const int row = lane & 15, kq = lane >> 4;
  const bool rok = r0 + row < K, sok = row < Krho;
  const double* fr = f + (size_t)(rok ? r0 + row : 0) * N;
  const double* dr = D + (size_t)(sok ? row : 0) * N;
  const double fs = rok ? 1.0 : 0.0, ds = sok ? 1.0 : 0.0;
  typename G::acc_t acc = {0, 0, 0, 0};
  int c0 = c_beg;
  // whole 16-cell steps with 16-byte loads when the rows start 16-byte
  // aligned (N even; c is a multiple of 4), then the rest with masked loads,
  // in the same order of cells
  if ((N & 1) == 0) {
    // four steps at a time: all sixteen loads issued before the MFMAs
    for (; c0 + 64 <= c_end; c0 += 64) {
      double2 fa[4][2], da[4][2];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int c = c0 + 16 * u + 4 * kq;
        fa[u][0] = *reinterpret_cast<const double2*>(fr + c);
        fa[u][1] = *reinterpret_cast<const double2*>(fr + c + 2);
        da[u][0] = *reinterpret_cast<const double2*>(dr + c);
        da[u][1] = *reinterpret_cast<const double2*>(dr + c + 2);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double fv[4] = {fa[u][0].x * fs, fa[u][0].y * fs, fa[u][1].x * fs, fa[u][1].y * fs};
        const double dv[4] = {da[u][0].x * ds, da[u][0].y * ds, da[u][1].x * ds, da[u][1].y * ds};
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = G::mma((T)dv[j], (T)fv[j], acc);
      }
    }
    for (; c0 + 16 <= c_end; c0 += 16) {
      const int c = c0 + 4 * kq;
      const double2 f01 = *reinterpret_cast<const double2*>(fr + c);
      const double2 f23 = *reinterpret_cast<const double2*>(fr + c + 2);
      const double2 d01 = *reinterpret_cast<const double2*>(dr + c);
      const double2 d23 = *reinterpret_cast<const double2*>(dr + c + 2);
      const double fv[4] = {f01.x * fs, f01.y * fs, f23.x * fs, f23.y * fs};
      const double dv[4] = {d01.x * ds, d01.y * ds, d23.x * ds, d23.y * ds};
#pragma unroll
      for (int j = 0; j < 4; ++j) acc = G::mma((T)dv[j], (T)fv[j], acc);
    }
  }
  for (; c0 < c_end; c0 += 16) {
    const int c = c0 + 4 * kq;
    double fv[4], dv[4];
    // loads at clamped cells (always in range), masked after
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cc = min(c + j, c_end - 1);
      const double m = (c + j < c_end) ? 1.0 : 0.0;
      fv[j] = fr[cc] * (fs * m);
      dv[j] = dr[cc] * (ds * m);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) acc = G::mma((T)dv[j], (T)fv[j], acc);
  }
  // acc[v] = G_l^T[s][r] with s = drow(lane, v), r = r0 + lane % 16
  double* out = part + ((size_t)q * 3 + l) * (size_t)K * Krho;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int s = G::drow(lane, v);
    if (s < Krho && rok) out[(size_t)(r0 + row) * Krho + s] = (double)acc[v];
  }
}

// Workgroup b takes the pairs i = 64 b + t (t < 64) of the n = K * Krho pairs
// (r, s): wave l sums the kGramChunks partials of G_l[i] in chunk order and
// stores G; wave 0 then adds the 64 terms coef[r] d[s] G0 G1 G2 (a fixed
// shuffle tree) into bsum[b].
__global__ __launch_bounds__(192) void k_energy_terms(const double* __restrict__ part, int n,
                                                      int Krho, const double* __restrict__ coef,
                                                      const double* __restrict__ d,
                                                      double* __restrict__ G,
                                                      double* __restrict__ bsum) {
  __shared__ double g[3][64];
  const int t = threadIdx.x & 63, l = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + t;
  double acc = 0.0;
  if (i < n) {
    // all partial loads in flight at once, then added in chunk order
    double v[kGramChunks];
#pragma unroll
    for (int q = 0; q < kGramChunks; ++q) v[q] = part[((size_t)q * 3 + l) * n + i];
#pragma unroll
    for (int q = 0; q < kGramChunks; ++q) acc += v[q];
    G[(size_t)l * n + i] = acc;
  }
  g[l][t] = acc;
  __syncthreads();
  if (l == 0) {
    double v = 0.0;
    if (i < n) {
      const int r = i / Krho, s = i - r * Krho;
      v = coef[r] * d[s] * g[0][t] * g[1][t] * g[2][t];
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (t == 0) bsum[blockIdx.x] = v;
  }
}

// one wave: E = the workgroup sums of k_energy_terms added in workgroup order
__global__ __launch_bounds__(64) void k_energy_sum(const double* __restrict__ bsum, int nb,
                                                   double* __restrict__ E) {
  if (threadIdx.x != 0) return;
  double e = 0.0;
  for (int b = 0; b < nb; ++b) e += bsum[b];
  *E = e;
}

// Phi[((l*W + i + X) * KP + s] = sum_{k in images} D_l[s][i + k n],  i in [-X, X + n - 1),
// cell-major with KP >= Krho values per cell (zero for s >= Krho), so the
// force Grams read one cell's densities as contiguous 16-byte loads
__global__ __launch_bounds__(256) void k_fold_density(const double* __restrict__ D0,
                                                       const double* __restrict__ D1,
                                                       const double* __restrict__ D2, Lat lat,
                                                       int Krho, int KP, int X, int W,
                                                       double* __restrict__ Phi) {
  const int ii = blockIdx.x * 256 + threadIdx.x;
  const int s = blockIdx.y;
  const int l = blockIdx.z;
  if (ii >= W) return;
  double acc = 0.0;
  if (s < Krho) {
    const double* D = (l == 0 ? D0 : (l == 1 ? D1 : D2)) + (size_t)s * lat.N[l];
    const int i = ii - X;
    for (int k = lat.kmin[l]; k < lat.kmin[l] + lat.L[l]; ++k) {
      const long long g = (long long)i + (long long)k * lat.n;
      if (g >= 0 && g < lat.N[l]) acc += D[g];
    }
  }
  Phi[((size_t)l * W + ii) * KP + s] = acc;
}

// Value and derivative Grams of one (atom, axis, q) against the folded density:
//   Gv[s] = sum_j h*B(j) Phi[s][j + p],  Gd[s] = sum_j dB(j) Phi[s][j + p]
// RHO: the density ranks the per-lane accumulators hold (8 or kMaxRho), also
// the folded density's values per cell (cell-major; 0.30 against 0.41 ms per
// FP64 forces call with the rank-major layout's eight strided loads per cell).
// Three waves per SIMD (0.30 / 0.29 ms per FP64 / FP32 forces call; four
// spill their 128 registers: 0.30 / 0.31 ms).
template <typename T, int RHO>
__global__ __launch_bounds__(256, 3) void k_force_grams(const double* __restrict__ pos, QuadArg qa,
                                                      Lat lat, const double* __restrict__ Phi,
                                                      int Krho, int X, int W, int K,
                                                      double* __restrict__ Gv,
                                                      double* __restrict__ Gd) {
  __shared__ double sh[256];
  __shared__ double eb[256];  // edge values erfc(tau |y|)
  __shared__ double gb[256];  // edge Gaussians exp(-tau^2 y^2)
  // (atom, axis) fastest: the widest Gaussians (smallest q, the most cells)
  // are dispatched first and the cheap narrow ones fill the tail
  const int q = blockIdx.y;
  const int c = blockIdx.x;  // nu*3 + l
  const int nu = c / 3, l = c - 3 * (c / 3);
  int p;
  double delta;
  node_offset(pos[c], lat.b, lat.h, lat.n, &p, &delta);
  const double tau = qa.tau[q];
  // ph[j * RHO + s] = Phi_l[s][j + p]
  const double* ph = Phi + ((size_t)l * W + p + X) * RHO;
  T av[RHO], ad[RHO];
#pragma unroll
  for (int s = 0; s < RHO; ++s) {
    av[s] = 0;
    ad[s] = 0;
  }
  // cells beyond the Gaussian's support contribute exactly 0
  const double hw = support_halfwidth(tau);
  const int jbeg = (int)fmax((double)-X, floor(delta - hw));
  const int jend = (int)fmin((double)X, ceil(delta + hw) + 1.0);
  // the node's constants of cell_value_deriv, once per workgroup
  const double knorm = cell_half_norm(tau), ec = exp(-0.25 * tau * tau);
  // chunks of 255 cells: thread t evaluates edge j0 + t once (shared edges):
  // its erfc value and its Gaussian, from which the cell values and
  // derivatives on both sides of it are formed
#pragma unroll 1
  for (int j0 = jbeg; j0 < jend; j0 += 255) {
    const int j = j0 + (int)threadIdx.x;
    // tau, delta and the node's constants opaque per chunk: the cell
    // integral's tau-dependent constants are recomputed instead of held live
    // across the loop
    double tq = tau, dq = delta, kq = knorm, eq = ec;
    asm volatile("" : "+v"(tq), "+v"(dq), "+v"(kq), "+v"(eq));
    // the cell's RHO densities (zero past Krho), 16 bytes per load; with FP32
    // Grams of 8 densities requested before the edge is evaluated, so that the
    // evaluation covers their latency (cells past the support read the last
    // one's and are not used); otherwise that would exceed the register budget
    // of three waves per SIMD (spills), so they are requested where used
    constexpr bool kEarly = sizeof(T) == 4 && RHO == 8;
    double fv[RHO];
    auto load_rho = [&](int jc) {
      const double2* c2 = reinterpret_cast<const double2*>(ph + (ptrdiff_t)jc * RHO);
#pragma unroll
      for (int q2 = 0; q2 < RHO / 2; ++q2) {
        const double2 v = c2[q2];
        fv[2 * q2] = v.x;
        fv[2 * q2 + 1] = v.y;
      }
    };
    if constexpr (kEarly) load_rho(min(j, jend - 1));
    double ev = 0.0, gv = 0.0;
    if (edge_needed(tq, j, dq)) ev = edge_value(tq, (double)j - dq, &gv);
    eb[threadIdx.x] = ev;
    gb[threadIdx.x] = gv;
    __syncthreads();
    if (threadIdx.x < 255 && j < jend) {
      const double y0 = (double)j - dq;
      double bd;
      const double bv = lat.h * cell_value_deriv(tq, y0, eb[threadIdx.x], eb[threadIdx.x + 1],
                                                 gb[threadIdx.x], gb[threadIdx.x + 1], kq, eq, &bd);
      if (bv != 0.0 || bd != 0.0) {
        if constexpr (!kEarly) load_rho(j);
#pragma unroll
        for (int s = 0; s < RHO; ++s) {
          av[s] += (T)bv * (T)fv[s];
          ad[s] += (T)bd * (T)fv[s];
        }
      }
    }
    __syncthreads();
  }
  // fixed-order reduction: shuffle tree per wave, then the four waves in order
  const int r = nu * qa.R + q;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < RHO; ++s) {
    if (s < Krho) {
      const double tv = wave_sum64((double)av[s]);
      const double td = wave_sum64((double)ad[s]);
      if (lane == 0) {
        sh[wv * 2 * kMaxRho + s] = tv;
        sh[wv * 2 * kMaxRho + kMaxRho + s] = td;
      }
    }
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i < 2 * kMaxRho && (i % kMaxRho) < Krho) {
    const double tot = ((sh[i] + sh[2 * kMaxRho + i]) + sh[4 * kMaxRho + i]) + sh[6 * kMaxRho + i];
    const int s = i % kMaxRho;
    double* dst = i < kMaxRho ? Gv : Gd;
    dst[((size_t)l * K + r) * Krho + s] = tot;
  }
}

// F[nu][l] = -Z_nu sum_q w_q sum_s d_s Gd_l[nu q][s] prod_{l' != l} Gv_l'[nu q][s]
// Eatom[nu] = Z_nu sum_q w_q sum_s d_s prod_l Gv_l[nu q][s]
__global__ __launch_bounds__(256) void k_force_combine(const double* __restrict__ Z, QuadArg qa,
                                                        int M0, int Krho,
                                                        const double* __restrict__ d,
                                                        const double* __restrict__ Gv,
                                                        const double* __restrict__ Gd,
                                                        double* __restrict__ F,
                                                        double* __restrict__ Eatom) {
  // one wave per (atom, l or 3 = energy); lanes over q, fixed-order shuffle sum
  const int lane = threadIdx.x & 63;
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);  // nu*4 + (l or 3)
  if (idx >= 4 * M0) return;
  const int nu = idx >> 2, l = idx & 3;
  const int K = M0 * qa.R;
  const size_t stride = (size_t)K * Krho;
  double acc = 0.0;
  for (int q = lane; q < qa.R; q += 64) {
    const size_t base = ((size_t)nu * qa.R + q) * Krho;
    double v = 0.0;
    for (int s = 0; s < Krho; ++s) {
      const double g0 = Gv[base + s], g1 = Gv[stride + base + s], g2 = Gv[2 * stride + base + s];
      double t;
      if (l == 0)
        t = Gd[base + s] * g1 * g2;
      else if (l == 1)
        t = g0 * Gd[stride + base + s] * g2;
      else if (l == 2)
        t = g0 * g1 * Gd[2 * stride + base + s];
      else
        t = g0 * g1 * g2;
      v += d[s] * t;
    }
    acc += qa.w[q] * v;
  }
  acc = wave_sum64(acc);
  if (lane == 0) {
    if (l < 3)
      F[nu * 3 + l] = -Z[nu] * acc;
    else
      Eatom[nu] = Z[nu] * acc;
  }
}

__global__ __launch_bounds__(256) void k_sum(const double* __restrict__ x, int n,
                                              double* __restrict__ out) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += x[i];
  const double tot = block_sum256(acc, sh);
  if (threadIdx.x == 0) *out = tot;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace ls

using namespace ls;

// workspace: G [3][K][Krho] | partial Grams [kGramChunks][3][K][Krho] |
// per-workgroup sums of k_energy_terms [ceil(K Krho / 64)]
static size_t energy_bsum_offset(int K, int Krho) {
  return align256((size_t)3 * K * Krho * sizeof(double)) +
         align256((size_t)kGramChunks * 3 * K * Krho * sizeof(double));
}
static int energy_blocks(int K, int Krho) { return (int)(((size_t)K * Krho + 63) / 64); }

extern "C" size_t ls_energy_workspace(int32_t K, int32_t Krho) {
  if (K < 1 || Krho < 1) return 0;
  return energy_bsum_offset(K, Krho) + align256((size_t)energy_blocks(K, Krho) * sizeof(double));
}

extern "C" ls_status ls_energy(const ls_canon* P, const ls_canon* rho, int32_t precision,
                               double* E_dev, void* ws_dev, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  LS_REQUIRE(P != nullptr && rho != nullptr && E_dev != nullptr, "null pointer");
  LS_REQUIRE(P->K >= 1 && rho->K >= 1, "ranks must be >= 1");
  LS_REQUIRE(P->f[0] && P->f[1] && P->f[2] && P->coef, "null factor pointer");
  LS_REQUIRE(rho->f[0] && rho->f[1] && rho->f[2] && rho->coef, "null density pointer");
  if (rho->K > kMaxRho) {
    set_error("density rank %d exceeds the supported %d", rho->K, kMaxRho);
    return LS_EUNSUPPORTED;
  }
  for (int l = 0; l < 3; ++l)
    LS_REQUIRE(P->len[l] == rho->len[l] && P->len[l] >= 1, "length mismatch on axis %d", l);
  if (precision != LS_F64 && precision != LS_F32) {
    set_error("energy supports LS_F64 and LS_F32 only");
    return LS_EUNSUPPORTED;
  }
  const size_t need = ls_energy_workspace(P->K, rho->K);
  if (ws_dev == nullptr || ws_bytes < need) {
    set_error("workspace of %zu bytes required", need);
    return LS_EWORKSPACE;
  }
  LS_REQUIRE(ws_aligned(ws_dev), "the workspace must be 256-byte aligned");
  double* G = (double*)ws_dev;
  double* part = (double*)((char*)ws_dev + align256((size_t)3 * P->K * rho->K * sizeof(double)));
  const size_t boff = energy_bsum_offset(P->K, rho->K);
  const int nblk = energy_blocks(P->K, rho->K);
  double* bsum = (double*)((char*)ws_dev + boff);
  const int Nmax = std::max(P->len[0], std::max(P->len[1], P->len[2]));
  const int chunk = ((Nmax + kGramChunks - 1) / kGramChunks + 15) / 16 * 16;
  // chunks past the end of a shorter axis still write their (zero) partials
  dim3 grid((P->K + 63) / 64, kGramChunks, 3);
  if (precision == LS_F64)
    hipLaunchKernelGGL(k_gram_mfma<double>, grid, dim3(256), 0, stream, P->f[0], P->f[1],
                       P->f[2], rho->f[0], rho->f[1], rho->f[2], P->K, rho->K, P->len[0],
                       P->len[1], P->len[2], chunk, part);
  else
    hipLaunchKernelGGL(k_gram_mfma<float>, grid, dim3(256), 0, stream, P->f[0], P->f[1],
                       P->f[2], rho->f[0], rho->f[1], rho->f[2], P->K, rho->K, P->len[0],
                       P->len[1], P->len[2], chunk, part);
  ls_status st = launch_status("ls_energy (gram)");
  if (st != LS_OK) return st;
  hipLaunchKernelGGL(k_energy_terms, dim3(nblk), dim3(192), 0, stream, part, P->K * rho->K, rho->K,
                     P->coef, rho->coef, G, bsum);
  st = launch_status("ls_energy (terms)");
  if (st != LS_OK) return st;
  hipLaunchKernelGGL(k_energy_sum, dim3(1), dim3(64), 0, stream, bsum, nblk, E_dev);
  return launch_status("ls_energy (sum)");
}

// densities per folded cell: the force Grams' accumulator count
static int fold_ranks(int Krho) { return Krho <= 8 ? 8 : kMaxRho; }

// workspace: Phi [3][W][fold_ranks] | Gv [3][K][Krho] | Gd [3][K][Krho] | Eatom [M0]
static void forces_layout(const Lat& L, int M0, int R, int Krho, size_t* off_gv, size_t* off_gd,
                          size_t* off_e, size_t* total, int* X, int* W) {
  *X = master_halfwidth(L);
  *W = 2 * (*X) + L.n;
  const size_t K = (size_t)M0 * R;
  size_t o = align256((size_t)3 * fold_ranks(Krho) * (*W) * sizeof(double));
  *off_gv = o;
  o += align256(3 * K * Krho * sizeof(double));
  *off_gd = o;
  o += align256(3 * K * Krho * sizeof(double));
  *off_e = o;
  o += align256((size_t)M0 * sizeof(double));
  *total = o;
}

extern "C" size_t ls_forces_workspace(const ls_lattice* lat, int32_t M0, int32_t R, int32_t Krho) {
  Lat L;
  if (check_lattice(lat, &L) != LS_OK || M0 < 1 || R < 1 || Krho < 1) return 0;
  size_t a, b, c, t;
  int X, W;
  forces_layout(L, M0, R, Krho, &a, &b, &c, &t, &X, &W);
  return t;
}

// The body of ls_forces and ls_forces_noalloc: `scratch_name` names the
// buffer in the error text when it is too small.
static ls_status forces_run(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                            const double* pos_dev, const double* Z_dev, const ls_canon* rho,
                            int32_t precision, double* F_dev, double* E_dev, void* ws_dev,
                            size_t ws_bytes, const char* scratch_name, hipStream_t stream) {
  Lat L;
  ls_status st = check_lattice(lat, &L);
  if (st != LS_OK) return st;
  QuadArg qa;
  st = check_quad(quad, L.h, &qa);
  if (st != LS_OK) return st;
  LS_REQUIRE(M0 >= 1 && M0 <= 20000, "M0 must be in [1, 20000] (got %d)", M0);
  LS_REQUIRE(pos_dev != nullptr && Z_dev != nullptr && F_dev != nullptr, "null device pointer");
  LS_REQUIRE(rho != nullptr && rho->K >= 1 && rho->f[0] && rho->f[1] && rho->f[2] && rho->coef,
             "density is null or empty");
  if (rho->K > kMaxRho) {
    set_error("density rank %d exceeds the supported %d", rho->K, kMaxRho);
    return LS_EUNSUPPORTED;
  }
  for (int l = 0; l < 3; ++l)
    LS_REQUIRE(rho->len[l] == L.N[l], "density length %d != grid %d on axis %d", rho->len[l],
               L.N[l], l);
  if (precision != LS_F64 && precision != LS_F32) {
    set_error("forces support LS_F64 and LS_F32 only");
    return LS_EUNSUPPORTED;
  }
  size_t off_gv, off_gd, off_e, total;
  int X, W;
  forces_layout(L, M0, qa.R, rho->K, &off_gv, &off_gd, &off_e, &total, &X, &W);
  if (ws_dev == nullptr || ws_bytes < total) {
    set_error("%s of %zu bytes required (%zu available)", scratch_name, total,
              ws_dev == nullptr ? (size_t)0 : ws_bytes);
    return LS_EWORKSPACE;
  }
  LS_REQUIRE(ws_aligned(ws_dev), "the %s must be 256-byte aligned", scratch_name);
  char* ws = (char*)ws_dev;
  double* Phi = (double*)ws;
  double* Gv = (double*)(ws + off_gv);
  double* Gd = (double*)(ws + off_gd);
  double* Eatom = (double*)(ws + off_e);
  const int K = M0 * qa.R;
  const int KP = fold_ranks(rho->K);
  hipLaunchKernelGGL(k_fold_density, dim3((W + 255) / 256, KP, 3), dim3(256), 0, stream,
                     rho->f[0], rho->f[1], rho->f[2], L, rho->K, KP, X, W, Phi);
  st = launch_status("ls_forces (fold)");
  if (st != LS_OK) return st;
  // accumulators for 8 density ranks where they suffice (fewer registers per
  // lane, more waves per SIMD for the cell integrals)
#define LS_FG(T, RH)                                                                           \
  hipLaunchKernelGGL((k_force_grams<T, RH>), dim3(3 * M0, qa.R), dim3(256), 0, stream, pos_dev, \
                     qa, L, Phi, rho->K, X, W, K, Gv, Gd)
  if (precision == LS_F64) {
    if (rho->K <= 8)
      LS_FG(double, 8);
    else
      LS_FG(double, kMaxRho);
  } else {
    if (rho->K <= 8)
      LS_FG(float, 8);
    else
      LS_FG(float, kMaxRho);
  }
#undef LS_FG
  st = launch_status("ls_forces (grams)");
  if (st != LS_OK) return st;
  hipLaunchKernelGGL(k_force_combine, dim3(M0), dim3(256), 0, stream, Z_dev, qa,
                     M0, rho->K, rho->coef, Gv, Gd, F_dev, Eatom);
  st = launch_status("ls_forces (combine)");
  if (st != LS_OK || E_dev == nullptr) return st;
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, stream, Eatom, M0, E_dev);
  return launch_status("ls_forces (energy)");
}

extern "C" ls_status ls_forces(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                               const double* pos_dev, const double* Z_dev, const ls_canon* rho,
                               int32_t precision, double* F_dev, double* E_dev, void* ws_dev,
                               size_t ws_bytes, hipStream_t stream) {
  clear_error();
  return forces_run(lat, quad, M0, pos_dev, Z_dev, rho, precision, F_dev, E_dev, ws_dev, ws_bytes,
                    "workspace", stream);
}

// ---------------------------------------------------------------------------
// ls_forces without a workspace argument: the folded density, the Grams and
// the per-atom energies go to a fixed device array of this library. Every
// kernel of the forces writes each scratch entry it later reads (nothing has
// to start at zero), so consecutive calls need no clearing.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[LS_FORCES_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The device address of `scratch` on the current device, resolved once per
// device (the host-side name of the array is not a device address).
static ls_status scratch_address(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    set_error("ls_forces_noalloc: no usable current device (%s)", hipGetErrorString(e));
    return LS_EHIP;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error("ls_forces_noalloc: scratch address on device %d: %s", dev, hipGetErrorString(e));
      return LS_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return LS_OK;
}

extern "C" ls_status ls_forces_noalloc(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                                       const double* pos_dev, const double* Z_dev,
                                       const ls_canon* rho, int32_t precision, double* F_dev,
                                       double* E_dev, hipStream_t stream) {
  clear_error();
  // the size check first, so that an oversized problem is refused on the
  // host before any device query
  if (lat != nullptr && quad != nullptr && rho != nullptr) {
    const size_t need = ls_forces_workspace(lat, M0, quad->R, rho->K);
    if (need > (size_t)LS_FORCES_NOALLOC_BYTES) {
      set_error("ls_forces_noalloc: the problem needs %zu bytes of scratch, above the fixed %zu "
                "(use ls_forces with a workspace)",
                need, (size_t)LS_FORCES_NOALLOC_BYTES);
      return LS_EWORKSPACE;
    }
  }
  void* ptr = nullptr;
  const ls_status st = scratch_address(&ptr);
  if (st != LS_OK) return st;
  return forces_run(lat, quad, M0, pos_dev, Z_dev, rho, precision, F_dev, E_dev, ptr,
                    (size_t)LS_FORCES_NOALLOC_BYTES, "fixed scratch", stream);
}
