// Operations on assembled canonical tensors beyond the potential itself.
//
// ls_canon_combine: alpha A + beta B by concatenating factor matrices
// (Appendix, eq. conc), e.g. the Richardson-regularised periodic sum
// 2 P_L - P_2L or (4 P_L - P_2L)/3 (Sec. 3.2).
//
// ls_nuclear_matrix: the nuclear-potential operator matrix of Example 2.1
// (eq. nuc_pot) in a separable basis, v_km = <G_k (.) G_m, P>. With rank-one
// G_k = g_k^(0) (x) g_k^(1) (x) g_k^(2) (cell-midpoint samples) the Hadamard and
// scalar products (eqs. had, scal) reduce to
//   T_l[(k,m)][r] = sum_i g_k^(l)(i) g_m^(l)(i) f_l[r][i],
//   v_km = sum_r coef[r] T_0[(k,m)][r] T_1[(k,m)][r] T_2[(k,m)][r].
// T_l is a GEMM (rows: basis pairs, columns: ranks, reduction: grid cells)
// whose left operand is the row-wise (face-splitting) product of the basis
// samples, formed while staging into LDS; it runs on the FP64 MFMA
// (v_mfma_f64_16x16x4f64, D rows l/16 + 4v). The final contraction over the
// rank is one wave per pair with a fixed shuffle tree.
#include "ls_common.hpp"

namespace ls {

typedef double d4x_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ src, int rows, int len,
                                                 double* __restrict__ dst) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < (size_t)rows * len) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_combine_coef(const double* __restrict__ ca, int Ka,
                                                      double alpha, const double* __restrict__ cb,
                                                      int Kb, double beta,
                                                      double* __restrict__ out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < Ka) out[i] = alpha * ca[i];
  else if (i < Ka + Kb) out[i] = beta * cb[i - Ka];
}

// coef[0..K) *= alpha, coef[K..2K) *= beta (the two lattices of a Richardson sum)
__global__ __launch_bounds__(256) void k_scale_coef(double* __restrict__ coef, int K, double alpha,
                                                    double beta) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < K) coef[i] *= alpha;
  else if (i < 2 * K) coef[i] *= beta;
}

// T[p][r] for pairs p = k*Nb + m, ranks r: 64 x 64 tiles, rank chunk of 16 cells.
constexpr int NM_BM = 64, NM_BN = 64, NM_BK = 16;

__global__ __launch_bounds__(256) void k_face_gemm(const double* __restrict__ g, int Nb,
                                                   const double* __restrict__ A, int K, int len,
                                                   double* __restrict__ T) {
  __shared__ double Hs[NM_BK][NM_BM + 2];
  __shared__ double Ys[NM_BK][NM_BN + 2];
  const int P = Nb * Nb;
  const int row0 = blockIdx.x * NM_BM;  // pairs
  const int col0 = blockIdx.y * NM_BN;  // ranks
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;
  d4x_t acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4x_t{0, 0, 0, 0};
  // staging map: lane kk = tid % 16 walks the reduction, rows tid/16 + 16e
  const int kk = tid & 15, rb = tid >> 4;
  for (int i0 = 0; i0 < len; i0 += NM_BK) {
    const int i = i0 + kk;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int pr = row0 + rb + 16 * e;
      double h = 0.0;
      if (pr < P && i < len) {
        const int k = pr / Nb, m = pr - k * Nb;
        h = g[(size_t)k * len + i] * g[(size_t)m * len + i];
      }
      Hs[kk][rb + 16 * e] = h;
      const int rr = col0 + rb + 16 * e;
      Ys[kk][rb + 16 * e] = (rr < K && i < len) ? A[(size_t)rr * len + i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < NM_BK; ks += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Hs[ks + lk][wr + a * 16 + lr];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Ys[ks + lk][wc + b * 16 + lr];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int pr = row0 + wr + a * 16 + lk + 4 * v;
        const int rr = col0 + wc + b * 16 + lr;
        if (pr < P && rr < K) T[(size_t)pr * K + rr] = acc[a][b][v];
      }
}

__global__ __launch_bounds__(256) void k_face_reduce(const double* __restrict__ T, int P, int K,
                                                     const double* __restrict__ coef,
                                                     double* __restrict__ V) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= P) return;
  const size_t st = (size_t)P * K;
  const double* t0 = T + (size_t)p * K;
  double acc = 0.0;
  for (int r = lane; r < K; r += 64) acc += coef[r] * t0[r] * t0[st + r] * t0[2 * st + r];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) V[p] = acc;
}

}  // namespace ls

using namespace ls;

extern "C" ls_status ls_canon_combine(const ls_canon* A, double alpha, const ls_canon* B,
                                      double beta, double* f0_dev, double* f1_dev, double* f2_dev,
                                      double* coef_dev, hipStream_t stream) {
  clear_error();
  LS_REQUIRE(A != nullptr && B != nullptr, "null canonical tensor");
  LS_REQUIRE(A->K >= 1 && B->K >= 1, "ranks must be >= 1");
  LS_REQUIRE(std::isfinite(alpha) && std::isfinite(beta), "weights must be finite");
  LS_REQUIRE(f0_dev && f1_dev && f2_dev && coef_dev, "null output pointer");
  LS_REQUIRE(A->coef && B->coef, "null coefficient pointer");
  double* out[3] = {f0_dev, f1_dev, f2_dev};
  for (int l = 0; l < 3; ++l) {
    LS_REQUIRE(A->f[l] && B->f[l], "null factor pointer");
    LS_REQUIRE(A->len[l] == B->len[l] && A->len[l] >= 1, "length mismatch on axis %d", l);
    const size_t na = (size_t)A->K * A->len[l], nb = (size_t)B->K * B->len[l];
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, stream,
                       A->f[l], A->K, A->len[l], out[l]);
    hipLaunchKernelGGL(k_combine, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, stream,
                       B->f[l], B->K, B->len[l], out[l] + na);
  }
  const int Kt = A->K + B->K;
  hipLaunchKernelGGL(k_combine_coef, dim3((Kt + 255) / 256), dim3(256), 0, stream, A->coef, A->K,
                     alpha, B->coef, B->K, beta, coef_dev);
  return launch_status("ls_canon_combine");
}

extern "C" size_t ls_nuclear_workspace(int32_t K, int32_t Nb) {
  if (K < 1 || Nb < 1) return 0;
  return (3 * (size_t)Nb * Nb * K * sizeof(double) + 255) & ~(size_t)255;
}

extern "C" ls_status ls_nuclear_matrix(const ls_canon* P, int32_t Nb, const double* g0_dev,
                                       const double* g1_dev, const double* g2_dev, double* V_dev,
                                       void* ws_dev, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  LS_REQUIRE(P != nullptr && P->K >= 1 && P->coef, "canonical tensor is null or empty");
  LS_REQUIRE(P->f[0] && P->f[1] && P->f[2], "null factor pointer");
  LS_REQUIRE(Nb >= 1 && Nb <= 4096, "Nb must be in [1, 4096]");
  LS_REQUIRE(g0_dev && g1_dev && g2_dev && V_dev, "null device pointer");
  for (int l = 0; l < 3; ++l) LS_REQUIRE(P->len[l] >= 1, "len[%d] must be >= 1", l);
  LS_REQUIRE((long long)Nb * Nb * P->K < (1LL << 40), "problem too large");
  const size_t need = ls_nuclear_workspace(P->K, Nb);
  if (ws_dev == nullptr || ws_bytes < need) {
    set_error("workspace of %zu bytes required", need);
    return LS_EWORKSPACE;
  }
  LS_REQUIRE(ws_aligned(ws_dev), "the workspace must be 256-byte aligned");
  double* T = (double*)ws_dev;
  const int Pn = Nb * Nb;
  const double* g[3] = {g0_dev, g1_dev, g2_dev};
  dim3 grid((Pn + NM_BM - 1) / NM_BM, (P->K + NM_BN - 1) / NM_BN);
  for (int l = 0; l < 3; ++l) {
    hipLaunchKernelGGL(k_face_gemm, grid, dim3(256), 0, stream, g[l], Nb, P->f[l], P->K, P->len[l],
                       T + (size_t)l * Pn * P->K);
  }
  ls_status st = launch_status("ls_nuclear_matrix (gemm)");
  if (st != LS_OK) return st;
  hipLaunchKernelGGL(k_face_reduce, dim3((Pn + 3) / 4), dim3(256), 0, stream, T, Pn, P->K, P->coef,
                     V_dev);
  return launch_status("ls_nuclear_matrix (reduce)");
}

extern "C" ls_status ls_richardson(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                                   const double* pos_dev, const double* Z_dev, int32_t order,
                                   double* f0_dev, double* f1_dev, double* f2_dev,
                                   double* coef_dev, hipStream_t stream) {
  clear_error();
  LS_REQUIRE(lat != nullptr && quad != nullptr, "null lattice or quadrature");
  LS_REQUIRE(lat->periodic != 0, "Richardson extrapolation applies to the periodic cell");
  LS_REQUIRE(order == 1 || order == 2, "order must be 1 (linear) or 2 (quadratic), got %d", order);
  LS_REQUIRE(f0_dev && f1_dev && f2_dev && coef_dev, "null output pointer");
  LS_REQUIRE(M0 >= 1 && quad->R >= 1, "M0 and R must be >= 1");
  for (int l = 0; l < 3; ++l)
    LS_REQUIRE(lat->L[l] >= 1 && lat->L[l] <= (1 << 29), "L[%d] out of range", l);
  // Sec. 3.2: with p_L = p + c L^m (m = 1: sums that grow linearly in L,
  // m = 2: quadratically), p = (2^m p_L - p_2L) / (2^m - 1)
  const double alpha = order == 1 ? 2.0 : 4.0 / 3.0;
  const double beta = order == 1 ? -1.0 : -1.0 / 3.0;
  ls_lattice lat2 = *lat;
  for (int l = 0; l < 3; ++l) lat2.L[l] = 2 * lat->L[l];
  const size_t K = (size_t)M0 * quad->R;
  const size_t n = (size_t)lat->n;
  // rows [0, K): the lattice L; rows [K, 2K): the lattice 2L (eq. conc)
  ls_status st = ls_assemble(lat, quad, M0, pos_dev, Z_dev, nullptr, 0, 0, f0_dev, f1_dev, f2_dev,
                             coef_dev, nullptr, stream);
  if (st != LS_OK) return st;
  st = ls_assemble(&lat2, quad, M0, pos_dev, Z_dev, nullptr, 0, 0, f0_dev + K * n,
                   f1_dev + K * n, f2_dev + K * n, coef_dev + K, nullptr, stream);
  if (st != LS_OK) return st;
  hipLaunchKernelGGL(k_scale_coef, dim3((unsigned)((2 * K + 255) / 256)), dim3(256), 0, stream,
                     coef_dev, (int)K, alpha, beta);
  return launch_status("ls_richardson");
}
