// Quantics-TT (QTT) compression of assembled canonical vectors (Sec. 4,
// eq. EwaldTensorQTT; Appendix: the TT format eq. tt and binary folding).
//
// A vector of length N <= 2^d (zero-padded) is folded into a 2 x ... x 2
// tensor of order d, most significant binary digit first, and decomposed by
// the TT-SVD (Oseledets 2011): at step k the unfolding C (rows
// (alpha_{k-1}, j_k), m = 2 r_{k-1} of them, n = 2^(d-k) columns, row-major)
// is decomposed as C = U S V^T; the left singular vectors of the kept values
// form core k, and S V^T, which as a row-major array already is the next
// unfolding (rows (alpha_k, j_{k+1})), goes on. The rank r_k is the smallest
// r >= 1 whose discarded singular values have Euclidean norm
// <= eps ||x||_2 / sqrt(d - 1), so ||x - x_QTT||_2 <= eps ||x||_2.
//
// One workgroup per vector, the unfolding in LDS (m n <= 2^d doubles at every
// step). Two launches: the first allows ranks up to 8 (a small rotation
// array, four workgroups per CU), the second, with ranks up to 32, redoes
// only the vectors the first refused for their rank (the same rotations in
// the same order: the result of a vector does not depend on which launch
// made it). The SVD is a one-sided Jacobi (Hestenes) iteration on the rows of C:
// plane rotations of row pairs, in a round-robin order (m/2 disjoint pairs
// per round, one group of lanes per pair, dot products by a shuffle tree
// inside the group), until every pair is orthogonal to 1e-15 of its norms
// (rows of squared norm below 1e-300 count as zero).
// The rotated rows are then sigma_i v_i^T, so S V^T needs no product, and the
// rotations applied to the identity give U^T. Row norms give the singular
// values; a fixed order of rounds and reductions makes the result bitwise
// reproducible.
#include "ls_common.hpp"

namespace ls {

constexpr int kQttMaxDigits = 12;      // N <= 4096: the unfolding fits in LDS
constexpr int kQttMaxRank = 32;        // so unfoldings have at most 64 rows
constexpr int kQttFirstRank = 8;       // the first launch's rank limit
constexpr int kQttMaxSweeps = 40;

// status values per vector
constexpr int kQttOk = 1, kQttRankLimit = -1, kQttCapacity = -2, kQttNoConvergence = -3;

__device__ __forceinline__ double group_sum(double v, int G) {
  // xor tree inside aligned groups of G lanes (G a power of two <= 64)
  for (int o = G >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// round-robin position i of round t among m players (m even): player 0 fixed,
// the others rotating
__device__ __forceinline__ int rr_player(int i, int t, int m) {
  return i == 0 ? 0 : 1 + (i - 1 + t) % (m - 1);
}

// MAXRANK: the largest rank this launch keeps (a larger one gives
// kQttRankLimit); REDO: work only on the vectors whose status is
// kQttRankLimit (a later launch with a larger MAXRANK).
template <int MAXRANK, bool REDO>
__global__ __launch_bounds__(256) void k_qtt_compress(const double* __restrict__ X, int len,
                                                       long long ld, int d, double eps, int cap,
                                                       double* __restrict__ cores,
                                                       int* __restrict__ ranks,
                                                       int* __restrict__ status) {
  constexpr int MR = 2 * MAXRANK;  // rows of an unfolding at most
  __shared__ double C[1 << kQttMaxDigits];
  __shared__ double W[MR * MR];  // U^T; also staging for the next C
  __shared__ double sig[MR];
  __shared__ double tails[MR];
  __shared__ int perm[MR];
  __shared__ double red[4];
  __shared__ int flag;
  __shared__ int rk_sh;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int v = blockIdx.x;
  if (REDO && status[v] != kQttRankLimit) return;  // uniform per workgroup
  const double* x = X + (long long)v * ld;
  double* out = cores + (long long)v * cap;
  int* rv = ranks + (long long)v * (d + 1);
  const int N = 1 << d;

  // load (zero-padded) and ||x||^2 in a fixed order
  double acc = 0.0;
  for (int i = tid; i < N; i += 256) {
    const double val = i < len ? x[i] : 0.0;
    C[i] = val;
    acc += val * val;
  }
  acc = group_sum(acc, 64);
  if (lane == 0) red[wave] = acc;
  __syncthreads();
  const double nrm2 = ((red[0] + red[1]) + red[2]) + red[3];
  const double delta = eps * sqrt(nrm2) / sqrt((double)(d - 1));
  const double delta2 = delta * delta;
  if (tid == 0) rv[0] = 1;

  int r = 1;      // r_{k-1}
  int off = 0;    // core offset in the vector's slot
  int st = kQttOk;
  for (int k = 1; k <= d - 1 && st == kQttOk; ++k) {
    const int m = 2 * r;
    const int n = N >> k;
    // W = identity (m x m)
    for (int i = tid; i < m * m; i += 256) W[i] = (i / m == i % m) ? 1.0 : 0.0;
    __syncthreads();
    // lanes per row pair: a power of two <= 64, 256 / (m/2) at most
    int G = 64;
    while (G * (m / 2) > 256) G >>= 1;
    const int grp = tid / G, gl = tid % G;
    int sweep = 0;
    for (; sweep < kQttMaxSweeps; ++sweep) {
      if (tid == 0) flag = 0;
      __syncthreads();
      for (int t = 0; t < m - 1; ++t) {
        if (grp < m / 2) {
          int p = rr_player(grp, t, m), q = rr_player(m - 1 - grp, t, m);
          if (p > q) {
            const int s = p;
            p = q;
            q = s;
          }
          double a = 0.0, b = 0.0, g = 0.0;
          for (int j = gl; j < n; j += G) {
            const double cp = C[p * n + j], cq = C[q * n + j];
            a += cp * cp;
            b += cq * cq;
            g += cp * cq;
          }
          a = group_sum(a, G);
          b = group_sum(b, G);
          g = group_sum(g, G);
          // rows of squared norm <= 1e-300 are numerically zero and left
          // alone (their denormal products would never settle)
          const double zeta = (b - a) / (2.0 * g);
          const double tt =
              fabs(zeta) < 1e150 ? (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta))
                                 : 0.5 / zeta;
          if (a > 1e-300 && b > 1e-300 && fabs(g) > 1e-15 * sqrt(a) * sqrt(b) && tt != 0.0) {
            const double c = 1.0 / sqrt(1.0 + tt * tt);
            const double s = c * tt;
            for (int j = gl; j < n; j += G) {
              const double cp = C[p * n + j], cq = C[q * n + j];
              C[p * n + j] = c * cp - s * cq;
              C[q * n + j] = s * cp + c * cq;
            }
            for (int j = gl; j < m; j += G) {
              const double wp = W[p * m + j], wq = W[q * m + j];
              W[p * m + j] = c * wp - s * wq;
              W[q * m + j] = s * wp + c * wq;
            }
            if (gl == 0) flag = 1;
          }
        }
        __syncthreads();
      }
      if (flag == 0) break;
      __syncthreads();
    }
    if (sweep == kQttMaxSweeps) st = kQttNoConvergence;
    // singular values: row norms (one group of G lanes per row, rows in turn)
    for (int i0 = 0; i0 < m; i0 += 256 / G) {
      const int i = i0 + grp;
      if (i < m) {
        double a = 0.0;
        for (int j = gl; j < n; j += G) a += C[i * n + j] * C[i * n + j];
        a = group_sum(a, G);
        if (gl == 0) sig[i] = a;  // squared
      }
    }
    __syncthreads();
    if (tid == 0) {
      // descending order of sigma^2 (stable), then the smallest rank whose
      // discarded tail is within delta; at most min(m, n) values exist
      for (int i = 0; i < m; ++i) perm[i] = i;
      for (int i = 1; i < m; ++i) {
        const int pi = perm[i];
        int j = i - 1;
        while (j >= 0 && sig[perm[j]] < sig[pi]) {
          perm[j + 1] = perm[j];
          --j;
        }
        perm[j + 1] = pi;
      }
      const int mn = m < n ? m : n;
      int rk = mn;
      double tail = 0.0;
      // squared tail norms from the smallest candidate upwards
      for (int i = mn - 1; i >= 0; --i) {
        tail += sig[perm[i]];
        tails[i] = tail;
      }
      for (int i = 1; i < mn; ++i)
        if (tails[i] <= delta2) {
          rk = i;
          break;
        }
      rk_sh = rk;
    }
    __syncthreads();
    const int rk = rk_sh;
    if (st != kQttOk) break;
    if (rk > MAXRANK) {
      st = kQttRankLimit;
      break;
    }
    if (off + m * rk > cap) {
      st = kQttCapacity;
      break;
    }
    // core k: G_k[alpha][j][beta] = U[(alpha, j)][perm[beta]] = W[perm[beta]][alpha * 2 + j]
    for (int e = tid; e < m * rk; e += 256) {
      const int row = e / rk, b = e - row * rk;
      out[off + e] = W[perm[b] * m + row];
    }
    off += m * rk;
    if (tid == 0) rv[k] = rk;
    __syncthreads();
    // next unfolding: rows perm[0..rk) of the rotated C (sigma v^T) moved to
    // rows 0..rk-1, staged through W a block of columns at a time (a block is
    // read from every kept row before any of it is written, and later blocks
    // read only columns not yet written)
    const int J = (MR * MR) / rk < n ? (MR * MR) / rk : n;
    for (int j0 = 0; j0 < n; j0 += J) {
      const int jn = n - j0 < J ? n - j0 : J;
      for (int e = tid; e < rk * jn; e += 256) {
        const int b = e / jn, j = e - b * jn;
        W[e] = C[perm[b] * n + j0 + j];
      }
      __syncthreads();
      for (int e = tid; e < rk * jn; e += 256) {
        const int b = e / jn, j = e - b * jn;
        C[b * n + j0 + j] = W[e];
      }
      __syncthreads();
    }
    r = rk;
  }
  if (st == kQttOk) {
    // last core: the remaining 2 r_{d-1} x 1 unfolding
    if (off + 2 * r > cap) {
      st = kQttCapacity;
    } else {
      for (int e = tid; e < 2 * r; e += 256) out[off + e] = C[e];
      if (tid == 0) rv[d] = 1;
    }
  }
  if (tid == 0) status[v] = st;
}

// Expansion (eq. tt): entry i = G_1[:, j_1, :] ... G_d[:, j_d, :] with the
// binary digits of i, most significant first; the cores of a vector staged in
// LDS (at most kQttExpandMax doubles), one row vector of length
// <= kQttMaxRank per lane. A vector whose compression failed, or whose ranks
// or core total are out of range, is written as NaN.
constexpr int kQttExpandMax = 8192;

__global__ __launch_bounds__(256) void k_qtt_expand(const double* __restrict__ cores,
                                                     const int* __restrict__ ranks,
                                                     const int* __restrict__ status, int d,
                                                     int cap, int len, long long ld,
                                                     double* __restrict__ Y) {
  __shared__ double Gs[kQttExpandMax];
  __shared__ int rs[kQttMaxDigits + 1];
  __shared__ int offs[kQttMaxDigits + 1];
  __shared__ int ok;
  const int v = blockIdx.y;
  const int tid = threadIdx.x;
  const double* src = cores + (long long)v * cap;
  if (tid == 0) {
    int good = status[v] == kQttOk;
    int o = 0;
    for (int k = 0; k <= d; ++k) {
      const int rk = good ? ranks[(long long)v * (d + 1) + k] : 1;
      if (rk < 1 || rk > kQttMaxRank) good = 0;
      rs[k] = good ? rk : 1;
    }
    if (rs[0] != 1 || rs[d] != 1) good = 0;
    for (int k = 1; k <= d; ++k) {
      offs[k] = o;
      o += 2 * rs[k - 1] * rs[k];
    }
    if (o > cap || o > kQttExpandMax) good = 0;
    offs[0] = good ? o : 0;
    ok = good;
  }
  __syncthreads();
  const int total = offs[0];
  for (int e = tid; e < total; e += 256) Gs[e] = src[e];
  __syncthreads();
  for (int i = blockIdx.x * 256 + tid; i < len; i += gridDim.x * 256) {
    if (!ok) {
      Y[(long long)v * ld + i] = __builtin_nan("");
      continue;
    }
    double a[kQttMaxRank], b[kQttMaxRank];
#pragma unroll
    for (int c = 0; c < kQttMaxRank; ++c) a[c] = c == 0 ? 1.0 : 0.0;
    int r0 = 1;
    for (int k = 1; k <= d; ++k) {
      const int j = (i >> (d - k)) & 1;
      const int r1 = rs[k];
      const double* Gk = Gs + offs[k];  // [r0][2][r1]
#pragma unroll
      for (int c = 0; c < kQttMaxRank; ++c) {
        double s = 0.0;
        if (c < r1) {
#pragma unroll
          for (int p = 0; p < kQttMaxRank; ++p)
            if (p < r0) s += a[p] * Gk[(p * 2 + j) * r1 + c];
        }
        b[c] = s;
      }
#pragma unroll
      for (int c = 0; c < kQttMaxRank; ++c) a[c] = b[c];
      r0 = r1;
    }
    Y[(long long)v * ld + i] = a[0];
  }
}

}  // namespace ls

using namespace ls;

extern "C" ls_status ls_qtt_compress(const double* x_dev, int32_t nvec, int32_t len, int64_t ld,
                                     double eps, int32_t cap, double* cores_dev,
                                     int32_t* ranks_dev, int32_t* status_dev,
                                     hipStream_t stream) {
  clear_error();
  LS_REQUIRE(x_dev && cores_dev && ranks_dev && status_dev, "null device pointer");
  LS_REQUIRE(nvec >= 1, "nvec must be >= 1");
  LS_REQUIRE(len >= 1 && len <= (1 << kQttMaxDigits), "len must be in [1, %d] (got %d)",
             1 << kQttMaxDigits, len);
  LS_REQUIRE(ld >= len, "ld must be >= len");
  LS_REQUIRE(std::isfinite(eps) && eps >= 0.0, "eps must be finite and >= 0");
  const int d = ls_qtt_digits(len);
  LS_REQUIRE(cap >= 2 * d, "cap must hold at least the rank-1 cores (%d doubles)", 2 * d);
  hipLaunchKernelGGL((k_qtt_compress<kQttFirstRank, false>), dim3(nvec), dim3(256), 0, stream,
                     x_dev, len, (long long)ld, d, eps, cap, cores_dev, ranks_dev, status_dev);
  hipLaunchKernelGGL((k_qtt_compress<kQttMaxRank, true>), dim3(nvec), dim3(256), 0, stream,
                     x_dev, len, (long long)ld, d, eps, cap, cores_dev, ranks_dev, status_dev);
  return launch_status("ls_qtt_compress");
}

extern "C" ls_status ls_qtt_expand(const double* cores_dev, const int32_t* ranks_dev,
                                   const int32_t* status_dev, int32_t nvec, int32_t len,
                                   int32_t cap, double* y_dev, int64_t ld, hipStream_t stream) {
  clear_error();
  LS_REQUIRE(cores_dev && ranks_dev && status_dev && y_dev, "null device pointer");
  LS_REQUIRE(nvec >= 1, "nvec must be >= 1");
  LS_REQUIRE(len >= 1 && len <= (1 << kQttMaxDigits), "len must be in [1, %d] (got %d)",
             1 << kQttMaxDigits, len);
  LS_REQUIRE(ld >= len, "ld must be >= len");
  LS_REQUIRE(cap >= 1, "cap must be >= 1");
  const int d = ls_qtt_digits(len);
  const int bx = (len + 255) / 256 < 16 ? (len + 255) / 256 : 16;
  hipLaunchKernelGGL(k_qtt_expand, dim3(bx, nvec), dim3(256), 0, stream, cores_dev, ranks_dev,
                     status_dev, d, cap, len, (long long)ld, y_dev);
  return launch_status("ls_qtt_expand");
}

extern "C" int32_t ls_qtt_digits(int32_t len) {
  int d = 2;
  while (d < 31 && (1 << d) < len) ++d;
  return d;
}
