// Reconstruction tile shared by the standalone reconstruction kernels and the
// batched persistent kernel (internal header). See ls_recon.hip for the
// formulation.
#pragma once

#include "ls_common.hpp"

namespace ls {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));
typedef short s8_t __attribute__((ext_vector_type(8)));

struct BoxArg {
  const double* A1;
  const double* A2;
  const double* A3;
  const double* coef;
  int K;
  int len0, len1, len2;
  int o0, o1, o2;
  int e0, e1, e2;
  double scale;
};

// A copy of a box descriptor whose integer fields are workgroup-uniform values
// held in scalar registers: read once through readfirstlane, so the compiler
// cannot re-load them from the kernel arguments inside the rank loop (each
// re-load would also wait on every outstanding LDS operation). The pointers
// keep their provenance (global address space).
__device__ __forceinline__ int rfl(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ BoxArg uniform_box(const BoxArg& a) {
  BoxArg u = a;
  u.K = rfl(a.K);
  u.len0 = rfl(a.len0);
  u.len1 = rfl(a.len1);
  u.len2 = rfl(a.len2);
  u.o0 = rfl(a.o0);
  u.o1 = rfl(a.o1);
  u.o2 = rfl(a.o2);
  u.e0 = rfl(a.e0);
  u.e1 = rfl(a.e1);
  u.e2 = rfl(a.e2);
  return u;
}

template <typename T>
struct Acc;
template <>
struct Acc<double> {
  typedef d4_t type;
};
template <>
struct Acc<float> {
  typedef f4_t type;
};

__device__ __forceinline__ d4_t mfma(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Operand staging shared by all precisions. One rank chunk of BK rows is
// staged per step; lane t of the workgroup owns rank row kk = t / TPR and
// rows m = q + TPR*e (q = t % TPR, e = 0..EPT-1) of the W operand, so every
// load instruction of a 16-lane group reads 16 consecutive doubles.
// ONEI (the BM rows of the tile share one i, uniform per workgroup):
// W[r][m] = alpha_r * f1[r][o1 + j0 + m - row0] with alpha_r = coef[r] f0[r][o0 + i]
// (two loads per rank row); otherwise every element loads its own f0 and f1
// values, at clamped ranks and rows without conditions (rank rows past K give
// 0 through w_value, rows past the box are never stored). The two cases are
// separate instantiations, so that the waits the compiler places for one do
// not follow the other's loads.
// load() only issues loads: the products are formed by w_value() when the
// chunk is written to LDS one step later, so the loads of chunk c+1 stay in
// flight while the MFMAs consume chunk c (a use right after the load would
// make the wave wait for memory there).
template <int BM, int BN, int BK, bool ONEI>
struct Stager {
  static constexpr int EPT_W = BK * BM / 256;
  static constexpr int TPR_W = BM / EPT_W;
  static constexpr int EPT_Y = BK * BN / 256;
  static constexpr int TPR_Y = BN / EPT_Y;
  static_assert(EPT_W >= 1 && EPT_Y >= 1 && TPR_W * BK == 256 && TPR_Y * BK == 256, "staging map");

  int wk, wq, yk, yq;
  int row0, col0, M, i0, j0;
  bool yfast;
  bool rv;        // !ONEI: the rank row of this chunk is below K
  double cr, a1;  // ONEI: alpha = cr * a1
  double w[EPT_W];
  double w0[ONEI ? 1 : EPT_W];  // !ONEI: each row's f0 value
  double y[EPT_Y];

  __device__ __forceinline__ void init(const BoxArg& a, int r0, int c0) {
    const int tid = threadIdx.x;
    wk = tid / TPR_W;
    wq = tid - wk * TPR_W;
    yk = tid / TPR_Y;
    yq = tid - yk * TPR_Y;
    row0 = r0;
    col0 = c0;
    M = a.e0 * a.e1;
    i0 = row0 / a.e1;
    j0 = row0 - i0 * a.e1;
    yfast = col0 + BN <= a.e2;
  }

  // (coef f0) f1 in this order on both paths
  __device__ __forceinline__ double w_value(int e) const {
    if constexpr (ONEI)
      return (cr * a1) * w[e];
    else
      return rv ? (cr * w0[e]) * w[e] : 0.0;
  }

  __device__ __forceinline__ void load(const BoxArg& a, int k0) {
    const int r = k0 + wk;
    if constexpr (ONEI) {
      cr = 1.0;
      a1 = 1.0;
      if (r < a.K) {
        cr = a.coef[r];
        a1 = a.A1[(size_t)r * a.len0 + a.o0 + i0];
        const double* src = a.A2 + (size_t)r * a.len1 + a.o1 + j0 + wq;
#pragma unroll
        for (int e = 0; e < EPT_W; ++e) w[e] = src[e * TPR_W];
      } else {
#pragma unroll
        for (int e = 0; e < EPT_W; ++e) w[e] = 0.0;
      }
    } else {
      rv = r < a.K;
      const int rc = min(r, a.K - 1);
      cr = a.coef[rc];
#pragma unroll
      for (int e = 0; e < EPT_W; ++e) {
        const int m = row0 + wq + e * TPR_W;
        const int mc = m < M ? m : row0;  // rows past the box: never stored
        const int i = mc / a.e1, j = mc - i * a.e1;
        w[e] = a.A2[(size_t)rc * a.len1 + a.o1 + j];
        w0[e] = a.A1[(size_t)rc * a.len0 + a.o0 + i];
      }
    }
    const int ry = k0 + yk;
    if (ry < a.K) {
      const double* src = a.A3 + (size_t)ry * a.len2 + a.o2 + col0 + yq;
      if (yfast) {
#pragma unroll
        for (int e = 0; e < EPT_Y; ++e) y[e] = src[e * TPR_Y];
      } else {
#pragma unroll
        for (int e = 0; e < EPT_Y; ++e) y[e] = (col0 + yq + e * TPR_Y < a.e2) ? src[e * TPR_Y] : 0.0;
      }
    } else {
#pragma unroll
      for (int e = 0; e < EPT_Y; ++e) y[e] = 0.0;
    }
  }
};

// rows of the tile in one value of i
template <int BM>
__device__ __forceinline__ bool tile_one_i(const BoxArg& a, int row0) {
  const int M = a.e0 * a.e1, i0 = row0 / a.e1;
  return (row0 + BM <= M) && ((row0 + BM - 1) / a.e1 == i0);
}

// FP64 / FP32 tile. T = operand type. Two LDS buffers: the global loads of
// chunk c+1 are in flight while the MFMAs consume chunk c. `smem` holds
// recon_smem_bytes<T, BM, BN, BK>() bytes.
template <typename T, int BM, int BN, int BK>
constexpr int recon_smem_bytes() {
  return 2 * BK * (BM + BN + 2 * ((sizeof(T) == 8) ? 2 : 16)) * (int)sizeof(T);
}

template <typename T, int BM, int BN, int WM, int WN, int BK, bool ONEI>
__device__ __forceinline__ void recon_tile_run(const BoxArg& a, int row0, int col0,
                                               T* __restrict__ out, char* smem) {
  static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");
  typedef typename Acc<T>::type acc_t;
  constexpr int FM = WM / 16, FN = WN / 16;
  // row padding: the four rank rows of one MFMA operand read (and of one
  // staging store) then start 16 banks apart (FP32: stride = 16 mod 64 words)
  constexpr int PAD = (sizeof(T) == 8) ? 2 : 16;
  typedef T WsRow[BK][BM + PAD];
  typedef T YsRow[BK][BN + PAD];
  WsRow* Ws = reinterpret_cast<WsRow*>(smem);
  YsRow* Ys = reinterpret_cast<YsRow*>(smem + 2 * sizeof(WsRow));

  const int M = a.e0 * a.e1;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave / (BN / WN)) * WM;
  const int wc = (wave % (BN / WN)) * WN;
  const int lr = lane & 15;
  const int lk = lane >> 4;

  acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

  typedef Stager<BM, BN, BK, ONEI> St;
  St st;
  st.init(a, row0, col0);
  st.load(a, 0);
  const int nchunk = (a.K + BK - 1) / BK;
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
#pragma unroll
    for (int e = 0; e < St::EPT_W; ++e) Ws[buf][st.wk][st.wq + e * St::TPR_W] = (T)st.w_value(e);
#pragma unroll
    for (int e = 0; e < St::EPT_Y; ++e) Ys[buf][st.yk][st.yq + e * St::TPR_Y] = (T)st.y[e];
    __syncthreads();
    if (c + 1 < nchunk) st.load(a, (c + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[FM], bv[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) av[i] = Ws[buf][kk + lk][wr + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < FN; ++j) bv[j] = Ys[buf][kk + lk][wc + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = mfma(av[i], bv[j], acc[i][j]);
    }
  }

  const T sc = (T)a.scale;
  constexpr bool f64_layout = sizeof(T) == 8;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wr + i * 16 + (f64_layout ? lk + 4 * v : 4 * lk + v);
        const int col = col0 + wc + j * 16 + lr;
        if (row < M && col < a.e2) out[(size_t)row * a.e2 + col] = sc * acc[i][j][v];
      }
}

template <typename T, int BM, int BN, int WM, int WN, int BK>
__device__ __forceinline__ void recon_tile(const BoxArg& a, int row0, int col0, T* __restrict__ out,
                                           char* smem) {
  if (tile_one_i<BM>(a, row0))
    recon_tile_run<T, BM, BN, WM, WN, BK, true>(a, row0, col0, out, smem);
  else
    recon_tile_run<T, BM, BN, WM, WN, BK, false>(a, row0, col0, out, smem);
}

typedef float f16v_t __attribute__((ext_vector_type(16)));

// FP32 tile on v_mfma_f32_32x32x2f32: each wave owns a WM x WN sub-tile of
// 32x32 blocks; lane l supplies A[l%32][k = l/32] and B[k = l/32][l%32] and
// receives D[8(v/4) + 4(l/32) + v%4][l%32], v = 0..15. Row stride of the LDS
// operands is 32 mod 64 words, so the two rank rows of one operand read fall
// on disjoint banks.
template <int BM, int BN, int BK>
constexpr int recon32_smem_bytes() {
  return 2 * BK * (BM + BN + 2 * 32) * (int)sizeof(float);
}

template <int BM, int BN, int WM, int WN, int BK, bool ONEI>
__device__ __forceinline__ void recon_tile32_run(const BoxArg& a, int row0, int col0,
                                                 float* __restrict__ out, char* smem) {
  static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");
  constexpr int FM = WM / 32, FN = WN / 32;
  constexpr int PAD = 32;
  typedef float WsRow[BK][BM + PAD];
  typedef float YsRow[BK][BN + PAD];
  WsRow* Ws = reinterpret_cast<WsRow*>(smem);
  YsRow* Ys = reinterpret_cast<YsRow*>(smem + 2 * sizeof(WsRow));

  const int M = a.e0 * a.e1;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave / (BN / WN)) * WM;
  const int wc = (wave % (BN / WN)) * WN;
  const int lr = lane & 31;
  const int lk = lane >> 5;

  f16v_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  typedef Stager<BM, BN, BK, ONEI> St;
  St st;
  st.init(a, row0, col0);
  st.load(a, 0);
  const int nchunk = (a.K + BK - 1) / BK;
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
#pragma unroll
    for (int e = 0; e < St::EPT_W; ++e) Ws[buf][st.wk][st.wq + e * St::TPR_W] = (float)st.w_value(e);
#pragma unroll
    for (int e = 0; e < St::EPT_Y; ++e) Ys[buf][st.yk][st.yq + e * St::TPR_Y] = (float)st.y[e];
    __syncthreads();
    if (c + 1 < nchunk) st.load(a, (c + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 2) {
      float av[FM], bv[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) av[i] = Ws[buf][kk + lk][wr + i * 32 + lr];
#pragma unroll
      for (int j = 0; j < FN; ++j) bv[j] = Ys[buf][kk + lk][wc + j * 32 + lr];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
  }

  const float sc = (float)a.scale;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = row0 + wr + i * 32 + 8 * (v >> 2) + 4 * lk + (v & 3);
        const int col = col0 + wc + j * 32 + lr;
        if (row < M && col < a.e2) out[(size_t)row * a.e2 + col] = sc * acc[i][j][v];
      }
}

template <int BM, int BN, int WM, int WN, int BK>
__device__ __forceinline__ void recon_tile32(const BoxArg& a, int row0, int col0,
                                             float* __restrict__ out, char* smem) {
  if (tile_one_i<BM>(a, row0))
    recon_tile32_run<BM, BN, WM, WN, BK, true>(a, row0, col0, out, smem);
  else
    recon_tile32_run<BM, BN, WM, WN, BK, false>(a, row0, col0, out, smem);
}

}  // namespace ls
