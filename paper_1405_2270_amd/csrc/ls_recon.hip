// Reconstruction of sub-boxes of a canonical tensor (Appendix, eq. CP_form)
// on MFMA.
//
// One box is one GEMM: rows m = (i, j) of the box (M = e0*e1), columns k
// (Nc = e2, contiguous in the C-order output), reduction over the rank r:
//   V[m][k] = scale * sum_r W[r][m] * Y[r][k],
//   W[r][m] = coef[r] f0[r][o0+i] f1[r][o1+j]   (Khatri-Rao operand, formed
//                                                  while staging into LDS)
//   Y[r][k] = f2[r][o2+k].
// A workgroup of four waves owns a BM x BN output tile and walks the rank in
// chunks of BK, staging W and Y in LDS; each wave owns a WM x WN sub-tile made
// of 16x16 MFMA blocks.
//
// Precisions
//   FP64 : v_mfma_f64_16x16x4f64, FP64 in and out.
//   FP32 : W, Y rounded to FP32, v_mfma_f32_16x16x4f32, FP32 out.
//   BF16x3 / BF16x6: W and Y split into bf16 terms x = x0 + x1 (+ x2) and
//          the products x0y0 + x0y1 + x1y0 (+ x0y2 + x2y0 + x1y1) on
//          v_mfma_f32_16x16x32_bf16 with FP32 accumulation, FP32 out.
//
// MFMA operand layout (16x16 blocks, wave of 64 lanes): lane l supplies
// A[l%16][k-group l/16] and B[k-group l/16][l%16]. It receives D[4*(l/16) + v][l%16]
// (v = 0..3) from the f32 and bf16 instructions, and D[l/16 + 4v][l%16] from the
// f64 one (checked on gfx950).
#include "ls_recon_tile.hpp"

namespace ls {

template <typename T, int BM, int BN, int WM, int WN, int BK>
__global__ __launch_bounds__(256) void k_recon(BoxArg a, T* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) char smem[recon_smem_bytes<T, BM, BN, BK>()];
  recon_tile<T, BM, BN, WM, WN, BK>(a, blockIdx.x * BM, blockIdx.y * BN, out, smem);
}

// ---------------------------------------------------------------------------
// split-bf16 kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  __bf16 h = (__bf16)x;  // round to nearest even
  return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_val(unsigned short u) {
  return __builtin_bit_cast(float, (unsigned int)u << 16);
}

// NT terms: 2 (x3 products) or 3 (x6 products). Operands in LDS as
// [term][row][BK] bf16 with the rank contiguous (16-byte MFMA operand loads);
// the staging writes transpose the rank-major global layout. Two LDS buffers
// as in the FP kernels.
template <int NT>
__device__ __forceinline__ void split_store(double v, unsigned short* dst, int plane) {
  double rem = v;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const unsigned short u = bf16_bits((float)rem);
    dst[t * plane] = u;
    rem -= (double)bf16_val(u);
  }
}

template <int NT, int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256) void k_recon_bf16(BoxArg a, float* __restrict__ out) {
  static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");
  constexpr int BK = 32;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int KP = BK + 8;  // padded row (elements)
  typedef Stager<BM, BN, BK> S;
  __shared__ __attribute__((aligned(16))) unsigned short Ws[2][NT][BM][KP];
  __shared__ __attribute__((aligned(16))) unsigned short Ys[2][NT][BN][KP];

  const int M = a.e0 * a.e1;
  const int row0 = blockIdx.x * BM;
  const int col0 = blockIdx.y * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = (wave / (BN / WN)) * WM;
  const int wc = (wave % (BN / WN)) * WN;
  const int lr = lane & 15;
  const int lk = lane >> 4;

  f4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

  S st;
  st.init(a, row0, col0);
  st.load(a, 0);
  const int nchunk = (a.K + BK - 1) / BK;
  for (int c = 0; c < nchunk; ++c) {
    const int buf = c & 1;
#pragma unroll
    for (int e = 0; e < S::EPT_W; ++e)
      split_store<NT>(st.w[e], &Ws[buf][0][st.wq + e * S::TPR_W][st.wk], BM * KP);
#pragma unroll
    for (int e = 0; e < S::EPT_Y; ++e)
      split_store<NT>(st.y[e], &Ys[buf][0][st.yq + e * S::TPR_Y][st.yk], BN * KP);
    __syncthreads();
    if (c + 1 < nchunk) st.load(a, (c + 1) * BK);
    s8_t av[NT][FM], bv[NT][FN];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
        av[t][i] = *reinterpret_cast<const s8_t*>(&Ws[buf][t][wr + i * 16 + lr][lk * 8]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bv[t][j] = *reinterpret_cast<const s8_t*>(&Ys[buf][t][wc + j * 16 + lr][lk * 8]);
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        // smallest terms first
        if (NT == 3) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf8_t, av[1][i]), __builtin_bit_cast(bf8_t, bv[1][j]), acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf8_t, av[0][i]), __builtin_bit_cast(bf8_t, bv[NT - 1][j]), acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf8_t, av[NT - 1][i]), __builtin_bit_cast(bf8_t, bv[0][j]), acc[i][j], 0, 0, 0);
        }
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8_t, av[0][i]), __builtin_bit_cast(bf8_t, bv[1][j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8_t, av[1][i]), __builtin_bit_cast(bf8_t, bv[0][j]), acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
            __builtin_bit_cast(bf8_t, av[0][i]), __builtin_bit_cast(bf8_t, bv[0][j]), acc[i][j], 0, 0, 0);
      }
  }

  const float sc = (float)a.scale;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = row0 + wr + i * 16 + 4 * lk + v;
        const int col = col0 + wc + j * 16 + lr;
        if (row < M && col < a.e2) out[(size_t)row * a.e2 + col] = sc * acc[i][j][v];
      }
}

// ---------------------------------------------------------------------------
// tile table
// ---------------------------------------------------------------------------
struct TileInfo {
  int bm, bn;
};

template <typename T>
static void launch_fp(int tile, dim3 block, hipStream_t s, const BoxArg& a, void* out, int* bm,
                      int* bn, bool dry) {
  const int M = a.e0 * a.e1;
#define LS_T(ID, BM_, BN_, WM_, WN_, BK_)                                                     \
  if (tile == ID) {                                                                          \
    *bm = BM_;                                                                               \
    *bn = BN_;                                                                               \
    if (!dry) {                                                                              \
      dim3 grid((M + BM_ - 1) / BM_, (a.e2 + BN_ - 1) / BN_);                                \
      hipLaunchKernelGGL((k_recon<T, BM_, BN_, WM_, WN_, BK_>), grid, block, 0, s, a, (T*)out); \
    }                                                                                        \
    return;                                                                                  \
  }
  LS_T(1, 128, 128, 64, 64, 16)
  LS_T(2, 64, 64, 32, 32, 16)
  LS_T(3, 128, 64, 64, 32, 16)
  LS_T(4, 64, 128, 32, 64, 16)
  LS_T(5, 128, 128, 64, 64, 32)
#undef LS_T
  *bm = 0;
}

template <int NT>
static void launch_bf(int tile, dim3 block, hipStream_t s, const BoxArg& a, void* out, int* bm,
                      int* bn, bool dry) {
  const int M = a.e0 * a.e1;
#define LS_T(ID, BM_, BN_, WM_, WN_)                                                          \
  if (tile == ID) {                                                                          \
    *bm = BM_;                                                                               \
    *bn = BN_;                                                                               \
    if (!dry) {                                                                              \
      dim3 grid((M + BM_ - 1) / BM_, (a.e2 + BN_ - 1) / BN_);                                \
      hipLaunchKernelGGL((k_recon_bf16<NT, BM_, BN_, WM_, WN_>), grid, block, 0, s, a, (float*)out); \
    }                                                                                        \
    return;                                                                                  \
  }
  LS_T(1, 128, 128, 64, 64)
  LS_T(2, 64, 64, 32, 32)
  LS_T(3, 128, 64, 64, 32)
  LS_T(4, 64, 128, 32, 64)
#undef LS_T
  *bm = 0;
}

static int n_tiles(int precision) { return precision == LS_F64 || precision == LS_F32 ? 5 : 4; }

static void dispatch(int precision, int tile, hipStream_t s, const BoxArg& a, void* out, int* bm,
                     int* bn, bool dry) {
  dim3 block(256);
  switch (precision) {
    case LS_F64: launch_fp<double>(tile, block, s, a, out, bm, bn, dry); break;
    case LS_F32: launch_fp<float>(tile, block, s, a, out, bm, bn, dry); break;
    case LS_BF16X3: launch_bf<2>(tile, block, s, a, out, bm, bn, dry); break;
    case LS_BF16X6: launch_bf<3>(tile, block, s, a, out, bm, bn, dry); break;
    default: *bm = 0;
  }
}

// Tile picked when the caller passes tile = 0: the largest tile that still
// gives every compute unit at least two workgroups.
static int auto_tile(int precision, long long M, long long Nc) {
  const long long big = ((M + 127) / 128) * ((Nc + 127) / 128);
  if (big >= 512) return 1;
  const long long mid = ((M + 127) / 128) * ((Nc + 63) / 64);
  if (mid >= 512) return 3;
  return 2;
}

}  // namespace ls

using namespace ls;

extern "C" int32_t ls_reconstruct_tiles(int32_t precision) {
  if (precision < LS_F64 || precision > LS_BF16X6) return 0;
  return n_tiles(precision);
}

extern "C" ls_status ls_reconstruct(const ls_canon* P, const ls_box* boxes, int32_t nbox,
                                    double scale, int32_t precision, int32_t tile, void* out_dev,
                                    hipStream_t stream) {
  clear_error();
  LS_REQUIRE(P != nullptr && boxes != nullptr && out_dev != nullptr, "null pointer");
  LS_REQUIRE(P->K >= 1, "rank K must be >= 1");
  LS_REQUIRE(P->f[0] && P->f[1] && P->f[2] && P->coef, "null factor pointer");
  LS_REQUIRE(nbox >= 1, "nbox must be >= 1");
  LS_REQUIRE(std::isfinite(scale), "scale must be finite");
  LS_REQUIRE(precision >= LS_F64 && precision <= LS_BF16X6, "unknown precision %d", precision);
  if (tile < 0 || tile > n_tiles(precision)) {
    set_error("tile %d not valid for precision %d", tile, precision);
    return LS_EUNSUPPORTED;
  }
  for (int b = 0; b < nbox; ++b) {
    for (int l = 0; l < 3; ++l) {
      LS_REQUIRE(P->len[l] >= 1, "len[%d] must be >= 1", l);
      LS_REQUIRE(boxes[b].e[l] >= 1 && boxes[b].o[l] >= 0 &&
                     (long long)boxes[b].o[l] + boxes[b].e[l] <= P->len[l],
                 "box %d outside the factors on axis %d", b, l);
    }
    LS_REQUIRE((long long)boxes[b].e[0] * boxes[b].e[1] < (1LL << 31), "box %d too large", b);
  }
  const size_t esz = precision == LS_F64 ? sizeof(double) : sizeof(float);
  char* out = (char*)out_dev;
  for (int b = 0; b < nbox; ++b) {
    BoxArg a;
    a.A1 = P->f[0];
    a.A2 = P->f[1];
    a.A3 = P->f[2];
    a.coef = P->coef;
    a.K = P->K;
    a.len0 = P->len[0];
    a.len1 = P->len[1];
    a.len2 = P->len[2];
    a.o0 = boxes[b].o[0];
    a.o1 = boxes[b].o[1];
    a.o2 = boxes[b].o[2];
    a.e0 = boxes[b].e[0];
    a.e1 = boxes[b].e[1];
    a.e2 = boxes[b].e[2];
    a.scale = scale;
    const int t = tile ? tile : auto_tile(precision, (long long)a.e0 * a.e1, a.e2);
    int bm = 0, bn = 0;
    dispatch(precision, t, stream, a, out, &bm, &bn, false);
    if (bm == 0) {
      set_error("tile %d not available for precision %d", t, precision);
      return LS_EUNSUPPORTED;
    }
    ls_status st = launch_status("ls_reconstruct");
    if (st != LS_OK) return st;
    out += esz * (size_t)a.e0 * a.e1 * a.e2;
  }
  return LS_OK;
}
