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

// All boxes of one call (up to kBoxesPerLaunch) share one launch, so the
// last partial round of workgroups is paid once, not once per box. Workgroup
// g runs on XCD g mod 8; the logical tile index is chosen so that each XCD
// takes a contiguous range of tiles (the tiles of one or two boxes), which
// keeps each box's factor slices in one XCD's L2.
constexpr int kBoxesPerLaunch = 24;

struct BoxSet {
  BoxArg box[kBoxesPerLaunch];
  long long tile_start[kBoxesPerLaunch + 1];  // prefix sums of tiles per box
  long long out_off[kBoxesPerLaunch];         // element offset of each box in out
  int tiles_n[kBoxesPerLaunch];               // column tiles per box
  int nbox;
  long long per_xcd;                          // tiles per XCD range
};

__device__ __forceinline__ bool locate(const BoxSet& bs, int* b, int* tm, int* tn) {
  const long long g = blockIdx.x;
  const long long t = (g & 7) * bs.per_xcd + (g >> 3);
  if (t >= bs.tile_start[bs.nbox]) return false;
  int i = 0;
  while (i + 1 < bs.nbox && bs.tile_start[i + 1] <= t) ++i;
  const long long local = t - bs.tile_start[i];
  *b = i;
  *tm = (int)(local / bs.tiles_n[i]);
  *tn = (int)(local - (long long)(*tm) * bs.tiles_n[i]);
  return true;
}

template <typename T, int BM, int BN, int WM, int WN, int BK>
__global__ __launch_bounds__(256) void k_recon(BoxSet bs, T* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) char smem[recon_smem_bytes<T, BM, BN, BK>()];
  int b, tm, tn;
  if (!locate(bs, &b, &tm, &tn)) return;
  recon_tile<T, BM, BN, WM, WN, BK>(bs.box[b], tm * BM, tn * BN, out + bs.out_off[b], smem);
}

template <int BM, int BN, int WM, int WN, int BK>
__global__ __launch_bounds__(256) void k_recon32(BoxSet bs, float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) char smem[recon32_smem_bytes<BM, BN, BK>()];
  int b, tm, tn;
  if (!locate(bs, &b, &tm, &tn)) return;
  recon_tile32<BM, BN, WM, WN, BK>(bs.box[b], tm * BM, tn * BN, out + bs.out_off[b], smem);
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
__global__ __launch_bounds__(256) void k_recon_bf16(BoxSet bs, float* __restrict__ out_all) {
  int bidx, tmi, tni;
  if (!locate(bs, &bidx, &tmi, &tni)) return;
  const BoxArg& a = bs.box[bidx];
  float* __restrict__ out = out_all + bs.out_off[bidx];
  static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");
  constexpr int BK = 32;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int KP = BK + 8;  // padded row (elements)
  typedef Stager<BM, BN, BK> S;
  __shared__ __attribute__((aligned(16))) unsigned short Ws[2][NT][BM][KP];
  __shared__ __attribute__((aligned(16))) unsigned short Ys[2][NT][BN][KP];

  const int M = a.e0 * a.e1;
  const int row0 = tmi * BM;
  const int col0 = tni * BN;
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
static void fill_tiles(BoxSet* bs, int bm, int bn) {
  long long acc = 0;
  for (int i = 0; i < bs->nbox; ++i) {
    const BoxArg& a = bs->box[i];
    const long long tm = ((long long)a.e0 * a.e1 + bm - 1) / bm;
    bs->tiles_n[i] = (a.e2 + bn - 1) / bn;
    bs->tile_start[i] = acc;
    acc += tm * bs->tiles_n[i];
  }
  bs->tile_start[bs->nbox] = acc;
  bs->per_xcd = (acc + 7) / 8;
}

template <typename T>
static bool launch_fp(int tile, hipStream_t s, BoxSet& bs, void* out, bool dry) {
  dim3 block(256);
#define LS_T(ID, BM_, BN_, WM_, WN_, BK_)                                                     \
  if (tile == ID) {                                                                          \
    if (!dry) {                                                                              \
      fill_tiles(&bs, BM_, BN_);                                                             \
      dim3 grid((unsigned)(8 * bs.per_xcd));                                                 \
      hipLaunchKernelGGL((k_recon<T, BM_, BN_, WM_, WN_, BK_>), grid, block, 0, s, bs, (T*)out); \
    }                                                                                        \
    return true;                                                                             \
  }
  LS_T(1, 128, 128, 64, 64, 16)
  LS_T(2, 64, 64, 32, 32, 16)
  LS_T(3, 128, 64, 64, 32, 16)
  LS_T(4, 64, 128, 32, 64, 16)
  LS_T(5, 128, 128, 64, 64, 32)
#undef LS_T
  if (sizeof(T) == 4) {
#define LS_T32(ID, BM_, BN_, WM_, WN_, BK_)                                                   \
  if (tile == ID) {                                                                          \
    if (!dry) {                                                                              \
      fill_tiles(&bs, BM_, BN_);                                                             \
      dim3 grid((unsigned)(8 * bs.per_xcd));                                                 \
      hipLaunchKernelGGL((k_recon32<BM_, BN_, WM_, WN_, BK_>), grid, block, 0, s, bs, (float*)out); \
    }                                                                                        \
    return true;                                                                             \
  }
    LS_T32(6, 128, 128, 64, 64, 16)
    LS_T32(7, 128, 64, 64, 32, 16)
    LS_T32(8, 128, 128, 64, 64, 32)
#undef LS_T32
  }
  return false;
}

template <int NT>
static bool launch_bf(int tile, hipStream_t s, BoxSet& bs, void* out, bool dry) {
  dim3 block(256);
#define LS_T(ID, BM_, BN_, WM_, WN_)                                                          \
  if (tile == ID) {                                                                          \
    if (!dry) {                                                                              \
      fill_tiles(&bs, BM_, BN_);                                                             \
      dim3 grid((unsigned)(8 * bs.per_xcd));                                                 \
      hipLaunchKernelGGL((k_recon_bf16<NT, BM_, BN_, WM_, WN_>), grid, block, 0, s, bs, (float*)out); \
    }                                                                                        \
    return true;                                                                             \
  }
  LS_T(1, 128, 128, 64, 64)
  LS_T(2, 64, 64, 32, 32)
  LS_T(3, 128, 64, 64, 32)
  LS_T(4, 64, 128, 32, 64)
#undef LS_T
  return false;
}

static int n_tiles(int precision) {
  return precision == LS_F32 ? 8 : (precision == LS_F64 ? 5 : 4);
}

static bool dispatch(int precision, int tile, hipStream_t s, BoxSet& bs, void* out, bool dry) {
  switch (precision) {
    case LS_F64: return launch_fp<double>(tile, s, bs, out, dry);
    case LS_F32: return launch_fp<float>(tile, s, bs, out, dry);
    case LS_BF16X3: return launch_bf<2>(tile, s, bs, out, dry);
    case LS_BF16X6: return launch_bf<3>(tile, s, bs, out, dry);
    default: return false;
  }
}

// Tile picked when the caller passes tile = 0 (measured on 256^3 boxes,
// K = 384: FP32 128x128 rank chunk 32, FP64 64x128).
static int auto_tile(int precision, long long M, long long Nc) {
  const long long big = ((M + 127) / 128) * ((Nc + 127) / 128);
  if (precision == LS_F32 && big >= 256) return 5;
  if (precision == LS_F64 && big >= 256) return 4;
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
  const int t = tile ? tile : auto_tile(precision, (long long)boxes[0].e[0] * boxes[0].e[1],
                                        boxes[0].e[2]);
  BoxSet probe;
  if (!dispatch(precision, t, stream, probe, nullptr, true)) {
    set_error("tile %d not available for precision %d", t, precision);
    return LS_EUNSUPPORTED;
  }
  long long off = 0;  // elements
  for (int b0 = 0; b0 < nbox; b0 += kBoxesPerLaunch) {
    BoxSet bs;
    bs.nbox = (nbox - b0) < kBoxesPerLaunch ? (nbox - b0) : kBoxesPerLaunch;
    long long local = 0;
    for (int i = 0; i < bs.nbox; ++i) {
      const ls_box& bx = boxes[b0 + i];
      BoxArg& a = bs.box[i];
      a.A1 = P->f[0];
      a.A2 = P->f[1];
      a.A3 = P->f[2];
      a.coef = P->coef;
      a.K = P->K;
      a.len0 = P->len[0];
      a.len1 = P->len[1];
      a.len2 = P->len[2];
      a.o0 = bx.o[0];
      a.o1 = bx.o[1];
      a.o2 = bx.o[2];
      a.e0 = bx.e[0];
      a.e1 = bx.e[1];
      a.e2 = bx.e[2];
      a.scale = scale;
      bs.out_off[i] = local;
      local += (long long)bx.e[0] * bx.e[1] * bx.e[2];
    }
    char* out = (char*)out_dev + off * (precision == LS_F64 ? 8 : 4);
    dispatch(precision, t, stream, bs, out, false);
    ls_status st = launch_status("ls_reconstruct");
    if (st != LS_OK) return st;
    off += local;
  }
  return LS_OK;
}
