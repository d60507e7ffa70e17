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
//   BF16x3 / BF16x6: W and Y rounded to FP32 and split into bf16 terms
//          x = x0 + x1 (+ x2), products x0y0 + x0y1 + x1y0 (+ x1y1 + x0y2 + x2y0)
//          on v_mfma_f32_16x16x32_bf16 with FP32 accumulation, FP32 out.
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
// Every operand value is rounded once to FP32 and cut into NT bf16 terms by
// truncation: x0 = x with its low 16 bits cleared, x1 = (x - x0) likewise,
// x2 = x - x0 - x1. Each difference is exact in FP32, and three 8-bit bf16
// significands hold the whole 24-bit FP32 significand, so x0 + x1 + x2 = x.
// With NT = 2 the last term is rounded to nearest (|x - x0 - x1| <= 2^-16 |x|).
// Products: x0y0 + x0y1 + x1y0, and for NT = 3 also x1y1 + x0y2 + x2y0, on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation, smallest terms first.
//
// Staging map: thread t owns operand row m = t % BM and the KW = BM/8
// consecutive ranks from (t / BM) * KW of each 32-rank chunk, so its terms go
// to LDS as packed 16-byte writes (8 ranks: what one MFMA lane reads). One LDS
// row holds the 32 ranks of one operand row (64 bytes); 16-byte slot s of row
// m sits at slot s ^ ((m >> 2) & 3), which keeps the packed writes of
// consecutive rows and the MFMA reads (16 rows, one slot) free of bank
// conflicts.
//
// The rank factor alpha_r = coef[r] f0[r][o0 + i] of a tile whose rows share
// one i (else coef[r], with f0 multiplied into each element) is kept in LDS:
// loaded two chunks ahead and written one chunk ahead. The loads of chunk
// c+1 stay raw in registers while the MFMAs consume chunk c; all arithmetic
// happens when the chunk is written to LDS.
constexpr int SPLIT_BK = 32;

template <int NT>
__device__ __forceinline__ void split_fp32(float x, unsigned (&u)[NT]) {
  unsigned b = __float_as_uint(x);
#pragma unroll
  for (int t = 0; t < NT - 1; ++t) {
    const unsigned hi = b & 0xffff0000u;
    u[t] = hi;
    x -= __uint_as_float(hi);
    b = __float_as_uint(x);
  }
  if (NT == 2) b += 0x7fffu + ((b >> 16) & 1u);
  u[NT - 1] = b;  // low half dropped when packed
}

__device__ __forceinline__ unsigned pack_hi(unsigned even, unsigned odd) {
  return (odd & 0xffff0000u) | (even >> 16);
}

template <int NT, int BM, int BN, int WM, int WN, int NBUF>
__global__ __launch_bounds__(256) void k_recon_split(BoxSet bs, float* __restrict__ out_all) {
  constexpr int BK = SPLIT_BK;
  constexpr int KW = BK * BM / 256, KY = BK * BN / 256;
  static_assert(BM >= 64 && BN >= 64 && 256 % BM == 0 && 256 % BN == 0, "staging map");
  static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");
  constexpr int FM = WM / 16, FN = WN / 16;
  __shared__ __attribute__((aligned(16))) unsigned Ws[NBUF][NT][BM][16];
  __shared__ __attribute__((aligned(16))) unsigned Ys[NBUF][NT][BN][16];
  __shared__ double alphaS[2][BK];

  int bidx, tmi, tni;
  if (!locate(bs, &bidx, &tmi, &tni)) return;
  const BoxArg& a = bs.box[bidx];
  float* __restrict__ out = out_all + bs.out_off[bidx];
  const int M = a.e0 * a.e1;
  const int row0 = tmi * BM, col0 = tni * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave / (BN / WN)) * WM, wc = (wave % (BN / WN)) * WN;
  const int lr = lane & 15, lk = lane >> 4;

  // staging ownership (tid / BM and tid / BN are uniform per wave: BM, BN >= 64)
  const int mw = tid % BM, ny = tid % BN;
  const int kbw = __builtin_amdgcn_readfirstlane(tid / BM) * KW;
  const int kby = __builtin_amdgcn_readfirstlane(tid / BN) * KY;
  const int i0 = row0 / a.e1;
  const bool wfast = (row0 + BM <= M) && ((row0 + BM - 1) / a.e1 == i0);
  const int m = row0 + mw;
  const bool mok = m < M;
  const int mi = mok ? m / a.e1 : 0;
  const int mj = mok ? m - mi * a.e1 : 0;
  const bool nok = col0 + ny < a.e2;
  const double* __restrict__ a1row = a.A1 + a.o0 + mi;
  const double* __restrict__ a2row = a.A2 + a.o1 + mj;
  const double* __restrict__ a3row = a.A3 + a.o2 + col0 + ny;
  const int nchunk = (a.K + BK - 1) / BK;

  double w[KW], y[KY];
  double cr = 0.0, ca = 1.0;  // raw parts of one alpha_r (threads tid < BK)

  auto load_ops = [&](int k0) {
#pragma unroll
    for (int kk = 0; kk < KW; ++kk) {
      const int r = k0 + kbw + kk;
      double v = 0.0;
      if (r < a.K && mok) {
        v = a2row[(size_t)r * a.len1];
        if (!wfast) v *= a1row[(size_t)r * a.len0];
      }
      w[kk] = v;
    }
#pragma unroll
    for (int kk = 0; kk < KY; ++kk) {
      const int r = k0 + kby + kk;
      y[kk] = (r < a.K && nok) ? a3row[(size_t)r * a.len2] : 0.0;
    }
  };
  auto load_alpha = [&](int k0) {
    const int r = k0 + tid;
    cr = 0.0;
    ca = 1.0;
    if (tid < BK && r < a.K) {
      cr = a.coef[r];
      if (wfast) ca = a.A1[(size_t)r * a.len0 + a.o0 + i0];
    }
  };
  auto put_alpha = [&](int ab) {
    if (tid < BK) alphaS[ab][tid] = cr * ca;
  };
  auto store = [&](int sb, int ab) {
#pragma unroll
    for (int g = 0; g < KW / 8; ++g) {
      unsigned pk[NT][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = g * 8 + 2 * q;
        unsigned u0[NT], u1[NT];
        split_fp32<NT>((float)(alphaS[ab][kbw + kk] * w[kk]), u0);
        split_fp32<NT>((float)(alphaS[ab][kbw + kk + 1] * w[kk + 1]), u1);
#pragma unroll
        for (int t = 0; t < NT; ++t) pk[t][q] = pack_hi(u0[t], u1[t]);
      }
      const int slot = ((kbw >> 3) + g) ^ ((mw >> 2) & 3);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        *reinterpret_cast<uint4*>(&Ws[sb][t][mw][slot * 4]) =
            make_uint4(pk[t][0], pk[t][1], pk[t][2], pk[t][3]);
    }
#pragma unroll
    for (int g = 0; g < KY / 8; ++g) {
      unsigned pk[NT][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = g * 8 + 2 * q;
        unsigned u0[NT], u1[NT];
        split_fp32<NT>((float)y[kk], u0);
        split_fp32<NT>((float)y[kk + 1], u1);
#pragma unroll
        for (int t = 0; t < NT; ++t) pk[t][q] = pack_hi(u0[t], u1[t]);
      }
      const int slot = ((kby >> 3) + g) ^ ((ny >> 2) & 3);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        *reinterpret_cast<uint4*>(&Ys[sb][t][ny][slot * 4]) =
            make_uint4(pk[t][0], pk[t][1], pk[t][2], pk[t][3]);
    }
  };

  f4_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f4_t{0, 0, 0, 0};

  // read slot of this lane: rows wr + 16 i + lr all have (row >> 2) & 3 = (lr >> 2) & 3
  const int rslot = (lk ^ ((lr >> 2) & 3)) * 4;

  load_alpha(0);
  put_alpha(0);
  load_alpha(BK);
  load_ops(0);
  __syncthreads();
  for (int c = 0; c < nchunk; ++c) {
    const int sb = (NBUF == 2) ? (c & 1) : 0;
    if (NBUF == 1 && c > 0) __syncthreads();
    store(sb, c & 1);
    put_alpha((c + 1) & 1);
    __syncthreads();
    if (c + 1 < nchunk) load_ops((c + 1) * BK);
    load_alpha((c + 2) * BK);
    s8_t av[NT][FM], bv[NT][FN];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
        av[t][i] = *reinterpret_cast<const s8_t*>(&Ws[sb][t][wr + i * 16 + lr][rslot]);
#pragma unroll
      for (int j = 0; j < FN; ++j)
        bv[t][j] = *reinterpret_cast<const s8_t*>(&Ys[sb][t][wc + j * 16 + lr][rslot]);
    }
    constexpr int NP = (NT == 3) ? 6 : 3;
    constexpr int PA[6] = {1, 2, 0, 1, 0, 0};  // NT = 3 order; NT = 2 uses the last three
    constexpr int PB[6] = {1, 0, 2, 0, 1, 0};
#pragma unroll
    for (int p = 6 - NP; p < 6; ++p)
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf8_t, av[PA[p]][i]), __builtin_bit_cast(bf8_t, bv[PB[p]][j]),
              acc[i][j], 0, 0, 0);
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
#define LS_T(ID, BM_, BN_, WM_, WN_, NB_)                                                     \
  if (tile == ID) {                                                                          \
    if (!dry) {                                                                              \
      fill_tiles(&bs, BM_, BN_);                                                             \
      dim3 grid((unsigned)(8 * bs.per_xcd));                                                 \
      hipLaunchKernelGGL((k_recon_split<NT, BM_, BN_, WM_, WN_, NB_>), grid, block, 0, s, bs, \
                         (float*)out);                                                       \
    }                                                                                        \
    return true;                                                                             \
  }
  LS_T(1, 128, 128, 64, 64, 2)
  LS_T(2, 128, 128, 64, 64, 1)
  LS_T(3, 64, 128, 32, 64, 2)
  LS_T(4, 128, 64, 64, 32, 2)
  LS_T(5, 64, 64, 32, 32, 2)
#undef LS_T
  return false;
}

static int n_tiles(int precision) {
  return precision == LS_F32 ? 8 : 5;
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
// K = 384: FP64 128x64, FP32 128x128 with rank chunk 16, BF16x6 128x128 single
// LDS buffer, BF16x3 128x128 double buffer).
static int auto_tile(int precision, long long M, long long Nc) {
  const long long big = ((M + 127) / 128) * ((Nc + 127) / 128);
  if (big >= 256) {
    switch (precision) {
      case LS_F64: return 3;
      case LS_F32: return 1;
      case LS_BF16X6: return 2;
      default: return 1;
    }
  }
  if (precision == LS_BF16X3 || precision == LS_BF16X6) return big >= 128 ? 4 : 5;
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
