// Split-bf16 GEMM tiles shared by the reconstruction kernels and the batch
// kernel (internal header).
#pragma once

#include "ls_recon_tile.hpp"

namespace ls {

// ---------------------------------------------------------------------------
// split-bf16 kernels
// ---------------------------------------------------------------------------
// Every operand value is rounded once to FP32 and cut into NT bf16 terms.
// NT = 3, by truncation: x0 = x with its low 16 bits cleared, x1 = (x - x0)
// likewise, x2 = x - x0 - x1. Each difference is exact in FP32, and three
// 8-bit bf16 significands hold the whole 24-bit FP32 significand, so
// x0 + x1 + x2 = x.
// NT = 2, by rounding to nearest (even): x0 = bf16(x), x1 = bf16(x - x0), so
// |x - x0| <= 2^-8 |x| and |x - x0 - x1| <= 2^-16 |x| (x - x0 is exact in
// FP32: x0 lies within a factor 2 of x). The dropped product x1 y1 then has
// either sign with equal odds; truncated terms would all share the sign of
// x y and drop a bias of about 2^-16 |x y| in every product.
// Products: x0y0 + x0y1 + x1y0, and for NT = 3 also x1y1 + x0y2 + x2y0, on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation, small terms first.
//
// Staging map: thread t owns operand row m = t % BM and the KW = BM/8
// consecutive ranks from (t / BM) * KW of each 32-rank chunk, so its terms go
// to LDS as packed 16-byte writes (8 ranks: what one MFMA lane reads). One LDS
// row holds the 32 ranks of one operand row (64 bytes), with its 16-byte
// slots permuted by lds_swz.
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
    const unsigned hi = (NT == 2 ? b + 0x7fffu + ((b >> 16) & 1u) : b) & 0xffff0000u;
    u[t] = hi;
    x -= __uint_as_float(hi);
    b = __float_as_uint(x);
  }
  if (NT == 2) b += 0x7fffu + ((b >> 16) & 1u);
  u[NT - 1] = b;  // low half dropped when packed
}

// LDS placement of the split operands: 16-byte slot s of row R sits at slot
// s ^ lds_swz(R). With 64-byte rows this keeps the 16-byte accesses of 16
// consecutive rows (one slot each) free of bank conflicts whether the LDS
// serves 8 or 16 lanes per cycle (32 or 64 banks).
__device__ __forceinline__ int lds_swz(int row) {
  const int r = row & 15;
  return ((r >> 1) ^ (r >> 3)) & 3;
}

// FP16 two-term split of an FP32 value (LS_F16X3, operands pre-scaled below
// 2^14 in magnitude): t0 = x rounded to FP16, t1 = the remainder x - t0 (exact
// in FP32) rounded to FP16, so |x - t0 - t1| <= 2^-22 |x| for normal terms.
// Returned in the high halves of 32-bit words, like split_fp32, so that
// pack_hi applies.
__device__ __forceinline__ void split_f16(float x, unsigned (&u)[2]) {
  // keep x an FP32 register value: the compiler would otherwise merge the
  // caller's double -> float rounding with this float -> FP16 one into a
  // software double -> FP16 conversion (two dozen instructions per value)
  asm("" : "+v"(x));
  const _Float16 h0 = (_Float16)x;
  const _Float16 h1 = (_Float16)(x - (float)h0);
  u[0] = (unsigned)__builtin_bit_cast(unsigned short, h0) << 16;
  u[1] = (unsigned)__builtin_bit_cast(unsigned short, h1) << 16;
}
typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef float fl2_t __attribute__((ext_vector_type(2)));

// split_f16 of two values at once, packed as pack_hi would pack them
// (w[t] = term t of `even` in the low half, of `odd` in the high half): the
// same roundings, on the packed FP32 -> FP16 conversion (two values per
// instruction, no packing step)
__device__ __forceinline__ void split_f16_pair(float even, float odd, unsigned (&w)[2]) {
  fl2_t v = {even, odd};
  asm("" : "+v"(v));  // FP32 register values, as in split_f16
  const h2_t h0 = __builtin_convertvector(v, h2_t);
  const h2_t h1 = __builtin_convertvector(v - __builtin_convertvector(h0, fl2_t), h2_t);
  w[0] = __builtin_bit_cast(unsigned, h0);
  w[1] = __builtin_bit_cast(unsigned, h1);
}

__device__ __forceinline__ unsigned pack_hi(unsigned even, unsigned odd) {
  return (odd & 0xffff0000u) | (even >> 16);
}

// MFMA shape of the split kernels. 16: v_mfma_f32_16x16x32_bf16, lane l
// supplies row l%16 and ranks 8(l/16)..+7 of the 32-rank chunk, receives
// D[4(l/16) + v][l%16], v < 4. 32: v_mfma_f32_32x32x16_bf16 on each half of
// the chunk, lane l supplies row l%32 and ranks 16h + 8(l/32)..+7, receives
// D[8(v/4) + 4(l/32) + v%4][l%32], v < 16. On gfx950 the 32x32 shape issues
// at twice the rate of the 16x16 one.
template <int MF>
struct SplitMma;
template <>
struct SplitMma<16> {
  typedef f4_t acc_t;
  static constexpr int NV = 4;
  static __device__ __forceinline__ int drow(int lane, int v) { return 4 * (lane >> 4) + v; }
  static __device__ __forceinline__ int dcol(int lane) { return lane & 15; }
};
template <>
struct SplitMma<32> {
  typedef f16v_t acc_t;
  static constexpr int NV = 16;
  static __device__ __forceinline__ int drow(int lane, int v) {
    return 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
  }
  static __device__ __forceinline__ int dcol(int lane) { return lane & 31; }
};

// The MFMAs of one 32-rank chunk: term planes W + t*wplane and Y + t*yplane
// (rows of 16 dwords, 16-byte slot s of row R at s ^ lds_swz(R)), A rows
// from arow, B rows from brow. Products x_ta y_tb with ta + tb <= NT - 1; the
// B fragments of all terms stay in registers, the A fragments are read one
// term at a time.
template <int NT, int MF, int FM, int FN>
__device__ __forceinline__ void split_products(typename SplitMma<MF>::acc_t (&acc)[FM][FN],
                                               const unsigned* W, int wplane, const unsigned* Y,
                                               int yplane, int arow, int brow, int lane) {
  constexpr int NH = MF == 16 ? 1 : 2;  // MFMA k-steps per chunk
  const int lr = lane & (MF - 1), lg = lane / MF;
  int slot[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) slot[h] = ((NH * h + lg) ^ lds_swz(lr)) * 4;
  s8_t bv[NT][FN][NH];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int h = 0; h < NH; ++h)
        bv[t][j][h] = *reinterpret_cast<const s8_t*>(Y + t * yplane + (brow + MF * j + lr) * 16 + slot[h]);
#pragma unroll
  for (int ta = NT - 1; ta >= 0; --ta) {
    s8_t av[FM][NH];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int h = 0; h < NH; ++h)
        av[i][h] = *reinterpret_cast<const s8_t*>(W + ta * wplane + (arow + MF * i + lr) * 16 + slot[h]);
#pragma unroll
    for (int tb = NT - 1 - ta; tb >= 0; --tb)
#pragma unroll
      for (int h = 0; h < NH; ++h)
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
          for (int j = 0; j < FN; ++j) {
            if constexpr (MF == 16)
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  __builtin_bit_cast(bf8_t, av[i][h]), __builtin_bit_cast(bf8_t, bv[tb][j][h]),
                  acc[i][j], 0, 0, 0);
            else
              acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  __builtin_bit_cast(bf8_t, av[i][h]), __builtin_bit_cast(bf8_t, bv[tb][j][h]),
                  acc[i][j], 0, 0, 0);
          }
  }
}

// A tile's rows (i, j) lie in the values i0 .. ilast of i. With at most
// kTileNI of them (FAST; with 128-row tiles, every tile of a box with 43 or
// more values of j) the rank factors coef_r f0[r][i] of each of them are
// formed once per rank chunk in LDS and each row reads its own, so staging
// loads only f1, without conditions; otherwise (narrow boxes) each element
// also loads its f0 value, in a loop of its own.
constexpr int kTileNI = 4;

template <int NT, int BM, int BN, int NBUF>
constexpr int split_smem_bytes() {
  return NBUF * NT * (BM + BN) * 16 * 4 + 2 * kTileNI * (SPLIT_BK + 1) * 8;
}

// One BM x BN tile (rows row0.., columns col0..) of the box GEMM with both
// operands split in the kernel; out is the box's output, smem holds
// split_smem_bytes<NT, BM, BN, NBUF>() bytes (16-byte aligned). All 256
// threads of the workgroup call it; it ends with the tile stored.
template <int NT, int BM, int BN, int WM, int WN, int NBUF, int MF, bool FAST>
__device__ __forceinline__ void split_tile_run(const BoxArg& a, int row0, int col0,
                                               float* __restrict__ out, char* smem) {
  constexpr int BK = SPLIT_BK;
  constexpr int KW = BK * BM / 256, KY = BK * BN / 256;
  static_assert(BM >= 64 && BN >= 64 && 256 % BM == 0 && 256 % BN == 0, "staging map");
  static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");
  constexpr int FM = WM / MF, FN = WN / MF;
  typedef SplitMma<MF> Mma;
  typedef unsigned WsT[NT][BM][16];
  typedef unsigned YsT[NT][BN][16];
  WsT* Ws = reinterpret_cast<WsT*>(smem);
  YsT* Ys = reinterpret_cast<YsT*>(smem + NBUF * sizeof(WsT));
  constexpr int NI = kTileNI, AST = BK + 1;  // alphaS row stride: rows of i in other banks
  double (*alphaS)[NI][AST] =
      reinterpret_cast<double (*)[NI][AST]>(smem + NBUF * (sizeof(WsT) + sizeof(YsT)));

  const int M = a.e0 * a.e1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave / (BN / WN)) * WM, wc = (wave % (BN / WN)) * WN;

  // staging ownership (tid / BM and tid / BN are uniform per wave: BM, BN >= 64)
  const int mw = tid % BM, ny = tid % BN;
  const int kbw = __builtin_amdgcn_readfirstlane(tid / BM) * KW;
  const int kby = __builtin_amdgcn_readfirstlane(tid / BN) * KY;
  const int i0 = row0 / a.e1;
  const int ilast = (min(row0 + BM, M) - 1) / a.e1;
  const int m = row0 + mw;
  const bool mok = m < M;
  const int mi = mok ? m / a.e1 : i0;
  const int mj = mok ? m - mi * a.e1 : 0;
  const int islot = FAST ? mi - i0 : 0;  // this row's factors in alphaS
  const double* __restrict__ a1row = a.A1 + a.o0 + mi;
  const double* __restrict__ a2row = a.A2 + a.o1 + mj;
  const int nchunk = (a.K + BK - 1) / BK;
  // f1 (FAST) and f2 through buffer resources: a uniform (scalar) byte offset
  // per rank row and a fixed 32-bit lane offset; rows past K read 0. Columns
  // past the box read its last column (computed, never stored).
  const __amdgpu_buffer_rsrc_t a2buf = uniform_rsrc(a.A2, a.K * a.len1 * 8);
  const __amdgpu_buffer_rsrc_t a3buf = uniform_rsrc(a.A3, a.K * a.len2 * 8);
  const int woff = (a.o1 + mj) * 8;
  const int yoff = (a.o2 + min(col0 + ny, a.e2 - 1)) * 8;
  const int rs1 = __builtin_amdgcn_readfirstlane(a.len1 * 8);  // bytes per rank row
  const int rs2 = __builtin_amdgcn_readfirstlane(a.len2 * 8);

  double w[KW], y[KY];
  double cr = 0.0, ca = 1.0;  // raw parts of one alpha_r (threads tid < NI BK)

  auto load_ops = [&](int k0) {
    if constexpr (FAST) {
      const int s0 = __builtin_amdgcn_readfirstlane((k0 + kbw) * a.len1 * 8);
#pragma unroll
      for (int kk = 0; kk < KW; ++kk)
        w[kk] = __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(a2buf, woff, s0 + kk * rs1, 0));
    } else {
#pragma unroll
      for (int kk = 0; kk < KW; ++kk) {
        const int r = k0 + kbw + kk;
        double v = 0.0;
        if (r < a.K && mok) v = a2row[(size_t)r * a.len1] * a1row[(size_t)r * a.len0];
        w[kk] = v;
      }
    }
    const int s0 = __builtin_amdgcn_readfirstlane((k0 + kby) * a.len2 * 8);
#pragma unroll
    for (int kk = 0; kk < KY; ++kk)
      y[kk] = __builtin_bit_cast(
          double, __builtin_amdgcn_raw_buffer_load_b64(a3buf, yoff, s0 + kk * rs2, 0));
  };
  // thread tid < NI BK: rank k0 + tid % BK and value i0 + tid / BK of i,
  // loaded at clamped indices without conditions; aval says whether the
  // factor is used (else it is written as 0)
  const int ai = tid / BK, ar = tid % BK;
  bool aval = false;
  auto load_alpha = [&](int k0) {
    const int r = k0 + ar;
    aval = ai < NI && r < a.K && (FAST ? i0 + ai <= ilast : ai == 0);
    const int rc = min(r, a.K - 1);
    cr = a.coef[rc];
    if constexpr (FAST) ca = a.A1[(size_t)rc * a.len0 + a.o0 + min(i0 + min(ai, NI - 1), ilast)];
  };
  auto put_alpha = [&](int ab) {
    if (ai < NI) alphaS[ab][ai][ar] = aval ? cr * ca : 0.0;
  };
  auto store = [&](int sb, int ab) {
#pragma unroll
    for (int g = 0; g < KW / 8; ++g) {
      unsigned pk[NT][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = g * 8 + 2 * q;
        unsigned u0[NT], u1[NT];
        split_fp32<NT>((float)(alphaS[ab][islot][kbw + kk] * w[kk]), u0);
        split_fp32<NT>((float)(alphaS[ab][islot][kbw + kk + 1] * w[kk + 1]), u1);
#pragma unroll
        for (int t = 0; t < NT; ++t) pk[t][q] = pack_hi(u0[t], u1[t]);
      }
      const int slot = ((kbw >> 3) + g) ^ lds_swz(mw);
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
      const int slot = ((kby >> 3) + g) ^ lds_swz(ny);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        *reinterpret_cast<uint4*>(&Ys[sb][t][ny][slot * 4]) =
            make_uint4(pk[t][0], pk[t][1], pk[t][2], pk[t][3]);
    }
  };

  typename Mma::acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < Mma::NV; ++v) acc[i][j][v] = 0.0f;


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
    if (FAST || c + 1 < nchunk) load_ops((c + 1) * BK);
    load_alpha((c + 2) * BK);
    split_products<NT, MF, FM, FN>(acc, &Ws[sb][0][0][0], BM * 16, &Ys[sb][0][0][0], BN * 16, wr,
                                   wc, lane);
  }

  const float sc = (float)a.scale;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < Mma::NV; ++v) {
        const int row = row0 + wr + i * MF + Mma::drow(lane, v);
        const int col = col0 + wc + j * MF + Mma::dcol(lane);
        if (row < M && col < a.e2) out[(size_t)row * a.e2 + col] = sc * acc[i][j][v];
      }
}

template <int NT, int BM, int BN, int WM, int WN, int NBUF, int MF>
__device__ __forceinline__ void split_tile(const BoxArg& a, int row0, int col0,
                                           float* __restrict__ out, char* smem) {
  const int M = a.e0 * a.e1;
  const int i0 = row0 / a.e1, ilast = (min(row0 + BM, M) - 1) / a.e1;
  if (ilast - i0 < kTileNI)
    split_tile_run<NT, BM, BN, WM, WN, NBUF, MF, true>(a, row0, col0, out, smem);
  else
    split_tile_run<NT, BM, BN, WM, WN, NBUF, MF, false>(a, row0, col0, out, smem);
}

}  // namespace ls
