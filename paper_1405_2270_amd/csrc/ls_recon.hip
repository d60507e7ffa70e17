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
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <type_traits>
#include <vector>

#include "ls_split_tile.hpp"

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
  const unsigned* P2;                         // pre-split f1 (tiles 6..9 of the split precisions)
  int nch;                                    // rank chunks of 32 in P2
  const double* coefS;                        // LS_F16X3: coef_r 2^(g - 13 + e_r)
  const int* gexp;                            // LS_F16X3: g
  const double* coefS32;                      // LS_F16X3: coefS_r 2^(e2_r)
  const float* f2f;                           // LS_F16X3: f2 2^(-e2_r) rounded to FP32
  // LS_F16X3: rank slot s holds rank perm[s] of the caller's factors (P2,
  // f2f, coefS and coefS32 are in slot order); cmask[x] bit c set when chunk
  // c has a nonzero FP16 term on plane x of axis 0 (null: every chunk runs)
  const int* perm;
  const unsigned* cmask;
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
  recon_tile<T, BM, BN, WM, WN, BK>(uniform_box(bs.box[b]), tm * BM, tn * BN, out + bs.out_off[b],
                                    smem);
}

template <int BM, int BN, int WM, int WN, int BK>
__global__ __launch_bounds__(256) void k_recon32(BoxSet bs, float* __restrict__ out) {
  __shared__ __attribute__((aligned(16))) char smem[recon32_smem_bytes<BM, BN, BK>()];
  int b, tm, tn;
  if (!locate(bs, &b, &tm, &tn)) return;
  recon_tile32<BM, BN, WM, WN, BK>(uniform_box(bs.box[b]), tm * BM, tn * BN, out + bs.out_off[b],
                                   smem);
}

// ---------------------------------------------------------------------------
// split-bf16 kernels (helpers and the in-kernel split tile: ls_split_tile.hpp)
// ---------------------------------------------------------------------------
typedef double d2_t __attribute__((ext_vector_type(2)));

template <int NT, int BM, int BN, int WM, int WN, int NBUF, int MF>
__global__ __launch_bounds__(256) void k_recon_split(BoxSet bs, float* __restrict__ out_all) {
  __shared__ __attribute__((aligned(16))) char smem[split_smem_bytes<NT, BM, BN, NBUF>()];
  int bidx, tmi, tni;
  if (!locate(bs, &bidx, &tmi, &tni)) return;
  split_tile<NT, BM, BN, WM, WN, NBUF, MF>(uniform_box(bs.box[bidx]), tmi * BM, tni * BN,
                                          out_all + bs.out_off[bidx], smem);
}

// ---------------------------------------------------------------------------
// split-bf16 with pre-split f1 (tiles 6..9, workspace)
// ---------------------------------------------------------------------------
// Per i the box is the GEMM out[i][j][k] = sum_r f1[r][o1+j] Y_i[r][k] with
// Y_i[r][k] = alpha_r(i) f2[r][o2+k], alpha_r(i) = coef[r] f0[r][o0+i]. The
// left operand does not depend on i, so f1 is split into bf16 terms once per
// call, into the workspace as P[t][c][x][32]: term t of f1[32c + q][x],
// q = 0..31 (zero beyond K), one 64-byte row per grid cell x and rank chunk c.
// A tile (one i, BM values of j, BN values of k) then copies its left operand
// rows into LDS as they are (16-byte loads and stores, no arithmetic) and
// splits only the BN x 32 values of Y_i per rank chunk.
template <int NT>
__global__ __launch_bounds__(64) void k_presplit(const double* __restrict__ f, int K, int len,
                                                  int nch, unsigned* __restrict__ P) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int c = blockIdx.y;
  if (x >= len) return;
  // all 32 loads first (rank clamped into range, zero beyond K), then the splits
  double v[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const int r = 32 * c + q;
    v[q] = f[(size_t)(r < K ? r : K - 1) * len + x];
  }
  unsigned pk[NT][16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int r0 = 32 * c + 2 * q;
    unsigned u0[NT], u1[NT];
    split_fp32<NT>(r0 < K ? (float)v[2 * q] : 0.0f, u0);
    split_fp32<NT>(r0 + 1 < K ? (float)v[2 * q + 1] : 0.0f, u1);
#pragma unroll
    for (int t = 0; t < NT; ++t) pk[t][q] = pack_hi(u0[t], u1[t]);
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    uint4* dst = reinterpret_cast<uint4*>(P + (((size_t)t * nch + c) * len + x) * 16);
#pragma unroll
    for (int s = 0; s < 4; ++s)
      dst[s] = make_uint4(pk[t][4 * s], pk[t][4 * s + 1], pk[t][4 * s + 2], pk[t][4 * s + 3]);
  }
}

// ---------------------------------------------------------------------------
// LS_F16X3: per-rank power-of-two scaling and two FP16 terms per operand
// ---------------------------------------------------------------------------
// FP16 holds 11 significant bits, so two terms keep 22 bits of an FP32 value
// (products x0y0 + x0y1 + x1y0, error of order 2^-21 |xy|), but only 5 exponent
// bits: the operands are scaled first. Rank r of f1 is multiplied by
// 2^(13 - e_r), e_r = floor(log2 max_x |f1[r][x]|), so its largest term lies in
// [2^13, 2^14); the scale cancels in every product f1[r][j] Y[r][k] when Y
// carries 2^-(13 - e_r). One more power of two, 2^g, lifts every Y value as far
// as the largest allows: g = 13 - floor(log2 B), B = max_r |coef_r| max|f0[r]|
// max|f2[r]| 2^(e_r - 13), so |Y| < 2^14; the output is multiplied by 2^-g.
// Both operands then use the FP16 normal range down to 2^-14 (2^-28 below
// their largest values), and values under 2^-24 of it flush to zero.

__device__ __forceinline__ double block_max256(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// one workgroup per rank and axis: rmax[axis][r] = max_x |f_axis[r][x]|
// (four independent loads per thread in flight)
__global__ __launch_bounds__(256) void k_rank_max(const double* __restrict__ f0,
                                                  const double* __restrict__ f1,
                                                  const double* __restrict__ f2, int K, int len0,
                                                  int len1, int len2, double* __restrict__ rmax) {
  __shared__ double sh[4];
  const int r = blockIdx.x, ax = blockIdx.y;
  const int len = ax == 0 ? len0 : (ax == 1 ? len1 : len2);
  const double* __restrict__ row = (ax == 0 ? f0 : (ax == 1 ? f1 : f2)) + (size_t)r * len;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  int x = threadIdx.x;
  for (; x + 768 < len; x += 1024)
#pragma unroll
    for (int u = 0; u < 4; ++u) m[u] = fmax(m[u], fabs(row[x + 256 * u]));
  for (; x < len; x += 256) m[0] = fmax(m[0], fabs(row[x]));
  const double v = block_max256(fmax(fmax(m[0], m[1]), fmax(m[2], m[3])), sh);
  if (threadIdx.x == 0) rmax[(size_t)ax * K + r] = v;
}

ls_status launch_rank_max(const double* f0, const double* f1, const double* f2, int K, int len0,
                          int len1, int len2, double* rmax, hipStream_t stream) {
  hipLaunchKernelGGL(k_rank_max, dim3(K, 3), dim3(256), 0, stream, f0, f1, f2, K, len0, len1,
                     len2, rmax);
  return launch_status("row maxima");
}

// floor(log2 m) for a row maximum m, 0 for a zero or non-finite row
__device__ __forceinline__ int row_exp(double m) { return (m > 0.0 && isfinite(m)) ? ilogb(m) : 0; }

// Rank order and scales of LS_F16X3 (one workgroup of 512 threads, which fits
// beside other work on a CU), from the
// row maxima rmax = [max|f0[r]|, max|f1[r]|, max|f2[r]|], e_r = row_exp of the
// f1 maximum, e2_r of the f2 maximum. Slot s of the reordered ranks holds rank
// perm[s]: with K <= kOrderRanks the ranks in decreasing max|f0[r]| (ties by
// index), so that terms of similar width, whose f0 vanishes on the same planes,
// share a chunk of 32; otherwise the given order. g from the largest bound
// b_r = |coef_r| max|f0[r]| max|f2[r]| 2^(e_r - 13), then in slot order
// coefS[s] = coef_r 2^(g - 13 + e_r) and coefS32[s] = coefS[s] 2^(e2_r),
// r = perm[s]. Clears the chunk masks (len0 words) when cmask is given.
constexpr int kOrderRanks = 1024;
__global__ __launch_bounds__(512) void k_f16_order(const double* __restrict__ coef,
                                                   const double* __restrict__ rmax, int K,
                                                   int len0, int* __restrict__ perm,
                                                   double* __restrict__ coefS,
                                                   double* __restrict__ coefS32,
                                                   int* __restrict__ gexp,
                                                   unsigned* __restrict__ cmask) {
  __shared__ double key[kOrderRanks];
  __shared__ double red[8];
  const int t = threadIdx.x;
  const double* __restrict__ m1 = rmax + K;
  const double* __restrict__ m2 = rmax + 2 * (size_t)K;
  const bool order = K <= kOrderRanks;
  if (order)
    for (int r = t; r < K; r += 512) key[r] = isfinite(rmax[r]) ? rmax[r] : 0.0;
  double m = 0.0;
  for (int r = t; r < K; r += 512)
    m = fmax(m, fabs(coef[r]) * rmax[r] * m2[r] * ldexp(1.0, row_exp(m1[r]) - 13));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((t & 63) == 0) red[t >> 6] = m;
  __syncthreads();
  m = red[0];
  for (int w = 1; w < 8; ++w) m = fmax(m, red[w]);
  const int g = (m > 0.0 && isfinite(m)) ? 13 - ilogb(m) : 0;
  for (int r = t; r < K; r += 512) {
    // the rank's values, requested before the ranking runs
    const double cr = coef[r], mr1 = m1[r], mr2 = m2[r];
    int s = r;
    if (order) {
      // the rank's place in the order: the ranks before it
      // (sixteen LDS reads in flight per step, and the tests combined with
      // bitwise operators: short-circuit ones become a branch per test)
      const double k = key[r];
      s = 0;
      int q = 0;
      for (; q + 16 <= K; q += 16) {
        double kq[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) kq[u] = key[q + u];
#pragma unroll
        for (int u = 0; u < 16; ++u) s += (int)(kq[u] > k) | ((int)(kq[u] == k) & (int)(q + u < r));
      }
      for (; q < K; ++q) s += (int)(key[q] > k) | ((int)(key[q] == k) & (int)(q < r));
    }
    const double cs = cr * ldexp(1.0, g - 13 + row_exp(mr1));
    perm[s] = r;
    coefS[s] = cs;
    coefS32[s] = ldexp(cs, row_exp(mr2));
  }
  if (t == 0) *gexp = g;
  if (cmask != nullptr)
    for (int x = t; x < len0; x += 512) cmask[x] = 0u;
}

// After k_f16_order, in slot order (r = perm[s]): blockIdx.y < nch: as
// k_presplit<2>, with rank r of f1 scaled by 2^(13 - e_r) and FP16 terms;
// nch <= y < nch + n8: slots 8 (y - nch) .. +7 of f2 scaled by 2^-e2_r and
// rounded to FP32 (the FP16 split of the other operand keeps 22 bits; f2 in
// FP32 halves the bytes the kernel loads for it); nch + n8 <= y (with cmask):
// the chunk c = y - nch - n8 of every plane x of axis 0 is marked in cmask[x]
// unless |coefS32[s] f0[r][x]| <= 2^-27 for each of its 32 slots. The
// reconstruction forms the same FP64 product as its rank factor; times the
// FP32 copy of f2 (below 2 in magnitude) it gives at most 2^-26, and so does
// the FP64-f2 tiles' product (their rank factor carries 2^-e2_r, their f2 is
// below 2^(e2_r + 1)); that is under half the smallest FP16 subnormal, so both
// FP16 terms round to zero, an unmarked chunk adds only zeros to the plane's
// outputs, and it is skipped without changing a bit.
__global__ __launch_bounds__(64) void k_prep_f16(const double* __restrict__ f,
                                                 const double* __restrict__ f2,
                                                 const double* __restrict__ f0,
                                                 const double* __restrict__ rmax,
                                                 const int* __restrict__ perm,
                                                 const double* __restrict__ coefS32, int K,
                                                 int len0, int len, int len2, int nch, int n8,
                                                 unsigned* __restrict__ P, float* __restrict__ f2f,
                                                 unsigned* __restrict__ cmask) {
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int c = blockIdx.y;
  const double* __restrict__ m1 = rmax + K;
  const double* __restrict__ m2 = rmax + 2 * (size_t)K;
  if (c >= nch + n8) {
    if (x >= len0) return;
    const int cc = c - nch - n8;
    // all 32 loads in flight, then the tests
    double a[32];
#pragma unroll
    for (int q = 0; q < 32; ++q) {
      const int sl = min(32 * cc + q, K - 1);
      a[q] = f0[(size_t)perm[sl] * len0 + x];
    }
    int act = 0;
#pragma unroll
    for (int q = 0; q < 32; ++q)
      act |= (int)(32 * cc + q < K) & (int)!(fabs(coefS32[min(32 * cc + q, K - 1)] * a[q]) <= 0x1p-27);
    if (act) atomicOr(&cmask[x], 1u << cc);
    return;
  }
  if (c >= nch) {
    if (x >= len2) return;
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = f2[(size_t)perm[min(8 * (c - nch) + q, K - 1)] * len2 + x];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int sl = 8 * (c - nch) + q;
      if (sl < K) f2f[(size_t)sl * len2 + x] = (float)ldexp(v[q], -row_exp(m2[perm[sl]]));
    }
    return;
  }
  if (x >= len) return;
  double v[32];
#pragma unroll
  for (int q = 0; q < 32; ++q) v[q] = f[(size_t)perm[min(32 * c + q, K - 1)] * len + x];
  unsigned pk[2][16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int s0 = 32 * c + 2 * q;
    unsigned u0[2], u1[2];
    split_f16(s0 < K ? (float)ldexp(v[2 * q], 13 - row_exp(m1[perm[min(s0, K - 1)]])) : 0.0f, u0);
    split_f16(s0 + 1 < K ? (float)ldexp(v[2 * q + 1], 13 - row_exp(m1[perm[min(s0 + 1, K - 1)]])) : 0.0f, u1);
#pragma unroll
    for (int t = 0; t < 2; ++t) pk[t][q] = pack_hi(u0[t], u1[t]);
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    uint4* dst = reinterpret_cast<uint4*>(P + (((size_t)t * nch + c) * len + x) * 16);
#pragma unroll
    for (int s = 0; s < 4; ++s)
      dst[s] = make_uint4(pk[t][4 * s], pk[t][4 * s + 1], pk[t][4 * s + 2], pk[t][4 * s + 3]);
  }
}

template <int NT, int BM, int BN, int WM, int WN, int NBUF, int MF>
__global__ __launch_bounds__(256, 2) void k_recon_presplit(BoxSet bs, float* __restrict__ out_all) {
  constexpr int BK = SPLIT_BK;
  constexpr int KY = BK * BN / 256;
  constexpr int PW = NT * BM * 4 / 256;  // 16-byte pieces of the left operand per thread
  static_assert(BN >= 64 && 256 % BN == 0 && (NT * BM * 4) % 256 == 0, "staging map");
  static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");
  constexpr int FM = WM / MF, FN = WN / MF;
  typedef SplitMma<MF> Mma;
  __shared__ __attribute__((aligned(16))) unsigned Ws[NBUF][NT][BM][16];
  __shared__ __attribute__((aligned(16))) unsigned Ys[NBUF][NT][BN][16];
  __shared__ double alphaS[2][BK];

  int bidx, tmi, tni;
  if (!locate(bs, &bidx, &tmi, &tni)) return;
  const BoxArg a = uniform_box(bs.box[bidx]);
  float* __restrict__ out = out_all + bs.out_off[bidx];
  const int jtn = (a.e1 + BM - 1) / BM;
  const int ib = tmi / jtn;
  const int j0 = (tmi - ib * jtn) * BM;
  const int col0 = tni * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave / (BN / WN)) * WM, wc = (wave % (BN / WN)) * WN;
  const int nch = rfl(bs.nch);
  const unsigned* __restrict__ P = bs.P2;

  const int ny = tid % BN;
  const int kby = __builtin_amdgcn_readfirstlane(tid / BN) * KY;
  const bool nok = col0 + ny < a.e2;
  const double* __restrict__ a3row = a.A3 + a.o2 + col0 + ny;
  const double* __restrict__ a1col = a.A1 + a.o0 + ib;
  const int nchunk = (a.K + BK - 1) / BK;

  uint4 wv[PW];
  double y[KY];
  double cr = 0.0, ca = 1.0;

  auto load_ops = [&](int c) {
#pragma unroll
    for (int e = 0; e < PW; ++e) {
      const int id = tid + 256 * e;
      const int slot = id & 3, row = (id >> 2) % BM, t = (id >> 2) / BM;
      uint4 v = make_uint4(0u, 0u, 0u, 0u);
      if (j0 + row < a.e1)
        v = *reinterpret_cast<const uint4*>(
            P + (((size_t)t * nch + c) * a.len1 + a.o1 + j0 + row) * 16 + slot * 4);
      wv[e] = v;
    }
#pragma unroll
    for (int kk = 0; kk < KY; ++kk) {
      const int r = c * BK + kby + kk;
      y[kk] = (r < a.K && nok) ? a3row[(size_t)r * a.len2] : 0.0;
    }
  };
  auto load_alpha = [&](int k0) {
    const int r = k0 + tid;
    cr = 0.0;
    ca = 1.0;
    if (tid < BK && r < a.K) {
      cr = a.coef[r];
      ca = a1col[(size_t)r * a.len0];
    }
  };
  auto put_alpha = [&](int ab) {
    if (tid < BK) alphaS[ab][tid] = cr * ca;
  };
  auto store = [&](int sb, int ab) {
#pragma unroll
    for (int e = 0; e < PW; ++e) {
      const int id = tid + 256 * e;
      const int slot = id & 3, row = (id >> 2) % BM, t = (id >> 2) / BM;
      *reinterpret_cast<uint4*>(&Ws[sb][t][row][(slot ^ lds_swz(row)) * 4]) = wv[e];
    }
#pragma unroll
    for (int g = 0; g < KY / 8; ++g) {
      unsigned pk[NT][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = g * 8 + 2 * q;
        unsigned u0[NT], u1[NT];
        split_fp32<NT>((float)(alphaS[ab][kby + kk] * y[kk]), u0);
        split_fp32<NT>((float)(alphaS[ab][kby + kk + 1] * y[kk + 1]), u1);
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
    if (c + 1 < nchunk) load_ops(c + 1);
    load_alpha((c + 2) * BK);
    split_products<NT, MF, FM, FN>(acc, &Ws[sb][0][0][0], BM * 16, &Ys[sb][0][0][0], BN * 16, wr,
                                   wc, lane);
  }

  const float sc = (float)a.scale;
  const size_t base = (size_t)ib * a.e1;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < Mma::NV; ++v) {
        const int jj = j0 + wr + i * MF + Mma::drow(lane, v);
        const int col = col0 + wc + j * MF + Mma::dcol(lane);
        if (jj < a.e1 && col < a.e2) out[(base + jj) * a.e2 + col] = sc * acc[i][j][v];
      }
}

// Pre-split f1, BM = 256 rows of j per tile with the four waves stacked along
// j (each wave 64 x BN): no two waves share a left-operand row, so each wave
// loads its bf16 fragments straight from the pre-split planes into registers
// (16-byte loads of consecutive 64-byte rows) and only the shared Y_i operand
// goes through LDS. The fragments of term t for the next chunk are loaded as
// soon as the MFMAs of this chunk are done with term t.
// PIPE = 0: per chunk, write the chunk to LDS, one barrier, then its MFMAs.
// PIPE = 1: software pipelined, the MFMAs of chunk c run while the same wave
// splits and writes chunk c+1 into the other LDS buffer (one barrier per
// chunk).
template <int NT, int BN, int MF, int PIPE>
__global__ __launch_bounds__(256, 2) void k_recon_direct(BoxSet bs, float* __restrict__ out_all) {
  constexpr int BM = 256, WM = 64, WN = BN;
  constexpr int BK = SPLIT_BK;
  constexpr int KY = BK * BN / 256;
  constexpr int FM = WM / MF, FN = WN / MF, NH = MF == 16 ? 1 : 2;
  static_assert(BN == 64, "four waves stacked along j, one column block of 64");
  typedef SplitMma<MF> Mma;
  // Y_i in LDS in fragment order: the 16-byte piece that lane l supplies for
  // term t, column block j and MFMA k-step h sits at ((t*FN + j)*NH + h)*64 + l,
  // so each fragment read is one contiguous 1 KB
  __shared__ uint4 Ysf[2][NT * FN * NH * 64];
  // rank factors of one chunk; the pipelined variants let every thread write
  // its slot (those past BK hold zeros) so that no branch splits the chunk's
  // instruction stream
  __shared__ double alphaS[2][PIPE ? 256 : BK];

  int bidx, tmi, tni;
  if (!locate(bs, &bidx, &tmi, &tni)) return;
  const BoxArg a = uniform_box(bs.box[bidx]);
  float* __restrict__ out = out_all + bs.out_off[bidx];
  const int jtn = (a.e1 + BM - 1) / BM;
  const int ib = tmi / jtn;
  const int j0 = (tmi - ib * jtn) * BM;
  const int col0 = tni * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave * WM;
  const int lr = lane & (MF - 1), lg = lane / MF;
  const int nch = rfl(bs.nch);
  const unsigned* __restrict__ P = bs.P2;

  const int ny = tid % BN;
  const int kby = __builtin_amdgcn_readfirstlane(tid / BN) * KY;
  const bool nok = col0 + ny < a.e2;
  const double* __restrict__ a1col = a.A1 + a.o0 + ib;
  const int nchunk = (a.K + BK - 1) / BK;

  // this lane's left-operand rows and their byte offsets in one term plane
  bool rok[FM];
  unsigned roff[FM];  // bytes
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    const int jj = j0 + wr + MF * i + lr;
    rok[i] = jj < a.e1;
    roff[i] = (unsigned)(a.o1 + (rok[i] ? jj : 0)) * 64u;
  }
  const size_t plane = (size_t)a.len1 * 64;  // bytes per rank chunk of one term
  // Global addresses are a wave-uniform base plus a 32-bit per-lane byte
  // offset (one SGPR pair and one VGPR per load).

  // Every load below is unconditional, at an address clamped into range, and
  // its raw value is kept until it is consumed: a load under a branch, or a
  // value used right after its load, would make the wave wait for memory
  // there. Left-operand rows past e1 read row o1 instead; their products land
  // in output rows that are never stored. f2 values and rank factors past K or
  // outside the box are zeroed when they are written to LDS.
  s8_t av[NT][FM][NH];
  auto load_a = [&](int t, int c) {
    const char* base = reinterpret_cast<const char*>(P) + ((size_t)t * nch + c) * plane;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int h = 0; h < NH; ++h)
        av[t][i][h] = *reinterpret_cast<const s8_t*>(base + (roff[i] + (NH * h + lg) * 16));
  };
  double y[KY];
  double cr = 0.0, ca = 1.0;
  bool aok = false;
  const int ycol = min(col0 + ny, a.e2 - 1);  // clamped column
  const char* __restrict__ a3c = reinterpret_cast<const char*>(a.A3 + a.o2);
  const unsigned yoff = (unsigned)ycol * 8u;
  auto load_y = [&](int c) {
#pragma unroll
    for (int kk = 0; kk < KY; ++kk) {
      const int r = c * BK + kby + kk;
      y[kk] = *reinterpret_cast<const double*>(a3c + (size_t)min(r, a.K - 1) * a.len2 * 8 + yoff);
    }
  };
  auto load_alpha = [&](int k0) {
    const int r = min(k0 + min(tid, BK - 1), a.K - 1);
    cr = a.coef[r];
    ca = a1col[(size_t)r * a.len0];
    aok = tid < BK && k0 + tid < a.K;
  };
  auto put_alpha = [&](int ab) {
    if constexpr (PIPE)
      alphaS[ab][tid] = aok ? cr * ca : 0.0;
    else if (tid < BK)
      alphaS[ab][tid] = aok ? cr * ca : 0.0;
  };
  auto store_y = [&](const double (&yv)[KY], int yb, int ab, int c) {
#pragma unroll
    for (int g = 0; g < KY / 8; ++g) {
      unsigned pk[NT][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = g * 8 + 2 * q;
        unsigned u0[NT], u1[NT];
        const int r = c * BK + kby + kk;
        const double m0 = (r < a.K && nok) ? 1.0 : 0.0;
        const double m1 = (r + 1 < a.K && nok) ? 1.0 : 0.0;
        split_fp32<NT>((float)(alphaS[ab][kby + kk] * (yv[kk] * m0)), u0);
        split_fp32<NT>((float)(alphaS[ab][kby + kk + 1] * (yv[kk + 1] * m1)), u1);
#pragma unroll
        for (int t = 0; t < NT; ++t) pk[t][q] = pack_hi(u0[t], u1[t]);
      }
      // rank slot s (8 ranks) of column ny: k-step h = s / (64/MF), lane group s % (64/MF)
      const int sl = (kby >> 3) + g;
      const int hh = sl / (64 / MF), lgw = sl % (64 / MF);
      const int piece = ((ny / MF) * NH + hh) * 64 + lgw * MF + (ny % MF);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        Ysf[yb][t * FN * NH * 64 + piece] = make_uint4(pk[t][0], pk[t][1], pk[t][2], pk[t][3]);
    }
  };

  typename Mma::acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < Mma::NV; ++v) acc[i][j][v] = 0.0f;

  if constexpr (!PIPE) {
    load_alpha(0);
    put_alpha(0);
    load_alpha(BK);
    load_y(0);
  #pragma unroll
    for (int t = 0; t < NT; ++t) load_a(t, 0);
    __syncthreads();
    // Y_i double-buffered: one barrier per chunk. Buffer c&1 is rewritten at
    // chunk c+2, after every wave has passed the barrier of chunk c+1, i.e.
    // finished its MFMAs of chunk c.
    for (int c = 0; c < nchunk; ++c) {
      const int yb = c & 1;
      store_y(y, yb, c & 1, c);
      put_alpha((c + 1) & 1);
      __syncthreads();
      const int cn = min(c + 1, nchunk - 1);  // the last chunk reloads itself (no branch)
      load_y(cn);
      load_alpha((c + 2) * BK);
      s8_t bv[NT][FN][NH];
  #pragma unroll
      for (int t = 0; t < NT; ++t)
  #pragma unroll
        for (int j = 0; j < FN; ++j)
  #pragma unroll
          for (int h = 0; h < NH; ++h)
            bv[t][j][h] = __builtin_bit_cast(s8_t, Ysf[yb][((t * FN + j) * NH + h) * 64 + lane]);
  #pragma unroll
      for (int ta = NT - 1; ta >= 0; --ta) {
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
                      __builtin_bit_cast(bf8_t, av[ta][i][h]), __builtin_bit_cast(bf8_t, bv[tb][j][h]),
                      acc[i][j], 0, 0, 0);
                else
                  acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                      __builtin_bit_cast(bf8_t, av[ta][i][h]), __builtin_bit_cast(bf8_t, bv[tb][j][h]),
                      acc[i][j], 0, 0, 0);
              }
        load_a(ta, cn);
      }
    }

  } else {
    // Chunk m's rank factors live in alphaS[m & 1] and its split f2 values in
    // Ysf[m & 1]. In the step of chunk c every wave loads the raw f2 values of
    // chunk c+2 and the rank factors of chunk c+3 into one register set,
    // reads Ysf[c & 1] for the MFMAs, writes chunk c+1 (raw values loaded one
    // step earlier, in the other set) into Ysf[(c+1) & 1], last read in the
    // step of chunk c-1, before the barrier that ends it, and the factors of
    // chunk c+2 into alphaS[c & 1], last read when chunk c was written. Every
    // load thus has a full step to arrive. Indices past the last chunk are
    // clamped: those writes go to a buffer that is never read again.
    double yr[2][KY], al[2][2];
    auto ld_y = [&](double (&yv)[KY], int c) {
#pragma unroll
      for (int kk = 0; kk < KY; ++kk) {
        const int r = c * BK + kby + kk;
        yv[kk] = *reinterpret_cast<const double*>(a3c + (size_t)min(r, a.K - 1) * a.len2 * 8 + yoff);
      }
    };
    auto ld_al = [&](double (&v)[2], int k0) {
      const int r = min(k0 + min(tid, BK - 1), a.K - 1);
      v[0] = a.coef[r];
      v[1] = a1col[(size_t)r * a.len0];
    };
    auto pt_al = [&](int ab, const double (&v)[2], int k0) {
      alphaS[ab][tid] = (tid < BK && k0 + tid < a.K) ? v[0] * v[1] : 0.0;
    };
    auto step = [&](int c, const double (&ys)[KY], double (&yl)[KY], const double (&as)[2],
                    double (&aload)[2]) {
      const int yb = c & 1;
      const int cn = min(c + 1, nchunk - 1);
      ld_y(yl, min(c + 2, nchunk - 1));
      ld_al(aload, (c + 3) * BK);
      s8_t bv[NT][FN][NH];
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int h = 0; h < NH; ++h)
            bv[t][j][h] = __builtin_bit_cast(s8_t, Ysf[yb][((t * FN + j) * NH + h) * 64 + lane]);
#pragma unroll
      for (int ta = NT - 1; ta >= 0; --ta) {
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
                      __builtin_bit_cast(bf8_t, av[ta][i][h]), __builtin_bit_cast(bf8_t, bv[tb][j][h]),
                      acc[i][j], 0, 0, 0);
                else
                  acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                      __builtin_bit_cast(bf8_t, av[ta][i][h]), __builtin_bit_cast(bf8_t, bv[tb][j][h]),
                      acc[i][j], 0, 0, 0);
              }
        load_a(ta, cn);
      }
      store_y(ys, yb ^ 1, yb ^ 1, cn);
      pt_al(yb, as, (c + 2) * BK);
      __syncthreads();
    };

    ld_al(al[0], 0);
    ld_y(yr[0], 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) load_a(t, 0);
    pt_al(0, al[0], 0);
    ld_al(al[1], BK);
    __syncthreads();
    store_y(yr[0], 0, 0, 0);
    pt_al(1, al[1], BK);
    ld_y(yr[0], min(1, nchunk - 1));
    ld_al(al[0], 2 * BK);
    __syncthreads();
    for (int c = 0; c < nchunk; c += 2) {
      step(c, yr[0], yr[1], al[0], al[1]);
      if (c + 1 < nchunk) step(c + 1, yr[1], yr[0], al[1], al[0]);
    }
  }
  const float sc = (float)a.scale;
  const size_t obase = (size_t)ib * a.e1;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < Mma::NV; ++v) {
        const int jj = j0 + wr + i * MF + Mma::drow(lane, v);
        const int col = col0 + j * MF + Mma::dcol(lane);
        if (jj < a.e1 && col < a.e2) out[(obase + jj) * a.e2 + col] = sc * acc[i][j][v];
      }
}

// ---------------------------------------------------------------------------
// persistent split-bf16 kernel
// ---------------------------------------------------------------------------
// One workgroup per resident slot. The workgroups of one XCD share that
// XCD's range of tiles (numbered as in fill_tiles with per-i row tiles):
// workgroup l of nbx takes tiles l, l + nbx, l + 2 nbx, ... of the range, so
// at any time the XCD works on neighbouring tiles, which read the same f1 and
// f2 slices from its L2. A workgroup walks its tiles as one stream of steps,
// step s being rank chunk s % nchunk of its tile s / nchunk (with chunk
// masks, only the chunks marked for the tile's plane of axis 0, in order),
// and runs the pipeline of the direct kernel (PIPE = 1) over the whole
// stream: the split
// of step s+1 and the loads of steps s+2 and s+3 overlap the MFMAs of step s
// also across tile boundaries, so a tile starts without waiting for memory,
// and its results are stored (non-temporal) while the stream goes on.
struct StreamPos {
  int c;       // rank chunk
  unsigned m;  // with chunk masks: the chunks of the tile's plane
  int g;       // tile number
  int ib, j0, col0;
  int o0, o1, o2, e1, e2;
  long long ooff;  // element offset of the tile's box in the output
};

template <int BN>
__device__ __forceinline__ void stream_tile(const BoxSet& bs, int g, StreamPos& p) {
  int i = 0;
  while (i + 1 < bs.nbox && bs.tile_start[i + 1] <= g) ++i;
  const BoxArg& a = bs.box[i];
  const int local = g - (int)bs.tile_start[i];
  const int tn = bs.tiles_n[i];
  const int tmi = local / tn;
  const int jtn = (a.e1 + 255) / 256;
  const int ib = tmi / jtn;
  p.g = g;
  p.ib = rfl(ib);
  p.j0 = rfl((tmi - ib * jtn) * 256);
  p.col0 = rfl((local - tmi * tn) * BN);
  p.o0 = rfl(a.o0);
  p.o1 = rfl(a.o1);
  p.o2 = rfl(a.o2);
  p.e1 = rfl(a.e1);
  p.e2 = rfl(a.e2);
  p.ooff = bs.out_off[i];
  // the chunks marked for the plane, or chunk 0 alone when none is (its terms
  // are then all zero, and so are the tile's outputs)
  if (bs.cmask != nullptr) {
    const unsigned m = (unsigned)rfl((int)bs.cmask[p.o0 + p.ib]);
    p.m = m ? m : 1u;
  }
}

// chunks of p's tile after chunk p.c (with chunk masks)
__device__ __forceinline__ unsigned chunks_after(const StreamPos& p) {
  return p.m & ~((2u << p.c) - 1u);
}

// position of the step after p (the caller keeps p at the stream's last step)
template <int BN>
__device__ __forceinline__ void stream_next(const BoxSet& bs, StreamPos& p, int nchunk, int nbx) {
  if (bs.cmask != nullptr) {
    const unsigned rest = chunks_after(p);
    if (rest != 0u) {
      p.c = __builtin_ctz(rest);
    } else {
      stream_tile<BN>(bs, p.g + nbx, p);
      p.c = __builtin_ctz(p.m);
    }
    return;
  }
  if (p.c + 1 < nchunk) {
    p.c += 1;
  } else {
    p.c = 0;
    stream_tile<BN>(bs, p.g + nbx, p);
  }
}

// FMT = 0: bf16 terms (split_fp32); FMT = 1: LS_F16X3, two FP16 terms of
// operands pre-scaled by powers of two (the rank factors come from bs.coefS,
// or bs.coefS32 with the FP32 copy of f2 (YV = 3), which carry the scales of
// both operands; the output is scaled by 2^-g).
// OPT bit 0: the rank factors are loaded and written to LDS by wave 0 alone
// (the other waves issue no load for them: fewer vector-memory instructions).
// OPT bit 2: tiles of 128 columns (FP16x3 with the FP32 copy of f2): each
// wave computes 64 x 128 outputs, so every f1 fragment it loads
// serves twice the columns; the f2 fragments are read from LDS per column
// fragment inside the MFMA loop to bound the live registers.
// OPT bit 4 (FP32 f2): each 64-slot fragment of the split f2 in LDS is
// followed by one unused 16-byte slot, so the 32-bit words one write
// instruction stores (four columns apart) fall in distinct banks; a fragment
// is still read as 64 consecutive slots.
template <int NT, int MF, int YV = 2, int FMT = 0, int OPT = 0>
__global__ __launch_bounds__(256, 2) void k_recon_stream(BoxSet bs, int nbx,
                                                         float* __restrict__ out_all) {
  static_assert(FMT == 0 || NT == 2, "FP16 operands have two terms");
  static_assert(YV != 3 || FMT == 1, "the FP32 copy of f2 exists for LS_F16X3");
  // raw f2 values held in registers: FP64, or FP32 with YV = 3
  typedef typename std::conditional<YV == 3, float, double>::type yt;
  constexpr int BM = 256, BN = (OPT & 4) ? 128 : 64, WM = 64, WN = BN;
  // raw f2 values are loaded one step ahead with wide tiles (one register
  // set; the step's MFMAs cover the latency), two steps ahead otherwise
  constexpr bool SH = BN == 128;
  static_assert(BN == 64 || (FMT == 1 && YV == 3), "wide tiles: FP16x3 with the FP32 copy of f2");
  constexpr int BK = SPLIT_BK;
  constexpr int KY = BK * BN / 256;
  constexpr int FM = WM / MF, FN = WN / MF, NH = MF == 16 ? 1 : 2;
  typedef SplitMma<MF> Mma;
  // Ysf and alphaS as in k_recon_direct: step m's split f2 values in Ysf[m & 1]
  // (fragment order) and its rank factors in alphaS[m & 1]
  constexpr int YP = (OPT & 16) ? 65 : 64;  // LDS slots per f2 fragment
  static_assert(YP == 64 || YV == 3, "padded fragments with the FP32 copy of f2");
  __shared__ uint4 Ysf[2][NT * FN * NH * YP];
  __shared__ double alphaS[2][256];

  // this workgroup's tiles: first, first + nbx, ... below lim
  const int xcd = blockIdx.x & 7, l = blockIdx.x >> 3;
  const int per = (int)bs.per_xcd;
  const int total = (int)bs.tile_start[bs.nbox];
  const int lim = min(per, total - xcd * per);
  if (l >= lim) return;
  const int ntile = (lim - l + nbx - 1) / nbx;

  const BoxArg a = uniform_box(bs.box[0]);  // factor pointers, K and lengths are common
  const int K = a.K, len0 = a.len0, len2 = a.len2;
  const int nchunk = (K + BK - 1) / BK;
  // steps of the stream: every chunk of every tile, or the marked ones
  int S = ntile * nchunk;
  if (bs.cmask != nullptr) {
    S = 0;
    for (int t = 0; t < ntile; ++t) {
      StreamPos q;
      stream_tile<BN>(bs, xcd * per + l + t * nbx, q);
      S += __builtin_popcount(q.m);
    }
  }
  const int nch = rfl(bs.nch);
  const int plane = a.len1 * 64;  // bytes per rank chunk of one term
  // f2 and the pre-split f1 are read through buffer resources: a uniform
  // (SGPR) byte offset for the rank row and a 32-bit per-lane offset, so no
  // per-lane 64-bit address arithmetic (the host keeps both below 2 GB)
  const __amdgpu_buffer_rsrc_t ybuf = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(a.A3), (short)0, K * len2 * 8, kBufferFlags);
  const __amdgpu_buffer_rsrc_t y32buf = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(bs.f2f), (short)0, YV == 3 ? K * len2 * 4 : 0, kBufferFlags);
  const __amdgpu_buffer_rsrc_t pbuf = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<unsigned*>(bs.P2), (short)0, (int)(NT * nch * plane), kBufferFlags);
  const double* __restrict__ A1 = a.A1;
  const double* __restrict__ coef = FMT ? (YV == 3 ? bs.coefS32 : bs.coefS) : a.coef;
  // LS_F16X3: the caller's rank of each slot, for the reads of f0 and the FP64 f2
  const int* __restrict__ perm = bs.perm;
  const float sc = FMT ? (float)(a.scale * ldexp(1.0, -rfl(*bs.gexp))) : (float)a.scale;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave * WM;
  const int lr = lane & (MF - 1), lg = lane / MF;
  const int ny = tid % BN;
  const int kby = __builtin_amdgcn_readfirstlane(tid / BN) * KY;

  // Loads are unconditional at clamped addresses and their raw values are
  // kept until use, as in k_recon_direct; rows past e1 read row o1, and f2
  // values and rank factors outside the box or past K are zeroed when written
  // to LDS.
  s8_t av[NT][FM][NH];
  auto load_a = [&](int t, const StreamPos& p) {
    const int soff = (t * nch + p.c) * plane;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const int jj = p.j0 + wr + MF * i + lr;
      const int off = (p.o1 + (jj < p.e1 ? jj : 0)) * 64;
#pragma unroll
      for (int h = 0; h < NH; ++h)
        av[t][i][h] = __builtin_bit_cast(
            s8_t, __builtin_amdgcn_raw_buffer_load_b128(pbuf, off + (NH * h + lg) * 16, soff, 0));
    }
  };
  // f2 staging, YV = 2: lane l of wave w reads columns 2(l%32), 2(l%32)+1
  // of ranks 8w + 4(l/32) .. +3 with 16-byte loads (four per chunk; the
  // second column past e2, or past the end of f2, is never used). YV = 1:
  // thread t reads column t%64 of ranks 8(t/64) .. +7 (eight 8-byte loads).
  const int yp = tid & 31, yh = (tid >> 5) & 1;
  // YV = 3: lane l of wave w reads FP32 columns 64 hc + 4(l%16) .. +3 of
  // ranks 8w + 2(l/16) and the next (two 16-byte loads per 64 columns) and
  // writes one 32-bit word (a rank pair) per column and term
  const int cg = lane & 15, yq = lane >> 4;
  const int kw = __builtin_amdgcn_readfirstlane(wave) * 8;
  constexpr int NHC = BN / 64;
  auto ld_y = [&](yt (&yv)[KY], const StreamPos& p) {
    if constexpr (YV == 3) {
#pragma unroll
      for (int hc = 0; hc < NHC; ++hc) {
        const int cb = (p.o2 + min(p.col0 + 64 * hc + 4 * cg, p.e2 - 1)) * 4;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int r = min(p.c * BK + kw + 2 * yq + e, K - 1);
          const f4_t v = __builtin_bit_cast(f4_t, __builtin_amdgcn_raw_buffer_load_b128(y32buf, r * len2 * 4 + cb, 0, 0));
#pragma unroll
          for (int q = 0; q < 4; ++q) yv[8 * hc + 4 * e + q] = v[q];
        }
      }
    } else if constexpr (YV == 2) {
      const int cb = (p.o2 + min(p.col0 + 2 * yp, p.e2 - 1)) * 8;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const int r = FMT ? perm[min(p.c * BK + kby + 4 * yh + kk, K - 1)]
                          : min(p.c * BK + kby + 4 * yh + kk, K - 1);
        const d2_t v = __builtin_bit_cast(d2_t, __builtin_amdgcn_raw_buffer_load_b128(ybuf, r * len2 * 8 + cb, 0, 0));
        yv[2 * kk] = v[0];
        yv[2 * kk + 1] = v[1];
      }
    } else {
      const int yoff = (p.o2 + min(p.col0 + ny, p.e2 - 1)) * 8;
#pragma unroll
      for (int kk = 0; kk < KY; ++kk) {
        const int r = FMT ? perm[min(p.c * BK + kby + kk, K - 1)] : min(p.c * BK + kby + kk, K - 1);
        yv[kk] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(ybuf, yoff, r * len2 * 8, 0));
      }
    }
  };
  const bool wave0 = __builtin_amdgcn_readfirstlane(wave) == 0;
  auto ld_al = [&](double (&v)[2], const StreamPos& p) {
    if (!(OPT & 1) || wave0) {
      const int r = min(p.c * BK + min(tid, BK - 1), K - 1);
      v[0] = coef[r];
      v[1] = A1[(size_t)(p.o0 + p.ib) + (size_t)(FMT ? perm[r] : r) * len0];
    }
  };
  auto pt_al = [&](int ab, const double (&v)[2], const StreamPos& p) {
    if (!(OPT & 1) || wave0) alphaS[ab][tid] = (tid < BK && p.c * BK + tid < K) ? v[0] * v[1] : 0.0;
  };
  auto split_val = [](float x, unsigned (&u)[NT]) {
    if constexpr (FMT == 1)
      split_f16(x, u);
    else
      split_fp32<NT>(x, u);
  };
  // No masks here: ranks past K have zero rank factors (and zero pre-split
  // f1), and the columns past e2 (clamped loads, finite values) only feed
  // output columns that are never stored.
  auto store_y = [&](const yt (&yv)[KY], int yb, int ab) {
    if constexpr (YV == 3) {
      const int hh = wave / (64 / MF), lgw = wave % (64 / MF);
      unsigned* Yw = reinterpret_cast<unsigned*>(Ysf[yb]);
      // the rank factors in FP32 (below 2^14 by the choice of g; one more
      // rounding of 2^-24 relative, far inside the FP16 terms' 2^-22)
      const float a0 = (float)alphaS[ab][kw + 2 * yq], a1 = (float)alphaS[ab][kw + 2 * yq + 1];
#pragma unroll
      for (int hc = 0; hc < NHC; ++hc)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // the two ranks of this lane's word, split together (packed)
          unsigned w[NT];
          split_f16_pair(a0 * yv[8 * hc + q], a1 * yv[8 * hc + 4 + q], w);
          const int n = 64 * hc + 4 * cg + q;
          const int piece = ((n / MF) * NH + hh) * YP + lgw * MF + (n % MF);
#pragma unroll
          for (int t = 0; t < NT; ++t) Yw[(t * FN * NH * YP + piece) * 4 + yq] = w[t];
        }
      return;
    }
    if constexpr (YV == 2) {
      // half a 16-byte piece (4 ranks) per column and term
      const int hh = wave / (64 / MF), lgw = wave % (64 / MF);
      uint2* Yh = reinterpret_cast<uint2*>(Ysf[yb]);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        unsigned pk[NT][2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          unsigned u0[NT], u1[NT];
          const int kk = 2 * e;
          split_val((float)(alphaS[ab][kby + 4 * yh + kk] * yv[2 * kk + q]), u0);
          split_val((float)(alphaS[ab][kby + 4 * yh + kk + 1] * yv[2 * kk + 2 + q]), u1);
#pragma unroll
          for (int t = 0; t < NT; ++t) pk[t][e] = pack_hi(u0[t], u1[t]);
        }
        const int n = 2 * yp + q;
        const int piece = ((n / MF) * NH + hh) * 64 + lgw * MF + (n % MF);
#pragma unroll
        for (int t = 0; t < NT; ++t) Yh[(t * FN * NH * 64 + piece) * 2 + yh] = make_uint2(pk[t][0], pk[t][1]);
      }
      return;
    }
#pragma unroll
    for (int g = 0; g < KY / 8; ++g) {
      unsigned pk[NT][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = g * 8 + 2 * q;
        unsigned u0[NT], u1[NT];
        split_val((float)(alphaS[ab][kby + kk] * yv[kk]), u0);
        split_val((float)(alphaS[ab][kby + kk + 1] * yv[kk + 1]), u1);
#pragma unroll
        for (int t = 0; t < NT; ++t) pk[t][q] = pack_hi(u0[t], u1[t]);
      }
      const int sl = (kby >> 3) + g;
      const int hh = sl / (64 / MF), lgw = sl % (64 / MF);
      const int piece = ((ny / MF) * NH + hh) * 64 + lgw * MF + (ny % MF);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        Ysf[yb][t * FN * NH * 64 + piece] = make_uint4(pk[t][0], pk[t][1], pk[t][2], pk[t][3]);
    }
  };

  typename Mma::acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < Mma::NV; ++v) acc[i][j][v] = 0.0f;

  // results of a finished tile; a tile that lies inside its box (the common
  // case, a uniform test) is stored without per-element tests
  auto epilogue = [&](const StreamPos& p) {
    float* __restrict__ out = out_all + p.ooff + (size_t)p.ib * p.e1 * p.e2;
    if (p.j0 + BM <= p.e1 && p.col0 + BN <= p.e2) {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int v = 0; v < Mma::NV; ++v) {
          float* __restrict__ rp = out + (size_t)(p.j0 + wr + i * MF + Mma::drow(lane, v)) * p.e2 +
                                   p.col0 + Mma::dcol(lane);
#pragma unroll
          for (int j = 0; j < FN; ++j) __builtin_nontemporal_store(sc * acc[i][j][v], rp + j * MF);
        }
    } else {
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int v = 0; v < Mma::NV; ++v) {
            const int jj = p.j0 + wr + i * MF + Mma::drow(lane, v);
            const int col = p.col0 + j * MF + Mma::dcol(lane);
            if (jj < p.e1 && col < p.e2)
              __builtin_nontemporal_store(sc * acc[i][j][v], &out[(size_t)jj * p.e2 + col]);
          }
    }
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < Mma::NV; ++v) acc[i][j][v] = 0.0f;
  };

  // p[0..3]: positions of steps s .. s+3 (clamped to the last step S-1)
  StreamPos p0, p1, p2, p3;
  p0.c = 0;
  stream_tile<BN>(bs, xcd * per + l, p0);
  if (bs.cmask != nullptr) p0.c = __builtin_ctz(p0.m);
  p1 = p0;
  if (S > 1) stream_next<BN>(bs, p1, nchunk, nbx);
  p2 = p1;
  if (S > 2) stream_next<BN>(bs, p2, nchunk, nbx);
  p3 = p2;
  if (S > 3) stream_next<BN>(bs, p3, nchunk, nbx);

  yt yr[2][KY];
  double al[2][2];
  // In step s every wave loads the raw f2 values of step s+2 and the rank
  // factors of step s+3 into one register set, reads Ysf[s & 1] for the
  // MFMAs, loads the left operand of step s+1 as each term's MFMAs finish,
  // writes step s+1 (raw values loaded in step s-1, other set) into
  // Ysf[(s+1) & 1] and the factors of step s+2 into alphaS[s & 1]; both
  // buffers were last read before the barrier that ended step s-1. With wide
  // tiles the raw f2 values loaded in step s are those of step s+1, written
  // at its end.
  auto step = [&](int s, const yt (&ys)[KY], yt (&yl)[KY], const double (&as)[2],
                  double (&aload)[2]) {
    const int yb = s & 1;
    if constexpr (SH)
      ld_y(yl, p1);
    else
      ld_y(yl, p2);
    ld_al(aload, p3);
    if constexpr (BN == 128) {
      // per column fragment: its f2 terms from LDS, then every product with
      // it (the products of each accumulator in the same order as below)
#pragma unroll
      for (int ta = NT - 1; ta >= 0; --ta) {
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          s8_t bj[NT][NH];
#pragma unroll
          for (int tb = NT - 1 - ta; tb >= 0; --tb)
#pragma unroll
            for (int h = 0; h < NH; ++h)
              bj[tb][h] = __builtin_bit_cast(s8_t, Ysf[yb][((tb * FN + j) * NH + h) * YP + lane]);
#pragma unroll
          for (int tb = NT - 1 - ta; tb >= 0; --tb)
#pragma unroll
            for (int h = 0; h < NH; ++h)
#pragma unroll
              for (int i = 0; i < FM; ++i) {
                if constexpr (MF == 16)
                  acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8_t, av[ta][i][h]),
                                                                     __builtin_bit_cast(h8_t, bj[tb][h]),
                                                                     acc[i][j], 0, 0, 0);
                else
                  acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(h8_t, av[ta][i][h]),
                                                                     __builtin_bit_cast(h8_t, bj[tb][h]),
                                                                     acc[i][j], 0, 0, 0);
              }
        }
        load_a(ta, p1);
      }
    } else {
      s8_t bv[NT][FN][NH];
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int j = 0; j < FN; ++j)
#pragma unroll
          for (int h = 0; h < NH; ++h)
            bv[t][j][h] = __builtin_bit_cast(s8_t, Ysf[yb][((t * FN + j) * NH + h) * YP + lane]);
#pragma unroll
      for (int ta = NT - 1; ta >= 0; --ta) {
#pragma unroll
        for (int tb = NT - 1 - ta; tb >= 0; --tb)
#pragma unroll
          for (int h = 0; h < NH; ++h)
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
              for (int j = 0; j < FN; ++j) {
                if constexpr (FMT == 1 && MF == 16)
                  acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                      __builtin_bit_cast(h8_t, av[ta][i][h]), __builtin_bit_cast(h8_t, bv[tb][j][h]),
                      acc[i][j], 0, 0, 0);
                else if constexpr (FMT == 1)
                  acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                      __builtin_bit_cast(h8_t, av[ta][i][h]), __builtin_bit_cast(h8_t, bv[tb][j][h]),
                      acc[i][j], 0, 0, 0);
                else if constexpr (MF == 16)
                  acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                      __builtin_bit_cast(bf8_t, av[ta][i][h]), __builtin_bit_cast(bf8_t, bv[tb][j][h]),
                      acc[i][j], 0, 0, 0);
                else
                  acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                      __builtin_bit_cast(bf8_t, av[ta][i][h]), __builtin_bit_cast(bf8_t, bv[tb][j][h]),
                      acc[i][j], 0, 0, 0);
              }
        load_a(ta, p1);
      }
    }
    if constexpr (SH)
      store_y(yl, yb ^ 1, yb ^ 1);
    else
      store_y(ys, yb ^ 1, yb ^ 1);
    pt_al(yb, as, p2);
    if (bs.cmask != nullptr ? chunks_after(p0) == 0u : p0.c == nchunk - 1) epilogue(p0);
    __syncthreads();
    p0 = p1;
    p1 = p2;
    p2 = p3;
    if (s + 4 < S) stream_next<BN>(bs, p3, nchunk, nbx);
  };

  ld_al(al[0], p0);
  ld_y(yr[0], p0);
#pragma unroll
  for (int t = 0; t < NT; ++t) load_a(t, p0);
  pt_al(0, al[0], p0);
  ld_al(al[1], p1);
  __syncthreads();
  store_y(yr[0], 0, 0);
  pt_al(1, al[1], p1);
  if constexpr (!SH) ld_y(yr[0], p1);
  ld_al(al[0], p2);
  __syncthreads();
  // the positions advance inside step: step s sees p0 = step s
  for (int s = 0; s < S; s += 2) {
    step(s, yr[0], yr[1], al[0], al[1]);
    if (s + 1 < S) step(s + 1, yr[1], yr[0], al[1], al[0]);
  }
}

// ---------------------------------------------------------------------------
// tile table
// ---------------------------------------------------------------------------
// Row tiles: BM rows of the (i, j) rows, or (per_i) BM values of j for each i.
static void fill_tiles(BoxSet* bs, int bm, int bn, bool per_i = false) {
  long long acc = 0;
  for (int i = 0; i < bs->nbox; ++i) {
    const BoxArg& a = bs->box[i];
    const long long tm = per_i ? (long long)a.e0 * ((a.e1 + bm - 1) / bm)
                               : ((long long)a.e0 * a.e1 + bm - 1) / bm;
    bs->tiles_n[i] = (a.e2 + bn - 1) / bn;
    bs->tile_start[i] = acc;
    acc += tm * bs->tiles_n[i];
  }
  bs->tile_start[bs->nbox] = acc;
  bs->per_xcd = (acc + 7) / 8;
}

// Workgroups of k_recon_stream<NT, MF> resident at once on the current device
// (occupancy per CU times CUs, cached per device); 0 if the query fails.
template <int NT, int MF, int YV = 2, int FMT = 0, int OPT = 0>
static int stream_slots() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  const int v = cache[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&k_recon_stream<NT, MF, YV, FMT, OPT>), 256, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  const int n = per_cu * cus;
  if (n > 0) cache[dev].store(n, std::memory_order_relaxed);
  return n;
}

// Persistent launch: nbx workgroups per XCD, at most one per resident slot
// and one per tile of the XCD's range. Tile numbers and buffer offsets are
// 32-bit in the kernel; a launch with over 2^31 tiles, or an f2 or pre-split
// f1 of 2 GB or more, uses the per-tile kernel instead.
template <int NT, int MF, int YV = 2, int FMT = 0, int OPT = 0>
static bool launch_stream(hipStream_t s, BoxSet& bs, float* out) {
  const long long total = bs.tile_start[bs.nbox];
  const BoxArg& a = bs.box[0];
  const long long ybytes = (long long)a.K * a.len2 * 8;
  const long long pbytes = (long long)NT * bs.nch * a.len1 * 64;
  if (total >= (1LL << 31) - (1LL << 20) || ybytes >= (1LL << 31) || pbytes >= (1LL << 31)) {
    if constexpr (FMT == 1) {
      return false;  // no per-tile FP16 kernel
    } else {
      dim3 grid((unsigned)(8 * bs.per_xcd));
      hipLaunchKernelGGL((k_recon_direct<NT, 64, MF, 0>), grid, dim3(256), 0, s, bs, out);
      return true;
    }
  }
  int slots = stream_slots<NT, MF, YV, FMT, OPT>();
  if (slots < 8) slots = 8 * 64;
  const long long nbx = std::max(1LL, std::min((long long)(slots / 8), bs.per_xcd));
  hipLaunchKernelGGL((k_recon_stream<NT, MF, YV, FMT, OPT>), dim3((unsigned)(8 * nbx)), dim3(256), 0, s,
                     bs, (int)nbx, out);
  return true;
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
  // the in-kernel split tiles address f1 and f2 with 32-bit buffer offsets
  auto split_fits = [&]() {
    return (long long)bs.box[0].K * std::max(bs.box[0].len1, bs.box[0].len2) * 8 < (1LL << 31);
  };
#define LS_T(ID, BM_, BN_, WM_, WN_, NB_, MF_)                                                \
  if (tile == ID) {                                                                          \
    if (!dry) {                                                                              \
      if (!split_fits()) return false;                                                       \
      fill_tiles(&bs, BM_, BN_);                                                             \
      dim3 grid((unsigned)(8 * bs.per_xcd));                                                 \
      hipLaunchKernelGGL((k_recon_split<NT, BM_, BN_, WM_, WN_, NB_, MF_>), grid, block, 0, s, \
                         bs, (float*)out);                                                   \
    }                                                                                        \
    return true;                                                                             \
  }
  LS_T(1, 128, 128, 64, 64, 1, 16)
  LS_T(2, 128, 128, 64, 64, 1, 32)
  LS_T(3, 128, 64, 64, 32, 1, 32)
  LS_T(4, 64, 128, 32, 64, 1, 32)
  LS_T(5, 64, 64, 32, 32, 2, 16)
#undef LS_T
#define LS_P(ID, BM_, BN_, WM_, WN_, NB_, MF_)                                                \
  if (tile == ID) {                                                                          \
    if (!dry) {                                                                              \
      fill_tiles(&bs, BM_, BN_, true);                                                       \
      dim3 grid((unsigned)(8 * bs.per_xcd));                                                 \
      hipLaunchKernelGGL((k_recon_presplit<NT, BM_, BN_, WM_, WN_, NB_, MF_>), grid, block, 0, \
                         s, bs, (float*)out);                                                \
    }                                                                                        \
    return true;                                                                             \
  }
  LS_P(6, 256, 64, 64, 64, 1, 16)
  LS_P(7, 256, 64, 64, 64, 1, 32)
  LS_P(8, 128, 128, 64, 64, 1, 32)
  LS_P(9, 128, 64, 64, 32, 1, 32)
#undef LS_P
#define LS_D(ID, MF_, PIPE_)                                                                  \
  if (tile == ID) {                                                                          \
    if (!dry) {                                                                              \
      fill_tiles(&bs, 256, 64, true);                                                        \
      dim3 grid((unsigned)(8 * bs.per_xcd));                                                 \
      hipLaunchKernelGGL((k_recon_direct<NT, 64, MF_, PIPE_>), grid, block, 0, s, bs,         \
                         (float*)out);                                                       \
    }                                                                                        \
    return true;                                                                             \
  }
  LS_D(10, 16, 0)
  LS_D(11, 32, 0)
  LS_D(12, 16, 1)
  LS_D(13, 32, 1)
#undef LS_D
  if (tile >= 14 && tile <= 16) {
    if (!dry) {
      fill_tiles(&bs, 256, 64, true);
      if (tile == 14) launch_stream<NT, 16>(s, bs, (float*)out);
      else if (tile == 15) launch_stream<NT, 32>(s, bs, (float*)out);
      else launch_stream<NT, 16, 1>(s, bs, (float*)out);
    }
    return true;
  }
  return false;
}

// LS_F16X3, all on the persistent kernel with the rank factors loaded by
// wave 0 unless stated. f2 from its FP32 copy in the workspace: tile 1 =
// 16x16 MFMA with 128-column tiles, 2 = 16x16 with 64-column tiles (both with
// padded f2 fragments in LDS), 3 = 32x32 with 64-column tiles, 4 = tile 2
// with every wave loading the rank factors, 8 = 32x32 with 128-column tiles.
// f2 from the FP64 factor: 5 = 16x16, 6 = 32x32, 7 = 16x16 with every wave
// loading the rank factors (64-column tiles). Tiles 1, 2 and 4 give the same
// results bit for bit, and so do 3 and 8, and 5 and 7. False when the launch
// exceeds the persistent kernel's 32-bit limits.
static bool launch_f16(int tile, hipStream_t s, BoxSet& bs, void* out, bool dry) {
  if (tile < 1 || tile > 8) return false;
  if (dry) return true;
  fill_tiles(&bs, 256, (tile == 1 || tile == 8) ? 128 : 64, true);
  switch (tile) {
    case 1: return launch_stream<2, 16, 3, 1, 21>(s, bs, (float*)out);
    case 2: return launch_stream<2, 16, 3, 1, 17>(s, bs, (float*)out);
    case 3: return launch_stream<2, 32, 3, 1, 1>(s, bs, (float*)out);
    case 4: return launch_stream<2, 16, 3, 1, 16>(s, bs, (float*)out);
    case 5: return launch_stream<2, 16, 2, 1, 1>(s, bs, (float*)out);
    case 6: return launch_stream<2, 32, 2, 1, 1>(s, bs, (float*)out);
    case 7: return launch_stream<2, 16, 2, 1, 0>(s, bs, (float*)out);
    // the 32x32 shape with 128-column tiles and padded f2 fragments: 0.57
    // against 0.64 ms unpadded on the headline boxes, still 5-7 % slower than
    // tile 1 (its two accumulators per column fragment leave each
    // accumulation chain of the 16-pass MFMA only one independent MFMA)
    default: return launch_stream<2, 32, 3, 1, 20>(s, bs, (float*)out);
  }
}

// tiles of the split precisions that read f1 pre-split from the workspace
static bool presplit_tile(int precision, int tile) {
  return ((precision == LS_BF16X3 || precision == LS_BF16X6) && tile >= 6) || precision == LS_F16X3;
}

static size_t align256(size_t n) { return (n + 255) / 256 * 256; }

// LS_F16X3 workspace: pre-split f1 (two FP16 terms) | row maxima of f0, f1,
// f2 (3 x K double) | coefS (double) | g (int) | coefS32 (double) | f2
// 2^(-e2_r) rounded to FP32 (K x len2) | rank order (K int) | chunk masks of
// the planes of axis 0 (len0 words, when the ranks fill at most 32 chunks)
struct F16Layout {
  size_t p, rmax, coefS, gexp, coefS32, f2f, perm, cmask, total;
};
static bool f16_masks(int K) { return (K + SPLIT_BK - 1) / SPLIT_BK <= 32; }
static F16Layout f16_layout(int K, int len0, int len1, int len2) {
  F16Layout L;
  const size_t nch = (size_t)((K + SPLIT_BK - 1) / SPLIT_BK);
  L.p = 0;
  L.rmax = align256(2 * nch * (size_t)len1 * 64);
  L.coefS = L.rmax + align256((size_t)K * 24);
  L.gexp = L.coefS + align256((size_t)K * 8);
  L.coefS32 = L.gexp + 256;
  L.f2f = L.coefS32 + align256((size_t)K * 8);
  L.perm = L.f2f + align256((size_t)K * len2 * 4);
  L.cmask = L.perm + align256((size_t)K * 4);
  L.total = L.cmask + (f16_masks(K) ? align256((size_t)len0 * 4) : 0);
  return L;
}

static size_t presplit_bytes(int precision, const ls_canon* P) {
  const int K = P->K, len1 = P->len[1];
  if (precision == LS_F16X3) return f16_layout(K, P->len[0], len1, P->len[2]).total;
  if (precision != LS_BF16X3 && precision != LS_BF16X6) return 0;
  const size_t nt = precision == LS_BF16X6 ? 3 : 2;
  return nt * (size_t)((K + SPLIT_BK - 1) / SPLIT_BK) * (size_t)len1 * 64;
}

static int n_tiles(int precision) {
  switch (precision) {
    case LS_F64: return 5;
    case LS_F32: return 8;
    case LS_F16X3: return 8;
    default: return 16;
  }
}

static bool dispatch(int precision, int tile, hipStream_t s, BoxSet& bs, void* out, bool dry) {
  switch (precision) {
    case LS_F64: return launch_fp<double>(tile, s, bs, out, dry);
    case LS_F32: return launch_fp<float>(tile, s, bs, out, dry);
    case LS_BF16X3: return launch_bf<2>(tile, s, bs, out, dry);
    case LS_BF16X6: return launch_bf<3>(tile, s, bs, out, dry);
    case LS_F16X3: return launch_f16(tile, s, bs, out, dry);
    default: return false;
  }
}

// Tile picked when the caller passes tile = 0 (measured on 256^3 boxes,
// K = 384: FP64 64x64, FP32 128x128 with rank chunk 16, split-bf16 with a
// workspace the persistent stream kernel, 256x64 tiles, 16x16 MFMA).
static int auto_tile(int precision, long long M, long long Nc, int e1, bool have_ws) {
  // FP16x3: 16x16 shape, FP32 f2, 128-column tiles unless the boxes are
  // narrower (measured fastest at K = 384, 768 on 256^3 boxes)
  if (precision == LS_F16X3) return Nc >= 128 ? 1 : 2;
  const long long big = ((M + 127) / 128) * ((Nc + 127) / 128);
  const bool split = precision == LS_BF16X3 || precision == LS_BF16X6;
  if (split && have_ws && big >= 256) {
    if (e1 >= 256) return 14;
    if (e1 >= 128) return 9;
  }
  if (big >= 256) {
    switch (precision) {
      case LS_F64: return 2;
      case LS_F32: return 1;
      case LS_BF16X6: return 2;
      default: return 1;
    }
  }
  if (split) return big >= 128 ? 4 : 5;
  const long long mid = ((M + 127) / 128) * ((Nc + 63) / 64);
  if (mid >= 512) return 3;
  return 2;
}

}  // namespace ls

using namespace ls;

extern "C" int32_t ls_reconstruct_tiles(int32_t precision) {
  if (precision < LS_F64 || precision > LS_F16X3) return 0;
  return n_tiles(precision);
}

extern "C" size_t ls_reconstruct_workspace(const ls_canon* P, int32_t precision) {
  if (P == nullptr || P->K < 1 || P->len[1] < 1) return 0;
  return presplit_bytes(precision, P);
}

// What a call with a workspace forms there before its reconstruction
// kernels: for LS_F16X3 the row maxima, the pre-split f1, the FP32 copy of f2
// and the scaled rank factors; for the split-bf16 precisions the pre-split f1.
static ls_status prepare_ws(const ls_canon* P, int precision, void* ws_dev, hipStream_t stream) {
  const int nch = (P->K + SPLIT_BK - 1) / SPLIT_BK;
  const F16Layout fl = f16_layout(P->K, P->len[0], P->len[1], P->len[2]);
  char* wsb = (char*)ws_dev;
  if (precision == LS_F16X3) {
    // the row maxima: those the assembly wrote, if the descriptor carries
    // them, else one pass over the three factor matrices
    const double* rmax = P->rowmax;
    if (rmax == nullptr) {
      hipLaunchKernelGGL(k_rank_max, dim3(P->K, 3), dim3(256), 0, stream, P->f[0], P->f[1],
                         P->f[2], P->K, P->len[0], P->len[1], P->len[2], (double*)(wsb + fl.rmax));
      rmax = (const double*)(wsb + fl.rmax);
    }
    const int n8 = (P->K + 7) / 8;
    unsigned* cmask = f16_masks(P->K) ? (unsigned*)(wsb + fl.cmask) : nullptr;
    hipLaunchKernelGGL(k_f16_order, dim3(1), dim3(512), 0, stream, P->coef, rmax, P->K, P->len[0],
                       (int*)(wsb + fl.perm), (double*)(wsb + fl.coefS),
                       (double*)(wsb + fl.coefS32), (int*)(wsb + fl.gexp), cmask);
    const int lx = std::max(std::max(P->len[1], P->len[2]), cmask ? P->len[0] : 1);
    hipLaunchKernelGGL(k_prep_f16, dim3((lx + 63) / 64, nch + n8 + (cmask ? nch : 0)), dim3(64), 0,
                       stream, P->f[1], P->f[2], P->f[0], rmax, (const int*)(wsb + fl.perm),
                       (const double*)(wsb + fl.coefS32), P->K, P->len[0], P->len[1], P->len[2],
                       nch, n8, (unsigned*)ws_dev, (float*)(wsb + fl.f2f), cmask);
    return launch_status("ls_reconstruct (scales and pre-split)");
  }
  dim3 grid((P->len[1] + 63) / 64, nch);
  if (precision == LS_BF16X6)
    hipLaunchKernelGGL(k_presplit<3>, grid, dim3(64), 0, stream, P->f[1], P->K, P->len[1], nch,
                       (unsigned*)ws_dev);
  else
    hipLaunchKernelGGL(k_presplit<2>, grid, dim3(64), 0, stream, P->f[1], P->K, P->len[1], nch,
                       (unsigned*)ws_dev);
  return launch_status("ls_reconstruct (pre-split)");
}

static ls_status check_canon(const ls_canon* P) {
  LS_REQUIRE(P != nullptr, "null pointer");
  LS_REQUIRE(P->K >= 1, "rank K must be >= 1");
  LS_REQUIRE(P->f[0] && P->f[1] && P->f[2] && P->coef, "null factor pointer");
  for (int l = 0; l < 3; ++l) LS_REQUIRE(P->len[l] >= 1, "len[%d] must be >= 1", l);
  return LS_OK;
}

// ---------------------------------------------------------------------------
// Measured tile choice: ls_reconstruct_autotune times every tile of a
// precision on the caller's own call and keeps the fastest per shape class;
// a call with tile 0 of a tuned class takes it, other calls the built-in
// choice (auto_tile).
// ---------------------------------------------------------------------------
namespace {
struct ReconTune {
  int tile;
  double ms;
};
std::mutex g_rtune_mu;
std::map<std::vector<long long>, ReconTune> g_rtune;

// shape class of a call: precision, rank, factor lengths, whether the
// workspace serves the pre-split tiles, and the boxes' extents in order
// (their offsets do not change the work)
std::vector<long long> recon_key(const ls_canon* P, const ls_box* boxes, int nbox,
                                 int precision, bool have_ws) {
  std::vector<long long> k = {precision, P->K, P->len[0], P->len[1], P->len[2],
                              have_ws ? 1 : 0, nbox};
  for (int b = 0; b < nbox; ++b)
    for (int l = 0; l < 3; ++l) k.push_back(boxes[b].e[l]);
  return k;
}

int tuned_tile(const ls_canon* P, const ls_box* boxes, int nbox, int precision, bool have_ws,
               double* ms) {
  std::lock_guard<std::mutex> lock(g_rtune_mu);
  const auto it = g_rtune.find(recon_key(P, boxes, nbox, precision, have_ws));
  if (it == g_rtune.end()) return 0;
  if (ms) *ms = it->second.ms;
  return it->second.tile;
}
}  // namespace

// ls_reconstruct, or with prepared = true ls_reconstruct_prepared (the
// workspace already holds the preparation of prepare_ws)
static ls_status reconstruct_common(const ls_canon* P, const ls_box* boxes, int32_t nbox,
                                    double scale, int32_t precision, int32_t tile, void* out_dev,
                                    void* ws_dev, size_t ws_bytes, hipStream_t stream, bool prepared) {
  clear_error();
  ls_status cs = check_canon(P);
  if (cs != LS_OK) return cs;
  LS_REQUIRE(boxes != nullptr && out_dev != nullptr, "null pointer");
  LS_REQUIRE(nbox >= 1, "nbox must be >= 1");
  LS_REQUIRE(std::isfinite(scale), "scale must be finite");
  LS_REQUIRE(precision >= LS_F64 && precision <= LS_F16X3, "unknown precision %d", precision);
  if (tile < 0 || tile > n_tiles(precision)) {
    set_error("tile %d not valid for precision %d", tile, precision);
    return LS_EUNSUPPORTED;
  }
  for (int b = 0; b < nbox; ++b) {
    for (int l = 0; l < 3; ++l) {
      LS_REQUIRE(boxes[b].e[l] >= 1 && boxes[b].o[l] >= 0 &&
                     (long long)boxes[b].o[l] + boxes[b].e[l] <= P->len[l],
                 "box %d outside the factors on axis %d", b, l);
    }
    LS_REQUIRE((long long)boxes[b].e[0] * boxes[b].e[1] < (1LL << 31), "box %d too large", b);
  }
  const size_t need = presplit_bytes(precision, P);
  const bool have_ws = need > 0 && ws_dev != nullptr && ws_bytes >= need;
  int t = tile ? tile : tuned_tile(P, boxes, nbox, precision, have_ws, nullptr);
  if (t == 0)
    t = auto_tile(precision, (long long)boxes[0].e[0] * boxes[0].e[1], boxes[0].e[2],
                  boxes[0].e[1], have_ws);
  BoxSet probe;
  if (!dispatch(precision, t, stream, probe, nullptr, true)) {
    set_error("tile %d not available for precision %d", t, precision);
    return LS_EUNSUPPORTED;
  }
  const bool pre = presplit_tile(precision, t);
  if (pre && !have_ws) {
    set_error("tile %d needs a workspace of %zu bytes", t, need);
    return LS_EWORKSPACE;
  }
  LS_REQUIRE(!pre || ws_aligned(ws_dev), "the workspace must be 256-byte aligned");
  const int nch = (P->K + SPLIT_BK - 1) / SPLIT_BK;
  const F16Layout fl = f16_layout(P->K, P->len[0], P->len[1], P->len[2]);
  char* wsb = (char*)ws_dev;
  if (pre && !prepared) {
    ls_status st = prepare_ws(P, precision, ws_dev, stream);
    if (st != LS_OK) return st;
  }
  long long off = 0;  // elements
  for (int b0 = 0; b0 < nbox; b0 += kBoxesPerLaunch) {
    BoxSet bs;
    bs.nbox = (nbox - b0) < kBoxesPerLaunch ? (nbox - b0) : kBoxesPerLaunch;
    bs.P2 = pre ? (const unsigned*)ws_dev : nullptr;
    bs.nch = nch;
    bs.coefS = precision == LS_F16X3 ? (const double*)(wsb + fl.coefS) : nullptr;
    bs.gexp = precision == LS_F16X3 ? (const int*)(wsb + fl.gexp) : nullptr;
    bs.coefS32 = precision == LS_F16X3 ? (const double*)(wsb + fl.coefS32) : nullptr;
    bs.f2f = precision == LS_F16X3 ? (const float*)(wsb + fl.f2f) : nullptr;
    bs.perm = precision == LS_F16X3 ? (const int*)(wsb + fl.perm) : nullptr;
    bs.cmask = precision == LS_F16X3 && f16_masks(P->K) ? (const unsigned*)(wsb + fl.cmask) : nullptr;
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
    if (!dispatch(precision, t, stream, bs, out, false)) {
      set_error("boxes %d.. exceed the limits of the persistent kernel (2^31 tiles, 2 GB operands)", b0);
      return LS_EUNSUPPORTED;
    }
    ls_status st = launch_status("ls_reconstruct");
    if (st != LS_OK) return st;
    off += local;
  }
  return LS_OK;
}

extern "C" ls_status ls_reconstruct(const ls_canon* P, const ls_box* boxes, int32_t nbox,
                                    double scale, int32_t precision, int32_t tile, void* out_dev,
                                    void* ws_dev, size_t ws_bytes, hipStream_t stream) {
  return reconstruct_common(P, boxes, nbox, scale, precision, tile, out_dev, ws_dev, ws_bytes,
                            stream, false);
}

extern "C" ls_status ls_reconstruct_prepared(const ls_canon* P, const ls_box* boxes, int32_t nbox,
                                             double scale, int32_t precision, int32_t tile,
                                             void* out_dev, void* ws_dev, size_t ws_bytes,
                                             hipStream_t stream) {
  return reconstruct_common(P, boxes, nbox, scale, precision, tile, out_dev, ws_dev, ws_bytes,
                            stream, true);
}

extern "C" ls_status ls_reconstruct_autotune(const ls_canon* P, const ls_box* boxes,
                                             int32_t nbox, double scale, int32_t precision,
                                             void* out_dev, void* ws_dev, size_t ws_bytes,
                                             int32_t reps, hipStream_t stream, int32_t* tile_out,
                                             double* ms_out) {
  clear_error();
  LS_REQUIRE(tile_out != nullptr, "null pointer");
  *tile_out = 0;
  if (ms_out) *ms_out = 0.0;
  LS_REQUIRE(reps >= 1 && reps <= 1000, "reps must be in [1, 1000] (got %d)", reps);
  // the call as given (tile 0) validates every argument before anything is timed
  ls_status st = reconstruct_common(P, boxes, nbox, scale, precision, 0, out_dev, ws_dev,
                                    ws_bytes, stream, false);
  if (st != LS_OK) return st;
  const size_t need = presplit_bytes(precision, P);
  const bool have_ws = need > 0 && ws_dev != nullptr && ws_bytes >= need;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) {
    set_error("event creation failed");
    return LS_EHIP;
  }
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    set_error("event creation failed");
    return LS_EHIP;
  }
  int best = 0;
  float best_ms = 0.f;
  for (int t = 1; t <= n_tiles(precision) && st == LS_OK; ++t) {
    BoxSet probe;
    if (!dispatch(precision, t, stream, probe, nullptr, true)) continue;
    if (presplit_tile(precision, t) && !have_ws) continue;
    // untimed first run; a tile that refuses this call's shapes is skipped
    st = reconstruct_common(P, boxes, nbox, scale, precision, t, out_dev, ws_dev, ws_bytes,
                            stream, false);
    if (st == LS_EUNSUPPORTED) {
      st = LS_OK;
      continue;
    }
    if (st != LS_OK) break;
    (void)hipEventRecord(e0, stream);
    for (int i = 0; i < reps && st == LS_OK; ++i)
      st = reconstruct_common(P, boxes, nbox, scale, precision, t, out_dev, ws_dev, ws_bytes,
                              stream, false);
    (void)hipEventRecord(e1, stream);
    if (st != LS_OK) break;
    if (hipEventSynchronize(e1) != hipSuccess) {
      set_error("autotune synchronisation failed");
      st = LS_EHIP;
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    ms /= (float)reps;
    if (best == 0 || ms < best_ms) {
      best = t;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LS_OK) return st;
  if (best == 0) {
    set_error("no tile of precision %d runs this call", precision);
    return LS_EUNSUPPORTED;
  }
  {
    std::lock_guard<std::mutex> lock(g_rtune_mu);
    g_rtune[recon_key(P, boxes, nbox, precision, have_ws)] = ReconTune{best, (double)best_ms};
  }
  *tile_out = best;
  if (ms_out) *ms_out = best_ms;
  return LS_OK;
}

extern "C" ls_status ls_reconstruct_tuned_tile(const ls_canon* P, const ls_box* boxes,
                                               int32_t nbox, int32_t precision,
                                               const void* ws_dev, size_t ws_bytes,
                                               int32_t* tile, double* ms) {
  clear_error();
  LS_REQUIRE(P != nullptr && boxes != nullptr && tile != nullptr, "null pointer");
  LS_REQUIRE(nbox >= 1, "nbox must be >= 1");
  LS_REQUIRE(precision >= LS_F64 && precision <= LS_F16X3, "unknown precision %d", precision);
  const size_t need = presplit_bytes(precision, P);
  const bool have_ws = need > 0 && ws_dev != nullptr && ws_bytes >= need;
  if (ms) *ms = 0.0;
  *tile = tuned_tile(P, boxes, nbox, precision, have_ws, ms);
  return LS_OK;
}

extern "C" ls_status ls_reconstruct_f16_plan(const ls_canon* P, const ls_box* boxes,
                                             int32_t nbox, const void* ws_dev, size_t ws_bytes,
                                             int32_t* perm_host, uint32_t* masks_host,
                                             int64_t* chunk_values) {
  clear_error();
  ls_status cs = check_canon(P);
  if (cs != LS_OK) return cs;
  LS_REQUIRE(boxes != nullptr && nbox >= 1, "nbox must be >= 1");
  for (int b = 0; b < nbox; ++b)
    for (int l = 0; l < 3; ++l)
      LS_REQUIRE(boxes[b].e[l] >= 1 && boxes[b].o[l] >= 0 &&
                     (long long)boxes[b].o[l] + boxes[b].e[l] <= P->len[l],
                 "box %d outside the factors on axis %d", b, l);
  const size_t need = presplit_bytes(LS_F16X3, P);
  if (ws_dev == nullptr || ws_bytes < need) {
    set_error("a workspace of %zu bytes is required", need);
    return LS_EWORKSPACE;
  }
  const F16Layout fl = f16_layout(P->K, P->len[0], P->len[1], P->len[2]);
  const char* wsb = (const char*)ws_dev;
  const int nch = (P->K + SPLIT_BK - 1) / SPLIT_BK;
  const bool masked = f16_masks(P->K);
  std::vector<uint32_t> m((size_t)P->len[0], masked ? 0u : ~0u);
  if (masked && hipMemcpy(m.data(), wsb + fl.cmask, m.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("copy of the chunk masks failed");
    return LS_EHIP;
  }
  if (perm_host != nullptr &&
      hipMemcpy(perm_host, wsb + fl.perm, (size_t)P->K * 4, hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("copy of the rank order failed");
    return LS_EHIP;
  }
  if (masks_host != nullptr) std::copy(m.begin(), m.end(), masks_host);
  if (chunk_values != nullptr) {
    long long cv = 0;
    for (int b = 0; b < nbox; ++b) {
      long long per_plane = 0;
      for (int i = 0; i < boxes[b].e[0]; ++i) {
        const uint32_t mi = m[(size_t)boxes[b].o[0] + i];
        per_plane += masked ? (mi ? __builtin_popcount(mi) : 1) : nch;
      }
      cv += per_plane * boxes[b].e[1] * boxes[b].e[2];
    }
    *chunk_values = cv;
  }
  return LS_OK;
}

extern "C" ls_status ls_reconstruct_prepare(const ls_canon* P, int32_t precision, void* ws_dev,
                                            size_t ws_bytes, hipStream_t stream) {
  clear_error();
  ls_status cs = check_canon(P);
  if (cs != LS_OK) return cs;
  LS_REQUIRE(precision >= LS_F64 && precision <= LS_F16X3, "unknown precision %d", precision);
  const size_t need = presplit_bytes(precision, P);
  if (need == 0) return LS_OK;  // FP64 and FP32 use no workspace
  if (ws_dev == nullptr || ws_bytes < need) {
    set_error("a workspace of %zu bytes is required", need);
    return LS_EWORKSPACE;
  }
  LS_REQUIRE(ws_aligned(ws_dev), "the workspace must be 256-byte aligned");
  return prepare_ws(P, precision, ws_dev, stream);
}
