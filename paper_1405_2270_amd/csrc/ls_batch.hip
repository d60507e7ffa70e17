// Batched lattice systems in one persistent launch (per system: Sec. 3.1,
// Theorem 3.1 assembly, the canonical scalar product of the Appendix,
// eq. scal, for the energy, and the reconstruction of one sub-box of at most
// one unit cell per axis).
//
// One kernel, k_batch, drains device work queues, one per XCD: every task of
// a system sits in one queue, so the system's folded density and factor
// columns, re-read by all its VEC and TILE tasks, stay in that XCD's L2.
// Workgroups take task indices from their own queue's counter (workgroup b
// runs on XCD b mod 8: the dispatcher deals workgroups to the XCDs in turn)
// and, once it is empty, from the other queues in turn. Each queue is a
// pipeline over groups of its systems taken by decreasing cost (the FOLDs of
// one group, the VECs of the previous one, the TILEs of the one before):
//   FOLD (system, axis)  Phi_l[s][i] = sum_k rho_l[s][i + k n], the density
//                        folded back over the lattice shifts (one lane per
//                        residue class, suffix/prefix sums, no subtraction).
//   VEC  (system, atom, axis)  for every q: the master cells j in [-X, X) are
//                        generated in registers; their dot products with Phi
//                        are the Gram entries G_l[nu q][s] (the assembled
//                        vector's scalar product with the density), and the
//                        cells that fall on the requested sub-box are summed
//                        per residue into its factor columns. The system's
//                        last VEC task forms E = sum_r coef_r sum_s d_s prod_l G.
//   TILE (system, tile)  one MFMA tile of the sub-box reconstruction.
// A VEC task waits until its system's FOLD tasks are done, a TILE until its
// VEC tasks are done and the last of them has formed the energy (and, for
// LS_F16X3, the per-rank scales of the FP16 tiles from the largest value of
// every sub-box column). Every awaited task is earlier in the same queue and
// was dequeued earlier by a running
// workgroup and never waits on a later one, so every wait ends; each wait is
// also bounded (a spin limit sets an error flag and skips the task).
// Producer: all lanes fence (agent scope), barrier, one lane increments the
// system's counter. Consumer: one lane polls with acquire loads, barrier, all
// lanes fence (acquire) before reading.
//
// Per-system device clock stamps (first task start, last task end) give the
// per-system latency distribution.
#include <algorithm>
#include <array>
#include <climits>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ls_split_tile.hpp"

namespace ls {

enum { TASK_FOLD = 0, TASK_VEC = 1, TASK_TILE = 2 };

struct Task {
  int type, sys, a, pad;
};

struct SysDev {
  double b, h;
  int n, L[3], N[3];
  int M0, R, K, Krho;
  int qoff, X, W;
  int o[3], e[3];
  int nvec, tiles_n;
  const double* pos;
  const double* Z;
  const double* D[3];
  const double* d;
  void* out;
  double* E;
  double* Phi;    // [3][Krho][W]
  double* G;      // [3][K][Krho]
  double* Fc[3];  // [K][e_l]
  double* coef;   // [K]
  double* fmax;   // [3][K] max_x |Fc_l[r][x]| (before the LS_F16X3 normalisation)
  double* fsc;    // [K + 1] FP16 tiles: left-operand rank factors, output scale
  uint4* yp;      // LS_F16X3: [2 terms][nch][e_2][32 ranks] FP16 of 2^13 Fc_2 / 2^e_2,r
};

struct BatchArg {
  const SysDev* sys;
  const Task* tasks;
  const double* tau;
  const double* w;
  const double* qhw;  // support_halfwidth(tau) per node
  const double* qk;   // cell_half_norm(tau) per node
  int* qhead;  // [kBatchQueues] next task of each queue
  int* err;
  int* fold_done;
  int* vec_done;
  unsigned long long* t_start;
  unsigned long long* t_end;
  unsigned long long* t_phase;  // [3][2]: first start, last end per task type
  int qstart[9];  // queue q holds tasks qstart[q] .. qstart[q + 1] - 1
  int nsys;
  int f16;  // LS_F16X3: the last VEC task also forms the FP16 scales
};
constexpr int kBatchQueues = 8;  // one per XCD

constexpr int kSpinLimit = 1 << 22;
// density rank handled by the batch kernel (per-lane accumulators)
constexpr int kBatchRho = 8;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Wait until *counter >= target. Returns false (and flags the error) if the
// spin limit is reached.
__device__ bool wait_counter(int* counter, int target, int* err, int* s_flag) {
  if (threadIdx.x == 0) {
    int spins = 0;
    bool ok = true;
    while (__hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(4);
      ++spins;
      // after any timed-out wait every later wait fails at once, so a broken
      // dependency cannot turn into a long series of timeouts
      if (spins > kSpinLimit ||
          ((spins & 1023) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
        atomicOr(err, 1);
        ok = false;
        break;
      }
    }
    *s_flag = ok ? 1 : 0;
  }
  __syncthreads();
  const bool ok = *s_flag != 0;
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  return ok;
}

// Returns the counter value before the increment (in lane 0; -1 elsewhere).
__device__ int signal_counter(int* counter) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  int prev = -1;
  if (threadIdx.x == 0) prev = __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  return prev;
}

// A pointer into device memory as a global-address-space pointer: its loads
// become global loads, which count only in the vector-memory counter (a flat
// load also counts in the LDS counter, so every wait for an LDS read would
// wait for the loads still in flight as well).
template <typename T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}

// A uniform pointer to data that no task writes during the launch, as a
// constant-address-space pointer (through readfirstlane): its loads become
// scalar loads (scalar cache), not vector loads waited for at full latency.
typedef const __attribute__((address_space(4))) double* cdptr;
__device__ __forceinline__ cdptr cmem(const double* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (cdptr)(((unsigned long long)hi << 32) | lo);
}

// Phi_l[s][i + X] = sum_{k=0}^{L-1} D_l[s][i + k n], i in [-X, X + n), D = 0 outside [0, N).
// For i = rho + c n: c >= 0 -> suffix sum of the residue column from c, c < 0 ->
// prefix sum up to c + L - 1.
__device__ void fold_task(const SysDev& S, int l) {
  const int n = S.n, L = S.L[l], N = S.N[l], X = S.X, W = S.W;
  for (int s = 0; s < S.Krho; ++s) {
    const double* D = S.D[l] + (size_t)s * N;
    double* P = S.Phi + ((size_t)l * S.Krho + s) * W;
    for (int rho = threadIdx.x; rho < n; rho += 256) {
      // zero the whole residue column first (c outside [-(L-1), L-1])
      for (int i = rho; i < W; i += n) P[i] = 0.0;
      double acc = 0.0;
      for (int c = L - 1; c >= 0; --c) {
        acc += D[rho + (size_t)c * n];
        const long long i = (long long)rho + (long long)c * n + X;
        if (i >= 0 && i < W) P[i] = acc;
      }
      acc = 0.0;
      for (int cp = 0; cp <= L - 2; ++cp) {
        acc += D[rho + (size_t)cp * n];
        const long long i = (long long)rho + (long long)(cp - L + 1) * n + X;
        if (i >= 0 && i < W) P[i] = acc;
      }
    }
  }
}

constexpr int kVecQ = 16;
// LDS row stride in doubles, 2 mod 32: the 16 rows x 2 cells that a half-wave
// reads as the MFMA A operand fall on distinct bank pairs
constexpr int kVecRow = 258;

// The cell values of one chunk for the nodes q0 .. q0 + ng - 1 (ng <= kVecQ):
// lane i evaluates the left edge of its cell j (y0 = j - delta) where a cell
// next to it needs it, takes the right edge from lane i + 1, and writes the
// cell value h * integral (0 outside the node's support or for cell_ok false)
// to col[g * kVecRow] (col null: lane 63, which only supplies an edge). Out of
// line: the persistent kernel's own register allocation stays that of its
// tile loops. The nodes' support half-widths and norms come precomputed.
__device__ __attribute__((noinline)) void vec_chunk_cells(const BatchArg& ba, int q0, int ng,
                                                          int j, double delta, double h,
                                                          bool cell_ok, double* col) {
  const double y0 = (double)j - delta;
  // the node tables through the constant address space (scalar loads)
  const cdptr ttau = cmem(ba.tau + q0);
  const cdptr thw = cmem(ba.qhw + q0);
  const cdptr tk = cmem(ba.qk + q0);
  ng = __builtin_amdgcn_readfirstlane(ng);
#pragma unroll 1
  for (int g = 0; g < kVecQ; ++g) {
    double cv = 0.0;
    if (g < ng) {
      const double tau = ttau[g], hw = thw[g];
      const bool in = (double)j >= delta - hw - 1.0 && (double)j <= delta + hw + 1.0;
      double eL = 0.0;
      if (in && edge_needed(tau, j, delta)) eL = edge_value(tau, y0);
      const double eR = __shfl_down(eL, 1, 64);
      if (cell_ok && in) cv = h * cell_from_edges(tau, y0, eL, eR, tk[g]);
    }
    if (col) col[g * kVecRow] = cv;
  }
}

// Vector task: atom nu, axis l, all q, in groups of kVecQ = 16 quadrature
// points. Per chunk of 4 x 63 master cells (63 per wave, each lane's right edge
// from the next lane: shared edges) the 16 integrals of every cell go to LDS
// as bq[g][cell]. The Gram sums G[q][s] = sum_j b_q(j) Phi_s(j)
// then run on v_mfma_f64_16x16x4f64 with the cell values as the A operand
// (rows q) and the folded density as B (columns s): each density value is
// loaded once per 16 points, and a wave keeps one 16x16 accumulator tile
// (four registers per lane). The central-cell factor columns are gathered
// from the same LDS values. All sums run in a fixed order.
constexpr int kVecSmem = (kVecQ * kVecRow + kVecQ * 256 + 4 * kVecQ * kBatchRho + kVecQ) * 8;
typedef double vec_d4_t __attribute__((ext_vector_type(4)));

__device__ void vec_task(const SysDev& S, const BatchArg& ba, int c, double* sbuf) {
  const int nu = c / 3, l = c - 3 * (c / 3);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = S.n, L = S.L[l], X = S.X, W = S.W, Krho = S.Krho;
  const int o = S.o[l], e = S.e[l];
  int p;
  double delta;
  node_offset(S.pos[c], S.b, S.h, n, &p, &delta);
  // the folded density of axis l, Krho rows of W, through a buffer resource:
  // Phi_l[s][j + p] at byte offset (s W + j + p + X) 8; the Gram loads need no
  // conditions (rows s >= Krho and offsets past the block read 0, and cells past
  // the group's support have value 0)
  const __amdgpu_buffer_rsrc_t phbuf = uniform_rsrc(S.Phi + (size_t)l * Krho * W, Krho * W * 8);
  const int qoff = S.qoff;
  const double hcell = S.h;
  // master cells that land on the sub-box: g = j + p + k n in [o, o+e), k in [0, L)
  const int jlo = o - p - (L - 1) * n, jhi = o + e - 1 - p;
  double* bq = sbuf;                          // [kVecQ][kVecRow] cell values
  double* vb = sbuf + kVecQ * kVecRow;        // [kVecQ][256] central-cell columns
  double* red = vb + kVecQ * 256;             // [4 waves][kVecQ][kBatchRho]
  double* cmax = red + 4 * kVecQ * kBatchRho;  // [kVecQ] column maxima
  // a chunk is 4 x 63 cells: wave wv covers cells 63 wv .. 63 wv + 62; lane i
  // evaluates the left edge of cell 63 wv + i and takes the right edge from
  // lane i + 1 (lane 63 only supplies an edge)
  constexpr int CH = 4 * 63;
  const int ci = 63 * wv + lane;              // this lane's cell within the chunk
  // MFMA lane roles: A row (point) gq = lane % 16, cell offset ck = lane / 16
  const int gq = lane & 15, ck = lane >> 4;
#pragma unroll 1
  for (int q0 = 0; q0 < S.R; q0 += kVecQ) {
    const int ng = min(kVecQ, S.R - q0);
    // support of the group: the union of the points' supports
    // (half-widths by scalar loads, all requested together; the indices past
    // the group repeat its last point, which leaves the union unchanged)
    int jbeg = X, jend = -X;
    const cdptr ghw = cmem(ba.qhw + qoff + q0);
#pragma unroll
    for (int g = 0; g < kVecQ; ++g) {
      const double hw = ghw[min(g, ng - 1)];
      jbeg = min(jbeg, (int)fmax((double)-X, floor(delta - hw)));
      jend = max(jend, (int)fmin((double)X, ceil(delta + hw) + 1.0));
    }
    vec_d4_t acc = {0.0, 0.0, 0.0, 0.0};
    // each thread tid < e owns column tid of vb (no other thread touches it)
#pragma unroll
    for (int g = 0; g < kVecQ; ++g) vb[g * 256 + tid] = 0.0;
#pragma unroll 1
    for (int j0 = jbeg; j0 < jend; j0 += CH) {
      const int j = j0 + ci;
      const bool cell_ok = lane < 63 && j < jend;
      vec_chunk_cells(ba, qoff + q0, ng, j, delta, hcell, cell_ok, lane < 63 ? bq + ci : nullptr);
      // Gram: wave wv takes cells 64 wv .. 64 wv + 63 of the chunk, 4 per
      // MFMA; the density values are requested before the barrier, whose
      // wait for the other waves' cells covers their latency
      double bvv[16];
      const int pb = (gq * W + p + X + j0 + 64 * wv + ck) * 8;
#pragma unroll
      for (int k4 = 0; k4 < 16; ++k4)
        bvv[k4] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(phbuf, pb + 32 * k4, 0, 0));
      __syncthreads();
#pragma unroll
      for (int k4 = 0; k4 < 16; ++k4) {
        const int i = 64 * wv + 4 * k4 + ck;  // cell within the chunk
        const double av = (i < CH) ? bq[gq * kVecRow + i] : 0.0;  // rows g >= ng hold 0
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bvv[k4], acc, 0, 0, 0);
      }
      if (j0 + CH - 1 >= jlo && j0 <= jhi) {  // uniform per chunk
        if (tid < e) {
          // cells i of this chunk with (j0 + i + p - o) == tid (mod n)
          int i0 = (tid + o - p - j0) % n;
          if (i0 < 0) i0 += n;
#pragma unroll 1
          for (int i = i0; i < CH; i += n) {
            const int jj = j0 + i;
            if (jj >= jlo && jj <= jhi) {
              const int k = (o + tid - jj - p) / n;  // exact
              if (k >= 0 && k < L) {
#pragma unroll
                for (int g = 0; g < kVecQ; ++g) vb[g * 256 + tid] += bq[g * kVecRow + i];
              }
            }
          }
        }
      }
      __syncthreads();  // bq is rewritten by the next chunk
    }
    // acc[vv] = G[q0 + row][s], row = lane / 16 + 4 vv, s = lane % 16 (f64 MFMA layout)
#pragma unroll
    for (int vv = 0; vv < 4; ++vv) {
      const int row = (lane >> 4) + 4 * vv;
      if (gq < kBatchRho) red[(wv * kVecQ + row) * kBatchRho + gq] = acc[vv];
    }
    __syncthreads();
    if (tid < kVecQ * kBatchRho) {
      const int g = tid / kBatchRho, sidx = tid % kBatchRho;
      if (g < ng && sidx < Krho) {
        const int r = nu * S.R + q0 + g;
        const int st = kVecQ * kBatchRho;
        S.G[((size_t)l * S.K + r) * Krho + sidx] =
            ((red[tid] + red[st + tid]) + red[2 * st + tid]) + red[3 * st + tid];
      }
    }
    // largest magnitude of each sub-box column; for LS_F16X3 the column is
    // stored divided by 2^floor(log2 max) (exact), so its maximum lies in [1, 2)
    for (int g = wv; g < ng; g += 4) {
      double m = 0.0;
      for (int x = lane; x < e; x += 64) m = fmax(m, fabs(vb[g * 256 + x]));
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
      if (lane == 0) cmax[g] = m;
    }
    __syncthreads();
#pragma unroll
    for (int g = 0; g < kVecQ; ++g) {
      if (g < ng) {
        const int r = nu * S.R + q0 + g;
        const double m = cmax[g];
        if (tid < e) {
          double v = vb[g * 256 + tid];
          if (ba.f16 && m > 0.0 && isfinite(m)) v = ldexp(v, -ilogb(m));
          if (ba.f16 && l == 2) {
            // the FP16 tiles' right operand, split once here: 2^13 v < 2^14
            unsigned u[2];
            split_f16((float)(8192.0 * v), u);
            unsigned short* y16 = reinterpret_cast<unsigned short*>(S.yp);
            const size_t nch = (size_t)(S.K + 31) >> 5;
            const size_t at = (((size_t)(r >> 5)) * e + tid) * 32 + (r & 31);
            y16[at] = (unsigned short)(u[0] >> 16);
            y16[nch * e * 32 + at] = (unsigned short)(u[1] >> 16);
          } else {
            S.Fc[l][(size_t)r * e + tid] = v;
          }
        }
        if (tid == 0) S.fmax[(size_t)l * S.K + r] = m;
        if (l == 0 && tid == 0) S.coef[r] = S.Z[nu] * ba.w[S.qoff + q0 + g];
      }
    }
    __syncthreads();
  }
  if (ba.f16 && l == 2 && nu == S.M0 - 1 && (S.K & 31) != 0) {
    // zero the padding ranks K .. 32 nch - 1 of the last chunk (the tiles
    // multiply them by zero rank factors; they must not hold NaN patterns)
    unsigned short* y16 = reinterpret_cast<unsigned short*>(S.yp);
    const size_t nch = (size_t)(S.K + 31) >> 5;
    const int r0 = S.K & 31, npad = 32 - r0;
    for (int idx = tid; idx < 2 * e * npad; idx += 256) {
      const int t = idx / (e * npad), rem = idx - t * e * npad;
      const int x = rem / npad, rr = r0 + rem - (rem / npad) * npad;
      y16[((size_t)t * nch + nch - 1) * e * 32 + (size_t)x * 32 + rr] = 0;
    }
  }
}

__device__ void energy_task(const SysDev& S, double* sbuf) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const size_t st = (size_t)S.K * S.Krho;
  double acc = 0.0;
  for (int r = tid; r < S.K; r += 256) {
    double v = 0.0;
    for (int s = 0; s < S.Krho; ++s) {
      const size_t i0 = (size_t)r * S.Krho + s;
      v += S.d[s] * S.G[i0] * S.G[st + i0] * S.G[2 * st + i0];
    }
    acc += S.coef[r] * v;
  }
  acc = wave_sum(acc);
  if (lane == 0) sbuf[wv] = acc;
  __syncthreads();
  if (tid == 0) *S.E = ((sbuf[0] + sbuf[1]) + sbuf[2]) + sbuf[3];
  __syncthreads();
}

// Scales of the FP16 tiles (LS_F16X3). The VEC tasks stored every sub-box
// column divided by 2^e_l,r, e_l,r = floor(log2 max_x |Fc_l[r][x]|), so the
// stored columns lie below 2 in magnitude, and the right operand already
// split as 2^13 Fc_2[r][k] (below 2^14). With E_r = e_0,r + e_1,r + e_2,r and
// t_r = floor(log2 |coef_r|) + E_r (the true rank term is below 2^(t_r + 4)),
// T = max_r t_r over the ranks not identically zero on the sub-box:
//   left operand   coef_r 2^(11 - T + E_r) Fc_0[r][i] Fc_1[r][j]  (below 2^14),
//   output scale   2^(T - 24) (undoes 2^13 2^(11 - T)).
// The rank factor is formed by ldexp of a finite value with a result below
// 2^13, so nothing overflows; ranks that vanish on the sub-box (a zero column
// or coefficient) get the factor 0. The power-of-two scheme of the LS_F16X3
// reconstruction, with the exponents kept as integers.
__device__ void f16_scales(const SysDev& S, int* ibuf) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = S.K;
  auto live = [&](int r) {
    return S.fmax[r] > 0.0 && S.fmax[K + r] > 0.0 && S.fmax[2 * K + r] > 0.0 &&
           isfinite(S.fmax[r]) && isfinite(S.fmax[K + r]) && isfinite(S.fmax[2 * K + r]) &&
           S.coef[r] != 0.0 && isfinite(S.coef[r]);
  };
  auto rexp = [&](int r) { return ilogb(S.fmax[r]) + ilogb(S.fmax[K + r]) + ilogb(S.fmax[2 * K + r]); };
  int T = INT_MIN;
  for (int r = tid; r < K; r += 256)
    if (live(r)) T = max(T, ilogb(fabs(S.coef[r])) + rexp(r));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) T = max(T, __shfl_xor(T, off, 64));
  if (lane == 0) ibuf[wv] = T;
  __syncthreads();
  T = max(max(ibuf[0], ibuf[1]), max(ibuf[2], ibuf[3]));
  __syncthreads();
  if (T == INT_MIN) T = 0;  // no live rank: every scale is 0
  for (int r = tid; r < K; r += 256) S.fsc[r] = live(r) ? ldexp(S.coef[r], 11 - T + rexp(r)) : 0.0;
  if (tid == 0) S.fsc[K] = ldexp(1.0, T - 24);
}

// One BM x BN tile of a sub-box for LS_F16X3: the left operand
// a.coef[r] f0[r][i] f1[r][j] is rounded to FP32 and split into two FP16
// terms in the tile (LDS, as split_tile), the right operand comes split from
// the VEC tasks (yp: per term and 32-rank chunk, 32 FP16 ranks of each
// column) and goes from global memory straight into the MFMA B fragments;
// products x0 y0 + x0 y1 + x1 y0 on the FP16 MFMA, FP32
// accumulation, out = a.scale * acc. smem holds f16_smem_bytes<BM>(): the
// split left operand in two buffers (chunk c in buffer c & 1), so one barrier
// per chunk suffices.
// The tile's rows lie in the values i0 .. ilast of i. With at most kTileNI of
// them (FAST: with BM = 128, every tile of a box with 43 or more values of
// j), the factor coef_r f0[r][i] of each of them and each rank of a chunk is
// formed once in LDS (alphaS[.][i - i0][r]) and a row reads its own, so
// staging loads only f1, without conditions, and those loads stay in flight
// through the chunk's MFMAs; otherwise (narrow boxes) each element also loads
// its f0 value. The two cases are separate loops, so that the waits the
// compiler places in the first do not follow the second's.

template <int BM>
constexpr int f16_smem_bytes() {
  return 2 * 2 * BM * 16 * 4 + 2 * kTileNI * (SPLIT_BK + 1) * 8;
}

template <int BM, int BN, int WM, int WN, int MF, bool FAST>
__device__ __forceinline__ void f16_tile_run(const BoxArg& a, int row0, int col0,
                                             float* __restrict__ out, char* smem,
                                             const uint4* __restrict__ yp) {
  constexpr int NT = 2, BK = SPLIT_BK;
  constexpr int KW = BK * BM / 256;
  static_assert(BM >= 64 && 256 % BM == 0, "staging map");
  static_assert((BM / WM) * (BN / WN) == 4, "four waves per workgroup");
  constexpr int FM = WM / MF, FN = WN / MF, NH = MF == 16 ? 1 : 2;
  typedef SplitMma<MF> Mma;
  constexpr int NI = kTileNI, AST = BK + 1;  // alphaS row stride: rows of i in other banks
  typedef unsigned WsT[NT][BM][16];
  static_assert(2 * sizeof(WsT) + 2 * NI * AST * sizeof(double) <= f16_smem_bytes<BM>(),
                "tile LDS");
  WsT* Wsb = reinterpret_cast<WsT*>(smem);
  double (*alphaS)[NI][AST] = reinterpret_cast<double (*)[NI][AST]>(smem + 2 * sizeof(WsT));

  const int M = a.e0 * a.e1, nch = (a.K + BK - 1) / BK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = (wave / (BN / WN)) * WM, wc = (wave % (BN / WN)) * WN;
  // a wave whose columns all lie past the sub-box (narrow boxes, the last
  // column tile) stages the left operand with the others but issues no
  // right-operand loads and no MFMAs (uniform per wave)
  const bool wlive = __builtin_amdgcn_readfirstlane(col0 + wc) < a.e2;
  const int mw = tid % BM;
  const int kbw = __builtin_amdgcn_readfirstlane(tid / BM) * KW;
  const int i0 = row0 / a.e1;
  const int ilast = (min(row0 + BM, M) - 1) / a.e1;
  constexpr bool wfast = FAST;
  const int m = row0 + mw;
  const bool mok = m < M;
  const int mi = mok ? m / a.e1 : i0;
  const int mj = mok ? m - mi * a.e1 : 0;
  const int islot = wfast ? mi - i0 : 0;  // this row's factors in alphaS
  const auto a1row = gmem(a.A1 + mi);
  const auto a2row = gmem(a.A2 + mj);
  const auto a1 = gmem(a.A1);
  const auto cf = gmem(a.coef);
  // f1 (FAST) and the split right operand through buffer resources: a
  // uniform (scalar) byte offset per rank row or chunk and a fixed 32-bit
  // offset per lane, so no per-lane 64-bit address arithmetic; f1 rows past
  // K read as 0
  const __amdgpu_buffer_rsrc_t a2buf = uniform_rsrc(a.A2, a.K * a.len1 * 8);
  const __amdgpu_buffer_rsrc_t ybuf = uniform_rsrc(yp, NT * nch * a.e2 * 64);
  const int woff = mj * 8;
  // this lane's B rows (output columns), clamped into the sub-box (columns
  // beyond it are computed from the last one and not stored)
  const int lr = lane & (MF - 1), lg = lane / MF;
  int brow[FN];
#pragma unroll
  for (int j = 0; j < FN; ++j) brow[j] = min(col0 + wc + MF * j + lr, a.e2 - 1);

  double w[KW];
  double cr = 0.0, ca = 1.0;
  // FAST: f1 values of ranks k0 + kbw + kk, without conditions (ranks past
  // K read as 0, rows past M are never stored); otherwise f1 f0
  auto load_w = [&](int k0) {
    if constexpr (FAST) {
      const int rs = __builtin_amdgcn_readfirstlane(a.len1 * 8);  // bytes per rank row
      const int s0 = __builtin_amdgcn_readfirstlane((k0 + kbw) * a.len1 * 8);
#pragma unroll
      for (int kk = 0; kk < KW; ++kk)
        w[kk] = __builtin_bit_cast(
            double, __builtin_amdgcn_raw_buffer_load_b64(a2buf, woff, s0 + kk * rs, 0));
      return;
    }
#pragma unroll
    for (int kk = 0; kk < KW; ++kk) {
      const int r = k0 + kbw + kk;
      double v = 0.0;
      if (r < a.K && mok) v = a2row[(size_t)r * a.len1] * a1row[(size_t)r * a.len0];
      w[kk] = v;
    }
  };
  // thread tid < NI BK: rank k0 + tid % BK and value i0 + tid / BK of i.
  // Loaded at clamped indices without conditions (so that no path through
  // the chunk loop has fewer loads in flight, which would make the waits for
  // the right operand wait for them too); aval says whether the factor is
  // used, else it is written as 0.
  const int ai = tid / BK, ar = tid % BK;
  bool aval = false;
  auto load_alpha = [&](int k0) {
    const int r = k0 + ar;
    aval = ai < NI && r < a.K && (FAST ? i0 + ai <= ilast : ai == 0);
    const int rc = min(r, a.K - 1);
    cr = cf[rc];
    if constexpr (FAST) ca = a1[(size_t)rc * a.len0 + min(i0 + min(ai, NI - 1), ilast)];
  };
  auto put_alpha = [&](int ab) {
    if (ai < NI) alphaS[ab][ai][ar] = aval ? cr * ca : 0.0;
  };
  auto store_w = [&](int ab) {
#pragma unroll
    for (int g = 0; g < KW / 8; ++g) {
      unsigned pk[NT][4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int kk = g * 8 + 2 * q;
        unsigned u0[NT], u1[NT];
        split_f16((float)(alphaS[ab][islot][kbw + kk] * w[kk]), u0);
        split_f16((float)(alphaS[ab][islot][kbw + kk + 1] * w[kk + 1]), u1);
#pragma unroll
        for (int t = 0; t < NT; ++t) pk[t][q] = pack_hi(u0[t], u1[t]);
      }
      const int slot = ((kbw >> 3) + g) ^ lds_swz(mw);
#pragma unroll
      for (int t = 0; t < NT; ++t)
        *reinterpret_cast<uint4*>(&Wsb[ab][t][mw][slot * 4]) = make_uint4(pk[t][0], pk[t][1], pk[t][2], pk[t][3]);
    }
  };
  typedef uint4 BFrag[NT][FN][NH];
  auto load_b = [&](int c, BFrag& bv) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int soff = __builtin_amdgcn_readfirstlane((t * nch + c) * a.e2 * 64);
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int h = 0; h < NH; ++h)
          bv[t][j][h] = __builtin_bit_cast(
              uint4, __builtin_amdgcn_raw_buffer_load_b128(ybuf, (brow[j] * 4 + NH * h + lg) * 16, soff, 0));
    }
  };

  typename Mma::acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < Mma::NV; ++v) acc[i][j][v] = 0.0f;

  auto products = [&](const BFrag& bv, int ab) {
    int slot[NH];
#pragma unroll
    for (int h = 0; h < NH; ++h) slot[h] = ((NH * h + lg) ^ lds_swz(lr)) * 4;
#pragma unroll
    for (int ta = NT - 1; ta >= 0; --ta) {
      s8_t av[FM][NH];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int h = 0; h < NH; ++h)
          av[i][h] = *reinterpret_cast<const s8_t*>(&Wsb[ab][ta][wr + MF * i + lr][slot[h]]);
#pragma unroll
      for (int tb = NT - 1 - ta; tb >= 0; --tb)
#pragma unroll
        for (int h = 0; h < NH; ++h)
#pragma unroll
          for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
              if constexpr (MF == 16)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(
                    __builtin_bit_cast(h8_t, av[i][h]), __builtin_bit_cast(h8_t, bv[tb][j][h]),
                    acc[i][j], 0, 0, 0);
              else
                acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                    __builtin_bit_cast(h8_t, av[i][h]), __builtin_bit_cast(h8_t, bv[tb][j][h]),
                    acc[i][j], 0, 0, 0);
            }
    }
  };
  // The right operand's fragments of chunk c + 1 are requested before the
  // products of chunk c (two register sets, the loop unrolled by two), so
  // that a whole chunk covers their latency; at the last chunk the request
  // repeats it (every path through the loop has the same loads in flight).
  BFrag bv0, bv1;
  load_alpha(0);
  put_alpha(0);
  load_alpha(BK);
  load_w(0);
  if (wlive) load_b(0, bv0);
  __syncthreads();
  // chunk c: its left operand goes to buffer c & 1, which the products of
  // chunk c - 2 read before the previous barrier; its rank factors were
  // written to alphaS[c & 1] before that barrier, and alphaS[(c + 1) & 1] was
  // last read by the staging of chunk c - 1, also before it
  auto step = [&](int c, const BFrag& cur, BFrag& nxt) {
    store_w(c & 1);
    put_alpha((c + 1) & 1);
    __syncthreads();
    // FAST: unconditional (past the last chunk the buffer reads 0), for the
    // same reason as the rank factors
    if (FAST || c + 1 < nch) load_w((c + 1) * BK);
    load_alpha((c + 2) * BK);
    if (wlive) load_b(min(c + 1, nch - 1), nxt);
    // keep these loads ahead of the MFMAs (the scheduler would otherwise sink
    // them below, and the next chunk would wait for them)
    __builtin_amdgcn_sched_barrier(0);
    if (wlive) products(cur, c & 1);
  };
  for (int c = 0; c < nch; c += 2) {
    step(c, bv0, bv1);
    if (c + 1 < nch) step(c + 1, bv1, bv0);
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

template <int BM, int BN, int WM, int WN, int MF>
__device__ __forceinline__ void f16_tile(const BoxArg& a, int row0, int col0,
                                         float* __restrict__ out, char* smem,
                                         const uint4* __restrict__ yp) {
  const int M = a.e0 * a.e1;
  const int i0 = row0 / a.e1, ilast = (min(row0 + BM, M) - 1) / a.e1;
  if (ilast - i0 < kTileNI)
    f16_tile_run<BM, BN, WM, WN, MF, true>(a, row0, col0, out, smem, yp);
  else
    f16_tile_run<BM, BN, WM, WN, MF, false>(a, row0, col0, out, smem, yp);
}

// NT = 0: FP64 / FP32 tiles (recon_tile<T>); NT = 2, 3: split tiles with NT
// terms (split_tile, FP32 output, MFMA shape MF): bf16 terms (FMT = 0) or, for
// LS_F16X3, scaled FP16 terms (FMT = 1).
template <typename T, int BM, int BN, int WM, int WN, int BK, int NT = 0, int MF = 16, int FMT = 0>
__global__ __launch_bounds__(256, 2) void k_batch(BatchArg ba) {
  constexpr int RB = FMT == 1 ? f16_smem_bytes<BM>()
                   : NT ? split_smem_bytes<NT, BM, BN, 1>() : recon_smem_bytes<T, BM, BN, BK>();
  constexpr int VB = kVecSmem;
  __shared__ __attribute__((aligned(16))) char smem[RB > VB ? RB : VB];
  __shared__ int s_task, s_flag;
  const int home = blockIdx.x & (kBatchQueues - 1);
  int tried = 0;  // thread 0: queues found empty so far (home first, then the next ones)
  for (;;) {
    if (threadIdx.x == 0) {
      int t = -1;
      while (tried < kBatchQueues) {
        const int q = (home + tried) & (kBatchQueues - 1);
        const int k = atomicAdd(&ba.qhead[q], 1);
        if (k < ba.qstart[q + 1] - ba.qstart[q]) {
          t = ba.qstart[q] + k;
          break;
        }
        ++tried;
      }
      s_task = t;
    }
    __syncthreads();
    // wave-uniform task index: descriptor loads become scalar loads
    const int t = __builtin_amdgcn_readfirstlane(s_task);
    __syncthreads();
    if (t < 0) return;
    const Task tk = ba.tasks[t];
    const SysDev& S = ba.sys[tk.sys];
    if (threadIdx.x == 0) {
      const unsigned long long now = wall_clock64();
      atomicMin(&ba.t_start[tk.sys], now);
      atomicMin(&ba.t_phase[2 * tk.type], now);
    }
    if (tk.type == TASK_FOLD) {
      fold_task(S, tk.a);
      signal_counter(&ba.fold_done[tk.sys]);
      if (threadIdx.x == 0) atomicMax(&ba.t_phase[1], (unsigned long long)wall_clock64());
    } else if (tk.type == TASK_VEC) {
      if (!wait_counter(&ba.fold_done[tk.sys], 3, ba.err, &s_flag)) continue;
      vec_task(S, ba, tk.a, reinterpret_cast<double*>(smem));
      const int prev = signal_counter(&ba.vec_done[tk.sys]);
      if (threadIdx.x == 0) s_flag = (prev == S.nvec - 1) ? 1 : 0;
      __syncthreads();
      if (s_flag) {
        // the system's last VEC task: energy and FP16 scales, then the second
        // signal that its TILE tasks wait for (count nvec + 1)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        energy_task(S, reinterpret_cast<double*>(smem));
        if (ba.f16) f16_scales(S, reinterpret_cast<int*>(smem));
        signal_counter(&ba.vec_done[tk.sys]);
        if (threadIdx.x == 0) atomicMax(&ba.t_end[tk.sys], (unsigned long long)wall_clock64());
      }
      if (threadIdx.x == 0) atomicMax(&ba.t_phase[3], (unsigned long long)wall_clock64());
    } else {
      if (!wait_counter(&ba.vec_done[tk.sys], S.nvec + 1, ba.err, &s_flag)) continue;
      BoxArg a;
      a.A1 = S.Fc[0];
      a.A2 = S.Fc[1];
      a.A3 = S.Fc[2];
      a.coef = S.coef;
      a.K = S.K;
      a.len0 = S.e[0];
      a.len1 = S.e[1];
      a.len2 = S.e[2];
      a.o0 = a.o1 = a.o2 = 0;
      a.e0 = S.e[0];
      a.e1 = S.e[1];
      a.e2 = S.e[2];
      a.scale = 1.0 / (S.h * S.h * S.h);
      const int tm = tk.a / S.tiles_n, tn = tk.a - tm * S.tiles_n;
      if constexpr (NT == 0) {
        recon_tile<T, BM, BN, WM, WN, BK>(a, tm * BM, tn * BN, reinterpret_cast<T*>(S.out), smem);
      } else if constexpr (FMT == 1) {
        a.coef = S.fsc;
        a.scale *= S.fsc[S.K];
        f16_tile<BM, BN, WM, WN, MF>(a, tm * BM, tn * BN, reinterpret_cast<float*>(S.out), smem, S.yp);
      } else {
        split_tile<NT, BM, BN, WM, WN, 1, MF>(a, tm * BM, tn * BN, reinterpret_cast<float*>(S.out),
                                              smem);
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        const unsigned long long now = wall_clock64();
        atomicMax(&ba.t_end[tk.sys], now);
        atomicMax(&ba.t_phase[5], now);
      }
    }
  }
}

__global__ void k_batch_reset(BatchArg ba) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kBatchQueues) ba.qhead[i] = 0;
  if (i == 0) *ba.err = 0;
  if (i < 3) {
    ba.t_phase[2 * i] = ~0ull;
    ba.t_phase[2 * i + 1] = 0ull;
  }
  if (i < ba.nsys) {
    ba.fold_done[i] = 0;
    ba.vec_done[i] = 0;
    ba.t_start[i] = ~0ull;
    ba.t_end[i] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct TileCfg {
  int bm, bn;
  const void* fn;
};

template <typename T>
static bool batch_tile(int tile, TileCfg* c) {
#define LS_BT(ID, BM_, BN_, WM_, WN_, BK_)                                \
  if (tile == ID) {                                                      \
    c->bm = BM_;                                                         \
    c->bn = BN_;                                                         \
    c->fn = (const void*)&k_batch<T, BM_, BN_, WM_, WN_, BK_>;           \
    return true;                                                         \
  }
  LS_BT(1, 128, 128, 64, 64, 16)
  LS_BT(2, 64, 64, 32, 32, 16)
  LS_BT(3, 128, 64, 64, 32, 16)
  LS_BT(4, 64, 128, 32, 64, 16)
#undef LS_BT
  return false;
}

// split-bf16 tiles: the in-kernel split of k_recon_split (tiles 1..4 there)
template <int NT>
static bool batch_tile_split(int tile, TileCfg* c) {
#define LS_BS(ID, BM_, BN_, WM_, WN_, MF_)                                 \
  if (tile == ID) {                                                      \
    c->bm = BM_;                                                         \
    c->bn = BN_;                                                         \
    c->fn = (const void*)&k_batch<float, BM_, BN_, WM_, WN_, 16, NT, MF_>; \
    return true;                                                         \
  }
  LS_BS(1, 128, 128, 64, 64, 16)
  LS_BS(2, 128, 128, 64, 64, 32)
  LS_BS(3, 128, 64, 64, 32, 32)
  LS_BS(4, 64, 128, 32, 64, 32)
#undef LS_BS
  return false;
}

// LS_F16X3 tiles (f16_tile)
static bool batch_tile_f16(int tile, TileCfg* c) {
#define LS_BH(ID, BM_, BN_, WM_, WN_, MF_)                                    \
  if (tile == ID) {                                                         \
    c->bm = BM_;                                                            \
    c->bn = BN_;                                                            \
    c->fn = (const void*)&k_batch<float, BM_, BN_, WM_, WN_, 16, 2, MF_, 1>; \
    return true;                                                            \
  }
  LS_BH(1, 128, 128, 64, 64, 16)
  LS_BH(2, 128, 128, 64, 64, 32)
  // the four waves side by side (128 rows x 32 columns each): no two waves
  // load the same right-operand fragments
  LS_BH(3, 128, 128, 128, 32, 16)
  LS_BH(4, 128, 128, 128, 32, 32)
#undef LS_BH
  return false;
}

static bool get_tile(int precision, int tile, TileCfg* c) {
  if (precision == LS_F64) return batch_tile<double>(tile, c);
  if (precision == LS_F32) return batch_tile<float>(tile, c);
  if (precision == LS_BF16X3) return batch_tile_split<2>(tile, c);
  if (precision == LS_BF16X6) return batch_tile_split<3>(tile, c);
  if (precision == LS_F16X3) return batch_tile_f16(tile, c);
  return false;
}
constexpr int kBatchTiles = 4;
#ifndef LS_BATCH_GROUP
#define LS_BATCH_GROUP 64
#endif
constexpr int kBatchGroup = LS_BATCH_GROUP;  // systems per pipeline stage, over all queues

struct SysHost {
  SysDev d;             // pointers into ws are offsets until bound
  size_t off_phi, off_g, off_fc[3], off_coef, off_fmax, off_fsc, off_yp;
  double cost;
};

}  // namespace ls

struct ls_batch {
  int precision;
  int count;
  std::vector<ls::SysHost> sys;
  std::vector<double> tau, w, qhw, qk;
  size_t off_ctrl, off_fold, off_vec, off_ts, off_te, off_sys, off_tau, off_w, off_hw, off_k, off_tasks,
      ws_bytes;
  // per bound tile: tasks differ only in the tile split of TILE tasks
  int bound_tile = -1;
  void* bound_ws = nullptr;
  int ntasks = 0;
  int qstart[ls::kBatchQueues + 1] = {};
  int best_tile = 0;
  uint64_t shape_key = 0;  // autotune cache key: precision and the multiset of system shapes
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<ls::Task> tasks;
  std::vector<ls::SysDev> devsys;
  ls::BatchArg arg;  // kernel-node arguments (kept alive with the graph)
};

namespace ls {

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

static ls_status build_tasks(ls_batch* B, int tile, TileCfg* cfg) {
  if (!get_tile(B->precision, tile, cfg)) {
    set_error("tile %d not available for the batch precision", tile);
    return LS_EUNSUPPORTED;
  }
  // Systems in decreasing cost (LPT), dealt to the queue with the least cost
  // so far. Each queue is a three-stage software pipeline over groups of its
  // systems (kBatchGroup / kBatchQueues each): chunk t holds the FOLD tasks of
  // group t, the VEC tasks of group t - 1 and the TILE tasks of group t - 2.
  // Every task still waits only on tasks of earlier chunks of its queue (its
  // system's FOLDs one chunk before its VECs, the VECs one chunk before its
  // TILEs), which running workgroups dequeued earlier, so every wait ends;
  // the chunk of other work between the stages covers most of the waiting,
  // and each system finishes about two chunks after it starts, so the
  // per-system times measure the system, not the whole queue.
  std::vector<int> order(B->count);
  for (int i = 0; i < B->count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return B->sys[a].cost > B->sys[b].cost; });
  std::vector<int> queue[kBatchQueues];
  double load[kBatchQueues] = {};
  for (int i : order) {
    int q = 0;
    for (int k = 1; k < kBatchQueues; ++k)
      if (load[k] < load[q]) q = k;
    queue[q].push_back(i);
    load[q] += B->sys[i].cost;
  }
  const int gsize = std::max(1, kBatchGroup / kBatchQueues);
  B->tasks.clear();
  for (int q = 0; q < kBatchQueues; ++q) {
    B->qstart[q] = (int)B->tasks.size();
    const std::vector<int>& sq = queue[q];
    const int ngroups = ((int)sq.size() + gsize - 1) / gsize;
    auto group = [&](int g, auto&& emit) {
      if (g < 0 || g >= ngroups) return;
      for (int k = g * gsize; k < std::min((int)sq.size(), (g + 1) * gsize); ++k) emit(sq[k]);
    };
    for (int t = 0; t < ngroups + 2; ++t) {
      group(t, [&](int i) {
        for (int l = 0; l < 3; ++l) B->tasks.push_back({TASK_FOLD, i, l, 0});
      });
      group(t - 1, [&](int i) {
        for (int c = 0; c < 3 * B->sys[i].d.M0; ++c) B->tasks.push_back({TASK_VEC, i, c, 0});
      });
      group(t - 2, [&](int i) {
        SysDev& d = B->sys[i].d;
        const long long M = (long long)d.e[0] * d.e[1];
        const int tm = (int)((M + cfg->bm - 1) / cfg->bm);
        d.tiles_n = (d.e[2] + cfg->bn - 1) / cfg->bn;
        for (int t2 = 0; t2 < tm * d.tiles_n; ++t2) B->tasks.push_back({TASK_TILE, i, t2, 0});
      });
    }
  }
  B->qstart[kBatchQueues] = (int)B->tasks.size();
  B->ntasks = (int)B->tasks.size();
  return LS_OK;
}

static BatchArg make_arg(ls_batch* B, char* ws) {
  BatchArg a;
  a.sys = (const SysDev*)(ws + B->off_sys);
  a.tasks = (const Task*)(ws + B->off_tasks);
  a.tau = (const double*)(ws + B->off_tau);
  a.w = (const double*)(ws + B->off_w);
  a.qhw = (const double*)(ws + B->off_hw);
  a.qk = (const double*)(ws + B->off_k);
  a.qhead = (int*)(ws + B->off_ctrl + 128);
  a.err = (int*)(ws + B->off_ctrl) + 1;
  a.fold_done = (int*)(ws + B->off_fold);
  a.vec_done = (int*)(ws + B->off_vec);
  a.t_start = (unsigned long long*)(ws + B->off_ts);
  a.t_end = (unsigned long long*)(ws + B->off_te);
  a.t_phase = (unsigned long long*)(ws + B->off_ctrl + 64);
  for (int q = 0; q <= kBatchQueues; ++q) a.qstart[q] = B->qstart[q];
  a.nsys = B->count;
  a.f16 = B->precision == LS_F16X3 ? 1 : 0;
  return a;
}

// Upload descriptors for (ws, tile) and build the graph [reset -> k_batch].
static ls_status bind(ls_batch* B, void* ws_dev, int tile, hipStream_t stream) {
  if (B->bound_ws == ws_dev && B->bound_tile == tile && B->exec) return LS_OK;
  TileCfg cfg;
  ls_status st = build_tasks(B, tile, &cfg);
  if (st != LS_OK) return st;
  const size_t task_bytes = sizeof(Task) * B->tasks.size();
  if (B->off_tasks + task_bytes > B->ws_bytes) {
    set_error("internal: task list exceeds the planned workspace");
    return LS_EWORKSPACE;
  }
  char* ws = (char*)ws_dev;
  B->devsys.resize(B->count);
  for (int i = 0; i < B->count; ++i) {
    SysDev d = B->sys[i].d;
    d.Phi = (double*)(ws + B->sys[i].off_phi);
    d.G = (double*)(ws + B->sys[i].off_g);
    for (int l = 0; l < 3; ++l) d.Fc[l] = (double*)(ws + B->sys[i].off_fc[l]);
    d.coef = (double*)(ws + B->sys[i].off_coef);
    d.fmax = (double*)(ws + B->sys[i].off_fmax);
    d.fsc = (double*)(ws + B->sys[i].off_fsc);
    d.yp = (uint4*)(ws + B->sys[i].off_yp);
    B->devsys[i] = d;
  }
  hipError_t e = hipMemcpyAsync(ws + B->off_sys, B->devsys.data(), sizeof(SysDev) * B->count,
                                hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + B->off_tasks, B->tasks.data(), task_bytes, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + B->off_tau, B->tau.data(), sizeof(double) * B->tau.size(),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + B->off_w, B->w.data(), sizeof(double) * B->w.size(),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + B->off_hw, B->qhw.data(), sizeof(double) * B->qhw.size(),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ws + B->off_k, B->qk.data(), sizeof(double) * B->qk.size(),
                       hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    set_error("batch descriptor upload: %s", hipGetErrorString(e));
    return LS_EHIP;
  }
  if (B->exec) {
    (void)hipStreamSynchronize(stream);
    (void)hipGraphExecDestroy(B->exec);
    B->exec = nullptr;
  }
  if (B->graph) {
    (void)hipGraphDestroy(B->graph);
    B->graph = nullptr;
  }
  int dev = 0, ncu = 0, per_cu = 0;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, cfg.fn, 256, 0);
  if (e != hipSuccess || ncu <= 0) {
    set_error("device query: %s", hipGetErrorString(e));
    return LS_EHIP;
  }
  if (per_cu < 1) per_cu = 1;
  B->arg = make_arg(B, ws);
  void* params[] = {&B->arg};
  e = hipGraphCreate(&B->graph, 0);
  hipGraphNode_t n_reset = nullptr, n_main = nullptr;
  if (e == hipSuccess) {
    hipKernelNodeParams kp = {};
    kp.func = (void*)&k_batch_reset;
    kp.gridDim = dim3((B->count + 255) / 256);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = params;
    kp.extra = nullptr;
    e = hipGraphAddKernelNode(&n_reset, B->graph, nullptr, 0, &kp);
  }
  if (e == hipSuccess) {
    hipKernelNodeParams kp = {};
    kp.func = (void*)cfg.fn;
    kp.gridDim = dim3(ncu * per_cu);
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = params;
    kp.extra = nullptr;
    e = hipGraphAddKernelNode(&n_main, B->graph, &n_reset, 1, &kp);
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    set_error("batch graph: %s", hipGetErrorString(e));
    return LS_EHIP;
  }
  B->bound_ws = ws_dev;
  B->bound_tile = tile;
  return LS_OK;
}

}  // namespace ls

using namespace ls;

// ---------------------------------------------------------------------------
// autotune cache: the fastest tile per (precision, shape class), where the
// shape class is the multiset of the systems' shapes (n, L, M0, R, density
// rank, sub-box extents), hashed (FNV-1a, 64 bits) in a canonical order. It
// lives in the process and, once ls_batch_cache_file names a file, in that
// text file too (one "key precision tile ms" line per entry, rewritten on
// every new entry).
// ---------------------------------------------------------------------------
namespace {
struct TuneEntry {
  int precision, tile;
  double ms;
};
std::mutex g_tune_mu;
std::map<uint64_t, TuneEntry> g_tune;
std::string g_tune_path;

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

void tune_save_locked() {
  if (g_tune_path.empty()) return;
  FILE* f = fopen(g_tune_path.c_str(), "w");
  if (f == nullptr) return;  // the in-process cache still holds the entry
  for (const auto& kv : g_tune)
    fprintf(f, "%016llx %d %d %.6f\n", (unsigned long long)kv.first, kv.second.precision,
            kv.second.tile, kv.second.ms);
  fclose(f);
}
}  // namespace

extern "C" ls_status ls_batch_cache_file(const char* path) {
  clear_error();
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
  g_tune_path = path ? path : "";
  if (path == nullptr) return LS_OK;
  FILE* f = fopen(path, "r");
  if (f == nullptr) return LS_OK;  // a new file: written by the next autotune
  unsigned long long key;
  int prec, tile;
  double ms;
  while (fscanf(f, "%llx %d %d %lf", &key, &prec, &tile, &ms) == 4)
    if (tile >= 1 && tile <= kBatchTiles) g_tune[(uint64_t)key] = TuneEntry{prec, tile, ms};
  fclose(f);
  return LS_OK;
}

extern "C" ls_status ls_batch_tuned_tile(ls_batch_t B, int32_t* tile, double* ms) {
  clear_error();
  LS_REQUIRE(B != nullptr && tile != nullptr, "null pointer");
  *tile = 0;
  if (ms) *ms = 0.0;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  const auto it = g_tune.find(B->shape_key);
  if (it != g_tune.end()) {
    *tile = it->second.tile;
    if (ms) *ms = it->second.ms;
  }
  return LS_OK;
}

extern "C" ls_status ls_batch_create(const ls_system* systems, int32_t count, int32_t precision,
                                     ls_batch_t* batch, size_t* ws_bytes) {
  clear_error();
  LS_REQUIRE(systems != nullptr && batch != nullptr && ws_bytes != nullptr, "null pointer");
  LS_REQUIRE(count >= 1 && count <= (1 << 20), "count must be in [1, 2^20]");
  if (precision < LS_F64 || precision > LS_F16X3) {
    set_error("unknown batch precision %d", precision);
    return LS_EUNSUPPORTED;
  }
  ls_batch* B = new ls_batch();
  B->precision = precision;
  B->count = count;
  B->sys.resize(count);
  size_t off = 0;
  B->off_ctrl = off;  // err at +4; phase stamps [6] u64 at +64; queue heads [8] at +128
  off += al(256);
  B->off_fold = off;
  off += al(sizeof(int) * count);
  B->off_vec = off;
  off += al(sizeof(int) * count);
  B->off_ts = off;
  off += al(8 * (size_t)count);
  B->off_te = off;
  off += al(8 * (size_t)count);
  B->off_sys = off;
  off += al(sizeof(SysDev) * (size_t)count);
  size_t nq = 0, max_tasks = 0;
  for (int i = 0; i < count; ++i) {
    const ls_system& S = systems[i];
    Lat L;
    ls_status st = check_lattice(&S.lat, &L);
    QuadArg qa;
    if (st == LS_OK) st = check_quad(&S.quad, L.h, &qa);
    if (st != LS_OK) {
      delete B;
      return st;
    }
    auto fail = [&](const char* msg) {
      set_error("system %d: %s", i, msg);
      delete B;
      return LS_EINVAL;
    };
    if (L.periodic) return fail("batches hold box lattices");
    if (S.M0 < 1 || S.M0 > 20000) return fail("M0 out of range");
    if (!S.pos_dev || !S.Z_dev || !S.out_dev || !S.E_dev) return fail("null device pointer");
    if (S.rho.K < 1 || S.rho.K > kBatchRho || !S.rho.coef) return fail("density rank not in [1, 8]");
    for (int l = 0; l < 3; ++l) {
      if (!S.rho.f[l] || S.rho.len[l] != L.N[l]) return fail("density length != grid");
      if (S.box.e[l] < 1 || S.box.e[l] > L.n || S.box.e[l] > 256 || S.box.o[l] < 0 ||
          S.box.o[l] + S.box.e[l] > L.N[l])
        return fail("sub-box must lie in the grid with extent in [1, min(n, 256)] per axis");
    }
    SysHost& h = B->sys[i];
    SysDev& d = h.d;
    memset(&d, 0, sizeof(d));
    d.b = L.b;
    d.h = L.h;
    d.n = L.n;
    for (int l = 0; l < 3; ++l) {
      d.L[l] = L.L[l];
      d.N[l] = L.N[l];
      d.o[l] = S.box.o[l];
      d.e[l] = S.box.e[l];
      d.D[l] = S.rho.f[l];
    }
    d.M0 = S.M0;
    d.R = qa.R;
    d.K = S.M0 * qa.R;
    d.Krho = S.rho.K;
    d.qoff = (int)nq;
    d.X = master_halfwidth(L);
    d.W = 2 * d.X + L.n;
    // the tiles and the vector tasks address the factor columns and the folded
    // density through buffer resources with 32-bit byte offsets
    if ((long long)d.K * 256 * 8 >= (1LL << 31) || (long long)d.Krho * d.W * 8 >= (1LL << 31))
      return fail("factor columns or folded density of 2 GB or more");
    d.nvec = 3 * S.M0;
    d.pos = S.pos_dev;
    d.Z = S.Z_dev;
    d.d = S.rho.coef;
    d.out = S.out_dev;
    d.E = S.E_dev;
    for (int q = 0; q < qa.R; ++q) {
      const double tau = qa.tau[q];
      B->tau.push_back(tau);
      B->w.push_back(qa.w[q]);
      // the device's support_halfwidth and cell_half_norm (IEEE division on
      // both sides: the same values)
      B->qhw.push_back(tau > 0.0 ? 28.0 / tau + 2.0 : 1e300);
      B->qk.push_back(0.88622692545275801365 / tau);
    }
    nq += qa.R;
    h.off_phi = off;
    off += al(sizeof(double) * 3 * (size_t)d.Krho * d.W);
    h.off_g = off;
    off += al(sizeof(double) * 3 * (size_t)d.K * d.Krho);
    for (int l = 0; l < 3; ++l) {
      h.off_fc[l] = off;
      off += al(sizeof(double) * (size_t)d.K * d.e[l]);
    }
    h.off_coef = off;
    off += al(sizeof(double) * (size_t)d.K);
    h.off_fmax = off;
    off += al(sizeof(double) * 3 * (size_t)d.K);
    h.off_fsc = off;
    off += al(sizeof(double) * ((size_t)d.K + 1));
    h.off_yp = off;
    if (precision == LS_F16X3) off += al(2 * (size_t)((d.K + 31) / 32) * d.e[2] * 64);
    h.cost = (double)d.K * (2.0 * d.X) + 2.0 * d.K * (double)d.e[0] * d.e[1] * d.e[2] / 64.0;
    // task count bound: smallest tile 64x64
    max_tasks += 3 + 3 * (size_t)S.M0 +
                 (size_t)(((long long)d.e[0] * d.e[1] + 63) / 64) * ((d.e[2] + 63) / 64);
  }
  B->off_tau = off;
  off += al(sizeof(double) * nq);
  B->off_w = off;
  off += al(sizeof(double) * nq);
  B->off_hw = off;
  off += al(sizeof(double) * nq);
  B->off_k = off;
  off += al(sizeof(double) * nq);
  B->off_tasks = off;
  off += al(sizeof(Task) * max_tasks);
  B->ws_bytes = off;
  // shape class for the autotune cache
  std::vector<std::array<int32_t, 10>> shapes(count);
  for (int i = 0; i < count; ++i) {
    const SysDev& d = B->sys[i].d;
    shapes[i] = {d.n, d.L[0], d.L[1], d.L[2], d.M0, d.R, d.Krho, d.e[0], d.e[1], d.e[2]};
  }
  std::sort(shapes.begin(), shapes.end());
  uint64_t key = 1469598103934665603ull;
  key = fnv1a(key, &precision, sizeof(precision));
  key = fnv1a(key, shapes.data(), shapes.size() * sizeof(shapes[0]));
  B->shape_key = key;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    const auto it = g_tune.find(key);
    if (it != g_tune.end()) B->best_tile = it->second.tile;
  }
  *ws_bytes = off;
  *batch = B;
  return LS_OK;
}

extern "C" int32_t ls_batch_tiles(void) { return kBatchTiles; }

extern "C" ls_status ls_batch_run(ls_batch_t B, void* ws_dev, size_t ws_bytes, int32_t tile,
                                  hipStream_t stream) {
  clear_error();
  LS_REQUIRE(B != nullptr, "null batch");
  if (ws_dev == nullptr || ws_bytes < B->ws_bytes) {
    set_error("workspace of %zu bytes required", B->ws_bytes);
    return LS_EWORKSPACE;
  }
  LS_REQUIRE(ws_aligned(ws_dev), "the workspace must be 256-byte aligned");
  if (tile == 0) tile = B->best_tile ? B->best_tile : 2;
  ls_status st = bind(B, ws_dev, tile, stream);
  if (st != LS_OK) return st;
  hipError_t e = hipGraphLaunch(B->exec, stream);
  if (e != hipSuccess) {
    set_error("batch graph launch: %s", hipGetErrorString(e));
    return LS_EHIP;
  }
  return LS_OK;
}

extern "C" ls_status ls_batch_autotune(ls_batch_t B, void* ws_dev, size_t ws_bytes,
                                       hipStream_t stream, int32_t* best, double* best_ms) {
  clear_error();
  LS_REQUIRE(B != nullptr && best != nullptr, "null pointer");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    set_error("event creation failed");
    return LS_EHIP;
  }
  float best_t = 1e30f;
  int best_id = 0;
  ls_status st = LS_OK;
  for (int t = 1; t <= kBatchTiles && st == LS_OK; ++t) {
    st = ls_batch_run(B, ws_dev, ws_bytes, t, stream);  // warm (binds the graph)
    if (st != LS_OK) break;
    (void)hipEventRecord(e0, stream);
    st = ls_batch_run(B, ws_dev, ws_bytes, t, stream);
    (void)hipEventRecord(e1, stream);
    if (hipEventSynchronize(e1) != hipSuccess) {
      set_error("autotune synchronisation failed");
      st = LS_EHIP;
      break;
    }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_t) {
      best_t = ms;
      best_id = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != LS_OK) return st;
  B->best_tile = best_id;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune[B->shape_key] = TuneEntry{B->precision, best_id, (double)best_t};
    tune_save_locked();
  }
  *best = best_id;
  if (best_ms) *best_ms = best_t;
  return LS_OK;
}

extern "C" ls_status ls_batch_report(ls_batch_t B, const void* ws_dev, double* seconds,
                                     double* phase_seconds, int32_t* error_flag) {
  clear_error();
  LS_REQUIRE(B != nullptr && ws_dev != nullptr, "null pointer");
  const char* ws = (const char*)ws_dev;
  std::vector<unsigned long long> ts(B->count), te(B->count);
  int ctrl[2] = {0, 0};
  hipError_t e = hipMemcpy(ts.data(), ws + B->off_ts, 8 * (size_t)B->count, hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(te.data(), ws + B->off_te, 8 * (size_t)B->count, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(ctrl, ws + B->off_ctrl, sizeof(ctrl), hipMemcpyDeviceToHost);
  unsigned long long ph[6] = {0, 0, 0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpy(ph, ws + B->off_ctrl + 64, sizeof(ph), hipMemcpyDeviceToHost);
  int dev = 0, khz = 0;
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess || khz <= 0) {
    set_error("batch report: %s", hipGetErrorString(e));
    return LS_EHIP;
  }
  if (seconds)
    for (int i = 0; i < B->count; ++i)
      seconds[i] = (te[i] >= ts[i] && ts[i] != ~0ull) ? (double)(te[i] - ts[i]) / (khz * 1e3) : -1.0;
  if (phase_seconds)
    for (int k = 0; k < 3; ++k)
      phase_seconds[k] = (ph[2 * k + 1] >= ph[2 * k] && ph[2 * k] != ~0ull)
                             ? (double)(ph[2 * k + 1] - ph[2 * k]) / (khz * 1e3)
                             : 0.0;
  if (error_flag) *error_flag = ctrl[1];
  return LS_OK;
}

extern "C" void ls_batch_destroy(ls_batch_t B) {
  if (!B) return;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  delete B;
}
