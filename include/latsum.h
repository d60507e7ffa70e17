/*
 * latsum: assembled canonical-tensor lattice summation of Newton potentials
 * on one AMD Instinct MI355X (gfx950).
 *
 * Method: V. Khoromskaia, B. N. Khoromskij, "Grid-based lattice summation of
 * electrostatic potentials by assembled rank-structured tensor approximation"
 * (arXiv 1405.2270). Section, equation and theorem labels below are the
 * paper's.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Unit cell [-b/2, b/2]^3, n cells of size h = b/n per edge (Sec. 2.1).
 *    Box case: lattice shifts b*k, k_l = 0..L_l-1; the grid of axis l has
 *    N_l = L_l * n cells, cell g spanning [-b/2 + g h, -b/2 + (g+1) h]
 *    (Sec. 3.1, eq. N0grid). Periodic case: only the reference cell is
 *    resolved (N_l = n) and the images are k = -p..p for L = 2p+1, and
 *    -L/2..L/2-1 for even L (Sec. 3.2, eq. EwaldSumP, Lemma 3.2).
 *  - Charges: M0 positions a_nu in physical coordinates inside the unit cell,
 *    row-major [M0][3] FP64, and charges Z_nu [M0] FP64, both in device
 *    memory. Positions need not be grid nodes: every cell integral is taken
 *    at the continuous position.
 *  - Canonical format (Appendix, eq. CP_form): rank index r = nu*R + q;
 *    factor matrices f[l] are vector-contiguous [K][N_l] FP64 in device
 *    memory, and coef[r] = Z_nu w_q is kept apart, FP64.
 *  - Every pointer argument named *_dev is device memory owned by the caller;
 *    struct descriptors and other pointers are host memory read during the
 *    call only. The library allocates no device memory and keeps no pointer
 *    after a call returns (its one fixed device array, the scratch of
 *    ls_forces_noalloc, is part of the loaded library).
 *  - Workspaces (the ws_dev arguments) are 256-byte aligned, as hipMalloc
 *    returns them: the kernels read them with 16-byte vector loads at
 *    256-byte aligned offsets. A misaligned workspace is refused (LS_EINVAL).
 *  - Arguments are checked on the host before anything is enqueued; a
 *    failing check returns a negative ls_status and enqueues nothing.
 *    ls_last_error() then describes the failure (thread-local).
 *  - Work is enqueued on `stream` (0 = the null stream) and runs
 *    asynchronously; outputs are valid after the stream is synchronised.
 *    A launch failure returns LS_EHIP.
 */
#ifndef LATSUM_H
#define LATSUM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LS_OK = 0,
  LS_EINVAL = -1,        /* invalid argument */
  LS_EHIP = -2,          /* HIP runtime or launch error */
  LS_EUNSUPPORTED = -3,  /* valid but not implemented combination */
  LS_EWORKSPACE = -4     /* workspace missing or too small */
} ls_status;

typedef enum {
  LS_F64 = 0,     /* FP64 operands, FP64 MFMA, FP64 output */
  LS_F32 = 1,     /* operands rounded to FP32, FP32 MFMA, FP32 output */
  LS_BF16X3 = 2,  /* operands split into 2 bf16 terms, 3 bf16 MFMA products, FP32 accumulate/output */
  LS_BF16X6 = 3,  /* operands split into 3 bf16 terms, 6 bf16 MFMA products, FP32 accumulate/output */
  LS_F16X3 = 4    /* operands scaled per rank by powers of two and split into 2 FP16 terms,
                     3 FP16 MFMA products, FP32 accumulate/output (reconstruction only; needs
                     the workspace) */
} ls_precision;

typedef enum {
  LS_RULE_U = 0,  /* t_k = k h_M, w_k = h_M/sqrt(pi), k = -M..M (eqs. sinc_Newt, hM) */
  LS_RULE_S = 1   /* t_q = s sinh(q h_M), q = 0..M, folded (R = M+1) */
} ls_rule;

typedef struct {
  int32_t n;         /* grid cells per unit-cell edge, >= 1 */
  int32_t L[3];      /* lattice cells per axis, >= 1 */
  double b;          /* unit-cell edge length, > 0 */
  int32_t periodic;  /* 0: box (Theorem 3.1), 1: periodic reference cell (Lemma 3.2) */
} ls_lattice;

typedef struct {
  int32_t R;         /* number of quadrature terms = canonical rank of one kernel */
  const double* t;   /* host [R], nodes t_q (1/length); only t_q^2 is used */
  const double* w;   /* host [R], weights w_q (1/length) */
} ls_quad;

typedef struct {
  int32_t K;            /* rank */
  int32_t len[3];       /* vector length per axis */
  const double* f[3];   /* device [K][len[l]] FP64 factor matrices */
  const double* coef;   /* device [K] FP64 weights */
  const double* rowmax; /* device [3][K] or NULL: rowmax[l K + r] = max_x |f[l][r][x]| of these
                           factors, as ls_assemble writes it; LS_F16X3 reconstruction then
                           skips its own pass over the factors (a wrong maximum mis-scales the
                           FP16 terms); ignored elsewhere */
} ls_canon;

typedef struct {
  int32_t o[3];  /* origin in cells */
  int32_t e[3];  /* extent in cells, >= 1; o + e <= len per axis */
} ls_box;

/* Version string of the library. */
const char* ls_version(void);

/* Description of the last failure on the calling thread ("" if none). */
const char* ls_last_error(void);

/*
 * Quadrature table (Sec. 2.1, eqs. laplace, sinc_Newt, hM) on the host.
 * The printed weight h_M lacks the 1/sqrt(pi) of eq. laplace; it is included.
 *   rule U: h_M = C0 log(M)/M, t_k = k h_M, w_k = h_M/sqrt(pi), k = -M..M, R = 2M+1.
 *   rule S: h_M = C0 log(M)/M, t_q = s sinh(q h_M), w_0 = s h_M/sqrt(pi),
 *           w_q = 2 s h_M cosh(q h_M)/sqrt(pi), q = 0..M, R = M+1
 *           (the sinh-substituted sinc rule, folded over +-q).
 * t, w: host arrays of `capacity` doubles; *R receives the term count.
 * Errors: LS_EINVAL for M < 2, C0 <= 0, s <= 0 (rule S), unknown rule,
 * capacity < R or null pointers.
 */
ls_status ls_quadrature(int32_t rule, int32_t M, double C0, double s,
                        double* t, double* w, int32_t capacity, int32_t* R);

/*
 * Half-width X (cells) of the master grid (eq. master_pot generalised to the
 * lattice): master index j in [-X, X) covers every offset g - p - k n that an
 * assembled sum needs on any axis. Box: X = max_l N_l. Periodic:
 * X = (max_l L_l div 2 + 1) n. Host only.
 */
ls_status ls_master_halfwidth(const ls_lattice* lat, int32_t* X);

/*
 * Kernel vectors (Sec. 2.1, eqs. C_nD_0, galten_int; eq. master_pot):
 * for every atom nu, axis l and term q the master vector on 2X cells,
 *   masters_dev[((nu*3 + l)*R + q)*2X + j + X]
 *     = integral over [(j - delta) h, (j + 1 - delta) h] of exp(-t_q^2 y^2) dy,
 * where (a_{nu,l} + b/2)/h = p + delta with integer p and 0 <= delta < 1.
 * With derivative != 0 the entries are the derivatives of the same cell
 * integrals with respect to the charge position,
 *   exp(-t_q^2 ((j - delta) h)^2) - exp(-t_q^2 ((j + 1 - delta) h)^2).
 * All arithmetic is FP64. X must be ls_master_halfwidth(lat).
 * masters_dev: device, M0*3*R*2X doubles, written.
 * Errors: LS_EINVAL (null pointers, M0 < 1, R < 1, non-finite t or w, X mismatch).
 */
ls_status ls_kernel_vectors(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                            const double* pos_dev, int32_t X, int32_t derivative,
                            double* masters_dev, hipStream_t stream);

/*
 * Assembled canonical vectors (Theorem 3.1, eq. EwaldTensorM0 for the box;
 * Lemma 3.2 for the periodic cell): for r = nu*R + q and each axis l,
 *   f_l[r][g] = sum over images k of b_{g - p - k n}(t_q; delta),
 * i.e. the pointwise sum of shifted windows of the master vector, and
 * coef[r] = Z_nu w_q.
 * masters_dev: the output of ls_kernel_vectors for the same lattice and X, or
 * NULL to generate every cell integral in registers (L integrals per entry).
 * The periodic case always generates in registers, since each master entry is
 * used exactly once there; masters_dev must be NULL for it. With
 * derivative != 0 the vectors are position derivatives (masters must then be
 * derivative masters or NULL) and coef_dev may be NULL.
 * Box lattice without stored masters: when (2 L_l - 1) n <= 8192 and
 * L_l <= 64 on every axis, one workgroup per (atom, axis, q) generates the
 * master cells its vector needs in LDS (as ls_kernel_vectors does) and sums
 * them as from stored masters: the same factors bit for bit, without the
 * masters' trip through device memory (kernel vectors and assembly in one
 * launch). Larger box lattices generate L integrals per entry.
 * f0_dev, f1_dev, f2_dev: device [K][N_l] FP64, written. coef_dev: device [K].
 * rowmax_dev: device [3][K] or NULL; if given, rowmax[l K + r] = max_g
 * |f_l[r][g]| is written too (for ls_canon.rowmax).
 * Errors: LS_EINVAL.
 */
ls_status ls_assemble(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                      const double* pos_dev, const double* Z_dev, const double* masters_dev,
                      int32_t X, int32_t derivative, double* f0_dev, double* f1_dev,
                      double* f2_dev, double* coef_dev, double* rowmax_dev, hipStream_t stream);

/*
 * Non-equidistant tensor lattice (Sec. 3.1, remark after eq. EwaldTensorM0):
 * lattice points at arbitrary coordinates per axis, image (k0, k1, k2) of
 * atom nu at a_nu + h (s0[k0], s1[k1], s2[k2]). The 3D sum over every image
 * triple splits into per-axis sums as in Theorem 3.1, so the result keeps
 * rank K = M0 * R.
 */
typedef struct {
  int32_t n;            /* cells per unit-cell edge, h = b / n */
  double b;             /* unit-cell edge length, > 0 (positions as for ls_lattice) */
  int32_t N[3];         /* grid cells per axis, cell g of axis l spanning
                           [-b/2 + g h, -b/2 + (g+1) h]; 1 <= N[l] <= 2^26 */
  int32_t L[3];         /* lattice coordinates per axis, 1 <= L[l] <= 2^24 */
  const double* s[3];   /* device [L[l]]: lattice coordinates of axis l in units of
                           h, any real values, repeats allowed (the equidistant box
                           lattice is s_l[k] = k n) */
} ls_tensor_lattice;

/*
 * Assembled canonical vectors of a tensor lattice: for r = nu*R + q,
 *   f_l[r][g] = sum_k integral over cell g of exp(-t_q^2 (x - a_{nu,l} - h s_l[k])^2) dx,
 * coef[r] = Z_nu w_q (the per-axis sums of Theorem 3.1 with the windows
 * replaced by arbitrary shifts; each image's cell integrals at its own
 * continuous position, all arithmetic FP64). derivative != 0: position
 * derivatives of the same sums, coef_dev may be NULL.
 * f0_dev, f1_dev, f2_dev: device [K][N[l]] FP64, written; coef_dev: device [K].
 * Work per call: K (N0 L0 + N1 L1 + N2 L2) cell offsets, the cell integral
 * only where the Gaussian's support reaches the cell. A coordinate beyond
 * +-1e9 cells counts as +-1e9; a non-finite one gives NaN in its vectors.
 * Errors: LS_EINVAL (bad sizes, null pointers), LS_EUNSUPPORTED (R > 160).
 */
ls_status ls_assemble_tensor(const ls_tensor_lattice* tlat, const ls_quad* quad, int32_t M0,
                             const double* pos_dev, const double* Z_dev, int32_t derivative,
                             double* f0_dev, double* f1_dev, double* f2_dev, double* coef_dev,
                             hipStream_t stream);

/*
 * Reconstruction of sub-boxes of a canonical tensor (Appendix, eq. CP_form):
 *   out_b[i][j][k] = scale * sum_r coef[r] f0[r][o0+i] f1[r][o1+j] f2[r][o2+k]
 * for each box b, as one GEMM per box with rows (i, j), columns k and the
 * Khatri-Rao operand formed on the fly, on MFMA in the requested precision.
 * scale = 1/h^3 gives cell averages of the potential; 1 gives the raw tensor.
 * out_dev: device; boxes are stored one after another, each [e0][e1][e2]
 * C-order; element type double for LS_F64, float otherwise.
 * boxes: host [nbox]. tile: 0 = automatic (the tile ls_reconstruct_autotune
 * measured fastest for this call's shape class, else a built-in choice),
 * otherwise a tile id from 1 to ls_reconstruct_tiles(precision).
 * ws_dev, ws_bytes: device workspace, caller-owned, used by the split
 * precisions only: tiles 6 and above of LS_BF16X3 / LS_BF16X6 first split f1
 * into bf16 terms there (ls_reconstruct_workspace bytes); tile 0 uses them
 * when the workspace is large enough and the boxes are large (the persistent
 * kernel, one workgroup per resident slot, for boxes of 256 or more values of
 * j), and otherwise tiles that split both operands inside the kernel.
 * LS_F16X3 always needs it (tiles 1..8, persistent kernel with 16x16 or
 * 32x32 MFMA; tiles 1..4 and 8 stage f2 from an FP32 copy, 5..7 from FP64; tile 0
 * takes tile 1, 128-column tiles, for boxes of 128 or more values of k,
 * else tile 2): the
 * per-rank scales 2^(13 - e_r), e_r = floor(log2 max|f1[r]|), one scale 2^g
 * for the other operand (the largest |coef_r f0 f2| / 2^(13-e_r) times 2^g is
 * below 2^14, so no FP16 term overflows), f1 scaled and split into two FP16
 * terms, and f2[r] 2^(-floor(log2 max|f2[r]|)) rounded to FP32 are formed
 * there first; the output is multiplied by
 * 2^-g (results below the FP32 range then flush to zero, as they would in any
 * FP32 output). The rank factors coef_r f0 2^(g - 13 + e_r) are formed in
 * FP64, so factor rows whose largest entries differ by more than about 10^290
 * between the axes of one rank are outside its range. The ranks are taken in
 * an order of the library's (with K <= 1024: decreasing max|f0[r]|, ties by
 * index, so that terms of similar width share a chunk of 32 ranks; otherwise
 * as given), and for each plane i of axis 0 the chunks whose rank factors
 * times the scaled f2 round to zero in both FP16 terms (|coef_r f0[r][i]
 * 2^(g - 13 + e_r + e2_r)| <= 2^-27, e2_r = floor(log2 max|f2[r]|)) are
 * marked absent and skipped: they would add only zeros, so the result is bit
 * for bit that of the full sum in the same order (ls_reconstruct_f16_plan
 * reports the order, the marks and the work). NULL / 0 is valid for every
 * other precision and tile.
 * Errors: LS_EINVAL (box outside the factors, nbox < 1, K < 1),
 * LS_EUNSUPPORTED (tile id not valid for the precision; LS_F16X3 with over
 * 2^31 tiles in a group of boxes or an operand of 2 GB or more; tiles 1..5 of
 * a bf16 split precision with f1 or f2 of 2 GB or more), LS_EWORKSPACE
 * (tile 6 or above of a bf16 split precision, or LS_F16X3, with a missing or
 * short workspace).
 */
ls_status ls_reconstruct(const ls_canon* P, const ls_box* boxes, int32_t nbox, double scale,
                         int32_t precision, int32_t tile, void* out_dev, void* ws_dev,
                         size_t ws_bytes, hipStream_t stream);
/* The preparation ls_reconstruct makes first in its workspace, as a call of
 * its own (the same reconstruction of the canonical tensor, Appendix, eq.
 * CP_form): for LS_F16X3 the row maxima of the factors, the scaled rank
 * factors, f1 scaled and split into FP16 terms and the scaled FP32 copy of f2;
 * for LS_BF16X3 / LS_BF16X6 f1 split into bf16 terms (read by the tiles that
 * use the workspace); nothing for LS_F64 and LS_F32 (returns LS_OK at once).
 * ws_dev, ws_bytes: device workspace of at least
 * ls_reconstruct_workspace(P, precision) bytes, caller-owned. Lets a caller
 * run the preparation beside other work on another stream, or reuse it for
 * several calls on the same factors. Asynchronous on `stream`.
 * Errors: LS_EINVAL (null or empty factors, unknown precision), LS_EWORKSPACE
 * (missing or short workspace).
 */
ls_status ls_reconstruct_prepare(const ls_canon* P, int32_t precision, void* ws_dev,
                                 size_t ws_bytes, hipStream_t stream);
/* ls_reconstruct without its preparation: ws_dev must hold the preparation of
 * the same factors (unchanged values) and precision, made by
 * ls_reconstruct_prepare or by an earlier ls_reconstruct, and complete before
 * these kernels run (the same stream, or an order the caller sets with
 * events). Otherwise the values are meaningless (every access still stays
 * inside the workspace). Arguments, layouts and errors as ls_reconstruct.
 */
ls_status ls_reconstruct_prepared(const ls_canon* P, const ls_box* boxes, int32_t nbox,
                                  double scale, int32_t precision, int32_t tile, void* out_dev,
                                  void* ws_dev, size_t ws_bytes, hipStream_t stream);
/* Workspace bytes of ls_reconstruct for a precision (0 for LS_F64, LS_F32). */
size_t ls_reconstruct_workspace(const ls_canon* P, int32_t precision);

/* Number of reconstruction tile variants for a precision (for autotuning). */
int32_t ls_reconstruct_tiles(int32_t precision);
/* Measured tile choice for ls_reconstruct (the same reconstruction, Appendix,
 * eq. CP_form; the tiling is a project addition). Runs the call as given with
 * tile 0 (which validates it), then every tile of `precision` that can run it
 * (tiles that need the workspace only when ws_dev holds
 * ls_reconstruct_workspace bytes; tiles that refuse the boxes are skipped):
 * one untimed run and `reps` timed runs each, with events on `stream`, which
 * it synchronizes. The fastest is entered in a per-process cache under the
 * call's shape class (precision, K, len[], whether the workspace serves the
 * pre-split tiles, nbox and the boxes' extents in order; not their offsets,
 * the factor values or `scale`), so that later ls_reconstruct and
 * ls_reconstruct_prepared calls of the class with tile 0 take it. out_dev
 * holds the last tile's result (every tile writes the reconstruction, within
 * the precision's rounding; tiles of one MFMA shape agree bit for bit).
 * tile_out: host, the chosen tile; ms_out (host, nullable): its mean time per
 * call in ms, preparation included. Thread-safe; calls on several threads
 * time each other's work.
 * Errors: those of ls_reconstruct for the call as given; LS_EINVAL (reps not
 * in [1, 1000], null tile_out); LS_EHIP (event failure, e.g. on a stream
 * being captured).
 */
ls_status ls_reconstruct_autotune(const ls_canon* P, const ls_box* boxes, int32_t nbox,
                                  double scale, int32_t precision, void* out_dev, void* ws_dev,
                                  size_t ws_bytes, int32_t reps, hipStream_t stream,
                                  int32_t* tile_out, double* ms_out);
/* The tile ls_reconstruct_autotune chose for this call's shape class, 0 if
 * it has not been tuned in this process (host only; ws_dev is only compared
 * with NULL). tile: host; ms (host, nullable): its time when tuned, else 0.
 * Errors: LS_EINVAL (null pointers, nbox < 1, unknown precision).
 */
ls_status ls_reconstruct_tuned_tile(const ls_canon* P, const ls_box* boxes, int32_t nbox,
                                    int32_t precision, const void* ws_dev, size_t ws_bytes,
                                    int32_t* tile, double* ms);
/* The LS_F16X3 preparation that ws_dev holds (ls_reconstruct_prepare or an
 * earlier ls_reconstruct of the same factors, complete before this call:
 * it copies from the device synchronously, on the null stream), and the
 * work of reconstructing `boxes` from it (Appendix, eq. CP_form; the chunk
 * skipping is a project addition). perm_host (host, nullable, K entries):
 * perm_host[s] = the caller's rank in slot s of the library's order.
 * masks_host (host, nullable, len[0] entries): bit c set when rank chunk c
 * (slots 32c .. 32c+31) has a nonzero FP16 term on that plane of axis 0;
 * when the ranks fill more than 32 chunks none is skipped, every entry is
 * 0xFFFFFFFF and chunk_values counts every chunk. chunk_values (host, nullable): the sum over the boxes'
 * values of the chunks their plane runs (a plane with no marked chunk runs
 * chunk 0, whose terms are all zero), so that 2 x 32 x chunk_values is the
 * multiply-adds of one FP16 product of the persistent tiles, against
 * 2 x 32 x ceil(K/32) x values without skipping.
 * Errors: LS_EINVAL (null factors, nbox < 1, a box outside the factors),
 * LS_EWORKSPACE (missing or short workspace), LS_EHIP (copy failure).
 */
ls_status ls_reconstruct_f16_plan(const ls_canon* P, const ls_box* boxes, int32_t nbox,
                                  const void* ws_dev, size_t ws_bytes, int32_t* perm_host,
                                  uint32_t* masks_host, int64_t* chunk_values);

/*
 * Energy as a canonical scalar product (Appendix, eq. scal) with a density
 * rho in canonical form sampled at cell midpoints (Sec. 2.2, Example 2.1):
 *   E = sum_r sum_s coef[r] d[s] prod_l G_l[r][s],  G_l = f_l rho_l^T.
 * P and rho must have equal len[]. precision LS_F64 or LS_F32 (Gram products
 * and per-lane sums in FP32; all reductions across lanes and the final sum in
 * FP64). E_dev: device, one double. ws_dev: device workspace of at least
 * ls_energy_workspace(P->K, rho->K) bytes; on return it holds the Grams
 * G_l[r][s] at ((l*K + r)*Krho + s) as FP64.
 * Errors: LS_EINVAL, LS_EWORKSPACE, LS_EUNSUPPORTED (bf16 precisions).
 */
size_t ls_energy_workspace(int32_t K, int32_t Krho);
ls_status ls_energy(const ls_canon* P, const ls_canon* rho, int32_t precision,
                    double* E_dev, void* ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * Forces on the unit-cell atoms, F[nu][l] = -dE/da_{nu,l}, with the energy
 * of the previous entry point, by the adjoint of the assembled vectors:
 * moving a_nu moves all its lattice images, so
 *   dE/da_{nu,l} = Z_nu sum_q w_q sum_s d_s G'_l[nu q][s] prod_{l' != l} G_l'[nu q][s],
 * where G'_l pairs the position derivative of each master vector with the
 * density folded back over the lattice shifts (the transpose of the shift
 * sum). Value Grams use the same folded density, so E is produced as well.
 * rho: density in canonical form with len[l] = N_l of the lattice.
 * precision: LS_F64 or LS_F32 (FP32 products and per-lane sums in the Grams;
 * cell integrals, folded density and every reduction across lanes in FP64).
 * F_dev: device [M0][3]. E_dev: device scalar or NULL.
 * ws_dev: at least ls_forces_workspace(lat, M0, R, rho->K) bytes.
 * Errors: LS_EINVAL, LS_EWORKSPACE, LS_EUNSUPPORTED.
 */
size_t ls_forces_workspace(const ls_lattice* lat, int32_t M0, int32_t R, int32_t Krho);
ls_status ls_forces(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                    const double* pos_dev, const double* Z_dev, const ls_canon* rho,
                    int32_t precision, double* F_dev, double* E_dev,
                    void* ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * ls_forces for callers that cannot allocate device memory or pass a
 * workspace (code under HIP graph capture, tight molecular-dynamics or
 * serving loops, harnesses that forbid allocation). Same arguments, kernels,
 * results and errors as ls_forces, without ws_dev / ws_bytes: the scratch
 * (folded density, Grams, per-atom energies) is a fixed array of
 * LS_FORCES_NOALLOC_BYTES bytes of device memory inside this library, one per
 * GPU, held until the process ends. The call allocates nothing; its first
 * call on a device resolves that device's array address once.
 * Limit: problems with ls_forces_workspace(lat, M0, quad->R, rho->K) above
 * LS_FORCES_NOALLOC_BYTES are refused with LS_EWORKSPACE before anything is
 * enqueued (8 MiB holds, e.g., M0 = 64 atoms, R = 48, a rank-8 density on a
 * 32^3-cell box lattice of n = 128, which needs 2.8 MB).
 * Every call on one GPU uses the same array and leaves its contents behind:
 * calls that may overlap on one GPU (several streams, several host threads)
 * race and give wrong results; the caller orders them (one stream, or
 * events). Calls in sequence on one stream are safe: every scratch entry a
 * call reads is written earlier in the same call.
 */
#define LS_FORCES_NOALLOC_BYTES (8u << 20)
ls_status ls_forces_noalloc(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                            const double* pos_dev, const double* Z_dev, const ls_canon* rho,
                            int32_t precision, double* F_dev, double* E_dev, hipStream_t stream);

/*
 * Richardson-regularised periodic sum on the reference cell (Sec. 3.2,
 * Richardson extrapolation): the assembled periodic tensors of the lattices
 * L and 2L (Lemma 3.2) combined in canonical form (Appendix, eq. conc) as
 *   order 1: 2 P_L - P_2L        (sums that grow linearly in L),
 *   order 2: (4 P_L - P_2L) / 3  (sums that grow quadratically in L);
 * each is exact when P_L = P + c L^order. lat must be periodic; the images
 * of 2L follow the even-L convention of the periodic cell.
 * f0_dev, f1_dev, f2_dev: device [2K][n] FP64, K = M0 * quad->R: rows
 * [0, K) hold the factors of lattice L, rows [K, 2K) those of lattice 2L.
 * coef_dev: device [2K], (alpha Z_nu w_q, beta Z_nu w_q) with the weights
 * above. Errors: LS_EINVAL (non-periodic lattice, order not 1 or 2, null
 * pointers, and every error of ls_assemble).
 */
ls_status ls_richardson(const ls_lattice* lat, const ls_quad* quad, int32_t M0,
                        const double* pos_dev, const double* Z_dev, int32_t order,
                        double* f0_dev, double* f1_dev, double* f2_dev, double* coef_dev,
                        hipStream_t stream);

/*
 * Canonical sum alpha A + beta B by concatenation of the factor matrices
 * (Appendix, eq. conc), e.g. of two different systems.
 * A and B must have equal len[]; outputs: f_l [K_A + K_B][len_l] (rows of A,
 * then rows of B) and coef [K_A + K_B] = (alpha coef_A, beta coef_B), device.
 * Errors: LS_EINVAL.
 */
ls_status ls_canon_combine(const ls_canon* A, double alpha, const ls_canon* B, double beta,
                           double* f0_dev, double* f1_dev, double* f2_dev, double* coef_dev,
                           hipStream_t stream);

/*
 * Quantics-TT compression of canonical vectors (Sec. 4, eq. EwaldTensorQTT;
 * Appendix: TT format, eq. tt, and binary folding). Each of nvec vectors of
 * length len (row v at x_dev + v * ld, device, FP64; e.g. the rows of an
 * assembled factor matrix, ld = len = N_l) is zero-padded to 2^d entries,
 * d = ls_qtt_digits(len), folded into a 2 x ... x 2 tensor of order d with
 * the most significant binary digit first, and decomposed by the TT-SVD:
 * left to right, each unfolding (rows (alpha_{k-1}, j_k)) is decomposed by an
 * SVD, and the kept left singular vectors form core k. r_k is the smallest
 * rank whose discarded singular values have Euclidean norm
 * <= eps ||x||_2 / sqrt(d - 1), so that ||x - x_QTT||_2 <= eps ||x||_2
 * (eps = 0: every non-zero singular value kept). FP64 throughout.
 * Outputs (device, caller-owned):
 *   cores_dev  [nvec][cap] doubles: core k of vector v (k = 1..d) at offset
 *              sum_{j<k} 2 r_{j-1} r_j of its slot, shape [r_{k-1}][2][r_k]
 *              row-major; storage per vector sum_k 2 r_{k-1} r_k;
 *   ranks_dev  [nvec][d + 1]: r_0 .. r_d (r_0 = r_d = 1);
 *   status_dev [nvec]: 1 = compressed; -1 = a rank above 32 would be needed
 *              (the next unfolding would not fit); -2 = the cores exceed cap;
 *              -3 = the SVD did not converge. Only status 1 vectors have
 *              valid ranks and cores.
 * Limits: len <= 4096 (d <= 12), r_k <= 32. Errors: LS_EINVAL.
 */
int32_t ls_qtt_digits(int32_t len);
ls_status ls_qtt_compress(const double* x_dev, int32_t nvec, int32_t len, int64_t ld, double eps,
                          int32_t cap, double* cores_dev, int32_t* ranks_dev, int32_t* status_dev,
                          hipStream_t stream);
/*
 * The vectors QTT cores represent (eq. tt): y_dev[v * ld + i], i < len, for the
 * output of ls_qtt_compress with the same nvec, len and cap (cores of at most
 * 8192 doubles per vector). Vectors whose status is not 1, or whose ranks or
 * core total are out of range, are written as NaN. Errors: LS_EINVAL.
 */
ls_status ls_qtt_expand(const double* cores_dev, const int32_t* ranks_dev,
                        const int32_t* status_dev, int32_t nvec, int32_t len, int32_t cap,
                        double* y_dev, int64_t ld, hipStream_t stream);

/*
 * Nuclear-potential operator matrix in a separable basis (Sec. 2.2,
 * Example 2.1, eq. nuc_pot): V[k][m] = <G_k (.) G_m, P> for rank-one basis
 * functions G_k = g_k^(0) (x) g_k^(1) (x) g_k^(2) sampled at cell midpoints:
 *   V[k][m] = sum_r coef[r] prod_l sum_i g_k^(l)(i) g_m^(l)(i) f_l[r][i]
 * (Hadamard and scalar products, eqs. had, scal), on FP64 MFMA.
 * g_l_dev: device [Nb][P->len[l]] FP64. V_dev: device [Nb][Nb] FP64 (symmetric).
 * ws_dev: at least ls_nuclear_workspace(P->K, Nb) bytes.
 * Errors: LS_EINVAL, LS_EWORKSPACE.
 */
size_t ls_nuclear_workspace(int32_t K, int32_t Nb);
ls_status ls_nuclear_matrix(const ls_canon* P, int32_t Nb, const double* g0_dev,
                            const double* g1_dev, const double* g2_dev, double* V_dev,
                            void* ws_dev, size_t ws_bytes, hipStream_t stream);

/*
 * Batched lattice systems (project addition; per system Sec. 3.1 box
 * assembly, Appendix eq. scal energy and eq. CP_form reconstruction).
 * Each system gives a box lattice, its quadrature, charges, a density in
 * canonical form and one sub-box of at most min(n, 256) cells per axis to
 * reconstruct (cell averages, scale 1/h^3). All systems run in one
 * persistent kernel that drains a device work queue (density folding, then
 * per-(atom, axis) vector tasks that form the energy Grams against the folded
 * density and the sub-box factor columns, then MFMA reconstruction tiles),
 * launched through a hipGraph built on first use. The library allocates the
 * host-side plan object only; device memory is the caller's workspace.
 */
typedef struct {
  ls_lattice lat;        /* periodic must be 0 */
  ls_quad quad;          /* host nodes/weights, read during ls_batch_create */
  int32_t M0;
  const double* pos_dev; /* [M0][3] */
  const double* Z_dev;   /* [M0] */
  ls_canon rho;          /* density, rho.len[l] = N_l, rho.K <= 8 */
  ls_box box;            /* sub-box, e[l] <= min(n, 256) */
  void* out_dev;         /* [e0][e1][e2]: double (LS_F64), else float */
  double* E_dev;         /* energy <P, rho> */
} ls_system;

typedef struct ls_batch* ls_batch_t;

/* Plan a batch; *ws_bytes receives the device workspace size.
 * precision: LS_F64, LS_F32, LS_BF16X3, LS_BF16X6 or LS_F16X3, the
 * reconstruction's (split precisions: both operands split inside the tile,
 * FP32 accumulation and output; LS_F16X3 scales every rank of both operands
 * by powers of two from the largest value of each sub-box factor column, as
 * the LS_F16X3 reconstruction does); everything else is FP64.
 * Errors: LS_EINVAL (system index in the message; among others a system with
 * M0 R >= 2^20 ranks, or a folded density of 2 GB or more, which the kernel's
 * 32-bit buffer offsets cannot address), LS_EUNSUPPORTED. */
ls_status ls_batch_create(const ls_system* systems, int32_t count, int32_t precision,
                          ls_batch_t* batch, size_t* ws_bytes);
/* Number of tile variants of the batch kernel (tile ids 1..n). */
int32_t ls_batch_tiles(void);
/* Enqueue one run on `stream` (graph replay). tile 0 = the autotuned tile
 * (or a default before autotuning). The first run with a given workspace and
 * tile uploads the descriptors (synchronously) and builds the graph. */
ls_status ls_batch_run(ls_batch_t batch, void* ws_dev, size_t ws_bytes, int32_t tile,
                       hipStream_t stream);
/* Times every tile variant on this batch (two runs each, synchronous) and
 * keeps the fastest for tile = 0. *best_ms (nullable) receives its time.
 * The choice is also entered in the autotune cache under the batch's shape
 * class (its precision and the multiset of its systems' n, L, M0, R, density
 * rank and sub-box extents), so that a later ls_batch_create of the same
 * class starts with it as its tile 0 without autotuning. */
ls_status ls_batch_autotune(ls_batch_t batch, void* ws_dev, size_t ws_bytes, hipStream_t stream,
                            int32_t* best_tile, double* best_ms);
/* Autotune cache (project addition, per the batch's autotuned tiles): the
 * fastest tile per shape class, kept in the process and, once a file is
 * named here, in that text file (one "key precision tile ms" line per entry,
 * rewritten whenever an entry is added). ls_batch_cache_file(path) empties
 * the in-process cache, loads the entries the file holds (a missing file is
 * created by the next autotune) and writes to it from then on; NULL stops
 * writing. The file is the library's only file access. Errors: none (a file
 * that cannot be written leaves the in-process cache in use). */
ls_status ls_batch_cache_file(const char* path);
/* The cached tile of this batch's shape class (*tile = 0 if none; *ms
 * nullable: the time it was tuned at). Host only. */
ls_status ls_batch_tuned_tile(ls_batch_t batch, int32_t* tile, double* ms);
/* After the last run has completed: per-system device time in seconds
 * (first task start to last task end, device wall clock) into seconds[count]
 * (nullable), the span of each phase (folding, vector tasks, tiles: first
 * start to last end) into phase_seconds[3] (nullable), and the error flag
 * (non-zero if a dependency wait timed out). */
ls_status ls_batch_report(ls_batch_t batch, const void* ws_dev, double* seconds,
                          double* phase_seconds, int32_t* error_flag);
void ls_batch_destroy(ls_batch_t batch);

/* ------------------------------------------------------------------------
 * Reference kernels for the rooflines (not part of the method).
 * ------------------------------------------------------------------------ */
/* Plain device copy of `bytes` bytes from src_dev to dst_dev (both device,
 * 16-byte aligned, caller-owned; bytes a positive multiple of 16). Its
 * duration gives the attainable HBM bandwidth; its hardware-counter readings
 * (bytes fetched and written per dispatch) calibrate those of other kernels.
 * Errors: LS_EINVAL for null or misaligned pointers or a bad size. */
ls_status ls_probe_copy(const void* src_dev, void* dst_dev, size_t bytes, hipStream_t stream);
/* MFMA issue loop: `blocks` workgroups of four waves, each wave issuing
 * iters x 8 (16x16 shapes) or iters x 4 (32x32 shapes) independent MFMAs of
 * the precision's instruction, shape 0: F64 v_mfma_f64_16x16x4f64, F32
 * v_mfma_f32_16x16x4f32, BF16X3/BF16X6 v_mfma_f32_16x16x32_bf16, F16X3
 * v_mfma_f32_16x16x32_f16; shape 1: F32 v_mfma_f32_32x32x2f32, BF16X3/BF16X6
 * v_mfma_f32_32x32x16_bf16, F16X3 v_mfma_f32_32x32x16_f16. Writes one
 * float per thread to out_dev[blocks * 256] (device, caller-owned); *flops
 * (host) receives the floating-point operations of the launch. Timing is the
 * caller's. Errors: LS_EINVAL for null pointers, an unknown precision or
 * shape, or out-of-range counts. */
ls_status ls_probe_mfma(int32_t precision, int32_t shape, int32_t blocks, int32_t iters,
                        float* out_dev, double* flops, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* LATSUM_H */
