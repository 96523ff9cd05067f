// Internal declarations shared by the HIP kernels and the host engine of
// the qtthom library.  Not part of the public C ABI (include/qtthom.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

namespace qtt {

using cplx = double2;  // interleaved complex double: x = re, y = im

// Householder columns with squared norm below this are treated as zero
// (identity reflector): beta^2 and |alpha - beta|^2 stay far from the
// bottom of the double range, so tau and 1/(alpha - beta) stay finite.
constexpr double QR_TINY = 1e-292;

// operand transform of a GEMM operand
enum Op : int { OP_N = 0, OP_T = 1, OP_C = 2 };

// Strided, two-level batched complex GEMM on row-major operands:
//   C[b1,b2] = alpha * op(A[b1,b2]) * op(B[b1,b2]) + beta * C[b1,b2]
// op(A) is M x K: OP_N reads A[m*lda + k], OP_T reads A[k*lda + m], OP_C
// reads conj(A[k*lda + m]).  op(B) is K x N likewise (OP_N: B[k*ldb + n]).
// C[m*ldc + n].  Batch element (b1, b2) offsets every operand by
// b1*s?1 + b2*s?2 complex entries.
struct GemmArgs {
  int M, N, K;
  int opA, opB;
  const cplx* A; long lda, sA1, sA2;
  const cplx* B; long ldb, sB1, sB2;
  cplx* C; long ldc, sC1, sC2;
  int nb1, nb2;
  cplx alpha, beta;
  // optional third batch level (innermost): element (b1, b2, b3) adds
  // b3 * s?3; the batch index is z = (b1 * nb2 + b2) * nb3 + b3
  int nb3 = 1;
  long sA3 = 0, sB3 = 0, sC3 = 0;
  // matrix-core path only: FP32 operands and accumulation (the vector
  // kernel for thin shapes always computes in FP64)
  bool fp32 = false;
  // matrix-core path only: split-BF16 operands (hi + lo, three bf16
  // products per real product) with FP32 accumulation
  bool bf16x3 = false;
  // split-K workspace of the matrix-core path (gemm_ws_elems entries for
  // ksplit slices); ksplit = 1 or ws = nullptr: no split
  cplx* ws = nullptr;
  int ksplit = 1;
  // matrix-core FP64 tile variant forced (0 .. gemm_num_tiles() - 1), or -1:
  // chosen per shape
  int tile = -1;
  // matrix-core path only: when set, the product kernel records its span
  // (earliest workgroup start into span[0] by atomic min, latest workgroup
  // end into span[1] by atomic max, device real-time counter ticks); the
  // caller arms the pair as {~0, 0} (span_arm)
  unsigned long long* span = nullptr;
};
__host__ __device__ inline long gemm_nbatch(const GemmArgs& g) { return (long)g.nb1 * g.nb2 * g.nb3; }
__host__ __device__ inline void gemm_batch_offsets(const GemmArgs& g, long z, long& oa, long& ob, long& oc) {
  const long b3 = z % g.nb3, t = z / g.nb3;
  const long b2 = t % g.nb2, b1 = t / g.nb2;
  oa = b1 * g.sA1 + b2 * g.sA2 + b3 * g.sA3;
  ob = b1 * g.sB1 + b2 * g.sB2 + b3 * g.sB3;
  oc = b1 * g.sC1 + b2 * g.sC2 + b3 * g.sC3;
}
// Returns true when the matrix-core kernel ran, false for the vector kernel.
bool gemm(const GemmArgs& g, hipStream_t s);
// Matrix-core path of gemm for M, N >= 16 and K >= 4 (kernels_mfma.hip);
// returns false when the shape is left to the vector kernel.
bool gemm_mfma(const GemmArgs& g, hipStream_t s);
// The two launches of gemm_mfma separately: the product (K slices into the
// workspace when ks_used > 1) and the ordered sum of the slices.
bool gemm_mfma_main(const GemmArgs& g, hipStream_t s, int& ks_used);
void gemm_mfma_reduce(const GemmArgs& g, int ks, hipStream_t s);
// The K split the matrix-core path wants for this shape and precision
// (1: none) and the workspace it then needs.
int gemm_ksplit(int M, int N, int K, long nbatch, bool fp32, int tile = -1);
int gemm_num_tiles();
size_t gemm_ws_elems(const GemmArgs& g, int ksplit);
// Vector-ALU path of gemm (any shape).
void gemm_vector(const GemmArgs& g, hipStream_t s);

// Strided matrix view used by the factorisation kernels: element (i, j) of
// batch element b is base[b*sb + i*rs + j*cs], conjugated when conj != 0.
struct MatView {
  const cplx* base;
  long rs, cs, sb;
  int conj;
};
struct MatOut {
  cplx* base;
  long rs, cs, sb;
};

// Householder QR of batched m x n matrices (any shape), k = min(m, n).
// Writes R (k x n, upper trapezoidal) to `R` and, when Q.base != nullptr,
// the explicit Q (m x k, orthonormal columns) to `Q`.  `ws` must hold
// batch * (m*n + m*k + k) complex entries.
void qr(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws,
        hipStream_t s);
size_t qr_ws(int batch, int m, int n);
// per-matrix slice of that workspace: the generic kernel's copy of A and
// Q (m n + m k + k entries), or V, T and tau of every 16-column panel
// (np (16 m + 256 + 16) entries: V[np][m][16], T[np][16][16], tau[np][16])
// followed by the large-shape kernel's working copy of A in panel-major
// order (nc 16 m entries, nc = ceil(n / 16)), whichever is larger
inline size_t qr_ws_per_matrix(int m, int n) {
  const long k = m < n ? m : n, np = (k + 15) / 16, nc = (n + 15) / 16;
  const long gen = (long)m * n + (long)m * k + k, blk = np * (16L * m + 256 + 16) + nc * 16L * m;
  return (size_t)(gen > blk ? gen : blk);
}
// The global-memory kernel behind qr() for shapes the register kernels do
// not hold (same contract as qr).
void qr_generic(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws,
                hipStream_t s);

// Register-resident Householder QR for m <= 256, n <= 128 (see
// kernels_fact.hip); returns false when the shape does not fit.  Uses
// qr_fast_ws(batch, m, n) <= qr_ws(batch, m, n) workspace entries.
bool qr_fast(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws, hipStream_t s);
// Blocked QR on the matrix cores (kernels_qr_blk.hip) for m >= n,
// 16 < n <= 96, m <= 192; false when the shape is not covered.  `ws` as
// for qr().
bool qr_blocked(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws, hipStream_t s);
// R of the unblocked 2D-wave register kernel, with the Householder
// vectors and tau per 16-column panel written to the workspace (layout of
// qr_ws_per_matrix's blocked part) instead of Q; false when no variant
// holds the shape (16 < n <= 96).  With `only` (a device array of batch
// flags) the matrices whose flag is zero are skipped.
bool qr_2d_vectors(int batch, int m, int n, MatView A, MatOut R, cplx* ws, hipStream_t s,
                   const int* only = nullptr);
// R (and, with vout, the panel vectors) from the kernel with one wave per
// 16-column group holding all rows (n <= 96, m <= 160); false otherwise.
bool qr_one_rowblock(int batch, int m, int n, const MatView& A, const MatOut& R, cplx* vout,
                     hipStream_t s);
// Q (m x k) from those vectors: T of each panel (compact WY), then the
// block reflectors applied on the matrix cores in reverse panel order;
// false when the shape is outside the blocked kernel's range.  `only` as
// for qr_2d_vectors.
bool qr_form_q(int batch, int m, int n, MatOut Q, cplx* ws, hipStream_t s, const int* only = nullptr);
// Orthonormal basis of the column space of batched m x n matrices (m >= n):
// Q (m x n) with Q^H Q = I and range(Q) = range(A), no R.  CholeskyQR2 on
// the FP64 matrix cores (kernels_cholqr.hip), one workgroup per matrix;
// a matrix whose Gram is too ill-conditioned for it (the first Cholesky
// breaks down, or the columns after the first pass are not within 0.5 of
// orthonormal in Frobenius norm) is flagged and factored by the Householder
// kernels instead, in the same stream order.  Covers 32 < m <= 192 for
// 16 < n <= 64 and 32 < m <= 168 for 64 < n <= 80 (m >= n); false
// otherwise.  `ws` holds orth_ws(batch, m, n) entries;
// on return its first batch ints hold the flags (1 = Householder).
// With drop, a column dependent on the earlier ones to rounding (Cholesky
// pivot at most 1e-13 of the largest) is not handed to Householder but
// gives an exactly zero column of Q: Q^H Q is then I on the kept columns
// and zero on the dropped ones, still an isometry on range(A) up to the
// dropped directions (relative size below 3e-7).
bool orth(int batch, int m, int n, MatView A, MatOut Q, cplx* ws, hipStream_t s, bool drop = false);
size_t orth_ws(int batch, int m, int n);
// The same basis with each pass spread over the device: partial Grams per
// 32-row slice, one workgroup per matrix for the Cholesky and R^-1, the
// products on the library's GEMM.  Needs unit column strides and no
// conjugation; false otherwise or outside orth_ok.  `ws` holds
// orth_split_ws(batch, m, n) entries, flags first as for orth.
bool orth_split(int batch, int m, int n, MatView A, MatOut Q, cplx* ws, hipStream_t s, bool drop = false);
size_t orth_split_ws(int batch, int m, int n);
bool orth_ok(int m, int n);
// Blocked QR for large shapes (m >= n, m <= 320, n <= 160): the matrix in
// the workspace, one workgroup walking over 16-column panels with the
// trailing updates on the matrix cores, Q formed afterwards from the
// panels' block reflectors (kernels_qr_big.hip); false when the shape is
// not covered.  `ws` as for qr().
bool qr_big(int batch, int m, int n, MatView A, MatOut R, MatOut Q, cplx* ws, hipStream_t s);
// Unblocked register kernel with two columns per lane (n <= 96).
bool qr_two_col(int batch, int m, int n, MatView A, MatOut R, MatOut Q, hipStream_t s);
size_t qr_fast_ws(int batch, int m, int n);

// One-sided Jacobi of batched square n x n matrices (n <= 96) resident in
// LDS: A V = U diag(S) with U orthonormal columns and S descending (V is not
// formed).  Returns false when n is too large.
bool jacobi_square(int batch, int n, MatView A, MatOut U, double* S, hipStream_t s);

// The same for 96 < n <= 160: the first columns in LDS, the others in `ws`
// (jacobi_ws(batch, n) entries); false when n is outside that range.
bool jacobi_big(int batch, int n, MatView A, MatOut U, double* S, cplx* ws, hipStream_t s);
size_t jacobi_ws(int batch, int n);

// One-sided Jacobi SVD of batched m x n matrices with m >= n:
// A = U diag(S) V^H with U (m x n) orthonormal columns, V (n x n) unitary,
// S descending.  `ws` must hold batch * (m*n + n*n) complex entries.
void svd(int batch, int m, int n, MatView A, MatOut U, double* S, MatOut V,
         cplx* ws, hipStream_t s);
size_t svd_ws(int batch, int m, int n);

// Complex standard normal numbers (Philox4x32-10 counter generator +
// Box-Muller), several blocks in one launch: block i (i < n) fills
// out[i][e], e < start[i+1] - start[i], with entry e of the stream
// (seed, stream[i]) scaled by scale[i].  Passed by value as the kernel
// argument.
constexpr int GAUSS_MULTI_MAX = 40;
struct GaussBlocks {
  int n = 0;
  cplx* out[GAUSS_MULTI_MAX];
  long start[GAUSS_MULTI_MAX + 1];
  uint64_t stream[GAUSS_MULTI_MAX];
  double scale[GAUSS_MULTI_MAX];
};
void gaussian_multi(const GaussBlocks& g, uint64_t seed, hipStream_t s);

// x / d for 0 <= x < 2^31 and 1 <= d < 2^31 by the high half of a 32-bit
// multiply and a shift (the round-up method of Granlund and Montgomery,
// 1994): with s = ceil(log2 d) >= 1 and m = floor(2^(31+s) / d) + 1
// (< 2^32), floor(x m / 2^(31+s)) = floor(x / d) because
// x (m d - 2^(31+s)) <= x d < 2^(31+s); d = 1 is marked by m = 0.
struct FastDiv {
  uint32_t m = 0, sh = 0, d = 1;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  if (d <= 1) return f;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.m = (uint32_t)(((1ull << (31 + s)) / d) + 1);
  f.sh = s - 1;
  return f;
}
__host__ __device__ inline uint32_t fdiv(uint32_t x, const FastDiv& f) {
#ifdef __HIP_DEVICE_COMPILE__
  const uint32_t hi = __umulhi(x, f.m);
#else
  const uint32_t hi = (uint32_t)(((uint64_t)x * f.m) >> 32);
#endif
  return f.m == 0 ? x : hi >> f.sh;
}

// One core of a materialised TTO x TT product (Table 2, contract):
// Z[b][(a,c)][i][(a2,c2)] = sum_j A[a][j][i][a2] x[b][c][j][c2] (A stored
// (rho, din, dout, rho2); diagonal operators pass din = 0 and A stored
// (rho, d, rho2)), batch folded into the row index, output Z of `total`
// entries, blocks [start_block, start_block + tto_apply_blocks(total,
// rho2)), one thread per rho2 outputs.
struct TtoDesc {
  const cplx* A;
  const cplx* x;
  cplx* Z;
  int batch, rho, din, dout, rho2, r, r2;
  long total, start_block;
  long a_stride;  // operator instance stride (0: one instance for all b)
  int group;      // train batch elements per operator instance
  // dividers of the thread index (i, column (b, a, c, c2)) and the instance
  FastDiv f_cols, f_r2, f_r, f_rho, f_group;
};
long tto_apply_blocks(long total, int rho2);
// Every core of a product in one launch; D_dev: ncores descriptors in
// device memory, nblocks = sum of the cores' blocks.
void tto_apply_all(int ncores, const TtoDesc* D_dev, long nblocks, hipStream_t s);

// out[b] = sqrt(sum |x[b*stride + e]|^2), e < len
void batch_norm(int batch, long len, long stride, const cplx* x,
                double* out, hipStream_t s);

// y[b][i][j] = scale * x[b][i][j]*S[b][j] for j < cols; S real per column.
void scale_cols(int batch, int rows, int cols, long ld, long sb, cplx* x,
                const double* S, long sS, hipStream_t s);

// out = conj transpose of a (rows x cols) strided view, out row-major
// (cols x rows_keep) keeping only the first `keep` columns of the input.
void conj_transpose(int batch, int rows, int keep, MatView in, MatOut out,
                    hipStream_t s);

// Generic strided 2D copy with optional scale: out(i,j) = alpha * in(i,j),
// times bscale[b] per batch element when bscale (device) is given.
void copy2d(int batch, int rows, int cols, MatView in, MatOut out,
            cplx alpha, hipStream_t s, const double* bscale = nullptr);

// Arm `slots` span pairs for timed launches: t[2i] = ~0, t[2i+1] = 0.
void span_arm(unsigned long long* t, int slots, hipStream_t s);

// Fill count complex entries with value v.
void fill(cplx* p, size_t count, cplx v, hipStream_t s);

// out[b][i][c] = sum over p of in[b][p][i][c] * w   (sum over the middle
// index p of length np), used by the volume averages.
void sum_middle(int batch, int outer, int np, int inner, const cplx* in,
                cplx* out, cplx w, hipStream_t s);

// out[p * NN + v] = (phase[v] == p) for p < nphase (device arrays); sets
// *bad (device int) when a phase id is >= nphase.
void onehot(const uint8_t* phase, long NN, int nphase, cplx* out, int* bad, hipStream_t s);
// Majority phase of every 2 x 2 x 2 block of the 2^n grid (2 x 2 blocks of a
// plane grid for dim 2; ties: lowest id) into the 2^(n-1) grid; n >= 1,
// nphase <= 16.
void coarsen_majority(const uint8_t* phase, int n, int nphase, uint8_t* out, hipStream_t s, int dim = 3);
// Unit momentum directions n^sigma_a of the Green factors on the 2^n grid
// (6 x 2^(3n) entries, control index (sigma, a) slowest, then x, y, z
// bits); f, f2: device arrays of one axis's frequencies (2^n each).
void direction(const double* f, const double* f2, int n, cplx* out, hipStream_t s);
// The plane version (4 x 2^(2n) entries, control (sigma, a), a in {x, y}).
void direction2d(const double* f, const double* f2, int n, cplx* out, hipStream_t s);
// Staggered-grid directions (6 x 2^(3n) entries, control index (t, a): t = 0
// the forward symbols kp_a / |kp|, t = 1 the backward ones km_a / |kp|);
// kp, km: device arrays of one axis's symbols in momentum order (2^n each).
void direction_staggered(const cplx* kp, const cplx* km, int n, cplx* out, hipStream_t s);
// The plane version (4 x 2^(2n) entries, control (t, a), a in {x, y}).
void direction_staggered2d(const cplx* kp, const cplx* km, int n, cplx* out, hipStream_t s);

void check(hipError_t e, const char* what);

}  // namespace qtt
