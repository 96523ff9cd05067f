/*
 * qtthom -- SFFT-based homogenization on quantized tensor trains (C ABI).
 *
 * Implements the hot path of the SFFT-based homogenization algorithm of
 * Hauck, Kabel, Ali and Gauger (arXiv 2412.11566): the Lippmann-Schwinger
 * fixed point of the FFT-based basic scheme (Sec. 2, Alg. 1) carried out on
 * strain fields held in controlled quantized tensor-train (QTT) format
 * (Sec. 4.3, Alg. 2), on one AMD Instinct GPU (gfx950).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * - A 3D periodic unit cell with N = 2^n voxels per axis.  Strain and stress
 *   fields carry a Voigt control core in front of the 3n binary cores
 *   (Sec. 4.3, controlled QTT): L = 3n + 1 cores.  Core 0 has physical
 *   dimension 6 (Voigt order 11, 22, 33, 23, 13, 12; strains with
 *   engineering shear, stresses plain); cores 1..n hold the bits of x, most
 *   significant first (Sec. 4.3, binary discretisation), then y, then z.
 *   Plane-strain problems (qtt_problem.dim = 2, the paper's 2D geometries)
 *   use N^2 pixels, a control core of dimension 3 (Voigt 11, 22, 12) and
 *   L = 2n + 1 cores.
 * - Tensor-train cores are stored row-major as (r_{k-1}, d_k, r_k) with r_k
 *   fastest; complex numbers are interleaved (re, im) doubles.  A tensor
 *   handle may hold a batch of B trains with common ranks (for instance the
 *   six unit load cases); batch element b of core k starts at
 *   b * r_{k-1} * d_k * r_k complex entries.
 * - Operators (TTOs, Sec. 3 eq. tto_format) are opaque handles.  Their
 *   cores have an (out, in) physical pair; "raised" operators (Sec. 3,
 *   eq. tt_to_tto; App. C) are stored diagonally.
 * - Device buffers: pointers documented as "device" must be device memory
 *   of the context's device; "host" pointers are ordinary host memory.
 * - Ownership: every qtt_tensor returned through an out-pointer is owned
 *   by the caller and released with qtt_tensor_destroy.  Input arrays stay
 *   owned by the caller.
 * - Errors: every call returns 0 (QTT_OK) or a negative QTT_E* code; no C++
 *   exception crosses the ABI.  qtt_last_error(ctx) returns a message for
 *   the last failure on that context.  A context is not thread-safe.
 * - Rounding parameters: delta is the relative Frobenius accuracy of
 *   TT-rounding, ||v - v~||_F <= delta ||v||_F (Sec. 3,
 *   eq. rounding_condition_tt), split evenly over the L-1 bonds; cap bounds
 *   every bond rank (cap <= 0 means no cap).
 */
#ifndef QTTHOM_H
#define QTTHOM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define QTT_OK          0
#define QTT_EINVAL     -1   /* invalid argument or shape mismatch          */
#define QTT_ENOMEM     -2   /* device or host allocation failed            */
#define QTT_ECAPACITY  -3   /* a size exceeds a documented maximum         */
#define QTT_EHIP       -4   /* HIP runtime error                           */
#define QTT_ENOCONV    -5   /* fixed point hit max_iter before tolerance   */
#define QTT_ENAN       -6   /* NaN or Inf met in a reduction               */
#define QTT_EDIVERGED  -7   /* residual grew beyond the divergence limit   */

/* ---- flags ------------------------------------------------------------- */
#define QTT_INVERSE     1   /* sfft_apply: apply S^H (the ISFFT)           */
#define QTT_NO_ROUND    2   /* products: materialise, do not round         */
#define QTT_EXACT       4   /* products: sketch at the full structural rank */

/* precision of the core contractions (rounding is always FP64) */
#define QTT_PREC_FP64   0
#define QTT_PREC_FP32   1
/* split-BF16: each operand of the operator x train contractions is rounded
 * to hi + lo (two bf16 values, 16 significant bits) and every real product
 * is formed from three bf16 products on the matrix cores with FP32
 * accumulation (Table 2's contractions); sketches, QR, SVD and residuals
 * stay FP64 */
#define QTT_PREC_BF16X3 2

/* orthonormalisation of the range finder's sketched unfoldings (Sec. 3:
 * only the basis is kept, not R).  The exact sketch always uses
 * Householder.
 * QTT_ORTH_AUTO (default): CholeskyQR2 on the FP64 matrix cores (qtt_zorth
 *   path 2) in the fixed-point updates whose iterate is cap-bound (a bond
 *   rank at a cap below that bond's structural rank, and the previous
 *   update's truncation discarded at least 1e-5 of it), where a column of the
 *   sketch that depends on the earlier ones to rounding is dropped (zero
 *   column of the basis) instead of refactored; Householder elsewhere.
 * QTT_ORTH_HOUSEHOLDER: Householder QR throughout.
 * QTT_ORTH_CHOLQR: CholeskyQR2 throughout, Householder QR for the matrices
 *   whose Gram is too ill-conditioned for it (qtt_zorth path 0). */
#define QTT_ORTH_AUTO        0
#define QTT_ORTH_HOUSEHOLDER 1
#define QTT_ORTH_CHOLQR      2

/* discretisation of the Green operator (App. A, Table 3):
 * QTT_SCHEME_DIRECT: k = i q (Moulinec-Suquet), Nyquist-symmetrised.
 * QTT_SCHEME_STAGGERED: the staggered grid, forward differences
 *   k+ = exp(i q) - 1 on the normal strains and backward differences
 *   k- = 1 - exp(-i q) on the shears; the constitutive law stays pointwise
 *   per voxel, as in Alg. 2. */
/* the Green step's products in Alg. 2 (truncated solves with a cap; exact
 * and untruncated solves always use the sketch):
 * QTT_MV_SKETCH (default): each factor product rounded by the randomized
 *   range finder of Sec. 3 (Gaussian TT sketch, QR sweep, truncated SVD).
 * QTT_MV_AMEN: each factor product by the AMEn-adapted product of App. B
 *   (tt_amen_apply), warm-started from the same product of the previous
 *   update (the first update from a random train at the cap's ranks; at
 *   most 3 sweeps warm, 6 cold; residual train of rank 16), its sweeps
 *   stopped when the product changes by less than a twentieth of the last
 *   relative update of the fixed point (at most 1e-3, at least delta). */
#define QTT_MV_SKETCH 0
#define QTT_MV_AMEN   1

#define QTT_SCHEME_DIRECT    0
#define QTT_SCHEME_STAGGERED 1

typedef struct qtt_ctx qtt_ctx;
typedef struct qtt_tensor qtt_tensor;

/* Problem statement: the corrector problem of Sec. 2 on a voxel grid. */
typedef struct qtt_problem {
    int n;                   /* bits per axis, N = 2^n, 1 <= n <= 10       */
    const uint8_t* phase;    /* N^3 phase ids, C order, x slowest; host
                                memory unless phase_on_device              */
    int nphase;              /* number of phases, 1..16                    */
    const double* lame;      /* host, [nphase][2] = (lambda, mu)           */
    double lame0[2];         /* reference medium (lambda0, mu0)            */
    int load_mask;           /* bit k set: solve unit load case e_k        */
    int phase_on_device;     /* nonzero: `phase` is device memory of the
                                context's device (read, never written or
                                kept beyond the call)                      */
    int scheme;              /* QTT_SCHEME_*: the Green operator's
                                discretisation (App. A, Table 3)           */
    int dim;                 /* 0 or 3: voxels N^3, Voigt 6; 2: plane
                                strain on N^2 pixels (C order, x slowest),
                                Voigt 3 (11, 22, 12), load cases bits 0..2,
                                C_eff in rows and columns 0..2 of the 6 x 6
                                output, n <= 12 (the paper's 2D problems,
                                Sec. 5); every solve entry point, the
                                adjoint included (there V = 3)             */
} qtt_problem;

typedef struct qtt_solve_opts {
    double delta;            /* rounding accuracy delta_acc                */
    double tol;              /* fixed-point tolerance delta_tol            */
    int cap;                 /* bond-rank cap (<= 0: none)                 */
    int max_iter;            /* iteration limit per load case              */
    int precision;           /* QTT_PREC_*                                 */
    int oversample;          /* extra sketch rank beyond cap (>= 0)        */
    int exact;               /* nonzero: sketch at full structural rank    */
    uint64_t seed;           /* seed of the sketching random numbers       */
    int streams;             /* load-case groups solved concurrently, each
                                on a stream of its own (<= 1: one stream);
                                in ls_adjoint also the number of groups of
                                the adjoint fixed point and of the gradient
                                terms; ls_batch_solve ignores it          */
    double* history;         /* host, optional (NULL: none), written by
                                ls_solve and ls_solve_prepared: entry
                                [k * history_len + m] receives the relative
                                update ||eps_{m+1} - eps_m|| / ||E|| of load
                                case k after update m + 1 (the stopping
                                test of Alg. 2), NaN where load case k made
                                no such update; ls_adjoint and
                                qtt_batch_solve leave it untouched          */
    int history_len;         /* entries per load case in `history`         */
    int orth;                /* QTT_ORTH_*: how the range finder of each
                                rounding orthonormalises its sketched
                                unfoldings (Sec. 3)                         */
    int matvec;              /* QTT_MV_*: how the Green step's products are
                                approximated (Alg. 2, App. B)               */
    int rank_buckets;        /* qtt_batch_solve: nonzero splits the
                                structures of one grid size by the
                                power-of-two bucket of their largest
                                one-hot bond rank (the geometry rank of
                                Sec. 5.2), so each batch pads to alike
                                ranks; others ignore it                    */
} qtt_solve_opts;

typedef struct qtt_report {
    int iterations[6];       /* fixed-point updates per load case          */
    double residual[6];      /* last relative update per load case         */
    int max_rank;            /* largest strain bond rank after rounding    */
    double discarded;        /* largest relative discarded mass, any round */
    int status;              /* QTT_OK or the failure code                 */
    double seconds_setup;    /* operator construction (not in the loop)    */
    double seconds_solve;    /* fixed-point loop, all load cases           */
} qtt_report;

/* ---- context ----------------------------------------------------------- */
/* Creates a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * to enqueue all work on, or NULL for a stream owned by the context. */
int qtt_create(int device, void* hip_stream, qtt_ctx** ctx);
int qtt_destroy(qtt_ctx* ctx);
const char* qtt_last_error(const qtt_ctx* ctx);
/* Blocks until all work enqueued by the context has finished. */
int qtt_sync(qtt_ctx* ctx);

/* ---- tensors ----------------------------------------------------------- */
/* A batch of `batch` tensor trains with L cores, physical dims dims[L] and
 * bond ranks ranks[L+1] (ranks[0] = ranks[L] = 1), copied from host
 * interleaved complex data laid out core by core, each core batch-major
 * (batch, r_{k-1}, d_k, r_k). */
int qtt_tt_from_host(qtt_ctx* ctx, int L, const int* dims, const int* ranks,
                     int batch, const double* data, qtt_tensor** out);
/* Shape query: kind (0 = TT, 1 = operator), L, batch, dims_out[L],
 * dims_in[L] (operators; TT: copies of dims_out), ranks[L+1].  Any output
 * pointer may be NULL. */
int qtt_tensor_shape(const qtt_tensor* t, int* kind, int* L, int* batch,
                     int* dims_out, int* dims_in, int* ranks);
/* Number of complex entries qtt_tensor_to_host writes. */
size_t qtt_tensor_size(const qtt_tensor* t);
/* Copies all cores to host, same layout as qtt_tt_from_host.  Operators
 * are written as full cores (r_{k-1}, d_out, d_in, r_k) even when stored
 * diagonally.  `capacity` is the number of complex entries available. */
int qtt_tensor_to_host(qtt_ctx* ctx, const qtt_tensor* t, double* data,
                       size_t capacity);
int qtt_tensor_destroy(qtt_tensor* t);

/* Device-resident trains without a host copy.
 *
 * qtt_tensor_create: a batch of `batch` trains (L cores, dims[L], ranks[L+1]
 * with ranks[0] = ranks[L] = 1) in memory the library allocates on the
 * context's device, zero-filled; released by qtt_tensor_destroy.
 *
 * qtt_tensor_wrap: the same shape over caller-owned DEVICE memory `dev`
 * of `bytes` bytes holding the cores one after another, each batch-major
 * (batch, r_{k-1}, d_k, r_k) in interleaved complex doubles (the layout of
 * qtt_tt_from_host); no copy is made.  QTT_ECAPACITY if `bytes` is smaller
 * than the cores need, QTT_EINVAL if `dev` is not 16-byte aligned.  The
 * caller keeps ownership and keeps the memory alive and unmodified while
 * the handle is used; qtt_tensor_destroy releases the handle only.
 * Wrapped trains are operands like any other (products, tt_round, ls_*);
 * an operation that replaces cores (tt_round in place) re-points the
 * handle to library memory and leaves the caller's buffer as it was.
 *
 * qtt_tensor_core: device address and size in bytes of core k of a train
 * (all batch elements), valid until the handle is destroyed or its cores
 * are replaced.
 *
 * qtt_tensor_export: device-to-device copy of all cores of a train, in the
 * qtt_tt_from_host layout, into caller DEVICE memory `dev` of `bytes`
 * bytes (QTT_ECAPACITY if too small); ordered on the context's stream and
 * complete when the call returns.
 *
 * These are how torch-owned device buffers enter and leave the library
 * (the caller's allocator owns the memory). */
int qtt_tensor_create(qtt_ctx* ctx, int L, const int* dims, const int* ranks,
                      int batch, qtt_tensor** out);
int qtt_tensor_wrap(qtt_ctx* ctx, int L, const int* dims, const int* ranks,
                    int batch, void* dev, size_t bytes, qtt_tensor** out);
int qtt_tensor_core(const qtt_tensor* t, int k, void** dev, size_t* bytes);
int qtt_tensor_export(qtt_ctx* ctx, const qtt_tensor* t, void* dev,
                      size_t bytes);

/* Constant strain field of each batch element: E[b][6] (host); rank-1
 * train of Sec. 4.3 (constant operands). */
int qtt_const_strain(qtt_ctx* ctx, int n, int batch, const double* E,
                     qtt_tensor** out);

/* ---- operators (Sec. 4) ------------------------------------------------ */
/* SFFT operator: the reduced QFT Q_n of Sec. 4.1 (QFT circuit without the
 * final SWAPs) on each spatial axis, identity on the Voigt core.  Built on
 * the host by contracting the circuit layer by layer (the Hadamard gate,
 * then the controlled phases carried on a bond of dimension 2) with SVD
 * truncation at `delta` after each layer; the paper's Zip-Up (Sec. 4.2)
 * yields the same operator.  On one axis, S maps the voxel index j to the
 * momentum index k with weight N^-1/2 exp(+2 pi i j rev_n(k) / N). */
int qtt_sfft_build(qtt_ctx* ctx, int n, double delta, qtt_tensor** S);

/* Green operator Gamma_0 of App. A (direct scheme, k = i q) for the
 * isotropic reference medium (lam0, mu0), Nyquist-symmetrised, in the SFFT
 * momentum convention of Sec. 4.3 (indices reversed per axis, then complex
 * conjugated).  It is held as four raised operators that share the spatial
 * cores of the unit direction n = xi/|xi| (n = 0 at xi = 0), each bounded by
 * one pointwise, so truncation errors are not amplified between them:
 * u_j = tau_jk n_k, s = n . u, q = u / (2 mu0) - (c/2) n s and
 * eps = sym(n (x) q) with c = (lam0 + mu0) / (mu0 (lam0 + 2 mu0)), which
 * is the closed form of eq. orig_green_eshelby for isotropic C0 (the
 * separable split of App. D with its 1/|xi|^2 factors cancelled).  The two
 * Nyquist representatives of a frequency carry a direction each (joint
 * control index), averaged in the last map. */
int qtt_green_build(qtt_ctx* ctx, int n, double lam0, double mu0,
                    double delta, qtt_tensor** G);

/* The Green operator of a discretisation scheme (QTT_SCHEME_*; App. A,
 * Table 3); QTT_SCHEME_DIRECT is qtt_green_build.  The staggered-grid
 * operator is B (B^H C0 B)^-1 B^H with B the strain symbol of its gradient
 * (the discrete form of eq. orig_green_eshelby).  For isotropic C0 its
 * acoustic tensor is mu0 |k+|^2 I + (lam0 + mu0) conj(k+) (k+)^T, so with
 * the unit vectors n = k+ / |k+| and m = k- / |k+| it is held, like the
 * direct one, as four factors over one train of (n_a, m_a):
 * u_k = -m_k tau_kk - sum_{j != k} n_j tau_kj, s = n . u,
 * q = u / mu0 + (lam0 + mu0) / (mu0 (lam0 + 2 mu0)) m s and
 * eps_kk = n_k q_k, gamma_ij = m_j q_i + m_i q_j.  The symbols are
 * 2 pi-periodic, so no Nyquist representative is chosen.  The train of
 * (n_a, m_a) is built by the device TT-SVD; QTT_ECAPACITY if a bond needs
 * more than 160.  QTT_EINVAL for an unknown scheme. */
int qtt_green_build_scheme(qtt_ctx* ctx, int n, double lam0, double mu0,
                           double delta, int scheme, qtt_tensor** G);

/* Raised stiffness operator C(x) - C0 (Sec. 4.3; App. D: recomputed per
 * geometry) from a voxel phase array (binary discretisation of Sec. 4.3
 * followed by TT-SVD).  phase: host or device (`phase_on_device`), N^3
 * uint8, C order, x slowest, values < nphase.  lame: host [nphase][2].
 * The optional `chi` receives the one-hot phase train (core 0 of
 * dimension nphase).  QTT_ECAPACITY if a rank would exceed `cap`. */
/* Applicability estimate from two discretisation orders (Sec. 5.2: the
 * geometry compressed at two orders indicates the rank and its growth):
 * the one-hot phase train of the voxel array (order n) and of its coarsened
 * copy (order n - 1: the majority phase of every 2 x 2 x 2 block, ties to
 * the lowest id) by the device TT-SVD at `delta`.  ranks[0], ranks[1]: the
 * largest bond rank at order n - 1 and n; growth (optional): their ratio
 * (about 2 per order when the rank grows exponentially with the
 * resolution, about 1 when it saturates).  phase: host or device
 * (`phase_on_device`), N^3 uint8, 2 <= n <= 8; trains whose bonds exceed
 * the device TT-SVD's 160 are decomposed on the host.  QTT_EINVAL for a
 * phase id >= nphase. */
int qtt_rank_estimate(qtt_ctx* ctx, const uint8_t* phase, int phase_on_device,
                      int n, int nphase, double delta, int* ranks,
                      double* growth);
/* qtt_rank_estimate for a grid of dimension `dim`: 3 as above, or 2 for a
 * plane geometry (N^2 pixels, C order, x slowest, 2 <= n <= 12; the
 * coarsened copy takes the majority phase of every 2 x 2 block).  Same
 * outputs and codes; QTT_EINVAL for another `dim`. */
int qtt_rank_estimate_dim(qtt_ctx* ctx, const uint8_t* phase,
                          int phase_on_device, int n, int nphase,
                          double delta, int dim, int* ranks,
                          double* growth);

int qtt_from_voxels(qtt_ctx* ctx, const uint8_t* phase, int phase_on_device,
                    int n, int nphase, const double* lame,
                    const double lame0[2], double delta, int cap,
                    qtt_tensor** C_minus_C0, qtt_tensor** chi);
/* qtt_from_voxels for a grid of dimension `dim`: 3 as above, or 2 for a
 * plane-strain geometry (N^2 pixels, C order, x slowest, 1 <= n <= 12):
 * core 0 of the operator is 3 x 3 (Voigt 11, 22, 12, the plane-strain
 * stiffness of each phase minus C0's), then 2n binary cores.  Same
 * outputs and codes; QTT_EINVAL for another `dim`. */
int qtt_from_voxels_dim(qtt_ctx* ctx, const uint8_t* phase,
                        int phase_on_device, int n, int nphase,
                        const double* lame, const double lame0[2],
                        double delta, int cap, int dim,
                        qtt_tensor** C_minus_C0, qtt_tensor** chi);

/* ---- products, each followed by TT-rounding --------------------------- */
/* y = S x (or S^H x with QTT_INVERSE), Sec. 4.3 Alg. 2 lines for the SFFT
 * and ISFFT.  Unless QTT_NO_ROUND, the product is rounded to (delta, cap)
 * by a randomized range sketch of the implicit product followed by
 * truncated SVDs; `seed` fixes the sketch.  QTT_NO_ROUND materialises the
 * product with ranks multiplied (Table 2, contract). */
int sfft_apply(qtt_ctx* ctx, const qtt_tensor* S, const qtt_tensor* x,
               qtt_tensor** y, int flags, double delta, int cap,
               uint64_t seed);

/* y = (C - C0) : x, the Hadamard stiffness product of Alg. 2 computed as
 * a raised TTO times a TT (Sec. 3, eq. tt_to_tto; App. C). */
int tt_hadamard(qtt_ctx* ctx, const qtt_tensor* A, const qtt_tensor* x,
                qtt_tensor** y, int flags, double delta, int cap,
                uint64_t seed);

/* y = Gamma_0 : x in momentum space (Alg. 2, Green step). */
int green_apply(qtt_ctx* ctx, const qtt_tensor* G, const qtt_tensor* x,
                qtt_tensor** y, int flags, double delta, int cap,
                uint64_t seed);

/* y ~ A x by the AMEn-adapted product of App. B: instead of forming A x
 * (ranks multiply, Table 2) and rounding it, ||y - A x|| is minimised core
 * by core.  A sweep runs left to right; at core k the local solution is the
 * projection of A x onto the frame of y's other cores (the Galerkin
 * condition, eq. galerkin_condition), truncated by SVD at
 * delta / sqrt(L - 1) of its norm and at `cap` (<= 0: none); the residual
 * A x - y is carried as a train z of its own (its cores the residual's
 * projections onto z's frame), and its core enriches the kept singular
 * vectors before the QR that makes y's core orthonormal.  Before every
 * sweep y and z are made right-orthonormal.  The sweeps stop when the
 * product changes by less than `tol` (relative, largest over the batch)
 * between two sweeps, or after `sweeps`.  The returned product keeps the
 * truncated ranks (the enrichment only steers the next sweep's frames).
 * A: an operator (kind 1; QTT_EINVAL for the factored Green operator);
 * x: a train; y0, z0: initial guesses (trains with A's output dims and x's
 * batch, any ranks; the caller draws them, typically at random), left
 * unchanged.  Optional outputs: the sweeps run and the last relative
 * change.  QTT_ECAPACITY when a local core exceeds 320 in its smaller
 * dimension. */
int tt_amen_apply(qtt_ctx* ctx, const qtt_tensor* A, const qtt_tensor* x,
                  const qtt_tensor* y0, const qtt_tensor* z0, double delta,
                  int cap, int sweeps, double tol, qtt_tensor** y,
                  int* sweeps_run, double* change);

/* In-place TT-rounding (Sec. 3): QR orthogonalisation sweep, then
 * truncated SVDs keeping per bond the smallest rank whose discarded
 * squared singular values sum to at most (delta / sqrt(L-1) ||x||)^2,
 * clipped to cap.  `discarded` (host, may be NULL) receives, per batch
 * element, sqrt(sum of discarded sigma^2) / ||x||. */
int tt_round(qtt_ctx* ctx, qtt_tensor* x, double delta, int cap,
             double* discarded);

/* Frobenius norms of each batch element (host out[batch]), computed from
 * an orthogonalisation sweep in FP64. */
int tt_norm(qtt_ctx* ctx, const qtt_tensor* x, double* out);

/* z = alpha x + beta y (ranks add, Table 2), alpha/beta real. */
int tt_axpby(qtt_ctx* ctx, double alpha, const qtt_tensor* x, double beta,
             const qtt_tensor* y, qtt_tensor** z);

/* Volume average of A(x) : x over all voxels (host out[batch][6], complex
 * interleaved): the mean stress term of Sec. 2 for A = C - C0 or C. */
int tt_mean_apply(qtt_ctx* ctx, const qtt_tensor* A, const qtt_tensor* x,
                  double* out);

/* ---- solvers ------------------------------------------------------------ */
/* Alg. 2 for the unit load cases selected by P->load_mask, then
 * C_eff[:, k] = < C eps^k > (Sec. 2).  Ceff: host [36], row-major.
 * eps_out (optional): receives the converged strain trains (batch = number
 * of solved load cases, in increasing k).  Returns QTT_ENOCONV when a load
 * case reached max_iter (Ceff and R still filled). */
int ls_solve(qtt_ctx* ctx, const qtt_problem* P, const qtt_solve_opts* O,
             double* Ceff, qtt_report* R, qtt_tensor** eps_out);

/* Adjoint Lippmann-Schwinger solve and gradient of C_eff with respect to
 * the phase Lame parameters theta = (lam_0, mu_0, lam_1, mu_1, ...), C0
 * held fixed.  For each load case k the adjoint fixed point
 * w_k = C e_k - (C - C0) G[w_k] (G = S^H Gamma S) is iterated with the
 * adjoint operators, then dC_kl/dtheta = <e_k, dC eps^l> - <w_k, G dC eps^l>.
 * V is the Voigt dimension of the problem: 6, or 3 for plane strain
 * (P->dim = 2).  eps: the V converged forward trains (from ls_solve with
 * every load case), else QTT_EINVAL.  gbar: host [V][V] row-major
 * cotangent of C_eff or NULL; grad: host, [2 nphase] if gbar is given,
 * else the full Jacobian [V][V][2 nphase]. */
int ls_adjoint(qtt_ctx* ctx, const qtt_problem* P, const qtt_solve_opts* O,
               const qtt_tensor* eps, const double* gbar, double* grad,
               qtt_report* R);

/* Operator setup separated from the fixed-point loop: builds the SFFT, the
 * Green operator and the stiffness operator of a problem once (the
 * preprocessing of App. D) so that ls_solve_prepared times only Alg. 2.
 * The prepared object keeps its own copies of the problem data. */
typedef struct qtt_prepared qtt_prepared;
int qtt_prepare(qtt_ctx* ctx, const qtt_problem* P, double delta,
                qtt_prepared** out);
int qtt_prepared_destroy(qtt_prepared* prep);
/* ls_solve on a prepared problem; load cases from P->load_mask as given
 * to qtt_prepare.  Same outputs and codes as ls_solve. */
int ls_solve_prepared(qtt_ctx* ctx, const qtt_prepared* prep,
                      const qtt_solve_opts* O, double* Ceff, qtt_report* R,
                      qtt_tensor** eps_out);
/* ls_adjoint on a prepared problem (the operators are not rebuilt): eps
 * from ls_solve_prepared of the same prepared object; same outputs and
 * codes as ls_adjoint. */
int ls_adjoint_prepared(qtt_ctx* ctx, const qtt_prepared* prep,
                        const qtt_solve_opts* O, const qtt_tensor* eps,
                        const double* gbar, double* grad, qtt_report* R);

/* The C_eff returned by exactly `steps` updates of Alg. 2 for all V unit
 * load cases (no stopping test; O->tol and O->max_iter are not used) and,
 * if grad is not NULL, its exact derivative with respect to the phase Lame
 * parameters (C0 fixed): the reverse mode of those updates (Sec. 2's
 * fixed point, Alg. 2's update), the rounding of each update held fixed.
 * It is the derivative of what a truncated solve returns, where
 * ls_adjoint gives that of the converged fixed point.  Every `every`-th
 * iterate is kept on the device (every = 0 or 1: all of them, nothing is
 * recomputed); the reverse sweep recomputes the others from them with the
 * forward pass's own sketches, one segment of `every` updates at a time. 
 * Ceff: host [36] (plane problems: rows and columns 0..2).  gbar, grad:
 * as in ls_adjoint ([V][V] cotangent or NULL; [2 nphase] or the Jacobian
 * [V][V][2 nphase]).  R->iterations = steps, R->residual = the last
 * update's relative change.  The V load cases run as one train batch on
 * the context's stream (O->streams is not used).  QTT_EINVAL: steps
 * outside 1..100000, every < 0, or O->matvec other than QTT_MV_SKETCH. */
int ls_unrolled(qtt_ctx* ctx, const qtt_problem* P, const qtt_solve_opts* O,
                int steps, int every, const double* gbar, double* Ceff,
                double* grad, qtt_report* R);
/* ls_unrolled on a prepared problem (the operators are not rebuilt). */
int ls_unrolled_prepared(qtt_ctx* ctx, const qtt_prepared* prep,
                         const qtt_solve_opts* O, int steps, int every,
                         const double* gbar, double* Ceff, double* grad,
                         qtt_report* R);

/* The strided batched complex FP64 GEMM that every core contraction of
 * the path runs on (the products of App. C and the factorisations of the
 * rounding, Sec. 3 around eq. rounding_condition_tt):
 *   C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b],   b < batch,
 * op(A) is M x K: op 0 (N) reads A[m*lda + k], op 1 (T) reads A[k*lda + m],
 * op 2 (C) reads conj(A[k*lda + m]); op(B) is K x N likewise.  A, B, C are
 * caller-owned DEVICE pointers to interleaved complex doubles, row-major,
 * batch strides sA/sB/sC in complex elements; alpha, beta are host
 * {re, im}.  The library cannot see the extent of caller memory: the
 * caller guarantees every addressed element lies in its allocation.
 * path: 0 automatic (matrix cores for M, N >= 16 and K >= 4, else vector
 * ALU), 1 vector ALU, 2 matrix cores (QTT_EINVAL if the shape is outside
 * its range), 3 matrix cores with FP32 operands and accumulation (the
 * contraction precision of QTT_PREC_FP32; results stored as doubles),
 * 4 + t matrix cores in FP64 with tile variant t forced instead of chosen
 * per shape (t = 0..6: 16x16, 32x32, 64x64, 80x80, 32x80, 80x32, 64x80;
 * for tests and tuning), QTT_GEMM_PATH_BF16X3 matrix cores with split-BF16
 * operands and FP32 accumulation (the contraction precision of
 * QTT_PREC_BF16X3; results stored as doubles).
 * Asynchronous on the context's stream.  QTT_EINVAL on null pointers,
 * K < 1, batch outside [1, 65535] or leading dimensions smaller than a
 * row. */
#define QTT_GEMM_PATH_BF16X3 16
int qtt_zgemm(qtt_ctx* ctx, int opA, int opB, int M, int N, int K,
              const double* alpha, const void* A, long lda, const void* B,
              long ldb, const double* beta, void* C, long ldc, int batch,
              long sA, long sB, long sC, int path);

/* The two small dense factorisations of TT-rounding (Sec. 3, QR sweep and
 * truncated SVD around eq. rounding_condition_tt),
 * exposed for direct testing and timing.  Device pointers, interleaved
 * complex doubles, row-major, batch stride = one matrix, caller-owned.
 *
 * qtt_zqr: Householder QR of batch m x n matrices A (k = min(m, n)):
 * R (k x n, upper trapezoidal, real diagonal) and, if Q != NULL, Q (m x k,
 * orthonormal columns) with A = Q R.  path 0: the kernels the library
 * uses, 1: the global-memory kernel, 2: the blocked matrix-core kernel
 * (m >= n, 16 < n <= 96, m <= 192), 3: the register-resident unblocked
 * kernels (m <= 256, n <= 128), 4: the two-columns-per-lane register
 * kernel (n <= 96), 5: the one-wave-per-column-group kernel for R (m <=
 * 160, n <= 96) with Q from the matrix-core block reflectors (Q needs
 * m >= n > 16), 6: the workspace-resident blocked kernel with trailing
 * updates and Q formation on the matrix cores (m >= n, m <= 320, n <= 160;
 * the library's choice beyond 192 rows or 96 columns); QTT_EINVAL when the
 * forced path does not cover the shape.
 * Synchronises the stream before returning.
 *
 * qtt_zjacobi: one-sided Jacobi of batch n x n matrices A (n <= 320):
 * A V = U diag(S) with U (n x n) orthonormal columns for the nonzero S
 * (zero columns otherwise) and S (batch x n) descending; V is not formed.
 * Up to n = 96 the matrix is held in LDS; beyond, its first columns stay
 * in LDS and the rest live in a library workspace.  QTT_EINVAL for
 * n > 320. */
int qtt_zqr(qtt_ctx* ctx, int batch, int m, int n, const void* A, void* R,
            void* Q, int path);
int qtt_zjacobi(qtt_ctx* ctx, int batch, int n, const void* A, void* U,
                double* S);

/* qtt_zorth: orthonormal basis of the column space of batch m x n
 * matrices A (m >= n, 32 < m <= 192 for 16 < n <= 64, 32 < m <= 168 for
 * 64 < n <= 80): Q (m x n) with
 * Q^H Q = I and range(Q) = range(A) -- the factor the range finder of
 * TT-rounding keeps (Sec. 3).  CholeskyQR2 on the FP64 matrix cores, one
 * workgroup per matrix; a matrix whose first Cholesky breaks down (a pivot
 * at or below 1e-12 of the largest diagonal entry of A^H A) or whose
 * first-pass columns are farther than 0.5 (Frobenius) from orthonormal is
 * factored by Householder QR instead.  fallback (host array of batch ints,
 * may be NULL) receives 1 for each matrix that took Householder, else 0.
 * Same layouts as qtt_zqr; QTT_EINVAL outside the covered shapes.
 * path 0: each pass spread over the device (partial Grams per 32-row
 * slice, one workgroup per matrix for the Cholesky and R^-1, the products
 * on the matrix-core GEMM; the library's choice); 1: one fused workgroup
 * per matrix; 2: as 0, but a column dependent on the earlier ones to
 * rounding (pivot at most 1e-13 of the largest) gives an exactly zero
 * column of Q instead of a fallback (Q^H Q is I on the kept columns, zero
 * on the dropped ones; the form the range finder uses).  Synchronises the
 * stream before returning. */
int qtt_zorth(qtt_ctx* ctx, int batch, int m, int n, const void* A, void* Q,
              int* fallback, int path);

/* qtt_zqr without any allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): the same factorisation as qtt_zqr with path 0 (same
 * arguments, layouts and results), but its workspace is a fixed device
 * array of QTT_ZQR_NOALLOC_MAX_ELEMS complex doubles (16 MiB) that the
 * library holds on every GPU it runs on until the process ends, and the
 * call neither allocates, frees nor synchronises: it is enqueued on the
 * context's stream and complete when that stream reaches it.
 * QTT_ECAPACITY (with a message) when batch * (workspace of one m x n
 * matrix) exceeds the array: 288 x 144 takes 85,392 entries per matrix, so
 * up to 12 such matrices per call.  Every call on one GPU shares that GPU's
 * array: calls whose execution overlaps on one GPU (other contexts or
 * streams) race on it and must be serialised by the caller. */
#define QTT_ZQR_NOALLOC_MAX_ELEMS 1048576
int qtt_zqr_noalloc(qtt_ctx* ctx, int batch, int m, int n, const void* A,
                    void* R, void* Q);

/* Kernel statistics for roofline accounting.  qtt_stats_enable(ctx, s)
 * with s >= 1 brackets every s-th launch of the library's kernels by HIP
 * events on the context's stream (s = 1: every launch; a larger s keeps
 * the event records' own cost out of a timed run), 0 turns statistics
 * off, negative s is QTT_EINVAL.  The matrix-core GEMM (QTT_K_MFMA,
 * QTT_K_MFMA32) is timed by the kernel itself: the span from its first
 * workgroup's start to its last workgroup's end on the device's
 * constant-rate real-time counter (the interval a kernel-trace profiler
 * reports).  Every other family is timed by a HIP event pair from the end
 * of the preceding work on the stream to the end of the launch, dispatch
 * gap included.  With concurrent load-case groups (qtt_solve_opts.streams
 * > 1) kernels of different groups share the device and each duration
 * includes that sharing.  qtt_stats_get synchronises and returns, for one kernel family
 * (QTT_K_*) and over the timed launches only, their number, the summed
 * event time in seconds, and their algorithmic FP64 flops and HBM bytes
 * (counted from the operand shapes, not measured); qtt_stats_get_all
 * returns the number, flops and bytes of every launch (timed or not).
 * qtt_stats_reset clears both and restarts the sampling. */
#define QTT_K_GEMM      0   /* batched complex GEMM, vector ALU kernel      */
#define QTT_K_QR        1   /* Householder QR                               */
#define QTT_K_JACOBI    2   /* one-sided Jacobi SVD                         */
#define QTT_K_APPLY     3   /* materialised TTO x TT core product           */
#define QTT_K_OTHER     4   /* elementwise helpers, RNG                     */
#define QTT_K_MFMA      5   /* batched complex GEMM on the matrix cores     */
#define QTT_K_MFMA32    6   /* the same in FP32 (QTT_PREC_FP32 contractions) */
#define QTT_K_CONTRACT  7   /* the operator x train core contractions inside
                               products (TTO apply as the rounding runs it:
                               operator core times partial contraction), any
                               GEMM path */
#define QTT_K_MFMA_BF16 8   /* matrix-core GEMM with split-BF16 operands
                               (QTT_PREC_BF16X3 products outside the
                               contraction family)                         */
#define QTT_K_COUNT     9
int qtt_stats_enable(qtt_ctx* ctx, int on);
int qtt_stats_get(qtt_ctx* ctx, int family, long long* launches,
                  double* seconds, double* flops, double* bytes);
int qtt_stats_get_all(qtt_ctx* ctx, int family, long long* launches,
                      double* flops, double* bytes);
int qtt_stats_reset(qtt_ctx* ctx);

/* Many problems in one call (the six load cases of each are batched
 * together; problems are grouped by grid size).  Ceff: host [count][36]. */
int qtt_batch_solve(qtt_ctx* ctx, int count, const qtt_problem* Ps,
                    const qtt_solve_opts* O, double* Ceff, qtt_report* Rs);

#ifdef __cplusplus
}
#endif
#endif /* QTTHOM_H */
