/*
 * sketchne.h -- C ABI of the MI355X (gfx950) SketchNE hot path.
 *
 * The method (SketchNE, TKDE 2023, arXiv 2110.12782) embeds a graph by
 *   1. a randomized eigendecomposition of D^-a A D^-a     (Alg. 5, Alg. 6 line 1)
 *   2. the low-rank factors L', R' of Eq. (11)            (Alg. 6 lines 2-3)
 *   3. the sparse-sign single-pass sketch of f(L'R')      (Alg. 3, Eq. 4, Alg. 4 lines 2-4, 6-7)
 *   4. the reduced matrix W, its SVD and E = U_d S_d^1/2  (Alg. 4 lines 5, 8-10, Alg. 6 line 5)
 * where f = trunc_log (Eq. 1).  The n x n matrix f(L'R') is never formed.
 *
 * Conventions for every entry point
 *   - Array arguments are DEVICE pointers unless marked "host".  Dense
 *     matrices are row-major with the stated leading dimension.
 *   - The caller owns every buffer, including the workspace.  The library
 *     allocates no device memory and keeps no pointer after a call returns,
 *     except for the work it enqueued on the context's stream; keep buffers
 *     alive until sketchne_sync() (or a sync of that stream).
 *   - Arguments are validated before anything is enqueued.  On SKETCHNE_E_ARG
 *     or SKETCHNE_E_WORKSPACE nothing was enqueued and outputs are untouched.
 *   - Numerical breakdown detected on the device (a Cholesky pivot that is
 *     not positive, an eigensolver that did not converge, a non-finite Ritz
 *     value) sets a device flag; sketchne_sync() reports it as
 *     SKETCHNE_E_NUMERIC.  Output contents are then unspecified.
 *   - No C++ exception crosses this boundary.
 *   - Workspace pointers must be 256-byte aligned.
 *   - Graphs are undirected and unweighted: the CSR pattern is symmetric,
 *     rows are sorted, there are no self loops and no duplicate entries
 *     (A_ij in {0,1}); vol(G) = nnz (Section 2).  An isolated vertex has all
 *     its degree powers taken as 0, so its rows of U, Y and E are 0.
 */
#ifndef SKETCHNE_H
#define SKETCHNE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SKETCHNE_OK = 0,
  SKETCHNE_E_ARG = 1,         /* invalid argument; nothing enqueued            */
  SKETCHNE_E_WORKSPACE = 2,   /* workspace null, too small or misaligned       */
  SKETCHNE_E_DEVICE = 3,      /* HIP runtime / launch failure                  */
  SKETCHNE_E_NUMERIC = 4,     /* device-side numerical breakdown (at sync)     */
  SKETCHNE_E_UNSUPPORTED = 5  /* size or option outside what this build runs   */
} sketchne_status;

/* Input type of the fused sketch GEMM (accumulation is FP32 in every case). */
typedef enum { SKETCHNE_FP32 = 0, SKETCHNE_BF16 = 1, SKETCHNE_FP16 = 2 } sketchne_precision;

/* Numeric flag bits returned by sketchne_sync(). */
#define SKETCHNE_FLAG_CHOL_SHIFT   0x1u  /* a Cholesky needed a diagonal shift        */
#define SKETCHNE_FLAG_CHOL_FAIL    0x2u  /* a Cholesky failed even after the shift    */
#define SKETCHNE_FLAG_EIG_NOCONV   0x4u  /* Jacobi reached its sweep limit            */
#define SKETCHNE_FLAG_NONFINITE    0x8u  /* non-finite eigenvalue / singular value    */
#define SKETCHNE_FLAG_BAD_INDEX    0x10u /* a test-matrix row outside [0, n) was read  */
#define SKETCHNE_FLAG_BARRIER      0x20u /* a grid barrier of the Cholesky or Jacobi
                                          * kernel waited over a second (workgroups not
                                          * all resident): the results are invalid   */

/* Workspace query operations (bitmask: the size covers every op named). */
#define SKETCHNE_OP_EIG    0x1
#define SKETCHNE_OP_SKETCH 0x2
#define SKETCHNE_OP_EMBED  0x4
#define SKETCHNE_OP_SPMM   0x8

typedef struct sketchne_ctx sketchne_ctx;

/* An undirected graph G = (V, E, A) in CSR, n vertices, nnz = 2m stored entries. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* rowptr; /* device, n+1 */
  const int32_t* colidx; /* device, nnz */
} sketchne_graph;

/* Hyper-parameters (Table 1 notation; Alg. 4, 5, 6). */
typedef struct {
  double alpha;      /* a in D^-a A D^-a, 0 < a <= 0.5 (Section 3.2)                 */
  int32_t T;         /* context window size, >= 1 (Eq. 1)                             */
  double b;          /* number of negative samples, > 0 (Eq. 1)                       */
  int32_t k;         /* eigen rank (Alg. 5)                                           */
  int32_t s_eig;     /* oversampling of Alg. 5; K = k + s_eig start columns           */
  int32_t q;         /* power iterations of Alg. 5, >= 0                              */
  int32_t d;         /* embedding dimension                                          */
  int32_t h;         /* columns of the test matrix S, d <= h (Alg. 4: h = d + s1)     */
  int32_t l;         /* columns of the test matrix O, h <= l (Alg. 4: l = d + s2)     */
  int32_t z;         /* nonzeros per test-matrix column, 1 <= z <= n (Alg. 3)         */
  uint64_t seed;     /* seed of the device generators (Omega, S, O)                   */
  int32_t precision; /* sketchne_precision of the fused sketch GEMM                   */
  int32_t split_r;   /* BF16/FP16: leading components carried as hi+lo pairs (0..k)  */
} sketchne_params;

/* A sparse-sign test matrix (Alg. 3) of size n x cols with z nonzeros per
 * column.  Column c owns rows[c*z .. c*z+z-1] (distinct, in [0, n)) with signs
 * signs[c*z .. c*z+z-1] in {-1, +1}; the entry value is sign / sqrt(z). */
typedef struct {
  int32_t cols;
  int32_t z;
  int32_t* rows;   /* device, cols*z */
  int8_t* signs;   /* device, cols*z */
} sketchne_sparse_sign;

const char* sketchne_status_str(sketchne_status s);

/* Context bound to a device and a caller-owned HIP stream (NULL = default
 * stream).  One context per host thread.  The context owns a few bytes of
 * device flags and pinned host memory, released by sketchne_destroy. */
sketchne_status sketchne_create(sketchne_ctx** ctx, int device, void* hip_stream);
sketchne_status sketchne_destroy(sketchne_ctx* ctx);
sketchne_status sketchne_set_stream(sketchne_ctx* ctx, void* hip_stream);

/* Bytes of workspace needed by the operations in op_mask for a graph of n
 * vertices and nnz entries (*bytes is host memory). */
sketchne_status sketchne_workspace_size(const sketchne_params* p, int64_t n, int64_t nnz,
                                        int op_mask, size_t* bytes);

/* Alg. 5 on X = D^-a A D^-a (Alg. 6 line 1): Y = X Omega, Q = orth(Y),
 * q times Q = orth(X(XQ)), Rayleigh-Ritz on Q^T X Q, eigenpairs sorted by
 * |lambda| descending (ties: lambda descending, then index).
 *   omega0: n x (k+s_eig) row-major start block, or NULL to draw a standard
 *           Gaussian block on the device from p->seed.
 *   U:      n x k row-major FP32 output (orthonormal columns).
 *   lambda: k FP64 output.
 * Requires k + s_eig <= 288 (order of the Rayleigh-Ritz eigensolver) and
 * (k + s_eig) % 4 == 0.
 * Orthonormalisation is Cholesky-QR with FP64 Gram and Cholesky; a second
 * pass runs only when the first factor's 1-norm condition number (Gram
 * scaled to unit diagonal) exceeds 1e5 or its Cholesky needed a shift. */
sketchne_status sketchne_eig(sketchne_ctx* ctx, const sketchne_graph* A, const sketchne_params* p,
                             const float* omega0, float* U, double* lambda,
                             void* ws, size_t ws_bytes);

/* Alg. 6 lines 2-3 and Alg. 4 lines 3-4, 6-7: forms L' and R' of Eq. (11)
 * from U, lambda and the degrees, then
 *   Y  = f(L'R') S           (n x h, written TRANSPOSED: Yt[c*n + i] = Y[i][c])
 *   Z  = O^T f(L'R') O       (l x l row-major)
 * visiting only the rows/columns of f(L'R') that S and O touch (Eq. 4).
 * If generate != 0, S and O are drawn on the device from p->seed and written
 * into S->rows/signs and O->rows/signs; otherwise they are read from there.
 * S->cols must equal h, O->cols must equal l, and both z must equal p->z.
 * Requires z <= 8 and k % 4 == 0. */
sketchne_status sketchne_sketch(sketchne_ctx* ctx, const sketchne_graph* A, const sketchne_params* p,
                                const float* U, const double* lambda,
                                sketchne_sparse_sign* S, sketchne_sparse_sign* O, int generate,
                                float* Yt, float* Z, void* ws, size_t ws_bytes);

/* Alg. 4 lines 5, 8-10 and Alg. 6 line 5: Q = orth(Y); W = (O^T Q)^+ Z (Q^T O)^+
 * by two least-squares solves (QR of O^T Q, FP64); SVD of W (W is symmetric
 * because Z is, so its SVD is taken from a symmetric eigendecomposition with
 * singular values |eigenvalue|); E = Q U^(:, 1:d) diag(sigma)^1/2.
 *   Yt: h x n (as written by sketchne_sketch); Z: l x l; O: the test matrix of Z.
 *   E:  n x d row-major FP32 output; sigma: d FP64 output, descending.
 * Requires h <= 288 (order of the eigensolver for W). */
sketchne_status sketchne_embed(sketchne_ctx* ctx, const sketchne_params* p, int64_t n,
                               const float* Yt, const float* Z, const sketchne_sparse_sign* O,
                               float* E, double* sigma, void* ws, size_t ws_bytes);

/* ---- Full-visit variant ------------------------------------------------ */
/* The sparse-sign test matrices of Alg. 3 with their z nonzeros placed in
 * every ROW (one set per vertex) instead of every column:
 *   Y = f(L'R') S (n x h, written transposed: Yt),  Z = O^T f(L'R') O (l x l),
 * with S (n x h) and O (n x l) holding z nonzeros +-1/sqrt(z) per row, so
 * every one of the n^2 entries of f(L'R') is formed (nothing is sampled).
 * Each tile of f(L'R') is formed on the matrix cores and multiplied by the
 * matching rows of S (or O) on the matrix cores, never leaving registers.
 * L', R' as in sketchne_sketch (Eq. 11); precision FP32 or BF16 (FP16 is
 * SKETCHNE_E_UNSUPPORTED); S->width = h, O->width = l <= 8192 (else
 * SKETCHNE_E_UNSUPPORTED), both z = p->z <= h.  Z = O^T T is summed in 64-bit
 * fixed point, so repeated calls give identical bits.
 * sketchne_embed_fullvisit is sketchne_embed (Alg. 4 lines 5, 8-10) with that
 * O.  Workspace: sketchne_fullvisit_workspace_size (the sketch's holds
 * f(L'R') O, l x n; the embed's holds O as a dense l-column matrix). */
typedef struct {
  int32_t width;   /* columns of the test matrix                               */
  int32_t z;       /* nonzeros per row                                          */
  int32_t* cols;   /* device, n*z: row i owns cols[i*z .. i*z+z-1], distinct in [0, width) */
  int8_t* signs;   /* device, n*z: +-1 (value sign / sqrt(z))                  */
} sketchne_row_sign;

sketchne_status sketchne_fullvisit_workspace_size(const sketchne_params* p, int64_t n, int op_mask, size_t* bytes);
sketchne_status sketchne_sketch_fullvisit(sketchne_ctx* ctx, const sketchne_graph* A, const sketchne_params* p,
                                          const float* U, const double* lambda, sketchne_row_sign* S,
                                          sketchne_row_sign* O, int generate, float* Yt, float* Z, void* ws,
                                          size_t ws_bytes);
sketchne_status sketchne_embed_fullvisit(sketchne_ctx* ctx, const sketchne_params* p, int64_t n, const float* Yt,
                                         const float* Z, const sketchne_row_sign* O, float* E, double* sigma,
                                         void* ws, size_t ws_bytes);

/* ---- General single pass (Eqs. 5-10) ---------------------------------- */
/* The single-pass SVD of a target f(LR) that need not be symmetric (for
 * instance the matrix of a directed graph), f = trunc_log, with four
 * sparse-sign test matrices C, S (n x h) and H, O (n x l), Eq. (5):
 *   K = f(LR)^T C   (n x h, written TRANSPOSED: Kt[c*n + i] = K[i][c])
 *   Y = f(LR) S     (n x h, written transposed: Yt)
 *   Z = H^T f(LR) O (l x l row-major)
 * visiting only the entries of f(LR) the test matrices touch.
 *   L:  n x k row-major FP32 (the left factor); Rt: n x k row-major FP32,
 *       the TRANSPOSE of the right factor R (k x n).
 *   p:  h, l, z, precision (FP32 or BF16; FP16 is SKETCHNE_E_UNSUPPORTED
 *       here: the factors carry no range bound) and split_r are read; k is
 *       the argument.  C, S have h columns, H, O have l, all with p->z
 *       nonzeros per column (z <= 8).
 * sketchne_embed_general then forms, Eqs. (6)-(10), P = orth(K), Q = orth(Y)
 * (Cholesky-QR, kept implicit), W = (H^T Q)^+ Z (P^T O)^+ by two FP64
 * least-squares solves, the SVD W = U^ Sigma V^^T (one-sided Jacobi, h <= 288)
 * and the two d-dimensional embeddings
 *   E  = Q U^(:, 1:d) Sigma_d^1/2      (n x d FP32, the column side)
 *   Ed = P V^(:, 1:d) Sigma_d^1/2      (n x d FP32, the row side)
 * with sigma (d FP64) descending.  For a symmetric target with C = S and
 * H = O this is the single pass of Alg. 4.
 * Workspace: sketchne_general_workspace_size(p, n, k, SKETCHNE_OP_SKETCH |
 * SKETCHNE_OP_EMBED); the embed step reads k = h. */
sketchne_status sketchne_general_workspace_size(const sketchne_params* p, int64_t n, int32_t k, int op_mask,
                                                size_t* bytes);
sketchne_status sketchne_sketch_general(sketchne_ctx* ctx, int64_t n, int32_t k, const float* L, const float* Rt,
                                        const sketchne_params* p, const sketchne_sparse_sign* C,
                                        const sketchne_sparse_sign* S, const sketchne_sparse_sign* H,
                                        const sketchne_sparse_sign* O, float* Kt, float* Yt, float* Z, void* ws,
                                        size_t ws_bytes);
sketchne_status sketchne_embed_general(sketchne_ctx* ctx, const sketchne_params* p, int64_t n, const float* Kt,
                                       const float* Yt, const float* Z, const sketchne_sparse_sign* H,
                                       const sketchne_sparse_sign* O, float* E, float* Ed, double* sigma, void* ws,
                                       size_t ws_bytes);

/* Wait for the context's stream; *flags (host, nullable) receives the OR of
 * the numeric flag bits raised since the previous sync.  Returns
 * SKETCHNE_E_NUMERIC if CHOL_FAIL, EIG_NOCONV or NONFINITE was raised, and
 * SKETCHNE_E_ARG if BAD_INDEX was raised (such a row contributes zero). */
sketchne_status sketchne_sync(sketchne_ctx* ctx, uint32_t* flags);

/* ---- Steps of the path, exposed for composition and testing ------------ */

/* C = D^-a A D^-a B (the SpMM of Alg. 5 lines 4, 6, 9; Section 3.4).
 * B: n x cols (ld ldb), C: n x cols (ld ldc), FP32; cols % 4 == 0, cols <= 512;
 * ldb, ldc multiples of 4.  B and C must not overlap. */
sketchne_status sketchne_spmm(sketchne_ctx* ctx, const sketchne_graph* A, double alpha,
                              const float* B, int64_t ldb, int32_t cols,
                              float* C, int64_t ldc, void* ws, size_t ws_bytes);

/* In-place orthonormalisation of the columns of B (n x cols, FP32, packed:
 * ldb == cols): Cholesky-QR with FP64 Gram and Cholesky, repeated once when
 * the first factor is ill-conditioned (the orth of Alg. 5).  cols <= 288
 * (SKETCHNE_E_UNSUPPORTED beyond, or when ldb != cols).
 * Workspace: sketchne_orth_workspace_size(). */
sketchne_status sketchne_orth_workspace_size(int64_t n, int32_t cols, size_t* bytes);
sketchne_status sketchne_orth(sketchne_ctx* ctx, int64_t n, int32_t cols, float* B, int64_t ldb,
                              void* ws, size_t ws_bytes);

/* Symmetric eigendecomposition of the m x m FP64 matrix A (only its upper
 * triangle is read) by one-sided block Jacobi on A + ||A||_F I:
 * A = V diag(w) V^T, pairs sorted by |w| descending (ties: w descending,
 * then index).  V: m x m row-major, column j = eigenvector j.  m <= 288. */
sketchne_status sketchne_symeig_workspace_size(int32_t m, size_t* bytes);
sketchne_status sketchne_symeig(sketchne_ctx* ctx, int32_t m, const double* A, double* V, double* w,
                                void* ws, size_t ws_bytes);

/* ---- Spectral propagation (Alg. 6 line 6) ------------------------------ */
/* E_out = sum_{r=0..p} c_r T_r(L - I) E with L = I - D^-1 A the random-walk
 * Laplacian of Alg. 6 and T_r the Chebyshev polynomials of the first kind
 * (T_0 = I, T_1(M) = M, T_{r+1}(M) = 2 M T_r(M) - T_{r-1}(M)); L - I = -D^-1 A
 * has its spectrum in [-1, 1], where this recurrence is stable.  The paper
 * names the Chebyshev coefficients c_r and the degree p (10 by default) and
 * takes the step from ProNE; sketchne_propagate_coeffs() gives the reading
 * used here: c_r interpolate ProNE's band-pass filter
 *     g(lambda) = exp(-theta/2 ((lambda - mu)^2 - 1))
 * on the Laplacian spectrum lambda in [0, 2] at the p + 1 Chebyshev nodes
 * lambda_j = 1 + cos(pi (j + 1/2) / (p + 1)) (theta = 0.5, mu = 0.2 in the
 * paper's ProNE settings).  An isolated vertex has a zero row in D^-1 A.
 *   E:    n x d FP32 (ld lde), read only; out: n x d FP32 (ld ldo), written;
 *         they must not overlap; both 16-byte aligned, d % 4 == 0, d <= 256,
 *         lde and ldo multiples of 4.
 *   coef: host, p + 1 doubles (c_0 .. c_p), 0 <= p <= 64.
 * Every step is one fused SpMM (neighbour sum, recurrence and running sum);
 * T_r lives in the workspace (two n x d blocks).  Arithmetic is FP32. */
sketchne_status sketchne_propagate_coeffs(int32_t p, double theta, double mu, double* coef /* host, p+1 */);
sketchne_status sketchne_propagate_workspace_size(int64_t n, int64_t nnz, int32_t d, size_t* bytes);
sketchne_status sketchne_propagate(sketchne_ctx* ctx, const sketchne_graph* A, int32_t d, const float* E,
                                   int64_t lde, int32_t p, const double* coef, float* out, int64_t ldo, void* ws,
                                   size_t ws_bytes);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): sketchne_symeig
 * without a workspace argument.  Its scratch (the padded column block,
 * rotation counts, grid barrier count and shift of the eigensolver, 664,064
 * bytes, enough for m <= 288) is a device array inside the library, one per
 * device, held until the process ends; its address is looked up once per
 * device by sketchne_create.  m > 288 returns SKETCHNE_E_UNSUPPORTED;
 * SKETCHNE_E_DEVICE if the scratch could not be located.  The call
 * allocates nothing (the eigensolver is four launches, the sweeps among
 * them one launch of at most nine workgroups that must all be resident at
 * once).  Every call on a device shares that device's scratch, which keeps
 * the last call's contents (each call initialises what it reads): calls that
 * overlap on one device -- from two streams or two contexts -- race and must
 * be serialised by the caller.  Results equal sketchne_symeig's. */
sketchne_status sketchne_symeig_noalloc(sketchne_ctx* ctx, int32_t m, const double* A, double* V, double* w);

/* Device generators (counter-based SplitMix64, Steele, Lea & Flood 2014).
 * gauss: n x cols standard normal block (Box-Muller in FP32).
 * sparse_sign: fills out->rows/signs for an n-row test matrix (Alg. 3). */
sketchne_status sketchne_gen_gauss(sketchne_ctx* ctx, int64_t n, int32_t cols, uint64_t seed,
                                   float* out);
sketchne_status sketchne_gen_sparse_sign(sketchne_ctx* ctx, int64_t n, uint64_t seed,
                                         sketchne_sparse_sign* out);

/* ---- Learned warm start of Alg. 5 ------------------------------------- */
/* An addition to the method (Alg. 5 draws a Gaussian start block Omega):
 * a 3-layer ReLU network maps per-vertex features to the first out <= k
 * columns of Omega; the other columns stay Gaussian, and the plain Gaussian
 * start remains the fallback.
 *   features   phi_i = [log max(deg_i,1), (X^3 G)_i1 .. (X^3 G)_i4,
 *                       (X^4 G)_i1 .. (X^4 G)_i3]
 *              with X = D^-a A D^-a and G an n x SKETCHNE_WS_PROBES block of
 *              Rademacher vectors (powers of independent probes are random
 *              combinations of the leading eigenvectors), each column
 *              standardised over the vertices to mean 0 and standard deviation
 *              1 (a column whose standard deviation is at most 1e-6 times its
 *              root mean square is set to 0); SKETCHNE_WS_RAW of the
 *              SKETCHNE_WS_FEAT columns are used (the rest are 0); phi is
 *              n x SKETCHNE_WS_FEAT FP32.
 *   network    F = relu(relu(phi W1 + b1) W2 + b2) W3 + b3   (n x out FP32)
 *   loss       L = ||(I - U U^T) F||_F^2 / ||F||_F^2
 *                  + mu || (out / ||F||_F^2) F^T F - I ||_F^2
 *              for reference eigenvectors U (n x out, orthonormal columns).
 * Parameters are one flat array in the order W1 (FEAT x width), b1 (width),
 * W2 (width x width), b2 (width), W3 (width x out), b3 (out), row-major.
 * The forward pass reads the BF16 copy; Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected) updates the FP32 master and rewrites the BF16
 * copy (round to nearest even).  Products run on the FP32 matrix cores with
 * FP32 accumulation; reductions over vertices use a fixed order. */
#define SKETCHNE_WS_FEAT 8
#define SKETCHNE_WS_RAW 8
#define SKETCHNE_WS_PROBES 4

typedef struct {
  int32_t width;     /* hidden width, >= 1                                    */
  int32_t out;       /* output columns (the k of the eigensolver it starts)   */
  float* master;     /* device, FP32 master parameters                         */
  uint16_t* bf16;    /* device, BF16 copy of the parameters (forward pass)      */
  float* adam_m;     /* device, Adam first moments (NULL: inference only)       */
  float* adam_v;     /* device, Adam second moments (NULL: inference only)      */
} sketchne_mlp;

#define SKETCHNE_WS_OP_FEATURES 0x1
#define SKETCHNE_WS_OP_FORWARD  0x2
#define SKETCHNE_WS_OP_GRAD     0x4
#define SKETCHNE_WS_OP_RESIDUAL 0x8   /* k = p->k                               */
#define SKETCHNE_WS_OP_EIG      0x10  /* sketchne_eig_learned with p            */

/* Number of parameters (host). */
sketchne_status sketchne_ws_param_count(int32_t width, int32_t out, int64_t* count);
/* Workspace bytes for the operations in op_mask (host); p is read for
 * SKETCHNE_WS_OP_RESIDUAL and SKETCHNE_WS_OP_EIG (out = p->k there). */
sketchne_status sketchne_ws_workspace_size(const sketchne_params* p, int32_t width, int32_t out, int64_t n,
                                           int64_t nnz, int op_mask, size_t* bytes);
/* He initialisation N(0, 2/fan_in) of the weights from seed (the padded rows
 * of W1 are 0), zero biases and moments, BF16 copy. */
sketchne_status sketchne_ws_init(sketchne_ctx* ctx, const sketchne_mlp* net, uint64_t seed);
/* phi (n x SKETCHNE_WS_FEAT) for the graph; g (n x SKETCHNE_WS_PROBES
 * row-major, +-1) is the probe block, or NULL to draw it on the device from
 * seed. */
sketchne_status sketchne_ws_features(sketchne_ctx* ctx, const sketchne_graph* A, double alpha, const float* g,
                                     uint64_t seed, float* phi, void* ws, size_t ws_bytes);
/* F = network(phi): n x out written with leading dimension ldf >= out. */
sketchne_status sketchne_ws_forward(sketchne_ctx* ctx, const sketchne_mlp* net, int64_t n, const float* phi,
                                    float* F, int64_t ldf, void* ws, size_t ws_bytes);
/* The inference pass that sketchne_eig_learned runs: as sketchne_ws_forward,
 * but each hidden layer's output is rounded to BF16 (round to nearest even)
 * and layers 2 and 3 run on the BF16 matrix cores with FP32 accumulation.
 * Requires width == 256 and out a multiple of 32 up to 256
 * (SKETCHNE_E_UNSUPPORTED otherwise).  Workspace: SKETCHNE_WS_OP_FORWARD. */
sketchne_status sketchne_ws_infer(sketchne_ctx* ctx, const sketchne_mlp* net, int64_t n, const float* phi,
                                  float* F, int64_t ldf, void* ws, size_t ws_bytes);
/* Loss and its gradient with respect to every parameter (grad: param_count
 * FP32, overwritten; loss: one FP32, device) for reference U (n x out, ldu). */
sketchne_status sketchne_ws_grad(sketchne_ctx* ctx, const sketchne_mlp* net, int64_t n, const float* phi,
                                 const float* U, int64_t ldu, float mu, float* grad, float* loss, void* ws,
                                 size_t ws_bytes);
/* One Adam step (step counts from 1) with learning rate lr. */
sketchne_status sketchne_ws_adam(sketchne_ctx* ctx, const sketchne_mlp* net, const float* grad, float lr,
                                 int32_t step);
/* Training loop: steps of (gradient on set t mod nsets, Adam step step0 + t + 1).
 * phi[s], U[s] (host arrays of nsets device pointers): features (n[s] x FEAT)
 * and reference eigenvectors (n[s] x out, ld out) of training set s; n is a
 * host array.  losses: steps FP32 (device), the loss of each step before its
 * update.  Workspace: SKETCHNE_WS_OP_GRAD for the largest n, plus
 * param_count floats. */
sketchne_status sketchne_ws_train(sketchne_ctx* ctx, const sketchne_mlp* net, int32_t nsets,
                                  const float* const* phi, const float* const* U, const int64_t* n, int32_t steps,
                                  int32_t step0, float lr, float mu, float* losses, void* ws, size_t ws_bytes);
/* Ritz residuals res_j = ||X U_j - lambda_j U_j||_2, j < k (U: n x k, ld k;
 * k % 4 == 0; res: k FP64, device). */
sketchne_status sketchne_ritz_residual(sketchne_ctx* ctx, const sketchne_graph* A, double alpha, int32_t k,
                                       const float* U, const double* lambda, double* res, void* ws,
                                       size_t ws_bytes);
/* Alg. 5 from the learned start: features (probe drawn from p->seed), F into
 * the first net->out columns of Omega (net->out <= p->k), Gaussian in the
 * other k + s_eig - net->out, q_warm power iterations.  If the largest Ritz
 * residual exceeds res_threshold (or is not finite) the result is discarded
 * and sketchne_eig runs from the Gaussian start with p->q iterations;
 * *used_fallback (host) says which ran.  The residuals come from the
 * Rayleigh-Ritz data of the warm run (||XQv||^2 - lambda^2 with XQ already
 * formed), not from a further SpMM; *worst_residual (host, may be NULL)
 * receives their maximum.  Synchronizes the stream once (the residual test).
 * Workspace: sketchne_ws_workspace_size(.., SKETCHNE_WS_OP_EIG, ..). */
sketchne_status sketchne_eig_learned(sketchne_ctx* ctx, const sketchne_graph* A, const sketchne_params* p,
                                     const sketchne_mlp* net, int32_t q_warm, double res_threshold, float* U,
                                     double* lambda, int32_t* used_fallback, double* worst_residual, void* ws,
                                     size_t ws_bytes);

/* ---- Per-kernel-class timing (measurement support) --------------------- */
/* When enabled, every launch of a timed kernel class is bracketed by HIP
 * events on the context's stream.  on = 0 stops timing (and resets the
 * sums), on = 1 times every class, and on = SKETCHNE_PROF_SELECT | (1 <<
 * class) | ... times only the named classes: the others then run without
 * events, which cost about 10 us of idle stream time per bracketed launch
 * group.  Any other value is SKETCHNE_E_ARG.  sketchne_profile_read()
 * synchronizes and returns, per class, the summed milliseconds and the
 * launch count since the last reset (host arrays of length
 * SKETCHNE_PROF_CLASSES). */
#define SKETCHNE_PROF_SPMM      0
#define SKETCHNE_PROF_SKETCH_Y  1
#define SKETCHNE_PROF_SKETCH_Z  2
#define SKETCHNE_PROF_GEMM64    3
#define SKETCHNE_PROF_SMALL     4
#define SKETCHNE_PROF_PREP      5
#define SKETCHNE_PROF_PROPAGATE 6
#define SKETCHNE_PROF_CLASSES   7
#define SKETCHNE_PROF_SELECT    0x40000000
sketchne_status sketchne_profile_enable(sketchne_ctx* ctx, int on);
sketchne_status sketchne_profile_read(sketchne_ctx* ctx, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* SKETCHNE_H */
