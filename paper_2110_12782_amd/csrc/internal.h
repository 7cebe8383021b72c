// Internal declarations shared by the translation units of libsketchne.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/sketchne.h"

struct sketchne_ctx {
  int device = 0;
  int n_cu = 0;                     // compute units of the device
  hipStream_t stream = nullptr;
  uint32_t* d_flags = nullptr;      // numeric flag word (device)
  uint32_t* h_flags = nullptr;      // pinned host copy
  int* h_counter = nullptr;         // pinned host scratch for convergence checks
  bool profiling = false;
  uint32_t prof_mask = 0;           // classes timed while profiling (bit = class)
  // per-class event pairs (recorded on the stream when profiling)
  static constexpr int kMaxEvents = 4096;
  hipEvent_t ev[kMaxEvents];
  int ev_class[kMaxEvents / 2];
  int n_ev = 0;
  double prof_ms[SKETCHNE_PROF_CLASSES] = {0};
  int64_t prof_n[SKETCHNE_PROF_CLASSES] = {0};
};

#define SK_TRY(expr)                    \
  do {                                  \
    sketchne_status _st = (expr);       \
    if (_st != SKETCHNE_OK) return _st; \
  } while (0)

namespace skne {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x, size_t a = kAlign) { return (x + a - 1) / a * a; }

// Bump allocator over a caller-provided workspace.  In "measure" mode (base
// == nullptr) it only accumulates the size.
struct Arena {
  char* base;
  size_t cap;
  size_t off = 0;
  bool overflow = false;
  Arena(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <class T>
  T* take(size_t count) {
    size_t bytes = align_up(count * sizeof(T));
    size_t at = off;
    off += bytes;
    if (base == nullptr) return nullptr;
    if (off > cap) { overflow = true; return nullptr; }
    return reinterpret_cast<T*>(base + at);
  }
};

// Profiling bracket: records an event pair around a launch when enabled.
struct ProfScope {
  sketchne_ctx* c;
  int cls;
  int slot = -1;
  ProfScope(sketchne_ctx* ctx, int klass) : c(ctx), cls(klass) {
    if (c && c->profiling && ((c->prof_mask >> cls) & 1u) && c->n_ev + 2 <= sketchne_ctx::kMaxEvents) {
      slot = c->n_ev;
      c->n_ev += 2;
      c->ev_class[slot / 2] = cls;
      hipEventRecord(c->ev[slot], c->stream);
    }
  }
  ~ProfScope() {
    if (slot >= 0) hipEventRecord(c->ev[slot + 1], c->stream);
  }
};

inline sketchne_status launch_status() {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? SKETCHNE_OK : SKETCHNE_E_DEVICE;
}

// ---- launchers implemented in the kernel translation units -------------

// rng.hip
sketchne_status gen_gauss(sketchne_ctx* c, int64_t n, int cols, int64_t ld, uint64_t seed, float* out);
sketchne_status gen_sparse_sign(sketchne_ctx* c, int64_t n, int cols, int z, uint64_t seed,
                                int32_t* rows, int8_t* signs);
sketchne_status gen_rademacher(sketchne_ctx* c, int64_t n, uint64_t seed, float* out);

// spmm.hip
size_t spmm_ws_bytes(int64_t nnz, int cols);
sketchne_status degree_scale(sketchne_ctx* c, int64_t n, const int64_t* rowptr, double alpha,
                             float* dscale);
sketchne_status spmm(sketchne_ctx* c, int64_t n, int64_t nnz, const int64_t* rowptr,
                     const int32_t* colidx, const float* dscale, const float* B, int64_t ldb,
                     int cols, float* C, int64_t ldc, float* partial);

// gemm64.hip : C(i,j) = alpha * sum_k A(i,k) * w(k) * B(k,j)  [+ diag_add * (i==j)]
// A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj], C(i,j) = C[i*sci + j*scj].
enum class Ty { F32 = 0, F64 = 1 };
struct GemmDesc {
  int64_t M = 0, N = 0, K = 0;
  const void* A = nullptr; Ty ta = Ty::F64; int64_t sai = 0, sak = 0;
  const void* B = nullptr; Ty tb = Ty::F64; int64_t sbk = 0, sbj = 0;
  void* C = nullptr; Ty tc = Ty::F64; int64_t sci = 0, scj = 0;
  const double* kw = nullptr;   // optional weights on the summation index
  double alpha = 1.0;
  double diag_add = 0.0;        // added to C(i,i)
  bool upper_only = false;      // compute tiles with i-tile <= j-tile and mirror
  const int* run_if = nullptr;  // device flag: when set and zero, the launch does nothing
};
// Split-K partial sums need splits*M*N doubles of scratch; gemm64 lowers the
// split count to what `partial_cap` bytes hold (down to 1, which needs none).
size_t gemm64_ws_bytes(const GemmDesc& g, int splits);
int gemm64_pick_splits(const GemmDesc& g);
size_t gemm64_partial_bytes(int64_t M, int64_t N, int64_t K, bool upper);
sketchne_status gemm64(sketchne_ctx* c, const GemmDesc& g, double* partial, size_t partial_cap);

// apply.hip : C = A B, A tall FP32 (n x K), B small FP64 (K x N), C FP32;
// N, K <= 288.  acol: A(i,k) = A[k*lda + i] (else A[i*lda + k]); bcol:
// B(k,j) = B[j*ldb + k] (else B[k*ldb + j]); ccol: C(i,j) = C[j*ldc + i];
// upper: B is upper triangular (N == K).  apply_tall_supported() says
// whether the fast kernel takes the shape.
struct ApplyDesc {
  int64_t n = 0; int K = 0, N = 0;
  const float* A = nullptr; int64_t lda = 0; bool acol = false;
  const double* B = nullptr; int64_t ldb = 0; bool bcol = false;
  bool upper = false;
  float* C = nullptr; int64_t ldc = 0; bool ccol = false;
  const int* run_if = nullptr;
  bool f32 = false;  // FP32 matrix cores (B rounded to FP32); only where a span is all that matters
  float* b32 = nullptr;  // f32: scratch for B's FP32 copy (as many floats as B spans); without it, FP64
};
bool apply_tall_supported(const ApplyDesc& d);
sketchne_status apply_tall(sketchne_ctx* c, const ApplyDesc& d);

// gram.hip : G = X^T diag(w) Y (symmetric products), X, Y tall FP32
int gram_nwg(int64_t n);
size_t gram_ws_bytes(int64_t n, int m);
sketchne_status gram_tall(sketchne_ctx* c, int64_t n, int m, const float* X, int64_t xr, int64_t xc, const float* Y,
                          int64_t yr, int64_t yc, const double* w, double* G, double* partial, size_t partial_cap,
                          const int* run_if, bool f32 = false);

// dense_small.hip
// Cholesky G = R^T R of an SPD m x m FP64 matrix (row-major, ld = m) and the
// inverse factor; writes RinvT (= R^-T, lower triangular, row-major m x m).
// The Gram matrix is first scaled to unit diagonal.  need_more (nullable):
// set to 1 when the scaled factor's 1-norm condition number exceeds
// repeat_kappa (or a shift was needed), else 0.  run_if (nullable):
// when it points to 0 the launch does nothing.
//   kCholQRRepeat: a basis that is used as an orthonormal basis (Rayleigh-
//     Ritz, the embedding); one FP64 pass below it leaves the FP32 basis
//     orthonormal to its storage rounding.
//   kCholQRRepeatInner: a power-iteration basis that only feeds the next
//     X (X Q).  Any invertible R keeps the span, which is all the next step
//     uses, and the next orthonormalisation restores orthogonality, so a
//     second pass is spent only when the Cholesky needed a shift (or the
//     estimate is not finite).
constexpr double kCholQRRepeat = 1e5;
constexpr double kCholQRRepeatInner = __builtin_inf();
size_t chol_ws_bytes(int m);
sketchne_status chol_inv(sketchne_ctx* c, int m, const double* G, double* RinvT, double* work,
                         int* need_more = nullptr, const int* run_if = nullptr,
                         double repeat_kappa = kCholQRRepeat);
sketchne_status copy_if(sketchne_ctx* c, int64_t count, const float* src, float* dst, const int* run_if);
constexpr int kSymeigMax = 288;  // largest order of the Jacobi eigensolver
size_t symeig_ws_bytes(int m);
// general = false: eigendecomposition of the symmetric A (upper triangle
// read), pairs by |w| descending.  general = true: singular values w >= 0
// (descending) and left singular vectors V of the general row-major A, by
// the same one-sided Jacobi on A itself (A J = V diag(w)).
sketchne_status symeig(sketchne_ctx* c, int m, const double* A, double* V, double* w, void* ws, bool general = false);
// The eigensolver's scratch for orders up to kSymeigMax in a device array of
// the library (one per device, held until the process ends).  init looks up
// its address on `device` (once; called by sketchne_create); scratch returns
// it, or nullptr when init has not succeeded on that device.
size_t symeig_scratch_bytes();
sketchne_status symeig_scratch_init(int device);
void* symeig_scratch(int device);

// propagate.hip (spectral propagation, Alg. 6 line 6)
constexpr int kPropagateMaxDegree = 64;
size_t propagate_ws_bytes(int64_t n, int64_t nnz, int d);
sketchne_status propagate(sketchne_ctx* c, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colidx,
                          int d, const float* E, int64_t lde, int p, const double* coef, float* out, int64_t ldo,
                          void* ws);

// mlp.hip (learned warm start)
int64_t ws_param_count(int width, int out);
size_t ws_part_floats(int64_t n, int width, int out);
size_t ws_forward_bytes(int64_t n, int width);
size_t ws_grad_bytes(int64_t n, int width, int out);
size_t ws_features_bytes(int64_t n, int64_t nnz);
size_t ritz_residual_bytes(int64_t n, int64_t nnz, int k);
// res_j = sqrt(max(v_j^T G v_j - lam_j^2, 0)), j < k: G m x m symmetric,
// V m x m row-major with v_j its column j
sketchne_status ritz_from_gram(sketchne_ctx* c, int m, int k, const double* G, const double* V, const double* lam,
                               double* res);
sketchne_status ws_init(sketchne_ctx* c, const sketchne_mlp* net, uint64_t seed);
sketchne_status ws_features(sketchne_ctx* c, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colidx,
                            double alpha, const float* g, uint64_t seed, float* phi, void* ws, size_t ws_bytes);
// BF16-activation inference pass (width 256, out % 32 == 0, out <= 256)
bool ws_infer_supported(const sketchne_mlp* net);
size_t ws_infer_bytes();
sketchne_status ws_infer(sketchne_ctx* c, const sketchne_mlp* net, int64_t n, const float* phi, float* F, int64_t ldf,
                         void* ws, size_t ws_bytes);
sketchne_status ws_forward(sketchne_ctx* c, const sketchne_mlp* net, int64_t n, const float* phi, float* F,
                           int64_t ldf, void* ws, size_t ws_bytes);
sketchne_status ws_grad(sketchne_ctx* c, const sketchne_mlp* net, int64_t n, const float* phi, const float* U,
                        int64_t ldu, float mu, float* grad, float* loss, void* ws, size_t ws_bytes);
sketchne_status ws_adam(sketchne_ctx* c, const sketchne_mlp* net, const float* grad, float lr, int step, double beta1,
                        double beta2, double eps);
sketchne_status ritz_residual(sketchne_ctx* c, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colidx,
                              double alpha, int k, const float* U, const double* lambda, double* res, void* ws,
                              size_t ws_bytes);
}  // namespace skne
