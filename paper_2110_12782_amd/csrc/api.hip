// Host side of the C ABI: argument validation, workspace carving and the
// orchestration of the three calls of the path (Alg. 6 lines 1-5).
#include <math.h>
#include <initializer_list>
#include <new>
#include <string.h>

#include "internal.h"
#include "sketch.h"

using namespace skne;

namespace {

__global__ void k_symmetrize(int m, const double* __restrict__ A, double* __restrict__ S) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  int i = idx / m, j = idx % m;
  S[idx] = 0.5 * (A[idx] + A[j * m + i]);
}

// Map[i][j] = V[i][j] * sqrt(|w_j|) (j < d), sigma[j] = |w_j|
__global__ void k_embed_map(int h, int d, const double* __restrict__ V, const double* __restrict__ w,
                            double* __restrict__ Map, double* __restrict__ sigma) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < d) sigma[idx] = fabs(w[idx]);
  if (idx >= h * d) return;
  int i = idx / d, j = idx % d;
  Map[idx] = V[i * h + j] * sqrt(fabs(w[j]));
}

// out = A^T (m x m)
__global__ void k_transpose(int m, const double* __restrict__ A, double* __restrict__ out) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  int i = idx / m, j = idx % m;
  out[idx] = A[j * m + i];
}

bool aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & (kAlign - 1)) == 0; }

// ------------------------------------------------------------- orthonormalise
// Cholesky-QR twice with FP64 Gram and Cholesky.  The tall matrix is either
// row-major n x m (element (i,j) at X[i*ld + j]) or "transposed" m x n
// (element (i,j) at Xt[j*ld + i]); src -> tmp -> dst, src may equal dst.
struct OrthWs {
  double* partial;
  size_t partial_cap;
  double* G;
  double* RinvT;
  double* cwork;
  int* need2;
  float* B32;  // FP32 copy of an m x m apply operand (the FP32 applies)
};

GemmDesc apply_desc(int64_t n, int m, const float* X, int64_t ld, bool transposed, const double* RinvT, float* out) {
  GemmDesc g;
  if (!transposed) {  // out (n x m) = X (n x m) * R^-1 ;  R^-1 (k, j) = RinvT[j][k]
    g.M = n; g.N = m; g.K = m;
    g.A = X; g.ta = Ty::F32; g.sai = ld; g.sak = 1;
    g.B = RinvT; g.tb = Ty::F64; g.sbk = 1; g.sbj = m;
    g.C = out; g.tc = Ty::F32; g.sci = ld; g.scj = 1;
  } else {            // out^T (m x n) = R^-T (m x m) * X^T (m x n)
    g.M = m; g.N = n; g.K = m;
    g.A = RinvT; g.ta = Ty::F64; g.sai = m; g.sak = 1;
    g.B = X; g.tb = Ty::F32; g.sbk = ld; g.sbj = 1;
    g.C = out; g.tc = Ty::F32; g.sci = ld; g.scj = 1;
  }
  return g;
}

size_t max_bytes(std::initializer_list<size_t> v) {
  size_t m = 0;
  for (size_t x : v) m = x > m ? x : m;
  return m;
}

size_t orth_partial_bytes(int64_t n, int m, bool transposed) {
  GemmDesc a = apply_desc(n, m, nullptr, transposed ? n : m, transposed, nullptr, nullptr);
  return max_bytes({gram_ws_bytes(n, m), gemm64_partial_bytes(a.M, a.N, a.K, a.upper_only)});
}

OrthWs carve_orth(Arena& ar, int64_t n, int m, bool transposed) {
  OrthWs w;
  w.partial_cap = orth_partial_bytes(n, m, transposed);
  w.partial = ar.take<double>(w.partial_cap / sizeof(double) + 1);
  w.G = ar.take<double>((size_t)m * m);
  w.RinvT = ar.take<double>((size_t)m * m);
  w.cwork = ar.take<double>(chol_ws_bytes(m) / sizeof(double) + 1);
  w.need2 = ar.take<int>(1);
  w.B32 = ar.take<float>((size_t)m * m);
  return w;
}

// dst = src R^-1 (R^-1 upper triangular, given as RinvT = R^-T row-major):
// the tall FP64 apply when it takes the shape, the general GEMM otherwise.
sketchne_status apply_rinv(sketchne_ctx* c, int64_t n, int m, const float* src, int64_t ld, bool transposed,
                           const double* RinvT, float* dst, const OrthWs& w, const int* run_if, bool f32 = false) {
  ApplyDesc d;
  d.f32 = f32;
  d.b32 = w.B32;
  d.n = n; d.K = m; d.N = m;
  d.A = src; d.lda = ld; d.acol = transposed;
  // R^-1(k, j) = RinvT[j][k]: column-major reads of B (measured faster here
  // than transposing R^-T and reading rows)
  d.B = RinvT; d.ldb = m; d.bcol = true; d.upper = true;
  d.C = dst; d.ldc = ld; d.ccol = transposed;
  d.run_if = run_if;
  if (apply_tall_supported(d)) return apply_tall(c, d);
  GemmDesc a = apply_desc(n, m, src, ld, transposed, RinvT, dst);
  a.run_if = run_if;
  return gemm64(c, a, w.partial, w.partial_cap);
}

// One Cholesky-QR pass src -> dst.  need_more: set by the Cholesky when a
// second pass is needed; run_if: the pass runs only when it points to 1.
// f32: Gram and apply on the FP32 matrix cores (the Cholesky stays FP64), for
// a power-iteration basis: its factor only has to keep the basis well
// conditioned, since any invertible factor keeps its span.
sketchne_status orth_pass(sketchne_ctx* c, int64_t n, int m, const float* src, float* dst, int64_t ld,
                          bool transposed, const OrthWs& w, int* need_more, const int* run_if,
                          double repeat_kappa = kCholQRRepeat, bool f32 = false) {
  if (!transposed)
    SK_TRY(gram_tall(c, n, m, src, ld, 1, nullptr, 0, 0, nullptr, w.G, w.partial, w.partial_cap, run_if, f32));
  else SK_TRY(gram_tall(c, n, m, src, 1, ld, nullptr, 0, 0, nullptr, w.G, w.partial, w.partial_cap, run_if));
  SK_TRY(chol_inv(c, m, w.G, w.RinvT, w.cwork, need_more, run_if, repeat_kappa));
  return apply_rinv(c, n, m, src, ld, transposed, w.RinvT, dst, w, run_if, f32);
}

// Cholesky-QR with FP64 Gram and Cholesky: src -> dst, and a second pass
// (dst -> tmp -> dst) only when the first factor's 1-norm condition number
// (Gram scaled to unit diagonal) exceeds repeat_kappa or its Cholesky needed
// a shift (kCholQRRepeat for a basis used as orthonormal, kCholQRRepeatInner
// for a power-iteration basis).
sketchne_status orth2(sketchne_ctx* c, int64_t n, int m, const float* src, float* tmp, float* dst, int64_t ld,
                      bool transposed, const OrthWs& w, double repeat_kappa = kCholQRRepeat) {
  // a power-iteration basis takes its first pass on the FP32 matrix cores;
  // the second pass (after a shifted Cholesky) is FP64
  const bool inner = repeat_kappa == kCholQRRepeatInner;
  SK_TRY(orth_pass(c, n, m, src, dst, ld, transposed, w, w.need2, nullptr, repeat_kappa, inner));
  SK_TRY(orth_pass(c, n, m, dst, tmp, ld, transposed, w, nullptr, w.need2));
  int64_t count = transposed ? (int64_t)m * ld : n * ld;
  return copy_if(c, count, tmp, dst, w.need2);
}

// ------------------------------------------------------------- validation
sketchne_status check_params(const sketchne_params* p, int64_t n) {
  if (!p) return SKETCHNE_E_ARG;
  if (!(p->alpha > 0.0 && p->alpha <= 0.5)) return SKETCHNE_E_ARG;
  if (p->T < 1 || !(p->b > 0.0)) return SKETCHNE_E_ARG;
  if (p->k < 1 || p->s_eig < 0 || p->q < 0) return SKETCHNE_E_ARG;
  int64_t K = (int64_t)p->k + p->s_eig;
  if (K > n) return SKETCHNE_E_ARG;
  if (p->d < 1 || p->h < p->d || p->l < p->h) return SKETCHNE_E_ARG;
  if (p->z < 1 || p->z > n) return SKETCHNE_E_ARG;
  if (p->precision < 0 || p->precision > 2) return SKETCHNE_E_ARG;
  if (p->split_r < 0 || p->split_r > p->k) return SKETCHNE_E_ARG;
  return SKETCHNE_OK;
}

sketchne_status check_graph(const sketchne_graph* A) {
  if (!A || A->n < 1 || A->nnz < 0 || !A->rowptr || (A->nnz > 0 && !A->colidx)) return SKETCHNE_E_ARG;
  if (A->n >= (int64_t)1 << 31) return SKETCHNE_E_UNSUPPORTED;
  return SKETCHNE_OK;
}

// ------------------------------------------------------------- eig
struct EigWs {
  float* dscale;
  float* Q;
  float* P1;
  float* P2;
  float* spmm_part;
  OrthWs ow;
  double* H;
  double* Vh;
  double* wv;
  double* rr_partial;
  size_t rr_cap;
  void* symws;
};

EigWs carve_eig(Arena& ar, const sketchne_params* p, int64_t n, int64_t nnz) {
  const int K = p->k + p->s_eig;
  EigWs w;
  w.dscale = ar.take<float>(n);
  w.Q = ar.take<float>((size_t)n * K);
  w.P1 = ar.take<float>((size_t)n * K);
  w.P2 = ar.take<float>((size_t)n * K);
  w.spmm_part = ar.take<float>(spmm_ws_bytes(nnz, K) / sizeof(float) + 1);
  w.ow = carve_orth(ar, n, K, false);
  w.H = ar.take<double>((size_t)K * K);
  w.Vh = ar.take<double>((size_t)K * K);
  w.wv = ar.take<double>(K);
  w.rr_cap = max_bytes({gram_ws_bytes(n, K), gemm64_partial_bytes(n, p->k, K, false)});
  w.rr_partial = ar.take<double>(w.rr_cap / sizeof(double) + 1);
  w.symws = ar.take<char>(symeig_ws_bytes(K));
  return w;
}

// ------------------------------------------------------------- sketch
struct SketchGeo {
  bool ok;       // k and r fit a compiled kernel
  int prec, r;
  int KSM, KSS;  // k-step sections (A: KSM + 2*KSS, B: KSM + KSS)
  int ntS, ntO, FB;
  int64_t nvt_pad, nvtO_pad, zl;
};

SketchGeo sketch_geo(const sketchne_params* p, int64_t n) {
  SketchGeo g;
  g.prec = p->precision;
  g.r = g.prec == SKETCHNE_FP32 ? 0 : p->split_r;
  g.KSM = g.KSS = 0;
  g.ok = sketch_sections(g.prec, p->k, g.r, &g.KSM, &g.KSS);
  g.FB = sketch_frag_bytes(g.prec);
  g.ntS = (p->h + 3) / 4;
  g.ntO = (p->l + 3) / 4;
  const int wg_tiles = 4 * sketch_vt(g.prec);
  int64_t nvt = (n + 31) / 32;
  g.nvt_pad = (nvt + wg_tiles - 1) / wg_tiles * wg_tiles;
  g.zl = (int64_t)p->z * p->l;
  int64_t nvtO = (g.zl + 31) / 32;
  g.nvtO_pad = (nvtO + wg_tiles - 1) / wg_tiles * wg_tiles;
  return g;
}

struct SketchWs {
  double* d1;
  double* d2;
  double* Kmat;
  double* Sa;
  double* Sb;
  double* Cc;
  double* k_partial;
  size_t k_cap;
  double* Gsel;
  double* RtT;
  void* ApS;
  void* ApO;
  float* sgnS;
  float* sgnO;
  void* Bp;
  float* T1t;
  double* pscale;
};

SketchWs carve_sketch(Arena& ar, const sketchne_params* p, int64_t n) {
  SketchGeo g = sketch_geo(p, n);
  const int k = p->k;
  SketchWs w;
  w.d1 = ar.take<double>(n);
  w.d2 = ar.take<double>(n);
  w.Kmat = ar.take<double>((size_t)k * k);
  w.Sa = ar.take<double>((size_t)k * k);
  w.Sb = ar.take<double>((size_t)k * k);
  w.Cc = ar.take<double>((size_t)k * k);
  int ntmax = g.ntS > g.ntO ? g.ntS : g.ntO;
  w.k_cap = max_bytes({gram_ws_bytes(n, k), gemm64_partial_bytes(k, k, k, false),
                       gemm64_partial_bytes((int64_t)g.ntS * 32, k, k, false),
                       gemm64_partial_bytes((int64_t)g.ntO * 32, k, k, false)});
  w.k_partial = ar.take<double>(w.k_cap / sizeof(double) + 1);
  w.Gsel = ar.take<double>((size_t)ntmax * 32 * k);
  w.RtT = ar.take<double>((size_t)ntmax * 32 * k);
  w.ApS = ar.take<char>((size_t)g.ntS * (g.KSM + 2 * g.KSS) * 64 * g.FB);
  w.ApO = ar.take<char>((size_t)g.ntO * (g.KSM + 2 * g.KSS) * 64 * g.FB);
  w.sgnS = ar.take<float>((size_t)g.ntS * 32);
  w.sgnO = ar.take<float>((size_t)g.ntO * 32);
  int64_t nvtmax = g.nvt_pad > g.nvtO_pad ? g.nvt_pad : g.nvtO_pad;
  w.Bp = ar.take<char>((size_t)nvtmax * (g.KSM + g.KSS) * 64 * g.FB);
  w.T1t = ar.take<float>((size_t)p->l * g.zl);
  w.pscale = ar.take<double>(3);
  return w;
}

// ------------------------------------------------------------- embed
struct EmbedWs {
  float* Q1;        // Y R1^-1 (transposed), formed only for the second Cholesky-QR pass
  OrthWs ow;        // ow.RinvT holds R1^-T
  double* RT2;
  double* Rci;      // Rc^-1 with Y = Q Rc
  double* OY;
  double* Bm;
  double* Bq1;
  double* Bq;
  double* Gb;
  double* Rb1;
  double* Rb2;
  double* cwork;
  double* Rinv;
  double* M1;
  double* M2;
  double* M3;
  double* W;
  double* Vw;
  double* ww;
  double* Map;
  double* Map2;
  double* s_partial;
  size_t s_cap;
  void* symws;
  int* needB;       // set by the Cholesky of B^T B when B = O^T Q needs a second pass
};

EmbedWs carve_embed(Arena& ar, const sketchne_params* p, int64_t n, bool dense_o = false) {
  const int h = p->h, l = p->l, d = p->d;
  EmbedWs w;
  w.Q1 = ar.take<float>((size_t)h * n);
  w.ow = carve_orth(ar, n, h, true);
  w.RT2 = ar.take<double>((size_t)h * h);
  w.Rci = ar.take<double>((size_t)h * h);
  w.OY = ar.take<double>((size_t)l * h);
  w.Bm = ar.take<double>((size_t)l * h);
  w.Bq1 = ar.take<double>((size_t)l * h);
  w.Bq = ar.take<double>((size_t)l * h);
  w.Gb = ar.take<double>((size_t)h * h);
  w.Rb1 = ar.take<double>((size_t)h * h);
  w.Rb2 = ar.take<double>((size_t)h * h);
  w.cwork = ar.take<double>(chol_ws_bytes(h) / sizeof(double) + 1);
  w.Rinv = ar.take<double>((size_t)h * h);
  w.M1 = ar.take<double>((size_t)h * l);
  w.M2 = ar.take<double>((size_t)h * h);
  w.M3 = ar.take<double>((size_t)h * h);
  w.W = ar.take<double>((size_t)h * h);
  w.Vw = ar.take<double>((size_t)h * h);
  w.ww = ar.take<double>(h);
  w.Map = ar.take<double>((size_t)h * d);
  w.Map2 = ar.take<double>((size_t)h * d);
  w.needB = ar.take<int>(1);
  // the largest split-K partial of the small products and of E = Y Map2
  w.s_cap = max_bytes({gemm64_partial_bytes(h, h, l, true), gemm64_partial_bytes(l, h, h, false),
                       gemm64_partial_bytes(h, h, h, false), gemm64_partial_bytes(h, l, l, false),
                       gemm64_partial_bytes(h, h, l, false), gemm64_partial_bytes(h, d, h, false),
                       gemm64_partial_bytes(n, d, h, false),
                       dense_o ? gemm64_partial_bytes(l, h, n, false) : (size_t)0});
  w.s_partial = ar.take<double>(w.s_cap / sizeof(double) + 1);
  w.symws = ar.take<char>(symeig_ws_bytes(h));
  return w;
}

size_t op_bytes(const sketchne_params* p, int64_t n, int64_t nnz, int mask) {
  size_t best = 0;
  if (mask & SKETCHNE_OP_EIG) { Arena a(nullptr, 0); carve_eig(a, p, n, nnz); best = a.off > best ? a.off : best; }
  if (mask & SKETCHNE_OP_SKETCH) { Arena a(nullptr, 0); carve_sketch(a, p, n); best = a.off > best ? a.off : best; }
  if (mask & SKETCHNE_OP_EMBED) { Arena a(nullptr, 0); carve_embed(a, p, n); best = a.off > best ? a.off : best; }
  if (mask & SKETCHNE_OP_SPMM) {
    size_t s = align_up(sizeof(float) * n) + spmm_ws_bytes(nnz, 512);
    best = s > best ? s : best;
  }
  return best;
}

sketchne_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return SKETCHNE_OK;
  if (!ws || ws_bytes < need || !aligned(ws)) return SKETCHNE_E_WORKSPACE;
  return SKETCHNE_OK;
}

// Alg. 6 lines 2-3 (Eq. 11): Kmat = U^T D^(-1+2a) U Lambda, then
// C = Lambda sum_{r=1..T} Kmat^(r-1) by Horner (Sa, Sb: k x k scratch)
sketchne_status eq11_core(sketchne_ctx* c, int64_t n, int k, int T, const float* U, const double* lambda,
                          const double* d2, double* Kmat, double* Sa, double* Sb, double* Cc, double* k_partial,
                          size_t k_cap) {
  // U^T D U is symmetric (upper blocks, mirrored); Lambda is applied after
  SK_TRY(gram_tall(c, n, k, U, k, 1, nullptr, 0, 0, d2, Kmat, k_partial, k_cap, nullptr));
  SK_TRY(scale_cols(c, k, k, Kmat, lambda));
  SK_TRY(identity(c, k, Sa));
  double* cur = Sa;
  double* nxt = Sb;
  for (int r = 1; r < T; ++r) {
    GemmDesc gd;
    gd.M = k; gd.N = k; gd.K = k;
    gd.A = Kmat; gd.ta = Ty::F64; gd.sai = k; gd.sak = 1;
    gd.B = cur; gd.tb = Ty::F64; gd.sbk = k; gd.sbj = 1;
    gd.C = nxt; gd.tc = Ty::F64; gd.sci = k; gd.scj = 1;
    gd.diag_add = 1.0;
    SK_TRY(gemm64(c, gd, k_partial, k_cap));
    double* t = cur; cur = nxt; nxt = t;
  }
  return scale_rows(c, k, k, cur, lambda, Cc);
}

// ------------------------------------------------------------- learned warm start
sketchne_status check_net(const sketchne_mlp* net) {
  if (!net || !net->master || !net->bf16 || net->width < 1 || net->out < 1) return SKETCHNE_E_ARG;
  if (net->width > 4096 || net->out > 4096) return SKETCHNE_E_UNSUPPORTED;
  return SKETCHNE_OK;
}

struct LearnedWs {
  float* omega;
  char* rest;     // reused in turn: phi + features/forward scratch, eig, residual
  size_t rest_bytes;
};

size_t learned_rest_bytes(const sketchne_params* p, int width, int64_t n, int64_t nnz) {
  size_t phi = align_up(sizeof(float) * (size_t)n * SKETCHNE_WS_FEAT);
  size_t a = phi + max_bytes({ws_features_bytes(n, nnz), ws_forward_bytes(n, width), ws_infer_bytes()});
  size_t b = op_bytes(p, n, nnz, SKETCHNE_OP_EIG);
  return max_bytes({a, b});
}

// start block, Ritz residuals, then the space shared by the network and Alg. 5
size_t learned_bytes(const sketchne_params* p, int width, int64_t n, int64_t nnz) {
  return align_up(sizeof(float) * (size_t)n * (p->k + p->s_eig)) + align_up(sizeof(double) * p->k) +
         learned_rest_bytes(p, width, n, nnz);
}

}  // namespace

// ===================================================================== ABI

extern "C" {

const char* sketchne_status_str(sketchne_status s) {
  switch (s) {
    case SKETCHNE_OK: return "ok";
    case SKETCHNE_E_ARG: return "invalid argument";
    case SKETCHNE_E_WORKSPACE: return "workspace missing, too small or misaligned";
    case SKETCHNE_E_DEVICE: return "HIP device or launch error";
    case SKETCHNE_E_NUMERIC: return "numerical breakdown on the device";
    case SKETCHNE_E_UNSUPPORTED: return "unsupported size or option";
  }
  return "unknown status";
}

sketchne_status sketchne_create(sketchne_ctx** out, int device, void* stream) {
  if (!out) return SKETCHNE_E_ARG;
  *out = nullptr;
  sketchne_ctx* c = new (std::nothrow) sketchne_ctx();
  if (!c) return SKETCHNE_E_DEVICE;
  c->device = device;
  c->stream = static_cast<hipStream_t>(stream);
  if (hipSetDevice(device) != hipSuccess) { delete c; return SKETCHNE_E_DEVICE; }
  if (hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
    delete c;
    return SKETCHNE_E_DEVICE;
  }
  if (hipMalloc(&c->d_flags, sizeof(uint32_t)) != hipSuccess) { delete c; return SKETCHNE_E_DEVICE; }
  if (hipHostMalloc(&c->h_flags, sizeof(uint32_t) + sizeof(int) * 4, hipHostMallocDefault) != hipSuccess) {
    hipFree(c->d_flags);
    delete c;
    return SKETCHNE_E_DEVICE;
  }
  c->h_counter = reinterpret_cast<int*>(c->h_flags + 1);
  hipMemset(c->d_flags, 0, sizeof(uint32_t));
  // address of this device's eigensolver scratch (sketchne_symeig_noalloc);
  // a failure here only disables that entry point, which then reports it
  symeig_scratch_init(device);
  for (int i = 0; i < sketchne_ctx::kMaxEvents; ++i) hipEventCreate(&c->ev[i]);
  *out = c;
  return SKETCHNE_OK;
}

sketchne_status sketchne_destroy(sketchne_ctx* c) {
  if (!c) return SKETCHNE_E_ARG;
  hipStreamSynchronize(c->stream);
  for (int i = 0; i < sketchne_ctx::kMaxEvents; ++i) hipEventDestroy(c->ev[i]);
  hipFree(c->d_flags);
  hipHostFree(c->h_flags);
  delete c;
  return SKETCHNE_OK;
}

sketchne_status sketchne_set_stream(sketchne_ctx* c, void* stream) {
  if (!c) return SKETCHNE_E_ARG;
  c->stream = static_cast<hipStream_t>(stream);
  return SKETCHNE_OK;
}

sketchne_status sketchne_workspace_size(const sketchne_params* p, int64_t n, int64_t nnz, int op_mask,
                                        size_t* bytes) {
  if (!bytes || n < 1 || nnz < 0) return SKETCHNE_E_ARG;
  SK_TRY(check_params(p, n));
  *bytes = op_bytes(p, n, nnz, op_mask);
  return SKETCHNE_OK;
}

// Alg. 5; when res is given (device, k doubles) it also receives the Ritz
// residuals ||X u_j - lambda_j u_j|| of the returned pairs, from the
// Rayleigh-Ritz data rather than a further SpMM: with Q orthonormal, H = Q^T X Q,
// u_j = Q v_j and v_j^T H v_j = lambda_j,
//   ||X Q v_j - lambda_j Q v_j||^2 = v_j^T (XQ)^T (XQ) v_j - lambda_j^2.
static sketchne_status eig_impl(sketchne_ctx* c, const sketchne_graph* A, const sketchne_params* p,
                                const float* omega0, float* U, double* lambda, double* res, void* ws,
                                size_t ws_bytes);

sketchne_status sketchne_eig(sketchne_ctx* c, const sketchne_graph* A, const sketchne_params* p,
                             const float* omega0, float* U, double* lambda, void* ws, size_t ws_bytes) {
  return eig_impl(c, A, p, omega0, U, lambda, nullptr, ws, ws_bytes);
}

static sketchne_status eig_impl(sketchne_ctx* c, const sketchne_graph* A, const sketchne_params* p,
                                const float* omega0, float* U, double* lambda, double* res, void* ws,
                                size_t ws_bytes) {
  if (!c || !U || !lambda) return SKETCHNE_E_ARG;
  SK_TRY(check_graph(A));
  SK_TRY(check_params(p, A->n));
  const int K = p->k + p->s_eig;
  if (K > kSymeigMax) return SKETCHNE_E_UNSUPPORTED;
  if (K % 4) return SKETCHNE_E_UNSUPPORTED;  // row length of the SpMM float4 path
  SK_TRY(check_ws(ws, ws_bytes, op_bytes(p, A->n, A->nnz, SKETCHNE_OP_EIG)));
  const int64_t n = A->n;
  Arena ar(ws, ws_bytes);
  EigWs w = carve_eig(ar, p, n, A->nnz);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;

  SK_TRY(degree_scale(c, n, A->rowptr, p->alpha, w.dscale));
  const float* start = omega0;
  if (!start) {
    SK_TRY(gen_gauss(c, n, K, K, p->seed, w.Q));
    start = w.Q;
  }
  // line 4-5: Y = X Omega, Q = orth(Y).  Every basis but the last one only
  // feeds the next X (X Q), so it takes the relaxed second-pass bound.
  SK_TRY(spmm(c, n, A->nnz, A->rowptr, A->colidx, w.dscale, start, K, K, w.P1, K, w.spmm_part));
  SK_TRY(orth2(c, n, K, w.P1, w.P2, w.Q, K, false, w.ow, p->q > 0 ? kCholQRRepeatInner : kCholQRRepeat));
  // lines 6-8: q times Q = orth(X (X Q))
  for (int it = 0; it < p->q; ++it) {
    SK_TRY(spmm(c, n, A->nnz, A->rowptr, A->colidx, w.dscale, w.Q, K, K, w.P1, K, w.spmm_part));
    SK_TRY(spmm(c, n, A->nnz, A->rowptr, A->colidx, w.dscale, w.P1, K, K, w.P2, K, w.spmm_part));
    SK_TRY(orth2(c, n, K, w.P2, w.P1, w.Q, K, false, w.ow, it + 1 < p->q ? kCholQRRepeatInner : kCholQRRepeat));
  }
  // line 9: H = Q^T X Q
  SK_TRY(spmm(c, n, A->nnz, A->rowptr, A->colidx, w.dscale, w.Q, K, K, w.P1, K, w.spmm_part));
  // Q^T X Q is symmetric: upper blocks computed and mirrored
  SK_TRY(gram_tall(c, n, K, w.Q, K, 1, w.P1, K, 1, nullptr, w.H, w.rr_partial, w.rr_cap, nullptr));
  // line 10: eigendecomposition, sorted by |lambda|
  SK_TRY(symeig(c, K, w.H, w.Vh, w.wv, w.symws));
  // line 11: U = Q U^(:, 1:k), on the FP32 matrix cores: Q and the columns of
  // U^ are orthonormal, so the sums have no cancellation to amplify the FP32
  // rounding (U is stored in FP32 either way)
  ApplyDesc ad;
  ad.f32 = true;
  ad.b32 = w.ow.B32;  // K x K floats, free once the last basis is formed
  ad.n = n; ad.K = K; ad.N = p->k;
  ad.A = w.Q; ad.lda = K;
  ad.B = w.Vh; ad.ldb = K;
  ad.C = U; ad.ldc = p->k;
  if (apply_tall_supported(ad)) {
    SK_TRY(apply_tall(c, ad));
  } else {
    GemmDesc g;
    g.M = n; g.N = p->k; g.K = K;
    g.A = w.Q; g.ta = Ty::F32; g.sai = K; g.sak = 1;
    g.B = w.Vh; g.tb = Ty::F64; g.sbk = K; g.sbj = 1;
    g.C = U; g.tc = Ty::F32; g.sci = p->k; g.scj = 1;
    SK_TRY(gemm64(c, g, w.rr_partial, w.rr_cap));
  }
  if (hipMemcpyAsync(lambda, w.wv, sizeof(double) * p->k, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return SKETCHNE_E_DEVICE;
  if (res) {
    // (XQ)^T (XQ) into H (free once the eigensolver has read it); P1 still holds XQ
    SK_TRY(gram_tall(c, n, K, w.P1, K, 1, nullptr, 0, 0, nullptr, w.H, w.rr_partial, w.rr_cap, nullptr));
    SK_TRY(ritz_from_gram(c, K, p->k, w.H, w.Vh, w.wv, res));
  }
  return SKETCHNE_OK;
}

sketchne_status sketchne_sketch(sketchne_ctx* c, const sketchne_graph* A, const sketchne_params* p,
                                const float* U, const double* lambda, sketchne_sparse_sign* S,
                                sketchne_sparse_sign* O, int generate, float* Yt, float* Z, void* ws,
                                size_t ws_bytes) {
  if (!c || !U || !lambda || !S || !O || !Yt || !Z) return SKETCHNE_E_ARG;
  SK_TRY(check_graph(A));
  SK_TRY(check_params(p, A->n));
  if (S->cols != p->h || O->cols != p->l || S->z != p->z || O->z != p->z) return SKETCHNE_E_ARG;
  if (!S->rows || !S->signs || !O->rows || !O->signs) return SKETCHNE_E_ARG;
  if (p->z > 8) return SKETCHNE_E_UNSUPPORTED;  // group of one lane's accumulators
  if (p->k % 4) return SKETCHNE_E_UNSUPPORTED;  // float4 rows of U
  SketchGeo g = sketch_geo(p, A->n);
  if (!g.ok) return SKETCHNE_E_UNSUPPORTED;
  if (g.zl >= ((int64_t)1 << 31)) return SKETCHNE_E_UNSUPPORTED;
  SK_TRY(check_ws(ws, ws_bytes, op_bytes(p, A->n, A->nnz, SKETCHNE_OP_SKETCH)));
  const int64_t n = A->n;
  const int k = p->k;
  Arena ar(ws, ws_bytes);
  SketchWs w = carve_sketch(ar, p, n);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;

  if (generate) {
    SK_TRY(gen_sparse_sign(c, n, p->h, p->z, p->seed ^ 0x5555555555555555ULL, S->rows, S->signs));
    SK_TRY(gen_sparse_sign(c, n, p->l, p->z, p->seed ^ 0xaaaaaaaaaaaaaaaaULL, O->rows, O->signs));
  }
  SK_TRY(degree_powers(c, n, A->rowptr, p->alpha, w.d1, w.d2));
  SK_TRY(eq11_core(c, n, k, p->T, U, lambda, w.d2, w.Kmat, w.Sa, w.Sb, w.Cc, w.k_partial, w.k_cap));

  const double vol = (double)A->nnz;
  const double scale = vol / (p->b * p->T);
  const float ln2 = 0.69314718055994530942f;
  const float inv_sqrt_z = (float)(1.0 / sqrt((double)p->z));

  // expanded columns R~^T = scale * D1(p) U(p,:) C^T  for one test matrix
  auto build_A = [&](const sketchne_sparse_sign* T, int ntiles, int groups, void* Ap, float* sgn) -> sketchne_status {
    SK_TRY(gather_expanded(c, n, ntiles, groups, p->z, T->rows, U, k, k, w.d1, scale, w.Gsel));
    GemmDesc gd;
    gd.M = (int64_t)ntiles * 32; gd.N = k; gd.K = k;
    gd.A = w.Gsel; gd.ta = Ty::F64; gd.sai = k; gd.sak = 1;
    gd.B = w.Cc; gd.tb = Ty::F64; gd.sbk = 1; gd.sbj = k;
    gd.C = w.RtT; gd.tc = Ty::F64; gd.sci = k; gd.scj = 1;
    SK_TRY(gemm64(c, gd, w.k_partial, w.k_cap));
    SK_TRY(balance(c, g.prec, (int64_t)ntiles * 32 * k, w.RtT, w.pscale));
    SK_TRY(pack_A(c, g.prec, ntiles, g.KSM, g.KSS, k, g.r, w.RtT, w.pscale, Ap));
    return pack_signs(c, ntiles, groups, p->z, T->signs, sgn);
  };

  // Alg. 4 line 4: Y = f(L' R'(:, p)) S(p, :)
  SK_TRY(build_A(S, g.ntS, p->h, w.ApS, w.sgnS));
  SK_TRY(pack_B(c, g.prec, n, n, g.nvt_pad, g.KSM, g.KSS, k, g.r, nullptr, U, k, w.d1, w.pscale, w.Bp));
  SK_TRY(fused_sketch(c, SKETCHNE_PROF_SKETCH_Y, g.prec, n, p->h, g.ntS, g.KSM, g.KSS, w.Bp, w.ApS, w.sgnS, Yt, n,
                      ln2 * inv_sqrt_z));
  // Alg. 4 line 7: Z = O(p,:)^T f(L'(p,:) R'(:, p)) O(p,:)
  SK_TRY(build_A(O, g.ntO, p->l, w.ApO, w.sgnO));
  SK_TRY(pack_B(c, g.prec, n, g.zl, g.nvtO_pad, g.KSM, g.KSS, k, g.r, O->rows, U, k, w.d1, w.pscale, w.Bp));
  SK_TRY(fused_sketch(c, SKETCHNE_PROF_SKETCH_Z, g.prec, g.zl, p->l, g.ntO, g.KSM, g.KSS, w.Bp, w.ApO, w.sgnO, w.T1t,
                      g.zl,
                      ln2 * inv_sqrt_z));
  SK_TRY(z_reduce(c, p->l, p->z, O->signs, w.T1t, g.zl, inv_sqrt_z, Z));
  return SKETCHNE_OK;
}

static sketchne_status embed_impl(sketchne_ctx* c, const sketchne_params* p, int64_t n, const float* Yt,
                                  const float* Z, const sketchne_sparse_sign* O, const float* Odense, float* E,
                                  double* sigma, void* ws, size_t ws_bytes);

sketchne_status sketchne_embed(sketchne_ctx* c, const sketchne_params* p, int64_t n, const float* Yt,
                               const float* Z, const sketchne_sparse_sign* O, float* E, double* sigma, void* ws,
                               size_t ws_bytes) {
  if (!c || !Yt || !Z || !O || !E || !sigma || n < 1) return SKETCHNE_E_ARG;
  SK_TRY(check_params(p, n));
  if (O->cols != p->l || O->z != p->z || !O->rows || !O->signs) return SKETCHNE_E_ARG;
  if (p->h > kSymeigMax) return SKETCHNE_E_UNSUPPORTED;
  if (p->h > n) return SKETCHNE_E_ARG;
  SK_TRY(check_ws(ws, ws_bytes, op_bytes(p, n, 0, SKETCHNE_OP_EMBED)));
  return embed_impl(c, p, n, Yt, Z, O, nullptr, E, sigma, ws, ws_bytes);
}

// Alg. 4 lines 5, 8-10 with O given by its columns' coordinates (O) or, for
// the full-visit variant, as a dense n x l matrix (Odense)
static sketchne_status embed_impl(sketchne_ctx* c, const sketchne_params* p, int64_t n, const float* Yt,
                                  const float* Z, const sketchne_sparse_sign* O, const float* Odense, float* E,
                                  double* sigma, void* ws, size_t ws_bytes) {
  const int h = p->h, l = p->l, d = p->d;
  Arena ar(ws, ws_bytes);
  EmbedWs w = carve_embed(ar, p, n, Odense != nullptr);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;

  auto small = [&](int64_t M, int64_t N, int64_t K, const void* Ap, Ty ta, int64_t sai, int64_t sak, const void* Bp,
                   Ty tb, int64_t sbk, int64_t sbj, double* C, bool upper, const int* run_if) -> sketchne_status {
    GemmDesc gd;
    gd.M = M; gd.N = N; gd.K = K;
    gd.A = Ap; gd.ta = ta; gd.sai = sai; gd.sak = sak;
    gd.B = Bp; gd.tb = tb; gd.sbk = sbk; gd.sbj = sbj;
    gd.C = C; gd.tc = Ty::F64; gd.sci = N; gd.scj = 1;
    gd.upper_only = upper;
    gd.run_if = run_if;
    return gemm64(c, gd, w.s_partial, w.s_cap);
  };
  // Alg. 4 line 5: Q = orth(Y), kept implicit as Q = Y Rc^-1 (Y = Q Rc), so
  // the n x h matrix Q is never written: Cholesky-QR factor of Y (Y held
  // transposed, h x n), and a second pass only when Y is ill-conditioned.
  const OrthWs& ow = w.ow;
  SK_TRY(gram_tall(c, n, h, Yt, 1, n, nullptr, 0, 0, nullptr, ow.G, ow.partial, ow.partial_cap, nullptr));
  SK_TRY(chol_inv(c, h, ow.G, ow.RinvT, ow.cwork, ow.need2, nullptr));
  hipLaunchKernelGGL(k_transpose, dim3((h * h + 255) / 256), dim3(256), 0, c->stream, h, ow.RinvT, w.Rci);
  SK_TRY(launch_status());
  {  // second pass (device-side condition): Q1 = Y R1^-1, R2 from Q1^T Q1, Rc^-1 = R1^-1 R2^-1
    SK_TRY(apply_rinv(c, n, h, Yt, n, true, ow.RinvT, w.Q1, ow, ow.need2));
    SK_TRY(gram_tall(c, n, h, w.Q1, 1, n, nullptr, 0, 0, nullptr, ow.G, ow.partial, ow.partial_cap, ow.need2));
    SK_TRY(chol_inv(c, h, ow.G, w.RT2, ow.cwork, nullptr, ow.need2));
    SK_TRY(small(h, h, h, ow.RinvT, Ty::F64, 1, h, w.RT2, Ty::F64, 1, h, w.Rci, false, ow.need2));
  }
  // B = O^T Q = (O^T Y) Rc^-1   (l x h)
  if (Odense) {
    GemmDesc gd;  // O^T Y: O(k, i) = Odense[k l + i], Y(k, j) = Yt[j n + k]
    gd.M = l; gd.N = h; gd.K = n;
    gd.A = Odense; gd.ta = Ty::F32; gd.sai = 1; gd.sak = l;
    gd.B = Yt; gd.tb = Ty::F32; gd.sbk = 1; gd.sbj = n;
    gd.C = w.OY; gd.tc = Ty::F64; gd.sci = h; gd.scj = 1;
    SK_TRY(gemm64(c, gd, w.s_partial, w.s_cap));
  } else {
    SK_TRY(ot_q(c, l, p->z, h, O->rows, O->signs, Yt, n, 1.0 / sqrt((double)p->z), w.OY));
  }
  SK_TRY(small(l, h, h, w.OY, Ty::F64, h, 1, w.Rci, Ty::F64, h, 1, w.Bm, false, nullptr));
  // QR of B by Cholesky-QR in FP64: B = Bq R.  B = O^T Q is an l x h
  // sparse-sign projection of orthonormal columns (l > h), so it is well
  // conditioned and one pass leaves Bq orthonormal to FP64 rounding; the
  // second pass (R^-1 = R1^-1 R2^-1) runs only when the first factor's
  // condition number exceeds the orthonormal-basis bound or its Cholesky
  // needed a shift (a device flag, no host round trip).
  SK_TRY(small(h, h, l, w.Bm, Ty::F64, 1, h, w.Bm, Ty::F64, h, 1, w.Gb, true, nullptr));
  SK_TRY(chol_inv(c, h, w.Gb, w.Rb1, w.cwork, w.needB, nullptr));
  SK_TRY(small(l, h, h, w.Bm, Ty::F64, h, 1, w.Rb1, Ty::F64, 1, h, w.Bq, false, nullptr));
  // Rinv = R1^-1 (R^-1(i, j) = RinvT[j][i]), replaced by R1^-1 R2^-1 after a second pass
  hipLaunchKernelGGL(k_transpose, dim3((h * h + 255) / 256), dim3(256), 0, c->stream, h, w.Rb1, w.Rinv);
  SK_TRY(launch_status());
  SK_TRY(small(h, h, l, w.Bq, Ty::F64, 1, h, w.Bq, Ty::F64, h, 1, w.Gb, true, w.needB));
  SK_TRY(chol_inv(c, h, w.Gb, w.Rb2, w.cwork, nullptr, w.needB));
  SK_TRY(small(l, h, h, w.Bq, Ty::F64, h, 1, w.Rb2, Ty::F64, 1, h, w.Bq1, false, w.needB));
  SK_TRY(copy_if(c, 2 * (int64_t)l * h, reinterpret_cast<const float*>(w.Bq1), reinterpret_cast<float*>(w.Bq),
                 w.needB));
  SK_TRY(small(h, h, h, w.Rb1, Ty::F64, 1, h, w.Rb2, Ty::F64, 1, h, w.Rinv, false, w.needB));
  // W = Rinv (Bq^T Z Bq) Rinv^T  (Alg. 4 line 8, two least-squares solves)
  SK_TRY(small(h, l, l, w.Bq, Ty::F64, 1, h, Z, Ty::F32, l, 1, w.M1, false, nullptr));
  SK_TRY(small(h, h, l, w.M1, Ty::F64, l, 1, w.Bq, Ty::F64, h, 1, w.M2, false, nullptr));
  SK_TRY(small(h, h, h, w.Rinv, Ty::F64, h, 1, w.M2, Ty::F64, h, 1, w.M3, false, nullptr));
  SK_TRY(small(h, h, h, w.M3, Ty::F64, h, 1, w.Rinv, Ty::F64, 1, h, w.W, false, nullptr));
  hipLaunchKernelGGL(k_symmetrize, dim3((h * h + 255) / 256), dim3(256), 0, c->stream, h, w.W, w.M2);
  SK_TRY(launch_status());
  // Alg. 4 line 9: SVD of the symmetric W from its eigendecomposition
  SK_TRY(symeig(c, h, w.M2, w.Vw, w.ww, w.symws));
  hipLaunchKernelGGL(k_embed_map, dim3((h * d + 255) / 256), dim3(256), 0, c->stream, h, d, w.Vw, w.ww, w.Map,
                     sigma);
  SK_TRY(launch_status());
  // Alg. 4 line 10 and Alg. 6 line 5: E = Q U^(:, 1:d) Sigma^(1/2) = Y (Rc^-1 U^ Sigma^(1/2))
  SK_TRY(small(h, d, h, w.Rci, Ty::F64, h, 1, w.Map, Ty::F64, d, 1, w.Map2, false, nullptr));
  ApplyDesc ad;
  ad.n = n; ad.K = h; ad.N = d;
  ad.A = Yt; ad.lda = n; ad.acol = true;
  ad.B = w.Map2; ad.ldb = d;
  ad.C = E; ad.ldc = d;
  if (apply_tall_supported(ad)) return apply_tall(c, ad);
  GemmDesc gd;
  gd.M = n; gd.N = d; gd.K = h;
  gd.A = Yt; gd.ta = Ty::F32; gd.sai = 1; gd.sak = n;
  gd.B = w.Map2; gd.tb = Ty::F64; gd.sbk = d; gd.sbj = 1;
  gd.C = E; gd.tc = Ty::F32; gd.sci = d; gd.scj = 1;
  return gemm64(c, gd, w.s_partial, w.s_cap);
}

// ===================================================== general single pass
// Eqs. (5)-(10): four test matrices for a target f(LR) that need not be
// symmetric.  The three sketches reuse the fused kernel: Y with the rows of
// L against the columns of R at S, K = f(LR)^T C as f(R^T L^T) C with the
// roles of the factors exchanged, and Z with the rows of L at H's
// coordinates against the columns of R at O.
}  // extern "C"

namespace {

// k_general_map: Map_v(:, j) = W^T u_j / sqrt(sigma_j)  (zero when sigma_j = 0),
// from WtU = W^T U^_d (h x d); V^_d Sigma_d^(1/2) = W^T U^_d Sigma_d^(-1/2)
__global__ void k_scale_inv_sqrt(int h, int d, const double* __restrict__ WtU, const double* __restrict__ sigma,
                                 double* __restrict__ out) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= h * d) return;
  const double s = sigma[idx % d];
  out[idx] = s > 0.0 ? WtU[idx] / sqrt(s) : 0.0;
}

struct GenSketchWs {
  double* Gsel;
  void* Ap;
  float* sgn;
  void* Bp;
  float* T1t;
  double* pscale;
};

sketchne_params general_params(const sketchne_params* p, int k) {
  sketchne_params q = *p;
  q.k = k;
  return q;
}

GenSketchWs carve_gen_sketch(Arena& ar, const sketchne_params* q, int64_t n) {
  SketchGeo g = sketch_geo(q, n);
  GenSketchWs w;
  const int ntmax = g.ntS > g.ntO ? g.ntS : g.ntO;
  w.Gsel = ar.take<double>((size_t)ntmax * 32 * q->k);
  w.Ap = ar.take<char>((size_t)ntmax * (g.KSM + 2 * g.KSS) * 64 * g.FB);
  w.sgn = ar.take<float>((size_t)ntmax * 32);
  int64_t nvtmax = g.nvt_pad > g.nvtO_pad ? g.nvt_pad : g.nvtO_pad;
  w.Bp = ar.take<char>((size_t)nvtmax * (g.KSM + g.KSS) * 64 * g.FB);
  w.T1t = ar.take<float>((size_t)q->l * g.zl);
  w.pscale = ar.take<double>(3);
  return w;
}

struct GenEmbedWs {
  float* Q1;
  OrthWs ow;
  double* RT2;
  double* RciY;
  double* RciK;
  double* T;      // H^T Y, then O^T K (l x h)
  double* B1;
  double* B2;
  double* Bq1;
  double* Bq2;
  double* Bqt;
  double* Gb;
  double* Rb1;
  double* Rb2;
  double* cwork;
  double* Rinv1;
  double* Rinv2;
  double* M1;
  double* M2;
  double* M3;
  double* W;
  double* Vw;
  double* ww;
  double* Mu;
  double* Mv;
  double* WtU;
  double* Map2;
  double* s_partial;
  size_t s_cap;
  void* symws;
};

GenEmbedWs carve_gen_embed(Arena& ar, const sketchne_params* p, int64_t n) {
  const int h = p->h, l = p->l, d = p->d;
  GenEmbedWs w;
  w.Q1 = ar.take<float>((size_t)h * n);
  w.ow = carve_orth(ar, n, h, true);
  w.RT2 = ar.take<double>((size_t)h * h);
  w.RciY = ar.take<double>((size_t)h * h);
  w.RciK = ar.take<double>((size_t)h * h);
  w.T = ar.take<double>((size_t)l * h);
  w.B1 = ar.take<double>((size_t)l * h);
  w.B2 = ar.take<double>((size_t)l * h);
  w.Bq1 = ar.take<double>((size_t)l * h);
  w.Bq2 = ar.take<double>((size_t)l * h);
  w.Bqt = ar.take<double>((size_t)l * h);
  w.Gb = ar.take<double>((size_t)h * h);
  w.Rb1 = ar.take<double>((size_t)h * h);
  w.Rb2 = ar.take<double>((size_t)h * h);
  w.cwork = ar.take<double>(chol_ws_bytes(h) / sizeof(double) + 1);
  w.Rinv1 = ar.take<double>((size_t)h * h);
  w.Rinv2 = ar.take<double>((size_t)h * h);
  w.M1 = ar.take<double>((size_t)h * l);
  w.M2 = ar.take<double>((size_t)h * h);
  w.M3 = ar.take<double>((size_t)h * h);
  w.W = ar.take<double>((size_t)h * h);
  w.Vw = ar.take<double>((size_t)h * h);
  w.ww = ar.take<double>(h);
  w.Mu = ar.take<double>((size_t)h * d);
  w.Mv = ar.take<double>((size_t)h * d);
  w.WtU = ar.take<double>((size_t)h * d);
  w.Map2 = ar.take<double>((size_t)h * d);
  w.s_cap = max_bytes({gemm64_partial_bytes(h, h, l, true), gemm64_partial_bytes(l, h, h, false),
                       gemm64_partial_bytes(h, h, h, false), gemm64_partial_bytes(h, l, l, false),
                       gemm64_partial_bytes(h, h, l, false), gemm64_partial_bytes(h, d, h, false),
                       gemm64_partial_bytes(n, d, h, false)});
  w.s_partial = ar.take<double>(w.s_cap / sizeof(double) + 1);
  w.symws = ar.take<char>(symeig_ws_bytes(h));
  return w;
}

sketchne_status check_general(const sketchne_params* p, int64_t n, int k) {
  if (!p || n < 1 || k < 1 || k > n) return SKETCHNE_E_ARG;
  if (p->d < 1 || p->h < p->d || p->l < p->h || p->h > n) return SKETCHNE_E_ARG;
  if (p->z < 1 || p->z > n) return SKETCHNE_E_ARG;
  if (p->precision < 0 || p->precision > 2 || p->split_r < 0 || p->split_r > k) return SKETCHNE_E_ARG;
  if (n >= ((int64_t)1 << 31)) return SKETCHNE_E_UNSUPPORTED;
  return SKETCHNE_OK;
}

bool test_matrix_ok(const sketchne_sparse_sign* T, int cols, int z) {
  return T && T->cols == cols && T->z == z && T->rows && T->signs;
}

}  // namespace

extern "C" {

sketchne_status sketchne_general_workspace_size(const sketchne_params* p, int64_t n, int32_t k, int op_mask,
                                                size_t* bytes) {
  if (!bytes) return SKETCHNE_E_ARG;
  SK_TRY(check_general(p, n, k));
  sketchne_params q = general_params(p, k);
  size_t best = 0;
  if (op_mask & SKETCHNE_OP_SKETCH) { Arena a(nullptr, 0); carve_gen_sketch(a, &q, n); best = a.off > best ? a.off : best; }
  if (op_mask & SKETCHNE_OP_EMBED) { Arena a(nullptr, 0); carve_gen_embed(a, &q, n); best = a.off > best ? a.off : best; }
  *bytes = best;
  return SKETCHNE_OK;
}

sketchne_status sketchne_sketch_general(sketchne_ctx* c, int64_t n, int32_t k, const float* L, const float* Rt,
                                        const sketchne_params* p, const sketchne_sparse_sign* C,
                                        const sketchne_sparse_sign* S, const sketchne_sparse_sign* H,
                                        const sketchne_sparse_sign* O, float* Kt, float* Yt, float* Z, void* ws,
                                        size_t ws_bytes) {
  if (!c || !L || !Rt || !Kt || !Yt || !Z) return SKETCHNE_E_ARG;
  SK_TRY(check_general(p, n, k));
  if (!test_matrix_ok(C, p->h, p->z) || !test_matrix_ok(S, p->h, p->z) || !test_matrix_ok(H, p->l, p->z) ||
      !test_matrix_ok(O, p->l, p->z))
    return SKETCHNE_E_ARG;
  if (p->z > 8 || p->precision == SKETCHNE_FP16) return SKETCHNE_E_UNSUPPORTED;
  sketchne_params q = general_params(p, k);
  SketchGeo g = sketch_geo(&q, n);
  if (!g.ok || g.zl >= ((int64_t)1 << 31)) return SKETCHNE_E_UNSUPPORTED;
  size_t need = 0;
  SK_TRY(sketchne_general_workspace_size(p, n, k, SKETCHNE_OP_SKETCH, &need));
  SK_TRY(check_ws(ws, ws_bytes, need));
  Arena ar(ws, ws_bytes);
  GenSketchWs w = carve_gen_sketch(ar, &q, n);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  const float ln2 = 0.69314718055994530942f;
  const float inv_sqrt_z = (float)(1.0 / sqrt((double)p->z));
  // one product f(B_rows A_cols^T) T of the fused kernel: the expanded columns
  // are rows of `acols` (n x k) at T's coordinates, the vertex rows are rows
  // of `brows` (n x k), gathered at `gather` when given
  auto pass = [&](int cls, const sketchne_sparse_sign* T, int ntiles, int groups, const float* acols,
                  const float* brows, const int32_t* gather, int64_t nrows, int64_t nvt_pad, float* out,
                  int64_t ld_out) -> sketchne_status {
    SK_TRY(gather_expanded(c, n, ntiles, groups, p->z, T->rows, acols, k, k, nullptr, 1.0, w.Gsel));
    SK_TRY(balance(c, g.prec, (int64_t)ntiles * 32 * k, w.Gsel, w.pscale));
    SK_TRY(pack_A(c, g.prec, ntiles, g.KSM, g.KSS, k, g.r, w.Gsel, w.pscale, w.Ap));
    SK_TRY(pack_signs(c, ntiles, groups, p->z, T->signs, w.sgn));
    SK_TRY(pack_B(c, g.prec, n, nrows, nvt_pad, g.KSM, g.KSS, k, g.r, gather, brows, k, nullptr, w.pscale, w.Bp));
    return fused_sketch(c, cls, g.prec, nrows, groups, ntiles, g.KSM, g.KSS, w.Bp, w.Ap, w.sgn, out, ld_out,
                        ln2 * inv_sqrt_z);
  };
  // Eq. (5): Y = f(LR) S
  SK_TRY(pass(SKETCHNE_PROF_SKETCH_Y, S, g.ntS, p->h, Rt, L, nullptr, n, g.nvt_pad, Yt, n));
  // K = f(LR)^T C = f(R^T L^T) C
  SK_TRY(pass(SKETCHNE_PROF_SKETCH_Y, C, g.ntS, p->h, L, Rt, nullptr, n, g.nvt_pad, Kt, n));
  // Z = H^T f(LR) O: rows of L at H's coordinates against the columns of R at O
  SK_TRY(pass(SKETCHNE_PROF_SKETCH_Z, O, g.ntO, p->l, Rt, L, H->rows, g.zl, g.nvtO_pad, w.T1t, g.zl));
  return z_reduce(c, p->l, p->z, H->signs, w.T1t, g.zl, inv_sqrt_z, Z);
}

sketchne_status sketchne_embed_general(sketchne_ctx* c, const sketchne_params* p, int64_t n, const float* Kt,
                                       const float* Yt, const float* Z, const sketchne_sparse_sign* H,
                                       const sketchne_sparse_sign* O, float* E, float* Ed, double* sigma, void* ws,
                                       size_t ws_bytes) {
  if (!c || !Kt || !Yt || !Z || !E || !Ed || !sigma) return SKETCHNE_E_ARG;
  SK_TRY(check_general(p, n, p ? p->h : 1));
  if (!test_matrix_ok(H, p->l, p->z) || !test_matrix_ok(O, p->l, p->z)) return SKETCHNE_E_ARG;
  if (p->h > kSymeigMax) return SKETCHNE_E_UNSUPPORTED;
  size_t need = 0;
  SK_TRY(sketchne_general_workspace_size(p, n, p->h, SKETCHNE_OP_EMBED, &need));
  SK_TRY(check_ws(ws, ws_bytes, need));
  const int h = p->h, l = p->l, d = p->d;
  Arena ar(ws, ws_bytes);
  GenEmbedWs w = carve_gen_embed(ar, p, n);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  auto small = [&](int64_t M, int64_t N, int64_t K, const void* Ap, Ty ta, int64_t sai, int64_t sak, const void* Bp,
                   Ty tb, int64_t sbk, int64_t sbj, double* C, bool upper, const int* run_if) -> sketchne_status {
    GemmDesc gd;
    gd.M = M; gd.N = N; gd.K = K;
    gd.A = Ap; gd.ta = ta; gd.sai = sai; gd.sak = sak;
    gd.B = Bp; gd.tb = tb; gd.sbk = sbk; gd.sbj = sbj;
    gd.C = C; gd.tc = Ty::F64; gd.sci = N; gd.scj = 1;
    gd.upper_only = upper;
    gd.run_if = run_if;
    return gemm64(c, gd, w.s_partial, w.s_cap);
  };
  const OrthWs& ow = w.ow;
  // Eq. (6) kept implicit: X = orth(X) Rc for X = Y, K (both held transposed,
  // h x n); Rci = Rc^-1, with a second Cholesky-QR pass when X is
  // ill-conditioned
  auto implicit_orth = [&](const float* Xt, double* Rci) -> sketchne_status {
    SK_TRY(gram_tall(c, n, h, Xt, 1, n, nullptr, 0, 0, nullptr, ow.G, ow.partial, ow.partial_cap, nullptr));
    SK_TRY(chol_inv(c, h, ow.G, ow.RinvT, ow.cwork, ow.need2, nullptr));
    hipLaunchKernelGGL(k_transpose, dim3((h * h + 255) / 256), dim3(256), 0, c->stream, h, ow.RinvT, Rci);
    SK_TRY(launch_status());
    SK_TRY(apply_rinv(c, n, h, Xt, n, true, ow.RinvT, w.Q1, ow, ow.need2));
    SK_TRY(gram_tall(c, n, h, w.Q1, 1, n, nullptr, 0, 0, nullptr, ow.G, ow.partial, ow.partial_cap, ow.need2));
    SK_TRY(chol_inv(c, h, ow.G, w.RT2, ow.cwork, nullptr, ow.need2));
    return small(h, h, h, ow.RinvT, Ty::F64, 1, h, w.RT2, Ty::F64, 1, h, Rci, false, ow.need2);
  };
  // B = Bq R by Cholesky-QR twice in FP64; Rinv = R^-1 (row-major)
  auto small_qr = [&](const double* Bm, double* Bq, double* Rinv) -> sketchne_status {
    SK_TRY(small(h, h, l, Bm, Ty::F64, 1, h, Bm, Ty::F64, h, 1, w.Gb, true, nullptr));
    SK_TRY(chol_inv(c, h, w.Gb, w.Rb1, w.cwork));
    SK_TRY(small(l, h, h, Bm, Ty::F64, h, 1, w.Rb1, Ty::F64, 1, h, w.Bqt, false, nullptr));
    SK_TRY(small(h, h, l, w.Bqt, Ty::F64, 1, h, w.Bqt, Ty::F64, h, 1, w.Gb, true, nullptr));
    SK_TRY(chol_inv(c, h, w.Gb, w.Rb2, w.cwork));
    SK_TRY(small(l, h, h, w.Bqt, Ty::F64, h, 1, w.Rb2, Ty::F64, 1, h, Bq, false, nullptr));
    return small(h, h, h, w.Rb1, Ty::F64, 1, h, w.Rb2, Ty::F64, 1, h, Rinv, false, nullptr);
  };
  const double isz = 1.0 / sqrt((double)p->z);
  SK_TRY(implicit_orth(Yt, w.RciY));
  SK_TRY(implicit_orth(Kt, w.RciK));
  // H^T Q = (H^T Y) Rq^-1 and O^T P = (O^T K) Rp^-1   (l x h)
  SK_TRY(ot_q(c, l, p->z, h, H->rows, H->signs, Yt, n, isz, w.T));
  SK_TRY(small(l, h, h, w.T, Ty::F64, h, 1, w.RciY, Ty::F64, h, 1, w.B1, false, nullptr));
  SK_TRY(ot_q(c, l, p->z, h, O->rows, O->signs, Kt, n, isz, w.T));
  SK_TRY(small(l, h, h, w.T, Ty::F64, h, 1, w.RciK, Ty::F64, h, 1, w.B2, false, nullptr));
  // Eq. (9): W = (H^T Q)^+ Z (P^T O)^+ = R1^-1 Bq1^T Z Bq2 R2^-T
  SK_TRY(small_qr(w.B1, w.Bq1, w.Rinv1));
  SK_TRY(small_qr(w.B2, w.Bq2, w.Rinv2));
  SK_TRY(small(h, l, l, w.Bq1, Ty::F64, 1, h, Z, Ty::F32, l, 1, w.M1, false, nullptr));
  SK_TRY(small(h, h, l, w.M1, Ty::F64, l, 1, w.Bq2, Ty::F64, h, 1, w.M2, false, nullptr));
  SK_TRY(small(h, h, h, w.Rinv1, Ty::F64, h, 1, w.M2, Ty::F64, h, 1, w.M3, false, nullptr));
  SK_TRY(small(h, h, h, w.M3, Ty::F64, h, 1, w.Rinv2, Ty::F64, 1, h, w.W, false, nullptr));
  // Eq. (10): SVD of W (general) by one-sided Jacobi: W J = U^ Sigma
  SK_TRY(symeig(c, h, w.W, w.Vw, w.ww, w.symws, true));
  hipLaunchKernelGGL(k_embed_map, dim3((h * d + 255) / 256), dim3(256), 0, c->stream, h, d, w.Vw, w.ww, w.Mu,
                     sigma);
  SK_TRY(launch_status());
  // V^_d Sigma_d^(1/2) = W^T U^_d Sigma_d^(-1/2)
  SK_TRY(small(h, d, h, w.W, Ty::F64, 1, h, w.Vw, Ty::F64, h, 1, w.WtU, false, nullptr));
  hipLaunchKernelGGL(k_scale_inv_sqrt, dim3((h * d + 255) / 256), dim3(256), 0, c->stream, h, d, w.WtU, sigma, w.Mv);
  SK_TRY(launch_status());
  // E = Q U^_d Sigma_d^(1/2) = Y (Rq^-1 Mu);  Ed = P V^_d Sigma_d^(1/2) = K (Rp^-1 Mv)
  auto tall = [&](const float* Xt, const double* Map, float* out) -> sketchne_status {
    ApplyDesc ad;
    ad.n = n; ad.K = h; ad.N = d;
    ad.A = Xt; ad.lda = n; ad.acol = true;
    ad.B = Map; ad.ldb = d;
    ad.C = out; ad.ldc = d;
    if (apply_tall_supported(ad)) return apply_tall(c, ad);
    GemmDesc gd;
    gd.M = n; gd.N = d; gd.K = h;
    gd.A = Xt; gd.ta = Ty::F32; gd.sai = 1; gd.sak = n;
    gd.B = Map; gd.tb = Ty::F64; gd.sbk = d; gd.sbj = 1;
    gd.C = out; gd.tc = Ty::F32; gd.sci = d; gd.scj = 1;
    return gemm64(c, gd, w.s_partial, w.s_cap);
  };
  SK_TRY(small(h, d, h, w.RciY, Ty::F64, h, 1, w.Mu, Ty::F64, d, 1, w.Map2, false, nullptr));
  SK_TRY(tall(Yt, w.Map2, E));
  SK_TRY(small(h, d, h, w.RciK, Ty::F64, h, 1, w.Mv, Ty::F64, d, 1, w.Map2, false, nullptr));
  return tall(Kt, w.Map2, Ed);
}

// ===================================================== full-visit variant
// Test matrices with z nonzeros per ROW: every entry of f(L'R') is formed,
// by two chained matrix-core products per tile (fullvisit.hip).
}  // extern "C"

namespace {

constexpr int kFullVisitMaxL = 8192;

struct FvGeo {
  int prec, KSM, KSS;
  int64_t npad, njt, nvt_pad;
  int nct_h, nct_l;
  int fb;   // bytes per lane of one fragment
  int ks2;  // k-steps of the second product per 32 columns
};

FvGeo fv_geo(const sketchne_params* p, int64_t n) {
  FvGeo g;
  g.prec = p->precision;
  g.KSM = g.KSS = 0;
  sketch_sections(g.prec, p->k, 0, &g.KSM, &g.KSS);
  g.npad = (n + 31) / 32 * 32;
  g.njt = g.npad / 32;
  g.nvt_pad = (g.njt + 3) / 4 * 4;
  // output tiles of 32 columns, padded (with zero blocks of S or O) to whole
  // launch chunks of the kernel
  const int ch = fullvisit_nct(g.prec);
  g.nct_h = ((p->h + 31) / 32 + ch - 1) / ch * ch;
  g.nct_l = ((p->l + 31) / 32 + ch - 1) / ch * ch;
  g.fb = g.prec == SKETCHNE_FP32 ? 4 : 16;
  g.ks2 = g.prec == SKETCHNE_FP32 ? 16 : 2;
  return g;
}

struct FvWs {
  double* d1;
  double* d2;
  double* Kmat;
  double* Sa;
  double* Sb;
  double* Cc;
  double* k_partial;
  size_t k_cap;
  double* Gsel;
  double* RtT;
  void* A1;
  void* Bp;
  void* A2;
  float* T;
  unsigned* tmax;
  double* pscale;
};

FvWs carve_fv(Arena& ar, const sketchne_params* p, int64_t n) {
  FvGeo g = fv_geo(p, n);
  const int k = p->k;
  FvWs w;
  w.d1 = ar.take<double>(n);
  w.d2 = ar.take<double>(n);
  w.Kmat = ar.take<double>((size_t)k * k);
  w.Sa = ar.take<double>((size_t)k * k);
  w.Sb = ar.take<double>((size_t)k * k);
  w.Cc = ar.take<double>((size_t)k * k);
  w.k_cap = max_bytes({gram_ws_bytes(n, k), gemm64_partial_bytes(k, k, k, false),
                       gemm64_partial_bytes(g.npad, k, k, false)});
  w.k_partial = ar.take<double>(w.k_cap / sizeof(double) + 1);
  w.Gsel = ar.take<double>((size_t)g.npad * k);
  w.RtT = ar.take<double>((size_t)g.npad * k);
  w.A1 = ar.take<char>((size_t)g.njt * g.KSM * 64 * g.fb);
  w.Bp = ar.take<char>((size_t)g.nvt_pad * g.KSM * 64 * g.fb);
  const int nct = g.nct_h > g.nct_l ? g.nct_h : g.nct_l;
  w.A2 = ar.take<char>((size_t)g.njt * nct * g.ks2 * 64 * g.fb);
  w.T = ar.take<float>((size_t)p->l * n);
  w.tmax = ar.take<unsigned>(1);
  w.pscale = ar.take<double>(3);
  return w;
}

bool row_sign_ok(const sketchne_row_sign* T, int width, int z) {
  return T && T->width == width && T->z == z && T->cols && T->signs;
}

}  // namespace

extern "C" {

sketchne_status sketchne_fullvisit_workspace_size(const sketchne_params* p, int64_t n, int op_mask, size_t* bytes) {
  if (!bytes || n < 1) return SKETCHNE_E_ARG;
  SK_TRY(check_params(p, n));
  size_t best = 0;
  if (op_mask & SKETCHNE_OP_SKETCH) { Arena a(nullptr, 0); carve_fv(a, p, n); best = a.off > best ? a.off : best; }
  if (op_mask & SKETCHNE_OP_EMBED) {
    Arena a(nullptr, 0);
    carve_embed(a, p, n, true);
    a.take<float>((size_t)n * p->l);
    best = a.off > best ? a.off : best;
  }
  *bytes = best;
  return SKETCHNE_OK;
}

sketchne_status sketchne_sketch_fullvisit(sketchne_ctx* c, const sketchne_graph* A, const sketchne_params* p,
                                          const float* U, const double* lambda, sketchne_row_sign* S,
                                          sketchne_row_sign* O, int generate, float* Yt, float* Z, void* ws,
                                          size_t ws_bytes) {
  if (!c || !U || !lambda || !Yt || !Z) return SKETCHNE_E_ARG;
  SK_TRY(check_graph(A));
  SK_TRY(check_params(p, A->n));
  if (!row_sign_ok(S, p->h, p->z) || !row_sign_ok(O, p->l, p->z) || p->z > p->h) return SKETCHNE_E_ARG;
  if (p->precision == SKETCHNE_FP16 || p->k % 4) return SKETCHNE_E_UNSUPPORTED;
  if (p->l > kFullVisitMaxL) return SKETCHNE_E_UNSUPPORTED;  // the Z pass keeps l 64-bit sums in LDS
  const int64_t n = A->n;
  FvGeo g = fv_geo(p, n);
  if (g.KSM == 0) return SKETCHNE_E_UNSUPPORTED;
  size_t need = 0;
  SK_TRY(sketchne_fullvisit_workspace_size(p, n, SKETCHNE_OP_SKETCH, &need));
  SK_TRY(check_ws(ws, ws_bytes, need));
  Arena ar(ws, ws_bytes);
  FvWs w = carve_fv(ar, p, n);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  const int k = p->k;
  if (generate) {  // z distinct columns per row: the column draw of Alg. 3 with the roles of n and width exchanged
    SK_TRY(gen_sparse_sign(c, p->h, (int)n, p->z, p->seed ^ 0x1111111111111111ULL, S->cols, S->signs));
    SK_TRY(gen_sparse_sign(c, p->l, (int)n, p->z, p->seed ^ 0x2222222222222222ULL, O->cols, O->signs));
  }
  SK_TRY(degree_powers(c, n, A->rowptr, p->alpha, w.d1, w.d2));
  SK_TRY(eq11_core(c, n, k, p->T, U, lambda, w.d2, w.Kmat, w.Sa, w.Sb, w.Cc, w.k_partial, w.k_cap));
  // R'^T rows for every vertex: RtT = scale D1 U C^T (Eq. 11)
  const double scale = (double)A->nnz / (p->b * p->T);
  SK_TRY(gather_rows(c, n, g.npad, k, U, k, w.d1, scale, w.Gsel));
  {
    GemmDesc gd;
    gd.M = g.npad; gd.N = k; gd.K = k;
    gd.A = w.Gsel; gd.ta = Ty::F64; gd.sai = k; gd.sak = 1;
    gd.B = w.Cc; gd.tb = Ty::F64; gd.sbk = 1; gd.sbj = k;
    gd.C = w.RtT; gd.tc = Ty::F64; gd.sci = k; gd.scj = 1;
    SK_TRY(gemm64(c, gd, w.k_partial, w.k_cap));
  }
  SK_TRY(balance(c, g.prec, g.npad * k, w.RtT, w.pscale));
  SK_TRY(pack_A(c, g.prec, (int)g.njt, g.KSM, 0, k, 0, w.RtT, w.pscale, w.A1));
  SK_TRY(pack_B(c, g.prec, n, n, g.nvt_pad, g.KSM, 0, k, 0, nullptr, U, k, w.d1, w.pscale, w.Bp));
  const float inv_sqrt_z = (float)(1.0 / sqrt((double)p->z));
  const float out_scale = 0.69314718055994530942f * inv_sqrt_z;
  // Y = f(L'R') S
  SK_TRY(pack_s_full(c, g.prec, n, g.njt, g.nct_h, p->z, S->cols, S->signs, p->h, w.A2));
  SK_TRY(fullvisit(c, SKETCHNE_PROF_SKETCH_Y, g.prec, g.KSM, n, g.njt, g.nct_h, p->h, w.Bp, w.A1, w.A2, Yt, n,
                   out_scale));
  // T = f(L'R') O, then Z = O^T T
  SK_TRY(pack_s_full(c, g.prec, n, g.njt, g.nct_l, p->z, O->cols, O->signs, p->l, w.A2));
  SK_TRY(fullvisit(c, SKETCHNE_PROF_SKETCH_Z, g.prec, g.KSM, n, g.njt, g.nct_l, p->l, w.Bp, w.A1, w.A2, w.T, n,
                   out_scale));
  return fv_z(c, n, p->l, p->z, O->cols, O->signs, w.T, n, w.tmax, 1.0 / sqrt((double)p->z), Z);
}

sketchne_status sketchne_embed_fullvisit(sketchne_ctx* c, const sketchne_params* p, int64_t n, const float* Yt,
                                         const float* Z, const sketchne_row_sign* O, float* E, double* sigma,
                                         void* ws, size_t ws_bytes) {
  if (!c || !Yt || !Z || !E || !sigma || n < 1) return SKETCHNE_E_ARG;
  SK_TRY(check_params(p, n));
  if (!row_sign_ok(O, p->l, p->z)) return SKETCHNE_E_ARG;
  if (p->h > kSymeigMax) return SKETCHNE_E_UNSUPPORTED;
  if (p->h > n) return SKETCHNE_E_ARG;
  size_t need = 0;
  SK_TRY(sketchne_fullvisit_workspace_size(p, n, SKETCHNE_OP_EMBED, &need));
  SK_TRY(check_ws(ws, ws_bytes, need));
  // the dense O goes after the embedding's own workspace
  Arena ar(nullptr, 0);
  carve_embed(ar, p, n, true);
  const size_t off = ar.off;
  float* Od = reinterpret_cast<float*>(static_cast<char*>(ws) + off);
  SK_TRY(dense_rows(c, n, p->l, p->z, O->cols, O->signs, (float)(1.0 / sqrt((double)p->z)), Od));
  return embed_impl(c, p, n, Yt, Z, nullptr, Od, E, sigma, ws, off);
}

sketchne_status sketchne_sync(sketchne_ctx* c, uint32_t* flags) {
  if (!c) return SKETCHNE_E_ARG;
  if (hipMemcpyAsync(c->h_flags, c->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
    return SKETCHNE_E_DEVICE;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SKETCHNE_E_DEVICE;
  uint32_t f = *c->h_flags;
  if (f) hipMemsetAsync(c->d_flags, 0, sizeof(uint32_t), c->stream);
  if (flags) *flags = f;
  if (f & SKETCHNE_FLAG_BAD_INDEX) return SKETCHNE_E_ARG;
  if (f & (SKETCHNE_FLAG_CHOL_FAIL | SKETCHNE_FLAG_EIG_NOCONV | SKETCHNE_FLAG_NONFINITE)) return SKETCHNE_E_NUMERIC;
  return SKETCHNE_OK;
}

sketchne_status sketchne_spmm(sketchne_ctx* c, const sketchne_graph* A, double alpha, const float* B, int64_t ldb,
                              int32_t cols, float* C, int64_t ldc, void* ws, size_t ws_bytes) {
  if (!c || !B || !C) return SKETCHNE_E_ARG;
  SK_TRY(check_graph(A));
  if (!(alpha > 0.0 && alpha <= 0.5)) return SKETCHNE_E_ARG;
  if (cols < 0 || cols % 4 || cols > 512 || ldb < cols || ldc < cols || ldb % 4 || ldc % 4) return SKETCHNE_E_ARG;
  size_t need = align_up(sizeof(float) * A->n) + spmm_ws_bytes(A->nnz, cols);
  SK_TRY(check_ws(ws, ws_bytes, need));
  Arena ar(ws, ws_bytes);
  float* dscale = ar.take<float>(A->n);
  float* part = ar.take<float>(spmm_ws_bytes(A->nnz, cols) / sizeof(float));
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  SK_TRY(degree_scale(c, A->n, A->rowptr, alpha, dscale));
  return spmm(c, A->n, A->nnz, A->rowptr, A->colidx, dscale, B, ldb, cols, C, ldc, part);
}

sketchne_status sketchne_orth_workspace_size(int64_t n, int32_t cols, size_t* bytes) {
  if (!bytes || n < 1 || cols < 1 || cols > n) return SKETCHNE_E_ARG;
  Arena a(nullptr, 0);
  a.take<float>((size_t)n * cols);
  carve_orth(a, n, cols, false);
  *bytes = a.off;
  return SKETCHNE_OK;
}

sketchne_status sketchne_orth(sketchne_ctx* c, int64_t n, int32_t cols, float* B, int64_t ldb, void* ws,
                              size_t ws_bytes) {
  if (!c || !B || n < 1 || cols < 1 || cols > n || ldb < cols) return SKETCHNE_E_ARG;
  if (cols > kSymeigMax || ldb != cols) return SKETCHNE_E_UNSUPPORTED;  // Gram kernel order; tmp shares ldb
  size_t need = 0;
  SK_TRY(sketchne_orth_workspace_size(n, cols, &need));
  SK_TRY(check_ws(ws, ws_bytes, need));
  Arena ar(ws, ws_bytes);
  float* tmp = ar.take<float>((size_t)n * cols);
  OrthWs ow = carve_orth(ar, n, cols, false);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  // in place: B -> tmp, copy back, then the conditional second pass B -> tmp -> B
  SK_TRY(orth_pass(c, n, cols, B, tmp, ldb, false, ow, ow.need2, nullptr));
  SK_TRY(copy_if(c, n * ldb, tmp, B, nullptr));
  SK_TRY(orth_pass(c, n, cols, B, tmp, ldb, false, ow, nullptr, ow.need2));
  return copy_if(c, n * ldb, tmp, B, ow.need2);
}

sketchne_status sketchne_symeig_workspace_size(int32_t m, size_t* bytes) {
  if (!bytes || m < 1) return SKETCHNE_E_ARG;
  *bytes = symeig_ws_bytes(m);
  return SKETCHNE_OK;
}

sketchne_status sketchne_symeig(sketchne_ctx* c, int32_t m, const double* A, double* V, double* w, void* ws,
                                size_t ws_bytes) {
  if (!c || !A || !V || !w || m < 1) return SKETCHNE_E_ARG;
  if (m > kSymeigMax) return SKETCHNE_E_UNSUPPORTED;
  SK_TRY(check_ws(ws, ws_bytes, symeig_ws_bytes(m)));
  return symeig(c, m, A, V, w, ws);
}

sketchne_status sketchne_symeig_noalloc(sketchne_ctx* c, int32_t m, const double* A, double* V, double* w) {
  if (!c || !A || !V || !w || m < 1) return SKETCHNE_E_ARG;
  if (m > kSymeigMax) return SKETCHNE_E_UNSUPPORTED;
  void* ws = symeig_scratch(c->device);
  if (!ws) {
    // first call on a device whose lookup failed at create: try once more
    SK_TRY(symeig_scratch_init(c->device));
    ws = symeig_scratch(c->device);
  }
  if (!ws || symeig_ws_bytes(m) > symeig_scratch_bytes()) return SKETCHNE_E_DEVICE;
  return symeig(c, m, A, V, w, ws);
}

sketchne_status sketchne_propagate_coeffs(int32_t p, double theta, double mu, double* coef) {
  if (!coef || p < 0 || p > kPropagateMaxDegree || !(theta >= 0.0) || !isfinite(mu)) return SKETCHNE_E_ARG;
  // interpolation at the p + 1 Chebyshev nodes x_j = cos(phi_j) of [-1, 1],
  // lambda_j = 1 + x_j: c_r = (2 - [r == 0]) / (p + 1) sum_j g(lambda_j) cos(r phi_j)
  const double pi = 3.14159265358979323846;
  double gv[kPropagateMaxDegree + 1];
  for (int j = 0; j <= p; ++j) {
    const double phi = pi * (j + 0.5) / (p + 1);
    const double lam = 1.0 + cos(phi) - mu;
    gv[j] = exp(-0.5 * theta * (lam * lam - 1.0));
  }
  for (int r = 0; r <= p; ++r) {
    double acc = 0.0;
    for (int j = 0; j <= p; ++j) acc += gv[j] * cos(r * pi * (j + 0.5) / (p + 1));
    coef[r] = acc * (r == 0 ? 1.0 : 2.0) / (p + 1);
  }
  return SKETCHNE_OK;
}

sketchne_status sketchne_propagate_workspace_size(int64_t n, int64_t nnz, int32_t d, size_t* bytes) {
  if (!bytes || n < 1 || nnz < 0 || d < 1) return SKETCHNE_E_ARG;
  *bytes = propagate_ws_bytes(n, nnz, d);
  return SKETCHNE_OK;
}

sketchne_status sketchne_propagate(sketchne_ctx* c, const sketchne_graph* A, int32_t d, const float* E, int64_t lde,
                                   int32_t p, const double* coef, float* out, int64_t ldo, void* ws,
                                   size_t ws_bytes) {
  if (!c || !E || !out || !coef) return SKETCHNE_E_ARG;
  SK_TRY(check_graph(A));
  if (d < 1 || d % 4 || lde < d || ldo < d || lde % 4 || ldo % 4 || p < 0) return SKETCHNE_E_ARG;
  if (d > 256 || p > kPropagateMaxDegree) return SKETCHNE_E_UNSUPPORTED;
  if (reinterpret_cast<uintptr_t>(E) % 16 || reinterpret_cast<uintptr_t>(out) % 16) return SKETCHNE_E_ARG;
  for (int r = 0; r <= p; ++r)
    if (!isfinite(coef[r])) return SKETCHNE_E_ARG;
  SK_TRY(check_ws(ws, ws_bytes, propagate_ws_bytes(A->n, A->nnz, d)));
  return propagate(c, A->n, A->nnz, A->rowptr, A->colidx, d, E, lde, p, coef, out, ldo, ws);
}

sketchne_status sketchne_gen_gauss(sketchne_ctx* c, int64_t n, int32_t cols, uint64_t seed, float* out) {
  if (!c || !out || n < 0 || cols < 0) return SKETCHNE_E_ARG;
  return gen_gauss(c, n, cols, cols, seed, out);
}

sketchne_status sketchne_gen_sparse_sign(sketchne_ctx* c, int64_t n, uint64_t seed, sketchne_sparse_sign* out) {
  if (!c || !out || !out->rows || !out->signs || n < 1 || out->cols < 0 || out->z < 1 || out->z > n)
    return SKETCHNE_E_ARG;
  if (n >= ((int64_t)1 << 31)) return SKETCHNE_E_UNSUPPORTED;
  return gen_sparse_sign(c, n, out->cols, out->z, seed, out->rows, out->signs);
}

sketchne_status sketchne_ws_param_count(int32_t width, int32_t out, int64_t* count) {
  if (!count || width < 1 || out < 1) return SKETCHNE_E_ARG;
  *count = ws_param_count(width, out);
  return SKETCHNE_OK;
}

sketchne_status sketchne_ws_workspace_size(const sketchne_params* p, int32_t width, int32_t out, int64_t n,
                                           int64_t nnz, int op_mask, size_t* bytes) {
  if (!bytes || width < 1 || out < 1 || n < 1 || nnz < 0) return SKETCHNE_E_ARG;
  size_t best = 0;
  if (op_mask & SKETCHNE_WS_OP_FEATURES) best = max_bytes({best, ws_features_bytes(n, nnz)});
  if (op_mask & SKETCHNE_WS_OP_FORWARD) best = max_bytes({best, ws_forward_bytes(n, width), ws_infer_bytes()});
  if (op_mask & SKETCHNE_WS_OP_GRAD) best = max_bytes({best, ws_grad_bytes(n, width, out)});
  if (op_mask & (SKETCHNE_WS_OP_RESIDUAL | SKETCHNE_WS_OP_EIG)) {
    if (!p) return SKETCHNE_E_ARG;
    SK_TRY(check_params(p, n));
    if (op_mask & SKETCHNE_WS_OP_RESIDUAL) best = max_bytes({best, ritz_residual_bytes(n, nnz, p->k)});
    if (op_mask & SKETCHNE_WS_OP_EIG) best = max_bytes({best, learned_bytes(p, width, n, nnz)});
  }
  *bytes = best;
  return SKETCHNE_OK;
}

sketchne_status sketchne_ws_init(sketchne_ctx* c, const sketchne_mlp* net, uint64_t seed) {
  if (!c) return SKETCHNE_E_ARG;
  SK_TRY(check_net(net));
  return ws_init(c, net, seed);
}

sketchne_status sketchne_ws_features(sketchne_ctx* c, const sketchne_graph* A, double alpha, const float* g,
                                     uint64_t seed, float* phi, void* ws, size_t ws_bytes) {
  if (!c || !phi) return SKETCHNE_E_ARG;
  SK_TRY(check_graph(A));
  if (!(alpha > 0.0 && alpha <= 0.5)) return SKETCHNE_E_ARG;
  SK_TRY(check_ws(ws, ws_bytes, ws_features_bytes(A->n, A->nnz)));
  return ws_features(c, A->n, A->nnz, A->rowptr, A->colidx, alpha, g, seed, phi, ws, ws_bytes);
}

sketchne_status sketchne_ws_forward(sketchne_ctx* c, const sketchne_mlp* net, int64_t n, const float* phi, float* F,
                                    int64_t ldf, void* ws, size_t ws_bytes) {
  if (!c || !phi || !F || n < 0) return SKETCHNE_E_ARG;
  SK_TRY(check_net(net));
  if (ldf < net->out) return SKETCHNE_E_ARG;
  if (n == 0) return SKETCHNE_OK;
  SK_TRY(check_ws(ws, ws_bytes, ws_forward_bytes(n, net->width)));
  return ws_forward(c, net, n, phi, F, ldf, ws, ws_bytes);
}

sketchne_status sketchne_ws_infer(sketchne_ctx* c, const sketchne_mlp* net, int64_t n, const float* phi, float* F,
                                  int64_t ldf, void* ws, size_t ws_bytes) {
  if (!c || !phi || !F || n < 0) return SKETCHNE_E_ARG;
  SK_TRY(check_net(net));
  if (ldf < net->out) return SKETCHNE_E_ARG;
  if (!ws_infer_supported(net)) return SKETCHNE_E_UNSUPPORTED;
  SK_TRY(check_ws(ws, ws_bytes, ws_infer_bytes()));
  return ws_infer(c, net, n, phi, F, ldf, ws, ws_bytes);
}

sketchne_status sketchne_ws_grad(sketchne_ctx* c, const sketchne_mlp* net, int64_t n, const float* phi,
                                 const float* U, int64_t ldu, float mu, float* grad, float* loss, void* ws,
                                 size_t ws_bytes) {
  if (!c || !phi || !U || !grad || !loss || n < 1 || !(mu >= 0.f)) return SKETCHNE_E_ARG;
  SK_TRY(check_net(net));
  if (ldu < net->out) return SKETCHNE_E_ARG;
  SK_TRY(check_ws(ws, ws_bytes, ws_grad_bytes(n, net->width, net->out)));
  return ws_grad(c, net, n, phi, U, ldu, mu, grad, loss, ws, ws_bytes);
}

sketchne_status sketchne_ws_adam(sketchne_ctx* c, const sketchne_mlp* net, const float* grad, float lr,
                                 int32_t step) {
  if (!c || !grad || step < 1 || !(lr > 0.f)) return SKETCHNE_E_ARG;
  SK_TRY(check_net(net));
  if (!net->adam_m || !net->adam_v) return SKETCHNE_E_ARG;
  return ws_adam(c, net, grad, lr, step, 0.9, 0.999, 1e-8);
}

sketchne_status sketchne_ws_train(sketchne_ctx* c, const sketchne_mlp* net, int32_t nsets,
                                  const float* const* phi, const float* const* U, const int64_t* n, int32_t steps,
                                  int32_t step0, float lr, float mu, float* losses, void* ws, size_t ws_bytes) {
  if (!c || !phi || !U || !n || !losses || nsets < 1 || steps < 0 || step0 < 0 || !(lr > 0.f) || !(mu >= 0.f))
    return SKETCHNE_E_ARG;
  SK_TRY(check_net(net));
  if (!net->adam_m || !net->adam_v) return SKETCHNE_E_ARG;
  int64_t nmax = 0;
  for (int s = 0; s < nsets; ++s) {
    if (!phi[s] || !U[s] || n[s] < 1) return SKETCHNE_E_ARG;
    nmax = n[s] > nmax ? n[s] : nmax;
  }
  const int64_t count = ws_param_count(net->width, net->out);
  const size_t gb = ws_grad_bytes(nmax, net->width, net->out);
  SK_TRY(check_ws(ws, ws_bytes, align_up(sizeof(float) * count) + gb));
  Arena ar(ws, ws_bytes);
  float* grad = ar.take<float>(count);
  char* scratch = ar.take<char>(gb);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  for (int t = 0; t < steps; ++t) {
    const int s = t % nsets;
    SK_TRY(ws_grad(c, net, n[s], phi[s], U[s], net->out, mu, grad, losses + t, scratch, gb));
    SK_TRY(ws_adam(c, net, grad, lr, step0 + t + 1, 0.9, 0.999, 1e-8));
  }
  return SKETCHNE_OK;
}

sketchne_status sketchne_ritz_residual(sketchne_ctx* c, const sketchne_graph* A, double alpha, int32_t k,
                                       const float* U, const double* lambda, double* res, void* ws,
                                       size_t ws_bytes) {
  if (!c || !U || !lambda || !res) return SKETCHNE_E_ARG;
  SK_TRY(check_graph(A));
  if (!(alpha > 0.0 && alpha <= 0.5) || k < 4 || k % 4 || k > A->n) return SKETCHNE_E_ARG;
  if (k > 512) return SKETCHNE_E_UNSUPPORTED;
  SK_TRY(check_ws(ws, ws_bytes, ritz_residual_bytes(A->n, A->nnz, k)));
  return ritz_residual(c, A->n, A->nnz, A->rowptr, A->colidx, alpha, k, U, lambda, res, ws, ws_bytes);
}

sketchne_status sketchne_eig_learned(sketchne_ctx* c, const sketchne_graph* A, const sketchne_params* p,
                                     const sketchne_mlp* net, int32_t q_warm, double res_threshold, float* U,
                                     double* lambda, int32_t* used_fallback, double* worst_residual, void* ws,
                                     size_t ws_bytes) {
  if (!c || !U || !lambda || !used_fallback || q_warm < 0) return SKETCHNE_E_ARG;
  SK_TRY(check_graph(A));
  SK_TRY(check_params(p, A->n));
  SK_TRY(check_net(net));
  if (net->out > p->k) return SKETCHNE_E_ARG;
  const int K = p->k + p->s_eig;
  if (K > kSymeigMax || K % 4 || p->k % 4) return SKETCHNE_E_UNSUPPORTED;
  const int64_t n = A->n;
  SK_TRY(check_ws(ws, ws_bytes, learned_bytes(p, net->width, n, A->nnz)));
  Arena ar(ws, ws_bytes);
  float* omega = ar.take<float>((size_t)n * K);
  double* res = ar.take<double>(p->k);
  const size_t rest_bytes = learned_rest_bytes(p, net->width, n, A->nnz);
  char* rest = ar.take<char>(rest_bytes);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  *used_fallback = 0;
  // start block: [F | Gaussian]
  {
    Arena r(rest, rest_bytes);
    float* phi = r.take<float>((size_t)n * SKETCHNE_WS_FEAT);
    char* scratch = r.take<char>(rest_bytes - r.off);
    size_t sb = rest_bytes - align_up(sizeof(float) * (size_t)n * SKETCHNE_WS_FEAT);
    if (r.overflow) return SKETCHNE_E_WORKSPACE;
    SK_TRY(ws_features(c, n, A->nnz, A->rowptr, A->colidx, p->alpha, nullptr, p->seed ^ 0x7f4a7c159e3779b9ULL, phi,
                       scratch, sb));
    if (ws_infer_supported(net)) SK_TRY(ws_infer(c, net, n, phi, omega, K, scratch, sb));
    else SK_TRY(ws_forward(c, net, n, phi, omega, K, scratch, sb));
    SK_TRY(gen_gauss(c, n, K - net->out, K, p->seed, omega + net->out));
  }
  sketchne_params pw = *p;
  pw.q = q_warm;
  SK_TRY(eig_impl(c, A, &pw, omega, U, lambda, res, rest, rest_bytes));
  // residual test on the Ritz residuals of the warm-started pairs
  {
    double* host = new (std::nothrow) double[p->k];
    if (!host) return SKETCHNE_E_DEVICE;
    hipError_t e = hipMemcpyAsync(host, res, sizeof(double) * p->k, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    double worst = 0.0;
    bool finite = true;
    for (int j = 0; j < p->k; ++j) {
      if (!(host[j] == host[j]) || host[j] > 1e300) finite = false;
      else if (host[j] > worst) worst = host[j];
    }
    delete[] host;
    if (e != hipSuccess) return SKETCHNE_E_DEVICE;
    if (worst_residual) *worst_residual = finite ? worst : HUGE_VAL;
    if (finite && worst <= res_threshold) return SKETCHNE_OK;
  }
  *used_fallback = 1;
  return sketchne_eig(c, A, p, nullptr, U, lambda, rest, rest_bytes);
}

sketchne_status sketchne_profile_enable(sketchne_ctx* c, int on) {
  if (!c) return SKETCHNE_E_ARG;
  const uint32_t all = (1u << SKETCHNE_PROF_CLASSES) - 1;
  if (on != 0 && on != 1 && ((on & SKETCHNE_PROF_SELECT) == 0 || ((uint32_t)on & ~(SKETCHNE_PROF_SELECT | all))))
    return SKETCHNE_E_ARG;
  c->profiling = on != 0;
  c->prof_mask = on == 1 ? all : (uint32_t)on & all;
  c->n_ev = 0;
  for (int i = 0; i < SKETCHNE_PROF_CLASSES; ++i) { c->prof_ms[i] = 0; c->prof_n[i] = 0; }
  return SKETCHNE_OK;
}

sketchne_status sketchne_profile_read(sketchne_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return SKETCHNE_E_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return SKETCHNE_E_DEVICE;
  for (int e = 0; e + 1 < c->n_ev; e += 2) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, c->ev[e], c->ev[e + 1]) == hipSuccess) {
      int cls = c->ev_class[e / 2];
      c->prof_ms[cls] += t;
      c->prof_n[cls] += 1;
    }
  }
  c->n_ev = 0;
  for (int i = 0; i < SKETCHNE_PROF_CLASSES; ++i) {
    ms[i] = c->prof_ms[i];
    launches[i] = c->prof_n[i];
    c->prof_ms[i] = 0;
    c->prof_n[i] = 0;
  }
  return SKETCHNE_OK;
}

}  // extern "C"
