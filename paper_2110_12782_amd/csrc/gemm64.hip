// FP64-accumulating GEMM on the FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
//   C(i,j) = alpha * sum_k A(i,k) * w(k) * B(k,j)  [+ diag_add if i == j]
//
// with arbitrary element strides for A, B and C, FP32 or FP64 operands
// (FP32 inputs are widened exactly to FP64), an optional weight on the
// summation index (used for U^T D^p U) and split-K with a deterministic
// second-pass reduction.  This one kernel serves every dense FP64 product of
// the path: the Gram matrices of Cholesky-QR, the Rayleigh-Ritz matrix
// Q^T (XQ), the applies B R^-1 and Q U^, the k x k Horner products of
// Eq. (11) and the small products of Alg. 4 line 8.
//
// Tiling: 64 x 64 output tile per 256-thread workgroup, 2 x 2 wavefronts of
// 32 x 32 (2 x 2 MFMA blocks of 16 x 16), K step 16 staged through LDS with
// a register prefetch of the next step.  Workgroups that share an operand
// panel (the row tiles of one output row block, or the tiles of one K split)
// are given linear ids congruent mod 8 so that they run on the same XCD and
// share its L2.
#include "internal.h"

namespace skne {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int BM = 64, BN = 64, BK = 16, LDP = BM + 2;

struct GemmArgs {
  int64_t M, N, K;
  const void* A; int ta; int64_t sai, sak;
  const void* B; int tb; int64_t sbk, sbj;
  void* C; int tc; int64_t sci, scj;
  const double* kw;
  double alpha, diag_add;
  int upper_only;
  int splits;
  int64_t kchunk;       // K range per split (multiple of BK)
  int tiles_m, tiles_n;
  int ntile_items;      // tiles per split (grid items per group)
  int groups;           // number of "groups" mapped to one XCD (row tiles or splits)
  int group_is_split;   // 1: group = split, item = tile; 0: group = row tile, item = col tile
  double* partial;      // splits x M x N when splits > 1
};

__device__ __forceinline__ double ld_elem(const void* p, int t, int64_t off) {
  return t == 0 ? (double)static_cast<const float*>(p)[off] : static_cast<const double*>(p)[off];
}

// enumerate upper-triangular tile pairs (tm <= tn) in row order
__device__ __forceinline__ void upper_tile(int idx, int nt, int& tm, int& tn) {
  int r = 0;
  int rowlen = nt;
  while (idx >= rowlen) { idx -= rowlen; ++r; --rowlen; }
  tm = r;
  tn = r + idx;
}

__global__ __launch_bounds__(256) void k_gemm64(GemmArgs g) {
  __shared__ double As[2][BK][LDP];
  __shared__ double Bs[2][BK][LDP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // ---- XCD-aware decode of the linear workgroup id
  const int L = blockIdx.x;
  int item, group;
  if (g.groups >= 8) {
    const int xcd = L & 7, q = L >> 3;
    item = q % g.ntile_items;
    group = (q / g.ntile_items) * 8 + xcd;
  } else {
    item = L % g.ntile_items;
    group = L / g.ntile_items;
  }
  if (group >= g.groups) return;
  int split, tm, tn;
  if (g.group_is_split) {
    split = group;
    if (g.upper_only) upper_tile(item, g.tiles_m, tm, tn);
    else { tm = item / g.tiles_n; tn = item % g.tiles_n; }
  } else {
    split = 0;
    tm = group;
    tn = item;
  }
  const int64_t i0 = (int64_t)tm * BM, j0 = (int64_t)tn * BN;
  const int64_t kbeg = (int64_t)split * g.kchunk;
  const int64_t kend = min(g.K, kbeg + g.kchunk);

  const bool a_kfast = (g.sak == 1);
  const bool b_jfast = (g.sbj == 1) || (g.sbk != 1);

  double ra[4], rb[4];
  auto load_regs = [&](int64_t k0) {
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      int ii, kk;
      if (a_kfast) { kk = tid & 15; ii = (tid >> 4) + 16 * rep; }
      else { ii = tid & 63; kk = (tid >> 6) + 4 * rep; }
      int64_t i = i0 + ii, k = k0 + kk;
      double v = 0.0;
      if (i < g.M && k < kend) {
        v = ld_elem(g.A, g.ta, i * g.sai + k * g.sak);
        if (g.kw) v *= g.kw[k];
      }
      ra[rep] = v;
      int jj, kb;
      if (b_jfast) { jj = tid & 63; kb = (tid >> 6) + 4 * rep; }
      else { kb = tid & 15; jj = (tid >> 4) + 16 * rep; }
      int64_t j = j0 + jj, kq = k0 + kb;
      rb[rep] = (j < g.N && kq < kend) ? ld_elem(g.B, g.tb, kq * g.sbk + j * g.sbj) : 0.0;
    }
  };
  auto store_lds = [&](int buf) {
#pragma unroll
    for (int rep = 0; rep < 4; ++rep) {
      int ii, kk;
      if (a_kfast) { kk = tid & 15; ii = (tid >> 4) + 16 * rep; }
      else { ii = tid & 63; kk = (tid >> 6) + 4 * rep; }
      As[buf][kk][ii] = ra[rep];
      int jj, kb;
      if (b_jfast) { jj = tid & 63; kb = (tid >> 6) + 4 * rep; }
      else { kb = tid & 15; jj = (tid >> 4) + 16 * rep; }
      Bs[buf][kb][jj] = rb[rep];
    }
  };

  doublex4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = doublex4{0.0, 0.0, 0.0, 0.0};

  int buf = 0;
  if (kbeg < kend) {
    load_regs(kbeg);
    store_lds(0);
  }
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load_regs(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      const int kr = kk * 4 + (lane >> 4);
      double a0 = As[buf][kr][wm * 32 + (lane & 15)];
      double a1 = As[buf][kr][wm * 32 + 16 + (lane & 15)];
      double b0 = Bs[buf][kr][wn * 32 + (lane & 15)];
      double b1 = Bs[buf][kr][wn * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    if (more) store_lds(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // ---- epilogue
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // v_mfma_f64_16x16x4f64 output: lane l, register r holds row (l / 16) + 4 r, column l % 16
        int64_t i = i0 + wm * 32 + mt * 16 + (lane >> 4) + 4 * r;
        int64_t j = j0 + wn * 32 + nt * 16 + (lane & 15);
        if (i >= g.M || j >= g.N) continue;
        double v = acc[mt][nt][r];
        if (g.splits > 1) {
          g.partial[((int64_t)split * g.M + i) * g.N + j] = v;
        } else {
          v = g.alpha * v + (i == j ? g.diag_add : 0.0);
          int64_t off = i * g.sci + j * g.scj;
          if (g.tc == 0) static_cast<float*>(g.C)[off] = (float)v;
          else static_cast<double*>(g.C)[off] = v;
          if (g.upper_only && tm != tn) {
            int64_t off2 = j * g.sci + i * g.scj;
            if (g.tc == 0) static_cast<float*>(g.C)[off2] = (float)v;
            else static_cast<double*>(g.C)[off2] = v;
          }
        }
      }
}

__global__ void k_gemm64_reduce(GemmArgs g) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.M * g.N) return;
  int64_t i = idx / g.N, j = idx - i * g.N;
  int64_t si = i, sj = j;
  if (g.upper_only && (i / BM) > (j / BN)) { si = j; sj = i; }
  double s = 0.0;
  for (int sp = 0; sp < g.splits; ++sp) s += g.partial[((int64_t)sp * g.M + si) * g.N + sj];
  double v = g.alpha * s + (i == j ? g.diag_add : 0.0);
  int64_t off = i * g.sci + j * g.scj;
  if (g.tc == 0) static_cast<float*>(g.C)[off] = (float)v;
  else static_cast<double*>(g.C)[off] = v;
}

}  // namespace

int gemm64_pick_splits(const GemmDesc& d) {
  int64_t tm = (d.M + BM - 1) / BM, tn = (d.N + BN - 1) / BN;
  int64_t tiles = d.upper_only ? tm * (tm + 1) / 2 : tm * tn;
  if (tiles >= 512 || d.K <= 4 * BK) return 1;
  int64_t want = (1024 + tiles - 1) / tiles;
  int64_t maxs = (d.K + 8 * BK - 1) / (8 * BK);  // at least 8 K steps per split
  int64_t s = want < maxs ? want : maxs;
  if (s > 128) s = 128;
  return s < 1 ? 1 : (int)s;
}

size_t gemm64_ws_bytes(const GemmDesc& d, int splits) {
  return splits > 1 ? align_up(sizeof(double) * (size_t)splits * d.M * d.N) : 0;
}

size_t gemm64_partial_bytes(int64_t M, int64_t N, int64_t K, bool upper) {
  GemmDesc d;
  d.M = M; d.N = N; d.K = K; d.upper_only = upper;
  return gemm64_ws_bytes(d, gemm64_pick_splits(d));
}

sketchne_status gemm64(sketchne_ctx* c, const GemmDesc& d, double* partial, size_t partial_cap) {
  if (d.M == 0 || d.N == 0) return SKETCHNE_OK;
  if (d.upper_only && d.M != d.N) return SKETCHNE_E_ARG;
  int splits = gemm64_pick_splits(d);
  if (splits > 1) {
    size_t per = sizeof(double) * (size_t)d.M * (size_t)d.N;
    size_t fit = partial ? partial_cap / per : 0;
    if ((size_t)splits > fit) splits = fit >= 2 ? (int)fit : 1;
  }
  ProfScope ps(c, SKETCHNE_PROF_GEMM64);
  GemmArgs g{};
  g.M = d.M; g.N = d.N; g.K = d.K;
  g.A = d.A; g.ta = (int)d.ta; g.sai = d.sai; g.sak = d.sak;
  g.B = d.B; g.tb = (int)d.tb; g.sbk = d.sbk; g.sbj = d.sbj;
  g.C = d.C; g.tc = (int)d.tc; g.sci = d.sci; g.scj = d.scj;
  g.kw = d.kw; g.alpha = d.alpha; g.diag_add = d.diag_add; g.upper_only = d.upper_only ? 1 : 0;
  g.splits = splits < 1 ? 1 : splits;
  int64_t kc = (d.K + g.splits - 1) / g.splits;
  g.kchunk = (kc + BK - 1) / BK * BK;
  if (g.kchunk == 0) g.kchunk = BK;
  g.tiles_m = (int)((d.M + BM - 1) / BM);
  g.tiles_n = (int)((d.N + BN - 1) / BN);
  g.partial = partial;
  if (g.splits > 1 || d.upper_only) {
    g.group_is_split = 1;
    g.groups = g.splits;
    g.ntile_items = d.upper_only ? g.tiles_m * (g.tiles_m + 1) / 2 : g.tiles_m * g.tiles_n;
  } else {
    g.group_is_split = 0;
    g.groups = g.tiles_m;
    g.ntile_items = g.tiles_n;
  }
  int64_t gpad = g.groups >= 8 ? ((int64_t)g.groups + 7) / 8 * 8 : g.groups;
  int64_t blocks = gpad * g.ntile_items;
  hipLaunchKernelGGL(k_gemm64, dim3((unsigned)blocks), dim3(256), 0, c->stream, g);
  if (g.splits > 1) {
    int64_t tot = d.M * d.N;
    hipLaunchKernelGGL(k_gemm64_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, g);
  }
  return launch_status();
}

}  // namespace skne
