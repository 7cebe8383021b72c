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
// Tiling: a 64 x 64 or 96 x 96 output tile per 256-thread workgroup (the one
// that pads the output less), 2 x 2 wavefronts each holding 2 x 2 or 3 x 3
// MFMA blocks of 16 x 16, K step 16 staged through LDS with a register
// prefetch of the next step.  Workgroups that share an operand
// panel (the row tiles of one output row block, or the tiles of one K split)
// are given linear ids congruent mod 8 so that they run on the same XCD and
// share its L2.
#include "internal.h"

namespace skne {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));

constexpr int BK = 16;

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
  int tile;             // square output tile edge (64 or 96)
  int tiles_m, tiles_n;
  int ntile_items;      // tiles per split (grid items per group)
  int groups;           // number of "groups" mapped to one XCD (row tiles or splits)
  int group_is_split;   // 1: group = split, item = tile; 0: group = row tile, item = col tile
  double* partial;      // splits x M x N when splits > 1
  const int* run_if;    // when non-null and zero: do nothing
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

// T x T output tile per workgroup (4 wavefronts in 2 x 2, each (T/2) x (T/2)
// = TT x TT MFMA blocks of 16 x 16).
template <int T, bool AKF, bool BJF>
__global__ __launch_bounds__(256) void k_gemm64(GemmArgs g) {
  constexpr int TT = T / 32;           // MFMA blocks per wave and dimension
  constexpr int LDP = T + 2;
  constexpr int PER = T * BK / 256;    // elements of each operand tile per thread
  __shared__ double As[2][BK][LDP];
  __shared__ double Bs[2][BK][LDP];
  if (g.run_if && *g.run_if == 0) return;
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
  const int64_t i0 = (int64_t)tm * T, j0 = (int64_t)tn * T;
  const int64_t kbeg = (int64_t)split * g.kchunk;
  const int64_t kend = min(g.K, kbeg + g.kchunk);

  // element e = tid + 256 rep of a tile: (fast index, slow index); AKF: the
  // summation index is contiguous in A, BJF: the column index is contiguous in B
  auto a_coord = [&](int e, int& ii, int& kk) {
    if (AKF) { kk = e % BK; ii = e / BK; } else { ii = e % T; kk = e / T; }
  };
  auto b_coord = [&](int e, int& jj, int& kk) {
    if (BJF) { jj = e % T; kk = e / T; } else { kk = e % BK; jj = e / BK; }
  };

  double ra[PER], rb[PER];
  auto load_regs = [&](int64_t k0) {
#pragma unroll
    for (int rep = 0; rep < PER; ++rep) {
      const int e = tid + 256 * rep;
      int ii, kk;
      a_coord(e, ii, kk);
      const int64_t i = i0 + ii, k = k0 + kk;
      double v = 0.0;
      if (i < g.M && k < kend) {
        const int64_t off = AKF ? (i * g.sai + k) : (i + k * g.sak);
        v = ld_elem(g.A, g.ta, off);
        if (g.kw) v *= g.kw[k];
      }
      ra[rep] = v;
      int jj, kb;
      b_coord(e, jj, kb);
      const int64_t j = j0 + jj, kq = k0 + kb;
      const int64_t offb = BJF ? (kq * g.sbk + j * g.sbj) : (kq + j * g.sbj);
      rb[rep] = (j < g.N && kq < kend) ? ld_elem(g.B, g.tb, offb) : 0.0;
    }
  };
  auto store_lds = [&](int buf) {
#pragma unroll
    for (int rep = 0; rep < PER; ++rep) {
      const int e = tid + 256 * rep;
      int ii, kk;
      a_coord(e, ii, kk);
      As[buf][kk][ii] = ra[rep];
      int jj, kb;
      b_coord(e, jj, kb);
      Bs[buf][kb][jj] = rb[rep];
    }
  };

  doublex4 acc[TT][TT];
#pragma unroll
  for (int a = 0; a < TT; ++a)
#pragma unroll
    for (int b = 0; b < TT; ++b) acc[a][b] = doublex4{0.0, 0.0, 0.0, 0.0};

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
      double af[TT], bf[TT];
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        af[t] = As[buf][kr][wm * (T / 2) + t * 16 + (lane & 15)];
        bf[t] = Bs[buf][kr][wn * (T / 2) + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int a = 0; a < TT; ++a)
#pragma unroll
        for (int b = 0; b < TT; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
    if (more) store_lds(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }

  // ---- epilogue
#pragma unroll
  for (int mt = 0; mt < TT; ++mt)
#pragma unroll
    for (int nt = 0; nt < TT; ++nt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // v_mfma_f64_16x16x4f64 output: lane l, register r holds row (l / 16) + 4 r, column l % 16
        int64_t i = i0 + wm * (T / 2) + mt * 16 + (lane >> 4) + 4 * r;
        int64_t j = j0 + wn * (T / 2) + nt * 16 + (lane & 15);
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
  if (g.run_if && *g.run_if == 0) return;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= g.M * g.N) return;
  int64_t i = idx / g.N, j = idx - i * g.N;
  int64_t si = i, sj = j;
  if (g.upper_only && (i / g.tile) > (j / g.tile)) { si = j; sj = i; }
  double s = 0.0;
  for (int sp = 0; sp < g.splits; ++sp) s += g.partial[((int64_t)sp * g.M + si) * g.N + sj];
  double v = g.alpha * s + (i == j ? g.diag_add : 0.0);
  int64_t off = i * g.sci + j * g.scj;
  if (g.tc == 0) static_cast<float*>(g.C)[off] = (float)v;
  else static_cast<double*>(g.C)[off] = v;
}

}  // namespace

// square tile edge: the one of {64, 96} that pads the output least (96 on ties)
static int pick_tile(int64_t M, int64_t N, bool upper) {
  auto area = [&](int64_t t) {
    int64_t a = (M + t - 1) / t, b = (N + t - 1) / t;
    return (upper ? a * (a + 1) / 2 : a * b) * t * t;
  };
  return area(96) <= area(64) ? 96 : 64;
}

int gemm64_pick_splits(const GemmDesc& d) {
  const int T = pick_tile(d.M, d.N, d.upper_only);
  int64_t tm = (d.M + T - 1) / T, tn = (d.N + T - 1) / T;
  int64_t tiles = d.upper_only ? tm * (tm + 1) / 2 : tm * tn;
  if (tiles >= 512 || d.K <= 4 * BK) return 1;
  int64_t want = (1024 + tiles - 1) / tiles;
  int64_t maxs = (d.K + 8 * BK - 1) / (8 * BK);  // at least 8 K steps per split
  int64_t s = want < maxs ? want : maxs;
  if (s > 256) s = 256;
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
  g.tile = pick_tile(d.M, d.N, d.upper_only);
  g.tiles_m = (int)((d.M + g.tile - 1) / g.tile);
  g.tiles_n = (int)((d.N + g.tile - 1) / g.tile);
  g.partial = partial;
  g.run_if = d.run_if;
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
  // load layouts: A contiguous along the summation index (sak == 1) or along
  // rows (sai == 1); B contiguous along columns (sbj == 1) or along the
  // summation index (sbk == 1)
  const bool akf = d.sak == 1 && d.sai != 1 ? true : (d.sai == 1 ? false : d.sak == 1);
  const bool bjf = !(d.sbk == 1 && d.sbj != 1);
  if (!akf && d.sai != 1) return SKETCHNE_E_ARG;
  if (!bjf && d.sbk != 1) return SKETCHNE_E_ARG;
  dim3 grid((unsigned)blocks), blk(256);
#define SKNE_GEMM_LAUNCH(T)                                                                  \
  do {                                                                                       \
    if (akf && bjf) hipLaunchKernelGGL((k_gemm64<T, true, true>), grid, blk, 0, c->stream, g);  \
    else if (akf) hipLaunchKernelGGL((k_gemm64<T, true, false>), grid, blk, 0, c->stream, g);   \
    else if (bjf) hipLaunchKernelGGL((k_gemm64<T, false, true>), grid, blk, 0, c->stream, g);   \
    else hipLaunchKernelGGL((k_gemm64<T, false, false>), grid, blk, 0, c->stream, g);           \
  } while (0)
  if (g.tile == 96) SKNE_GEMM_LAUNCH(96);
  else SKNE_GEMM_LAUNCH(64);
#undef SKNE_GEMM_LAUNCH
  if (g.splits > 1) {
    int64_t tot = d.M * d.N;
    hipLaunchKernelGGL(k_gemm64_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, g);
  }
  return launch_status();
}

}  // namespace skne
