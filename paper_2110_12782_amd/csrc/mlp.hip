// Learned warm start for the randomized eigensolver (an addition to Alg. 5,
// which starts from a Gaussian block): per-vertex features, a 3-layer ReLU
// network whose output replaces the first k columns of the start block, the
// subspace loss that trains it, backpropagation and Adam.
//
//   features  phi_i = standardised [log max(deg_i,1), (Xg)_i, (X^2g)_i, (X^3g)_i, (X^4g)_i, 0, 0, 0]
//             X = D^-a A D^-a, g Rademacher; a column whose standard deviation is at
//             most 1e-6 times its root mean square is set to 0.
//   network   F = relu(relu(phi W1 + b1) W2 + b2) W3 + b3
//   loss      L = ||(I - UU^T)F||^2/||F||^2 + mu ||(k/||F||^2) F^T F - I||^2
//             dL/dF = U A + F B,  A = -(2/s) P,
//             B = (4 mu k/s) M + (2||P||^2/s^2 - 4 mu k <M,G>/s^2) I
//             with s = ||F||^2, P = U^T F, G = F^T F, M = (k/s) G - I.
//
// Weights are stored in BF16 (an FP32 master copy is what Adam updates);
// activations are FP32 and every product runs on the FP32 matrix cores
// (v_mfma_f32_32x32x2_f32) with FP32 accumulation.  Reductions over vertices
// (weight gradients, F^T F, U^T F, column sums) are split over fixed row
// ranges and summed in a fixed order, so results are deterministic.
#include "internal.h"

#include <type_traits>

namespace skne {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int FEAT = SKETCHNE_WS_FEAT;

__device__ __forceinline__ float bf16_val(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
template <typename WT> __device__ __forceinline__ float wval(const WT* w, int64_t i);
template <> __device__ __forceinline__ float wval<uint16_t>(const uint16_t* w, int64_t i) { return bf16_val(w[i]); }
template <> __device__ __forceinline__ float wval<float>(const float* w, int64_t i) { return w[i]; }

// ---------------------------------------------------------------- dense layer
// C(i, j) = act( sum_k A(i,k) W(k,j) + b(j) ) * [mask(i,j) > 0] (+ C(i,j) if accumulate)
// A: n x K FP32 row-major (lda); W(k, j) = W[k*wsk + j*wsj]; b: N or null.
// Workgroup: 256 threads = 4 waves in a 2 x 2 grid of 32 x 32 MFMA tiles
// (64 rows x 64 columns); the summation runs in chunks of KC through LDS.
template <typename WT>
struct DenseArgs {
  int64_t n; int K, N;
  const float* A; int64_t lda;
  const WT* W; int64_t wsk, wsj;
  const WT* bias;
  const float* mask; int64_t ldm;
  float* C; int64_t ldc;
  int relu, accumulate;
};

template <typename WT, int KC>
__global__ __launch_bounds__(256) void k_dense(DenseArgs<WT> a) {
  __shared__ float As[64][KC + 1];
  __shared__ float Bs[KC][64 + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  const int col0 = blockIdx.y * 64;
  floatx16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int k0 = 0; k0 < a.K; k0 += KC) {
    for (int e = tid; e < 64 * KC; e += 256) {
      int r = e / KC, kk = e % KC;
      int64_t gi = row0 + r;
      int gk = k0 + kk;
      As[r][kk] = (gi < a.n && gk < a.K) ? a.A[gi * a.lda + gk] : 0.f;
    }
    for (int e = tid; e < 64 * KC; e += 256) {
      int kk = e / 64, j = e % 64;
      int gk = k0 + kk, gj = col0 + j;
      Bs[kk][j] = (gk < a.K && gj < a.N) ? wval<WT>(a.W, (int64_t)gk * a.wsk + (int64_t)gj * a.wsj) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC; kk += 2) {
      float av = As[wr * 32 + (lane & 31)][kk + (lane >> 5)];
      float bv = Bs[kk + (lane >> 5)][wc * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int gj = col0 + wc * 32 + (lane & 31);
  if (gj >= a.N) return;
  const float bj = a.bias ? wval<WT>(a.bias, gj) : 0.f;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    int64_t gi = row0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (gi >= a.n) continue;
    float v = acc[r] + bj;
    if (a.relu) v = fmaxf(v, 0.f);
    if (a.mask && !(a.mask[gi * a.ldm + gj] > 0.f)) v = 0.f;
    float* dst = a.C + gi * a.ldc + gj;
    if (a.accumulate) v += *dst;
    *dst = v;
  }
}

// Wide variant for the inference shapes: W is BF16 row-major (W(k, j) =
// W[k*ldw + j]), N <= 256 with N % 8 == 0, K % 16 == 0, lda % 4 == 0.  A
// workgroup of 512 threads owns 128 rows and all N columns, so each row of A
// is read from HBM once; wave w computes rows 32(w&3).. x columns
// 128(w>>2).. (four 32 x 32 tiles).  The summation runs in chunks of 16
// through double-buffered LDS, the next chunk prefetched into registers.
struct WideArgs {
  int64_t n; int K, N;
  const float* A; int64_t lda;
  const uint16_t* W; int64_t ldw;
  const uint16_t* bias;
  float* C; int64_t ldc;
  int relu;
};

constexpr int WKC = 16;

__global__ __launch_bounds__(512) void k_dense_wide(WideArgs a) {
  __shared__ float As[2][128][WKC + 1];
  __shared__ float Bs[2][WKC][256 + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rt = wave & 3, cg = wave >> 2;
  const int64_t row0 = (int64_t)blockIdx.x * 128;
  // loader roles: A -- one float4 per thread (128 rows x 4 float4);
  //               W -- one 8 x BF16 vector per thread (16 rows x 32 vectors)
  const int ar = tid >> 2, ac = (tid & 3) * 4;
  const int64_t agi = row0 + ar;
  const int wk = tid >> 5, wj = (tid & 31) * 8;
  const bool a_ok = agi < a.n;
  const bool w_ok = wj < a.N;
  floatx16 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;
  float4 ra = make_float4(0.f, 0.f, 0.f, 0.f);
  uint4 rw = make_uint4(0u, 0u, 0u, 0u);
  auto fetch = [&](int k0) {
    ra = a_ok ? *reinterpret_cast<const float4*>(a.A + agi * a.lda + k0 + ac) : make_float4(0.f, 0.f, 0.f, 0.f);
    rw = w_ok ? *reinterpret_cast<const uint4*>(a.W + (int64_t)(k0 + wk) * a.ldw + wj) : make_uint4(0u, 0u, 0u, 0u);
  };
  auto stash = [&](int buf) {
    As[buf][ar][ac + 0] = ra.x;
    As[buf][ar][ac + 1] = ra.y;
    As[buf][ar][ac + 2] = ra.z;
    As[buf][ar][ac + 3] = ra.w;
    const uint32_t wv[4] = {rw.x, rw.y, rw.z, rw.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      Bs[buf][wk][wj + 2 * q] = __uint_as_float(wv[q] << 16);
      Bs[buf][wk][wj + 2 * q + 1] = __uint_as_float(wv[q] & 0xffff0000u);
    }
  };
  const int nchunk = a.K / WKC;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) fetch((ch + 1) * WKC);
#pragma unroll
    for (int kk = 0; kk < WKC; kk += 2) {
      const float av = As[buf][rt * 32 + (lane & 31)][kk + (lane >> 5)];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float bv = Bs[buf][kk + (lane >> 5)][cg * 128 + t * 32 + (lane & 31)];
        acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc[t], 0, 0, 0);
      }
    }
    if (ch + 1 < nchunk) stash(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int gj = cg * 128 + t * 32 + (lane & 31);
    if (gj >= a.N) continue;
    const float bj = a.bias ? bf16_val(a.bias[gj]) : 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t gi = row0 + rt * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (gi >= a.n) continue;
      float v = acc[t][r] + bj;
      if (a.relu) v = fmaxf(v, 0.f);
      a.C[gi * a.ldc + gj] = v;
    }
  }
}

// ---------------------------------------------------------------- inference pass in BF16
// The start block only seeds the power iteration, so inference may round the
// hidden activations to BF16 and run layers 2 and 3 on the BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16, FP32 accumulation):
//   H1 = bf16(relu(phi W1 + b1)),  H2 = bf16(relu(H1 W2 + b2)),  F = H2 W3 + b3.
// Width 256, out a multiple of 32 up to 256.  Persistent workgroups of 512
// threads walk blocks of 128 rows.  Wave w keeps the MFMA B fragments of
// column tile w of W2 and W3 (packed once per call by k_pack_wfrag) in
// registers for the whole launch, so no weight moves after the start.  Per
// row block: layer 1 on the vector ALU, H1 and then H2 in LDS (BF16, rows
// padded by 8 elements), each wave multiplying all four 32-row tiles of H by
// its column tile; nothing but F is written to memory.
constexpr int IW = 256;          // hidden width of the BF16 inference kernel
constexpr int IROWS = 128;       // rows per row block
constexpr int IHS = IW + 8;      // LDS row stride of H (BF16 elements)
constexpr int IPERSIST = 256;    // persistent workgroups (one per CU of the MI355X)

typedef __bf16 ibf16x8 __attribute__((ext_vector_type(8)));

// W (K x N, row-major BF16, K = 256, N <= 256, N % 32 == 0) -> fragments
// out[((ks * 8) + jt) * 64 + lane] = W[16ks + 8(lane/32) + e][32jt + lane%32], e < 8
// (zero for jt >= N/32)
__global__ void k_pack_wfrag(int N, const uint16_t* __restrict__ W, uint4* __restrict__ out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // (ks, jt, lane)
  if (idx >= 16 * 8 * 64) return;
  const int lane = idx & 63, jt = (idx >> 6) & 7, ks = idx >> 9;
  const int j = 32 * jt + (lane & 31);
  const int k0 = 16 * ks + 8 * (lane >> 5);
  uint16_t v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) v[e] = j < N ? W[(int64_t)(k0 + e) * N + j] : (uint16_t)0;
  out[idx] = make_uint4(v[0] | ((uint32_t)v[1] << 16), v[2] | ((uint32_t)v[3] << 16), v[4] | ((uint32_t)v[5] << 16),
                        v[6] | ((uint32_t)v[7] << 16));
}

struct InferArgs {
  int64_t n; int out;
  const float* phi;            // n x FEAT
  const uint16_t* W1;          // FEAT x IW
  const uint16_t* b1;          // IW
  const uint4* W2f;            // packed fragments of W2 (IW x IW)
  const uint16_t* b2;          // IW
  const uint4* W3f;            // packed fragments of W3 (IW x out)
  const uint16_t* b3;          // out
  float* F; int64_t ldf;
};

__global__ __launch_bounds__(512, 1) void k_mlp_infer(InferArgs a) {
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  uint16_t* Hs = reinterpret_cast<uint16_t*>(lds_raw);                     // IROWS x IHS
  float* W1s = reinterpret_cast<float*>(lds_raw + (size_t)IROWS * IHS * 2);  // FEAT x IW
  float* b1s = W1s + FEAT * IW;                                             // IW
  const int tid = threadIdx.x, lane = tid & 63;
  const int ct = __builtin_amdgcn_readfirstlane(tid >> 6);  // this wave's 32-column tile
  for (int i = tid; i < FEAT * IW; i += 512) W1s[i] = bf16_val(a.W1[i]);
  for (int i = tid; i < IW; i += 512) b1s[i] = bf16_val(a.b1[i]);
  // the B fragments of column tile ct of W2 and W3, all 16 k-steps, stay in
  // registers for every row block of the workgroup
  ibf16x8 w2[16], w3[16];
  const ibf16x8* W2f = reinterpret_cast<const ibf16x8*>(a.W2f);
  const ibf16x8* W3f = reinterpret_cast<const ibf16x8*>(a.W3f);
#pragma unroll
  for (int ks = 0; ks < 16; ++ks) {
    w2[ks] = W2f[(ks * 8 + ct) * 64 + lane];
    w3[ks] = W3f[(ks * 8 + ct) * 64 + lane];
  }
  const int col = 32 * ct + (lane & 31);
  const bool has3 = 32 * ct < a.out;
  const float bias2 = bf16_val(a.b2[col]);
  const float bias3 = has3 ? bf16_val(a.b3[col]) : 0.f;
  const int64_t nblocks = (a.n + IROWS - 1) / IROWS;
  floatx16 acc[4];
  // one wavefront's product of the four 32-row tiles of Hs with its column
  // tile, k-steps in order
  auto layer = [&](const ibf16x8 (&w)[16]) {
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
      floatx16 c = {};
#pragma unroll
      for (int ks = 0; ks < 16; ++ks) {
        const ibf16x8 av = *reinterpret_cast<const ibf16x8*>(Hs + (32 * rt + (lane & 31)) * IHS + 16 * ks +
                                                              8 * (lane >> 5));
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, w[ks], c, 0, 0, 0);
      }
      acc[rt] = c;
    }
  };
  for (int64_t blk = blockIdx.x; blk < nblocks; blk += gridDim.x) {
    const int64_t row0 = blk * IROWS;
    __syncthreads();  // Hs is free (and W1s, b1s are written on the first pass)
    // layer 1 (vector ALU): thread -> row tid/4, columns 64*(tid%4) .. +63
    {
      const int r = tid >> 2, c0 = (tid & 3) * 64;
      const int64_t gr = row0 + r;
      float x[FEAT];
#pragma unroll
      for (int f = 0; f < FEAT; ++f) x[f] = gr < a.n ? a.phi[gr * FEAT + f] : 0.f;
      for (int c = c0; c < c0 + 64; c += 2) {
        float v0 = b1s[c], v1 = b1s[c + 1];
#pragma unroll
        for (int f = 0; f < FEAT; ++f) {
          v0 = fmaf(x[f], W1s[f * IW + c], v0);
          v1 = fmaf(x[f], W1s[f * IW + c + 1], v1);
        }
        const uint32_t pk = (uint32_t)bf16_rne(fmaxf(v0, 0.f)) | ((uint32_t)bf16_rne(fmaxf(v1, 0.f)) << 16);
        *reinterpret_cast<uint32_t*>(Hs + r * IHS + c) = pk;
      }
    }
    __syncthreads();  // H1 complete
    layer(w2);
    __syncthreads();  // every wave has finished reading H1
    // H2 = bf16(relu(acc + b2)) over H1
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = 32 * rt + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
        Hs[row * IHS + col] = bf16_rne(fmaxf(acc[rt][e] + bias2, 0.f));
      }
    __syncthreads();  // H2 complete
    if (has3) {
      layer(w3);
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int64_t row = row0 + 32 * rt + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
          if (row < a.n) a.F[row * a.ldf + col] = acc[rt][e] + bias3;
        }
    }
  }
}

// ---------------------------------------------------------------- A^T B over row ranges
// part[p](i, j) = sum_{r in range p} A(r, i) B(r, j), i < K1, j < K2.
// Grid: (ceil(K1/64) * ceil(K2/64), parts).  Rows run in chunks of 32 via LDS.
struct GramArgs32 {
  int64_t n; int K1, K2; int64_t rows_per_part;
  const float* A; int64_t lda;
  const float* B; int64_t ldb;
  float* part;  // parts x K1 x K2
};

__global__ __launch_bounds__(256) void k_gram32(GramArgs32 g) {
  __shared__ float As[32][64 + 4];
  __shared__ float Bs[32][64 + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int tj = (g.K2 + 63) / 64;
  const int i0 = (blockIdx.x / tj) * 64, j0 = (blockIdx.x % tj) * 64;
  const int64_t rb = (int64_t)blockIdx.y * g.rows_per_part;
  const int64_t re = min(g.n, rb + g.rows_per_part);
  floatx16 acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int64_t r0 = rb; r0 < re; r0 += 32) {
    for (int e = tid; e < 32 * 64; e += 256) {
      int r = e / 64, c = e % 64;
      int64_t gr = r0 + r;
      bool ok = gr < re;
      As[r][c] = (ok && i0 + c < g.K1) ? g.A[gr * g.lda + i0 + c] : 0.f;
      Bs[r][c] = (ok && j0 + c < g.K2) ? g.B[gr * g.ldb + j0 + c] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 32; kk += 2) {
      float av = As[kk + (lane >> 5)][wr * 32 + (lane & 31)];
      float bv = Bs[kk + (lane >> 5)][wc * 32 + (lane & 31)];
      acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  const int j = j0 + wc * 32 + (lane & 31);
  if (j >= g.K2) return;
  float* out = g.part + (int64_t)blockIdx.y * g.K1 * g.K2;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    int i = i0 + wr * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (i < g.K1) out[(int64_t)i * g.K2 + j] = acc[r];
  }
}

// out[e] = sum_p part[p][e], p in order
__global__ void k_sum_parts(int64_t count, int parts, const float* __restrict__ part, float* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float s = 0.f;
  for (int p = 0; p < parts; ++p) s += part[(int64_t)p * count + e];
  out[e] = s;
}

// part[p][j] = sum_{r in range p} A(r, j)
__global__ void k_colsum_part(int64_t n, int N, int64_t rows_per_part, const float* __restrict__ A, int64_t lda,
                              float* __restrict__ part) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  int64_t rb = (int64_t)blockIdx.y * rows_per_part, re = min(n, rb + rows_per_part);
  float s = 0.f;
  for (int64_t r = rb; r < re; ++r) s += A[r * lda + j];
  part[(int64_t)blockIdx.y * N + j] = s;
}

// ---------------------------------------------------------------- loss and dL/dF coefficients
// One workgroup.  P = U^T F, G = F^T F (k x k FP32).  Writes the loss and the
// k x k matrices Acoef, Bcoef with dL/dF = U Acoef + F Bcoef.
__device__ double block_sum(double v, double* red) {
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (tid == 0) {
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    red[16] = s;
  }
  __syncthreads();
  s = red[16];
  __syncthreads();
  return s;
}

__global__ __launch_bounds__(1024) void k_ws_loss(int k, float mu, const float* __restrict__ P,
                                                  const float* __restrict__ G, float* __restrict__ Acoef,
                                                  float* __restrict__ Bcoef, float* __restrict__ loss) {
  __shared__ double red[17];
  const int tid = threadIdx.x;
  const int64_t kk = (int64_t)k * k;
  double tr = 0.0, pp = 0.0;
  for (int64_t e = tid; e < kk; e += blockDim.x) {
    double p = P[e];
    pp += p * p;
    if (e / k == e % k) tr += G[e];
  }
  const double s = block_sum(tr, red);
  pp = block_sum(pp, red);
  double mm = 0.0, mg = 0.0;
  for (int64_t e = tid; e < kk; e += blockDim.x) {
    double g = G[e];
    double m = (double)k / s * g - (e / k == e % k ? 1.0 : 0.0);
    mm += m * m;
    mg += m * g;
  }
  mm = block_sum(mm, red);
  mg = block_sum(mg, red);
  const double cm = 4.0 * mu * k / s;
  const double cdiag = 2.0 * pp / (s * s) - 4.0 * mu * k * mg / (s * s);
  for (int64_t e = tid; e < kk; e += blockDim.x) {
    bool diag = e / k == e % k;
    double m = (double)k / s * G[e] - (diag ? 1.0 : 0.0);
    Acoef[e] = (float)(-2.0 / s * P[e]);
    Bcoef[e] = (float)(cm * m + (diag ? cdiag : 0.0));
  }
  if (tid == 0) *loss = (float)(1.0 - pp / s + mu * mm);
}

// ---------------------------------------------------------------- Adam and parameter set-up
// b1, b2 and their complements om1 = 1 - b1, om2 = 1 - b2 are rounded to FP32
// from exact values on the host (1 - 0.999f is not 0.001 to FP32 accuracy);
// c1 = 1 - b1^step, c2 = 1 - b2^step likewise.
__global__ void k_adam(int64_t count, float lr, float b1, float b2, float om1, float om2, float eps, float c1,
                       float c2, const float* __restrict__ g, float* __restrict__ w, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ wb) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float ge = g[e];
  float me = b1 * m[e] + om1 * ge;
  float ve = b2 * v[e] + om2 * ge * ge;
  m[e] = me;
  v[e] = ve;
  float we = w[e] - lr * (me / c1) / (sqrtf(ve / c2) + eps);
  w[e] = we;
  wb[e] = bf16_rne(we);
}

// master[e] *= scale for e in [0, count) ; zero rows / biases handled by k_fill
__global__ void k_scale_f(int64_t count, float scale, float* __restrict__ x) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) x[e] *= scale;
}
__global__ void k_fill_f(int64_t count, float val, float* __restrict__ x) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) x[e] = val;
}
__global__ void k_to_bf16(int64_t count, const float* __restrict__ x, uint16_t* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) out[e] = bf16_rne(x[e]);
}

// ---------------------------------------------------------------- features
// raw(i, 0) = log max(deg_i, 1); T0 = [g, 0, 0, 0] (n x 4)
// raw column 0 = log max(deg, 1); T0 = the probe block G (n x 4)
__global__ void k_feat_seed(int64_t n, const int64_t* __restrict__ rowptr, const float* __restrict__ g,
                            float* __restrict__ raw, float* __restrict__ T0) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double deg = (double)(rowptr[i + 1] - rowptr[i]);
  raw[i * FEAT] = (float)log(deg > 1.0 ? deg : 1.0);
  for (int j = 0; j < 4; ++j) T0[i * 4 + j] = g[i * 4 + j];
}
// raw columns col0 .. col0 + ncols - 1 = the first ncols columns of T (n x 4)
__global__ void k_feat_take(int64_t n, int col0, int ncols, const float* __restrict__ T, float* __restrict__ raw) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int j = 0; j < ncols; ++j) raw[i * FEAT + col0 + j] = T[i * 4 + j];
}
// Column moments of the raw features in two passes over fixed row ranges
// (FP64, fixed order): pass 0 sums x, pass 1 sums (x - mean)^2 and x^2.
// part[(b * SKETCHNE_WS_RAW + j) * 2 + {0, 1}] for block b.
constexpr int FS_BLOCKS = 256;
__global__ __launch_bounds__(256) void k_feat_moments(int64_t n, int pass, const float* __restrict__ raw,
                                                      const double* __restrict__ stat, double* __restrict__ part) {
  __shared__ double red[2][SKETCHNE_WS_RAW][256];
  const int64_t per = (n + FS_BLOCKS - 1) / FS_BLOCKS;
  const int64_t rb = (int64_t)blockIdx.x * per, re = min(n, rb + per);
  double a[SKETCHNE_WS_RAW], b[SKETCHNE_WS_RAW];
  for (int j = 0; j < SKETCHNE_WS_RAW; ++j) a[j] = b[j] = 0.0;
  for (int64_t i = rb + threadIdx.x; i < re; i += 256) {
    for (int j = 0; j < SKETCHNE_WS_RAW; ++j) {
      double x = raw[i * FEAT + j];
      if (pass == 0) {
        a[j] += x;
      } else {
        double d = x - stat[2 * j];
        a[j] += d * d;
        b[j] += x * x;
      }
    }
  }
  for (int j = 0; j < SKETCHNE_WS_RAW; ++j) {
    red[0][j][threadIdx.x] = a[j];
    red[1][j][threadIdx.x] = b[j];
  }
  __syncthreads();
  if (threadIdx.x < 2 * SKETCHNE_WS_RAW) {
    const int which = threadIdx.x / SKETCHNE_WS_RAW, j = threadIdx.x % SKETCHNE_WS_RAW;
    double s = 0.0;
    for (int t = 0; t < 256; ++t) s += red[which][j][t];
    part[((int64_t)blockIdx.x * SKETCHNE_WS_RAW + j) * 2 + which] = s;
  }
}
// stat[2j] = mean, stat[2j+1] = 1/std, or 0 when the column has no spread
__global__ void k_feat_finish(int64_t n, int pass, const double* __restrict__ part, double* __restrict__ stat) {
  const int j = threadIdx.x;
  if (j >= SKETCHNE_WS_RAW) return;
  double s0 = 0.0, s1 = 0.0;
  for (int b = 0; b < FS_BLOCKS; ++b) {
    s0 += part[((int64_t)b * SKETCHNE_WS_RAW + j) * 2 + 0];
    s1 += part[((int64_t)b * SKETCHNE_WS_RAW + j) * 2 + 1];
  }
  if (pass == 0) {
    stat[2 * j] = s0 / (double)n;
  } else {
    const double sd = sqrt(s0 / (double)n), rms = sqrt(s1 / (double)n);
    stat[2 * j + 1] = sd > 1e-6 * rms ? 1.0 / sd : 0.0;
  }
}
__global__ void k_feat_apply(int64_t n, int nraw, const double* __restrict__ stat, float* __restrict__ phi) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * FEAT) return;
  int j = (int)(e % FEAT);
  float v = 0.f;
  if (j < nraw && stat[2 * j + 1] != 0.0) v = (float)(((double)phi[e] - stat[2 * j]) * stat[2 * j + 1]);
  phi[e] = v;
}

// ---------------------------------------------------------------- Ritz residuals
// part[p][j] = sum_{r in range p} (XU(r,j) - lambda_j U(r,j))^2   (FP64)
// Block (x, y): columns 64x .. 64x+63, rows of part y; the 256 threads split
// the part's rows four ways and combine in LDS in a fixed order.
__global__ __launch_bounds__(256) void k_resid_part(int64_t n, int k, int64_t rows_per_part,
                                                    const float* __restrict__ XU, const float* __restrict__ U,
                                                    const double* __restrict__ lambda, double* __restrict__ part) {
  __shared__ double red[4][64];
  const int c = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + c;
  const int64_t rb = (int64_t)blockIdx.y * rows_per_part, re = min(n, rb + rows_per_part);
  double s = 0.0;
  if (j < k) {
    const double lj = lambda[j];
    for (int64_t r = rb + q; r < re; r += 4) {
      double d = (double)XU[r * k + j] - lj * (double)U[r * k + j];
      s += d * d;
    }
  }
  red[q][c] = s;
  __syncthreads();
  if (q == 0 && j < k) part[(int64_t)blockIdx.y * k + j] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
}
__global__ void k_resid_final(int k, int parts, const double* __restrict__ part, double* __restrict__ res) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double s = 0.0;
  for (int p = 0; p < parts; ++p) s += part[(int64_t)p * k + j];
  res[j] = sqrt(s);
}

inline unsigned nblk(int64_t count, int t = 256) { return (unsigned)((count + t - 1) / t); }

}  // namespace

// ---------------------------------------------------------------- launchers
int64_t ws_param_count(int width, int out) {
  return (int64_t)FEAT * width + width + (int64_t)width * width + width + (int64_t)width * out + out;
}

namespace {
struct Off { int64_t W1, b1, W2, b2, W3, b3; };
Off offsets(int w, int o) {
  Off f;
  f.W1 = 0;
  f.b1 = f.W1 + (int64_t)FEAT * w;
  f.W2 = f.b1 + w;
  f.b2 = f.W2 + (int64_t)w * w;
  f.W3 = f.b2 + w;
  f.b3 = f.W3 + (int64_t)w * o;
  return f;
}

int64_t resid_parts(int64_t n) {
  int64_t parts = (n + 511) / 512;
  return parts < 1 ? 1 : (parts > 1024 ? 1024 : parts);
}

int64_t parts_for(int64_t n) {
  int64_t parts = (n + 2047) / 2048;
  return parts < 1 ? 1 : (parts > 128 ? 128 : parts);
}

template <typename WT>
sketchne_status dense(sketchne_ctx* c, int64_t n, int K, int N, const float* A, int64_t lda, const WT* W, int64_t wsk,
                      int64_t wsj, const WT* bias, const float* mask, int64_t ldm, float* C, int64_t ldc, bool relu,
                      bool accumulate) {
  if (n == 0) return SKETCHNE_OK;
  if constexpr (std::is_same<WT, uint16_t>::value) {
    // the wide kernel covers the forward shapes (row-major BF16 weights, no mask)
    if (!mask && !accumulate && wsj == 1 && N <= 256 && N % 8 == 0 && K % WKC == 0 && lda % 4 == 0 && wsk % 8 == 0 &&
        reinterpret_cast<uintptr_t>(A) % 16 == 0 && reinterpret_cast<uintptr_t>(W) % 16 == 0) {
      WideArgs w{n, K, N, A, lda, W, wsk, bias, C, ldc, relu ? 1 : 0};
      hipLaunchKernelGGL(k_dense_wide, dim3((unsigned)((n + 127) / 128)), dim3(512), 0, c->stream, w);
      return launch_status();
    }
  }
  DenseArgs<WT> a{n, K, N, A, lda, W, wsk, wsj, bias, mask, ldm, C, ldc, relu ? 1 : 0, accumulate ? 1 : 0};
  dim3 grid((unsigned)((n + 63) / 64), (unsigned)((N + 63) / 64));
  if (K <= 8)
    hipLaunchKernelGGL((k_dense<WT, 8>), grid, dim3(256), 0, c->stream, a);
  else
    hipLaunchKernelGGL((k_dense<WT, 32>), grid, dim3(256), 0, c->stream, a);
  return launch_status();
}

// C (K1 x K2) = A^T B over all n rows; part: parts_for(n) * K1 * K2 floats
sketchne_status gram32(sketchne_ctx* c, int64_t n, int K1, int K2, const float* A, int64_t lda, const float* B,
                       int64_t ldb, float* part, float* C) {
  int64_t parts = parts_for(n);
  int64_t rpp = (n + parts - 1) / parts;
  rpp = (rpp + 31) / 32 * 32;
  parts = (n + rpp - 1) / rpp;
  if (parts < 1) parts = 1;
  GramArgs32 g{n, K1, K2, rpp, A, lda, B, ldb, part};
  dim3 grid((unsigned)(((K1 + 63) / 64) * ((K2 + 63) / 64)), (unsigned)parts);
  hipLaunchKernelGGL(k_gram32, grid, dim3(256), 0, c->stream, g);
  int64_t cnt = (int64_t)K1 * K2;
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(cnt)), dim3(256), 0, c->stream, cnt, (int)parts, part, C);
  return launch_status();
}

sketchne_status colsum(sketchne_ctx* c, int64_t n, int N, const float* A, int64_t lda, float* part, float* out) {
  int64_t parts = parts_for(n);
  int64_t rpp = (n + parts - 1) / parts;
  parts = (n + rpp - 1) / rpp;
  if (parts < 1) parts = 1;
  hipLaunchKernelGGL(k_colsum_part, dim3(nblk(N), (unsigned)parts), dim3(256), 0, c->stream, n, N, rpp, A, lda, part);
  hipLaunchKernelGGL(k_sum_parts, dim3(nblk(N)), dim3(256), 0, c->stream, (int64_t)N, (int)parts, part, out);
  return launch_status();
}
}  // namespace

size_t ws_part_floats(int64_t n, int width, int out) {
  int64_t m = width > out ? width : out;
  return (size_t)parts_for(n) * (size_t)(m * m > FEAT * m ? m * m : FEAT * m);
}

size_t ws_forward_bytes(int64_t n, int width) {
  return 2 * align_up(sizeof(float) * (size_t)n * width);
}

size_t ws_grad_bytes(int64_t n, int width, int out) {
  size_t b = 0;
  b += 2 * align_up(sizeof(float) * (size_t)n * width);   // H1, H2
  b += 2 * align_up(sizeof(float) * (size_t)n * out);     // F, dF
  b += 2 * align_up(sizeof(float) * (size_t)n * width);   // dZ2, dZ1
  b += align_up(sizeof(float) * ws_part_floats(n, width, out));
  b += 4 * align_up(sizeof(float) * (size_t)out * out);   // P, G, Acoef, Bcoef
  return b;
}

size_t ws_features_bytes(int64_t n, int64_t nnz) {
  return 2 * align_up(sizeof(float) * (size_t)n * 4) + align_up(sizeof(float) * (size_t)n * SKETCHNE_WS_PROBES) +
         align_up(sizeof(double) * 2 * FEAT) + align_up(sizeof(double) * FS_BLOCKS * SKETCHNE_WS_RAW * 2) +
         align_up(sizeof(float) * (size_t)n) + spmm_ws_bytes(nnz, 4);
}

size_t ritz_residual_bytes(int64_t n, int64_t nnz, int k) {
  return align_up(sizeof(float) * (size_t)n * k) + align_up(sizeof(float) * (size_t)n) +
         align_up(sizeof(double) * (size_t)resid_parts(n) * k) + spmm_ws_bytes(nnz, k);
}

sketchne_status ws_init(sketchne_ctx* c, const sketchne_mlp* net, uint64_t seed) {
  const int w = net->width, o = net->out;
  const Off f = offsets(w, o);
  const int64_t total = ws_param_count(w, o);
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  // He initialisation: N(0, 2 / fan_in); the padded rows of W1 start at 0
  SK_TRY(gen_gauss(c, SKETCHNE_WS_RAW, w, w, seed ^ 0x1111, net->master + f.W1));
  SK_TRY(gen_gauss(c, w, w, w, seed ^ 0x2222, net->master + f.W2));
  SK_TRY(gen_gauss(c, w, o, o, seed ^ 0x3333, net->master + f.W3));
  hipLaunchKernelGGL(k_scale_f, dim3(nblk((int64_t)SKETCHNE_WS_RAW * w)), dim3(256), 0, c->stream,
                     (int64_t)SKETCHNE_WS_RAW * w, sqrtf(2.f / SKETCHNE_WS_RAW), net->master + f.W1);
  if (FEAT > SKETCHNE_WS_RAW)
    hipLaunchKernelGGL(k_fill_f, dim3(nblk((int64_t)(FEAT - SKETCHNE_WS_RAW) * w)), dim3(256), 0, c->stream,
                       (int64_t)(FEAT - SKETCHNE_WS_RAW) * w, 0.f, net->master + f.W1 + (int64_t)SKETCHNE_WS_RAW * w);
  hipLaunchKernelGGL(k_scale_f, dim3(nblk((int64_t)w * w)), dim3(256), 0, c->stream, (int64_t)w * w,
                     sqrtf(2.f / w), net->master + f.W2);
  hipLaunchKernelGGL(k_scale_f, dim3(nblk((int64_t)w * o)), dim3(256), 0, c->stream, (int64_t)w * o,
                     sqrtf(2.f / w), net->master + f.W3);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(w)), dim3(256), 0, c->stream, (int64_t)w, 0.f, net->master + f.b1);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(w)), dim3(256), 0, c->stream, (int64_t)w, 0.f, net->master + f.b2);
  hipLaunchKernelGGL(k_fill_f, dim3(nblk(o)), dim3(256), 0, c->stream, (int64_t)o, 0.f, net->master + f.b3);
  if (net->adam_m)
    hipLaunchKernelGGL(k_fill_f, dim3(nblk(total)), dim3(256), 0, c->stream, total, 0.f, net->adam_m);
  if (net->adam_v)
    hipLaunchKernelGGL(k_fill_f, dim3(nblk(total)), dim3(256), 0, c->stream, total, 0.f, net->adam_v);
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(total)), dim3(256), 0, c->stream, total, net->master, net->bf16);
  return launch_status();
}

sketchne_status ws_features(sketchne_ctx* c, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colidx,
                            double alpha, const float* g, uint64_t seed, float* phi, void* ws, size_t ws_bytes) {
  Arena ar(ws, ws_bytes);
  float* T0 = ar.take<float>((size_t)n * 4);
  float* T1 = ar.take<float>((size_t)n * 4);
  float* gdraw = ar.take<float>((size_t)n * SKETCHNE_WS_PROBES);
  double* stat = ar.take<double>(2 * FEAT);
  double* mom = ar.take<double>((size_t)FS_BLOCKS * SKETCHNE_WS_RAW * 2);
  float* dscale = ar.take<float>((size_t)n);
  float* part = ar.take<float>(spmm_ws_bytes(nnz, 4) / sizeof(float));
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  if (!g) {
    SK_TRY(gen_rademacher(c, n * SKETCHNE_WS_PROBES, seed, gdraw));
    g = gdraw;
  }
  SK_TRY(degree_scale(c, n, rowptr, alpha, dscale));
  hipLaunchKernelGGL(k_feat_seed, dim3(nblk(n)), dim3(256), 0, c->stream, n, rowptr, g, phi, T0);
  SK_TRY(launch_status());
  float* src = T0;
  float* dst = T1;
  // X^t G for t = 1 .. 4; X^3 G fills raw columns 1-4, X^4 G columns 5-7
  static_assert(SKETCHNE_WS_PROBES == 4 && SKETCHNE_WS_RAW == 8, "feature layout");
  for (int t = 1; t <= 4; ++t) {
    SK_TRY(spmm(c, n, nnz, rowptr, colidx, dscale, src, 4, 4, dst, 4, part));
    if (t == 3)
      hipLaunchKernelGGL(k_feat_take, dim3(nblk(n)), dim3(256), 0, c->stream, n, 1, 4, dst, phi);
    else if (t == 4)
      hipLaunchKernelGGL(k_feat_take, dim3(nblk(n)), dim3(256), 0, c->stream, n, 5, 3, dst, phi);
    float* tmp = src;
    src = dst;
    dst = tmp;
  }
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(k_feat_moments, dim3(FS_BLOCKS), dim3(256), 0, c->stream, n, pass, phi, stat, mom);
    hipLaunchKernelGGL(k_feat_finish, dim3(1), dim3(64), 0, c->stream, n, pass, mom, stat);
  }
  hipLaunchKernelGGL(k_feat_apply, dim3(nblk(n * FEAT)), dim3(256), 0, c->stream, n, (int)SKETCHNE_WS_RAW, stat,
                     phi);
  return launch_status();
}

sketchne_status ws_forward(sketchne_ctx* c, const sketchne_mlp* net, int64_t n, const float* phi, float* F,
                           int64_t ldf, void* ws, size_t ws_bytes) {
  const int w = net->width, o = net->out;
  const Off f = offsets(w, o);
  Arena ar(ws, ws_bytes);
  float* H1 = ar.take<float>((size_t)n * w);
  float* H2 = ar.take<float>((size_t)n * w);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  const uint16_t* Wb = net->bf16;
  SK_TRY(dense<uint16_t>(c, n, FEAT, w, phi, FEAT, Wb + f.W1, w, 1, Wb + f.b1, nullptr, 0, H1, w, true, false));
  SK_TRY(dense<uint16_t>(c, n, w, w, H1, w, Wb + f.W2, w, 1, Wb + f.b2, nullptr, 0, H2, w, true, false));
  return dense<uint16_t>(c, n, w, o, H2, w, Wb + f.W3, o, 1, Wb + f.b3, nullptr, 0, F, ldf, false, false);
}

bool ws_infer_supported(const sketchne_mlp* net) {
  return net->width == IW && net->out >= 32 && net->out <= IW && net->out % 32 == 0;
}

size_t ws_infer_bytes() { return 2 * align_up((size_t)16 * 8 * 64 * 16); }

sketchne_status ws_infer(sketchne_ctx* c, const sketchne_mlp* net, int64_t n, const float* phi, float* F, int64_t ldf,
                         void* ws, size_t ws_bytes) {
  if (!ws_infer_supported(net)) return SKETCHNE_E_UNSUPPORTED;
  const int w = net->width, o = net->out;
  const Off f = offsets(w, o);
  Arena ar(ws, ws_bytes);
  uint4* W2f = ar.take<uint4>(16 * 8 * 64);
  uint4* W3f = ar.take<uint4>(16 * 8 * 64);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  if (n == 0) return SKETCHNE_OK;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  const uint16_t* Wb = net->bf16;
  hipLaunchKernelGGL(k_pack_wfrag, dim3(32), dim3(256), 0, c->stream, w, Wb + f.W2, W2f);
  hipLaunchKernelGGL(k_pack_wfrag, dim3(32), dim3(256), 0, c->stream, o, Wb + f.W3, W3f);
  InferArgs a;
  a.n = n; a.out = o; a.phi = phi;
  a.W1 = Wb + f.W1; a.b1 = Wb + f.b1;
  a.W2f = W2f; a.b2 = Wb + f.b2;
  a.W3f = W3f; a.b3 = Wb + f.b3;
  a.F = F; a.ldf = ldf;
  const size_t shmem = (size_t)IROWS * IHS * 2 + sizeof(float) * (size_t)(FEAT + 1) * IW;
  hipFuncSetAttribute(reinterpret_cast<const void*>(k_mlp_infer), hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shmem);
  // persistent workgroups, one per CU: each loads the weights once and walks
  // row blocks blockIdx.x, blockIdx.x + gridDim.x, ...
  const int64_t nblocks = (n + IROWS - 1) / IROWS;
  const unsigned grid = (unsigned)(nblocks < IPERSIST ? nblocks : IPERSIST);
  hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(512), shmem, c->stream, a);
  return launch_status();
}

sketchne_status ws_grad(sketchne_ctx* c, const sketchne_mlp* net, int64_t n, const float* phi, const float* U,
                        int64_t ldu, float mu, float* grad, float* loss, void* ws, size_t ws_bytes) {
  const int w = net->width, o = net->out;
  const Off f = offsets(w, o);
  Arena ar(ws, ws_bytes);
  float* H1 = ar.take<float>((size_t)n * w);
  float* H2 = ar.take<float>((size_t)n * w);
  float* F = ar.take<float>((size_t)n * o);
  float* dF = ar.take<float>((size_t)n * o);
  float* dZ2 = ar.take<float>((size_t)n * w);
  float* dZ1 = ar.take<float>((size_t)n * w);
  float* part = ar.take<float>(ws_part_floats(n, w, o));
  float* P = ar.take<float>((size_t)o * o);
  float* G = ar.take<float>((size_t)o * o);
  float* Ac = ar.take<float>((size_t)o * o);
  float* Bc = ar.take<float>((size_t)o * o);
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  const uint16_t* Wb = net->bf16;
  // forward
  SK_TRY(dense<uint16_t>(c, n, FEAT, w, phi, FEAT, Wb + f.W1, w, 1, Wb + f.b1, nullptr, 0, H1, w, true, false));
  SK_TRY(dense<uint16_t>(c, n, w, w, H1, w, Wb + f.W2, w, 1, Wb + f.b2, nullptr, 0, H2, w, true, false));
  SK_TRY(dense<uint16_t>(c, n, w, o, H2, w, Wb + f.W3, o, 1, Wb + f.b3, nullptr, 0, F, o, false, false));
  // loss and dL/dF = U Acoef + F Bcoef
  SK_TRY(gram32(c, n, o, o, U, ldu, F, o, part, P));
  SK_TRY(gram32(c, n, o, o, F, o, F, o, part, G));
  hipLaunchKernelGGL(k_ws_loss, dim3(1), dim3(1024), 0, c->stream, o, mu, P, G, Ac, Bc, loss);
  SK_TRY(dense<float>(c, n, o, o, U, ldu, Ac, o, 1, nullptr, nullptr, 0, dF, o, false, false));
  SK_TRY(dense<float>(c, n, o, o, F, o, Bc, o, 1, nullptr, nullptr, 0, dF, o, false, true));
  // layer 3
  SK_TRY(gram32(c, n, w, o, H2, w, dF, o, part, grad + f.W3));
  SK_TRY(colsum(c, n, o, dF, o, part, grad + f.b3));
  SK_TRY(dense<uint16_t>(c, n, o, w, dF, o, Wb + f.W3, 1, o, nullptr, H2, w, dZ2, w, false, false));
  // layer 2
  SK_TRY(gram32(c, n, w, w, H1, w, dZ2, w, part, grad + f.W2));
  SK_TRY(colsum(c, n, w, dZ2, w, part, grad + f.b2));
  SK_TRY(dense<uint16_t>(c, n, w, w, dZ2, w, Wb + f.W2, 1, w, nullptr, H1, w, dZ1, w, false, false));
  // layer 1
  SK_TRY(gram32(c, n, FEAT, w, phi, FEAT, dZ1, w, part, grad + f.W1));
  return colsum(c, n, w, dZ1, w, part, grad + f.b1);
}

sketchne_status ws_adam(sketchne_ctx* c, const sketchne_mlp* net, const float* grad, float lr, int step, double beta1,
                        double beta2, double eps) {
  const int64_t total = ws_param_count(net->width, net->out);
  const float c1 = (float)(1.0 - pow(beta1, (double)step));
  const float c2 = (float)(1.0 - pow(beta2, (double)step));
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  hipLaunchKernelGGL(k_adam, dim3(nblk(total)), dim3(256), 0, c->stream, total, lr, (float)beta1, (float)beta2,
                     (float)(1.0 - beta1), (float)(1.0 - beta2), (float)eps, c1, c2, grad, net->master, net->adam_m,
                     net->adam_v, net->bf16);
  return launch_status();
}

sketchne_status ritz_residual(sketchne_ctx* c, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colidx,
                              double alpha, int k, const float* U, const double* lambda, double* res, void* ws,
                              size_t ws_bytes) {
  Arena ar(ws, ws_bytes);
  float* XU = ar.take<float>((size_t)n * k);
  float* dscale = ar.take<float>((size_t)n);
  double* part = ar.take<double>((size_t)resid_parts(n) * k);
  float* sp = ar.take<float>(spmm_ws_bytes(nnz, k) / sizeof(float));
  if (ar.overflow) return SKETCHNE_E_WORKSPACE;
  SK_TRY(degree_scale(c, n, rowptr, alpha, dscale));
  SK_TRY(spmm(c, n, nnz, rowptr, colidx, dscale, U, k, k, XU, k, sp));
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  int64_t parts = resid_parts(n);
  int64_t rpp = (n + parts - 1) / parts;
  parts = (n + rpp - 1) / rpp;
  hipLaunchKernelGGL(k_resid_part, dim3((unsigned)((k + 63) / 64), (unsigned)parts), dim3(256), 0, c->stream, n, k,
                     rpp, XU, U, lambda, part);
  hipLaunchKernelGGL(k_resid_final, dim3(nblk(k)), dim3(256), 0, c->stream, k, (int)parts, part, res);
  return launch_status();
}

}  // namespace skne
