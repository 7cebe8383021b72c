// Tall-skinny apply on the FP64 matrix cores:  C = A B  with A an n x K FP32
// block (n large) and B a small K x N FP64 matrix (N, K <= 288).
//
// This is the shape of every apply of the path: Q = B R^-1 in Cholesky-QR
// (R^-1 upper triangular), U = Q U^(:, 1:k) after Rayleigh-Ritz, and
// E = Y (R^-1 U^ Sigma^1/2) in the embedding.  A workgroup owns 128 rows and
// every output column, so each row of A is read from HBM once and written
// once.  A and B stream in chunks of 16 summation indices through two LDS
// buffers: chunk c + 1 is stored into one while chunk c is multiplied out of
// the other (one barrier per chunk), and the registers already hold chunk
// c + 2, fetched from HBM (A) and L2 (B).  With a triangular B a
// chunk only meets the column blocks at or right of its diagonal, which
// halves the work of the Cholesky-QR apply; entries below the diagonal are
// masked on load, whatever the buffer holds there.
//
// F32 selects the FP32 matrix cores (v_mfma_f32_16x16x4f32, FP32 operands in
// LDS, B rounded to FP32): twice the FP64 rate and half the LDS bytes, for the
// applies whose result only has to span the right space (the power-iteration
// bases of Alg. 5), not to be accurate to FP64 working precision.  This form
// reads B from an FP32 copy made just before the launch, so the chunk held in
// registers takes half the VGPRs and four wavefronts fit per SIMD (two
// workgroups per CU) instead of two.
//
// 8 wavefronts: wave w owns rows 32 (w & 3) .. +32 (two 16-row MFMA blocks)
// and the column blocks (16 columns each) of parity w >> 2, i.e. 2 x NBH
// v_mfma_f64_16x16x4f64 accumulators; interleaving the blocks keeps the two
// halves equally loaded when a triangular B skips blocks.
#include <type_traits>

#include "internal.h"

namespace skne {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

// operand and accumulator types of the two forms
template <bool F32>
struct ApplyTy {
  typedef double T;
  typedef doublex4 Acc;
  static constexpr int PAD = 2;  // LDS row padding (elements)
  static __device__ __forceinline__ Acc mma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output element (lane, r) -> row within the 16-row block
  static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <>
struct ApplyTy<true> {
  typedef float T;
  typedef floatx4 Acc;
  static constexpr int PAD = 16;  // rows 16 banks apart: the 4 k-rows of a fragment read hit distinct banks
  static __device__ __forceinline__ Acc mma(T a, T b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int AR = 128;   // rows per workgroup
constexpr int ABK = 16;   // summation chunk

struct ApplyArgs {
  int64_t n; int K, N;
  const float* A; int64_t lda;
  const double* B; int64_t ldb;
  float* C; int64_t ldc;
  const int* run_if;
  const float* B32;  // the FP32 form's copy of B (same layout)
};

// FP32 copy of a B given by `rows` strided rows of ldb doubles
__global__ void k_b_to_f32(int64_t count, const double* __restrict__ B, float* __restrict__ B32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) B32[i] = (float)B[i];
}

// One chunk's products for the wave's column blocks 2t + ch, t = T0 .. NBH-1,
// k-steps in order, as straight-line code.
template <int T0, int NBH, bool F32>
__device__ __forceinline__ void chunk_mfma(const typename ApplyTy<F32>::T (*As)[AR + ApplyTy<F32>::PAD],
                                           const typename ApplyTy<F32>::T (*Bs)[32 * NBH + ApplyTy<F32>::PAD], int rg,
                                           int ch, int lane, typename ApplyTy<F32>::Acc (&acc)[2][NBH]) {
  typedef ApplyTy<F32> Ty;
#pragma unroll
  for (int kk = 0; kk < ABK / 4; ++kk) {
    const int kr = kk * 4 + (lane >> 4);
    const typename Ty::T a0 = As[kr][32 * rg + (lane & 15)];
    const typename Ty::T a1 = As[kr][32 * rg + 16 + (lane & 15)];
#pragma unroll
    for (int t = T0; t < NBH; ++t) {
      const typename Ty::T b = Bs[kr][16 * (2 * t + ch) + (lane & 15)];
      acc[0][t] = Ty::mma(a0, b, acc[0][t]);
      acc[1][t] = Ty::mma(a1, b, acc[1][t]);
    }
  }
}

template <int C, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (C < N) {
    f(std::integral_constant<int, C>{});
    static_for<C + 1, N>(f);
  }
}

// ACOL: A(i,k) = A[k*lda + i] (else A[i*lda + k]); BCOL: B(k,j) = B[j*ldb + k]
// (else B[k*ldb + j]); CCOL: C(i,j) = C[j*ldc + i] (else C[i*ldc + j]);
// TRI: B(k,j) = 0 for k > j.
template <int NBH, bool ACOL, bool BCOL, bool CCOL, bool TRI, bool F32 = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(F32 ? 4 : 1))) void k_apply_tall(ApplyArgs g) {
  typedef ApplyTy<F32> Ty;
  typedef typename Ty::T T;
  constexpr int NC = 32 * NBH;                        // columns held by the workgroup
  constexpr int AVEC = AR * ABK / 4;                  // float4 per A chunk
  constexpr int APER = AVEC / 512;
  constexpr int BVEC = ABK * NC / 2;                  // double2 per B chunk
  constexpr int BPER = (BVEC + 511) / 512;
  __shared__ T As[2][ABK][AR + Ty::PAD];
  __shared__ T Bs[2][ABK][NC + Ty::PAD];
  if (g.run_if && *g.run_if == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rg = wave & 3, ch = __builtin_amdgcn_readfirstlane(wave >> 2);
  const int64_t i0 = (int64_t)blockIdx.x * AR;
  const int kend = TRI ? min(g.K, g.N) : g.K;

  typedef std::conditional_t<F32, float2, double2> BPair;
  float4 ra[APER];
  BPair rb[BPER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int p = 0; p < APER; ++p) {
      const int e = tid + 512 * p;
      if (!ACOL) {
        // consecutive lanes take consecutive rows, so that the LDS stores
        // below (one k-row of As per store) are conflict-free
        const int r = e % AR, q = (e / AR) * 4;
        const int64_t i = i0 + r;
        const int k = k0 + q;
        ra[p] = (i < g.n && k < kend) ? *reinterpret_cast<const float4*>(g.A + i * g.lda + k)
                                      : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        const int kk = e / (AR / 4), q = (e % (AR / 4)) * 4;
        const int k = k0 + kk;
        const int64_t i = i0 + q;
        if (k < kend && i + 3 < g.n) {
          ra[p] = *reinterpret_cast<const float4*>(g.A + (int64_t)k * g.lda + i);
        } else {
          const float* ptr = g.A + (int64_t)k * g.lda + i;
          ra[p].x = (k < kend && i + 0 < g.n) ? ptr[0] : 0.f;
          ra[p].y = (k < kend && i + 1 < g.n) ? ptr[1] : 0.f;
          ra[p].z = (k < kend && i + 2 < g.n) ? ptr[2] : 0.f;
          ra[p].w = (k < kend && i + 3 < g.n) ? ptr[3] : 0.f;
        }
      }
    }
#pragma unroll
    for (int p = 0; p < BPER; ++p) {
      const int e = tid + 512 * p;
      BPair v;
      v.x = 0;
      v.y = 0;
      if (e < BVEC) {
        int j, k;
        // BCOL: eight consecutive lanes read one column's 16 indices
        if (BCOL) { j = e / (ABK / 2); k = k0 + (e % (ABK / 2)) * 2; }
        else { k = k0 + e / (NC / 2); j = (e % (NC / 2)) * 2; }
        // with a triangular B, whole columns j < k0 are zero in this chunk
        if (j < g.N && k < kend && !(TRI && j < k0)) {
          const int64_t at = BCOL ? (int64_t)j * g.ldb + k : (int64_t)k * g.ldb + j;
          if constexpr (F32) v = *reinterpret_cast<const float2*>(g.B32 + at);
          else v = *reinterpret_cast<const double2*>(g.B + at);
          if (TRI) {
            // BCOL: (k, j) and (k+1, j); else (k, j) and (k, j+1)
            if (BCOL) { if (k > j) v.x = 0; if (k + 1 > j) v.y = 0; }
            else { if (k > j) v.x = 0; if (k > j + 1) v.y = 0; }
          }
        }
      }
      rb[p] = v;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int p = 0; p < APER; ++p) {
      const int e = tid + 512 * p;
      if (!ACOL) {
        const int r = e % AR, q = (e / AR) * 4;
        As[buf][q + 0][r] = ra[p].x;
        As[buf][q + 1][r] = ra[p].y;
        As[buf][q + 2][r] = ra[p].z;
        As[buf][q + 3][r] = ra[p].w;
      } else {
        const int kk = e / (AR / 4), q = (e % (AR / 4)) * 4;
        As[buf][kk][q + 0] = ra[p].x;
        As[buf][kk][q + 1] = ra[p].y;
        As[buf][kk][q + 2] = ra[p].z;
        As[buf][kk][q + 3] = ra[p].w;
      }
    }
#pragma unroll
    for (int p = 0; p < BPER; ++p) {
      const int e = tid + 512 * p;
      if (e < BVEC) {
        if (BCOL) {
          const int j = e / (ABK / 2), kk = (e % (ABK / 2)) * 2;
          Bs[buf][kk][j] = (T)rb[p].x;
          Bs[buf][kk + 1][j] = (T)rb[p].y;
        } else {
          const int kk = e / (NC / 2), j = (e % (NC / 2)) * 2;
          Bs[buf][kk][j] = (T)rb[p].x;
          Bs[buf][kk][j + 1] = (T)rb[p].y;
        }
      }
    }
  };

  typename Ty::Acc acc[2][NBH];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int t = 0; t < NBH; ++t) acc[m][t] = typename Ty::Acc{0, 0, 0, 0};

  // two LDS buffers; the registers run two chunks ahead
  const int nchunk = (kend + ABK - 1) / ABK;
  if (nchunk > 0) {
    fetch(0);
    stash(0);
  }
  if (nchunk > 1) fetch(ABK);
  __syncthreads();
  // after chunk c's MFMAs are issued: chunk c + 1 into the other buffer (last
  // read by chunk c - 1, before the previous barrier), then fetch chunk c + 2
  auto advance = [&](int c) {
    if (c + 1 < nchunk) {
      stash((c + 1) & 1);
      if (c + 2 < nchunk) fetch((c + 2) * ABK);
    }
    __syncthreads();
  };
  // column blocks are interleaved over the two halves: block 2t + ch
  if constexpr (TRI) {
    // Chunk c (indices 16c .. 16c+15) meets block 2t + ch only if its last
    // column 32t + 16ch + 15 >= 16c.  Both halves start at t = c / 2 (for odd
    // c the even half's first block lies left of the diagonal; B was zeroed
    // there on load, so it adds zeros).  N = K <= 32 NBH, so there are at
    // most 2 NBH chunks: the loop is unrolled and each chunk gets a
    // branch-free body over its blocks.
    static_for<0, 2 * NBH>([&](auto cc) {
      constexpr int c = decltype(cc)::value;
      if (c < nchunk) {
        chunk_mfma<c / 2, NBH, F32>(As[c & 1], Bs[c & 1], rg, ch, lane, acc);
        advance(c);
      }
    });
  } else {
    for (int c = 0; c < nchunk; ++c) {
      chunk_mfma<0, NBH, F32>(As[c & 1], Bs[c & 1], rg, ch, lane, acc);
      advance(c);
    }
  }

  // output: lane l, register r -> row Ty::row(l, r) of the 16-row block, column l % 16
#pragma unroll
  for (int t = 0; t < NBH; ++t) {
    const int j = 16 * (2 * t + ch) + (lane & 15);
    if (j >= g.N) continue;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 32 * rg + 16 * m + Ty::row(lane, r);
        if (i >= g.n) continue;
        const float v = (float)acc[m][t][r];
        if (CCOL) g.C[(int64_t)j * g.ldc + i] = v;
        else g.C[i * g.ldc + j] = v;
      }
  }
}

}  // namespace

bool apply_tall_supported(const ApplyDesc& d) {
  if (d.N < 1 || d.N > 288 || d.K < 1 || d.K > 288) return false;
  if (d.N % 2 || d.K % 4 || d.lda % 4 || d.ldb % 2) return false;
  if (d.ccol && !d.acol) return false;
  if (d.upper && d.N != d.K) return false;
  if (reinterpret_cast<uintptr_t>(d.A) % 16 || reinterpret_cast<uintptr_t>(d.B) % 16) return false;
  return true;
}

sketchne_status apply_tall(sketchne_ctx* c, const ApplyDesc& d) {
  if (d.n == 0) return SKETCHNE_OK;
  if (!apply_tall_supported(d)) return SKETCHNE_E_UNSUPPORTED;
  ProfScope ps(c, SKETCHNE_PROF_GEMM64);
  ApplyArgs g{d.n, d.K, d.N, d.A, d.lda, d.B, d.ldb, d.C, d.ldc, d.run_if, d.b32};
  dim3 grid((unsigned)((d.n + AR - 1) / AR)), blk(512);
  const int nbh = d.N <= 128 ? 4 : (d.N <= 256 ? 8 : 9);
  // the FP32 form is built for two shapes of a row-major block: the
  // Cholesky-QR apply (B = R^-1 read by columns) and a plain B read by rows;
  // it needs the scratch for B's FP32 copy
  if (d.f32 && d.b32 && !d.acol && !d.ccol && d.upper == d.bcol) {
    // B spans (N columns or K rows) of ldb doubles; the last one only to K or N
    const int64_t count = (int64_t)((d.bcol ? d.N : d.K) - 1) * d.ldb + (d.bcol ? d.K : d.N);
    hipLaunchKernelGGL(k_b_to_f32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, c->stream, count, d.B, d.b32);
    if (d.upper) {
      if (nbh == 4) hipLaunchKernelGGL((k_apply_tall<4, false, true, false, true, true>), grid, blk, 0, c->stream, g);
      else if (nbh == 8) hipLaunchKernelGGL((k_apply_tall<8, false, true, false, true, true>), grid, blk, 0, c->stream, g);
      else hipLaunchKernelGGL((k_apply_tall<9, false, true, false, true, true>), grid, blk, 0, c->stream, g);
    } else {
      if (nbh == 4) hipLaunchKernelGGL((k_apply_tall<4, false, false, false, false, true>), grid, blk, 0, c->stream, g);
      else if (nbh == 8) hipLaunchKernelGGL((k_apply_tall<8, false, false, false, false, true>), grid, blk, 0, c->stream, g);
      else hipLaunchKernelGGL((k_apply_tall<9, false, false, false, false, true>), grid, blk, 0, c->stream, g);
    }
    return launch_status();
  }
#define SKNE_APPLY(NBH)                                                                                       \
  do {                                                                                                        \
    if (d.upper && d.bcol) {                                                                                  \
      if (d.ccol) hipLaunchKernelGGL((k_apply_tall<NBH, true, true, true, true>), grid, blk, 0, c->stream, g); \
      else if (d.acol) hipLaunchKernelGGL((k_apply_tall<NBH, true, true, false, true>), grid, blk, 0, c->stream, g); \
      else hipLaunchKernelGGL((k_apply_tall<NBH, false, true, false, true>), grid, blk, 0, c->stream, g);      \
    } else if (d.upper) {                                                                                     \
      if (d.ccol) hipLaunchKernelGGL((k_apply_tall<NBH, true, false, true, true>), grid, blk, 0, c->stream, g); \
      else if (d.acol) hipLaunchKernelGGL((k_apply_tall<NBH, true, false, false, true>), grid, blk, 0, c->stream, g); \
      else hipLaunchKernelGGL((k_apply_tall<NBH, false, false, false, true>), grid, blk, 0, c->stream, g);     \
    } else if (d.bcol) {                                                                                      \
      if (d.ccol) hipLaunchKernelGGL((k_apply_tall<NBH, true, true, true, false>), grid, blk, 0, c->stream, g); \
      else if (d.acol) hipLaunchKernelGGL((k_apply_tall<NBH, true, true, false, false>), grid, blk, 0, c->stream, g); \
      else hipLaunchKernelGGL((k_apply_tall<NBH, false, true, false, false>), grid, blk, 0, c->stream, g);     \
    } else {                                                                                                  \
      if (d.ccol) hipLaunchKernelGGL((k_apply_tall<NBH, true, false, true, false>), grid, blk, 0, c->stream, g); \
      else if (d.acol) hipLaunchKernelGGL((k_apply_tall<NBH, true, false, false, false>), grid, blk, 0, c->stream, g); \
      else hipLaunchKernelGGL((k_apply_tall<NBH, false, false, false, false>), grid, blk, 0, c->stream, g);    \
    }                                                                                                         \
  } while (0)
  if (nbh == 4) SKNE_APPLY(4);
  else if (nbh == 8) SKNE_APPLY(8);
  else SKNE_APPLY(9);
#undef SKNE_APPLY
  return launch_status();
}

}  // namespace skne
