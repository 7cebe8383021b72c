// The full-visit variant of the sparse-sign sketch: test matrices with z
// nonzeros in every ROW (one set per vertex) instead of every column, so
//     Y = f(L'R') S,   T = f(L'R') O,   Z = O^T T
// touch every one of the n^2 entries of f(L'R') (Alg. 3 read with the
// nonzeros of a test matrix spread over its rows).  Nothing is sampled, so
// the product becomes two chained GEMMs, as in attention:
//     X^T tile (32 columns j x 32 vertices i) = R'(:, j)^T L'(i, :)^T   (MFMA)
//     F = trunc_log(X) in registers
//     Y^T tile (32 outputs c x 32 vertices i) += S(j, c)^T F            (MFMA)
// The accumulator layout of the first product is the B-operand layout of
// the second once the summation index j of the second is taken in the order
// the accumulators hold it, so F never leaves registers; S is packed in that
// order (exact +-1 in BF16 or FP32, 1/sqrt(z) and ln 2 applied at the store).
// A workgroup of four wavefronts takes 128 vertices (one 32-vertex tile per
// wave, its L' fragments in registers) and streams the column tiles of R'
// and the matching S blocks through two LDS buffers by LDS-DMA.  The output
// columns are taken NCT tiles of 32 at a time (blockIdx.y), each launch chunk
// recomputing the first product.
#include <type_traits>

#include "internal.h"

#include "sketch.h"

namespace skne {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

template <int PREC>
struct FvOp;
template <>
struct FvOp<SKETCHNE_FP32> {
  typedef float frag;
  static constexpr int KS2 = 16;  // k-steps of the second product over 32 columns j
  static __device__ __forceinline__ floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct FvOp<SKETCHNE_BF16> {
  typedef bf16x8 frag;
  static constexpr int KS2 = 2;
  static __device__ __forceinline__ floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

__device__ __forceinline__ uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// column j (0..31) of a 32-column tile that k-step s, lane half hf, element u
// of the second product's operands stands for: the order in which the first
// product's accumulators hold the columns (register e of lane half hf holds
// row 8 (e / 4) + 4 hf + e % 4 of the 32 x 32 output)
__device__ __forceinline__ int fv_col(int prec, int s, int hf, int u) {
  if (prec == SKETCHNE_FP32) return 8 * (s >> 2) + 4 * hf + (s & 3);
  return 16 * s + (u < 4 ? 4 * hf + u : 8 + 4 * hf + (u - 4));
}

// S^T blocks in MFMA A-fragment order: [column tile jt][output tile ct][k-step s][lane]
// (lane l: output c = 32 ct + l % 32, columns j of k-step s from fv_col)
// value = sign if c is among the z columns of row j (of n rows), else 0
template <int PREC>
__global__ void k_pack_s_full(int64_t n, int64_t njt, int nct, int z, const int32_t* __restrict__ cols,
                              const int8_t* __restrict__ signs, void* __restrict__ out, uint32_t* __restrict__ flags,
                              int width) {
  constexpr int KS2 = FvOp<PREC>::KS2;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = njt * nct * KS2 * 64;
  if (idx >= total) return;
  const int lane = (int)(idx & 63);
  int64_t q = idx >> 6;
  const int s = (int)(q % KS2);
  q /= KS2;
  const int ct = (int)(q % nct);
  const int64_t jt = q / nct;
  const int c = 32 * ct + (lane & 31), hf = lane >> 5;
  auto value = [&](int u) -> float {
    const int64_t j = 32 * jt + fv_col(PREC, s, hf, u);
    if (j >= n) return 0.0f;
    float v = 0.0f;
    for (int t = 0; t < z; ++t) {
      const int col = cols[j * z + t];
      if (col < 0 || col >= width) atomicOr(flags, SKETCHNE_FLAG_BAD_INDEX);
      if (col == c) v = (float)signs[j * z + t];
    }
    return v;
  };
  if (PREC == SKETCHNE_FP32) {
    static_cast<float*>(out)[idx] = value(0);
  } else {
    uint16_t w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) w[u] = bf16_rne(value(u));
    static_cast<uint4*>(out)[idx] = make_uint4(w[0] | ((uint32_t)w[1] << 16), w[2] | ((uint32_t)w[3] << 16),
                                               w[4] | ((uint32_t)w[5] << 16), w[6] | ((uint32_t)w[7] << 16));
  }
}

// rows of R'^T before the core product: Gsel[j][:] = scale d1[j] U[j][:] (zero for j >= n)
__global__ void k_gather_rows(int64_t n, int64_t npad, int k, const float* __restrict__ U, int64_t ldu,
                              const double* __restrict__ d1, double scale, double* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= npad * k) return;
  const int64_t j = idx / k;
  const int col = (int)(idx - j * k);
  out[idx] = j < n ? scale * d1[j] * (double)U[j * ldu + col] : 0.0;
}

// dense O (n x l, FP32) from the per-row coordinates: O[i][cols[i][t]] = signs[i][t] / sqrt(z)
__global__ void k_dense_rows(int64_t n, int width, int z, const int32_t* __restrict__ cols,
                             const int8_t* __restrict__ signs, float inv_sqrt_z, float* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * z) return;
  const int64_t i = idx / z;
  const int col = cols[idx];
  if (col >= 0 && col < width) out[i * width + col] = inv_sqrt_z * (float)signs[idx];
}

// Z = O^T T for the row-sparse O (z signed entries per row, value s / sqrt z)
// and T = f(L'R') O held transposed (Tt, l x n: row c is column c of T).
// Workgroup c forms column c of Z, Z[c'][c] = (1 / sqrt z) sum over rows j and
// their entries (c', s) of s T[j][c], streaming row c of Tt once (coalesced)
// with the entries of O (read by every workgroup, so served from L2).  The
// terms are added as 64-bit integers at a power-of-two scale 2^e chosen from
// max |T| so that no sum can leave the range (|sum| <= n max |T| <= 2^62):
// integer addition is associative, so the LDS atomics that scatter the terms
// give the same bits in any order, and the only rounding is each term's, at
// 2^-e (2^-46 of max |T| at n = 2^16).
__global__ void k_fv_tmax_clear(unsigned* __restrict__ tmax) {
  if (threadIdx.x == 0) *tmax = 0u;
}

__global__ __launch_bounds__(256) void k_fv_tmax(int64_t count, const float* __restrict__ T, unsigned* __restrict__ tmax) {
  float m = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
    const float a = fabsf(T[i]);
    m = (a == a) ? fmaxf(m, a) : __builtin_inff();  // a NaN is carried as +inf
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  // non-negative floats order as their bit patterns
  if ((threadIdx.x & 63) == 0) atomicMax(tmax, __float_as_uint(m));
}

__global__ __launch_bounds__(256) void k_fv_z(int64_t n, int l, int z, const int32_t* __restrict__ cols,
                                              const int8_t* __restrict__ signs, const float* __restrict__ Tt,
                                              int64_t ldt, const unsigned* __restrict__ tmax_bits, double inv_sqrt_z,
                                              float* __restrict__ Z, uint32_t* __restrict__ flags) {
  extern __shared__ long long zacc[];  // l
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < l; i += blockDim.x) zacc[i] = 0;
  const float tmax = __uint_as_float(*tmax_bits);
  __syncthreads();
  if (!(tmax <= 3.4e38f)) {  // T holds a non-finite value
    for (int i = threadIdx.x; i < l; i += blockDim.x) Z[(int64_t)i * l + c] = __builtin_nanf("");
    if (threadIdx.x == 0) atomicOr(flags, (uint32_t)SKETCHNE_FLAG_NONFINITE);
    return;
  }
  const int e = tmax > 0.0f ? 62 - (int)ceil(log2((double)n * (double)tmax)) : 0;
  const double scale = ldexp(1.0, e);
  const float* trow = Tt + (int64_t)c * ldt;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
    const double v = (double)trow[j] * scale;
    for (int t = 0; t < z; ++t) {
      const int col = cols[j * z + t];
      if (col >= 0 && col < l) {
        const long long q = llrint(signs[j * z + t] > 0 ? v : -v);
        atomicAdd(reinterpret_cast<unsigned long long*>(&zacc[col]), (unsigned long long)q);
      }
    }
  }
  __syncthreads();
  const double back = ldexp(inv_sqrt_z, -e);
  for (int i = threadIdx.x; i < l; i += blockDim.x) Z[(int64_t)i * l + c] = (float)((double)zacc[i] * back);
}

__global__ void k_fill0(int64_t count, float* __restrict__ out) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < count) out[idx] = 0.0f;
}

template <int N>
using cint = std::integral_constant<int, N>;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t fv_rsrc(const void* base, uint32_t bytes) {
  // wave-uniform by construction; readfirstlane keeps the descriptor scalar
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  void* ptr = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  // dword 3 = 0x00020000: 32-bit data format, the raw-buffer setting of gfx9
  return __builtin_amdgcn_make_buffer_rsrc(ptr, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

template <int PREC, int KSM, int NCT>
__global__ __launch_bounds__(256, 1) void k_fullvisit(int64_t nrows, int64_t njt, int nct_all, int width,
                                                      const void* __restrict__ Bpack, const void* A1pack,
                                                      const void* A2pack, float* __restrict__ out, int64_t ld_out,
                                                      float out_scale) {
  typedef FvOp<PREC> Op;
  typedef typename Op::frag frag;
  constexpr int FB = sizeof(frag) * 64;  // bytes of one fragment (64 lanes)
  constexpr int KS2 = Op::KS2;
  constexpr int NF = KSM + NCT * KS2;    // fragments per column tile in LDS
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  // wave index made visibly uniform, so that branches on it are scalar
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t vt = (int64_t)blockIdx.x * 4 + wave;
  const int ct0 = blockIdx.y * NCT;  // nct_all is a multiple of NCT (padded with zero blocks)

  frag bfr[KSM];
  const frag* Bp = static_cast<const frag*>(Bpack);
#pragma unroll
  for (int ks = 0; ks < KSM; ++ks) bfr[ks] = Bp[(vt * KSM + ks) * 64 + lane];
  // column tile jt -> LDS buffer B: its KSM fragments of R'^T, then the S^T
  // fragments of this launch's output tiles; fragment f is one DMA by wave
  // f % 4.  Buffer (MUBUF) LDS-DMA, so that no FLAT operation is pending while
  // the fragments are read (that would turn every LDS-read wait into
  // lgkmcnt(0)); the host keeps both packed arrays below 4 GiB.
  const __amdgpu_buffer_rsrc_t a1_rs = fv_rsrc(A1pack, (uint32_t)(njt * KSM * FB));
  const __amdgpu_buffer_rsrc_t a2_rs = fv_rsrc(A2pack, (uint32_t)(njt * nct_all * KS2 * FB));
  auto dma = [&](int64_t jt, auto Bc) {
    constexpr int B = decltype(Bc)::value;
    char* dst = lds_raw + B * NF * FB;
#pragma unroll
    for (int f0 = 0; f0 < NF; f0 += 4) {
      const int f = f0 + wave;
      if (NF % 4 != 0 && f >= NF) break;
      const bool first = f < KSM;
      const uint32_t off = first ? (uint32_t)((jt * KSM + f) * FB)
                                 : (uint32_t)(((jt * nct_all + ct0) * KS2 + (f - KSM)) * FB);
      if constexpr (sizeof(frag) == 16)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(first ? a1_rs : a2_rs, (lds_void*)(dst + f * FB), 16,
                                                 off + (uint32_t)(lane * 16), 0, 0, 0);
      else
        __builtin_amdgcn_raw_ptr_buffer_load_lds(first ? a1_rs : a2_rs, (lds_void*)(dst + f * FB), 4,
                                                 off + (uint32_t)(lane * 4), 0, 0, 0);
    }
  };
  floatx16 accY[NCT];
#pragma unroll
  for (int q = 0; q < NCT; ++q)
#pragma unroll
    for (int e = 0; e < 16; ++e) accY[q][e] = 0.0f;
  dma(0, cint<0>());
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // one column tile; the loop below is unrolled by two so that both LDS
  // buffer offsets are compile-time constants and the reads of one buffer
  // never wait on the copy into the other
  auto step = [&](int64_t jt, auto Bc) {
    constexpr int B = decltype(Bc)::value;
    if (jt + 1 < njt) dma(jt + 1, cint<B ^ 1>());
    const frag* L = reinterpret_cast<const frag*>(lds_raw + B * NF * FB);
    // first product: X^T (32 columns x 32 vertices)
    floatx16 x = {};
#pragma unroll
    for (int ks = 0; ks < KSM; ++ks) x = Op::mma(L[ks * 64 + lane], bfr[ks], x);
    // fragment reads RA ahead of their MFMAs
    constexpr int RA = KSM < 6 ? KSM : 6;
    __builtin_amdgcn_sched_group_barrier(0x100, RA, 0);
#pragma unroll
    for (int g = 0; g < KSM - RA; ++g) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, RA, 0);
    __builtin_amdgcn_sched_barrier(0);
    // F = max(log2 x, 0) as the B operand of the second product
    frag fb[KS2];
    if constexpr (PREC == SKETCHNE_FP32) {
#pragma unroll
      for (int s = 0; s < KS2; ++s) fb[s] = fmaxf(__builtin_amdgcn_logf(x[s]), 0.0f);
    } else {
#pragma unroll
      for (int s = 0; s < KS2; ++s) {
        uint16_t w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) w[u] = bf16_rne(fmaxf(__builtin_amdgcn_logf(x[8 * s + u]), 0.0f));
        uint4 pk = make_uint4(w[0] | ((uint32_t)w[1] << 16), w[2] | ((uint32_t)w[3] << 16),
                              w[4] | ((uint32_t)w[5] << 16), w[6] | ((uint32_t)w[7] << 16));
        fb[s] = __builtin_bit_cast(frag, pk);
      }
    }
    // second product: Y^T tiles += S^T F, its first fragments read during
    // the vector work above
#pragma unroll
    for (int q = 0; q < NCT; ++q)
#pragma unroll
      for (int s = 0; s < KS2; ++s) accY[q] = Op::mma(L[(KSM + q * KS2 + s) * 64 + lane], fb[s], accY[q]);
    constexpr int N2 = NCT * KS2;
    constexpr int RB = N2 < 6 ? N2 : 6;
    __builtin_amdgcn_sched_group_barrier(0x100, RB, 0);
    __builtin_amdgcn_sched_group_barrier(0x002, 256, 0);
#pragma unroll
    for (int g = 0; g < N2 - RB; ++g) {
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, RB, 0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  int64_t jt = 0;
  for (; jt + 2 <= njt; jt += 2) {
    step(jt, cint<0>());
    step(jt + 1, cint<1>());
  }
  if (jt < njt) step(jt, cint<0>());
  // Y^T[c][i], c = 32 (ct0 + q) + 8 (e / 4) + 4 hf + e % 4, i = 32 vt + lane % 32
  const int64_t i = vt * 32 + (lane & 31);
  if (i >= nrows) return;
#pragma unroll
  for (int q = 0; q < NCT; ++q) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int c = 32 * (ct0 + q) + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
      if (c < width) out[(int64_t)c * ld_out + i] = out_scale * accY[q][e];
    }
  }
}

template <int PREC, int KSM, int NCT>
sketchne_status launch_fullvisit(sketchne_ctx* c, int cls, int64_t nrows, int64_t njt, int nct_all, int width,
                                 const void* Bp, const void* A1, const void* A2, float* out, int64_t ld_out,
                                 float out_scale) {
  typedef typename FvOp<PREC>::frag frag;
  constexpr int NF = KSM + NCT * FvOp<PREC>::KS2;
  const size_t shmem = (size_t)2 * NF * 64 * sizeof(frag);
  // the tile copies address the packed operands with 32-bit offsets
  if (nct_all % NCT != 0) return SKETCHNE_E_ARG;
  const int64_t fb = 64 * (int64_t)sizeof(frag);
  if (njt * KSM * fb >= ((int64_t)1 << 32) || njt * nct_all * FvOp<PREC>::KS2 * fb >= ((int64_t)1 << 32))
    return SKETCHNE_E_UNSUPPORTED;
  auto kern = k_fullvisit<PREC, KSM, NCT>;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)shmem) != hipSuccess)
    return SKETCHNE_E_DEVICE;
  const int64_t nvt = (nrows + 31) / 32;
  ProfScope ps(c, cls);
  hipLaunchKernelGGL(kern, dim3((unsigned)((nvt + 3) / 4), (unsigned)((nct_all + NCT - 1) / NCT)), dim3(256), shmem,
                     c->stream, nrows, njt, nct_all, width, Bp, A1, A2, out, ld_out, out_scale);
  return launch_status();
}

}  // namespace

// output tiles per launch chunk (accumulators held per lane: 16 per tile)
int fullvisit_nct(int prec) { return prec == SKETCHNE_FP32 ? 3 : 9; }

sketchne_status gather_rows(sketchne_ctx* c, int64_t n, int64_t npad, int k, const float* U, int64_t ldu,
                            const double* d1, double scale, double* out) {
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)((npad * k + 255) / 256)), dim3(256), 0, c->stream, n, npad, k, U,
                     ldu, d1, scale, out);
  return launch_status();
}

sketchne_status pack_s_full(sketchne_ctx* c, int prec, int64_t n, int64_t njt, int nct, int z, const int32_t* cols,
                            const int8_t* signs, int width, void* out) {
  const int ks2 = prec == SKETCHNE_FP32 ? FvOp<SKETCHNE_FP32>::KS2 : FvOp<SKETCHNE_BF16>::KS2;
  const int64_t tot = njt * nct * ks2 * 64;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  if (prec == SKETCHNE_FP32)
    hipLaunchKernelGGL(k_pack_s_full<SKETCHNE_FP32>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, n,
                       njt, nct, z, cols, signs, out, c->d_flags, width);
  else
    hipLaunchKernelGGL(k_pack_s_full<SKETCHNE_BF16>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, n,
                       njt, nct, z, cols, signs, out, c->d_flags, width);
  return launch_status();
}

sketchne_status fv_z(sketchne_ctx* c, int64_t n, int l, int z, const int32_t* cols, const int8_t* signs,
                     const float* Tt, int64_t ldt, unsigned* tmax, double inv_sqrt_z, float* Z) {
  if ((size_t)l * sizeof(long long) > 65536) return SKETCHNE_E_UNSUPPORTED;
  ProfScope ps(c, SKETCHNE_PROF_SKETCH_Z);
  hipLaunchKernelGGL(k_fv_tmax_clear, dim3(1), dim3(64), 0, c->stream, tmax);
  const int64_t cnt = (int64_t)l * ldt;
  int64_t blocks = (cnt + 4 * 256 - 1) / (4 * 256);
  blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
  hipLaunchKernelGGL(k_fv_tmax, dim3((unsigned)blocks), dim3(256), 0, c->stream, cnt, Tt, tmax);
  hipLaunchKernelGGL(k_fv_z, dim3((unsigned)l), dim3(256), (size_t)l * sizeof(long long), c->stream, n, l, z, cols,
                     signs, Tt, ldt, tmax, inv_sqrt_z, Z, c->d_flags);
  return launch_status();
}

sketchne_status dense_rows(sketchne_ctx* c, int64_t n, int width, int z, const int32_t* cols, const int8_t* signs,
                           float inv_sqrt_z, float* out) {
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  const int64_t cnt = n * width;
  hipLaunchKernelGGL(k_fill0, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, c->stream, cnt, out);
  hipLaunchKernelGGL(k_dense_rows, dim3((unsigned)((n * z + 255) / 256)), dim3(256), 0, c->stream, n, width, z, cols,
                     signs, inv_sqrt_z, out);
  return launch_status();
}

sketchne_status fullvisit(sketchne_ctx* c, int cls, int prec, int KSM, int64_t nrows, int64_t njt, int nct_all,
                          int width, const void* Bp, const void* A1, const void* A2, float* out, int64_t ld_out,
                          float out_scale) {
  if (nrows == 0 || width == 0) return SKETCHNE_OK;
  if (prec == SKETCHNE_FP32) {
    switch (KSM) {
      case 32: return launch_fullvisit<SKETCHNE_FP32, 32, 3>(c, cls, nrows, njt, nct_all, width, Bp, A1, A2, out, ld_out, out_scale);
      case 64: return launch_fullvisit<SKETCHNE_FP32, 64, 3>(c, cls, nrows, njt, nct_all, width, Bp, A1, A2, out, ld_out, out_scale);
      case 128: return launch_fullvisit<SKETCHNE_FP32, 128, 3>(c, cls, nrows, njt, nct_all, width, Bp, A1, A2, out, ld_out, out_scale);
    }
  } else if (prec == SKETCHNE_BF16) {
    switch (KSM) {
      case 8: return launch_fullvisit<SKETCHNE_BF16, 8, 9>(c, cls, nrows, njt, nct_all, width, Bp, A1, A2, out, ld_out, out_scale);
      case 16: return launch_fullvisit<SKETCHNE_BF16, 16, 9>(c, cls, nrows, njt, nct_all, width, Bp, A1, A2, out, ld_out, out_scale);
    }
  }
  return SKETCHNE_E_UNSUPPORTED;
}

}  // namespace skne
