// The single-pass sparse-sign sketch of f(L'R') (Section 3.1, Eq. 4, Alg. 4).
//
// Column sampling (Eq. 4) means only the columns of f(L'R') that a test
// matrix touches are ever formed.  Each test-matrix column c has z nonzeros
// (row p_ct, sign s_ct), so with the columns of R' "expanded" to one column
// per nonzero,
//
//     Y[i][c] = (1/sqrt z) * sum_t s_ct * f(L'_i . R'(:, p_ct)),
//
// one row of Y is a GEMM row followed by a signed sum over groups of z
// adjacent expanded columns.  The fused kernel computes the GEMM on the
// matrix cores with the vertex block held in registers and the expanded
// columns streamed through LDS; the expanded columns are ordered so that the
// z (<= 8) members of a group land in the accumulator registers of one lane
// (32x32 MFMA output: lane l, register r holds row 8(r/4) + 4(l/32) + r%4),
// so trunc_log and the signed group sum finish in registers and each output
// is written exactly once, without atomics.  Duplicate coordinates across
// columns are recomputed rather than de-duplicated.  f = trunc_log is
// evaluated as ln2 * log2(max(x, 1)), with ln2 and 1/sqrt(z) folded into one
// final multiply.
//
// The same kernel forms Z: its "vertex" rows are then the rows p_O of O
// (Alg. 4 line 7), giving T1 = f(L'(p_O,:) R'(:, p_O)) O(p_O,:), and
// k_z_reduce applies O(p_O,:)^T.
//
// Precision forms: FP32 operands (v_mfma_f32_32x32x2_f32), or BF16 / FP16
// operands (v_mfma_f32_32x32x16_{bf16,f16}) with FP32 accumulation.  In the
// BF16/FP16 forms the first split_r components are carried as hi + lo pairs.
// The summation index runs over three sections, each zero-padded to whole
// 16-wide k-steps (KSM main steps, KSS split steps):
//     A (expanded columns of R'):  [hi(0..k) | hi(0..r) | lo(0..r)]
//     B (rows of L'):              [hi(0..k) | lo(0..r)]
// and A's third section meets B's first KSS k-steps (hi(0..r)) again, so the
// GEMM forms hi.hi + hi.lo + lo.hi on the dominant components in one pass
// while B stores only KSM + KSS fragments per vertex.
#include <type_traits>

#include "internal.h"

#include "sketch.h"

namespace skne {
namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 halfx8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t bf16_bits_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f16_bits(float f) {
  _Float16 h = (_Float16)f;
  return *reinterpret_cast<uint16_t*>(&h);
}
__device__ __forceinline__ float f16_to_float(uint16_t b) {
  _Float16 h = *reinterpret_cast<_Float16*>(&b);
  return (float)h;
}

// hi / lo parts of x in the packed type
__device__ __forceinline__ void split2(double x, int prec, uint16_t& hi, uint16_t& lo) {
  float xf = (float)x;
  if (prec == SKETCHNE_BF16) {
    hi = bf16_bits_rne(xf);
    lo = bf16_bits_rne((float)(x - (double)bf16_to_float(hi)));
  } else {
    hi = f16_bits(xf);
    lo = f16_bits((float)(x - (double)f16_to_float(hi)));
  }
}

// value at summation index kappa of an operand row in the sectioned layout
// (16*KSM main entries, then 16*KSS split entries, then, A side only, 16*KSS
// more); zero in the padding
__device__ __forceinline__ uint16_t sect_val(const double* row, double scale, int k, int r, int KSM, int KSS, int kappa,
                                             int prec, bool a_side) {
  int comp;
  bool want_lo;
  if (kappa < 16 * KSM) {
    comp = kappa < k ? kappa : -1;
    want_lo = false;
  } else if (kappa < 16 * (KSM + KSS)) {
    comp = kappa - 16 * KSM;
    comp = comp < r ? comp : -1;
    want_lo = !a_side;
  } else {
    comp = kappa - 16 * (KSM + KSS);
    comp = (a_side && comp < r) ? comp : -1;
    want_lo = true;
  }
  if (comp < 0) return 0;
  uint16_t hi, lo;
  split2(row[comp] * scale, prec, hi, lo);
  return want_lo ? lo : hi;
}

// map tile row i (0..31) of expanded-column tile rt to (group, member)
__device__ __forceinline__ void tile_row_to_group(int rt, int i, int& group, int& member) {
  group = 4 * rt + 2 * (i >> 4) + ((i >> 2) & 1);
  member = 4 * ((i >> 3) & 1) + (i & 3);
}

__global__ void k_degree_powers(int64_t n, const int64_t* __restrict__ rowptr, double alpha,
                                double* __restrict__ d1, double* __restrict__ d2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t deg = rowptr[i + 1] - rowptr[i];
  d1[i] = deg > 0 ? pow((double)deg, -1.0 + alpha) : 0.0;
  d2[i] = deg > 0 ? pow((double)deg, -1.0 + 2.0 * alpha) : 0.0;
}

// M(:, j) *= s[j]   (ld = cols)
__global__ void k_scale_cols(int rows, int cols, double* __restrict__ M, const double* __restrict__ s) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  M[idx] *= s[idx % cols];
}
// out(i, :) = s[i] * M(i, :)
__global__ void k_scale_rows(int rows, int cols, const double* __restrict__ M, const double* __restrict__ s,
                             double* __restrict__ out) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * cols) return;
  out[idx] = s[idx / cols] * M[idx];
}
__global__ void k_identity(int m, double* __restrict__ M) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  M[idx] = (idx / m == idx % m) ? 1.0 : 0.0;
}

// Rows of the expanded column matrix before the core product:
//   Gsel[rho][:] = scale * d1[p] * U[p][:], p = coordinate of expanded column rho
// (zero for padding; d1 == nullptr reads as 1).  rho runs over ntiles*32 rows
// in tile order.
__global__ void k_gather_expanded(int64_t n, int ntiles, int groups, int z, const int32_t* __restrict__ rows,
                                  const float* __restrict__ U, int64_t ldu, int k, const double* __restrict__ d1,
                                  double scale, double* __restrict__ Gsel, uint32_t* __restrict__ flags) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)ntiles * 32 * k;
  if (idx >= total) return;
  int rho = (int)(idx / k), col = (int)(idx % k);
  int rt = rho >> 5, i = rho & 31, g, t;
  tile_row_to_group(rt, i, g, t);
  double v = 0.0;
  if (g < groups && t < z) {
    int64_t p = rows[(int64_t)g * z + t];
    if (p >= 0 && p < n) v = scale * (d1 ? d1[p] : 1.0) * (double)U[p * ldu + col];
    else atomicOr(flags, SKETCHNE_FLAG_BAD_INDEX);
  }
  Gsel[idx] = v;
}

// whether eight packed 16-bit values are finite (an FP16 conversion that
// overflowed gives +-inf; BF16 keeps the FP32 exponent range)
template <int PREC>
__device__ __forceinline__ bool packed_finite(const uint16_t (&v)[8]) {
  const uint16_t expmask = PREC == SKETCHNE_FP16 ? 0x7c00 : 0x7f80;
  bool ok = true;
#pragma unroll
  for (int e = 0; e < 8; ++e) ok &= (v[e] & expmask) != expmask;
  return ok;
}

// A operand (expanded columns of R'), MFMA fragment order, KS = KSM + 2*KSS
// k-steps per tile (FP32: KSS = 0, no split).
//   RtT: (ntiles*32) x k FP64, row rho in tile order.
template <int PREC>
__global__ void k_pack_A(int ntiles, int KSM, int KSS, int k, int r, const double* __restrict__ RtT,
                         const double* __restrict__ pscale, void* __restrict__ out, uint32_t* __restrict__ flags) {
  constexpr int KSTEP = (PREC == SKETCHNE_FP32) ? 2 : 16;
  constexpr int E = (PREC == SKETCHNE_FP32) ? 1 : 8;
  const int KS = KSM + 2 * KSS;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one (tile, ks, lane)
  int64_t total = (int64_t)ntiles * KS * 64;
  if (idx >= total) return;
  int lane = (int)(idx & 63);
  int64_t q = idx >> 6;
  int ks = (int)(q % KS);
  int rt = (int)(q / KS);
  int rho = rt * 32 + (lane & 31);
  const double* row = RtT + (int64_t)rho * k;
  int kb = ks * KSTEP + (lane >> 5) * (KSTEP / 2);
  if (PREC == SKETCHNE_FP32) {
    static_cast<float*>(out)[idx] = kb < k ? (float)row[kb] : 0.0f;
  } else {
    const double sa = pscale[0];
    uint16_t v[8];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = sect_val(row, sa, k, r, KSM, KSS, kb + e, PREC, true);
    if (!packed_finite<PREC>(v)) atomicOr(flags, SKETCHNE_FLAG_NONFINITE);
    uint4 w;
    w.x = v[0] | ((uint32_t)v[1] << 16);
    w.y = v[2] | ((uint32_t)v[3] << 16);
    w.z = v[4] | ((uint32_t)v[5] << 16);
    w.w = v[6] | ((uint32_t)v[7] << 16);
    static_cast<uint4*>(out)[idx] = w;
  }
}

// B operand (rows of L' = D^(-1+a) U, optionally gathered; d1 == nullptr
// reads as 1, giving the rows of U itself), fragment order, KB = KSM + KSS
// k-steps per vertex tile (FP32: KSS = 0).
template <int PREC>
__global__ void k_pack_B(int64_t n, int64_t nrows, int64_t nvt, int KSM, int KSS, int k, int r,
                         const int32_t* __restrict__ gather, const float* __restrict__ U, int64_t ldu,
                         const double* __restrict__ d1, const double* __restrict__ pscale, void* __restrict__ out,
                         uint32_t* __restrict__ flags) {
  constexpr int KSTEP = (PREC == SKETCHNE_FP32) ? 2 : 16;
  constexpr int E = (PREC == SKETCHNE_FP32) ? 1 : 8;
  const int KS = KSM + KSS;
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = nvt * KS * 64;
  if (idx >= total) return;
  int lane = (int)(idx & 63);
  int64_t q = idx >> 6;
  int ks = (int)(q % KS);
  int64_t vt = q / KS;
  int64_t v = vt * 32 + (lane & 31);
  int kb = ks * KSTEP + (lane >> 5) * (KSTEP / 2);
  int64_t row = -1;
  if (v < nrows) row = gather ? (int64_t)gather[v] : v;
  if (row >= n) row = -1;
  if (v < nrows && row < 0 && (lane >> 5) == 0 && ks == 0) atomicOr(flags, SKETCHNE_FLAG_BAD_INDEX);
  if (PREC == SKETCHNE_FP32) {
    float val = 0.0f;
    if (row >= 0 && kb < k) val = (float)((d1 ? d1[row] : 1.0) * (double)U[row * ldu + kb]);
    static_cast<float*>(out)[idx] = val;
  } else {
    // the E = 8 summation indices kb .. kb+7 of this lane lie in one section
    // (sections are whole 16-wide k-steps): components comp0 .. comp0+7 of
    // the main part (hi, below k) or of the split part (lo, below r)
    const bool want_lo = kb >= 16 * KSM;
    const int comp0 = want_lo ? kb - 16 * KSM : kb;
    const int lim = want_lo ? r : k;
    uint16_t vv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (row >= 0 && comp0 < lim) {
      const double s = (d1 ? d1[row] : 1.0) * pscale[1];
      const float* src = U + row * ldu + comp0;
      float u[8];
      if (comp0 + 8 <= lim && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
        const float4 a = *reinterpret_cast<const float4*>(src);
        const float4 b = *reinterpret_cast<const float4*>(src + 4);
        u[0] = a.x; u[1] = a.y; u[2] = a.z; u[3] = a.w;
        u[4] = b.x; u[5] = b.y; u[6] = b.z; u[7] = b.w;
      } else {
#pragma unroll
        for (int e = 0; e < E; ++e) u[e] = comp0 + e < lim ? src[e] : 0.0f;
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (comp0 + e < lim) {
          uint16_t hi, lo;
          split2(s * (double)u[e], PREC, hi, lo);
          vv[e] = want_lo ? lo : hi;
        }
      }
    }
    if (!packed_finite<PREC>(vv)) atomicOr(flags, SKETCHNE_FLAG_NONFINITE);
    uint4 w;
    w.x = vv[0] | ((uint32_t)vv[1] << 16);
    w.y = vv[2] | ((uint32_t)vv[3] << 16);
    w.z = vv[4] | ((uint32_t)vv[5] << 16);
    w.w = vv[6] | ((uint32_t)vv[7] << 16);
    static_cast<uint4*>(out)[idx] = w;
  }
}

// Range balancing of the FP16 operands.  The product L'_i . R'(:, j) does not
// change when L' is multiplied by 2^e and R' by 2^-e, and power-of-two
// scaling is exact, but FP16 holds only |x| < 65504: R' carries the factor
// vol / (bT) (Eq. 11) and reaches about 3e5 on a graph of 2^20 vertices,
// while |L'_it| = d_i^(-1+a) |U_it| <= 1 (U has orthonormal columns and
// degrees are at least 1).  With M = max |R'| over the expanded columns,
// e = floor(log2(sqrt(M))) (clamped to [0, 15]) leaves both operands below
// sqrt(M) <= 65504 for M up to 4e9, and lifts the small entries of L' out of
// the FP16 subnormal range.  pscale = {2^-e (R' side), 2^e (L' side), M};
// BF16 and FP32 take e = 0 and skip the scan.  M is a grid-wide maximum: the
// bit patterns of non-negative doubles order as unsigned integers, so an
// integer atomic max over them is exact and independent of the order.
__global__ void k_balance_clear(double* __restrict__ pscale) {
  if (threadIdx.x == 0) pscale[2] = 0.0;
}

__global__ __launch_bounds__(256) void k_balance_max(int64_t count, const double* __restrict__ RtT,
                                                     double* __restrict__ pscale) {
  double m = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < count; i += 4 * stride)
    m = fmax(fmax(m, fabs(RtT[i])), fmax(fmax(fabs(RtT[i + stride]), fabs(RtT[i + 2 * stride])),
                                         fabs(RtT[i + 3 * stride])));
  for (; i < count; i += stride) m = fmax(m, fabs(RtT[i]));
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  // NaN compares false with everything: carry it as +inf so that it is seen
  if (m != m) m = __builtin_huge_val();
  if ((threadIdx.x & 63) == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(pscale + 2), (unsigned long long)__double_as_longlong(m));
}

__global__ void k_balance_finish(int prec, double* __restrict__ pscale) {
  if (threadIdx.x != 0) return;
  int e = 0;
  if (prec == SKETCHNE_FP16) {
    const double t = pscale[2];
    if (t > 1.0 && isfinite(t)) {
      e = (int)floor(0.5 * log2(t));
      e = e < 0 ? 0 : (e > 15 ? 15 : e);
    }
  }
  pscale[0] = ldexp(1.0, -e);
  pscale[1] = ldexp(1.0, e);
}

// signs in accumulator order: sgn[(rt*2 + hf)*16 + r] for lane half hf, register r
__global__ void k_pack_signs(int ntiles, int groups, int z, const int8_t* __restrict__ signs, float* __restrict__ sgn) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= ntiles * 32) return;
  int rt = idx >> 5, hf = (idx >> 4) & 1, r = idx & 15;
  int g = 4 * rt + 2 * (r >> 3) + hf;
  int t = r & 7;
  float s = 0.0f;
  if (g < groups && t < z) s = (float)signs[(int64_t)g * z + t];
  sgn[idx] = s;
}

template <int PREC>
struct MfmaOp;
template <>
struct MfmaOp<SKETCHNE_FP32> {
  typedef float frag;
  static constexpr int KSTEP = 2;
  static __device__ __forceinline__ floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfmaOp<SKETCHNE_BF16> {
  typedef bf16x8 frag;
  static constexpr int KSTEP = 16;
  static __device__ __forceinline__ floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfmaOp<SKETCHNE_FP16> {
  typedef halfx8 frag;
  static constexpr int KSTEP = 16;
  static __device__ __forceinline__ floatx16 mma(frag a, frag b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// Fused block GEMM + trunc_log + signed group sum.
//   8 wavefronts: wave w owns vertex tiles (w & 3) * VT .. +VT of the
//   workgroup's 4*VT tiles and, in each chunk of two expanded-column tiles,
//   the tile (w >> 2).  The chunk's A fragments are staged in LDS (double
//   buffered, next chunk prefetched through registers during the MFMAs).
//   out[g * ld_out + v] = out_scale * sum_t s_gt log2(max(x_{v, (g,t)}, 1))
template <int PREC, int VT, int KS>
__global__ __launch_bounds__(512) void k_fused_sketch(int64_t nrows, int groups, int ntiles,
                                                      const void* __restrict__ Bpack, const void* __restrict__ Apack,
                                                      const float* __restrict__ sgn, float* __restrict__ out,
                                                      int64_t ld_out, float out_scale) {
  typedef MfmaOp<PREC> Op;
  typedef typename Op::frag frag;
  constexpr int FB = sizeof(frag);
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int vg = wave & 3, rh = wave >> 2;
  const int64_t vt0 = (int64_t)blockIdx.x * (4 * VT) + vg * VT;

  // vertex fragments for the whole summation range, kept in registers
  frag bfr[VT][KS];
  const frag* Bp = static_cast<const frag*>(Bpack);
#pragma unroll
  for (int v = 0; v < VT; ++v)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) bfr[v][ks] = Bp[((vt0 + v) * KS + ks) * 64 + lane];

  constexpr int64_t chunk_bytes = (int64_t)2 * KS * 64 * FB;
  constexpr int nvec = (int)(chunk_bytes / 16);
  const int nchunks = (ntiles + 1) / 2;
  const char* Ag = static_cast<const char*>(Apack);
  const int64_t tile_bytes = (int64_t)KS * 64 * FB;
  const int64_t total_bytes = (int64_t)ntiles * tile_bytes;

  constexpr int MAXPRE = (nvec + 511) / 512;
  uint4 pre[MAXPRE];
  auto fetch = [&](int ch) {
#pragma unroll
    for (int u = 0; u < MAXPRE; ++u) {
      int vi = tid + u * 512;
      int64_t off = (int64_t)ch * 2 * tile_bytes + (int64_t)vi * 16;
      if (vi < nvec && off < total_bytes)
        pre[u] = *reinterpret_cast<const uint4*>(Ag + off);
      else
        pre[u] = make_uint4(0, 0, 0, 0);
    }
  };
  auto stash = [&](int buf) {
    char* dst = lds_raw + (int64_t)buf * chunk_bytes;
#pragma unroll
    for (int u = 0; u < MAXPRE; ++u) {
      int vi = tid + u * 512;
      if (vi < nvec) *reinterpret_cast<uint4*>(dst + (int64_t)vi * 16) = pre[u];
    }
  };

  fetch(0);
  stash(0);
  __syncthreads();
  int buf = 0;
  for (int ch = 0; ch < nchunks; ++ch) {
    const bool more = ch + 1 < nchunks;
    if (more) fetch(ch + 1);
    const int rt = 2 * ch + rh;
    if (rt < ntiles) {
      floatx16 acc[VT];
#pragma unroll
      for (int v = 0; v < VT; ++v)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[v][e] = 0.0f;
      const frag* Al = reinterpret_cast<const frag*>(lds_raw + (int64_t)buf * chunk_bytes) + (int64_t)rh * KS * 64;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        frag a = Al[ks * 64 + lane];
#pragma unroll
        for (int v = 0; v < VT; ++v) acc[v] = Op::mma(a, bfr[v][ks], acc[v]);
      }
      // the other buffer was last read before the previous barrier: refill it
      // now so the prefetch registers are free during the epilogue
      if (more) stash(buf ^ 1);
      // epilogue: trunc_log and signed group sums, finished in registers
      const float4* sp = reinterpret_cast<const float4*>(sgn + ((int64_t)rt * 2 + (lane >> 5)) * 16);
      float s[16];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        float4 t4 = sp[u];
        s[4 * u] = t4.x; s[4 * u + 1] = t4.y; s[4 * u + 2] = t4.z; s[4 * u + 3] = t4.w;
      }
      const int g0 = 4 * rt + (lane >> 5), g1 = g0 + 2;
#pragma unroll
      for (int v = 0; v < VT; ++v) {
        float y0 = 0.0f, y1 = 0.0f;
#pragma unroll
        for (int e = 0; e < 8; ++e) y0 = fmaf(s[e], __builtin_amdgcn_logf(fmaxf(acc[v][e], 1.0f)), y0);
#pragma unroll
        for (int e = 8; e < 16; ++e) y1 = fmaf(s[e], __builtin_amdgcn_logf(fmaxf(acc[v][e], 1.0f)), y1);
        const int64_t vert = (vt0 + v) * 32 + (lane & 31);
        if (vert < nrows) {
          if (g0 < groups) out[(int64_t)g0 * ld_out + vert] = out_scale * y0;
          if (g1 < groups) out[(int64_t)g1 * ld_out + vert] = out_scale * y1;
        }
      }
    }
    else if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
}

// Low-precision fused kernel (BF16 / FP16 operands, FP32 accumulation).
//   Workgroup: 4 wavefronts (one per SIMD; two workgroups share a CU), wave w
//   owns vertex tiles 2w, 2w+1 of the workgroup's 8 (256 vertices).  The
//   vertex fragments of the main section stay in registers for the whole
//   launch; the split-section (lo) fragments sit in the wave's LDS region.
//   All waves walk the same sequence of expanded-column tiles through three
//   LDS buffers: tile t+1 is copied global -> LDS by the LDS-DMA path (no
//   registers) while tile t is multiplied, then the trunc_log / signed group
//   sums of tile t run on the vector ALU; the two workgroups that share a CU
//   keep the matrix cores busy during each other's vector phases.  (A second
//   accumulator set that overlapped tile t-1's vector work with tile t's
//   MFMAs inside one wave left too few registers for reading the A
//   fragments ahead, and measured slower; so did two wave groups per
//   workgroup alternating the phases under barriers, and split-K chains.)
//   A buffer holds a tile's fragments and its 32 signs (register e of lane
//   half hf).  The loop is unrolled over the period 3 of the buffers, so every
//   LDS offset is a compile-time constant and the reads of the current buffer
//   never wait on the copy into the next one.  Results leave through buffer
//   stores whose descriptor covers exactly the tile's output rows, so rows
//   past `groups` and vertices past `nrows` are dropped by the hardware range
//   check.
//   out[g * ld_out + v] = out_scale * sum_t s_gt log2(max(x_{v, (g,t)}, 1))
typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t out_rsrc(const float* base, uint32_t bytes) {
  // wave-uniform by construction; readfirstlane keeps the descriptor scalar
  const uint64_t a = reinterpret_cast<uint64_t>(base);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  void* ptr = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  // dword 3 = 0x00020000: 32-bit data format, the raw-buffer setting of gfx9
  return __builtin_amdgcn_make_buffer_rsrc(ptr, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}

template <int N>
using cint = std::integral_constant<int, N>;


template <int PREC, int KSM, int KSS>
__global__ __launch_bounds__(256, 2) void k_fused_lowp(int64_t nrows, int groups, int ntiles, int tiles_per_block,
                                                       const void* __restrict__ Bpack, const void* Apack,
                                                       const float* __restrict__ sgn, float* out, int64_t ld_out,
                                                       float out_scale) {
  typedef MfmaOp<PREC> Op;
  typedef typename Op::frag frag;
  constexpr int VT = 2;
  constexpr int KS = KSM + 2 * KSS;  // A k-steps per tile
  constexpr int KB = KSM + KSS;      // B k-steps per vertex tile
  constexpr int TB = KS * 1024;      // bytes of one A tile
  // dynamic LDS: the three fragment buffers; separate static arrays hold each
  // buffer's signs and the split-section B fragments, so that the compiler
  // sees them as objects apart from the buffer being filled
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  __shared__ __attribute__((aligned(16))) float sg0[32], sg1[32], sg2[32];
  __shared__ __attribute__((aligned(16))) char blo_all[4 * VT * KSS * 1024 + 16];
  // wave index made visibly uniform, so that branches on it are scalar
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t vt0 = (int64_t)blockIdx.x * (4 * VT) + wave * VT;
  // this workgroup's expanded-column tiles: tb .. tb + nt - 1 (blockIdx.y splits
  // the tile range when there are too few vertex blocks to fill the chip)
  const int tb = blockIdx.y * tiles_per_block;
  const int nt = ntiles - tb < tiles_per_block ? ntiles - tb : tiles_per_block;
  if (nt <= 0) return;

  frag bfr[VT][KSM];
  const frag* Bp = static_cast<const frag*>(Bpack);
#pragma unroll
  for (int v = 0; v < VT; ++v)
#pragma unroll
    for (int ks = 0; ks < KSM; ++ks) bfr[v][ks] = Bp[((vt0 + v) * KB + ks) * 64 + lane];
  char* blo = blo_all + wave * (VT * KSS * 1024);
#pragma unroll
  for (int v = 0; v < VT; ++v)
#pragma unroll
    for (int j = 0; j < KSS; ++j)
      __builtin_amdgcn_global_load_lds((const void*)(Bp + ((vt0 + v) * KB + KSM + j) * 64 + lane),
                                       (lds_void*)(blo + (v * KSS + j) * 1024), 16, 0, 0);
  const frag* Blo = reinterpret_cast<const frag*>(blo);
  const char* Ag = static_cast<const char*>(Apack);
  auto signs_of = [&](auto Bc) -> float* {
    constexpr int B = decltype(Bc)::value;
    if constexpr (B == 0) return sg0;
    else if constexpr (B == 1) return sg1;
    else return sg2;
  };
  // tile t -> LDS buffer B: fragment c of the tile is one 1 KiB DMA by wave
  // c % 4, the 128 bytes of signs one DMA by eight lanes of wave 3
  // The copies are buffer (MUBUF) LDS-DMA loads, not global (FLAT) ones: the
  // compiler cannot tell whether a pending FLAT operation counts in lgkmcnt,
  // so with a global DMA in flight every wait for an LDS fragment read became
  // lgkmcnt(0), a full LDS round trip per four k-steps, instead of a count.
  const __amdgpu_buffer_rsrc_t a_rs = out_rsrc(reinterpret_cast<const float*>(Ag), (uint32_t)ntiles * (uint32_t)TB);
  const __amdgpu_buffer_rsrc_t s_rs = out_rsrc(sgn, (uint32_t)ntiles * 128u);
  auto dma = [&](int t, auto Bc) {
    constexpr int B = decltype(Bc)::value;
#pragma unroll
    for (int u = 0; u < (KS + 3) / 4; ++u) {
      const int c = u * 4 + wave;
      if (KS % 4 == 0 || c < KS)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(a_rs, (lds_void*)(lds_raw + B * TB + c * 1024), 16,
                                                 (uint32_t)(t * TB + c * 1024 + lane * 16), 0, 0, 0);
    }
    if (wave == 3 && lane < 8)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(s_rs, (lds_void*)signs_of(Bc), 16, (uint32_t)(t * 128 + lane * 16), 0,
                                               0, 0);
  };
  const int64_t vbase = vt0 * 32 + (lane & 31);
  floatx16 accC[VT];
  float yv[VT][2];
  // stores of finished tile tt (nothing for tt < 0): output rows 4tt .. 4tt+3
  auto store_tile = [&](int tt) {
    int64_t rows = (int64_t)groups - 4 * (int64_t)tt;
    rows = tt < 0 ? 0 : (rows < 4 ? rows : 4);
    const uint32_t nrec = (uint32_t)(rows * ld_out * 4);
    const __amdgpu_buffer_rsrc_t rs = out_rsrc(out + (int64_t)4 * (tt < 0 ? 0 : tt) * ld_out, nrec);
    const int r0 = lane >> 5;
#pragma unroll
    for (int v = 0; v < VT; ++v) {
      const int64_t vert = vbase + v * 32;
      const bool ok = vert < nrows;
      const uint32_t o0 = ok ? (uint32_t)((r0 * ld_out + vert) * 4) : nrec;
      const uint32_t o1 = ok ? (uint32_t)(((r0 + 2) * ld_out + vert) * 4) : nrec;
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(yv[v][0]), rs, o0, 0, 0);
      __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(yv[v][1]), rs, o1, 0, 0);
    }
  };
  // trunc_log and signed group sums: registers 0..7 form group 4tt + hf,
  // registers 8..15 group 4tt + 2 + hf; the signs of register e of this
  // lane half are entry hf * 16 + e of the tile's sign block, read four at a
  // time (all lanes of a half read the same 16 bytes)
  auto epilogue = [&](floatx16 (&acc)[VT], const float* signs) {
    const float4* sl = reinterpret_cast<const float4*>(signs + (lane >> 5) * 16);
    float y[VT][2];
#pragma unroll
    for (int v = 0; v < VT; ++v) y[v][0] = y[v][1] = 0.0f;
#pragma unroll
    for (int c4 = 0; c4 < 4; ++c4) {
      const float4 s4 = sl[c4];
      const float sv[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
      for (int v = 0; v < VT; ++v)
#pragma unroll
        for (int u = 0; u < 4; ++u)
          y[v][c4 >> 1] = fmaf(sv[u], fmaxf(__builtin_amdgcn_logf(acc[v][4 * c4 + u]), 0.0f), y[v][c4 >> 1]);
    }
#pragma unroll
    for (int v = 0; v < VT; ++v) {
      yv[v][0] = out_scale * y[v][0];
      yv[v][1] = out_scale * y[v][1];
    }
  };

  dma(tb, cint<0>());
#pragma unroll
  for (int v = 0; v < VT; ++v) yv[v][0] = yv[v][1] = 0.0f;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // step J of the period: stores of tile t-1, DMA of tile t+1 into buffer
  // (J+1) % 3, MFMAs of tile t (buffer J % 3), four A fragments read ahead,
  // then the epilogue of tile t (its signs in the same buffer)
  auto step = [&](auto Jc, int t) {
    constexpr int J = decltype(Jc)::value;
    store_tile(t >= 1 ? tb + t - 1 : -1);
    dma(tb + (t + 1 < nt ? t + 1 : nt - 1), cint<(J + 1) % 3>());
    __builtin_amdgcn_sched_barrier(0);
    const frag* Al = reinterpret_cast<const frag*>(lds_raw + (J % 3) * TB);
    const floatx16 zero = {};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const frag a = Al[ks * 64 + lane];
#pragma unroll
      for (int v = 0; v < VT; ++v) {
        frag b;
        if (ks < KSM) b = bfr[v][ks];
        else if (ks < KB) b = Blo[(v * KSS + ks - KSM) * 64 + lane];
        else b = bfr[v][ks - KB];
        accC[v] = Op::mma(a, b, ks == 0 ? zero : accC[v]);
      }
    }
    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
    for (int g = 0; g < KS; ++g) {
      __builtin_amdgcn_sched_group_barrier(0x008, VT, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_barrier(0);
    epilogue(accC, signs_of(cint<J % 3>()));
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  };
  int t = 0;
  for (; t + 3 <= nt; t += 3) {
    step(cint<0>(), t);
    step(cint<1>(), t + 1);
    step(cint<2>(), t + 2);
  }
  const int rem = nt - t;
  if (rem > 0) step(cint<0>(), t);
  if (rem > 1) step(cint<1>(), t + 1);
  store_tile(tb + nt - 1);
}

// Z[c'][c] = inv_sqrt_z * sum_t s_{c't} * T1t[c][c' z + t]
__global__ void k_z_reduce(int l, int z, const int8_t* __restrict__ signs, const float* __restrict__ T1t,
                           int64_t ld_t1, float inv_sqrt_z, float* __restrict__ Z) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)l * l) return;
  int cp = (int)(idx / l), c = (int)(idx % l);
  float s = 0.0f;
  for (int t = 0; t < z; ++t) s = fmaf((float)signs[(int64_t)cp * z + t], T1t[(int64_t)c * ld_t1 + (int64_t)cp * z + t], s);
  Z[idx] = inv_sqrt_z * s;
}

// B = O^T Q with Q given transposed (Qt: cols x n):  B[c][j] = inv_sqrt_z sum_t s_ct Qt[j][p_ct]
__global__ void k_ot_q(int l, int z, int hcols, const int32_t* __restrict__ rows, const int8_t* __restrict__ signs,
                       const float* __restrict__ Qt, int64_t n, double inv_sqrt_z, double* __restrict__ Bm,
                       uint32_t* __restrict__ flags) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)l * hcols) return;
  int c = (int)(idx / hcols), j = (int)(idx % hcols);
  double s = 0.0;
  for (int t = 0; t < z; ++t) {
    int64_t p = rows[(int64_t)c * z + t];
    if (p < 0 || p >= n) { atomicOr(flags, SKETCHNE_FLAG_BAD_INDEX); continue; }
    s += (double)signs[(int64_t)c * z + t] * (double)Qt[(int64_t)j * n + p];
  }
  Bm[idx] = inv_sqrt_z * s;
}

template <int PREC, int VT, int KS>
sketchne_status launch_fused(sketchne_ctx* c, int cls, int64_t nrows, int groups, int ntiles, const void* Bpack,
                             const void* Apack, const float* sgn, float* out, int64_t ld_out, float out_scale) {
  typedef typename MfmaOp<PREC>::frag frag;
  size_t shmem = (size_t)2 * 2 * KS * 64 * sizeof(frag);
  int64_t nvt = (nrows + 31) / 32;
  int64_t blocks = (nvt + 4 * VT - 1) / (4 * VT);
  auto kern = k_fused_sketch<PREC, VT, KS>;
  hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  ProfScope ps(c, cls);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(512), shmem, c->stream, nrows, groups, ntiles, Bpack, Apack,
                     sgn, out, ld_out, out_scale);
  return launch_status();
}

template <int PREC, int KSM, int KSS>
sketchne_status launch_lowp(sketchne_ctx* c, int cls, int64_t nrows, int groups, int ntiles, const void* Bpack,
                            const void* Apack, const float* sgn, float* out, int64_t ld_out, float out_scale) {
  constexpr int KS = KSM + 2 * KSS;
  const size_t shmem = (size_t)3 * KS * 1024;  // plus the kernel's static signs and split fragments
  const int64_t nvt = (nrows + 31) / 32;
  const int64_t blocks = (nvt + 7) / 8;
  // few vertex blocks (the Z pass): split the tile range so that about 1024
  // workgroups run, keeping at least 8 tiles per workgroup
  int64_t ysplit = (1024 + blocks - 1) / blocks;
  const int64_t ymax = ntiles / 8 > 1 ? ntiles / 8 : 1;
  ysplit = ysplit < ymax ? ysplit : ymax;
  const int tpb = (int)((ntiles + ysplit - 1) / ysplit);
  const int64_t ny = (ntiles + tpb - 1) / tpb;
  auto kern = k_fused_lowp<PREC, KSM, KSS>;
  hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
  ProfScope ps(c, cls);
  hipLaunchKernelGGL(kern, dim3((unsigned)blocks, (unsigned)ny), dim3(256), shmem, c->stream, nrows, groups, ntiles,
                     tpb, Bpack, Apack, sgn, out, ld_out, out_scale);
  return launch_status();
}

template <int PREC>
sketchne_status fused_lowp(sketchne_ctx* c, int cls, int64_t nrows, int groups, int ntiles, int KSM, int KSS,
                           const void* Bpack, const void* Apack, const float* sgn, float* out, int64_t ld_out,
                           float out_scale) {
#define SK_LOWP(m, s)                                                                                             \
  if (KSM == m && KSS == s)                                                                                       \
    return launch_lowp<PREC, m, s>(c, cls, nrows, groups, ntiles, Bpack, Apack, sgn, out, ld_out, out_scale);
  SK_LOWP(8, 0) SK_LOWP(8, 1) SK_LOWP(8, 2) SK_LOWP(16, 0) SK_LOWP(16, 1) SK_LOWP(16, 2)
#undef SK_LOWP
  return SKETCHNE_E_UNSUPPORTED;
}

}  // namespace

// ---------------------------------------------------------------- launchers

int sketch_kstep(int prec) { return prec == SKETCHNE_FP32 ? 2 : 16; }
int sketch_frag_bytes(int prec) { return prec == SKETCHNE_FP32 ? 4 : 16; }
int sketch_vt(int prec) { return prec == SKETCHNE_FP32 ? 1 : 2; }

// k-step sections with a compiled kernel (each section zero-padded up to the
// next one): FP32 KSM in {32, 64, 128} steps of 2, KSS = 0; BF16/FP16 KSM in
// {8, 16} steps of 16 (k <= 256) and KSS = ceil(r/16) <= 2 (r <= 32).
// Returns false when k or r is beyond them.
bool sketch_sections(int prec, int k, int r, int* KSM, int* KSS) {
  if (prec == SKETCHNE_FP32) {
    static const int f32[] = {32, 64, 128};
    const int need = (k + 1) / 2;
    for (int v : f32)
      if (need <= v) { *KSM = v; *KSS = 0; return true; }
    return false;
  }
  const int need = (k + 15) / 16;
  const int kss = (r + 15) / 16;
  if (need > 16 || kss > 2) return false;
  *KSM = need <= 8 ? 8 : 16;
  *KSS = kss;
  return true;
}

sketchne_status degree_powers(sketchne_ctx* c, int64_t n, const int64_t* rowptr, double alpha, double* d1,
                              double* d2) {
  if (n == 0) return SKETCHNE_OK;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  hipLaunchKernelGGL(k_degree_powers, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, rowptr, alpha,
                     d1, d2);
  return launch_status();
}

sketchne_status scale_cols(sketchne_ctx* c, int rows, int cols, double* M, const double* s) {
  int tot = rows * cols;
  hipLaunchKernelGGL(k_scale_cols, dim3((tot + 255) / 256), dim3(256), 0, c->stream, rows, cols, M, s);
  return launch_status();
}
sketchne_status scale_rows(sketchne_ctx* c, int rows, int cols, const double* M, const double* s, double* out) {
  int tot = rows * cols;
  hipLaunchKernelGGL(k_scale_rows, dim3((tot + 255) / 256), dim3(256), 0, c->stream, rows, cols, M, s, out);
  return launch_status();
}
sketchne_status identity(sketchne_ctx* c, int m, double* M) {
  hipLaunchKernelGGL(k_identity, dim3((m * m + 255) / 256), dim3(256), 0, c->stream, m, M);
  return launch_status();
}

sketchne_status gather_expanded(sketchne_ctx* c, int64_t n, int ntiles, int groups, int z, const int32_t* rows,
                                const float* U, int64_t ldu, int k, const double* d1, double scale, double* Gsel) {
  int64_t tot = (int64_t)ntiles * 32 * k;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  hipLaunchKernelGGL(k_gather_expanded, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, n, ntiles,
                     groups, z, rows, U, ldu, k, d1, scale, Gsel, c->d_flags);
  return launch_status();
}

sketchne_status balance(sketchne_ctx* c, int prec, int64_t count, const double* RtT, double* pscale) {
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  if (prec == SKETCHNE_FP16 && count > 0) {
    hipLaunchKernelGGL(k_balance_clear, dim3(1), dim3(64), 0, c->stream, pscale);
    int64_t blocks = (count + 4 * 256 - 1) / (4 * 256);
    blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
    hipLaunchKernelGGL(k_balance_max, dim3((unsigned)blocks), dim3(256), 0, c->stream, count, RtT, pscale);
  }
  hipLaunchKernelGGL(k_balance_finish, dim3(1), dim3(64), 0, c->stream, prec, pscale);
  return launch_status();
}

sketchne_status pack_A(sketchne_ctx* c, int prec, int ntiles, int KSM, int KSS, int k, int r, const double* RtT,
                       const double* pscale, void* out) {
  int64_t tot = (int64_t)ntiles * (KSM + 2 * KSS) * 64;
  unsigned blocks = (unsigned)((tot + 255) / 256);
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  if (prec == SKETCHNE_FP32)
    hipLaunchKernelGGL(k_pack_A<SKETCHNE_FP32>, dim3(blocks), dim3(256), 0, c->stream, ntiles, KSM, KSS, k, r, RtT,
                       pscale, out, c->d_flags);
  else if (prec == SKETCHNE_BF16)
    hipLaunchKernelGGL(k_pack_A<SKETCHNE_BF16>, dim3(blocks), dim3(256), 0, c->stream, ntiles, KSM, KSS, k, r, RtT,
                       pscale, out, c->d_flags);
  else
    hipLaunchKernelGGL(k_pack_A<SKETCHNE_FP16>, dim3(blocks), dim3(256), 0, c->stream, ntiles, KSM, KSS, k, r, RtT,
                       pscale, out, c->d_flags);
  return launch_status();
}

sketchne_status pack_B(sketchne_ctx* c, int prec, int64_t n, int64_t nrows, int64_t nvt, int KSM, int KSS, int k,
                       int r, const int32_t* gather, const float* U, int64_t ldu, const double* d1, const double* pscale,
                       void* out) {
  int64_t tot = nvt * (KSM + KSS) * 64;
  unsigned blocks = (unsigned)((tot + 255) / 256);
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  if (prec == SKETCHNE_FP32)
    hipLaunchKernelGGL(k_pack_B<SKETCHNE_FP32>, dim3(blocks), dim3(256), 0, c->stream, n, nrows, nvt, KSM, KSS, k, r,
                       gather, U, ldu, d1, pscale, out, c->d_flags);
  else if (prec == SKETCHNE_BF16)
    hipLaunchKernelGGL(k_pack_B<SKETCHNE_BF16>, dim3(blocks), dim3(256), 0, c->stream, n, nrows, nvt, KSM, KSS, k, r,
                       gather, U, ldu, d1, pscale, out, c->d_flags);
  else
    hipLaunchKernelGGL(k_pack_B<SKETCHNE_FP16>, dim3(blocks), dim3(256), 0, c->stream, n, nrows, nvt, KSM, KSS, k, r,
                       gather, U, ldu, d1, pscale, out, c->d_flags);
  return launch_status();
}

sketchne_status pack_signs(sketchne_ctx* c, int ntiles, int groups, int z, const int8_t* signs, float* sgn) {
  int tot = ntiles * 32;
  hipLaunchKernelGGL(k_pack_signs, dim3((tot + 255) / 256), dim3(256), 0, c->stream, ntiles, groups, z, signs, sgn);
  return launch_status();
}

sketchne_status fused_sketch(sketchne_ctx* c, int cls, int prec, int64_t nrows, int groups, int ntiles, int KSM,
                             int KSS, const void* Bpack, const void* Apack, const float* sgn, float* out,
                             int64_t ld_out, float out_scale) {
  if (nrows == 0 || groups == 0) return SKETCHNE_OK;
  if (prec == SKETCHNE_FP32) {
    switch (KSM) {
      case 32:
        return launch_fused<SKETCHNE_FP32, 1, 32>(c, cls, nrows, groups, ntiles, Bpack, Apack, sgn, out, ld_out,
                                                  out_scale);
      case 64:
        return launch_fused<SKETCHNE_FP32, 1, 64>(c, cls, nrows, groups, ntiles, Bpack, Apack, sgn, out, ld_out,
                                                  out_scale);
      case 128:
        return launch_fused<SKETCHNE_FP32, 1, 128>(c, cls, nrows, groups, ntiles, Bpack, Apack, sgn, out, ld_out,
                                                   out_scale);
    }
    return SKETCHNE_E_UNSUPPORTED;
  }
  // the buffer descriptor of one tile's four output rows holds < 2^32 bytes,
  // and the tile copies address the packed columns with 32-bit offsets
  if (ld_out >= ((int64_t)1 << 28)) return SKETCHNE_E_UNSUPPORTED;
  if ((int64_t)ntiles * (KSM + 2 * KSS) * 1024 >= ((int64_t)1 << 31)) return SKETCHNE_E_UNSUPPORTED;
  if (prec == SKETCHNE_BF16)
    return fused_lowp<SKETCHNE_BF16>(c, cls, nrows, groups, ntiles, KSM, KSS, Bpack, Apack, sgn, out, ld_out,
                                     out_scale);
  return fused_lowp<SKETCHNE_FP16>(c, cls, nrows, groups, ntiles, KSM, KSS, Bpack, Apack, sgn, out, ld_out,
                                   out_scale);
}

sketchne_status z_reduce(sketchne_ctx* c, int l, int z, const int8_t* signs, const float* T1t, int64_t ld_t1,
                         float inv_sqrt_z, float* Z) {
  int64_t tot = (int64_t)l * l;
  ProfScope ps(c, SKETCHNE_PROF_SKETCH_Z);
  hipLaunchKernelGGL(k_z_reduce, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, l, z, signs, T1t, ld_t1,
                     inv_sqrt_z, Z);
  return launch_status();
}

sketchne_status ot_q(sketchne_ctx* c, int l, int z, int hcols, const int32_t* rows, const int8_t* signs,
                     const float* Qt, int64_t n, double inv_sqrt_z, double* Bm) {
  int64_t tot = (int64_t)l * hcols;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  hipLaunchKernelGGL(k_ot_q, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, l, z, hcols, rows, signs,
                     Qt, n, inv_sqrt_z, Bm, c->d_flags);
  return launch_status();
}

}  // namespace skne
