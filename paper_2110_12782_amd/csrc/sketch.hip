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
// BF16/FP16 forms the first split_r components are carried as hi + lo pairs:
// the summation index is extended to k + 2r with A = [hi | hi(:r) | lo(:r)]
// and B = [hi | lo(:r) | hi(:r)], so the GEMM computes
// hi.hi + hi.lo + lo.hi on the dominant components in one pass.
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

// value of extended column kappa of an operand row, as hi/lo selection
//   A side (R~): [hi(0..k) | hi(0..r) | lo(0..r)]
//   B side (L'): [hi(0..k) | lo(0..r) | hi(0..r)]
__device__ __forceinline__ uint16_t ext_val(const double* row, int k, int r, int kappa, int prec, bool a_side) {
  if (kappa >= k + 2 * r) return 0;
  int comp;
  bool want_lo;
  if (kappa < k) { comp = kappa; want_lo = false; }
  else if (kappa < k + r) { comp = kappa - k; want_lo = !a_side; }
  else { comp = kappa - k - r; want_lo = a_side; }
  uint16_t hi, lo;
  split2(row[comp], prec, hi, lo);
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
// (zero for padding).  rho runs over ntiles*32 rows in tile order.
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
    if (p >= 0 && p < n) v = scale * d1[p] * (double)U[p * ldu + col];
    else atomicOr(flags, SKETCHNE_FLAG_BAD_INDEX);
  }
  Gsel[idx] = v;
}

// A operand (expanded columns of R'), MFMA fragment order.
//   RtT: (ntiles*32) x k FP64, row rho in tile order.
template <int PREC>
__global__ void k_pack_A(int ntiles, int KS, int k, int r, const double* __restrict__ RtT, void* __restrict__ out) {
  constexpr int KSTEP = (PREC == SKETCHNE_FP32) ? 2 : 16;
  constexpr int E = (PREC == SKETCHNE_FP32) ? 1 : 8;
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
    uint16_t v[8];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = ext_val(row, k, r, kb + e, PREC, true);
    uint4 w;
    w.x = v[0] | ((uint32_t)v[1] << 16);
    w.y = v[2] | ((uint32_t)v[3] << 16);
    w.z = v[4] | ((uint32_t)v[5] << 16);
    w.w = v[6] | ((uint32_t)v[7] << 16);
    static_cast<uint4*>(out)[idx] = w;
  }
}

// B operand (rows of L' = D^(-1+a) U, optionally gathered), fragment order.
template <int PREC>
__global__ void k_pack_B(int64_t n, int64_t nrows, int64_t nvt, int KS, int k, int r,
                         const int32_t* __restrict__ gather, const float* __restrict__ U, int64_t ldu,
                         const double* __restrict__ d1, void* __restrict__ out, uint32_t* __restrict__ flags) {
  constexpr int KSTEP = (PREC == SKETCHNE_FP32) ? 2 : 16;
  constexpr int E = (PREC == SKETCHNE_FP32) ? 1 : 8;
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
    if (row >= 0 && kb < k) val = (float)(d1[row] * (double)U[row * ldu + kb]);
    static_cast<float*>(out)[idx] = val;
  } else {
    double rowv[1];
    (void)rowv;
    uint16_t vv[8];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      vv[e] = 0;
      if (row >= 0) {
        int kappa = kb + e;
        int comp;
        bool want_lo;
        if (kappa < k) { comp = kappa; want_lo = false; }
        else if (kappa < k + r) { comp = kappa - k; want_lo = true; }
        else if (kappa < k + 2 * r) { comp = kappa - k - r; want_lo = false; }
        else { comp = -1; want_lo = false; }
        if (comp >= 0) {
          uint16_t hi, lo;
          split2(d1[row] * (double)U[row * ldu + comp], PREC, hi, lo);
          vv[e] = want_lo ? lo : hi;
        }
      }
    }
    uint4 w;
    w.x = vv[0] | ((uint32_t)vv[1] << 16);
    w.y = vv[2] | ((uint32_t)vv[3] << 16);
    w.z = vv[4] | ((uint32_t)vv[5] << 16);
    w.w = vv[6] | ((uint32_t)vv[7] << 16);
    static_cast<uint4*>(out)[idx] = w;
  }
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

template <int PREC>
sketchne_status fused_lowp(sketchne_ctx* c, int cls, int64_t nrows, int groups, int ntiles, int KS, const void* Bpack,
                           const void* Apack, const float* sgn, float* out, int64_t ld_out, float out_scale) {
  switch (KS) {
    case 8: return launch_fused<PREC, 2, 8>(c, cls, nrows, groups, ntiles, Bpack, Apack, sgn, out, ld_out, out_scale);
    case 12: return launch_fused<PREC, 2, 12>(c, cls, nrows, groups, ntiles, Bpack, Apack, sgn, out, ld_out, out_scale);
    case 16: return launch_fused<PREC, 2, 16>(c, cls, nrows, groups, ntiles, Bpack, Apack, sgn, out, ld_out, out_scale);
    case 20: return launch_fused<PREC, 2, 20>(c, cls, nrows, groups, ntiles, Bpack, Apack, sgn, out, ld_out, out_scale);
  }
  return SKETCHNE_E_UNSUPPORTED;
}

}  // namespace

// ---------------------------------------------------------------- launchers

int sketch_kstep(int prec) { return prec == SKETCHNE_FP32 ? 2 : 16; }
int sketch_frag_bytes(int prec) { return prec == SKETCHNE_FP32 ? 4 : 16; }
int sketch_vt(int prec) { return prec == SKETCHNE_FP32 ? 1 : 2; }

// k-step counts with a compiled kernel; the summation range is zero-padded up
// to the next one (0 if the range is too long)
int sketch_ks_supported(int prec, int ks_needed) {
  static const int f32[] = {32, 64, 128};
  static const int lowp[] = {8, 12, 16, 20};
  if (prec == SKETCHNE_FP32) {
    for (int v : f32) if (ks_needed <= v) return v;
  } else {
    for (int v : lowp) if (ks_needed <= v) return v;
  }
  return 0;
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

sketchne_status pack_A(sketchne_ctx* c, int prec, int ntiles, int KS, int k, int r, const double* RtT, void* out) {
  int64_t tot = (int64_t)ntiles * KS * 64;
  unsigned blocks = (unsigned)((tot + 255) / 256);
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  if (prec == SKETCHNE_FP32)
    hipLaunchKernelGGL(k_pack_A<SKETCHNE_FP32>, dim3(blocks), dim3(256), 0, c->stream, ntiles, KS, k, r, RtT, out);
  else if (prec == SKETCHNE_BF16)
    hipLaunchKernelGGL(k_pack_A<SKETCHNE_BF16>, dim3(blocks), dim3(256), 0, c->stream, ntiles, KS, k, r, RtT, out);
  else
    hipLaunchKernelGGL(k_pack_A<SKETCHNE_FP16>, dim3(blocks), dim3(256), 0, c->stream, ntiles, KS, k, r, RtT, out);
  return launch_status();
}

sketchne_status pack_B(sketchne_ctx* c, int prec, int64_t n, int64_t nrows, int64_t nvt, int KS, int k, int r,
                       const int32_t* gather, const float* U, int64_t ldu, const double* d1, void* out) {
  int64_t tot = nvt * KS * 64;
  unsigned blocks = (unsigned)((tot + 255) / 256);
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  if (prec == SKETCHNE_FP32)
    hipLaunchKernelGGL(k_pack_B<SKETCHNE_FP32>, dim3(blocks), dim3(256), 0, c->stream, n, nrows, nvt, KS, k, r,
                       gather, U, ldu, d1, out, c->d_flags);
  else if (prec == SKETCHNE_BF16)
    hipLaunchKernelGGL(k_pack_B<SKETCHNE_BF16>, dim3(blocks), dim3(256), 0, c->stream, n, nrows, nvt, KS, k, r,
                       gather, U, ldu, d1, out, c->d_flags);
  else
    hipLaunchKernelGGL(k_pack_B<SKETCHNE_FP16>, dim3(blocks), dim3(256), 0, c->stream, n, nrows, nvt, KS, k, r,
                       gather, U, ldu, d1, out, c->d_flags);
  return launch_status();
}

sketchne_status pack_signs(sketchne_ctx* c, int ntiles, int groups, int z, const int8_t* signs, float* sgn) {
  int tot = ntiles * 32;
  hipLaunchKernelGGL(k_pack_signs, dim3((tot + 255) / 256), dim3(256), 0, c->stream, ntiles, groups, z, signs, sgn);
  return launch_status();
}

sketchne_status fused_sketch(sketchne_ctx* c, int cls, int prec, int64_t nrows, int groups, int ntiles, int KS,
                             const void* Bpack, const void* Apack, const float* sgn, float* out, int64_t ld_out,
                             float out_scale) {
  if (nrows == 0 || groups == 0) return SKETCHNE_OK;
  if (prec == SKETCHNE_FP32) {
    switch (KS) {
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
  if (prec == SKETCHNE_BF16)
    return fused_lowp<SKETCHNE_BF16>(c, cls, nrows, groups, ntiles, KS, Bpack, Apack, sgn, out, ld_out, out_scale);
  return fused_lowp<SKETCHNE_FP16>(c, cls, nrows, groups, ntiles, KS, Bpack, Apack, sgn, out, ld_out, out_scale);
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
