// Counter-based random draws on the device.
//
// Each value is SplitMix64's output function (Steele, Lea & Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014) applied to
// the state seed + gamma * (counter + 1): the counter-th output of a SplitMix64
// generator, computable independently per thread.  Independent streams use
// seeds derived by mixing the user seed with a stream constant.
#include "internal.h"

namespace skne {
namespace {

constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ULL;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t ctr) {
  return mix64(seed + kGamma * (ctr + 1));
}

// Box-Muller in FP32: one pair of uniforms gives two normals, written to
// consecutive elements 2e and 2e+1 of the row-major block.
__global__ void k_gauss(int64_t n, int cols, int64_t ld, uint64_t seed, double inv_cols, float* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = n * cols;
  int64_t i0 = 2 * e;
  if (i0 >= total) return;
  uint64_t s = mix64(seed ^ 0x6a09e667f3bcc909ULL);
  uint64_t r = draw(s, (uint64_t)e);
  // two 32-bit uniforms in (0, 1]
  float u1 = ((float)((uint32_t)(r >> 40)) + 1.0f) * (1.0f / 16777216.0f);
  float u2 = (float)((uint32_t)(r >> 8) & 0xffffffu) * (1.0f / 16777216.0f);
  // Box-Muller on the hardware transcendentals: log2, and sin / cos of an
  // angle given in revolutions (u2 in [0, 1))
  const float rad = __builtin_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));  // -2 ln 2 log2(u1)
  const float sn = __builtin_amdgcn_sinf(u2), cs = __builtin_amdgcn_cosf(u2);
  // row a = i0 / cols from an FP64 quotient (exact below 2^53) corrected by
  // one step either way, instead of a 64-bit integer division
  int64_t a = (int64_t)((double)i0 * inv_cols);
  if (a * cols > i0) --a;
  else if ((a + 1) * cols <= i0) ++a;
  int b = (int)(i0 - a * cols);
  out[a * ld + b] = rad * cs;
  if (i0 + 1 < total) {
    if (++b == cols) { b = 0; ++a; }
    out[a * ld + b] = rad * sn;
  }
}

// Even column counts: pair e = a cols / 2 + b / 2 lies in row a, so one thread
// takes four pairs of a row (columns 8q .. 8q+7) with the same counters and
// positions as k_gauss, the row found once and the SplitMix64 states stepped
// by gamma instead of multiplied.
__global__ void k_gauss_row8(int64_t n, int cols, int64_t ld, uint64_t seed, int chunks, double inv_chunks,
                             float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * chunks) return;
  int64_t a = (int64_t)((double)t * inv_chunks);
  if (a * chunks > t) --a;
  else if ((a + 1) * chunks <= t) ++a;
  const int b0 = 8 * (int)(t - a * chunks);
  const uint64_t s = mix64(seed ^ 0x6a09e667f3bcc909ULL);
  const uint64_t e0 = (uint64_t)a * (uint64_t)(cols / 2) + (uint64_t)(b0 / 2);
  uint64_t state = s + kGamma * (e0 + 1);
  float v[8];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const uint64_t r = mix64(state);
    state += kGamma;
    const float u1 = ((float)((uint32_t)(r >> 40)) + 1.0f) * (1.0f / 16777216.0f);
    const float u2 = (float)((uint32_t)(r >> 8) & 0xffffffu) * (1.0f / 16777216.0f);
    const float rad = __builtin_sqrtf(-1.38629436111989061883f * __builtin_amdgcn_logf(u1));
    v[2 * p] = rad * __builtin_amdgcn_cosf(u2);
    v[2 * p + 1] = rad * __builtin_amdgcn_sinf(u2);
  }
  float* o = out + a * ld + b0;
  if (b0 + 8 <= cols && (reinterpret_cast<uintptr_t>(o) & 15) == 0) {
    reinterpret_cast<float4*>(o)[0] = make_float4(v[0], v[1], v[2], v[3]);
    reinterpret_cast<float4*>(o)[1] = make_float4(v[4], v[5], v[6], v[7]);
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (b0 + u < cols) o[u] = v[u];
  }
}

// One thread per column: z distinct rows uniformly from [0, n), independent
// fair signs.  A duplicate is redrawn with a fresh counter; after a bounded
// number of redraws the next free row (cyclically) is taken, which keeps the
// loop finite for z close to n.
__global__ void k_sparse_sign(int64_t n, int cols, int z, uint64_t seed,
                              int32_t* __restrict__ rows, int8_t* __restrict__ signs) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  uint64_t s = mix64(seed ^ 0xbb67ae8584caa73bULL);
  uint64_t base = (uint64_t)c * (uint64_t)z * 64u;
  int32_t* rc = rows + (int64_t)c * z;
  for (int t = 0; t < z; ++t) {
    int64_t r = 0;
    bool ok = false;
    for (int a = 0; a < 32 && !ok; ++a) {
      uint64_t x = draw(s, base + (uint64_t)t * 32u + a);
      r = (int64_t)__umul64hi(x, (uint64_t)n);
      ok = true;
      for (int u = 0; u < t; ++u) ok = ok && (rc[u] != r);
    }
    while (!ok) {  // deterministic fallback: next unused row
      r = (r + 1) % n;
      ok = true;
      for (int u = 0; u < t; ++u) ok = ok && (rc[u] != r);
    }
    rc[t] = (int32_t)r;
    uint64_t y = draw(s ^ 0x3c6ef372fe94f82bULL, (uint64_t)c * z + t);
    signs[(int64_t)c * z + t] = (y >> 63) ? (int8_t)1 : (int8_t)-1;
  }
}

// out[i] = +1 or -1 with probability 1/2 each (top bit of draw i)
__global__ void k_rademacher(int64_t n, uint64_t seed, float* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t s = mix64(seed ^ 0xa54ff53a5f1d36f1ULL);
  out[i] = (draw(s, (uint64_t)i) >> 63) ? 1.f : -1.f;
}

}  // namespace

sketchne_status gen_rademacher(sketchne_ctx* c, int64_t n, uint64_t seed, float* out) {
  if (n == 0) return SKETCHNE_OK;
  hipLaunchKernelGGL(k_rademacher, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, seed, out);
  return launch_status();
}

sketchne_status gen_gauss(sketchne_ctx* c, int64_t n, int cols, int64_t ld, uint64_t seed, float* out) {
  int64_t total = n * cols;
  if (total == 0) return SKETCHNE_OK;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  if (cols % 2 == 0) {
    const int chunks = (cols + 7) / 8;
    const int64_t blocks = (n * chunks + 255) / 256;
    hipLaunchKernelGGL(k_gauss_row8, dim3((unsigned)blocks), dim3(256), 0, c->stream, n, cols, ld, seed, chunks,
                       1.0 / chunks, out);
    return launch_status();
  }
  int64_t blocks = ((total + 1) / 2 + 255) / 256;
  hipLaunchKernelGGL(k_gauss, dim3((unsigned)blocks), dim3(256), 0, c->stream, n, cols, ld, seed, 1.0 / cols, out);
  return launch_status();
}

sketchne_status gen_sparse_sign(sketchne_ctx* c, int64_t n, int cols, int z, uint64_t seed,
                                int32_t* rows, int8_t* signs) {
  if (cols == 0) return SKETCHNE_OK;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  hipLaunchKernelGGL(k_sparse_sign, dim3((cols + 127) / 128), dim3(128), 0, c->stream, n, cols, z,
                     seed, rows, signs);
  return launch_status();
}

}  // namespace skne
