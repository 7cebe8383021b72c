// Spectral propagation (Alg. 6 line 6): E_out = sum_{r=0..p} c_r T_r(M) E with
// M = L - I = -D^-1 A, L = I - D^-1 A the random-walk Laplacian and T_r the
// Chebyshev polynomials of the first kind.  M has its spectrum in [-1, 1],
// where the three-term recurrence
//     T_0 E = E,  T_1 E = M E,  T_{r+1} E = 2 M T_r E - T_{r-1} E
// is stable.  Each step is one CSR SpMM fused with the recurrence and the
// running sum: row i of the step's output is
//     t_i = s_i * sum_{j in N(i)} T_r[j] - T_{r-1}[i],   s_i = -2 / deg_i
// (s_i = -1 / deg_i and no T_{r-1} term for the first step), and
// out_i += c_{r+1} t_i.  T_{r+1} overwrites T_{r-1} in place: row i of
// T_{r-1} is read only by the lanes that then write row i of T_{r+1}.
//
// Work split as in the eigensolver's SpMM: fixed slices of kP stored entries
// per wavefront, rows crossing a slice boundary summed by a fixup in slice
// order (deterministic, no atomics).  A row of d <= 256 FP32 values is
// covered by d / 4 lanes in float4 chunks; the 64 lanes of a wavefront form
// 64 / LPS slots (LPS = lanes per slot, a power of two >= d / 4) that walk
// alternate neighbours of the same row, combined by xor shuffles, so a
// 128-column block keeps both halves of the wavefront gathering.
// An isolated vertex (no stored entries) has a zero row in M: its t_i is
// -T_{r-1}[i] (0 for the first step).
#include "internal.h"

namespace skne {
namespace {

constexpr int kP = 256;  // stored entries per wavefront slice

__device__ __forceinline__ int64_t row_of(const int64_t* __restrict__ rowptr, int64_t n, int64_t e) {
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (rowptr[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void k_prop_bounds(int64_t n, const int64_t* __restrict__ rowptr, int64_t nwaves,
                              int64_t* __restrict__ brow) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwaves) return;
  brow[w] = row_of(rowptr, n, w * kP);
}

// One recurrence step's arguments.  first: T_1 = M E and out = c0 E + c1 T_1;
// otherwise T_{r+1} = 2 M T_r - T_{r-1} (into Tn, which may alias Tp) and
// out += c T_{r+1}.
struct ChebStep {
  const float* Tc; int64_t ldc;  // T_r, gathered
  const float* Tp; int64_t ldp;  // T_{r-1} (first step: unused)
  float* Tn; int64_t ldn;        // T_{r+1}
  const float* E; int64_t lde;   // first step: E (for c0 E)
  float* out; int64_t ldo;
  float c0, c;                   // first step: c0 and c1; otherwise c = c_{r+1}
  int first;
};

__device__ __forceinline__ void fma4(float s, const float4& v, float4& a) {
  a.x = fmaf(s, v.x, a.x); a.y = fmaf(s, v.y, a.y); a.z = fmaf(s, v.z, a.z); a.w = fmaf(s, v.w, a.w);
}

// the recurrence and the running sum for row r, column quad q, given the
// neighbour sum v of T_r and the row's degree
__device__ __forceinline__ void cheb_row(const ChebStep& st, int64_t r, int q, int64_t deg, float4 v) {
  float4 t;
  if (st.first) {
    const float s = deg > 0 ? -1.0f / (float)deg : 0.0f;
    t = make_float4(s * v.x, s * v.y, s * v.z, s * v.w);
    const float4 e = *reinterpret_cast<const float4*>(st.E + r * st.lde + 4 * q);
    *reinterpret_cast<float4*>(st.Tn + r * st.ldn + 4 * q) = t;
    *reinterpret_cast<float4*>(st.out + r * st.ldo + 4 * q) =
        make_float4(fmaf(st.c, t.x, st.c0 * e.x), fmaf(st.c, t.y, st.c0 * e.y), fmaf(st.c, t.z, st.c0 * e.z),
                    fmaf(st.c, t.w, st.c0 * e.w));
    return;
  }
  const float s = deg > 0 ? -2.0f / (float)deg : 0.0f;
  const float4 p = *reinterpret_cast<const float4*>(st.Tp + r * st.ldp + 4 * q);
  t = make_float4(fmaf(s, v.x, -p.x), fmaf(s, v.y, -p.y), fmaf(s, v.z, -p.z), fmaf(s, v.w, -p.w));
  *reinterpret_cast<float4*>(st.Tn + r * st.ldn + 4 * q) = t;
  float4* o = reinterpret_cast<float4*>(st.out + r * st.ldo + 4 * q);
  float4 a = *o;
  *o = make_float4(fmaf(st.c, t.x, a.x), fmaf(st.c, t.y, a.y), fmaf(st.c, t.z, a.z), fmaf(st.c, t.w, a.w));
}

// LPS lanes per slot, 64 / LPS slots per wavefront (d / 4 <= LPS)
template <int LPS>
__global__ __launch_bounds__(256) void k_cheb_spmm(int64_t n, int64_t nnz, const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ colidx, int nq, ChebStep st,
                                                   float* __restrict__ partial, const int64_t* __restrict__ brow,
                                                   int64_t nwaves) {
  constexpr int NS = 64 / LPS;
  const int lane = threadIdx.x & 63;
  int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  w = __builtin_amdgcn_readfirstlane((int)w);
  if (w >= nwaves) return;
  const int slot = lane / LPS, q = lane % LPS;
  const bool qok = q < nq;
  const int64_t e0 = w * kP;
  const int64_t e1 = min(e0 + (int64_t)kP, nnz);
  int64_t r = brow[w];
  while (true) {
    const int64_t rs = rowptr[r], re = rowptr[r + 1];
    const int64_t a = max(rs, e0), bnd = min(re, e1);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int64_t e = a + slot;
    // four neighbours per slot in flight
    for (; e + 3 * NS < bnd; e += 4 * NS) {
      int j[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) j[u] = colidx[e + u * NS];
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        v[u] = qok ? *reinterpret_cast<const float4*>(st.Tc + (int64_t)j[u] * st.ldc + 4 * q)
                   : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 4; ++u) fma4(1.0f, v[u], acc);
    }
    for (; e < bnd; e += NS) {
      const int jj = colidx[e];
      if (qok) fma4(1.0f, *reinterpret_cast<const float4*>(st.Tc + (int64_t)jj * st.ldc + 4 * q), acc);
    }
    // slots hold interleaved neighbours of the same row
#pragma unroll
    for (int off = LPS; off < 64; off <<= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
      acc.z += __shfl_xor(acc.z, off, 64);
      acc.w += __shfl_xor(acc.w, off, 64);
    }
    if (slot == 0 && qok) {
      if (rs >= e0 && re <= e1) {
        cheb_row(st, r, q, re - rs, acc);
      } else {
        float* dst = partial + (2 * w + (rs < e0 ? 0 : 1)) * (int64_t)(4 * nq);
        *reinterpret_cast<float4*>(dst + 4 * q) = acc;
      }
    }
    if (re >= e1) break;
    ++r;
    while (rowptr[r + 1] == rowptr[r]) ++r;  // isolated vertices: k_cheb_isolated
  }
}

// rows split by slice boundaries: sum the partials in slice order, then the
// recurrence (the boundary that first cuts a row owns it)
__global__ __launch_bounds__(256) void k_cheb_fixup(int64_t nnz, const int64_t* __restrict__ rowptr, int nq,
                                                    ChebStep st, const float* __restrict__ partial,
                                                    const int64_t* __restrict__ brow, int64_t nwaves) {
  const int lane = threadIdx.x & 63;
  int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6) + 1;
  if (b >= nwaves) return;
  const int64_t e = b * kP;
  const int64_t r = brow[b];
  const int64_t rs = rowptr[r], re = rowptr[r + 1];
  if (rs >= e) return;
  const int64_t ws = rs / kP;
  if (ws + 1 != b) return;
  const int64_t we = (re - 1) / kP;
  const int64_t cols = 4 * (int64_t)nq;
  for (int q = lane; q < nq; q += 64) {
    float4 acc = *reinterpret_cast<const float4*>(partial + (2 * ws + 1) * cols + 4 * q);
    int64_t wv = ws + 1;
    for (; wv + 8 <= we + 1; wv += 8) {
      float4 p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) p[u] = *reinterpret_cast<const float4*>(partial + (2 * (wv + u)) * cols + 4 * q);
#pragma unroll
      for (int u = 0; u < 8; ++u) fma4(1.0f, p[u], acc);
    }
    for (; wv <= we; ++wv) fma4(1.0f, *reinterpret_cast<const float4*>(partial + (2 * wv) * cols + 4 * q), acc);
    cheb_row(st, r, q, re - rs, acc);
  }
}

// isolated vertices: M has a zero row there.  One thread per vertex; the
// rare isolated ones write all their column quads.
__global__ void k_cheb_isolated(int64_t n, const int64_t* __restrict__ rowptr, int nq, ChebStep st) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  if (rowptr[r + 1] != rowptr[r]) return;
  for (int q = 0; q < nq; ++q) cheb_row(st, r, q, 0, make_float4(0.f, 0.f, 0.f, 0.f));
}

// out = c0 E (a degree-0 polynomial)
__global__ void k_cheb_scale(int64_t n, int nq, const float* __restrict__ E, int64_t lde, float c0,
                             float* __restrict__ out, int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = idx / nq;
  if (r >= n) return;
  const int q = (int)(idx - r * nq);
  const float4 e = *reinterpret_cast<const float4*>(E + r * lde + 4 * q);
  *reinterpret_cast<float4*>(out + r * ldo + 4 * q) = make_float4(c0 * e.x, c0 * e.y, c0 * e.z, c0 * e.w);
}

size_t brow_bytes(int64_t nwaves) { return align_up(sizeof(int64_t) * (size_t)(nwaves + 1)); }

}  // namespace

size_t propagate_ws_bytes(int64_t n, int64_t nnz, int d) {
  const int64_t nwaves = (nnz + kP - 1) / kP;
  return 2 * align_up(sizeof(float) * (size_t)n * d) + brow_bytes(nwaves) +
         align_up(sizeof(float) * (size_t)(2 * nwaves + 2) * d);
}

sketchne_status propagate(sketchne_ctx* c, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colidx,
                          int d, const float* E, int64_t lde, int p, const double* coef, float* out, int64_t ldo,
                          void* ws) {
  if (n == 0 || d == 0) return SKETCHNE_OK;
  ProfScope ps(c, SKETCHNE_PROF_PROPAGATE);
  const int nq = d / 4;
  const int64_t nwaves = nnz > 0 ? (nnz + kP - 1) / kP : 0;
  Arena ar(ws, propagate_ws_bytes(n, nnz, d));
  float* Ta = ar.take<float>((size_t)n * d);
  float* Tb = ar.take<float>((size_t)n * d);
  int64_t* brow = ar.take<int64_t>((size_t)nwaves + 1);
  float* partial = ar.take<float>((size_t)(2 * nwaves + 2) * d);
  const unsigned eblocks = (unsigned)((n * nq + 255) / 256);
  if (p == 0) {
    hipLaunchKernelGGL(k_cheb_scale, dim3(eblocks), dim3(256), 0, c->stream, n, nq, E, lde, (float)coef[0], out, ldo);
    return launch_status();
  }
  if (nwaves > 0)
    hipLaunchKernelGGL(k_prop_bounds, dim3((unsigned)((nwaves + 255) / 256)), dim3(256), 0, c->stream, n, rowptr,
                       nwaves, brow);
  const unsigned blocks = (unsigned)((nwaves + 3) / 4);
  // T_1 -> Ta; then T_2 -> Tb (T_0 = E is never overwritten), T_3 -> Ta, ...
  const float* prev = E;
  int64_t ldprev = lde;
  const float* cur = E;
  int64_t ldcur = lde;
  for (int r = 0; r < p; ++r) {
    ChebStep st;
    st.first = r == 0;
    st.Tc = cur; st.ldc = ldcur;
    st.Tp = prev; st.ldp = ldprev;
    float* dst = (r % 2 == 0) ? Ta : Tb;
    st.Tn = dst; st.ldn = d;
    st.E = E; st.lde = lde;
    st.out = out; st.ldo = ldo;
    st.c0 = (float)coef[0];
    st.c = (float)coef[r + 1];
    if (nwaves > 0) {
      if (nq <= 8) hipLaunchKernelGGL(k_cheb_spmm<8>, dim3(blocks), dim3(256), 0, c->stream, n, nnz, rowptr, colidx, nq, st, partial, brow, nwaves);
      else if (nq <= 16) hipLaunchKernelGGL(k_cheb_spmm<16>, dim3(blocks), dim3(256), 0, c->stream, n, nnz, rowptr, colidx, nq, st, partial, brow, nwaves);
      else if (nq <= 32) hipLaunchKernelGGL(k_cheb_spmm<32>, dim3(blocks), dim3(256), 0, c->stream, n, nnz, rowptr, colidx, nq, st, partial, brow, nwaves);
      else hipLaunchKernelGGL(k_cheb_spmm<64>, dim3(blocks), dim3(256), 0, c->stream, n, nnz, rowptr, colidx, nq, st, partial, brow, nwaves);
      if (nwaves > 1)
        hipLaunchKernelGGL(k_cheb_fixup, dim3((unsigned)((nwaves - 1 + 3) / 4)), dim3(256), 0, c->stream, nnz, rowptr,
                           nq, st, partial, brow, nwaves);
    }
    hipLaunchKernelGGL(k_cheb_isolated, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, rowptr, nq,
                       st);
    SK_TRY(launch_status());
    prev = cur; ldprev = ldcur;
    cur = dst; ldcur = d;
  }
  return SKETCHNE_OK;
}

}  // namespace skne
