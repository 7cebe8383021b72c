// CSR SpMM with the modified Laplacian: C = D^-a A D^-a B.
//
// The paper's CPU version walks vertices in parallel and, for each neighbour
// v of u, adds D(u,u)^-a D(v,v)^-a times row v of the row-major dense matrix
// to row u of the output (Section 3.4).  Here the work unit is a fixed slice
// of P stored entries per wavefront instead of a vertex, so a hub with
// thousands of neighbours is spread over many wavefronts and no wavefront
// waits on one long row.  Inside a wavefront the 64 lanes cover one dense
// row in float4 chunks, so every neighbour gather is a contiguous, coalesced
// read of cols*4 bytes.  A row that crosses a slice boundary is written as
// partial sums (one "head" and one "tail" slot per wavefront) and a fixup
// kernel adds the partials of each such row in slice order, so the result is
// deterministic (no floating-point atomics).  The row containing the first
// entry of every slice is found once per call (one binary search per slice,
// all in parallel) and read by both kernels.
#include "internal.h"

namespace skne {
namespace {

constexpr int kP = 256;  // stored entries per wavefront slice

__global__ void k_degree_scale(int64_t n, const int64_t* __restrict__ rowptr, double alpha,
                               float* __restrict__ dscale) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t deg = rowptr[i + 1] - rowptr[i];
  dscale[i] = deg > 0 ? (float)pow((double)deg, -alpha) : 0.0f;
}

__device__ __forceinline__ int64_t row_of(const int64_t* __restrict__ rowptr, int64_t n, int64_t e) {
  // largest r with rowptr[r] <= e  (rowptr[0] = 0 <= e < rowptr[n])
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (rowptr[mid] <= e) lo = mid; else hi = mid;
  }
  return lo;
}

// brow[w] = row containing stored entry w*P, for every slice w
__global__ void k_spmm_bounds(int64_t n, const int64_t* __restrict__ rowptr, int64_t nwaves,
                              int64_t* __restrict__ brow) {
  const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= nwaves) return;
  brow[w] = row_of(rowptr, n, w * kP);
}

template <int NIT>
__global__ __launch_bounds__(256) void k_spmm(int64_t n, int64_t nnz, const int64_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ colidx,
                                              const float* __restrict__ dscale,
                                              const float* __restrict__ B, int64_t ldb, int cols,
                                              float* __restrict__ C, int64_t ldc,
                                              float* __restrict__ partial, const int64_t* __restrict__ brow,
                                              int64_t nwaves) {
  const int lane = threadIdx.x & 63;
  int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  w = __builtin_amdgcn_readfirstlane((int)w);
  if (w >= nwaves) return;
  const int nc4 = cols >> 2;
  const int64_t e0 = w * kP;
  const int64_t e1 = min(e0 + (int64_t)kP, nnz);
  int64_t r = brow[w];
  while (true) {
    const int64_t rs = rowptr[r], re = rowptr[r + 1];
    const int64_t a = max(rs, e0), bnd = min(re, e1);
    float4 acc[NIT];
#pragma unroll
    for (int it = 0; it < NIT; ++it) acc[it] = make_float4(0.f, 0.f, 0.f, 0.f);
    int64_t e = a;
    for (; e + 4 <= bnd; e += 4) {
      int j[4];
      float s[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) j[u] = colidx[e + u];
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] = dscale[j[u]];
      float4 v[4][NIT];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
          int c4 = lane + 64 * it;
          v[u][it] = c4 < nc4 ? *reinterpret_cast<const float4*>(B + (int64_t)j[u] * ldb + 4 * c4)
                              : make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
          acc[it].x = fmaf(s[u], v[u][it].x, acc[it].x);
          acc[it].y = fmaf(s[u], v[u][it].y, acc[it].y);
          acc[it].z = fmaf(s[u], v[u][it].z, acc[it].z);
          acc[it].w = fmaf(s[u], v[u][it].w, acc[it].w);
        }
    }
    for (; e < bnd; ++e) {
      int jj = colidx[e];
      float ss = dscale[jj];
#pragma unroll
      for (int it = 0; it < NIT; ++it) {
        int c4 = lane + 64 * it;
        if (c4 < nc4) {
          float4 vv = *reinterpret_cast<const float4*>(B + (int64_t)jj * ldb + 4 * c4);
          acc[it].x = fmaf(ss, vv.x, acc[it].x);
          acc[it].y = fmaf(ss, vv.y, acc[it].y);
          acc[it].z = fmaf(ss, vv.z, acc[it].z);
          acc[it].w = fmaf(ss, vv.w, acc[it].w);
        }
      }
    }
    const float sr = dscale[r];
    const bool whole = (rs >= e0) && (re <= e1);
    float* dst = whole ? (C + r * ldc) : (partial + (2 * w + (rs < e0 ? 0 : 1)) * (int64_t)cols);
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      int c4 = lane + 64 * it;
      if (c4 < nc4) {
        float4 o = make_float4(sr * acc[it].x, sr * acc[it].y, sr * acc[it].z, sr * acc[it].w);
        *reinterpret_cast<float4*>(dst + 4 * c4) = o;
      }
    }
    if (re >= e1) break;
    ++r;
    while (rowptr[r + 1] == rowptr[r]) ++r;  // skip empty rows (written by k_zero_empty)
  }
}

// Narrow variant for blocks of at most 32 columns (CWP <= 8 float4 column
// quads, a power of two).  A row is taken by a group of 8 * CWP lanes: lane
// slot (sub / CWP) walks every 8th neighbour and column quad sub % CWP, and
// the 8 slots are summed with xor shuffles inside the group.  A wavefront
// runs 8 / CWP row groups side by side over the rows of its slice, so a
// 4-column block (the warm-start probes) has eight rows' dependent load
// chains in flight instead of one.  (Splitting a wide block into 32-column
// launches was measured slower than k_spmm: 5.6 TB/s of 128-byte gathers
// against 7.3 TB/s of whole-row gathers.)  Rows that cross a slice boundary
// use the same head/tail partial slots as k_spmm.
template <int CWP>
__global__ __launch_bounds__(256) void k_spmm_narrow(int64_t n, int64_t nnz, const int64_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ colidx,
                                                     const float* __restrict__ dscale,
                                                     const float* __restrict__ B, int64_t ldb, int cw,
                                                     float* __restrict__ C, int64_t ldc,
                                                     float* __restrict__ partial, const int64_t* __restrict__ brow,
                                                     int64_t nwaves) {
  constexpr int GL = 8 * CWP;  // lanes per row group
  constexpr int NG = 64 / GL;  // row groups per wavefront
  const int lane = threadIdx.x & 63;
  int64_t w = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  w = __builtin_amdgcn_readfirstlane((int)w);
  if (w >= nwaves) return;
  const int grp = lane / GL, sub = lane % GL, slot = sub / CWP, c4 = sub % CWP;
  const bool colok = c4 < cw;
  const int64_t e0 = w * kP;
  const int64_t e1 = min(e0 + (int64_t)kP, nnz);
  // rows [rfirst, rend) hold this slice's entries (empty rows among them are
  // skipped; k_zero_empty writes them)
  const int64_t rfirst = brow[w];
  int64_t rend;
  if (w + 1 < nwaves) {
    const int64_t rb = brow[w + 1];
    rend = rowptr[rb] < e1 ? rb + 1 : rb;
  } else {
    rend = row_of(rowptr, n, e1 - 1) + 1;
  }
  for (int64_t r = rfirst + grp; r < rend; r += NG) {
    const int64_t rs = rowptr[r], re = rowptr[r + 1];
    const int64_t a = max(rs, e0), bnd = min(re, e1);
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    int64_t e = a + slot;
    for (; e + 8 < bnd; e += 16) {
      const int j0 = colidx[e], j1 = colidx[e + 8];
      const float s0 = dscale[j0], s1 = dscale[j1];
      float4 v0 = make_float4(0.f, 0.f, 0.f, 0.f), v1 = v0;
      if (colok) {
        v0 = *reinterpret_cast<const float4*>(B + (int64_t)j0 * ldb + 4 * c4);
        v1 = *reinterpret_cast<const float4*>(B + (int64_t)j1 * ldb + 4 * c4);
      }
      acc.x = fmaf(s0, v0.x, acc.x); acc.y = fmaf(s0, v0.y, acc.y);
      acc.z = fmaf(s0, v0.z, acc.z); acc.w = fmaf(s0, v0.w, acc.w);
      acc.x = fmaf(s1, v1.x, acc.x); acc.y = fmaf(s1, v1.y, acc.y);
      acc.z = fmaf(s1, v1.z, acc.z); acc.w = fmaf(s1, v1.w, acc.w);
    }
    if (e < bnd) {
      const int j0 = colidx[e];
      const float s0 = dscale[j0];
      if (colok) {
        const float4 v0 = *reinterpret_cast<const float4*>(B + (int64_t)j0 * ldb + 4 * c4);
        acc.x = fmaf(s0, v0.x, acc.x); acc.y = fmaf(s0, v0.y, acc.y);
        acc.z = fmaf(s0, v0.z, acc.z); acc.w = fmaf(s0, v0.w, acc.w);
      }
    }
    // the xor partners stay inside the group, which shares r
#pragma unroll
    for (int off = CWP; off < GL; off <<= 1) {
      acc.x += __shfl_xor(acc.x, off, 64);
      acc.y += __shfl_xor(acc.y, off, 64);
      acc.z += __shfl_xor(acc.z, off, 64);
      acc.w += __shfl_xor(acc.w, off, 64);
    }
    if (slot == 0 && colok && a < bnd) {
      const float sr = dscale[r];
      const bool whole = (rs >= e0) && (re <= e1);
      float* dst = whole ? (C + r * ldc) : (partial + (2 * w + (rs < e0 ? 0 : 1)) * (int64_t)(4 * cw));
      *reinterpret_cast<float4*>(dst + 4 * c4) = make_float4(sr * acc.x, sr * acc.y, sr * acc.z, sr * acc.w);
    }
  }
}

// For each slice boundary b*P: the row containing entry b*P, if it began in an
// earlier slice and b is the first boundary it crosses, is finished here.
__global__ __launch_bounds__(256) void k_spmm_fixup(int64_t n, int64_t nnz, const int64_t* __restrict__ rowptr,
                                                    int cols, float* __restrict__ C, int64_t ldc,
                                                    const float* __restrict__ partial,
                                                    const int64_t* __restrict__ brow, int64_t nwaves) {
  const int lane = threadIdx.x & 63;
  int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6) + 1;
  if (b >= nwaves) return;
  const int64_t e = b * kP;
  const int64_t r = brow[b];
  const int64_t rs = rowptr[r], re = rowptr[r + 1];
  if (rs >= e) return;                 // row starts at this boundary: not split here
  const int64_t ws = rs / kP;
  if (ws + 1 != b) return;             // an earlier boundary owns this row
  const int64_t we = (re - 1) / kP;
  const int nc4 = cols >> 2;
  for (int c4 = lane; c4 < nc4; c4 += 64) {
    float4 acc = *reinterpret_cast<const float4*>(partial + (2 * ws + 1) * (int64_t)cols + 4 * c4);
    // a hub row spans many slices: eight partial loads in flight per step,
    // added in slice order
    int64_t wv = ws + 1;
    for (; wv + 8 <= we + 1; wv += 8) {
      float4 p[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        p[u] = *reinterpret_cast<const float4*>(partial + (2 * (wv + u)) * (int64_t)cols + 4 * c4);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        acc.x += p[u].x; acc.y += p[u].y; acc.z += p[u].z; acc.w += p[u].w;
      }
    }
    for (; wv <= we; ++wv) {
      float4 p = *reinterpret_cast<const float4*>(partial + (2 * wv) * (int64_t)cols + 4 * c4);
      acc.x += p.x; acc.y += p.y; acc.z += p.z; acc.w += p.w;
    }
    *reinterpret_cast<float4*>(C + r * ldc + 4 * c4) = acc;
  }
}

__global__ void k_zero_empty(int64_t n, const int64_t* __restrict__ rowptr, int cols,
                             float* __restrict__ C, int64_t ldc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (rowptr[i + 1] != rowptr[i]) return;
  for (int c = 0; c < cols; ++c) C[i * ldc + c] = 0.0f;
}

}  // namespace

// workspace: the slice rows (nwaves int64), then the head/tail partials
static size_t spmm_brow_bytes(int64_t nwaves) { return align_up(sizeof(int64_t) * (size_t)(nwaves + 1)); }

size_t spmm_ws_bytes(int64_t nnz, int cols) {
  int64_t nwaves = (nnz + kP - 1) / kP;
  return spmm_brow_bytes(nwaves) + align_up(sizeof(float) * (size_t)(2 * nwaves + 2) * (size_t)cols);
}

sketchne_status degree_scale(sketchne_ctx* c, int64_t n, const int64_t* rowptr, double alpha, float* dscale) {
  if (n == 0) return SKETCHNE_OK;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  hipLaunchKernelGGL(k_degree_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, rowptr,
                     alpha, dscale);
  return launch_status();
}

sketchne_status spmm(sketchne_ctx* c, int64_t n, int64_t nnz, const int64_t* rowptr, const int32_t* colidx,
                     const float* dscale, const float* B, int64_t ldb, int cols, float* C, int64_t ldc,
                     float* partial) {
  if (n == 0 || cols == 0) return SKETCHNE_OK;
  ProfScope ps(c, SKETCHNE_PROF_SPMM);
  hipLaunchKernelGGL(k_zero_empty, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, n, rowptr, cols,
                     C, ldc);
  if (nnz == 0) return launch_status();
  int64_t nwaves = (nnz + kP - 1) / kP;
  unsigned blocks = (unsigned)((nwaves + 3) / 4);
  int64_t* brow = reinterpret_cast<int64_t*>(partial);
  partial = reinterpret_cast<float*>(reinterpret_cast<char*>(partial) + spmm_brow_bytes(nwaves));
  hipLaunchKernelGGL(k_spmm_bounds, dim3((unsigned)((nwaves + 255) / 256)), dim3(256), 0, c->stream, n, rowptr, nwaves,
                     brow);
  if (cols > 32) {
    if (cols <= 256)
      hipLaunchKernelGGL(k_spmm<1>, dim3(blocks), dim3(256), 0, c->stream, n, nnz, rowptr, colidx, dscale, B, ldb,
                         cols, C, ldc, partial, brow, nwaves);
    else
      hipLaunchKernelGGL(k_spmm<2>, dim3(blocks), dim3(256), 0, c->stream, n, nnz, rowptr, colidx, dscale, B, ldb,
                         cols, C, ldc, partial, brow, nwaves);
    if (nwaves > 1)
      hipLaunchKernelGGL(k_spmm_fixup, dim3((unsigned)((nwaves - 1 + 3) / 4)), dim3(256), 0, c->stream, n, nnz,
                         rowptr, cols, C, ldc, partial, brow, nwaves);
    return launch_status();
  }
  // narrow blocks (<= 32 columns): 8 / CWP rows per wavefront at once
  const int cw = cols / 4;
#define SKNE_NARROW(CWP)                                                                                         \
  hipLaunchKernelGGL(k_spmm_narrow<CWP>, dim3(blocks), dim3(256), 0, c->stream, n, nnz, rowptr, colidx, dscale, B, \
                     ldb, cw, C, ldc, partial, brow, nwaves)
  if (cw <= 1) SKNE_NARROW(1);
  else if (cw <= 2) SKNE_NARROW(2);
  else if (cw <= 4) SKNE_NARROW(4);
  else SKNE_NARROW(8);
#undef SKNE_NARROW
  if (nwaves > 1)
    hipLaunchKernelGGL(k_spmm_fixup, dim3((unsigned)((nwaves - 1 + 3) / 4)), dim3(256), 0, c->stream, n, nnz,
                       rowptr, cols, C, ldc, partial, brow, nwaves);
  return launch_status();
}

}  // namespace skne
