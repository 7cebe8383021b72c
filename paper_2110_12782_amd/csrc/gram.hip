// Tall-skinny symmetric products on the FP64 matrix cores:
//
//   G = X^T diag(w) Y      (X, Y: n x m FP32, m <= 288; w optional FP64)
//
// computed on the upper 16 x 16 blocks only and mirrored, which is exact for
// the symmetric products of the path (Gram matrices B^T B, Q^T (X Q) and
// U^T D U).  Each workgroup owns a contiguous range of rows: it (512 threads)
// streams them through LDS in chunks of 32 rows (double buffered, next chunk
// prefetched through registers) and keeps the accumulators of its share of
// the upper 16 x 16 blocks of the m x m result in registers.  The blocks are
// dealt one by one to the sixteen wavefronts of two workgroups on the same
// XCD (so the rows are read from memory once and from the XCD's L2 the
// second time): m = 288 has 171 upper blocks, 11 per wavefront at most.  Per-workgroup partial sums are added in a
// fixed order by a second kernel.  The F32 form runs the FP32 matrix cores
// (v_mfma_f32_16x16x4f32: twice the FP64 rate, no conversion of the rows) and
// keeps FP32 partial sums per workgroup; it serves the Cholesky-QR of
// power-iteration bases, whose factor only has to keep the basis well
// conditioned (any invertible factor keeps its span).
#include <type_traits>

#include "internal.h"

namespace skne {
namespace {

typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int GR_CHUNK = 32;      // rows per LDS chunk
constexpr int GR_MAXB = 18;       // m <= 16 * GR_MAXB
constexpr int GR_GROUPS = 2;      // block groups (workgroups per row range)
constexpr int GR_THREADS = 512;
constexpr int GR_WAVES = GR_THREADS / 64;
// LDS row stride of a row-major chunk: room for 288 columns, 48 floats past
// a multiple of 64 so the 4 rows read by one MFMA fragment fall in distinct
// banks; a compile-time stride turns every row step into an immediate offset
constexpr int GR_RSTRIDE = 304;
// column-major chunks are stored [column][row]: GR_CHUNK + 2 floats per
// column, so the 16 columns x 2 rows a half-wave reads fall in distinct banks
constexpr int GR_CSTRIDE = 34;

struct GramArgs {
  int64_t n;
  int m, nbk, nblk, stride;     // stride: LDS row length in floats
  const float* X; int64_t xr, xc;   // element (r, i) at X[r*xr + i*xc]
  const float* Y; int64_t yr, yc;
  const double* w;
  int64_t rows_per_wg;
  int nranges;                  // row ranges
  int crows;                    // !ROWMAJ: rows of a chunk buffer (one per matrix column i, padded)
  double* partial;              // nranges x nblk x 256
  const int* run_if;            // when non-null and zero: do nothing
};

__device__ __forceinline__ void blk_coords(int b, int nbk, int& I, int& J) {
  int r = 0, len = nbk;
  while (b >= len) { b -= len; ++r; --len; }
  I = r;
  J = r + b;
}

// Wavefront g (0..15 over the two workgroups of a row range) takes the upper
// blocks g, g + 16, g + 32, ... of the row-by-row enumeration; a slot past
// the last block repeats the wavefront's first block and is not stored.
// (2 x 2 super-tiles of blocks, which share fragment reads, cost 12% more
// MFMA work at m = 288 from the lower block of each diagonal super-tile and
// from uneven shares, 17% at m = 272 and 33% at m = 256.)
constexpr int GR_WG = GR_GROUPS * GR_WAVES;  // wavefronts per row range

// WGT: G = X^T diag(w) X (w given).  The one-operand FP64 forms stage their
// chunks in LDS already converted to FP64 (S64): each value is converted
// once instead of once per block that reads it, and a fragment read is one
// 8-byte LDS read with no conversion after it.
template <bool TWO, bool ROWMAJ, bool F32, int NSL, bool WGT>
__global__ __launch_bounds__(GR_THREADS) void k_gram_st(GramArgs g) {
  typedef std::conditional_t<F32, floatx4, doublex4> Acc;
  constexpr bool S64 = !F32;
  // rows per chunk: the two-operand FP64 form takes 16 so that its four
  // FP64 chunk buffers fit the LDS
  constexpr int CHK = (TWO && S64) ? 16 : GR_CHUNK;
  typedef std::conditional_t<S64, double, float> LT;  // LDS element
  if (g.run_if && *g.run_if == 0) return;
  const int L = blockIdx.x;
  const int q = L >> 3;
  const int grp = q % GR_GROUPS;
  const int range = (q / GR_GROUPS) * 8 + (L & 7);
  if (range >= g.nranges) return;
  extern __shared__ __attribute__((aligned(16))) char lds_raw[];
  LT* lds = reinterpret_cast<LT*>(lds_raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // chunk buffers: ROWMAJ [data row][column i] (row stride S); otherwise
  // [column i][data row] (stride S = GR_CHUNK + 2), so that a column-major
  // input is stored as it is read, without a transposing scatter
  constexpr int S = ROWMAJ ? GR_RSTRIDE : GR_CSTRIDE;
  const int CH = ROWMAJ ? CHK * S : g.crows * S;
  constexpr int rstep = ROWMAJ ? S : 1, cstep = ROWMAJ ? 1 : S;
  // the two chunk buffers as offsets from the LDS array itself (an array of
  // pointers indexed at run time would lose the LDS address space, and every
  // fragment read would become a FLAT load waiting on the row prefetch)
  auto offX = [&](int b) { return b ? (TWO ? 2 : 1) * CH : 0; };
  auto offY = [&](int b) { return TWO ? (b ? 3 * CH : CH) : offX(b); };
  __shared__ double wsh[2][GR_CHUNK];

  const int64_t r0 = (int64_t)range * g.rows_per_wg;
  const int64_t r1 = min(g.n, r0 + g.rows_per_wg);

  // blocks of this wavefront
  const int uw = __builtin_amdgcn_readfirstlane(wave);
  const int gw = grp * GR_WAVES + uw;
  int pI[NSL], pJ[NSL];
#pragma unroll
  for (int t = 0; t < NSL; ++t) {
    int b = gw + GR_WG * t;
    if (b >= g.nblk) b = gw < g.nblk ? gw : 0;
    blk_coords(b, g.nbk, pI[t], pJ[t]);
  }
  Acc acc[NSL];
#pragma unroll
  for (int t = 0; t < NSL; ++t) acc[t] = Acc{0, 0, 0, 0};

  const int cols4 = (g.m + 3) / 4;
  constexpr int MAXV = (CHK * GR_MAXB * 16 / 4 + GR_THREADS - 1) / GR_THREADS;
  float4 px[MAXV], py[MAXV];
  double pw = 1.0;
  auto fetch = [&](int64_t c0) {
#pragma unroll
    for (int u = 0; u < MAXV; ++u) {
      int v = tid + GR_THREADS * u;
      float4 a = make_float4(0.f, 0.f, 0.f, 0.f), b = a;
      if (ROWMAJ) {
        int rr = v / cols4, c4 = v - rr * cols4;
        int64_t r = c0 + rr;
        if (rr < CHK && r < r1) {
          a = *reinterpret_cast<const float4*>(g.X + r * g.xr + 4 * c4);
          if (TWO) b = *reinterpret_cast<const float4*>(g.Y + r * g.yr + 4 * c4);
        }
      } else {
        int i = v / (GR_CHUNK / 4), qq = v - i * (GR_CHUNK / 4);
        int64_t r = c0 + 4 * qq;
        if (i < g.m) {
          const float* px0 = g.X + (int64_t)i * g.xc + r;
          if (r + 3 < r1 && (reinterpret_cast<uintptr_t>(px0) & 15) == 0) {
            a = *reinterpret_cast<const float4*>(px0);
          } else {
            a.x = r < r1 ? px0[0] : 0.f;
            a.y = r + 1 < r1 ? px0[1] : 0.f;
            a.z = r + 2 < r1 ? px0[2] : 0.f;
            a.w = r + 3 < r1 ? px0[3] : 0.f;
          }
          if (TWO) {
            const float* py0 = g.Y + (int64_t)i * g.yc + r;
            if (r + 3 < r1 && (reinterpret_cast<uintptr_t>(py0) & 15) == 0) {
              b = *reinterpret_cast<const float4*>(py0);
            } else {
              b.x = r < r1 ? py0[0] : 0.f;
              b.y = r + 1 < r1 ? py0[1] : 0.f;
              b.z = r + 2 < r1 ? py0[2] : 0.f;
              b.w = r + 3 < r1 ? py0[3] : 0.f;
            }
          }
        }
      }
      px[u] = a;
      py[u] = b;
    }
    if (WGT && tid < CHK) pw = (c0 + tid < r1) ? g.w[c0 + tid] : 0.0;
  };
  auto stash = [&](int buf) {
    LT* dx = lds + offX(buf);
    LT* dy = lds + offY(buf);
#pragma unroll
    for (int u = 0; u < MAXV; ++u) {
      int v = tid + GR_THREADS * u;
      if (ROWMAJ) {
        int rr = v / cols4, c4 = v - rr * cols4;
        if (rr < CHK) {
          if constexpr (S64) {
            *reinterpret_cast<double2*>(dx + rr * S + 4 * c4) = make_double2(px[u].x, px[u].y);
            *reinterpret_cast<double2*>(dx + rr * S + 4 * c4 + 2) = make_double2(px[u].z, px[u].w);
            if (TWO) {
              *reinterpret_cast<double2*>(dy + rr * S + 4 * c4) = make_double2(py[u].x, py[u].y);
              *reinterpret_cast<double2*>(dy + rr * S + 4 * c4 + 2) = make_double2(py[u].z, py[u].w);
            }
          } else {
            *reinterpret_cast<float4*>(dx + rr * S + 4 * c4) = px[u];
            if (TWO) *reinterpret_cast<float4*>(dy + rr * S + 4 * c4) = py[u];
          }
        }
      } else {
        int i = v / (GR_CHUNK / 4), qq = v - i * (GR_CHUNK / 4);
        if (i < g.m) {
          if constexpr (S64) {
            *reinterpret_cast<double2*>(dx + i * S + 4 * qq) = make_double2(px[u].x, px[u].y);
            *reinterpret_cast<double2*>(dx + i * S + 4 * qq + 2) = make_double2(px[u].z, px[u].w);
          } else {
            // S is even: 8-byte stores
            *reinterpret_cast<float2*>(dx + i * S + 4 * qq) = make_float2(px[u].x, px[u].y);
            *reinterpret_cast<float2*>(dx + i * S + 4 * qq + 2) = make_float2(px[u].z, px[u].w);
            if (TWO) {
              *reinterpret_cast<float2*>(dy + i * S + 4 * qq) = make_float2(py[u].x, py[u].y);
              *reinterpret_cast<float2*>(dy + i * S + 4 * qq + 2) = make_float2(py[u].z, py[u].w);
            }
          }
        }
      }
    }
    if (tid < CHK) wsh[buf][tid] = pw;
  };

  // columns i >= m are never stored: zero them once
  for (int idx = tid; idx < 2 * (TWO ? 2 : 1) * CH; idx += GR_THREADS) {
    const int col = ROWMAJ ? (idx % CH) % S : (idx % CH) / S;
    if (col >= g.m) lds[idx] = LT(0);
  }
  int buf = 0;
  if (r0 < r1) {
    fetch(r0);
    stash(0);
  }
  __syncthreads();
  for (int64_t c0 = r0; c0 < r1; c0 += CHK) {
    const bool more = c0 + CHK < r1;
    if (more) fetch(c0 + CHK);
    // this lane's fragment address in each slot's blocks; the row steps of
    // the chunk are compile-time offsets from it
    const LT* xa[NSL];
    const LT* ya[NSL];
#pragma unroll
    for (int t = 0; t < NSL; ++t) {
      xa[t] = lds + offX(buf) + (lane >> 4) * rstep + ((lane & 15) + 16 * pI[t]) * cstep;
      ya[t] = lds + offY(buf) + (lane >> 4) * rstep + ((lane & 15) + 16 * pJ[t]) * cstep;
    }
#pragma unroll
    for (int st = 0; st < CHK / 4; ++st) {
      const double wr = WGT ? wsh[buf][4 * st + (lane >> 4)] : 1.0;
#pragma unroll
      for (int t = 0; t < NSL; ++t) {
        if constexpr (F32) {
          const float a0 = xa[t][4 * st * rstep];
          const float a = WGT ? a0 * (float)wr : a0;
          const float b = ya[t][4 * st * rstep];
          acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[t], 0, 0, 0);
        } else {
          const double a0 = (double)xa[t][4 * st * rstep];
          const double a = WGT ? a0 * wr : a0;
          const double b = (double)ya[t][4 * st * rstep];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        }
      }
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double* part = g.partial + (int64_t)range * g.nblk * 256;
#pragma unroll
  for (int t = 0; t < NSL; ++t) {
    const int b = gw + GR_WG * t;
    if (b >= g.nblk) continue;
    if constexpr (F32) {
      // v_mfma_f32_16x16x4f32 holds row 4 (l / 16) + r, column l % 16 in
      // lane l, register r; the partial keeps the FP64 form's order
      // (row l' / 16 + 4 r', column l' % 16 at element 4 l' + r')
      double* pb = part + (int64_t)b * 256;
#pragma unroll
      for (int r = 0; r < 4; ++r) pb[4 * ((lane & 15) + 16 * r) + (lane >> 4)] = (double)acc[t][r];
    } else {
      double* pb = part + (int64_t)b * 256 + lane * 4;
      pb[0] = acc[t][0];
      pb[1] = acc[t][1];
      pb[2] = acc[t][2];
      pb[3] = acc[t][3];
    }
  }
}

// G[i][j] = G[j][i] = sum over workgroups; element (block, lane, r) of the
// MFMA output is row I*16 + lane/16 + 4r, column J*16 + lane%16.
__global__ void k_gram_reduce(int m, int nbk, int nblk, int nwg, const double* __restrict__ partial,
                              double* __restrict__ G, const int* __restrict__ run_if) {
  if (run_if && *run_if == 0) return;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nblk * 256) return;
  int b = idx >> 8, e = idx & 255, lane = e >> 2, r = e & 3;
  int I, J;
  blk_coords(b, nbk, I, J);
  int i = I * 16 + (lane >> 4) + 4 * r, j = J * 16 + (lane & 15);
  if (i >= m || j >= m) return;
  // eight partials in flight per step, added in workgroup order
  double s = 0.0;
  int w = 0;
  for (; w + 8 <= nwg; w += 8) {
    double p[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) p[u] = partial[((int64_t)(w + u) * nblk + b) * 256 + e];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += p[u];
  }
  for (; w < nwg; ++w) s += partial[((int64_t)w * nblk + b) * 256 + e];
  G[(int64_t)i * m + j] = s;
  if (I != J) G[(int64_t)j * m + i] = s;
}

}  // namespace

int gram_nwg(int64_t n) {
  int64_t chunks = (n + GR_CHUNK - 1) / GR_CHUNK;
  int64_t nr = chunks < 256 ? chunks : 256;
  return nr < 1 ? 1 : (int)nr;
}

size_t gram_ws_bytes(int64_t n, int m) {
  int nbk = (m + 15) / 16;
  int nblk = nbk * (nbk + 1) / 2;
  return align_up(sizeof(double) * (size_t)gram_nwg(n) * nblk * 256);
}

// X, Y: element (r, i) at X[r*xr + i*xc]; either xc == 1 (rows contiguous)
// or xr == 1 (columns contiguous).  Y may equal X (then pass Y = nullptr);
// two operands and weights take row-major blocks.
sketchne_status gram_tall(sketchne_ctx* c, int64_t n, int m, const float* X, int64_t xr, int64_t xc, const float* Y,
                          int64_t yr, int64_t yc, const double* w, double* G, double* partial, size_t partial_cap,
                          const int* run_if, bool f32) {
  if (m < 1 || m > 16 * GR_MAXB) return SKETCHNE_E_UNSUPPORTED;
  const bool rowmaj = (xc == 1);
  if (!rowmaj && xr != 1) return SKETCHNE_E_ARG;
  if (Y && ((rowmaj && yc != 1) || (!rowmaj && yr != 1))) return SKETCHNE_E_ARG;
  if (rowmaj && ((m % 4) || (xr % 4) || (Y && (yr % 4)))) return SKETCHNE_E_ARG;  // float4 rows
  if (partial_cap < gram_ws_bytes(n, m)) return SKETCHNE_E_WORKSPACE;
  GramArgs g{};
  g.n = n;
  g.m = m;
  g.nbk = (m + 15) / 16;
  g.nblk = g.nbk * (g.nbk + 1) / 2;
  g.stride = rowmaj ? GR_RSTRIDE : GR_CSTRIDE;
  g.crows = 16 * g.nbk;  // column-major buffers: one LDS row per matrix column
  g.X = X; g.xr = xr; g.xc = xc;
  g.Y = Y ? Y : X; g.yr = Y ? yr : xr; g.yc = Y ? yc : xc;
  g.w = w;
  const int nr = gram_nwg(n);
  int64_t rpw = (n + nr - 1) / nr;
  g.rows_per_wg = (rpw + GR_CHUNK - 1) / GR_CHUNK * GR_CHUNK;
  g.nranges = nr;
  // blocks per wavefront (instantiated for 3, 6, 9, 10 and 11)
  const int need = (g.nblk + GR_WG - 1) / GR_WG;
  const int nsl = need <= 3 ? 3 : need <= 6 ? 6 : need <= 9 ? 9 : need <= 10 ? 10 : 11;
  if (need > 11) return SKETCHNE_E_UNSUPPORTED;
  g.partial = partial;
  g.run_if = run_if;
  const bool two = Y != nullptr;
  const bool s64 = !(f32 && !w && !two && rowmaj);  // the FP64 forms stage FP64
  const int chk = (two && s64) ? 16 : GR_CHUNK;
  const size_t shmem = (s64 ? sizeof(double) : sizeof(float)) * (size_t)2 * (two ? 2 : 1) *
                       (rowmaj ? chk : g.crows) * g.stride;
  // weights: the one-operand row-major form; two operands: row-major
  if ((w && (two || !rowmaj)) || (two && !rowmaj)) return SKETCHNE_E_UNSUPPORTED;
  const unsigned blocks = (unsigned)((nr + 7) / 8 * 8 * GR_GROUPS);
  ProfScope ps(c, SKETCHNE_PROF_GEMM64);
#define SKNE_GRAM_N(T, R, F, N, W)                                                                         \
  do {                                                                                                     \
    hipFuncSetAttribute(reinterpret_cast<const void*>(k_gram_st<T, R, F, N, W>),                           \
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);                           \
    hipLaunchKernelGGL((k_gram_st<T, R, F, N, W>), dim3(blocks), dim3(GR_THREADS), shmem, c->stream, g);   \
  } while (0)
#define SKNE_GRAM(T, R, F, W)                                                                              \
  do {                                                                                                     \
    switch (nsl) {                                                                                         \
      case 3: SKNE_GRAM_N(T, R, F, 3, W); break;                                                           \
      case 6: SKNE_GRAM_N(T, R, F, 6, W); break;                                                           \
      case 9: SKNE_GRAM_N(T, R, F, 9, W); break;                                                           \
      case 10: SKNE_GRAM_N(T, R, F, 10, W); break;                                                         \
      default: SKNE_GRAM_N(T, R, F, 11, W); break;                                                         \
    }                                                                                                      \
  } while (0)
  if (w) SKNE_GRAM(false, true, false, true);
  else if (f32 && !two && rowmaj) SKNE_GRAM(false, true, true, false);
  else if (two) SKNE_GRAM(true, true, false, false);
  else { if (rowmaj) SKNE_GRAM(false, true, false, false); else SKNE_GRAM(false, false, false, false); }
#undef SKNE_GRAM_N
#undef SKNE_GRAM
  hipLaunchKernelGGL(k_gram_reduce, dim3((g.nblk * 256 + 255) / 256), dim3(256), 0, c->stream, m, g.nbk, g.nblk, nr,
                     partial, G, run_if);
  return launch_status();
}

}  // namespace skne
