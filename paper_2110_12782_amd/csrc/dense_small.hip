// Small dense FP64 solvers: Cholesky with inverse factor, symmetric eigensolver.
//
// Cholesky: G = R^T R for an SPD m x m matrix (m <= 512), right-looking and
// blocked by 32 inside one 512-thread workgroup (diagonal blocks factored by
// one wavefront in registers, row panels and trailing updates on the FP64
// matrix cores).  The same row operations are
// applied to an appended identity, so the right half ends up holding R^-T
// (block row J of [R | R^-T] is R_JJ^-T times the updated block row J of
// [G | I]).  A pivot that is not positive restarts the factorization once with
// a small diagonal shift (shifted Cholesky-QR) and raises a flag; a second
// failure raises CHOL_FAIL.
//
// Eigensolver: one-sided block Jacobi (see the comment above oj_cross_round).
#include <mutex>

#include "internal.h"

namespace skne {
namespace {

constexpr int NB = 32;
constexpr int CH_MAXM = 512;            // largest order
constexpr int CH_CHUNKS = CH_MAXM / 64;  // 64-column chunks of a row

typedef double doublex4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double readlane_d(double v, int lane) {
  int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Grid barrier for the few-workgroup kernels below (at most 9 workgroups of
// one CU each, launched on the stream after the previous kernel has ended, so
// all of them are resident together).  *bar is zero at launch; barrier b
// (1, 2, ...) is passed once all workgroups have added their arrival, i.e.
// when *bar reaches b times the grid size.  The workgroup barrier before the
// arrival and thread 0's agent-scope release publish the workgroup's stores;
// thread 0's acquire fence once the count is seen (the polling itself is
// relaxed, so the caches are invalidated once) and the closing workgroup
// barrier make the other workgroups' stores visible to every thread.  A wait
// longer than kBarSpinLimit polls (over a second) raises
// SKETCHNE_FLAG_BARRIER and returns false, and the caller then leaves the
// kernel, so a grid that were not all resident ends with an error instead of
// hanging.
constexpr uint32_t kBarSpinLimit = 1u << 22;

__device__ __forceinline__ bool grid_barrier(uint32_t* bar, uint32_t& target, uint32_t* flags, int* s_abort) {
  __syncthreads();
  target += gridDim.x;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int abort = 0;
    uint32_t spins = 0;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++spins > kBarSpinLimit) {
        atomicOr(flags, SKETCHNE_FLAG_BARRIER);
        abort = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *s_abort = abort;
  }
  __syncthreads();
  return *s_abort == 0;
}

__global__ void k_zero_u32(uint32_t* __restrict__ p) { *p = 0u; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Factorization of the jb x jb diagonal block by one wavefront.  Lanes 0..31
// hold the columns of the block (upper triangle, read from D: LDS, row stride
// NB + 1; padded with the identity beyond jb), lanes 32..63 the columns of an
// identity, and the row operations of the factorization turn the pair into
// [R_JJ | R_JJ^-T].  Row t is passed between lanes through LDS (xrow; LDS
// operations of one wavefront complete in order).  On return the left lanes
// have written R_JJ to W (unless W is null) (and added the column sums of |R_JJ| to colsum when
// it is non-null), and D holds R_JJ^-T, padded with the identity.  Sets
// *fail when a pivot is not positive.
__device__ __forceinline__ void chol_diag_wave(double* D, double* xrow, double* W, int64_t m2, int j0, int jb, int lane,
                               double* colsum, int* fail) {
  const int b = lane & (NB - 1);
  const bool right = lane >= NB;
  double c[NB];
#pragma unroll
  for (int a = 0; a < NB; ++a) {
    double v = a == b ? 1.0 : 0.0;
    if (!right && b < jb && a < jb) v = a <= b ? D[a * (NB + 1) + b] : 0.0;
    c[a] = v;
  }
  bool bad = false;
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    double piv = readlane_d(c[t], t);
    if (!(piv > 0.0) || !isfinite(piv)) { bad = true; piv = 1.0; }
    // 1 / R(t, t) from one reciprocal square root and R(t, t) = piv / R(t, t):
    // a shorter dependent chain than a square root followed by a division
    const double rd = rsqrt(piv);
    const double d = piv * rd;
    // (entries below the diagonal of a left column are never read, so they
    // take the same unconditional operations as the rest)
    c[t] = (!right && b == t) ? d : c[t] * rd;
    xrow[lane] = c[t];  // row t of [R_JJ | R_JJ^-T]
    // read back the part of the row this step needs, every 16-byte read
    // issued before the first use (one LDS round trip per step)
    double xr[NB];
#pragma unroll
    for (int a = (t + 1) & ~1; a < NB; a += 2) {
      const double2 v = *reinterpret_cast<const double2*>(xrow + a);
      xr[a] = v.x;
      xr[a + 1] = v.y;
    }
    __builtin_amdgcn_sched_group_barrier(0x100, NB / 2, 0);  // the DS reads first (at most NB / 2)
    __builtin_amdgcn_sched_group_barrier(0x002, NB, 0);      // then the FMAs
#pragma unroll
    for (int a = t + 1; a < NB; ++a) c[a] = fma(-xr[a], c[t], c[a]);  // xr[a] = R(t, a)
  }
  if (!right) {
    if (b < jb) {
      double cs = 0.0;
#pragma unroll
      for (int a = 0; a < NB; ++a)
        if (a <= b) {
          if (W) W[(int64_t)(j0 + a) * m2 + j0 + b] = c[a];
          cs += fabs(c[a]);
        }
      if (colsum) colsum[j0 + b] += cs;
    }
  } else {
#pragma unroll
    for (int a = 0; a < NB; ++a) D[a * (NB + 1) + b] = c[a];
  }
  if (bad && lane == 0) *fail = 1;
}

// W (m x 2m, row-major) holds [Gs | I] and is reduced in place to [Rs | Rs^-T].
// Only the parts the factorization reads are ever written or read: the left
// half on and above the diagonal, the right half below the diagonal and in
// the diagonal blocks.  Every loop over W keeps many loads in flight (a row
// per wavefront, its 64-column chunks over the lanes, several rows at once),
// since one workgroup is bound by the latency of its loads, not by their
// bandwidth.
__global__ __launch_bounds__(512) void k_chol_inv(int m, const double* __restrict__ G, double* __restrict__ W,
                                                  double* __restrict__ RinvT, uint32_t* __restrict__ flags,
                                                  int* __restrict__ need_more, const int* __restrict__ run_if,
                                                  double repeat_kappa) {
  if (run_if && *run_if == 0) return;
  extern __shared__ double smem[];
  double* D = smem;                  // NB x (NB+1)
  double* P = smem + NB * (NB + 1);  // NB x m panel
  __shared__ double rsc[CH_MAXM];     // 1 / sqrt(G_ii) (1 for a zero or invalid diagonal)
  __shared__ double colsum[CH_MAXM];  // column sums of |Rs|, added as block rows of Rs are finished
  __shared__ __attribute__((aligned(16))) double xrow[64];         // row exchange of the diagonal-block factorization
  __shared__ double s_red[2][8];
  __shared__ int s_fail;
  __shared__ int s_shifted;
  __shared__ int s_abort;
  uint32_t target = 0;  // grid barrier count
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), nw = nt >> 6;
  const int64_t m2 = 2 * (int64_t)m;

  // The scaled matrix Gs = S^-1 G S^-1 (S = diag(sqrt(G_ii))) is factored:
  // Gs = Rs^T Rs gives R = Rs S and R^-T = Rs^-T S^-1.  The span of the
  // Cholesky-QR basis does not depend on the scaling, and the condition
  // number that decides a second pass is the scaled one (power iterates
  // differ mostly in column scale).
  double trp = 0.0;
  for (int i = tid; i < m; i += nt) {
    const double g = G[(int64_t)i * m + i];
    const double r = (g > 0.0 && isfinite(g)) ? 1.0 / sqrt(g) : 1.0;
    rsc[i] = r;
    trp += fabs(g) * r * r;
  }
  trp = wave_sum(trp);
  if (lane == 0) s_red[0][wv] = trp;
  if (tid == 0) s_shifted = 0;
  __syncthreads();
  double tr = 0.0;
  for (int w = 0; w < nw; ++w) tr += s_red[0][w];
  // shifted retry: s = 11 (m^2 + m) u trace(Gs)  (shifted Cholesky-QR)
  const double retry_shift = 11.0 * ((double)m * m + m) * 1.1102230246251565e-16 * (tr > 0 ? tr : 1.0);

  for (int attempt = 0; attempt < 2; ++attempt) {
    const double shift = attempt == 0 ? 0.0 : retry_shift;
    for (int r0 = 4 * wv; r0 < m; r0 += 4 * nw) {
      double v[4][CH_CHUNKS];
#pragma unroll
      for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int cc = 0; cc < CH_CHUNKS; ++cc) {
          const int r = r0 + h, c = lane + 64 * cc;
          v[h][cc] = (r < m && c < m && c >= r) ? G[(int64_t)r * m + c] : 0.0;
        }
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int r = r0 + h;
        if (r >= m) break;
        double* row = W + (int64_t)r * m2;
        const int rend = min(m, (r / NB + 1) * NB);  // right half: up to the end of the diagonal block
        const double rr = rsc[r];
#pragma unroll
        for (int cc = 0; cc < CH_CHUNKS; ++cc) {
          const int c = lane + 64 * cc;
          if (c < m && c >= r) row[c] = v[h][cc] * rr * rsc[c] + (c == r ? shift : 0.0);
          if (c < rend) row[m + c] = c == r ? 1.0 : 0.0;
        }
      }
    }
    for (int j = tid; j < m; j += nt) colsum[j] = 0.0;
    if (tid == 0) s_fail = 0;
    __syncthreads();

    for (int j0 = 0; j0 < m; j0 += NB) {
      const int jb = min(NB, m - j0);
      // 1. factor the diagonal block in LDS (one wavefront)
      for (int idx = tid; idx < NB * NB; idx += nt) {
        const int a = idx / NB, b = idx % NB;
        D[a * (NB + 1) + b] = (b < jb && a <= b) ? W[(int64_t)(j0 + a) * m2 + j0 + b] : 0.0;
      }
      __syncthreads();
      if (tid < 64) chol_diag_wave(D, xrow, W, m2, j0, jb, tid, need_more ? colsum : nullptr, &s_fail);
      __syncthreads();
      if (s_fail) break;
      // 2. row panel X = R_JJ^-T W[J, c] for the left columns right of the
      //    block and the right columns that can be non-zero (< j0 + jb), on
      //    the FP64 matrix cores: 16 x 16 tiles of X (rows i, columns pc),
      //    A(i, k) = R_JJ^-T(i, k) from D, B(k, j) = W[j0 + k, col(pc0 + j)].
      //    X goes back to W and, zero-padded to NB rows, to the panel P.
      const int nleft = m - j0 - jb;
      for (int ct = wv; ct < (m + 15) / 16; ct += nw) {
        const int pc = 16 * ct + (lane & 15);
        const bool okc = pc < m;
        const int64_t col = pc < nleft ? (int64_t)(j0 + jb + pc) : (int64_t)m + (pc - nleft);
        double bv[NB / 4];
#pragma unroll
        for (int kk = 0; kk < NB / 4; ++kk) {
          const int k = 4 * kk + (lane >> 4);
          bv[kk] = (okc && k < jb) ? W[(int64_t)(j0 + k) * m2 + col] : 0.0;
        }
        doublex4 x0 = {0.0, 0.0, 0.0, 0.0}, x1 = x0;
#pragma unroll
        for (int kk = 0; kk < NB / 4; ++kk) {
          const int k = 4 * kk + (lane >> 4);
          x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(D[(lane & 15) * (NB + 1) + k], bv[kk], x0, 0, 0, 0);
          x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(D[(16 + (lane & 15)) * (NB + 1) + k], bv[kk], x1, 0, 0, 0);
        }
        double cs = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i0 = (lane >> 4) + 4 * q, i1 = i0 + 16;
          if (okc) {
            if (i0 < jb) W[(int64_t)(j0 + i0) * m2 + col] = x0[q];
            if (i1 < jb) W[(int64_t)(j0 + i1) * m2 + col] = x1[q];
            P[i0 * m + pc] = x0[q];
            P[i1 * m + pc] = x1[q];
          }
          cs += fabs(x0[q]) + fabs(x1[q]);
        }
        if (need_more) {
          cs += __shfl_xor(cs, 16, 64);
          cs += __shfl_xor(cs, 32, 64);
          if (lane < 16 && pc < nleft) colsum[col] += cs;
        }
      }
      __syncthreads();
      // 3. trailing update of the rows below the block on the FP64 matrix
      //    cores: W[r, col(pc)] -= sum_t P[t][pr] P[t][pc] in 16 x 16 tiles
      //    (v_mfma_f64_16x16x4f64; A(i, k) = -P[k][pr0 + i], B(k, j) = P[k][pc0 + j];
      //    output lane l, register q: row (l / 16) + 4 q, column l % 16).
      //    Only live tiles are enumerated: tile row tr of the left part starts
      //    at the diagonal (tiles wholly below it are never read), and only
      //    the upper triangle of the left part is written.
      {
        const int nrows = nleft;
        const int tr_n = (nrows + 15) / 16, tc_n = (m + 15) / 16;
        const int FL = nleft / 16;  // tiles tc < FL lie wholly in the left part
        int nlive = 0;
        for (int tr = 0; tr < tr_n; ++tr) nlive += tc_n - min(tr, FL);
        // four tiles per pass, so that their 16 loads per lane overlap
        constexpr int UT = 4;
        for (int base = UT * wv; base < nlive; base += UT * nw) {
          doublex4 acc[UT];
          int64_t gofs[UT][4];
          bool ok[UT][4];
          bool live[UT];
          int pras[UT], pcs[UT];
#pragma unroll
          for (int u = 0; u < UT; ++u) {
            int li = base + u;
            live[u] = li < nlive;
            if (!live[u]) li = 0;
            int tr = 0, len = tc_n;
            while (li >= len) { li -= len; ++tr; len = tc_n - min(tr, FL); }
            const int tc = min(tr, FL) + li;
            pras[u] = 16 * tr + (lane & 15);
            const int pc = 16 * tc + (lane & 15);
            pcs[u] = pc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int pr = 16 * tr + (lane >> 4) + 4 * q;
              ok[u][q] = live[u] && pr < nrows && pc < m && (pc >= nleft || pc >= pr);
              const int64_t col = pc < nleft ? (int64_t)(j0 + jb + pc) : (int64_t)m + (pc - nleft);
              gofs[u][q] = (int64_t)(j0 + jb + pr) * m2 + col;
              acc[u][q] = ok[u][q] ? W[gofs[u][q]] : 0.0;
            }
          }
          // k outer, tiles inner: the UT accumulation chains interleave
#pragma unroll
          for (int k0 = 0; k0 < NB; k0 += 4) {
            const int t = k0 + (lane >> 4);
#pragma unroll
            for (int u = 0; u < UT; ++u) {
              const double av = (live[u] && pras[u] < nrows) ? -P[t * m + pras[u]] : 0.0;
              const double bv = (live[u] && pcs[u] < m) ? P[t * m + pcs[u]] : 0.0;
              acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
            }
          }
#pragma unroll
          for (int u = 0; u < UT; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (ok[u][q]) W[gofs[u][q]] = acc[u][q];
        }
      }
      __syncthreads();
    }
    __syncthreads();
    if (!s_fail) break;
    if (tid == 0) {
      atomicOr(flags, attempt == 0 ? SKETCHNE_FLAG_CHOL_SHIFT : SKETCHNE_FLAG_CHOL_FAIL);
      s_shifted = 1;
    }
    __syncthreads();
  }
  // R^-T = Rs^-T S^-1 from the lower triangle of the right half (zeros above
  // it), and the row sums of |Rs^-T| for the condition number
  double rmax = 0.0;
  for (int r0 = 4 * wv; r0 < m; r0 += 4 * nw) {
    double x[4][CH_CHUNKS];
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int cc = 0; cc < CH_CHUNKS; ++cc) {
        const int r = r0 + h, c = lane + 64 * cc;
        x[h][cc] = (r < m && c <= r) ? W[(int64_t)r * m2 + m + c] : 0.0;
      }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int r = r0 + h;
      if (r >= m) break;
      double rs = 0.0;
#pragma unroll
      for (int cc = 0; cc < CH_CHUNKS; ++cc) {
        const int c = lane + 64 * cc;
        if (c < m) RinvT[(int64_t)r * m + c] = x[h][cc] * rsc[c];
        rs += fabs(x[h][cc]);
      }
      rmax = fmax(rmax, wave_sum(rs));
    }
  }
  if (need_more) {
    // kappa_1(Rs) = ||Rs||_1 ||Rs^-1||_1: the largest column sum of Rs and
    // the largest row sum of Rs^-T
    double cmax = 0.0;
    for (int j = tid; j < m; j += nt) cmax = fmax(cmax, colsum[j]);
    cmax = wave_max(cmax);
    if (lane == 0) { s_red[0][wv] = cmax; s_red[1][wv] = rmax; }
    __syncthreads();
    if (tid == 0) {
      double a = 0.0, b = 0.0;
      for (int w = 0; w < nw; ++w) { a = fmax(a, s_red[0][w]); b = fmax(b, s_red[1][w]); }
      double kappa = a * b;
      *need_more = (s_shifted || !(kappa <= repeat_kappa)) ? 1 : 0;
    }
  }
}

// grid-stride copy over a fixed grid, so that a skipped copy costs one launch
__global__ void k_copy_if(int64_t count, const float* __restrict__ src, float* __restrict__ dst,
                          const int* __restrict__ run_if) {
  if (run_if && *run_if == 0) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4;
  for (; i + 3 < count; i += 4 * stride) *reinterpret_cast<float4*>(dst + i) = *reinterpret_cast<const float4*>(src + i);
  for (; i < count; ++i) dst[i] = src[i];
}

// ---------------------------------------------------------------- Jacobi
//
// One-sided (Hestenes) block Jacobi on B = A + c I with c = 1.5 ||A||_F, so
// the eigenvalues of B lie in [0.5, 2.5] ||A||_F: B is positive definite with
// condition number at most 5, eigenvalues +-lambda of A cannot mix, and at
// convergence the columns of G = B V are (lambda_j + c) v_j.  The
// eigenvectors are therefore the normalised columns of G (accurate to a few
// units of rounding because B is well conditioned) and lambda_j =
// ||g_j|| - c; V itself is never formed.  The same sweeps on a general
// (non-symmetric) matrix A with c = 0 give its singular value decomposition:
// at convergence G = A J has orthogonal columns sigma_j u_j, so the
// normalised columns are the left singular vectors and the norms the
// singular values (J, the right singular vectors, is not formed).
//
// Columns are grouped in blocks of NBJ = 16.  A sweep is one "intra" round
// (the pairs inside each block) and nb - 1 "cross" rounds that pair the
// blocks by the round-robin (circle) schedule.  In a cross round one
// workgroup takes a block pair (P, Q); group g of 16 lanes keeps column g of P
// in registers for all 16 rounds and meets column (g + round) mod 16 of Q,
// which is the only data that moves (through LDS).  Columns are stored with
// 288 rows (zero below m), a lane holds pairs of adjacent rows strided by 32,
// and the three inner products are reduced by DPP.
// Every sweep counts its rotations and its "large" rotations (|g| above
// OJ_BIG sqrt(ab)).  A sweep without a large rotation ends the iteration:
// the off-diagonal it leaves is of the order of the square of that bound
// (cyclic Jacobi converges quadratically), so a further sweep would only
// confirm it.
constexpr int NBJ = 16;           // columns per block
constexpr int OJ_GL = 16;         // lanes per column (one DPP row)
constexpr int OJ_MAXR = 18;       // rows per lane: m <= OJ_GL * OJ_MAXR = 288
constexpr int OJ_ROWS = OJ_GL * OJ_MAXR;  // stored column length; rows m.. are zero
constexpr int OJ_THREADS = NBJ * OJ_GL;
constexpr double OJ_SHIFT = 1.5;  // c = OJ_SHIFT * ||A||_F
constexpr double OJ_BIG = 1e-8;   // a rotation with |g| > OJ_BIG sqrt(ab) is large
constexpr int kMaxSweeps = 30;

__device__ __forceinline__ void pair_of(int s, int pi, int mp, int& p, int& q) {
  const int ring = mp - 1;
  int a, b;
  if (pi == 0) { a = mp - 1; b = s; }
  else { a = (s + pi) % ring; b = (s - pi + ring) % ring; }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

// one DPP move of a double (two 32-bit halves)
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, true);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, true);
  return __hiloint2double(hi, lo);
}

// sum over the 16 lanes of a DPP row; every lane of the row gets the total
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0x141>(v);  // row_half_mirror
  v += dpp_d<0x140>(v);  // row_mirror
  return v;
}

// sum over the OJ_GL lanes of a column group; every lane gets it
__device__ __forceinline__ double group_sum(double v) {
  v = row16_sum(v);
  if (OJ_GL == 32) v += __shfl_xor(v, 16, 64);
  return v;
}

// c = OJ_SHIFT * ||A||_F over the symmetric matrix given by its upper
// triangle; c = 0 for a general matrix (its singular value decomposition)
__global__ __launch_bounds__(1024) void k_oj_norm(int m, const double* __restrict__ A, int general,
                                                  double* __restrict__ shift) {
  if (general) {
    if (threadIdx.x == 0) *shift = 0.0;
    return;
  }
  __shared__ double part[16];
  // ||A||_F^2 from the upper triangle (off-diagonal entries twice), eight
  // loads in flight per thread
  constexpr int BATCH = 8;
  const int mm = m * m, nt = blockDim.x;
  double s = 0.0;
  for (int base = threadIdx.x; base < mm; base += nt * BATCH) {
    double a[BATCH], wt[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int idx = base + nt * u;
      const int r = idx / m, c = idx - r * m;
      a[u] = (idx < mm && c >= r) ? A[idx] : 0.0;
      wt[u] = c > r ? 2.0 : 1.0;
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) s = fma(a[u] * wt[u], a[u], s);
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += part[w];
    *shift = OJ_SHIFT * sqrt(t);
  }
}

// G (column-major, mp columns of OJ_ROWS rows) = A + c I, zero-padded in both
// directions (zero rows stay zero under rotations, so the kernels below need
// no row bounds), counters = 0
__global__ void k_oj_init(int m, int mp, const double* __restrict__ A, int general, const double* __restrict__ shift,
                          double* __restrict__ G, int* __restrict__ counters, int max_sweeps) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < max_sweeps) counters[idx] = 0;
  if (idx >= mp * OJ_ROWS) return;
  int c = idx / OJ_ROWS, r = idx - c * OJ_ROWS;
  double g = 0.0;
  if (c < m && r < m) {
    if (general) {
      g = A[r * m + c];
    } else {
      g = r <= c ? A[r * m + c] : A[c * m + r];
      if (r == c) g += *shift;
    }
  }
  G[idx] = g;
}

// Jacobi rotation that orthogonalises the pair (x, y) given a = x.x, b = y.y,
// g = x.y; returns false when the pair is already orthogonal to 1e-14; `big`
// reports |g| > OJ_BIG sqrt(ab).  The angle is the smaller one,
// |theta| <= pi / 4: with d = b - a and h = sqrt(d^2 + 4 g^2),
// cos(2 theta) = |d| / h and sin(2 theta) = sgn(d) 2 g / h, so
// c^2 = (1 + |d| / h) / 2 and s = sgn(d) g / (h c) (tan(theta) =
// sgn(d) 2g / (|d| + h)); two reciprocal square roots and no division keep
// the dependent chain short.  t = tan(theta) = s / c is returned for the
// norm update: the rotated pair x' = c x - s y, y' = s x + c y has
// x'.x' = a - t g and y'.y' = b + t g (its Gram matrix keeps its trace and
// loses the off-diagonal g).
__device__ __forceinline__ bool oj_angle(double a, double b, double g, double& c, double& sn, double& t, bool& big) {
  const double tol = 1e-14;
  const double g2 = g * g, ab = a * b;
  big = false;
  if (!(a > 0.0 && b > 0.0 && g2 > (tol * tol) * ab)) return false;
  big = g2 > (OJ_BIG * OJ_BIG) * ab;
  const double d = b - a;
  const double rh = rsqrt(fma(d, d, 4.0 * g2));  // 1 / h
  const double c2 = fma(fabs(d), 0.5 * rh, 0.5);  // c^2
  const double rc = rsqrt(c2);                    // 1 / c
  c = c2 * rc;
  sn = (d >= 0.0 ? g : -g) * rh * rc;
  t = sn * rc;
  return true;
}

// Lane sub of a column group holds rows 2 sub + 2 OJ_GL i and the row after
// it (i < OJ_MAXR / 2): one 16-byte access per pair, and the 16 lanes of a
// group cover 256 contiguous bytes.
__device__ __forceinline__ int oj_row(int sub, int i) { return 2 * sub + 2 * OJ_GL * i; }

// this lane's share of x.y, in three interleaved partial sums so that the
// FMAs do not form one dependent chain
__device__ __forceinline__ double oj_dot(const double* x, const double* y) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int i = 0; i < OJ_MAXR; i += 3) {
    s0 = fma(x[i], y[i], s0);
    s1 = fma(x[i + 1], y[i + 1], s1);
    s2 = fma(x[i + 2], y[i + 2], s2);
  }
  return (s0 + s1) + s2;
}

__device__ __forceinline__ void oj_load_col(const double* __restrict__ col, int sub, double* x) {
#pragma unroll
  for (int i = 0; i < OJ_MAXR / 2; ++i) {
    const double2 u = *reinterpret_cast<const double2*>(col + oj_row(sub, i));
    x[2 * i] = u.x;
    x[2 * i + 1] = u.y;
  }
}

// The squared column norms are computed once per round and then carried
// through the rotations (a - t g, b + t g) instead of being recomputed, so a
// rotation step computes one inner product.  With the shift c >= 1.5 ||A||_F
// every column norm stays above (c - ||A||_2)^2 > 0, so the update never
// cancels.

// orthogonalise columns p and q of sG (LDS, column-major, OJ_ROWS rows) by
// the lanes of one column group, nrm holding their squared norms; returns
// whether a rotation was applied
__device__ __forceinline__ bool oj_rotate_lds(double* __restrict__ sG, double* __restrict__ nrm, int p, int q, int sub,
                                              bool& big) {
  double* gp = sG + p * OJ_ROWS;
  double* gq = sG + q * OJ_ROWS;
  double x[OJ_MAXR], y[OJ_MAXR];
  oj_load_col(gp, sub, x);
  oj_load_col(gq, sub, y);
  const double a = nrm[p], b = nrm[q];
  const double g = group_sum(oj_dot(x, y));
  double c, sn, t;
  if (!oj_angle(a, b, g, c, sn, t, big)) return false;
#pragma unroll
  for (int i = 0; i < OJ_MAXR / 2; ++i) {
    *reinterpret_cast<double2*>(gp + oj_row(sub, i)) =
        make_double2(c * x[2 * i] - sn * y[2 * i], c * x[2 * i + 1] - sn * y[2 * i + 1]);
    *reinterpret_cast<double2*>(gq + oj_row(sub, i)) =
        make_double2(sn * x[2 * i] + c * y[2 * i], sn * x[2 * i + 1] + c * y[2 * i + 1]);
  }
  if (sub == 0) {
    nrm[p] = a - t * g;
    nrm[q] = b + t * g;
  }
  return true;
}

// load / store contiguous columns of OJ_ROWS doubles with double2,
// `batch` transfers in flight per thread
__device__ __forceinline__ void oj_block_load(const double* __restrict__ src, double* __restrict__ dst, int count) {
  constexpr int BATCH = NBJ * OJ_ROWS / (2 * OJ_THREADS);  // one block in a single batch
  for (int base = 2 * threadIdx.x; base < count; base += 2 * blockDim.x * BATCH) {
    double2 v[BATCH];
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int idx = base + 2 * blockDim.x * u;
      v[u] = idx < count ? *reinterpret_cast<const double2*>(src + idx) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < BATCH; ++u) {
      const int idx = base + 2 * blockDim.x * u;
      if (idx < count) *reinterpret_cast<double2*>(dst + idx) = v[u];
    }
  }
}

// workgroup w orthogonalises the pairs inside blocks 2w and 2w+1 (both in LDS)
__device__ __forceinline__ void oj_intra_round(int w, int sweep, double* __restrict__ G, int* __restrict__ counters,
                                               double* __restrict__ sG, double* __restrict__ nrm, int* s_cnt) {
  const int tid = threadIdx.x;
  if (tid == 0) s_cnt[0] = s_cnt[1] = 0;
  const int blk = NBJ * OJ_ROWS;
  double* g0 = G + (int64_t)(2 * w) * blk;  // blocks 2w, 2w+1 are contiguous
  oj_block_load(g0, sG, 2 * blk);
  __syncthreads();
  const int grp = tid / OJ_GL, sub = tid % OJ_GL;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    double x[OJ_MAXR];
    const int col = grp + NBJ * h;
    oj_load_col(sG + col * OJ_ROWS, sub, x);
    const double a = group_sum(oj_dot(x, x));
    if (sub == 0) nrm[col] = a;
  }
  __syncthreads();
  int my_rot = 0, my_big = 0;
  for (int rnd = 0; rnd < NBJ - 1; ++rnd) {
    const int half = grp >> 3;  // 8 groups per block
    int p, q;
    pair_of(rnd, grp & 7, NBJ, p, q);
    bool big;
    if (oj_rotate_lds(sG, nrm, p + half * NBJ, q + half * NBJ, sub, big) && sub == 0) {
      ++my_rot;
      my_big += big;
    }
    __syncthreads();
  }
  if (sub == 0 && my_rot) atomicAdd(&s_cnt[0], my_rot);
  if (sub == 0 && my_big) atomicAdd(&s_cnt[1], my_big);
  oj_block_load(sG, g0, 2 * blk);
  __syncthreads();
  if (tid == 0 && s_cnt[0]) atomicAdd(&counters[sweep], s_cnt[0]);
  if (tid == 0 && s_cnt[1]) atomicAdd(&counters[kMaxSweeps + sweep], s_cnt[1]);
}

// workgroup w takes the block pair w of round s: column g of block P stays
// in the registers of lane group g, the 16 columns of block Q rotate past it
// (their squared norms travel with them in nrm)
__device__ __forceinline__ void oj_cross_round(int w, int nb, int s, int sweep, double* __restrict__ G,
                                               int* __restrict__ counters, double* __restrict__ sQ,
                                               double* __restrict__ nrm, int* s_cnt) {
  int P, Q;
  pair_of(s, w, nb, P, Q);
  const int tid = threadIdx.x, grp = tid / OJ_GL, sub = tid % OJ_GL;
  if (tid == 0) s_cnt[0] = s_cnt[1] = 0;
  const int blk = NBJ * OJ_ROWS;
  double* gpcol = G + (int64_t)P * blk + (int64_t)grp * OJ_ROWS;
  double* gQ = G + (int64_t)Q * blk;
  double x[OJ_MAXR];
  oj_load_col(gpcol, sub, x);
  oj_block_load(gQ, sQ, blk);
  double a = group_sum(oj_dot(x, x));
  __syncthreads();
  {
    double y[OJ_MAXR];
    oj_load_col(sQ + grp * OJ_ROWS, sub, y);
    const double b = group_sum(oj_dot(y, y));
    if (sub == 0) nrm[grp] = b;
  }
  __syncthreads();
  int my_rot = 0, my_big = 0;
  for (int rnd = 0; rnd < NBJ; ++rnd) {
    const int qc = (grp + rnd) & (NBJ - 1);
    double* gq = sQ + qc * OJ_ROWS;
    double y[OJ_MAXR];
    oj_load_col(gq, sub, y);
    const double b = nrm[qc];
    const double g = group_sum(oj_dot(x, y));
    double c, sn, t;
    bool big;
    if (oj_angle(a, b, g, c, sn, t, big)) {
#pragma unroll
      for (int i = 0; i < OJ_MAXR / 2; ++i) {
        const double x0 = x[2 * i], x1 = x[2 * i + 1];
        x[2 * i] = c * x0 - sn * y[2 * i];
        x[2 * i + 1] = c * x1 - sn * y[2 * i + 1];
        *reinterpret_cast<double2*>(gq + oj_row(sub, i)) =
            make_double2(sn * x0 + c * y[2 * i], sn * x1 + c * y[2 * i + 1]);
      }
      a -= t * g;
      if (sub == 0) {
        nrm[qc] = b + t * g;
        ++my_rot;
        my_big += big;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < OJ_MAXR / 2; ++i)
    *reinterpret_cast<double2*>(gpcol + oj_row(sub, i)) = make_double2(x[2 * i], x[2 * i + 1]);
  if (sub == 0 && my_rot) atomicAdd(&s_cnt[0], my_rot);
  if (sub == 0 && my_big) atomicAdd(&s_cnt[1], my_big);
  oj_block_load(sQ, gQ, blk);
  __syncthreads();
  if (tid == 0 && s_cnt[0]) atomicAdd(&counters[sweep], s_cnt[0]);
  if (tid == 0 && s_cnt[1]) atomicAdd(&counters[kMaxSweeps + sweep], s_cnt[1]);
}

// All sweeps in one launch of nb / 2 workgroups (one per block pair of a
// round): a grid barrier separates the rounds, and after the last
// round of a sweep every workgroup reads that sweep's count of large
// rotations (final once the barrier has passed) and leaves the loop when it is
// zero, so the stopping rule needs no host round trip.  The rounds and their
// arithmetic are those of a sweep-per-launch schedule, so the results do not
// depend on the launch shape.
// counters[2 * kMaxSweeps] is the grid barrier's arrival count.
__global__ __launch_bounds__(OJ_THREADS) void k_oj_sweeps(int nb, double* __restrict__ G, int* __restrict__ counters,
                                                          uint32_t* __restrict__ flags) {
  extern __shared__ __attribute__((aligned(16))) double lds[];
  __shared__ double s_nrm[2 * NBJ];  // squared column norms of the blocks in LDS
  __shared__ int s_cnt[2];
  __shared__ int s_stop;
  __shared__ int s_abort;
  uint32_t* bar = reinterpret_cast<uint32_t*>(counters + 2 * kMaxSweeps);
  uint32_t target = 0;
  const int w = blockIdx.x;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    oj_intra_round(w, sweep, G, counters, lds, s_nrm, s_cnt);
    if (!grid_barrier(bar, target, flags, &s_abort)) return;
    for (int s = 0; s < nb - 1; ++s) {
      oj_cross_round(w, nb, s, sweep, G, counters, lds, s_nrm, s_cnt);
      if (!grid_barrier(bar, target, flags, &s_abort)) return;
    }
    if (threadIdx.x == 0)
      s_stop = __hip_atomic_load(&counters[kMaxSweeps + sweep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
    __syncthreads();
    if (s_stop) break;
    __syncthreads();  // s_stop is rewritten only after every thread has read it
  }
}

// lambda_j = ||g_j|| - c and v_j = g_j / ||g_j||; sort by |lambda| desc
// (ties: lambda desc, then index); write w and the eigenvectors as the
// columns of the row-major Vout.  Workgroup b writes rows 32 b .. 32 b + 31
// of Vout: every workgroup computes all norms and the order itself (a few
// microseconds), then moves the 32-row segments of every column (256-byte
// reads) through LDS and writes whole output rows.
constexpr int OJF_ROWS = 32;  // output rows per workgroup
__global__ __launch_bounds__(1024) void k_oj_finish(int m, const double* __restrict__ G,
                                                    const double* __restrict__ shift, const int* __restrict__ counters,
                                                    int sweeps_run, double* __restrict__ Vout,
                                                    double* __restrict__ wout, uint32_t* __restrict__ flags) {
  extern __shared__ __attribute__((aligned(16))) double tile[];  // m x OJF_ROWS, row stride OJF_ROWS + 1
  __shared__ double w[OJ_ROWS];
  __shared__ double inv[OJ_ROWS];
  __shared__ int perm[OJ_ROWS];  // perm[p] = column of G that goes to position p
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nwv = blockDim.x >> 6, nt = blockDim.x;
  const bool lead = blockIdx.x == 0;
  const int r0 = OJF_ROWS * blockIdx.x;
  if (lead && tid == 0) {
    bool conv = false;
    for (int s = 0; s < sweeps_run; ++s)
      if (counters[kMaxSweeps + s] == 0) { conv = true; break; }
    if (!conv) atomicOr(flags, SKETCHNE_FLAG_EIG_NOCONV);
  }
  const double cs = *shift;
  // this workgroup's row segments: issued first, stored to LDS after the norms
  constexpr int TB = (OJ_ROWS * OJF_ROWS + 1023) / 1024;
  double seg[TB];
#pragma unroll
  for (int u = 0; u < TB; ++u) {
    const int idx = tid + nt * u;
    const int j = idx / OJF_ROWS, rr = idx - j * OJF_ROWS;
    seg[u] = (j < m && r0 + rr < m) ? G[(int64_t)j * OJ_ROWS + r0 + rr] : 0.0;
  }
  // column norms: a wavefront takes three columns at a time, all their loads
  // in flight
  constexpr int RPL = (OJ_ROWS + 63) / 64;  // rows per lane
  for (int j0 = 3 * wave; j0 < m; j0 += 3 * nwv) {
    double v[3][RPL];
#pragma unroll
    for (int u = 0; u < 3; ++u)
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int j = j0 + u, r = lane + 64 * i;
        v[u][i] = (j < m && r < m) ? G[(int64_t)j * OJ_ROWS + r] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      double d = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) d = fma(v[u][i], v[u][i], d);
      d = wave_sum(d);
      const int j = j0 + u;
      if (lane == 0 && j < m) {
        const double nrm = sqrt(d);
        w[j] = nrm - cs;
        inv[j] = nrm > 0.0 ? 1.0 / nrm : 0.0;
        if (lead && !isfinite(w[j])) atomicOr(flags, SKETCHNE_FLAG_NONFINITE);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < TB; ++u) {
    const int idx = tid + nt * u;
    const int j = idx / OJF_ROWS, rr = idx - j * OJF_ROWS;
    if (j < m) tile[j * (OJF_ROWS + 1) + rr] = seg[u];
  }
  __syncthreads();
  for (int i = tid; i < m; i += nt) {
    double ai = fabs(w[i]);
    int rk = 0;
    for (int j = 0; j < m; ++j) {
      double aj = fabs(w[j]);
      bool before = (aj > ai) || (aj == ai && (w[j] > w[i] || (w[j] == w[i] && j < i)));
      rk += before ? 1 : 0;
    }
    perm[rk] = i;
    if (lead) wout[rk] = w[i];
  }
  __syncthreads();
  // Vout[r][p] = G[perm[p]][r] / ||g||, consecutive threads along a row
  for (int idx = tid; idx < OJF_ROWS * m; idx += nt) {
    const int rr = idx / m, p = idx - rr * m, r = r0 + rr;
    if (r >= m) break;
    const int j = perm[p];
    const double s = inv[j];
    // a zero matrix (c = 0) has G = 0: its eigenvectors are the unit vectors
    Vout[(int64_t)r * m + p] = s > 0.0 ? tile[j * (OJF_ROWS + 1) + rr] * s : (r == j ? 1.0 : 0.0);
  }
}

constexpr int oj_nblocks(int m) {
  return (m + NBJ - 1) / NBJ + (((m + NBJ - 1) / NBJ) & 1);
}

constexpr size_t oj_align(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// workspace of the eigensolver of order m: the padded column block, the
// per-sweep rotation counts and the grid barrier's count, and the shift
constexpr size_t oj_ws_bytes(int m) {
  return oj_align(sizeof(double) * (size_t)(oj_nblocks(m) * NBJ) * OJ_ROWS) +
         oj_align(sizeof(int) * (2 * kMaxSweeps + 1)) + oj_align(sizeof(double));
}

// The no-allocation variant's scratch: the workspace of the largest order, in
// a file-scope device array.  Every device that loads the library holds its
// own copy until the process ends.  On the host the name `scratch` is only a
// stand-in for the symbol, never a device address: host code uses the
// address hipGetSymbolAddress returns for the current device.
constexpr size_t kSymeigScratchBytes = oj_ws_bytes(kSymeigMax);
static __device__ __align__(256) char scratch[kSymeigScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The same factorization spread over a few workgroups of one launch, for
// orders where the trailing updates of a single workgroup (one
// CU's FP64 matrix cores) dominate.  Every workgroup factors the diagonal
// block and forms the whole row panel itself (both are small), so that only
// the trailing update is divided: its live tiles are dealt to all wavefronts
// of the grid, and one grid barrier per block step publishes the updated rows.
// Entries of the left half are never read once their block row is done, so
// R itself is not stored: the row panel lives in LDS (its column sums feed the
// condition estimate), and its right-half part, the block row of R^-T, is
// written to W at the start of the next step, after the barrier, when no
// workgroup reads those entries any more.  Decisions (a failed pivot, the
// shifted retry) depend only on data every workgroup reads identically, so all
// workgroups take the same path and meet the same barriers.
__global__ __launch_bounds__(512) void k_chol_inv_coop(int m, const double* __restrict__ G, double* __restrict__ W,
                                                       double* __restrict__ rpart, double* __restrict__ RinvT,
                                                       uint32_t* __restrict__ flags, int* __restrict__ need_more,
                                                       const int* __restrict__ run_if, double repeat_kappa,
                                                       uint32_t* __restrict__ bar) {
  if (run_if && *run_if == 0) return;
  extern __shared__ double smem[];
  // two NB x (NB+1) diagonal-block buffers (this step's, the next one's),
  // then the NB x m panel; buffers are offsets from the LDS array
  constexpr int DSZ = NB * (NB + 1);
  double* P = smem + 2 * DSZ;
  __shared__ double rsc[CH_MAXM];
  __shared__ double colsum[CH_MAXM];
  __shared__ __attribute__((aligned(16))) double xrow[64];
  __shared__ double s_red[2][8];
  __shared__ int s_fail;
  __shared__ int s_shifted;
  __shared__ int s_abort;
  uint32_t target = 0;  // grid barrier count
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), nw = nt >> 6;
  const int wg = blockIdx.x, nwg = gridDim.x;
  const int gw = wg * nw + wv, gnw = nwg * nw;  // wavefront index in the grid
  const int64_t m2 = 2 * (int64_t)m;

  double trp = 0.0;
  for (int i = tid; i < m; i += nt) {
    const double g = G[(int64_t)i * m + i];
    const double r = (g > 0.0 && isfinite(g)) ? 1.0 / sqrt(g) : 1.0;
    rsc[i] = r;
    trp += fabs(g) * r * r;
  }
  trp = wave_sum(trp);
  if (lane == 0) s_red[0][wv] = trp;
  if (tid == 0) s_shifted = 0;
  __syncthreads();
  double tr = 0.0;
  for (int w = 0; w < nw; ++w) tr += s_red[0][w];
  const double retry_shift = 11.0 * ((double)m * m + m) * 1.1102230246251565e-16 * (tr > 0 ? tr : 1.0);

  // block row (pj0, pjb) of R^-T from the panel in LDS to W
  auto store_right = [&](int pj0, int pjb) {
    const int pleft = m - pj0 - pjb, wr = pj0 + pjb;
    for (int idx = wg * nt + tid; idx < pjb * wr; idx += nwg * nt) {
      const int i = idx / wr, j = idx - i * wr;
      W[(int64_t)(pj0 + i) * m2 + m + j] = P[i * m + pleft + j];
    }
  };

  int pj0 = 0, pjb = 0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    const double shift = attempt == 0 ? 0.0 : retry_shift;
    for (int r0 = 4 * gw; r0 < m; r0 += 4 * gnw) {
      double v[4][CH_CHUNKS];
#pragma unroll
      for (int h = 0; h < 4; ++h)
#pragma unroll
        for (int cc = 0; cc < CH_CHUNKS; ++cc) {
          const int r = r0 + h, c = lane + 64 * cc;
          v[h][cc] = (r < m && c < m && c >= r) ? G[(int64_t)r * m + c] : 0.0;
        }
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        const int r = r0 + h;
        if (r >= m) break;
        double* row = W + (int64_t)r * m2;
        const int rend = min(m, (r / NB + 1) * NB);
        const double rr = rsc[r];
#pragma unroll
        for (int cc = 0; cc < CH_CHUNKS; ++cc) {
          const int c = lane + 64 * cc;
          if (c < m && c >= r) row[c] = v[h][cc] * rr * rsc[c] + (c == r ? shift : 0.0);
          if (c < rend) row[m + c] = c == r ? 1.0 : 0.0;
        }
      }
    }
    for (int j = tid; j < m; j += nt) colsum[j] = 0.0;
    if (tid == 0) s_fail = 0;
    pjb = 0;
    if (!grid_barrier(bar, target, flags, &s_abort)) return;

    int dcur = 0;         // buffer of this step's diagonal block
    bool have_d = false;  // already factored during the previous step
    for (int j0 = 0; j0 < m; j0 += NB) {
      const int jb = min(NB, m - j0);
      if (pjb) store_right(pj0, pjb);
      double* D = smem + dcur * DSZ;
      if (!have_d) {
        for (int idx = tid; idx < NB * NB; idx += nt) {
          const int a = idx / NB, b = idx % NB;
          D[a * (NB + 1) + b] = (b < jb && a <= b) ? W[(int64_t)(j0 + a) * m2 + j0 + b] : 0.0;
        }
        __syncthreads();
        if (tid < 64) chol_diag_wave(D, xrow, nullptr, m2, j0, jb, tid, need_more ? colsum : nullptr, &s_fail);
        __syncthreads();
      }
      if (s_fail) break;
      // row panel of the whole block row (every workgroup), into LDS only
      const int nleft = m - j0 - jb;
      for (int ct = wv; ct < (m + 15) / 16; ct += nw) {
        const int pc = 16 * ct + (lane & 15);
        const bool okc = pc < m;
        const int64_t col = pc < nleft ? (int64_t)(j0 + jb + pc) : (int64_t)m + (pc - nleft);
        double bv[NB / 4];
#pragma unroll
        for (int kk = 0; kk < NB / 4; ++kk) {
          const int k = 4 * kk + (lane >> 4);
          bv[kk] = (okc && k < jb) ? W[(int64_t)(j0 + k) * m2 + col] : 0.0;
        }
        doublex4 x0 = {0.0, 0.0, 0.0, 0.0}, x1 = x0;
#pragma unroll
        for (int kk = 0; kk < NB / 4; ++kk) {
          const int k = 4 * kk + (lane >> 4);
          x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(D[(lane & 15) * (NB + 1) + k], bv[kk], x0, 0, 0, 0);
          x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(D[(16 + (lane & 15)) * (NB + 1) + k], bv[kk], x1, 0, 0, 0);
        }
        double cs = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i0 = (lane >> 4) + 4 * q, i1 = i0 + 16;
          if (okc) {
            P[i0 * m + pc] = x0[q];
            P[i1 * m + pc] = x1[q];
          }
          cs += fabs(x0[q]) + fabs(x1[q]);
        }
        if (need_more) {
          cs += __shfl_xor(cs, 16, 64);
          cs += __shfl_xor(cs, 32, 64);
          if (lane < 16 && pc < nleft) colsum[col] += cs;
        }
      }
      __syncthreads();
      // Look-ahead: wavefront 0 of every workgroup forms the next diagonal
      // block from the panel (its entries before this step's update minus
      // P^T P; nobody writes them back, since no later step reads them) and
      // factors it, while the other wavefronts run the trailing update.
      const int jbn = min(NB, nleft);
      const bool ahead = nleft > 0;
      if (ahead && wv == 0) {
        double* Dn = smem + (dcur ^ 1) * DSZ;
        for (int ti = 0; ti < 2; ++ti)
          for (int tj = ti; tj < 2; ++tj) {
            doublex4 acc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int a = 16 * ti + (lane >> 4) + 4 * q, b = 16 * tj + (lane & 15);
              acc[q] = (a < jbn && b < jbn && a <= b) ? W[(int64_t)(j0 + jb + a) * m2 + j0 + jb + b] : 0.0;
            }
#pragma unroll
            for (int k0 = 0; k0 < NB; k0 += 4) {
              const int t = k0 + (lane >> 4);
              const int pa = 16 * ti + (lane & 15), pb = 16 * tj + (lane & 15);
              const double av = (t < jb && pa < jbn) ? -P[t * m + pa] : 0.0;
              const double bv = (t < jb && pb < jbn) ? P[t * m + pb] : 0.0;
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int a = 16 * ti + (lane >> 4) + 4 * q, b = 16 * tj + (lane & 15);
              Dn[a * (NB + 1) + b] = (a < jbn && b < jbn && a <= b) ? acc[q] : 0.0;
            }
          }
        // (one wavefront: its LDS writes complete before its reads below)
        chol_diag_wave(Dn, xrow, nullptr, m2, j0 + jb, jbn, lane, need_more ? colsum : nullptr, &s_fail);
      }
      // trailing update: the live tiles over the other wavefronts of the
      // grid, without the next diagonal block's tiles
      {
        const int nrows = nleft;
        const int tr_n = (nrows + 15) / 16, tc_n = (m + 15) / 16;
        const int FL = nleft / 16;
        int nlive = 0;
        for (int tr = 0; tr < tr_n; ++tr) nlive += tc_n - min(tr, FL);
        constexpr int UT = 4;
        const int tw = ahead ? wg * (nw - 1) + (wv - 1) : gw;  // wavefront 0 is busy when ahead
        const int tnw = ahead ? nwg * (nw - 1) : gnw;
        for (int base = UT * tw; (!ahead || wv > 0) && base < nlive; base += UT * tnw) {
          doublex4 acc[UT];
          int64_t gofs[UT][4];
          bool ok[UT][4];
          bool live[UT];
          int pras[UT], pcs[UT];
#pragma unroll
          for (int u = 0; u < UT; ++u) {
            int li = base + u;
            live[u] = li < nlive;
            if (!live[u]) li = 0;
            int tr = 0, len = tc_n;
            while (li >= len) { li -= len; ++tr; len = tc_n - min(tr, FL); }
            const int tc = min(tr, FL) + li;
            pras[u] = 16 * tr + (lane & 15);
            const int pc = 16 * tc + (lane & 15);
            pcs[u] = pc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int pr = 16 * tr + (lane >> 4) + 4 * q;
              // the next diagonal block (rows and columns < jbn of the left
              // part) is formed by the look-ahead and not stored
              const bool dblk = ahead && pr < jbn && pc < jbn;
              ok[u][q] = live[u] && !dblk && pr < nrows && pc < m && (pc >= nleft || pc >= pr);
              const int64_t col = pc < nleft ? (int64_t)(j0 + jb + pc) : (int64_t)m + (pc - nleft);
              gofs[u][q] = (int64_t)(j0 + jb + pr) * m2 + col;
              acc[u][q] = ok[u][q] ? W[gofs[u][q]] : 0.0;
            }
          }
#pragma unroll
          for (int k0 = 0; k0 < NB; k0 += 4) {
            const int t = k0 + (lane >> 4);
#pragma unroll
            for (int u = 0; u < UT; ++u) {
              const double av = (live[u] && pras[u] < nrows) ? -P[t * m + pras[u]] : 0.0;
              const double bv = (live[u] && pcs[u] < m) ? P[t * m + pcs[u]] : 0.0;
              acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[u], 0, 0, 0);
            }
          }
#pragma unroll
          for (int u = 0; u < UT; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q)
              if (ok[u][q]) W[gofs[u][q]] = acc[u][q];
        }
      }
      pj0 = j0;
      pjb = jb;
      if (ahead) dcur ^= 1;
      have_d = ahead;
      if (!grid_barrier(bar, target, flags, &s_abort)) return;
    }
    if (!s_fail) break;
    // every workgroup saw the same failed pivot: retry once with the shift
    if (wg == 0 && tid == 0) atomicOr(flags, attempt == 0 ? SKETCHNE_FLAG_CHOL_SHIFT : SKETCHNE_FLAG_CHOL_FAIL);
    if (tid == 0) s_shifted = 1;
    if (!grid_barrier(bar, target, flags, &s_abort)) return;  // no workgroup still reads W before it is initialised again
  }
  if (!s_fail && pjb) store_right(pj0, pjb);
  if (!grid_barrier(bar, target, flags, &s_abort)) return;
  // R^-T = Rs^-T S^-1 from the lower triangle of the right half, rows over
  // the wavefronts of the grid; the largest row sum of |Rs^-T| per workgroup
  double rmax = 0.0;
  for (int r0 = 4 * gw; r0 < m; r0 += 4 * gnw) {
    double x[4][CH_CHUNKS];
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int cc = 0; cc < CH_CHUNKS; ++cc) {
        const int r = r0 + h, c = lane + 64 * cc;
        x[h][cc] = (r < m && c <= r) ? W[(int64_t)r * m2 + m + c] : 0.0;
      }
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int r = r0 + h;
      if (r >= m) break;
      double rs = 0.0;
#pragma unroll
      for (int cc = 0; cc < CH_CHUNKS; ++cc) {
        const int c = lane + 64 * cc;
        if (c < m) RinvT[(int64_t)r * m + c] = x[h][cc] * rsc[c];
        rs += fabs(x[h][cc]);
      }
      rmax = fmax(rmax, wave_sum(rs));
    }
  }
  if (need_more) {
    if (lane == 0) s_red[1][wv] = rmax;
    __syncthreads();
    if (tid == 0) {
      double b = 0.0;
      for (int w = 0; w < nw; ++w) b = fmax(b, s_red[1][w]);
      rpart[wg] = b;
    }
    if (!grid_barrier(bar, target, flags, &s_abort)) return;
    if (wg == 0) {
      // kappa_1(Rs) = ||Rs||_1 ||Rs^-1||_1 (column sums of Rs gathered in
      // every workgroup's LDS, row sums of Rs^-T from all workgroups)
      double cmax = 0.0;
      for (int j = tid; j < m; j += nt) cmax = fmax(cmax, colsum[j]);
      cmax = wave_max(cmax);
      if (lane == 0) s_red[0][wv] = cmax;
      __syncthreads();
      if (tid == 0) {
        double a = 0.0, b = 0.0;
        for (int w = 0; w < nw; ++w) a = fmax(a, s_red[0][w]);
        for (int w = 0; w < nwg; ++w) b = fmax(b, rpart[w]);
        const double kappa = a * b;
        *need_more = (s_shifted || !(kappa <= repeat_kappa)) ? 1 : 0;
      }
    }
  }
}

}  // namespace

constexpr int CHC_MAXWG = 8;  // workgroups of the multi-workgroup form
// W (m x 2m), the per-workgroup row-sum maxima, the grid barrier's count
size_t chol_ws_bytes(int m) { return align_up(sizeof(double) * ((size_t)m * 2 * m + CHC_MAXWG + 1)); }

namespace {

// The grid barrier needs all `blocks` workgroups resident at once.
sketchne_status check_resident(sketchne_ctx* c, const void* kernel, int blocks, int threads, size_t shmem) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, shmem) != hipSuccess)
    return SKETCHNE_E_DEVICE;
  return (int64_t)per_cu * c->n_cu >= blocks ? SKETCHNE_OK : SKETCHNE_E_UNSUPPORTED;
}

}  // namespace

sketchne_status copy_if(sketchne_ctx* c, int64_t count, const float* src, float* dst, const int* run_if) {
  if (count == 0) return SKETCHNE_OK;
  ProfScope ps(c, SKETCHNE_PROF_PREP);
  const int64_t want = (count / 4 + 255) / 256;
  const unsigned blocks = (unsigned)(want < 1 ? 1 : (want > 4096 ? 4096 : want));
  if (reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16) return SKETCHNE_E_UNSUPPORTED;
  hipLaunchKernelGGL(k_copy_if, dim3(blocks), dim3(256), 0, c->stream, count, src, dst, run_if);
  return launch_status();
}

sketchne_status chol_inv(sketchne_ctx* c, int m, const double* G, double* RinvT, double* work, int* need_more,
                         const int* run_if, double repeat_kappa) {
  if (m <= 0) return SKETCHNE_OK;
  if (m > CH_MAXM) return SKETCHNE_E_UNSUPPORTED;
  ProfScope ps(c, SKETCHNE_PROF_SMALL);
  size_t shmem = sizeof(double) * (NB * (NB + 1) + (size_t)NB * m);
  if (m <= 2 * NB) {
    hipFuncSetAttribute(reinterpret_cast<const void*>(k_chol_inv), hipFuncAttributeMaxDynamicSharedMemorySize,
                        (int)shmem);
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(512), shmem, c->stream, m, G, work, RinvT, c->d_flags, need_more,
                       run_if, repeat_kappa);
    return launch_status();
  }
  // workgroups: the first (largest) trailing update in passes of four tiles
  // per wavefront, eight wavefronts per workgroup
  const int nleft0 = m - NB, tr_n = (nleft0 + 15) / 16, tc_n = (m + 15) / 16, FL = nleft0 / 16;
  int nlive0 = 0;
  for (int tr = 0; tr < tr_n; ++tr) nlive0 += tc_n - (tr < FL ? tr : FL);
  int nwg = (nlive0 + 31) / 32;
  nwg = nwg < 2 ? 2 : (nwg > CHC_MAXWG ? CHC_MAXWG : nwg);
  shmem += sizeof(double) * NB * (NB + 1);  // the look-ahead's second diagonal-block buffer
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(k_chol_inv_coop), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)shmem) != hipSuccess)
    return SKETCHNE_E_DEVICE;
  SK_TRY(check_resident(c, reinterpret_cast<const void*>(k_chol_inv_coop), nwg, 512, shmem));
  double* W = work;
  double* rpart = work + (size_t)m * 2 * m;
  uint32_t* bar = reinterpret_cast<uint32_t*>(rpart + CHC_MAXWG);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, c->stream, bar);
  hipLaunchKernelGGL(k_chol_inv_coop, dim3(nwg), dim3(512), shmem, c->stream, m, G, W, rpart, RinvT, c->d_flags,
                     need_more, run_if, repeat_kappa, bar);
  return launch_status();
}

namespace {

// one wavefront per column j: t = G v_j (lanes over rows), s = v_j . t
__global__ __launch_bounds__(256) void k_ritz_from_gram(int m, int k, const double* __restrict__ G,
                                                        const double* __restrict__ V, const double* __restrict__ lam,
                                                        double* __restrict__ res) {
  const int lane = threadIdx.x & 63;
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= k) return;
  double s = 0.0;
  for (int r = lane; r < m; r += 64) {
    double t = 0.0;
    for (int col = 0; col < m; ++col) t = fma(G[(int64_t)r * m + col], V[(int64_t)col * m + j], t);
    s = fma(V[(int64_t)r * m + j], t, s);
  }
  s = wave_sum(s);
  if (lane == 0) {
    const double d = s - lam[j] * lam[j];
    res[j] = d > 0.0 ? sqrt(d) : 0.0;
  }
}

}  // namespace

sketchne_status ritz_from_gram(sketchne_ctx* c, int m, int k, const double* G, const double* V, const double* lam,
                               double* res) {
  if (k <= 0) return SKETCHNE_OK;
  ProfScope ps(c, SKETCHNE_PROF_SMALL);
  hipLaunchKernelGGL(k_ritz_from_gram, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, c->stream, m, k, G, V, lam, res);
  return launch_status();
}

size_t symeig_ws_bytes(int m) { return oj_ws_bytes(m); }

size_t symeig_scratch_bytes() { return kSymeigScratchBytes; }

sketchne_status symeig_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return SKETCHNE_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return SKETCHNE_OK;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return SKETCHNE_E_DEVICE;
  if (prev != device && hipSetDevice(device) != hipSuccess) return SKETCHNE_E_DEVICE;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (prev != device) hipSetDevice(prev);
  if (e != hipSuccess || !ptr) return SKETCHNE_E_DEVICE;
  g_scratch_ptr[device] = ptr;
  return SKETCHNE_OK;
}

void* symeig_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

sketchne_status symeig(sketchne_ctx* c, int m, const double* A, double* Vout, double* wout, void* ws, bool general) {
  if (m <= 0) return SKETCHNE_OK;
  if (m > OJ_GL * OJ_MAXR) return SKETCHNE_E_UNSUPPORTED;
  const int nb = oj_nblocks(m), mp = nb * NBJ;
  Arena ar(ws, symeig_ws_bytes(m));
  double* G = ar.take<double>((size_t)mp * OJ_ROWS);
  // rotations, then large rotations, per sweep; then the grid barrier's count
  int* counters = ar.take<int>(2 * kMaxSweeps + 1);
  double* shift = ar.take<double>(1);
  ProfScope ps(c, SKETCHNE_PROF_SMALL);
  hipLaunchKernelGGL(k_oj_norm, dim3(1), dim3(1024), 0, c->stream, m, A, (int)general, shift);
  int tot = mp * OJ_ROWS;
  hipLaunchKernelGGL(k_oj_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, m, mp, A, (int)general,
                     shift, G, counters, 2 * kMaxSweeps + 1);
  const size_t sh_intra = sizeof(double) * (size_t)(2 * NBJ) * OJ_ROWS;  // the larger of the two rounds
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(k_oj_sweeps), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)sh_intra) != hipSuccess)
    return SKETCHNE_E_DEVICE;
  SK_TRY(check_resident(c, reinterpret_cast<const void*>(k_oj_sweeps), nb / 2, OJ_THREADS, sh_intra));
  hipLaunchKernelGGL(k_oj_sweeps, dim3(nb / 2), dim3(OJ_THREADS), sh_intra, c->stream, nb, G, counters, c->d_flags);
  // every sweep slot not reached keeps its zero count, so the finish kernel's
  // convergence test may scan them all
  const int run = kMaxSweeps;
  const size_t sh_fin = sizeof(double) * (size_t)m * (OJF_ROWS + 1);
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(k_oj_finish), hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)sh_fin) != hipSuccess)
    return SKETCHNE_E_DEVICE;
  hipLaunchKernelGGL(k_oj_finish, dim3((unsigned)((m + OJF_ROWS - 1) / OJF_ROWS)), dim3(1024), sh_fin, c->stream, m,
                     G, shift, counters, run, Vout, wout, c->d_flags);
  return launch_status();
}

}  // namespace skne
