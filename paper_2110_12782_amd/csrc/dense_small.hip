// Small dense FP64 solvers: Cholesky with inverse factor, symmetric eigensolver.
//
// Cholesky: G = R^T R for an SPD m x m matrix (m <= 512), right-looking and
// blocked by 32 inside one 1024-thread workgroup.  The same row operations are
// applied to an appended identity, so the right half ends up holding R^-T
// (block row J of [R | R^-T] is R_JJ^-T times the updated block row J of
// [G | I]).  A pivot that is not positive restarts the factorization once with
// a small diagonal shift (shifted Cholesky-QR) and raises a flag; a second
// failure raises CHOL_FAIL.
//
// Eigensolver: two-sided cyclic Jacobi with the round-robin ("circle")
// ordering, so each step rotates m/2 disjoint index pairs at once.  One
// kernel per step updates every 2 x 2 block A[{p1,q1},{p2,q2}] <- J1^T A J2
// into a second buffer (rotations are recomputed from the 2 x 2 diagonal
// blocks of the input buffer) and rotates the pairs of columns of V in place.
// A per-sweep rotation counter stops the iteration: once a whole sweep
// performs no rotation, later step kernels return immediately.  Pairs are
// finally sorted by |w| descending, ties by w descending, then index.
#include "internal.h"

namespace skne {
namespace {

constexpr int NB = 32;

__global__ __launch_bounds__(1024) void k_chol_inv(int m, const double* __restrict__ G, double* __restrict__ W,
                                                   double* __restrict__ RinvT, uint32_t* __restrict__ flags) {
  extern __shared__ double smem[];
  double* D = smem;               // NB x (NB+1)
  double* P = smem + NB * (NB + 1);  // NB x m panel
  __shared__ int s_fail;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t m2 = 2 * (int64_t)m;

  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < m; ++i) tr += fabs(G[(int64_t)i * m + i]);
    s_fail = 0;
    // shifted retry: s = 11 (m^2 + m) u trace(G)  (shifted Cholesky-QR)
    D[0] = 11.0 * ((double)m * m + m) * 1.1102230246251565e-16 * (tr > 0 ? tr : 1.0);
  }
  __syncthreads();
  const double retry_shift = D[0];
  __syncthreads();

  for (int attempt = 0; attempt < 2; ++attempt) {
    const double shift = attempt == 0 ? 0.0 : retry_shift;
    for (int64_t idx = tid; idx < (int64_t)m * m2; idx += nt) {
      int64_t r = idx / m2, c = idx - r * m2;
      double v;
      if (c < m) {
        int64_t a = r < c ? r : c, b = r < c ? c : r;  // symmetric: read the upper triangle
        v = G[a * m + b] + (r == c ? shift : 0.0);
      } else {
        v = (c - m == r) ? 1.0 : 0.0;
      }
      W[idx] = v;
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();

    for (int j0 = 0; j0 < m; j0 += NB) {
      const int jb = min(NB, m - j0);
      // 1. factor the diagonal block in LDS
      for (int idx = tid; idx < jb * jb; idx += nt) {
        int a = idx / jb, b = idx % jb;
        D[a * (NB + 1) + b] = (b >= a) ? W[(int64_t)(j0 + a) * m2 + j0 + b] : 0.0;
      }
      __syncthreads();
      for (int t = 0; t < jb; ++t) {
        if (tid == 0) {
          double d = D[t * (NB + 1) + t];
          if (!(d > 0.0) || !isfinite(d)) { s_fail = 1; d = 1.0; }
          D[t * (NB + 1) + t] = sqrt(d);
        }
        __syncthreads();
        if (tid > t && tid < jb) D[t * (NB + 1) + tid] /= D[t * (NB + 1) + t];
        __syncthreads();
        for (int idx = tid; idx < jb * jb; idx += nt) {
          int a = idx / jb, b = idx % jb;
          if (a > t && b >= a) D[a * (NB + 1) + b] -= D[t * (NB + 1) + a] * D[t * (NB + 1) + b];
        }
        __syncthreads();
      }
      if (s_fail) break;
      // 2. row panel: W[J, c] <- R_JJ^-T W[J, c] for the left columns right of
      //    the block and the right columns that can be non-zero (< j0 + jb)
      const int nleft = m - j0 - jb;
      for (int pc = tid; pc < m; pc += nt) {
        int64_t col = pc < nleft ? (int64_t)(j0 + jb + pc) : (int64_t)m + (pc - nleft);
        double x[NB];
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          if (t < jb) {
            double v = W[(int64_t)(j0 + t) * m2 + col];
            for (int s2 = 0; s2 < t; ++s2) v -= D[s2 * (NB + 1) + t] * x[s2];
            x[t] = v / D[t * (NB + 1) + t];
            W[(int64_t)(j0 + t) * m2 + col] = x[t];
            P[t * m + pc] = x[t];
          }
        }
      }
      __syncthreads();
      // 3. trailing update of the rows below the block
      const int64_t nrows = nleft;
      for (int64_t idx = tid; idx < nrows * m; idx += nt) {
        int pr = (int)(idx / m);
        int pc = (int)(idx - (int64_t)pr * m);
        if (pc < nleft && pc < pr) continue;  // left part: upper triangle only
        int64_t r = j0 + jb + pr;
        int64_t col = pc < nleft ? (int64_t)(j0 + jb + pc) : (int64_t)m + (pc - nleft);
        double s = 0.0;
        for (int t = 0; t < jb; ++t) s += P[t * m + pr] * P[t * m + pc];
        W[r * m2 + col] -= s;
      }
      __syncthreads();
    }
    __syncthreads();
    if (!s_fail) break;
    if (tid == 0) atomicOr(flags, attempt == 0 ? SKETCHNE_FLAG_CHOL_SHIFT : SKETCHNE_FLAG_CHOL_FAIL);
    __syncthreads();
  }
  for (int64_t idx = tid; idx < (int64_t)m * m; idx += nt) {
    int64_t r = idx / m, c = idx - r * m;
    RinvT[idx] = c <= r ? W[r * m2 + m + c] : 0.0;
  }
}

// ---------------------------------------------------------------- Jacobi

__device__ __forceinline__ void pair_of(int s, int pi, int mp, int& p, int& q) {
  const int ring = mp - 1;
  int a, b;
  if (pi == 0) { a = mp - 1; b = s; }
  else { a = (s + pi) % ring; b = (s - pi + ring) % ring; }
  p = a < b ? a : b;
  q = a < b ? b : a;
}

__device__ __forceinline__ void rotation(double app, double aqq, double apq, double tol_abs, double& c,
                                         double& s, bool& rot) {
  const double eps = 2.220446049250313e-16;
  rot = fabs(apq) > tol_abs && fabs(apq) > eps * sqrt(fabs(app) * fabs(aqq));
  if (!rot) { c = 1.0; s = 0.0; return; }
  double tau = (aqq - app) / (2.0 * apq);
  double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
  c = 1.0 / sqrt(1.0 + t * t);
  s = t * c;
}

__global__ void k_jac_init(int m, int mp, const double* __restrict__ A, double* __restrict__ A0,
                           double* __restrict__ V, int* __restrict__ counters, int max_sweeps,
                           double* __restrict__ frob) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < max_sweeps) counters[idx] = 0;
  if (idx >= (int64_t)mp * mp) return;
  int r = (int)(idx / mp), c = (int)(idx % mp);
  double v = 0.0;
  if (r < m && c < m) v = r <= c ? A[(int64_t)r * m + c] : A[(int64_t)c * m + r];
  A0[idx] = v;
  V[idx] = r == c ? 1.0 : 0.0;
  if (idx == 0) {
    double s = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        double a = i <= j ? A[(int64_t)i * m + j] : A[(int64_t)j * m + i];
        s += a * a;
      }
    *frob = sqrt(s);
  }
}

__global__ __launch_bounds__(256) void k_jac_step(int mp, int s, int sweep, const double* __restrict__ Ain,
                                                  double* __restrict__ Aout, double* __restrict__ V,
                                                  int* __restrict__ counters, const double* __restrict__ frob) {
  if (sweep > 0 && counters[sweep - 1] == 0) return;
  const int P = mp / 2;
  const int64_t nA = (int64_t)P * P;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double tol_abs = 1e-17 * (*frob) + 1e-300;
  if (idx < nA) {
    const int pi = (int)(idx / P), pj = (int)(idx % P);
    int p1, q1, p2, q2;
    pair_of(s, pi, mp, p1, q1);
    pair_of(s, pj, mp, p2, q2);
    double c1, s1, c2, s2;
    bool r1, r2;
    rotation(Ain[(int64_t)p1 * mp + p1], Ain[(int64_t)q1 * mp + q1], Ain[(int64_t)p1 * mp + q1], tol_abs, c1, s1, r1);
    rotation(Ain[(int64_t)p2 * mp + p2], Ain[(int64_t)q2 * mp + q2], Ain[(int64_t)p2 * mp + q2], tol_abs, c2, s2, r2);
    double b00 = Ain[(int64_t)p1 * mp + p2], b01 = Ain[(int64_t)p1 * mp + q2];
    double b10 = Ain[(int64_t)q1 * mp + p2], b11 = Ain[(int64_t)q1 * mp + q2];
    // J = [[c, s], [-s, c]];  B' = J1^T B J2
    double t00 = c1 * b00 - s1 * b10, t01 = c1 * b01 - s1 * b11;
    double t10 = s1 * b00 + c1 * b10, t11 = s1 * b01 + c1 * b11;
    double n00 = t00 * c2 - t01 * s2, n01 = t00 * s2 + t01 * c2;
    double n10 = t10 * c2 - t11 * s2, n11 = t10 * s2 + t11 * c2;
    if (pi == pj && r1) { n01 = 0.0; n10 = 0.0; atomicAdd(&counters[sweep], 1); }
    Aout[(int64_t)p1 * mp + p2] = n00;
    Aout[(int64_t)p1 * mp + q2] = n01;
    Aout[(int64_t)q1 * mp + p2] = n10;
    Aout[(int64_t)q1 * mp + q2] = n11;
    return;
  }
  const int64_t j = idx - nA;
  if (j >= (int64_t)mp * P) return;
  const int r = (int)(j / P), pi = (int)(j % P);
  int p, q;
  pair_of(s, pi, mp, p, q);
  double c, sn;
  bool rot;
  rotation(Ain[(int64_t)p * mp + p], Ain[(int64_t)q * mp + q], Ain[(int64_t)p * mp + q], tol_abs, c, sn, rot);
  if (!rot) return;
  double vp = V[(int64_t)r * mp + p], vq = V[(int64_t)r * mp + q];
  V[(int64_t)r * mp + p] = c * vp - sn * vq;
  V[(int64_t)r * mp + q] = sn * vp + c * vq;
}

// Sort eigenpairs and write the outputs.  The final matrix sits in buffer
// ((S+1)*(mp-1)) % 2 where S is the first sweep without rotations.
__global__ __launch_bounds__(1024) void k_jac_finish(int m, int mp, const double* __restrict__ A0,
                                                     const double* __restrict__ A1, const double* __restrict__ V,
                                                     const int* __restrict__ counters, int sweeps_run,
                                                     double* __restrict__ Vout, double* __restrict__ wout,
                                                     uint32_t* __restrict__ flags) {
  __shared__ double w[1024];
  __shared__ int rank[1024];
  __shared__ int s_final;
  const int tid = threadIdx.x;
  if (tid == 0) {
    int S = -1;
    for (int s = 0; s < sweeps_run; ++s)
      if (counters[s] == 0) { S = s; break; }
    int steps;
    if (S < 0) { steps = sweeps_run * (mp - 1); atomicOr(flags, SKETCHNE_FLAG_EIG_NOCONV); }
    else steps = (S + 1) * (mp - 1);
    s_final = steps & 1;
  }
  __syncthreads();
  const double* Af = s_final ? A1 : A0;
  for (int i = tid; i < m; i += blockDim.x) {
    w[i] = Af[(int64_t)i * mp + i];
    if (!isfinite(w[i])) atomicOr(flags, SKETCHNE_FLAG_NONFINITE);
  }
  __syncthreads();
  for (int i = tid; i < m; i += blockDim.x) {
    double ai = fabs(w[i]);
    int rk = 0;
    for (int j = 0; j < m; ++j) {
      double aj = fabs(w[j]);
      bool before = (aj > ai) || (aj == ai && (w[j] > w[i] || (w[j] == w[i] && j < i)));
      rk += before ? 1 : 0;
    }
    rank[i] = rk;
  }
  __syncthreads();
  for (int i = tid; i < m; i += blockDim.x) wout[rank[i]] = w[i];
  for (int64_t idx = tid; idx < (int64_t)m * m; idx += blockDim.x) {
    int r = (int)(idx / m), i = (int)(idx % m);
    Vout[(int64_t)r * m + rank[i]] = V[(int64_t)r * mp + i];
  }
}

constexpr int kMaxSweeps = 40;

}  // namespace

size_t chol_ws_bytes(int m) { return align_up(sizeof(double) * (size_t)m * 2 * m); }

sketchne_status chol_inv(sketchne_ctx* c, int m, const double* G, double* RinvT, double* work) {
  if (m <= 0) return SKETCHNE_OK;
  if (m > 512) return SKETCHNE_E_UNSUPPORTED;
  ProfScope ps(c, SKETCHNE_PROF_SMALL);
  size_t shmem = sizeof(double) * (NB * (NB + 1) + (size_t)NB * m);
  hipFuncSetAttribute(reinterpret_cast<const void*>(k_chol_inv), hipFuncAttributeMaxDynamicSharedMemorySize,
                      (int)shmem);
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(1024), shmem, c->stream, m, G, work, RinvT, c->d_flags);
  return launch_status();
}

size_t symeig_ws_bytes(int m) {
  int mp = m + (m & 1);
  size_t mat = align_up(sizeof(double) * (size_t)mp * mp);
  return 3 * mat + align_up(sizeof(int) * kMaxSweeps) + align_up(sizeof(double));
}

sketchne_status symeig(sketchne_ctx* c, int m, const double* A, double* Vout, double* wout, void* ws) {
  if (m <= 0) return SKETCHNE_OK;
  if (m > 1024) return SKETCHNE_E_UNSUPPORTED;
  const int mp = m + (m & 1);
  Arena ar(ws, symeig_ws_bytes(m));
  double* A0 = ar.take<double>((size_t)mp * mp);
  double* A1 = ar.take<double>((size_t)mp * mp);
  double* V = ar.take<double>((size_t)mp * mp);
  int* counters = ar.take<int>(kMaxSweeps);
  double* frob = ar.take<double>(1);
  ProfScope ps(c, SKETCHNE_PROF_SMALL);
  int64_t tot = (int64_t)mp * mp;
  hipLaunchKernelGGL(k_jac_init, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, c->stream, m, mp, A, A0, V,
                     counters, kMaxSweeps, frob);
  const int P = mp / 2;
  const int64_t threads = (int64_t)P * P + (int64_t)mp * P;
  const unsigned blocks = (unsigned)((threads + 255) / 256);
  int sweeps_run = 0;
  int buf = 0;
  for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
    for (int s = 0; s < mp - 1; ++s) {
      const double* Ain = buf ? A1 : A0;
      double* Aout = buf ? A0 : A1;
      hipLaunchKernelGGL(k_jac_step, dim3(blocks), dim3(256), 0, c->stream, mp, s, sweep, Ain, Aout, V, counters,
                         frob);
      buf ^= 1;
    }
    sweeps_run = sweep + 1;
    if (sweep >= 3) {  // converged?  (one small host read per sweep from the fourth on)
      hipMemcpyAsync(c->h_counter, counters + sweep, sizeof(int), hipMemcpyDeviceToHost, c->stream);
      if (hipStreamSynchronize(c->stream) != hipSuccess) return SKETCHNE_E_DEVICE;
      if (*c->h_counter == 0) break;
    }
  }
  hipLaunchKernelGGL(k_jac_finish, dim3(1), dim3(1024), 0, c->stream, m, mp, A0, A1, V, counters, sweeps_run, Vout,
                     wout, c->d_flags);
  return launch_status();
}

}  // namespace skne
