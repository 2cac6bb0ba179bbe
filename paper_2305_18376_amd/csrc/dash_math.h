// Device helpers shared by the update and initialisation kernels: wave-level
// reductions and broadcasts, and the small dense R x R algebra (FP64) that the
// lemmas need -- Gauss-Jordan solves and inverses with the Cholesky acceptance
// rule, cyclic Jacobi eigendecomposition, eigen pseudo-inverses.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "dash_dev.h"

namespace dash {

// ---------------------------------------------------------------------------
// wave / block helpers
// ---------------------------------------------------------------------------
// Order LDS accesses of one wave.  The LDS executes a wave's instructions in
// issue order, so only the compiler must not move accesses across this point
// (wavefront-scope fences emit no wait on outstanding global memory traffic).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over c in [c0, c1) of src[c * stride + e], in ascending c, with the loads
// issued in batches of 16 so their latencies overlap (missing terms add 0).
__device__ __forceinline__ double ordered_sum(const double *src, int64_t stride, int e, int c0, int c1) {
  double s = 0.0;
  for (int c = c0; c < c1; c += 16) {
    double v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = (c + i < c1) ? src[(int64_t)(c + i) * stride + e] : 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) s += v[i];
  }
  return s;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long x = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)x, l);
  const int hi = __builtin_amdgcn_readlane((int)(x >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Solve M x = b for an SPD n x n matrix (n <= RM) held by one wave in
// registers: lane i owns row i of M in m[] and b_i in b.  Cholesky with the
// pivots and factor columns broadcast by readlane; the factor is transposed
// once through LDS (`scratch`, n*n doubles) for the back substitution.
// Returns false, uniformly, when a pivot is not above kPivotRel times the
// largest diagonal entry (the oracle's acceptance rule); m and b are then
// undefined.
// Cholesky factorisation of the n x n SPD matrix M (row-major, LDS) by one
// wave, lane i owning row i.  The lower factor overwrites the lower triangle.
// Fails (returns false, uniformly) when a pivot is not above kPivotRel times the
// largest diagonal entry -- the same acceptance rule as the oracle.
__device__ inline bool wave_cholesky(double *M, int n) {
  const int lane = threadIdx.x & 63;
  const double dmax = wave_max(lane < n ? M[lane * n + lane] : 0.0);
  if (!(dmax > 0.0)) return false;
  const double thr = kPivotRel * dmax;
  for (int p = 0; p < n; ++p) {
    const double piv = M[p * n + p];
    if (!(piv > thr)) return false;
    const double lp = sqrt(piv);
    wave_sync();
    if (lane == p) M[p * n + p] = lp;
    if (lane > p && lane < n) M[lane * n + p] /= lp;
    wave_sync();
    if (lane > p && lane < n) {
      const double lip = M[lane * n + p];
      for (int j = p + 1; j <= lane; ++j) M[lane * n + j] -= lip * M[j * n + p];
    }
    wave_sync();
  }
  return true;
}

// Solve L L^T x = b in place (x in LDS), L from wave_cholesky.  One wave.
__device__ inline void wave_chol_apply(const double *L, double *x, int n) {
  const int lane = threadIdx.x & 63;
  for (int p = 0; p < n; ++p) {
    const double yp = x[p] / L[p * n + p];
    wave_sync();
    if (lane == p) x[p] = yp;
    if (lane > p && lane < n) x[lane] -= L[lane * n + p] * yp;
    wave_sync();
  }
  for (int p = n - 1; p >= 0; --p) {
    const double zp = x[p] / L[p * n + p];
    wave_sync();
    if (lane == p) x[p] = zp;
    if (lane < p) x[lane] -= L[p * n + lane] * zp;
    wave_sync();
  }
}

// Symmetric eigendecomposition A = Z diag(A_out) Z^T of an n x n matrix
// (n <= 64) by one wave: cyclic parallel Jacobi (Golub & Van Loan, Sec. 8.5,
// "parallel ordering"), disjoint rotation pairs per round from the round-robin
// tournament.  A (lda = n) is diagonalised in place, Z receives the
// eigenvectors as columns.  `rot` needs 2*32 doubles, `pair` 2*32 ints.
__device__ inline void wave_jacobi(double *A, double *Z, int n, double *rot, int *pair) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < n * n; e += 64) Z[e] = (e / n == e % n) ? 1.0 : 0.0;
  wave_sync();
  if (n < 2) return;
  const int np = n + (n & 1);
  const int half = np / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = lane; e < n * n; e += 64) {
      const double v = A[e] * A[e];
      tot += v;
      if (e / n != e % n) off += v;
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    // converged when the off-diagonal part is at rounding level
    if (!(off > 1e-30 * tot) || !(off > (double)(n * n) * 5e-32 * tot)) break;
    for (int t = 0; t < np - 1; ++t) {
      if (lane < half) {
        // circle method: player 0 fixed, the others rotate by t
        auto pos = [&](int i) { return i == 0 ? 0 : ((i - 1 + t) % (np - 1)) + 1; };
        int p = pos(lane), q = pos(np - 1 - lane);
        if (p > q) { int tmp = p; p = q; q = tmp; }
        double c = 1.0, s = 0.0;
        if (q < n) {
          const double apq = A[p * n + q];
          if (apq != 0.0) {
            const double tau = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
          }
        }
        rot[2 * lane] = c;
        rot[2 * lane + 1] = s;
        pair[2 * lane] = p;
        pair[2 * lane + 1] = (q < n) ? q : -1;
      }
      wave_sync();
      // A <- A J and Z <- Z J (columns p, q of every pair)
      for (int e = lane; e < n * half; e += 64) {
        const int i = e / n, r = e % n;
        const int p = pair[2 * i], q = pair[2 * i + 1];
        if (q < 0) continue;
        const double c = rot[2 * i], s = rot[2 * i + 1];
        const double ap = A[r * n + p], aq = A[r * n + q];
        A[r * n + p] = c * ap - s * aq;
        A[r * n + q] = s * ap + c * aq;
        const double zp = Z[r * n + p], zq = Z[r * n + q];
        Z[r * n + p] = c * zp - s * zq;
        Z[r * n + q] = s * zp + c * zq;
      }
      wave_sync();
      // A <- J^T A (rows p, q of every pair)
      for (int e = lane; e < n * half; e += 64) {
        const int i = e / n, col = e % n;
        const int p = pair[2 * i], q = pair[2 * i + 1];
        if (q < 0) continue;
        const double c = rot[2 * i], s = rot[2 * i + 1];
        const double ap = A[p * n + col], aq = A[q * n + col];
        A[p * n + col] = c * ap - s * aq;
        A[q * n + col] = s * ap + c * aq;
      }
      wave_sync();
    }
  }
}

// x <- pinv(M) x for symmetric PSD M (n x n, LDS, destroyed), eigenvalues kept
// above kEigCutoff * max|eigenvalue|.  One wave; scratch >= n*n + n doubles.
__device__ inline void wave_pinv_apply(double *M, double *x, int n, double *Z, double *tmp, double *rot,
                                int *pair) {
  const int lane = threadIdx.x & 63;
  wave_jacobi(M, Z, n, rot, pair);
  double top = 0.0;
  for (int i = 0; i < n; ++i) top = fmax(top, fabs(M[i * n + i]));
  // tmp_i = (z_i . x) / lambda_i for kept i
  if (lane < n) {
    const double li = M[lane * n + lane];
    double d = 0.0;
    for (int r = 0; r < n; ++r) d += Z[r * n + lane] * x[r];
    tmp[lane] = (top > 0.0 && li > kEigCutoff * top) ? d / li : 0.0;
  }
  wave_sync();
  if (lane < n) {
    double v = 0.0;
    for (int i = 0; i < n; ++i) v += Z[lane * n + i] * tmp[i];
    x[lane] = v;
  }
  wave_sync();
}

// Gauss-Jordan elimination without pivoting of an SPD n x n system held by
// one wave in registers (n <= RM): lane i < n owns row i of A in m[] (m[c] =
// A_ic, zero for c >= n; zero rows on lanes >= n) and the i-th entries of NB
// right-hand sides in b[].  The system is padded to RM x RM with a decoupled
// diagonal block, so the elimination is straight-line code over compile-time
// indices; pivot rows are broadcast with readlane.  Pivot p < n is the Schur
// complement diagonal -- the square of the Cholesky diagonal entry -- and is
// accepted when above kPivotRel times the largest diagonal entry of A: the
// oracle's Cholesky acceptance rule.  On success d holds lane i's final pivot
// and x_i = b[.] / d; returns false, uniformly across the wave, otherwise.
template <int RM, int NB>
__device__ __forceinline__ bool wave_gj_reg(double (&m)[RM], double (&b)[NB], double &d, int n) {
  const int lane = threadIdx.x & 63;
  double dmax = 0.0;
#pragma unroll
  for (int p = 0; p < RM; ++p) {
    const double v = readlane_d(m[p], p);
    dmax = (p < n) ? fmax(dmax, v) : dmax;
  }
  if (!(dmax > 0.0)) return false;
  const double thr = kPivotRel * dmax;
#pragma unroll
  for (int c = 0; c < RM; ++c) m[c] = (lane == c && c >= n) ? dmax : m[c];
  d = 1.0;
#pragma unroll
  for (int p = 0; p < RM; ++p) {
    const double piv = readlane_d(m[p], p);
    if (p < n && !(piv > thr)) return false;
    d = (lane == p) ? piv : d;
    const double f = (lane != p) ? m[p] / piv : 0.0;
#pragma unroll
    for (int c = p + 1; c < RM; ++c) m[c] = fma(-f, readlane_d(m[c], p), m[c]);
#pragma unroll
    for (int k = 0; k < NB; ++k) b[k] = fma(-f, readlane_d(b[k], p), b[k]);
  }
  return true;
}

// Ainv = A^{-1} for SPD A (n x n, n <= RM, LDS, row-major) by the first four
// waves of the block (one per SIMD): wave w eliminates its own copy of A with
// the unit vectors e_{w*NB} .. e_{w*NB+NB-1} as right-hand sides, so the
// columns of the inverse come out in parallel.  Every wave runs the same
// elimination, hence takes the same acceptance decision; the return value is
// that decision on waves 0..3 and true elsewhere (the caller combines it
// through LDS and synchronises the block before reading Ainv).
// With piv, wave 0 also stores the elimination pivots (piv[i] = lane i's d,
// the Schur complement diagonal) when the elimination is accepted.
template <int RM>
__device__ bool block_spd_inverse(const double *A, double *Ainv, int n, double *piv = nullptr) {
  constexpr int NB = RM / 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (wv >= 4) return true;
  double m[RM];
#pragma unroll
  for (int c = 0; c < RM; ++c) m[c] = (lane < n && c < n) ? A[lane * n + c] : 0.0;
  double rhs[NB];
#pragma unroll
  for (int k = 0; k < NB; ++k) rhs[k] = (lane == wv * NB + k) ? 1.0 : 0.0;
  double d;
  if (!wave_gj_reg<RM, NB>(m, rhs, d, n)) return false;
  if (piv && wv == 0 && lane < n) piv[lane] = d;
#pragma unroll
  for (int k = 0; k < NB; ++k) {
    const int col = wv * NB + k;
    if (lane < n && col < n) Ainv[lane * n + col] = rhs[k] / d;
  }
  return true;
}

// out = pinv(src) for a symmetric PSD n x n matrix (LDS), the whole block
// taking part: wave 0 diagonalises a copy (work, eigenvectors in Z), then every
// thread forms entries of Z diag(1/lambda_kept) Z^T with the relative cutoff.
__device__ inline void block_pinv_of(const double *src, double *out, double *work, double *Z, int n,
                              double *rot, int *pair) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int q = tid; q < n * n; q += nt) work[q] = src[q];
  __syncthreads();
  if ((tid >> 6) == 0) wave_jacobi(work, Z, n, rot, pair);
  __syncthreads();
  double top = 0.0;
  for (int i = 0; i < n; ++i) top = fmax(top, fabs(work[i * n + i]));
  for (int q = tid; q < n * n; q += nt) {
    const int r = q / n, c = q - r * n;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
      const double li = work[i * n + i];
      if (top > 0.0 && li > kEigCutoff * top) acc += Z[r * n + i] * Z[c * n + i] / li;
    }
    out[q] = acc;
  }
  __syncthreads();
}

}  // namespace dash
