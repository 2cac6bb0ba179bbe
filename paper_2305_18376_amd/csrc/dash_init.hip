// gfx950 kernels of the initial decomposition (Sec. 3.2.1): PARAFAC2-ALS on
// the initial tensor {X_k}, then the hand-off to the streaming state
// (eq. [updateC_init]-[updateG_init] in the exact form Y_k = U_k^T X_k,
// D_k = U_k^T U_k with U_k = Q_k H).
//
// One ALS iteration (host loop in dash_host.cpp):
//   accum   per slice: T_k = X_k V; Yh_k = T_k^T X_k (R x J), Dh_k = T_k^T T_k
//           (one pass over X; n_k = ||X_k||^2).  Dh_k is summed and kept in FP64:
//           for I_k < R it has rank I_k, and P_k's retained eigenspace (the
//           1e-12 relative cutoff) must see that rank as the oracle does.
//   slice   per slice: A_k = X_k V S_k H^T, so P_k = A_k^T A_k = Hw Dh_k Hw^T and
//           A_k^T X_k = Hw Yh_k with Hw = H S_k; Jacobi eigen of P_k gives
//           P_k^{-1/2} and the projector Pi_k; Y_k = Q_k^T X_k = P_k^{-1/2} Hw Yh_k;
//           partials of M1 = sum Y_k V S_k and of W^T W
//   solve H H = M1 ((V^T V) * (W^T W))^{-1}
//   m2      partials of M2 = sum Y_k^T H S_k
//   solve V V = M2 ((H^T H) * (W^T W))^{-1}, then ((H^T H) * (V^T V))^{-1}
//   w       per slice: c = diag(H^T Y_k V), w_k = ((H^T H) * (V^T V))^{-1} c, loss
//           ||X_k||^2 - 2 w.c + w^T ((H^T Pi_k H) * (V^T V)) w
//   solve L loss = sum of the slice losses
// Partials are written per chunk of slices and summed in chunk order.
#include <hip/hip_runtime.h>
#include <math.h>

#include "dash_dev.h"
#include "dash_math.h"

namespace dash {

// ---------------------------------------------------------------------------
// V0: top-R eigenvectors of sum_k X_k^T X_k
// ---------------------------------------------------------------------------
constexpr int kGT = 64;   // Gram tile edge

// Gram partial of one chunk of rows: part[c] = X_rows^T X_rows (FP64 sums of
// exact products).  Grid (tiles^2, n_gc); 256 threads, 4 x 4 entries each.
__global__ __launch_bounds__(256) void k_gram_partial(int J, int64_t N, int64_t rows_per_chunk,
                                                      const float *X, double *part) {
  __shared__ float sA[32][kGT + 1];
  __shared__ float sB[32][kGT + 1];
  const int nt = (J + kGT - 1) / kGT;
  const int ti = blockIdx.x / nt, tj = blockIdx.x - ti * nt;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = min(N, r0 + rows_per_chunk);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += 32) {
    const int m = (int)min((int64_t)32, r1 - rb);
    __syncthreads();
    for (int e = threadIdx.x; e < 32 * kGT; e += 256) {
      const int rr = e / kGT, cc = e - rr * kGT;
      const int ci = ti * kGT + cc, cj = tj * kGT + cc;
      sA[rr][cc] = (rr < m && ci < J) ? X[(rb + rr) * J + ci] : 0.f;
      sB[rr][cc] = (rr < m && cj < J) ? X[(rb + rr) * J + cj] : 0.f;
    }
    __syncthreads();
    for (int rr = 0; rr < m; ++rr) {
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = (double)sA[rr][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = (double)sB[rr][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(av[i], bv[j], acc[i][j]);
    }
  }
  double *out = part + (int64_t)blockIdx.y * J * J;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int gi = ti * kGT + ty + 16 * i, gj = tj * kGT + tx + 16 * j;
      if (gi < J && gj < J) out[gi * J + gj] = acc[i][j];
    }
}

__global__ void k_gram_reduce(int JJ, int n_gc, const double *part, double *Gm) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < JJ) Gm[e] = ordered_sum(part, JJ, e, 0, n_gc);
}

// Symmetric eigendecomposition A = Z diag(evals) Z^T of an n x n matrix
// (n <= 256, global memory) by one workgroup: cyclic Jacobi with the parallel
// round-robin ordering (Golub & Van Loan, Sec. 8.5); the n/2 rotations of a
// round touch disjoint index pairs and are applied together.  A is destroyed.
constexpr int kEigThreads = 1024;

__global__ __launch_bounds__(kEigThreads) void k_sym_eig(int n, double *A, double *Z, double *evals) {
  __shared__ double sc[128], ss[128];
  __shared__ int sp[128], sq[128];
  __shared__ double red[2][kEigThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nt = blockDim.x;
  for (int e = tid; e < n * n; e += nt) Z[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  const int np = n + (n & 1), half = np / 2;
  for (int sweep = 0; sweep < 60 && n > 1; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += nt) {
      const double v = A[e] * A[e];
      tot += v;
      if (e / n != e % n) off += v;
    }
    off = wave_sum(off);
    tot = wave_sum(tot);
    if (lane == 0) {
      red[0][wv] = off;
      red[1][wv] = tot;
    }
    __syncthreads();
    off = 0.0;
    tot = 0.0;
    for (int w = 0; w < nt / 64; ++w) {
      off += red[0][w];
      tot += red[1][w];
    }
    __syncthreads();
    if (!(off > 1e-30 * tot) || !(off > (double)n * (double)n * 5e-32 * tot)) break;
    for (int t = 0; t < np - 1; ++t) {
      if (tid < half) {
        auto pos = [&](int i) { return i == 0 ? 0 : ((i - 1 + t) % (np - 1)) + 1; };
        int p = pos(tid), q = pos(np - 1 - tid);
        if (p > q) {
          const int tmp = p;
          p = q;
          q = tmp;
        }
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
        sc[tid] = c;
        ss[tid] = s;
        sp[tid] = p;
        sq[tid] = (q < n) ? q : -1;
      }
      __syncthreads();
      // A <- J^T A: rows p, q of every pair
      for (int e = tid; e < half * n; e += nt) {
        const int i = e / n, col = e - i * n;
        const int p = sp[i], q = sq[i];
        if (q < 0) continue;
        const double c = sc[i], s = ss[i];
        const double ap = A[p * n + col], aq = A[q * n + col];
        A[p * n + col] = c * ap - s * aq;
        A[q * n + col] = s * ap + c * aq;
      }
      __syncthreads();
      // A <- A J and Z <- Z J: columns p, q of every pair
      for (int e = tid; e < half * n; e += nt) {
        const int i = e % half, r = e / half;
        const int p = sp[i], q = sq[i];
        if (q < 0) continue;
        const double c = sc[i], s = ss[i];
        const double ap = A[r * n + p], aq = A[r * n + q];
        A[r * n + p] = c * ap - s * aq;
        A[r * n + q] = s * ap + c * aq;
        const double zp = Z[r * n + p], zq = Z[r * n + q];
        Z[r * n + p] = c * zp - s * zq;
        Z[r * n + q] = s * zp + c * zq;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += nt) evals[i] = A[i * n + i];
}

// V64 (J x R) = the eigenvectors of the R largest eigenvalues, in descending
// order, each column signed so that its entry of largest magnitude is positive
// (first such entry on ties).  One workgroup of 256 threads.
__global__ __launch_bounds__(256) void k_top_vectors(int J, int R, const double *evals, const double *Z,
                                                     double *V64) {
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ unsigned char taken[256];
  __shared__ int chosen;
  __shared__ double sgn;
  const int tid = threadIdx.x;
  for (int i = tid; i < J; i += 256) taken[i] = 0;
  __syncthreads();
  for (int r = 0; r < R; ++r) {
    // largest remaining eigenvalue (lowest index on ties)
    double best = -INFINITY;
    int bi = J;
    for (int i = tid; i < J; i += 256)
      if (!taken[i] && (evals[i] > best || (evals[i] == best && i < bi))) {
        best = evals[i];
        bi = i;
      }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) {
        const double v2 = sv[tid + o];
        const int i2 = si[tid + o];
        if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) {
          sv[tid] = v2;
          si[tid] = i2;
        }
      }
      __syncthreads();
    }
    if (tid == 0) {
      int ch = si[0];
      if (ch >= J) {   // only non-comparable (NaN) eigenvalues remain: take the first free one
        ch = 0;
        while (ch < J - 1 && taken[ch]) ++ch;
      }
      chosen = ch;
      taken[ch] = 1;
    }
    __syncthreads();
    const int col = chosen;
    // entry of largest magnitude of the column (first on ties)
    double bm = -1.0;
    int bj = J;
    for (int j = tid; j < J; j += 256) {
      const double v = fabs(Z[j * J + col]);
      if (v > bm) {
        bm = v;
        bj = j;
      }
    }
    sv[tid] = bm;
    si[tid] = bj;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) {
        const double v2 = sv[tid + o];
        const int i2 = si[tid + o];
        if (v2 > sv[tid] || (v2 == sv[tid] && i2 < si[tid])) {
          sv[tid] = v2;
          si[tid] = i2;
        }
      }
      __syncthreads();
    }
    if (tid == 0) sgn = (Z[si[0] * J + col] < 0.0) ? -1.0 : 1.0;
    __syncthreads();
    for (int j = tid; j < J; j += 256) V64[j * R + r] = sgn * Z[j * J + col];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// ALS iteration
// ---------------------------------------------------------------------------
__global__ void k_init_start(InitArgs a) {
  // H = I, S_k = I
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int RR = a.R * a.R;
  if (e < RR) a.H[e] = ((int)e / a.R == (int)e % a.R) ? 1.0 : 0.0;
  if (e < (int64_t)a.K * a.R) a.W[e] = 1.0;
}

// Per slice k (one 256-thread workgroup): T = X_k V (rows staged 64 at a time),
// Yh_k = T^T X_k into Y buffer 1, Dh_k = T^T T into D buffer 1, n_k = ||X_k||^2.
constexpr int kInitMB = 64;

template <int RW, int JW>
__global__ __launch_bounds__(256) void k_init_accum(InitArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int k = blockIdx.x;
  const int J = a.J, R = a.R, RR = R * R;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int XS = J | 1;
  float *sV = (float *)smem;                    // J x R
  float *sX = sV + J * R;                       // kInitMB x XS
  float *sU = sX + kInitMB * XS;                // kInitMB x (R + 1)
  for (int e = tid; e < J * R; e += 256) sV[e] = (float)a.V64[e];
  float dY[RW][JW];
#pragma unroll
  for (int rr = 0; rr < RW; ++rr)
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) dY[rr][jj] = 0.f;
  double dD[4] = {0.0, 0.0, 0.0, 0.0};
  double dn = 0.0;
  const int64_t a0 = a.row_ptr[k], a1 = a.row_ptr[k + 1];
  for (int64_t r0 = a0; r0 < a1; r0 += kInitMB) {
    const int m = (int)min((int64_t)kInitMB, a1 - r0);
    __syncthreads();
    for (int e = tid; e < m * J; e += 256) {
      const int row = e / J, col = e - row * J;
      const float x = a.X[r0 * J + e];
      sX[row * XS + col] = x;
      dn = fma((double)x, (double)x, dn);
    }
    __syncthreads();
    {
      // lane = row (rows >= m compute unused values), waves split the ranks
      float t[RW];
#pragma unroll
      for (int rr = 0; rr < RW; ++rr) t[rr] = 0.f;
      const float *xr = sX + lane * XS;
      for (int j = 0; j < J; ++j) {
        const float xv = xr[j];
#pragma unroll
        for (int rr = 0; rr < RW; ++rr) {
          const int r = wv + 4 * rr;
          if (r < R) t[rr] = fmaf(xv, sV[j * R + r], t[rr]);
        }
      }
#pragma unroll
      for (int rr = 0; rr < RW; ++rr) {
        const int r = wv + 4 * rr;
        if (r < R) sU[lane * (R + 1) + r] = t[rr];
      }
    }
    __syncthreads();
    for (int row = 0; row < m; ++row) {
      float u[RW];
#pragma unroll
      for (int rr = 0; rr < RW; ++rr) {
        const int r = wv + 4 * rr;
        u[rr] = (r < R) ? sU[row * (R + 1) + r] : 0.f;
      }
#pragma unroll
      for (int jj = 0; jj < JW; ++jj) {
        const int j = min(lane + 64 * jj, J - 1);
        const float x = sX[row * XS + j];
#pragma unroll
        for (int rr = 0; rr < RW; ++rr) dY[rr][jj] = fmaf(u[rr], x, dY[rr][jj]);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = min(tid + 256 * i, RR - 1);
      const int r = q / R, s2 = q - r * R;
      double acc = dD[i];
      for (int row = 0; row < m; ++row)
        acc = fma((double)sU[row * (R + 1) + r], (double)sU[row * (R + 1) + s2], acc);
      dD[i] = acc;
    }
  }
  float *Yh = a.Y + (a.K_cap + k) * (int64_t)a.ys;
#pragma unroll
  for (int rr = 0; rr < RW; ++rr) {
    const int r = wv + 4 * rr;
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
      const int j = lane + 64 * jj;
      if (r < R && j < J) Yh[r * J + j] = dY[rr][jj];
    }
  }
  double *Dh = a.Dh + (int64_t)k * RR;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = tid + 256 * i;
    if (q < RR) Dh[q] = dD[i];
  }
  __shared__ double red[4];
  dn = wave_sum(dn);
  if (lane == 0) red[wv] = dn;
  __syncthreads();
  if (tid == 0) a.n[k] = ((red[0] + red[1]) + red[2]) + red[3];
}

// small dense products in LDS, the whole block taking part:
// C (m x p) = A (m x q) * B (q x p), all row-major FP64
__device__ __forceinline__ void blk_mm(const double *A, const double *B, double *C, int m, int q, int p) {
  for (int e = threadIdx.x; e < m * p; e += blockDim.x) {
    const int i = e / p, j = e - i * p;
    double acc = 0.0;
    for (int t = 0; t < q; ++t) acc = fma(A[i * q + t], B[t * p + j], acc);
    C[e] = acc;
  }
}
// C = A * B^T (A m x q, B p x q)
__device__ __forceinline__ void blk_mmt(const double *A, const double *B, double *C, int m, int q, int p) {
  for (int e = threadIdx.x; e < m * p; e += blockDim.x) {
    const int i = e / p, j = e - i * p;
    double acc = 0.0;
    for (int t = 0; t < q; ++t) acc = fma(A[i * q + t], B[j * q + t], acc);
    C[e] = acc;
  }
}
// C = A^T * B (A q x m, B q x p)
__device__ __forceinline__ void blk_mtm(const double *A, const double *B, double *C, int m, int q, int p) {
  for (int e = threadIdx.x; e < m * p; e += blockDim.x) {
    const int i = e / p, j = e - i * p;
    double acc = 0.0;
    for (int t = 0; t < q; ++t) acc = fma(A[t * m + i], B[t * p + j], acc);
    C[e] = acc;
  }
}

struct SliceLds {
  size_t oV, oYh, oH, oHw, oDh, oT, oP, oZ, oPis, oW, oRot, oPair, bytes;
};

__host__ __device__ inline SliceLds slice_lds(int J, int R) {
  SliceLds L;
  const size_t RR = (size_t)R * R;
  size_t o = 0;
  L.oV = o;   o += (size_t)J * R * 8;
  L.oYh = o;  o += align_up((size_t)R * J * 4, 16);
  L.oH = o;   o += RR * 8;
  L.oHw = o;  o += RR * 8;
  L.oDh = o;  o += RR * 8;
  L.oT = o;   o += RR * 8;
  L.oP = o;   o += RR * 8;
  L.oZ = o;   o += RR * 8;
  L.oPis = o; o += RR * 8;
  L.oW = o;   o += 32 * 8;
  L.oRot = o; o += 64 * 8;
  L.oPair = o; o += 64 * 4;
  L.bytes = align_up(o, 16);
  return L;
}

// Procrustes step per slice (a chunk of slices per 256-thread workgroup):
// P_k^{-1/2}, Pi_k, Y_k = P_k^{-1/2} Hw Yh_k (Y buffer 0), Pi_k (D buffer 0),
// chunk partials [M1 | W^T W].
__global__ __launch_bounds__(256) void k_init_slice(InitArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int J = a.J, R = a.R, RR = R * R;
  const int tid = threadIdx.x;
  const SliceLds L = slice_lds(J, R);
  double *sV = (double *)(smem + L.oV);
  float *sYh = (float *)(smem + L.oYh);
  double *sH = (double *)(smem + L.oH);
  double *sHw = (double *)(smem + L.oHw);
  double *sDh = (double *)(smem + L.oDh);
  double *sT = (double *)(smem + L.oT);
  double *sP = (double *)(smem + L.oP);
  double *sZ = (double *)(smem + L.oZ);
  double *sPis = (double *)(smem + L.oPis);
  double *sYV = sP;   // P is dead once P^{-1/2} and Pi are formed
  double *sw = (double *)(smem + L.oW);
  double *sRot = (double *)(smem + L.oRot);
  int *sPair = (int *)(smem + L.oPair);
  for (int e = tid; e < J * R; e += 256) sV[e] = a.V64[e];
  for (int e = tid; e < RR; e += 256) sH[e] = a.H[e];
  double m1[4] = {0.0, 0.0, 0.0, 0.0}, ww[4] = {0.0, 0.0, 0.0, 0.0};
  const int k0 = blockIdx.x * a.chunk, k1 = min(a.K, k0 + a.chunk);
  for (int k = k0; k < k1; ++k) {
    __syncthreads();
    const float *Yh = a.Y + (a.K_cap + k) * (int64_t)a.ys;
    for (int e = tid; e < R * J; e += 256) sYh[e] = Yh[e];
    for (int e = tid; e < RR; e += 256) sDh[e] = a.Dh[(int64_t)k * RR + e];
    if (tid < R) sw[tid] = a.W[(int64_t)k * R + tid];
    __syncthreads();
    for (int e = tid; e < RR; e += 256) sHw[e] = sH[e] * sw[e % R];
    __syncthreads();
    blk_mm(sHw, sDh, sT, R, R, R);   // Hw Dh
    __syncthreads();
    blk_mmt(sT, sHw, sP, R, R, R);   // P = Hw Dh Hw^T
    __syncthreads();
    for (int e = tid; e < RR; e += 256) {
      const int i = e / R, j = e - i * R;
      if (i < j) {
        const double v = 0.5 * (sP[e] + sP[j * R + i]);
        sP[e] = v;
        sP[j * R + i] = v;
      }
    }
    __syncthreads();
    if ((tid >> 6) == 0) wave_jacobi(sP, sZ, R, sRot, sPair);
    __syncthreads();
    double top = 0.0;
    for (int i = 0; i < R; ++i) top = fmax(top, sP[i * R + i]);
    // P^{-1/2} and Pi on the retained eigenspace
    float *Pi = a.D + (int64_t)k * RR;
    for (int e = tid; e < RR; e += 256) {
      const int r = e / R, s2 = e - r * R;
      double ps = 0.0, pp = 0.0;
      for (int i = 0; i < R; ++i) {
        const double li = sP[i * R + i];
        if (top > 0.0 && li > kEigCutoff * top) {
          const double z = sZ[r * R + i] * sZ[s2 * R + i];
          ps += z / sqrt(li);
          pp += z;
        }
      }
      sPis[e] = ps;
      Pi[e] = (float)pp;
    }
    __syncthreads();
    blk_mm(sPis, sHw, sT, R, R, R);  // T = P^{-1/2} Hw
    __syncthreads();
    // Y_k = T Yh_k (stored FP32) and Yh_k V
    float *Yk = a.Y + (int64_t)k * a.ys;
    for (int e = tid; e < R * J; e += 256) {
      const int r = e / J, j = e - r * J;
      double acc = 0.0;
      for (int t = 0; t < R; ++t) acc = fma(sT[r * R + t], (double)sYh[t * J + j], acc);
      Yk[e] = (float)acc;
    }
    for (int e = tid; e < RR; e += 256) {
      const int r = e / R, s2 = e - r * R;
      double acc = 0.0;
      for (int j = 0; j < J; ++j) acc = fma((double)sYh[r * J + j], sV[j * R + s2], acc);
      sYV[e] = acc;
    }
    __syncthreads();
    // M1 += (T Yh V) S_k, W^T W += w w^T
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = tid + 256 * i;
      if (q < RR) {
        const int r = q / R, s2 = q - r * R;
        double acc = 0.0;
        for (int t = 0; t < R; ++t) acc = fma(sT[r * R + t], sYV[t * R + s2], acc);
        m1[i] += acc * sw[s2];
        ww[i] += sw[r] * sw[s2];
      }
    }
  }
  double *out = a.part + (int64_t)blockIdx.x * a.plen;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = tid + 256 * i;
    if (q < RR) {
      out[q] = m1[i];
      out[RR + q] = ww[i];
    }
  }
}

// Partials of M2 = sum_k Y_k^T H S_k (J x R), a chunk of slices per workgroup.
__global__ __launch_bounds__(256) void k_init_m2(InitArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int J = a.J, R = a.R, RR = R * R, JR = J * R;
  const int tid = threadIdx.x;
  double *sAcc = (double *)smem;          // J x R
  double *sHw = sAcc + JR;                // R x R
  double *sH = sHw + RR;                  // R x R
  float *sY = (float *)(sH + RR);         // R x J
  for (int e = tid; e < JR; e += 256) sAcc[e] = 0.0;
  for (int e = tid; e < RR; e += 256) sH[e] = a.H[e];
  const int k0 = blockIdx.x * a.chunk, k1 = min(a.K, k0 + a.chunk);
  for (int k = k0; k < k1; ++k) {
    __syncthreads();
    const float *Yk = a.Y + (int64_t)k * a.ys;
    for (int e = tid; e < R * J; e += 256) sY[e] = Yk[e];
    for (int e = tid; e < RR; e += 256) sHw[e] = sH[e] * a.W[(int64_t)k * R + e % R];
    __syncthreads();
    for (int e = tid; e < JR; e += 256) {
      const int j = e / R, r = e - j * R;
      double acc = sAcc[e];
      for (int s2 = 0; s2 < R; ++s2) acc = fma((double)sY[s2 * J + j], sHw[s2 * R + r], acc);
      sAcc[e] = acc;
    }
  }
  __syncthreads();
  double *out = a.part + (int64_t)blockIdx.x * a.plen;
  for (int e = tid; e < JR; e += 256) out[e] = sAcc[e];
}

// W step and slice losses, a chunk of slices per workgroup: c = diag(H^T Y_k V),
// w_k = Mw^{-1} c, loss_k = n_k - 2 w.c + w^T ((H^T Pi_k H) * (V^T V)) w.
__global__ __launch_bounds__(256) void k_init_w(InitArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int J = a.J, R = a.R, RR = R * R;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double *sV = (double *)smem;            // J x R
  double *sH = sV + J * R;
  double *sMi = sH + RR;
  double *sVtV = sMi + RR;
  double *sYV = sVtV + RR;
  double *sPi = sYV + RR;
  double *sT = sPi + RR;
  double *sHPH = sT + RR;
  double *sc = sHPH + RR;                 // 32
  double *sw = sc + 32;                   // 32
  double *sred = sw + 32;                 // 4
  float *sY = (float *)(sred + 4);        // R x J
  for (int e = tid; e < J * R; e += 256) sV[e] = a.V64[e];
  for (int e = tid; e < RR; e += 256) {
    sH[e] = a.H[e];
    sMi[e] = a.Mwinv[e];
    sVtV[e] = a.VtV[e];
  }
  double loss_acc = 0.0, n_acc = 0.0;
  const int k0 = blockIdx.x * a.chunk, k1 = min(a.K, k0 + a.chunk);
  for (int k = k0; k < k1; ++k) {
    __syncthreads();
    const float *Yk = a.Y + (int64_t)k * a.ys;
    for (int e = tid; e < R * J; e += 256) sY[e] = Yk[e];
    for (int e = tid; e < RR; e += 256) sPi[e] = (double)a.D[(int64_t)k * RR + e];
    __syncthreads();
    for (int e = tid; e < RR; e += 256) {
      const int r = e / R, s2 = e - r * R;
      double acc = 0.0;
      for (int j = 0; j < J; ++j) acc = fma((double)sY[r * J + j], sV[j * R + s2], acc);
      sYV[e] = acc;
    }
    blk_mtm(sH, sPi, sT, R, R, R);   // H^T Pi
    __syncthreads();
    blk_mm(sT, sH, sHPH, R, R, R);   // H^T Pi H
    if (tid < R) {
      double acc = 0.0;
      for (int s2 = 0; s2 < R; ++s2) acc = fma(sH[s2 * R + tid], sYV[s2 * R + tid], acc);
      sc[tid] = acc;
    }
    __syncthreads();
    if (tid < R) {
      double acc = 0.0;
      for (int s2 = 0; s2 < R; ++s2) acc = fma(sMi[tid * R + s2], sc[s2], acc);
      sw[tid] = acc;
      a.W[(int64_t)k * R + tid] = acc;
    }
    __syncthreads();
    double q = 0.0;
    for (int e = tid; e < RR; e += 256) {
      const int r = e / R, s2 = e - r * R;
      q += sw[r] * sHPH[e] * sVtV[e] * sw[s2];
    }
    q = wave_sum(q);
    if (lane == 0) sred[wv] = q;
    __syncthreads();
    if (tid == 0) {
      double wc = 0.0;
      for (int r = 0; r < R; ++r) wc += sw[r] * sc[r];
      const double nk = a.n[k];
      loss_acc += nk - 2.0 * wc + (((sred[0] + sred[1]) + sred[2]) + sred[3]);
      n_acc += nk;
    }
  }
  if (tid == 0) {
    double *out = a.part + (int64_t)blockIdx.x * a.plen;
    out[0] = loss_acc;
    out[1] = n_acc;
  }
}

// Solves on the reduced partials (one 512-thread workgroup).
//   mode 0: H = M1 ((V^T V) * (W^T W))^{-1}; keeps W^T W
//   mode 1: V = M2 ((H^T H) * (W^T W))^{-1}; V^T V; ((H^T H) * (V^T V))^{-1}
//   mode 2: loss and sum n
constexpr int kInitSolveThreads = 512;

template <int RM>
__global__ __launch_bounds__(kInitSolveThreads) void k_init_solve(InitArgs a, int mode) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int J = a.J, R = a.R, RR = R * R, JR = J * R;
  const int tid = threadIdx.x, lane = tid & 63;
  double *sA = (double *)smem;   // RR (M1) or J x R (M2, then the new V)
  double *sM = sA + (JR > RR ? JR : RR);
  double *sMi = sM + RR;
  double *sG = sMi + RR;         // H^T H
  double *sWork = sG + RR;
  double *sZ = sWork + RR;
  double *sRot = sZ + RR;        // 64
  int *sPair = (int *)(sRot + 64);
  int *sFlag = sPair + 64;
  if (mode == 2) {
    if (tid < 2) a.result[tid] = ordered_sum(a.part, a.plen, tid, 0, a.n_chunks);
    return;
  }
  if (tid == 0) sFlag[0] = 1;
  if (mode == 0) {
    for (int e = tid; e < 2 * RR; e += blockDim.x) {
      const double v = ordered_sum(a.part, a.plen, e, 0, a.n_chunks);
      if (e < RR) sA[e] = v;
      else a.WtW[e - RR] = v;
    }
    __syncthreads();
    // (V^T V) * (W^T W)
    for (int e = tid; e < RR; e += blockDim.x) {
      const int r = e / R, s2 = e - r * R;
      double acc = 0.0;
      for (int j = 0; j < J; ++j) acc = fma(a.V64[j * R + r], a.V64[j * R + s2], acc);
      sM[e] = acc * a.WtW[e];
    }
  } else {
    for (int e = tid; e < JR; e += blockDim.x) sA[e] = ordered_sum(a.part, a.plen, e, 0, a.n_chunks);
    for (int e = tid; e < RR; e += blockDim.x) {
      const int r = e / R, s2 = e - r * R;
      double acc = 0.0;
      for (int t = 0; t < R; ++t) acc = fma(a.H[t * R + r], a.H[t * R + s2], acc);
      sG[e] = acc;
      sM[e] = acc * a.WtW[e];
    }
  }
  __syncthreads();
  if (!block_spd_inverse<RM>(sM, sMi, R) && lane == 0) sFlag[0] = 0;
  __syncthreads();
  if (!sFlag[0]) block_pinv_of(sM, sMi, sWork, sZ, R, sRot, sPair);
  __syncthreads();
  if (mode == 0) {
    for (int e = tid; e < RR; e += blockDim.x) {
      const int r = e / R, s2 = e - r * R;
      double acc = 0.0;
      for (int t = 0; t < R; ++t) acc = fma(sA[r * R + t], sMi[t * R + s2], acc);
      a.H[e] = acc;
    }
    return;
  }
  // V = M2 Mv^{-1}: every thread forms its entries in registers, then (after
  // the barrier, once M2 is no longer read) V replaces M2 in LDS
  constexpr int kPer = (kMaxJ * kMaxR + kInitSolveThreads - 1) / kInitSolveThreads;
  double vloc[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int e = tid + kInitSolveThreads * i;
    vloc[i] = 0.0;
    if (e < JR) {
      const int j = e / R, r = e - j * R;
      double acc = 0.0;
      for (int t = 0; t < R; ++t) acc = fma(sA[j * R + t], sMi[t * R + r], acc);
      vloc[i] = acc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int e = tid + kInitSolveThreads * i;
    if (e < JR) {
      a.V64[e] = vloc[i];
      sA[e] = vloc[i];
    }
  }
  __syncthreads();
  if (tid == 0) sFlag[0] = 1;
  for (int e = tid; e < RR; e += blockDim.x) {
    const int r = e / R, s2 = e - r * R;
    double acc = 0.0;
    for (int j = 0; j < J; ++j) acc = fma(sA[j * R + r], sA[j * R + s2], acc);
    a.VtV[e] = acc;
    sM[e] = sG[e] * acc;
  }
  __syncthreads();
  if (!block_spd_inverse<RM>(sM, sMi, R) && lane == 0) sFlag[0] = 0;
  __syncthreads();
  if (!sFlag[0]) block_pinv_of(sM, sMi, sWork, sZ, R, sRot, sPair);
  __syncthreads();
  for (int e = tid; e < RR; e += blockDim.x) a.Mwinv[e] = sMi[e];
}

// Hand-off per slice: Y_k <- H^T Y_k, D_k <- H^T Pi_k H (buffer 0).
__global__ __launch_bounds__(256) void k_init_handoff(InitArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int k = blockIdx.x;
  const int J = a.J, R = a.R, RR = R * R;
  const int tid = threadIdx.x;
  double *sH = (double *)smem;
  double *sPi = sH + RR;
  double *sT = sPi + RR;
  float *sY = (float *)(sT + RR);
  float *Yk = a.Y + (int64_t)k * a.ys;
  float *Dk = a.D + (int64_t)k * RR;
  for (int e = tid; e < RR; e += 256) {
    sH[e] = a.H[e];
    sPi[e] = (double)Dk[e];
  }
  for (int e = tid; e < R * J; e += 256) sY[e] = Yk[e];
  __syncthreads();
  blk_mtm(sH, sPi, sT, R, R, R);
  __syncthreads();
  for (int e = tid; e < RR; e += 256) {
    const int r = e / R, s2 = e - r * R;
    double acc = 0.0;
    for (int t = 0; t < R; ++t) acc = fma(sT[r * R + t], sH[t * R + s2], acc);
    Dk[e] = (float)acc;
  }
  for (int e = tid; e < R * J; e += 256) {
    const int r = e / J, j = e - r * J;
    double acc = 0.0;
    for (int t = 0; t < R; ++t) acc = fma(sH[t * R + r], (double)sY[t * J + j], acc);
    Yk[e] = (float)acc;
  }
  for (int e = R * J + tid; e < a.ys; e += 256) Yk[e] = 0.f;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename F>
static int allow_lds_init(F *fn, size_t bytes) {
  if (bytes <= 65536) return 0;
  return (int)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

int init_gram_chunks(int J) {
  const int nt = (J + kGT - 1) / kGT;
  int g = 1024 / (nt * nt);
  return g < 1 ? 1 : (g > 256 ? 256 : g);
}

int launch_init_gram(int J, int64_t N, int n_gc, const float *X, double *part, double *Gm, hipStream_t s) {
  const int nt = (J + kGT - 1) / kGT;
  const int64_t rpc = (N + n_gc - 1) / n_gc;
  hipLaunchKernelGGL(k_gram_partial, dim3(nt * nt, n_gc), dim3(256), 0, s, J, N, rpc, X, part);
  if (int e = (int)hipGetLastError()) return e;
  hipLaunchKernelGGL(k_gram_reduce, dim3((J * J + 255) / 256), dim3(256), 0, s, J * J, n_gc, part, Gm);
  return (int)hipGetLastError();
}

int launch_sym_eig(int n, double *A, double *Z, double *evals, hipStream_t s) {
  hipLaunchKernelGGL(k_sym_eig, dim3(1), dim3(kEigThreads), 0, s, n, A, Z, evals);
  return (int)hipGetLastError();
}

int launch_top_vectors(int J, int R, const double *evals, const double *Z, double *V64, hipStream_t s) {
  hipLaunchKernelGGL(k_top_vectors, dim3(1), dim3(256), 0, s, J, R, evals, Z, V64);
  return (int)hipGetLastError();
}

int launch_init_start(const InitArgs &a, hipStream_t s) {
  const int64_t cnt = std::max<int64_t>((int64_t)a.K * a.R, (int64_t)a.R * a.R);
  hipLaunchKernelGGL(k_init_start, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, a);
  return (int)hipGetLastError();
}

template <int RW, int JW>
static int launch_accum_init_t(const InitArgs &a, hipStream_t s) {
  const size_t bytes = (size_t)a.J * a.R * 4 + (size_t)kInitMB * (a.J | 1) * 4 + (size_t)kInitMB * (a.R + 1) * 4;
  if (int e = allow_lds_init(k_init_accum<RW, JW>, bytes)) return e;
  hipLaunchKernelGGL((k_init_accum<RW, JW>), dim3(a.K), dim3(256), bytes, s, a);
  return (int)hipGetLastError();
}

static int launch_init_accum(const InitArgs &a, hipStream_t s) {
  const int rw = (a.R + 3) / 4, jw = (a.J + 63) / 64;
  switch (rw * 8 + jw) {
#define C(RW, JW) case RW * 8 + JW: return launch_accum_init_t<RW, JW>(a, s);
    C(1, 1) C(1, 2) C(1, 3) C(1, 4) C(2, 1) C(2, 2) C(2, 3) C(2, 4)
    C(3, 1) C(3, 2) C(3, 3) C(3, 4) C(4, 1) C(4, 2) C(4, 3) C(4, 4)
    C(5, 1) C(5, 2) C(5, 3) C(5, 4) C(6, 1) C(6, 2) C(6, 3) C(6, 4)
    C(7, 1) C(7, 2) C(7, 3) C(7, 4) C(8, 1) C(8, 2) C(8, 3) C(8, 4)
#undef C
    default: return (int)hipErrorInvalidValue;
  }
}

template <int RM>
static int launch_init_solve_t(const InitArgs &a, int mode, hipStream_t s) {
  const size_t RR = (size_t)a.R * a.R, JR = (size_t)a.J * a.R;
  const size_t bytes = ((JR > RR ? JR : RR) + 5 * RR + 64) * 8 + 70 * 4;
  if (int e = allow_lds_init(k_init_solve<RM>, bytes)) return e;
  hipLaunchKernelGGL((k_init_solve<RM>), dim3(1), dim3(kInitSolveThreads), bytes, s, a, mode);
  return (int)hipGetLastError();
}

static int launch_init_solve(const InitArgs &a, int mode, hipStream_t s) {
  if (a.R <= 8) return launch_init_solve_t<8>(a, mode, s);
  if (a.R <= 12) return launch_init_solve_t<12>(a, mode, s);
  if (a.R <= 16) return launch_init_solve_t<16>(a, mode, s);
  if (a.R <= 24) return launch_init_solve_t<24>(a, mode, s);
  return launch_init_solve_t<32>(a, mode, s);
}

int launch_init_iteration(const InitArgs &a, hipStream_t s) {
  const size_t RR = (size_t)a.R * a.R, JR = (size_t)a.J * a.R;
  if (int e = launch_init_accum(a, s)) return e;
  {
    const size_t bytes = slice_lds(a.J, a.R).bytes;
    if (int e = allow_lds_init(k_init_slice, bytes)) return e;
    hipLaunchKernelGGL(k_init_slice, dim3(a.n_chunks), dim3(256), bytes, s, a);
    if (int e = (int)hipGetLastError()) return e;
  }
  if (int e = launch_init_solve(a, 0, s)) return e;
  {
    const size_t bytes = (JR + 2 * RR) * 8 + JR * 4;
    if (int e = allow_lds_init(k_init_m2, bytes)) return e;
    hipLaunchKernelGGL(k_init_m2, dim3(a.n_chunks), dim3(256), bytes, s, a);
    if (int e = (int)hipGetLastError()) return e;
  }
  if (int e = launch_init_solve(a, 1, s)) return e;
  {
    const size_t bytes = (JR + 7 * RR + 68) * 8 + JR * 4;
    if (int e = allow_lds_init(k_init_w, bytes)) return e;
    hipLaunchKernelGGL(k_init_w, dim3(a.n_chunks), dim3(256), bytes, s, a);
    if (int e = (int)hipGetLastError()) return e;
  }
  return launch_init_solve(a, 2, s);
}

int launch_init_handoff(const InitArgs &a, hipStream_t s) {
  const size_t RR = (size_t)a.R * a.R;
  const size_t bytes = 3 * RR * 8 + (size_t)a.R * a.J * 4;
  if (int e = allow_lds_init(k_init_handoff, bytes)) return e;
  hipLaunchKernelGGL(k_init_handoff, dim3(a.K), dim3(256), bytes, s, a);
  return (int)hipGetLastError();
}

}  // namespace dash
