// gfx950 kernels of the streaming PARAFAC2 update (DASH).
//
// One update = per ALS pass: k_pass (fused Lemma 1 + Lemma 2 + slice sweep),
// k_reduce + k_solve (Lemma 3 and the next pass's V-derived operands), then
// k_commit.  See dash_dev.h for layouts.
//
// Thread mapping used for every R x J per-slice matrix (Y_k, its increment and
// the F^T accumulator): wave w of the 4 waves owns rows r = w, w+4, w+8, ...
// (RW of them) and lane l owns columns j = l, l+64, ... (JW of them), so a row
// of Y_k is a coalesced 64-float access per wave and diag(Y_k V) is a wave
// reduction.  R x R matrices use a flat mapping q = tid + 256 i.
#include <hip/hip_runtime.h>
#include <math.h>

#include "dash_dev.h"

namespace dash {

// ---------------------------------------------------------------------------
// wave / block helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
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

// Cholesky factorisation of the n x n SPD matrix M (row-major, LDS) by one
// wave, lane i owning row i.  The lower factor overwrites the lower triangle.
// Fails (returns false, uniformly) when a pivot is not above kPivotRel times the
// largest diagonal entry -- the same acceptance rule as the oracle.
__device__ bool wave_cholesky(double *M, int n) {
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
__device__ void wave_chol_apply(const double *L, double *x, int n) {
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
__device__ void wave_jacobi(double *A, double *Z, int n, double *rot, int *pair) {
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
    if (!(off > 1e-30 * tot)) break;
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
__device__ void wave_pinv_apply(double *M, double *x, int n, double *Z, double *tmp, double *rot,
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

// ---------------------------------------------------------------------------
// LDS plan of the pass / accumulate kernels
// ---------------------------------------------------------------------------
struct PassLds {
  int XS, MB;
  size_t oP, oVt, oX, oU, oW, oWinv, oC, oC2, oM, oDc, oVtV, oZ, oTmp, oRot, oPair, bytes;
};

__host__ __device__ inline PassLds pass_lds(int J, int R) {
  PassLds L;
  L.XS = J | 1;
  L.MB = (J <= 128) ? 64 : 32;
  size_t o = 0;
  L.oP = o;    o += (size_t)J * R * 4;
  L.oVt = o;   o += (size_t)R * J * 4;
  L.oX = o;    o += (size_t)L.MB * L.XS * 4;
  L.oU = o;    o += (size_t)L.MB * (R + 1) * 4;
  o = align_up(o, 16);
  L.oW = o;    o += (size_t)R * 8;
  L.oWinv = o; o += (size_t)R * 4;
  o = align_up(o, 8);
  L.oC = o;    o += (size_t)R * 8;
  L.oC2 = o;   o += (size_t)R * 8;
  L.oM = o;    o += (size_t)R * R * 8;
  L.oDc = o;   o += (size_t)R * R * 4;
  o = align_up(o, 8);
  L.oVtV = o;  o += (size_t)R * R * 8;
  L.oZ = o;    o += (size_t)R * R * 8;
  L.oTmp = o;  o += (size_t)64 * 8;
  L.oRot = o;  o += (size_t)64 * 8;
  L.oPair = o; o += (size_t)64 * 4;
  L.bytes = align_up(o, 16);
  return L;
}

// Accumulate one block of m (<= MB) rows already staged in sX (stride XS) and
// their U rows in sU (stride R+1): dY += U^T X, dD += U^T U.
template <int RW, int JW>
__device__ __forceinline__ void accum_block(const float *sX, const float *sU, int XS, int m, int J,
                                            int R, float (&dY)[RW][JW], float (&dD)[4]) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int row = 0; row < m; ++row) {
    float u[RW];
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) {
      const int r = wv + 4 * rr;
      u[rr] = (r < R) ? sU[row * (R + 1) + r] : 0.f;
    }
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
      const int j = lane + 64 * jj;
      const float x = (j < J) ? sX[row * XS + j] : 0.f;
#pragma unroll
      for (int rr = 0; rr < RW; ++rr) dY[rr][jj] = fmaf(u[rr], x, dY[rr][jj]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = tid + 256 * i;
    if (q < R * R) {
      const int r = q / R, s = q - r * R;
      float acc = dD[i];
      for (int row = 0; row < m; ++row) acc = fmaf(sU[row * (R + 1) + r], sU[row * (R + 1) + s], acc);
      dD[i] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// k_pass: one ALS pass over a chunk of slices.
//   for each slice k of the chunk (ascending id):
//     new rows x (if any):  u = (x P) * (1/w_k)          Lemma 1, P = V (V^T V)^{-1}
//                           dY += u^T x, dD += u^T u, dn += ||x||^2
//     fold:   Y_k = lambda^dt Y_k,stored + dY   (touched slices; dt = step - t_k)
//     Lemma 2: c = diag(Y_k V), (V^T V * D_k) w_k = c     (FP64 Cholesky, pinv fallback)
//     sweep:  F^T += sigma w_k * Y_k, G += sigma diag(w_k) D_k diag(w_k), sum n
//   then one F/G/n partial per chunk (reduced in fixed order by k_reduce/k_solve).
// Untouched slices are solved from their stored (undecayed) Y_k, D_k -- the
// solution w_k is invariant to the common factor lambda^dt -- and enter F, G
// with sigma = lambda^dt.
// ---------------------------------------------------------------------------
template <int RW, int JW>
__global__ __launch_bounds__(256) void k_pass(PassArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const StepHeader *h = a.hdr;
  const int chunk = blockIdx.x;
  if (chunk >= h->n_chunks) return;
  const int J = a.J, R = a.R;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = h->K, Kp = h->K_prev;
  const int64_t step = h->step;
  const int gcur = a.ctl->gcur;
  const int win = (a.pass == 0) ? gcur : 1 - gcur;
  const int wout = 1 - gcur;
  const VBundleView vb = vb_view(a.vb + (int64_t)win * a.vb_stride, J, R);
  const PassLds L = pass_lds(J, R);
  float *sP = (float *)(smem + L.oP);
  float *sVt = (float *)(smem + L.oVt);
  float *sX = (float *)(smem + L.oX);
  float *sU = (float *)(smem + L.oU);
  double *sW = (double *)(smem + L.oW);
  float *sWinv = (float *)(smem + L.oWinv);
  double *sC = (double *)(smem + L.oC);
  double *sC2 = (double *)(smem + L.oC2);
  double *sM = (double *)(smem + L.oM);
  float *sDc = (float *)(smem + L.oDc);
  double *sVtV = (double *)(smem + L.oVtV);
  double *sZ = (double *)(smem + L.oZ);
  double *sTmp = (double *)(smem + L.oTmp);
  double *sRot = (double *)(smem + L.oRot);
  int *sPair = (int *)(smem + L.oPair);
  const int XS = L.XS, MB = L.MB;
  const int RR = R * R;

  for (int e = tid; e < J * R; e += 256) sP[e] = vb.P32[e];
  for (int e = tid; e < R * J; e += 256) sVt[e] = vb.Vt32[e];
  for (int e = tid; e < RR; e += 256) sVtV[e] = vb.VtV[e];

  double facc[RW][JW];
  double gacc[4] = {0.0, 0.0, 0.0, 0.0};
  double nacc = 0.0;
#pragma unroll
  for (int rr = 0; rr < RW; ++rr)
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) facc[rr][jj] = 0.0;

  const int k0 = chunk * h->chunk;
  const int k1 = min(K, k0 + h->chunk);
  int t = a.chunk_tptr[chunk];
  const int tend = a.chunk_tptr[chunk + 1];
  const int plen = partial_len(J, R);

  for (int k = k0; k < k1; ++k) {
    const bool touched = (t < tend) && (a.touched[t].slice == k);
    const bool is_new = k >= Kp;
    __syncthreads();  // LDS of the previous slice is free
    if (tid < R) {
      const double w = (is_new && a.pass == 0) ? 1.0 : a.W[((int64_t)win * a.K_cap + k) * R + tid];
      sW[tid] = w;
    }
    __syncthreads();
    if (tid < R) {
      double top = 0.0;
      for (int r = 0; r < R; ++r) top = fmax(top, fabs(sW[r]));
      const double w = sW[tid];
      sWinv[tid] = (fabs(w) > kWCutoff * top) ? (float)(1.0 / w) : 0.f;
    }

    float dY[RW][JW];
    float dD[4] = {0.f, 0.f, 0.f, 0.f};
    double dn = 0.0;
#pragma unroll
    for (int rr = 0; rr < RW; ++rr)
#pragma unroll
      for (int jj = 0; jj < JW; ++jj) dY[rr][jj] = 0.f;

    if (touched && a.mode == 0) {
      const Touched te = a.touched[t];
      for (int g = te.g_begin; g < te.g_end; ++g) {
        const Group gr = a.groups[g];
        for (int r0 = 0; r0 < gr.nrows; r0 += MB) {
          const int m = min(MB, gr.nrows - r0);
          __syncthreads();
          const float *src = gr.src + (int64_t)r0 * J;
          for (int e = tid; e < m * J; e += 256) {
            const int row = e / J, col = e - row * J;
            sX[row * XS + col] = src[e];
          }
          __syncthreads();
          if (lane < m) {
            float tacc[RW];
#pragma unroll
            for (int rr = 0; rr < RW; ++rr) tacc[rr] = 0.f;
            float nx = 0.f;
            const float *xr = sX + lane * XS;
            for (int j = 0; j < J; ++j) {
              const float xv = xr[j];
              nx = fmaf(xv, xv, nx);
#pragma unroll
              for (int rr = 0; rr < RW; ++rr) {
                const int r = wv + 4 * rr;
                if (r < R) tacc[rr] = fmaf(xv, sP[j * R + r], tacc[rr]);
              }
            }
#pragma unroll
            for (int rr = 0; rr < RW; ++rr) {
              const int r = wv + 4 * rr;
              if (r < R) {
                const float u = tacc[rr] * sWinv[r];
                sU[lane * (R + 1) + r] = u;
                if (a.write_u) a.U_out[(gr.out_row + r0 + lane) * R + r] = u;
              }
            }
            if (wv == 0) dn += (double)nx;
          }
          __syncthreads();
          accum_block<RW, JW>(sX, sU, XS, m, J, R, dY, dD);
        }
      }
      if (wv == 0) dn = wave_sum(dn);
    }

    const int b = a.cur[k];
    const double s_old = is_new ? 0.0 : pow(a.lambda, (double)(step - a.tlast[k]));
    const float s_old_f = (float)s_old;
    const float *Yst = a.Y + ((int64_t)b * a.K_cap + k) * R * J;
    float yv[RW][JW];
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) {
      const int r = wv + 4 * rr;
#pragma unroll
      for (int jj = 0; jj < JW; ++jj) {
        const int j = lane + 64 * jj;
        const float yo = (!is_new && r < R && j < J) ? Yst[r * J + j] : 0.f;
        yv[rr][jj] = touched ? fmaf(s_old_f, yo, dY[rr][jj]) : yo;
      }
    }
    // c_r = sum_j Y_k[r][j] V[j][r]  (wave reduction, FP64)
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) {
      const int r = wv + 4 * rr;
      double part = 0.0;
#pragma unroll
      for (int jj = 0; jj < JW; ++jj) {
        const int j = lane + 64 * jj;
        if (r < R && j < J) part += (double)yv[rr][jj] * (double)sVt[r * J + j];
      }
      part = wave_sum(part);
      if (lane == 0 && r < R) {
        sC[r] = part;
        sC2[r] = part;
      }
    }
    const float *Dst = a.D + ((int64_t)b * a.K_cap + k) * RR;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = tid + 256 * i;
      if (q < RR) {
        const float dold = is_new ? 0.f : Dst[q];
        const float dc = touched ? fmaf(s_old_f, dold, dD[i]) : dold;
        sDc[q] = dc;
        sM[q] = sVtV[q] * (double)dc;
      }
    }
    __syncthreads();
    if (a.mode == 0) {
      if (wv == 0) {
        if (!wave_cholesky(sM, R)) {
          for (int q = lane; q < RR; q += 64) sM[q] = sVtV[q] * (double)sDc[q];
          if (lane < R) sC[lane] = sC2[lane];
          wave_sync();
          wave_pinv_apply(sM, sC, R, sZ, sTmp, sRot, sPair);
        } else {
          wave_chol_apply(sM, sC, R);
        }
      }
      __syncthreads();
      if (tid < R) a.W[((int64_t)wout * a.K_cap + k) * R + tid] = sC[tid];
    } else {
      if (tid < R) sC[tid] = sW[tid];
      __syncthreads();
    }
    const double sigma = touched ? 1.0 : s_old;
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) {
      const int r = wv + 4 * rr;
      if (r < R) {
        const double wr = sigma * sC[r];
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) facc[rr][jj] += wr * (double)yv[rr][jj];
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = tid + 256 * i;
      if (q < RR) {
        const int r = q / R, s = q - r * R;
        gacc[i] += sigma * sC[r] * sC[s] * (double)sDc[q];
      }
    }
    if (tid == 0) {
      const double nold = is_new ? 0.0 : a.n[(int64_t)b * a.K_cap + k];
      const double ncur = s_old * nold + dn;
      nacc += ncur;
      if (touched && a.mode == 0) a.n[(int64_t)(1 - b) * a.K_cap + k] = ncur;
    }
    if (touched && a.mode == 0) {
      float *Ynx = a.Y + ((int64_t)(1 - b) * a.K_cap + k) * R * J;
#pragma unroll
      for (int rr = 0; rr < RW; ++rr) {
        const int r = wv + 4 * rr;
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
          const int j = lane + 64 * jj;
          if (r < R && j < J) Ynx[r * J + j] = yv[rr][jj];
        }
      }
      float *Dnx = a.D + ((int64_t)(1 - b) * a.K_cap + k) * RR;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = tid + 256 * i;
        if (q < RR) Dnx[q] = sDc[q];
      }
    }
    if (touched) ++t;
  }

  double *part = a.partials + (int64_t)chunk * plen;
#pragma unroll
  for (int rr = 0; rr < RW; ++rr) {
    const int r = wv + 4 * rr;
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
      const int j = lane + 64 * jj;
      if (r < R && j < J) part[r * J + j] = facc[rr][jj];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = tid + 256 * i;
    if (q < RR) part[R * J + q] = gacc[i];
  }
  if (tid == 0) part[R * J + RR] = nacc;
}

// ---------------------------------------------------------------------------
// k_reduce: first level of the fixed-order reduction of chunk partials.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(const double *partials, double *gpart,
                                                const StepHeader *h, int plen) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  const int g = blockIdx.y;
  if (e >= plen || g >= h->n_rgroups) return;
  const int c0 = g * h->chunks_per_rgroup;
  const int c1 = min(h->n_chunks, c0 + h->chunks_per_rgroup);
  double s = 0.0;
  for (int c = c0; c < c1; ++c) s += partials[(int64_t)c * plen + e];
  gpart[(int64_t)g * plen + e] = s;
}

// ---------------------------------------------------------------------------
// k_solve: Lemma 3 and the V-derived operands of the next pass (one workgroup).
//   mode 0: F, G, n from the group partials; V = F G^{-1} into the spare bundle;
//           V^T V, B = (V^T V)^{-1}, P = V B; loss / fit; ok flag.
//   mode 1: bundle of the committed buffer from its V64 (V^T V, V^T, P).
//   mode 2: loss / fit of the committed V with F, G from the partials.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_solve(int J, int R, const double *gpart, int n_rgroups,
                                               char *vbase, int64_t vb_stride, Ctl *ctl, int mode) {
  __shared__ double sG[kMaxR * kMaxR];
  __shared__ double sL[kMaxR * kMaxR];
  __shared__ double sB[kMaxR * kMaxR];
  __shared__ double sVtV[kMaxR * kMaxR];
  __shared__ double sZ[kMaxR * kMaxR];
  __shared__ double sRot[64];
  __shared__ int sPair[64];
  __shared__ double sRed[kWaves];
  __shared__ double sSumN;
  __shared__ int sFlag;
  __shared__ int sBad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int RR = R * R, RJ = R * J;
  const int plen = partial_len(J, R);
  const int gcur = ctl->gcur;
  const int out = (mode == 0) ? 1 - gcur : gcur;
  const VBundleView vo = vb_view(vbase + (int64_t)out * vb_stride, J, R);
  if (tid == 0) sBad = 0;
  if (mode != 1) {
    for (int q = tid; q < RR; q += 256) {
      double s = 0.0;
      for (int g = 0; g < n_rgroups; ++g) s += gpart[(int64_t)g * plen + RJ + q];
      sG[q] = s;
      sL[q] = s;
    }
    if (tid == 0) {
      double s = 0.0;
      for (int g = 0; g < n_rgroups; ++g) s += gpart[(int64_t)g * plen + RJ + RR];
      sSumN = s;
    }
  }
  __syncthreads();
  double vf = 0.0;  // <V, F>
  if (mode == 0) {
    if (wv == 0) {
      const bool okc = wave_cholesky(sL, R);
      if (lane == 0) sFlag = okc ? 1 : 0;
      if (!okc) {
        for (int q = lane; q < RR; q += 64) sL[q] = sG[q];
        wave_sync();
        wave_jacobi(sL, sZ, R, sRot, sPair);  // eigenvalues on the diagonal of sL
      }
    }
    __syncthreads();
    double top = 0.0;
    if (!sFlag)
      for (int i = 0; i < R; ++i) top = fmax(top, fabs(sL[i * R + i]));
    for (int j = tid; j < J; j += 256) {
      double f[kMaxR], v[kMaxR];
      for (int r = 0; r < R; ++r) {
        double s = 0.0;
        for (int g = 0; g < n_rgroups; ++g) s += gpart[(int64_t)g * plen + r * J + j];
        f[r] = s;
      }
      if (sFlag) {
        // v = G^{-1} f (G symmetric): L y = f, L^T v = y
        for (int p = 0; p < R; ++p) {
          double s = f[p];
          for (int q = 0; q < p; ++q) s -= sL[p * R + q] * v[q];
          v[p] = s / sL[p * R + p];
        }
        for (int p = R - 1; p >= 0; --p) {
          double s = v[p];
          for (int q = p + 1; q < R; ++q) s -= sL[q * R + p] * v[q];
          v[p] = s / sL[p * R + p];
        }
      } else {
        double tmp[kMaxR];
        for (int i = 0; i < R; ++i) {
          double d = 0.0;
          for (int r = 0; r < R; ++r) d += sZ[r * R + i] * f[r];
          const double li = sL[i * R + i];
          tmp[i] = (top > 0.0 && li > kEigCutoff * top) ? d / li : 0.0;
        }
        for (int r = 0; r < R; ++r) {
          double s = 0.0;
          for (int i = 0; i < R; ++i) s += sZ[r * R + i] * tmp[i];
          v[r] = s;
        }
      }
      for (int r = 0; r < R; ++r) {
        vo.V64[(int64_t)j * R + r] = v[r];
        vf += v[r] * f[r];
        if (!isfinite(v[r])) sBad = 1;
      }
    }
  } else if (mode == 2) {
    for (int j = tid; j < J; j += 256)
      for (int r = 0; r < R; ++r) {
        double s = 0.0;
        for (int g = 0; g < n_rgroups; ++g) s += gpart[(int64_t)g * plen + r * J + j];
        vf += vo.V64[(int64_t)j * R + r] * s;
      }
  }
  vf = wave_sum(vf);
  if (lane == 0) sRed[wv] = vf;
  __syncthreads();
  const double VF = sRed[0] + sRed[1] + sRed[2] + sRed[3];

  if (mode != 2) {
    // V^T V and V^T (float)
    for (int q = tid; q < RR; q += 256) {
      const int r = q / R, s = q - r * R;
      double acc = 0.0;
      for (int j = 0; j < J; ++j) acc += vo.V64[(int64_t)j * R + r] * vo.V64[(int64_t)j * R + s];
      sVtV[q] = acc;
      sL[q] = acc;
      vo.VtV[q] = acc;
    }
    for (int e = tid; e < RJ; e += 256) {
      const int r = e / J, j = e - r * J;
      vo.Vt32[e] = (float)vo.V64[(int64_t)j * R + r];
    }
    __syncthreads();
    // B = (V^T V)^{-1}
    if (wv == 0) {
      const bool okc = wave_cholesky(sL, R);
      if (lane == 0) sFlag = okc ? 1 : 0;
      if (!okc) {
        for (int q = lane; q < RR; q += 64) sL[q] = sVtV[q];
        wave_sync();
        wave_jacobi(sL, sZ, R, sRot, sPair);
      }
    }
    __syncthreads();
    if (sFlag) {
      if (tid < R) {
        double col[kMaxR];
        for (int p = 0; p < R; ++p) {
          double s = (p == tid) ? 1.0 : 0.0;
          for (int q = 0; q < p; ++q) s -= sL[p * R + q] * col[q];
          col[p] = s / sL[p * R + p];
        }
        for (int p = R - 1; p >= 0; --p) {
          double s = col[p];
          for (int q = p + 1; q < R; ++q) s -= sL[q * R + p] * col[q];
          col[p] = s / sL[p * R + p];
        }
        for (int p = 0; p < R; ++p) sB[p * R + tid] = col[p];
      }
    } else {
      double top = 0.0;
      for (int i = 0; i < R; ++i) top = fmax(top, fabs(sL[i * R + i]));
      for (int q = tid; q < RR; q += 256) {
        const int r = q / R, s = q - r * R;
        double acc = 0.0;
        for (int i = 0; i < R; ++i) {
          const double li = sL[i * R + i];
          if (top > 0.0 && li > kEigCutoff * top) acc += sZ[r * R + i] * sZ[s * R + i] / li;
        }
        sB[q] = acc;
      }
    }
    __syncthreads();
    for (int e = tid; e < J * R; e += 256) {
      const int j = e / R, s = e - j * R;
      double acc = 0.0;
      for (int r = 0; r < R; ++r) acc += vo.V64[(int64_t)j * R + r] * sB[r * R + s];
      vo.P32[e] = (float)acc;
    }
  } else {
    for (int q = tid; q < RR; q += 256) sVtV[q] = vo.VtV[q];
    __syncthreads();
  }
  if (mode != 1 && tid == 0) {
    double vg = 0.0;
    for (int q = 0; q < RR; ++q) vg += sVtV[q] * sG[q];
    const double sn = sSumN;
    const double loss = sn - 2.0 * VF + vg;
    const double fit = sn > 0.0 ? 1.0 - sqrt(fmax(0.0, loss)) / sqrt(sn) : 1.0;
    ctl->loss = loss;
    ctl->fit = fit;
    ctl->sum_n = sn;
    ctl->ok = (isfinite(loss) && !sBad) ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// k_commit: make the update's state current if every pass produced finite
// factors and no earlier in-flight update failed; write the pinned report.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_commit(const StepHeader *h, const Touched *touched,
                                                uint8_t *cur, int32_t *tlast, Ctl *ctl) {
  const bool ok = ctl->ok && !ctl->poison;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (ok) {
    for (int t = i; t < h->n_touched; t += gridDim.x * 256) {
      const int k = touched[t].slice;
      cur[k] ^= (uint8_t)1;
      tlast[k] = (int32_t)h->step;
    }
  }
  if (i == 0) {
    Report *rep = (Report *)h->report;
    rep->step = h->step;
    rep->rows = h->M;
    rep->K = h->K;
    rep->committed = ok ? 1 : 0;
    rep->fit = ctl->fit;
    rep->loss = ctl->loss;
    rep->sum_n = ctl->sum_n;
    if (ok)
      ctl->gcur ^= 1;
    else
      ctl->poison = 1;
    __threadfence_system();
    rep->done = 1;
  }
}

// ---------------------------------------------------------------------------
// k_accum_given_u: helper terms of the initial tensor from given U rows
// (eq. [updateC_init]-[updateG_init] in exact form): Y_k = U_k^T X_k,
// D_k = U_k^T U_k, n_k = ||X_k||^2, written to buffer 0.
// ---------------------------------------------------------------------------
template <int RW, int JW>
__global__ __launch_bounds__(256) void k_accum_given_u(int J, int R, const int64_t *row_ptr,
                                                       const float *X, const float *U, float *Y,
                                                       float *D, double *n) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int k = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const PassLds L = pass_lds(J, R);
  float *sX = (float *)(smem + L.oX);
  float *sU = (float *)(smem + L.oU);
  const int XS = L.XS, MB = L.MB;
  float dY[RW][JW];
  float dD[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int rr = 0; rr < RW; ++rr)
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) dY[rr][jj] = 0.f;
  double dn = 0.0;
  const int64_t a0 = row_ptr[k], a1 = row_ptr[k + 1];
  for (int64_t r0 = a0; r0 < a1; r0 += MB) {
    const int m = (int)min((int64_t)MB, a1 - r0);
    __syncthreads();
    for (int e = tid; e < m * J; e += 256) {
      const int row = e / J, col = e - row * J;
      const float x = X[r0 * J + e];
      sX[row * XS + col] = x;
      dn += (double)x * (double)x;
    }
    for (int e = tid; e < m * R; e += 256) {
      const int row = e / R, col = e - row * R;
      sU[row * (R + 1) + col] = U[r0 * R + e];
    }
    __syncthreads();
    accum_block<RW, JW>(sX, sU, XS, m, J, R, dY, dD);
  }
  float *Yk = Y + (int64_t)k * R * J;
#pragma unroll
  for (int rr = 0; rr < RW; ++rr) {
    const int r = wv + 4 * rr;
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
      const int j = lane + 64 * jj;
      if (r < R && j < J) Yk[r * J + j] = dY[rr][jj];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = tid + 256 * i;
    if (q < R * R) D[(int64_t)k * R * R + q] = dD[i];
  }
  // block reduction of dn (fixed order)
  __shared__ double red[kWaves];
  dn = wave_sum(dn);
  if (lane == 0) red[wv] = dn;
  __syncthreads();
  if (tid == 0) n[k] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// small conversion kernels
// ---------------------------------------------------------------------------
__global__ void k_v_from_f32(int JR, const float *V, double *V64) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e < JR) V64[e] = (double)V[e];
}

__global__ void k_f32_to_f64(int64_t count, const float *src, double *dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) dst[e] = (double)src[e];
}

__global__ void k_f64_to_f32(int64_t count, const double *src, float *dst) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < count) dst[e] = (float)src[e];
}

__global__ void k_export_state(int J, int R, int K, int64_t step, double lambda, const float *Y,
                               const float *D, const double *n, const uint8_t *cur,
                               const int32_t *tlast, int64_t K_cap, double *Yo, double *Do,
                               double *no) {
  const int k = blockIdx.x;
  if (k >= K) return;
  const int b = cur[k];
  const double s = pow(lambda, (double)(step - tlast[k]));
  const int64_t RJ = (int64_t)R * J, RR = (int64_t)R * R;
  for (int e = threadIdx.x; e < RJ; e += 256)
    Yo[k * RJ + e] = s * (double)Y[((int64_t)b * K_cap + k) * RJ + e];
  for (int e = threadIdx.x; e < RR; e += 256)
    Do[k * RR + e] = s * (double)D[((int64_t)b * K_cap + k) * RR + e];
  if (threadIdx.x == 0) no[k] = s * n[(int64_t)b * K_cap + k];
}

// Raw committed state (no decay applied) of slices [0, K), for checkpoints.
__global__ void k_gather_state(int J, int R, int K, const float *Y, const float *D, const double *n,
                               const uint8_t *cur, int64_t K_cap, float *Yo, float *Do, double *no) {
  const int k = blockIdx.x;
  if (k >= K) return;
  const int b = cur[k];
  const int64_t RJ = (int64_t)R * J, RR = (int64_t)R * R;
  for (int e = threadIdx.x; e < RJ; e += 256) Yo[k * RJ + e] = Y[((int64_t)b * K_cap + k) * RJ + e];
  for (int e = threadIdx.x; e < RR; e += 256) Do[k * RR + e] = D[((int64_t)b * K_cap + k) * RR + e];
  if (threadIdx.x == 0) no[k] = n[(int64_t)b * K_cap + k];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int rw_of(int R) { return (R + 3) / 4; }
static inline int jw_of(int J) { return (J + 63) / 64; }

// Kernels whose dynamic LDS exceeds 64 KB must opt in once.
template <typename F>
static int allow_lds(F *fn, size_t bytes) {
  if (bytes <= 65536) return 0;
  return (int)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

template <int RW, int JW>
static int launch_pass_t(const PassArgs &a, int n_chunks, hipStream_t s) {
  const PassLds L = pass_lds(a.J, a.R);
  if (int e = allow_lds(k_pass<RW, JW>, L.bytes)) return e;
  hipLaunchKernelGGL((k_pass<RW, JW>), dim3(n_chunks), dim3(256), L.bytes, s, a);
  return (int)hipGetLastError();
}

template <int RW, int JW>
static int launch_accum_t(int J, int R, int K, const int64_t *rp, const float *X, const float *U,
                          float *Y, float *D, double *n, hipStream_t s) {
  const PassLds L = pass_lds(J, R);
  if (int e = allow_lds(k_accum_given_u<RW, JW>, L.bytes)) return e;
  hipLaunchKernelGGL((k_accum_given_u<RW, JW>), dim3(K), dim3(256), L.bytes, s, J, R, rp, X, U, Y, D, n);
  return (int)hipGetLastError();
}

int launch_pass(const PassArgs &a, int n_chunks, hipStream_t s) {
  if (n_chunks <= 0) return 0;
  switch (rw_of(a.R) * 8 + jw_of(a.J)) {
#define C(RW, JW) case RW * 8 + JW: return launch_pass_t<RW, JW>(a, n_chunks, s);
    C(1, 1) C(1, 2) C(1, 3) C(1, 4) C(2, 1) C(2, 2) C(2, 3) C(2, 4)
    C(3, 1) C(3, 2) C(3, 3) C(3, 4) C(4, 1) C(4, 2) C(4, 3) C(4, 4)
    C(5, 1) C(5, 2) C(5, 3) C(5, 4) C(6, 1) C(6, 2) C(6, 3) C(6, 4)
    C(7, 1) C(7, 2) C(7, 3) C(7, 4) C(8, 1) C(8, 2) C(8, 3) C(8, 4)
#undef C
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_accum_given_u(int J, int R, int K, const int64_t *rp, const float *X, const float *U,
                         float *Y, float *D, double *n, hipStream_t s) {
  if (K <= 0) return 0;
  switch (rw_of(R) * 8 + jw_of(J)) {
#define C(RW, JW) case RW * 8 + JW: return launch_accum_t<RW, JW>(J, R, K, rp, X, U, Y, D, n, s);
    C(1, 1) C(1, 2) C(1, 3) C(1, 4) C(2, 1) C(2, 2) C(2, 3) C(2, 4)
    C(3, 1) C(3, 2) C(3, 3) C(3, 4) C(4, 1) C(4, 2) C(4, 3) C(4, 4)
    C(5, 1) C(5, 2) C(5, 3) C(5, 4) C(6, 1) C(6, 2) C(6, 3) C(6, 4)
    C(7, 1) C(7, 2) C(7, 3) C(7, 4) C(8, 1) C(8, 2) C(8, 3) C(8, 4)
#undef C
    default: return (int)hipErrorInvalidValue;
  }
}

int launch_reduce(const double *partials, double *gpart, const StepHeader *hdr, int plen,
                  int n_chunks, int n_rgroups, int chunks_per_rgroup, hipStream_t s) {
  (void)n_chunks;
  (void)chunks_per_rgroup;
  dim3 grid((plen + 255) / 256, n_rgroups);
  hipLaunchKernelGGL(k_reduce, grid, dim3(256), 0, s, partials, gpart, hdr, plen);
  return (int)hipGetLastError();
}

int launch_solve(int J, int R, const double *gpart, int n_rgroups, char *vb, int64_t vb_stride,
                 Ctl *ctl, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_solve, dim3(1), dim3(256), 0, s, J, R, gpart, n_rgroups, vb, vb_stride, ctl, mode);
  return (int)hipGetLastError();
}

int launch_commit(const StepHeader *hdr, const Touched *touched, uint8_t *cur, int32_t *tlast,
                  Ctl *ctl, int n_touched, hipStream_t s) {
  int blocks = (n_touched + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_commit, dim3(blocks), dim3(256), 0, s, hdr, touched, cur, tlast, ctl);
  return (int)hipGetLastError();
}

int launch_v_from_f32(int J, int R, const float *V, char *vb_committed, hipStream_t s) {
  const VBundleView v = vb_view(vb_committed, J, R);
  hipLaunchKernelGGL(k_v_from_f32, dim3((J * R + 255) / 256), dim3(256), 0, s, J * R, V, v.V64);
  return (int)hipGetLastError();
}

int launch_w_from_f32(int R, int K, const float *W, double *Wc, hipStream_t s) {
  const int64_t cnt = (int64_t)R * K;
  if (cnt == 0) return 0;
  hipLaunchKernelGGL(k_f32_to_f64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, cnt, W, Wc);
  return (int)hipGetLastError();
}

int launch_to_f32(const double *src, float *dst, int64_t count, hipStream_t s) {
  if (count == 0) return 0;
  hipLaunchKernelGGL(k_f64_to_f32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, src, dst);
  return (int)hipGetLastError();
}

int launch_export_state(int J, int R, int K, int64_t step, double lambda, const float *Y,
                        const float *D, const double *n, const uint8_t *cur, const int32_t *tlast,
                        int64_t K_cap, double *Yo, double *Do, double *no, hipStream_t s) {
  if (K <= 0) return 0;
  hipLaunchKernelGGL(k_export_state, dim3(K), dim3(256), 0, s, J, R, K, step, lambda, Y, D, n, cur,
                     tlast, K_cap, Yo, Do, no);
  return (int)hipGetLastError();
}

int launch_gather_state(int J, int R, int K, const float *Y, const float *D, const double *n,
                        const uint8_t *cur, int64_t K_cap, float *Yo, float *Do, double *no,
                        hipStream_t s) {
  if (K <= 0) return 0;
  hipLaunchKernelGGL(k_gather_state, dim3(K), dim3(256), 0, s, J, R, K, Y, D, n, cur, K_cap, Yo, Do, no);
  return (int)hipGetLastError();
}

}  // namespace dash
