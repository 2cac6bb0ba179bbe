// gfx950 kernels of the streaming PARAFAC2 update (DASH): the final phase of a
// pass and the fused one-wave-per-slice sweep.
//
// Fused sweep: one launch per ALS pass.  Every workgroup sweeps a chunk of
// slices (Lemma 1 on their new rows, the forgetting-factor fold, Lemma 2) and
// writes an F/G/n partial; the last workgroup to arrive reduces the partials in
// a fixed order, solves Lemma 3 and prepares the next pass's V operands, and
// on the last pass commits the update.  The split sweep (dash_split.hip) runs
// the same pass as four launches.  See dash_dev.h for layouts.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "dash_dev.h"
#include "dash_math.h"
#include "dash_tiles.h"

namespace dash {

// ---------------------------------------------------------------------------
// Final phase of a pass: one workgroup of 512 threads.
//   mode 0: F, G, n from the group partials; Lemma 3: V = F G^{-1} into the
//           spare bundle with V^T V, B = (V^T V)^{-1}, P = V B, V^T; loss and
//           fit; on the last pass the commit (switch of touched slices and of
//           the W / V buffers) and the pinned report.
//   mode 1: build the committed bundle from its V64 (no reduction, no fit).
//   mode 2: loss and fit of the committed V with F, G from the partials.
// The R x R inverses come from block_spd_inverse (FP64); when a pivot fails
// the acceptance rule the eigen pseudo-inverse replaces it, as in the oracle.
// ---------------------------------------------------------------------------
constexpr int kFinishThreads = 512;   // 2 waves per SIMD: up to 256 VGPRs for the R x R eliminations
constexpr int kFinishRed = 48;        // doubles of the reduction scratch
constexpr int kFinishScr = 1024;      // doubles of the split-product scratch (>= R^2)

// F^T (R rows of stride J | 1), G, G^{-1}, (V^T V)^{-1}, V^T V, the
// pseudo-inverse scratch, reductions and flags
__host__ __device__ inline size_t finish_lds_bytes(int J, int R) {
  return (size_t)(R * (J | 1) + 5 * R * R + 64 + kFinishRed + kFinishScr) * 8 + 68 * 4;
}


template <int RM>
__device__ void finish_pass(const PassArgs &a, const StepHeader *h, int n_rgroups, int mode,
                            unsigned char *smem, size_t lds_avail) {
  (void)lds_avail;
  const int nt = blockDim.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, nwv = nt >> 6;
  const int J = a.J, R = a.R, RR = R * R, RJ = R * J;
  const int JS = J | 1;            // row stride of F^T and V^T: a column's rows in different banks
  const int plen = partial_len(J, R);
  // F^T (R x J); V^T replaces it in place once V is formed, and every later
  // product reads V from there
  double *sF = (double *)smem;
  double *sG = sF + R * JS;
  double *sGi = sG + RR;         // G^{-1}
  double *sB = sGi + RR;         // (V^T V)^{-1}
  double *sVtV = sB + RR;
  double *sZ = sVtV + RR;        // pseudo-inverse scratch (and sW below)
  double *sRot = sZ + RR;        // 64
  double *sRed = sRot + 64;      // kFinishRed
  double *sScr = sRed + kFinishRed;   // kFinishScr: split products
  int *sPair = (int *)(sScr + kFinishScr);
  int *sFlag = sPair + 64;       // [0], [2]: inverse ok, [1]: non-finite seen
  const int gcur = a.ctl->gcur;
  const int out = (mode == 0) ? 1 - gcur : gcur;
  const VBundleView vo = vb_view(a.vb + (int64_t)out * a.vb_stride, J, R);
  if (tid == 0) {
    sFlag[0] = 1;
    sFlag[1] = 0;
    sFlag[2] = 1;
  }
  double sum_n = 0.0;
  if (mode != 1) {
    for (int e = tid; e < plen; e += nt) {
      const double s = ordered_sum(a.gpart, plen, e, 0, n_rgroups);
      if (e < RJ) sF[(e / J) * JS + e % J] = s;
      else if (e < RJ + RR) sG[e - RJ] = s;
      else sRed[kFinishRed - 1] = s;
    }
  }
  __syncthreads();
  if (mode != 1) sum_n = sRed[kFinishRed - 1];
  if (mode == 0 && a.lagged) {
    // Algorithm 1's recursions (eq. [obtain_FandF], [obtain_FandG]): the old
    // terms are the committed F, G scaled by lambda; the partials hold the
    // new rows' terms
    const double *fg = a.FG + (int64_t)gcur * (RJ + RR);
    for (int e = tid; e < RJ + RR; e += nt) {
      double *d = e < RJ ? sF + (e / J) * JS + e % J : sG + (e - RJ);
      *d = fma(a.lambda, fg[e], *d);
    }
    __syncthreads();
  }
  if (a.lagged && mode != 1) {
    // the lagged F, G of this pass (committed with it), or, evaluating the
    // initial state, the exact ones the recursions start from
    double *fg = a.FG + (int64_t)(mode == 0 ? 1 - gcur : gcur) * (RJ + RR);
    for (int e = tid; e < RJ + RR; e += nt) fg[e] = e < RJ ? sF[(e / J) * JS + e % J] : sG[e - RJ];
  }
  double vf = 0.0;
  if (mode == 0) {
    // Lemma 3: V = F G^{-1}, formed as V^T[:, j] = G^{-T} F^T[:, j] by one
    // thread per column j, in place (the column is read into registers first)
    if (!block_spd_inverse<RM>(sG, sGi, R) && lane == 0) sFlag[0] = 0;
    __syncthreads();
    if (!sFlag[0]) block_pinv_of(sG, sGi, sB, sZ, R, sRot, sPair);
    bool bad = false;
    for (int j = tid; j < J; j += nt) {
      double f[RM];
#pragma unroll
      for (int c = 0; c < RM; ++c) f[c] = (c < R) ? sF[c * JS + j] : 0.0;
      for (int r = 0; r < R; ++r) {
        double x = 0.0;
#pragma unroll
        for (int c = 0; c < RM; ++c)
          if (c < R) x = fma(f[c], sGi[c * R + r], x);
        const double fr = sF[r * JS + j];   // F^T[r][j], not yet replaced
        vf = fma(x, fr, vf);
        bad |= !isfinite(x);
        sF[r * JS + j] = x;
        vo.V64[(size_t)j * R + r] = x;
      }
    }
    if (bad) sFlag[1] = 1;
  } else {
    for (int e = tid; e < J * R; e += nt) {
      const int j = e / R, r = e - j * R;
      const double x = vo.V64[e];
      if (mode == 2) vf = fma(x, sF[r * JS + j], vf);
      sF[r * JS + j] = x;
    }
  }
  __syncthreads();

  if (mode != 2) {
    // next pass operands: V^T V, B = (V^T V)^{-1}, P = V B, V^T in float32.
    // V^T V by 2 x 2 blocks on and above the diagonal (each entry one FMA
    // chain over j in order; the mirror entry is the same chain)
    const int RH = (R + 1) >> 1;
    for (int t = tid; t < RH * RH; t += nt) {
      const int rb = t / RH, cb = t - rb * RH;
      if (cb < rb) continue;
      const int r0 = 2 * rb, c0 = 2 * cb, r1 = min(r0 + 1, R - 1), c1 = min(c0 + 1, R - 1);
      const double *v0 = sF + r0 * JS, *v1 = sF + r1 * JS, *w0 = sF + c0 * JS, *w1 = sF + c1 * JS;
      double a00 = 0.0, a01 = 0.0, a10 = 0.0, a11 = 0.0;
#pragma unroll 4
      for (int j = 0; j < J; ++j) {
        const double x0 = v0[j], x1 = v1[j], y0 = w0[j], y1 = w1[j];
        a00 = fma(x0, y0, a00);
        a01 = fma(x0, y1, a01);
        a10 = fma(x1, y0, a10);
        a11 = fma(x1, y1, a11);
      }
      const double acc[2][2] = {{a00, a01}, {a10, a11}};
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int r = r0 + i, c = c0 + k;
          if (r < R && c < R) {
            sVtV[r * R + c] = acc[i][k];
            sVtV[c * R + r] = acc[i][k];
            vo.VtV[r * R + c] = acc[i][k];
            vo.VtV[c * R + r] = acc[i][k];
          }
        }
    }
    for (int e = tid; e < RJ; e += nt) {
      const int r = e / J, j = e - r * J;
      vo.Vt32[e] = (float)sF[r * JS + j];
    }
    __syncthreads();
    if (!block_spd_inverse<RM>(sVtV, sB, R, vo.piv) && lane == 0) sFlag[2] = 0;
    __syncthreads();
    if (!sFlag[2]) {
      // no pivots: every slice's Lemma 1 system takes the pseudo-inverse form
      if (tid < R) vo.piv[tid] = 0.0;
      block_pinv_of(sVtV, sB, sGi, sZ, R, sRot, sPair);
    }
    // P = V B, four columns per thread
    const int CB = (R + 3) >> 2;
    for (int e = tid; e < J * CB; e += nt) {
      const int j = e / CB, c0 = 4 * (e - j * CB);
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for (int r = 0; r < R; ++r) {
        const double v = sF[r * JS + j];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] = fma(v, sB[r * R + min(c0 + i, R - 1)], acc[i]);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (c0 + i < R) vo.P32[(size_t)j * R + c0 + i] = (float)acc[i];
    }
  } else {
    for (int q = tid; q < RR; q += nt) sVtV[q] = vo.VtV[q];
    __syncthreads();
  }
  if (mode == 1) return;
  // loss = sum n - 2 <V, F> + <V^T V, G>
  double vg = 0.0;
  for (int q = tid; q < RR; q += nt) vg = fma(sVtV[q], sG[q], vg);
  vf = wave_sum(vf);
  vg = wave_sum(vg);
  if (lane == 0) {
    sRed[wv] = vf;
    sRed[16 + wv] = vg;
  }
  __syncthreads();
  double VF = 0.0, VG = 0.0;
  for (int w = 0; w < nwv; ++w) {
    VF += sRed[w];
    VG += sRed[16 + w];
  }
  const double loss = sum_n - 2.0 * VF + VG;
  const double fit = sum_n > 0.0 ? 1.0 - sqrt(fmax(0.0, loss)) / sqrt(sum_n) : 1.0;
  // (an injected failure takes the same path as non-finite factors)
  const bool ok = isfinite(loss) && !sFlag[1] && !(mode == 0 && h->force_fail);
  if (tid == 0) {
    a.ctl->loss = loss;
    a.ctl->fit = fit;
    a.ctl->sum_n = sum_n;
  }
  if (mode != 0) return;
  // every pass of an update must be finite for it to commit
  if (tid == 0 && !ok) a.ctl->ok = 0;
  if (!a.last_pass) return;
  __syncthreads();
  // the sweep wrote the next state beside the committed one (Y, D, n per slice,
  // the slice bookkeeping, W, the V bundle): committing switches buffers
  const bool commit = ok && a.ctl->ok && !a.ctl->poison;
  if (tid == 0) {
    Report *rep = (Report *)h->report;
    rep->t_end = __builtin_amdgcn_s_memrealtime();
    rep->step = h->step;
    rep->rows = h->M;
    rep->K = h->K;
    rep->committed = commit ? 1 : 0;
    rep->fit = fit;
    rep->loss = loss;
    rep->sum_n = sum_n;
    if (commit)
      a.ctl->gcur = 1 - gcur;
    else
      a.ctl->poison = 1;
    a.ctl->ok = 1;  // reset for the next update
    // the host polls `done`: every other field must be visible before it
    // (with anomaly scores on, their kernel sets it after this launch)
    if (!a.defer_done) {
      __threadfence_system();
      rep->done = 1;
    }
  }
}

// R bucket of the final phase's register eliminations
template <int RQ>
struct FinishBucket {
  static constexpr int value = RQ <= 8 ? 8 : RQ <= 12 ? 12 : RQ <= 16 ? 16 : RQ <= 24 ? 24 : 32;
};

// Final phase of a pass as its own single-workgroup launch (modes as finish_pass).
__host__ __device__ inline size_t finish_launch_lds(int J, int R) { return finish_lds_bytes(J, R); }

template <int RM>
__global__ __launch_bounds__(kFinishThreads) void k_finish(PassArgs a, int mode) {
  extern __shared__ __align__(16) unsigned char smem[];
  const StepHeader *h = a.hdr;
  finish_pass<RM>(a, h, mode == 1 ? 0 : h->n_rgroups, mode, smem, finish_launch_lds(a.J, a.R));
}

// The same with its arguments in device memory (one workgroup per context).
template <int RM>
__global__ __launch_bounds__(kFinishThreads) void k_finish_dev(const PassArgs *args, const BlockMap *map, int mode) {
  extern __shared__ __align__(16) unsigned char smem[];
  const PassArgs a = map ? *map[blockIdx.x].args : *args;
  const StepHeader *h = a.hdr;
  const int ng = mode == 1 ? 0 : (a.pre_reduced ? 1 : h->n_rgroups);
  finish_pass<RM>(a, h, ng, mode, smem, finish_launch_lds(a.J, a.R));
}

// ---------------------------------------------------------------------------
// Sweep variant 1: one wave per slice ("wave" variant, R*J <= 2048, J <= 128).
// 8 waves per workgroup; wave w handles slices k0+w, k0+w+8, ... of the chunk.
// A slice's R x J state is spread flat over the wave: lane l holds elements
// e = l + 64 i (i < EPT) of the contiguous row-major Y_k, so every load and
// store of Y_k is one coalesced access with a single base address.
// Per slice, within the wave only (no block barriers):
//   new rows (16-row blocks staged in the wave's LDS):
//     u = (x P) * (1/w_k)  (Lemma 1; 4 lanes per row, R/4 outputs per lane)
//     dY += u^T x, dD += u^T u, dn += ||x||^2
//   fold:    Y_k = lambda^dt Y_k,stored + dY  (touched), else the stored Y_k
//   Lemma 2: c = diag(Y_k V) (products transposed through LDS, FP64 row sums);
//            (V^T V * D_k) w = c by FP64 Cholesky (pseudo-inverse fallback)
//   sweep:   F^T += sigma w_k Y_k, G += sigma w_k w_k^T * D_k, sum n
// Untouched slices solve on their stored (undecayed) Y_k, D_k -- w_k does not
// depend on the common factor lambda^dt -- and enter F, G with sigma = lambda^dt.
// ---------------------------------------------------------------------------
constexpr int kWaveRows = 16;   // rows per staged block

struct WaveLds {
  int XS;
  size_t oP, oVt, oVtV, oWave, wave_bytes, oSmall, oX, oU, oM, oZ, oRot, oTmp, oPair, oProd, oDcur, bytes;
};

// padded rank of the wave variant's register tiles (R <= 16)
__host__ __device__ inline int wave_rc(int R) { return R <= 8 ? 8 : (R <= 11 ? 12 : 16); }

// bytes of one wave's slot in the end-of-chunk combine: F^T (float, padded)
// then G and n (double)
__host__ __device__ inline size_t wave_slot_bytes(int J, int R) {
  return align_up(align_up((size_t)y_stride(J, R) * 4, 16) + (size_t)(R * R + 1) * 8, 16);
}

__host__ __device__ inline WaveLds wave_lds(int J, int R) {
  WaveLds L;
  const int RC = wave_rc(R);
  L.XS = J | 1;
  size_t o = 0;
  L.oP = o;   o += (size_t)J * RC * 4;   // P = V (V^T V)^{-1}, J x RC, zero-padded columns
  L.oVt = o;  o += (size_t)y_stride(J, R) * 4;
  o = align_up(o, 8);
  L.oVtV = o; o += (size_t)R * R * 8;
  o = align_up(o, 16);
  L.oWave = o;
  // per-wave region: small vectors, then a union of the row block, the
  // products of diag(Y_k V), and the solve scratch
  size_t w = 0;
  // sW, sC, sC2 (f64, R+1), sWinv (f32, RC), sZf (f32, RC x RC: Lemma 1's pseudo-inverse form)
  L.oSmall = w; w += (size_t)(R + 1) * 8 * 3 + (size_t)RC * 4 + (size_t)RC * RC * 4;
  w = align_up(w, 16);
  const size_t blk = w;
  L.oX = blk;
  L.oU = blk + (size_t)kWaveRows * L.XS * 4;
  const size_t rows_end = L.oU + (size_t)kWaveRows * RC * 4;
  L.oProd = blk;
  const size_t prod_end = blk + (size_t)y_stride(J, R) * 4;
  L.oDcur = blk;
  L.oM = blk + align_up((size_t)R * R * 4, 16);
  L.oZ = L.oM + (size_t)R * (R + 1) * 8;
  L.oRot = L.oZ + (size_t)R * R * 8;
  L.oTmp = L.oRot + 64 * 8;
  L.oPair = L.oTmp + 64 * 8;
  size_t end = L.oPair + 64 * 4;
  if (rows_end > end) end = rows_end;
  if (prod_end > end) end = prod_end;
  L.wave_bytes = align_up(end, 16);
  o += L.wave_bytes * kWaveWarps;
  const size_t comb = wave_slot_bytes(J, R) * kWaveWarps;
  L.bytes = align_up(o > comb ? o : comb, 16);
  return L;
}

template <int EPT, int DQ>
__global__ __launch_bounds__(512) void k_pass_wave(PassArgs a) {
  constexpr int RC = DQ == 1 ? 8 : DQ == 2 ? 12 : 16;  // == wave_rc(R): R <= RC
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sflag;
  const StepHeader *h = a.hdr;
  const int chunk = blockIdx.x;
  if (chunk >= h->n_chunks) return;
  if (a.stamp_start && chunk == 0 && threadIdx.x == 0 && a.pass == 0 && a.mode == 0 && h->report)
    ((Report *)h->report)->t_start = __builtin_amdgcn_s_memrealtime();
  const int J = a.J, R = a.R, RR = R * R, RJ = R * J, YS = a.ys;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int K = h->K, Kp = h->K_prev;
  const int64_t step = h->step;
  const int gcur = a.ctl->gcur;
  const int win = (a.pass == 0) ? gcur : 1 - gcur;
  const int wout = 1 - gcur;
  const VBundleView vb = vb_view(a.vb + (int64_t)win * a.vb_stride, J, R);
  const WaveLds L = wave_lds(J, R);
  float *sP = (float *)(smem + L.oP);
  float *sVt = (float *)(smem + L.oVt);
  double *sVtV = (double *)(smem + L.oVtV);
  unsigned char *wbase = smem + L.oWave + (size_t)wv * L.wave_bytes;
  double *sW = (double *)(wbase + L.oSmall);
  double *sC = sW + (R + 1);
  double *sC2 = sC + (R + 1);
  float *sWinv = (float *)(sC2 + (R + 1));
  float *sZf = sWinv + RC;
  float *sX = (float *)(wbase + L.oX);
  float *sU = (float *)(wbase + L.oU);
  float *sProd = (float *)(wbase + L.oProd);
  double *sM = (double *)(wbase + L.oM);
  double *sZ = (double *)(wbase + L.oZ);
  double *sRot = (double *)(wbase + L.oRot);
  double *sTmp = (double *)(wbase + L.oTmp);
  int *sPair = (int *)(wbase + L.oPair);
  const int XS = L.XS;
  const float invJ = 1.0f / (float)J;   // e / J below is exact: e < 2^11, J <= 128
  constexpr int NB = kWaveRows * 2;     // staged floats per lane for a 16 x 128 row block

  for (int e = tid; e < J * RC; e += 512) {
    const int j = e / RC, r = e - j * RC;
    sP[e] = (r < R) ? vb.P32[j * R + r] : 0.f;
  }
  for (int e = tid; e < YS; e += 512) sVt[e] = (e < RJ) ? vb.Vt32[e] : 0.f;
  for (int e = tid; e < RR; e += 512) sVtV[e] = vb.VtV[e];
  __syncthreads();

  float facc[EPT];   // this wave's F^T partial (one slice per wave up to 4096 slices)
  double gacc[DQ];
  double nacc = 0.0;
#pragma unroll
  for (int i = 0; i < EPT; ++i) facc[i] = 0.f;
#pragma unroll
  for (int i = 0; i < DQ; ++i) gacc[i] = 0.0;

  const int k0 = chunk * h->chunk;
  const int k1 = min(K, k0 + h->chunk);
  const int g0 = a.chunk_gptr[chunk], g1 = a.chunk_gptr[chunk + 1];
  // pivots and diagonal of V^T V for Lemma 1's acceptance rule (lane r)
  const double pivl = lane < R ? vb.piv[lane] : 0.0;
  const double arrl = lane < R ? vb.VtV[lane * R + lane] : 0.0;

  for (int k = k0 + wv; k < k1; k += kWaveWarps) {
    const bool is_new = k >= Kp;
    // issue every load of the slice's state first so their latencies overlap;
    // slice-level values are wave-uniform
    const int b = __builtin_amdgcn_readfirstlane((int)a.cur[(int64_t)gcur * a.K_cap + k]);
    const int tl = __builtin_amdgcn_readfirstlane(a.tlast[(int64_t)gcur * a.K_cap + k]);
    double w = 0.0;
    if (lane < R) w = (is_new && a.pass == 0) ? 1.0 : a.W[((int64_t)win * a.K_cap + k) * R + lane];
    const float *Yst = a.Y + ((int64_t)b * a.K_cap + k) * YS;
    const float *Dst = a.D + ((int64_t)b * a.K_cap + k) * RR;
    float dold[DQ];
#pragma unroll
    for (int i = 0; i < DQ; ++i) {
      const int q = lane + 64 * i;
      dold[i] = (q < RR && !is_new) ? Dst[q] : 0.f;
    }
    const double nold = (lane == 0 && !is_new) ? a.n[(int64_t)b * a.K_cap + k] : 0.0;
    float yo[EPT];   // stored Y_k, in flight while the rows are processed
#pragma unroll
    for (int i = 0; i < EPT; ++i) yo[i] = (64 * i < YS && !is_new) ? Yst[lane + 64 * i] : 0.f;
    // groups of slice k: contiguous run inside [g0, g1)
    int gb = -1, ge = -1;
    for (int base = g0; base < g1; base += 64) {
      const int g = base + lane;
      const int sl = (g < g1) ? a.groups[g].slice : -1;
      const unsigned long long m = __ballot(sl == k);
      if (m) {
        const int first = base + __ffsll((long long)m) - 1;
        const int last = base + 63 - __clzll((long long)m);
        if (gb < 0) gb = first;
        ge = last + 1;
      } else if (gb >= 0) {
        break;
      }
    }
    const bool touched = gb >= 0;
    // Lemma 1's system S_k V^T V S_k: the division by w when it passes the
    // acceptance rule, else its pseudo-inverse form u = t Z
    const bool regular = lemma1_regular(w, pivl, arrl, R);
    {
      if (lane < R) sW[lane] = w;
      if (lane < RC) sWinv[lane] = (lane < R && regular) ? (float)(1.0 / w) : 0.f;
      if (lane == 0) sC[R] = 0.0;   // weight of the padding elements of Y_k
    }
    wave_sync();
    const bool slow = !regular && touched && a.mode == 0;
    if (slow) lemma1_pinv_matrix(sVtV, sW, R, sM, sZ, sTmp, sRot, sPair, sZf, RC);

    float dD[DQ];
    double dn = 0.0;
#pragma unroll
    for (int i = 0; i < DQ; ++i) dD[i] = 0.f;
    // dY = U_new^T X_new as MFMA tiles (16 ranks x 16 columns each): lane
    // holds dY[4 (lane / 16) + i][16 t + lane % 16] in accY[t]
    f32x4 accY[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) accY[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int NT = (J + 15) >> 4;
    const int li = lane & 15, lq = lane >> 4;

    if (touched && a.mode == 0) {
      for (int g = gb; g < ge; ++g) {
        const Group *gp = a.groups + g;
        const int nrows = __builtin_amdgcn_readfirstlane(gp->nrows);
        const int64_t out_row = ((int64_t)__builtin_amdgcn_readfirstlane((int)(gp->out_row >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)gp->out_row);
        const uint64_t srcbits = (uint64_t)gp->src;
        const float *gsrc = (const float *)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(srcbits >> 32)) << 32) |
                                            (uint32_t)__builtin_amdgcn_readfirstlane((int)srcbits));
        for (int r0 = 0; r0 < nrows; r0 += kWaveRows) {
          const int m = min(kWaveRows, nrows - r0);
          const int tot = m * J;
          const float *src = gsrc + (int64_t)r0 * J;
          wave_sync();  // the previous block's readers are done
          // stage the block (m x J) in LDS; the loads are clamped in bounds and
          // only the stores are predicated, so every batch is one round trip
          for (int i0 = 0; i0 < NB; i0 += 8) {
            if (64 * i0 >= tot) break;
            float buf[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const int e = lane + 64 * (i0 + i);
              const float v = src[min(e, tot - 1)];
              buf[i] = (e < tot) ? v : 0.f;
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
              const int e = lane + 64 * (i0 + i);
              const int row = (int)(((float)e + 0.5f) * invJ);
              dn = fma((double)buf[i], (double)buf[i], dn);
              if (e < tot) sX[row * XS + (e - row * J)] = buf[i];
            }
          }
          // zero rows m .. m rounded up to 4: the accumulation MFMAs take
          // four rows at a time
          for (int e = tot + lane; e < (((m + 3) & ~3) * J); e += 64) {
            const int row = (int)(((float)e + 0.5f) * invJ);
            sX[row * XS + (e - row * J)] = 0.f;
          }
          wave_sync();
          {
            // Lemma 1 on MFMA: the 16 x RC tile U = (X P) * (1/w); u is set
            // to 0 on rows >= m of the block, whatever stale X holds there
            const float *xr = sX + li * XS;
            const int n = min(li, RC - 1);
            f32x4 t0 = {0.f, 0.f, 0.f, 0.f}, t1 = {0.f, 0.f, 0.f, 0.f};
            int ks = 0;
            for (; ks + 8 <= J; ks += 8) {
              t0 = mfma_f32(xr[ks + lq], sP[(ks + lq) * RC + n], t0);
              t1 = mfma_f32(xr[ks + 4 + lq], sP[(ks + 4 + lq) * RC + n], t1);
            }
            for (; ks < J; ks += 4) {
              const int kk = ks + lq;
              t0 = mfma_f32(kk < J ? xr[kk] : 0.f, kk < J ? sP[kk * RC + n] : 0.f, t0);
            }
            const f32x4 t = t0 + t1;
            if (slow) {
              // u = t Z: the tile goes through LDS so every lane sees whole rows
              if (li < RC) {
#pragma unroll
                for (int i = 0; i < 4; ++i) sU[(4 * lq + i) * RC + li] = (li < R) ? t[i] : 0.f;
              }
              wave_sync();
              float uq[4];
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int row = 4 * lq + i;
                float acc = 0.f;
                if (li < R)
                  for (int mm = 0; mm < R; ++mm) acc = fmaf(sU[row * RC + mm], sZf[mm * RC + li], acc);
                uq[i] = (row < m && li < R) ? acc : 0.f;
              }
              wave_sync();
              if (li < RC) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  const int row = 4 * lq + i;
                  sU[row * RC + li] = uq[i];
                  if (a.last_pass && row < m && li < R) a.U_out[(out_row + r0 + row) * R + li] = uq[i];
                }
              }
            } else if (li < RC) {
              const float wi = sWinv[li];
#pragma unroll
              for (int i = 0; i < 4; ++i) {
                const int row = 4 * lq + i;
                const float u = (row < m) ? t[i] * wi : 0.f;
                sU[row * RC + li] = u;
                if (a.last_pass && row < m && li < R) a.U_out[(out_row + r0 + row) * R + li] = u;
              }
            }
          }
          wave_sync();
          // dY += U^T X on MFMA over the block's rows in steps of 4 (u = 0
          // on rows >= m); dD += u^T u (lane = entry), padded ranks are zero
          {
            const int rn = min(li, RC - 1);
            const int mp = (m + 3) & ~3;
            for (int ks = 0; ks < mp; ks += 4) {
              const float au = (li < RC) ? sU[(ks + lq) * RC + rn] : 0.f;
              const float *xrow = sX + (ks + lq) * XS;
#pragma unroll
              for (int t = 0; t < 8; ++t)
                if (t < NT) accY[t] = mfma_f32(au, xrow[min(16 * t + li, J - 1)], accY[t]);
            }
          }
#pragma unroll
          for (int i = 0; i < DQ; ++i) {
            const int q = min(lane + 64 * i, RR - 1);
            const int r = q / R, s = q - r * R;
            float acc = dD[i];
#pragma unroll 4
            for (int row = 0; row < m; ++row) acc = fmaf(sU[row * RC + r], sU[row * RC + s], acc);
            dD[i] = acc;
          }
        }
      }
      dn = wave_sum(dn);
    }
    // hand dY to the flat layout through LDS (zero on the padding)
    wave_sync();
    float *sDY = sProd;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int j = 16 * t + li;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 4 * lq + i;
        if (t < NT && r < R && j < J) sDY[r * J + j] = accY[t][i];
      }
    }
    if (RJ + lane < YS) sDY[RJ + lane] = 0.f;
    wave_sync();

    const double s_old = is_new ? 0.0 : exp2((double)(step - tl) * a.log2_lambda);
    const float s_old_f = (float)s_old;
    wave_sync();  // the row block is dead: the product buffer may overwrite it
    float yc[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      yc[i] = 0.f;
      if (64 * i >= YS) continue;   // uniform: the slice has YS / 64 flat blocks
      const int e = lane + 64 * i;
      yc[i] = touched ? fmaf(s_old_f, yo[i], sDY[e]) : yo[i];
      sProd[e] = yc[i] * sVt[e];   // same element as sDY[e]: read before written
    }
    wave_sync();
    // c_r = sum_j Y_k[r][j] V[j][r]: lane r sums row r of the products in FP64
    double cr = 0.0;
    {
      const float *pr = sProd + min(lane, R - 1) * J;
#pragma unroll 8
      for (int j = 0; j < J; ++j) cr += (double)pr[j];
      if (lane >= R) cr = 0.0;
    }
    wave_sync();  // products consumed: the buffer takes the current D_k
    float *sDcur = (float *)(wbase + L.oDcur);
#pragma unroll
    for (int i = 0; i < DQ; ++i) {
      const int q = lane + 64 * i;
      if (q < RR) {
        const float dc = touched ? fmaf(s_old_f, dold[i], dD[i]) : dold[i];
        dD[i] = dc;
        sDcur[q] = dc;
      }
    }
    wave_sync();
    if (a.mode == 0) {
      // Lemma 2: (V^T V * D_k) w = c in FP64, Gauss-Jordan in registers (lane r
      // holds row r of the system)
      double m[RC];
#pragma unroll
      for (int c = 0; c < RC; ++c)
        m[c] = (lane < R && c < R) ? sVtV[lane * R + c] * (double)sDcur[lane * R + c] : 0.0;
      double rhs[1] = {cr};
      double dpiv;
      if (wave_gj_reg<RC, 1>(m, rhs, dpiv, R)) {
        if (lane < R) sC[lane] = rhs[0] / dpiv;
      } else {
        for (int q = lane; q < RR; q += 64) sM[q] = sVtV[q] * (double)sDcur[q];
        if (lane < R) sC[lane] = cr;
        wave_sync();
        wave_pinv_apply(sM, sC, R, sZ, sTmp, sRot, sPair);
      }
      if (lane < R) a.W[((int64_t)wout * a.K_cap + k) * R + lane] = sC[lane];
    } else {
      if (lane < R) sC[lane] = sW[lane];
    }
    wave_sync();
    const double sigma = touched ? 1.0 : s_old;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      if (64 * i >= YS) continue;
      const int e = lane + 64 * i;
      const int r = min((int)(((float)e + 0.5f) * invJ), R);
      facc[i] = fmaf((float)(sigma * sC[r]), yc[i], facc[i]);
    }
#pragma unroll
    for (int i = 0; i < DQ; ++i) {
      const int q = min(lane + 64 * i, RR - 1);
      const int r = q / R, s = q - r * R;
      const double gv = sigma * sC[r] * sC[s] * (double)dD[i];
      gacc[i] += (lane + 64 * i < RR) ? gv : 0.0;
    }
    if (lane == 0) {
      const double ncur = s_old * nold + dn;
      nacc += ncur;
      if (touched && a.mode == 0) a.n[(int64_t)(1 - b) * a.K_cap + k] = ncur;
      if (a.mode == 0) {
        // slice bookkeeping of the next state (made current by the commit)
        a.cur[(int64_t)(1 - gcur) * a.K_cap + k] = (uint8_t)(touched ? 1 - b : b);
        a.tlast[(int64_t)(1 - gcur) * a.K_cap + k] = touched ? (int32_t)step : tl;
      }
    }
    if (touched && a.mode == 0) {
      float *Ynx = a.Y + ((int64_t)(1 - b) * a.K_cap + k) * YS;
#pragma unroll
      for (int i = 0; i < EPT; ++i)
        if (64 * i < YS) Ynx[lane + 64 * i] = yc[i];
      float *Dnx = a.D + ((int64_t)(1 - b) * a.K_cap + k) * RR;
#pragma unroll
      for (int i = 0; i < DQ; ++i) {
        const int q = lane + 64 * i;
        if (q < RR) Dnx[q] = dD[i];
      }
    }
  }

  // combine the waves' accumulators: every wave parks its sums in a slot of
  // its own, then each thread adds the slots of its elements in wave order
  __syncthreads();
  const int plen = partial_len(J, R);
  const size_t slot = wave_slot_bytes(J, R);
  {
    unsigned char *mine = smem + (size_t)wv * slot;
    float *cf = (float *)mine;
    double *cg = (double *)(mine + align_up((size_t)YS * 4, 16));
#pragma unroll
    for (int i = 0; i < EPT; ++i)
      if (64 * i < YS) cf[lane + 64 * i] = facc[i];
#pragma unroll
    for (int i = 0; i < DQ; ++i) {
      const int q = lane + 64 * i;
      if (q < RR) cg[q] = gacc[i];
    }
    if (lane == 0) cg[RR] = nacc;
  }
  __syncthreads();
  double *part = a.partials + (int64_t)chunk * plen;
  const size_t goff = align_up((size_t)YS * 4, 16);
  for (int e = tid; e < plen; e += 512) {
    double v[kWaveWarps];
    if (e < RJ) {
#pragma unroll
      for (int w = 0; w < kWaveWarps; ++w) v[w] = (double)((const float *)(smem + w * slot))[e];
    } else {
#pragma unroll
      for (int w = 0; w < kWaveWarps; ++w) v[w] = ((const double *)(smem + w * slot + goff))[e - RJ];
    }
    double acc = 0.0;
#pragma unroll
    for (int w = 0; w < kWaveWarps; ++w) acc += v[w];
    part[e] = acc;
  }
  if (arrive(a, h, chunk, &sflag))
    finish_pass<FinishBucket<RC>::value>(a, h, h->n_rgroups, a.mode == 0 ? 0 : 2, smem, (size_t)a.lds_bytes);
}

// ---------------------------------------------------------------------------
// Sweep variant 2: one workgroup per slice ("block" variant, any R <= 32,
// J <= 256), for slices whose R x J state does not fit one wave's registers.
// Same arithmetic as the wave variant; the 4 waves split the R x J matrices by
// rows (wave w owns r = w, w+4, ...) and lanes own columns.
// ---------------------------------------------------------------------------
struct PassLds {
  int XS, MB;
  size_t oP, oVt, oX, oU, oW, oWinv, oC, oC2, oM, oDc, oDlo, oVtV, oZ, oTmp, oRot, oPair, bytes;
};

__host__ __device__ inline PassLds pass_lds(int J, int R, bool with_finish = true) {
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
  L.oDlo = o;  o += (size_t)R * R * 4;   // compensation of D_k (mixed precision)
  o = align_up(o, 8);
  L.oVtV = o;  o += (size_t)R * R * 8;
  L.oZ = o;    o += (size_t)R * R * 8;
  L.oTmp = o;  o += (size_t)64 * 8;
  L.oRot = o;  o += (size_t)64 * 8;
  L.oPair = o; o += (size_t)64 * 4;
  (void)with_finish;
  L.bytes = align_up(o, 16);
  return L;
}

// dY += U^T X and dD += U^T U for one staged block of m rows (block variant).
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
  const PassLds L = pass_lds(J, R, false);
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
  float *Yk = Y + (int64_t)k * y_stride(J, R);
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
  __shared__ double red[kWaves];
  dn = wave_sum(dn);
  if (lane == 0) red[wv] = dn;
  __syncthreads();
  if (tid == 0) n[k] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// small copy and conversion kernels
// ---------------------------------------------------------------------------
// dst[0, bytes) = src[0, bytes); src is pinned host memory mapped for the
// device.  16-byte words, one per thread, all loads in flight at once.
__global__ void k_fetch(const uint4 *src, uint4 *dst, int64_t n16, const unsigned char *src_tail,
                        unsigned char *dst_tail, int tail, Report *rep) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i == 0 && rep) rep->t_start = __builtin_amdgcn_s_memrealtime();
  if (i < n16) dst[i] = src[i];
  if (i < tail) dst_tail[i] = src_tail[i];
}

// Batched descriptor fetch: workgroup row y copies job y with a grid-stride
// loop of 16-byte words.
__global__ void k_fetch_list(const FetchJob *jobs, int n_jobs) {
  const int y = blockIdx.y;
  if (y >= n_jobs) return;
  const FetchJob j = jobs[y];
  const int64_t n16 = j.bytes / 16;
  const int64_t i0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i0 == 0 && j.report) ((Report *)j.report)->t_start = __builtin_amdgcn_s_memrealtime();
  const uint4 *src = (const uint4 *)j.src;
  uint4 *dst = (uint4 *)j.dst;
  for (int64_t i = i0; i < n16; i += (int64_t)gridDim.x * 256) dst[i] = src[i];
}

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
                               double *no, const uint16_t *Yc, const float *Dc) {
  const int k = blockIdx.x;
  if (k >= K) return;
  const int b = cur[k];
  const double s = pow(lambda, (double)(step - tlast[k]));
  const int64_t RJ = (int64_t)R * J, RR = (int64_t)R * R, YS = y_stride(J, R);
  for (int e = threadIdx.x; e < RJ; e += 256) {
    const int64_t i = ((int64_t)b * K_cap + k) * YS + e;
    Yo[k * RJ + e] = s * ((double)Y[i] + (Yc ? (double)__uint_as_float((uint32_t)Yc[i] << 16) : 0.0));
  }
  for (int e = threadIdx.x; e < RR; e += 256) {
    const int64_t i = ((int64_t)b * K_cap + k) * RR + e;
    Do[k * RR + e] = s * ((double)D[i] + (Dc ? (double)Dc[i] : 0.0));
  }
  if (threadIdx.x == 0) no[k] = s * n[(int64_t)b * K_cap + k];
}

// Raw committed state (no decay applied) of slices [0, K), for checkpoints.
__global__ void k_gather_state(int J, int R, int K, const float *Y, const float *D, const double *n,
                               const uint8_t *cur, int64_t K_cap, float *Yo, float *Do, double *no) {
  const int k = blockIdx.x;
  if (k >= K) return;
  const int b = cur[k];
  const int64_t RJ = (int64_t)R * J, RR = (int64_t)R * R, YS = y_stride(J, R);
  for (int e = threadIdx.x; e < RJ; e += 256) Yo[k * RJ + e] = Y[((int64_t)b * K_cap + k) * YS + e];
  for (int e = threadIdx.x; e < RR; e += 256) Do[k * RR + e] = D[((int64_t)b * K_cap + k) * RR + e];
  if (threadIdx.x == 0) no[k] = n[(int64_t)b * K_cap + k];
}

// The compensation words of the current buffers (Y's as BF16, widened), same
// layout as k_gather_state's output.
__global__ void k_gather_carry(int J, int R, int K, const uint16_t *Yc, const float *Dc, const uint8_t *cur,
                               int64_t K_cap, float *Yo, float *Do) {
  const int k = blockIdx.x;
  if (k >= K) return;
  const int b = cur[k];
  const int64_t RJ = (int64_t)R * J, RR = (int64_t)R * R, YS = y_stride(J, R);
  for (int e = threadIdx.x; e < RJ; e += 256)
    Yo[k * RJ + e] = __uint_as_float((uint32_t)Yc[((int64_t)b * K_cap + k) * YS + e] << 16);
  for (int e = threadIdx.x; e < RR; e += 256) Do[k * RR + e] = Dc[((int64_t)b * K_cap + k) * RR + e];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline int rw_of(int R) { return (R + 3) / 4; }
static inline int jw_of(int J) { return (J + 63) / 64; }

// Kernels whose dynamic LDS exceeds 64 KB must opt in.
template <typename F>
static int allow_lds(F *fn, size_t bytes) {
  if (bytes <= 65536) return 0;
  return (int)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static inline int ept_of(int J, int R) {
  const int e = (R * J + 63) / 64;
  if (e <= 4) return 4;
  if (e <= 8) return 8;
  if (e <= 16) return 16;
  if (e <= 24) return 24;
  return 32;
}

static inline int dq_of(int R) {
  const int q = (R * R + 63) / 64;
  if (q <= 1) return 1;
  if (q <= 2) return 2;
  return 4;   // R <= 16
}

int pass_variant(int J, int R, int precision, int lagged) {
  // the fused sweep: float32 exact mode, per-wave register tiles that fit
  // without spilling (R <= 16)
  if (precision == 0 && !lagged && J <= 128 && R <= 16 && R * J <= 2048 && wave_lds(J, R).bytes <= 150 * 1024)
    return kPassWave;
  return kPassSplit;
}

int pass_chunk(int variant, int K, int n_cu) {
  int ch;
  if (variant == kPassWave) {
    // one workgroup per CU is resident (register bound): give every wave the
    // same number of slices and launch at most one workgroup per CU
    const int slots = kWaveWarps * (n_cu > 0 ? n_cu : 256);
    const int per = (K + slots - 1) / slots;
    ch = kWaveWarps * (per < 1 ? 1 : per);
  } else {
    ch = (K + 511) / 512;
    if (ch < 1) ch = 1;
  }
  while ((K + ch - 1) / ch > kMaxChunks) ++ch;
  return ch;
}

template <int EPT, int DQ>
static int launch_wave_t(const PassArgs &a, int n_chunks, hipStream_t s) {
  const size_t bytes = a.fuse ? (size_t)a.lds_bytes : wave_lds(a.J, a.R).bytes;
  if (int e = allow_lds(k_pass_wave<EPT, DQ>, bytes)) return e;
  hipLaunchKernelGGL((k_pass_wave<EPT, DQ>), dim3(n_chunks), dim3(512), bytes, s, a);
  return (int)hipGetLastError();
}

size_t fused_pass_lds(int variant, int J, int R) {
  if (variant != kPassWave) return 0;   // the split sweep ends in a separate final-phase launch
  const size_t sweep = wave_lds(J, R).bytes;
  const size_t cap = 160 * 1024 - 1024;   // the kernels' static LDS (flags, small sums) stays under 1 KiB
  const size_t need = std::max(sweep, finish_lds_bytes(J, R));
  return need <= cap ? need : 0;
}

template <int RW, int JW>
static int launch_accum_t(int J, int R, int K, const int64_t *rp, const float *X, const float *U,
                          float *Y, float *D, double *n, hipStream_t s) {
  const PassLds L = pass_lds(J, R, false);
  if (int e = allow_lds(k_accum_given_u<RW, JW>, L.bytes)) return e;
  hipLaunchKernelGGL((k_accum_given_u<RW, JW>), dim3(K), dim3(256), L.bytes, s, J, R, rp, X, U, Y, D, n);
  return (int)hipGetLastError();
}

int launch_pass(const PassArgs &a, int variant, int n_chunks, hipStream_t s) {
  if (n_chunks <= 0) return 0;
  if (variant == kPassWave) {
    switch (ept_of(a.J, a.R) * 32 + dq_of(a.R)) {
#define C(E, Q) case E * 32 + Q: return launch_wave_t<E, Q>(a, n_chunks, s);
      C(4, 1) C(4, 2) C(4, 4) C(8, 1) C(8, 2) C(8, 4) C(16, 1) C(16, 2) C(16, 4)
      C(24, 1) C(24, 2) C(24, 4) C(32, 1) C(32, 2) C(32, 4)
#undef C
      default: return (int)hipErrorInvalidValue;
    }
  }
  return (int)hipErrorInvalidValue;   // the split sweep has launchers of its own
}

template <int RM>
static int launch_finish_t(const PassArgs &a, int mode, hipStream_t s) {
  const size_t bytes = finish_launch_lds(a.J, a.R);
  if (int e = allow_lds(k_finish<RM>, bytes)) return e;
  hipLaunchKernelGGL((k_finish<RM>), dim3(1), dim3(kFinishThreads), bytes, s, a, mode);
  return (int)hipGetLastError();
}

template <int RM>
static int launch_finish_dev_t(const PassArgs *args, const BlockMap *map, int n_blocks, int mode, size_t bytes,
                               hipStream_t s) {
  if (int e = allow_lds(k_finish_dev<RM>, bytes)) return e;
  hipLaunchKernelGGL((k_finish_dev<RM>), dim3(n_blocks), dim3(kFinishThreads), bytes, s, args, map, mode);
  return (int)hipGetLastError();
}

int finish_class(int R) { return R <= 8 ? 8 : R <= 12 ? 12 : R <= 16 ? 16 : R <= 24 ? 24 : 32; }
size_t finish_dev_lds(int J, int R) { return finish_launch_lds(J, R); }

int launch_finish_dev(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks, int mode,
                      hipStream_t s, size_t lds) {
  if (n_blocks <= 0) return 0;
  const size_t bytes = lds ? lds : finish_launch_lds(a.J, a.R);
  switch (finish_class(a.R)) {
    case 8: return launch_finish_dev_t<8>(args, map, n_blocks, mode, bytes, s);
    case 12: return launch_finish_dev_t<12>(args, map, n_blocks, mode, bytes, s);
    case 16: return launch_finish_dev_t<16>(args, map, n_blocks, mode, bytes, s);
    case 24: return launch_finish_dev_t<24>(args, map, n_blocks, mode, bytes, s);
    default: return launch_finish_dev_t<32>(args, map, n_blocks, mode, bytes, s);
  }
}

int launch_finish(const PassArgs &a, int mode, hipStream_t s) {
  if (a.R <= 8) return launch_finish_t<8>(a, mode, s);
  if (a.R <= 12) return launch_finish_t<12>(a, mode, s);
  if (a.R <= 16) return launch_finish_t<16>(a, mode, s);
  if (a.R <= 24) return launch_finish_t<24>(a, mode, s);
  return launch_finish_t<32>(a, mode, s);
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

FetchArgs fetch_args(const char *src, char *dst, size_t bytes, void *report) {
  FetchArgs f;
  f.report = report;
  f.n16 = (int64_t)(bytes / 16);
  f.tail = (int)(bytes - (size_t)f.n16 * 16);
  f.src = src;
  f.dst = dst;
  f.src_tail = src + f.n16 * 16;
  f.dst_tail = dst + f.n16 * 16;
  const int64_t threads = std::max<int64_t>(std::max<int64_t>(f.n16, f.tail), 1);
  f.grid = (unsigned)((threads + 255) / 256);
  return f;
}

int launch_fetch(const char *src, char *dst, size_t bytes, void *report, hipStream_t s) {
  const FetchArgs f = fetch_args(src, dst, bytes, report);
  hipLaunchKernelGGL(k_fetch, dim3(f.grid), dim3(256), 0, s, (const uint4 *)f.src, (uint4 *)f.dst, f.n16,
                     (const unsigned char *)f.src_tail, (unsigned char *)f.dst_tail, f.tail, (Report *)f.report);
  return (int)hipGetLastError();
}

int launch_fetch_list(const FetchJob *jobs, int n_jobs, int64_t max_bytes, hipStream_t s) {
  if (n_jobs <= 0) return 0;
  const int64_t w = std::max<int64_t>(max_bytes / 16, 1);
  const unsigned gx = (unsigned)std::min<int64_t>((w + 255) / 256, 64);
  hipLaunchKernelGGL(k_fetch_list, dim3(gx, (unsigned)n_jobs), dim3(256), 0, s, jobs, n_jobs);
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
                        int64_t K_cap, double *Yo, double *Do, double *no, const uint16_t *Yc, const float *Dc,
                        hipStream_t s) {
  if (K <= 0) return 0;
  hipLaunchKernelGGL(k_export_state, dim3(K), dim3(256), 0, s, J, R, K, step, lambda, Y, D, n, cur,
                     tlast, K_cap, Yo, Do, no, Yc, Dc);
  return (int)hipGetLastError();
}

int launch_gather_state(int J, int R, int K, const float *Y, const float *D, const double *n,
                        const uint8_t *cur, int64_t K_cap, float *Yo, float *Do, double *no,
                        hipStream_t s) {
  if (K <= 0) return 0;
  hipLaunchKernelGGL(k_gather_state, dim3(K), dim3(256), 0, s, J, R, K, Y, D, n, cur, K_cap, Yo, Do, no);
  return (int)hipGetLastError();
}

int launch_gather_carry(int J, int R, int K, const uint16_t *Yc, const float *Dc, const uint8_t *cur, int64_t K_cap,
                        float *Yo, float *Do, hipStream_t s) {
  if (K <= 0) return 0;
  hipLaunchKernelGGL(k_gather_carry, dim3(K), dim3(256), 0, s, J, R, K, Yc, Dc, cur, K_cap, Yo, Do);
  return (int)hipGetLastError();
}

}  // namespace dash
