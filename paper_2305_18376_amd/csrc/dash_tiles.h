// Device building blocks shared by the sweep kernels (dash_kernels.hip,
// dash_split.hip): MFMA tile products of the new rows, row staging, the
// two-level arrival reduction of chunk partials, and the guard and
// pseudo-inverse form of Lemma 1.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#include "dash_dev.h"
#include "dash_math.h"

namespace dash {

// MFMA tiles.  v_mfma_f32_16x16x4_f32: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; v_mfma_f32_16x16x32_bf16: A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16] (i < 8), BF16-rounded operands; both return
// C[4 (l / 16) + i][l % 16] (i < 4) with FP32 accumulation.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma_bf16(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma_f32(float a, float b, const f32x4 &c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Raw buffer access through a bounds-checked descriptor: a load at a byte
// offset outside [0, bytes) returns zero and a store there is dropped, so
// ragged tiles and empty slices need no branches around their memory
// operations.  kNoOff lies outside every buffer.
constexpr int kNoOff = (int)0x80000000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}

__device__ __forceinline__ float buf_ldf(__amdgpu_buffer_rsrc_t r, int off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

__device__ __forceinline__ void buf_stf(__amdgpu_buffer_rsrc_t r, int off, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), r, off, 0, 0);
}

// N consecutive float words (N = 1, 2, 4) in one access; with a range check
// per access, all N must lie inside or outside the buffer together.
template <int N>
__device__ __forceinline__ void buf_ldfn(__amdgpu_buffer_rsrc_t r, int off, float (&o)[N]) {
  if constexpr (N == 1) {
    o[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  } else if constexpr (N == 2) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    o[0] = __uint_as_float(v[0]);
    o[1] = __uint_as_float(v[1]);
  } else {
    const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) o[i] = __uint_as_float(v[i]);
  }
}

template <int N>
__device__ __forceinline__ void buf_stfn(__amdgpu_buffer_rsrc_t r, int off, const float (&x)[N]) {
  if constexpr (N == 1) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x[0]), r, off, 0, 0);
  } else if constexpr (N == 2) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 v = {__float_as_uint(x[0]), __float_as_uint(x[1])};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
  } else {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 v = {__float_as_uint(x[0]), __float_as_uint(x[1]), __float_as_uint(x[2]), __float_as_uint(x[3])};
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, 0);
  }
}

// N consecutive BF16 words widened to float (N = 1, 2, 4: 2, 4 or 8 bytes)
template <int N>
__device__ __forceinline__ void buf_ldbfn(__amdgpu_buffer_rsrc_t r, int off, float (&o)[N]) {
  if constexpr (N == 1) {
    o[0] = __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0) << 16);
  } else if constexpr (N == 2) {
    const uint32_t v = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0);
    o[0] = __uint_as_float(v << 16);
    o[1] = __uint_as_float(v & 0xffff0000u);
  } else {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
    o[0] = __uint_as_float(v[0] << 16);
    o[1] = __uint_as_float(v[0] & 0xffff0000u);
    o[2] = __uint_as_float(v[1] << 16);
    o[3] = __uint_as_float(v[1] & 0xffff0000u);
  }
}

// N floats rounded to nearest even BF16 and stored as N consecutive words
template <int N>
__device__ __forceinline__ void buf_stbfn(__amdgpu_buffer_rsrc_t r, int off, const float (&x)[N]) {
  uint32_t b[N];
#pragma unroll
  for (int i = 0; i < N; ++i) b[i] = __builtin_bit_cast(uint16_t, (__bf16)x[i]);
  if constexpr (N == 1) {
    __builtin_amdgcn_raw_buffer_store_b16((uint16_t)b[0], r, off, 0, 0);
  } else if constexpr (N == 2) {
    __builtin_amdgcn_raw_buffer_store_b32(b[0] | (b[1] << 16), r, off, 0, 0);
  } else {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 v = {b[0] | (b[1] << 16), b[2] | (b[3] << 16)};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, off, 0, 0);
  }
}

// BF16 words (the compensation words of Y): loaded widened to float, stored
// rounded to nearest even
__device__ __forceinline__ float buf_ldbf(__amdgpu_buffer_rsrc_t r, int off) {
  return __uint_as_float((uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0) << 16);
}

__device__ __forceinline__ void buf_stbf(__amdgpu_buffer_rsrc_t r, int off, float v) {
  __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, (__bf16)v), r, off, 0, 0);
}

// A value the whole wave shares, read from lane 0 (so that the compiler keeps
// it, and what is derived from it, in scalar registers).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni64(int64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T *uniptr(T *p) {
  return (T *)(uintptr_t)uni64((int64_t)(uintptr_t)p);
}

// Zero rows m .. mp - 1 (all J16 columns) and columns J .. J16 - 1 of rows
// 0 .. m - 1 of a staged row block (stride XS).
__device__ __forceinline__ void zero_block_pad(float *sX, int XS, int m, int mp, int J, int J16, int tid) {
  for (int e = tid; e < (mp - m) * J16; e += 256) {
    const int row = e / J16;
    sX[(m + row) * XS + (e - row * J16)] = 0.f;
  }
  const int pc = J16 - J;
  if (pc > 0)
    for (int e = tid; e < m * pc; e += 256) {
      const int row = e / pc;
      sX[row * XS + J + (e - row * pc)] = 0.f;
    }
}


// Mixed precision (BF16 MFMA) row products of the block variant.
// v_mfma_f32_16x16x32_bf16: lane l holds A[l % 16][8 (l / 16) + i] and
// B[8 (l / 16) + i][l % 16] (i < 8) and receives C[4 (l / 16) + i][l % 16]
// (i < 4); products of BF16-rounded operands, FP32 accumulation.
// ---------------------------------------------------------------------------
// the mixed-precision tiles of one slice: wave w owns the dY column tiles
// w, w+4, w+8, w+12 (16 columns each) for both rank tiles (accY[2 c + mt]), and
// the dD tile w of the (R / 16)^2 rank-tile pairs
constexpr int kMxTiles = 8;
// One 16 x 16 tile of X P in FP32 with P held transposed: xrow is the lane's
// row of the 16-row tile and prow the lane's rank of the 16-rank tile, both
// with J16 (J rounded up to 16) entries, zero beyond J, 16-byte aligned.  The
// sum over j is split so that lane quad q takes columns 16 s + 4 q .. + 3 of
// each 16-column step s (four MFMAs, one float4 of each operand), so every
// operand comes from one vector LDS read.
__device__ __forceinline__ f32x4 rows_times_pt(const float *xrow, const float *prow, int J16, int lq) {
  f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
  const float4 *xa = reinterpret_cast<const float4 *>(xrow) + lq;
  const float4 *pb = reinterpret_cast<const float4 *>(prow) + lq;
  const int n4 = J16 >> 2;
  // the next step's operands are read while this step's MFMAs run
  float4 a = xa[0], b = pb[0];
  for (int q = 4; q < n4; q += 4) {
    const float4 an = xa[q], bn = pb[q];
    acc0 = mfma_f32(a.x, b.x, acc0);
    acc1 = mfma_f32(a.y, b.y, acc1);
    acc0 = mfma_f32(a.z, b.z, acc0);
    acc1 = mfma_f32(a.w, b.w, acc1);
    a = an;
    b = bn;
  }
  acc0 = mfma_f32(a.x, b.x, acc0);
  acc1 = mfma_f32(a.y, b.y, acc1);
  acc0 = mfma_f32(a.z, b.z, acc0);
  acc1 = mfma_f32(a.w, b.w, acc1);
  return acc0 + acc1;
}

// The same tile with BF16-rounded operands (16x16x32 MFMA, FP32 sums).
__device__ __forceinline__ f32x4 rows_times_pt_bf(const float *xrow, const float *prow, int J, int lane) {
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const int lk = (lane >> 4) * 8;
  for (int ks = 0; ks < J; ks += 32) {
    bf16x8 av, bv;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int kk = ks + lk + q;
      av[q] = (__bf16)((kk < J) ? xrow[kk] : 0.f);
      bv[q] = (__bf16)((kk < J) ? prow[kk] : 0.f);
    }
    acc = mfma_bf16(av, bv, acc);
  }
  return acc;
}

// dY += U^T X, dD += U^T U in FP32 on MFMA (16x16x4) for one staged block:
// sX rows of stride XS and sU rows of stride US, rows m .. mp - 1 zero in
// both (mp = m rounded up to 16), sX columns J .. J16 - 1 and sU columns
// R .. 16 MT - 1 zero.  Lane quad q takes rows 4 q .. 4 q + 3 of each 16-row
// step, four MFMAs per tile and step; a step's LDS reads all go out before
// its MFMAs.  Wave w owns the column tiles w, w + 4, w + 8, w + 12 of both
// rank tiles and the rank-tile pair w of dD.
__device__ __forceinline__ void accum_block_f32(const float *sX, const float *sU, int XS, int US, int mp, int J,
                                                int R, f32x4 (&accY)[kMxTiles], f32x4 &accD, int tid) {
  const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int MT = (R + 15) >> 4, NT = (J + 15) >> 4;
  const int li = lane & 15, lq = lane >> 4;
  const bool dtile = wv < MT * MT;
  const int mt = dtile ? wv / MT : 0, st = dtile ? wv - mt * MT : 0;
#pragma unroll 1
  for (int ks = 0; ks < mp; ks += 16) {
    const float *urow = sU + (ks + 4 * lq) * US + li;
    const float *xrow = sX + (ks + 4 * lq) * XS + li;
    float au0[4], au1[4], bx[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      au0[i] = urow[i * US];
      au1[i] = (MT > 1) ? urow[i * US + 16] : 0.f;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int nt = wv + 4 * c;
#pragma unroll
      for (int i = 0; i < 4; ++i) bx[c][i] = (nt < NT) ? xrow[i * XS + 16 * nt] : 0.f;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (wv + 4 * c < NT) {
          accY[2 * c] = mfma_f32(au0[i], bx[c][i], accY[2 * c]);
          if (MT > 1) accY[2 * c + 1] = mfma_f32(au1[i], bx[c][i], accY[2 * c + 1]);
        }
      }
      if (dtile) accD = mfma_f32(mt == 0 ? au0[i] : au1[i], st == 0 ? au0[i] : au1[i], accD);
    }
  }
}

// dY += U^T X, dD += U^T U on MFMA for one staged block (rows >= m are zero
// in both sX and sU; mp = m rounded up to 32).  The U^T operand of a rank
// tile is loaded once per 32-row step and serves every column tile, and, as
// the B operand of dD, the rank-tile pairs too.
__device__ __forceinline__ void accum_block_mx(const float *sX, const float *sU, int XS, int US, int mp, int J,
                                               int R, f32x4 (&accY)[kMxTiles], f32x4 &accD, int tid) {
  const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int MT = (R + 15) >> 4, NT = (J + 15) >> 4;
  const int li = lane & 15, lk = (lane >> 4) * 8;
  for (int ks = 0; ks < mp; ks += 32) {
    bf16x8 au[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const int r = mt * 16 + li;
#pragma unroll
      for (int q = 0; q < 8; ++q) au[mt][q] = (__bf16)((r < R) ? sU[(ks + lk + q) * US + r] : 0.f);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int nt = wv + 4 * c;
      if (nt < NT) {
        const int j = min(nt * 16 + li, J - 1);
        bf16x8 bv;
#pragma unroll
        for (int q = 0; q < 8; ++q) bv[q] = (__bf16)sX[(ks + lk + q) * XS + j];
        accY[2 * c] = mfma_bf16(au[0], bv, accY[2 * c]);
        if (MT > 1) accY[2 * c + 1] = mfma_bf16(au[1], bv, accY[2 * c + 1]);
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    if (wv < MT * MT) {
      const int mt = wv / MT, st = wv - mt * MT;
      accD = mfma_bf16(mt == 0 ? au[0] : au[1], st == 0 ? au[0] : au[1], accD);
    }
  }
}

// Copy m contiguous rows of J floats from HBM into sX (row stride XS) with NTH
// threads (tid < NTH); m * J <= 8192.  A thread's loads go out in batches of
// four float4 (eight floats) before its LDS stores, so the copy waits for a few
// memory latencies, not one per element.  Float4 loads when the rows allow
// them.  With SQ the thread's sum of squares of what it loaded is returned
// (FP64).
template <bool SQ, int NTH = 256>
__device__ __forceinline__ double stage_rows(const float *__restrict__ src, int m, int J, int XS, float *sX,
                                             int tid) {
  double sq = 0.0;
  const int n = m * J;
  if ((J & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
    const int n4 = n >> 2;
    constexpr int PER = (2048 + NTH - 1) / NTH;
#pragma unroll 1
    for (int i0 = 0; i0 < PER; i0 += 4) {
      if (tid + NTH * i0 >= n4) break;
      float4 v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = tid + NTH * (i0 + i);
        v[i] = (q < n4) ? reinterpret_cast<const float4 *>(src)[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = tid + NTH * (i0 + i);
        if (q < n4) {
          const int e = 4 * q, row = e / J, col = e - row * J;
          float *d = sX + row * XS + col;
          d[0] = v[i].x;
          d[1] = v[i].y;
          d[2] = v[i].z;
          d[3] = v[i].w;
        }
        if constexpr (SQ) {
          sq = fma((double)v[i].x, (double)v[i].x, sq);
          sq = fma((double)v[i].y, (double)v[i].y, sq);
          sq = fma((double)v[i].z, (double)v[i].z, sq);
          sq = fma((double)v[i].w, (double)v[i].w, sq);
        }
      }
    }
  } else {
    constexpr int PER = (8192 + NTH - 1) / NTH;
#pragma unroll 1
    for (int i0 = 0; i0 < PER; i0 += 8) {
      if (tid + NTH * i0 >= n) break;
      float v[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = tid + NTH * (i0 + i);
        v[i] = (e < n) ? src[e] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int e = tid + NTH * (i0 + i);
        if (e < n) {
          const int row = e / J;
          sX[row * XS + (e - row * J)] = v[i];
        }
        if constexpr (SQ) sq = fma((double)v[i], (double)v[i], sq);
      }
    }
  }
  return sq;
}

// Arrival of a workgroup whose chunk partial is written: the last of each group
// of kChunksPerRGroup chunks to arrive sums the group's partials in chunk order
// into gpart (a first reduction level inside the sweep launch; the final phase
// does the second).  With a.fuse, the last group reducer to finish takes a
// second ticket and returns true: it then runs the final phase.  Every ticket is
// reset by the workgroup that drew the last number, so all are zero again when
// the launch ends.
template <typename A>
__device__ bool arrive(const A &a, const StepHeader *h, int chunk, int *sflag) {
  const int tid = threadIdx.x, nt = blockDim.x;
  const int plen = partial_len(a.J, a.R);
  const int cpr = h->chunks_per_rgroup;
  const int rg = chunk / cpr;
  const int c0 = rg * cpr, c1 = min(h->n_chunks, c0 + cpr);
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const int old = atomicAdd(&a.counters[rg], 1);
    *sflag = (old == c1 - c0 - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!*sflag) return false;
  __threadfence();
  for (int e = tid; e < plen; e += nt) a.gpart[(int64_t)rg * plen + e] = ordered_sum(a.partials, plen, e, c0, c1);
  if (!a.fuse) {
    if (tid == 0) a.counters[rg] = 0;
    return false;
  }
  __syncthreads();
  if (tid == 0) {
    a.counters[rg] = 0;
    __threadfence();
    const int old = atomicAdd(&a.counters[kMaxChunks], 1);
    *sflag = (old == h->n_rgroups - 1) ? 1 : 0;
    if (*sflag) a.counters[kMaxChunks] = 0;
  }
  __syncthreads();
  if (!*sflag) return false;
  __threadfence();
  return true;
}


// ---------------------------------------------------------------------------
// Lemma 1 (eq. [updateU_lemma]): U_new = X_new V S_k (S_k V^T V S_k)^{-1},
// one R x R system per slice.  With A = V^T V eliminated once per pass
// (pivots piv_r: the Schur complement diagonals, i.e. the squared Cholesky
// diagonal), the system S_k A S_k has pivots w_r^2 piv_r and diagonal
// w_r^2 A_rr, so the Cholesky acceptance rule for it is
//     min_r w_r^2 piv_r  >  kPivotRel * max_r w_r^2 A_rr.
// When it holds, U_new = X_new V A^{-1} S_k^{-1}: the row product with
// P = V A^{-1} followed by a division by w.  One wave, lane r < R holding
// w_r, piv_r and A_rr; the decision comes back wave-uniform.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool lemma1_regular(double w, double piv, double arr, int R) {
  const int lane = threadIdx.x & 63;
  const double w2 = w * w;
  const double lo = wave_min(lane < R ? w2 * piv : INFINITY);
  const double hi = wave_max(lane < R ? w2 * arr : 0.0);
  return hi > 0.0 && lo > kPivotRel * hi;
}

// Otherwise the system is solved by its eigen pseudo-inverse (the minimum-norm
// least-squares reading of a singular system): u = x V S (S A S)^+.  The row
// product still gives t = x V B with B = A^{-1} (or A^+ when A itself failed the
// rule), and t A = x V because the rows of V lie in the row space of A, so
// u = t Z with Z = A S (S A S)^+.  One wave computes Z in FP64 (cyclic Jacobi,
// eigenvalues kept above kEigCutoff times the largest) and stores it as float
// into Zf (row-major, leading dimension ldz).  A and w may live in LDS or
// global memory; M and E take R*R doubles each, lam R, rot 64, pair 64 ints.
__device__ inline void lemma1_pinv_matrix(const double *A, const double *w, int R, double *M, double *E,
                                          double *lam, double *rot, int *pair, float *Zf, int ldz) {
  const int lane = threadIdx.x & 63;
  for (int q = lane; q < R * R; q += 64) {
    const int r = q / R, c = q - r * R;
    M[q] = w[r] * A[q] * w[c];
  }
  wave_sync();
  wave_jacobi(M, E, R, rot, pair);
  double top = 0.0;
  for (int i = 0; i < R; ++i) top = fmax(top, fabs(M[i * R + i]));
  if (lane < R) {
    const double li = M[lane * R + lane];
    lam[lane] = (top > 0.0 && li > kEigCutoff * top) ? 1.0 / li : 0.0;
  }
  wave_sync();
  // T = A S E (into M; its eigenvalues were read above)
  for (int q = lane; q < R * R; q += 64) {
    const int r = q / R, i = q - r * R;
    double acc = 0.0;
    for (int p = 0; p < R; ++p) acc = fma(A[r * R + p] * w[p], E[p * R + i], acc);
    M[q] = acc;
  }
  wave_sync();
  // Z = T diag(lam) E^T
  for (int q = lane; q < R * R; q += 64) {
    const int r = q / R, c = q - r * R;
    double acc = 0.0;
    for (int i = 0; i < R; ++i) acc = fma(M[r * R + i] * lam[i], E[c * R + i], acc);
    Zf[r * ldz + c] = (float)acc;
  }
  wave_sync();
}

}  // namespace dash
