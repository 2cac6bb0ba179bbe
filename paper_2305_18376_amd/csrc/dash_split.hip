// Split sweep of one ALS pass of the DASH update on gfx950 (Algorithm 1 with
// Lemmas 1-3), as four launches on the context's stream:
//
//   row stage   k_rows:   the touched slices, most rows first, pulled from a
//                         device work queue by persistent workgroups.  Lemma 1
//                         on the new rows (MFMA), the new-row sums dY = U^T X,
//                         dD = U^T U, dn = sum ||x||^2, the fold under the
//                         forgetting factor (eq. [obtain_CandD]) into the spare
//                         state buffer, and c_k = diag(Y_k V) (Lemma 2) -- or,
//                         in lagged mode, its recursion (eq. [obtain_CandC]).
//   solve stage k_solve:  every slice, one wave each: c_k of the untouched
//                         slices from their stored Y_k, Lemma 2's system
//                         (V^T V * D_k) w_k = c_k in FP64 (pseudo-inverse when
//                         it fails the acceptance rule), the slice bookkeeping
//                         of the next state, and G / sum-n partials.
//   F stage     k_fsum:   F^T = sum_k sigma_k diag(w_k) Y_k streamed over every
//                         slice (exact mode), or k_fsum_rows: the new rows'
//                         terms of eq. [obtain_FandF], [obtain_FandG] (lagged
//                         mode); chunk partials in FP64, the first level of the
//                         fixed-order reduction by the last arrival of each group.
//   final phase k_finish (dash_kernels.hip): Lemma 3 and, on the last pass,
//                         the commit.
//
// Every slice's work stays on one workgroup (row stage) or one wave (solve
// stage) and every sum that spans slices is a fixed-order reduction of
// per-chunk partials, so the results do not depend on which workgroup ran a
// slice.  Untouched slices are solved on their stored, undecayed Y_k and D_k
// (w_k does not depend on the common factor lambda^dt) and enter F and G with
// sigma_k = lambda^dt.  See dash_dev.h for the layouts.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <math.h>

#include <algorithm>

#include "dash_dev.h"
#include "dash_math.h"
#include "dash_tiles.h"

namespace dash {

// ---------------------------------------------------------------------------
// Row stage
// ---------------------------------------------------------------------------
struct RowsLds {
  int XS, US, J16, MB;
  size_t oP, oX, oU, oZf, oW, oWinv, bytes;
};

// P^T (ranks padded to a multiple of 16, row stride XS, zero beyond R and J),
// a row block (MB rows of stride XS = J16 + 4, where J16 is J rounded up to
// 16: 16-byte rows whose four-row steps fall in different banks) that is also
// the hand-off buffer of dY (R x J) and the scratch of Lemma 1's
// pseudo-inverse form, the U block (MB x US, US = 16 MT + 4; also dD), that
// form's matrix Z (R x R), w and 1/w.
__host__ __device__ inline RowsLds rows_lds(int J, int R) {
  RowsLds L;
  L.J16 = (J + 15) / 16 * 16;
  L.XS = L.J16 + 4;
  L.US = (R + 15) / 16 * 16 + 4;
  L.MB = (J <= 128) ? 64 : 32;
  size_t o = 0;
  L.oP = o;
  o = align_up(o + (size_t)((R + 15) / 16 * 16) * L.XS * 4, 16);
  L.oX = o;
  size_t xb = (size_t)L.MB * L.XS * 4;
  const size_t scr = (size_t)(2 * R * R + R + 64) * 8 + 64 * 4;
  xb = std::max(xb, scr);
  xb = std::max(xb, (size_t)R * J * 4);
  // the waves' c_k partials after the fold: 4 waves x RW ranks x 64 lanes
  // (RW = 8: the deferred-slice kernel is the RW = 8 instantiation for every R)
  xb = std::max(xb, (size_t)4 * 8 * 64 * 8);
  o = align_up(o + xb, 16);
  L.oU = o;
  o = align_up(o + (size_t)L.MB * L.US * 4, 16);
  L.oZf = o;
  o = align_up(o + (size_t)R * R * 4, 16);
  L.oW = o;
  o += (size_t)R * 8;
  L.oWinv = o;
  o += (size_t)R * 4;
  L.bytes = align_up(o, 16);
  return L;
}

// Row-stage layout of the mixed-precision path: the new rows staged once as
// BF16 in two layouts -- Xr row-major (stride XS) for U^T = P^T X^T and Xc
// column-major (stride XC) for dY = U^T X -- with P^T (Pt, stride XS) and U^T
// (Ut, stride XC) in BF16 as well, so that every MFMA operand (eight
// consecutive k per lane) is one 16-byte LDS read.  Columns are padded to
// Jp = 32 * ceil(J / 32) (the k steps of P^T X^T), ranks to 16 * ceil(R / 16).
// The Xr + Xc region also takes the dY hand-off (R x J float) and the c_k
// partials after the fold; dD gets a region of its own.
struct RowsLdsBf {
  int Jp, XS, XC, MB, R16, J16;
  size_t oPt, oX, oXc, oUt, oDD, oW, oWinv, bytes;
};

__host__ __device__ inline RowsLdsBf rows_lds_bf(int J, int R) {
  RowsLdsBf L;
  L.Jp = (J + 31) / 32 * 32;
  L.XS = L.Jp + 8;
  L.MB = (J <= 128) ? 64 : 32;
  L.XC = L.MB + 8;
  L.R16 = (R + 15) / 16 * 16;
  L.J16 = (J + 15) / 16 * 16;
  size_t o = 0;
  L.oPt = o;
  o = align_up(o + (size_t)L.R16 * L.XS * 2, 16);
  L.oX = o;
  L.oXc = align_up(o + (size_t)L.MB * L.XS * 2, 16);
  size_t xend = L.oXc + (size_t)L.J16 * L.XC * 2;
  xend = std::max(xend, L.oX + (size_t)R * J * 4);
  xend = std::max(xend, L.oX + (size_t)4 * 8 * 64 * 8);
  o = align_up(xend, 16);
  L.oUt = o;
  o = align_up(o + (size_t)L.R16 * L.XC * 2, 16);
  L.oDD = o;
  o = align_up(o + (size_t)R * R * 4, 16);
  L.oW = o;
  o += (size_t)R * 8;
  L.oWinv = o;
  o += (size_t)R * 4;
  L.bytes = align_up(o, 16);
  return L;
}

// Stage m rows of J floats (HBM, row-major) into Xr and Xc as BF16, with rows
// m .. mp - 1 and columns J .. Jp - 1 (Xr) / J .. J16 - 1 (Xc) zero; returns
// this thread's sum of squares of the float values (FP64).
__device__ inline double stage_rows_bf(const float *__restrict__ src, int m, int mp, int J, const RowsLdsBf &L,
                                       __bf16 *Xr, __bf16 *Xc, int tid) {
  double sq = 0.0;
  const __bf16 z = (__bf16)0.f;
  // padding
  for (int e = tid; e < mp * (L.Jp - J); e += 256) {
    const int row = e / (L.Jp - J);
    Xr[row * L.XS + J + (e - row * (L.Jp - J))] = z;
  }
  for (int e = tid; e < (mp - m) * J; e += 256) {
    const int row = m + e / J, col = e % J;
    Xr[row * L.XS + col] = z;
    Xc[col * L.XC + row] = z;
  }
  for (int e = tid; e < (L.J16 - J) * mp; e += 256) {
    const int col = J + e / mp, row = e % mp;
    Xc[col * L.XC + row] = z;
  }
  const int n = m * J;
  if ((J & 3) == 0 && (reinterpret_cast<uintptr_t>(src) & 15) == 0) {
    const int n4 = n >> 2;
#pragma unroll 1
    for (int q0 = tid; q0 < n4; q0 += 4 * 256) {
      float4 v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = q0 + 256 * i;
        v[i] = (q < n4) ? reinterpret_cast<const float4 *>(src)[q] : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = q0 + 256 * i;
        if (q < n4) {
          const int e = 4 * q, row = e / J, col = e - row * J;
          const __bf16 b0 = (__bf16)v[i].x, b1 = (__bf16)v[i].y, b2 = (__bf16)v[i].z, b3 = (__bf16)v[i].w;
          __bf16 *d = Xr + row * L.XS + col;
          d[0] = b0;
          d[1] = b1;
          d[2] = b2;
          d[3] = b3;
          Xc[col * L.XC + row] = b0;
          Xc[(col + 1) * L.XC + row] = b1;
          Xc[(col + 2) * L.XC + row] = b2;
          Xc[(col + 3) * L.XC + row] = b3;
          sq = fma((double)v[i].x, (double)v[i].x, sq);
          sq = fma((double)v[i].y, (double)v[i].y, sq);
          sq = fma((double)v[i].z, (double)v[i].z, sq);
          sq = fma((double)v[i].w, (double)v[i].w, sq);
        }
      }
    }
  } else {
    for (int e = tid; e < n; e += 256) {
      const float x = src[e];
      const int row = e / J, col = e - row * J;
      const __bf16 b = (__bf16)x;
      Xr[row * L.XS + col] = b;
      Xc[col * L.XC + row] = b;
      sq = fma((double)x, (double)x, sq);
    }
  }
  return sq;
}

// RW ranks x JW columns per thread in the [rank][column] layout: thread
// (wave w, lane l) owns r = w + 4 rr (rr < RW) and j = l + 64 jj (jj < JW).
// SLOW = false: the slices whose Lemma 1 system passes the acceptance rule;
// the others are deferred to a list.  SLOW = true: the deferred slices, with
// the pseudo-inverse form (a separate launch, so that its code does not weigh
// on the registers of the common case).
template <int RW, int JW, bool MX, bool SLOW, bool VEC = false>
__global__ __launch_bounds__(256, 2) void k_rows(const PassArgs *args, const BlockMap *map) {
  extern __shared__ __align__(16) unsigned char smem[];
  CPassArgs &a = *(CPassArgs *)(map ? map[blockIdx.x].args : args);
  const int blk = map ? map[blockIdx.x].local : (int)blockIdx.x;
  const int nblk = map ? map[blockIdx.x].pad : (int)gridDim.x;   // this context's workgroups
  __shared__ int sItem, sDefer;
  __shared__ int sNext[5];   // the deferred-slice kernel's item: index, slice, g0, g1, rows
  __shared__ double sDn[4];
  // The fast kernel's look-ahead: the descriptors of its items i, i + 1, i + 2
  // (a ring of three) and the state words of items i, i + 1 (a ring of two),
  // so that a slice starts its HBM loads without dependent round trips.
  // Words of sMeta: [0, 32) W row, 32 + b n in buffer b, 34 first row group's
  // source, 35 its first output row, 36 its row count (low half), 37 the
  // slice's buffer (low half) and last fold (high half).
  __shared__ __align__(16) Item sDesc[3];
  __shared__ uint64_t sMeta[2][38];
  const StepHeader *h = a.hdr;
  const int J = a.J, R = a.R, RR = R * R;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int Kp = h->K_prev, n_items = h->n_items, seq = h->seq;
  const int64_t step = h->step;
  const int gcur = a.ctl->gcur;
  const int win = (a.pass == 0) ? gcur : 1 - gcur;
  const VBundleView vb = vb_view(a.vb + (int64_t)win * a.vb_stride, J, R);
  // the mixed path's fast kernel stages BF16 operands; the float32 path and
  // the deferred-slice kernel keep float rows and Lemma 1's scratch
  constexpr bool BF = MX && !SLOW;
  const RowsLds L = rows_lds(J, R);
  const RowsLdsBf LB = rows_lds_bf(J, R);
  float *sP = (float *)(smem + L.oP);
  float *sX = BF ? (float *)(smem + LB.oX) : (float *)(smem + L.oX);
  double *sScr = (double *)(smem + L.oX);   // Lemma 1 pseudo-inverse scratch (before the rows)
  float *sU = (float *)(smem + L.oU);
  float *sZf = (float *)(smem + L.oZf);
  double *sW = BF ? (double *)(smem + LB.oW) : (double *)(smem + L.oW);
  float *sWinv = BF ? (float *)(smem + LB.oWinv) : (float *)(smem + L.oWinv);
  __bf16 *bPt = (__bf16 *)(smem + LB.oPt);
  __bf16 *bXr = (__bf16 *)(smem + LB.oX);
  __bf16 *bXc = (__bf16 *)(smem + LB.oXc);
  __bf16 *bUt = (__bf16 *)(smem + LB.oUt);
  const int XS = L.XS, MB = BF ? LB.MB : L.MB;
  const bool write_u = a.last_pass || a.lagged;
  if (a.stamp_start && blk == 0 && tid == 0 && a.pass == 0 && h->report)
    ((Report *)h->report)->t_start = __builtin_amdgcn_s_memrealtime();

  if constexpr (BF) {
    // P^T in BF16, ranks padded to a multiple of 16 and columns to Jp (zero)
    for (int e = tid; e < LB.R16 * LB.Jp; e += 256) {
      const int r = e / LB.Jp, j = e - r * LB.Jp;
      bPt[r * LB.XS + j] = (__bf16)((r < R && j < J) ? vb.P32[j * R + r] : 0.f);
    }
  } else {
    // P^T, ranks padded to a multiple of 16 and columns to J16 (zero)
    const int R16 = (R + 15) & ~15;
    for (int e = tid; e < R16 * L.XS; e += 256) {
      const int r = e / L.XS, j = e - r * L.XS;
      sP[e] = (r < R && j < J) ? vb.P32[j * R + r] : 0.f;
    }
  }
  // Column ownership in the [rank][column] layout: VEC (J a multiple of JW)
  // gives lane l the JW consecutive columns JW l .. JW l + JW - 1, so each of
  // its ranks is one 4 JW-byte access (a CU's outstanding memory requests,
  // not bytes, bound this stage); otherwise it owns columns l, l + 64, ...
  // (separate instantiations: carrying both costs the registers of both)
  constexpr bool vecj = VEC;
  // the entries of V^T this thread multiplies for c_k
  float vt[RW][JW];
  {
    const auto rv = buf_rsrc(vb.Vt32, R * J * 4);
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) {
      const int r = wv + 4 * rr;
      if (vecj) {
        buf_ldfn<JW>(rv, (r < R && lane * JW < J) ? (r * J + lane * JW) * 4 : kNoOff, vt[rr]);
      } else {
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
          const int j = lane + 64 * jj;
          vt[rr][jj] = buf_ldf(rv, (r < R && j < J) ? (r * J + j) * 4 : kNoOff);
        }
      }
    }
  }
  // pivots and diagonal of V^T V for Lemma 1's acceptance rule (wave 0, lane r)
  const double pivl = lane < R ? vb.piv[lane] : 0.0;
  const double arrl = lane < R ? vb.VtV[lane * R + lane] : 0.0;

  // Wave 0's gather for the fast kernel: lane l loads word l of item it1's
  // state words (descriptor d1) and lanes 37, 38 the descriptor of item it2;
  // the values stay in registers until put() stores them, so their latency
  // hides behind a slice's work.
  auto gather = [&](int it1, const Item &d1, int it2, uint64_t &g64, uint32_t &g32) {
    const int l = threadIdx.x & 63;
    g64 = 0;
    g32 = 0;
    if (it1 >= n_items) return;
    const int k1 = d1.slice;
    const bool grp = d1.g0 < d1.g1;
    if (l < R) g64 = (uint64_t)__double_as_longlong(a.W[((int64_t)win * a.K_cap + k1) * R + l]);
    else if (l == 32 || l == 33) g64 = (uint64_t)__double_as_longlong(a.n[(int64_t)(l - 32) * a.K_cap + k1]);
    else if (l == 34 && grp) g64 = (uint64_t)(uintptr_t)a.groups[d1.g0].src;
    else if (l == 35 && grp) g64 = (uint64_t)a.groups[d1.g0].out_row;
    else if (l == 36 && grp) g64 = *(const uint64_t *)&a.groups[d1.g0].nrows;
    else if ((l == 37 || l == 38) && it2 < n_items) g64 = ((const uint64_t *)(a.items + it2))[l - 37];
    if (l == 39) g32 = a.cur[(int64_t)gcur * a.K_cap + k1];
    else if (l == 40) g32 = (uint32_t)a.tlast[(int64_t)gcur * a.K_cap + k1];
  };
  auto put = [&](int slot, int dslot, uint64_t g64, uint32_t g32) {
    const int l = threadIdx.x & 63;
    if (l < 37) sMeta[slot][l] = g64;
    else if (l < 39) ((uint64_t *)&sDesc[dslot])[l - 37] = g64;
    else if (l < 41) ((uint32_t *)&sMeta[slot][37])[l - 39] = g32;
  };
  // the fast kernel takes the items blk, blk + nblk, ... (heaviest first, so
  // the static stride balances like a greedy list schedule)
  if constexpr (!SLOW) {
    if (threadIdx.x == 0 && blk < n_items) sDesc[0] = a.items[blk];
    __syncthreads();
    if (threadIdx.x < 64) {
      uint64_t g64;
      uint32_t g32;
      gather(blk, sDesc[0], blk + nblk, g64, g32);
      put(0, 1, g64, g32);
    }
  }
  for (int cnt = 0;; ++cnt) {
    __syncthreads();   // the previous slice is done with LDS; the look-ahead is stored
    if constexpr (SLOW) {
      if (threadIdx.x == 0) {
        const int q = atomicAdd(&a.queue[2], 1);
        sItem = (q < __atomic_load_n(&a.queue[1], __ATOMIC_RELAXED)) ? a.slow_list[q] : n_items;
        if (sItem < n_items) {
          const Item x = a.items[sItem];
          sNext[1] = x.slice;
          sNext[2] = x.g0;
          sNext[3] = x.g1;
          sNext[4] = x.rows;
        }
      }
      __syncthreads();
    }
    const int it = SLOW ? sItem : blk + cnt * nblk;
    if (it >= n_items) break;
    // the thread index, opaque to the compiler inside the loop: per-thread
    // address arithmetic is redone per slice instead of being hoisted out of
    // the loop into registers
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    const int lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    Item item;
    const int ms = cnt & 1;   // this item's slot of sMeta
    if constexpr (SLOW) {
      item.slice = sNext[1];
      item.g0 = sNext[2];
      item.g1 = sNext[3];
      item.rows = sNext[4];
    } else {
      item = sDesc[cnt % 3];
    }
    const int k = uni(item.slice);
    item.g0 = uni(item.g0);
    item.g1 = uni(item.g1);
    // the next item's state words and the descriptor after it, in flight
    // during this slice (wave 0)
    uint64_t g64 = 0;
    uint32_t g32 = 0;
    if (!SLOW && wv == 0) gather(it + nblk, sDesc[(cnt + 1) % 3], it + 2 * nblk, g64, g32);
    const bool is_new = k >= Kp;
    const uint32_t btl0 = SLOW ? 0u : ((const uint32_t *)&sMeta[ms][37])[0];
    const uint32_t btl1 = SLOW ? 0u : ((const uint32_t *)&sMeta[ms][37])[1];
    const int b = uni(SLOW ? (int)a.cur[(int64_t)gcur * a.K_cap + k] : (int)btl0);
    const int tl = uni(SLOW ? a.tlast[(int64_t)gcur * a.K_cap + k] : (int)btl1);
    const int64_t ybase = ((int64_t)b * a.K_cap + k) * a.ys;
    const int64_t ynext = ((int64_t)(1 - b) * a.K_cap + k) * a.ys;
    const int64_t dbase = ((int64_t)b * a.K_cap + k) * RR;
    const int64_t dnext = ((int64_t)(1 - b) * a.K_cap + k) * RR;
    // the stored state: loaded before the rows in the float32 path (the row
    // work hides its latency), after them in the mixed path (registers)
    float yo[RW][JW];
    float yl[MX ? RW : 1][MX ? JW : 1];
    float dold[4], dlo[4];
    // (a new slice's buffers have no bytes: every load returns zero)
    auto load_state = [&]() {
      const int yb = is_new ? 0 : R * J * 4, db = is_new ? 0 : RR * 4;
      const auto ry = buf_rsrc(a.Y + ybase, yb);
      const auto rd = buf_rsrc(a.D + dbase, db);
#pragma unroll
      for (int rr = 0; rr < RW; ++rr) {
        const int r = wv + 4 * rr;
        if (vecj) {
          buf_ldfn<JW>(ry, (r < R && lane * JW < J) ? (r * J + lane * JW) * 4 : kNoOff, yo[rr]);
        } else {
#pragma unroll
          for (int jj = 0; jj < JW; ++jj) {
            const int j = lane + 64 * jj;
            yo[rr][jj] = buf_ldf(ry, (r < R && j < J) ? (r * J + j) * 4 : kNoOff);
          }
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = tid + 256 * i;
        dold[i] = buf_ldf(rd, q < RR ? q * 4 : kNoOff);
      }
      if constexpr (MX) {
        // Y's compensation words are BF16 (the residual of the float32 word:
        // 8 more bits, 2^-33 relative per fold, half the bytes)
        const auto ryc = buf_rsrc(a.Yc + ybase, yb / 2);
        const auto rdc = buf_rsrc(a.Dc + dbase, db);
#pragma unroll
        for (int rr = 0; rr < RW; ++rr) {
          const int r = wv + 4 * rr;
          if (vecj) {
            buf_ldbfn<JW>(ryc, (r < R && lane * JW < J) ? (r * J + lane * JW) * 2 : kNoOff, yl[rr]);
          } else {
#pragma unroll
            for (int jj = 0; jj < JW; ++jj) {
              const int j = lane + 64 * jj;
              yl[rr][jj] = buf_ldbf(ryc, (r < R && j < J) ? (r * J + j) * 2 : kNoOff);
            }
          }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int q = tid + 256 * i;
          dlo[i] = buf_ldf(rdc, q < RR ? q * 4 : kNoOff);
        }
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) dlo[i] = 0.f;
      }
    };
    if (wv == 0) {
      // the weights Lemma 1 uses (1 for a new slice's first pass) and the
      // acceptance rule of its system S_k V^T V S_k
      const double w =
          (lane < R) ? ((is_new && a.pass == 0) ? 1.0
                        : SLOW ? a.W[((int64_t)win * a.K_cap + k) * R + lane]
                               : __longlong_as_double((long long)sMeta[ms][lane]))
                     : 0.0;
      const bool regular = SLOW || lemma1_regular(w, pivl, arrl, R);
      if (lane < R) {
        sW[lane] = w;
        sWinv[lane] = regular ? (float)(1.0 / w) : 0.f;
      }
      if (lane == 0) {
        sDefer = regular ? 0 : 1;
        if (!regular) a.slow_list[atomicAdd(&a.queue[1], 1)] = it;
      }
    }
    __syncthreads();
    if (!SLOW && sDefer) {
      if (wv == 0) put((cnt + 1) & 1, (cnt + 2) % 3, g64, g32);
      continue;
    }
    if constexpr (!MX) load_state();
    constexpr bool slow = SLOW;
    if (slow) {
      if (wv == 0)
        lemma1_pinv_matrix(vb.VtV, sW, R, sScr, sScr + RR, sScr + 2 * RR, sScr + 2 * RR + R,
                           (int *)(sScr + 2 * RR + R + 64), sZf, R);
      __syncthreads();
    }

    // Lemma 1 and the new-row sums on MFMA (FP32 16x16x4, or BF16 16x16x32
    // with FP32 sums in the mixed path); the dY, dD tiles stay in the waves'
    // accumulators over every block of the slice
    f32x4 accY[kMxTiles];
    f32x4 accD = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < kMxTiles; ++i) accY[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    double dn = 0.0;
    const int NTu = (R + 15) >> 4;
    for (int gi = item.g0; gi < item.g1; ++gi) {
      Group gr;
      if (!SLOW && gi == item.g0) {
        gr.src = (const float *)(uintptr_t)sMeta[ms][34];
        gr.out_row = (int64_t)sMeta[ms][35];
        gr.nrows = (int32_t)(uint32_t)sMeta[ms][36];
        gr.slice = k;
      } else {
        gr = a.groups[gi];
      }
      gr.src = uniptr(gr.src);
      gr.out_row = uni64(gr.out_row);
      gr.nrows = uni(gr.nrows);
      for (int r0 = 0; r0 < gr.nrows; r0 += MB) {
        const int m = min(MB, gr.nrows - r0);
        const int mp = MX ? (m + 31) & ~31 : (m + 15) & ~15;
        if constexpr (BF) {
          __syncthreads();
          dn += stage_rows_bf(gr.src + (int64_t)r0 * J, m, mp, J, LB, bXr, bXc, tid);
          __syncthreads();
          // U^T = P^T X^T per (row tile, rank tile) on BF16 MFMA: wave w takes
          // jobs w and w + 4; u = (x P) / w into U^T (BF16) and U_new
          const int jobs = (mp >> 4) * NTu;
#pragma unroll
          for (int jb = 0; jb < 2; ++jb) {
            const int job = wv + 4 * jb;
            if (job < jobs) {
              const int rt = job / NTu, nt = job - rt * NTu;
              const __bf16 *pa = bPt + (16 * nt + (lane & 15)) * LB.XS + 8 * (lane >> 4);
              const __bf16 *pb = bXr + (16 * rt + (lane & 15)) * LB.XS + 8 * (lane >> 4);
              f32x4 acc = {0.f, 0.f, 0.f, 0.f};
              for (int ks = 0; ks < LB.Jp; ks += 32)
                acc = mfma_bf16(*(const bf16x8 *)(pa + ks), *(const bf16x8 *)(pb + ks), acc);
              const int row = 16 * rt + (lane & 15);
              const auto ru = buf_rsrc(a.U_out + (gr.out_row + r0) * R, write_u ? m * R * 4 : 0);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const int r = 16 * nt + (lane >> 4) * 4 + q;
                const bool in = r < R && row < m;
                const float u = in ? acc[q] * sWinv[min(r, R - 1)] : 0.f;
                bUt[r * LB.XC + row] = (__bf16)u;
                buf_stf(ru, in ? (row * R + r) * 4 : kNoOff, u);
              }
            }
          }
          __syncthreads();
          // dY += U^T X, dD += U^T U: every operand eight consecutive rows
          const int MT = NTu, NT = (J + 15) >> 4;
          const int li = lane & 15, lk = 8 * (lane >> 4);
          for (int ks = 0; ks < mp; ks += 32) {
            bf16x8 au[2];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
              au[mt] = (mt < MT) ? *(const bf16x8 *)(bUt + (16 * mt + li) * LB.XC + ks + lk) : bf16x8{};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              const int nt = wv + 4 * c;
              if (nt < NT) {
                const bf16x8 bv = *(const bf16x8 *)(bXc + (16 * nt + li) * LB.XC + ks + lk);
                accY[2 * c] = mfma_bf16(au[0], bv, accY[2 * c]);
                if (MT > 1) accY[2 * c + 1] = mfma_bf16(au[1], bv, accY[2 * c + 1]);
              }
            }
            if (wv < MT * MT) {
              const int mt = wv / MT, st = wv - mt * MT;
              accD = mfma_bf16(mt == 0 ? au[0] : au[1], st == 0 ? au[0] : au[1], accD);
            }
          }
          continue;
        }
        __syncthreads();
        dn += stage_rows<true>(gr.src + (int64_t)r0 * J, m, J, XS, sX, tid);
        zero_block_pad(sX, XS, m, mp, J, L.J16, tid);
        __syncthreads();
        // t = x P per (row tile, rank tile): wave w takes jobs w and w + 4;
        // U's columns R .. 16 NTu - 1 come out zero
        const int jobs = (mp >> 4) * NTu;
        const auto ru = buf_rsrc(a.U_out + (gr.out_row + r0) * R, (write_u && !slow) ? m * R * 4 : 0);
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
          const int job = wv + 4 * jb;
          if (job < jobs) {
            const int rt = job / NTu, nt = job - rt * NTu;
            const float *xr = sX + (16 * rt + (lane & 15)) * XS;
            const float *pr = sP + (16 * nt + (lane & 15)) * XS;
            f32x4 acc;
            if constexpr (MX)
              acc = rows_times_pt_bf(xr, pr, J, lane);
            else
              acc = rows_times_pt(xr, pr, L.J16, lane >> 4);
            const int n = nt * 16 + (lane & 15);
            const float wi = sWinv[min(n, R - 1)];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int rr = 16 * rt + (lane >> 4) * 4 + q;
              const bool in = rr < m && n < R;
              if (slow) {
                sU[rr * L.US + n] = in ? acc[q] : 0.f;
              } else {
                const float u = in ? acc[q] * wi : 0.f;
                sU[rr * L.US + n] = u;
                buf_stf(ru, in ? (rr * R + n) * 4 : kNoOff, u);
              }
            }
          }
        }
        if (slow) {
          // u = t Z, row by row (at most 8 entries per thread)
          __syncthreads();
          float uq[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int e = tid + 256 * i;
            uq[i] = 0.f;
            if (e < mp * R) {
              const int row = e / R, n = e - row * R;
              float acc = 0.f;
              for (int mm = 0; mm < R; ++mm) acc = fmaf(sU[row * L.US + mm], sZf[mm * R + n], acc);
              uq[i] = (row < m) ? acc : 0.f;
            }
          }
          __syncthreads();
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const int e = tid + 256 * i;
            if (e < mp * R) {
              const int row = e / R, n = e - row * R;
              sU[row * L.US + n] = uq[i];
              if (write_u && row < m) a.U_out[(gr.out_row + r0 + row) * R + n] = uq[i];
            }
          }
        }
        __syncthreads();
        if constexpr (MX)
          accum_block_mx(sX, sU, XS, L.US, mp, J, R, accY, accD, tid);
        else
          accum_block_f32(sX, sU, XS, L.US, mp, J, R, accY, accD, tid);
      }
    }
    if constexpr (MX) load_state();
    // hand the tiles to the [rank][column] layout through LDS
    __syncthreads();
    float *sDY = sX;   // R x J
    float *sDD = BF ? (float *)(smem + LB.oDD) : sU;   // R x R
    {
      const int li = lane & 15;
      const int MT = (R + 15) >> 4, NT = (J + 15) >> 4;
#pragma unroll
      for (int i = 0; i < kMxTiles; ++i) {
        const int c = i >> 1, mt = i & 1;
        const int nt = wv + 4 * c;
        if (nt >= NT || mt >= MT) continue;
        const int j = nt * 16 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = mt * 16 + (lane >> 4) * 4 + q;
          if (r < R && j < J) sDY[r * J + j] = accY[i][q];
        }
      }
      if (wv < MT * MT) {
        const int mt = wv / MT, st = wv - mt * MT;
        const int cc = st * 16 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = mt * 16 + (lane >> 4) * 4 + q;
          if (r < R && cc < R) sDD[r * R + cc] = accD[q];
        }
      }
    }
    dn = wave_sum(dn);
    if (lane == 0) sDn[wv] = dn;
    __syncthreads();

    // fold: Y_k = lambda^dt Y_k,stored + dY into the spare buffer; c_k
    const double s_old = is_new ? 0.0 : exp2((double)(step - tl) * a.log2_lambda);
    const float s_old_f = (float)s_old;
    double cpart[RW];
    {
      const auto wy = buf_rsrc(a.Y + ynext, R * J * 4);
      const auto wyc = buf_rsrc(MX ? (const void *)(a.Yc + ynext) : (const void *)a.Y, MX ? R * J * 2 : 0);
      const bool lag = a.lagged;
#pragma unroll
      for (int rr = 0; rr < RW; ++rr) {
        const int r = wv + 4 * rr;
        cpart[rr] = 0.0;
        float yv[JW], lo[JW];
#pragma unroll
        for (int jj = 0; jj < JW; ++jj) {
          const int j = vecj ? lane * JW + jj : lane + 64 * jj;
          const bool in = r < R && j < J;
          const float dyl = sDY[min(r, R - 1) * J + min(j, J - 1)];
          const float dy = in ? dyl : 0.f;
          double cv;
          if constexpr (MX) {
            // compensated running sum: (hi, lo) folded in FP64 and split again
            const double v = s_old * ((double)yo[rr][jj] + (double)yl[rr][jj]) + (double)dy;
            const float hi = (float)v;
            yv[jj] = hi;
            lo[jj] = (float)(v - (double)hi);
            cv = lag ? (double)dy : v;
          } else {
            yv[jj] = fmaf(s_old_f, yo[rr][jj], dy);
            lo[jj] = 0.f;
            cv = lag ? (double)dy : (double)yv[jj];
          }
          // V^T's entry converted here, not hoisted out of the slice loop
          // as 32 more double registers
          float vtc = vt[rr][jj];
          asm volatile("" : "+v"(vtc));
          cpart[rr] = fma(cv, (double)vtc, cpart[rr]);
        }
        if (vecj) {
          const bool in = r < R && lane * JW < J;
          buf_stfn<JW>(wy, in ? (r * J + lane * JW) * 4 : kNoOff, yv);
          if constexpr (MX) buf_stbfn<JW>(wyc, in ? (r * J + lane * JW) * 2 : kNoOff, lo);
        } else {
#pragma unroll
          for (int jj = 0; jj < JW; ++jj) {
            const int j = lane + 64 * jj;
            const bool in = r < R && j < J;
            buf_stf(wy, in ? (r * J + j) * 4 : kNoOff, yv[jj]);
            if constexpr (MX) buf_stbf(wyc, in ? (r * J + j) * 2 : kNoOff, lo[jj]);
          }
        }
      }
    }
    // c_r: each wave sums its ranks' partials across lanes through LDS (the
    // row block, dead after the fold): lanes 8 rr .. 8 rr + 7 add eight
    // partials each, then three exchanges
    __syncthreads();
    double *sCp = (double *)sX + wv * (RW * 64);
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) sCp[rr * 64 + lane] = cpart[rr];
    wave_sync();
    double csum = 0.0;
    if (lane < RW * 8) {
      const double *src = sCp + (lane >> 3) * 64 + (lane & 7) * 8;
#pragma unroll
      for (int u = 0; u < 8; ++u) csum += src[u];
    }
    csum += __shfl_xor(csum, 1, 64);
    csum += __shfl_xor(csum, 2, 64);
    csum += __shfl_xor(csum, 4, 64);
#pragma unroll
    for (int rr = 0; rr < RW; ++rr) {
      const int r = wv + 4 * rr;
      const double part = __shfl(csum, rr * 8, 64);
      if (lane == 0 && r < R) {
        if (a.lagged) {
          // eq. [obtain_CandC]: the stored c_k decayed, plus diag(U^T X V)
          const double cold = is_new ? 0.0 : a.cst[((int64_t)b * a.K_cap + k) * R + r];
          const double cc = fma(s_old, cold, part);
          a.cst[((int64_t)(1 - b) * a.K_cap + k) * R + r] = cc;
          a.cbuf[(int64_t)k * R + r] = cc;
        } else {
          a.cbuf[(int64_t)k * R + r] = part;
        }
      }
    }
    {
      const auto wd = buf_rsrc(a.D + dnext, RR * 4);
      const auto wdc = buf_rsrc(MX ? a.Dc + dnext : a.D, MX ? RR * 4 : 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = tid + 256 * i;
        const float dd = sDD[min(q, RR - 1)];
        const int off = q < RR ? q * 4 : kNoOff;
        if constexpr (MX) {
          const double v = s_old * ((double)dold[i] + (double)dlo[i]) + (double)dd;
          const float hi = (float)v;
          buf_stf(wd, off, hi);
          buf_stf(wdc, off, (float)(v - (double)hi));
        } else {
          buf_stf(wd, off, fmaf(s_old_f, dold[i], dd));
        }
      }
    }
    if (tid == 0) {
      const double nold = is_new ? 0.0
                          : SLOW ? a.n[(int64_t)b * a.K_cap + k]
                                 : __longlong_as_double((long long)sMeta[ms][32 + b]);
      a.n[(int64_t)(1 - b) * a.K_cap + k] = s_old * nold + (((sDn[0] + sDn[1]) + sDn[2]) + sDn[3]);
      a.tag[k] = seq;
    }
    if (!SLOW && wv == 0) put((cnt + 1) & 1, (cnt + 2) % 3, g64, g32);
  }
}

// ---------------------------------------------------------------------------
// Solve stage
// ---------------------------------------------------------------------------
struct SolveLds {
  size_t oVtV, oVt, oW, oScr, bytes;
  int vts;   // row stride of V^T in LDS (floats)
};

constexpr int kSolveWaves = 4;   // waves of a solve workgroup

// V^T V (FP64, row stride R + 1), V^T (float, row stride J + 4: the rows a
// lane group reads side by side fall in different banks), a deferred slice's
// w, and a scratch shared by the pseudo-inverse of deferred slices, their G
// terms and the final combination of the waves' G partials.
__host__ __device__ inline SolveLds solve_lds(int J, int R) {
  SolveLds L;
  L.vts = J + 4;
  size_t o = 0;
  L.oVtV = o;
  o += (size_t)R * (R + 1) * 8;
  L.oVt = o = align_up(o, 16);
  o = align_up(o + (size_t)R * L.vts * 4, 16);
  L.oW = o;
  o += (size_t)R * 8;
  L.oScr = o;
  const size_t pinv = (size_t)(2 * R * R + 2 * R + 3 * 64) * 8 + 64 * 4;
  // pseudo-inverse scratch, deferred G, combined G; during the solve loop the
  // same space holds each lane group's D_k rows (solve_drows_bytes)
  const size_t scr = pinv + (size_t)2 * (R * R + 1) * 8;
  const size_t rm = R <= 8 ? 8 : (R <= 16 ? 16 : 32);
  const size_t drows = (size_t)kSolveWaves * 64 * (rm + 1) * 4;
  o += scr > drows ? scr : drows;
  L.bytes = align_up(o, 16);
  return L;
}

// One slice's state as the solve stage sees it.
struct SolveSlice {
  int b, tl;
  bool touched;
  double sig;
  const float *Dp, *Dcp, *Yk;
};

__device__ inline SolveSlice solve_slice(CPassArgs &a, int k, int gcur, int64_t step, int seq, bool upd, int RR) {
  SolveSlice x;
  x.b = a.cur[(int64_t)gcur * a.K_cap + k];
  x.tl = a.tlast[(int64_t)gcur * a.K_cap + k];
  x.touched = upd && a.tag[k] == seq;
  const int bs = x.touched ? 1 - x.b : x.b;
  x.sig = x.touched ? 1.0 : exp2((double)(step - x.tl) * a.log2_lambda);
  x.Dp = a.D + ((int64_t)bs * a.K_cap + k) * RR;
  x.Dcp = a.Dc ? a.Dc + ((int64_t)bs * a.K_cap + k) * RR : nullptr;
  x.Yk = a.Y + ((int64_t)x.b * a.K_cap + k) * a.ys;
  return x;
}

// c_r = sum_j Y_k[r][j] V[j][r] for one row: FP64 sum of the float products in
// column order; float4 loads, eight in flight, when rows are 16-byte aligned.
__device__ inline double row_c(const float *__restrict__ yr, const float *vr, int J) {
  double p = 0.0;
  if ((J & 3) == 0) {
    const float4 *y4 = reinterpret_cast<const float4 *>(yr);
    const float4 *v4 = reinterpret_cast<const float4 *>(vr);
    const int J4 = J >> 2;
    for (int t0 = 0; t0 < J4; t0 += 8) {
      float4 y[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) y[u] = (t0 + u < J4) ? y4[t0 + u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (t0 + u < J4) {
          const float4 v = v4[t0 + u];
          p = fma((double)y[u].x, (double)v.x, p);
          p = fma((double)y[u].y, (double)v.y, p);
          p = fma((double)y[u].z, (double)v.z, p);
          p = fma((double)y[u].w, (double)v.w, p);
        }
      }
    }
  } else {
    for (int j = 0; j < J; ++j) p = fma((double)yr[j], (double)vr[j], p);
  }
  return p;
}

// c_k of Lemma 2, row r (update pass): the row stage's sums for a touched
// slice, the lagged recursion's stored value, or diag(Y_k V).
__device__ inline double solve_c_row(CPassArgs &a, const SolveSlice &x, int k, int J, int R, int r, const float *sVt,
                                     int vts) {
  if (r >= R) return 0.0;
  if (x.touched) return a.cbuf[(int64_t)k * R + r];
  if (a.lagged) return a.cst[((int64_t)x.b * a.K_cap + k) * R + r];
  return row_c(x.Yk + r * J, sVt + r * vts, J);
}

// Row r of D_k (plus its compensation word), as doubles, 0 beyond R.
template <int RM>
__device__ __forceinline__ void load_d_row(const SolveSlice &x, int R, int r, double (&d)[RM]) {
  if ((R & 3) == 0) {
    const float4 *d4 = reinterpret_cast<const float4 *>(x.Dp + r * R);
    const float4 *e4 = x.Dcp ? reinterpret_cast<const float4 *>(x.Dcp + r * R) : nullptr;
#pragma unroll
    for (int c4 = 0; c4 < RM / 4; ++c4) {
      const bool in = r < R && 4 * c4 < R;
      const float4 v = in ? d4[c4] : make_float4(0.f, 0.f, 0.f, 0.f);
      const float4 e = (in && e4) ? e4[c4] : make_float4(0.f, 0.f, 0.f, 0.f);
      d[4 * c4 + 0] = (double)v.x + (double)e.x;
      d[4 * c4 + 1] = (double)v.y + (double)e.y;
      d[4 * c4 + 2] = (double)v.z + (double)e.z;
      d[4 * c4 + 3] = (double)v.w + (double)e.w;
    }
  } else {
#pragma unroll
    for (int c = 0; c < RM; ++c)
      d[c] = (r < R && c < R) ? (double)x.Dp[r * R + c] + (x.Dcp ? (double)x.Dcp[r * R + c] : 0.0) : 0.0;
  }
}

// Row r of D_k and its compensation words as loaded (R a multiple of 4):
// issued early, converted where the row is used.
template <int RM>
struct DRowRaw {
  float4 v[RM / 4], e[RM / 4];
};

template <int RM>
__device__ __forceinline__ void load_d_row_raw(const SolveSlice &x, int R, int r, DRowRaw<RM> &o) {
  const float4 *d4 = reinterpret_cast<const float4 *>(x.Dp + min(r, R - 1) * R);
  const float4 *e4 = x.Dcp ? reinterpret_cast<const float4 *>(x.Dcp + min(r, R - 1) * R) : d4;
#pragma unroll
  for (int c4 = 0; c4 < RM / 4; ++c4) {
    const int cc = min(c4, R / 4 - 1);
    o.v[c4] = d4[cc];
    o.e[c4] = e4[cc];
  }
}

template <int RM>
__device__ __forceinline__ void d_row_from_raw(const DRowRaw<RM> &o, bool comp, int R, int r, double (&d)[RM]) {
#pragma unroll
  for (int c4 = 0; c4 < RM / 4; ++c4) {
    const bool in = r < R && 4 * c4 < R;
    const float4 v = o.v[c4], e = o.e[c4];
    d[4 * c4 + 0] = in ? (double)v.x + (comp ? (double)e.x : 0.0) : 0.0;
    d[4 * c4 + 1] = in ? (double)v.y + (comp ? (double)e.y : 0.0) : 0.0;
    d[4 * c4 + 2] = in ? (double)v.z + (comp ? (double)e.z : 0.0) : 0.0;
    d[4 * c4 + 3] = in ? (double)v.w + (comp ? (double)e.w : 0.0) : 0.0;
  }
}

// Gauss-Jordan of one group of RM lanes: lane base + r holds row r of an
// RM x RM system (rows n .. RM - 1 are padding) and entry r of the right-hand
// side; pivot rows are exchanged within the group.  The acceptance rule of the
// oracle's Cholesky: every pivot of a real row above kPivotRel times the
// largest diagonal entry (ok is uniform over the group; a failing group runs
// on harmlessly).  On ok, x_r = b / d.
template <int RM>
__device__ __forceinline__ bool group_gj(double (&m)[RM], double &b, double &d, int n, int base, int r) {
  double diag = 0.0;
#pragma unroll
  for (int c = 0; c < RM; ++c) diag = (c == r) ? m[c] : diag;
  double dmax = (r < n) ? diag : 0.0;
#pragma unroll
  for (int o = 1; o < RM; o <<= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
  bool ok = dmax > 0.0;
  const double thr = kPivotRel * dmax;
  const double pad = ok ? dmax : 1.0;
#pragma unroll
  for (int c = 0; c < RM; ++c) m[c] = (r >= n) ? ((c == r) ? pad : 0.0) : m[c];
  d = 1.0;
#pragma unroll
  for (int p = 0; p < RM; ++p) {
    double piv = __shfl(m[p], base + p, 64);
    ok = ok && (p >= n || piv > thr);
    piv = (piv > 0.0) ? piv : 1.0;
    d = (r == p) ? piv : d;
    const double f = (r != p) ? m[p] / piv : 0.0;
#pragma unroll
    for (int c = p + 1; c < RM; ++c) m[c] = fma(-f, __shfl(m[c], base + p, 64), m[c]);
    b = fma(-f, __shfl(b, base + p, 64), b);
  }
  return ok;
}

// The deferred slices of a solve chunk (systems that failed the acceptance
// rule), in slice order, by one wave: the eigen pseudo-inverse in the shared
// scratch; their G terms go to sGd (LDS, RR entries) and their n to *nd_sum.
__device__ inline void solve_deferred(CPassArgs &a, int32_t *sDef, int nd, int gcur, int wout, int64_t step, int seq,
                                      bool upd, bool do_g, const double *sVtV, const float *sVt, int vts, double *sScr,
                                      double *sw, double *sGd, double *nd_sum) {
  const int lane = threadIdx.x & 63;
  const int J = a.J, R = a.R, RR = R * R;
  if (lane == 0)
    for (int i = 1; i < nd; ++i)   // insertion sort: the list is short
      for (int j = i; j > 0 && sDef[j - 1] > sDef[j]; --j) {
        const int t = sDef[j];
        sDef[j] = sDef[j - 1];
        sDef[j - 1] = t;
      }
  for (int q = lane; q < RR; q += 64) sGd[q] = 0.0;
  double *sM = sScr, *sZ = sM + RR, *sx = sZ + RR, *sTmp = sx + 2 * R, *sRot = sTmp + 64;
  int *sPair = (int *)(sRot + 128);
  double nsum = 0.0;
  for (int i = 0; i < nd; ++i) {
    int k = lane == 0 ? sDef[i] : 0;   // lane 0 sorted the list: its view is current
    k = __shfl(k, 0, 64);
    const SolveSlice x = solve_slice(a, k, gcur, step, seq, upd, RR);
    const double c = solve_c_row(a, x, k, J, R, lane, sVt, vts);
    for (int q = lane; q < RR; q += 64) {
      const int r = q / R, cc = q - r * R;
      sM[q] = sVtV[r * (R + 1) + cc] * ((double)x.Dp[q] + (x.Dcp ? (double)x.Dcp[q] : 0.0));
    }
    if (lane < R) sx[lane] = c;
    wave_sync();
    wave_pinv_apply(sM, sx, R, sZ, sTmp, sRot, sPair);
    const double w = lane < R ? sx[lane] : 0.0;
    if (lane < R) {
      a.W[((int64_t)wout * a.K_cap + k) * R + lane] = w;
      sw[lane] = w;
    }
    if (lane == 0) {
      a.cur[(int64_t)(1 - gcur) * a.K_cap + k] = (uint8_t)(x.touched ? 1 - x.b : x.b);
      a.tlast[(int64_t)(1 - gcur) * a.K_cap + k] = x.touched ? (int32_t)step : x.tl;
    }
    wave_sync();
    if (do_g)
      for (int q = lane; q < RR; q += 64) {
        const int r = q / R, s2 = q - r * R;
        const double d = (double)x.Dp[q] + (x.Dcp ? (double)x.Dcp[q] : 0.0);
        sGd[q] = fma(x.sig * sw[r] * sw[s2], d, sGd[q]);
      }
    nsum = fma(x.sig, a.n[(int64_t)(x.touched ? 1 - x.b : x.b) * a.K_cap + k], nsum);
    wave_sync();
  }
  if (lane == 0) *nd_sum = nsum;
}

// mode 0 (update pass) or 1 (evaluation of the committed state: w_k is the
// committed W, no solve; in lagged mode c_k = diag(Y_k V) is stored as the
// recursion's starting value).  Workgroup = one solve chunk of kSolveWaves
// waves; a wave splits into 64 / RM lane groups, each taking one slice at a
// time (lane r of a group owns row r of the slice's R x R system, its c_r, its
// w_r and row r of its G terms), so 64 / RM slices are in flight per wave and
// no workgroup barrier separates slices.  Group g of wave v takes the chunk's
// slices v S + g + 4 S i (S = 64 / RM).  Each lane keeps its G row partial in
// registers; at the end the groups of a wave are summed by a fixed exchange
// tree, then the waves in order, then the deferred slices (systems that
// failed the acceptance rule) are listed in the chunk's range of the row
// stage's deferred-slice array (free once that stage is done) and solved by
// the next launch.
template <int RM>
__device__ __forceinline__ void solve_body(const PassArgs *args, const BlockMap *map) {
  constexpr int S = 64 / RM;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sNDef;
  __shared__ double sN[kSolveWaves];
  CPassArgs &a = *(CPassArgs *)(map ? map[blockIdx.x].args : args);
  const int blk = map ? map[blockIdx.x].local : (int)blockIdx.x;
  const StepHeader *h = a.hdr;
  const int J = a.J, R = a.R, RR = R * R;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane % RM, grp = lane / RM, base = grp * RM;
  const int K = h->K, seq = h->seq;
  const int64_t step = h->step;
  const int gcur = a.ctl->gcur;
  const int win = (a.pass == 0) ? gcur : 1 - gcur;
  const int wout = 1 - gcur;
  const bool upd = a.mode == 0;
  const VBundleView vb = vb_view(a.vb + (int64_t)(upd ? win : gcur) * a.vb_stride, J, R);
  const SolveLds L = solve_lds(J, R);
  double *sVtV = (double *)(smem + L.oVtV);
  float *sVt = (float *)(smem + L.oVt);
  double *sScr = (double *)(smem + L.oScr);
  double *sG = sScr;   // the waves' combined G
  // this lane group's D_k rows (row stride RM + 1: the lanes of a wave fall in
  // distinct banks), kept from the system's load for the G terms
  float *sD = (float *)sScr + (wv * S + grp) * RM * (RM + 1) + r * (RM + 1);
  const int chunk2 = blk;
  const int k0 = chunk2 * h->chunk2;
  const int k1 = min(K, k0 + h->chunk2);
  int32_t *sDef = a.slow_list + k0;   // at most k1 - k0 entries
  // the row stage has finished: its counters are free for the next launch
  if (upd && chunk2 == 0 && tid < 3) a.queue[tid] = 0;
  const bool need_c = upd ? !a.lagged : (a.lagged != 0);
  for (int e = tid; e < RR; e += blockDim.x) sVtV[(e / R) * (R + 1) + e % R] = vb.VtV[e];
  if (need_c)
    for (int e = tid; e < R * J; e += blockDim.x) sVt[(e / J) * L.vts + e % J] = vb.Vt32[e];
  if (tid == 0) sNDef = 0;
  __syncthreads();

  double gacc[RM];
#pragma unroll
  for (int i = 0; i < RM; ++i) gacc[i] = 0.0;
  double nacc = 0.0;
  const bool do_g = !a.lagged || !upd;

  for (int kb = k0 + wv * S; kb < k1; kb += kSolveWaves * S) {
    const int k = kb + grp;
    if (k < k1) {
      const SolveSlice x = solve_slice(a, k, gcur, step, seq, upd, RR);
      double w = 0.0;
      bool use = true;
      // n_k goes out with the first loads of the slice (the 32-rank kernel,
      // short of registers, loads it where it is used)
      double nk = 0.0;
      if (RM < 32 && r == 0) nk = a.n[(int64_t)(x.touched ? 1 - x.b : x.b) * a.K_cap + k];
      if (upd) {
        // the D row too (R a multiple of 4, and only where the registers
        // allow it without spills or a lower occupancy: the 16-rank kernel):
        // one round trip with the first c_k loads instead of one after them;
        // the empty asm keeps these loads ahead of the dot products
        const bool raw = RM == 16 && (R & 3) == 0;
        DRowRaw<RM> dr;
        if (raw) load_d_row_raw<RM>(x, R, r, dr);
        asm volatile("" ::: "memory");
        double b = solve_c_row(a, x, k, J, R, r, sVt, L.vts);
        // Lemma 2: (V^T V * D_k) w = c
        double m[RM];
        if (raw)
          d_row_from_raw<RM>(dr, x.Dcp != nullptr, R, r, m);
        else
          load_d_row<RM>(x, R, r, m);
        if (do_g) {
          // D_k's row rounded to float (the mixed path's (hi, lo) pair to its
          // nearest float, the G terms' FP32 operand); zeros beyond R
#pragma unroll
          for (int c = 0; c < RM; ++c) sD[c] = (float)m[c];
        }
#pragma unroll
        for (int c = 0; c < RM; ++c) m[c] = (r < R && c < R) ? sVtV[r * (R + 1) + c] * m[c] : 0.0;
        double dpiv;
        const bool ok = group_gj<RM>(m, b, dpiv, R, base, r);
        if (!ok) {
          if (r == 0) sDef[atomicAdd(&sNDef, 1)] = k;
          use = false;
        } else {
          w = r < R ? b / dpiv : 0.0;
          if (r < R) a.W[((int64_t)wout * a.K_cap + k) * R + r] = w;
          if (r == 0) {
            a.cur[(int64_t)(1 - gcur) * a.K_cap + k] = (uint8_t)(x.touched ? 1 - x.b : x.b);
            a.tlast[(int64_t)(1 - gcur) * a.K_cap + k] = x.touched ? (int32_t)step : x.tl;
          }
        }
      } else {
        if (a.lagged && r < R)
          a.cst[((int64_t)x.b * a.K_cap + k) * R + r] = row_c(x.Yk + r * J, sVt + r * L.vts, J);
        w = r < R ? a.W[((int64_t)gcur * a.K_cap + k) * R + r] : 0.0;
      }
      if (use) {
        // row r of G += sigma_k diag(w_k) D_k diag(w_k)
        if (do_g) {
          double d[RM];
          if (upd) {
#pragma unroll
            for (int i = 0; i < RM; ++i) d[i] = (double)sD[i];
          } else {
            load_d_row<RM>(x, R, r, d);
          }
          const double sr = x.sig * w;
#pragma unroll
          for (int i = 0; i < RM; ++i) {
            const double wi = __shfl(w, base + i, 64);
            gacc[i] = fma(sr * wi, d[i], gacc[i]);
          }
        }
        if (r == 0) {
          if (RM == 32) nk = a.n[(int64_t)(x.touched ? 1 - x.b : x.b) * a.K_cap + k];
          nacc = fma(x.sig, nk, nacc);
        }
      }
    }
  }
  // the groups of this wave: a fixed exchange tree
#pragma unroll
  for (int o = RM; o < 64; o <<= 1) {
#pragma unroll
    for (int i = 0; i < RM; ++i) gacc[i] += __shfl_xor(gacc[i], o, 64);
    nacc += __shfl_xor(nacc, o, 64);
  }
  // the waves' partials in wave order (lanes 0 .. R - 1 of each hold the rows),
  // once every wave is done with its D_k rows in the same space
  __syncthreads();
  for (int v = 0; v < kSolveWaves; ++v) {
    if (wv == v && lane < R) {
#pragma unroll
      for (int i = 0; i < RM; ++i)
        if (i < R) sG[lane * R + i] = (v == 0) ? gacc[i] : sG[lane * R + i] + gacc[i];
    }
    if (wv == v && lane == 0) sN[v] = nacc;
    __syncthreads();
  }
  double *p2 = a.part2 + (int64_t)chunk2 * (RR + 1);
  for (int q = tid; q < RR; q += blockDim.x) p2[q] = sG[q];
  if (tid == 0) {
    double n = 0.0;
    for (int v = 0; v < kSolveWaves; ++v) n += sN[v];
    p2[RR] = n;
    a.solve_defer[chunk2] = sNDef;   // the next launch solves these
  }
}

// The deferred systems of each solve chunk (launched after the solve stage,
// one workgroup per chunk): wave 0 solves them in slice order by the
// pseudo-inverse and adds their G and n terms to the chunk's partial after the
// waves' terms.  Chunks without deferred systems leave at once.
__global__ __launch_bounds__(64 * kSolveWaves) void k_solve_fix(const PassArgs *args, const BlockMap *map) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double sNd;
  CPassArgs &a = *(CPassArgs *)(map ? map[blockIdx.x].args : args);
  const int chunk2 = map ? map[blockIdx.x].local : (int)blockIdx.x;
  const int nd = a.solve_defer[chunk2];
  if (nd == 0) return;
  const StepHeader *h = a.hdr;
  const int J = a.J, R = a.R, RR = R * R;
  const int tid = threadIdx.x, wv = tid >> 6;
  const int seq = h->seq;
  const int64_t step = h->step;
  const int gcur = a.ctl->gcur;
  const int win = (a.pass == 0) ? gcur : 1 - gcur;
  const bool upd = a.mode == 0;
  const VBundleView vb = vb_view(a.vb + (int64_t)(upd ? win : gcur) * a.vb_stride, J, R);
  const SolveLds L = solve_lds(J, R);
  double *sVtV = (double *)(smem + L.oVtV);
  float *sVt = (float *)(smem + L.oVt);
  double *sw = (double *)(smem + L.oW);
  double *sScr = (double *)(smem + L.oScr);
  double *sGd = sScr + (size_t)(2 * R * R + 2 * R + 3 * 64) + 32;
  for (int e = tid; e < RR; e += blockDim.x) sVtV[(e / R) * (R + 1) + e % R] = vb.VtV[e];
  if (upd && !a.lagged)
    for (int e = tid; e < R * J; e += blockDim.x) sVt[(e / J) * L.vts + e % J] = vb.Vt32[e];
  __syncthreads();
  const int k0 = chunk2 * h->chunk2;
  if (wv == 0)
    solve_deferred(a, a.slow_list + k0, nd, gcur, 1 - gcur, step, seq, upd, !a.lagged || !upd, sVtV, sVt, L.vts,
                   sScr, sw, sGd, &sNd);
  __syncthreads();
  double *p2 = a.part2 + (int64_t)chunk2 * (RR + 1);
  for (int q = tid; q < RR; q += blockDim.x) p2[q] += sGd[q];
  if (tid == 0) p2[RR] += sNd;
}

template <int RM>
__global__ __launch_bounds__(64 * kSolveWaves, 2) void k_solve(const PassArgs *args, const BlockMap *map) {
  solve_body<RM>(args, map);
}

// ---------------------------------------------------------------------------
// F stage, exact mode: F^T = sum_k sigma_k diag(w_k) Y_k over every slice of
// the chunk, streamed as float4 from the flat R x J layout.  512 threads; TPS
// threads per slice (a power of two, <= 512), 512 / TPS slices side by side,
// up to two slices per thread group in flight; each thread owns the float4
// positions q = tq + TPS e (e < EPT) of a slice.
// ---------------------------------------------------------------------------
constexpr int kFsumThreads = 512;
constexpr int kFsumBatch = 64;   // slices whose weights are staged at a time

__host__ __device__ inline int fsum_tps(int ys) {
  const int nq = ys / 4;
  if (nq > kFsumThreads) return kFsumThreads;
  int tps = 1;
  while (tps < nq) tps <<= 1;
  return tps;
}

// WHOLE: J is a multiple of 4, so each float4 of a slice lies in one row of
// Y_k (one weight); otherwise every float's row is found where it is used
// (a separate kernel, so that this code does not weigh on the common one's
// registers).
template <int EPT, bool WHOLE>
__device__ __forceinline__ void fsum_body(const PassArgs *args, const BlockMap *map) {
  extern __shared__ __align__(16) unsigned char smem[];
  CPassArgs &a = *(CPassArgs *)(map ? map[blockIdx.x].args : args);
  const int blk = map ? map[blockIdx.x].local : (int)blockIdx.x;
  const int tps = fsum_tps(a.ys);
  __shared__ int sflag;
  __shared__ int sb[kFsumBatch];
  const StepHeader *h = a.hdr;
  const int J = a.J, R = a.R, RR = R * R, RJ = R * J;
  const int tid = threadIdx.x;
  const int K = h->K;
  const int64_t step = h->step;
  const int gcur = a.ctl->gcur;
  const bool upd = a.mode == 0;
  const int bsel = upd ? 1 - gcur : gcur;   // bookkeeping of the pass's state
  const int wsel = upd ? 1 - gcur : gcur;   // the pass's weights
  const int chunk = blk;
  const int k0 = chunk * h->chunk;
  const int k1 = min(K, k0 + h->chunk);
  double *sw = (double *)smem;   // [kFsumBatch][R]: sigma_k w_k
  const int spi = kFsumThreads / tps, sg = tid / tps, tq = tid - sg * tps;
  const int nq = a.ys >> 2;
  // the row of this thread's float4 e (WHOLE)
  int r0[EPT];
#pragma unroll
  for (int e = 0; e < EPT; ++e) r0[e] = min(4 * (tq + tps * e) / max(J, 1), R - 1);
  double acc[EPT][4];
#pragma unroll
  for (int e = 0; e < EPT; ++e)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[e][c] = 0.0;

  for (int kb = k0; kb < k1; kb += kFsumBatch) {
    const int nb = min(kFsumBatch, k1 - kb);
    __syncthreads();
    // sigma_k w_k of the batch's slices and their buffers: a thread's loads
    // (four entries at a time) all go out before their first use
    for (int e0 = tid; e0 < nb * R; e0 += 4 * kFsumThreads) {
      int tl[4];
      double wv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = min(e0 + u * kFsumThreads, nb * R - 1);
        const int i = e / R, r = e - i * R, k = kb + i;
        tl[u] = a.tlast[(int64_t)bsel * a.K_cap + k];
        wv[u] = a.W[((int64_t)wsel * a.K_cap + k) * R + r];
      }
      const int ib = min(e0, nb - 1);
      const int cb = a.cur[(int64_t)bsel * a.K_cap + kb + ib];
      if (e0 < nb) sb[e0] = cb;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int e = e0 + u * kFsumThreads;
        if (e < nb * R) sw[e] = exp2((double)(step - tl[u]) * a.log2_lambda) * wv[u];
      }
    }
    __syncthreads();
    // Two slices per thread group per step where the registers allow it,
    // and the next step's slices loaded while this step's are summed.  A
    // slice's Y comes through a bounds-checked buffer of its a.ys floats: the
    // lanes beyond it, and a missing second slice, read zeros.
    constexpr int NS = EPT <= 2 ? 2 : 1;
    struct V4 {
      float4 v[EPT];
    };
    // (a thread group may be narrower than a wave, so the slice address is
    // per lane: plain loads from clamped addresses; what a lane loads beyond
    // its slice, or for a slice past the batch, is never summed)
    auto load = [&](int i) {
      V4 o;
      const int ic = min(i, nb - 1);
      const float4 *y = (const float4 *)(a.Y + ((int64_t)sb[ic] * a.K_cap + kb + ic) * a.ys);
#pragma unroll
      for (int e = 0; e < EPT; ++e) o.v[e] = y[min(tq + tps * e, nq - 1)];
      return o;
    };
    // the sums of one step: slices i and, with NS = 2, i + spi; weights of
    // entries outside the slice, or of a missing second slice, are zero, so
    // every lane runs the same FMAs
    auto sum_step = [&](V4 &x1, V4 &x2, int i) {
      // this step's floats as floats: their wait and conversion happen here,
      // one step after their loads went out
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        asm volatile("" : "+v"(x1.v[e].x), "+v"(x1.v[e].y), "+v"(x1.v[e].z), "+v"(x1.v[e].w));
        if constexpr (NS == 2)
          asm volatile("" : "+v"(x2.v[e].x), "+v"(x2.v[e].y), "+v"(x2.v[e].z), "+v"(x2.v[e].w));
      }
      const int i2 = i + spi;
      const bool two = NS == 2 && i2 < nb;
      const double *w1 = sw + i * R, *w2 = sw + (two ? i2 : i) * R;
#pragma unroll
      for (int e = 0; e < EPT; ++e) {
        const int el = 4 * (tq + tps * e);
        const float a1[4] = {x1.v[e].x, x1.v[e].y, x1.v[e].z, x1.v[e].w};
        if constexpr (WHOLE) {
          const bool in = el < RJ;
          const double wa1 = w1[r0[e]];
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[e][c] = fma(in ? wa1 : 0.0, (double)a1[c], acc[e][c]);
          if constexpr (NS == 2) {
            const float a2[4] = {x2.v[e].x, x2.v[e].y, x2.v[e].z, x2.v[e].w};
            const double wa2 = w2[r0[e]];
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[e][c] = fma((in && two) ? wa2 : 0.0, (double)a2[c], acc[e][c]);
          }
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const bool in = el + c < RJ;
            const int r = min((el + c) / J, R - 1);
            const double wr1 = w1[r];
            acc[e][c] = fma(in ? wr1 : 0.0, (double)a1[c], acc[e][c]);
            if constexpr (NS == 2) {
              const float a2c = c == 0 ? x2.v[e].x : c == 1 ? x2.v[e].y : c == 2 ? x2.v[e].z : x2.v[e].w;
              const double wr2 = w2[r];
              acc[e][c] = fma((in && two) ? wr2 : 0.0, (double)a2c, acc[e][c]);
            }
          }
        }
      }
    };
    // Two register sets in turn (A, B): a step's sums run while the next
    // step's slices load into the other set.  The next loads go out
    // unconditionally (past the batch the clamped load repeats its last
    // slice, which is not summed again); the empty asm keeps them ahead of
    // the sums (without it the compiler proves a set equals a fresh load of
    // its slice and moves the load down to its use).
    const int step = NS * spi;
    V4 a1 = load(sg), a2, b1, b2;
    if constexpr (NS == 2) a2 = load(sg + spi);
#pragma unroll 1
    for (int i = sg; i < nb; i += 2 * step) {
      b1 = load(i + step);
      if constexpr (NS == 2) b2 = load(i + step + spi);
      asm volatile("" ::: "memory");
      sum_step(a1, a2, i);
      if (i + step >= nb) break;
      a1 = load(i + 2 * step);
      if constexpr (NS == 2) a2 = load(i + 2 * step + spi);
      asm volatile("" ::: "memory");
      sum_step(b1, b2, i + step);
    }
  }
  // the slice groups' sums added in group order
  double *part = a.partials + (int64_t)chunk * partial_len(J, R);
  double *scomb = (double *)smem;   // kFsumThreads x 4
#pragma unroll
  for (int e = 0; e < EPT; ++e) {
    const int el = 4 * (tq + tps * e);
    if (spi == 1) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (el + c < RJ) part[el + c] = acc[e][c];
    } else {
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 4; ++c) scomb[tid * 4 + c] = acc[e][c];
      __syncthreads();
      if (sg == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (el + c < RJ) {
            double sum = 0.0;
            for (int g = 0; g < spi; ++g) sum += scomb[(g * tps + tq) * 4 + c];
            part[el + c] = sum;
          }
        }
      }
    }
  }
  // G and sum n from the solve chunks of this chunk, in order
  const int per = h->chunk / h->chunk2;
  const int c2a = chunk * per, c2b = min(h->n_chunks2, c2a + per);
  for (int e = tid; e <= RR; e += kFsumThreads) part[RJ + e] = ordered_sum(a.part2, RR + 1, e, c2a, c2b);
  (void)arrive(a, h, chunk, &sflag);
}

template <int EPT>
__global__ __launch_bounds__(kFsumThreads, 4) void k_fsum(const PassArgs *args, const BlockMap *map) {
  fsum_body<EPT, true>(args, map);
}

// J not a multiple of 4 (any slice size up to 4 float4 per thread)
__global__ __launch_bounds__(kFsumThreads, 4) void k_fsum_odd(const PassArgs *args, const BlockMap *map) {
  fsum_body<4, false>(args, map);
}

// float4 positions per thread of a slice's F-stage work (1, 2 or 4).
__host__ __device__ inline int ept_bucket(int ys) {
  const int tps = fsum_tps(ys), e = (ys / 4 + tps - 1) / tps;
  return e <= 1 ? 1 : (e <= 2 ? 2 : 4);
}


// ---------------------------------------------------------------------------
// Second reduction level before the final phase: the group partials summed in
// group order into group 0, one thread per entry, so the single-workgroup
// final phase reads one partial.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce_groups(const PassArgs *args, const BlockMap *map) {
  CPassArgs &a = *(CPassArgs *)(map ? map[blockIdx.x].args : args);
  const int blk = map ? map[blockIdx.x].local : (int)blockIdx.x;
  const int plen = partial_len(a.J, a.R);
  const int e = blk * 256 + threadIdx.x;
  if (e >= plen) return;
  const int ng = a.hdr->n_rgroups;
  a.gpart[e] = ordered_sum(a.gpart, plen, e, 0, ng);
}

int reduce_groups_blocks(int J, int R) { return (partial_len(J, R) + 255) / 256; }

int launch_reduce_groups(const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return 0;
  hipLaunchKernelGGL(k_reduce_groups, dim3(n_blocks), dim3(256), 0, s, args, map);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// F stage, lagged mode: the new rows' terms of eq. [obtain_FandF] and
// [obtain_FandG], sum over touched slices of (U_k S_k)^T X_k and
// S_k U_k^T U_k S_k with the pass's new S_k.  Workgroup c takes the items
// c, c + n_chunks, ... (static, so the sums do not depend on scheduling).
// ---------------------------------------------------------------------------
template <int RW, int JW, bool MX>
__global__ __launch_bounds__(256) void k_fsum_rows(const PassArgs *args, const BlockMap *map) {
  extern __shared__ __align__(16) unsigned char smem[];
  CPassArgs &a = *(CPassArgs *)(map ? map[blockIdx.x].args : args);
  const int blk = map ? map[blockIdx.x].local : (int)blockIdx.x;
  __shared__ int sflag;
  const StepHeader *h = a.hdr;
  const int J = a.J, R = a.R, RR = R * R, RJ = R * J;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int gcur = a.ctl->gcur;
  const int wout = 1 - gcur;
  const RowsLds L = rows_lds(J, R);
  float *sX = (float *)(smem + L.oX);
  float *sU = (float *)(smem + L.oU);
  double *sW = (double *)(smem + L.oW);
  const int XS = L.XS, MB = L.MB;
  const int chunk = blk;
  double facc[RW][JW];
  double gacc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int rr = 0; rr < RW; ++rr)
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) facc[rr][jj] = 0.0;

  for (int it = chunk; it < h->n_items; it += h->n_chunks) {
    const Item item = a.items[it];
    const int k = item.slice;
    __syncthreads();
    if (tid < R) sW[tid] = a.W[((int64_t)wout * a.K_cap + k) * R + tid];
    f32x4 accY[kMxTiles];
    f32x4 accD = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int i = 0; i < kMxTiles; ++i) accY[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int gi = item.g0; gi < item.g1; ++gi) {
      const Group gr = a.groups[gi];
      for (int r0 = 0; r0 < gr.nrows; r0 += MB) {
        const int m = min(MB, gr.nrows - r0);
        const int mp = MX ? (m + 31) & ~31 : (m + 15) & ~15;
        __syncthreads();
        (void)stage_rows<false>(gr.src + (int64_t)r0 * J, m, J, XS, sX, tid);
        zero_block_pad(sX, XS, m, mp, J, L.J16, tid);
        const int R16 = (R + 15) & ~15;
        for (int e = tid; e < mp * R16; e += 256) {
          const int row = e / R16, n = e - row * R16;
          sU[row * L.US + n] =
              (row < m && n < R) ? (float)(a.U_out[(gr.out_row + r0 + row) * R + n] * sW[n]) : 0.f;
        }
        __syncthreads();
        if constexpr (MX)
          accum_block_mx(sX, sU, XS, L.US, mp, J, R, accY, accD, tid);
        else
          accum_block_f32(sX, sU, XS, L.US, mp, J, R, accY, accD, tid);
      }
    }
    // the slice's tiles into the FP64 sums through LDS
    __syncthreads();
    float *sDY = sX, *sDD = sU;
    {
      const int li = lane & 15;
      const int MT = (R + 15) >> 4, NT = (J + 15) >> 4;
#pragma unroll
      for (int i = 0; i < kMxTiles; ++i) {
        const int c = i >> 1, mt = i & 1;
        const int nt = wv + 4 * c;
        if (nt >= NT || mt >= MT) continue;
        const int j = nt * 16 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = mt * 16 + (lane >> 4) * 4 + q;
          if (r < R && j < J) sDY[r * J + j] = accY[i][q];
        }
      }
      if (wv < MT * MT) {
        const int mt = wv / MT, st = wv - mt * MT;
        const int cc = st * 16 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int r = mt * 16 + (lane >> 4) * 4 + q;
          if (r < R && cc < R) sDD[r * R + cc] = accD[q];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int rr = 0; rr < RW; ++rr)
#pragma unroll
      for (int jj = 0; jj < JW; ++jj) {
        const int r = wv + 4 * rr, j = lane + 64 * jj;
        if (r < R && j < J) facc[rr][jj] += (double)sDY[r * J + j];
      }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int q = tid + 256 * i;
      if (q < RR) gacc[i] += (double)sDD[q];
    }
  }
  double *part = a.partials + (int64_t)chunk * partial_len(J, R);
#pragma unroll
  for (int rr = 0; rr < RW; ++rr)
#pragma unroll
    for (int jj = 0; jj < JW; ++jj) {
      const int r = wv + 4 * rr, j = lane + 64 * jj;
      if (r < R && j < J) part[r * J + j] = facc[rr][jj];
    }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int q = tid + 256 * i;
    if (q < RR) part[RJ + q] = gacc[i];
  }
  // sum n from the solve chunks of this chunk, in order
  const int per = h->chunk / h->chunk2;
  const int c2a = chunk * per, c2b = min(h->n_chunks2, c2a + per);
  if (tid == 0) part[RJ + RR] = ordered_sum(a.part2, RR + 1, RR, c2a, c2b);
  (void)arrive(a, h, chunk, &sflag);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename F>
static int allow_lds_s(F *fn, size_t bytes) {
  if (bytes <= 65536) return 0;
  return (int)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

static inline int rw_bucket(int R) { return R <= 8 ? 2 : (R <= 16 ? 4 : 8); }
static inline int jw_bucket(int J) { return J <= 64 ? 1 : (J <= 128 ? 2 : 4); }
static inline int rm_bucket(int R) { return R <= 8 ? 8 : (R <= 16 ? 16 : 32); }

int split_rows_class(int J, int R, int mixed) {
  return ((rw_bucket(R) * 8 + jw_bucket(J)) * 2 + (mixed ? 1 : 0)) * 2 + (J % jw_bucket(J) == 0 ? 1 : 0);
}
int split_solve_class(int R) { return rm_bucket(R); }
int split_fsum_class(int J, int R, int lagged, int mixed) {
  return lagged ? 1000 + split_rows_class(J, R, mixed) : (J & 3) ? 5 : ept_bucket(y_stride(J, R));
}

// the fast row kernel's LDS: BF16-staged blocks in the mixed path
static size_t rows_fast_lds(int J, int R, bool mixed) {
  return mixed ? rows_lds_bf(J, R).bytes : rows_lds(J, R).bytes;
}

size_t split_rows_lds(int J, int R, int mixed) { return rows_fast_lds(J, R, mixed != 0); }
size_t split_rows_slow_lds(int J, int R) { return rows_lds(J, R).bytes; }

int launch_split_solve_fix(const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s, size_t lds) {
  if (n_blocks <= 0) return 0;
  if (int e = allow_lds_s(k_solve_fix, lds)) return e;
  hipLaunchKernelGGL(k_solve_fix, dim3(n_blocks), dim3(64 * kSolveWaves), lds, s, args, map);
  return (int)hipGetLastError();
}

void split_kernel_name(int stage, const PassArgs &a, char *buf, size_t n) {
  const int mx = a.mixed ? 1 : 0;
  switch (stage) {
    case 0:
      snprintf(buf, n, "k_rows<%d, %d, %s, false, %s>", rw_bucket(a.R), jw_bucket(a.J), mx ? "true" : "false",
               a.J % jw_bucket(a.J) == 0 ? "true" : "false");
      break;
    case 1: snprintf(buf, n, "k_rows<8, 4, %s, true>", mx ? "true" : "false"); break;
    case 2: snprintf(buf, n, "k_solve<%d>", rm_bucket(a.R)); break;
    case 3:
      if (a.lagged && a.mode == 0)
        snprintf(buf, n, "k_fsum_rows<%d, %d, %s>", rw_bucket(a.R), jw_bucket(a.J), mx ? "true" : "false");
      else if (a.J & 3)
        snprintf(buf, n, "k_fsum_odd");
      else
        snprintf(buf, n, "k_fsum<%d>", ept_bucket(a.ys));
      break;
    case 4: snprintf(buf, n, "k_reduce_groups"); break;
    default: snprintf(buf, n, "k_finish_dev<%d>", finish_class(a.R)); break;
  }
}
size_t split_solve_lds(int J, int R) { return solve_lds(J, R).bytes; }
size_t split_fsum_lds(int J, int R, int lagged) {
  if (lagged) return rows_lds(J, R).bytes;
  return std::max((size_t)kFsumBatch * R * 8, (size_t)kFsumThreads * 4 * 8);
}

template <int RW, int JW, bool MX>
static int launch_rows_t(const PassArgs *args, const BlockMap *map, int n_blocks, size_t bytes, hipStream_t s,
                         bool vec) {
  if (vec) {
    if (int e = allow_lds_s(k_rows<RW, JW, MX, false, true>, bytes)) return e;
    hipLaunchKernelGGL((k_rows<RW, JW, MX, false, true>), dim3(n_blocks), dim3(256), bytes, s, args, map);
  } else {
    if (int e = allow_lds_s(k_rows<RW, JW, MX, false>, bytes)) return e;
    hipLaunchKernelGGL((k_rows<RW, JW, MX, false>), dim3(n_blocks), dim3(256), bytes, s, args, map);
  }
  return (int)hipGetLastError();
}

template <int RW, int JW, bool MX>
static int rows_occupancy_t(int J, int R) {
  const size_t bytes = rows_fast_lds(J, R, MX);
  if (allow_lds_s(k_rows<RW, JW, MX, false, true>, bytes)) return 1;
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_rows<RW, JW, MX, false, true>, 256, bytes) != hipSuccess ||
      n < 1)
    return 1;
  return n;
}

template <int RW, int JW, bool MX>
static int launch_fsum_rows_t(const PassArgs *args, const BlockMap *map, int n_blocks, size_t bytes,
                              hipStream_t s) {
  if (int e = allow_lds_s(k_fsum_rows<RW, JW, MX>, bytes)) return e;
  hipLaunchKernelGGL((k_fsum_rows<RW, JW, MX>), dim3(n_blocks), dim3(256), bytes, s, args, map);
  return (int)hipGetLastError();
}

#define DASH_RW_JW_SWITCH(FN, MX, ...)                                                              \
  switch (rw_bucket(a.R) * 8 + jw_bucket(a.J)) {                                                    \
    case 2 * 8 + 1: return FN<2, 1, MX>(__VA_ARGS__);                                               \
    case 2 * 8 + 2: return FN<2, 2, MX>(__VA_ARGS__);                                               \
    case 2 * 8 + 4: return FN<2, 4, MX>(__VA_ARGS__);                                               \
    case 4 * 8 + 1: return FN<4, 1, MX>(__VA_ARGS__);                                               \
    case 4 * 8 + 2: return FN<4, 2, MX>(__VA_ARGS__);                                               \
    case 4 * 8 + 4: return FN<4, 4, MX>(__VA_ARGS__);                                               \
    case 8 * 8 + 1: return FN<8, 1, MX>(__VA_ARGS__);                                               \
    case 8 * 8 + 2: return FN<8, 2, MX>(__VA_ARGS__);                                               \
    case 8 * 8 + 4: return FN<8, 4, MX>(__VA_ARGS__);                                               \
    default: return (int)hipErrorInvalidValue;                                                      \
  }

int launch_split_rows(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s,
                      size_t lds) {
  if (n_blocks <= 0) return 0;
  const size_t bytes = lds ? lds : rows_fast_lds(a.J, a.R, a.mixed != 0);
  if (a.mixed) {
    DASH_RW_JW_SWITCH(launch_rows_t, true, args, map, n_blocks, bytes, s, a.J % jw_bucket(a.J) == 0)
  } else {
    DASH_RW_JW_SWITCH(launch_rows_t, false, args, map, n_blocks, bytes, s, a.J % jw_bucket(a.J) == 0)
  }
}

int launch_split_rows_slow(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks,
                           hipStream_t s, size_t lds) {
  if (n_blocks <= 0) return 0;
  // the deferred slices (Lemma 1's pseudo-inverse form): one instantiation for
  // every shape; its workgroups leave at once when nothing was deferred
  const size_t bytes = lds ? lds : rows_lds(a.J, a.R).bytes;
  if (a.mixed) {
    if (int e = allow_lds_s(k_rows<8, 4, true, true>, bytes)) return e;
    hipLaunchKernelGGL((k_rows<8, 4, true, true>), dim3(n_blocks), dim3(256), bytes, s, args, map);
  } else {
    if (int e = allow_lds_s(k_rows<8, 4, false, true>, bytes)) return e;
    hipLaunchKernelGGL((k_rows<8, 4, false, true>), dim3(n_blocks), dim3(256), bytes, s, args, map);
  }
  return (int)hipGetLastError();
}

int split_rows_blocks_per_cu(int J, int R, int mixed) {
  PassArgs a{};
  a.J = J;
  a.R = R;
  if (mixed) {
    DASH_RW_JW_SWITCH(rows_occupancy_t, true, J, R)
  } else {
    DASH_RW_JW_SWITCH(rows_occupancy_t, false, J, R)
  }
}

template <int RM>
static int launch_solve_t(const PassArgs *args, const BlockMap *map, int n_blocks, size_t bytes, hipStream_t s) {
  if (int e = allow_lds_s(k_solve<RM>, bytes)) return e;
  hipLaunchKernelGGL((k_solve<RM>), dim3(n_blocks), dim3(64 * kSolveWaves), bytes, s, args, map);
  return (int)hipGetLastError();
}

int launch_split_solve(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s,
                       size_t lds) {
  if (n_blocks <= 0) return 0;
  const size_t bytes = lds ? lds : solve_lds(a.J, a.R).bytes;
  switch (rm_bucket(a.R)) {
    case 8: return launch_solve_t<8>(args, map, n_blocks, bytes, s);
    case 16: return launch_solve_t<16>(args, map, n_blocks, bytes, s);
    default: return launch_solve_t<32>(args, map, n_blocks, bytes, s);
  }
}

template <int EPT>
static int launch_fsum_t(const PassArgs *args, const BlockMap *map, int n_blocks, size_t bytes, hipStream_t s) {
  hipLaunchKernelGGL((k_fsum<EPT>), dim3(n_blocks), dim3(kFsumThreads), bytes, s, args, map);
  return (int)hipGetLastError();
}

int launch_split_fsum(const PassArgs &a, const PassArgs *args, const BlockMap *map, int n_blocks, hipStream_t s,
                      size_t lds) {
  if (n_blocks <= 0) return 0;
  const size_t bytes = lds ? lds : split_fsum_lds(a.J, a.R, a.lagged && a.mode == 0);
  if (a.lagged && a.mode == 0) {
    if (a.mixed) {
      DASH_RW_JW_SWITCH(launch_fsum_rows_t, true, args, map, n_blocks, bytes, s)
    } else {
      DASH_RW_JW_SWITCH(launch_fsum_rows_t, false, args, map, n_blocks, bytes, s)
    }
  }
  if (a.J & 3) {
    hipLaunchKernelGGL(k_fsum_odd, dim3(n_blocks), dim3(kFsumThreads), bytes, s, args, map);
    return (int)hipGetLastError();
  }
  switch (ept_bucket(a.ys)) {
    case 1: return launch_fsum_t<1>(args, map, n_blocks, bytes, s);
    case 2: return launch_fsum_t<2>(args, map, n_blocks, bytes, s);
    default: return launch_fsum_t<4>(args, map, n_blocks, bytes, s);
  }
}

#undef DASH_RW_JW_SWITCH

}  // namespace dash
