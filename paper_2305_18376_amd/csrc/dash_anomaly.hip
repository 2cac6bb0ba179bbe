// Anomaly scores of an update on gfx950 (the paper's application of the
// update, Sec. 3.4): the slice-level reconstruction error of Definition 1,
//   se_k = sum_{i,j} |X_{k,new}(i,j) - (U_{k,new} S_k V^T)(i,j)| / (I_{k,new} J),
// with the updated S_k and V, for every slice that received rows; the
// tensor-level error of Definition 2 as the mean of se_k over those slices;
// and, per slice, the moving threshold of Sec. 4.5 (mean plus population
// standard deviation of the slice's previous `window` errors): a slice whose
// se_k exceeds it is flagged.
//
// One launch after the update's final phase.  Workgroup b takes the touched
// slices b, b + gridDim.x, ... (static, so every sum has a fixed order); thread
// t owns column j = t mod J of rows t / J, t / J + 256 / J, ... of a block and
// keeps V's row j (R floats) in registers.  The last workgroup to finish sums
// se_k in item order into te, writes it to the update's report and publishes
// the report (the final phase leaves `done` to this kernel when scores are on).
#include <hip/hip_runtime.h>
#include <math.h>

#include "dash_dev.h"
#include "dash_math.h"

namespace dash {

constexpr int kAnomThreads = 256;
constexpr int kAnomRows = 32;   // rows of U S staged at a time

template <int RP>   // R rounded up: 8, 16 or 32
__global__ __launch_bounds__(kAnomThreads) void k_slice_errors(PassArgs a, AnomalyArgs x) {
  __shared__ float sUS[kAnomRows * 33];
  __shared__ double sRed[kAnomThreads / 64];
  __shared__ int sLast;
  const StepHeader *h = a.hdr;
  const int J = a.J, R = a.R;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool committed = !a.ctl->poison;   // the final phase poisons the context on a failed update
  const int gcur = a.ctl->gcur;            // after the commit: the new state
  const VBundleView vb = vb_view(a.vb + (int64_t)gcur * a.vb_stride, J, R);
  const int n_items = h->n_items;
  // this thread's column and V row
  const int rows_per = max(1, kAnomThreads / J);   // rows side by side (J <= 256)
  const int j = tid % J, rsub = tid / J;
  const bool active = rsub < rows_per && j < J;
  float vrow[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r) vrow[r] = (active && r < R) ? vb.Vt32[r * J + j] : 0.f;

  if (committed) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
      const Item item = a.items[it];
      const int k = item.slice;
      const double *w = a.W + ((int64_t)gcur * a.K_cap + k) * R;
      double acc = 0.0;
      for (int gi = item.g0; gi < item.g1; ++gi) {
        const Group gr = a.groups[gi];
        for (int r0 = 0; r0 < gr.nrows; r0 += kAnomRows) {
          const int m = min(kAnomRows, gr.nrows - r0);
          __syncthreads();
          for (int e = tid; e < m * R; e += kAnomThreads) {
            const int row = e / R, r = e - row * R;
            sUS[row * 33 + r] = (float)((double)a.U_out[(gr.out_row + r0 + row) * R + r] * w[r]);
          }
          __syncthreads();
          if (active) {
            for (int row = rsub; row < m; row += rows_per) {
              float xh = 0.f;
#pragma unroll
              for (int r = 0; r < RP; ++r)
                if (r < R) xh = fmaf(sUS[row * 33 + r], vrow[r], xh);
              const float xv = gr.src[(int64_t)(r0 + row) * J + j];
              acc += fabs((double)xv - (double)xh);
            }
          }
        }
      }
      acc = wave_sum(acc);
      __syncthreads();
      if (lane == 0) sRed[wv] = acc;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int q = 0; q < kAnomThreads / 64; ++q) s += sRed[q];
        const float se = (float)(s / ((double)item.rows * J));
        // moving threshold over the slice's previous errors (Sec. 4.5)
        const int cnt = x.hcnt[k];
        const int n = min(cnt, x.window);
        float *hk = x.hist + (int64_t)k * x.window;
        int flag = 0;
        if (n > 0) {
          double mean = 0.0, var = 0.0;
          for (int q = 0; q < n; ++q) mean += hk[q];
          mean /= n;
          for (int q = 0; q < n; ++q) var += (hk[q] - mean) * (hk[q] - mean);
          const double thr = mean + sqrt(var / n);
          flag = (double)se > thr ? 1 : 0;
        }
        hk[cnt % x.window] = se;
        x.hcnt[k] = cnt + 1;
        x.se[it] = se;
        x.flag[it] = flag;
        x.sid[it] = k;
      }
    }
  }
  // the last workgroup: te (Definition 2) in item order, then the report
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    sLast = (atomicAdd(x.ticket, 1) == (int)gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!sLast) return;
  __threadfence();
  double s = 0.0;
  int nf = 0;
  if (committed)
    for (int it = tid; it < n_items; it += kAnomThreads) {
      s += (double)x.se[it];
      nf += x.flag[it];
    }
  // fixed-order block sum: per-wave partials, then in wave order
  s = wave_sum(s);
  double fn = wave_sum((double)nf);
  __shared__ double sF[kAnomThreads / 64];
  if (lane == 0) {
    sRed[wv] = s;
    sF[wv] = fn;
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0, flags = 0.0;
    for (int q = 0; q < kAnomThreads / 64; ++q) {
      tot += sRed[q];
      flags += sF[q];
    }
    *x.ticket = 0;
    Report *rep = (Report *)h->report;
    if (rep) {
      rep->te = (committed && n_items > 0) ? tot / n_items : 0.0;
      rep->n_anomalies = committed ? (int32_t)flags : 0;
      __threadfence_system();
      rep->done = 1;
    }
  }
}

int launch_slice_errors(const PassArgs &a, const AnomalyArgs &x, int n_blocks, hipStream_t s) {
  if (n_blocks < 1) n_blocks = 1;
  if (a.R <= 8)
    hipLaunchKernelGGL((k_slice_errors<8>), dim3(n_blocks), dim3(kAnomThreads), 0, s, a, x);
  else if (a.R <= 16)
    hipLaunchKernelGGL((k_slice_errors<16>), dim3(n_blocks), dim3(kAnomThreads), 0, s, a, x);
  else
    hipLaunchKernelGGL((k_slice_errors<32>), dim3(n_blocks), dim3(kAnomThreads), 0, s, a, x);
  return (int)hipGetLastError();
}

}  // namespace dash
