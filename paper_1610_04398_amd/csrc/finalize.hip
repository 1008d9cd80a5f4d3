// Final assembly of P at each target (Appendix A, superposition of the group
// contributions): far field from the local expansion plus the near field, with
// the 1/(2 pi) of eq. green2D, scattered back to the caller's target order.
//
// The near-field kernel sums w ln(r^2 / h^2) over the near sources; with the
// near weight W = sum w (FP64, from the leaf sums) the physical near field is
// 0.5 * that sum + W ln h.  A target that coincides with a grid node (exact FP64
// equality with x0 + (i + 1/2) h) contributed 0 for that node inside the
// near-field kernel but w ln h through W: the self rule then subtracts w ln h
// (skip) or w kappa (cell average: w (ln h - kappa) in total).  In mixed
// precision a target within 2^-20 h of a node was snapped onto it (FP32 cannot
// resolve that distance); the exact FP64 term w ln d is restored here.
// Scattered sources that coincide exactly with a target were skipped by the
// near-field kernel the same way; their share w ln u of the near weight term
// is removed here (G(0) := 0).
#include <algorithm>

#include "internal.h"

namespace pp {

namespace {
constexpr int kFinBlock = 256;
constexpr int kTotItems = 16;  // statistics items per thread in the blocks that sum them

// The first workgroups also sum the statistics (per-wave pair counts, per-cell
// list lengths) into zeroed slots with integer atomics, so they need no launch of
// their own.
__global__ __launch_bounds__(kFinBlock) void k_finalize(
    int64_t m, int ncells, int nparts, const int* __restrict__ perm, const int* __restrict__ tleaf,
    const double* __restrict__ far, const double* __restrict__ near_sum, const double* __restrict__ leaf_wnear,
    const int* __restrict__ self_idx, const double* __restrict__ self_logd, const double* __restrict__ self_w,
    const double* __restrict__ f, double h, double lnh, int self_mode, const int* __restrict__ flags,
    double* __restrict__ out, FinalizeTotals tot) {
  const int64_t tot_n = std::max<int64_t>(tot.pairs ? tot.nwaves : 0, tot.cnt_m ? tot.ncells : 0);
  const int64_t tot_base = (int64_t)blockIdx.x * kFinBlock * kTotItems;
  if (tot_base < tot_n) {  // uniform per workgroup
    __shared__ long long part[3][kFinBlock];
    long long acc = 0, am = 0, ap = 0;
    for (int q = 0; q < kTotItems; ++q) {
      const int64_t i = tot_base + (int64_t)q * kFinBlock + threadIdx.x;
      if (tot.pairs && i < tot.nwaves) acc += tot.pair_counts[i];
      if (tot.cnt_m && i < tot.ncells) {
        am += tot.cnt_m[i];
        ap += tot.cnt_p[i];
      }
    }
    part[0][threadIdx.x] = acc;
    part[1][threadIdx.x] = am;
    part[2][threadIdx.x] = ap;
    __syncthreads();
    for (int w = kFinBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w)
        for (int q = 0; q < 3; ++q) part[q][threadIdx.x] += part[q][threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (tot.pairs && part[0][0]) atomicAdd(tot.pairs, (unsigned long long)part[0][0]);
      if (tot.cnt_m && part[1][0]) atomicAdd(tot.tot_m, (int)part[1][0]);
      if (tot.cnt_m && part[2][0]) atomicAdd(tot.tot_p, (int)part[2][0]);
    }
  }
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  if (*flags != 0) return;
  const int c = tleaf[k];
  double ns = near_sum[k], wn = leaf_wnear[c];
  for (int q = 1; q < nparts; ++q) {
    ns += near_sum[(int64_t)q * m + k];
    wn += leaf_wnear[(int64_t)q * ncells + c];
  }
  double v = (far ? far[k] : 0.0) + 0.5 * ns + lnh * wn;
  if (self_w) v -= self_w[k] * lnh;
  const int si = self_idx ? self_idx[k] : -1;
  if (si >= 0) {
    const double w = f[si] * (h * h);
    const double lg = self_logd[k];
    if (isinf(lg)) {
      v -= (self_mode == 1) ? w * kKappa : w * lnh;
    } else {
      v += w * (lg - lnh);
    }
  }
  out[perm[k]] = v * kInv2Pi;
}
}  // namespace

void finalize(int64_t m, int ncells, int nparts, const int* perm, const int* tleaf, const double* far,
              const double* near_sum, const double* leaf_wnear, const int* self_idx, const double* self_logd,
              const double* self_w, const double* f, double h, int self_mode, const int* flags, double* out,
              const FinalizeTotals& tot, hipStream_t s) {
  const int64_t tot_n = std::max<int64_t>(tot.pairs ? tot.nwaves : 0, tot.cnt_m ? tot.ncells : 0);
  const int64_t blocks = std::max((m + kFinBlock - 1) / kFinBlock,
                                  (tot_n + (int64_t)kFinBlock * kTotItems - 1) / ((int64_t)kFinBlock * kTotItems));
  if (blocks <= 0) return;
  k_finalize<<<(unsigned)blocks, kFinBlock, 0, s>>>(m, ncells, nparts, perm, tleaf, far, near_sum, leaf_wnear,
                                                    self_idx, self_logd, self_w, f, h, log(h), self_mode, flags, out,
                                                    tot);
}

}  // namespace pp
