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
#include "internal.h"

namespace pp {

namespace {
__global__ void k_finalize(int64_t m, int ncells, int nparts, const int* __restrict__ perm, const int* __restrict__ tleaf,
                           const double* __restrict__ far, const double* __restrict__ near_sum,
                           const double* __restrict__ leaf_wnear, const int* __restrict__ self_idx,
                           const double* __restrict__ self_logd, const double* __restrict__ self_w,
                           const double* __restrict__ f, double h, double lnh,
                           int self_mode, const int* __restrict__ flags, double* __restrict__ out) {
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
              hipStream_t s) {
  if (m <= 0) return;
  k_finalize<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(m, ncells, nparts, perm, tleaf, far, near_sum, leaf_wnear,
                                                         self_idx, self_logd, self_w, f, h, log(h), self_mode, flags,
                                                         out);
}

}  // namespace pp
