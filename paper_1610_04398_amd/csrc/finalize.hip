// Final assembly of P at each target (Appendix A, superposition of the group
// contributions): far field from the local expansion (read, or evaluated here
// by L2P) plus the near field, with the 1/(2 pi) of eq. green2D, scattered back
// to the caller's target order.
//
// The near-field kernel leaves, per target and list part, sum w ln r over the
// part's near sources (its own leaf included).  A target that coincides with a
// grid node (exact FP64 equality with x0 + (i + 1/2) h) contributed 0 for that
// node's pair inside the near-field kernel, but w ln h through the near weight
// term: the self rule then subtracts w ln h (skip) or w kappa (cell average:
// w (ln h - kappa) in total).  In mixed precision a target within 2^-20 h of a
// node was snapped onto it (FP32 cannot resolve that distance); the exact FP64
// term w ln d is restored here.  Scattered sources that coincide exactly with a
// target were skipped by the near-field kernel the same way; their share w ln h
// is removed here (G(0) := 0).
#include <algorithm>

#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {
constexpr int kFinBlock = 256;
constexpr int kFinWaves = kFinBlock / kWave;

__device__ inline long long wave_sum(long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// The first workgroups also sum the statistics (per-wave pair counts, per-cell
// list lengths; one item per thread, wave sums, one atomic per workgroup and
// counter) into zeroed slots, so they need no launch of their own and add
// little to the launch's critical path.
__global__ __launch_bounds__(kFinBlock) void k_finalize(int64_t m, int nparts, const int* __restrict__ perm,
                                                         double* __restrict__ far,
                                                         const double* __restrict__ near_sum,
                                                         const double* __restrict__ self_w,
                                                         const double* __restrict__ self_logd, double lnh,
                                                         int self_mode, const int* __restrict__ flags,
                                                         double* __restrict__ out, FinalizeTotals tot, FarEval fe,
                                                         GridBatch bt) {
  const int64_t tot_n = std::max<int64_t>(tot.pairs ? tot.nwaves : 0, tot.cnt_m ? tot.ncells : 0);
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((int64_t)blockIdx.x * kFinBlock < tot_n) {  // uniform per workgroup
    __shared__ long long part[3][kFinWaves];
    long long acc = 0, am = 0, ap = 0;
    if (tot.pairs && k < tot.nwaves) acc = tot.pair_counts[k];
    if (tot.cnt_m && k < tot.ncells) {
      am = tot.cnt_m[k];
      ap = tot.cnt_p[k];
    }
    acc = wave_sum(acc);
    am = wave_sum(am);
    ap = wave_sum(ap);
    const int w = threadIdx.x / kWave;
    if (threadIdx.x % kWave == 0) {
      part[0][w] = acc;
      part[1][w] = am;
      part[2][w] = ap;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      long long t = 0;
      for (int q = 0; q < kFinWaves; ++q) t += part[threadIdx.x][q];
      if (t) {
        if (threadIdx.x == 0 && tot.pairs) atomicAdd(tot.pairs, (unsigned long long)t);
        if (threadIdx.x == 1 && tot.cnt_m) atomicAdd(tot.tot_m, (int)t);
        if (threadIdx.x == 2 && tot.cnt_m) atomicAdd(tot.tot_p, (int)t);
      }
    }
  }
  if (k >= m) return;
  if (*flags != 0) return;
  // the parts' loads issued together, then summed in part order
  double nsq[kMaxNearParts];
#pragma unroll
  for (int q = 0; q < kMaxNearParts; ++q) nsq[q] = q < nparts ? near_sum[(int64_t)q * m + k] : 0.0;
  double ns = nsq[0];
#pragma unroll
  for (int q = 1; q < kMaxNearParts; ++q)
    if (q < nparts) ns += nsq[q];
  double fv;
  if (fe.loc) {
    const int c = fe.tleaf[k];
    fv = l2p_eval(fe.loc + (int64_t)c * (fe.p + 1), fe.p, fe.rel64[k], fe.D, fe.lvl[c], fe.fp32 != 0);
    if (far) far[k] = fv;  // kept for the far-field array read-back
  } else {
    fv = far ? far[k] : 0.0;
    if (far && fe.far_parts > 1) {
      for (int q = 1; q < fe.far_parts; ++q) fv += far[(int64_t)q * m + k];
      far[k] = fv;  // the total, for the far-field array read-back
    }
  }
  double v = fv + ns;
  if (self_w) {
    const double w = self_w[k];
    const double lg = self_logd ? self_logd[k] : -INFINITY;
    if (isinf(lg)) {
      v -= (self_mode == 1) ? w * kKappa : w * lnh;
    } else {
      v += w * (lg - lnh);
    }
  }
  const int o = perm[k];
  if (bt.nreq) {  // a forest of requests: target o - toff[r] of request r
    const int r = batch_request(bt, o);
    bt.out[r][o - bt.toff[r]] = v * kInv2Pi;
  } else {
    out[o] = v * kInv2Pi;
  }
}
}  // namespace

void finalize(int64_t m, int nparts, const int* perm, double* far, const double* near_sum,
              const double* self_w, const double* self_logd, double h, int self_mode, const int* flags, double* out,
              const FinalizeTotals& tot, const FarEval& fe, const GridBatch* bt, hipStream_t s) {
  const int64_t tot_n = std::max<int64_t>(tot.pairs ? tot.nwaves : 0, tot.cnt_m ? tot.ncells : 0);
  const int64_t blocks = (std::max(m, tot_n) + kFinBlock - 1) / kFinBlock;
  if (blocks <= 0) return;
  k_finalize<<<(unsigned)blocks, kFinBlock, 0, s>>>(m, nparts, perm, far, near_sum, self_w, self_logd, log(h),
                                                    self_mode, flags, out, tot, fe, bt ? *bt : GridBatch{});
}

}  // namespace pp
