// Ingest of scattered sources (w_i = f_i h_i^2 given per source, so a source
// may carry its own cell area, eq. greenSum with a varying h) and the per-leaf
// packing of those sources and of the targets.
//
// The root square is anchored at the lower-left corner (x0, y0) of the
// bounding box of the weighted sources and the targets, and its finest cells
// have the power-of-two side u for which 2^D u first exceeds the box's extent
// (D = kPointsDepth).  Keys are floor((x - x0) / u) interleaved, the same FP64
// operations as for grid targets, so every point falls inside the root.
// Sources with w = 0 take the key 0xFFFFFFFF, above every cell key, and sort
// to the end where the tree does not see them.
#include <cmath>

#include "blockscan.h"
#include "internal.h"
#include "leafpass.h"

namespace pp {

namespace {
constexpr int kBoxBlock = 256;

// Per-block bounding box of the weighted sources and the targets, the number
// of weighted sources, and flags for non-finite input.
__global__ __launch_bounds__(kBoxBlock) void k_box_partial(const double* __restrict__ sx,
                                                            const double* __restrict__ sy,
                                                            const double* __restrict__ w, int64_t n,
                                                            const double* __restrict__ tx,
                                                            const double* __restrict__ ty, int64_t m,
                                                            double4* __restrict__ part, int* __restrict__ cnt,
                                                            int* __restrict__ flags) {
  __shared__ double red[4][kBoxBlock];
  __shared__ int rc[kBoxBlock];
  double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
  int c = 0, bad_s = 0, bad_t = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n + m; i += stride) {
    double x, y;
    if (i < n) {
      const double wi = w[i];
      x = sx[i];
      y = sy[i];
      if (!isfinite(wi) || !isfinite(x) || !isfinite(y)) {
        bad_s = 1;
        continue;
      }
      if (wi == 0.0) continue;
      ++c;
    } else {
      x = tx[i - n];
      y = ty[i - n];
      if (!isfinite(x) || !isfinite(y)) {
        bad_t = 1;
        continue;
      }
    }
    x0 = fmin(x0, x);
    x1 = fmax(x1, x);
    y0 = fmin(y0, y);
    y1 = fmax(y1, y);
  }
  if (bad_s) atomicOr(flags, kFlagNonFiniteSource);
  if (bad_t) atomicOr(flags, kFlagNonFiniteTarget);
  const int t = threadIdx.x;
  red[0][t] = x0;
  red[1][t] = -x1;
  red[2][t] = y0;
  red[3][t] = -y1;
  rc[t] = c;
  __syncthreads();
  for (int o = kBoxBlock / 2; o > 0; o >>= 1) {
    if (t < o) {
      for (int q = 0; q < 4; ++q) red[q][t] = fmin(red[q][t], red[q][t + o]);
      rc[t] += rc[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    part[blockIdx.x] = make_double4(red[0][0], -red[1][0], red[2][0], -red[3][0]);
    cnt[blockIdx.x] = rc[0];
  }
}

__global__ __launch_bounds__(kBoxBlock) void k_box_final(const double4* __restrict__ part,
                                                          const int* __restrict__ cnt, int nparts,
                                                          double* __restrict__ box, int* __restrict__ nsrc) {
  __shared__ double red[4][kBoxBlock];
  __shared__ int rc[kBoxBlock];
  const int t = threadIdx.x;
  double v[4] = {INFINITY, INFINITY, INFINITY, INFINITY};
  int c = 0;
  for (int i = t; i < nparts; i += kBoxBlock) {
    const double4 p = part[i];
    v[0] = fmin(v[0], p.x);
    v[1] = fmin(v[1], -p.y);
    v[2] = fmin(v[2], p.z);
    v[3] = fmin(v[3], -p.w);
    c += cnt[i];
  }
  for (int q = 0; q < 4; ++q) red[q][t] = v[q];
  rc[t] = c;
  __syncthreads();
  for (int o = kBoxBlock / 2; o > 0; o >>= 1) {
    if (t < o) {
      for (int q = 0; q < 4; ++q) red[q][t] = fmin(red[q][t], red[q][t + o]);
      rc[t] += rc[t + o];
    }
    __syncthreads();
  }
  if (t == 0) {
    box[0] = red[0][0];
    box[1] = -red[1][0];
    box[2] = red[2][0];
    box[3] = -red[3][0];
    *nsrc = rc[0];
  }
}

__global__ void k_point_keys(const double* __restrict__ sx, const double* __restrict__ sy,
                             const double* __restrict__ w, int64_t n, double x0, double y0, double u, int D,
                             uint32_t* __restrict__ key, int* __restrict__ idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t k = 0xFFFFFFFFu;
  if (w[i] != 0.0) {
    const double lim = (double)(1u << D);
    const double qx = floor((sx[i] - x0) / u);
    const double qy = floor((sy[i] - y0) / u);
    // inside by construction of the root; clamp defensively
    const uint32_t ix = (uint32_t)fmin(fmax(qx, 0.0), lim - 1.0);
    const uint32_t iy = (uint32_t)fmin(fmax(qy, 0.0), lim - 1.0);
    k = morton(ix, iy);
  }
  key[i] = k;
  idx[i] = (int)i;
}

__global__ void k_gather_points(const int* __restrict__ perm, const int* __restrict__ nsrc_dev,
                                const double* __restrict__ sx, const double* __restrict__ sy,
                                const double* __restrict__ w, double* __restrict__ xs, double* __restrict__ ys,
                                double* __restrict__ ws) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= *nsrc_dev) return;
  const int o = perm[i];
  xs[i] = sx[o];
  ys[i] = sy[o];
  ws[i] = w[o];
}

// Both per-leaf passes in one launch: the first workgroups pack the source
// leaves, the rest prepare the target leaves.
__global__ __launch_bounds__(256) void k_pack_prep_points(TreeArrays t, int D, PointFrame fr,
                                                           const int* __restrict__ sleaves, int ns,
                                                           float* __restrict__ s32, int64_t stride,
                                                           double2* __restrict__ s64, double* __restrict__ leaf_w,
                                                           int pack_blocks, const int* __restrict__ tleaves, int nt,
                                                           const double* __restrict__ tx,
                                                           const double* __restrict__ ty,
                                                           const int* __restrict__ perm, float2* __restrict__ rel32,
                                                           double2* __restrict__ rel64, int* __restrict__ tleaf,
                                                           double* __restrict__ self_w) {
  const int lane = threadIdx.x % kWave;
  if ((int)blockIdx.x < pack_blocks) {
    const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (wid < ns)
      pack_point_leaf(wid, lane, t, sleaves, D, fr.xs, fr.ys, fr.ws, fr.x0, fr.y0, fr.u, s32, stride, s64, leaf_w);
  } else {
    const int wid = (blockIdx.x - pack_blocks) * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (wid < nt)
      prep_point_leaf(wid, lane, t, tleaves, D, tx, ty, perm, fr.x0, fr.y0, fr.u, fr.xs, fr.ys, fr.ws, rel32, rel64,
                      tleaf, self_w);
  }
}
}  // namespace

int points_box_blocks(int64_t n_total) {
  const int64_t b = (n_total + kBoxBlock * 8 - 1) / (kBoxBlock * 8);
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 1024);
}

void points_box(const double* sx, const double* sy, const double* w, int64_t n, const double* tx, const double* ty,
                int64_t m, double4* part, int* cnt, double* box, int* nsrc, int* flags, hipStream_t s) {
  const int g = points_box_blocks(n + m);
  k_box_partial<<<g, kBoxBlock, 0, s>>>(sx, sy, w, n, tx, ty, m, part, cnt, flags);
  k_box_final<<<1, kBoxBlock, 0, s>>>(part, cnt, g, box, nsrc);
}

void points_keys(const double* sx, const double* sy, const double* w, int64_t n, double x0, double y0, double u,
                 int D, uint32_t* key, int* idx, hipStream_t s) {
  if (n <= 0) return;
  k_point_keys<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(sx, sy, w, n, x0, y0, u, D, key, idx);
}

void points_gather(const int* perm, const int* nsrc_dev, int64_t nmax, const double* sx, const double* sy,
                   const double* w, double* xs, double* ys, double* ws, hipStream_t s) {
  if (nmax <= 0) return;
  k_gather_points<<<(unsigned)((nmax + 255) / 256), 256, 0, s>>>(perm, nsrc_dev, sx, sy, w, xs, ys, ws);
}

LeafPass leaf_pass_points(TreeArrays t, int D, double x0, double y0, double u, const double* xs, const double* ys,
                          const double* ws, const int* sleaves, int nsleaves, float* s32, int64_t stride,
                          double2* s64, double* leaf_w, const int* tleaves, int ntleaves, const double* tx,
                          const double* ty, const int* perm, float2* rel32, double2* rel64, int* tleaf,
                          double* self_w) {
  LeafPass lp;
  lp.kind = 2;
  lp.pack_blocks = std::max(nsleaves, 0) / 4 + (nsleaves % 4 > 0);
  lp.prep_blocks = std::max(ntleaves, 0) / 4 + (ntleaves % 4 > 0);
  lp.t = t;
  lp.D = D;
  lp.pa = PointArgs{PointFrame{x0, y0, u, xs, ys, ws}, sleaves, nsleaves, s32, stride, s64, leaf_w, tleaves, ntleaves,
                    tx, ty, perm, rel32, rel64, tleaf, self_w};
  return lp;
}

void leaf_pack_prep_points(TreeArrays t, int D, double x0, double y0, double u, const double* xs, const double* ys,
                           const double* ws, const int* sleaves, int nsleaves, float* s32, int64_t stride,
                           double2* s64, double* leaf_w, const int* tleaves, int ntleaves, const double* tx,
                           const double* ty, const int* perm, float2* rel32, double2* rel64, int* tleaf,
                           double* self_w, hipStream_t s) {
  const int gp = std::max(nsleaves, 0) / 4 + (nsleaves % 4 > 0);
  const int gt = std::max(ntleaves, 0) / 4 + (ntleaves % 4 > 0);
  if (gp + gt <= 0) return;
  const PointFrame fr{x0, y0, u, xs, ys, ws};
  k_pack_prep_points<<<gp + gt, 256, 0, s>>>(t, D, fr, sleaves, nsleaves, s32, stride, s64, leaf_w, gp, tleaves,
                                             ntleaves, tx, ty, perm, rel32, rel64, tleaf, self_w);
}

}  // namespace pp
