// Quadtree construction over the Morton-ordered sources and sorted targets,
// and the per-leaf packing of sources and targets for the evaluation passes.
//
// The paper groups sources hierarchically in a quadtree (Appendix A, Fig.
// multipole) without saying how it is built.  Here the tree is built top
// down, one level per launch pair: a cell at level l < D is split when it holds
// more than leaf_max sources or more than leaf_max targets, and its children
// (quadrant order q = qx + 2 qy) are kept when non-empty.  A child's source
// and target ranges are found by binary search of its key prefix inside the
// parent's ranges.
#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {

__device__ inline int lower_bound_u32(const uint32_t* __restrict__ a, int lo, int hi, uint64_t key) {
  while (lo < hi) {
    const int mid = lo + ((hi - lo) >> 1);
    if ((uint64_t)a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ void k_root(TreeArrays t, const int* __restrict__ nsrc_dev, int ntgt) {
  const int nsrc = *nsrc_dev;
  t.lvl[0] = 0;
  t.ix[0] = 0;
  t.iy[0] = 0;
  t.sb[0] = 0;
  t.se[0] = nsrc;
  t.tb[0] = 0;
  t.te[0] = ntgt;
  t.child[0] = -1;
  t.nchild[0] = 0;
  t.parent[0] = -1;
}

__global__ void k_level_count(TreeArrays t, int c0, int c1, int level, int D, int leaf_max,
                              const uint32_t* __restrict__ skey, const uint32_t* __restrict__ tkey,
                              int* __restrict__ cnt, int* __restrict__ cr) {
  const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  const int sb = t.sb[c], se = t.se[c], tb = t.tb[c], te = t.te[c];
  const bool split = level < D && (se - sb > leaf_max || te - tb > leaf_max);
  int n = 0;
  if (split) {
    const int shift = 2 * (D - level - 1);
    const uint32_t ix = t.ix[c], iy = t.iy[c];
    int* out = cr + (int64_t)(c - c0) * 16;
    for (int q = 0; q < 4; ++q) {
      const uint32_t prefix = morton(2 * ix + (q & 1), 2 * iy + (q >> 1));
      const uint64_t lo = (uint64_t)prefix << shift;
      const uint64_t hi = (uint64_t)(prefix + 1) << shift;
      const int csb = lower_bound_u32(skey, sb, se, lo);
      const int cse = lower_bound_u32(skey, csb, se, hi);
      const int ctb = lower_bound_u32(tkey, tb, te, lo);
      const int cte = lower_bound_u32(tkey, ctb, te, hi);
      out[4 * q + 0] = csb;
      out[4 * q + 1] = cse;
      out[4 * q + 2] = ctb;
      out[4 * q + 3] = cte;
      n += (cse > csb || cte > ctb) ? 1 : 0;
    }
  }
  cnt[c - c0] = n;
}

__global__ void k_level_emit(TreeArrays t, int c0, int c1, int level, const int* __restrict__ cnt,
                             const int* __restrict__ off, const int* __restrict__ cr, int first_child) {
  const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  const int n = cnt[c - c0];
  if (n == 0) {
    t.child[c] = -1;
    t.nchild[c] = 0;
    return;
  }
  int dst = first_child + off[c - c0];
  t.child[c] = dst;
  t.nchild[c] = n;
  const int ix = t.ix[c], iy = t.iy[c];
  const int* in = cr + (int64_t)(c - c0) * 16;
  for (int q = 0; q < 4; ++q) {
    const int csb = in[4 * q], cse = in[4 * q + 1], ctb = in[4 * q + 2], cte = in[4 * q + 3];
    if (!(cse > csb || cte > ctb)) continue;
    t.lvl[dst] = level + 1;
    t.ix[dst] = 2 * ix + (q & 1);
    t.iy[dst] = 2 * iy + (q >> 1);
    t.sb[dst] = csb;
    t.se[dst] = cse;
    t.tb[dst] = ctb;
    t.te[dst] = cte;
    t.child[dst] = -1;
    t.nchild[dst] = 0;
    t.parent[dst] = c;
    ++dst;
  }
}

__global__ void k_cell_flags(TreeArrays t, int c0, int c1, int kind, int* __restrict__ flag) {
  const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  const bool leaf = t.child[c] < 0;
  const bool hs = t.se[c] > t.sb[c];
  const bool ht = t.te[c] > t.tb[c];
  bool v = false;
  switch (kind) {
    case 0: v = leaf && hs; break;
    case 1: v = leaf && ht; break;
    case 2: v = ht; break;
    case 3: v = !leaf && hs; break;
    default: v = false;
  }
  flag[c - c0] = v ? 1 : 0;
}

__global__ void k_compact(const int* __restrict__ flag, const int* __restrict__ off, int c0, int c1,
                          int* __restrict__ out) {
  const int c = c0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= c1) return;
  if (flag[c - c0]) out[off[c - c0]] = c;
}

// One wave per source leaf: FP32 record (x, y relative to the leaf corner in
// units of h, w) per source; leaf weight sum in FP64 in a fixed order.
__global__ __launch_bounds__(256) void k_pack_sources(TreeArrays t, const int* __restrict__ sleaves, int n, int D,
                                                       const uint32_t* __restrict__ ij, const double* __restrict__ w64,
                                                       float4* __restrict__ src4, double* __restrict__ leaf_w) {
  const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (wid >= n) return;
  const int lane = threadIdx.x % kWave;
  const int c = sleaves[wid];
  const int sh = D - t.lvl[c];
  const int cx = t.ix[c] << sh, cy = t.iy[c] << sh;
  const int sb = t.sb[c], se = t.se[c];
  double acc = 0.0;
  for (int s = sb + lane; s < se; s += kWave) {
    const uint32_t v = ij[s];
    const int i = (int)(v & 0xFFFFu), j = (int)(v >> 16);
    const double w = w64[s];
    src4[s] = make_float4((float)(i - cx) + 0.5f, (float)(j - cy) + 0.5f, (float)w, 0.0f);
    acc += w;
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (lane == 0) leaf_w[c] = acc;
}

// x0 + (i + 1/2) h without contraction: the node coordinate exactly as the
// oracle forms it, so that coincidence is the same FP64 equality on both sides.
__device__ inline double node_coord(double x0, int i, double h) {
#pragma clang fp contract(off)
  const double a = ((double)i + 0.5) * h;
  return x0 + a;
}

__global__ __launch_bounds__(256) void k_prep_targets(TreeArrays t, const int* __restrict__ tleaves, int n, int D,
                                                       const double* __restrict__ tx, const double* __restrict__ ty,
                                                       const int* __restrict__ perm, double x0, double y0, double h,
                                                       int nx, int ny, double snap_frac2,
                                                       float2* __restrict__ rel32, double2* __restrict__ rel64,
                                                       int* __restrict__ tleaf, int* __restrict__ self_idx,
                                                       double* __restrict__ self_logd) {
#pragma clang fp contract(off)
  const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (wid >= n) return;
  const int lane = threadIdx.x % kWave;
  const int c = tleaves[wid];
  const int sh = D - t.lvl[c];
  const double cx = (double)(t.ix[c] << sh), cy = (double)(t.iy[c] << sh);
  const int tb = t.tb[c], te = t.te[c];
  // squared distance below which a target is snapped onto its nearest node
  const double snap2 = h * h * snap_frac2;
  for (int k = tb + lane; k < te; k += kWave) {
    const int o = perm[k];
    const double x = tx[o], y = ty[o];
    const double ux = (x - x0) / h;
    const double uy = (y - y0) / h;
    double rx = ux - cx, ry = uy - cy;
    const double fx = floor(ux), fy = floor(uy);
    const bool inside = fx >= 0.0 && fy >= 0.0 && fx < 65536.0 && fy < 65536.0;
    const int i = inside ? (int)fx : -1, j = inside ? (int)fy : -1;
    int sidx = -1;
    double lg = 0.0;
    if (i >= 0 && j >= 0 && i < nx && j < ny) {
      const double dx = x - node_coord(x0, i, h);
      const double dy = y - node_coord(y0, j, h);
      const double d2 = dx * dx + dy * dy;
      if (d2 == 0.0 || d2 < snap2) {
        sidx = j * nx + i;
        lg = (d2 == 0.0) ? -INFINITY : 0.5 * log(d2);
        rx = ((double)i + 0.5) - cx;
        ry = ((double)j + 0.5) - cy;
      }
    }
    rel64[k] = make_double2(rx, ry);
    rel32[k] = make_float2((float)rx, (float)ry);
    tleaf[k] = c;
    self_idx[k] = sidx;
    self_logd[k] = lg;
  }
}

}  // namespace

void tree_init_root(TreeArrays t, const int* nsrc_dev, int ntgt, hipStream_t s) {
  k_root<<<1, 1, 0, s>>>(t, nsrc_dev, ntgt);
}

void tree_level_count(TreeArrays t, int c0, int c1, int level, int D, int leaf_max, const uint32_t* skey,
                      const uint32_t* tkey, int* cnt, int* cr, hipStream_t s) {
  const int n = c1 - c0;
  if (n <= 0) return;
  k_level_count<<<(n + 127) / 128, 128, 0, s>>>(t, c0, c1, level, D, leaf_max, skey, tkey, cnt, cr);
}

void tree_level_emit(TreeArrays t, int c0, int c1, int level, const int* cnt, const int* off, const int* cr,
                     int first_child, hipStream_t s) {
  const int n = c1 - c0;
  if (n <= 0) return;
  k_level_emit<<<(n + 127) / 128, 128, 0, s>>>(t, c0, c1, level, cnt, off, cr, first_child);
}

void cell_flags(TreeArrays t, int c0, int c1, int kind, int* flag, hipStream_t s) {
  const int n = c1 - c0;
  if (n <= 0) return;
  k_cell_flags<<<(n + 255) / 256, 256, 0, s>>>(t, c0, c1, kind, flag);
}

void compact_indices(const int* flag, const int* off, int c0, int c1, int* out, hipStream_t s) {
  const int n = c1 - c0;
  if (n <= 0) return;
  k_compact<<<(n + 255) / 256, 256, 0, s>>>(flag, off, c0, c1, out);
}

void leaf_pack_sources(TreeArrays t, const int* sleaves, int nsleaves, int D, const uint32_t* ij, const double* w64,
                       float4* src4, double* leaf_w, hipStream_t s) {
  if (nsleaves <= 0) return;
  k_pack_sources<<<(nsleaves + 3) / 4, 256, 0, s>>>(t, sleaves, nsleaves, D, ij, w64, src4, leaf_w);
}

void leaf_prep_targets(TreeArrays t, const int* tleaves, int ntleaves, int D, const double* tx, const double* ty,
                       const int* perm, double x0, double y0, double h, int nx, int ny, double snap_frac2,
                       float2* rel32, double2* rel64, int* tleaf, int* self_idx, double* self_logd, hipStream_t s) {
  if (ntleaves <= 0) return;
  k_prep_targets<<<(ntleaves + 3) / 4, 256, 0, s>>>(t, tleaves, ntleaves, D, tx, ty, perm, x0, y0, h, nx, ny,
                                                     snap_frac2, rel32, rel64, tleaf, self_idx, self_logd);
}

}  // namespace pp
