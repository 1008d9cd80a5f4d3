// Per-leaf passes before the near field: packing of the source leaves and
// preparation of the target leaves, for grid sources and for scattered
// sources.  One wave per leaf.  Shared by their own launch and by the
// interaction-list launch, which runs them in extra workgroups.
#pragma once

#include "blockscan.h"
#include "internal.h"

namespace pp {

// One wave packs source leaf c.
__device__ inline void pack_leaf_cell(int c, int lane, const TreeArrays& t, int D, const uint32_t* __restrict__ ij,
                                      const double* __restrict__ w64, float* __restrict__ s32, int64_t stride,
                                      double* __restrict__ leaf_w) {
  const int sh = D - t.lvl[c];
  const int cx = t.ix[c] << sh, cy = t.iy[c] << sh;
  const int sb = t.sb[c], se = t.se[c];
  double acc = 0.0;
  for (int s = sb + lane; s < se; s += kWave) {
    const uint32_t v = ij[s];
    const int i = (int)(v & 0xFFFFu), j = (int)(v >> 16);
    const double w = w64[s];
    s32[s] = (float)(i - cx) + 0.5f;
    s32[stride + s] = (float)(j - cy) + 0.5f;
    s32[2 * stride + s] = (float)w;
    acc += w;
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (lane == 0) leaf_w[c] = acc;
}

// One wave packs the grid source leaves cs[0..n) (n <= 4, the same for every
// lane) with their loads issued together; per leaf the same records and the
// same weight sum (per-lane order, then the butterfly) as pack_leaf_cell.
__device__ inline void pack_leaf_cells4(const int* cs, int n, int lane, const TreeArrays& t, int D,
                                        const uint32_t* __restrict__ ij, const double* __restrict__ w64,
                                        float* __restrict__ s32, int64_t stride, double* __restrict__ leaf_w) {
  int cx[4], cy[4], sb[4], se[4];
  int span = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    cx[q] = cy[q] = sb[q] = se[q] = 0;
    if (q < n) {
      const int c = cs[q];
      const int sh = D - t.lvl[c];
      cx[q] = t.ix[c] << sh;
      cy[q] = t.iy[c] << sh;
      sb[q] = t.sb[c];
      se[q] = t.se[c];
      span = max(span, se[q] - sb[q]);
    }
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int o = lane; o < span; o += kWave) {
    uint32_t v[4];
    double w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int s = sb[q] + o;
      const bool ok = s < se[q];
      v[q] = ok ? ij[s] : 0u;
      w[q] = ok ? w64[s] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int s = sb[q] + o;
      if (s < se[q]) {
        const int i = (int)(v[q] & 0xFFFFu), j = (int)(v[q] >> 16);
        s32[s] = (float)(i - cx[q]) + 0.5f;
        s32[stride + s] = (float)(j - cy[q]) + 0.5f;
        s32[2 * stride + s] = (float)w[q];
        acc[q] += w[q];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) acc[q] += __shfl_xor(acc[q], o, kWave);
    if (q < n && lane == 0) leaf_w[cs[q]] = acc[q];
  }
}

// One wave packs source leaf sleaves[wid].
__device__ inline void pack_leaf(int wid, int lane, const TreeArrays& t, const int* __restrict__ sleaves, int D,
                                 const uint32_t* __restrict__ ij, const double* __restrict__ w64,
                                 float* __restrict__ s32, int64_t stride, double* __restrict__ leaf_w) {
  pack_leaf_cell(sleaves[wid], lane, t, D, ij, w64, s32, stride, leaf_w);
}

// x0 + (i + 1/2) h without contraction: the node coordinate exactly as the
// oracle forms it, so that coincidence is the same FP64 equality on both sides.
__device__ inline double node_coord(double x0, int i, double h) {
#pragma clang fp contract(off)
  const double a = ((double)i + 0.5) * h;
  return x0 + a;
}

// One wave prepares the targets of target leaf tleaves[wid].
// bt.nreq > 0: a forest of requests; target o is target o - toff[r] of
// request r, whose grid f[r] sits at offset (vx, vy) of the joint index space,
// and offsets are formed in the request's own frame (bit for bit its lone
// solve's).
__device__ inline void prep_leaf(int wid, int lane, const TreeArrays& t, const int* __restrict__ tleaves, int D,
                                 const double* __restrict__ tx, const double* __restrict__ ty,
                                 const int* __restrict__ perm, double x0, double y0, double h, int nx, int ny,
                                 double snap_frac2, const double* __restrict__ f, float2* __restrict__ rel32,
                                 double2* __restrict__ rel64, int* __restrict__ tleaf, double* __restrict__ self_w,
                                 double* __restrict__ self_logd, const GridBatch& bt) {
#pragma clang fp contract(off)
  const int c = tleaves[wid];
  const int sh = D - t.lvl[c];
  const int tb = t.tb[c], te = t.te[c];
  // squared distance below which a target is snapped onto its nearest node
  const double snap2 = h * h * snap_frac2;
  for (int k = tb + lane; k < te; k += kWave) {
    const int o = perm[k];
    double x, y;
    const double* fr = f;
    int vx = 0, vy = 0;
    if (bt.nreq) {
      const int r = batch_request(bt, o);
      const int64_t j = o - bt.toff[r];
      x = bt.tx[r][j];
      y = bt.ty[r][j];
      fr = bt.f[r];
      vx = (int)compact_bits((uint32_t)r) << bt.D;
      vy = (int)compact_bits((uint32_t)r >> 1) << bt.D;
    } else {
      x = tx[o];
      y = ty[o];
    }
    const double cx = (double)((t.ix[c] << sh) - vx), cy = (double)((t.iy[c] << sh) - vy);
    const double ux = (x - x0) / h;
    const double uy = (y - y0) / h;
    double rx = ux - cx, ry = uy - cy;
    const double fx = floor(ux), fy = floor(uy);
    const bool inside = fx >= 0.0 && fy >= 0.0 && fx < 65536.0 && fy < 65536.0;
    const int i = inside ? (int)fx : -1, j = inside ? (int)fy : -1;
    double sw = 0.0, lg = 0.0;
    if (i >= 0 && j >= 0 && i < nx && j < ny) {
      const double dx = x - node_coord(x0, i, h);
      const double dy = y - node_coord(y0, j, h);
      const double d2 = dx * dx + dy * dy;
      if (d2 == 0.0 || d2 < snap2) {
        sw = fr[(int64_t)j * nx + i] * (h * h);
        lg = (d2 == 0.0) ? -INFINITY : 0.5 * log(d2);
        rx = ((double)i + 0.5) - cx;
        ry = ((double)j + 0.5) - cy;
      }
    }
    rel64[k] = make_double2(rx, ry);
    rel32[k] = make_float2((float)rx, (float)ry);
    tleaf[k] = c;
    self_w[k] = sw;
    self_logd[k] = lg;
  }
}

// One wave per source leaf: offsets from the leaf corner in units of u, FP32
// (with the weight) and FP64, and the FP64 leaf weight in a fixed order.
__device__ inline void pack_point_cell(int c, int lane, const TreeArrays& t, int D, const double* __restrict__ xs,
                                       const double* __restrict__ ys, const double* __restrict__ ws, double x0,
                                       double y0, double u, float* __restrict__ s32, int64_t stride,
                                       double2* __restrict__ s64, double* __restrict__ leaf_w) {
  const int sh = D - t.lvl[c];
  const double cx = (double)(t.ix[c] << sh), cy = (double)(t.iy[c] << sh);
  const int sb = t.sb[c], se = t.se[c];
  double acc = 0.0;
  for (int s = sb + lane; s < se; s += kWave) {
    const double rx = (xs[s] - x0) / u - cx;
    const double ry = (ys[s] - y0) / u - cy;
    const double w = ws[s];
    s32[s] = (float)rx;
    s32[stride + s] = (float)ry;
    s32[2 * stride + s] = (float)w;
    s64[s] = make_double2(rx, ry);
    acc += w;
  }
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
  if (lane == 0) leaf_w[c] = acc;
}
__device__ inline void pack_point_leaf(int wid, int lane, const TreeArrays& t, const int* __restrict__ sleaves, int D,
                                       const double* __restrict__ xs, const double* __restrict__ ys,
                                       const double* __restrict__ ws, double x0, double y0, double u,
                                       float* __restrict__ s32, int64_t stride, double2* __restrict__ s64,
                                       double* __restrict__ leaf_w) {
  pack_point_cell(sleaves[wid], lane, t, D, xs, ys, ws, x0, y0, u, s32, stride, s64, leaf_w);
}

// One wave per target leaf: offsets from the leaf corner (the same FP64
// operations as for the sources, so coincident points get identical offsets),
// the owning leaf, and the summed weight of the sources that coincide exactly
// with the target (they are skipped by the near-field kernel, and the finalize
// step removes their share of the near weight).
__device__ inline void prep_point_leaf(int wid, int lane, const TreeArrays& t, const int* __restrict__ tleaves, int D,
                                       const double* __restrict__ tx, const double* __restrict__ ty,
                                       const int* __restrict__ perm, double x0, double y0, double u,
                                       const double* __restrict__ xs, const double* __restrict__ ys,
                                       const double* __restrict__ ws, float2* __restrict__ rel32,
                                       double2* __restrict__ rel64, int* __restrict__ tleaf,
                                       double* __restrict__ self_w) {
  const int c = tleaves[wid];
  const int sh = D - t.lvl[c];
  const double cx = (double)(t.ix[c] << sh), cy = (double)(t.iy[c] << sh);
  const int tb = t.tb[c], te = t.te[c], sb = t.sb[c], se = t.se[c];
  for (int k = tb + lane; k < te; k += kWave) {
    const int o = perm[k];
    const double x = tx[o], y = ty[o];
    const double rx = (x - x0) / u - cx;
    const double ry = (y - y0) / u - cy;
    double sw = 0.0;
    for (int s = sb; s < se; ++s)
      if (xs[s] == x && ys[s] == y) sw += ws[s];
    rel64[k] = make_double2(rx, ry);
    rel32[k] = make_float2((float)rx, (float)ry);
    tleaf[k] = c;
    self_w[k] = sw;
  }
}

// Arguments of the two passes for grid sources.
struct PackArgs {
  const int* sleaves;
  int ns;
  const uint32_t* ij;
  const double* w64;
  float* s32;
  int64_t stride;
  double* leaf_w;
};
struct PrepArgs {
  const int* tleaves;
  int nt;
  const double* tx;
  const double* ty;
  const int* perm;
  double x0, y0, h;
  int nx, ny;
  double snap_frac2;
  const double* f;
  float2* rel32;
  double2* rel64;
  int* tleaf;
  double* self_w;
  double* self_logd;
  GridBatch bt;
};

// Arguments of the two passes for scattered sources.
struct PointFrame {
  double x0, y0, u;
  const double* xs;
  const double* ys;
  const double* ws;
};
struct PointArgs {
  PointFrame fr;
  const int* sleaves;
  int ns;
  float* s32;
  int64_t stride;
  double2* s64;
  double* leaf_w;
  const int* tleaves;
  int nt;
  const double* tx;
  const double* ty;
  const int* perm;
  float2* rel32;
  double2* rel64;
  int* tleaf;
  double* self_w;
};

// The passes as extra workgroups of another launch (256 threads, one wave per
// leaf): blocks [0, pack_blocks) pack source leaves, the next prep_blocks
// prepare target leaves.  kind 0: none, 1: grid sources, 2: scattered sources.
struct LeafPass {
  int kind = 0;
  int pack_blocks = 0, prep_blocks = 0;
  TreeArrays t{};
  int D = 0;
  PackArgs ga{};
  PrepArgs gb{};
  PointArgs pa{};
};

__device__ inline void run_leaf_pass(const LeafPass& lp, int blk) {
  const int lane = threadIdx.x % kWave;
  const bool pack = blk < lp.pack_blocks;
  const int wid = (pack ? blk : blk - lp.pack_blocks) * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (lp.kind == 1) {
    if (pack) {
      if (wid < lp.ga.ns) pack_leaf(wid, lane, lp.t, lp.ga.sleaves, lp.D, lp.ga.ij, lp.ga.w64, lp.ga.s32, lp.ga.stride,
                                    lp.ga.leaf_w);
    } else if (wid < lp.gb.nt) {
      const PrepArgs& b = lp.gb;
      prep_leaf(wid, lane, lp.t, b.tleaves, lp.D, b.tx, b.ty, b.perm, b.x0, b.y0, b.h, b.nx, b.ny, b.snap_frac2, b.f,
                b.rel32, b.rel64, b.tleaf, b.self_w, b.self_logd, b.bt);
    }
  } else if (lp.kind == 2) {
    const PointArgs& a = lp.pa;
    if (pack) {
      if (wid < a.ns)
        pack_point_leaf(wid, lane, lp.t, a.sleaves, lp.D, a.fr.xs, a.fr.ys, a.fr.ws, a.fr.x0, a.fr.y0, a.fr.u, a.s32,
                        a.stride, a.s64, a.leaf_w);
    } else if (wid < a.nt) {
      prep_point_leaf(wid, lane, lp.t, a.tleaves, lp.D, a.tx, a.ty, a.perm, a.fr.x0, a.fr.y0, a.fr.u, a.fr.xs, a.fr.ys,
                      a.fr.ws, a.rel32, a.rel64, a.tleaf, a.self_w);
    }
  }
}

// One wave packs source leaf c, for either kind of source.
__device__ inline void run_pack_cell(const LeafPass& lp, int c, int lane) {
  if (lp.kind == 1)
    pack_leaf_cell(c, lane, lp.t, lp.D, lp.ga.ij, lp.ga.w64, lp.ga.s32, lp.ga.stride, lp.ga.leaf_w);
  else if (lp.kind == 2)
    pack_point_cell(c, lane, lp.t, lp.D, lp.pa.fr.xs, lp.pa.fr.ys, lp.pa.fr.ws, lp.pa.fr.x0, lp.pa.fr.y0, lp.pa.fr.u,
                    lp.pa.s32, lp.pa.stride, lp.pa.s64, lp.pa.leaf_w);
}

// Host side: the descriptor of the passes for one solve.
LeafPass leaf_pass_grid(TreeArrays t, int D, const int* sleaves, int nsleaves, const uint32_t* ij, const double* w64,
                        float* s32, int64_t stride, double* leaf_w, const int* tleaves, int ntleaves, const double* tx,
                        const double* ty, const int* perm, double x0, double y0, double h, int nx, int ny,
                        double snap_frac2, const double* f, float2* rel32, double2* rel64, int* tleaf, double* self_w,
                        double* self_logd, const GridBatch* bt);
LeafPass leaf_pass_points(TreeArrays t, int D, double x0, double y0, double u, const double* xs, const double* ys,
                          const double* ws, const int* sleaves, int nsleaves, float* s32, int64_t stride,
                          double2* s64, double* leaf_w, const int* tleaves, int ntleaves, const double* tx,
                          const double* ty, const int* perm, float2* rel32, double2* rel64, int* tleaf,
                          double* self_w);
// The passes as a launch of their own.
void leaf_pass_launch(const LeafPass& lp, hipStream_t s);
// The same passes with the source packing left out (target preparation only).
LeafPass leaf_pass_prep_only(const LeafPass& lp);
// Packing of only the source leaves that the near field reads: those in the
// list (list_src + list_off[A], list_cnt[A] entries) of some target leaf A of
// tleaves, each packed once (claim: ncells ints, all zero before).  lp: the
// descriptor of the full passes.
void pack_listed(const LeafPass& lp, const int* tleaves, int ntleaves, const int* list_off, const int* list_cnt,
                 const int* list_src, int ncells, int* claim, hipStream_t s);

}  // namespace pp
