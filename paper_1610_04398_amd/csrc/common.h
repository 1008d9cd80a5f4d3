// Internal definitions shared by the HIP kernels and the host pipeline of the
// pressure-Poisson tree-code library.  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pp {

// Largest supported expansion order; kernels are instantiated for the order
// buckets below and take the exact order p <= bucket at run time.
constexpr int kMaxP = 20;
constexpr int kMaxDepth = 16;  // finest level; keys are 2*16 bits

// 1/(2 pi), ln 2, and the cell-average constant kappa = 3/2 - pi/4 + ln(2)/2
constexpr double kInv2Pi = 0.15915494309189533577;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kKappa = 1.0611754268825244;

// Error flags raised by kernels (bit mask in a device word).
enum : int {
  kFlagNonFiniteSource = 1,
  kFlagNonFiniteTarget = 2,
  kFlagTargetOutside = 4,
  kFlagFrontierOverflow = 8,
  kFlagCellOverflow = 16,
  kFlagListOverflow = 32,
  kFlagBadIndex = 64,  // a list entry outside the tree (an internal error); the entry is skipped
  kFlagStale = 128,    // resident solve: the retained tree does not fit the new sources or targets
};

struct cplx {
  double x, y;
};

__host__ __device__ inline cplx cadd(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline cplx cscale(cplx a, double s) { return {a.x * s, a.y * s}; }

// Error-free transformations in FP32: a + b = s + e exactly (Knuth's TwoSum),
// and a b = p + e exactly (with a fused multiply-add).  Contraction is off in
// both (and wherever their results are combined): a product fused into a
// later sum would no longer be the value whose error was captured.
__device__ inline float two_sum(float a, float b, float& e) {
#pragma clang fp contract(off)
  const float s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
  return s;
}
__device__ inline float two_prod(float a, float b, float& e) {
#pragma clang fp contract(off)
  const float q = a * b;
  e = fmaf(a, b, -q);
  return q;
}

// L2P at one target: Re sum_l L'_l u^l with u = (t - z_c) / s_c, from the
// target's offset r to its leaf's corner (units of h) and the leaf at level
// lvl of a root with 2^D cells per side.
// FP64: Horner.  FP32 (mixed path): compensated Horner (Graillat, Langlois and
// Louvet's scheme, in complex arithmetic): every step's rounding errors, exact
// through the transformations above, are collected in a second Horner
// recurrence that runs beside the first and is added at the end; u and each
// coefficient are carried as an FP32 pair (high part + rounding remainder),
// whose low parts enter that error recurrence.  The result is as accurate as
// an evaluation in twice FP32's precision.
__device__ inline double l2p_eval(const double2* __restrict__ Lg, int p, double2 r, int D, int lvl, bool fp32) {
  const double side = (double)(1 << (D - lvl)), inv = ldexp(1.0, lvl - D);
  // every coefficient's load issued before the evaluation needs the first
  double2 L[kMaxP + 1];
#pragma unroll
  for (int l = 0; l <= kMaxP; ++l) L[l] = l <= p ? Lg[l] : make_double2(0.0, 0.0);
  if (fp32) {
#pragma clang fp contract(off)
    const double uxd = (r.x - 0.5 * side) * inv, uyd = (r.y - 0.5 * side) * inv;
    const float ux = (float)uxd, uy = (float)uyd;
    const float uxl = (float)(uxd - (double)ux), uyl = (float)(uyd - (double)uy);
    float ax = 0.f, ay = 0.f;  // the running value
    float ex = 0.f, ey = 0.f;  // the running error
#pragma unroll
    for (int l = kMaxP; l >= 0; --l) {
      if (l > p) continue;
      const double2 v = L[l];
      const float cx = (float)v.x, cy = (float)v.y;
      const float cxl = (float)(v.x - (double)cx), cyl = (float)(v.y - (double)cy);
      // a * u, exactly as rounded parts plus errors
      float e1, e2, e3, e4, e5, e6, e7, e8;
      const float p1 = two_prod(ax, ux, e1), p2 = two_prod(ay, uy, e2);
      const float p3 = two_prod(ax, uy, e3), p4 = two_prod(ay, ux, e4);
      const float pr = two_sum(p1, -p2, e5), pi = two_sum(p3, p4, e6);
      // + the coefficient
      const float nx = two_sum(pr, cx, e7), ny = two_sum(pi, cy, e8);
      // this step's error: the transformations' parts, the low parts of the
      // coefficient, and a times the low part of u
      const float lx = ((e1 - e2) + e5 + e7) + (cxl + (ax * uxl - ay * uyl));
      const float ly = ((e3 + e4) + e6 + e8) + (cyl + (ax * uyl + ay * uxl));
      // the error recurrence: e = e u + this step's error
      const float tx = ex * ux - ey * uy + lx;
      const float ty = ex * uy + ey * ux + ly;
      ex = tx;
      ey = ty;
      ax = nx;
      ay = ny;
    }
    return (double)ax + (double)ex;
  }
  const cplx u = {(r.x - 0.5 * side) * inv, (r.y - 0.5 * side) * inv};
  cplx acc = {0.0, 0.0};
#pragma unroll
  for (int l = kMaxP; l >= 0; --l) {
    if (l > p) continue;
    const double2 v = L[l];
    acc = cadd(cmul(acc, u), {v.x, v.y});
  }
  return acc.x;
}

// Morton bit spreading: bit b of v goes to bit 2b.
__host__ __device__ inline uint32_t spread_bits(uint32_t v) {
  v &= 0xFFFFu;
  v = (v | (v << 8)) & 0x00FF00FFu;
  v = (v | (v << 4)) & 0x0F0F0F0Fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}
__host__ __device__ inline uint32_t compact_bits(uint32_t v) {
  v &= 0x55555555u;
  v = (v | (v >> 1)) & 0x33333333u;
  v = (v | (v >> 2)) & 0x0F0F0F0Fu;
  v = (v | (v >> 4)) & 0x00FF00FFu;
  v = (v | (v >> 8)) & 0x0000FFFFu;
  return v;
}
__host__ __device__ inline uint32_t morton(uint32_t ix, uint32_t iy) { return spread_bits(ix) | (spread_bits(iy) << 1); }

// Finest-cell Morton key of a target: floor((t - x0) / h) per axis with the
// same FP64 operations (subtract, then divide; no contraction) as the
// reference tree, in a root of 2^k cells per side.  *err: 1 for a non-finite
// coordinate, 2 for a target outside the root (the key is then 0).
__device__ inline uint32_t target_key(double x, double y, double x0, double y0, double h, int k, int* err) {
#pragma clang fp contract(off)
  if (!isfinite(x) || !isfinite(y)) {
    *err = 1;
    return 0;
  }
  const double ux = floor((x - x0) / h);
  const double uy = floor((y - y0) / h);
  const double lim = (double)(1u << k);
  if (!(ux >= 0.0 && ux < lim && uy >= 0.0 && uy < lim)) {
    *err = 2;
    return 0;
  }
  return morton((uint32_t)ux, (uint32_t)uy);
}

// Device view of the quadtree: structure-of-arrays over all cells, numbered
// level by level (root = 0), children of a cell contiguous and in quadrant
// order q = qx + 2 qy.
// Workgroups are dispatched to the 8 XCDs round-robin (workgroup b runs on
// XCD b % 8), and each XCD has its own L2.  This maps the hardware index to a
// logical one so that each XCD receives one contiguous 1/8 of the logical
// range: work that is close in the logical order (neighbouring leaves) shares
// an L2.  A bijection of [0, G).
constexpr int kXcds = 8;
__device__ inline int xcd_contiguous(int b, int G) {
  const int q = G / kXcds, r = G % kXcds, x = b % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}

struct TreeView {
  int D;               // finest level
  int ncells;
  const int* lvl;
  const int* ix;
  const int* iy;
  const int* sb;       // source range [sb, se) into the Morton-ordered sources
  const int* se;
  const int* tb;       // target range [tb, te) into the sorted targets
  const int* te;
  const int* child;    // first child, or -1 for a leaf
  const int* nchild;
  const int* parent;   // -1 for the root
};

// Per-cell setup of the interaction lists: the cell's packed traversal record
// {ix, iy, first child, meta} with meta = level | nchild << 5 |
// (children-with-sources mask) << 8 | has_src << 12, its list counts cleared,
// and for the one-pass lists (cap_m > 0) the fixed-capacity offsets c * cap.
struct RecordArgs {
  TreeView t;
  int4* rec;
  int* cnt_m;
  int* cnt_p;
  int* off_m;
  int* off_p;
  int cap_m, cap_p;
};
__device__ inline void cell_setup(const RecordArgs& a, int c) {
  a.cnt_m[c] = 0;
  a.cnt_p[c] = 0;
  if (a.cap_m > 0) {
    a.off_m[c] = c * a.cap_m;
    a.off_p[c] = c * a.cap_p;
  }
  const int k0 = a.t.child[c], nk = a.t.nchild[c];
  int mask = 0;
  for (int q = 0; q < nk; ++q) mask |= (a.t.se[k0 + q] > a.t.sb[k0 + q]) ? (1 << q) : 0;
  const int meta = a.t.lvl[c] | (nk << 5) | (mask << 8) | ((a.t.se[c] > a.t.sb[c]) ? (1 << 12) : 0);
  a.rec[c] = make_int4(a.t.ix[c], a.t.iy[c], k0, meta);
}

// Exact acceptance test (r_A + r_B) < theta d with theta = num/den, all in
// units of half a finest cell: (S_A + S_B)^2 den^2 < 2 num^2 d^2.
__host__ __device__ inline bool mac_accept(int D, int la, int ixa, int iya, int lb, int ixb, int iyb, int num,
                                           int den) {
  const int64_t cax = (int64_t)(2 * ixa + 1) << (D - la);
  const int64_t cay = (int64_t)(2 * iya + 1) << (D - la);
  const int64_t cbx = (int64_t)(2 * ixb + 1) << (D - lb);
  const int64_t cby = (int64_t)(2 * iyb + 1) << (D - lb);
  const int64_t s = ((int64_t)1 << (D - la + 1)) + ((int64_t)1 << (D - lb + 1));
  const int64_t dx = cax - cbx, dy = cay - cby;
  const int64_t lhs = s * s * (int64_t)den * (int64_t)den;
  const int64_t rhs = 2 * (int64_t)num * (int64_t)num * (dx * dx + dy * dy);
  return lhs < rhs;
}

// Acceptance of source cell B for every target of leaf A in the paper's
// tree-code (a group is used through its expansion when it is far enough from
// the target): S_B / d < theta with d the distance from A's square to B's
// centre, exactly in integers (half-finest-cell units): S_B^2 den^2 < num^2 d^2.
__host__ __device__ inline bool treecode_accept(int D, int la, int ixa, int iya, int lb, int ixb, int iyb, int num,
                                                int den) {
  const int64_t ax0 = (int64_t)(2 * ixa) << (D - la), ax1 = (int64_t)(2 * ixa + 2) << (D - la);
  const int64_t ay0 = (int64_t)(2 * iya) << (D - la), ay1 = (int64_t)(2 * iya + 2) << (D - la);
  const int64_t cx = (int64_t)(2 * ixb + 1) << (D - lb);
  const int64_t cy = (int64_t)(2 * iyb + 1) << (D - lb);
  const int64_t dx = ax0 > cx ? ax0 - cx : (cx > ax1 ? cx - ax1 : 0);
  const int64_t dy = ay0 > cy ? ay0 - cy : (cy > ay1 ? cy - ay1 : 0);
  const int64_t s = (int64_t)1 << (D - lb + 1);
  return s * s * (int64_t)den * (int64_t)den < (int64_t)num * (int64_t)num * (dx * dx + dy * dy);
}

}  // namespace pp
