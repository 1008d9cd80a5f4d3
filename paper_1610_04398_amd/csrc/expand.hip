// Expansion passes in FP64: P2M, M2M, M2L, L2L, L2P.
//
// Notation: the sources of a cell with centre z_c and side s have the
// multipole expansion  Phi(z) = a_0 log(z - z_c) + sum_{k=1..p} a_k (z - z_c)^-k
// with a_0 = S = sum w and a_k = -alpha_k = -sum w (z_i - z_c)^k / k
// (Appendix A, eq. alphaK and eq. pressTruncated; P = Re Phi / 2pi).  Stored
// coefficients are scaled by the cell side, a'_k = a_k / s^k, and locals
// L'_l = L_l s^l, so every operator acts on O(1) numbers and depends only on
// offsets measured in cell sides.  Positions are in units of the finest cell
// (h), where every cell centre is exact in FP64.
//
// M2M is the re-centring of eq. expandedShift with the S term's sign derived
// from eq. logExpansion (+S z0^k / k in the paper's alpha convention; the
// printed minus sign does not reproduce the parent's expansion).  M2L, L2L and
// L2P are the local-expansion operators of the fast multipole method that the
// paper cites, derived from the same series:
//   M2L (z0 = z_B - z_A, t = s_A / z0, r = s_B / z0):
//     L'_0 = a_0 ln|z0| + sum_k a'_k (-r)^k
//     L'_l = t^l [ -a_0 / l + sum_k C(l+k-1, k-1) a'_k (-r)^k ],  l >= 1
//   L2L (d = (z_child - z_parent) / s_parent):
//     L'_m(child) = 2^-m sum_{k>=m} C(k, m) d^(k-m) L'_k(parent)
//   M2M (d as above):
//     a'_l(parent) += -a_0 d^l / l + sum_{k=1..l} C(l-1, k-1) 2^-k d^(l-k) a'_k(child)
//   L2P: far(z) = Re sum_l L'_l u^l,  u = (z - z_c) / s.
#include <algorithm>
#include <cstdlib>
#include <mutex>

#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {

struct BinomTable {
  double v[2 * kMaxP + 1][2 * kMaxP + 1];
};
constexpr BinomTable make_binom() {
  BinomTable b{};
  for (int n = 0; n <= 2 * kMaxP; ++n) {
    b.v[n][0] = 1.0;
    for (int k = 1; k <= n; ++k) b.v[n][k] = b.v[n - 1][k - 1] + (k <= n - 1 ? b.v[n - 1][k] : 0.0);
  }
  return b;
}
__constant__ BinomTable c_binom = make_binom();

__device__ inline double binom(int n, int k) { return c_binom.v[n][k]; }

__device__ inline double cell_side(int D, int l) { return (double)(1 << (D - l)); }
// 1 / cell_side, exact (a power of two): x * inv_cell_side equals x / cell_side.
__device__ inline double inv_cell_side(int D, int l) { return ldexp(1.0, l - D); }

// Offset of child quadrant from its parent's centre, in parent sides.
__device__ inline cplx quadrant_offset(int ix, int iy) {
  return {(ix & 1) ? 0.25 : -0.25, (iy & 1) ? 0.25 : -0.25};
}

// P2M: LANES lanes per source leaf (8 by default: eight leaves per wave);
// lanes stride over the leaf's sources, four sources per lane per step with
// their loads issued together, and the per-lane powers are summed across the
// lane group by DPP moves (plain VALU, no LDS round trips): within quads
// (lane xor 1, xor 2), then half rows (mirror: lane i with 7 - i), then rows
// (rotate by 8).  After each step the lanes of a group hold bitwise equal
// sums (the partner's value is added in the same order).  The source offsets
// from the leaf corner (units of the finest cell) are formed here from the
// ordered sources, as the packing step forms them for the near field, so P2M
// does not wait for that step: grid nodes from their packed index (exact
// half-integers), scattered sources from their FP64 coordinates.
template <int CTRL>
__device__ inline double dpp_add(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return v + __hiloint2double(hi, lo);
}

template <int LANES>
__device__ inline double group_sum(double v) {
  v = dpp_add<0xB1>(v);                     // quad_perm [1, 0, 3, 2]
  v = dpp_add<0x4E>(v);                     // quad_perm [2, 3, 0, 1]
  if (LANES >= 8) v = dpp_add<0x141>(v);    // row_half_mirror
  if (LANES >= 16) v = dpp_add<0x128>(v);   // row_ror:8
  return v;
}

// One source leaf c, LANES lanes (sub = the lane's index in its group); only
// a group with store set writes the leaf's coefficients.
template <int PM, int LANES>
__device__ inline void p2m_leaf(const TreeView& t, int c, int sub, bool store, const uint32_t* __restrict__ ij,
                                const double* __restrict__ xs, const double* __restrict__ ys, double x0, double y0,
                                double u, const double* __restrict__ w64, int p, double2* __restrict__ mp) {
  const double side = cell_side(t.D, t.lvl[c]);
  const double inv = 1.0 / side;
  const int sh = t.D - t.lvl[c];
  const int cxi = t.ix[c] << sh, cyi = t.iy[c] << sh;
  cplx acc[PM + 1];
#pragma unroll
  for (int k = 0; k <= PM; ++k) acc[k] = {0.0, 0.0};
  const int sb = t.sb[c], se = t.se[c];
  // four sources per lane per step (a missing source gets weight 0 at the
  // leaf corner and adds nothing)
  constexpr int kR = 4;
  for (int s = sb + sub; s < se; s += kR * LANES) {
    double ox[kR], oy[kR], w[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int sr = s + r * LANES;
      const bool ok = sr < se;
      if (ij) {
        const uint32_t v = ok ? ij[sr] : (uint32_t)cxi | ((uint32_t)cyi << 16);
        ox[r] = (double)((int)(v & 0xFFFFu) - cxi) + 0.5;
        oy[r] = (double)((int)(v >> 16) - cyi) + 0.5;
      } else {
        ox[r] = ok ? (xs[sr] - x0) / u - (double)cxi : 0.0;
        oy[r] = ok ? (ys[sr] - y0) / u - (double)cyi : 0.0;
      }
      w[r] = ok ? w64[sr] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const cplx z = {ox[r] * inv - 0.5, oy[r] * inv - 0.5};
      acc[0].x += w[r];
      cplx zk = {w[r] * z.x, w[r] * z.y};
#pragma unroll
      for (int k = 1; k <= PM; ++k) {
        acc[k] = cadd(acc[k], zk);
        zk = cmul(zk, z);
      }
    }
  }
#pragma unroll
  for (int k = 0; k <= PM; ++k) {
    acc[k].x = group_sum<LANES>(acc[k].x);
    acc[k].y = group_sum<LANES>(acc[k].y);
  }
  if (!store) return;
  double2* out = mp + (int64_t)c * (p + 1);
#pragma unroll
  for (int k = 0; k <= PM; ++k)
    if (k <= p && (k % LANES) == sub)
      out[k] = (k == 0) ? make_double2(acc[0].x, 0.0) : make_double2(-acc[k].x / k, -acc[k].y / k);
}

template <int PM, int LANES>
__global__ __launch_bounds__(256) void k_p2m(TreeView t, const int* __restrict__ sleaves, int n,
                                             const uint32_t* __restrict__ ij, const double* __restrict__ xs,
                                             const double* __restrict__ ys, double x0, double y0, double u,
                                             const double* __restrict__ w64, int p, double2* __restrict__ mp) {
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int li = (int)(gtid / LANES);
  const int sub = (int)(gtid % LANES);
  // every lane of a group takes part in the group sums: lanes past the last
  // leaf work on a copy of it and store nothing
  const int c = sleaves[li < n ? li : n - 1];
  p2m_leaf<PM, LANES>(t, c, sub, li < n, ij, xs, ys, x0, y0, u, w64, p, mp);
}

// P2M of grid leaves 8 nodes wide, the usual leaf of a grid source: the 64
// node positions of such a leaf, relative to its centre, are the same for
// every leaf (zeta = ((x + 1/2) / 8 - 1/2, (y + 1/2) / 8 - 1/2), x, y = 0..7).
// So a'_k = -(1/k) sum_s w_s zeta_s^k (and a'_0 = sum_s w_s) is the product of
// the leaf's weights by position (zero where a node was culled) with one fixed
// 64 x 2(p + 1) real matrix Z (columns Re and Im of -zeta^k / k; 1 and 0 for
// k = 0): a dense contraction, run on the matrix cores as FP64 16x16x4
// products, 16 leaves per wave (rows), 4 positions per product, 16 columns per
// tile.  Leaves of other sizes in the wave's 16 are done by the lane-group path
// above, 8 lanes per leaf.
// 1 / k, k = 1..kMaxP, each the correctly rounded quotient.
struct InvIntTable {
  double v[kMaxP + 1];
};
constexpr InvIntTable make_inv_int() {
  InvIntTable t{};
  for (int k = 1; k <= kMaxP; ++k) t.v[k] = 1.0 / k;
  return t;
}
__constant__ InvIntTable c_inv_int = make_inv_int();

template <int PM>
__global__ __launch_bounds__(256) void k_p2m_lattice(TreeView t, const int* __restrict__ sleaves, int n,
                                                     const uint32_t* __restrict__ ij, const double* __restrict__ w64,
                                                     int p, double2* __restrict__ mp) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  constexpr int kCols = 2 * (PM + 1);
  constexpr int kTiles = (kCols + 15) / 16;
  constexpr int kZW = kTiles * 16;  // row length of Z
  constexpr int kWP = 68;           // padded row of a wave's weight block (doubles)
  __shared__ double zt[64 * kZW];
  __shared__ double wb[4 * 16 * kWP];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  // the wave's 16 leaves: lane i < 16 holds leaf i's cell, source range and corner
  const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 16;
  int c = 0, sb = 0, cnt = 0, cx = 0, cy = 0;
  bool valid = false, lat = false;
  if (lane < 16 && base + lane < n) {
    c = sleaves[base + lane];
    const int sh = t.D - t.lvl[c];
    sb = t.sb[c];
    cnt = t.se[c] - sb;
    cx = t.ix[c] << sh;
    cy = t.iy[c] << sh;
    valid = true;
    lat = sh == 3 && cnt <= 64;
  }
  const uint64_t latm = __ballot(lat);
  const uint64_t genm = __ballot(valid && !lat);
  uint32_t v[16];
  double w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int sbi = __builtin_amdgcn_readlane(sb, i), cnti = __builtin_amdgcn_readlane(cnt, i);
    const bool ok = ((latm >> i) & 1) && lane < cnti;
    v[i] = ok ? ij[sbi + lane] : 0u;
    w[i] = ok ? w64[sbi + lane] : 0.0;
  }
  // while the loads are in flight: Z (first wave) and the cleared weight blocks
  if (threadIdx.x < 64) {
    const int pos = threadIdx.x;
    const cplx z = {((double)(pos & 7) + 0.5) * 0.125 - 0.5, ((double)(pos >> 3) + 0.5) * 0.125 - 0.5};
    double* row = zt + pos * kZW;
    row[0] = 1.0;
    row[1] = 0.0;
    cplx zk = z;
#pragma unroll
    for (int k = 1; k <= PM; ++k) {
      row[2 * k] = -zk.x * c_inv_int.v[k];
      row[2 * k + 1] = -zk.y * c_inv_int.v[k];
      zk = cmul(zk, z);
    }
#pragma unroll
    for (int col = kCols; col < kZW; ++col) row[col] = 0.0;
  }
  double* W = wb + wave * 16 * kWP;
  for (int q = lane; q < 16 * kWP; q += kWave) W[q] = 0.0;
  __syncthreads();  // Z and the cleared weight blocks
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int cxi = __builtin_amdgcn_readlane(cx, i), cyi = __builtin_amdgcn_readlane(cy, i);
    const int cnti = __builtin_amdgcn_readlane(cnt, i);
    const int dx = (int)(v[i] & 0xFFFFu) - cxi, dy = (int)(v[i] >> 16) - cyi;
    if (((latm >> i) & 1) && lane < cnti && (unsigned)dx < 8u && (unsigned)dy < 8u) W[i * kWP + dx + 8 * dy] = w[i];
  }
  __syncthreads();
  // D (16 leaves x 16 columns per tile) += A (16 leaves x 4 positions) B (4 positions x 16 columns)
  const int r16 = lane % 16, kq = lane / 16;
  v4d acc[kTiles];
#pragma unroll
  for (int tl = 0; tl < kTiles; ++tl) acc[tl] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const double a = W[r16 * kWP + 4 * s + kq];
#pragma unroll
    for (int tl = 0; tl < kTiles; ++tl) {
      const double b = zt[(4 * s + kq) * kZW + tl * 16 + r16];
      acc[tl] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[tl], 0, 0, 0);
    }
  }
  // lane (r16, kq), element e: leaf 4 e + kq, column 16 tl + r16
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = 4 * e + kq;
    const int ci = __shfl(c, i);
    if (!((latm >> i) & 1)) continue;
    double* out = reinterpret_cast<double*>(mp + (int64_t)ci * (p + 1));
#pragma unroll
    for (int tl = 0; tl < kTiles; ++tl) {
      const int col = tl * 16 + r16;
      if (col < 2 * (p + 1)) out[col] = acc[tl][e];
    }
  }
  // the wave's other leaves, eight at a time, 8 lanes each
  uint64_t gen = genm;
  while (gen) {
    const int grp = lane / 8;
    uint64_t m = gen;
    for (int q = 0; q < grp && m; ++q) m &= m - 1;
    const bool st = m != 0;
    const int i = st ? __builtin_ctzll(m) : __builtin_ctzll(gen);
    const int ci = __shfl(c, i);
    p2m_leaf<PM, 8>(t, ci, lane % 8, st, ij, nullptr, nullptr, 0.0, 0.0, 1.0, w64, p, mp);
    for (int q = 0; q < 8 && gen; ++q) gen &= gen - 1;
  }
}

// M2M as fixed matrices.  With coefficients scaled by the cell side, the shift
// of a child's expansion to its parent's centre depends only on the child's
// quadrant q, through d_q = (+-1/4, +-1/4) (the child centre's offset in parent
// sides).  From eq. expandedShift with the corrected S term:
//   a'_l(parent) = sum_q sum_{k=0..l} T_q[l][k] a'_k(child q),
//   T_q[0][0] = 1,  T_q[l][0] = -d_q^l / l,  T_q[l][k] = C(l-1, k-1) 2^-k d_q^(l-k).
// The table is built at compile time; every entry but the 1/l ones is exact.
struct M2MTable {
  double v[4][kMaxP + 1][kMaxP + 1][2];
};
constexpr M2MTable make_m2m_table() {
  M2MTable t{};
  for (int q = 0; q < 4; ++q) {
    const double dx = (q & 1) ? 0.25 : -0.25, dy = (q & 2) ? 0.25 : -0.25;
    // powers d^n, n = 0..kMaxP
    double pw[kMaxP + 1][2] = {};
    pw[0][0] = 1.0;
    for (int n = 1; n <= kMaxP; ++n) {
      pw[n][0] = pw[n - 1][0] * dx - pw[n - 1][1] * dy;
      pw[n][1] = pw[n - 1][0] * dy + pw[n - 1][1] * dx;
    }
    t.v[q][0][0][0] = 1.0;
    for (int l = 1; l <= kMaxP; ++l) {
      t.v[q][l][0][0] = -pw[l][0] / l;
      t.v[q][l][0][1] = -pw[l][1] / l;
      double c = 1.0;  // C(l-1, k-1), k = 1
      double two = 0.5;  // 2^-k
      for (int k = 1; k <= l; ++k) {
        t.v[q][l][k][0] = c * two * pw[l - k][0];
        t.v[q][l][k][1] = c * two * pw[l - k][1];
        c = c * (l - k) / k;
        two *= 0.5;
      }
    }
  }
  return t;
}
__constant__ M2MTable c_m2m = make_m2m_table();

// One child's share of the M2M output coefficient a'_l of its parent: the sum
// over k <= l of row[k] a[k], with a the child's coefficients and row the
// table tm[quadrant][l] (both in LDS).
__device__ inline cplx m2m_child(int l, const double2* __restrict__ a, const double2* __restrict__ row) {
  double bx0 = 0.0, by0 = 0.0, bx1 = 0.0, by1 = 0.0;
  // two accumulators shorten the dependent chain
  int k = 0;
  for (; k + 1 <= l; k += 2) {
    const double2 t0 = row[k], a0 = a[k], t1 = row[k + 1], a1 = a[k + 1];
    bx0 += t0.x * a0.x - t0.y * a0.y;
    by0 += t0.x * a0.y + t0.y * a0.x;
    bx1 += t1.x * a1.x - t1.y * a1.y;
    by1 += t1.x * a1.y + t1.y * a1.x;
  }
  if (k == l) {
    const double2 t0 = row[k], a0 = a[k];
    bx0 += t0.x * a0.x - t0.y * a0.y;
    by0 += t0.x * a0.y + t0.y * a0.x;
  }
  return {bx0 + bx1, by0 + by1};
}

// M2M for up to three levels per launch (eq. expandedShift applied
// recursively from the finest level up).  One workgroup per cell R at level L
// computes, bottom up, the expansions of R's descendants at levels L+2, L+1
// and of R itself from the final expansions one level below the subtree.
// The subtree's structure is read level by level with one thread per cell;
// then every expansion the subtree needs from global memory (the level below
// it and the leaves inside it) is staged into LDS in one parallel sweep, so
// the arithmetic never waits on a global load.  Leaves keep their P2M
// expansions.
// 512 threads: a workgroup of 8 waves finds room on a compute unit as soon as
// two near-field workgroups (4 waves each) leave it, when the near field runs
// beside the upward pass on another stream; 1024-thread workgroups waited far
// longer for a whole free half of a compute unit.  (Launches of a few
// workgroups, but more than one, use 256 threads; see m2m_levels.)
constexpr int kM2MThreads = 512;
constexpr int kM2MLevels = 3;
constexpr int kM2MSlots = 85;  // 1 + 4 + 16 + 64
__host__ __device__ constexpr int m2m_first(int d) { return ((1 << (2 * d)) - 1) / 3; }

// LDS: five int arrays of kM2MSlots (padded to a 16-byte boundary), the
// expansions and the four shift tables: 30 KB at p = 12 (four workgroups of
// 512 threads fill a compute unit), 58 KB at p = 20.
constexpr int kM2MIntWords = 5 * kM2MSlots + 3;
size_t m2m_lds_bytes(int p) {
  return kM2MIntWords * sizeof(int) + ((size_t)kM2MSlots * (p + 1) + 4 * (size_t)(p + 1) * (p + 1)) * sizeof(double2);
}

// dense_flag/dense_off: the existence flags and cell numbers of the dense prefix
// table the tree build used for its top levels (index ((4^L - 1) / 3) + prefix at
// level L).  When the launch's levels all lie in that table (dense != 0), every
// slot finds its cell there directly (slot offsets within a depth are Morton
// offsets within R's subtree), instead of walking down the child links one
// level at a time.
__global__ __launch_bounds__(kM2MThreads) void k_m2m(TreeView t, int c0, int c1, int L, int levels, int p,
                                                      double2* __restrict__ mp, const int* __restrict__ dense_flag,
                                                      const int* __restrict__ dense_off, int dense) {
  // slots: [0] = R, [1..4] its children, [5..20] grandchildren (4 per parent
  // slot), ... ; depth d holds slots [m2m_first(d), m2m_first(d + 1)).
  extern __shared__ int smem[];
  int* cell = smem;
  int* kid0 = cell + kM2MSlots;
  int* nkid = kid0 + kM2MSlots;
  int* hsrc = nkid + kM2MSlots;
  int* quad = hsrc + kM2MSlots;
  double2* e = (double2*)(smem + kM2MIntWords);
  const int R = c0 + blockIdx.x;
  if (R >= c1) return;
  const int P1 = p + 1;
  const int tid = threadIdx.x;
  double2* tm = e + (size_t)kM2MSlots * P1;
  for (int w = tid; w < 4 * P1 * P1; w += blockDim.x) {
    const int q = w / (P1 * P1), l = (w / P1) % P1, k = w % P1;
    tm[w] = make_double2(c_m2m.v[q][l][k][0], c_m2m.v[q][l][k][1]);
  }
  if (dense) {
    const int64_t PR = (int64_t)morton((uint32_t)t.ix[R], (uint32_t)t.iy[R]);
    for (int i = tid; i < m2m_first(levels + 1); i += blockDim.x) {
      int d = 0;
      while (m2m_first(d + 1) <= i) ++d;
      const int j = i - m2m_first(d);
      int c = R;
      if (d > 0) {
        const int64_t idx = ((((int64_t)1 << (2 * (L + d))) - 1) / 3) + (PR << (2 * d)) + j;
        c = dense_flag[idx] ? dense_off[idx] : -1;
      }
      cell[i] = c;
      kid0[i] = c >= 0 ? t.child[c] : -1;
      nkid[i] = 4;  // children sit at their quadrant's slot; missing ones have no sources
      hsrc[i] = c >= 0 ? (t.se[c] > t.sb[c]) : 0;
      quad[i] = d > 0 ? (j & 3) : 0;
    }
    __syncthreads();
  } else {
    for (int d = 0; d <= levels; ++d) {
      const int lo = m2m_first(d), hi = m2m_first(d + 1);
      for (int i = lo + tid; i < hi; i += blockDim.x) {
        int c = -1;
        if (d == 0) {
          c = R;
        } else {
          const int par = m2m_first(d - 1) + (i - lo) / 4;
          const int q = (i - lo) % 4;
          if (cell[par] >= 0 && hsrc[par] && q < nkid[par] && kid0[par] >= 0) c = kid0[par] + q;
        }
        cell[i] = c;
        kid0[i] = c >= 0 ? t.child[c] : -1;
        nkid[i] = c >= 0 ? t.nchild[c] : 0;
        hsrc[i] = c >= 0 ? (t.se[c] > t.sb[c]) : 0;
        quad[i] = c >= 0 ? ((t.ix[c] & 1) | ((t.iy[c] & 1) << 1)) : 0;
      }
      __syncthreads();
    }
  }
  // stage: slots of depth `levels`, and leaves above it, hold final expansions
  const int nstage = m2m_first(levels + 1);
  const int deepest = m2m_first(levels);
  for (int w = tid; w < nstage * P1; w += blockDim.x) {
    const int i = w / P1, l = w % P1;
    const int c = cell[i];
    if (c < 0 || !hsrc[i]) continue;
    if (i >= deepest || kid0[i] < 0) e[i * P1 + l] = mp[(int64_t)c * P1 + l];
  }
  __syncthreads();
  // Each (parent, coefficient) item takes four adjacent lanes, one per child
  // slot; the four partial sums meet through two cross-lane adds, in the same
  // order on every lane.  The trip count is the same for every lane, so whole
  // wavefronts reach the exchanges.
  for (int d = levels - 1; d >= 0; --d) {
    const int lo = m2m_first(d), hi = m2m_first(d + 1);
    const int items = 4 * (hi - lo) * P1;
    for (int base = 0; base < items; base += blockDim.x) {
      const int w = base + tid, q = w & 3, item = w >> 2;
      const int i = lo + item / P1, l = item % P1;
      const int c = w < items ? cell[i] : -1;
      const bool live = c >= 0 && hsrc[i] && kid0[i] >= 0;
      const int slot = m2m_first(d + 1) + 4 * (i - lo) + q;
      cplx v = {0.0, 0.0};
      if (live && q < nkid[i] && hsrc[slot]) v = m2m_child(l, e + (int64_t)slot * P1, tm + ((int64_t)quad[slot] * P1 + l) * P1);
      v.x += __shfl_xor(v.x, 1);
      v.y += __shfl_xor(v.y, 1);
      v.x += __shfl_xor(v.x, 2);
      v.y += __shfl_xor(v.y, 2);
      if (live && q == 0) {
        e[i * P1 + l] = make_double2(v.x, v.y);
        mp[(int64_t)c * P1 + l] = make_double2(v.x, v.y);
      }
    }
    __syncthreads();
  }
}

// G lanes per target cell: lane j of the group takes list entries j, j+G, ...
// and accumulates their local contributions in registers.  The group then
// sums them through LDS: every lane stores its 2 (p + 1) partial values, and
// lane q of the group adds value q over the G lanes in lane order (a fixed
// order, so the result is reproducible).
constexpr int kM2LBlock = 128;
template <int PM, int G>
__global__ __launch_bounds__(kM2LBlock) void k_m2l(TreeView t, const int* __restrict__ tcells, int n,
                                             const int* __restrict__ off, const int* __restrict__ cnt,
                                             const int* __restrict__ src, int p, double lnh,
                                             const double2* __restrict__ mp, double2* __restrict__ loc,
                                             int* __restrict__ flags) {
  static_assert(2 * (PM + 1) <= 2 * G, "two partial values per coefficient and at most two per lane");
  __builtin_assume(p >= 1);  // the orders the library accepts
  __shared__ double red[kM2LBlock][2 * (PM + 1)];
  const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int gi = (int)(gtid / G);
  const int sub = (int)(gtid % G);
  const bool live = gi < n;  // whole groups agree; every lane reaches the barrier
  const int A = live ? tcells[gi] : 0;
  const int D = t.D;
  const int lA = t.lvl[A];
  const double sA = cell_side(D, lA);
  const double cax = (t.ix[A] + 0.5) * sA, cay = (t.iy[A] + 0.5) * sA;
  cplx L[PM + 1];
#pragma unroll
  for (int k = 0; k <= PM; ++k) L[k] = {0.0, 0.0};
  const int e0 = live ? off[A] : 0, ne = live ? cnt[A] : 0;
  for (int e = sub; e < ne; e += G) {
    const int B = src[e0 + e];
    if ((unsigned)B >= (unsigned)t.ncells) {
      atomicOr(flags, kFlagBadIndex);
      continue;
    }
    const int lB = t.lvl[B];
    const double sB = cell_side(D, lB);
    const cplx z0 = {(t.ix[B] + 0.5) * sB - cax, (t.iy[B] + 0.5) * sB - cay};
    const double r2 = z0.x * z0.x + z0.y * z0.y;
    const double ir2 = 1.0 / r2;
    const cplx inv = {z0.x * ir2, -z0.y * ir2};  // 1 / z0
    const cplx tt = cscale(inv, sA);
    const cplx mr = cscale(inv, -sB);           // -s_B / z0
    const double2* a = mp + (int64_t)B * (p + 1);
    // all p + 1 coefficients are requested before the first is used: the
    // index is clamped to p (inside the cell's own block; p >= 1) and the
    // terms past p are zeroed, so no load waits behind a branch
    double2 av[PM + 1];
#pragma unroll
    for (int k = 0; k <= PM; ++k) av[k] = a[k <= p ? k : p];
    const double a0 = av[0].x;
    cplx bk[PM + 1];
    cplx pw = mr;
    cplx sum0 = {a0 * (0.5 * log(r2) + lnh), 0.0};
#pragma unroll
    for (int k = 1; k <= PM; ++k) {
      bk[k] = k <= p ? cmul({av[k].x, av[k].y}, pw) : cplx{0.0, 0.0};
      pw = cmul(pw, mr);
      sum0 = cadd(sum0, bk[k]);
    }
    L[0] = cadd(L[0], sum0);
    cplx tl = tt;
#pragma unroll
    for (int l = 1; l <= PM; ++l) {
      cplx s = {-a0 * (1.0 / l), 0.0};  // 1 / l is a compile-time constant of the unrolled loop
#pragma unroll
      for (int k = 1; k <= PM; ++k) s = cadd(s, cscale(bk[k], binom(l + k - 1, k - 1)));
      L[l] = cadd(L[l], cmul(tl, s));
      tl = cmul(tl, tt);
    }
  }
#pragma unroll
  for (int k = 0; k <= PM; ++k) {
    red[threadIdx.x][2 * k] = L[k].x;
    red[threadIdx.x][2 * k + 1] = L[k].y;
  }
  __syncthreads();
  if (!live) return;
  const int g0 = (int)(threadIdx.x - sub);  // the group's first lane in the block
  double* out = (double*)(loc + (int64_t)A * (p + 1));
  for (int q = sub; q < 2 * (p + 1); q += G) {
    double v = 0.0;
    for (int j = 0; j < G; ++j) v += red[g0 + j][q];
    out[q] = v;
  }
}

// Downward pass in one launch.  L2L is exact for a degree-p polynomial, so the
// recursion "local(child) = own M2L + L2L(local(parent))" equals the sum, over
// the cell and each of its ancestors X, of X's own M2L local shifted from X's
// centre to the cell:  L'_m = sum_X 2^{-m (l_c - l_X)} sum_{k>=m} C(k, m) d_X^{k-m} L'_k(X),
// d_X = (z_c - z_X) / s_X.  Sixteen lanes per cell with targets (four cells per
// wave): lane j takes the ancestor at level j (and j + 16), loads its p + 1 own
// coefficients once, shifts them to the cell in place by synthetic division (a
// Taylor shift by d_X: p (p + 1) / 2 complex multiply-adds) and scales
// coefficient m by 2^{-m (l_c - l_X)}; the cell itself (j = l_c) contributes its
// own local unshifted.  The lanes' terms are then added through LDS, lane m of
// the cell summing coefficient m over the levels in ascending order (a fixed
// order, so the result is reproducible).  An ancestor at a level of the dense
// prefix table is found there directly from the cell's coordinates; deeper ones
// by following parent links.
constexpr int kDownLanes = 16;
template <int PM>
__global__ __launch_bounds__(kWave) void k_downward(TreeView t, const int* __restrict__ tcells, int n, int p,
                                                    const double2* __restrict__ own, double2* __restrict__ loc,
                                                    const int* __restrict__ dense_off, int dense_levels, int top) {
  __shared__ double2 red[kWave][PM + 1];
  const int lane = threadIdx.x;
  const int sub = lane % kDownLanes;
  const int grp = lane / kDownLanes;
  const int i = blockIdx.x * (kWave / kDownLanes) + grp;
  const bool live = i < n;
  const int P1 = p + 1;
  const int D = t.D;
  const int c = live ? tcells[i] : 0;
  const int lc = live ? t.lvl[c] : -1;
  const int icx = live ? t.ix[c] : 0, icy = live ? t.iy[c] : 0;
  const double sc = cell_side(D, live ? lc : 0);
  const double cx = (icx + 0.5) * sc, cy = (icy + 0.5) * sc;
  cplx acc[PM + 1];
#pragma unroll
  for (int k = 0; k <= PM; ++k) acc[k] = {0.0, 0.0};
  // ancestors from level top (a forest's request roots; 0 otherwise): the
  // levels above it have no interactions, and starting there gives each
  // request's cells the lane assignment (and sums) of its lone solve
  for (int a = top + sub; a <= lc; a += kDownLanes) {
    if (a == lc) {
      // every coefficient requested before the first is added (index clamped
      // to p, terms past p dropped), so no load waits behind a branch
      double2 v[PM + 1];
#pragma unroll
      for (int k = 0; k <= PM; ++k) v[k] = own[(int64_t)c * P1 + (k <= p ? k : p)];
#pragma unroll
      for (int k = 0; k <= PM; ++k)
        if (k <= p) acc[k] = cadd(acc[k], {v[k].x, v[k].y});
      continue;
    }
    const int sh = lc - a;
    const int ax = icx >> sh, ay = icy >> sh;  // the ancestor's coordinates at level a
    int X;
    if (a <= dense_levels) {
      X = dense_off[((((int64_t)1 << (2 * a)) - 1) / 3) + (int64_t)morton((uint32_t)ax, (uint32_t)ay)];
    } else {
      X = c;
      for (int l = lc; l > a; --l) X = t.parent[X];
    }
    const double sX = cell_side(D, a), iX = inv_cell_side(D, a);
    const cplx d = {(cx - (ax + 0.5) * sX) * iX, (cy - (ay + 0.5) * sX) * iX};
    cplx L[PM + 1];
#pragma unroll
    for (int k = 0; k <= PM; ++k) {
      if (k <= p) {
        const double2 v = own[(int64_t)X * P1 + k];
        L[k] = {v.x, v.y};
      } else {
        L[k] = {0.0, 0.0};
      }
    }
    // Taylor shift by d: afterwards L[m] = sum_{k>=m} C(k, m) d^{k-m} L[k]
#pragma unroll
    for (int r = 0; r < PM; ++r)
#pragma unroll
      for (int k = PM - 1; k >= r; --k)
        if (k < p) L[k] = cadd(L[k], cmul(d, L[k + 1]));
    const double f = ldexp(1.0, -sh);  // s_c / s_X
    double g = 1.0;
#pragma unroll
    for (int k = 0; k <= PM; ++k) {
      acc[k] = cadd(acc[k], cscale(L[k], g));
      g *= f;  // exact: a power of two
    }
  }
#pragma unroll
  for (int k = 0; k <= PM; ++k) red[lane][k] = make_double2(acc[k].x, acc[k].y);
  __syncthreads();
  if (!live) return;
  for (int m = sub; m <= p; m += kDownLanes) {
    cplx s = {0.0, 0.0};
    for (int q = 0; q < kDownLanes; ++q) {
      const double2 v = red[grp * kDownLanes + q][m];
      s = cadd(s, {v.x, v.y});
    }
    loc[(int64_t)c * P1 + m] = make_double2(s.x, s.y);
  }
}

__global__ void k_l2p(TreeView t, int64_t m, const int* __restrict__ tleaf, int p, const double2* __restrict__ loc,
                      const double2* __restrict__ rel64, int fp32, double* __restrict__ far) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int c = tleaf[k];
  far[k] = l2p_eval(loc + (int64_t)c * (p + 1), p, rel64[k], t.D, t.lvl[c], fp32 != 0);
}

// M2P of the paper's tree-code (eq. pressTruncated evaluated at the targets):
// one wave per target leaf A, lane j on target j of each 64-target chunk, and
// for every source cell B of A's list
//   far += a_0 (ln|w| + ln s_B) + Re sum_{k=1..p} a'_k w^-k,   w = (t - z_B) / s_B,
// by Horner in u = 1/w.  The list is consumed 64 cells at a time: lane i
// loads cell i's geometry (corner difference to A in units of h, 1/s_B, the
// ln s_B term) and its coefficients into the wave's LDS slice, so the
// evaluation loop reads only LDS broadcasts.  The slice holds PM + 1
// coefficients per cell, zero above p (Horner over zeros leaves the sum
// unchanged), so the loop is fully unrolled and its reads are issued ahead of
// the arithmetic.  T = float for mixed precision (coefficients rounded when
// staged, each cell's term added to an FP64 sum), double otherwise.
constexpr double kLn2d = 0.69314718055994530942;
constexpr int kM2PWaves = 4;

template <class T>
struct Cx2 {
  T x, y;
};

template <class T, int PM>
__global__ __launch_bounds__(kM2PWaves* kWave) void k_m2p(TreeView t, const int* __restrict__ tleaves, int n,
                                                          const int* __restrict__ off, const int* __restrict__ cnt,
                                                          const int* __restrict__ src, int p, double lnh,
                                                          const double2* __restrict__ mp,
                                                          const double2* __restrict__ rel64, int nparts,
                                                          int64_t m, double* __restrict__ far,
                                                          int* __restrict__ flags) {
  extern __shared__ double m2p_lds[];
  const int w = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int P1 = p + 1;
  constexpr int kSlot = PM + 3;  // per cell: 2 geometry slots and PM + 1 coefficients
  Cx2<T>* coef = (Cx2<T>*)m2p_lds + (size_t)w * kWave * kSlot;
  const int wid = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * kM2PWaves + w));
  if (wid >= n * nparts) return;
  // wave (leaf, part): the part's share of the leaf's list, its partial far
  // field stored at far[part * m + k] (the finalize step adds the parts)
  const int part = wid % nparts;
  const int A = tleaves[wid / nparts];
  const int shA = t.D - t.lvl[A];
  const int64_t ax2 = (int64_t)(2 * t.ix[A]) << shA, ay2 = (int64_t)(2 * t.iy[A]) << shA;
  const int nall = cnt[A];
  const int e0 = off[A] + (int)((int64_t)nall * part / nparts);
  const int ne = (int)((int64_t)nall * (part + 1) / nparts) - (int)((int64_t)nall * part / nparts);
  double* far_part = far + (int64_t)part * m;
  const int tb = t.tb[A], te = t.te[A];
  bool bad = false;
  for (int chunk = tb; chunk < te; chunk += kWave) {
    const int k = chunk + lane;
    const bool active = k < te;
    const double2 r64 = active ? rel64[k] : make_double2(0.0, 0.0);
    const T rx = (T)r64.x, ry = (T)r64.y;
    double acc_far = 0.0;
    for (int base = 0; base < ne; base += kWave) {
      const int nb = min(kWave, ne - base);
      // stage: lane i takes list entry base + i
      if (lane < nb) {
        int B = src[e0 + base + lane];
        Cx2<T>* cb = coef + (size_t)lane * kSlot;
        for (int q = P1; q <= PM; ++q) cb[2 + q] = {(T)0, (T)0};
        if ((unsigned)B >= (unsigned)t.ncells) {
          bad = true;
          cb[0] = {(T)0, (T)0};
          cb[1] = {(T)1, (T)0};
          for (int q = 0; q < P1; ++q) cb[2 + q] = {(T)0, (T)0};
        } else {
          const int shB = t.D - t.lvl[B];
          const double dx = 0.5 * (double)(ax2 - ((int64_t)(2 * t.ix[B] + 1) << shB));
          const double dy = 0.5 * (double)(ay2 - ((int64_t)(2 * t.iy[B] + 1) << shB));
          cb[0] = {(T)dx, (T)dy};
          cb[1] = {(T)ldexp(1.0, -shB), (T)((double)shB * kLn2d + lnh)};
          const double2* a = mp + (int64_t)B * P1;
          for (int q = 0; q < P1; ++q) {
            const double2 v = a[q];
            cb[2 + q] = {(T)v.x, (T)v.y};
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int j = 0; j < nb; ++j) {
        const Cx2<T>* cb = coef + (size_t)j * kSlot;
        const Cx2<T> g0 = cb[0], g1 = cb[1];
        const T wx = (rx + g0.x) * g1.x, wy = (ry + g0.y) * g1.x;
        const T r2 = wx * wx + wy * wy;
        T ir2;
        if constexpr (sizeof(T) == 4)
          ir2 = __builtin_amdgcn_rcpf(r2);  // v_rcp_f32 (1 ulp): the mixed-precision path rounds to FP32 anyway
        else
          ir2 = (T)1 / r2;
        const T ux = wx * ir2, uy = -wy * ir2;
        T hx = (T)0, hy = (T)0;
#pragma unroll
        for (int q = PM; q >= 1; --q) {
          const Cx2<T> c = cb[2 + q];
          const T nx = hx * ux - hy * uy + c.x;
          const T ny = hx * uy + hy * ux + c.y;
          hx = nx;
          hy = ny;
        }
        const T re = hx * ux - hy * uy;
        T lg;
        if constexpr (sizeof(T) == 4)
          lg = (T)(0.5 * kLn2d) * __builtin_amdgcn_logf(r2) + g1.y;
        else
          lg = (T)0.5 * log(r2) + g1.y;
        acc_far += (double)(re + cb[2].x * lg);
      }
      // the slice is rewritten by the next batch only after every lane is done with it
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if (active) far_part[k] = acc_far;
  }
  if (bad && lane == 0) atomicOr(flags, kFlagBadIndex);
}

#define PP_DISPATCH(p, KERNEL, GRID, BLOCK, STREAM, ...)                      \
  do {                                                                        \
    if ((p) <= 4)                                                             \
      KERNEL<4><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);                     \
    else if ((p) <= 8)                                                        \
      KERNEL<8><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);                     \
    else if ((p) <= 12)                                                       \
      KERNEL<12><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);                    \
    else if ((p) <= 16)                                                       \
      KERNEL<16><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);                    \
    else                                                                      \
      KERNEL<20><<<GRID, BLOCK, 0, STREAM>>>(__VA_ARGS__);                    \
  } while (0)

}  // namespace

template <int LANES>
void p2m_lanes(TreeView t, const int* sleaves, int n, const uint32_t* ij, const double* xs, const double* ys,
               double x0, double y0, double u, const double* w64, int p, double2* mp, hipStream_t s) {
  const unsigned g = (unsigned)(((int64_t)n * LANES + 255) / 256);
  if (p <= 4)
    k_p2m<4, LANES><<<g, 256, 0, s>>>(t, sleaves, n, ij, xs, ys, x0, y0, u, w64, p, mp);
  else if (p <= 8)
    k_p2m<8, LANES><<<g, 256, 0, s>>>(t, sleaves, n, ij, xs, ys, x0, y0, u, w64, p, mp);
  else if (p <= 12)
    k_p2m<12, LANES><<<g, 256, 0, s>>>(t, sleaves, n, ij, xs, ys, x0, y0, u, w64, p, mp);
  else if (p <= 16)
    k_p2m<16, LANES><<<g, 256, 0, s>>>(t, sleaves, n, ij, xs, ys, x0, y0, u, w64, p, mp);
  else
    k_p2m<kMaxP, LANES><<<g, 256, 0, s>>>(t, sleaves, n, ij, xs, ys, x0, y0, u, w64, p, mp);
}

void p2m(TreeView t, const int* sleaves, int n, const uint32_t* ij, const double* xs, const double* ys, double x0,
         double y0, double u, const double* w64, int p, double2* mp, int64_t lattice_min, hipStream_t s) {
  if (n <= 0) return;
  // grid sources with at least lattice_min leaves: leaves 8 nodes wide on
  // the matrix cores
  if (ij && lattice_min > 0 && n >= lattice_min) {
    const unsigned g = (unsigned)(((int64_t)n + 63) / 64);
    if (p <= 4)
      k_p2m_lattice<4><<<g, 256, 0, s>>>(t, sleaves, n, ij, w64, p, mp);
    else if (p <= 8)
      k_p2m_lattice<8><<<g, 256, 0, s>>>(t, sleaves, n, ij, w64, p, mp);
    else if (p <= 12)
      k_p2m_lattice<12><<<g, 256, 0, s>>>(t, sleaves, n, ij, w64, p, mp);
    else if (p <= 16)
      k_p2m_lattice<16><<<g, 256, 0, s>>>(t, sleaves, n, ij, w64, p, mp);
    else
      k_p2m_lattice<kMaxP><<<g, 256, 0, s>>>(t, sleaves, n, ij, w64, p, mp);
    return;
  }
  // lanes per leaf: PP_P2M_LANES = 4, 8 (default) or 16
  static const int lanes = [] {
    const char* e = std::getenv("PP_P2M_LANES");
    const int v = e ? std::atoi(e) : 8;
    return (v == 4 || v == 16) ? v : 8;
  }();
  if (lanes == 4)
    p2m_lanes<4>(t, sleaves, n, ij, xs, ys, x0, y0, u, w64, p, mp, s);
  else if (lanes == 16)
    p2m_lanes<16>(t, sleaves, n, ij, xs, ys, x0, y0, u, w64, p, mp, s);
  else
    p2m_lanes<8>(t, sleaves, n, ij, xs, ys, x0, y0, u, w64, p, mp, s);
}

int m2m_max_levels() { return kM2MLevels; }

void m2m_levels(TreeView t, int c0, int c1, int L, int levels, int p, double2* mp, const int* dense_flag,
                const int* dense_off, int dense_levels, hipStream_t s) {
  if (c1 <= c0 || levels < 1) return;
  levels = std::min(levels, kM2MLevels);
  const int dense = (dense_flag && dense_off && L + levels <= dense_levels) ? 1 : 0;
  static std::once_flag lds_opt_in;
  std::call_once(lds_opt_in, [] {
    (void)hipFuncSetAttribute((const void*)k_m2m, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)m2m_lds_bytes(kMaxP));
  });
  // A launch of few workgroups (the top levels) uses 256-thread workgroups:
  // beside the near field they find room on a compute unit sooner.  Alone
  // they are slower (M2M 50.6 -> 56.4 us at 4096^2), beside the near field
  // faster (cold solves +1.5 %, resident +1.4 %; 128 threads: -5 %).  A
  // launch of one workgroup (the root's subtree) keeps 512 threads: its
  // chain of levels is the whole launch (+0.8 % timed, +1.6 % untimed).
  const int nb = c1 - c0;
  const int th = nb > 1 && nb <= 1024 ? 256 : kM2MThreads;
  k_m2m<<<c1 - c0, th, m2m_lds_bytes(p), s>>>(t, c0, c1, L, levels, p, mp, dense_flag, dense_off, dense);
}

void m2l(TreeView t, const int* tcells, int n, const int* m2l_off, const int* m2l_cnt, const int* m2l_src, int p,
         double h, const double2* mp, double2* loc, int* flags, hipStream_t s) {
  if (n <= 0) return;
  constexpr int G = 32;
  const unsigned g = (unsigned)(((int64_t)n * G + kM2LBlock - 1) / kM2LBlock);
  const double lnh = log(h);
  if (p <= 4)
    k_m2l<4, G><<<g, kM2LBlock, 0, s>>>(t, tcells, n, m2l_off, m2l_cnt, m2l_src, p, lnh, mp, loc, flags);
  else if (p <= 8)
    k_m2l<8, G><<<g, kM2LBlock, 0, s>>>(t, tcells, n, m2l_off, m2l_cnt, m2l_src, p, lnh, mp, loc, flags);
  else if (p <= 12)
    k_m2l<12, G><<<g, kM2LBlock, 0, s>>>(t, tcells, n, m2l_off, m2l_cnt, m2l_src, p, lnh, mp, loc, flags);
  else if (p <= 16)
    k_m2l<16, G><<<g, kM2LBlock, 0, s>>>(t, tcells, n, m2l_off, m2l_cnt, m2l_src, p, lnh, mp, loc, flags);
  else
    k_m2l<20, G><<<g, kM2LBlock, 0, s>>>(t, tcells, n, m2l_off, m2l_cnt, m2l_src, p, lnh, mp, loc, flags);
}

void downward(TreeView t, const int* tcells, int n, int p, const double2* own, double2* loc, const int* dense_off,
              int dense_levels, int top, hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)((n + kWave / kDownLanes - 1) / (kWave / kDownLanes));
  PP_DISPATCH(p, k_downward, g, kWave, s, t, tcells, n, p, own, loc, dense_off, dense_levels, top);
}

void l2p(TreeView t, int64_t m, const int* tleaf, int p, const double2* loc, const double2* rel64, int fp32,
         double* far, hipStream_t s) {
  if (m <= 0) return;
  k_l2p<<<(unsigned)((m + 255) / 256), 256, 0, s>>>(t, m, tleaf, p, loc, rel64, fp32, far);
}

template <class T, int PM>
void m2p_launch(unsigned g, TreeView t, const int* tleaves, int n, const int* off, const int* cnt, const int* src,
                int p, double h, const double2* mp, const double2* rel64, int nparts, int64_t m, double* far,
                int* flags, hipStream_t s) {
  // up to 94 KB of LDS at PM = 20 in FP64 (gfx950 allows 160 KB per workgroup)
  const size_t bytes = (size_t)kM2PWaves * kWave * (PM + 3) * sizeof(Cx2<T>);
  static std::once_flag lds_opt_in;
  std::call_once(lds_opt_in, [bytes] {
    (void)hipFuncSetAttribute((const void*)k_m2p<T, PM>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  });
  k_m2p<T, PM><<<g, kM2PWaves * kWave, bytes, s>>>(t, tleaves, n, off, cnt, src, p, log(h), mp, rel64, nparts, m,
                                                   far, flags);
}

template <class T>
void m2p_dispatch(unsigned g, TreeView t, const int* tleaves, int n, const int* off, const int* cnt, const int* src,
                  int p, double h, const double2* mp, const double2* rel64, int nparts, int64_t m, double* far,
                  int* flags, hipStream_t s) {
  if (p <= 4)
    m2p_launch<T, 4>(g, t, tleaves, n, off, cnt, src, p, h, mp, rel64, nparts, m, far, flags, s);
  else if (p <= 8)
    m2p_launch<T, 8>(g, t, tleaves, n, off, cnt, src, p, h, mp, rel64, nparts, m, far, flags, s);
  else if (p <= 12)
    m2p_launch<T, 12>(g, t, tleaves, n, off, cnt, src, p, h, mp, rel64, nparts, m, far, flags, s);
  else if (p <= 16)
    m2p_launch<T, 16>(g, t, tleaves, n, off, cnt, src, p, h, mp, rel64, nparts, m, far, flags, s);
  else
    m2p_launch<T, 20>(g, t, tleaves, n, off, cnt, src, p, h, mp, rel64, nparts, m, far, flags, s);
}

void m2p(TreeView t, const int* tleaves, int n, const int* off, const int* cnt, const int* src, int p, double h,
         const double2* mp, const double2* rel64, int fp32, int nparts, int64_t m, double* far, int* flags,
         hipStream_t s) {
  if (n <= 0) return;
  const unsigned g = (unsigned)(((int64_t)n * nparts + kM2PWaves - 1) / kM2PWaves);
  if (fp32)
    m2p_dispatch<float>(g, t, tleaves, n, off, cnt, src, p, h, mp, rel64, nparts, m, far, flags, s);
  else
    m2p_dispatch<double>(g, t, tleaves, n, off, cnt, src, p, h, mp, rel64, nparts, m, far, flags, s);
}

}  // namespace pp
