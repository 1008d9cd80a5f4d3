// Quadtree construction over the Morton-ordered sources and sorted targets,
// and the per-leaf packing of sources and targets for the evaluation passes.
//
// The paper groups sources hierarchically in a quadtree (Appendix A, Fig.
// multipole) without saying how it is built.  Here a cell at level l < D is
// split when it holds more than leaf_max sources or more than leaf_max
// targets, and its children (quadrant order q = qx + 2 qy) are kept when
// non-empty.  Cells are numbered level by level, in Morton order within a
// level.  The top levels (up to 9, the default) come from one dense table of Morton
// prefixes in a fixed number of launches; deeper levels are built top down,
// one launch group per level, a child's source and target ranges found by
// binary search of its key prefix inside the parent's ranges.
#include <algorithm>

#include "blockscan.h"
#include "internal.h"
#include "leafpass.h"

namespace pp {

namespace {

// lower_bound of key in a[lo, hi) by one wave: 64 probes per step shrink the
// range 64-fold, so a range of 2^18 keys takes three dependent loads instead
// of eighteen.  All lanes return the same index.
__device__ inline int wave_lower_bound(const uint32_t* __restrict__ a, int lo, int hi, uint64_t key) {
  const int lane = threadIdx.x % kWave;
  while (hi > lo) {
    const int L = hi - lo;
    if (L <= kWave) {
      const bool lt = lane < L && (uint64_t)a[lo + lane] < key;
      return lo + __popcll(__ballot(lt));
    }
    const int step = (L + kWave - 1) / kWave;
    const int pos = min(lo + (lane + 1) * step - 1, hi - 1);
    const int cnt = __popcll(__ballot((uint64_t)a[pos] < key));
    if (cnt == kWave) return hi;  // the last probe is hi - 1
    // a[lo + cnt*step - 1] < key <= a[min(lo + (cnt+1)*step - 1, hi - 1)]
    const int newhi = min(lo + (cnt + 1) * step - 1, hi - 1);
    lo = lo + cnt * step;
    hi = newhi;
  }
  return lo;
}

// One wave per (cell of the level, split point j): j = 0..2 find where source
// quadrants 1..3 of the cell begin, j = 3..5 the same for targets.
__global__ __launch_bounds__(256) void k_level_split(TreeArrays t, const int* __restrict__ ls, int level, int D,
                                                      int leaf_max, const uint32_t* __restrict__ skey,
                                                      const uint32_t* __restrict__ tkey, int* __restrict__ sp,
                                                      int* __restrict__ n4_out) {
  const int c0 = ls[level], c1 = ls[level + 1];
  const int gw = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + threadIdx.x / kWave));
  if (gw == 0 && threadIdx.x % kWave == 0) *n4_out = 4 * (c1 - c0);
  const int nw = 6 * (c1 - c0);
  for (int w = gw; w < nw; w += gridDim.x * 4) {
    const int ci = w / 6, j = w % 6;
    const int c = c0 + ci;
    const int sb = t.sb[c], se = t.se[c], tb = t.tb[c], te = t.te[c];
    const bool split = level < D && (se - sb > leaf_max || te - tb > leaf_max);
    if (!split) continue;
    const int q = j % 3 + 1;
    const int shift = 2 * (D - level - 1);
    const uint32_t prefix = morton(2 * (uint32_t)t.ix[c] + (q & 1), 2 * (uint32_t)t.iy[c] + (q >> 1));
    const uint64_t lo = (uint64_t)prefix << shift;
    const int r = j < 3 ? wave_lower_bound(skey, sb, se, lo) : wave_lower_bound(tkey, tb, te, lo);
    if (threadIdx.x % kWave == 0) sp[6 * ci + j] = r;
  }
}

// Work item w = 4 (c - c0) + q: child quadrant q's source/target ranges from
// the split points, and whether it exists (split parent, non-empty child).
__global__ void k_level_exists(TreeArrays t, const int* __restrict__ ls, int level, int D, int leaf_max,
                               const int* __restrict__ sp, int4* __restrict__ cr, int* __restrict__ exists) {
  const int c0 = ls[level], c1 = ls[level + 1];
  const int n4 = 4 * (c1 - c0);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w < n4; w += stride) {
    const int ci = (int)(w >> 2), q = (int)(w & 3);
    const int c = c0 + ci;
    const int sb = t.sb[c], se = t.se[c], tb = t.tb[c], te = t.te[c];
    const bool split = level < D && (se - sb > leaf_max || te - tb > leaf_max);
    if (!split) {
      exists[w] = 0;
      continue;
    }
    const int* v = sp + 6 * ci;
    const int csb = q == 0 ? sb : v[q - 1], cse = q == 3 ? se : v[q];
    const int ctb = q == 0 ? tb : v[3 + q - 1], cte = q == 3 ? te : v[3 + q];
    cr[w] = make_int4(csb, cse, ctb, cte);
    exists[w] = (cse > csb || cte > ctb) ? 1 : 0;
  }
}

// Children of the level go to c1 + off[w] (off = exclusive scan of exists);
// parents get their first child and child count; ls[level + 2] = c1 + total.
__global__ void k_level_link(TreeArrays t, int* __restrict__ ls, int level, const int4* __restrict__ cr,
                             const int* __restrict__ exists, const int* __restrict__ off,
                             const int* __restrict__ total, int cap, int* __restrict__ flags) {
  const int c0 = ls[level], c1 = ls[level + 1];
  const int n4 = 4 * (c1 - c0);
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int tot = *total;
  const bool fits = (int64_t)c1 + tot <= cap;
  if (gid == 0) {
    ls[level + 2] = fits ? c1 + tot : c1;
    if (!fits) atomicOr(flags, kFlagCellOverflow);
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = gid; w < n4; w += stride) {
    const int c = c0 + (int)(w >> 2);
    const int q = (int)(w & 3);
    if (q == 0) {
      const int n = exists[w] + exists[w + 1] + exists[w + 2] + exists[w + 3];
      t.child[c] = (n > 0 && fits) ? c1 + off[w] : -1;
      t.nchild[c] = fits ? n : 0;
    }
    if (!exists[w] || !fits) continue;
    const int d = c1 + off[w];
    const int4 r = cr[w];
    t.lvl[d] = level + 1;
    t.ix[d] = 2 * t.ix[c] + (q & 1);
    t.iy[d] = 2 * t.iy[c] + (q >> 1);
    t.sb[d] = r.x;
    t.se[d] = r.y;
    t.tb[d] = r.z;
    t.te[d] = r.w;
    t.child[d] = -1;
    t.nchild[d] = 0;
    t.parent[d] = c;
  }
}

// Dense top of the tree.  For the levels L <= Ld every Morton prefix of the
// level is a candidate cell; its source and target ranges come from one table
// of range starts at level Ld (a binary search per prefix), read at stride
// 4^(Ld - L) for the coarser levels.  A candidate exists when its parent was
// split (the parent holds more than leaf_max sources or targets; counts only
// shrink going down, so every further ancestor was split too) and it is not
// empty.  An exclusive scan of the existence flags in (level, prefix) order
// numbers the cells exactly as the level-by-level construction does (level
// major, Morton order within a level), so both give the same tree.
__device__ inline int64_t dense_level_offset(int L) { return (((int64_t)1 << (2 * L)) - 1) / 3; }

__device__ inline int dense_level_of(int64_t idx) {
  int L = 0;
  while (dense_level_offset(L + 1) <= idx) ++L;
  return L;
}

// lower_bound of key in a[0, n) starting from a guess g: gallop away from g until
// the answer is bracketed, then bisect the bracket.  For keys spread evenly over
// the key range a guess proportional to the key needs only a few probes.
__device__ inline int lower_bound_from(const uint32_t* __restrict__ a, int n, uint64_t key, int64_t guess) {
  const int64_t g = guess < 0 ? 0 : (guess > n ? n : guess);
  int64_t lo, hi;
  if (g < n && (uint64_t)a[g] < key) {
    lo = g + 1;
    int64_t step = 1;
    while (lo + step - 1 < n && (uint64_t)a[lo + step - 1] < key) {
      lo += step;
      step *= 2;
    }
    hi = min((int64_t)n, lo + step - 1);
  } else {
    hi = g;
    int64_t step = 1;
    while (hi - step >= 0 && (uint64_t)a[hi - step] >= key) {
      hi -= step;
      step *= 2;
    }
    lo = max((int64_t)0, hi - step + 1);
  }
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if ((uint64_t)a[mid] < key)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (int)lo;
}

// lower_bound of key in a[0, n) by one wave: 64 lanes probe 64 evenly spaced
// entries of the bracket [lo, hi) at once and the ballot of "entry < key"
// narrows it to one gap, so the search takes log64(n) rounds of loads (3 for
// 32,768 keys) instead of the log2(n) rounds of a bisection.  Every lane
// returns the same index.
__device__ inline int wave_lower_bound(const uint32_t* __restrict__ a, int n, uint64_t key) {
  const int lane = threadIdx.x % kWave;
  int64_t lo = 0, hi = n;  // the answer lies in [lo, hi]
  while (lo < hi) {
    const int64_t len = hi - lo;
    const int64_t pos = lo + (len * lane) / kWave;  // < hi
    const uint64_t below = __ballot((uint64_t)a[pos] < key);
    const int c = __popcll(below);  // probes 0 .. c-1 lie below the key
    if (c == 0) {
      hi = lo;
    } else {
      const int64_t plast = lo + (len * (c - 1)) / kWave;
      hi = c == kWave ? hi : lo + (len * c) / kWave;
      lo = plast + 1;
    }
  }
  return (int)lo;
}

// Target starts of one workgroup's kDenseStartsBlock consecutive prefixes:
// two waves find the range [tlo, thi) of target keys that the workgroup's
// prefixes span (wave_lower_bound); if it fits, the range is staged in LDS
// and each thread bisects there, otherwise in global memory within the range.
constexpr int kDenseStartsBlock = 256;
constexpr int kDenseStartsLds = 2048;

// src_done: the source starts ss[0..np) were written by the ingest (grid
// sources, whose ingest visits every Morton index in order); only ss[np].
__global__ __launch_bounds__(kDenseStartsBlock) void k_dense_starts(
    const uint32_t* __restrict__ skey, const int* __restrict__ nsrc_dev, const uint32_t* __restrict__ tkey, int ntgt,
    int D, int Ld, int src_done, int* __restrict__ ss, int* __restrict__ ts) {
  __shared__ uint32_t kv[kDenseStartsLds];
  __shared__ int range[2];
  const int64_t np = (int64_t)1 << (2 * Ld);
  const int sh = 2 * (D - Ld);
  const int64_t P0 = (int64_t)blockIdx.x * kDenseStartsBlock;
  const int64_t P = P0 + threadIdx.x;
  const int w = threadIdx.x / kWave;
  if (w < 2) {
    // prefixes P0 and P0 + block (past np the key exceeds every target key)
    const int64_t Pb = w == 0 ? P0 : P0 + kDenseStartsBlock;
    const int r = wave_lower_bound(tkey, ntgt, (uint64_t)Pb << sh);
    if (threadIdx.x % kWave == 0) range[w] = r;
  }
  __syncthreads();
  const int tlo = range[0], thi = range[1];
  const bool staged = thi - tlo <= kDenseStartsLds;
  if (staged)
    for (int i = threadIdx.x; i < thi - tlo; i += kDenseStartsBlock) kv[i] = tkey[tlo + i];
  __syncthreads();
  if (P > np) return;
  const uint64_t key = (uint64_t)P << sh;
  const int ns = *nsrc_dev;
  if (!src_done || P == np) ss[P] = P == np ? ns : lower_bound_from(skey, ns, key, (P * (int64_t)ns) / np);
  int t;
  if (staged) {
    int lo = 0, hi = thi - tlo;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((uint64_t)kv[mid] < key)
        lo = mid + 1;
      else
        hi = mid;
    }
    t = tlo + lo;
  } else {
    t = tlo + lower_bound_from(tkey + tlo, thi - tlo, key, ((P - P0) * (int64_t)(thi - tlo)) / kDenseStartsBlock);
  }
  ts[P] = t;
}

// Existence flag of every prefix-table cell, and per workgroup (kDenseBlock
// consecutive cells) the number of cells that exist, for k_dense_offsets.
constexpr int kDenseBlock = 256;
// Cells of the levels above split_above are split whatever they hold (the
// top levels of a forest of requests).
__global__ __launch_bounds__(kDenseBlock) void k_dense_flags(const int* __restrict__ ss, const int* __restrict__ ts,
                                                              int D, int Ld, int leaf_max, int split_above,
                                                              int* __restrict__ flag, int* __restrict__ part) {
  __shared__ int lds[kDenseBlock / kWave + 1];
  const int64_t F = dense_level_offset(Ld + 1);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int f = 0;
  if (idx < F) {
    const int L = dense_level_of(idx);
    if (L == 0) {
      f = 1;
    } else {
      const int64_t P = idx - dense_level_offset(L);
      const int sh = 2 * (Ld - L), shp = sh + 2;
      const int64_t Q = P >> 2;
      const int ns = ss[(P + 1) << sh] - ss[P << sh], nt = ts[(P + 1) << sh] - ts[P << sh];
      const int nps = ss[(Q + 1) << shp] - ss[Q << shp], npt = ts[(Q + 1) << shp] - ts[Q << shp];
      const bool split = L - 1 < D && (nps > leaf_max || npt > leaf_max || L - 1 < split_above);
      f = (split && (ns > 0 || nt > 0)) ? 1 : 0;
    }
    flag[idx] = f;
  }
  int total;
  block_excl_scan<kDenseBlock>(f, lds, &total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

// Exclusive scan of the flags (the cell numbers): each workgroup adds up the
// counts of the workgroups before it, then scans its own cells; workgroup 0
// also stores the total.
__global__ __launch_bounds__(kDenseBlock) void k_dense_offsets(const int* __restrict__ flag,
                                                                const int* __restrict__ part, int Ld,
                                                                int* __restrict__ off, int* __restrict__ total_out) {
  __shared__ int lds[kDenseBlock / kWave + 1];
  const int64_t F = dense_level_offset(Ld + 1);
  const int nb = (int)((F + kDenseBlock - 1) / kDenseBlock);
  const int upto = blockIdx.x == 0 ? nb : (int)blockIdx.x;
  // eight loads in flight per thread, added in index order
  int acc = 0;
  for (int i0 = threadIdx.x; i0 < upto; i0 += 8 * kDenseBlock) {
    int v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = i0 + u * kDenseBlock < upto ? part[i0 + u * kDenseBlock] : 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  int before;
  block_excl_scan<kDenseBlock>(acc, lds, &before);
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) *total_out = before;
    before = 0;
  }
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int f = idx < F ? flag[idx] : 0;
  int tot;
  const int ex = block_excl_scan<kDenseBlock>(f, lds, &tot) + before;
  if (idx < F) off[idx] = ex;
}

// The levels below Ld are left empty (ls[Ld+2..D+1] = ls[Ld+1]); *deep
// becomes nonzero when a cell of level Ld is split after all (more than
// leaf_max sources or targets, Ld < D), so the levels below have to be built.
__global__ void k_dense_write(TreeArrays t, const int* __restrict__ flag, const int* __restrict__ off,
                              const int* __restrict__ total_dev, const int* __restrict__ ss,
                              const int* __restrict__ ts, int D, int Ld, int leaf_max, int cap,
                              int* __restrict__ ls, int* __restrict__ deep, int* __restrict__ flags) {
  const int64_t F = dense_level_offset(Ld + 1);
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int total = *total_dev;
  if (idx == 0) {
    // level starts; clamped to the capacity so later launches stay in bounds
    for (int L = 0; L <= Ld; ++L) ls[L] = min(off[dense_level_offset(L)], cap);
    for (int L = Ld + 1; L <= D + 1; ++L) ls[L] = min(total, cap);
    if (total > cap) atomicOr(flags, kFlagCellOverflow);
  }
  if (idx >= F) return;
  const int L = dense_level_of(idx);
  const int64_t P = idx - dense_level_offset(L);
  const int sh = 2 * (Ld - L);
  // everything the cell's record needs is requested at once (indices that
  // depend only on its place in the table), before its flag is tested
  const int fl = flag[idx], id = off[idx];
  const int sb = ss[P << sh], se = ss[(P + 1) << sh], tb = ts[P << sh], te = ts[(P + 1) << sh];
  const int par = L == 0 ? -1 : off[dense_level_offset(L - 1) + (P >> 2)];
  const int64_t c0 = L < Ld ? dense_level_offset(L + 1) + 4 * P : idx;  // (idx: an in-bounds stand-in)
  const int64_t c1 = L < Ld ? c0 + 1 : idx, c2 = L < Ld ? c0 + 2 : idx, c3 = L < Ld ? c0 + 3 : idx;
  int f0 = flag[c0], f1 = flag[c1], f2 = flag[c2], f3 = flag[c3], o0 = off[c0];
  // (an empty statement that takes the values keeps the compiler from moving
  // these loads behind the test below)
  asm volatile("" : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3), "+v"(o0));
  const int n4 = f0 + f1 + f2 + f3;
  if (!fl || id >= cap) return;
  t.lvl[id] = L;
  t.ix[id] = (int)compact_bits((uint32_t)P);
  t.iy[id] = (int)compact_bits((uint32_t)(P >> 1));
  t.sb[id] = sb;
  t.se[id] = se;
  t.tb[id] = tb;
  t.te[id] = te;
  t.parent[id] = par;
  int n = 0, first = -1;
  if (L < Ld) {
    n = n4;
    first = n > 0 && o0 + n <= cap ? o0 : -1;
    if (first < 0) n = 0;
  }
  t.child[id] = first;
  t.nchild[id] = n;
  if (L == Ld && Ld < D && (se - sb > leaf_max || te - tb > leaf_max)) atomicOr(deep, 1);
}

// flag[kind * n + c] for kind 0 = leaf with sources, 1 = leaf with targets,
// 2 = any cell with targets; the cell count n is read on the device (the
// tree's last level start) and 3n is left in *n3 for the scan.
// Cell classification: source leaves, target leaves and cells with targets,
// each compacted in cell order.  Two launches over tiles of kClsTile cells:
// the first counts the three kinds per tile, the second adds up the counts of
// the tiles before its own (few: the tree's cells / kClsTile) and compacts its
// tile with block scans.  The cell count is read from the device.
constexpr int kClsBlock = 256;
constexpr int kClsItems = 1;
constexpr int kClsTile = kClsBlock * kClsItems;

__device__ inline int cls_bits(const TreeArrays& t, int c) {
  const bool leaf = t.child[c] < 0;
  const bool hs = t.se[c] > t.sb[c];
  const bool ht = t.te[c] > t.tb[c];
  return (leaf && hs ? 1 : 0) | (leaf && ht ? 2 : 0) | (ht ? 4 : 0);
}

__global__ __launch_bounds__(kClsBlock) void k_classify_count(TreeArrays t, const int* __restrict__ n_dev,
                                                               int* __restrict__ part, RecordArgs rec) {
  __shared__ int lds[kClsBlock / kWave + 1];
  const int n = *n_dev;
  const int64_t base = (int64_t)blockIdx.x * kClsTile;
  if (base >= n) return;  // uniform per workgroup
  int c0 = 0, c1 = 0, c2 = 0;
  for (int q = 0; q < kClsItems; ++q) {
    const int64_t c = base + (int64_t)threadIdx.x * kClsItems + q;
    if (c < n) {
      if (rec.rec) cell_setup(rec, (int)c);
      const int b = cls_bits(t, (int)c);
      c0 += b & 1;
      c1 += (b >> 1) & 1;
      c2 += (b >> 2) & 1;
    }
  }
  int tot0, tot1, tot2;
  block_excl_scan<kClsBlock>(c0, lds, &tot0);
  block_excl_scan<kClsBlock>(c1, lds, &tot1);
  block_excl_scan<kClsBlock>(c2, lds, &tot2);
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = tot0;
    part[3 * blockIdx.x + 1] = tot1;
    part[3 * blockIdx.x + 2] = tot2;
  }
}

__global__ __launch_bounds__(kClsBlock) void k_classify_emit(TreeArrays t, const int* __restrict__ n_dev,
                                                              const int* __restrict__ part, int* __restrict__ out0,
                                                              int* __restrict__ out1, int* __restrict__ out2,
                                                              int* __restrict__ counts) {
  __shared__ int lds[kClsBlock / kWave + 1];
  const int n = *n_dev;
  const int ntiles = (int)(((int64_t)n + kClsTile - 1) / kClsTile);
  const int64_t base = (int64_t)blockIdx.x * kClsTile;
  if (blockIdx.x > 0 && base >= n) return;  // uniform per workgroup
  // offsets of this tile (and, in workgroup 0, the totals of all tiles)
  const int upto = blockIdx.x == 0 ? ntiles : (int)blockIdx.x;
  // four tiles' counts in flight per thread, added in index order
  int p0 = 0, p1 = 0, p2 = 0;
  for (int i0 = threadIdx.x; i0 < upto; i0 += 4 * kClsBlock) {
    int v[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = i0 + u * kClsBlock;
#pragma unroll
      for (int r = 0; r < 3; ++r) v[u][r] = i < upto ? part[3 * i + r] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      p0 += v[u][0];
      p1 += v[u][1];
      p2 += v[u][2];
    }
  }
  int s0, s1, s2;
  block_excl_scan<kClsBlock>(p0, lds, &s0);
  block_excl_scan<kClsBlock>(p1, lds, &s1);
  block_excl_scan<kClsBlock>(p2, lds, &s2);
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      counts[0] = s0;
      counts[1] = s1;
      counts[2] = s2;
    }
    s0 = s1 = s2 = 0;
  }
  if (base >= n) return;
  int bits[kClsItems];
  int c0 = 0, c1 = 0, c2 = 0;
  for (int q = 0; q < kClsItems; ++q) {
    const int64_t c = base + (int64_t)threadIdx.x * kClsItems + q;
    bits[q] = c < n ? cls_bits(t, (int)c) : 0;
    c0 += bits[q] & 1;
    c1 += (bits[q] >> 1) & 1;
    c2 += (bits[q] >> 2) & 1;
  }
  int tot;
  int o0 = block_excl_scan<kClsBlock>(c0, lds, &tot) + s0;
  int o1 = block_excl_scan<kClsBlock>(c1, lds, &tot) + s1;
  int o2 = block_excl_scan<kClsBlock>(c2, lds, &tot) + s2;
  for (int q = 0; q < kClsItems; ++q) {
    const int c = (int)(base + (int64_t)threadIdx.x * kClsItems + q);
    if (bits[q] & 1) out0[o0++] = c;
    if (bits[q] & 2) out1[o1++] = c;
    if (bits[q] & 4) out2[o2++] = c;
  }
}

// One wave per source leaf: FP32 record (x, y relative to the leaf corner in
// units of h, w) per source; leaf weight sum in FP64 in a fixed order.
// Both per-leaf passes in one launch: the first workgroups pack the source
// leaves, the rest prepare the target leaves.
__global__ __launch_bounds__(256) void k_pack_prep(TreeArrays t, int D, PackArgs a, int pack_blocks, PrepArgs b) {
  const int lane = threadIdx.x % kWave;
  if ((int)blockIdx.x < pack_blocks) {
    const int wid = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (wid < a.ns) pack_leaf(wid, lane, t, a.sleaves, D, a.ij, a.w64, a.s32, a.stride, a.leaf_w);
  } else {
    const int wid = (blockIdx.x - pack_blocks) * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (wid < b.nt)
      prep_leaf(wid, lane, t, b.tleaves, D, b.tx, b.ty, b.perm, b.x0, b.y0, b.h, b.nx, b.ny, b.snap_frac2, b.f,
                b.rel32, b.rel64, b.tleaf, b.self_w, b.self_logd, b.bt);
  }
}

// Packing of the listed source leaves: one wave per target leaf claims the
// leaves of its list that no wave has claimed yet (claim[B] 0 -> 1) and packs
// the ones it claimed with all lanes, grid leaves four at a time (their loads
// issued together).  (Queueing the claimed leaves for a
// second, wide launch was measured slower at 4096^2: that launch fills the
// compute units the upward pass is using.)
__global__ __launch_bounds__(256) void k_pack_listed(LeafPass lp, const int* __restrict__ tleaves, int ntleaves,
                                                     const int* __restrict__ list_off, const int* __restrict__ list_cnt,
                                                     const int* __restrict__ list_src, int ncells,
                                                     int* __restrict__ claim) {
  const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave);
  if (wid >= ntleaves) return;
  const int lane = threadIdx.x % kWave;
  const int A = tleaves[wid];
  const int nb = list_cnt[A];
  const int* lst = list_src + list_off[A];
  for (int e0 = 0; e0 < nb; e0 += kWave) {
    const int e = e0 + lane;
    const int B = e < nb ? lst[e] : -1;
    const bool mine = (unsigned)B < (unsigned)ncells && atomicExch(&claim[B], 1) == 0;
    uint64_t m = __ballot(mine);
    if (lp.kind == 1) {
      while (m) {  // the leaves this wave claimed, up to four at a time
        int cs[4];
        int n = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          cs[q] = 0;
          if (m) {
            cs[q] = __shfl(B, __builtin_ctzll(m), kWave);
            m &= m - 1;
            n = q + 1;
          }
        }
        pack_leaf_cells4(cs, n, lane, lp.t, lp.D, lp.ga.ij, lp.ga.w64, lp.ga.s32, lp.ga.stride, lp.ga.leaf_w);
      }
    } else {
      while (m) {  // the leaves this wave claimed, one at a time
        const int l = __builtin_ctzll(m);
        m &= m - 1;
        run_pack_cell(lp, __shfl(B, l, kWave), lane);
      }
    }
  }
}

// The per-leaf passes of a descriptor as a launch of their own.
__global__ __launch_bounds__(256) void k_leaf_pass(LeafPass lp) { run_leaf_pass(lp, (int)blockIdx.x); }

}  // namespace

void leaf_pass_launch(const LeafPass& lp, hipStream_t s) {
  const int g = lp.pack_blocks + lp.prep_blocks;
  if (g > 0) k_leaf_pass<<<(unsigned)g, 256, 0, s>>>(lp);
}

LeafPass leaf_pass_prep_only(const LeafPass& lp) {
  LeafPass q = lp;
  q.pack_blocks = 0;
  return q;
}

void pack_listed(const LeafPass& lp, const int* tleaves, int ntleaves, const int* list_off, const int* list_cnt,
                 const int* list_src, int ncells, int* claim, hipStream_t s) {
  if (ntleaves <= 0) return;
  k_pack_listed<<<(unsigned)((ntleaves + 3) / 4), 256, 0, s>>>(lp, tleaves, ntleaves, list_off, list_cnt, list_src,
                                                                 ncells, claim);
}

static unsigned level_blocks(int64_t max_cells) {
  const int64_t items = 4 * std::max<int64_t>(max_cells, 1);
  return (unsigned)std::min<int64_t>((items + 255) / 256, 2048);
}

void tree_level(TreeArrays t, int* ls, int level, int D, int leaf_max, int64_t max_cells, int cap,
                const uint32_t* skey, const uint32_t* tkey, int* sp, int4* cr, int* exists, int* off, int* scan_tmp,
                int* n4_slot, int* total_slot, int* flags, hipStream_t s) {
  const int64_t mc = std::max<int64_t>(max_cells, 1);
  const unsigned gs = (unsigned)std::min<int64_t>((6 * mc + 3) / 4, 4096);
  k_level_split<<<gs, 256, 0, s>>>(t, ls, level, D, leaf_max, skey, tkey, sp, n4_slot);
  const unsigned g = level_blocks(mc);
  k_level_exists<<<g, 256, 0, s>>>(t, ls, level, D, leaf_max, sp, cr, exists);
  scan_exclusive_dev(exists, off, n4_slot, 4 * mc, scan_tmp, total_slot, s);
  k_level_link<<<g, 256, 0, s>>>(t, ls, level, cr, exists, off, total_slot, cap, flags);
}

int64_t tree_dense_part_ints(int Ld) { return (tree_dense_cells(Ld) + kDenseBlock - 1) / kDenseBlock + 1; }

int64_t tree_dense_cells(int Ld) { return ((((int64_t)1) << (2 * (Ld + 1))) - 1) / 3; }

void tree_dense_top(TreeArrays t, int* ls, int D, int Ld, int leaf_max, int split_above, int cap,
                    const uint32_t* skey, const int* nsrc_dev, int src_done, const uint32_t* tkey, int ntgt, int* ss,
                    int* ts, int* flag, int* off, int* scan_tmp, int* total_slot, int* deep, int* flags,
                    hipStream_t s) {
  const int64_t np = ((int64_t)1 << (2 * Ld)) + 1;
  k_dense_starts<<<(unsigned)((np + kDenseStartsBlock - 1) / kDenseStartsBlock), kDenseStartsBlock, 0, s>>>(
      skey, nsrc_dev, tkey, ntgt, D, Ld, src_done, ss, ts);
  const int64_t F = tree_dense_cells(Ld);
  const unsigned g = (unsigned)((F + kDenseBlock - 1) / kDenseBlock);
  k_dense_flags<<<g, kDenseBlock, 0, s>>>(ss, ts, D, Ld, leaf_max, split_above, flag, scan_tmp);
  k_dense_offsets<<<g, kDenseBlock, 0, s>>>(flag, scan_tmp, Ld, off, total_slot);
  k_dense_write<<<g, 256, 0, s>>>(t, flag, off, total_slot, ss, ts, D, Ld, leaf_max, cap, ls, deep, flags);
}

int64_t classify_part_ints(int64_t cap) { return 3 * ((cap + kClsTile - 1) / kClsTile) + 3; }

void classify_cells(TreeArrays t, const int* ncells_dev, int cap, int* part, int* sleaves, int* tleaves,
                    int* tcells, int* counts, const RecordArgs* rec, hipStream_t s) {
  if (cap <= 0) return;
  const unsigned g = (unsigned)(((int64_t)cap + kClsTile - 1) / kClsTile);
  k_classify_count<<<g, kClsBlock, 0, s>>>(t, ncells_dev, part, rec ? *rec : RecordArgs{});
  k_classify_emit<<<g, kClsBlock, 0, s>>>(t, ncells_dev, part, sleaves, tleaves, tcells, counts);
}

LeafPass leaf_pass_grid(TreeArrays t, int D, const int* sleaves, int nsleaves, const uint32_t* ij, const double* w64,
                        float* s32, int64_t stride, double* leaf_w, const int* tleaves, int ntleaves, const double* tx,
                        const double* ty, const int* perm, double x0, double y0, double h, int nx, int ny,
                        double snap_frac2, const double* f, float2* rel32, double2* rel64, int* tleaf, double* self_w,
                        double* self_logd, const GridBatch* bt) {
  LeafPass lp;
  lp.kind = 1;
  lp.pack_blocks = std::max(nsleaves, 0) / 4 + (nsleaves % 4 > 0);
  lp.prep_blocks = std::max(ntleaves, 0) / 4 + (ntleaves % 4 > 0);
  lp.t = t;
  lp.D = D;
  lp.ga = PackArgs{sleaves, nsleaves, ij, w64, s32, stride, leaf_w};
  lp.gb = PrepArgs{tleaves, ntleaves, tx, ty, perm, x0, y0, h, nx, ny, snap_frac2, f, rel32, rel64, tleaf, self_w,
                   self_logd, bt ? *bt : GridBatch{}};
  return lp;
}

void leaf_pack_prep(TreeArrays t, int D, const int* sleaves, int nsleaves, const uint32_t* ij, const double* w64,
                    float* s32, int64_t stride, double* leaf_w, const int* tleaves, int ntleaves, const double* tx,
                    const double* ty, const int* perm, double x0, double y0, double h, int nx, int ny,
                    double snap_frac2, const double* f, float2* rel32, double2* rel64, int* tleaf, double* self_w,
                    double* self_logd, const GridBatch* bt, hipStream_t s) {
  const int gp = std::max(nsleaves, 0) / 4 + (nsleaves % 4 > 0);
  const int gt = std::max(ntleaves, 0) / 4 + (ntleaves % 4 > 0);
  if (gp + gt <= 0) return;
  const PackArgs a{sleaves, nsleaves, ij, w64, s32, stride, leaf_w};
  const PrepArgs b{tleaves, ntleaves, tx, ty, perm, x0, y0, h, nx, ny, snap_frac2, f, rel32, rel64, tleaf, self_w,
                   self_logd, bt ? *bt : GridBatch{}};
  k_pack_prep<<<gp + gt, 256, 0, s>>>(t, D, a, gp, b);
}

}  // namespace pp
