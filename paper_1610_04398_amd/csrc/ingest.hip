// Ingest of grid sources and target keys (steps: source weights w = f h^2 of
// eq. greenSum, Morton keys of the quadtree).
//
// Grid sources need no sort: enumerating Morton indices m of the root's finest
// cells in increasing order and keeping nodes with f != 0 yields the sources
// already in key order.  Two passes over f: nonzero counts per Morton tile,
// then the emission of each tile at its offset.  A resident solve (the tree of
// the last solve on the same grid kept) runs the emitting pass alone, with the
// retained tile counts, and checks that the nonzero nodes are still the same.
#include <algorithm>

#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {
constexpr int kIngBlock = 256;
// A tile: 2^11 consecutive Morton indices, i.e. a block of 64 columns by 32
// rows (x takes the even key bits).  Its rows are read whole (each lane two
// neighbouring nodes, 32 lanes a 512-byte row), so the loads stay coalesced
// although the output is in Morton order.
constexpr int kTileBits = 11;
constexpr int kIngTile = 1 << kTileBits;
constexpr int kTileW = 64, kTileH = 32;
constexpr int kPairLanes = kTileW / 2;                // lanes per tile row
constexpr int kRowsPerPass = kIngBlock / kPairLanes;  // 8
constexpr int kPasses = kTileH / kRowsPerPass;        // 4 row passes per tile
constexpr int kItems = kIngTile / kIngBlock;          // 8 consecutive indices per thread
// Tiles are counted in groups (one counting workgroup each); at most this many
// groups, so that an emitting workgroup adds up few group totals.
constexpr int64_t kMaxGroups = 1024;
constexpr int kGroupReads = (int)(kMaxGroups / kIngBlock);  // group totals read per lane

// Two horizontally neighbouring nodes (i, j) and (i + 1, j); zero outside the
// grid.  VEC: f is 16-byte aligned and nx even, so a pair is one 16-byte load
// and lies wholly inside or outside the grid.
template <bool VEC>
__device__ inline void load_pair(const double* __restrict__ f, int nx, int ny, int i, int j, double* a,
                                 double* b) {
  *a = 0.0;
  *b = 0.0;
  if (i >= nx || j >= ny) return;
  const double* p = f + (int64_t)j * nx + i;
  if (VEC) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    *a = v.x;
    *b = v.y;
  } else {
    *a = p[0];
    if (i + 1 < nx) *b = p[1];
  }
}

// Local Morton index of column x, row y inside a tile.
__device__ inline uint32_t tile_index(uint32_t x, uint32_t y) { return spread_bits(x) | (spread_bits(y) << 1); }

// Position in the LDS staging array of a tile's node li (Morton order).  The
// pairs of doubles are permuted (bits 4-7 of the pair index XORed into bits
// 0-3, a bijection) so that both access patterns spread over the LDS banks:
// a row pass (32 lanes on the pairs of one row: pair-index bits 1, 3, 5, 7, 9)
// and the per-thread reads of 8 consecutive nodes (pair-index bits 2-7 from
// the thread).  Unpermuted, each went to 4 of the 16 bank groups of a pair.
__device__ inline uint32_t stage_pos(uint32_t li) {
  const uint32_t d = li >> 1;
  const uint32_t g = ((d >> 5) & 1u) | (((d >> 4) & 1u) << 1) | (((d >> 7) & 1u) << 2) | (((d >> 6) & 1u) << 3);
  return ((d ^ g) << 1) | (li & 1u);
}

// Tile t of the (joint) Morton order: the grid it reads (null: an empty
// forest cell), the tile's first node (i0, j0) in that grid, its first key
// and the offset (vx, vy) of the grid's nodes in the joint index space.
struct TileSrc {
  const double* f;
  int i0, j0;
  uint32_t key0;
  int vx, vy;
};
__device__ inline TileSrc tile_src(const double* f, int64_t t, const GridBatch& b) {
  if (b.nreq == 0) {
    const uint32_t m0 = (uint32_t)(t << kTileBits);
    return {f, (int)compact_bits(m0), (int)compact_bits(m0 >> 1), m0, 0, 0};
  }
  const int64_t per = ((int64_t)1 << (2 * b.D)) >> kTileBits;  // tiles per request (b.D >= 6)
  const int r = (int)(t / per);
  const uint32_t m0 = (uint32_t)((t - (int64_t)r * per) << kTileBits);
  return {r < b.nreq ? b.f[r] : nullptr, (int)compact_bits(m0), (int)compact_bits(m0 >> 1),
          ((uint32_t)r << (2 * b.D)) | m0, (int)compact_bits((uint32_t)r) << b.D,
          (int)compact_bits((uint32_t)r >> 1) << b.D};
}

// Tile counts.  Workgroup g counts the nonzero nodes of tiles [g G, g G + G)
// two tiles at a time (eight row loads in flight per lane), then stores, per
// tile, the count of the tiles before it in the group (tile_pre) and the group
// total (grp[g]).  Non-finite values raise kFlagNonFiniteSource.
template <bool VEC>
__global__ __launch_bounds__(kIngBlock) void k_ingest_count(const double* __restrict__ f, int nx, int ny, int G,
                                                             int* __restrict__ tile_pre, int* __restrict__ grp,
                                                             int* __restrict__ flags, GridBatch bt) {
  extern __shared__ int cnt[];  // G counts
  __shared__ int lds[kIngBlock / kWave + 1];
  const int g = blockIdx.x;
  for (int q = threadIdx.x; q < G; q += kIngBlock) cnt[q] = 0;
  __syncthreads();
  const int c = threadIdx.x % kPairLanes, r = threadIdx.x / kPairLanes;
  int bad = 0;
  for (int q = 0; q < G; q += 2) {
    int n[2] = {0, 0};
    double a[2][kPasses], b[2][kPasses];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const TileSrc ts = tile_src(f, (int64_t)g * G + q + u, bt);
      const bool live = q + u < G && ts.f;
#pragma unroll
      for (int s = 0; s < kPasses; ++s) {
        a[u][s] = b[u][s] = 0.0;
        if (live) load_pair<VEC>(ts.f, nx, ny, ts.i0 + 2 * c, ts.j0 + r + s * kRowsPerPass, &a[u][s], &b[u][s]);
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
#pragma unroll
      for (int s = 0; s < kPasses; ++s) {
        bad |= !isfinite(a[u][s]) || !isfinite(b[u][s]);
        n[u] += (a[u][s] != 0.0) + (b[u][s] != 0.0);
      }
      n[u] = wave_sum(n[u]);
    }
    if (lane_id() == 0) {
      if (n[0]) atomicAdd(&cnt[q], n[0]);
      if (n[1] && q + 1 < G) atomicAdd(&cnt[q + 1], n[1]);
    }
  }
  if (bad) atomicOr(flags, kFlagNonFiniteSource);
  __syncthreads();
  // exclusive scan of the G counts (G / 256 per thread, in order)
  const int per = (G + kIngBlock - 1) / kIngBlock;
  const int q0 = threadIdx.x * per;
  int mine = 0;
  for (int q = q0; q < q0 + per && q < G; ++q) mine += cnt[q];
  int total;
  int run = block_excl_scan<kIngBlock>(mine, lds, &total);
  for (int q = q0; q < q0 + per && q < G; ++q) {
    tile_pre[(int64_t)g * G + q] = run;
    run += cnt[q];
  }
  if (threadIdx.x == 0) grp[g] = total;
}

// Emission of tile blockIdx.x: its offset is the sum of the group totals
// before its group plus its prefix inside the group (both from the counting
// pass).  The tile's rows are staged in LDS in Morton order; each thread then
// takes 8 consecutive indices, the workgroup scans the nonzero counts, the
// kept nodes are compacted in LDS (weight and local index) and written out
// with consecutive lanes on consecutive sources.  A tile the counting pass
// found empty is not read again (only its prefix starts are written).
// starts (may be null): for every Morton prefix of 2 * sh bits (the cells of
// the tree's dense table), the position of its first source, i.e. the number
// of sources with a smaller key.
template <bool VEC>
__global__ __launch_bounds__(kIngBlock) void k_ingest_emit(const double* __restrict__ f, int nx, int ny, int k,
                                                            double h2, const int* __restrict__ tile_pre,
                                                            const int* __restrict__ grp, int G,
                                                            int* __restrict__ total_out,
                                                            uint32_t* __restrict__ ij, double* __restrict__ w64,
                                                            int* __restrict__ starts, int sh, GridBatch bt) {
  __shared__ double wv[kIngTile];     // node values in Morton order, then the kept weights
  __shared__ uint16_t lix[kIngTile];  // local Morton index of each kept node
  __shared__ int lds[kIngBlock / kWave + 1];
  const int64_t t = blockIdx.x;
  const TileSrc ts = tile_src(f, t, bt);
  const uint32_t m0 = ts.key0;
  const int i0 = ts.i0, j0 = ts.j0;
  const int c = threadIdx.x % kPairLanes, r = threadIdx.x / kPairLanes;
  // offset of the tile: the group totals before its group (read first, so
  // that adding them up need not wait for the rows) and its prefix in the group
  const int g = (int)(t / G);
  int gv[kGroupReads];
#pragma unroll
  for (int u = 0; u < kGroupReads; ++u) {
    const int q = threadIdx.x + u * kIngBlock;
    gv[u] = q < g ? grp[q] : 0;
  }
  const int inner = tile_pre[t];
  const int next = (t + 1) % G == 0 ? grp[g] : tile_pre[t + 1];
  const bool any = ts.f && next != inner;  // uniform over the workgroup
  double a[kPasses], b[kPasses];
#pragma unroll
  for (int s = 0; s < kPasses; ++s) {
    a[s] = b[s] = 0.0;
    if (any) load_pair<VEC>(ts.f, nx, ny, i0 + 2 * c, j0 + r + s * kRowsPerPass, &a[s], &b[s]);
  }
  int acc = 0;
#pragma unroll
  for (int u = 0; u < kGroupReads; ++u) acc += gv[u];
  int before;
  block_excl_scan<kIngBlock>(acc, lds, &before);  // ends with a barrier
  before += inner;
  const uint64_t mend = (uint64_t)1 << (2 * k);
  const uint32_t pmask = (uint32_t)(((uint64_t)1 << (2 * sh)) - 1);
  const int l0 = threadIdx.x * kItems;
  if (!any) {
    if (starts) {
#pragma unroll
      for (int q = 0; q < kItems; ++q) {
        const uint32_t m = m0 | (uint32_t)(l0 + q);
        if ((uint64_t)m < mend && (m & pmask) == 0) starts[m >> (2 * sh)] = before;
      }
    }
    if (t == (int64_t)gridDim.x - 1 && threadIdx.x == 0) *total_out = before;
    return;
  }
#pragma unroll
  for (int s = 0; s < kPasses; ++s) {
    const uint32_t li = tile_index(2 * c, r + s * kRowsPerPass);  // even: the pair is adjacent
    *reinterpret_cast<double2*>(&wv[stage_pos(li)]) = make_double2(a[s], b[s]);
  }
  __syncthreads();
  double v[kItems];
#pragma unroll
  for (int q = 0; q < kItems; q += 2) {
    const double2 p = *reinterpret_cast<const double2*>(&wv[stage_pos(l0 + q)]);
    v[q] = p.x;
    v[q + 1] = p.y;
  }
  int cn = 0;
#pragma unroll
  for (int q = 0; q < kItems; ++q) cn += v[q] != 0.0;
  int total;
  int pos = block_excl_scan<kIngBlock>(cn, lds, &total);  // ends with a barrier: wv is free
#pragma unroll
  for (int q = 0; q < kItems; ++q) {
    const uint32_t m = m0 | (uint32_t)(l0 + q);
    if (starts && (uint64_t)m < mend && (m & pmask) == 0) starts[m >> (2 * sh)] = before + pos;
    if (v[q] != 0.0) {
      wv[pos] = v[q] * h2;
      lix[pos] = (uint16_t)(l0 + q);
      ++pos;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < total; q += kIngBlock) {
    const int64_t o = (int64_t)before + q;
    const uint32_t li = lix[q];
    ij[o] = (uint32_t)(ts.vx + i0 + (int)compact_bits(li)) | ((uint32_t)(ts.vy + j0 + (int)compact_bits(li >> 1)) << 16);
    w64[o] = wv[q];
  }
  if (t == (int64_t)gridDim.x - 1 && threadIdx.x == 0) *total_out = before + total;
}

// Resident weights: tile blockIdx.x of the new f is staged in LDS in Morton
// order as above; its retained sources (the range the counting pass of the
// retained tree gave the tile; their node indices locate them in the tile)
// take w = f h^2 from it and mark their nodes (a byte each: plain stores, the
// retained nodes being distinct), and a nonzero node left unmarked (a node
// outside the retained tree) raises kFlagStale.  Nodes that became zero keep
// their place with w = 0.
template <bool VEC>
__global__ __launch_bounds__(kIngBlock) void k_resident_weights(const double* __restrict__ f, int nx, int ny,
                                                                 double h2, const int* __restrict__ tile_pre,
                                                                 const int* __restrict__ grp, int G,
                                                                 const uint32_t* __restrict__ ij, int64_t n,
                                                                 double* __restrict__ w64, int* __restrict__ flags) {
  __shared__ double wv[kIngTile];
  __shared__ uint64_t kept[kIngTile / 8];  // a byte per node of the tile
  __shared__ int lds[kIngBlock / kWave + 1];
  const int64_t t = blockIdx.x;
  const uint32_t m0 = (uint32_t)(t << kTileBits);
  const int i0 = (int)compact_bits(m0), j0 = (int)compact_bits(m0 >> 1);
  const int c = threadIdx.x % kPairLanes, r = threadIdx.x / kPairLanes;
  const int g = (int)(t / G);
  int gv[kGroupReads];
#pragma unroll
  for (int u = 0; u < kGroupReads; ++u) {
    const int q = threadIdx.x + u * kIngBlock;
    gv[u] = q < g ? grp[q] : 0;
  }
  const int inner = tile_pre[t];
  const int next = (t + 1) % G == 0 ? grp[g] : tile_pre[t + 1];
  double a[kPasses], b[kPasses];
#pragma unroll
  for (int s = 0; s < kPasses; ++s) load_pair<VEC>(f, nx, ny, i0 + 2 * c, j0 + r + s * kRowsPerPass, &a[s], &b[s]);
  kept[threadIdx.x] = 0;  // kIngTile / 8 == kIngBlock
  int acc = 0;
#pragma unroll
  for (int u = 0; u < kGroupReads; ++u) acc += gv[u];
  int before;
  block_excl_scan<kIngBlock>(acc, lds, &before);  // (its barriers also order the bitmap's clearing)
  const int cnt = next - inner;
  before += inner;
  int bad = 0;
#pragma unroll
  for (int s = 0; s < kPasses; ++s) {
    bad |= !isfinite(a[s]) || !isfinite(b[s]);
    const uint32_t li = tile_index(2 * c, r + s * kRowsPerPass);
    *reinterpret_cast<double2*>(&wv[stage_pos(li)]) = make_double2(a[s], b[s]);
  }
  if (bad) atomicOr(flags, kFlagNonFiniteSource);
  __syncthreads();
  int stale = 0;
  uint8_t* kept8 = reinterpret_cast<uint8_t*>(kept);
  // the retained node indices of the tile (at most 2048: eight per thread), loaded together
  for (int q0 = threadIdx.x; q0 < cnt; q0 += kItems * kIngBlock) {
    uint32_t vq[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
      const int q = q0 + u * kIngBlock;
      const int64_t o = (int64_t)before + q;
      vq[u] = q < cnt && o < n ? ij[o] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
      const int q = q0 + u * kIngBlock;
      if (q >= cnt) continue;
      const int64_t o = (int64_t)before + q;
      if (o >= n) {
        stale = 1;
        continue;
      }
      const uint32_t dx = (vq[u] & 0xFFFFu) - (uint32_t)i0, dy = (vq[u] >> 16) - (uint32_t)j0;
      if (dx >= (uint32_t)kTileW || dy >= (uint32_t)kTileH) {
        stale = 1;
        continue;
      }
      const uint32_t li = tile_index(dx, dy);
      w64[o] = wv[stage_pos(li)] * h2;
      kept8[li] = 1;
    }
  }
  __syncthreads();
  const int l0 = threadIdx.x * kItems;
  const uint64_t mask = kept[threadIdx.x];  // the bytes of nodes l0 .. l0 + 7
#pragma unroll
  for (int q = 0; q < kItems; ++q) stale |= wv[stage_pos(l0 + q)] != 0.0 && !((mask >> (8 * q)) & 1u);
  if (stale) atomicOr(flags, kFlagStale);
}

__global__ void k_target_keys(const double* __restrict__ tx, const double* __restrict__ ty, int64_t m, double x0,
                              double y0, double h, int k, uint32_t* __restrict__ key, int* __restrict__ idx,
                              int* __restrict__ flags) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  int err = 0;
  const uint32_t kk = target_key(tx[t], ty[t], x0, y0, h, k, &err);
  if (err) atomicOr(flags, err == 1 ? kFlagNonFiniteTarget : kFlagTargetOutside);
  key[t] = kk;
  idx[t] = (int)t;
}

// ---- resident solves: the check that the sorted targets still fit the
// retained tree (its new weights come from the emitting pass above) ----

// Every target must still lie in the finest cell it was sorted into.
__global__ void k_resident_targets(const double* __restrict__ tx, const double* __restrict__ ty, int64_t m,
                                   const int* __restrict__ perm, const uint32_t* __restrict__ key, double x0,
                                   double y0, double h, int k, int* __restrict__ flags) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= m) return;
  const int t = perm[q];
  int err = 0;
  const uint32_t kk = target_key(tx[t], ty[t], x0, y0, h, k, &err);
  if (err) atomicOr(flags, err == 1 ? kFlagNonFiniteTarget : kFlagTargetOutside);
  else if (kk != key[q]) atomicOr(flags, kFlagStale);
}

}  // namespace

void resident_targets(const double* tx, const double* ty, int64_t m, const int* perm, const uint32_t* key, double x0,
                      double y0, double h, int k, int* flags, hipStream_t s) {
  if (m <= 0) return;
  const int b = 256;
  k_resident_targets<<<(unsigned)((m + b - 1) / b), b, 0, s>>>(tx, ty, m, perm, key, x0, y0, h, k, flags);
}

int64_t ingest_num_tiles(int k) {
  const int64_t cells = (int64_t)1 << (2 * k);
  return (cells + kIngTile - 1) / kIngTile;
}

namespace {
int group_tiles(int k) { return (int)std::max<int64_t>(1, ingest_num_tiles(k) / kMaxGroups); }
bool vec_ok(const double* f, int nx) { return (nx % 2) == 0 && ((uintptr_t)f % 16) == 0; }
}  // namespace

int64_t ingest_count_ints(int k) {
  const int64_t nt = ingest_num_tiles(k);
  return nt + nt / group_tiles(k);
}

namespace {
bool vec_ok_all(const double* f, int nx, const GridBatch* bt) {
  if (!bt || bt->nreq == 0) return vec_ok(f, nx);
  for (int r = 0; r < bt->nreq; ++r)
    if (!vec_ok(bt->f[r], nx)) return false;
  return true;
}
}  // namespace

void ingest_grid_count(const double* f, int nx, int ny, int k, int* tile_cnt, int* flags, const GridBatch* bt,
                       hipStream_t s) {
  const int G = group_tiles(k);
  const int64_t nt = ingest_num_tiles(k);
  const unsigned ng = (unsigned)(nt / G);
  const size_t lds = (size_t)G * sizeof(int);
  const GridBatch b = bt ? *bt : GridBatch{};
  if (vec_ok_all(f, nx, bt))
    k_ingest_count<true><<<ng, kIngBlock, lds, s>>>(f, nx, ny, G, tile_cnt, tile_cnt + nt, flags, b);
  else
    k_ingest_count<false><<<ng, kIngBlock, lds, s>>>(f, nx, ny, G, tile_cnt, tile_cnt + nt, flags, b);
}

void ingest_grid_emit(const double* f, int nx, int ny, int k, double h2, const int* tile_cnt, int* total_out,
                      uint32_t* ij, double* w64, int* starts, int sh, const GridBatch* bt, hipStream_t s) {
  const int G = group_tiles(k);
  const int64_t nt = ingest_num_tiles(k);
  const GridBatch b = bt ? *bt : GridBatch{};
  if (vec_ok_all(f, nx, bt))
    k_ingest_emit<true><<<(unsigned)nt, kIngBlock, 0, s>>>(f, nx, ny, k, h2, tile_cnt, tile_cnt + nt, G, total_out,
                                                            ij, w64, starts, sh, b);
  else
    k_ingest_emit<false><<<(unsigned)nt, kIngBlock, 0, s>>>(f, nx, ny, k, h2, tile_cnt, tile_cnt + nt, G, total_out,
                                                             ij, w64, starts, sh, b);
}

__global__ void k_keys_from_ij(const uint32_t* __restrict__ ij, const int* __restrict__ n_dev, int64_t n,
                               uint32_t* __restrict__ key) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t lim = n_dev ? std::min<int64_t>(*n_dev, n) : n;
  if (i >= lim) return;
  const uint32_t v = ij[i];
  key[i] = spread_bits(v & 0xFFFFu) | (spread_bits(v >> 16) << 1);
}

void keys_from_ij(const uint32_t* ij, const int* n_dev, int64_t n, uint32_t* key, hipStream_t s) {
  if (n <= 0) return;
  k_keys_from_ij<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ij, n_dev, n, key);
}

void resident_weights(const double* f, int nx, int ny, int k, double h2, const int* tile_cnt, const uint32_t* ij,
                      int64_t n, double* w64, int* flags, hipStream_t s) {
  const int G = group_tiles(k);
  const int64_t nt = ingest_num_tiles(k);
  if (vec_ok(f, nx))
    k_resident_weights<true><<<(unsigned)nt, kIngBlock, 0, s>>>(f, nx, ny, h2, tile_cnt, tile_cnt + nt, G, ij, n,
                                                                 w64, flags);
  else
    k_resident_weights<false><<<(unsigned)nt, kIngBlock, 0, s>>>(f, nx, ny, h2, tile_cnt, tile_cnt + nt, G, ij, n,
                                                                  w64, flags);
}

void target_keys(const double* tx, const double* ty, int64_t m, double x0, double y0, double h, int k, uint32_t* key,
                 int* idx, int* flags, hipStream_t s) {
  if (m <= 0) return;
  const int b = 256;
  k_target_keys<<<(unsigned)((m + b - 1) / b), b, 0, s>>>(tx, ty, m, x0, y0, h, k, key, idx, flags);
}

}  // namespace pp
