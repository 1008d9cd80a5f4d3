// Ingest of grid sources and target keys (steps: source weights w = f h^2 of
// eq. greenSum, Morton keys of the quadtree).
//
// Grid sources need no sort: enumerating Morton indices m of the root's finest
// cells in increasing order and keeping nodes with f != 0 yields the sources
// already in key order.  Each workgroup owns a tile of 1024 consecutive Morton
// indices (a 32 x 32 block of the grid), so its reads of f stay within 32 rows.
#include <algorithm>

#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {
constexpr int kIngBlock = 256;
constexpr int kIngItems = 4;
constexpr int kIngTile = kIngBlock * kIngItems;

__device__ inline bool node_value(const double* __restrict__ f, int nx, int ny, uint64_t m, uint64_t mend,
                                  double* v, int* bad) {
  if (m >= mend) return false;
  const uint32_t i = compact_bits((uint32_t)m);
  const uint32_t j = compact_bits((uint32_t)(m >> 1));
  if (i >= (uint32_t)nx || j >= (uint32_t)ny) return false;
  const double x = f[(int64_t)j * nx + i];
  if (!isfinite(x)) {
    *bad = 1;
    return false;
  }
  *v = x;
  return x != 0.0;
}

__global__ __launch_bounds__(kIngBlock) void k_ingest_count(const double* __restrict__ f, int nx, int ny, int k,
                                                             int* __restrict__ tile_cnt, int* __restrict__ flags) {
  __shared__ int lds[kIngBlock / kWave + 1];
  const uint64_t mend = (uint64_t)1 << (2 * k);
  const uint64_t base = (uint64_t)blockIdx.x * kIngTile + (uint64_t)threadIdx.x * kIngItems;
  int c = 0, bad = 0;
  for (int q = 0; q < kIngItems; ++q) {
    double v;
    c += node_value(f, nx, ny, base + q, mend, &v, &bad) ? 1 : 0;
  }
  if (bad) atomicOr(flags, kFlagNonFiniteSource);
  int total;
  block_excl_scan<kIngBlock>(c, lds, &total);
  if (threadIdx.x == 0) tile_cnt[blockIdx.x] = total;
}

// tile_sum: tile_off holds the per-tile counts instead of their exclusive
// scan; each workgroup then adds up the counts before its own tile (few
// tiles: at most kIngFusedTiles), and the last one stores the total.
// starts (may be null): for every Morton prefix of 2 * sh bits (the cells of
// the tree's dense table), the position of its first source, i.e. the number
// of sources with a smaller key: written by the item whose index begins the
// prefix, before it emits.
__global__ __launch_bounds__(kIngBlock) void k_ingest_emit(const double* __restrict__ f, int nx, int ny, int k,
                                                            double h2, const int* __restrict__ tile_off,
                                                            int tile_sum, int* __restrict__ total_out,
                                                            uint32_t* __restrict__ key, uint32_t* __restrict__ ij,
                                                            double* __restrict__ w64, int* __restrict__ starts,
                                                            int sh) {
  __shared__ int lds[kIngBlock / kWave + 1];
  int before = 0;
  if (tile_sum) {
    int acc = 0;
    for (int t = threadIdx.x; t < (int)blockIdx.x; t += kIngBlock) acc += tile_off[t];
    int all;
    block_excl_scan<kIngBlock>(acc, lds, &all);
    before = all;
    __syncthreads();
  } else {
    before = tile_off[blockIdx.x];
  }
  const uint64_t mend = (uint64_t)1 << (2 * k);
  const uint64_t base = (uint64_t)blockIdx.x * kIngTile + (uint64_t)threadIdx.x * kIngItems;
  double v[kIngItems];
  bool ok[kIngItems];
  int c = 0, bad = 0;
  for (int q = 0; q < kIngItems; ++q) {
    ok[q] = node_value(f, nx, ny, base + q, mend, &v[q], &bad);
    c += ok[q] ? 1 : 0;
  }
  int total;
  int pos = block_excl_scan<kIngBlock>(c, lds, &total) + before;
  if (tile_sum && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_out = before + total;
  const uint64_t pmask = ((uint64_t)1 << (2 * sh)) - 1;
  for (int q = 0; q < kIngItems; ++q) {
    if (starts && base + q < mend && ((base + q) & pmask) == 0) starts[(base + q) >> (2 * sh)] = pos;
    if (!ok[q]) continue;
    const uint64_t m = base + q;
    const uint32_t i = compact_bits((uint32_t)m);
    const uint32_t j = compact_bits((uint32_t)(m >> 1));
    key[pos] = (uint32_t)m;
    ij[pos] = i | (j << 16);
    w64[pos] = v[q] * h2;
    ++pos;
  }
}

// Single pass (count, prefix, emit) over the tiles with a decoupled look-back:
// a workgroup takes the next tile number from a ticket counter (so every
// smaller tile belongs to a workgroup that is already running), counts its
// tile's nonzero nodes and publishes that count.  Its first wave then reads
// the published words of the 64 tiles before it at once: when the nearest
// one that carries a prefix (the count of everything before that tile plus
// its own) is found and every tile after it has published its count, the
// counts and that prefix are added (a wave sum) and the walk ends; a window
// with no prefix is added whole and the walk moves 64 tiles back.  The tile
// then publishes its own prefix and emits.  Status word of a tile: 0 not yet,
// 1 << 62 | count, 2 << 62 | prefix; the array and the ticket start at zero.
// The words carry their own values and nothing else is read through them, so
// relaxed device-scope atomics suffice (acquire loads would invalidate the
// compute unit's caches on every poll).
// A window that is not complete after kSpinLimit reads raises kFlagBadIndex
// and the tile goes on with what it has (the solve is then reported as
// failed), so the kernel always finishes.
constexpr unsigned long long kStAgg = 1ull << 62, kStPre = 2ull << 62, kStVal = (1ull << 62) - 1;
constexpr int kSpinLimit = 1 << 20;

__device__ inline long long wave_sum_ll(long long v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Tiles of kFusedItems nodes per thread (4,096 nodes): a quarter as many tiles
// as the two-pass ingest, so the look-back walks a quarter as far.
constexpr int kFusedItems = 16;
constexpr int kFusedTile = kIngBlock * kFusedItems;

__global__ __launch_bounds__(kIngBlock) void k_ingest_fused(const double* __restrict__ f, int nx, int ny, int k,
                                                             double h2, unsigned long long* __restrict__ status,
                                                             int* __restrict__ ticket, int* __restrict__ total_out,
                                                             uint32_t* __restrict__ key, uint32_t* __restrict__ ij,
                                                             double* __restrict__ w64, int* __restrict__ starts,
                                                             int sh, int* __restrict__ flags) {
  __shared__ int lds[kIngBlock / kWave + 1];
  __shared__ int tile_s, before_s;
  if (threadIdx.x == 0) tile_s = atomicAdd(ticket, 1);
  __syncthreads();
  const int tile = tile_s;
  const uint64_t mend = (uint64_t)1 << (2 * k);
  const uint64_t base = (uint64_t)tile * kFusedTile + (uint64_t)threadIdx.x * kFusedItems;
  double v[kFusedItems];
  bool ok[kFusedItems];
  int c = 0, bad = 0;
#pragma unroll
  for (int q = 0; q < kFusedItems; ++q) {
    ok[q] = node_value(f, nx, ny, base + q, mend, &v[q], &bad);
    c += ok[q] ? 1 : 0;
  }
  if (bad) atomicOr(flags, kFlagNonFiniteSource);
  int total;
  int pos = block_excl_scan<kIngBlock>(c, lds, &total);
  if (threadIdx.x < kWave) {  // the first wave publishes and looks back
    const int lane = threadIdx.x;
    long long before = 0;
    if (lane == 0)
      __hip_atomic_store(&status[tile], (tile == 0 ? kStPre : kStAgg) | (unsigned long long)total, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    if (tile > 0) {
      int top = tile - 1, reads = 0;
      for (;;) {
        const int j = top - lane;
        const unsigned long long st =
            j >= 0 ? __hip_atomic_load(&status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kStPre;
        const unsigned long long kind = st & ~kStVal;
        const unsigned long long pre = __ballot(kind == kStPre);
        const unsigned long long wait = __ballot(kind == 0);
        const int first = pre ? __builtin_ctzll(pre) : kWave;  // nearest tile with a prefix
        const unsigned long long upto = first >= kWave - 1 ? ~0ull : ((2ull << first) - 1);
        if (wait & upto) {  // a tile at or after the prefix has not published yet
          if (++reads > kSpinLimit) {
            if (lane == 0) atomicOr(flags, kFlagBadIndex);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          continue;
        }
        before += wave_sum_ll(lane <= first ? (long long)(st & kStVal) : 0);
        if (first < kWave) break;
        top -= kWave;
      }
      if (lane == 0)
        __hip_atomic_store(&status[tile], kStPre | (unsigned long long)(before + total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      before_s = (int)before;
      if (tile == (int)gridDim.x - 1) *total_out = (int)(before + total);
    }
  }
  __syncthreads();
  pos += before_s;
  const uint64_t pmask = ((uint64_t)1 << (2 * sh)) - 1;
#pragma unroll
  for (int q = 0; q < kFusedItems; ++q) {
    if (starts && base + q < mend && ((base + q) & pmask) == 0) starts[(base + q) >> (2 * sh)] = pos;
    if (!ok[q]) continue;
    const uint64_t m = base + q;
    const uint32_t i = compact_bits((uint32_t)m);
    const uint32_t j = compact_bits((uint32_t)(m >> 1));
    key[pos] = (uint32_t)m;
    ij[pos] = i | (j << 16);
    w64[pos] = v[q] * h2;
    ++pos;
  }
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
// ---- resident solves: new weights on a retained tree, and the checks that
// the tree still fits the input ----

constexpr int kResBlock = 256;

__device__ inline int block_sum_int(int v, int* lds) {
  int total;
  block_excl_scan<kResBlock>(v, lds, &total);
  return total;
}

// w = f h^2 of every retained source (its packed node index), the number of
// retained sources with f != 0, and the number of nonzero nodes of the whole
// grid: the retained tree fits the new f exactly when the two counts agree
// (no node outside it has become nonzero).
__global__ __launch_bounds__(kResBlock) void k_resident_weights(const double* __restrict__ f, int nx, int64_t ngrid,
                                                                 double h2, const uint32_t* __restrict__ ij,
                                                                 int64_t n, double* __restrict__ w64,
                                                                 int* __restrict__ cnt_kept,
                                                                 int* __restrict__ cnt_all, int* __restrict__ flags) {
  __shared__ int lds[kResBlock / kWave + 1];
  const int64_t stride = (int64_t)gridDim.x * kResBlock;
  int kept = 0, all = 0, bad = 0;
  for (int64_t q = (int64_t)blockIdx.x * kResBlock + threadIdx.x; q < n; q += stride) {
    const uint32_t c = ij[q];
    const double v = f[(int64_t)(c >> 16) * nx + (c & 0xFFFFu)];
    w64[q] = v * h2;
    kept += v != 0.0;
  }
  for (int64_t q = (int64_t)blockIdx.x * kResBlock + threadIdx.x; q < ngrid; q += stride) {
    const double v = f[q];
    bad |= !isfinite(v);
    all += v != 0.0;
  }
  if (bad) atomicOr(flags, kFlagNonFiniteSource);
  kept = block_sum_int(kept, lds);
  __syncthreads();
  all = block_sum_int(all, lds);
  if (threadIdx.x == 0) {
    if (kept) atomicAdd(cnt_kept, kept);
    if (all) atomicAdd(cnt_all, all);
  }
}

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

__global__ void k_resident_verdict(const int* __restrict__ cnt_kept, const int* __restrict__ cnt_all,
                                   int* __restrict__ flags) {
  if (threadIdx.x == 0 && *cnt_kept != *cnt_all) atomicOr(flags, kFlagStale);
}
}  // namespace

void resident_weights(const double* f, int nx, int ny, double h2, const uint32_t* ij, int64_t n, double* w64,
                      int* cnt_kept, int* cnt_all, int* flags, hipStream_t s) {
  const int64_t ngrid = (int64_t)nx * ny;
  const int64_t work = std::max<int64_t>(ngrid, 1);
  const unsigned blocks = (unsigned)std::min<int64_t>((work + kResBlock - 1) / kResBlock, 4096);
  k_resident_weights<<<blocks, kResBlock, 0, s>>>(f, nx, ngrid, h2, ij, n, w64, cnt_kept, cnt_all, flags);
  k_resident_verdict<<<1, kWave, 0, s>>>(cnt_kept, cnt_all, flags);
}

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

void ingest_grid_count(const double* f, int nx, int ny, int k, int* tile_cnt, int* flags, hipStream_t s) {
  k_ingest_count<<<(unsigned)ingest_num_tiles(k), kIngBlock, 0, s>>>(f, nx, ny, k, tile_cnt, flags);
}

void ingest_grid_emit(const double* f, int nx, int ny, int k, double h2, const int* tile_off, int tile_sum,
                      int* total_out, uint32_t* key, uint32_t* ij, double* w64, int* starts, int sh, hipStream_t s) {
  k_ingest_emit<<<(unsigned)ingest_num_tiles(k), kIngBlock, 0, s>>>(f, nx, ny, k, h2, tile_off, tile_sum, total_out,
                                                                     key, ij, w64, starts, sh);
}

int64_t ingest_fused_tiles(int k) {
  const int64_t cells = (int64_t)1 << (2 * k);
  return (cells + kFusedTile - 1) / kFusedTile;
}

void ingest_grid_fused(const double* f, int nx, int ny, int k, double h2, unsigned long long* status, int* ticket,
                       int* total_out, uint32_t* key, uint32_t* ij, double* w64, int* starts, int sh, int* flags,
                       hipStream_t s) {
  k_ingest_fused<<<(unsigned)ingest_fused_tiles(k), kIngBlock, 0, s>>>(f, nx, ny, k, h2, status, ticket, total_out,
                                                                        key, ij, w64, starts, sh, flags);
}

void target_keys(const double* tx, const double* ty, int64_t m, double x0, double y0, double h, int k, uint32_t* key,
                 int* idx, int* flags, hipStream_t s) {
  if (m <= 0) return;
  const int b = 256;
  k_target_keys<<<(unsigned)((m + b - 1) / b), b, 0, s>>>(tx, ty, m, x0, y0, h, k, key, idx, flags);
}

}  // namespace pp
