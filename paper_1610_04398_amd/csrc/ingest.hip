// Ingest of grid sources and target keys (steps: source weights w = f h^2 of
// eq. greenSum, Morton keys of the quadtree).
//
// Grid sources need no sort: enumerating Morton indices m of the root's finest
// cells in increasing order and keeping nodes with f != 0 yields the sources
// already in key order.  Each workgroup owns a tile of 1024 consecutive Morton
// indices (a 32 x 32 block of the grid), so its reads of f stay within 32 rows.
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
__global__ __launch_bounds__(kIngBlock) void k_ingest_emit(const double* __restrict__ f, int nx, int ny, int k,
                                                            double h2, const int* __restrict__ tile_off,
                                                            int tile_sum, int* __restrict__ total_out,
                                                            uint32_t* __restrict__ key, uint32_t* __restrict__ ij,
                                                            double* __restrict__ w64) {
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
  for (int q = 0; q < kIngItems; ++q) {
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
}  // namespace

int64_t ingest_num_tiles(int k) {
  const int64_t cells = (int64_t)1 << (2 * k);
  return (cells + kIngTile - 1) / kIngTile;
}

void ingest_grid_count(const double* f, int nx, int ny, int k, int* tile_cnt, int* flags, hipStream_t s) {
  k_ingest_count<<<(unsigned)ingest_num_tiles(k), kIngBlock, 0, s>>>(f, nx, ny, k, tile_cnt, flags);
}

void ingest_grid_emit(const double* f, int nx, int ny, int k, double h2, const int* tile_off, int tile_sum,
                      int* total_out, uint32_t* key, uint32_t* ij, double* w64, hipStream_t s) {
  k_ingest_emit<<<(unsigned)ingest_num_tiles(k), kIngBlock, 0, s>>>(f, nx, ny, k, h2, tile_off, tile_sum, total_out,
                                                                     key, ij, w64);
}

void target_keys(const double* tx, const double* ty, int64_t m, double x0, double y0, double h, int k, uint32_t* key,
                 int* idx, int* flags, hipStream_t s) {
  if (m <= 0) return;
  const int b = 256;
  k_target_keys<<<(unsigned)((m + b - 1) / b), b, 0, s>>>(tx, ty, m, x0, y0, h, k, key, idx, flags);
}

}  // namespace pp
