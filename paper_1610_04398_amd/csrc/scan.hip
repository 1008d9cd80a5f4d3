// Device-wide exclusive prefix sum of int32 counts (three-phase: tile
// reductions, one-workgroup scan of the tile sums, tile scans).  Used for
// every compaction in the pipeline (sources, tree levels, lists, sort bins).
#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__global__ __launch_bounds__(kScanBlock) void scan_tile_reduce(const int* __restrict__ in, int n,
                                                                int* __restrict__ partial) {
  __shared__ int lds[kScanBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
  int total;
  block_excl_scan<kScanBlock>(s, lds, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// One workgroup: exclusive scan of partial[0..nb) in place; total to *total.
__global__ __launch_bounds__(kScanBlock) void scan_partials(int* __restrict__ partial, int nb,
                                                             int* __restrict__ total_out) {
  __shared__ int lds[kScanBlock / kWave + 1];
  int carry = 0;
  for (int base = 0; base < nb; base += kScanBlock) {
    int i = base + threadIdx.x;
    int v = i < nb ? partial[i] : 0;
    int tot;
    int ex = block_excl_scan<kScanBlock>(v, lds, &tot);
    if (i < nb) partial[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kScanBlock) void scan_tiles(const int* __restrict__ in, int n,
                                                          const int* __restrict__ partial, int* __restrict__ out) {
  __shared__ int lds[kScanBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  // each thread owns kScanItems consecutive elements
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  int tot;
  int ex = block_excl_scan<kScanBlock>(s, lds, &tot) + partial[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    if (i < n) out[i] = ex;
    ex += v[k];
  }
}
}  // namespace

namespace {
__global__ void k_fill_i32(int* __restrict__ p, int v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
}  // namespace

void fill_i32(int* p, int v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
}

size_t scan_temp_ints(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

void scan_exclusive(const int* in, int* out, int64_t n, int* temp, int* total_dev, hipStream_t s) {
  if (n <= 0) {
    if (total_dev) fill_i32(total_dev, 0, 1, s);
    return;
  }
  const int nb = (int)((n + kScanTile - 1) / kScanTile);
  scan_tile_reduce<<<nb, kScanBlock, 0, s>>>(in, (int)n, temp);
  scan_partials<<<1, kScanBlock, 0, s>>>(temp, nb, total_dev);
  scan_tiles<<<nb, kScanBlock, 0, s>>>(in, (int)n, temp, out);
}

}  // namespace pp
