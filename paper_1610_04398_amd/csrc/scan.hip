// Device-wide exclusive prefix sum of int32 counts, used for every compaction
// in the pipeline (sources, tree levels, lists, sort bins).
//
// The element count is either a host value or read from device memory (so a
// level of the tree can be compacted without a host round trip); grids are then
// sized for an upper bound and surplus workgroups exit.  Up to kSmallMax
// elements one workgroup scans everything in a single launch; larger inputs use
// tile reductions and then tile scans that each add up the tile sums before
// their own.
#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;
constexpr int kSmallBlock = 1024;
constexpr int kSmallItems = 8;
constexpr int64_t kSmallMax = (int64_t)kSmallBlock * kSmallItems;

// Element count: the device value (clamped to the launch's upper bound) or the host value.
__device__ inline int64_t count_of(int64_t n_host, const int* n_dev) {
  if (!n_dev) return n_host;
  const int64_t v = *n_dev;
  return v < 0 ? 0 : (v > n_host ? n_host : v);
}

__global__ __launch_bounds__(kSmallBlock) void scan_small(const int* __restrict__ in, int64_t n_host,
                                                           const int* __restrict__ n_dev, int* __restrict__ out,
                                                           int* __restrict__ total_out) {
  __shared__ int lds[kSmallBlock / kWave + 1];
  const int64_t n = count_of(n_host, n_dev);
  int carry = 0;
  for (int64_t base = 0; base < n; base += (int64_t)kSmallBlock * kSmallItems) {
    int v[kSmallItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kSmallItems; ++k) {
      const int64_t i = base + (int64_t)threadIdx.x * kSmallItems + k;
      v[k] = i < n ? in[i] : 0;
      s += v[k];
    }
    int tot;
    int ex = block_excl_scan<kSmallBlock>(s, lds, &tot) + carry;
#pragma unroll
    for (int k = 0; k < kSmallItems; ++k) {
      const int64_t i = base + (int64_t)threadIdx.x * kSmallItems + k;
      if (i < n) out[i] = ex;
      ex += v[k];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

__global__ __launch_bounds__(kScanBlock) void scan_tile_reduce(const int* __restrict__ in, int64_t n_host,
                                                                const int* __restrict__ n_dev,
                                                                int* __restrict__ partial) {
  __shared__ int lds[kScanBlock / kWave + 1];
  const int64_t n = count_of(n_host, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n && blockIdx.x > 0) return;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;
    if (i < n) s += in[i];
  }
  int total;
  block_excl_scan<kScanBlock>(s, lds, &total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Tile scans: each workgroup first sums the tile totals before its own (at
// most a few thousand ints, read from L2), so no separate pass over the tile
// sums is needed; workgroup 0 also writes the grand total.
__global__ __launch_bounds__(kScanBlock) void scan_tiles(const int* __restrict__ in, int64_t n_host,
                                                          const int* __restrict__ n_dev,
                                                          const int* __restrict__ partial, int* __restrict__ out,
                                                          int* __restrict__ total_out) {
  __shared__ int lds[kScanBlock / kWave + 1];
  const int64_t n = count_of(n_host, n_dev);
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  if (base >= n && blockIdx.x > 0) return;
  const int nb = (int)((n + kScanTile - 1) / kScanTile);
  // prefix of this tile (and, for workgroup 0, the total of all tiles)
  const int upto = blockIdx.x == 0 ? nb : (int)blockIdx.x;
  int acc = 0;
  for (int i = threadIdx.x; i < upto; i += kScanBlock) acc += partial[i];
  int sum_upto;
  block_excl_scan<kScanBlock>(acc, lds, &sum_upto);
  const int prefix = blockIdx.x == 0 ? 0 : sum_upto;
  if (blockIdx.x == 0 && threadIdx.x == 0 && total_out) *total_out = sum_upto;
  if (base >= n) return;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    v[k] = i < n ? in[i] : 0;
    s += v[k];
  }
  int tot;
  int ex = block_excl_scan<kScanBlock>(s, lds, &tot) + prefix;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + (int64_t)threadIdx.x * kScanItems + k;
    if (i < n) out[i] = ex;
    ex += v[k];
  }
}

__global__ void k_fill_i32(int* __restrict__ p, int v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

constexpr int kPublishBlock = 256;

// One workgroup: lane i copies src[i] to the host mailbox, then (after a
// system-scope fence and a barrier) lane 0 advances the device counter and
// stores its new value into mail[seq_slot] with release semantics.
__global__ __launch_bounds__(kPublishBlock) void k_publish(const int* __restrict__ src, int count,
                                                           int* __restrict__ ctr, int* mail, int seq_slot) {
  const int i = threadIdx.x;
  if (i < count) mail[i] = src[i];
  __threadfence_system();
  __syncthreads();
  if (i == 0) {
    const int v = *ctr + 1;
    *ctr = v;
    __hip_atomic_store(mail + seq_slot, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
}
}  // namespace

void publish(const int* src, int count, int* ctr, int* mail, int seq_slot, hipStream_t s) {
  if (count < 0 || count > kPublishBlock) count = kPublishBlock;
  k_publish<<<1, kPublishBlock, 0, s>>>(src, count, ctr, mail, seq_slot);
}

void fill_i32(int* p, int v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_fill_i32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, v, n);
}

size_t scan_temp_ints(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

void scan_exclusive_dev(const int* in, int* out, const int* n_dev, int64_t max_n, int* temp, int* total_dev,
                        hipStream_t s) {
  if (max_n <= 0) {
    if (total_dev) fill_i32(total_dev, 0, 1, s);
    return;
  }
  if (max_n <= kSmallMax) {
    scan_small<<<1, kSmallBlock, 0, s>>>(in, max_n, n_dev, out, total_dev);
    return;
  }
  const int nb = (int)((max_n + kScanTile - 1) / kScanTile);
  scan_tile_reduce<<<nb, kScanBlock, 0, s>>>(in, max_n, n_dev, temp);
  scan_tiles<<<nb, kScanBlock, 0, s>>>(in, max_n, n_dev, temp, out, total_dev);
}

void scan_exclusive(const int* in, int* out, int64_t n, int* temp, int* total_dev, hipStream_t s) {
  scan_exclusive_dev(in, out, nullptr, n, temp, total_dev, s);
}

}  // namespace pp
