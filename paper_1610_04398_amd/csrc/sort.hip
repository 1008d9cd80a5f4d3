// Stable LSD radix sort of (uint32 Morton key, int32 index) pairs, 8-bit
// digits.  Used to order the targets along the quadtree's Morton curve; ties
// keep their input order, so the permutation is unique.
//
// Per digit pass: per-tile digit histograms -> one device-wide exclusive scan
// of the digit-major histogram table -> stable scatter.  Within a tile the
// scatter ranks keys round by round (256 keys per round, in thread order),
// matching equal digits across a wave with eight ballots.
#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {
constexpr int kRsBlock = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsBlock * kRsItems;
constexpr int kRsWaves = kRsBlock / kWave;

__global__ __launch_bounds__(kRsBlock) void k_radix_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                          int nblocks, int* __restrict__ hist) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kRsTile;
  for (int q = 0; q < kRsItems; ++q) {
    const int i = base + q * kRsBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFF], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kRsBlock) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                             const int* __restrict__ vin, int n, int shift, int nblocks,
                                                             const int* __restrict__ off, uint32_t* __restrict__ kout,
                                                             int* __restrict__ vout) {
  __shared__ int goff[256];
  __shared__ int run[256];
  __shared__ int wcnt[kRsWaves][256];
  const int t = threadIdx.x;
  const int lane = t % kWave;
  const int w = t / kWave;
  goff[t] = off[t * nblocks + blockIdx.x];
  run[t] = 0;
  for (int ww = 0; ww < kRsWaves; ++ww) wcnt[ww][t] = 0;
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
  const int base = blockIdx.x * kRsTile;
  for (int q = 0; q < kRsItems; ++q) {
    const int i = base + q * kRsBlock + t;
    const bool valid = i < n;
    uint32_t key = 0;
    int val = 0;
    if (valid) {
      key = kin[i];
      val = vin[i];
    }
    const int d = (key >> shift) & 0xFF;
    // lanes holding the same digit (valid lanes only)
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt_mask);
    const bool leader = valid && (peers & lt_mask) == 0;
    if (leader) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pre = 0;
      for (int ww = 0; ww < w; ++ww) pre += wcnt[ww][d];
      const int pos = goff[d] + run[d] + pre + rank;
      kout[pos] = key;
      vout[pos] = val;
    }
    __syncthreads();
    int add = 0;
    for (int ww = 0; ww < kRsWaves; ++ww) {
      add += wcnt[ww][t];
      wcnt[ww][t] = 0;
    }
    run[t] += add;
    __syncthreads();
  }
}

__global__ void k_copy_pairs(const uint32_t* __restrict__ ks, const int* __restrict__ vs, int n,
                             uint32_t* __restrict__ kd, int* __restrict__ vd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    kd[i] = ks[i];
    vd[i] = vs[i];
  }
}
}  // namespace

size_t radix_temp_ints(int64_t n) {
  const int64_t nb = (n + kRsTile - 1) / kRsTile;
  const int64_t table = 256 * nb;
  return (size_t)(table + scan_temp_ints(table) + 1);
}

void radix_sort_pairs(uint32_t* keys, int* vals, uint32_t* keys_tmp, int* vals_tmp, int64_t n, int bits, int* temp,
                      hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  const int nb = (int)((n + kRsTile - 1) / kRsTile);
  int* table = temp;
  int* scan_tmp = temp + 256 * (int64_t)nb;
  uint32_t* ka = keys;
  int* va = vals;
  uint32_t* kb = keys_tmp;
  int* vb = vals_tmp;
  const int passes = (bits + 7) / 8;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = 8 * ps;
    k_radix_hist<<<nb, kRsBlock, 0, s>>>(ka, (int)n, shift, nb, table);
    scan_exclusive(table, table, 256 * (int64_t)nb, scan_tmp, nullptr, s);
    k_radix_scatter<<<nb, kRsBlock, 0, s>>>(ka, va, (int)n, shift, nb, table, kb, vb);
    uint32_t* tk = ka;
    ka = kb;
    kb = tk;
    int* tv = va;
    va = vb;
    vb = tv;
  }
  if (ka != keys) k_copy_pairs<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ka, va, (int)n, keys, vals);
}

}  // namespace pp
