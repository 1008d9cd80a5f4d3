// Stable LSD radix sort of (uint32 Morton key, int32 index) pairs with digits
// of up to 9 bits (the 18-bit keys of a 512^2 root take two passes).  Used to
// order the targets along the quadtree's Morton curve; ties keep their input
// order, so the permutation is unique.
//
// Per digit pass: per-tile digit histograms -> one device-wide exclusive scan
// of the digit-major histogram table -> stable scatter (for at most 64 tiles
// the scatter's workgroups form their offsets from the table themselves, and
// the scan launch is skipped).  Within a tile the
// scatter ranks keys round by round (256 keys per round, in thread order),
// matching equal digits across a wave with one ballot per digit bit.
#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {
constexpr int kRsBlock = 256;
constexpr int kRsItems = 4;  // 1024-key tiles: enough workgroups to fill the GPU at ~2.6e5 keys
constexpr int kRsTile = kRsBlock * kRsItems;
constexpr int kRsWaves = kRsBlock / kWave;
constexpr int kRsMaxBits = 9;

template <int BITS>
__global__ __launch_bounds__(kRsBlock) void k_radix_hist(const uint32_t* __restrict__ keys, int n, int shift,
                                                          int nblocks, int* __restrict__ hist) {
  constexpr int BINS = 1 << BITS;
  __shared__ int h[BINS];
  for (int b = threadIdx.x; b < BINS; b += kRsBlock) h[b] = 0;
  __syncthreads();
  const int base = blockIdx.x * kRsTile;
  // the tile's keys are all requested before the first count
  uint32_t kv[kRsItems];
#pragma unroll
  for (int q = 0; q < kRsItems; ++q) {
    const int i = base + q * kRsBlock + threadIdx.x;
    kv[q] = i < n ? keys[i] : 0u;
  }
  // (an empty statement that takes the keys keeps the compiler from moving a
  // load down into the branch of its count)
#pragma unroll
  for (int q = 0; q < kRsItems; ++q) asm volatile("" : "+v"(kv[q]));
#pragma unroll
  for (int q = 0; q < kRsItems; ++q)
    if (base + q * kRsBlock + (int)threadIdx.x < n) atomicAdd(&h[(kv[q] >> shift) & (BINS - 1)], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < BINS; b += kRsBlock) hist[b * nblocks + blockIdx.x] = h[b];
}

// The first pass's histogram fused with the computation of the target keys
// (finest-cell Morton keys, see target_key): each workgroup computes and stores
// the keys and indices of its tile and counts their lowest digit.
// bt.nreq > 0: the targets of a forest of requests, joint index i is target
// i - toff[r] of request r, whose key is prefixed by r (its cell of the
// forest's top levels; k is then one request's root exponent).
template <int BITS>
__global__ __launch_bounds__(kRsBlock) void k_keys_hist(const double* __restrict__ tx, const double* __restrict__ ty,
                                                        int n, double x0, double y0, double h, int k, int nblocks,
                                                        uint32_t* __restrict__ keys, int* __restrict__ vals,
                                                        int* __restrict__ hist, int* __restrict__ flags,
                                                        GridBatch bt) {
  constexpr int BINS = 1 << BITS;
  __shared__ int hs[BINS];
  for (int b = threadIdx.x; b < BINS; b += kRsBlock) hs[b] = 0;
  __syncthreads();
  const int base = blockIdx.x * kRsTile;
  int errs = 0;
  for (int q = 0; q < kRsItems; ++q) {
    const int i = base + q * kRsBlock + threadIdx.x;
    if (i < n) {
      int err = 0;
      uint32_t key;
      if (bt.nreq) {
        const int r = batch_request(bt, i);
        const int64_t j = i - bt.toff[r];
        key = ((uint32_t)r << (2 * k)) | target_key(bt.tx[r][j], bt.ty[r][j], x0, y0, h, k, &err);
      } else {
        key = target_key(tx[i], ty[i], x0, y0, h, k, &err);
      }
      errs |= err;
      keys[i] = key;
      vals[i] = i;
      atomicAdd(&hs[key & (BINS - 1)], 1);
    }
  }
  if (errs & 1) atomicOr(flags, kFlagNonFiniteTarget);
  if (errs & 2) atomicOr(flags, kFlagTargetOutside);
  __syncthreads();
  for (int b = threadIdx.x; b < BINS; b += kRsBlock) hist[b * nblocks + blockIdx.x] = hs[b];
}

// FOLD: `off` holds the raw per-tile digit counts (digit-major) instead of
// their exclusive scan, and each workgroup forms its own offsets from them:
// the totals of all smaller digits plus the counts of its digit in the tiles
// before it.  For few tiles (at most kRsFoldTiles) this replaces the scan
// launch between the histogram and the scatter.
constexpr int kRsFoldTiles = 64;

template <int BITS, bool FOLD>
__global__ __launch_bounds__(kRsBlock) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                             const int* __restrict__ vin, int n, int shift, int nblocks,
                                                             const int* __restrict__ off, uint32_t* __restrict__ kout,
                                                             int* __restrict__ vout) {
  constexpr int BINS = 1 << BITS;
  constexpr int PER = (BINS + kRsBlock - 1) / kRsBlock;  // digits per thread
  __shared__ int goff[BINS];
  __shared__ int run[BINS];
  __shared__ int wcnt[kRsWaves][BINS];
  __shared__ int lds[kRsWaves + 1];
  const int t = threadIdx.x;
  const int lane = t % kWave;
  const int w = t / kWave;
  // the tile's keys and values, loaded before anything waits on them
  const int base = blockIdx.x * kRsTile;
  uint32_t kq[kRsItems];
  int vq[kRsItems];
#pragma unroll
  for (int q = 0; q < kRsItems; ++q) {
    const int i = base + q * kRsBlock + t;
    kq[q] = i < n ? kin[i] : 0u;
    vq[q] = i < n ? vin[i] : 0;
  }
  if (FOLD) {
    // thread t owns digits [t PER, t PER + PER)
    int tot[PER], pre[PER], sum = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int b = t * PER + q;
      tot[q] = pre[q] = 0;
      if (b < BINS) {
        // 16 loads in flight at a time (clamped indices, no branch around them)
        for (int b0 = 0; b0 < nblocks; b0 += 16) {
          int c[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) c[u] = off[b * nblocks + min(b0 + u, nblocks - 1)];
#pragma unroll
          for (int u = 0; u < 16; ++u) {
            const int blk = b0 + u;
            tot[q] += blk < nblocks ? c[u] : 0;
            pre[q] += blk < (int)blockIdx.x ? c[u] : 0;
          }
        }
      }
      sum += tot[q];
    }
    int all;
    int base = block_excl_scan<kRsBlock>(sum, lds, &all);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int b = t * PER + q;
      if (b < BINS) goff[b] = base + pre[q];
      base += tot[q];
    }
  } else {
    for (int b = t; b < BINS; b += kRsBlock) goff[b] = off[b * nblocks + blockIdx.x];
  }
  for (int b = t; b < BINS; b += kRsBlock) {
    run[b] = 0;
    for (int ww = 0; ww < kRsWaves; ++ww) wcnt[ww][b] = 0;
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
#pragma unroll
  for (int q = 0; q < kRsItems; ++q) {
    const int i = base + q * kRsBlock + t;
    const bool valid = i < n;
    const uint32_t key = kq[q];
    const int val = vq[q];
    const int d = (key >> shift) & (BINS - 1);
    // lanes holding the same digit (valid lanes only), in lane order
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
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
    for (int b = t; b < BINS; b += kRsBlock) {
      int add = 0;
      for (int ww = 0; ww < kRsWaves; ++ww) {
        add += wcnt[ww][b];
        wcnt[ww][b] = 0;
      }
      run[b] += add;
    }
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

// The target coordinates when the first pass also computes the keys.
struct KeySource {
  const double* tx = nullptr;
  const double* ty = nullptr;
  double x0 = 0.0, y0 = 0.0, h = 1.0;
  int k = 0;
  int* flags = nullptr;
  GridBatch bt{};
};

template <int BITS>
void radix_pass(uint32_t* ka, int* va, uint32_t* kb, int* vb, int n, int shift, int nb, int* table, int* scan_tmp,
                const KeySource* ks, hipStream_t s) {
  if (ks)
    k_keys_hist<BITS><<<nb, kRsBlock, 0, s>>>(ks->tx, ks->ty, n, ks->x0, ks->y0, ks->h, ks->k, nb, ka, va, table,
                                              ks->flags, ks->bt);
  else
    k_radix_hist<BITS><<<nb, kRsBlock, 0, s>>>(ka, n, shift, nb, table);
  if (nb <= kRsFoldTiles) {
    k_radix_scatter<BITS, true><<<nb, kRsBlock, 0, s>>>(ka, va, n, shift, nb, table, kb, vb);
  } else {
    scan_exclusive(table, table, (int64_t)(1 << BITS) * nb, scan_tmp, nullptr, s);
    k_radix_scatter<BITS, false><<<nb, kRsBlock, 0, s>>>(ka, va, n, shift, nb, table, kb, vb);
  }
}

void sort_impl(uint32_t* keys, int* vals, uint32_t* keys_tmp, int* vals_tmp, int64_t n, int bits, int* temp,
               const KeySource* ks, hipStream_t s) {
  const int nb = (int)((n + kRsTile - 1) / kRsTile);
  int* table = temp;
  int* scan_tmp = temp + (1 << kRsMaxBits) * (int64_t)nb;
  const int passes = (bits + kRsMaxBits - 1) / kRsMaxBits;
  const int width = (bits + passes - 1) / passes;
  // keys computed by the first pass start in the buffer from which an odd
  // number of passes ends in the result buffers (no final copy)
  const bool start_tmp = ks && (passes & 1);
  uint32_t* ka = start_tmp ? keys_tmp : keys;
  int* va = start_tmp ? vals_tmp : vals;
  uint32_t* kb = start_tmp ? keys : keys_tmp;
  int* vb = start_tmp ? vals : vals_tmp;
  for (int ps = 0; ps < passes; ++ps) {
    const int shift = width * ps;
    const KeySource* kp = ps == 0 ? ks : nullptr;
    switch (width) {
      case 1: radix_pass<1>(ka, va, kb, vb, (int)n, shift, nb, table, scan_tmp, kp, s); break;
      case 2: radix_pass<2>(ka, va, kb, vb, (int)n, shift, nb, table, scan_tmp, kp, s); break;
      case 3: radix_pass<3>(ka, va, kb, vb, (int)n, shift, nb, table, scan_tmp, kp, s); break;
      case 4: radix_pass<4>(ka, va, kb, vb, (int)n, shift, nb, table, scan_tmp, kp, s); break;
      case 5: radix_pass<5>(ka, va, kb, vb, (int)n, shift, nb, table, scan_tmp, kp, s); break;
      case 6: radix_pass<6>(ka, va, kb, vb, (int)n, shift, nb, table, scan_tmp, kp, s); break;
      case 7: radix_pass<7>(ka, va, kb, vb, (int)n, shift, nb, table, scan_tmp, kp, s); break;
      case 8: radix_pass<8>(ka, va, kb, vb, (int)n, shift, nb, table, scan_tmp, kp, s); break;
      default: radix_pass<9>(ka, va, kb, vb, (int)n, shift, nb, table, scan_tmp, kp, s); break;
    }
    uint32_t* tk = ka;
    ka = kb;
    kb = tk;
    int* tv = va;
    va = vb;
    vb = tv;
  }
  if (ka != keys) k_copy_pairs<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(ka, va, (int)n, keys, vals);
}
}  // namespace

size_t radix_temp_ints(int64_t n) {
  const int64_t nb = (n + kRsTile - 1) / kRsTile;
  const int64_t table = (1 << kRsMaxBits) * nb;
  return (size_t)(table + scan_temp_ints(table) + 1);
}

// Digits of up to 9 bits: the fewest passes that cover `bits`, equal widths.
void radix_sort_pairs(uint32_t* keys, int* vals, uint32_t* keys_tmp, int* vals_tmp, int64_t n, int bits, int* temp,
                      hipStream_t s) {
  if (n <= 1 || bits <= 0) return;
  sort_impl(keys, vals, keys_tmp, vals_tmp, n, bits, temp, nullptr, s);
}

void target_keys_sorted(const double* tx, const double* ty, int64_t m, double x0, double y0, double h, int k,
                        uint32_t* keys, int* vals, uint32_t* keys_tmp, int* vals_tmp, int* temp, int* flags,
                        const GridBatch* bt, hipStream_t s) {
  if (m <= 0) return;
  if (bt && bt->nreq) {  // keys of one request's root prefixed by the request's forest cell
    KeySource ks;
    ks.x0 = x0;
    ks.y0 = y0;
    ks.h = h;
    ks.k = bt->D;
    ks.flags = flags;
    ks.bt = *bt;
    sort_impl(keys, vals, keys_tmp, vals_tmp, m, 2 * (bt->D + bt->levels), temp, &ks, s);
    return;
  }
  if (m == 1 || k <= 0) {
    target_keys(tx, ty, m, x0, y0, h, k, keys, vals, flags, s);
    return;
  }
  KeySource ks;
  ks.tx = tx;
  ks.ty = ty;
  ks.x0 = x0;
  ks.y0 = y0;
  ks.h = h;
  ks.k = k;
  ks.flags = flags;
  sort_impl(keys, vals, keys_tmp, vals_tmp, m, 2 * k, temp, &ks, s);
}

}  // namespace pp
