// Near field (P2P): the direct part of the group superposition, Appendix A,
// eq. greenSum restricted to the source leaves that are not accepted for an
// expansion.  Also serves as the all-pairs direct sum when every source leaf
// is listed for every target leaf.
//
// Work item: one wave per (target leaf, part of its source list); lane j owns
// target j of each 64-target chunk.  Every lane of a wave needs the same
// source at the same time, so sources are read with wave-uniform addresses
// (scalar loads, no LDS staging) and each source costs one pass of ~7 VALU
// instructions over the 64 lanes.
//
// Coordinates are offsets in units of h: sources relative to their own leaf
// corner (exact half-integers for grid nodes), targets relative to their leaf
// corner, shifted per source leaf by the integer corner difference.  This keeps
// FP32 positions accurate to ~1e-6 h however large the grid.  The kernel sums
// w log2(r^2 / h^2); per target and list part it then stores, in FP64, half
// that sum times ln 2 plus ln(h) times the part's near weight W = sum w, which
// is the part's share of sum w ln r.
//
// Mixed precision: FP32 with Kahan-compensated accumulation in a fixed order.
// The pair of a target with a coincident node only occurs inside its own leaf;
// that leaf is processed by a guarded loop where r^2 = 0 contributes 0.
#include <algorithm>

#include "blockscan.h"
#include "internal.h"

namespace pp {

namespace {
constexpr int kP2PWaves = 4;

// Kahan step with the group's partial sum y (which already carries -comp).
__device__ inline void kahan_fold(float y, float& sum, float& comp) {
  const float tt = sum + y;
  comp = (tt - sum) - y;
  sum = tt;
}

__device__ inline float pair_log2(float tx, float ty, float qx, float qy, bool guard) {
  const float dx = tx - qx;
  const float dy = ty - qy;
  float r2 = fmaf(dy, dy, dx * dx);
  if (guard) r2 = (r2 == 0.0f) ? 1.0f : r2;
  return __builtin_amdgcn_logf(r2);  // v_log_f32: log2
}

// Source planes (offsets x, y and weights w of the sorted sources).
struct Planes {
  const float* __restrict__ x;
  const float* __restrict__ y;
  const float* __restrict__ w;
};

// G consecutive sources from s: their terms are summed in order (the first
// product starts from -comp) and the group is folded into the running sum with
// Kahan compensation.
template <int G, bool GUARD>
__device__ inline void p2p32_group(const Planes& q, int s, float tx, float ty, float& sum, float& comp) {
  float qx[G], qy[G], qw[G], l[G];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    qx[i] = q.x[s + i];
    qy[i] = q.y[s + i];
    qw[i] = q.w[s + i];
  }
#pragma unroll
  for (int i = 0; i < G; ++i) l[i] = pair_log2(tx, ty, qx[i], qy[i], GUARD);
  float y = fmaf(qw[0], l[0], -comp);
#pragma unroll
  for (int i = 1; i < G; ++i) y = fmaf(qw[i], l[i], y);
  kahan_fold(y, sum, comp);
}

// Sources [s0, s1) of one leaf against this lane's target: groups of eight
// (3 VALU of compensation per 8 pairs), then the ragged tail as at most one
// group each of four, two and one.
template <bool GUARD>
__device__ inline void p2p32_leaf(const Planes& q, int s0, int s1, float tx, float ty, float& sum, float& comp) {
  int s = s0;
  for (; s + 8 <= s1; s += 8) p2p32_group<8, GUARD>(q, s, tx, ty, sum, comp);
  if (s + 4 <= s1) {
    p2p32_group<4, GUARD>(q, s, tx, ty, sum, comp);
    s += 4;
  }
  if (s + 2 <= s1) {
    p2p32_group<2, GUARD>(q, s, tx, ty, sum, comp);
    s += 2;
  }
  if (s < s1) p2p32_group<1, GUARD>(q, s, tx, ty, sum, comp);
}

// Sparse target leaves (at most kSparseTargets targets, e.g. surface points
// crossing a leaf): one lane per (target, source slot), Q source slots per
// target (Q = 4, 8 or 16 for up to 16, 8 or 4 targets), so that Q times
// more lanes do useful work than with one lane per target.  (Two slots for
// up to 32 targets were measured slower than one lane per target.)  Lane (t, q) takes the
// sources q, q + Q, q + 2Q, ... of every source leaf of its list part, sums
// their terms four at a time in FP32 and folds each group into a Kahan-
// compensated running sum; the Q slots' compensated totals are then added in
// FP64 in a fixed order (a butterfly over the Q lanes).
constexpr int kSparseTargets = 16;

template <bool GUARD>
__device__ inline void p2p32_strided(const Planes& q, int s, int s1, int stride, float tx, float ty, float& sum,
                                     float& comp) {
  for (; s < s1; s += 4 * stride) {
    float y = -comp;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int sj = s + j * stride;
      if (sj < s1) y = fmaf(q.w[sj], pair_log2(tx, ty, q.x[sj], q.y[sj], GUARD), y);
    }
    kahan_fold(y, sum, comp);
  }
}

template <bool DIRECT>
__device__ inline void p2p32_sparse(const P2PArgs& a, const Planes& q, int A, int part, int e0, int e1, const int* lst,
                                    int wid) {
  const TreeView& t = a.t;
  const int lane = threadIdx.x % kWave;
  const int tb = t.tb[A], nt = t.te[A] - tb;
  const int Q = nt <= 4 ? 16 : nt <= 8 ? 8 : 4;
  const int ti = lane / Q, qi = lane % Q;
  const bool active = ti < nt;
  const int k = tb + (active ? ti : 0);
  const int shA = t.D - t.lvl[A];
  const int cax = t.ix[A] << shA, cay = t.iy[A] << shA;
  const float2 r = a.rel32[k];
  float sum = 0.0f, comp = 0.0f;
  double wn = 0.0;
  int64_t nsrc = 0;
  bool bad = false;
  for (int e = e0; e < e1; ++e) {
    const int B = lst[e];
    if ((unsigned)B >= (unsigned)t.ncells) {
      bad = true;
      continue;
    }
    const int shB = t.D - t.lvl[B];
    const float tx = r.x + (float)(cax - (t.ix[B] << shB));
    const float ty = r.y + (float)(cay - (t.iy[B] << shB));
    const int s0 = t.sb[B], s1 = t.se[B];
    nsrc += s1 - s0;
    wn += a.leaf_w[B];
    if (B == A)
      p2p32_strided<true>(q, s0 + qi, s1, Q, tx, ty, sum, comp);
    else
      p2p32_strided<false>(q, s0 + qi, s1, Q, tx, ty, sum, comp);
  }
  double v = (double)sum - (double)comp;
  for (int o = 1; o < Q; o <<= 1) v += __shfl_xor(v, o, kWave);
  if (active && qi == 0) a.near_sum[(int64_t)part * a.m + k] = 0.5 * (v * kLn2) + a.lnh * wn;
  if (lane == 0 && a.pair_counts) a.pair_counts[wid] = (int64_t)nt * nsrc;
  if (bad && lane == 0 && a.flags) atomicOr(a.flags, kFlagBadIndex);
}

// Work: wave w (workgroups spread over the XCDs in contiguous runs, so an
// XCD's L2 holds the sources of a compact region) handles target leaf
// tleaves[w / nparts] and the list part
// w % nparts (entries [part * nb / nparts, (part + 1) * nb / nparts)), looping
// over the leaf's targets 64 at a time.  Partial sums go to
// near_sum[part * m + k] and are added in a fixed order by the finalize step;
// pair_counts[w] receives the number of (target, source) pairs the wave
// evaluated.
// The source planes come in as separate __restrict__ arguments: with no
// possible aliasing the compiler keeps their wave-uniform loads on the scalar
// path although the kernel stores partial sums between chunks.
template <bool DIRECT>
__global__ __launch_bounds__(kP2PWaves* kWave) __attribute__((amdgpu_waves_per_eu(8, 8))) void k_p2p32(
    P2PArgs a, const float* __restrict__ sx, const float* __restrict__ sy, const float* __restrict__ sw) {
  const Planes q{sx, sy, sw};
  // wave-uniform work index (keeps all per-item data in scalar registers)
  const int wid = __builtin_amdgcn_readfirstlane(xcd_contiguous(blockIdx.x, gridDim.x) * kP2PWaves +
                                                    threadIdx.x / kWave);
  if (wid >= a.ntleaves * a.nparts) return;
  const int part = wid % a.nparts;
  const int lane = threadIdx.x % kWave;
  const TreeView& t = a.t;
  const int A = a.tleaves[wid / a.nparts];
  const int shA = t.D - t.lvl[A];
  const int cax = t.ix[A] << shA, cay = t.iy[A] << shA;
  const int nb = DIRECT ? a.nsleaves : a.list_cnt[A];
  const int* lst = DIRECT ? a.sleaves : a.list_src + a.list_off[A];
  const int e0 = (int)((int64_t)part * nb / a.nparts);
  const int e1 = (int)((int64_t)(part + 1) * nb / a.nparts);
  const int tb = t.tb[A], te = t.te[A];
  if (te - tb <= kSparseTargets) {  // wave-uniform
    p2p32_sparse<DIRECT>(a, q, A, part, e0, e1, lst, wid);
    return;
  }
  int64_t pairs = 0;
  bool bad = false;
  for (int chunk = tb; chunk < te; chunk += kWave) {
    const int k = chunk + lane;
    const bool active = k < te;
    const float2 r = active ? a.rel32[k] : make_float2(0.0f, 0.0f);
    float sum = 0.0f, comp = 0.0f;
    double wn = 0.0;
    int64_t nsrc = 0;
    for (int e = e0; e < e1; ++e) {
      const int B = lst[e];
      if ((unsigned)B >= (unsigned)t.ncells) {
        bad = true;
        continue;
      }
      const int shB = t.D - t.lvl[B];
      const float tx = r.x + (float)(cax - (t.ix[B] << shB));
      const float ty = r.y + (float)(cay - (t.iy[B] << shB));
      const int s0 = t.sb[B], s1 = t.se[B];
      nsrc += s1 - s0;
      wn += a.leaf_w[B];
      if (B == A)
        p2p32_leaf<true>(q, s0, s1, tx, ty, sum, comp);
      else
        p2p32_leaf<false>(q, s0, s1, tx, ty, sum, comp);
    }
    if (active) a.near_sum[(int64_t)part * a.m + k] = 0.5 * (((double)sum - (double)comp) * kLn2) + a.lnh * wn;
    pairs += (int64_t)min(kWave, te - chunk) * nsrc;
  }
  if (lane == 0 && a.pair_counts) a.pair_counts[wid] = pairs;
  if (bad && lane == 0 && a.flags) atomicOr(a.flags, kFlagBadIndex);
}

// FP64 near field.  Grid-node targets and grid sources sit at exact
// half-integer offsets, so r^2 is an exact integer there; below kLogTable it
// is looked up in a table of ln n computed on the device with the same log
// (bitwise the same term), any other r^2 calls log.
template <bool GUARD>
__device__ inline void p2p64_leaf(const float* __restrict__ sx, const float* __restrict__ sy,
                                  const double2* __restrict__ s64, const double* __restrict__ w64,
                                  const double* __restrict__ log_tab, int s0, int s1, double tx, double ty,
                                  double& sum) {
#pragma unroll 2
  for (int s = s0; s < s1; ++s) {
    double ox, oy;
    if (s64) {
      const double2 o = s64[s];
      ox = o.x;
      oy = o.y;
    } else {
      ox = (double)sx[s];
      oy = (double)sy[s];
    }
    const double w = w64[s];
    const double dx = tx - ox;
    const double dy = ty - oy;
    const double r2 = fma(dy, dy, dx * dx);
    if (GUARD && r2 == 0.0) continue;
    double lg;
    if (r2 < (double)kLogTable && r2 == floor(r2))
      lg = log_tab[(int)r2];
    else
      lg = log(r2);
    sum = fma(w, lg, sum);
  }
}

__global__ void k_log_table(double* __restrict__ tab) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n < kLogTable) tab[n] = n > 0 ? log((double)n) : 0.0;
}

template <bool DIRECT>
__global__ __launch_bounds__(kP2PWaves* kWave) void k_p2p64(P2PArgs a, const float* __restrict__ sx,
                                                             const float* __restrict__ sy,
                                                             const double2* __restrict__ s64,
                                                             const double* __restrict__ w64,
                                                             const double* __restrict__ log_tab) {
  const int wid = __builtin_amdgcn_readfirstlane(xcd_contiguous(blockIdx.x, gridDim.x) * kP2PWaves +
                                                    threadIdx.x / kWave);
  if (wid >= a.ntleaves * a.nparts) return;
  const int part = wid % a.nparts;
  const int lane = threadIdx.x % kWave;
  const TreeView& t = a.t;
  const int A = a.tleaves[wid / a.nparts];
  const int shA = t.D - t.lvl[A];
  const int cax = t.ix[A] << shA, cay = t.iy[A] << shA;
  const int nb = DIRECT ? a.nsleaves : a.list_cnt[A];
  const int* lst = DIRECT ? a.sleaves : a.list_src + a.list_off[A];
  const int e0 = (int)((int64_t)part * nb / a.nparts);
  const int e1 = (int)((int64_t)(part + 1) * nb / a.nparts);
  const int tb = t.tb[A], te = t.te[A];
  int64_t pairs = 0;
  bool bad = false;
  for (int chunk = tb; chunk < te; chunk += kWave) {
    const int k = chunk + lane;
    const bool active = k < te;
    const double2 r = active ? a.rel64[k] : make_double2(0.0, 0.0);
    double sum = 0.0;
    double wn = 0.0;
    int64_t nsrc = 0;
    for (int e = e0; e < e1; ++e) {
      const int B = lst[e];
      if ((unsigned)B >= (unsigned)t.ncells) {
        bad = true;
        continue;
      }
      const int shB = t.D - t.lvl[B];
      const double tx = r.x + (double)(cax - (t.ix[B] << shB));
      const double ty = r.y + (double)(cay - (t.iy[B] << shB));
      const int s0 = t.sb[B], s1 = t.se[B];
      nsrc += s1 - s0;
      wn += a.leaf_w[B];
      if (B == A)
        p2p64_leaf<true>(sx, sy, s64, w64, log_tab, s0, s1, tx, ty, sum);
      else
        p2p64_leaf<false>(sx, sy, s64, w64, log_tab, s0, s1, tx, ty, sum);
    }
    if (active) a.near_sum[(int64_t)part * a.m + k] = 0.5 * sum + a.lnh * wn;
    pairs += (int64_t)min(kWave, te - chunk) * nsrc;
  }
  if (lane == 0 && a.pair_counts) a.pair_counts[wid] = pairs;
  if (bad && lane == 0 && a.flags) atomicOr(a.flags, kFlagBadIndex);
}

}  // namespace

void log_table(double* tab, hipStream_t s) { k_log_table<<<(kLogTable + 255) / 256, 256, 0, s>>>(tab); }

void p2p(const P2PArgs& a, int fp64, hipStream_t s) {
  const int64_t waves = (int64_t)a.ntleaves * a.nparts;
  if (waves <= 0) return;
  const unsigned g = (unsigned)((waves + kP2PWaves - 1) / kP2PWaves);
  const bool direct = a.list_cnt == nullptr;
  if (fp64) {
    if (direct)
      k_p2p64<true><<<g, kP2PWaves * kWave, 0, s>>>(a, a.sx, a.sy, a.s64, a.w64, a.log_tab);
    else
      k_p2p64<false><<<g, kP2PWaves * kWave, 0, s>>>(a, a.sx, a.sy, a.s64, a.w64, a.log_tab);
  } else {
    if (direct)
      k_p2p32<true><<<g, kP2PWaves * kWave, 0, s>>>(a, a.sx, a.sy, a.sw);
    else
      k_p2p32<false><<<g, kP2PWaves * kWave, 0, s>>>(a, a.sx, a.sy, a.sw);
  }
}

}  // namespace pp
