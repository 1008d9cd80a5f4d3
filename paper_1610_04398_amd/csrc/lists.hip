// Interaction lists of the dual-tree traversal.
//
// The paper sums group contributions, treating a group through its expansion
// once it is far enough away and the rest directly (Appendix A, the
// superposition equation after Fig. multipole).  The traversal read here pairs
// a target cell A with a source cell B starting from the roots: accepted by
// the exact integer test -> M2L; both leaves -> P2P; A leaf -> split B; B leaf
// -> split A; otherwise split both.  Only cells with sources are used as
// sources and only cells with targets as targets.
//
// GPU form: one wave per target cell A walks the traversal restricted to A's
// ancestor path.  The pairs (X, B) with X the current path cell form a
// frontier of source cells kept in LDS; the 64 lanes classify 64 candidates at
// a time and compact what they emit with ballots, so each cell's lists come out
// in a fixed order without atomics.  Down to A the frontier advances one level
// at a time; at A itself it becomes a stack popped 64 cells at a time, so that a
// target leaf much larger than the source cells beside it (whose breadth-first
// frontier would hold every source cell of a level near it) needs only about
// 3 x 64 entries per level below A.  A count pass sizes the lists, an emit pass
// writes them.
#include <algorithm>
#include <climits>

#include "blockscan.h"
#include "internal.h"
#include "leafpass.h"

namespace pp {

namespace {
constexpr int kListWaves = 4;
// Frontier capacity per wave (two level buffers, or one stack of twice the
// size at the target cell), in three tiers.  The frontier of a target cell holds
// the non-accepted source cells near its path, ~4 (2/theta + 1)^2 in a uniform
// tree (about 100 at theta = 0.5).  Tier 0 (256 entries, 8 KB of LDS per
// workgroup, so LDS no longer limits the waves per CU) serves theta >= 0.5;
// tier 1 (1024) theta >= 0.3; tier 2 (2048) smaller theta.  Overflow is flagged
// and the solve repeats at the next tier.
constexpr int kFrontierTiers[3] = {256, 1024, 2048};
int frontier_tier_for(int num, int den) {
  if (2 * num >= den) return 0;       // theta >= 0.5
  if (num * 10 >= 3 * den) return 1;  // theta >= 0.3
  return 2;
}

// Packed per-cell record for the traversal: {ix, iy, first child, meta} with
// meta = level | nchild << 5 | (children-with-sources mask) << 8 | has_src << 12.
__device__ inline int rec_level(int4 r) { return r.w & 31; }
__device__ inline int rec_nchild(int4 r) { return (r.w >> 5) & 7; }
__device__ inline int rec_kidmask(int4 r) { return (r.w >> 8) & 15; }
__device__ inline bool rec_has_src(int4 r) { return (r.w >> 12) & 1; }

// The traversal at the target cell A itself, from the source cells left on the
// stack st[0, top): accepted -> A's far list (M2L, or M2P for the tree-code);
// not accepted and a leaf -> A's near list when A is a leaf; not accepted and
// not a leaf -> its children with sources pushed when A is a leaf (for a
// non-leaf A the rest belongs to A's children).  Pops the top 64 entries at a
// time.  Returns true when the stack would exceed `cap` (the lists are then
// incomplete).
template <bool kTreecode>
__device__ bool lists_at_target(int* st, int top, int cap, int D, int4 rA, bool leafA, int num, int den,
                                const int4* __restrict__ rec, int emit, int* __restrict__ m_src, int64_t mbase,
                                int mlim, int* __restrict__ p_src, int64_t pbase, int plim, int& nm, int& np,
                                int lane, uint64_t lt_mask) {
  const int lA = rec_level(rA);
  while (top > 0) {
    const int n = min(kWave, top);
    const bool valid = lane < n;
    const int B = valid ? st[top - n + lane] : 0;
    top -= n;
    __syncwarp();  // the popped slots take this round's pushes
    bool acc = false, leafB = false;
    int kid0 = 0, kmask = 0;
    if (valid) {
      const int4 rB = rec[B];
      acc = kTreecode ? treecode_accept(D, lA, rA.x, rA.y, rec_level(rB), rB.x, rB.y, num, den)
                      : mac_accept(D, lA, rA.x, rA.y, rec_level(rB), rB.x, rB.y, num, den);
      kid0 = rB.z;
      leafB = kid0 < 0;
      kmask = rec_kidmask(rB);
    }
    const bool em = valid && acc;
    const bool ep = valid && !acc && leafB && leafA;
    const bool push = valid && !acc && !leafB && leafA;
    const uint64_t bm = __ballot(em);
    const uint64_t bp = __ballot(ep);
    if (emit) {
      const int im = nm + __popcll(bm & lt_mask), ip = np + __popcll(bp & lt_mask);
      if (em && im < mlim) m_src[mbase + im] = B;
      if (ep && ip < plim) p_src[pbase + ip] = B;
    }
    nm += __popcll(bm);
    np += __popcll(bp);
    const int npush = push ? __popc(kmask) : 0;
    const int incl = wave_incl_scan(npush);
    const int total = __shfl(incl, kWave - 1, kWave);
    if (top + total > cap) return true;
    if (push) {
      int pos = top + incl - npush;
      for (int q = 0; q < 4; ++q)
        if ((kmask >> q) & 1) st[pos++] = kid0 + q;
    }
    top += total;
    __syncwarp();
  }
  return false;
}

template <int kFrontierCap, bool kLeafPass>
__global__ __launch_bounds__(kListWaves * kWave) void k_lists(int D, const int4* __restrict__ rec,
                                                               const int* __restrict__ parent,
                                                               const int* __restrict__ tcells, int ntcells, int num,
                                                               int den, int emit, int* __restrict__ cnt_m2l,
                                                               int* __restrict__ cnt_p2p,
                                                               const int* __restrict__ off_m2l,
                                                               const int* __restrict__ off_p2p,
                                                               int* __restrict__ m2l_src, int* __restrict__ p2p_src,
                                                               int cap_m, int cap_p, int* __restrict__ flags,
                                                               int top, LeafPass lp) {
  __shared__ int front[kListWaves][2 * kFrontierCap];
  __shared__ int path[kListWaves][kMaxDepth + 1];
  if constexpr (kLeafPass) {  // the per-leaf passes riding on this launch
    const int list_blocks = (ntcells + kListWaves - 1) / kListWaves;
    if ((int)blockIdx.x >= list_blocks) {
      run_leaf_pass(lp, (int)blockIdx.x - list_blocks);
      return;
    }
  }
  const int w = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * kListWaves + w);
  if (wid >= ntcells) return;
  const int A = tcells[wid];
  const int4 rA = rec[A];
  const int lA = rec_level(rA);
  if (lane == 0) {
    int c = A;
    for (int l = lA; l >= 0; --l) {
      path[w][l] = c;
      c = parent[c];
    }
  }
  const bool leafA = rA.z < 0;
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
  int* const buf = front[w];
  int* cur = buf;
  int* nxt = buf + kFrontierCap;
  int ncur = 0;
  // top > 0 (a forest of requests): the walk starts at A's ancestor of level
  // top, its request's root, and cells above that level have no lists
  __syncwarp();
  const int R0 = lA >= top ? path[w][top] : -1;
  if (R0 >= 0 && rec_has_src(rec[R0])) {
    if (lane == 0) cur[0] = R0;
    ncur = 1;
  }
  __syncwarp();
  // emit 1: exact offsets from a count pass; emit 2: fixed capacity per cell
  const int64_t mbase = emit == 1 ? off_m2l[A] : (int64_t)A * cap_m;
  const int64_t pbase = emit == 1 ? off_p2p[A] : (int64_t)A * cap_p;
  const int mlim = emit == 2 ? cap_m : INT_MAX;
  const int plim = emit == 2 ? cap_p : INT_MAX;
  bool overflow = false;
  // Down the path: X (level xl) is a proper ancestor of A, so not a leaf, and a
  // pair accepted here belongs to X's lists.  A source leaf that is not
  // accepted stays for the next level, any other source cell is replaced by its
  // children with sources.
  for (int xl = top; xl < lA && ncur > 0; ++xl) {
    const int4 rX = rec[path[w][xl]];
    int nnext = 0;
    for (int base = 0; base < ncur; base += kWave) {
      const int i = base + lane;
      const bool valid = i < ncur;
      const int B = valid ? cur[i] : 0;
      bool keep = false, leafB = false;
      int kid0 = 0, kmask = 0;
      if (valid) {
        const int4 rB = rec[B];
        keep = !mac_accept(D, xl, rX.x, rX.y, rec_level(rB), rB.x, rB.y, num, den);
        kid0 = rB.z;
        leafB = kid0 < 0;
        kmask = rec_kidmask(rB);
      }
      const int npush = keep ? (leafB ? 1 : __popc(kmask)) : 0;
      const int incl = wave_incl_scan(npush);
      const int total = __shfl(incl, kWave - 1, kWave);
      int pos = nnext + incl - npush;
      if (nnext + total > kFrontierCap) {
        overflow = true;
      } else {
        if (keep && leafB) nxt[pos] = B;
        if (keep && !leafB) {
          for (int q = 0; q < 4; ++q)
            if ((kmask >> q) & 1) nxt[pos++] = kid0 + q;
        }
        nnext += total;
      }
    }
    __syncwarp();
    if (overflow) break;
    int* tmp = cur;
    cur = nxt;
    nxt = tmp;
    ncur = nnext;
  }
  int nm = 0, np = 0;
  if (!overflow && ncur > 0) {
    if (cur != buf) {  // the stack starts at the bottom of the buffer (no overlap: ncur <= kFrontierCap)
      for (int i = lane; i < ncur; i += kWave) buf[i] = cur[i];
      __syncwarp();
    }
    overflow = lists_at_target<false>(buf, ncur, 2 * kFrontierCap, D, rA, leafA, num, den, rec, emit, m2l_src,
                                      mbase, mlim, p2p_src, pbase, plim, nm, np, lane, lt_mask);
  }
  if (overflow && lane == 0) atomicOr(flags, kFlagFrontierOverflow);
  if (emit == 2 && (nm > cap_m || np > cap_p) && lane == 0) atomicOr(flags, kFlagListOverflow);
  if (emit != 1 && lane == 0) {
    // in the capacity layout a list never reaches past its cell's slots: an
    // overflowing list is cut at the capacity (and flagged for an exact re-run),
    // so the kernels that read it stay inside the allocation
    cnt_m2l[A] = emit == 2 ? min(nm, cap_m) : nm;
    cnt_p2p[A] = emit == 2 ? min(np, cap_p) : np;
  }
}

// Lists of the paper's tree-code: one wave per target leaf A walks the source
// tree from the root.  A source cell accepted for all of A's targets goes to
// A's M2P list; a leaf that is not accepted goes to its P2P list; any other
// cell is replaced by its children with sources.  The cells still to visit
// form a stack in LDS, popped and classified 64 at a time; ballots compact the
// output in a fixed order.  Same emit modes and layouts as k_lists.
template <int kFrontierCap, bool kLeafPass>
__global__ __launch_bounds__(kListWaves * kWave) void k_lists_treecode(
    int D, const int4* __restrict__ rec, const int* __restrict__ tleaves, int ntleaves, int num, int den, int emit,
    int* __restrict__ cnt_m, int* __restrict__ cnt_p, const int* __restrict__ off_m, const int* __restrict__ off_p,
    int* __restrict__ m_src, int* __restrict__ p_src, int cap_m, int cap_p, int* __restrict__ flags, LeafPass lp) {
  __shared__ int front[kListWaves][2 * kFrontierCap];
  if constexpr (kLeafPass) {  // the per-leaf passes riding on this launch
    const int list_blocks = (ntleaves + kListWaves - 1) / kListWaves;
    if ((int)blockIdx.x >= list_blocks) {
      run_leaf_pass(lp, (int)blockIdx.x - list_blocks);
      return;
    }
  }
  const int w = threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * kListWaves + w);
  if (wid >= ntleaves) return;
  const int A = tleaves[wid];
  const int4 rA = rec[A];
  const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (kWave - lane));
  int* const buf = front[w];
  int top = 0;
  if (rec_has_src(rec[0])) {
    if (lane == 0) buf[0] = 0;
    top = 1;
  }
  __syncwarp();
  int nm = 0, np = 0;
  const int64_t mbase = emit == 1 ? off_m[A] : (int64_t)A * cap_m;
  const int64_t pbase = emit == 1 ? off_p[A] : (int64_t)A * cap_p;
  const int mlim = emit == 2 ? cap_m : INT_MAX;
  const int plim = emit == 2 ? cap_p : INT_MAX;
  const bool overflow = lists_at_target<true>(buf, top, 2 * kFrontierCap, D, rA, true, num, den, rec, emit, m_src,
                                              mbase, mlim, p_src, pbase, plim, nm, np, lane, lt_mask);
  if (overflow && lane == 0) atomicOr(flags, kFlagFrontierOverflow);
  if (emit == 2 && (nm > cap_m || np > cap_p) && lane == 0) atomicOr(flags, kFlagListOverflow);
  if (emit != 1 && lane == 0) {
    cnt_m[A] = emit == 2 ? min(nm, cap_m) : nm;
    cnt_p[A] = emit == 2 ? min(np, cap_p) : np;
  }
}

}  // namespace

#define PP_LIST_TIER(tier, LP, KERNEL, G, S, ...)                                      \
  do {                                                                                 \
    if ((tier) <= 0 && (LP))                                                           \
      KERNEL<kFrontierTiers[0], true><<<G, kListWaves * kWave, 0, S>>>(__VA_ARGS__);   \
    else if ((tier) <= 0)                                                              \
      KERNEL<kFrontierTiers[0], false><<<G, kListWaves * kWave, 0, S>>>(__VA_ARGS__);  \
    else if ((tier) == 1 && (LP))                                                      \
      KERNEL<kFrontierTiers[1], true><<<G, kListWaves * kWave, 0, S>>>(__VA_ARGS__);   \
    else if ((tier) == 1)                                                              \
      KERNEL<kFrontierTiers[1], false><<<G, kListWaves * kWave, 0, S>>>(__VA_ARGS__);  \
    else if (LP)                                                                       \
      KERNEL<kFrontierTiers[2], true><<<G, kListWaves * kWave, 0, S>>>(__VA_ARGS__);   \
    else                                                                               \
      KERNEL<kFrontierTiers[2], false><<<G, kListWaves * kWave, 0, S>>>(__VA_ARGS__);  \
  } while (0)

void lists_pass(TreeView t, const int4* rec, const int* tcells, int ntcells, int num, int den, int emit, int* cnt_m2l,
                int* cnt_p2p, const int* off_m2l, const int* off_p2p, int* m2l_src, int* p2p_src, int cap_m, int cap_p,
                int* flags, int tier_boost, int top, const LeafPass* lp, hipStream_t s) {
  const int nlist = std::max(ntcells, 0);
  const int extra = lp ? lp->pack_blocks + lp->prep_blocks : 0;
  const unsigned g = (unsigned)((nlist + kListWaves - 1) / kListWaves + extra);
  if (g == 0) return;
  const int tier = std::min(2, frontier_tier_for(num, den) + tier_boost);
  PP_LIST_TIER(tier, lp != nullptr, k_lists, g, s, t.D, rec, t.parent, tcells, nlist, num, den, emit, cnt_m2l, cnt_p2p, off_m2l,
               off_p2p, m2l_src, p2p_src, cap_m, cap_p, flags, top, lp ? *lp : LeafPass{});
}

void lists_treecode_pass(TreeView t, const int4* rec, const int* tleaves, int ntleaves, int num, int den, int emit,
                         int* cnt_m, int* cnt_p, const int* off_m, const int* off_p, int* m_src, int* p_src, int cap_m,
                         int cap_p, int* flags, int tier_boost, const LeafPass* lp, hipStream_t s) {
  const int nlist = std::max(ntleaves, 0);
  const int extra = lp ? lp->pack_blocks + lp->prep_blocks : 0;
  const unsigned g = (unsigned)((nlist + kListWaves - 1) / kListWaves + extra);
  if (g == 0) return;
  const int tier = std::min(2, frontier_tier_for(num, den) + tier_boost);
  PP_LIST_TIER(tier, lp != nullptr, k_lists_treecode, g, s, t.D, rec, tleaves, nlist, num, den, emit, cnt_m, cnt_p, off_m, off_p,
               m_src, p_src, cap_m, cap_p, flags, lp ? *lp : LeafPass{});
}

bool frontier_at_top(int num, int den, int tier_boost) { return frontier_tier_for(num, den) + tier_boost >= 2; }

}  // namespace pp
