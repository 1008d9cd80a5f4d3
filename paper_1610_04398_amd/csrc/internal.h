// Host-side launchers of the HIP kernels (one translation unit each) and the
// mutable tree arrays the pipeline owns.  Internal: not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "../../include/pp.h"

namespace pp {

// Several grid requests of one geometry (nx, ny, x0, y0, h and parameters)
// solved as one forest: request r's grid lies in cell r (Morton order) of
// level `levels` of a root 2^levels times as wide, so its sources, targets
// and cells keep their relative positions, keys and order; every cell above
// that level is split, and no interaction crosses from one request's cell to
// another's.  Each request's arithmetic is then that of its lone solve.
constexpr int kMaxBatch = 16;
struct GridBatch {
  int nreq = 0;    // 0: a single solve
  int levels = 0;  // levels above the requests' roots: 4^levels >= nreq
  int D = 0;       // root exponent of one request's grid
  const double* f[kMaxBatch] = {};
  const double* tx[kMaxBatch] = {};
  const double* ty[kMaxBatch] = {};
  double* out[kMaxBatch] = {};
  int64_t toff[kMaxBatch + 1] = {};  // request r's targets are [toff[r], toff[r + 1]) of the joint order
};
// The request of joint target index i.
__host__ __device__ inline int batch_request(const GridBatch& b, int64_t i) {
  int r = 0;
  while (r + 1 < b.nreq && b.toff[r + 1] <= i) ++r;
  return r;
}

// ---- scan.hip: exclusive prefix sums and fills --------------------------------
size_t scan_temp_ints(int64_t n);
// out[i] = sum_{j<i} in[j]; *total_dev = sum of all (may be null). in == out allowed.
// temp holds scan_temp_ints(n) ints.
void scan_exclusive(const int* in, int* out, int64_t n, int* temp, int* total_dev, hipStream_t s);
// Same with the count read from device memory (*n_dev, clamped to max_n).
void scan_exclusive_dev(const int* in, int* out, const int* n_dev, int64_t max_n, int* temp, int* total_dev,
                        hipStream_t s);
void fill_i32(int* p, int v, int64_t n, hipStream_t s);
// Copies src[0..count) (count <= 256) into host-visible coherent memory `mail`,
// then increments the device counter *ctr and stores its new value into
// mail[seq_slot] after a system-scope fence: the host spins on that slot
// instead of synchronising the stream.
void publish(const int* src, int count, int* ctr, int* mail, int seq_slot, hipStream_t s);
// Whether the context runs the near field on a second stream beside the
// expansions (on by default; the server turns it off when it runs several slots).
void ctx_set_near_stream(pp_ctx* c, bool on);
// Device bytes the context's buffers hold, and releasing all of them (the
// next solve allocates again).
size_t ctx_held_bytes(const pp_ctx* c);
void ctx_trim(pp_ctx* c);

// ---- ingest.hip: sources in Morton order, target keys ------------------------------
// Morton tiles of 2048 indices (64 x 32 nodes) cover [0, 4^k).
int64_t ingest_num_tiles(int k);
// Ints of the tile-count buffer: per tile the nonzero count of the tiles before
// it in its group, then one total per group.
int64_t ingest_count_ints(int k);
// First pass: tile counts (tile_cnt: ingest_count_ints(k) ints; no clearing needed).
// bt (may be null): a forest of requests (f is then unused; k is the forest's
// root exponent).
void ingest_grid_count(const double* f, int nx, int ny, int k, int* tile_cnt, int* flags, const GridBatch* bt,
                       hipStream_t s);
// Second pass: the sources in Morton order (packed node index ij = i | j << 16
// in the forest's index space, w = f h^2) and *total_out = their count; a
// source's key is the Morton index of (i, j) (keys_from_ij).  starts (may be
// null): the source range start of every Morton prefix of 2 * sh bits (cells
// of the dense table sh levels above the finest).
void ingest_grid_emit(const double* f, int nx, int ny, int k, double h2, const int* tile_cnt, int* total_out,
                      uint32_t* ij, double* w64, int* starts, int sh, const GridBatch* bt, hipStream_t s);
// key[i] = Morton index of source i's node (from ij), i < *n_dev (n_dev may be
// null: n sources); n bounds *n_dev.
void keys_from_ij(const uint32_t* ij, const int* n_dev, int64_t n, uint32_t* key, hipStream_t s);
// Resident solves (the tree of the last solve kept, new f on the same grid):
// w = f h^2 of the n retained sources (node indices ij, tile counts tile_cnt
// of the retained solve), in one pass over f; kFlagStale when a node outside
// them is nonzero (retained nodes may have become zero).
void resident_weights(const double* f, int nx, int ny, int k, double h2, const int* tile_cnt, const uint32_t* ij,
                      int64_t n, double* w64, int* flags, hipStream_t s);
// kFlagStale unless every target (caller index perm[q]) still has the sorted key key[q].
void resident_targets(const double* tx, const double* ty, int64_t m, const int* perm, const uint32_t* key, double x0,
                      double y0, double h, int k, int* flags, hipStream_t s);
void target_keys(const double* tx, const double* ty, int64_t m, double x0, double y0, double h, int k,
                 uint32_t* key, int* idx, int* flags, hipStream_t s);

// ---- points.hip: scattered sources -----------------------------------------------
// Finest level of the root for scattered input: keys use 2 * 15 bits, so the
// key of a zero-weight source (0xFFFFFFFF) sorts after every cell key.
constexpr int kPointsDepth = 15;
int points_box_blocks(int64_t n_total);
// box[0..3] = xmin, xmax, ymin, ymax of the weighted sources and the targets;
// *nsrc = number of sources with w != 0.  part/cnt: points_box_blocks entries.
void points_box(const double* sx, const double* sy, const double* w, int64_t n, const double* tx, const double* ty,
                int64_t m, double4* part, int* cnt, double* box, int* nsrc, int* flags, hipStream_t s);
void points_keys(const double* sx, const double* sy, const double* w, int64_t n, double x0, double y0, double u,
                 int D, uint32_t* key, int* idx, hipStream_t s);
// Sorted copies of the first *nsrc_dev sources in the order perm.
void points_gather(const int* perm, const int* nsrc_dev, int64_t nmax, const double* sx, const double* sy,
                   const double* w, double* xs, double* ys, double* ws, hipStream_t s);

// ---- sort.hip: stable LSD radix sort of (uint32 key, int32 value) pairs -----------
size_t radix_temp_ints(int64_t n);
// Sorts the low `bits` bits of keys; results end in (keys, vals).  tmp arrays of n.
void radix_sort_pairs(uint32_t* keys, int* vals, uint32_t* keys_tmp, int* vals_tmp, int64_t n, int bits,
                      int* temp, hipStream_t s);
// Target keys (as target_keys) sorted with their indices (as radix_sort_pairs
// over 2k bits); the first pass computes the keys while it counts digits.
// bt (may be null): the joint targets of a forest (tx, ty and k unused).
void target_keys_sorted(const double* tx, const double* ty, int64_t m, double x0, double y0, double h, int k,
                        uint32_t* keys, int* vals, uint32_t* keys_tmp, int* vals_tmp, int* temp, int* flags,
                        const GridBatch* bt, hipStream_t s);

struct LeafPass;  // leafpass.h: per-leaf passes that ride on the list launch (lp may be null)
// ---- tree.hip: top-down construction, per-leaf packing ------------------------------
struct TreeArrays {
  int* lvl;
  int* ix;
  int* iy;
  int* sb;
  int* se;
  int* tb;
  int* te;
  int* child;
  int* nchild;
  int* parent;
};
// Levels 0..Ld of the tree in one pass over a dense table of Morton prefixes
// (4^Ld + 1 range starts per key array, tree_dense_cells(Ld) flags); writes
// ls[0..D+1] on the device (the levels below Ld empty), and level Ld's cells
// are left as leaves for tree_level to continue from, which is needed only
// when *deep becomes nonzero (a cell of level Ld holds more than leaf_max
// sources or targets).  Gives the same cells and numbering as building the
// levels one at a time from the root.  src_done: ss[0..4^Ld) was written by
// the grid ingest.  Cells of the levels above split_above are split whatever
// they hold (a forest's top levels; split_above <= Ld).
int64_t tree_dense_cells(int Ld);
// ints of scan_tmp that tree_dense_top needs (per-workgroup counts of the flags)
int64_t tree_dense_part_ints(int Ld);
void tree_dense_top(TreeArrays t, int* ls, int D, int Ld, int leaf_max, int split_above, int cap,
                    const uint32_t* skey, const int* nsrc_dev, int src_done, const uint32_t* tkey, int ntgt, int* ss,
                    int* ts, int* flag, int* off, int* scan_tmp, int* total_slot, int* deep, int* flags,
                    hipStream_t s);
// One level of the top-down construction, with no host round trip: the level's
// cells are [ls[level], ls[level+1]) read on the device; its children are
// appended and ls[level+2] is written.  max_cells bounds the level's size (grid
// and scan sizing), cap the total cell count (overflow raises a flag).
void tree_level(TreeArrays t, int* ls, int level, int D, int leaf_max, int64_t max_cells, int cap,
                const uint32_t* skey, const uint32_t* tkey, int* sp, int4* cr, int* exists, int* off, int* scan_tmp,
                int* n4_slot, int* total_slot, int* flags, hipStream_t s);
// Compacted cell lists: source leaves, target leaves, cells with targets, for
// the *ncells_dev cells of the tree (cap = allocated cells; flag3/off3 scratch
// of 3 * cap); counts[0..2] receive their lengths.
// part: classify_part_ints(cap) ints of scratch.  counts[0..2]: the three list lengths.
// rec (may be null): the same launch also sets up every cell for the lists
// (cell_setup; rec->t's arrays are the tree's, its ncells unused).
int64_t classify_part_ints(int64_t cap);
void classify_cells(TreeArrays t, const int* ncells_dev, int cap, int* part, int* sleaves, int* tleaves,
                    int* tcells, int* counts, const RecordArgs* rec, hipStream_t s);
// One launch for two independent per-leaf passes.
// Per source leaf: FP32 source records relative to the leaf corner, in finest
// cell units, as three planes (x at s32[s], y at s32[stride + s], w at
// s32[2 stride + s]), and the FP64 leaf weight.
// Per target leaf: offsets relative to the leaf corner (FP32 and FP64, in units
// of h), owning leaf, and for the self rule the weight f h^2 of the node the
// target coincides with (0 if none) and ln of its distance to it (-inf on it).
// A target at squared distance d2 from its nearest node with d2 == 0 or
// d2 < snap_frac2 h^2 is snapped onto the node (its exact term is restored by
// the finalize step); FP32 near fields use snap_frac2 = 2^-40, FP64 ones 0.
void leaf_pack_prep(TreeArrays t, int D, const int* sleaves, int nsleaves, const uint32_t* ij, const double* w64,
                    float* s32, int64_t stride, double* leaf_w, const int* tleaves, int ntleaves, const double* tx,
                    const double* ty, const int* perm, double x0, double y0, double h, int nx, int ny,
                    double snap_frac2, const double* f, float2* rel32, double2* rel64, int* tleaf, double* self_w,
                    double* self_logd, const GridBatch* bt, hipStream_t s);
// Scattered-source counterpart, in one launch: FP32 records and FP64 offsets
// (units of u) per source leaf; per target leaf the offsets, owning leaf, and
// the weight of the sources that coincide exactly with the target.
void leaf_pack_prep_points(TreeArrays t, int D, double x0, double y0, double u, const double* xs, const double* ys,
                           const double* ws, const int* sleaves, int nsleaves, float* s32, int64_t stride,
                           double2* s64, double* leaf_w, const int* tleaves, int ntleaves, const double* tx,
                           const double* ty, const int* perm, float2* rel32, double2* rel64, int* tleaf,
                           double* self_w, hipStream_t s);

// ---- lists.hip: dual-tree interaction lists ------------------------------------
// One wave per target cell in `tcells`; pass 0 counts into cnt_m2l / cnt_p2p
// (indexed by cell id), pass 1 writes the lists at off_m2l / off_p2p (by cell id).
// Lists of the tree-code variant, per target leaf (indexed by cell id): the
// source cells whose multipoles are evaluated at the leaf's targets (M2P) and
// the source leaves summed directly (P2P).  Same emit modes as lists_pass.
void lists_treecode_pass(TreeView t, const int4* rec, const int* tleaves, int ntleaves, int num, int den, int emit,
                         int* cnt_m, int* cnt_p, const int* off_m, const int* off_p, int* m_src, int* p_src, int cap_m,
                         int cap_p, int* flags, int tier_boost, const struct LeafPass* lp, hipStream_t s);
// emit 0: counts only; 1: write at the exact offsets of a count pass;
// 2: one pass, counts plus lists at cell * cap (kFlagListOverflow if a list
// is longer than its capacity; its tail is then dropped).  top > 0: a forest
// whose requests' roots are at level top (the walk of a target cell starts
// at its request's root; cells above that level get empty lists).
void lists_pass(TreeView t, const int4* rec, const int* tcells, int ntcells, int num, int den, int emit, int* cnt_m2l,
                int* cnt_p2p, const int* off_m2l, const int* off_p2p, int* m2l_src, int* p2p_src, int cap_m, int cap_p,
                int* flags, int tier_boost, int top, const struct LeafPass* lp, hipStream_t s);
// The traversal frontier has three capacity tiers chosen from theta; tier_boost
// raises it after an overflow.  True when no higher tier is left.
bool frontier_at_top(int num, int den, int tier_boost);
// ---- expand.hip: multipole and local passes (FP64) ---------------------------------
// P2M of every source leaf (16 lanes per leaf), from the ordered sources: grid
// nodes by their packed index ij (i | j << 16), or (ij null) scattered sources
// by their coordinates xs, ys in a root square anchored at (x0, y0) with
// finest cell side u.
void p2m(TreeView t, const int* sleaves, int n, const uint32_t* ij, const double* xs, const double* ys, double x0,
         double y0, double u, const double* w64, int p, double2* mp, int64_t lattice_min, hipStream_t s);
// M2M for the `levels` (1..m2m_max_levels()) levels starting at the level
// whose cells are [c0, c1): one workgroup per cell computes its subtree
// bottom up.
// L is the level of [c0, c1); dense_flag/dense_off/dense_levels describe the dense
// prefix table of the tree build (its top dense_levels levels), used to find the
// subtree cells directly when the launch lies inside it (may be null).
int m2m_max_levels();
void m2m_levels(TreeView t, int c0, int c1, int L, int levels, int p, double2* mp, const int* dense_flag,
                const int* dense_off, int dense_levels, hipStream_t s);
void m2l(TreeView t, const int* tcells, int n, const int* m2l_off, const int* m2l_cnt, const int* m2l_src, int p,
         double h, const double2* mp, double2* loc, int* flags, hipStream_t s);
// List parts per target leaf in the tree-code's M2P (more, shorter waves than
// one per leaf: the leaves with the longest lists no longer set the time).
constexpr int kM2PParts = 4;
// Largest number of near-field list parts per target leaf.
constexpr int kMaxNearParts = 8;
// M2P of the tree-code variant: the far field of every target of the n target
// leaves from the multipoles of their M2P lists (off/cnt by cell id), each list
// split into nparts parts whose partial sums go to far[part * m + k] (m
// targets); fp32 != 0 evaluates in FP32.
void m2p(TreeView t, const int* tleaves, int n, const int* off, const int* cnt, const int* src, int p, double h,
         const double2* mp, const double2* rel64, int fp32, int nparts, int64_t m, double* far, int* flags,
         hipStream_t s);
// Final local expansion of every cell with targets from its own M2L local
// (`own`) and its ancestors' (exact L2L shifts), one launch.
// dense_off/dense_levels: the cell numbers of the tree build's dense prefix
// table (levels 0..dense_levels), where ancestors are looked up directly.
// top: the first ancestor level with interactions (a forest's request roots; 0 otherwise).
void downward(TreeView t, const int* tcells, int n, int p, const double2* own, double2* loc, const int* dense_off,
              int dense_levels, int top, hipStream_t s);
// far[k] = Re sum_l c'_l u^l for every sorted target k (u: offset from its
// leaf centre over the leaf side); fp32 != 0 evaluates in FP32.
void l2p(TreeView t, int64_t m, const int* tleaf, int p, const double2* loc, const double2* rel64, int fp32,
         double* far, hipStream_t s);

// ---- p2p.hip: near field --------------------------------------------------------------
struct P2PArgs {
  TreeView t;
  const int* tleaves;   // target leaves (work: one wave per leaf and list part)
  int ntleaves;
  const int* list_off;  // per cell id: P2P list begin
  const int* list_cnt;  // and length; null => all source leaves (direct mode)
  const int* list_src;  // source leaf ids
  const int* sleaves;   // all source leaves (direct mode)
  int nsleaves;
  // FP32 source records as three planes of the sorted sources: offsets from the
  // leaf corner (x, y, units of the finest cell) and weights
  const float* sx;
  const float* sy;
  const float* sw;
  const double2* s64;   // FP64 source offsets for the FP64 kernel (null: those of sx, sy, exact for grid nodes)
  const double* w64;
  const double* leaf_w;
  const float2* rel32;
  const double2* rel64;
  int nparts;           // each target chunk's list is split over nparts waves
  int64_t m;            // number of targets
  long long* pair_counts;     // per wave: (target, source) pairs evaluated (may be null)
  int* flags;                 // error flags (kFlagBadIndex for a list entry outside the tree)
  unsigned long long* pairs;  // if set with pair_counts, receives their sum
  double lnh;           // ln of the grid spacing (the unit of the offsets)
  const double* log_tab;  // FP64 kernel: kLogTable values of ln n (log_table)
  double* near_sum;     // [nparts][m]: per sorted target, sum w ln(r) over the part's near sources
};
void p2p(const P2PArgs& a, int fp64, hipStream_t s);
// ln n for n in [1, kLogTable) (tab[0] = 0), for the FP64 near field.
constexpr int kLogTable = 4096;
void log_table(double* tab, hipStream_t s);

// ---- finalize.hip ----------------------------------------------------------------------
// P at every target, scattered to the caller's order; writes nothing if *flags != 0.
// near_sum holds nparts partial sums (stride m).
// Statistics summed by the finalize launch into zeroed slots: the per-wave pair
// counts (pair_counts[0..nwaves) into *pairs, if pairs is set) and the per-cell list
// lengths (cnt_m/cnt_p[0..ncells) into *tot_m/*tot_p, if cnt_m is set).
struct FinalizeTotals {
  const long long* pair_counts = nullptr;
  int64_t nwaves = 0;
  unsigned long long* pairs = nullptr;
  const int* cnt_m = nullptr;
  const int* cnt_p = nullptr;
  int64_t ncells = 0;
  int* tot_m = nullptr;
  int* tot_p = nullptr;
};
// The far field evaluated inside the finalize launch (L2P, as l2p) when loc is
// set; it is then written to far (if not null) rather than read from it.
// Otherwise far holds far_parts partial sums per target (far[q * m + k]),
// added here and the total written back to far[k].
struct FarEval {
  const double2* loc = nullptr;
  const double2* rel64 = nullptr;
  const int* tleaf = nullptr;
  const int* lvl = nullptr;
  int D = 0, p = 0, fp32 = 0;
  int far_parts = 1;
};
// self_w (may be null): per target the weight of the source it coincides with
// (grid node or scattered sources), 0 for none; self_logd (may be null: exact
// coincidence throughout) the log of the distance to that node, -inf if exact.
void finalize(int64_t m, int nparts, const int* perm, double* far, const double* near_sum,
              const double* self_w, const double* self_logd, double h, int self_mode, const int* flags, double* out,
              const FinalizeTotals& tot, const FarEval& fe, const GridBatch* bt, hipStream_t s);

// ---- forces.hip: pressure forces on surfaces -----------------------------------------
// One workgroup per segment seg[s]..seg[s+1] (device array of nseg + 1); dfx/dfy may be null.
void surface_forces(const double* p, const double* nx, const double* ny, const double* ds, int nseg,
                    const int64_t* seg, double ux, double uy, double rho, double area, double* dfx, double* dfy,
                    pp_force* out, hipStream_t s);

// ---- assembly.hip: source from the gridded velocity, viscous forces -------------------
// f at every node of the nx x ny grid (eq. PoissonFinal); chi/us/vs null: no penalisation term.
void pressure_source(const double* u, const double* v, const double* chi, const double* us, const double* vs, int nx,
                     int ny, double h, double rho, double lam, double* f, int* flags, hipStream_t s);
// Viscous forces per panel and per segment (eq. Fvisc, FviscNet, CdNu) from nearest-node gradients.
void viscous_forces(const double* u, const double* v, int nx, int ny, double x0, double y0, double h, const double* lx,
                    const double* ly, const double* pnx, const double* pny, const double* ds, int nseg,
                    const int64_t* seg, double mu, double uxi, double uyi, double rho, double area, double* dfx,
                    double* dfy, pp_force* out, hipStream_t s);

}  // namespace pp
