// Host pipeline and C ABI of the pressure-Poisson tree-code library.
//
// One solve (eq. greenSum of Appendix A evaluated with a quadtree):
//   ingest (w = f h^2, Morton order) -> target keys + radix sort -> tree levels
//   -> cell lists -> interaction lists -> P2M -> M2M (levels up) -> M2L ->
//   L2L (levels down) -> L2P -> P2P -> finalize (1/2pi, self rule, caller order).
// Every step runs on the GPU; the host only sizes buffers from counts the
// kernels produce (a few small read-backs per solve) and sequences launches on
// the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/pp.h"
#include "internal.h"
#include "leafpass.h"

using namespace pp;

// Device memory of the allocation-free solve (pp_solve_grid_noalloc): one
// array per GPU, alive while the library is loaded.  Host code never uses its
// name as an address: the device address comes from hipGetSymbolAddress, once
// per device (scratch_address below).
constexpr size_t kScratchBytes = (size_t)256 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

struct PPError {
  pp_status code;
  std::string msg;
};
// Thrown once the traversal frontier overflowed below its largest tier: the tier
// has been raised and the solve is repeated (nothing was written to the output).
struct FrontierRetry {};

#define HIPCHK(x)                                                                             \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess) throw PPError{PP_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
  } while (0)

enum BufId {
  B_F, B_TX, B_TY, B_OUT, B_MISC, B_TILE, B_SCAN, B_SKEY, B_SIJ, B_SW, B_SRC4, B_TKEY, B_TPERM, B_TKEY2,
  B_TPERM2, B_SORT, B_LVL, B_IX, B_IY, B_SB, B_SE, B_TB, B_TE, B_CHILD, B_NCHILD, B_PARENT, B_CNT, B_OFF, B_CR,
  B_FLAG, B_SLEAF, B_TLEAF, B_TCELL, B_M2MC, B_L2LC, B_CM2L, B_OM2L, B_CP2P, B_OP2P, B_M2LSRC, B_P2PSRC,
  B_CHCNT, B_CHOFF, B_ITEMS, B_LEAFW, B_REL32, B_REL64, B_TGTLEAF, B_SELFD, B_MP, B_LOC, B_FAR, B_NEAR, B_OWNLOC, B_SPLIT, B_REC, B_PCOUNT,
  B_DSS, B_DTS, B_DFLAG, B_DOFF, B_PSX, B_PSY, B_PW, B_PXS, B_PYS, B_PWS, B_SPERM2, B_SKEY2, B_BOXP, B_BOXC,
  B_S64, B_SELFW, B_FP, B_FNX, B_FNY, B_FDS, B_FSEG, B_FDFX, B_FDFY, B_FOUT,
  B_AU, B_AV, B_ACHI, B_AUS, B_AVS, B_AF, B_VLX, B_VLY, B_LOGT, B_CLAIM,
  B_COUNT
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// The address of `scratch` on each device, looked up once per device with
// that device current (each GPU holds its own copy at its own address).
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

void* scratch_address(int device) {
  if (device < 0 || device >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

// Metadata of the last successful solve (for pp_debug_copy).
struct Last {
  bool valid = false;
  int64_t n_src = 0, m = 0;
  int ncells = 0, p = 0;
  int64_t n_m2l = 0, n_p2p = 0;
  bool has_expansions = false;
  bool has_locals = false;
  int nparts = 1;
  bool arena = false;  // its arrays are pieces of the workspace (pp_solve_grid_noalloc)
  bool keys_from_ij = false;  // grid sources: the source keys are formed from the node indices on request
};

// The tree of the last successful grid solve, kept for resident solves
// (new f on the same grid, targets in the same finest cells): everything the
// second segment is sized from.  Its device arrays are the context's buffers.
struct Resident {
  bool valid = false;
  int32_t nx = 0, ny = 0;
  double x0 = 0.0, y0 = 0.0, h = 0.0;
  int64_t m = 0;
  pp_params prm{};
  bool exact_lists = false;
  int cap_far = 0, cap_near = 0, frontier_boost = 0;
  int64_t N = 0, n_m2l = 0, n_p2pl = 0;
  std::vector<int> lstart;
  int nsl = 0, ntl = 0, ntc = 0;
};

constexpr int kMiscInts = 128;
constexpr int kMailExtra = 32;
constexpr int kSeqSlot = kMiscInts;
// misc layout: [0] flags, [1] source count, [2] scratch total, [3] level work items,
// [4..8] cell-list and interaction-list totals, [12] levels below the dense
// table needed, [16..17] near-field pair count (u64),
// [32..32+D+2] level starts of the tree, [96..103] bounding box of scattered input (4 doubles).
constexpr int M_FLAGS = 0, M_NSRC = 1, M_TOT = 2, M_N4 = 3, M_NSL = 4, M_NTL = 5, M_NTC = 6, M_NM2L = 7,
              M_NP2P = 8, M_DEEP = 12, M_PAIRS = 16, M_LS = 32,
              M_BOX = 96;

}  // namespace

struct pp_ctx {
  int device = 0;
  int p2p_parts = 5;  // near-field list split per target leaf (PP_P2P_PARTS overrides, 1..8)
  int cap_m2l = 128;  // per-cell list capacities of the one-pass lists (doubled on overflow)
  int cap_p2p = 64;
  int cap_m2p = 512;  // the same for the tree-code variant's per-leaf lists
  int cap_tp2p = 96;
  bool exact_lists = false;  // PP_EXACT_LISTS=1 forces the two-pass lists
  // untimed calls issue the second segment directly, as the timed ones do,
  // instead of replaying it from a graph (PP_DIRECT_ISSUE=0 replays it)
  int direct_issue = 1;
  int dense_levels = 9;      // levels built from the dense prefix table (PP_DENSE_LEVELS overrides, 0..9)
  // in the directly issued schedule, pack only the source leaves some near-field list holds (PP_LAZY_PACK=0:
  // every source leaf)
  bool lazy_pack = true;
  bool resident_graph = false;  // PP_RESIDENT_GRAPH=1: a resident solve replayed as one graph
  // P2M of grid sources on the matrix cores from this many source leaves up
  // (PP_P2M_LATTICE; 0: never).  With few leaves its long workgroups (64
  // leaves each, 51 KB of LDS) leave most of the chip idle and crowd the list
  // launch beside them: at 512^2 (4,300 leaves) P2M took 17.7 µs against 10.8
  // for the lane groups and the solve was 4-12 % slower.
  int64_t p2m_lattice_min = 32768;
  int profiling = 0;  // 0 off, 1 every phase, 2 the near-field launch only, 16 + phase that phase's launches
  hipEvent_t ev[13] = {};
  // launch replay: each of the two segments of a solve (up to the tree read-back, and
  // from the lists to the end) is captured into a HIP graph on the second call with
  // the same inputs and replayed while they stay the same (PP_GRAPHS=0 disables)
  bool graphs = true;
  uint64_t gen = 0;  // bumped by every device (re)allocation; part of every graph key
  uint64_t res_gen = 0;  // bumped whenever a solve keeps its tree for resident solves
  // work of calls on the null stream runs on this blocking stream (ordered with the
  // null stream like the null stream itself), which can be captured
  hipStream_t own_stream = nullptr;
  // the near field runs on this second stream (default priority, non-blocking)
  // while the expansions run on the caller's stream; fork and join are events
  // (PP_NEAR_STREAM=0 keeps it on the caller's stream after the expansions)
  bool near_stream = true;
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_lists = nullptr, ev_join = nullptr;
  struct Segment {
    std::vector<uint64_t> key;
    int seen = 0;
    hipGraphExec_t exec = nullptr;
    uint64_t used = 0;  // last use (a counter), to pick the slot to replace
  };
  // 0: up to the tree read-back; 1: the rest (not replayed in timing mode 2);
  // 2..5: whole resident solves, one per set of input and output buffers (a
  // caller that alternates between buffers replays a graph for each)
  static constexpr int kResidentSlots = 4;
  static constexpr int kSegments = 2 + kResidentSlots;
  Segment seg[kSegments];
  uint64_t seg_clock = 0;
  uint64_t budget = 0;
  size_t held = 0;
  DevBuf bufs[B_COUNT];
  // Planning pass: ensure() records the bytes each buffer needs instead of
  // allocating, so that a call can check its footprint against the budget
  // before it allocates or enqueues anything.
  bool planning = false;
  size_t plan_need[B_COUNT] = {};
  // Workspace mode (pp_solve_grid_noalloc): ensure() hands out 256-byte
  // aligned pieces of the device's scratch array instead of allocating; the
  // pieces of one call are laid out from its start, in the order asked for.
  bool arena = false;
  char* arena_base = nullptr;
  size_t arena_used = 0;
  DevBuf abufs[B_COUNT];
  void* scratch_ptr = nullptr;  // this device's scratch array (looked up at creation)
  // kMiscInts + kMailExtra ints of coherent pinned host memory for read-backs;
  // slot kSeqSlot receives the sequence number of the last published read-back
  int* pinned = nullptr;
  int* pub_ctr = nullptr;      // device counter of published read-backs
  double* log_tab = nullptr;  // ln n table of the FP64 near field, filled at its first use
  int frontier_boost = 0;     // traversal frontier tiers above theta's own (raised after an overflow)
  hipStream_t cur_stream = nullptr;  // the running call's stream (drained after a failure)
  std::string err;
  bool dead = false;
  Last last;
  Resident res;
  pp_stats stats{};
};

namespace {

void release(pp_ctx& c, int id) {
  DevBuf& b = c.bufs[id];
  if (b.p) {
    (void)hipFree(b.p);
    c.held -= b.bytes;
  }
  b = DevBuf{};
}

template <class T>
T* ensure(pp_ctx& c, int id, int64_t count) {
  const size_t bytes = (size_t)std::max<int64_t>(count, 1) * sizeof(T);
  if (c.planning) {
    c.plan_need[id] = std::max(c.plan_need[id], bytes);
    return (T*)(uintptr_t)256;  // never dereferenced: nothing is enqueued while planning
  }
  if (c.arena) {
    DevBuf& a = c.abufs[id];
    if (a.bytes >= bytes) return (T*)a.p;
    const size_t start = (c.arena_used + 255) & ~(size_t)255;
    if (start + bytes > kScratchBytes)
      throw PPError{PP_ERR_NOMEM, "the solve needs more than the " + std::to_string(kScratchBytes >> 20) +
                                      " MiB of the allocation-free workspace"};
    a.p = c.arena_base + start;
    a.bytes = bytes;
    c.arena_used = start + bytes;
    return (T*)a.p;
  }
  DevBuf& b = c.bufs[id];
  if (b.bytes >= bytes) return (T*)b.p;
  const size_t others = c.held - b.bytes;
  size_t want = c.budget ? bytes : bytes + bytes / 4;  // headroom only without a budget
  if (c.budget && others + want > c.budget)
    throw PPError{PP_ERR_NOMEM, "device-memory budget exceeded (" + std::to_string(others + want) + " > " +
                                    std::to_string(c.budget) + " bytes)"};
  release(c, id);
  c.gen += 1;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, want);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) {
    (void)hipGetLastError();
    throw PPError{PP_ERR_NOMEM, "hipMalloc of " + std::to_string(want) + " bytes failed"};
  }
  HIPCHK(e);
  b.p = p;
  b.bytes = want;
  c.held += want;
  return (T*)p;
}

// Runs `alloc` (a block of ensure() calls with no other effect) once as a
// plan, checks that the buffers it asks for fit the context's budget together
// with everything else the context holds (PP_ERR_NOMEM before anything is
// allocated or enqueued), then runs it for real.  While a budget is set, the
// buffers of a planned block get no growth headroom, so the check is exact.
template <class F>
void reserve(pp_ctx& c, F&& alloc) {
  if (c.arena) {
    // workspace mode: the pieces this block asks for must fit after those
    // already handed out in this call
    std::fill(std::begin(c.plan_need), std::end(c.plan_need), (size_t)0);
    c.planning = true;
    try {
      alloc();
    } catch (...) {
      c.planning = false;
      throw;
    }
    c.planning = false;
    size_t total = c.arena_used;
    for (int i = 0; i < B_COUNT; ++i)
      if (c.plan_need[i] > c.abufs[i].bytes) total = ((total + 255) & ~(size_t)255) + c.plan_need[i];
    if (total > kScratchBytes)
      throw PPError{PP_ERR_NOMEM, "the solve needs " + std::to_string(total) + " bytes of workspace, more than the " +
                                      std::to_string(kScratchBytes >> 20) + " MiB of the allocation-free entry point"};
    alloc();
    return;
  }
  if (!c.budget) {
    alloc();
    return;
  }
  std::fill(std::begin(c.plan_need), std::end(c.plan_need), (size_t)0);
  c.planning = true;
  try {
    alloc();
  } catch (...) {
    c.planning = false;
    throw;
  }
  c.planning = false;
  size_t total = 0;
  for (int i = 0; i < B_COUNT; ++i) total += std::max(c.bufs[i].bytes, c.plan_need[i]);
  if (total > c.budget)
    throw PPError{PP_ERR_NOMEM, "the solve needs " + std::to_string(total) + " bytes of device memory, more than the "
                                "context's budget of " + std::to_string(c.budget) + " bytes"};
  alloc();
}

bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  std::memset(&a, 0, sizeof(a));
  const hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

template <class T>
const T* stage_in(pp_ctx& c, int id, const T* src, int64_t n, hipStream_t s) {
  if (n <= 0 || is_device_ptr(src)) return src;
  T* d = ensure<T>(c, id, n);
  HIPCHK(hipMemcpyAsync(d, src, (size_t)n * sizeof(T), hipMemcpyHostToDevice, s));
  return d;
}

void readback_enqueue(pp_ctx& c, const int* dev, int first, int count, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(c.pinned + first, dev + first, (size_t)count * sizeof(int), hipMemcpyDeviceToHost, s));
}

// Read-back of misc[0..count) at the end of a segment: a kernel writes the
// values into the coherent pinned buffer and then a sequence number, and the
// host spins on that number (a few microseconds sooner than a stream
// synchronisation).  published_seq() before the segment is enqueued gives the
// number to wait for (one more); every earlier read-back has been waited for.
int published_seq(const pp_ctx& c) { return __atomic_load_n(c.pinned + kSeqSlot, __ATOMIC_ACQUIRE); }

void publish_enqueue(pp_ctx& c, const int* misc, int count, hipStream_t s) {
  publish(misc, count, c.pub_ctr, c.pinned, kSeqSlot, s);
}

// Spins until read-back `expect` has arrived.  After 20 ms it also asks the
// stream every 2 ms (rarely: a query takes the runtime's locks, which other
// threads launching work need): an error is reported, and a stream that
// finished without the number arriving is a device error, so the wait always
// ends when the stream does.
void wait_published(pp_ctx& c, hipStream_t s, int expect) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  auto next = t0 + std::chrono::milliseconds(20);
  for (uint64_t n = 1;; ++n) {
    if (published_seq(c) == expect) return;
    if ((n & 255) == 0 && clk::now() >= next) {
      next = clk::now() + std::chrono::milliseconds(2);
      const hipError_t e = hipStreamQuery(s);
      if (e == hipErrorNotReady) continue;
      HIPCHK(e);
      if (published_seq(c) == expect) return;
      throw PPError{PP_ERR_DEVICE, "a read-back did not arrive"};
    }
    __builtin_ia32_pause();
  }
}

void readback(pp_ctx& c, const int* dev, int first, int count, hipStream_t s) {
  readback_enqueue(c, dev, first, count, s);
  HIPCHK(hipStreamSynchronize(s));
}

void drop_graph(pp_ctx::Segment& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  g.exec = nullptr;
}

uint64_t bits(double v) {
  uint64_t u;
  std::memcpy(&u, &v, sizeof(u));
  return u;
}

uint64_t bits(const void* p) { return (uint64_t)(uintptr_t)p; }

// Enqueues one segment of a solve on s: `enqueue` only enqueues device work (every
// buffer it touches was sized before).  Eager the first time a key is seen; on the
// second call with the same key the work is captured into a graph, which is then
// launched, and later calls with that key only launch the graph.  Any failure to
// capture or instantiate falls back to eager launches for the rest of the context.
template <class F>
void run_segment(pp_ctx& c, int which, bool allowed, std::vector<uint64_t> key, hipStream_t s, F&& enqueue) {
  if (which < 0 || which >= pp_ctx::kSegments) throw PPError{PP_ERR_LIMIT, "bad graph segment"};
  pp_ctx::Segment& g = c.seg[which];
  if (!allowed || !c.graphs || s == nullptr) {
    enqueue();
    return;
  }
  key.push_back(c.gen);
  if (g.key != key) {
    drop_graph(g);
    g.key = key;
    g.seen = 0;
  }
  if (g.exec) {
    HIPCHK(hipGraphLaunch(g.exec, s));
    return;
  }
  if (g.seen++ == 0) {
    enqueue();
    return;
  }
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    c.graphs = false;
    enqueue();
    return;
  }
  bool ok = true;
  try {
    enqueue();
  } catch (const PPError&) {
    ok = false;
  }
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &graph);
  if (!ok || e != hipSuccess || !graph || c.gen != key.back() ||
      hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    // nothing captured ran: disable replay and do the work eagerly
    (void)hipGetLastError();
    if (graph) (void)hipGraphDestroy(graph);
    drop_graph(g);
    c.graphs = false;
    enqueue();
    return;
  }
  (void)hipGraphDestroy(graph);
  HIPCHK(hipGraphLaunch(g.exec, s));
}

// The resident-solve graph slot for key (with the allocation generation
// appended, as run_segment keys it): the slot that holds it, else the one
// used least recently.
int resident_slot(pp_ctx& c, std::vector<uint64_t> key) {
  key.push_back(c.gen);
  int pick = 2;
  for (int i = 2; i < pp_ctx::kSegments; ++i) {
    if (c.seg[i].key == key) {
      pick = i;
      break;
    }
    if (c.seg[i].used < c.seg[pick].used) pick = i;
  }
  c.seg[pick].used = ++c.seg_clock;
  return pick;
}

int root_exponent(int nx, int ny) {
  int n = std::max(nx, ny), k = 0;
  while ((1 << k) < n) ++k;
  return k;
}

void check_flags(int flags) {
  if (flags & (kFlagNonFiniteSource | kFlagNonFiniteTarget))
    throw PPError{PP_ERR_ARG, "non-finite source value or target coordinate"};
  if (flags & kFlagTargetOutside) throw PPError{PP_ERR_DOMAIN, "a target lies outside the root square"};
  if (flags & kFlagFrontierOverflow) throw PPError{PP_ERR_LIMIT, "traversal frontier exceeded its capacity"};
  if (flags & kFlagCellOverflow) throw PPError{PP_ERR_LIMIT, "cell capacity exceeded"};
  if (flags & kFlagBadIndex) throw PPError{PP_ERR_LIMIT, "internal index check failed"};
  if (flags & kFlagStale)
    throw PPError{PP_ERR_ARG, "the retained tree does not fit: f is nonzero at a node that was zero when the tree "
                              "was built, or a target left its finest cell"};
  if (flags) throw PPError{PP_ERR_DEVICE, "unknown kernel flag"};
}

void validate_common(int64_t m, const double* tx, const double* ty, const pp_params* prm, const double* p_out) {
  if (!prm) throw PPError{PP_ERR_ARG, "params is null"};
  if (m < 0 || m >= ((int64_t)1 << 31)) throw PPError{PP_ERR_ARG, "target count out of range"};
  if (m > 0 && (!tx || !ty || !p_out)) throw PPError{PP_ERR_ARG, "target or output pointer is null"};
  if (prm->p < 1 || prm->p > kMaxP) throw PPError{PP_ERR_ARG, "p must lie in [1, 20]"};
  if (!(prm->theta > 0.0 && prm->theta < 1.0)) throw PPError{PP_ERR_ARG, "theta must lie in (0, 1)"};
  const int num = (int)std::lround(prm->theta * 1000.0);
  if (num < 1 || num > 999) throw PPError{PP_ERR_ARG, "theta rounds to 0 or 1"};
  if (prm->leaf_max < 1 || prm->leaf_max > 4096) throw PPError{PP_ERR_ARG, "leaf_max must lie in [1, 4096]"};
  if (prm->precision != PP_FP64 && prm->precision != PP_MIXED) throw PPError{PP_ERR_ARG, "unknown precision"};
  if (prm->self_mode != PP_SELF_SKIP && prm->self_mode != PP_SELF_CELLAVG) throw PPError{PP_ERR_ARG, "unknown self mode"};
  if (prm->method != PP_METHOD_FMM && prm->method != PP_METHOD_TREECODE) throw PPError{PP_ERR_ARG, "unknown method"};
}

void validate(int32_t nx, int32_t ny, double x0, double y0, double h, const double* f, int64_t m, const double* tx,
              const double* ty, const pp_params* prm, const double* p_out) {
  if (nx < 1 || ny < 1 || nx > 65536 || ny > 65536 || (int64_t)nx * ny >= ((int64_t)1 << 31))
    throw PPError{PP_ERR_ARG, "grid size out of range"};
  if (!(h > 0.0) || !std::isfinite(h) || !std::isfinite(x0) || !std::isfinite(y0))
    throw PPError{PP_ERR_ARG, "h must be positive and finite, x0/y0 finite"};
  if (!f) throw PPError{PP_ERR_ARG, "f is null"};
  validate_common(m, tx, ty, prm, p_out);
}

// The two source forms: grid nodes (f on an nx x ny grid of spacing h, weight
// f h^2) or scattered points with their own weights.
struct Sources {
  bool grid = true;
  int32_t nx = 0, ny = 0;
  double x0 = 0.0, y0 = 0.0, h = 0.0;
  const double* f = nullptr;
  int64_t n = 0;
  const double* sx = nullptr;
  const double* sy = nullptr;
  const double* w = nullptr;
};

void validate_points(int64_t n, const double* sx, const double* sy, const double* w, int64_t m, const double* tx,
                     const double* ty, const pp_params* prm, const double* p_out) {
  if (n < 0 || n >= ((int64_t)1 << 31)) throw PPError{PP_ERR_ARG, "source count out of range"};
  if (n > 0 && (!sx || !sy || !w)) throw PPError{PP_ERR_ARG, "source pointer is null"};
  validate_common(m, tx, ty, prm, p_out);
  if (prm->self_mode != PP_SELF_SKIP)
    throw PPError{PP_ERR_ARG, "scattered sources support only the skip self rule (there is no cell to average over)"};
}

// One solve.  Two host round trips: after the tree (its level starts and the
// cell-list counts size the later launches) and at the end (flags, statistics).
// The launches between them form two segments, each of which is replayed from a
// captured HIP graph when a call repeats the previous one's shape, device
// pointers and (for the second) tree; every buffer is sized before a segment.
// `exact_lists` selects the two-pass interaction lists (count, scan, emit);
// otherwise the lists are written in one pass into a fixed capacity per cell,
// and a list that does not fit makes the solve report kFlagListOverflow (the
// caller then repeats it with exact lists).
// batch (may be null): a forest of grid requests (device inputs and outputs;
// src describes the first request's grid, m is the joint target count).
pp_status run_solve(pp_ctx& c, bool direct, bool exact_lists, const Sources& src, int64_t m, const double* tx,
                    const double* ty, const pp_params& prm, double* p_out, hipStream_t s, bool resident = false,
                    const GridBatch* batch = nullptr) {
  const auto t_start = std::chrono::steady_clock::now();
  HIPCHK(hipSetDevice(c.device));
  if (s == nullptr) {
    if (!c.own_stream) HIPCHK(hipStreamCreate(&c.own_stream));  // blocking, default priority
    s = c.own_stream;
  }
  c.cur_stream = s;
  c.last.valid = false;
  // a resident solve reuses the retained tree (its sizes and list layout);
  // any other solve rebuilds the buffers the tree lives in
  const Resident R = c.res;
  if (resident) exact_lists = R.exact_lists;
  else c.res.valid = false;
  if (c.arena) {  // every piece of the workspace is handed out anew
    c.arena_used = 0;
    for (auto& a : c.abufs) a = DevBuf{};
  }
  const int32_t nx = src.grid ? src.nx : 0, ny = src.grid ? src.ny : 0;
  const int64_t ngrid = src.grid ? (int64_t)nx * ny : 0;
  const int nreq = batch ? batch->nreq : 0;
  const int top = batch ? batch->levels : 0;  // levels above a forest's request roots
  const int64_t nmax = src.grid ? ngrid * std::max(nreq, 1) : src.n;  // sources before culling zeros
  const int p = prm.p;
  const int g = std::gcd((int)std::lround(prm.theta * 1000.0), 1000);
  const int num = (int)std::lround(prm.theta * 1000.0) / g, den = 1000 / g;
  const bool mixed = prm.precision == PP_MIXED;
  const int lm = prm.leaf_max;

  // profiling 1: events between all phases (no graph replay); 2: events around the
  // near-field launch only, which then runs outside the replayed segments
  auto mark = [&](int i) {
    if (c.profiling == 1) HIPCHK(hipEventRecord(c.ev[i], s));
  };
  // profiling 2 / 16 + phase: events around one phase's launches, on the
  // stream they run on, in the schedule of an untimed call
  const int timed_phase = c.profiling == 2 ? PP_PHASE_P2P : c.profiling >= 16 ? c.profiling - 16 : -1;
  auto tbegin = [&](int ph, hipStream_t q) {
    if (ph == timed_phase) HIPCHK(hipEventRecord(c.ev[0], q));
  };
  auto tend = [&](int ph, hipStream_t q) {
    if (ph == timed_phase) HIPCHK(hipEventRecord(c.ev[1], q));
  };
  // Every buffer of the first segment (staging copies of host inputs included)
  // depends on the input sizes only: sized, and checked against the budget,
  // before anything is allocated or enqueued.
  const bool f_host = src.grid && ngrid > 0 && !is_device_ptr(src.f);
  const bool t_host = m > 0 && !is_device_ptr(tx);
  const bool ty_host = m > 0 && !is_device_ptr(ty);
  const bool out_on_device = is_device_ptr(p_out);
  const bool pts_host = !src.grid && src.n > 0 && !is_device_ptr(src.sx);
  const bool ptsy_host = !src.grid && src.n > 0 && !is_device_ptr(src.sy);
  const bool ptsw_host = !src.grid && src.n > 0 && !is_device_ptr(src.w);
  const int D = src.grid ? root_exponent(nx, ny) + top : kPointsDepth;
  const int k = D;
  // capacities from the input sizes (the source count is only known on the device)
  int64_t geo = 0;
  for (int l = 0; l <= D; ++l) geo += (int64_t)1 << (2 * l);
  const int64_t per_level = 4 * (nmax / (lm + 1) + m / (lm + 1) + 1);  // children of split cells
  const int64_t cap = std::min<int64_t>(geo, 1 + (int64_t)std::max(D, 1) * per_level) + 1;
  if (cap >= ((int64_t)1 << 31) / 4) throw PPError{PP_ERR_LIMIT, "tree capacity exceeds the index range"};
  const bool treecode = prm.method == PP_METHOD_TREECODE;
  const int cap_far = resident ? R.cap_far : treecode ? c.cap_m2p : c.cap_m2l;
  const int cap_near = resident ? R.cap_near : treecode ? c.cap_tp2p : c.cap_p2p;
  // levels 0..Ld from the dense prefix table, the rest one level at a time
  const int Ld = std::min(D, c.dense_levels);
  const int64_t dense_np = ((int64_t)1 << (2 * Ld)) + 1;
  const int64_t dense_F = tree_dense_cells(Ld);
  const int64_t wmax = std::min<int64_t>(cap, per_level);
  const int nbox = src.grid ? 0 : points_box_blocks(src.n + m);

  double* f_stage = nullptr;
  double *tx_stage = nullptr, *ty_stage = nullptr, *out_d = p_out;
  double *psx_stage = nullptr, *psy_stage = nullptr, *pw_stage = nullptr;
  int* misc = nullptr;
  double4* boxp = nullptr;
  int* boxc = nullptr;
  uint32_t *skey = nullptr, *sij = nullptr, *skey2 = nullptr, *tkey = nullptr, *tkey2 = nullptr;
  double *sw = nullptr, *pxs = nullptr, *pys = nullptr;
  int *tile = nullptr, *sort_tmp = nullptr, *sperm2 = nullptr, *tperm = nullptr, *tperm2 = nullptr;
  TreeArrays ta{};
  int4* rec = nullptr;
  int *cm2l = nullptr, *om2l = nullptr, *cp2p = nullptr, *op2p = nullptr;
  int *dss = nullptr, *dts = nullptr, *dflag = nullptr, *doff = nullptr;
  int4* cr = nullptr;
  int *sp = nullptr, *ex = nullptr, *off = nullptr, *scan = nullptr;
  int *sleaves = nullptr, *tleaves = nullptr, *tcells = nullptr, *flag3 = nullptr;
  reserve(c, [&] {
    if (f_host) f_stage = ensure<double>(c, B_F, ngrid);
    if (t_host) tx_stage = ensure<double>(c, B_TX, m);
    if (ty_host) ty_stage = ensure<double>(c, B_TY, m);
    out_d = out_on_device ? p_out : ensure<double>(c, B_OUT, m);
    misc = ensure<int>(c, B_MISC, kMiscInts);
    if (!src.grid) {
      if (pts_host) psx_stage = ensure<double>(c, B_PSX, src.n);
      if (ptsy_host) psy_stage = ensure<double>(c, B_PSY, src.n);
      if (ptsw_host) pw_stage = ensure<double>(c, B_PW, src.n);
      boxp = ensure<double4>(c, B_BOXP, nbox);
      boxc = ensure<int>(c, B_BOXC, nbox);
    }
    scan = ensure<int>(c, B_SCAN,
                       std::max<int64_t>((int64_t)scan_temp_ints(std::max<int64_t>({4 * per_level, cap, m, nmax, 1})),
                                         tree_dense_part_ints(Ld)));
    skey = ensure<uint32_t>(c, B_SKEY, nmax);
    sij = ensure<uint32_t>(c, B_SIJ, nmax);  // grid: packed (i, j); points: input index
    sw = ensure<double>(c, B_SW, nmax);
    tile = src.grid ? ensure<int>(c, B_TILE, ingest_count_ints(k)) : nullptr;
    sort_tmp = ensure<int>(c, B_SORT, (int64_t)radix_temp_ints(std::max<int64_t>(src.grid ? 0 : src.n, m)));
    skey2 = src.grid ? nullptr : ensure<uint32_t>(c, B_SKEY2, src.n);
    sperm2 = src.grid ? nullptr : ensure<int>(c, B_SPERM2, src.n);
    if (!src.grid) {
      pxs = ensure<double>(c, B_PXS, src.n);
      pys = ensure<double>(c, B_PYS, src.n);
    }
    tkey = ensure<uint32_t>(c, B_TKEY, m);
    tperm = ensure<int>(c, B_TPERM, m);
    tkey2 = ensure<uint32_t>(c, B_TKEY2, m);
    tperm2 = ensure<int>(c, B_TPERM2, m);
    ta = TreeArrays{ensure<int>(c, B_LVL, cap),  ensure<int>(c, B_IX, cap),    ensure<int>(c, B_IY, cap),
                    ensure<int>(c, B_SB, cap),   ensure<int>(c, B_SE, cap),    ensure<int>(c, B_TB, cap),
                    ensure<int>(c, B_TE, cap),   ensure<int>(c, B_CHILD, cap), ensure<int>(c, B_NCHILD, cap),
                    ensure<int>(c, B_PARENT, cap)};
    // the lists' per-cell setup (records, counts, one-pass offsets) is written by
    // the first segment's cell classification, so its buffers hold `cap` cells
    rec = direct ? nullptr : ensure<int4>(c, B_REC, cap);
    cm2l = ensure<int>(c, B_CM2L, cap);
    om2l = ensure<int>(c, B_OM2L, cap);
    cp2p = ensure<int>(c, B_CP2P, cap);
    op2p = ensure<int>(c, B_OP2P, cap);
    dss = ensure<int>(c, B_DSS, dense_np);
    dts = ensure<int>(c, B_DTS, dense_np);
    dflag = ensure<int>(c, B_DFLAG, dense_F);
    doff = ensure<int>(c, B_DOFF, dense_F);
    cr = ensure<int4>(c, B_CR, 4 * wmax);
    sp = ensure<int>(c, B_SPLIT, 6 * wmax);
    ex = ensure<int>(c, B_CNT, 4 * wmax);
    off = ensure<int>(c, B_OFF, 4 * wmax);
    sleaves = ensure<int>(c, B_SLEAF, cap);
    tleaves = ensure<int>(c, B_TLEAF, cap);
    tcells = ensure<int>(c, B_TCELL, cap);
    flag3 = ensure<int>(c, B_FLAG, classify_part_ints(cap));  // per-tile counts of the classification
  });
  auto copy_in = [&](double* dst, const double* srcp, int64_t n) -> const double* {
    if (!dst) return srcp;
    HIPCHK(hipMemcpyAsync(dst, srcp, (size_t)n * sizeof(double), hipMemcpyHostToDevice, s));
    return dst;
  };
  const double* f_d = src.grid ? copy_in(f_stage, src.f, ngrid) : nullptr;
  const double* tx_d = copy_in(tx_stage, tx, m);
  const double* ty_d = copy_in(ty_stage, ty, m);
  unsigned long long* pairs = (unsigned long long*)(misc + M_PAIRS);  // 8-byte aligned slot

  // root square: anchor (x0, y0), finest cell side `unit`, finest level D
  double x0 = 0.0, y0 = 0.0, unit = 1.0;
  const double *psx = nullptr, *psy = nullptr, *pw = nullptr;
  if (src.grid) {
    x0 = src.x0;
    y0 = src.y0;
    unit = src.h;
  } else {
    fill_i32(misc, 0, kMiscInts, s);
    psx = copy_in(psx_stage, src.sx, src.n);
    psy = copy_in(psy_stage, src.sy, src.n);
    pw = copy_in(pw_stage, src.w, src.n);
    double* box = (double*)(misc + M_BOX);
    points_box(psx, psy, pw, src.n, tx_d, ty_d, m, boxp, boxc, box, misc + M_NSRC, misc + M_FLAGS, s);
    readback(c, misc, 0, M_BOX + 8, s);
    check_flags(c.pinned[M_FLAGS]);
    double bx[4];
    std::memcpy(bx, c.pinned + M_BOX, sizeof(bx));
    x0 = bx[0];
    y0 = bx[2];
    // the same FP64 differences the key kernels form for the extreme points
    const double ext = std::max(bx[1] - bx[0], bx[3] - bx[2]);
    unit = 1.0;
    if (ext > 0.0 && ext < 1e-280) throw PPError{PP_ERR_ARG, "the points span less than 1e-280"};
    if (ext > 0.0) {
      int e = std::ilogb(ext) - D;
      while (std::ldexp(1.0, e + D) <= ext) ++e;
      while (e > -1000 && std::ldexp(1.0, e + D - 1) > ext) --e;
      unit = std::ldexp(1.0, e);
    }
  }
  int* ls_d = misc + M_LS;

  // ---- segment 1: ingest, target sort, tree, cell lists; ends with the read-back ----
  // (graph replay only for device-resident grid input: host input is staged by copies)
  const bool replayable = src.grid && !batch && !exact_lists && !direct && !resident && !c.arena && f_d == src.f && tx_d == tx &&
                          ty_d == ty && out_on_device && c.profiling != 1 &&
                          !(timed_phase >= PP_PHASE_INGEST && timed_phase <= PP_PHASE_TREE);
  const std::vector<uint64_t> key1 = {(uint64_t)nx, (uint64_t)ny, bits(x0), bits(y0), bits(unit), (uint64_t)m,
                                      (uint64_t)lm, (uint64_t)c.dense_levels, (uint64_t)c.profiling, bits(f_d),
                                      bits(tx_d), bits(ty_d), (uint64_t)direct, (uint64_t)cap_far,
                                      (uint64_t)cap_near};
  // the levels below the dense table, one launch group per level (on the device sizes)
  auto build_levels_below = [&] {
    for (int l = Ld; l < D; ++l) {
      const int64_t lmax = std::min<int64_t>(wmax, (int64_t)1 << std::min(2 * l, 40));
      tree_level(ta, ls_d, l, D, lm, lmax, (int)cap, skey, tkey, sp, cr, ex, off, scan, misc + M_N4, misc + M_TOT,
                 misc + M_FLAGS, s);
    }
  };
  // cell lists over the whole tree (its size is the last level start, on the
  // device; bound: at least that many cells, the launch's size)
  auto classify = [&](int64_t bound) {
    const TreeView tv0{D, 0, ta.lvl, ta.ix, ta.iy, ta.sb, ta.se, ta.tb, ta.te, ta.child, ta.nchild, ta.parent};
    const RecordArgs rec0{tv0, rec, cm2l, cp2p, om2l, op2p, cap_far, cap_near};
    classify_cells(ta, ls_d + D + 1, (int)std::min<int64_t>(bound, cap), flag3, sleaves, tleaves, tcells,
                   misc + M_NSL, direct ? nullptr : &rec0, s);
  };
  const int seq1 = published_seq(c) + 1;
  // the retained tree: new weights for its sources, and the checks that it
  // still fits (no new nonzero node, every target in its finest cell); no
  // round trip follows, so it is issued with the second segment below
  auto resident_first = [&] {
    mark(PP_PHASE_INGEST);
    fill_i32(misc, 0, kMiscInts, s);
    tbegin(PP_PHASE_INGEST, s);
    resident_weights(f_d, nx, ny, k, unit * unit, tile, sij, R.N, sw, misc + M_FLAGS, s);
    tend(PP_PHASE_INGEST, s);
    mark(PP_PHASE_SORT);
    tbegin(PP_PHASE_SORT, s);
    resident_targets(tx_d, ty_d, m, tperm, tkey, x0, y0, unit, k, misc + M_FLAGS, s);
    tend(PP_PHASE_SORT, s);
    mark(PP_PHASE_TREE);
  };
  if (!resident) run_segment(c, 0, replayable, key1, s, [&] {
    mark(PP_PHASE_INGEST);
    if (src.grid) fill_i32(misc, 0, kMiscInts, s);  // scattered input: cleared before its bounding box
    tbegin(PP_PHASE_INGEST, s);
    if (src.grid) {
      // ---- ingest: sources in Morton order (no sort needed for a grid) ----
      ingest_grid_count(f_d, nx, ny, k, tile, misc + M_FLAGS, batch, s);
      ingest_grid_emit(f_d, nx, ny, k, unit * unit, tile, misc + M_NSRC, sij, sw, dss, D - Ld, batch, s);
    } else if (src.n > 0) {
      // ---- ingest: keys of the scattered sources, stable sort, sorted copies ----
      int* sperm = (int*)sij;
      points_keys(psx, psy, pw, src.n, x0, y0, unit, D, skey, sperm, s);
      radix_sort_pairs(skey, sperm, skey2, sperm2, src.n, 32, sort_tmp, s);
      points_gather(sperm, misc + M_NSRC, src.n, psx, psy, pw, pxs, pys, sw, s);
    }
    tend(PP_PHASE_INGEST, s);
    // ---- targets: Morton keys and a stable radix sort ----
    mark(PP_PHASE_SORT);
    tbegin(PP_PHASE_SORT, s);
    target_keys_sorted(tx_d, ty_d, m, x0, y0, unit, k, tkey, tperm, tkey2, tperm2, sort_tmp, misc + M_FLAGS, batch,
                       s);
    tend(PP_PHASE_SORT, s);
    // ---- tree: dense top levels, then (scattered sources) one launch group per level ----
    mark(PP_PHASE_TREE);
    tbegin(PP_PHASE_TREE, s);
    tree_dense_top(ta, ls_d, D, Ld, lm, top, (int)cap, skey, misc + M_NSRC, src.grid ? 1 : 0, tkey, (int)m, dss, dts,
                   dflag, doff, scan, misc + M_TOT, misc + M_DEEP, misc + M_FLAGS, s);
    // Grid sources: a cell of the dense table's last level holds at most
    // 4^(D - Ld) nodes, so it is split only by its targets, which is rare:
    // the levels below are built after the read-back, only if one is.
    if (!src.grid) build_levels_below();
    // grid sources: every cell so far is a cell of the dense table
    classify(src.grid ? dense_F : cap);
    tend(PP_PHASE_TREE, s);
    publish_enqueue(c, misc, M_LS + D + 2, s);
  });
  if (!resident) {
    wait_published(c, s, seq1);
    check_flags(c.pinned[M_FLAGS]);
    if (src.grid && c.pinned[M_DEEP]) {
      // a cell of the dense table's last level has more than leaf_max targets;
      // the levels below search the source keys, which the grid ingest leaves
      // implicit in the node indices
      const int seq_deep = published_seq(c) + 1;
      keys_from_ij(sij, misc + M_NSRC, nmax, skey, s);
      build_levels_below();
      classify(cap);
      publish_enqueue(c, misc, M_LS + D + 2, s);
      wait_published(c, s, seq_deep);
      check_flags(c.pinned[M_FLAGS]);
    }
  }
  const int64_t N = resident ? R.N : c.pinned[M_NSRC];
  std::vector<int> lstart;  // level l holds cells [lstart[l], lstart[l+1])
  if (resident) {
    lstart = R.lstart;
  } else {
    const int* ls_h = c.pinned + M_LS;
    lstart = {ls_h[0], ls_h[1]};
    for (int l = 1; l <= D; ++l) {
      if (ls_h[l + 1] == ls_h[l]) break;
      lstart.push_back(ls_h[l + 1]);
    }
  }
  const int ncells = lstart.back();
  const int depth = (int)lstart.size() - 2;
  const int nsl = resident ? R.nsl : c.pinned[M_NSL], ntl = resident ? R.ntl : c.pinned[M_NTL],
            ntc = resident ? R.ntc : c.pinned[M_NTC];
  const TreeView tv{D, ncells, ta.lvl, ta.ix, ta.iy, ta.sb, ta.se, ta.tb, ta.te, ta.child, ta.nchild, ta.parent};

  // ---- every buffer of the second segment, sized (and checked against the
  // budget) from the tree's counts before anything of it is allocated ----
  int* m2l_src = nullptr;
  int* p2p_src = nullptr;
  int64_t n_m2l = 0, n_p2pl = 0;
  // the tree-code's M2P leaves its list parts' partial sums side by side
  const int far_parts = treecode ? kM2PParts : 1;
  const int nparts = c.p2p_parts;
  float* s32 = nullptr;
  double *leaf_w = nullptr, *selfd = nullptr, *selfw = nullptr, *far = nullptr, *near = nullptr;
  float2* rel32 = nullptr;
  double2 *rel64 = nullptr, *s64 = nullptr, *mp = nullptr, *loc = nullptr, *own = nullptr;
  int *tgtleaf = nullptr, *claim = nullptr;
  long long* pcount = nullptr;
  reserve(c, [&] {
    // the tree-code variant lists per target leaf (M2P cells, P2P leaves); the
    // multipole method lists per cell with targets (M2L cells, P2P leaves)
    if (!direct && !exact_lists) {
      m2l_src = ensure<int>(c, B_M2LSRC, (int64_t)ncells * cap_far);
      p2p_src = ensure<int>(c, B_P2PSRC, (int64_t)ncells * cap_near);
    }
    s32 = ensure<float>(c, B_SRC4, 3 * std::max<int64_t>(N, 1));  // x, y, w planes of stride N
    leaf_w = ensure<double>(c, B_LEAFW, ncells);
    rel32 = ensure<float2>(c, B_REL32, m);
    rel64 = ensure<double2>(c, B_REL64, m);
    tgtleaf = ensure<int>(c, B_TGTLEAF, m);
    selfd = src.grid ? ensure<double>(c, B_SELFD, m) : nullptr;
    selfw = ensure<double>(c, B_SELFW, m);
    s64 = src.grid ? nullptr : ensure<double2>(c, B_S64, N);
    mp = direct ? nullptr : ensure<double2>(c, B_MP, (int64_t)ncells * (p + 1));
    loc = (direct || treecode) ? nullptr : ensure<double2>(c, B_LOC, (int64_t)ncells * (p + 1));
    own = (direct || treecode) ? nullptr : ensure<double2>(c, B_OWNLOC, (int64_t)ncells * (p + 1));
    far = direct ? nullptr : ensure<double>(c, B_FAR, m * far_parts);
    near = ensure<double>(c, B_NEAR, (int64_t)nparts * m);
    pcount = ensure<long long>(c, B_PCOUNT, (int64_t)nparts * std::max(ntl, 1));
    claim = ensure<int>(c, B_CLAIM, ncells);
  });
  if (resident && exact_lists) {  // the retained two-pass lists
    m2l_src = (int*)c.bufs[B_M2LSRC].p;
    p2p_src = (int*)c.bufs[B_P2PSRC].p;
    n_m2l = R.n_m2l;
    n_p2pl = R.n_p2pl;
  }
  P2PArgs pa{};
  pa.t = tv;
  pa.tleaves = tleaves;
  pa.ntleaves = ntl;
  pa.list_off = direct ? nullptr : op2p;
  pa.list_cnt = direct ? nullptr : cp2p;
  pa.sleaves = sleaves;
  pa.nsleaves = nsl;
  pa.sx = s32;
  pa.sy = s32 + std::max<int64_t>(N, 1);
  pa.sw = s32 + 2 * std::max<int64_t>(N, 1);
  pa.s64 = s64;
  pa.w64 = sw;
  pa.leaf_w = leaf_w;
  pa.rel32 = rel32;
  pa.rel64 = rel64;
  pa.nparts = nparts;
  pa.m = m;
  pa.pair_counts = pcount;
  pa.flags = misc + M_FLAGS;
  pa.pairs = pairs;
  pa.near_sum = near;
  pa.lnh = std::log(unit);
  if (!mixed && c.arena) {  // a piece of the workspace, filled on every call (one stream)
    double* lt = ensure<double>(c, B_LOGT, kLogTable);
    log_table(lt, s);
    pa.log_tab = lt;
  } else {
    if (!mixed && !c.log_tab) {  // filled once, outside any captured segment
      HIPCHK(hipMalloc((void**)&c.log_tab, kLogTable * sizeof(double)));
      log_table(c.log_tab, s);
      HIPCHK(hipStreamSynchronize(s));  // the near field may run on the side stream without waiting on s
    }
    pa.log_tab = c.log_tab;
  }
  pa.list_src = direct ? nullptr : p2p_src;  // set again below once exact lists are allocated
  // statistics: pair count, and the list totals of the one-pass lists
  const bool list_totals = !direct && !exact_lists;

  // a frontier that overflowed below the top tier: raise the tier for this and later solves
  auto frontier_retry = [&](int flags) {
    if (!(flags & kFlagFrontierOverflow) || frontier_at_top(num, den, c.frontier_boost)) return;
    ++c.frontier_boost;
    c.cur_stream = nullptr;
    throw FrontierRetry{};
  };
  auto list_pass = [&](int emit, const int* om, const int* op, int* ms, int* ps, int cm, int cp,
                       const LeafPass* lp, hipStream_t q) {
    if (treecode)
      lists_treecode_pass(tv, rec, tleaves, ntl, num, den, emit, cm2l, cp2p, om, op, ms, ps, cm, cp, misc + M_FLAGS,
                          c.frontier_boost, lp, q);
    else
      lists_pass(tv, rec, tcells, ntc, num, den, emit, cm2l, cp2p, om, op, ms, ps, cm, cp, misc + M_FLAGS,
                 c.frontier_boost, top, lp, q);
  };
  std::vector<uint64_t> key2 = key1;
  for (uint64_t v : {(uint64_t)N, (uint64_t)ncells, (uint64_t)nsl, (uint64_t)ntl, (uint64_t)ntc, (uint64_t)depth,
                     (uint64_t)p, (uint64_t)num, (uint64_t)den, (uint64_t)prm.precision, (uint64_t)prm.self_mode,
                     (uint64_t)prm.method, (uint64_t)cap_far, (uint64_t)cap_near, (uint64_t)nparts, bits(out_d),
                     (uint64_t)c.frontier_boost})
    key2.push_back(v);
  for (int v : lstart) key2.push_back((uint64_t)v);

  // ---- segment 2: lists, expansions, near field, finalize; ends with the read-back ----
  // Dependencies: the upward pass and the lists need only segment 1 (P2M forms
  // its source offsets itself); the near field needs the lists and both
  // packings; the M2L (or M2P) needs the lists and the upward pass.  So the
  // work forks: the side stream builds the lists, prepares the targets and
  // runs the near field, while the caller's stream runs the upward pass, waits
  // for the lists, runs the M2L and downward passes, and finally waits for the
  // near field before the finalize step.
  // Each stream's work fills compute units the other leaves idle.  Timing mode
  // 1 keeps every phase on one stream, in phase order, so that its per-phase
  // events mean something.
  hipStream_t ss = s;
  // (the allocation-free solve keeps one stream: no stream or event is created for it)
  if (c.profiling != 1 && c.near_stream && !c.arena) {
    if (!c.side_stream) HIPCHK(hipStreamCreateWithFlags(&c.side_stream, hipStreamNonBlocking));
    // the events order work between two streams of one device: a device-scope
    // release and acquire suffice (the host never inspects them)
    for (hipEvent_t* e : {&c.ev_fork, &c.ev_lists, &c.ev_join})
      if (!*e) HIPCHK(hipEventCreateWithFlags(e, hipEventDisableTiming | hipEventDisableSystemFence));
    ss = c.side_stream;
  }
  // `from` signals `to` through event e (no-op without the side stream)
  auto signal = [&](hipEvent_t e, hipStream_t from, hipStream_t to) {
    if (ss == s) return;
    HIPCHK(hipEventRecord(e, from));
    HIPCHK(hipStreamWaitEvent(to, e, 0));
  };
  // the two-pass lists read a total back to the host, so they run first, on s
  const bool lists_early = exact_lists && !direct && !resident;

  // lp (one-pass lists only): the per-leaf packing rides on the list launch
  auto do_lists = [&](hipStream_t q, const LeafPass* lp) {
    if (direct) return;
    if (resident) {  // retained
      pa.list_src = p2p_src;
      return;
    }
    if (exact_lists) {
      list_pass(0, nullptr, nullptr, nullptr, nullptr, 0, 0, nullptr, q);  // records, cleared counts: segment 1
      scan_exclusive(cm2l, om2l, ncells, scan, misc + M_NM2L, q);
      scan_exclusive(cp2p, op2p, ncells, scan, misc + M_NP2P, q);
      readback(c, misc, 0, 16, q);
      frontier_retry(c.pinned[M_FLAGS]);
      check_flags(c.pinned[M_FLAGS]);
      n_m2l = c.pinned[M_NM2L];
      n_p2pl = c.pinned[M_NP2P];
      m2l_src = ensure<int>(c, B_M2LSRC, n_m2l);
      p2p_src = ensure<int>(c, B_P2PSRC, n_p2pl);
      list_pass(1, om2l, op2p, m2l_src, p2p_src, 0, 0, nullptr, q);
    } else {
      list_pass(2, om2l, op2p, m2l_src, p2p_src, cap_far, cap_near, lp, q);  // records, offsets: segment 1
    }
    pa.list_src = p2p_src;
  };
  // source packing and target preparation, one launch
  auto do_pack_prep = [&](hipStream_t q) {
    if (src.grid)
      leaf_pack_prep(ta, D, sleaves, nsl, sij, sw, s32, std::max<int64_t>(N, 1), leaf_w, tleaves, ntl, tx_d, ty_d,
                     tperm, x0, y0, unit, nx, ny, mixed ? 0x1p-40 : 0.0, f_d, rel32, rel64, tgtleaf, selfw, selfd,
                     batch, q);
    else
      leaf_pack_prep_points(ta, D, x0, y0, unit, pxs, pys, sw, sleaves, nsl, s32, std::max<int64_t>(N, 1), s64,
                            leaf_w, tleaves, ntl, tx_d, ty_d, tperm, rel32, rel64, tgtleaf, selfw, q);
  };
  // The one-pass lists (records and offsets written by segment 1) carry the
  // per-leaf packing in extra workgroups of their launch, so the two overlap,
  // in the directly issued schedule.  (In the graph, lists and packing before
  // the fork made the replay 10% slower: there the packing stays its own
  // launch before the fork, and the lists run on the side stream.)
  // The second segment issued directly: timed calls, and by default untimed
  // ones too (the replayed graph runs the side branch's kernels first, which
  // made the multipole solve 2-4 % and the tree-code 15 % slower).
  const bool issue2 = timed_phase >= 0 || (c.profiling == 0 && (c.direct_issue || resident) && ss != s);
  const bool fused = !direct && !exact_lists && issue2 && !resident;
  const LeafPass lpass =
      src.grid ? leaf_pass_grid(ta, D, sleaves, nsl, sij, sw, s32, std::max<int64_t>(N, 1), leaf_w, tleaves, ntl, tx_d,
                                ty_d, tperm, x0, y0, unit, nx, ny, mixed ? 0x1p-40 : 0.0, f_d, rel32, rel64, tgtleaf,
                                selfw, selfd, batch)
               : leaf_pass_points(ta, D, x0, y0, unit, pxs, pys, sw, sleaves, nsl, s32, std::max<int64_t>(N, 1), s64,
                                  leaf_w, tleaves, ntl, tx_d, ty_d, tperm, rel32, rel64, tgtleaf, selfw);
  auto do_p2m = [&] {
    mark(PP_PHASE_P2M);
    tbegin(PP_PHASE_P2M, s);
    if (!direct)
      p2m(tv, sleaves, nsl, src.grid ? sij : nullptr, pxs, pys, x0, y0, unit, sw, p, mp, c.p2m_lattice_min, s);
    tend(PP_PHASE_P2M, s);
  };
  auto do_m2m = [&] {
    mark(PP_PHASE_M2M);
    if (direct) return;
    tbegin(PP_PHASE_M2M, s);
    // the recursion from the finest level up, several levels per launch
    const int ml = m2m_max_levels();
    for (int top = depth - 1; top >= 0; top -= ml) {
      const int L = std::max(top - (ml - 1), 0);
      m2m_levels(tv, lstart[L], lstart[L + 1], L, top - L + 1, p, mp, dflag, doff, Ld, s);
    }
    tend(PP_PHASE_M2M, s);
  };
  auto do_upward = [&] {
    do_p2m();
    do_m2m();
  };
  // L2P runs inside the finalize launch (one launch fewer after the near
  // field), except in timing mode 1, which times it as a phase of its own
  const bool fuse_l2p = !direct && !treecode && c.profiling != 1;
  auto do_downward = [&] {
    if (direct) {
      for (int ph = PP_PHASE_M2L; ph <= PP_PHASE_L2P; ++ph) mark(ph);
      return;
    }
    mark(PP_PHASE_M2L);
    tbegin(PP_PHASE_M2L, s);
    if (treecode) {
      // multipoles evaluated at the targets; no local expansions
      m2p(tv, tleaves, ntl, om2l, cm2l, m2l_src, p, unit, mp, rel64, mixed ? 1 : 0, far_parts, m, far,
          misc + M_FLAGS, s);
      tend(PP_PHASE_M2L, s);
      mark(PP_PHASE_L2L);
      mark(PP_PHASE_L2P);
    } else {
      m2l(tv, tcells, ntc, om2l, cm2l, m2l_src, p, unit, mp, own, misc + M_FLAGS, s);
      tend(PP_PHASE_M2L, s);
      mark(PP_PHASE_L2L);
      tbegin(PP_PHASE_L2L, s);
      downward(tv, tcells, ntc, p, own, loc, doff, Ld, top, s);
      tend(PP_PHASE_L2L, s);
      mark(PP_PHASE_L2P);
      if (!fuse_l2p) l2p(tv, m, tgtleaf, p, loc, rel64, mixed ? 1 : 0, far, s);
    }
  };
  auto do_near = [&](hipStream_t q) { p2p(pa, mixed ? 0 : 1, q); };
  auto do_finalize = [&] {
    mark(PP_PHASE_FINALIZE);
    FinalizeTotals tot;
    tot.pair_counts = pcount;
    tot.nwaves = (int64_t)ntl * nparts;
    tot.pairs = pairs;
    tot.cnt_m = list_totals ? cm2l : nullptr;
    tot.cnt_p = list_totals ? cp2p : nullptr;
    tot.ncells = ncells;
    tot.tot_m = misc + M_NM2L;
    tot.tot_p = misc + M_NP2P;
    FarEval fe;
    fe.far_parts = far_parts;
    if (fuse_l2p) {
      fe.loc = loc;
      fe.rel64 = rel64;
      fe.tleaf = tgtleaf;
      fe.lvl = tv.lvl;
      fe.D = D;
      fe.p = p;
      fe.fp32 = mixed ? 1 : 0;
    }
    tbegin(PP_PHASE_FINALIZE, s);
    finalize(m, nparts, tperm, far, near, selfw, selfd, unit, prm.self_mode, misc + M_FLAGS, out_d, tot, fe, batch,
             s);
    tend(PP_PHASE_FINALIZE, s);
    mark(12);
    publish_enqueue(c, misc, M_PAIRS + 2, s);
  };
  // The two streams' launches before the near field, interleaved for the
  // directly issued schedule: the host issues launches one at a time, so each
  // stream gets its first kernel at once rather than after all of the other
  // stream's launches, and the upward pass runs beside the list building
  // (kernels that leave most of the GPU idle) rather than beside the near
  // field, which fills it.
  // Lazy packing (directly issued schedule, lists on the device, target
  // leaves few beside the source leaves): the list launch prepares the
  // targets only, and a launch after it packs just the source leaves that
  // some near-field list holds (at 4096^2 with surface targets, a fraction of
  // them), so that less traffic competes with the upward pass.  With targets
  // spread over the whole grid nearly every leaf is listed, and packing them
  // all beside the list building is faster.
  const bool lazy = c.lazy_pack && !direct && (fused || resident) && 4 * (int64_t)ntl < nsl;
  const LeafPass lpass_prep = leaf_pass_prep_only(lpass);
  auto do_pack_listed = [&](hipStream_t q) {
    pack_listed(lpass, tleaves, ntl, op2p, cp2p, p2p_src, ncells, claim, q);
  };
  auto fork_work = [&] {
    if (fused) {
      // one launch: the lists, with the packing (or the target preparation) in extra workgroups
      if (lazy) fill_i32(claim, 0, ncells, ss);
      tbegin(PP_PHASE_LISTS, ss);
      do_lists(ss, lazy ? &lpass_prep : &lpass);
      tend(PP_PHASE_LISTS, ss);
      do_p2m();
      if (lazy) do_pack_listed(ss);
      do_m2m();
      return;
    }
    tbegin(PP_PHASE_PACK, ss);
    if (lazy) {  // resident: the retained lists are there already
      fill_i32(claim, 0, ncells, ss);
      leaf_pass_launch(lpass_prep, ss);
      do_pack_listed(ss);
    } else {
      do_pack_prep(ss);
    }
    tend(PP_PHASE_PACK, ss);
    do_p2m();
    tbegin(PP_PHASE_LISTS, ss);
    if (!lists_early) do_lists(ss, nullptr);
    tend(PP_PHASE_LISTS, ss);
    do_m2m();
  };

  const int seq2 = published_seq(c) + 1;
  // With PP_RESIDENT_GRAPH=1 a resident solve with device inputs and output,
  // untimed, is one graph: its first launches and the whole second segment,
  // captured on the second call with the same retained tree and buffers and
  // replayed after that (the round trip at the end is its only host
  // synchronisation; up to four sets of buffers keep a graph each).  Off by
  // default: at 4096^2 the replay was 8 % slower than issuing the launches
  // (3,449 against 3,766 solves/s, A/B), the graph's executor starting the
  // side stream's branch before the upward pass.
  const bool resident_graph = resident && c.resident_graph && c.profiling == 0 && ss != s && f_d == src.f &&
                              tx_d == tx && ty_d == ty && out_on_device;
  std::vector<uint64_t> key3;
  if (resident_graph)
    key3 = {c.res_gen, bits(f_d), bits(tx_d), bits(ty_d), bits(out_d), (uint64_t)m, (uint64_t)lazy,
            (uint64_t)c.frontier_boost, (uint64_t)nparts};
  auto resident_issue = [&](auto&& second) {
    if (resident_graph) {
      run_segment(c, resident_slot(c, key3), true, key3, s, [&] {
        resident_first();
        second();
      });
    } else {
      if (resident) resident_first();
      second();
    }
  };
  if (issue2) resident_issue([&] {
    // The schedule of a call with the near field on its own stream (bracketed
    // by events in timing mode 2), every launch of this segment issued directly (a
    // captured graph drops event records, and replaying the pieces around the
    // near field as four small graphs was measured slower than issuing their
    // launches: each graph launch delays its first kernel).  Segment 1 is
    // complete (the host has seen its read-back), so the side stream starts
    // without waiting on s: the lists with the packing and target preparation
    // riding on their launch, then the near field.  The upward pass runs
    // meanwhile on s (its launches issued after the side stream's first),
    // which then waits for the lists (M2L, L2L) and for the near field
    // (finalize, with L2P).
    if (lists_early) {
      // the two-pass lists are emitted on s: the near field on the side stream
      // reads them, so that stream waits for the emit pass
      do_lists(s, nullptr);
      signal(c.ev_fork, s, ss);
    }
    // a resident solve wrote its new weights on s without a host round trip:
    // the packing on the side stream reads them
    if (resident) signal(c.ev_fork, s, ss);
    fork_work();
    if (ss != s) HIPCHK(hipEventRecord(c.ev_lists, ss));
    tbegin(PP_PHASE_P2P, ss);
    do_near(ss);
    tend(PP_PHASE_P2P, ss);
    if (ss != s) HIPCHK(hipStreamWaitEvent(s, c.ev_lists, 0));
    do_downward();
    signal(c.ev_join, ss, s);
    do_finalize();
  });
  else if (ss == s) {
    // one stream, phases in order (timing mode 1, or the side stream disabled)
    if (resident) resident_first();
    run_segment(c, 1, replayable, key2, s, [&] {
      mark(PP_PHASE_LISTS);
      do_lists(s, nullptr);
      mark(PP_PHASE_PACK);
      do_pack_prep(s);
      do_upward();
      do_downward();
      mark(PP_PHASE_P2P);
      do_near(s);
      do_finalize();
    });
  } else {
    // Captured in phase order: the graph runs the side branch's kernels before
    // the upward pass whatever the order of capture, and a fork at the start of
    // the segment (two root nodes) was measured to delay the first kernels.
    if (resident) resident_first();
    if (lists_early) do_lists(s, nullptr);
    run_segment(c, 1, replayable, key2, s, [&] {
      do_pack_prep(s);
      signal(c.ev_fork, s, ss);
      if (!lists_early) do_lists(ss, nullptr);
      HIPCHK(hipEventRecord(c.ev_lists, ss));
      do_near(ss);
      do_upward();
      HIPCHK(hipStreamWaitEvent(s, c.ev_lists, 0));
      do_downward();
      signal(c.ev_join, ss, s);
      do_finalize();
    });
  }
  wait_published(c, s, seq2);
  const int flags = c.pinned[M_FLAGS];
  frontier_retry(flags);
  if (flags & kFlagListOverflow) {  // nothing written; repeat with exact lists
    c.cur_stream = nullptr;
    return PP_ERR_LIMIT;
  }
  check_flags(flags);
  for (int i = 0; i < 12; ++i) c.stats.ms_phase[i] = 0.0;
  if (c.profiling == 1) {
    HIPCHK(hipEventSynchronize(c.ev[12]));
    for (int i = 0; i < 12; ++i) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, c.ev[i], c.ev[i + 1]));
      c.stats.ms_phase[i] = ms;
    }
  } else if (timed_phase >= 0) {
    float ms = 0.f;
    HIPCHK(hipEventSynchronize(c.ev[1]));
    HIPCHK(hipEventElapsedTime(&ms, c.ev[0], c.ev[1]));
    c.stats.ms_phase[timed_phase] = ms;
  }
  if (!out_on_device && m > 0) {
    HIPCHK(hipMemcpyAsync(p_out, out_d, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  unsigned long long npairs = 0;
  std::memcpy(&npairs, c.pinned + M_PAIRS, sizeof(npairs));
  if (!direct && !exact_lists) {
    n_m2l = c.pinned[M_NM2L];
    n_p2pl = c.pinned[M_NP2P];
  }

  c.stats.depth = depth;
  c.stats.ncells = ncells;
  c.stats.nsrc_leaves = nsl;
  c.stats.ntgt_leaves = ntl;
  c.stats.nsources = N;
  c.stats.ntargets = m;
  c.stats.n_m2l = n_m2l;
  c.stats.n_p2p_lists = direct ? (int64_t)nsl * ntl : n_p2pl;
  c.stats.n_p2p_pairs = (int64_t)npairs;
  c.stats.ms_total =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  if (src.grid && !direct && !resident && !c.arena && !batch) {
    Resident& r = c.res;
    r.valid = true;
    ++c.res_gen;
    r.nx = nx;
    r.ny = ny;
    r.x0 = x0;
    r.y0 = y0;
    r.h = unit;
    r.m = m;
    r.prm = prm;
    r.exact_lists = exact_lists;
    r.cap_far = cap_far;
    r.cap_near = cap_near;
    r.frontier_boost = c.frontier_boost;
    r.N = N;
    r.n_m2l = n_m2l;
    r.n_p2pl = n_p2pl;
    r.lstart = lstart;
    r.nsl = nsl;
    r.ntl = ntl;
    r.ntc = ntc;
  }
  c.last.valid = true;
  c.last.n_src = N;
  c.last.m = m;
  c.last.ncells = ncells;
  c.last.p = p;
  c.last.n_m2l = exact_lists ? n_m2l : (int64_t)ncells * cap_far;
  c.last.n_p2p = exact_lists ? n_p2pl : (int64_t)ncells * cap_near;
  c.last.has_expansions = !direct;
  c.last.has_locals = !direct && !treecode;
  c.last.nparts = nparts;
  c.last.arena = c.arena;
  c.last.keys_from_ij = src.grid;
  c.cur_stream = nullptr;
  return PP_OK;
}

pp_status guard(pp_ctx* c, bool direct, const Sources& src, int64_t m, const double* tx, const double* ty,
                const pp_params* prm, double* p_out, void* stream, bool resident = false,
                const GridBatch* batch = nullptr) {
  if (!c) return PP_ERR_ARG;
  if (c->dead) {
    c->err = "context is unusable after a device error";
    return PP_ERR_DEVICE;
  }
  try {
    if (src.grid)
      validate(src.nx, src.ny, src.x0, src.y0, src.h, src.f, m, tx, ty, prm, p_out);
    else
      validate_points(src.n, src.sx, src.sy, src.w, m, tx, ty, prm, p_out);
    if (resident) {
      // the retained tree is used once as it is: no list rebuild, no retry
      const pp_status st = m == 0 ? PP_OK
                                  : run_solve(*c, false, c->res.exact_lists, src, m, tx, ty, *prm, p_out,
                                              (hipStream_t)stream, true);
      if (st != PP_OK) throw PPError{st, "resident solve failed"};
      c->err.clear();
      return st;
    }
    if (m == 0) return PP_OK;
    // A solve is repeated (at most a few times) when the traversal frontier
    // overflowed below its top tier, or when a one-pass list outgrew its per-cell
    // capacity (then exactly, with room made for next time).
    bool exact = c->exact_lists;
    pp_status st = PP_OK;
    for (;;) {
      try {
        st = run_solve(*c, direct, exact, src, m, tx, ty, *prm, p_out, (hipStream_t)stream, false, batch);
      } catch (const FrontierRetry&) {
        continue;
      }
      if (st != PP_ERR_LIMIT || exact) break;
      if (prm->method == PP_METHOD_TREECODE) {
        c->cap_m2p *= 2;
        c->cap_tp2p *= 2;
      } else {
        c->cap_m2l *= 2;
        c->cap_p2p *= 2;
      }
      exact = true;
    }
    c->err.clear();
    return st;
  } catch (const PPError& e) {
    c->err = e.msg;
    if (e.code == PP_ERR_DEVICE) c->dead = true;
    c->last.valid = false;
    return e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    c->last.valid = false;
    return PP_ERR_DEVICE;
  }
}

Sources grid_sources(int32_t nx, int32_t ny, double x0, double y0, double h, const double* f) {
  Sources q;
  q.grid = true;
  q.nx = nx;
  q.ny = ny;
  q.x0 = x0;
  q.y0 = y0;
  q.h = h;
  q.f = f;
  return q;
}

Sources point_sources(int64_t n, const double* sx, const double* sy, const double* w) {
  Sources q;
  q.grid = false;
  q.n = n;
  q.sx = sx;
  q.sy = sy;
  q.w = w;
  return q;
}

}  // namespace

extern "C" {

pp_status pp_create(int32_t device, uint64_t hbm_budget_bytes, pp_ctx** out) {
  if (!out) return PP_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
    (void)hipGetLastError();
    return PP_ERR_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return PP_ERR_DEVICE;
  pp_ctx* c = new pp_ctx();
  c->device = device;
  if (const char* e = std::getenv("PP_P2P_PARTS")) c->p2p_parts = std::min(kMaxNearParts, std::max(1, std::atoi(e)));
  if (const char* e = std::getenv("PP_EXACT_LISTS")) c->exact_lists = std::atoi(e) != 0;
  if (const char* e = std::getenv("PP_DIRECT_ISSUE")) c->direct_issue = std::atoi(e) != 0;
  if (const char* e = std::getenv("PP_DENSE_LEVELS")) c->dense_levels = std::min(9, std::max(0, std::atoi(e)));
  if (const char* e = std::getenv("PP_LAZY_PACK")) c->lazy_pack = std::atoi(e) != 0;
  if (const char* e = std::getenv("PP_RESIDENT_GRAPH")) c->resident_graph = std::atoi(e) != 0;
  if (const char* e = std::getenv("PP_P2M_LATTICE")) c->p2m_lattice_min = std::max(0LL, std::atoll(e));
  if (const char* e = std::getenv("PP_GRAPHS")) c->graphs = std::atoi(e) != 0;
  if (const char* e = std::getenv("PP_NEAR_STREAM")) c->near_stream = std::atoi(e) != 0;
  if (const char* e = std::getenv("PP_LIST_CAPS")) {  // "m2l,p2p[,m2p,tree-code p2p]" initial capacities
    int a = 0, b = 0, x = 0, y = 0;
    const int got = std::sscanf(e, "%d,%d,%d,%d", &a, &b, &x, &y);
    if (got >= 2 && a > 0 && b > 0) {
      c->cap_m2l = a;
      c->cap_p2p = b;
    }
    if (got == 4 && x > 0 && y > 0) {
      c->cap_m2p = x;
      c->cap_tp2p = y;
    }
  }
  c->budget = hbm_budget_bytes;
  if (hipHostMalloc((void**)&c->pinned, (kMiscInts + kMailExtra) * sizeof(int), hipHostMallocCoherent) !=
      hipSuccess) {
    delete c;
    return PP_ERR_DEVICE;
  }
  std::memset(c->pinned, 0, (kMiscInts + kMailExtra) * sizeof(int));
  // set-up of the allocation-free entry point: this device's workspace address,
  // and the stream that calls on the null stream use (created here, not there)
  c->scratch_ptr = scratch_address(device);
  if (!c->scratch_ptr || hipStreamCreate(&c->own_stream) != hipSuccess) {
    (void)hipHostFree(c->pinned);
    delete c;
    return PP_ERR_DEVICE;
  }
  const int zeros[64] = {};
  if (hipMalloc((void**)&c->pub_ctr, sizeof(zeros)) != hipSuccess ||
      hipMemcpy(c->pub_ctr, zeros, sizeof(zeros), hipMemcpyHostToDevice) != hipSuccess) {
    if (c->pub_ctr) (void)hipFree(c->pub_ctr);
    (void)hipStreamDestroy(c->own_stream);
    (void)hipHostFree(c->pinned);
    delete c;
    return PP_ERR_DEVICE;
  }
  *out = c;
  return PP_OK;
}

void pp_destroy(pp_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (auto& g : c->seg) drop_graph(g);
  if (c->own_stream) (void)hipStreamDestroy(c->own_stream);
  if (c->side_stream) (void)hipStreamDestroy(c->side_stream);
  for (hipEvent_t e : {c->ev_fork, c->ev_lists, c->ev_join})
    if (e) (void)hipEventDestroy(e);
  for (int i = 0; i < B_COUNT; ++i) release(*c, i);
  for (int i = 0; i < 13; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->pub_ctr) (void)hipFree(c->pub_ctr);
  if (c->log_tab) (void)hipFree(c->log_tab);
  delete c;
}

pp_status pp_solve_grid(pp_ctx* c, int32_t nx, int32_t ny, double x0, double y0, double h, const double* f, int64_t m,
                        const double* tx, const double* ty, const pp_params* params, double* p_out, void* stream) {
  return guard(c, false, grid_sources(nx, ny, x0, y0, h, f), m, tx, ty, params, p_out, stream);
}

pp_status pp_solve_grid_batch(pp_ctx* c, int32_t nreq, int32_t nx, int32_t ny, double x0, double y0, double h,
                              const double* const* f, const int64_t* m, const double* const* tx,
                              const double* const* ty, const pp_params* params, double* const* p_out, void* stream) {
  if (!c) return PP_ERR_ARG;
  auto refuse = [&](const char* why) {
    c->err = why;
    return PP_ERR_ARG;
  };
  if (nreq < 1 || nreq > kMaxBatch || !f || !m || !tx || !ty || !p_out || !params)
    return refuse("batch: 1 to 16 requests, every array given");
  if (nreq == 1) return pp_solve_grid(c, nx, ny, x0, y0, h, f[0], m[0], tx[0], ty[0], params, p_out[0], stream);
  if (params->method != PP_METHOD_FMM) return refuse("batch: the multipole method only");
  int levels = 0;
  while ((1 << (2 * levels)) < nreq) ++levels;
  const int D = root_exponent(std::max(nx, 1), std::max(ny, 1));
  if (D < 6 || D + levels > 16) return refuse("batch: grids of 33 to 65536 nodes a side, and the forest within 65536");
  if (levels > c->dense_levels) return refuse("batch: the forest's top levels must lie in the dense table");
  GridBatch b;
  b.nreq = nreq;
  b.levels = levels;
  b.D = D;
  int64_t M = 0;
  for (int r = 0; r < nreq; ++r) {
    if (m[r] < 0) return refuse("batch: negative target count");
    if (!f[r] || !is_device_ptr(f[r]) || (m[r] > 0 && (!tx[r] || !ty[r] || !p_out[r] || !is_device_ptr(tx[r]) ||
                                                       !is_device_ptr(ty[r]) || !is_device_ptr(p_out[r]))))
      return refuse("batch: device memory only, every pointer given");
    b.f[r] = f[r];
    b.tx[r] = tx[r];
    b.ty[r] = ty[r];
    b.out[r] = p_out[r];
    b.toff[r] = M;
    M += m[r];
  }
  b.toff[nreq] = M;
  if (M >= ((int64_t)1 << 31)) return refuse("batch: too many targets");
  int r0 = 0;  // a request with targets stands for the batch in the argument checks
  while (r0 + 1 < nreq && m[r0] == 0) ++r0;
  return guard(c, false, grid_sources(nx, ny, x0, y0, h, f[0]), M, tx[r0], ty[r0], params, p_out[r0], stream, false,
               &b);
}

pp_status pp_solve_grid_noalloc(pp_ctx* c, int32_t nx, int32_t ny, double x0, double y0, double h,
                                const double* f, int64_t m, const double* tx, const double* ty,
                                const pp_params* params, double* p_out, void* stream) {
  if (!c) return PP_ERR_ARG;
  if ((f && !is_device_ptr(f)) || (m > 0 && ((tx && !is_device_ptr(tx)) || (ty && !is_device_ptr(ty)) ||
                                              (p_out && !is_device_ptr(p_out))))) {
    c->err = "the allocation-free solve takes device memory only (no staging copies)";
    return PP_ERR_ARG;
  }
  c->arena = true;
  c->arena_base = (char*)c->scratch_ptr;
  const pp_status st = guard(c, false, grid_sources(nx, ny, x0, y0, h, f), m, tx, ty, params, p_out, stream);
  c->arena = false;
  return st;
}

pp_status pp_solve_grid_resident(pp_ctx* c, const double* f, const double* tx, const double* ty, double* p_out,
                                 void* stream) {
  if (!c) return PP_ERR_ARG;
  if (!c->res.valid) {
    c->err = "no retained tree: the last call on this context was not a successful pp_solve_grid";
    return PP_ERR_ARG;
  }
  const Resident R = c->res;
  return guard(c, false, grid_sources(R.nx, R.ny, R.x0, R.y0, R.h, f), R.m, tx, ty, &R.prm, p_out, stream, true);
}

pp_status pp_solve_points(pp_ctx* c, int64_t n, const double* sx, const double* sy, const double* w, int64_t m,
                          const double* tx, const double* ty, const pp_params* params, double* p_out, void* stream) {
  return guard(c, false, point_sources(n, sx, sy, w), m, tx, ty, params, p_out, stream);
}

pp_status pp_direct_points(pp_ctx* c, int64_t n, const double* sx, const double* sy, const double* w, int64_t m,
                           const double* tx, const double* ty, const pp_params* params, double* p_out, void* stream) {
  return guard(c, true, point_sources(n, sx, sy, w), m, tx, ty, params, p_out, stream);
}

pp_status pp_direct_grid(pp_ctx* c, int32_t nx, int32_t ny, double x0, double y0, double h, const double* f, int64_t m,
                         const double* tx, const double* ty, const pp_params* params, double* p_out, void* stream) {
  return guard(c, true, grid_sources(nx, ny, x0, y0, h, f), m, tx, ty, params, p_out, stream);
}

}  // extern "C"

namespace {
void validate_segments(int64_t m, int32_t nseg, const int64_t* seg_start, double ux, double uy, double rho,
                       double area) {
  if (m < 0 || nseg < 1 || !seg_start) throw PPError{PP_ERR_ARG, "bad sizes or null segment offsets"};
  if (is_device_ptr(seg_start)) throw PPError{PP_ERR_ARG, "seg_start must be host memory"};
  if (seg_start[0] != 0 || seg_start[nseg] != m) throw PPError{PP_ERR_ARG, "seg_start must run from 0 to m"};
  for (int i = 0; i < nseg; ++i)
    if (seg_start[i + 1] < seg_start[i]) throw PPError{PP_ERR_ARG, "seg_start decreases"};
  const double speed = std::hypot(ux, uy);
  if (!(speed > 0.0) || !std::isfinite(speed) || !(rho > 0.0) || !(area > 0.0) || !std::isfinite(rho) ||
      !std::isfinite(area))
    throw PPError{PP_ERR_ARG, "|U|, rho and area must be positive and finite"};
}

// Stages the per-panel outputs and the segment table, runs `launch`, copies results to host buffers.
template <class Launch>
void run_force_kernel(pp_ctx& c, int64_t m, int32_t nseg, const int64_t* seg_start, double* dfx, double* dfy,
                      pp_force* out, hipStream_t s, Launch launch) {
  int64_t* seg_d = ensure<int64_t>(c, B_FSEG, nseg + 1);
  HIPCHK(hipMemcpyAsync(seg_d, seg_start, (size_t)(nseg + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
  const bool dfx_dev = dfx && is_device_ptr(dfx), dfy_dev = dfy && is_device_ptr(dfy);
  const bool out_dev = is_device_ptr(out);
  double* dfx_d = dfx ? (dfx_dev ? dfx : ensure<double>(c, B_FDFX, m)) : nullptr;
  double* dfy_d = dfy ? (dfy_dev ? dfy : ensure<double>(c, B_FDFY, m)) : nullptr;
  pp_force* out_d = out_dev ? out : ensure<pp_force>(c, B_FOUT, nseg);
  launch(seg_d, dfx_d, dfy_d, out_d);
  HIPCHK(hipGetLastError());
  if (dfx && !dfx_dev && m > 0) HIPCHK(hipMemcpyAsync(dfx, dfx_d, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
  if (dfy && !dfy_dev && m > 0) HIPCHK(hipMemcpyAsync(dfy, dfy_d, (size_t)m * sizeof(double), hipMemcpyDeviceToHost, s));
  if (!out_dev) HIPCHK(hipMemcpyAsync(out, out_d, (size_t)nseg * sizeof(pp_force), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
}

}  // namespace

void pp::ctx_set_near_stream(pp_ctx* c, bool on) {
  if (c) c->near_stream = on;
}

size_t pp::ctx_held_bytes(const pp_ctx* c) { return c ? c->held : 0; }

void pp::ctx_trim(pp_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  for (auto& g : c->seg) drop_graph(g);
  for (int i = 0; i < B_COUNT; ++i) release(*c, i);
  c->gen += 1;
  c->last.valid = false;
  c->res.valid = false;
}

namespace {

// A call that failed after forking the near field must not return while that
// launch may still use the context's buffers.
void drain_side(pp_ctx* c) {
  if (c->side_stream) (void)hipStreamSynchronize(c->side_stream);
  if (c->cur_stream) (void)hipStreamSynchronize(c->cur_stream);
  c->cur_stream = nullptr;
}

template <class Body>
pp_status guarded(pp_ctx* c, Body body) {
  if (!c) return PP_ERR_ARG;
  if (c->dead) {
    c->err = "context is unusable after a device error";
    return PP_ERR_DEVICE;
  }
  try {
    body();
    c->err.clear();
    return PP_OK;
  } catch (const PPError& e) {
    c->err = e.msg;
    if (e.code == PP_ERR_DEVICE) c->dead = true;
    drain_side(c);
    return e.code;
  } catch (const std::exception& e) {
    c->err = e.what();
    drain_side(c);
    return PP_ERR_DEVICE;
  }
}
}  // namespace

extern "C" {

pp_status pp_pressure_source(pp_ctx* c, int32_t nx, int32_t ny, double h, const double* u, const double* v,
                             double rho, double lambda, const double* chi, const double* us, const double* vs,
                             double* f_out, void* stream) {
  return guarded(c, [&] {
    if (nx < 1 || ny < 1 || nx > 65536 || ny > 65536 || (int64_t)nx * ny >= ((int64_t)1 << 31))
      throw PPError{PP_ERR_ARG, "grid size out of range"};
    if (!(h > 0.0) || !std::isfinite(h) || !std::isfinite(rho) || !std::isfinite(lambda))
      throw PPError{PP_ERR_ARG, "h must be positive, rho and lambda finite"};
    if (!u || !v || !f_out) throw PPError{PP_ERR_ARG, "null velocity or output"};
    const bool pen = chi || us || vs;
    if (pen && !(chi && us && vs)) throw PPError{PP_ERR_ARG, "chi, us and vs must be given together"};
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)nx * ny;
    int* misc = ensure<int>(*c, B_MISC, kMiscInts);
    fill_i32(misc, 0, kMiscInts, s);
    const double* u_d = stage_in(*c, B_AU, u, n, s);
    const double* v_d = stage_in(*c, B_AV, v, n, s);
    const double* chi_d = pen ? stage_in(*c, B_ACHI, chi, n, s) : nullptr;
    const double* us_d = pen ? stage_in(*c, B_AUS, us, n, s) : nullptr;
    const double* vs_d = pen ? stage_in(*c, B_AVS, vs, n, s) : nullptr;
    const bool out_dev = is_device_ptr(f_out);
    double* f_d = out_dev ? f_out : ensure<double>(*c, B_AF, n);
    pressure_source(u_d, v_d, chi_d, us_d, vs_d, nx, ny, h, rho, lambda, f_d, misc + M_FLAGS, s);
    HIPCHK(hipGetLastError());
    readback(*c, misc, 0, 1, s);
    if (c->pinned[M_FLAGS]) throw PPError{PP_ERR_ARG, "non-finite velocity data (the source is not finite)"};
    if (!out_dev) {
      HIPCHK(hipMemcpyAsync(f_out, f_d, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
  });
}

pp_status pp_viscous_forces(pp_ctx* c, int32_t nx, int32_t ny, double x0, double y0, double h, const double* u,
                            const double* v, int64_t m, const double* lx, const double* ly, const double* pnx,
                            const double* pny, const double* ds, int32_t nseg, const int64_t* seg_start, double mu,
                            double ux, double uy, double rho, double area, double* dfx, double* dfy, pp_force* out,
                            void* stream) {
  return guarded(c, [&] {
    if (nx < 1 || ny < 1 || nx > 65536 || ny > 65536 || (int64_t)nx * ny >= ((int64_t)1 << 31))
      throw PPError{PP_ERR_ARG, "grid size out of range"};
    if (!(h > 0.0) || !std::isfinite(h) || !std::isfinite(x0) || !std::isfinite(y0) || !std::isfinite(mu))
      throw PPError{PP_ERR_ARG, "h must be positive, x0, y0 and mu finite"};
    if (!u || !v || !out || (m > 0 && (!lx || !ly || !pnx || !pny || !ds)))
      throw PPError{PP_ERR_ARG, "null pointer"};
    validate_segments(m, nseg, seg_start, ux, uy, rho, area);
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)nx * ny;
    const double* u_d = stage_in(*c, B_AU, u, n, s);
    const double* v_d = stage_in(*c, B_AV, v, n, s);
    const double* lx_d = stage_in(*c, B_VLX, lx, m, s);
    const double* ly_d = stage_in(*c, B_VLY, ly, m, s);
    const double* nx_d = stage_in(*c, B_FNX, pnx, m, s);
    const double* ny_d = stage_in(*c, B_FNY, pny, m, s);
    const double* ds_d = stage_in(*c, B_FDS, ds, m, s);
    run_force_kernel(*c, m, nseg, seg_start, dfx, dfy, out, s,
                     [&](const int64_t* seg_d, double* dfx_d, double* dfy_d, pp_force* out_d) {
                       viscous_forces(u_d, v_d, nx, ny, x0, y0, h, lx_d, ly_d, nx_d, ny_d, ds_d, nseg, seg_d, mu, ux,
                                      uy, rho, area, dfx_d, dfy_d, out_d, s);
                     });
  });
}

pp_status pp_surface_forces(pp_ctx* c, int64_t m, const double* p, const double* nx, const double* ny,
                            const double* ds, int32_t nseg, const int64_t* seg_start, double ux, double uy, double rho,
                            double area, double* dfx, double* dfy, pp_force* out, void* stream) {
  return guarded(c, [&] {
    if (!out || (m > 0 && (!p || !nx || !ny || !ds))) throw PPError{PP_ERR_ARG, "null pointer"};
    validate_segments(m, nseg, seg_start, ux, uy, rho, area);
    HIPCHK(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const double* p_d = stage_in(*c, B_FP, p, m, s);
    const double* nx_d = stage_in(*c, B_FNX, nx, m, s);
    const double* ny_d = stage_in(*c, B_FNY, ny, m, s);
    const double* ds_d = stage_in(*c, B_FDS, ds, m, s);
    run_force_kernel(*c, m, nseg, seg_start, dfx, dfy, out, s,
                     [&](const int64_t* seg_d, double* dfx_d, double* dfy_d, pp_force* out_d) {
                       surface_forces(p_d, nx_d, ny_d, ds_d, nseg, seg_d, ux, uy, rho, area, dfx_d, dfy_d, out_d, s);
                     });
  });
}

pp_status pp_set_profiling(pp_ctx* c, int32_t on) {
  if (!c || on < 0 || (on > 2 && on < 16) || on >= 16 + 12) return PP_ERR_ARG;
  if (on && !c->profiling) {
    if (hipSetDevice(c->device) != hipSuccess) return PP_ERR_DEVICE;
    for (int i = 0; i < 13; ++i) {
      if (!c->ev[i] && hipEventCreate(&c->ev[i]) != hipSuccess) return PP_ERR_DEVICE;
    }
  }
  c->profiling = on;
  return PP_OK;
}

pp_status pp_get_stats(const pp_ctx* c, pp_stats* out) {
  if (!c || !out) return PP_ERR_ARG;
  *out = c->stats;
  return PP_OK;
}

pp_status pp_debug_copy(const pp_ctx* cc, int32_t what, void* dst, int64_t capacity, int64_t* length) {
  if (!cc || (capacity > 0 && !dst)) return PP_ERR_ARG;
  pp_ctx* c = const_cast<pp_ctx*>(cc);
  if (!c->last.valid) {
    c->err = "no successful solve to inspect";
    return PP_ERR_ARG;
  }
  const Last& L = c->last;
  int id = -1;
  int64_t n = 0;
  size_t esz = 4;
  switch (what) {
    case PP_ARR_SRC_KEY: id = B_SKEY; n = L.n_src; break;
    case PP_ARR_SRC_INDEX: id = B_SIJ; n = L.n_src; break;
    case PP_ARR_TGT_KEY: id = B_TKEY; n = L.m; break;
    case PP_ARR_TGT_PERM: id = B_TPERM; n = L.m; break;
    case PP_ARR_CELL_LEVEL: id = B_LVL; n = L.ncells; break;
    case PP_ARR_CELL_IX: id = B_IX; n = L.ncells; break;
    case PP_ARR_CELL_IY: id = B_IY; n = L.ncells; break;
    case PP_ARR_CELL_SB: id = B_SB; n = L.ncells; break;
    case PP_ARR_CELL_SE: id = B_SE; n = L.ncells; break;
    case PP_ARR_CELL_TB: id = B_TB; n = L.ncells; break;
    case PP_ARR_CELL_TE: id = B_TE; n = L.ncells; break;
    case PP_ARR_CELL_CHILD: id = B_CHILD; n = L.ncells; break;
    case PP_ARR_CELL_NCHILD: id = B_NCHILD; n = L.ncells; break;
    case PP_ARR_CELL_PARENT: id = B_PARENT; n = L.ncells; break;
    case PP_ARR_M2L_OFF: id = L.has_expansions ? B_OM2L : -1; n = L.ncells; break;
    case PP_ARR_M2L_CNT: id = L.has_expansions ? B_CM2L : -1; n = L.ncells; break;
    case PP_ARR_M2L_SRC: id = L.has_expansions ? B_M2LSRC : -1; n = L.n_m2l; break;
    case PP_ARR_P2P_OFF: id = L.has_expansions ? B_OP2P : -1; n = L.ncells; break;
    case PP_ARR_P2P_CNT: id = L.has_expansions ? B_CP2P : -1; n = L.ncells; break;
    case PP_ARR_P2P_SRC: id = L.has_expansions ? B_P2PSRC : -1; n = L.n_p2p; break;
    case PP_ARR_MULTIPOLE: id = L.has_expansions ? B_MP : -1; n = (int64_t)L.ncells * (L.p + 1) * 2; esz = 8; break;
    case PP_ARR_LOCAL: id = L.has_locals ? B_LOC : -1; n = (int64_t)L.ncells * (L.p + 1) * 2; esz = 8; break;
    case PP_ARR_FAR: id = L.has_expansions ? B_FAR : -1; n = L.m; esz = 8; break;
    case PP_ARR_NEAR: id = B_NEAR; n = L.m * L.nparts; esz = 8; break;
    case PP_ARR_TGT_LEAF: id = B_TGTLEAF; n = L.m; break;
    default: c->err = "unknown array id"; return PP_ERR_ARG;
  }
  if (id < 0) {
    c->err = "array not produced by the last call";
    return PP_ERR_ARG;
  }
  if (length) *length = n;
  const int64_t cnt = std::min(n, std::max<int64_t>(capacity, 0));
  if (cnt <= 0) return PP_OK;
  DevBuf* bufs = L.arena ? c->abufs : c->bufs;
  if (what == PP_ARR_SRC_KEY && L.keys_from_ij) {
    if (hipSetDevice(c->device) != hipSuccess) {
      c->err = "copy failed";
      return PP_ERR_DEVICE;
    }
    keys_from_ij((const uint32_t*)bufs[B_SIJ].p, nullptr, n, (uint32_t*)bufs[B_SKEY].p, nullptr);
    if (hipDeviceSynchronize() != hipSuccess) {
      c->err = "forming the source keys failed";
      return PP_ERR_DEVICE;
    }
  }
  if (hipSetDevice(c->device) != hipSuccess ||
      hipMemcpy(dst, (L.arena ? c->abufs : c->bufs)[id].p, (size_t)cnt * esz, hipMemcpyDeviceToHost) != hipSuccess) {
    c->err = "copy failed";
    return PP_ERR_DEVICE;
  }
  return PP_OK;
}

const char* pp_status_string(pp_status s) {
  switch (s) {
    case PP_OK: return "ok";
    case PP_ERR_ARG: return "invalid argument";
    case PP_ERR_DOMAIN: return "target outside the root square";
    case PP_ERR_NOMEM: return "device-memory budget exceeded";
    case PP_ERR_DEVICE: return "device error";
    case PP_ERR_LIMIT: return "internal limit exceeded";
    case PP_ERR_TIMEOUT: return "timed out";
    case PP_ERR_CANCELLED: return "cancelled";
    case PP_ERR_BUSY: return "already started";
    default: return "unknown status";
  }
}

const char* pp_last_error(const pp_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
