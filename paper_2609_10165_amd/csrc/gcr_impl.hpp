// gcr_impl.hpp -- host-side internals shared by the library's translation
// units: the plan and batch objects, the device memory pool, error helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <vector>

#include "../../include/gcr.h"
#include "gcr_device.hpp"

namespace gcr {

constexpr int kStages = 13;   // plan-build stages timed by gcr_last_build_times


// Per-instance results of plan building, written by the device.
struct InstInfo {
  uint32_t err;
  int32_t nlev;
  int32_t nunits;
  int32_t maxunit;
  int32_t maxwidth;
  int32_t nfluid;
  int32_t rmax[3];      // largest stencil multiplier per axis
  int32_t layered;      // set when the LDS layering finished the instance
  unsigned long long max_alpha_bits[3];
};

// Device memory pool: power-of-two size classes, blocks are kept for reuse
// until the process ends, so rebuilding plans does not call hipMalloc.
void* pool_alloc(size_t bytes);
void* pinned_alloc(size_t bytes);
void pinned_free(void* p);
// pooled events without timing (event_give after the last wait on one)
hipEvent_t event_take();
void event_give(hipEvent_t e);

// Pinned staging block of one plan build.  Until `pending` is cleared, an
// exit synchronises the stream first, so no queued copy still uses the block
// when it returns to the pool.
struct PinnedStage {
  char* p = nullptr;
  hipStream_t st = nullptr;
  bool pending = false;
  ~PinnedStage() {
    if (pending) (void)hipStreamSynchronize(st);
    pinned_free(p);
  }
};
void pool_free(void* p);

template <class T>
T* palloc(size_t n) {
  return static_cast<T*>(pool_alloc(sizeof(T) * (n ? n : 1)));
}

// Owner of every device array of one batch of plans (a single plan is a
// batch of one).  Ghost-indexed arrays are concatenated over instances and
// structure-of-arrays with stride `cap`.
struct BatchData {
  int ninst = 0;
  int64_t ncells_total = 0, nchunks = 0, nif = 0, cap = 0, ng_total = 0;
  int64_t nband = 0;                 // row segments tested by the band pass
  std::vector<Inst> inst;            // host copies
  std::vector<int64_t> if_off, g_off;  // host [ninst+1]
  std::vector<int64_t> iface_off;      // host [ninst+1] interface cells alone
  std::vector<InstInfo> info;        // host [ninst]
  std::vector<int32_t> lev_off;      // host [ninst][kMaxLevels+1]
  // device
  Inst* d_inst = nullptr;
  int8_t* d_tags = nullptr;
  int64_t* d_chunk_start = nullptr;  // [ninst+1]
  int32_t* d_chunk_cnt = nullptr;
  int8_t* d_span = nullptr;          // [chunks * 4] settled flag of each wave's span
  int32_t* d_chunk_list = nullptr;   // chunks holding interface cells, ascending
  int32_t* d_nchunk_list = nullptr;
  int32_t* d_band = nullptr;         // band masks of the chunks (classification scratch)
  int32_t* d_chunk_inst = nullptr;   // instance of each chunk
  int32_t* d_nband = nullptr;        // their number
  int32_t* d_dirty = nullptr;        // chunks the store pass classifies (flags, then list)
  int32_t* d_dirty_list = nullptr;
  int32_t* d_ndirty = nullptr;
  int64_t* d_scan_tmp = nullptr;     // tile totals of the long chunk scan
  int64_t* d_iface_off = nullptr;    // interface cells per instance (second layer)
  int64_t* d_chunk_excl = nullptr;
  int64_t* d_if_off = nullptr;       // [ninst+1]
  int64_t* d_g_off = nullptr;        // [ninst+1]
  InstInfo* d_info = nullptr;
  int32_t* d_lev_off = nullptr;      // [ninst][kMaxLevels+1]
  // interface cells
  int32_t* d_if_cell = nullptr;
  double* d_if_psi = nullptr;
  double* d_if_n = nullptr;          // [3][cap]
  uint8_t* d_if_flag = nullptr;
  int32_t* d_blkcnt = nullptr;
  int64_t* d_blkexcl = nullptr;
  // ghosts, linear-index order
  int32_t* d_g_cell = nullptr;
  uint8_t* d_g_ext = nullptr;        // ghost on the extended stencil (second layer)
  double* d_g_psi = nullptr;
  double* d_g_n = nullptr;           // [3][cap]
  uint32_t* d_g_code = nullptr;
  int32_t* d_deps = nullptr;         // [7][cap]
  int32_t* d_lev = nullptr;
  int32_t* d_blk_idx = nullptr;
  int32_t* d_perm = nullptr;         // linear-order position -> canonical (instance-local)
  // ghosts, canonical order
  int32_t* d_cell = nullptr;
  double* d_delta = nullptr;         // [3][cap]
  double* d_nrm = nullptr;           // [3][cap]
  double* d_psi = nullptr;
  uint32_t* d_code = nullptr;
  int32_t* d_level = nullptr;
  int32_t* d_blk = nullptr;
  int32_t* d_unit_mem = nullptr;     // [ninst][kMaxUnits][kMaxUnit]
  int32_t* d_unit_cnt = nullptr;     // [ninst][kMaxUnits]
  int32_t* d_unit_lev = nullptr;     // [ninst][kMaxUnits] level of each unit
  uint32_t* d_reach = nullptr;       // [ninst] residual closure bitsets (cyclic graphs)
  int32_t* d_listA = nullptr;        // [cap] level lists of the layering
  int32_t* d_rcnt = nullptr;         // [2][cap] reverse-edge counts, fill pointers
  int32_t* d_roff = nullptr;         // [cap+1] reverse-edge offsets (all ghosts)
  int32_t* d_radj = nullptr;         // [7][cap] reverse edges (linear-order ghost ids)
  uint8_t* d_dcnt = nullptr;         // [cap] ghost dependencies per ghost
  uint32_t* d_cnt = nullptr;         // byte counters in HBM (instances beyond LDS)
  uint32_t* d_bits = nullptr;        // level bitmaps in HBM (instances beyond LDS)
  std::vector<int32_t> unit_lev;     // host copy
  // cell -> ghost hash tables, concatenated per instance
  unsigned long long* d_htab = nullptr;
  int64_t* d_hoff = nullptr;
  uint32_t* d_hmask = nullptr;
  std::vector<int64_t> hoff;
  std::vector<uint32_t> hmask;
  std::vector<void*> owned;
  char* arena_cur = nullptr;         // bump allocator over pooled chunks
  size_t arena_left = 0;
  ~BatchData();
};

// Arguments of the layering kernel (levels.hip).
struct LevelsArgs {
  const Inst* insts;
  const int64_t* g_off;
  const int32_t* deps;
  int64_t cap;
  int32_t* lev;
  int32_t* blk_idx;
  int32_t* perm;
  int32_t* lev_off;
  int32_t* unit_mem;
  int32_t* unit_cnt;
  int32_t* unit_lev;
  uint32_t* reach;
  int32_t* listA;
  const uint8_t* dcnt;
  const int32_t* roff;
  const int32_t* radj;
  uint32_t* cnt;
  uint32_t* bits;
  InstInfo* info;
  // wide layering of a single large instance (null: not used)
  int32_t* listB;        // [cap] second level list
  int32_t* wide;         // [kWideState] completion flag, sizes of the levels
  int32_t* hist;         // [kWideLevels][cap / 256 + 1] per-tile level counts
  int cur_cap;           // entries of a level list held in LDS (set at launch)
  int wave_res;          // residuals up to this size go to the one-wave solver
  int wide_cap;          // entries of the wide layering's per-workgroup release buffer
};
constexpr int kWideBuf = 4096;   // its LDS capacity
constexpr int kWideLevels = 128;               // deepest graph the wide layering orders
constexpr int kWideState = kWideLevels + 8;
constexpr int64_t kWideMinInterface = 65536;   // default; smaller instances: one workgroup
void set_wide_layering(int64_t min_interface);   // 0: the default
int64_t wide_layering_min();
constexpr int kWaveResidual = 64;   // most ghosts left by Kahn that one wave resolves
void set_wave_residual(int max_ghosts);
int wave_residual();
void set_wide_buffer(int entries);   // 0: the default (kWideBuf)
int wide_buffer();
bool wide_layering_forced();         // a threshold set explicitly
gcr_status launch_levels(const LevelsArgs& L, int ninst, int64_t max_n, hipStream_t st);

// Classification of every cell of a batch into tags (0 fluid, 1 solid, 0x40
// interface mark) and per-chunk interface counts; chunk_inst [chunks]
// receives each chunk's instance, band [chunks][8] is scratch.  ev_prepass / ev_store
// (either may be null) are recorded after the span pre-pass and after the
// store pass.
//
// The chunks the span pass leaves (or, with U, those a move can change)
// are flagged in W.flag [chunks] and listed in W.list[0, *W.nlist),
// ascending.  With U (a re-plan of a single instance whose tags hold the
// previous plan's): only the chunks the move can change are classified
// again, those with a span unsettled now or settled differently before,
// and those holding a ghost of the previous plan.
struct ClassifyWork {
  int32_t* flag;               // [chunks]
  int32_t* list;               // [chunks]
  int32_t* nlist;              // [1]
  int64_t* scan_excl;          // [chunks + 1] scan scratch
  int64_t* scan_tmp;           // scan tile totals
  bool every_chunk;            // full build: the store pass takes every chunk (2D grids)
};
struct ClassifyUpdate {
  const int8_t* span_prev;     // [chunks * 4] the previous plan's span flags
  const int32_t* ghost_prev;   // [ng_prev] the previous plan's ghost cells
  int64_t ng_prev;
};
constexpr int kListGrid = 32768;   // workgroups striding over a chunk list (one entry each below)
void launch_classify(const Inst* insts, int ninst, const int64_t* chunk_start, int64_t chunks,
                     int8_t* span, int32_t* chunk_inst, int8_t* tags, int32_t* chunk_cnt,
                     int32_t* band, int32_t* nband, hipEvent_t ev_prepass, hipEvent_t ev_store,
                     hipStream_t st, const ClassifyWork& W,
                     const ClassifyUpdate* U = nullptr);


// instance holding global index x of a batch: the last i with off[i] <= x
__device__ __forceinline__ int find_inst(const int64_t* off, int ninst, int64_t x) {
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Schedule of the fill.
enum { kSchedAuto = 0, kSchedLevels = 1, kSchedWorkgroup = 2, kSchedGraph = 3 };
constexpr int kScratchSlots = 7;

struct GraphCache;

}  // namespace gcr

// A plan: a view of one instance of a BatchData.
struct gcr_plan {
  std::shared_ptr<gcr::BatchData> batch;
  int index = 0;
  gcr::Inst inst;          // host copy
  int dim = 0;
  int64_t ncell = 0, ng = 0, nif = 0, stride = 0, goff = 0;
  int32_t nlev = 0;
  gcr::InstInfo info{};
  std::vector<int32_t> lev_off;   // host [nlev+1]
  // device views
  int8_t* tags = nullptr;
  const int8_t* span = nullptr;     // span flags of the plan's chunks (4 a chunk)
  int32_t* cell = nullptr;
  double* delta[3] = {nullptr, nullptr, nullptr};
  double* nrm[3] = {nullptr, nullptr, nullptr};
  double* psi = nullptr;
  uint32_t* code = nullptr;
  int32_t* level = nullptr;
  int32_t* blk = nullptr;
  int32_t* unit_mem = nullptr;
  int32_t* unit_cnt = nullptr;
  int32_t* sorted_cell = nullptr;   // ghost cells in linear-index order
  int32_t* sorted_pos = nullptr;    // their canonical positions
  int32_t* d_lev_off = nullptr;
  int32_t* unit_lev = nullptr;      // device [nunits]
  std::vector<int32_t> unit_lev_host;
  unsigned long long* htab = nullptr;
  uint32_t hmask = 0;
  int schedule = gcr::kSchedAuto;
  int tuned = -1;                   // schedule picked by the tuner
  // scratch buffers owned by the plan (forces partials, adjoint state);
  // calls that use them must not overlap on one plan
  void* scr[gcr::kScratchSlots] = {};
  size_t scr_bytes[gcr::kScratchSlots] = {};
  // ghost weights per boundary-condition kind, [2][8][ng], computed on first use
  double* wts = nullptr;
  bool wts_ok[2] = {false, false};
  // transposed stencil of the adjoints, built on first use (adjoint.hip)
  void* sup = nullptr;
  int64_t sup_bound = 0;
  uint32_t sup_hmask = 0;
  std::unique_ptr<gcr::GraphCache> graph;
  // set when a re-plan failed and the plan could not be rebuilt as it was:
  // every call but destroy then returns GCR_E_ARG
  bool dead = false;
  ~gcr_plan();
};

inline bool plan_ok(const gcr_plan* p) { return p && !p->dead; }

namespace gcr {
// Cached ghost weights of plan p for the kinds used (capi.hip).
gcr_status plan_weights(gcr_plan* p, int nf, const int* kind, const double* w[2],
                        hipStream_t st);
}  // namespace gcr

struct gcr_batch {
  std::shared_ptr<gcr::BatchData> data;
  std::vector<std::unique_ptr<gcr_plan>> plans;
  void* fwd_args = nullptr;         // device table for the batched forward
  size_t fwd_args_bytes = 0;
  ~gcr_batch();
};

namespace gcr {

gcr_status build_batch(int ninst, const gcr_grid* grids, const gcr_shape* shapes,
                       const int32_t* schemes, hipStream_t st, std::shared_ptr<BatchData>* out);
// A plan of prev's single instance (same grid, scheme and second layer) for
// the body `shape`.  incremental: prev's tags are taken over (prev is left
// without them, so it can no longer serve a plan) and only the chunks the
// move can change are classified again; else a full build.
gcr_status build_update(BatchData& prev, const gcr_shape& shape, bool incremental,
                        hipStream_t st, std::shared_ptr<BatchData>* out);
gcr_status build_update(BatchData& prev, const ShapeD& shape, bool incremental, hipStream_t st,
                        std::shared_ptr<BatchData>* out);
void make_plan_view(const std::shared_ptr<BatchData>& B, int i, gcr_plan* p);
void set_profiling(int mask);
int profiling_mask();   // bit 0 build stages, bit 1 batched forward
// Exclusive scan of n counts into excl[n + 1] (total last); where list is
// set, the indices with a nonzero count go there in order and their number
// to nlist[0].  tsum: ceil(n / 8192) + 1 int64 of scratch (plan.hip).
void launch_scan(const int32_t* cnt, int64_t n, int64_t* excl, int32_t* list,
                 int32_t* nlist, int64_t* tsum, hipStream_t st);
// Tiled batched fill: 0 off, 1 from a batch's second forward call (the
// default), 2 from its first (process-wide).
void set_batch_tiling(int mode);
int batch_tiling();
void set_batch_shape(int threads, int grid);
void* plan_scratch(gcr_plan* p, int slot, size_t bytes);
void last_build_times(float* ms);
gcr_status status_from_err(uint32_t err);

extern thread_local hipError_t g_last_hip_error;

}  // namespace gcr

// drops the batched-forward tables of a batch (defined with the batched kernel)
void gcr_batch_release_state(const gcr_batch* b);

#define GCR_HIP(x)                                  \
  do {                                              \
    hipError_t e_ = (x);                            \
    if (e_ != hipSuccess) {                         \
      gcr::g_last_hip_error = e_;                   \
      return GCR_E_HIP;                             \
    }                                               \
  } while (0)
