// capi.hip -- the C-ABI of libgcr: argument checks, plan objects, the
// device memory pool, fill schedules (per-level launches, single-workgroup
// sweep, per-level launches replayed from a HIP graph) and the tuner that
// picks among them by timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "gcr_apply.hpp"
#include "gcr_impl.hpp"

namespace gcr {

thread_local hipError_t g_last_hip_error = hipSuccess;

// --------------------------------------------------------------------------
// device memory pool
// --------------------------------------------------------------------------

namespace {
std::mutex g_pool_mu;
std::unordered_map<size_t, std::vector<void*>> g_free_blocks;
std::unordered_map<void*, size_t> g_live_blocks;

size_t size_class(size_t b) {
  size_t c = 256;
  while (c < b) c <<= 1;
  return c;
}
}  // namespace

void* pool_alloc(size_t bytes) {
  const size_t c = size_class(bytes);
  {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    auto& v = g_free_blocks[c];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      g_live_blocks[p] = c;
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, c) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_pool_mu);
  g_live_blocks[p] = c;
  return p;
}

void pool_free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pool_mu);
  auto it = g_live_blocks.find(p);
  if (it == g_live_blocks.end()) return;
  g_free_blocks[it->second].push_back(p);
  g_live_blocks.erase(it);
}

// Events without timing, pooled like the memory blocks (creating one per
// use costs more host time than a short kernel launch)
namespace {
std::mutex g_ev_mu;
std::vector<hipEvent_t> g_ev_free;
}  // namespace

hipEvent_t event_take() {
  {
    std::lock_guard<std::mutex> lk(g_ev_mu);
    if (!g_ev_free.empty()) {
      hipEvent_t e = g_ev_free.back();
      g_ev_free.pop_back();
      return e;
    }
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return e;
}

void event_give(hipEvent_t e) {
  if (!e) return;
  std::lock_guard<std::mutex> lk(g_ev_mu);
  g_ev_free.push_back(e);
}

// Pinned host staging blocks (hipHostMalloc), pooled like the device blocks:
// copies from and to them are asynchronous, so a plan build does not wait
// for earlier work on its stream when it uploads its tables.
namespace {
std::mutex g_pin_mu;
std::map<size_t, std::vector<void*>> g_pin_free;
std::unordered_map<void*, size_t> g_pin_live;
}  // namespace

void* pinned_alloc(size_t bytes) {
  const size_t c = size_class(bytes);
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto& v = g_pin_free[c];
    if (!v.empty()) {
      void* p = v.back();
      v.pop_back();
      g_pin_live[p] = c;
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, c, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_live[p] = c;
  return p;
}

void pinned_free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  auto it = g_pin_live.find(p);
  if (it == g_pin_live.end()) return;
  g_pin_free[it->second].push_back(p);
  g_pin_live.erase(it);
}

// --------------------------------------------------------------------------
// helpers
// --------------------------------------------------------------------------

PlanD plan_view(const gcr_plan* p) {
  PlanD P;
  std::memset(&P, 0, sizeof(P));
  P.g = p->inst.g;
  P.ng = (int)p->ng;
  P.tags = p->tags;
  P.cell = p->cell;
  for (int a = 0; a < 3; ++a) {
    P.dl[a] = p->delta[a];
    P.nn[a] = p->nrm[a];
  }
  P.code = p->code;
  P.blk = p->blk;
  P.unit_mem = p->unit_mem;
  P.unit_cnt = p->unit_cnt;
  P.sorted_cell = p->sorted_cell;
  P.sorted_pos = p->sorted_pos;
  for (int a = 0; a < 3; ++a) P.rmax[a] = a < p->dim ? std::max(1, p->info.rmax[a]) : 0;
  P.htab = p->htab;
  P.hmask = p->hmask;
  P.nunits = p->info.nunits;
  P.unit_lev = p->unit_lev;
  P.cgi = nullptr;
  return P;
}

struct GraphCache {
  hipStream_t cap = nullptr;
  std::vector<std::pair<FillArgs, hipGraphExec_t>> entries;
  ~GraphCache() {
    for (auto& e : entries) (void)hipGraphExecDestroy(e.second);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// per-level launches; a level holding coupled units gets a second, small
// launch that solves them
static void launch_levels_fill(const gcr_plan* p, const FillArgs& A, hipStream_t st) {
  for (int l = 0; l < p->nlev; ++l) {
    launch_fill_range(A, p->lev_off[l], p->lev_off[l + 1], st);
    for (int32_t ul : p->unit_lev_host)
      if (ul == l + 1) {
        launch_fill_units(A, l + 1, st);
        break;
      }
  }
}

static gcr_status fill_levels(const gcr_plan* p, const FillArgs& A, hipStream_t st) {
  launch_levels_fill(p, A, st);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

static gcr_status fill_wg(const gcr_plan* p, const FillArgs& A, hipStream_t st) {
  launch_fill_wg(A, p->d_lev_off, p->nlev, 1024, st);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

static gcr_status fill_graph(gcr_plan* p, const FillArgs& A, hipStream_t st) {
  if (!p->graph) p->graph.reset(new GraphCache());
  GraphCache& G = *p->graph;
  for (auto& e : G.entries)
    if (std::memcmp(&e.first, &A, sizeof(FillArgs)) == 0) {
      GCR_HIP(hipGraphLaunch(e.second, st));
      return GCR_OK;
    }
  if (!G.cap) GCR_HIP(hipStreamCreateWithFlags(&G.cap, hipStreamNonBlocking));
  hipGraph_t graph = nullptr;
  GCR_HIP(hipStreamBeginCapture(G.cap, hipStreamCaptureModeThreadLocal));
  launch_levels_fill(p, A, G.cap);
  GCR_HIP(hipStreamEndCapture(G.cap, &graph));
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  GCR_HIP(e);
  if (G.entries.size() >= 8) {
    (void)hipGraphExecDestroy(G.entries.front().second);
    G.entries.erase(G.entries.begin());
  }
  G.entries.emplace_back(A, exec);
  GCR_HIP(hipGraphLaunch(exec, st));
  return GCR_OK;
}

static gcr_status run_fill(gcr_plan* p, const FillArgs& A, int sched, hipStream_t st) {
  switch (sched) {
    case kSchedWorkgroup: return fill_wg(p, A, st);
    case kSchedGraph: return fill_graph(p, A, st);
    default: return fill_levels(p, A, st);
  }
}

// Tuner: times the three schedules on the caller's data (the fill is
// idempotent: ghost values depend only on non-ghost cells and boundary data)
// and remembers the winner per (dim, ghost-count bucket, level bucket, nf).
namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune_cache;
int bucket(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}
}  // namespace

constexpr int64_t kWgMaxGhosts = 8192;

static gcr_status tuned_fill(gcr_plan* p, const FillArgs& A, hipStream_t st) {
  if (p->tuned < 0) {
    auto key = std::make_tuple(p->dim, bucket(p->ng), bucket(p->nlev), A.nf);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) p->tuned = it->second;
    }
    if (p->tuned < 0) {
      hipEvent_t e0, e1;
      GCR_HIP(hipEventCreate(&e0));
      GCR_HIP(hipEventCreate(&e1));
      float best = 1e30f;
      int pick = kSchedLevels;
      const int cands[3] = {kSchedLevels, kSchedWorkgroup, kSchedGraph};
      for (int c : cands) {
        // one workgroup cannot keep up once a level spans many rounds of it
        if (c == kSchedWorkgroup && p->ng > kWgMaxGhosts) continue;
        gcr_status s = run_fill(p, A, c, st);  // warm (and graph capture)
        if (s != GCR_OK) continue;
        GCR_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 5; ++r) run_fill(p, A, c, st);
        GCR_HIP(hipEventRecord(e1, st));
        GCR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        GCR_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          pick = c;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      p->tuned = pick;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[key] = pick;
    }
  }
  return run_fill(p, A, p->tuned, st);
}

__global__ void k_export_r(const uint32_t* __restrict__ code, int ng, int dim,
                           int32_t* __restrict__ r) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < ng)
    for (int a = 0; a < dim; ++a) r[(int64_t)a * ng + p] = code_r(code[p], a);
}

// Foot points S = x_c + delta and the normals, [dim][ng] each
__global__ void k_foot_points(GridD g, const int32_t* __restrict__ cell, const double* d0,
                              const double* d1, const double* d2, const double* n0,
                              const double* n1, const double* n2, int ng,
                              double* __restrict__ S, double* __restrict__ nrm) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ng) return;
  int i, j, k;
  unlinear(g, cell[p], i, j, k);
  const double* dl[3] = {d0, d1, d2};
  const double* nn[3] = {n0, n1, n2};
  const int q[3] = {i, j, k};
  for (int a = 0; a < g.dim; ++a) {
    if (S) S[(int64_t)a * ng + p] = centre(g, a, q[a]) + dl[a][p];
    if (nrm) nrm[(int64_t)a * ng + p] = nn[a][p];
  }
}

// The same for every ghost of a batch, instances one after another: ghost p
// belongs to the last instance i with g_off[i] <= p (empty instances skipped)
__global__ void k_batch_foot_points(const Inst* __restrict__ insts, int ninst,
                                    const int64_t* __restrict__ g_off, int64_t cap,
                                    const int32_t* __restrict__ cell,
                                    const double* __restrict__ delta,
                                    const double* __restrict__ nrm_in, int dim, int64_t ng,
                                    double* __restrict__ S, double* __restrict__ nrm) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= ng) return;
  int lo = 0, hi = ninst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (g_off[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  const GridD& g = insts[lo].g;
  int q[3];
  unlinear(g, cell[p], q[0], q[1], q[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a < dim) {
      if (S) S[a * ng + p] = centre(g, a, q[a]) + delta[a * cap + p];
      if (nrm) nrm[a * ng + p] = nrm_in[a * cap + p];
    }
}

__global__ void k_export_unit(const int32_t* __restrict__ blk,
                              const int32_t* __restrict__ unit_mem, int ng,
                              int32_t* __restrict__ unit) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < ng) unit[p] = blk[p] < 0 ? -1 : unit_mem[blk[p] * kMaxUnit];
}

static bool check_fields(int32_t nf, const void* const* f) {
  if (nf < 1 || nf > kMaxFields || !f) return false;
  for (int i = 0; i < nf; ++i)
    if (!f[i]) return false;
  return true;
}

static gcr_status make_fill_args(const gcr_plan* p, int32_t nf, double* const* fields,
                                 const int32_t* bc_kind, const uint8_t* const* bc_type,
                                 const double* const* bc_val, FillArgs* A) {
  // (a plan without ghosts reads no boundary data)
  const bool reads_bc = p->ng > 0;
  if (!check_fields(nf, (const void* const*)fields) || !bc_kind || (reads_bc && !bc_val) ||
      (reads_bc && !check_fields(nf, (const void* const*)bc_val)))
    return GCR_E_ARG;
  std::memset(A, 0, sizeof(FillArgs));
  A->P = plan_view(p);
  A->nf = nf;
  for (int f = 0; f < nf; ++f) {
    if (bc_kind[f] < 0 || bc_kind[f] > 2) return GCR_E_ARG;
    if (reads_bc && bc_kind[f] == GCR_MIXED && (!bc_type || !bc_type[f])) return GCR_E_ARG;
    A->kind[f] = bc_kind[f];
    A->f[f] = fields[f];
    A->b[f] = bc_val ? bc_val[f] : nullptr;
    A->bt[f] = bc_kind[f] == GCR_MIXED && bc_type ? bc_type[f] : nullptr;
  }
  return GCR_OK;
}

// The plan's cached weights for the kinds in kind[0..nf) (computed on
// `st` the first time a kind is used); w[b] receives kind b's array.
gcr_status plan_weights(gcr_plan* p, int nf, const int* kind, const double* w[2],
                        hipStream_t st) {
  bool need[2] = {false, false};
  for (int f = 0; f < nf; ++f) {
    if (kind[f] == 0 || kind[f] == 2) need[0] = true;
    if (kind[f] == 1 || kind[f] == 2) need[1] = true;
  }
  const size_t nw = 16 * (size_t)std::max<int64_t>(p->ng, 1);
  if (!p->wts) {
    // the weights, then the {0, 1} kind table read by uniform-kind fields
    p->wts = (double*)pool_alloc(sizeof(double) * (nw + 1));
    if (!p->wts) return GCR_E_NOMEM;
  }
  uint8_t* kinds = reinterpret_cast<uint8_t*>(p->wts + nw);
  for (int b = 0; b < 2; ++b) {
    double* wb = p->wts + (size_t)b * 8 * p->ng;
    if (need[b] && !p->wts_ok[b]) {
      launch_weights(plan_view(p), b, wb, kinds, st);
      GCR_HIP(hipGetLastError());
      p->wts_ok[b] = true;
    }
    w[b] = wb;
  }
  return GCR_OK;
}

}  // namespace gcr

using namespace gcr;

// --------------------------------------------------------------------------
// object lifetimes and per-plan scratch
// --------------------------------------------------------------------------

gcr_plan::~gcr_plan() {
  for (int i = 0; i < kScratchSlots; ++i)
    if (scr[i]) pool_free(scr[i]);
  if (sup) pool_free(sup);
  if (wts) pool_free(wts);
}

gcr_batch::~gcr_batch() {
  if (fwd_args) pool_free(fwd_args);
}

namespace gcr {
void* plan_scratch(gcr_plan* p, int slot, size_t bytes) {
  if (slot < 0 || slot >= kScratchSlots) return nullptr;
  if (p->scr_bytes[slot] < bytes) {
    if (p->scr[slot]) pool_free(p->scr[slot]);
    p->scr[slot] = pool_alloc(bytes);
    p->scr_bytes[slot] = p->scr[slot] ? bytes : 0;
  }
  return p->scr[slot];
}
}  // namespace gcr

extern "C" {

const char* gcr_status_str(gcr_status s) {
  switch (s) {
    case GCR_OK: return "ok";
    case GCR_E_ARG: return "invalid argument";
    case GCR_E_HIP: return "HIP runtime error";
    case GCR_E_NOMEM: return "out of memory";
    case GCR_E_CYCLE: return "ghost graph could not be layered";
    case GCR_E_STENCIL: return "stencil leaves the grid or reaches a solid cell";
    case GCR_E_DEGENERATE: return "degenerate relation (zero denominator)";
    case GCR_E_GEOMETRY: return "closest-point projection failed";
    case GCR_E_UNSUPPORTED: return "unsupported size or combination";
    case GCR_E_TIMEOUT: return "a wait between workgroups gave up; outputs not valid";
  }
  return "unknown status";
}

const char* gcr_version(void) { return "gcr 0.1 (gfx950, FP64)"; }

gcr_status gcr_plan_create(const gcr_grid* grid, const gcr_shape* shape, int32_t scheme,
                           void* stream, gcr_plan** out) {
  if (!out) return GCR_E_ARG;
  *out = nullptr;
  if (!grid || !shape) return GCR_E_ARG;
  std::shared_ptr<BatchData> B;
  gcr_status s = build_batch(1, grid, shape, &scheme, (hipStream_t)stream, &B);
  if (s != GCR_OK) return s;
  gcr_plan* p = new (std::nothrow) gcr_plan();
  if (!p) return GCR_E_NOMEM;
  make_plan_view(B, 0, p);
  *out = p;
  return GCR_OK;
}

void gcr_plan_destroy(gcr_plan* plan) {
  if (!plan) return;
  delete plan;
}

gcr_status gcr_plan_update(gcr_plan* p, const gcr_shape* shape, void* stream) {
  if (!plan_ok(p) || !shape) return GCR_E_ARG;
  // a plan made alone, not a view of a batch (whose other plans share its arrays)
  if (!p->batch || p->batch->ninst != 1 || p->batch.use_count() != 1) return GCR_E_UNSUPPORTED;
  const hipStream_t st = (hipStream_t)stream;
  std::shared_ptr<BatchData> nb;
  gcr_status s = build_update(*p->batch, *shape, true, st, &nb);
  const gcr_status result = s;
  if (s != GCR_OK) {
    if (p->batch->d_tags) return s;   // failed before the tags were taken: plan unchanged
    // the previous tags are partly rewritten: build the plan as it was
    s = build_update(*p->batch, p->inst.s, false, st, &nb);
    if (s != GCR_OK) {
      p->dead = true;
      p->batch.reset();
      return result;
    }
  }
  // the build synchronised the stream: the previous plan's arrays are idle
  // on it.  Caches derived from the ghosts go with them.
  for (int i = 0; i < kScratchSlots; ++i) {
    if (p->scr[i]) pool_free(p->scr[i]);
    p->scr[i] = nullptr;
    p->scr_bytes[i] = 0;
  }
  if (p->sup) pool_free(p->sup);
  p->sup = nullptr;
  p->sup_bound = 0;
  p->sup_hmask = 0;
  if (p->wts) pool_free(p->wts);
  p->wts = nullptr;
  p->wts_ok[0] = p->wts_ok[1] = false;
  p->graph.reset();
  p->tuned = -1;
  make_plan_view(nb, 0, p);
  return result;
}

gcr_status gcr_plan_stats(const gcr_plan* p, gcr_stats* out) {
  if (!plan_ok(p) || !out) return GCR_E_ARG;
  std::memset(out, 0, sizeof(*out));
  out->dim = p->dim;
  out->n_levels = p->nlev;
  out->n_cells = p->ncell;
  out->n_interface = p->nif;
  out->n_ghost = p->ng;
  out->n_ghost_fluid_side = p->info.nfluid;
  out->n_units_coupled = p->info.nunits;
  out->max_unit = p->info.maxunit;
  out->max_level_width = p->info.maxwidth;
  out->schedule = p->schedule != kSchedAuto ? p->schedule : (p->tuned < 0 ? 0 : p->tuned);
  out->n_band_segments = p->batch ? p->batch->nband : 0;
  for (int a = 0; a < 3; ++a) {
    unsigned long long b = p->info.max_alpha_bits[a];
    double v;
    std::memcpy(&v, &b, sizeof(v));
    out->max_alpha[a] = v;
  }
  return GCR_OK;
}

gcr_status gcr_plan_level_offsets(const gcr_plan* p, int32_t* out) {
  if (!plan_ok(p) || !out) return GCR_E_ARG;
  std::memcpy(out, p->lev_off.data(), sizeof(int32_t) * (p->nlev + 1));
  return GCR_OK;
}

gcr_status gcr_plan_export(const gcr_plan* p, int8_t* tags, int32_t* cell, int32_t* level,
                           double* delta, double* normal, double* psi, int32_t* r,
                           int32_t* unit, void* stream) {
  if (!plan_ok(p)) return GCR_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t ng = p->ng;
  if (tags) GCR_HIP(hipMemcpyAsync(tags, p->tags, p->ncell, hipMemcpyDeviceToDevice, st));
  if (ng > 0) {
    if (cell) GCR_HIP(hipMemcpyAsync(cell, p->cell, 4 * ng, hipMemcpyDeviceToDevice, st));
    if (level) GCR_HIP(hipMemcpyAsync(level, p->level, 4 * ng, hipMemcpyDeviceToDevice, st));
    if (psi) GCR_HIP(hipMemcpyAsync(psi, p->psi, 8 * ng, hipMemcpyDeviceToDevice, st));
    for (int a = 0; a < p->dim; ++a) {
      if (delta)
        GCR_HIP(hipMemcpyAsync(delta + a * ng, p->delta[a], 8 * ng, hipMemcpyDeviceToDevice, st));
      if (normal)
        GCR_HIP(hipMemcpyAsync(normal + a * ng, p->nrm[a], 8 * ng, hipMemcpyDeviceToDevice, st));
    }
    const unsigned nb = (unsigned)((ng + 255) / 256);
    if (r) k_export_r<<<nb, 256, 0, st>>>(p->code, (int)ng, p->dim, r);
    if (unit) k_export_unit<<<nb, 256, 0, st>>>(p->blk, p->unit_mem, (int)ng, unit);
    GCR_HIP(hipGetLastError());
  }
  return GCR_OK;
}

gcr_status gcr_plan_foot_points(const gcr_plan* p, double* S, double* normal, void* stream) {
  if (!plan_ok(p)) return GCR_E_ARG;
  if (p->ng == 0 || (!S && !normal)) return GCR_OK;
  const int ng = (int)p->ng;
  const double* d2 = p->dim == 3 ? p->delta[2] : p->delta[0];
  const double* n2 = p->dim == 3 ? p->nrm[2] : p->nrm[0];
  k_foot_points<<<(unsigned)((ng + 255) / 256), 256, 0, (hipStream_t)stream>>>(
      p->inst.g, p->cell, p->delta[0], p->delta[1], d2, p->nrm[0], p->nrm[1], n2, ng, S, normal);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

gcr_status gcr_set_schedule(gcr_plan* p, int32_t schedule, int32_t param) {
  if (!plan_ok(p) || schedule < 0 || schedule > 3 || param != 0) return GCR_E_ARG;
  p->schedule = schedule;
  return GCR_OK;
}

gcr_status gcr_fill(const gcr_plan* plan, int32_t nf, double* const* fields,
                    const int32_t* bc_kind, const uint8_t* const* bc_type,
                    const double* const* bc_val, void* stream) {
  if (!plan_ok(plan)) return GCR_E_ARG;
  FillArgs A;
  gcr_status s = make_fill_args(plan, nf, fields, bc_kind, bc_type, bc_val, &A);
  if (s != GCR_OK) return s;
  if (plan->ng == 0) return GCR_OK;
  gcr_plan* p = const_cast<gcr_plan*>(plan);
  hipStream_t st = (hipStream_t)stream;
  s = plan_weights(p, A.nf, A.kind, A.w, st);
  if (s != GCR_OK) return s;
  {
    const uint8_t* kinds = reinterpret_cast<const uint8_t*>(p->wts + 16 * p->ng);
    for (int f = 0; f < nf; ++f)
      if (A.kind[f] != GCR_MIXED) {
        A.bt[f] = kinds + A.kind[f];
        A.bts[f] = 0;
      } else {
        A.bts[f] = 1;
      }
  }
  if (p->schedule == kSchedAuto) return tuned_fill(p, A, st);
  return run_fill(p, A, p->schedule, st);
}

gcr_status gcr_surface_ghost(const gcr_plan* p, int32_t nf, const double* const* fields,
                             double* val, double* grad, void* stream) {
  if (!plan_ok(p) || !check_fields(nf, (const void* const*)fields)) return GCR_E_ARG;
  SurfArgs S;
  std::memset(&S, 0, sizeof(S));
  S.P = plan_view(p);
  S.nf = nf;
  for (int f = 0; f < nf; ++f) S.f[f] = fields[f];
  S.val = val;
  S.grad = grad;
  launch_surface_ghost(S, (hipStream_t)stream);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

gcr_status gcr_surface(const gcr_plan* p, int64_t nq, const double* xq, int32_t nf,
                       const double* const* fields, double* val, double* grad, int32_t* anchor,
                       void* stream) {
  if (!plan_ok(p) || nq < 0 || (nq > 0 && !xq) || !check_fields(nf, (const void* const*)fields))
    return GCR_E_ARG;
  if (nq >= (int64_t(1) << 31)) return GCR_E_UNSUPPORTED;
  SurfArgs S;
  std::memset(&S, 0, sizeof(S));
  S.P = plan_view(p);
  S.nf = nf;
  for (int f = 0; f < nf; ++f) S.f[f] = fields[f];
  S.val = val;
  S.grad = grad;
  S.anchor = anchor;
  launch_surface_query(S, nq, xq, (hipStream_t)stream);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

gcr_status gcr_forces(const gcr_plan* p, int64_t nq, const double* xq, const double* nrm,
                      const double* wq, const double* pf, const double* const* u, double mu,
                      double* F, void* stream) {
  if (!plan_ok(p) || nq < 0 || !F || !pf || !u) return GCR_E_ARG;
  if (nq > 0 && (!xq || !nrm || !wq)) return GCR_E_ARG;
  for (int a = 0; a < p->dim; ++a)
    if (!u[a]) return GCR_E_ARG;
  if (nq >= (int64_t(1) << 31)) return GCR_E_UNSUPPORTED;
  ForceArgs A;
  std::memset(&A, 0, sizeof(A));
  A.nq = nq;
  A.xq = xq;
  A.nrm = nrm;
  A.wq = wq;
  A.p = pf;
  for (int a = 0; a < p->dim; ++a) A.u[a] = u[a];
  A.mu = mu;
  const int64_t nb = force_blocks(p->dim, nq);
  double* part = (double*)plan_scratch(const_cast<gcr_plan*>(p), 0, sizeof(double) * 3 * nb);
  if (!part) return GCR_E_NOMEM;
  launch_forces(plan_view(p), A, part, F, (hipStream_t)stream);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

}  // extern "C"

// Force partials of gcr_forces_noalloc: a file-scope device array instead of
// plan scratch, so the call allocates nothing.  Each device holds its own
// copy; host code reaches it only through the address hipGetSymbolAddress
// gives per device (the array's name on the host is a stand-in, not a
// device address).  Every block of the force kernel writes its partial, so
// nothing needs clearing between calls.
namespace {
constexpr int64_t kNoAllocForceBlocks = 65536;   // 1.5 MiB of partials
static __device__ __align__(256) double scratch[3 * kNoAllocForceBlocks];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of the array, looked up once per device.
gcr_status device_scratch(double** out) {
  int dev = 0;
  GCR_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return GCR_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    GCR_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return GCR_E_HIP;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return GCR_OK;
}
}  // namespace

extern "C" {

gcr_status gcr_forces_noalloc(const gcr_plan* p, int64_t nq, const double* xq,
                              const double* nrm, const double* wq, const double* pf,
                              const double* const* u, double mu, double* F, void* stream) {
  if (!plan_ok(p) || nq < 0 || !F || !pf || !u) return GCR_E_ARG;
  if (nq > 0 && (!xq || !nrm || !wq)) return GCR_E_ARG;
  for (int a = 0; a < p->dim; ++a)
    if (!u[a]) return GCR_E_ARG;
  const int64_t nb = force_blocks(p->dim, nq);
  if (nb > kNoAllocForceBlocks) return GCR_E_UNSUPPORTED;
  double* part = nullptr;
  const gcr_status s = device_scratch(&part);
  if (s != GCR_OK) return s;
  ForceArgs A;
  std::memset(&A, 0, sizeof(A));
  A.nq = nq;
  A.xq = xq;
  A.nrm = nrm;
  A.wq = wq;
  A.p = pf;
  for (int a = 0; a < p->dim; ++a) A.u[a] = u[a];
  A.mu = mu;
  launch_forces(plan_view(p), A, part, F, (hipStream_t)stream);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

gcr_status gcr_batch_create(int32_t ninst, const gcr_grid* grids, const gcr_shape* shapes,
                            const int32_t* schemes, void* stream, gcr_batch** out) {
  if (!out) return GCR_E_ARG;
  *out = nullptr;
  std::shared_ptr<BatchData> B;
  gcr_status s = build_batch(ninst, grids, shapes, schemes, (hipStream_t)stream, &B);
  if (s != GCR_OK) return s;
  gcr_batch* b = new (std::nothrow) gcr_batch();
  if (!b) return GCR_E_NOMEM;
  b->data = B;
  b->plans.resize(ninst);
  for (int i = 0; i < ninst; ++i) {
    b->plans[i].reset(new gcr_plan());
    make_plan_view(B, i, b->plans[i].get());
  }
  *out = b;
  return GCR_OK;
}

void gcr_batch_destroy(gcr_batch* b) {
  if (!b) return;
  gcr_batch_release_state(b);
  delete b;
}

gcr_status gcr_set_profiling(int32_t mask) {
  if (mask < 0 || mask > 3) return GCR_E_ARG;
  set_profiling(mask);
  return GCR_OK;
}

gcr_status gcr_set_batch_tiling(int32_t mode) {
  if (mode < 0 || mode > 2) return GCR_E_ARG;
  set_batch_tiling(mode);
  return GCR_OK;
}

gcr_status gcr_set_batch_shape(int32_t threads, int32_t grid) {
  if (threads == 0 && grid == 0) {
    set_batch_shape(0, 0);
    return GCR_OK;
  }
  if (threads < 64 || threads > 1024 || (threads & (threads - 1)) || grid == 0 || grid > 4 ||
      grid < -128)
    return GCR_E_ARG;
  set_batch_shape(threads, grid);
  return GCR_OK;
}

gcr_status gcr_set_wide_layering(int64_t min_interface) {
  if (min_interface < 0) return GCR_E_ARG;
  set_wide_layering(min_interface);
  return GCR_OK;
}

gcr_status gcr_set_wide_buffer(int32_t entries) {
  if (entries < 0 || entries > kWideBuf) return GCR_E_ARG;
  set_wide_buffer(entries);
  return GCR_OK;
}

gcr_status gcr_set_wave_residual(int32_t max_ghosts) {
  if (max_ghosts < 0 || max_ghosts > kWaveResidual) return GCR_E_ARG;
  set_wave_residual(max_ghosts);
  return GCR_OK;
}

gcr_status gcr_last_build_times(float* ms) {
  if (!ms) return GCR_E_ARG;
  last_build_times(ms);
  return GCR_OK;
}

gcr_status gcr_batch_plan(const gcr_batch* b, int32_t i, const gcr_plan** out) {
  if (!b || !out || i < 0 || i >= (int)b->plans.size()) return GCR_E_ARG;
  *out = b->plans[i].get();
  return GCR_OK;
}

gcr_status gcr_batch_counts(const gcr_batch* b, int64_t* n_ghost, int32_t* n_levels) {
  if (!b) return GCR_E_ARG;
  const int n = (int)b->plans.size();
  for (int i = 0; i < n; ++i) {
    if (n_ghost) n_ghost[i] = b->plans[i]->ng;
    if (n_levels) n_levels[i] = b->plans[i]->nlev;
  }
  return GCR_OK;
}

gcr_status gcr_batch_foot_points(const gcr_batch* b, double* S, double* normal, void* stream) {
  if (!b || !b->data) return GCR_E_ARG;
  const BatchData& D = *b->data;
  const int dim = b->plans[0]->dim;
  for (const auto& p : b->plans)
    if (p->dim != dim) return GCR_E_UNSUPPORTED;
  const int64_t ng = D.ng_total;
  if (ng == 0 || (!S && !normal)) return GCR_OK;
  k_batch_foot_points<<<(unsigned)((ng + 255) / 256), 256, 0, (hipStream_t)stream>>>(
      D.d_inst, D.ninst, D.d_g_off, D.cap, D.d_cell, D.d_delta, D.d_nrm, dim, ng, S, normal);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

}  // extern "C"
