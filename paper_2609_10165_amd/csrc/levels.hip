// levels.hip -- Kahn layering of the ghost dependency graph (Sec. 3.2) and
// the canonical order (level, linear index), one workgroup per instance.
//
// The reverse edges (ghost -> ghosts that read it) arrive as a CSR list and
// the number of ghosts each ghost reads as a byte per ghost, both built by
// grid-wide kernels.  Each ghost (or coupled unit) holds a byte counter of
// unplaced ghosts it reads, packed four to a word and kept in LDS when the
// instance fits.
// Level k is formed from the dependants of level k-1 whose counter drops to
// zero: they set their bit in a bitmap over the linear ghost order, and one
// workgroup scan over the bitmap words emits them in linear-index order with
// their canonical positions.  The work is O(ghosts + edges) plus one bitmap
// scan per level; the level of a ghost is the longest dependency path from a
// ghost that reads no ghost, independent of the order threads run in.
//
// If a level comes out empty while ghosts remain, the remaining ghosts hold
// cycles: their strongly connected groups (from the transitive closure of
// the remaining graph) become coupled units, and the layering restarts with
// each unit as one node, so a unit sits one level above the deepest level it
// needs.
//
// A single large instance is layered by the whole grid instead
// (k_levels_wide): one cooperative launch whose rounds each release the next
// level from the current one through the same counters (in HBM), with a grid
// barrier between rounds; the canonical order then comes from a stable
// counting sort of the ghosts by level.  A stall there (a cycle) or a graph
// deeper than the sort supports hands the instance to the one-workgroup
// layering, launched right after, which otherwise returns at once.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <mutex>

#include "gcr_impl.hpp"

namespace gcr {

__device__ __forceinline__ int64_t find_sorted(const int32_t* a, int64_t lo, int64_t hi, int v) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    int x = a[mid];
    if (x == v) return mid;
    if (x < v) lo = mid + 1; else hi = mid;
  }
  return -1;
}

// byte counters packed four per 32-bit word; a counter never goes below
// zero (one decrement per counted edge) and never exceeds 8 * 7, so no carry
// or borrow crosses into a neighbour
__device__ __forceinline__ void cnt_add(uint32_t* c, int i, uint32_t v) {
  atomicAdd(&c[i >> 2], v << ((i & 3) * 8));
}
__device__ __forceinline__ uint32_t cnt_dec(uint32_t* c, int i) {
  const uint32_t old = atomicSub(&c[i >> 2], 1u << ((i & 3) * 8));
  return (old >> ((i & 3) * 8)) & 0xffu;
}
__device__ __forceinline__ uint32_t cnt_get(const uint32_t* c, int i) {
  return (c[i >> 2] >> ((i & 3) * 8)) & 0xffu;
}

// Appends v to list (size counter *size) for the lanes with p set: one
// atomic per wave.  Lanes may be diverged; only active lanes take part.
__device__ __forceinline__ void wave_push(bool p, int v, int32_t* list, int32_t* size) {
  const unsigned long long m = __ballot(p);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(size, __popcll(m));
  base = __shfl(base, leader);
  if (p) list[base + __popcll(m & ((1ull << lane) - 1ull))] = v;
}

// Appends v for the lanes with p set to a workgroup's LDS buffer buf (fill
// count *s_n, capacity cap), one LDS atomic per wave; entries beyond the
// capacity go straight to the global list glist (length *gsize), one global
// atomic per wave that has any.  *s_n keeps counting past cap.
__device__ __forceinline__ void wave_push_buf(bool p, int v, int32_t* buf, int* s_n, int cap,
                                              int32_t* glist, int32_t* gsize) {
  const unsigned long long m = __ballot(p);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = (1ull << lane) - 1ull;
  const int leader = __ffsll((long long)m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(s_n, __popcll(m));
  base = __shfl(base, leader);
  const int idx = base + __popcll(m & lt);
  const bool spill = p && idx >= cap;
  if (p && !spill) buf[idx] = v;
  const unsigned long long ms = __ballot(spill);
  if (ms == 0ull) return;
  const int ls = __ffsll((long long)ms) - 1;
  int gb = 0;
  if (lane == ls) gb = atomicAdd(gsize, __popcll(ms));
  gb = __shfl(gb, ls);
  if (spill) glist[gb + __popcll(ms & lt)] = v;
}

// Wide layering of instance 0.  wide[0] = 1 when it finished (levels,
// canonical order, level offsets and info final), wide[r] = size of level r.
// Each round's releases collect in the workgroup's LDS buffer and join the
// next level's list with one global atomic per workgroup (the order inside
// a level's list is free: the counting sort orders the level).
__global__ __launch_bounds__(256) void k_levels_wide(LevelsArgs L) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const int tid = threadIdx.x;
  const int G = (int)gridDim.x;
  const int64_t GT = (int64_t)G * 256;
  const int64_t gt = (int64_t)blockIdx.x * 256 + tid;
  const int64_t lo = L.g_off[0];
  const int n = (int)(L.g_off[1] - lo);
  const int C = (n + 3) >> 2;
  uint32_t* __restrict__ cnt = L.cnt;
  int32_t* __restrict__ lev = L.lev + lo;
  int32_t* __restrict__ perm = L.perm + lo;
  const uint8_t* __restrict__ dcnt = L.dcnt + lo;
  const int32_t* __restrict__ roff = L.roff + lo;
  const int32_t* __restrict__ radj = L.radj;
  int32_t* __restrict__ size = L.wide;
  int32_t* lists[2] = {L.listA + lo, L.listB + lo};
  __shared__ int64_t sh[8];
  __shared__ int s_hist[kWideLevels];
  __shared__ int s_wc[4][kWideLevels];
  __shared__ int32_t s_buf[kWideBuf];
  __shared__ int s_n, s_base;
  const int wcap = min(max(L.wide_cap, 1), kWideBuf);
  if (L.info[0].layered) return;   // the LDS layering finished it (every workgroup leaves)

  // counters of ghosts read, four per word; no ghost is in a unit
  for (int64_t w = gt; w < C; w += GT) {
    uint32_t v = 0;
    for (int q = 0; q < 4; ++q)
      if (4 * w + q < n) v |= (uint32_t)dcnt[4 * w + q] << (8 * q);
    cnt[w] = v;
  }
  for (int64_t g = gt; g < n; g += GT) L.blk_idx[lo + g] = -1;
  if (blockIdx.x == 0)
    for (int r = tid; r < kWideState; r += 256) size[r] = 0;
  grid.sync();
  // level 1: ghosts that read no ghost (through the workgroup's buffer,
  // flushed as after each round)
  if (tid == 0) s_n = 0;
  __syncthreads();
  for (int64_t g0 = (int64_t)blockIdx.x * 256; g0 < n; g0 += GT) {
    const int g = (int)(g0 + tid);
    const bool p = g < n && dcnt[g] == 0;
    if (p) lev[g] = 1;
    wave_push_buf(p, g, s_buf, &s_n, wcap, lists[1], &size[1]);
  }
  __syncthreads();
  {
    const int mcount = min(s_n, wcap);
    if (tid == 0 && mcount > 0) s_base = atomicAdd(&size[1], mcount);
    __syncthreads();
    for (int k = tid; k < mcount; k += 256) lists[1][s_base + k] = s_buf[k];
  }
  grid.sync();

  // round r: the dependants of level r whose last counted edge comes from it
  // form level r + 1
  int r = 1, placed = 0, maxw = 0;
  bool ok = true;
  for (;;) {
    const int sz = __hip_atomic_load(&size[r], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (sz == 0) break;
    placed += sz;
    maxw = max(maxw, sz);
    if (r == kWideLevels - 1) {
      ok = false;
      break;
    }
    const int32_t* __restrict__ cur = lists[r & 1];
    int32_t* __restrict__ nxt = lists[(r + 1) & 1];
    if (tid == 0) s_n = 0;
    __syncthreads();
    for (int64_t i = gt; i < sz; i += GT) {
      const int g = cur[i];
      const int e1 = roff[g + 1];
      for (int e = roff[g]; e < e1; ++e) {
        const int q = (int)(radj[e] - lo);
        const bool rel = cnt_dec(cnt, q) == 1u;
        if (rel) lev[q] = r + 1;
        wave_push_buf(rel, q, s_buf, &s_n, wcap, nxt, &size[r + 1]);
      }
    }
    __syncthreads();
    {
      const int mcount = min(s_n, wcap);
      if (tid == 0 && mcount > 0) s_base = atomicAdd(&size[r + 1], mcount);
      __syncthreads();
      for (int k = tid; k < mcount; k += 256) nxt[s_base + k] = s_buf[k];
    }
    ++r;
    grid.sync();
  }
  if (!ok || placed != n) return;   // every workgroup leaves here alike
  const int nlev = r - 1;
  const int ntiles = (n + 255) >> 8;
  int32_t* __restrict__ hist = L.hist;   // [level][tile]

  // stable counting sort by level: per-tile counts ...
  for (int t = blockIdx.x; t < ntiles; t += G) {
    for (int l = tid; l < nlev; l += 256) s_hist[l] = 0;
    __syncthreads();
    const int g = t * 256 + tid;
    if (g < n) atomicAdd(&s_hist[lev[g] - 1], 1);
    __syncthreads();
    for (int l = tid; l < nlev; l += 256) hist[(int64_t)l * ntiles + t] = s_hist[l];
    __syncthreads();
  }
  grid.sync();
  // ... scanned over the tiles of each level, plus the level offsets ...
  for (int l = blockIdx.x; l < nlev; l += G) {
    int32_t* row = hist + (int64_t)l * ntiles;
    int64_t carry = 0;
    for (int t0 = 0; t0 < ntiles; t0 += 256) {
      const int t = t0 + tid;
      const int v = t < ntiles ? row[t] : 0;
      int64_t tot;
      const int64_t pre = block_excl_scan<256>(v, &tot, sh);
      if (t < ntiles) row[t] = (int32_t)(carry + pre);
      carry += tot;
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    int32_t* lev_off = L.lev_off;
    int run = 0;
    lev_off[0] = 0;
    for (int k = 1; k <= nlev; ++k) {
      run += size[k];
      lev_off[k] = run;
    }
    L.info[0].nlev = nlev;
    L.info[0].maxwidth = maxw;
    L.info[0].nunits = 0;
    L.info[0].maxunit = 0;
    size[0] = 1;
  }
  grid.sync();
  // ... and each ghost's rank among the same level's ghosts before it
  const int lane = tid & 63, wv = tid >> 6;
  for (int t = blockIdx.x; t < ntiles; t += G) {
    for (int i = tid; i < 4 * nlev; i += 256) s_wc[i / nlev][i % nlev] = 0;
    __syncthreads();
    const int g = t * 256 + tid;
    const bool valid = g < n;
    const int l = valid ? lev[g] - 1 : -1;
    unsigned long long rem = __ballot(valid);
    int inw = 0;
    while (rem) {
      const int leader = __ffsll((long long)rem) - 1;
      const int l0 = __shfl(l, leader);
      const bool same = valid && l == l0;
      const unsigned long long m = __ballot(same);
      if (same) inw = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == leader) s_wc[wv][l0] = __popcll(m);
      rem &= ~m;
    }
    __syncthreads();
    if (valid) {
      int pos = L.lev_off[l] + hist[(int64_t)l * ntiles + t] + inw;
      for (int w = 0; w < wv; ++w) pos += s_wc[w][l];
      perm[g] = pos;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Layering in LDS.  One workgroup per instance keeps the byte counters of
// unplaced ghosts read, each ghost's level and a Kahn queue in LDS (the
// queue in HBM when only the rest fits), and the instance's reverse edges
// too when they fit: level k is the queue segment
// its predecessor level released, so a level costs one pass over its own
// ghosts' reverse edges and one barrier.
//
// If the queue runs dry with ghosts left, those read a cycle directly or
// through others.  The ghosts that no unplaced ghost reads are trimmed
// away, repeatedly, leaving the cycles (and any ghost between two); their
// strongly connected groups (transitive closure, as in k_levels) become
// coupled units.  The unplaced ghosts and units are then placed in
// dependency order, each at 1 + the highest level it reads (the level of
// Sec. 3.2: the longest dependency path, units as single nodes).
//
// The canonical order (level, linear index) comes from a stable counting
// sort: per-wave level counts over contiguous ranges of the linear order,
// level offsets from their totals, a scan over the waves per level, and each
// ghost's rank among its wave's ghosts of the same level by ballots.  An
// instance that does not fit, is deeper than kFastLevels or whose units
// exceed the solver's limits is left to k_levels, launched right after,
// which skips the instances finished here (InstInfo::layered).
constexpr int kFastLevels = 256;
constexpr int kFastWaves = 16;     // 1024 threads
constexpr uint16_t kTrimmed = 0xffff;

// Appends v to list[base + ...] (length counter *size) for the lanes with p
// set, one atomic per wave; entries at or beyond cap are dropped (a node
// enters a queue once, so it never holds more than the instance's ghosts;
// the check keeps LDS writes in bounds regardless).
__device__ __forceinline__ void wave_push16(bool p, int v, uint16_t* list, int base,
                                            int* size, int cap) {
  const unsigned long long m = __ballot(p);
  if (m == 0ull) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)m) - 1;
  int at = 0;
  if (lane == leader) at = atomicAdd(size, __popcll(m));
  at = __shfl(at, leader);
  const int idx = base + at + __popcll(m & ((1ull << lane) - 1ull));
  if (p && idx < cap) list[idx] = (uint16_t)v;
}

__global__ __launch_bounds__(1024) void k_levels_fast(LevelsArgs L, int lds_bytes) {
  extern __shared__ uint32_t s_dyn[];
  __shared__ int s_off[kFastLevels + 2];
  __shared__ int s_tot[kFastLevels + 1];
  __shared__ int s_cnt[3];
  __shared__ int64_t sh[17];
  __shared__ int s_flag, s_units, s_maxunit, s_maxlev, s_placed, s_bad;
  const int ii = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t lo = L.g_off[ii];
  const int n = (int)(L.g_off[ii + 1] - lo);
  if (n > 65535) return;   // 16-bit ids in the queue
  const int np = (1 << L.insts[ii].g.dim) - 1;
  const int64_t cap = L.cap;
  const int32_t* __restrict__ deps = L.deps;
  const int32_t* __restrict__ roff = L.roff + lo;
  const int32_t* __restrict__ radj = L.radj;
  const uint8_t* __restrict__ dcnt = L.dcnt + lo;
  int32_t* __restrict__ blk_idx = L.blk_idx;      // global linear ids
  int32_t* unit_mem = L.unit_mem + (int64_t)ii * kMaxUnits * kMaxUnit;
  int32_t* unit_cnt = L.unit_cnt + (int64_t)ii * kMaxUnits;
  int32_t* unit_lev = L.unit_lev + (int64_t)ii * kMaxUnits;
  const int64_t e0 = roff[0];
  const int E = (int)(roff[n] - e0);
  auto al = [](int64_t b) { return (b + 15) & ~int64_t(15); };
  char* base = reinterpret_cast<char*>(s_dyn);
  int64_t o = 0;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(base + o);
  o += al(4 * (int64_t)((n + 3) >> 2));
  uint16_t* lvl = reinterpret_cast<uint16_t*>(base + o);
  o += al(2 * (int64_t)n);
  // the release queue: in LDS when it fits beside the rank table, else in the
  // instance's slice of listA (HBM, 2 bytes a ghost of its 4), which leaves
  // 3 bytes a ghost in LDS
  constexpr int64_t kTab = 4 * (int64_t)kFastWaves * kFastLevels;
  const bool qlds = o + al(2 * (int64_t)n) + kTab <= lds_bytes;
  uint16_t* que = qlds ? reinterpret_cast<uint16_t*>(base + o)
                       : reinterpret_cast<uint16_t*>(L.listA + lo);
  if (qlds) o += al(2 * (int64_t)n);
  // [kFastWaves][kFastLevels] rank counts; before that the cycle search's
  // residual list, representatives and unit slots (3 x kMaxResidual)
  int32_t* tab = reinterpret_cast<int32_t*>(base + o);
  o += kTab;
  if (o > lds_bytes) return;   // every thread leaves alike
  // reverse edges, then (used only after a stall) the forward dependencies
  // as local ids and each ghost's unit slot, each where LDS is left
  int32_t* eoff = reinterpret_cast<int32_t*>(base + o);
  const int64_t o_adj = o + al(4 * ((int64_t)n + 1));
  uint16_t* eadj = reinterpret_cast<uint16_t*>(base + o_adj);
  const int64_t o_eend = o_adj + al(2 * (int64_t)E);
  const bool elds = o_eend <= lds_bytes;
  const int64_t o_dep = elds ? o_eend : o;
  uint16_t* fdep = reinterpret_cast<uint16_t*>(base + o_dep);
  const int64_t o_slot = o_dep + al(2 * (int64_t)np * n);
  uint16_t* uslot = reinterpret_cast<uint16_t*>(base + o_slot);
  const bool dlds = o_slot + al(2 * (int64_t)n) <= lds_bytes;
  __shared__ uint16_t s_uhead[kMaxUnits];   // head (smallest member) of each unit
  __shared__ uint8_t s_usize[kMaxUnits];
  auto edge_range = [&](int g, int& ea, int& eb) {
    ea = elds ? eoff[g] : (int)(roff[g] - e0);
    eb = elds ? eoff[g + 1] : (int)(roff[g + 1] - e0);
  };
  auto dependant = [&](int e) { return elds ? (int)eadj[e] : (int)(radj[e0 + e] - lo); };
  // dependency q of ghost g as a local id, -1 if it reads no ghost there
  auto dep = [&](int g, int q) -> int {
    if (dlds) {
      const int v = fdep[q * n + g];
      return v == 0xffff ? -1 : v;
    }
    const int32_t d = deps[(int64_t)q * cap + lo + g];
    return d < 0 ? -1 : (int)(d - lo);
  };
  auto slot_of = [&](int g) -> int {
    if (dlds) {
      const int v = uslot[g];
      return v == 0xffff ? -1 : v;
    }
    return blk_idx[lo + g];
  };

  const int C = (n + 3) >> 2;
  for (int w = tid; w < C; w += 1024) {
    uint32_t v = 0;
    for (int q = 0; q < 4; ++q)
      if (4 * w + q < n) v |= (uint32_t)dcnt[4 * w + q] << (8 * q);
    cnt[w] = v;
  }
  for (int g = tid; g < n; g += 1024) {
    lvl[g] = 0;
    blk_idx[lo + g] = -1;
  }
  if (elds) {
    for (int g = tid; g <= n; g += 1024) eoff[g] = (int)(roff[g] - e0);
    for (int e = tid; e < E; e += 1024) eadj[e] = (uint16_t)(radj[e0 + e] - lo);
  }
  if (tid < 3) s_cnt[tid] = 0;
  if (tid == 0) {
    s_units = 0;
    s_maxunit = 0;
    s_bad = 0;
  }
  __syncthreads();
  // level 1: ghosts that read no ghost
  for (int g = tid; g < n; g += 1024) {
    const bool p = dcnt[g] == 0;
    if (p) lvl[g] = 1;
    wave_push16(p, g, que, 0, &s_cnt[0], n);
  }
  __syncthreads();
  int a = 0, b = s_cnt[0], k = 0;
  // iteration k: level k (queue[a, b)) releases level k + 1 into queue[b,
  // ...), its length accumulating in s_cnt[k % 3].  The counter of the next
  // iteration, s_cnt[(k + 1) % 3], was last read after the barrier that
  // ended iteration k - 2, which every thread has passed since, so thread 0
  // clears it now.
  while (a < b) {
    ++k;
    if (k > kFastLevels) return;   // uniform: every thread counts the same levels
    if (tid == 0) s_cnt[(k + 1) % 3] = 0;
    int* const tail = &s_cnt[k % 3];
    for (int i = a + tid; i < b; i += 1024) {
      const int g = que[i];
      int ea, eb;
      edge_range(g, ea, eb);
      for (int e = ea; e < eb; ++e) {
        const int q = dependant(e);
        const bool rel = cnt_dec(cnt, q) == 1u;
        if (rel) lvl[q] = (uint16_t)(k + 1);
        wave_push16(rel, q, que, b, tail, n);
      }
    }
    __syncthreads();
    a = b;
    b += *tail;
    if (b > n) return;   // cannot happen (each ghost released once)
  }
  if (tid == 0) {
    s_maxlev = k;
    s_placed = b;
  }

  if (b < n && n - b <= L.wave_res) {   // (wave_res <= 64)
    // ---- at most 64 ghosts left (they read a cycle): one wave finds the
    // cycles and places them, with no workgroup barrier.  Lane u holds
    // residual ghost res[u] and the set A of residual ghosts it reads; the
    // closure R = A+ comes from Warshall's pass over its lanes, the group of
    // a ghost on a cycle (u in R[u]) is R[u] & {v : u in R[v]}, whose
    // smallest member is its representative, and the groups' slots follow
    // their representatives' order.  Then every residual ghost or group is
    // placed, in dependency order, at 1 + the highest level it reads outside
    // its group.  The result is the one of the general path below, which
    // trims ghosts off the cycles first: a ghost on a cycle is never trimmed,
    // and the levels are the same longest-path levels.
    if (tid < 64) {
      const int lane = tid;
      int32_t* res = tab;          // [64] residual ghosts, ascending
      int32_t* s_c = tab + 128;    // [64] the placement order
      int m = 0;
      for (int g0 = 0; g0 < n; g0 += 64) {
        const int g = g0 + lane;
        const bool left = g < n && lvl[g] == 0;
        const unsigned long long bm = __ballot(left);
        if (left) res[m + __popcll(bm & ((1ull << lane) - 1ull))] = g;
        m += __popcll(bm);
      }
      __builtin_amdgcn_wave_barrier();
      // dependency q of ghost g as a local id, -1 if it reads no ghost there
      auto gdep = [&](int g, int q) -> int {
        const int32_t d = deps[(int64_t)q * cap + lo + g];
        return d < 0 ? -1 : (int)(d - lo);
      };
      // the residual ghosts each lane reads (A) and the highest level among
      // the ghosts it reads that the layering placed (ext), read once
      const int g = lane < m ? res[lane] : -1;
      unsigned long long A = 0ull;
      int ext = 0;
      if (lane < m)
        for (int q = 0; q < np; ++q) {
          const int d = gdep(g, q);
          if (d < 0) continue;
          if (lvl[d] != 0) {
            ext = max(ext, (int)lvl[d]);
            continue;
          }
          const int v = (int)find_sorted(res, 0, m, d);
          if (v >= 0) A |= 1ull << v;
        }
      // closure R = A+ by Warshall's pass: after step v, R[u] holds every
      // ghost u reaches through intermediates among the first v + 1; row v
      // is read from its lane with readlane (v is uniform), no LDS
      unsigned long long R = A;
      const int mu = __builtin_amdgcn_readfirstlane(m);   // (the same in every lane)
      for (int v = 0; v < mu; ++v) {
        const uint32_t rlo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)R, v);
        const uint32_t rhi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(R >> 32), v);
        if ((R >> v) & 1ull) R |= ((unsigned long long)rhi << 32) | rlo;
      }
      unsigned long long T = 0ull;   // {v : lane in R[v]}
      for (int u = 0; u < m; ++u) {
        const unsigned long long col = __ballot(lane < m && ((R >> u) & 1ull));
        if (lane == u) T = col;
      }
      const bool oncyc = lane < m && ((R >> lane) & 1ull);
      const unsigned long long M = oncyc ? (R & T) : (lane < m ? (1ull << lane) : 0ull);
      const int rep = oncyc ? __ffsll((long long)M) - 1 : -1;
      const int size = __popcll(M);
      const unsigned long long reps = __ballot(oncyc && rep == lane);
      const int nunits = __popcll(reps);
      const bool bad = __ballot(oncyc && size > kMaxUnit) != 0ull;
      int slot = -1;
      if (oncyc) slot = __popcll(reps & ((1ull << rep) - 1ull));
      if (!bad && oncyc) {
        unit_mem[slot * kMaxUnit + __popcll(M & ((1ull << lane) - 1ull))] = (int32_t)(lo + g);
        blk_idx[lo + g] = slot;
        if (rep == lane) unit_cnt[slot] = size;
      }
      // placement in dependency order, in one pass in registers.  Ghost u
      // reading ghost w of another group has a larger key 2 |R[u]| + (u not
      // on a cycle) than w: R[u] holds R[w], and u itself (u on a cycle) or
      // w's own group (w on a cycle) or w (neither) besides.  So the order
      // of (key, lane) places every group after all it reads; a group's
      // members share R and sit together.  c: the highest level the lane
      // reads outside its group (ext to start with), final when its group's
      // turn comes; the group's level is 1 + the highest c of its members.
      int Lown = 0;
      if (!bad) {
        const int key = lane < m ? 2 * __popcll(R) + (oncyc ? 0 : 1) : 0x7fffffff;
        int rank = 0;
        for (int v = 0; v < mu; ++v) {
          const int kv = __builtin_amdgcn_readlane(key, v);
          rank += (kv < key || (kv == key && v < lane)) ? 1 : 0;
        }
        if (lane < m) s_c[rank] = lane;
        __builtin_amdgcn_wave_barrier();
        const int ord = lane < m ? s_c[lane] : 0;
        const unsigned long long outside = A & ~M;
        int c = ext;
        for (int pos = 0; pos < mu; ++pos) {
          const int v = __builtin_amdgcn_readlane(ord, pos);
          if (__builtin_amdgcn_readlane(Lown, v) != 0) continue;   // placed with its group
          const unsigned long long Mv =
              ((unsigned long long)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(M >> 32), v) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)M, v);
          int mx = 0;
          for (unsigned long long w = Mv; w; w &= w - 1ull)
            mx = max(mx, __builtin_amdgcn_readlane(c, __ffsll((long long)w) - 1));
          if ((Mv >> lane) & 1ull) Lown = mx + 1;
          if (outside & Mv) c = max(c, mx + 1);
        }
      }
      if (bad) {
        if (lane == 0) s_bad = 1;
      } else {
        const int L = lane < m ? Lown : 0;
        if (lane < m && L > 0) lvl[g] = (uint16_t)L;
        if (oncyc && rep == lane) unit_lev[slot] = L;
        int mxl = L, mxs = oncyc ? size : 0, done = lane < m && L > 0 ? 1 : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
          mxl = max(mxl, __shfl_xor(mxl, o));
          mxs = max(mxs, __shfl_xor(mxs, o));
          done += __shfl_xor(done, o);
        }
        if (lane == 0) {
          s_units = nunits;
          s_maxunit = mxs;
          s_maxlev = max(s_maxlev, mxl);
          s_placed += done;
        }
      }
    }
    __syncthreads();
    if (s_bad) return;
  } else if (b < n) {
    // ---- the ghosts left read a cycle.  Trim those that no unplaced ghost
    // reads (counters: unplaced readers), repeatedly.
    if (dlds) {
      for (int t = tid; t < np * n; t += 1024) {
        const int q = t / n, g = t - q * n;
        const int32_t d = deps[(int64_t)q * cap + lo + g];
        fdep[t] = d < 0 ? (uint16_t)0xffff : (uint16_t)(d - lo);
      }
      for (int g = tid; g < n; g += 1024) uslot[g] = 0xffff;
    }
    for (int w = tid; w < C; w += 1024) cnt[w] = 0;
    __syncthreads();
    for (int g = tid; g < n; g += 1024) {
      if (lvl[g] != 0) continue;
      int ea, eb;
      edge_range(g, ea, eb);
      uint32_t c = 0;
      for (int e = ea; e < eb; ++e) c += lvl[dependant(e)] == 0 ? 1u : 0u;
      if (c) cnt_add(cnt, g, c);
    }
    if (tid < 3) s_cnt[tid] = 0;
    __syncthreads();
    for (int g = tid; g < n; g += 1024) {
      const bool p = lvl[g] == 0 && cnt_get(cnt, g) == 0;
      if (p) lvl[g] = kTrimmed;
      wave_push16(p, g, que, b, &s_cnt[0], n);
    }
    __syncthreads();
    {
      int ta = b, tb = b + s_cnt[0], r = 0;
      while (ta < tb) {
        ++r;
        if (tid == 0) s_cnt[(r + 1) % 3] = 0;
        int* const tail = &s_cnt[r % 3];
        for (int i = ta + tid; i < tb; i += 1024) {
          const int u = que[i];
          for (int q = 0; q < np; ++q) {
            const int dl = dep(u, q);
            bool rel = false;
            if (dl >= 0 && lvl[dl] == 0 && cnt_dec(cnt, dl) == 1u) {
              rel = true;
              lvl[dl] = kTrimmed;
            }
            wave_push16(rel, dl, que, tb, tail, n);
          }
        }
        __syncthreads();
        ta = tb;
        tb += *tail;
        if (tb > n) return;
      }
    }
    // ---- strongly connected groups of the untrimmed ghosts (ascending)
    int32_t* res = tab;
    int32_t* rep = tab + kMaxResidual;
    int32_t* slot = tab + 2 * kMaxResidual;
    int m = 0;
    for (int b0 = 0; b0 < n; b0 += 1024) {
      const int g = b0 + tid;
      const bool left = g < n && lvl[g] == 0;
      int64_t tot;
      const int64_t pre = block_excl_scan<1024>(left ? 1 : 0, &tot, sh);
      if (left && m + pre < kMaxResidual) res[m + pre] = g;
      m += (int)tot;
    }
    if (m == 0 || m > kMaxResidual) return;
    uint32_t* reach = L.reach + (int64_t)ii * kMaxResidual * (kMaxResidual / 32);
    const int RW = (m + 31) / 32;
    for (int t = tid; t < m * RW; t += 1024) reach[t] = 0;
    __threadfence_block();
    __syncthreads();
    for (int u = tid; u < m; u += 1024)
      for (int q = 0; q < np; ++q) {
        const int d = dep(res[u], q);
        if (d < 0 || lvl[d] != 0) continue;
        const int v = (int)find_sorted(res, 0, m, d);
        if (v >= 0) reach[u * RW + (v >> 5)] |= 1u << (v & 31);
      }
    __threadfence_block();
    __syncthreads();
    do {
      if (tid == 0) s_flag = 0;
      __syncthreads();
      int changed = 0;
      for (int u = tid; u < m; u += 1024)
        for (int q = 0; q < np; ++q) {
          const int d = dep(res[u], q);
          if (d < 0 || lvl[d] != 0) continue;
          const int v = (int)find_sorted(res, 0, m, d);
          if (v < 0) continue;
          for (int w = 0; w < RW; ++w) {
            const uint32_t ow = reach[u * RW + w], nw = ow | reach[v * RW + w];
            if (nw != ow) {
              reach[u * RW + w] = nw;
              changed = 1;
            }
          }
        }
      if (changed) s_flag = 1;
      __threadfence_block();
      __syncthreads();
    } while (s_flag);
    // representative: smallest member of the group; -1 off cycles
    for (int u = tid; u < m; u += 1024) {
      int rp = -1;
      if ((reach[u * RW + (u >> 5)] >> (u & 31)) & 1u)
        for (int v = 0; v < m; ++v)
          if (((reach[u * RW + (v >> 5)] >> (v & 31)) & 1u) &&
              ((reach[v * RW + (u >> 5)] >> (u & 31)) & 1u)) {
            rp = v;
            break;
          }
      rep[u] = rp;
    }
    __syncthreads();
    {
      int off = 0;
      for (int b0 = 0; b0 < m; b0 += 1024) {
        const int u = b0 + tid;
        const bool isrep = u < m && rep[u] == u;
        int64_t tot;
        const int64_t pre = block_excl_scan<1024>(isrep ? 1 : 0, &tot, sh);
        if (isrep) slot[u] = off + (int)pre;
        off += (int)tot;
      }
      if (tid == 0) s_units = off;
    }
    __syncthreads();
    if (s_units > kMaxUnits) return;
    for (int u = tid; u < m; u += 1024) {
      const int rp = rep[u];
      if (rp < 0) continue;
      int rank = 0, size = 0;
      for (int v = 0; v < m; ++v)
        if (rep[v] == rp) {
          if (v < u) ++rank;
          ++size;
        }
      if (size > kMaxUnit) {   // larger than the LDS solve's workspace
        s_bad = 1;
        continue;
      }
      const int sl = slot[rp];
      unit_mem[sl * kMaxUnit + rank] = (int32_t)(lo + res[u]);
      blk_idx[lo + res[u]] = sl;
      if (dlds) uslot[res[u]] = (uint16_t)sl;
      if (u == rp) {
        unit_cnt[sl] = size;
        s_uhead[sl] = (uint16_t)res[u];
        s_usize[sl] = (uint8_t)size;
        atomicMax(&s_maxunit, size);
      }
    }
    for (int g = tid; g < n; g += 1024)
      if (lvl[g] == kTrimmed) lvl[g] = 0;
    __threadfence_block();
    __syncthreads();
    if (s_bad) return;

    // ---- the unplaced ghosts and units in dependency order, each at 1 +
    // the highest level it reads (internal edges of a unit excluded)
    auto head_of = [&](int g) {
      const int u = slot_of(g);
      return u >= 0 ? (int)s_uhead[u] : g;
    };
    auto place = [&](int t) {   // level of node t, given to its members
      const int u = slot_of(t);
      const int sz = u >= 0 ? (int)s_usize[u] : 1;
      int mx = 0;
      for (int j = 0; j < sz; ++j) {
        const int gm = u >= 0 ? (int)(unit_mem[u * kMaxUnit + j] - lo) : t;
        for (int q = 0; q < np; ++q) {
          const int d = dep(gm, q);
          if (d < 0 || (u >= 0 && slot_of(d) == u)) continue;
          mx = max(mx, (int)lvl[d]);
        }
      }
      for (int j = 0; j < sz; ++j) {
        const int gm = u >= 0 ? (int)(unit_mem[u * kMaxUnit + j] - lo) : t;
        lvl[gm] = (uint16_t)(mx + 1);
      }
      if (u >= 0) unit_lev[u] = mx + 1;
      atomicAdd(&s_placed, sz);
      atomicMax(&s_maxlev, mx + 1);
    };
    for (int w = tid; w < C; w += 1024) cnt[w] = 0;
    __syncthreads();
    for (int g = tid; g < n; g += 1024) {
      if (lvl[g] != 0) continue;
      const int u = slot_of(g);
      uint32_t c = 0;
      for (int q = 0; q < np; ++q) {
        const int d = dep(g, q);
        if (d < 0 || lvl[d] != 0 || (u >= 0 && slot_of(d) == u)) continue;
        ++c;
      }
      if (c) cnt_add(cnt, head_of(g), c);
    }
    if (tid < 3) s_cnt[tid] = 0;
    __syncthreads();
    for (int g = tid; g < n; g += 1024) {
      bool p = false;
      if (lvl[g] == 0 && head_of(g) == g && cnt_get(cnt, g) == 0) p = true;
      if (p) place(g);
      wave_push16(p, g, que, b, &s_cnt[0], n);
    }
    __threadfence_block();
    __syncthreads();
    int ra = b, rb = b + s_cnt[0], r = 0;
    while (ra < rb) {
      ++r;
      if (tid == 0) s_cnt[(r + 1) % 3] = 0;
      int* const tail = &s_cnt[r % 3];
      for (int i = ra + tid; i < rb; i += 1024) {
        const int t = que[i];
        const int u = slot_of(t);
        const int sz = u >= 0 ? (int)s_usize[u] : 1;
        for (int j = 0; j < sz; ++j) {
          const int gm = u >= 0 ? (int)(unit_mem[u * kMaxUnit + j] - lo) : t;
          int ea, eb;
          edge_range(gm, ea, eb);
          for (int e = ea; e < eb; ++e) {
            const int q = dependant(e);
            bool rel = false;
            int tq = 0;
            if (lvl[q] == 0) {   // members of t's own unit are placed already
              tq = head_of(q);
              if (cnt_dec(cnt, tq) == 1u) {
                rel = true;
                place(tq);
              }
            }
            wave_push16(rel, tq, que, rb, tail, n);
          }
        }
      }
      __threadfence_block();
      __syncthreads();
      ra = rb;
      rb += *tail;
      if (rb > n) return;
    }
  }
  __syncthreads();
  if (s_placed != n || s_maxlev > kFastLevels) return;   // k_levels does it
  const int nlev = s_maxlev;

  // ---- stable counting sort by level: wave w takes linear positions
  // [w R, (w + 1) R)
  const int R = ((((n + kFastWaves - 1) / kFastWaves) + 63) / 64) * 64;
  const int wv = tid >> 6, lane = tid & 63;
  for (int t = tid; t < kFastWaves * nlev; t += 1024) tab[t] = 0;
  __syncthreads();
  const int r0 = wv * R, r1 = min(n, r0 + R);
  for (int g = r0 + lane; g < r1; g += 64) atomicAdd(&tab[wv * nlev + lvl[g] - 1], 1);
  __syncthreads();
  for (int l = tid; l < nlev; l += 1024) {
    int t = 0;
    for (int w = 0; w < kFastWaves; ++w) t += tab[w * nlev + l];
    s_tot[l] = t;
  }
  __syncthreads();
  {
    const int v = tid < nlev ? s_tot[tid] : 0;
    int64_t tot;
    const int64_t pre = block_excl_scan<1024>(v, &tot, sh);
    if (tid < nlev) s_off[tid] = (int)pre;
    if (tid == 0) s_off[nlev] = (int)tot;
  }
  __syncthreads();
  for (int l = tid; l < nlev; l += 1024) {
    int run = s_off[l];
    for (int w = 0; w < kFastWaves; ++w) {
      const int t = tab[w * nlev + l];
      tab[w * nlev + l] = run;
      run += t;
    }
  }
  __syncthreads();
  int32_t* __restrict__ lev = L.lev + lo;
  int32_t* __restrict__ perm = L.perm + lo;
  static_assert(kFastLevels <= 256, "a level index fits 8 ballots");
  for (int c = r0; c < r1; c += 64) {
    const int g = c + lane;
    const bool valid = g < r1;
    const int l = valid ? (int)lvl[g] - 1 : -1;
    // the lanes of this lane's level: those that agree with it on every bit
    // of the level index, one ballot a bit
    unsigned long long mk = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool on = (l >> bit) & 1;
      const unsigned long long bb = __ballot(valid && on);
      mk &= on ? bb : ~bb;
    }
    const int at = valid ? tab[wv * nlev + l] : 0;
    __builtin_amdgcn_wave_barrier();
    if (valid && lane == __ffsll((long long)mk) - 1) tab[wv * nlev + l] = at + __popcll(mk);
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      lev[g] = l + 1;
      perm[g] = at + __popcll(mk & ((1ull << lane) - 1ull));
    }
  }
  int32_t* lev_off = L.lev_off + (int64_t)ii * (kMaxLevels + 1);
  for (int l = tid; l <= nlev; l += 1024) lev_off[l] = s_off[l];
  if (tid == 0) {
    int maxw = 0;
    for (int l = 0; l < nlev; ++l) maxw = max(maxw, s_tot[l]);
    L.info[ii].nlev = nlev;
    L.info[ii].maxwidth = maxw;
    L.info[ii].nunits = s_units;
    L.info[ii].maxunit = s_maxunit;
    L.info[ii].layered = 1;
  }
}

constexpr int kRelU = 4;   // ghosts per thread whose releases are issued together
constexpr int kRelE = 4;   // their edges loaded up front (the rest, if any, one by one)

// InLds: byte counters and level bitmap in LDS; CurLds: the current level's
// list too (it is written and read back within each level)
template <bool InLds, bool CurLds>
__global__ __launch_bounds__(1024) void k_levels(LevelsArgs L) {
  extern __shared__ uint32_t s_dyn[];
  // after a finished wide or LDS layering there is nothing left to do
  if (L.wide && L.wide[0] == 1) return;
  const int ii = blockIdx.x;
  if (L.info[ii].layered) return;
  const int tid = threadIdx.x;
  const int np = (1 << L.insts[ii].g.dim) - 1;
  const int64_t lo = L.g_off[ii];
  const int n = (int)(L.g_off[ii + 1] - lo);
  const int W = (n + 31) >> 5;   // bitmap words
  const int C = (n + 3) >> 2;    // counter words
  const int64_t cap = L.cap;
  const int32_t* __restrict__ deps = L.deps;
  int32_t* __restrict__ lev = L.lev;
  int32_t* __restrict__ blk_idx = L.blk_idx;
  int32_t* __restrict__ perm = L.perm;
  const uint8_t* __restrict__ dcnt = L.dcnt + lo;
  const int32_t* __restrict__ roff = L.roff + lo;   // global ids in radj
  const int32_t* __restrict__ radj = L.radj;
  int32_t* lev_off = L.lev_off + (int64_t)ii * (kMaxLevels + 1);
  int32_t* unit_mem = L.unit_mem + (int64_t)ii * kMaxUnits * kMaxUnit;
  int32_t* unit_cnt = L.unit_cnt + (int64_t)ii * kMaxUnits;
  int32_t* unit_lev = L.unit_lev + (int64_t)ii * kMaxUnits;
  uint32_t* reach = L.reach + (int64_t)ii * kMaxResidual * (kMaxResidual / 32);
  // the level list: its first cur_cap entries in LDS after the counters
  // and bitmap (the rest, if a level is wider, in HBM)
  int32_t* gcur = L.listA + lo;
  int32_t* lcur = CurLds ? reinterpret_cast<int32_t*>(s_dyn + C + W) : nullptr;
  const int ccap = CurLds ? L.cur_cap : 0;
  // instance ii owns words [(lo >> 2) + ii, + C) and [(lo >> 5) + ii, + W):
  // the next instance starts at ((lo + n) >> 2) + ii + 1 >= that end
  uint32_t* cnt = InLds ? s_dyn : L.cnt + (lo >> 2) + ii;
  uint32_t* bits = InLds ? s_dyn + C : L.bits + (lo >> 5) + ii;

  __shared__ int64_t sh[17];
  __shared__ int s_flag, s_units, s_maxunit;
  __shared__ int32_t res[kMaxResidual];
  __shared__ int32_t rep[kMaxResidual];
  __shared__ int32_t slot[kMaxResidual];

  for (int g = tid; g < n; g += 1024) blk_idx[lo + g] = -1;
  if (tid == 0) {
    lev_off[0] = 0;
    s_units = 0;
    s_maxunit = 0;
  }
  __syncthreads();

  bool units = false;
  int k = 0, placed = 0, maxwidth = 0;
  uint32_t err = 0;
  for (;;) {
    // ---- counters of unplaced ghosts read (per ghost, or per unit on its
    // first member), internal edges of a unit excluded
    for (int g = tid; g < n; g += 1024) {
      lev[lo + g] = 0;
      perm[lo + g] = -1;
    }
    if (!units) {
      // four counters per word, and level 1 = ghosts that read no ghost
      for (int w = tid; w < C; w += 1024) {
        uint32_t v = 0;
        for (int q = 0; q < 4; ++q)
          if (4 * w + q < n) v |= (uint32_t)dcnt[4 * w + q] << (8 * q);
        cnt[w] = v;
      }
      // level-1 bitmap: each wave reads 64 consecutive counts (one byte per
      // lane) and writes the two words of their ballot
      for (int g0 = tid & ~63; g0 < n; g0 += 1024) {
        const int g = g0 + (tid & 63);
        const unsigned long long m = __ballot(g < n && dcnt[g] == 0);
        if ((tid & 63) == 0) {
          bits[g0 >> 5] = (uint32_t)m;
          if ((g0 >> 5) + 1 < W) bits[(g0 >> 5) + 1] = (uint32_t)(m >> 32);
        }
      }
      __syncthreads();
    } else {
      for (int w = tid; w < C; w += 1024) cnt[w] = 0;
      for (int w = tid; w < W; w += 1024) bits[w] = 0;
      __syncthreads();
      for (int g = tid; g < n; g += 1024) {
        const int u = blk_idx[lo + g];
        const int tgt = u >= 0 ? (int)(unit_mem[u * kMaxUnit] - lo) : g;
        uint32_t c = 0;
        for (int m = 0; m < np; ++m) {
          const int32_t d = deps[(int64_t)m * cap + lo + g];
          if (d >= 0 && !(u >= 0 && blk_idx[d] == u)) ++c;
        }
        if (c) cnt_add(cnt, tgt, c);
      }
      __syncthreads();
      // level 1: nodes that read no unplaced ghost
      for (int g = tid; g < n; g += 1024) {
        const int u = blk_idx[lo + g];
        if (u >= 0 && unit_mem[u * kMaxUnit] - lo != g) continue;
        if (cnt_get(cnt, g) != 0) continue;
        if (u >= 0) {
          unit_lev[u] = 1;
          for (int q = 0; q < unit_cnt[u]; ++q) {
            const int v = (int)(unit_mem[u * kMaxUnit + q] - lo);
            atomicOr(&bits[v >> 5], 1u << (v & 31));
          }
        } else {
          atomicOr(&bits[g >> 5], 1u << (g & 31));
        }
      }
      __syncthreads();
    }

    k = 0;
    placed = 0;
    maxwidth = 0;
    for (;;) {
      // ---- emit the next level from the bitmap, in linear-index order
      int newly = 0;
      for (int base = 0; base < W; base += 1024) {
        const int w = base + tid;
        uint32_t word = w < W ? bits[w] : 0u;
        int64_t tot;
        const int64_t pre = block_excl_scan<1024>(__popc(word), &tot, sh);
        if (word) {
          bits[w] = 0u;
          int pos = newly + (int)pre;
          while (word) {
            const int b = __ffs(word) - 1;
            word &= word - 1;
            const int g = w * 32 + b;
            if (pos < ccap) lcur[pos] = g;
            else gcur[pos] = g;
            perm[lo + g] = placed + pos;
            lev[lo + g] = k + 1;
            ++pos;
          }
        }
        newly += (int)tot;
      }
      if (newly == 0) break;
      ++k;
      if (k > kMaxLevels) {
        err |= kErrUnsupported;
        break;
      }
      placed += newly;
      maxwidth = max(maxwidth, newly);
      if (tid == 0) lev_off[k] = placed;
      __syncthreads();
      // ---- dependants of level k: the last edge into a node releases it.
      // A thread takes kRelU ghosts of the level at a time and issues their
      // loads together (list entry, edge range, first kRelE edges), so the
      // dependent global round trips are paid once per group, not per ghost;
      // the order of releases does not matter (a counter reaching zero sets
      // a bit of the next level's bitmap)
      auto release = [&](int rg, int ug) {
        const int r = (int)(rg - lo);
        const int ur = units ? blk_idx[lo + r] : -1;
        if (ur >= 0 && ur == ug) return;
        const int tgt = ur >= 0 ? (int)(unit_mem[ur * kMaxUnit] - lo) : r;
        if (cnt_dec(cnt, tgt) != 1u) return;
        if (ur >= 0) {
          unit_lev[ur] = k + 1;
          for (int q = 0; q < unit_cnt[ur]; ++q) {
            const int v = (int)(unit_mem[ur * kMaxUnit + q] - lo);
            atomicOr(&bits[v >> 5], 1u << (v & 31));
          }
        } else {
          atomicOr(&bits[r >> 5], 1u << (r & 31));
        }
      };
      for (int i0 = tid; i0 < newly; i0 += 1024 * kRelU) {
        int gg[kRelU], ea[kRelU], eb[kRelU], rr[kRelU][kRelE];
#pragma unroll
        for (int u = 0; u < kRelU; ++u) {
          const int i = i0 + u * 1024;
          gg[u] = i >= newly ? -1 : i < ccap ? lcur[i] : gcur[i];
        }
#pragma unroll
        for (int u = 0; u < kRelU; ++u) {
          ea[u] = gg[u] >= 0 ? roff[gg[u]] : 0;
          eb[u] = gg[u] >= 0 ? roff[gg[u] + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < kRelU; ++u)
#pragma unroll
          for (int q = 0; q < kRelE; ++q) rr[u][q] = ea[u] + q < eb[u] ? radj[ea[u] + q] : -1;
#pragma unroll
        for (int u = 0; u < kRelU; ++u) {
          if (gg[u] < 0) continue;
          const int ug = units ? blk_idx[lo + gg[u]] : -1;
#pragma unroll
          for (int q = 0; q < kRelE; ++q)
            if (rr[u][q] >= 0) release(rr[u][q], ug);
          for (int e = ea[u] + kRelE; e < eb[u]; ++e) release(radj[e], ug);
        }
      }
      __syncthreads();
    }
    if (err || placed == n) break;
    if (units) {
      err |= kErrCycle;
      break;
    }

    // ---- the unplaced ghosts (ascending) hold cycles
    int m = 0;
    for (int base = 0; base < n; base += 1024) {
      const int g = base + tid;
      const bool left = g < n && lev[lo + g] == 0;
      int64_t tot;
      const int64_t pre = block_excl_scan<1024>(left ? 1 : 0, &tot, sh);
      if (left && m + pre < kMaxResidual) res[m + pre] = g;
      m += (int)tot;
    }
    if (m > kMaxResidual) {   // workspace capacity, not a property of the graph
      err |= kErrUnsupported;
      break;
    }
    const int RW = (m + 31) / 32;
    for (int t = tid; t < m * RW; t += 1024) reach[t] = 0;
    __syncthreads();
    for (int u = tid; u < m; u += 1024) {
      for (int q = 0; q < np; ++q) {
        const int32_t d = deps[(int64_t)q * cap + lo + res[u]];
        if (d >= 0 && lev[d] == 0) {
          const int v = (int)find_sorted(res, 0, m, (int)(d - lo));
          if (v >= 0) reach[u * RW + (v >> 5)] |= 1u << (v & 31);
        }
      }
    }
    __threadfence_block();
    __syncthreads();
    do {
      if (tid == 0) s_flag = 0;
      __syncthreads();
      int changed = 0;
      for (int u = tid; u < m; u += 1024) {
        for (int q = 0; q < np; ++q) {
          const int32_t d = deps[(int64_t)q * cap + lo + res[u]];
          if (d < 0 || lev[d] != 0) continue;
          const int v = (int)find_sorted(res, 0, m, (int)(d - lo));
          if (v < 0) continue;
          for (int w = 0; w < RW; ++w) {
            const uint32_t o = reach[u * RW + w], nw = o | reach[v * RW + w];
            if (nw != o) {
              reach[u * RW + w] = nw;
              changed = 1;
            }
          }
        }
      }
      if (changed) s_flag = 1;
      __threadfence_block();
      __syncthreads();
    } while (s_flag);
    // representative = smallest member of the group; -1 off cycles
    for (int u = tid; u < m; u += 1024) {
      int rp = -1;
      if ((reach[u * RW + (u >> 5)] >> (u & 31)) & 1u) {
        for (int v = 0; v < m; ++v)
          if (((reach[u * RW + (v >> 5)] >> (v & 31)) & 1u) &&
              ((reach[v * RW + (u >> 5)] >> (u & 31)) & 1u)) {
            rp = v;
            break;
          }
      }
      rep[u] = rp;
    }
    __syncthreads();
    {
      int off = 0;
      for (int base = 0; base < m; base += 1024) {
        const int u = base + tid;
        const bool isrep = u < m && rep[u] == u;
        int64_t tot;
        const int64_t pre = block_excl_scan<1024>(isrep ? 1 : 0, &tot, sh);
        if (isrep) slot[u] = off + (int)pre;
        off += (int)tot;
      }
      if (tid == 0) s_units = off;
    }
    __syncthreads();
    if (s_units > kMaxUnits) {
      err |= kErrUnsupported;
      break;
    }
    for (int u = tid; u < m; u += 1024) {
      const int rp = rep[u];
      if (rp < 0) continue;
      int rank = 0, size = 0;
      for (int v = 0; v < m; ++v)
        if (rep[v] == rp) {
          if (v < u) ++rank;
          ++size;
        }
      if (size > kMaxUnit) {   // larger than the LDS solve's workspace
        atomicOr(&L.info[ii].err, kErrUnsupported);
        continue;
      }
      const int sl = slot[rp];
      unit_mem[sl * kMaxUnit + rank] = (int32_t)(lo + res[u]);
      blk_idx[lo + res[u]] = sl;
      if (u == rp) {
        unit_cnt[sl] = size;
        atomicMax(&s_maxunit, size);
      }
    }
    __syncthreads();
    if (L.info[ii].err & kErrUnsupported) break;
    units = true;   // restart the layering with the units as nodes
  }
  if (tid == 0) {
    if (err) atomicOr(&L.info[ii].err, err);
    L.info[ii].nlev = k;
    L.info[ii].maxwidth = maxwidth;
    L.info[ii].nunits = units ? s_units : 0;
    L.info[ii].maxunit = s_maxunit;
  }
}

// Counters and bitmap in LDS when the largest instance fits, else in HBM.
gcr_status launch_levels(const LevelsArgs& L, int ninst, int64_t max_n, hipStream_t st) {
  // device limits, taken once; the LDS attribute only grows, under the lock,
  // so builds on several host threads never launch beyond it
  static std::mutex mu;
  static int lds_max = -1;
  std::unique_lock<std::mutex> lk(mu);
  if (lds_max < 0) {
    int dev = 0, a = 0, b = 0;
    (void)hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      a = 0;
    if (hipDeviceGetAttribute(&b, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess)
      b = 0;
    (void)hipGetLastError();
    hipFuncAttributes fa{};
    int stat = 8192;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_levels<true, true>)) ==
        hipSuccess)
      stat = (int)fa.sharedSizeBytes;
    (void)hipGetLastError();
    lds_max = std::max(0, std::max(a, b) - stat - 256);
  }
  const int lds_avail = lds_max;
  lk.unlock();
  const int64_t nn = std::max<int64_t>(max_n, 1);
  const int64_t bytes = 4 * (((nn + 3) >> 2) + ((nn + 31) >> 5));
  LevelsArgs F = L;   // the one-workgroup layering
  F.wide = nullptr;
  if (!(L.wide && ninst == 1 && wide_layering_forced())) {
    // the LDS layering first (an instance that fits it is layered there even
    // when the wide layering is armed, unless a threshold set explicitly
    // forces it); k_levels_wide and k_levels below skip what it finished
    static int fast_lds = -1;
    lk.lock();
    if (fast_lds < 0) {
      int dev = 0, a = 0, b = 0;
      (void)hipGetDevice(&dev);
      if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        a = 0;
      if (hipDeviceGetAttribute(&b, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess)
        b = 0;
      hipFuncAttributes fa{};
      int stat = 4096;
      if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_levels_fast)) == hipSuccess)
        stat = (int)fa.sharedSizeBytes;
      (void)hipGetLastError();
      int v = std::max(0, std::max(a, b) - stat - 256) & ~255;
      if (v > 0 && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_levels_fast),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, v) != hipSuccess) {
        (void)hipGetLastError();
        v = 0;
      }
      fast_lds = v;
    }
    const int fl = fast_lds;
    lk.unlock();
    if (fl > 0) k_levels_fast<<<ninst, 1024, (size_t)fl, st>>>(L, fl);
  }
  if (L.wide && ninst == 1) {
    // grid: as many co-resident workgroups as fit, at most one per tile
    static int coop = -1;
    lk.lock();
    if (coop < 0) {
      int dev = 0, ncu = 0, per = 0;
      (void)hipGetDevice(&dev);
      if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
              &per, reinterpret_cast<const void*>(&k_levels_wide), 256, 0) != hipSuccess)
        per = 0;
      (void)hipGetLastError();
      coop = std::max(0, std::min(per, 1) * ncu);
    }
    const int coop_n = coop;
    lk.unlock();
    const int64_t G = std::min<int64_t>(coop_n, std::max<int64_t>(1, (nn + 255) >> 8));
    if (G > 0) {
      LevelsArgs A = L;
      void* args[] = {&A};
      GCR_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_levels_wide),
                                         dim3((unsigned)G), dim3(256), args, 0, st));
      F.wide = L.wide;
    }
  }
  // what LDS is left holds the level list (worth it from a few thousand)
  const int64_t cur_cap =
      bytes <= lds_avail ? std::min<int64_t>(nn, (lds_avail - bytes) / 4) : 0;
  const int64_t bytes_cur = bytes + 4 * cur_cap;
  F.cur_cap = (int)cur_cap;
  if (cur_cap >= 2048) {
    static int64_t attr = 0;
    lk.lock();
    if (bytes_cur > attr) {
      GCR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_levels<true, true>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes_cur));
      attr = bytes_cur;
    }
    lk.unlock();
    k_levels<true, true><<<ninst, 1024, (size_t)bytes_cur, st>>>(F);
  } else if (bytes <= lds_avail) {
    static int64_t attr = 0;
    lk.lock();
    if (bytes > attr) {
      GCR_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_levels<true, false>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
      attr = bytes;
    }
    lk.unlock();
    k_levels<true, false><<<ninst, 1024, (size_t)bytes, st>>>(F);
  } else {
    k_levels<false, false><<<ninst, 1024, 0, st>>>(F);
  }
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

}  // namespace gcr
