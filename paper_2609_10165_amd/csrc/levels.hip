// levels.hip -- Kahn layering of the ghost dependency graph (Sec. 3.2) and
// the canonical order (level, linear index), one workgroup per instance.
//
// Iteration k examines only the ghosts not yet placed, kept in linear-index
// order in a list; one packed workgroup scan per 1024 ghosts gives both the
// canonical positions of the ghosts placed at level k and the next list (so
// the work is the sum of the list lengths, not levels x ghosts).  Levels
// live in LDS when the instance fits.  A ghost is ready at k when every
// ghost it reads has a level in 1..k-1, so decisions do not depend on the
// order threads run in.  If an iteration places nothing, the remaining
// ghosts hold cycles: their strongly connected groups (from the transitive
// closure of the remaining graph) become coupled units and the layering
// restarts with them, so each unit sits one level above the deepest level it
// needs.
#include <hip/hip_runtime.h>

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

template <bool InLds>
__global__ __launch_bounds__(1024) void k_levels(LevelsArgs L) {
  extern __shared__ uint16_t s_lev[];
  const int ii = blockIdx.x;
  const int tid = threadIdx.x;
  const int np = (1 << L.insts[ii].g.dim) - 1;
  const int64_t lo = L.g_off[ii];
  const int n = (int)(L.g_off[ii + 1] - lo);
  const int64_t cap = L.cap;
  const int32_t* __restrict__ deps = L.deps;
  int32_t* __restrict__ lev = L.lev;
  int32_t* __restrict__ blk_idx = L.blk_idx;
  int32_t* __restrict__ perm = L.perm;
  int32_t* lev_off = L.lev_off + (int64_t)ii * (kMaxLevels + 1);
  int32_t* unit_mem = L.unit_mem + (int64_t)ii * kMaxUnits * kMaxUnit;
  int32_t* unit_cnt = L.unit_cnt + (int64_t)ii * kMaxUnits;
  int32_t* unit_lev = L.unit_lev + (int64_t)ii * kMaxUnits;
  uint32_t* reach = L.reach + (int64_t)ii * kMaxResidual * (kMaxResidual / 32);
  int32_t* listA = L.listA + lo;
  int32_t* listB = L.listB + lo;

  // level of ghost d (global linear-order position); 0 = not placed
  auto LEV = [&](int64_t d) -> int { return InLds ? (int)s_lev[d - lo] : lev[d]; };
  auto SET = [&](int g, int v) {
    if (InLds) s_lev[g] = (uint16_t)v;
    lev[lo + g] = v;
  };

  __shared__ int64_t sh[17];
  __shared__ int s_flag, s_units, s_maxunit;
  __shared__ int32_t res[kMaxResidual];
  __shared__ int32_t rep[kMaxResidual];
  __shared__ int32_t slot[kMaxResidual];

  for (int g = tid; g < n; g += 1024) {
    SET(g, 0);
    blk_idx[lo + g] = -1;
    perm[lo + g] = -1;
    listA[g] = g;
  }
  if (tid == 0) {
    lev_off[0] = 0;
    s_units = 0;
    s_maxunit = 0;
  }
  __syncthreads();

  int32_t* cur = listA;
  int32_t* nxt = listB;
  int nrem = n, placed = 0, k = 0, maxwidth = 0;
  bool units = false;
  uint32_t err = 0;
  while (nrem > 0) {
    ++k;
    if (k > kMaxLevels) {
      err |= kErrUnsupported;
      break;
    }
    int newly = 0, kept = 0;
    for (int base = 0; base < nrem; base += 1024) {
      const int idx = base + tid;
      const int g = idx < nrem ? cur[idx] : -1;
      bool ready = false;
      if (g >= 0) {
        const int u = units ? blk_idx[lo + g] : -1;
        ready = true;
        if (u < 0) {
          for (int m = 0; m < np && ready; ++m) {
            const int32_t d = deps[(int64_t)m * cap + lo + g];
            if (d >= 0) {
              const int ld = LEV(d);
              if (ld == 0 || ld >= k) ready = false;
            }
          }
        } else {
          const int cntu = unit_cnt[u];
          for (int q = 0; q < cntu && ready; ++q) {
            const int32_t w = unit_mem[u * kMaxUnit + q];
            for (int m = 0; m < np && ready; ++m) {
              const int32_t d = deps[(int64_t)m * cap + w];
              if (d >= 0 && blk_idx[d] != u) {
                const int ld = LEV(d);
                if (ld == 0 || ld >= k) ready = false;
              }
            }
          }
          if (ready) unit_lev[u] = k;
        }
      }
      const int64_t packed = ready ? 1 : (g >= 0 ? (int64_t(1) << 32) : 0);
      int64_t tot;
      const int64_t pre = block_excl_scan<1024>(packed, &tot, sh);
      if (ready) {
        perm[lo + g] = placed + newly + (int)(pre & 0xffffffff);
        SET(g, k);
      } else if (g >= 0) {
        nxt[kept + (int)(pre >> 32)] = g;
      }
      newly += (int)(tot & 0xffffffff);
      kept += (int)(tot >> 32);
    }
    __syncthreads();
    if (newly == 0) {
      if (units) {
        err |= kErrCycle;
        break;
      }
      // the remaining ghosts (ascending, in cur) hold cycles
      const int m = nrem;
      if (m > kMaxResidual) {
        err |= kErrCycle;
        break;
      }
      for (int u = tid; u < m; u += 1024) res[u] = cur[u];
      const int W = (m + 31) / 32;
      for (int t = tid; t < m * W; t += 1024) reach[t] = 0;
      __syncthreads();
      for (int u = tid; u < m; u += 1024) {
        for (int q = 0; q < np; ++q) {
          const int32_t d = deps[(int64_t)q * cap + lo + res[u]];
          if (d >= 0 && LEV(d) == 0) {
            const int v = (int)find_sorted(res, 0, m, (int)(d - lo));
            if (v >= 0) reach[u * W + (v >> 5)] |= 1u << (v & 31);
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
            if (d < 0 || LEV(d) != 0) continue;
            const int v = (int)find_sorted(res, 0, m, (int)(d - lo));
            if (v < 0) continue;
            for (int w = 0; w < W; ++w) {
              const uint32_t o = reach[u * W + w], nw = o | reach[v * W + w];
              if (nw != o) {
                reach[u * W + w] = nw;
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
        if ((reach[u * W + (u >> 5)] >> (u & 31)) & 1u) {
          for (int v = 0; v < m; ++v)
            if (((reach[u * W + (v >> 5)] >> (v & 31)) & 1u) &&
                ((reach[v * W + (u >> 5)] >> (u & 31)) & 1u)) {
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
        err |= kErrCycle;
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
        if (size > kMaxUnit) {
          atomicOr(&L.info[ii].err, kErrCycle);
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
      // restart the layering with the units
      for (int g = tid; g < n; g += 1024) {
        SET(g, 0);
        perm[lo + g] = -1;
        listA[g] = g;
      }
      __syncthreads();
      cur = listA;
      nxt = listB;
      units = true;
      nrem = n;
      placed = 0;
      k = 0;
      maxwidth = 0;
      continue;
    }
    placed += newly;
    maxwidth = max(maxwidth, newly);
    if (tid == 0) lev_off[k] = placed;
    int32_t* t = cur;
    cur = nxt;
    nxt = t;
    nrem = kept;
  }
  if (tid == 0) {
    if (err) atomicOr(&L.info[ii].err, err);
    L.info[ii].nlev = k;
    L.info[ii].maxwidth = maxwidth;
    L.info[ii].nunits = units ? s_units : 0;
    L.info[ii].maxunit = s_maxunit;
  }
}

// Levels in LDS when the largest instance fits (uint16 per ghost).
constexpr int kLdsLevelCap = 64 * 1024;

void launch_levels(const LevelsArgs& L, int ninst, int64_t max_n, hipStream_t st) {
  if (max_n <= kLdsLevelCap) {
    static bool attr = false;
    const size_t bytes = (size_t)std::max<int64_t>(max_n, 1) * sizeof(uint16_t);
    if (!attr) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_levels<true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                kLdsLevelCap * (int)sizeof(uint16_t));
      attr = true;
    }
    k_levels<true><<<ninst, 1024, bytes, st>>>(L);
  } else {
    k_levels<false><<<ninst, 1024, 0, st>>>(L);
  }
}

}  // namespace gcr
