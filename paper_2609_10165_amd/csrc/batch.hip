// batch.hip -- batched forward: many uneven instances, several fields each,
// reconstructed in one persistent launch.
//
// Work items are (instance, field) pairs, largest first.  A workgroup takes
// items round-robin; for each it sweeps the instance's levels for that
// field (barrier between levels), then evaluates that field at the
// instance's surface points and reduces its share of the force:
//   pressure p:      -w p n
//   velocity u_c:    mu w (e_c (grad u_c . n) + n_c grad u_c)
// which sum over the fields to w (-p n + mu (grad u + grad u^T) n).  The
// last item of an instance to finish (device-scope counter, reset after use)
// adds the shares in field order, so the result does not depend on timing.
// A batch of few large instances instead sweeps each level with many
// workgroups of the instance together (k_batch_split: a device-scope counter
// between levels), then does the surface items the same way.  Workgroup
// size, grid and which of the two are picked by timing candidates on the
// first call for a kind of batch and remembered for the process.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <numeric>
#include <vector>

#include "gcr_fill.hpp"
#include "gcr_impl.hpp"

namespace gcr {

struct BStatic {
  const PlanD* plans;        // [ninst]
  const int32_t* const* lev_off;
  const int32_t* nlev;
};

struct BCall {
  int nf, ninst, p_field, u_first, nitems, pad;
  double mu;
  int kind[kMaxFields];
  double* const* fields;         // [ninst*nf]
  const double* const* bcv;      // [ninst*nf]
  const uint8_t* const* bct;     // [ninst*nf] (may hold nulls)
  const int64_t* nq;             // [ninst] or null (no forces)
  const double* const* xq;
  const double* const* nrm;
  const double* const* wq;
  const int32_t* order;          // [nitems] items w = i*nf + f
  const int64_t* aoff;           // [ninst + 1] first point of each instance (forces)
  const int32_t* anchor;         // [aoff[ninst]] anchor ghost of every point
  double* const* sval;           // [ninst*nf] surface values [nq_i] (null: none)
  double* const* sgrad;          // [ninst*nf] surface gradients [dim][nq_i] (null: none)
  const int32_t* tile_flag;      // tiled fill ran when set and zero: items skip the levels
};

// Anchor ghost of every surface point of every instance, one group of lanes
// per point (the search is geometry only, so the fields' items share it).
// With a row of workgroups per instance (gridDim.y = instances) a workgroup
// knows its instance; otherwise (one row) each point searches the offsets.
template <int D>
__global__ __launch_bounds__(256) void k_batch_anchor(BStatic S, BCall C, int64_t npts,
                                                      int32_t* __restrict__ anchor) {
  constexpr int NL = anchor_lanes<D>();
  constexpr int PPB = 256 / NL;
  const int sub = (int)threadIdx.x % NL;
  const int64_t pb = (int64_t)blockIdx.x * PPB + (int)threadIdx.x / NL;
  int i = 0;
  int64_t q = 0, gq = 0;
  bool active;
  if (gridDim.y > 1) {
    i = (int)blockIdx.y;
    q = pb;
    active = q < C.nq[i];
    gq = C.aoff[i] + q;
  } else {
    gq = pb;
    active = gq < npts;
    if (active) {
      i = find_inst(C.aoff, C.ninst, gq);
      q = gq - C.aoff[i];
    }
  }
  double x[3] = {0.0, 0.0, 0.0};
  if (active) {
    const int64_t nq = C.nq[i];
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = C.xq[i][a * nq + q];
  }
  const int g = find_anchor_group<D, NL>(S.plans[i], x, sub, active);
  if (active && sub == 0) anchor[gq] = g;
}

// The surface part of item w = (instance, field), by a whole workgroup: the
// field's value and gradient at the instance's points (one box-polynomial
// evaluation serves both) and its share of the force, reduced over the
// workgroup in a fixed order; the last item of the instance to finish adds
// the shares in field order.
template <int D>
__device__ __forceinline__ void surface_item(const BStatic& S, const BCall& C, int w,
                                             double (*red)[3], double* __restrict__ part,
                                             int* __restrict__ counter,
                                             double* __restrict__ Fout) {
  const int T = blockDim.x;
  const int i = w / C.nf, f = w % C.nf;
  const PlanD& P = S.plans[i];
  const double* F = C.fields[w];
  // share of the force, and the field's value and gradient at the points
  // (one box-polynomial evaluation serves both)
  const int vc = f - C.u_first;
  const bool isp = f == C.p_field, isu = vc >= 0 && vc < D;
  double* const sv = C.sval ? C.sval[w] : nullptr;
  double* const sg = C.sgrad ? C.sgrad[w] : nullptr;
  double t[3] = {0.0, 0.0, 0.0};
  if (C.nq && (isp || isu || sv || sg)) {
    const int64_t nq = C.nq[i];
    const double* xq = C.xq[i];
    const double* nr = C.nrm[i];
    const double* wq = C.wq[i];
    for (int64_t q = threadIdx.x; q < nq; q += T) {
      double x[3] = {0.0, 0.0, 0.0}, n[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < D; ++a) {
        x[a] = xq[a * nq + q];
        n[a] = nr[a * nq + q];
      }
      const int g = C.anchor[C.aoff[i] + q];
      double val, gr[3];
      if (g < 0) {
        val = __longlong_as_double(0x7ff8000000000000LL);
        gr[0] = gr[1] = gr[2] = val;
      } else {
        int ii, jj, kk;
        unlinear(P.g, P.cell[g], ii, jj, kk);
        const int ijk[3] = {ii, jj, kk};
        double rel[3] = {0.0, 0.0, 0.0}, v[8];
#pragma unroll
        for (int a = 0; a < D; ++a) rel[a] = x[a] - centre(P.g, a, ijk[a]);
        corner_values<D>(P, g, F, v);
        double X[3];
        stencil_span(P.g, P.code[g], P.cell[g], X);
        box_eval<D>(rel, X, v, val, gr);
      }
      if (sv) sv[q] = val;
      if (sg)
#pragma unroll
        for (int a = 0; a < D; ++a) sg[a * nq + q] = gr[a];
      const double wt = wq[q];
      if (isp) {
#pragma unroll
        for (int a = 0; a < D; ++a) t[a] += -wt * val * n[a];
      } else if (isu) {
        double gn = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) gn += gr[a] * n[a];
#pragma unroll
        for (int a = 0; a < D; ++a) t[a] += C.mu * wt * ((a == vc ? gn : 0.0) + n[vc] * gr[a]);
      }
    }
  }
  for (int a = 0; a < 3; ++a) red[threadIdx.x][a] = t[a];
  __syncthreads();
  for (int s = T / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int a = 0; a < 3; ++a) red[threadIdx.x][a] += red[threadIdx.x + s][a];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    for (int a = 0; a < 3; ++a) part[(int64_t)w * 3 + a] = red[0][a];
    __threadfence();
    const int done = atomicAdd(&counter[i], 1);
    if (done == C.nf - 1) {
      __threadfence();
      double s3[3] = {0.0, 0.0, 0.0};
      for (int ff = 0; ff < C.nf; ++ff)
        for (int a = 0; a < 3; ++a)
          s3[a] += __hip_atomic_load(&part[((int64_t)i * C.nf + ff) * 3 + a], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
      for (int a = 0; a < 3; ++a) Fout[(int64_t)i * 3 + a] = s3[a];
      atomicExch(&counter[i], 0);
    }
  }
  __syncthreads();
}

// The levels of a 2D item, swept in LDS.  A prologue takes every ghost of
// the item at once: its weights (as fill_single computes them), the term of
// its boundary value, and per stencil corner either the product of weight
// and fluid value or, for a corner that is a ghost, the weight and that
// ghost's position, into a record of kRecWords doubles (bit 63 of the last
// word marks a member of a coupled unit).  The levels then read only LDS,
// the first word of each record becoming the ghost's value once computed;
// the terms are added in corner order, as fill_single adds them, and each
// level's coupled units are solved as fill_unit_field solves them, so the
// values are the same bits.  An epilogue stores the values into the field.
constexpr int kRecWords = 5;

// A load through a global-address-space pointer (the plan's and the
// field's arrays are device memory): a flat load would also count against
// the LDS wait counter that every LDS access of the sweep waits on.
template <class T>
__device__ __forceinline__ T gload(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}
constexpr int kRecUnitWS = 8;   // unit workspaces after the records
constexpr uint32_t kRecFluid = 0xffffu, kRecSkip = 0xfffeu;
constexpr uint64_t kRecMember = 1ull << 63;

// Coupled unit u of an LDS sweep: (I - W_int) phi = W_ext phi_ext + w0 b,
// assembled from the members' records in fill_unit_field's order.
__device__ __forceinline__ void unit_lds2(const PlanD& P, int u, double* rec, UnitWS& ws) {
  const int k = P.unit_cnt[u];
  for (int i = 0; i < k; ++i) ws.mem[i] = P.unit_mem[u * kMaxUnit + i];
  for (int i = 0; i < k; ++i) {
    const double* r = rec + (int64_t)kRecWords * ws.mem[i];
    const uint64_t pk = (uint64_t)__double_as_longlong(r[4]);
    for (int t = 0; t < k; ++t) ws.M[i * k + t] = (t == i) ? 1.0 : 0.0;
    double rr = r[0];
    for (int c = 1; c < 4; ++c) {
      const uint32_t id = (uint32_t)(pk >> (16 * (c - 1))) & 0xffffu;
      if (id == kRecSkip) continue;
      if (id == kRecFluid) {
        rr += r[c];
        continue;
      }
      int t = -1;
      for (int s = 0; s < k; ++s)
        if (ws.mem[s] == (int)id) t = s;
      if (t >= 0) ws.M[i * k + t] -= r[c];
      else rr += r[c] * rec[(int64_t)kRecWords * id];
    }
    ws.rhs[i] = rr;
  }
  ws_solve(ws, k);
  for (int i = 0; i < k; ++i) rec[(int64_t)kRecWords * ws.mem[i]] = ws.rhs[i];
}
__device__ __forceinline__ void sweep_lds2(const PlanD& P, const int32_t* __restrict__ lev_off,
                                           int nl, double* __restrict__ F,
                                           const double* __restrict__ b,
                                           const uint8_t* __restrict__ bt, int kind,
                                           double* rec, int rec_cap) {
  const int T = blockDim.x, tid = threadIdx.x;
  const int ng = P.ng;
  for (int p = tid; p < ng; p += T) {
    const int c = gload(P.cell + p);
    const uint32_t code = gload(P.code + p);
    double dl[3] = {gload(P.dl[0] + p), gload(P.dl[1] + p), 0.0},
           nn[3] = {gload(P.nn[0] + p), gload(P.nn[1] + p), 0.0}, w[8];
    const bool member = gload(P.blk + p) >= 0;
    const int bc = kind == 2 ? (int)gload(bt + p) : kind;
    const double bv = gload(b + p);
    int gi[4];
#pragma unroll
    for (int k = 1; k < 4; ++k) gi[k] = gload(P.cgi + (int64_t)(k - 1) * ng + p);
    double X[3];
    stencil_span(P.g, code, c, X);
    ghost_weights<2>(dl, nn, X, bc, w);
    double* r = rec + (int64_t)kRecWords * p;
    r[0] = w[0] * bv;
    uint64_t pk = member ? kRecMember : 0ull;
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      uint64_t id = kRecSkip;
      double t = 0.0;
      if (gi[k] >= 0) {
        id = (uint64_t)gi[k];
        t = w[k];
      } else if (gi[k] == -1) {
        id = kRecFluid;
        t = w[k] * gload(F + c + corner_offset(P.g, code, k));
      }
      r[k] = t;
      pk |= id << (16 * (k - 1));
    }
    r[4] = __longlong_as_double((long long)pk);
  }
  __syncthreads();
  // (read once: after a barrier every level would load it again)
  const int nunits = P.nunits;
  int unext = 0x7fffffff;
  if (tid < kRecUnitWS)
    for (int s = tid; s < nunits; s += kRecUnitWS) unext = min(unext, gload(P.unit_lev + s));
  // level offsets 64 at a time, lane j holding lev_off[base + j]: a level
  // reads its bounds from registers instead of memory
  const int lane = tid & 63;
  int vlev = 0, vnext = 0;
  for (int l = 0; l < nl; ++l) {
    if ((l & 63) == 0) {
      vlev = l + lane <= nl ? gload(lev_off + l + lane) : 0;
      vnext = l + 64 <= nl ? gload(lev_off + l + 64) : 0;
    }
    const int lo = __builtin_amdgcn_readlane(vlev, l & 63);
    const int hi = (l & 63) == 63 ? __builtin_amdgcn_readfirstlane(vnext)
                                  : __builtin_amdgcn_readlane(vlev, (l & 63) + 1);
    for (int p = lo + tid; p < hi; p += T) {
      // the record's words, then the three corners' ghost values, each
      // group read at once; the terms are added in corner order as before
      double* r = rec + (int64_t)kRecWords * p;
      double w[kRecWords];
#pragma unroll
      for (int k = 0; k < kRecWords; ++k) w[k] = r[k];
      const uint64_t pk = (uint64_t)__double_as_longlong(w[4]);
      if (pk & kRecMember) continue;   // solved with its unit below
      uint32_t id[3];
      double gv[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        id[k] = (uint32_t)(pk >> (16 * k)) & 0xffffu;
        gv[k] = rec[(int64_t)kRecWords * (id[k] < kRecSkip ? (int)id[k] : p)];
      }
      double v = w[0];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double t = id[k] == kRecFluid ? w[k + 1] : w[k + 1] * gv[k];
        v = id[k] == kRecSkip ? v : v + t;
      }
      r[0] = v;
    }
    __syncthreads();
    if (nunits) {
      // thread s < kRecUnitWS takes units s, s + kRecUnitWS, ...; unext is
      // the lowest level among those not solved yet
      if (unext == l + 1) {
        UnitWS* ws = reinterpret_cast<UnitWS*>(rec + (int64_t)kRecWords * rec_cap);
        unext = 0x7fffffff;
        for (int s = tid; s < nunits; s += kRecUnitWS) {
          const int ul = gload(P.unit_lev + s);
          if (ul == l + 1) unit_lds2(P, s, rec, ws[tid]);
          else if (ul > l + 1) unext = min(unext, ul);
        }
      }
      __syncthreads();
    }
  }
  for (int p = tid; p < ng; p += T)
    *(__attribute__((address_space(1))) double*)(F + gload(P.cell + p)) = rec[(int64_t)kRecWords * p];
  __syncthreads();
}

// (LDS, dynamic: the surface part's reduction rows, the coupled units'
// workspaces and the 2D sweep records share it; the records of an item are
// dead before the rows are used, and the sweep's unit workspaces follow the
// records.  rec_cap: the largest item, in ghosts, the records may hold.)
template <int D>
__global__ __launch_bounds__(1024) void k_batch_forward(BStatic S, BCall C, double* __restrict__ part,
                                                        int* __restrict__ counter,
                                                        double* __restrict__ Fout, int rec_cap) {
  extern __shared__ double s_lds[];
  double(*red)[3] = reinterpret_cast<double(*)[3]>(s_lds);
  UnitWS* ws = reinterpret_cast<UnitWS*>(s_lds);
  const int T = blockDim.x;
  for (int it = blockIdx.x; it < C.nitems; it += gridDim.x) {
    const int w = C.order[it];
    const int i = w / C.nf, f = w % C.nf;
    const PlanD& P = S.plans[i];
    double* F = C.fields[w];
    const double* b = C.bcv[w];
    const uint8_t* bt = C.bct ? C.bct[w] : nullptr;
    const int kind = C.kind[f];
    const int32_t* lo_ = S.lev_off[i];
    const int nl = (C.tile_flag && C.tile_flag[0] == 0) ? 0 : S.nlev[i];
    if (D == 2 && nl > 0 && P.ng <= rec_cap && P.cgi) {
      sweep_lds2(P, lo_, nl, F, b, bt, kind, s_lds, rec_cap);
      surface_item<D>(S, C, w, red, part, counter, Fout);
      continue;
    }
    for (int l = 0; l < nl; ++l) {
      const int lo = lo_[l], hi = lo_[l + 1];
      for (int p = lo + (int)threadIdx.x; p < hi; p += T) fill_single<D>(P, p, F, b, bt, kind);
      __syncthreads();
      if (P.nunits) {
        if (threadIdx.x < 64)
          for (int s = threadIdx.x; s < P.nunits; s += 64)
            if (P.unit_lev[s] == l + 1) fill_unit_field<D>(P, s, F, b, bt, kind, ws[threadIdx.x]);
        __syncthreads();
      }
    }
    surface_item<D>(S, C, w, red, part, counter, Fout);
  }
}

// The levels of an instance swept by G workgroups together.  Workgroup s of
// the instance takes every G-th block of T (ghost, field) pairs of a level,
// the fields of a ghost side by side (they share its stencil data), and the
// G workgroups meet at a device-scope counter after each level and after
// each level's coupled units (G = 1: the workgroup's own barrier, which
// orders its values for its own waves).  Every value is computed as by the per-item
// kernel, from the same inputs.  The launch is cooperative (the runtime
// refuses it unless every workgroup can be resident at once), and each wait
// is bounded as well, so every wave ends: a wait that gives up sets the
// batch's fault word, which gcr_batch_status reports, since the values of
// that call can then be wrong.  The instance's workgroups then take its
// (instance, field) surface items in turn, each computed as by the per-item
// kernel.  Two sets of counters serve launches in turn: each launch clears
// the set the next one uses (launches on one batch are ordered).
constexpr int kSpinMax = 1 << 22;

__device__ __forceinline__ void inst_barrier(int* bar, int target, int spin, int* fault, int G) {
  if (G == 1) {   // the instance's only workgroup: its own barrier orders its values
    __syncthreads();
    return;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();   // this workgroup's values, before its arrival
    atomicAdd(bar, 1);
    for (int k = 0;; ++k) {
      if (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
      if (k >= spin) {   // gave up: this call's values cannot be trusted
        atomicOr(fault, 1);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();   // the other workgroups' values, after theirs
  }
  __syncthreads();
}

template <int D>
__global__ __launch_bounds__(1024) void k_batch_split(BStatic S, BCall C, int G,
                                                      int* __restrict__ bar, int parity,
                                                      double* __restrict__ part,
                                                      int* __restrict__ counter,
                                                      double* __restrict__ Fout,
                                                      int* __restrict__ fault, int spin) {
  __shared__ double red[1024][3];
  __shared__ UnitWS ws[64];
  const int T = blockDim.x;
  const int i = (int)blockIdx.x / G, s = (int)blockIdx.x % G;
  if (blockIdx.x == 0)
    for (int k = threadIdx.x; k < C.ninst; k += T) bar[(parity ^ 1) * C.ninst + k] = 0;
  int* const cnt = bar + parity * C.ninst + i;
  const PlanD& P = S.plans[i];
  const int nf = C.nf;
  const int32_t* lo_ = S.lev_off[i];
  const int nl = (C.tile_flag && C.tile_flag[0] == 0) ? 0 : S.nlev[i];
  int arrivals = 0;
  for (int l = 0; l < nl; ++l) {
    const int lo = lo_[l], n = (lo_[l + 1] - lo) * nf;
    for (int e = s * T + (int)threadIdx.x; e < n; e += G * T) {
      const int p = lo + e / nf, f = e % nf, w = i * nf + f;
      fill_single<D>(P, p, C.fields[w], C.bcv[w], C.bct ? C.bct[w] : nullptr, C.kind[f]);
    }
    inst_barrier(cnt, G * ++arrivals, spin, fault, G);
    if (P.nunits) {
      if (threadIdx.x < 64)
        for (int u = s * 64 + (int)threadIdx.x; u < P.nunits; u += G * 64)
          if (P.unit_lev[u] == l + 1)
            for (int f = 0; f < nf; ++f) {
              const int w = i * nf + f;
              fill_unit_field<D>(P, u, C.fields[w], C.bcv[w], C.bct ? C.bct[w] : nullptr,
                                 C.kind[f], ws[threadIdx.x]);
            }
      inst_barrier(cnt, G * ++arrivals, spin, fault, G);
    }
  }
  for (int f = s; f < nf; f += G) surface_item<D>(S, C, i * nf + f, red, part, counter, Fout);
}

// ---------------------------------------------------------------------------
// Tiled fill.  Each instance's ghosts are grouped by the tile of cells that
// holds them (kTileB3^3 cells in 3D, kTileB2^2 in 2D).  A tile's closure is
// its own ghosts and every ghost they depend on, transitively; dependency
// chains stay local, so closures are barely larger than the tiles.  One
// workgroup per tile fills its closure level by level with the values in
// LDS and writes only the tile's own ghosts to the fields: every value is
// computed from the same inputs, in the same way, as by the per-level sweep,
// each ghost is written by one workgroup, and no workgroup waits for
// another.  The closures are found once per batch (first forward call).
// A closure or member store that would overflow, a coupled unit or a graph
// deeper than kTileLev levels sets a flag on the device; then the tiled fill
// writes nothing and the per-item kernel sweeps the levels itself.
constexpr int kTileB3 = 16, kTileB2 = 32;
constexpr int kTileCap = 1024;   // members of one closure
constexpr int kTileLev = 128;    // levels a closure may span

struct TileArgs {
  int ninst;
  int tb;                        // tile extent in cells per axis
  const int32_t* nt;             // [ninst][4] tiles per axis
  const int64_t* slot_base;      // [ninst + 1] first tile slot of each instance
  const int64_t* goff;           // [ninst + 1] first ghost of each instance
  int64_t ng_total;
  int32_t* count;                // [slots] ghosts per tile slot
  int32_t* fillc;                // [slots] bucket fill pointers
  const int64_t* off;            // [slots + 1] exclusive scan of count
  const int32_t* list;           // [slots] occupied slots in order
  const int32_t* nlist;          // [1] their number
  int32_t* bucket;               // [ng_total] ghosts by tile
  int32_t* mem;                  // [mcap] closure members (instance-local position | own << 31)
  int16_t* ref;                  // [mcap][7] local index of each ghost corner, -1: not a ghost
  int32_t* mbase;                // [tiles] first member of each closure
  int16_t* tlev;                 // [tiles][kTileLev + 1] members before each level
  int32_t* tinst;                // [tiles] instance of each closure
  int32_t* mtotal;               // [1] members stored
  int64_t mcap;
  int32_t* flag;                 // [1] nonzero: tiled fill not usable
};

__global__ void k_tile_zero(int32_t* __restrict__ a, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) a[t] = 0;
}

__device__ __forceinline__ int tile_key(const GridD& g, const int32_t* nt, int tb, int c) {
  int i, j, k;
  unlinear(g, c, i, j, k);
  return i / tb + nt[0] * (j / tb + nt[1] * (k / tb));
}

__global__ __launch_bounds__(256) void k_tile_count(BStatic S, TileArgs T, int bucket_pass) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= T.ng_total) return;
  const int i = find_inst(T.goff, T.ninst, g);
  const PlanD& P = S.plans[i];
  const int p = (int)(g - T.goff[i]);
  const int64_t slot = T.slot_base[i] + tile_key(P.g, T.nt + 4 * i, T.tb, P.cell[p]);
  if (!bucket_pass) {
    atomicAdd(&T.count[slot], 1);
  } else {
    const int at = atomicAdd(&T.fillc[slot], 1);
    T.bucket[T.off[slot] + at] = (int32_t)g;
  }
}

// one workgroup per occupied tile: mark the own ghosts in an LDS bitmap over
// the instance's positions, then, from the deepest level down, the ghosts
// the marked ones read (each level's marked positions first compacted into
// an LDS list, one per thread); emit the marked positions in ascending order
__device__ __forceinline__ uint32_t range_mask(int w, int a, int e) {
  const int lo = w == (a >> 5) ? (a & 31) : 0;
  const int hi = w == ((e - 1) >> 5) ? ((e - 1) & 31) : 31;
  const uint32_t upto = hi == 31 ? 0xffffffffu : ((1u << (hi + 1)) - 1u);
  return upto & ~((1u << lo) - 1u);
}

template <int D>
__global__ __launch_bounds__(256) void k_tile_closure(BStatic S, TileArgs T) {
  extern __shared__ uint32_t s_tile[];
  __shared__ int64_t sh[5];
  __shared__ int32_t s_list[kTileCap];
  __shared__ int s_m, s_base, s_bad;
  const int b = blockIdx.x;
  if (b >= T.nlist[0]) return;
  const int64_t slot = T.list[b];
  int i = 0;
  {
    int lo = 0, hi = T.ninst - 1;   // last instance whose first slot <= slot
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (T.slot_base[mid] <= slot) lo = mid;
      else hi = mid - 1;
    }
    i = lo;
  }
  const PlanD& P = S.plans[i];
  const int ng = P.ng, nl = S.nlev[i];
  const int32_t* lof = S.lev_off[i];
  const int W = (ng + 31) >> 5;
  uint32_t* bits = s_tile;
  int32_t* pre = reinterpret_cast<int32_t*>(s_tile + W);
  const int key = (int)(slot - T.slot_base[i]);
  const int tid = (int)threadIdx.x;
  if (tid == 0) {
    s_bad = (nl > kTileLev || P.nunits > 0) ? 1 : 0;
    s_m = 0;
  }
  for (int w = tid; w < W; w += 256) bits[w] = 0u;
  __syncthreads();
  if (s_bad) {
    if (tid == 0) atomicOr(T.flag, 1);
    return;
  }
  for (int64_t q = T.off[slot] + tid; q < T.off[slot + 1]; q += 256) {
    const int p = (int)(T.bucket[q] - T.goff[i]);
    atomicOr(&bits[p >> 5], 1u << (p & 31));
  }
  __syncthreads();
  for (int l = nl - 1; l >= 1; --l) {   // level l + 1 reads only levels <= l
    const int a = lof[l], e = lof[l + 1];
    if (a >= e) continue;
    const int wa = a >> 5, we = (e - 1) >> 5;
    int run = 0;
    for (int w0 = wa; w0 <= we; w0 += 256) {
      const int w = w0 + tid;
      uint32_t mm = w <= we ? (bits[w] & range_mask(w, a, e)) : 0u;
      int64_t tot;
      int pos = run + (int)block_excl_scan<256>(__popc(mm), &tot, sh);
      while (mm) {
        if (pos < kTileCap) s_list[pos] = (w << 5) + __ffs(mm) - 1;
        ++pos;
        mm &= mm - 1;
      }
      run += (int)tot;
    }
    if (run > kTileCap) {
      if (tid == 0) atomicOr(T.flag, 2);
      return;
    }
    __syncthreads();
    for (int t = tid; t < run; t += 256) {
      const int p = s_list[t];
      const uint32_t code = P.code[p];
      const uint32_t skip = code_skip(code);
      const int c = P.cell[p];
#pragma unroll
      for (int k = 1; k < (1 << D); ++k) {
        if (k & skip) continue;
        const int qc = c + corner_offset(P.g, code, k);
        const int8_t t8 = P.tags[qc];
        if (t8 != 2 && t8 != -2) continue;
        const int g2 = ghost_at(P, qc);
        if (g2 >= 0) atomicOr(&bits[g2 >> 5], 1u << (g2 & 31));
      }
    }
    __syncthreads();
  }
  // ranks: exclusive prefix of the word popcounts
  int run = 0;
  for (int w0 = 0; w0 < W; w0 += 256) {
    const int w = w0 + tid;
    int64_t tot;
    const int64_t ex = block_excl_scan<256>(w < W ? __popc(bits[w]) : 0, &tot, sh);
    if (w < W) pre[w] = run + (int)ex;
    run += (int)tot;
  }
  if (tid == 0) {
    s_m = run;
    if (run > kTileCap) {
      atomicOr(T.flag, 2);
      s_base = -1;
    } else {
      s_base = atomicAdd(T.mtotal, run);
      if ((int64_t)s_base + run > T.mcap) {
        atomicOr(T.flag, 4);
        s_base = -1;
      }
    }
  }
  __syncthreads();
  const int m = s_m, base = s_base;
  if (base < 0) return;
  auto rank = [&](int p) {
    const int w = p >> 5;
    return pre[w] + __popc(bits[w] & ((1u << (p & 31)) - 1u));
  };
  // the members in ascending order, then one per thread
  for (int w = tid; w < W; w += 256) {
    uint32_t mm = bits[w];
    int r = pre[w];
    while (mm) {
      s_list[r++] = (w << 5) + __ffs(mm) - 1;
      mm &= mm - 1;
    }
  }
  __syncthreads();
  for (int j = tid; j < m; j += 256) {
    const int p = s_list[j];
    const uint32_t code = P.code[p];
    const uint32_t skip = code_skip(code);
    const int c = P.cell[p];
    const bool own = tile_key(P.g, T.nt + 4 * i, T.tb, c) == key;
    T.mem[base + j] = p | (own ? (int32_t)0x80000000u : 0);
#pragma unroll
    for (int k = 1; k < 8; ++k) {
      int16_t r = -1;
      if (k < (1 << D) && !(k & skip)) {
        const int qc = c + corner_offset(P.g, code, k);
        const int8_t t8 = P.tags[qc];
        if (t8 == 2 || t8 == -2) {
          const int g2 = ghost_at(P, qc);
          if (g2 >= 0) r = (int16_t)rank(g2);
        }
      }
      T.ref[(int64_t)(base + j) * 7 + (k - 1)] = r;
    }
  }
  for (int l = tid; l <= nl; l += 256) {
    const int p = lof[l];
    T.tlev[(int64_t)b * (kTileLev + 1) + l] = (int16_t)(p >= ng ? m : rank(p));
  }
  if (tid == 0) {
    T.mbase[b] = base;
    T.tinst[b] = i;
  }
}

// one workgroup per closure: its members level by level, every field, with
// the values of the closure in LDS ([member][field]); own members also to
// the fields.  A (member, field) item reads, from HBM, only its metadata, its
// boundary datum and the corners that are not ghosts, none of which any
// level changes, so each thread loads its first item of the next level
// before it computes the current one: between levels only the ghost
// corners (LDS) remain on the path.
template <int D>
struct TileItem {
  int j, f, c, bc;
  uint32_t code;
  int16_t ref[8];
  double* F;
  double bv, dl[3], nn[3], val[8];
};

template <int D>
__device__ __forceinline__ void tile_load(const PlanD& P, const BCall& C, const TileArgs& T,
                                          int i, int base, int j, int f, TileItem<D>& it) {
  const int32_t mv = T.mem[base + j];
  const int p = mv & 0x7fffffff;
  const int w = i * C.nf + f;
  it.j = j;
  it.f = f;
  it.c = P.cell[p];
  it.code = P.code[p];
  it.bc = C.kind[f] == 2 ? (int)C.bct[w][p] : C.kind[f];
  it.bv = C.bcv[w][p];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    it.dl[a] = a < D ? P.dl[a][p] : 0.0;
    it.nn[a] = a < D ? P.nn[a][p] : 0.0;
  }
  const uint32_t skip = code_skip(it.code);
  it.F = C.fields[w];
#pragma unroll
  for (int k = 1; k < (1 << D); ++k) {
    const int r = T.ref[(int64_t)(base + j) * 7 + (k - 1)];
    it.ref[k] = (int16_t)r;
    it.val[k] = ((k & skip) || r >= 0) ? 0.0 : it.F[it.c + corner_offset(P.g, it.code, k)];
  }
  it.j = mv < 0 ? -(j + 1) : j;   // own member: written to the field too
}

template <int D>
__global__ __launch_bounds__(256) void k_tile_fill(BStatic S, BCall C, TileArgs T) {
  extern __shared__ double s_val[];
  const int b = blockIdx.x;
  if (b >= T.nlist[0] || T.flag[0] != 0) return;
  const int i = T.tinst[b];
  const PlanD& P = S.plans[i];
  const int nl = S.nlev[i], nf = C.nf;
  const int base = T.mbase[b];
  const int16_t* tl = T.tlev + (int64_t)b * (kTileLev + 1);
  const int nt = (int)blockDim.x;
  TileItem<D> cur, nxt;
  bool have = false;
  if (nl > 0 && (int)threadIdx.x < (tl[1] - tl[0]) * nf) {
    const int t = tl[0] * nf + (int)threadIdx.x;
    tile_load<D>(P, C, T, i, base, t / nf, t % nf, cur);
    have = true;
  }
  for (int l = 0; l < nl; ++l) {
    const int a = tl[l], e = tl[l + 1];
    // first item of the next level, loaded before this level is computed
    bool have_nxt = false;
    if (l + 1 < nl && (int)threadIdx.x < (tl[l + 2] - e) * nf) {
      const int t = e * nf + (int)threadIdx.x;
      tile_load<D>(P, C, T, i, base, t / nf, t % nf, nxt);
      have_nxt = true;
    }
    for (int t = a * nf + (int)threadIdx.x; t < e * nf; t += nt) {
      TileItem<D> it;
      if (t == a * nf + (int)threadIdx.x && have) it = cur;
      else tile_load<D>(P, C, T, i, base, t / nf, t % nf, it);
      const bool own = it.j < 0;
      const int j = own ? -it.j - 1 : it.j;
      const int f = it.f;
      const uint32_t skip = code_skip(it.code);
#pragma unroll
      for (int k = 1; k < (1 << D); ++k)
        if (!(k & skip) && it.ref[k] >= 0) it.val[k] = s_val[it.ref[k] * nf + f];
      double X[3], wt[8];
      stencil_span(P.g, it.code, it.c, X);
      ghost_weights<D>(it.dl, it.nn, X, it.bc, wt);
      double v = wt[0] * it.bv;
#pragma unroll
      for (int k = 1; k < (1 << D); ++k)
        if (!(k & skip)) v += wt[k] * it.val[k];
      s_val[j * nf + f] = v;
      if (own) it.F[it.c] = v;
    }
    cur = nxt;
    have = have_nxt;
    __syncthreads();
  }
}

struct BatchFwdState {
  PlanD* d_plans = nullptr;
  int32_t** d_levp = nullptr;
  int32_t* d_nlev = nullptr;
  int* d_counter = nullptr;
  int* d_bar = nullptr;            // [2][ninst] level counters of the split sweep
  int bar_parity = 0;              // the set the next split launch uses
  int* d_fault = nullptr;          // [1] set when a split sweep's wait gave up
  double* d_part = nullptr;
  size_t part_cap = 0;
  char* d_call = nullptr;
  size_t call_cap = 0;
  int32_t* d_anchor = nullptr;
  size_t anchor_cap = 0;
  // pinned staging of the call table, two slots used in turn; a slot is
  // rewritten only once the copy that last read it has run
  char* h_call[2] = {nullptr, nullptr};
  size_t h_call_cap[2] = {0, 0};
  hipEvent_t ev_call[2] = {nullptr, nullptr};
  bool call_pending[2] = {false, false};
  int call_slot = 0;
  // pinned source of the one upload of the static tables (kept until that
  // copy has run)
  char* h_static = nullptr;
  hipEvent_t ev_static = nullptr;
  // recorded after every forward launch: the state and the batch's memory
  // are released only once the last one has run, on whatever stream
  hipEvent_t ev_done = nullptr;
  int threads = 0, grid_mul = 0;   // tuned
  int rec_ng = 0;                  // ghosts of the largest 2D instance
  int32_t* d_cgi = nullptr;        // corners' ghosts of the 2D plans (PlanD::cgi)
  // tiled fill: 0 not set up yet, 1 set up, -1 not used for this batch
  int tiled = 0;
  int calls = 0;                   // forward calls so far
  TileArgs T{};
  int64_t tmax = 0;                // workgroups of the closure and fill launches
  char* h_tile = nullptr;          // pinned source of the tile tables
  hipEvent_t ev_tile = nullptr;
  std::vector<void*> owned;
  ~BatchFwdState() {
    if (ev_tile) {
      (void)hipEventSynchronize(ev_tile);
      event_give(ev_tile);
    }
    pinned_free(h_tile);
    if (ev_done) {
      (void)hipEventSynchronize(ev_done);
      event_give(ev_done);
    }
    if (ev_static) {
      (void)hipEventSynchronize(ev_static);
      event_give(ev_static);
    }
    pinned_free(h_static);
    for (int k = 0; k < 2; ++k) {
      if (call_pending[k]) (void)hipEventSynchronize(ev_call[k]);
      event_give(ev_call[k]);
      pinned_free(h_call[k]);
    }
    for (void* p : owned) pool_free(p);
    for (void* p : {(void*)d_part, (void*)d_call, (void*)d_anchor})
      if (p) pool_free(p);
  }
};

}  // namespace gcr

using namespace gcr;

namespace {
std::mutex g_shape_mu;
std::map<std::tuple<int, int, int, int, int, int>, std::pair<int, int>> g_shape;
std::mutex g_bfs_mu;
// never destroyed: states still held at exit are left to the process, since
// the device pool they return memory to may already be gone by then
auto& g_bfs = *new std::vector<std::pair<const gcr_batch*, std::unique_ptr<BatchFwdState>>>();

// The corners' ghosts of the batch's 2D plans, once per batch: one thread
// per ghost (flattened over the plans, off[i] the first of plan i), corner
// k + 1 of ghost p at cgi[3 off[i] + k ng + p]: the ghost's position from
// the lookup table, -1 for a fluid corner, -2 for a skipped one.
__global__ __launch_bounds__(256) void k_corner_ghosts(const PlanD* __restrict__ plans,
                                                       const int64_t* __restrict__ off, int n,
                                                       int32_t* __restrict__ cgi) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= off[n]) return;
  const int i = find_inst(off, n, e);
  const PlanD& P = plans[i];
  const int p = (int)(e - off[i]);
  const int c = P.cell[p];
  const uint32_t code = P.code[p];
  const uint32_t skip = code_skip(code);
  int32_t* out = cgi + 3 * off[i];
  for (int k = 1; k < 4; ++k)
    out[(int64_t)(k - 1) * P.ng + p] = (k & skip) ? -2 : ghost_at(P, c + corner_offset(P.g, code, k));
}

BatchFwdState* state_of(gcr_batch* b, hipStream_t st, gcr_status* err) {
  std::lock_guard<std::mutex> lk(g_bfs_mu);
  for (auto& e : g_bfs)
    if (e.first == b) return e.second.get();
  auto S = std::make_unique<BatchFwdState>();
  const int n = (int)b->plans.size();
  std::vector<PlanD> pv(n);
  std::vector<int32_t*> lp(n);
  std::vector<int32_t> nl(n);
  std::vector<int64_t> coff(n + 1, 0);   // ghosts of the 2D plans before plan i
  for (int i = 0; i < n; ++i) {
    pv[i] = plan_view(b->plans[i].get());
    lp[i] = b->plans[i]->d_lev_off;
    nl[i] = b->plans[i]->nlev;
    if (pv[i].g.dim == 2) S->rec_ng = std::max(S->rec_ng, pv[i].ng);
    coff[i + 1] = coff[i] + (pv[i].g.dim == 2 ? pv[i].ng : 0);
  }
  if (coff[n] > 0) {
    S->d_cgi = static_cast<int32_t*>(pool_alloc(sizeof(int32_t) * 3 * coff[n]));
    if (!S->d_cgi) {
      *err = GCR_E_NOMEM;
      return nullptr;
    }
    S->owned.push_back(S->d_cgi);
    for (int i = 0; i < n; ++i)
      if (pv[i].g.dim == 2) pv[i].cgi = S->d_cgi + 3 * coff[i];
  }
  // one upload from pinned staging: plans | level-offset pointers | level
  // counts | force counters and two sets of level counters (zero), each
  // region 256-byte aligned
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t o_lp = al(sizeof(PlanD) * n), o_nl = o_lp + al(sizeof(int32_t*) * n);
  const size_t o_ct = o_nl + al(sizeof(int32_t) * n), o_bar = o_ct + al(sizeof(int) * n);
  const size_t o_fault = o_bar + al(sizeof(int) * 2 * n);
  const size_t o_coff = o_fault + al(sizeof(int));
  const size_t bytes = o_coff + al(sizeof(int64_t) * (n + 1));
  char* d = static_cast<char*>(pool_alloc(bytes));
  if (d) S->owned.push_back(d);
  S->h_static = static_cast<char*>(pinned_alloc(bytes));
  if (!d || !S->h_static) {
    *err = GCR_E_NOMEM;
    return nullptr;
  }
  S->d_plans = reinterpret_cast<PlanD*>(d);
  S->d_levp = reinterpret_cast<int32_t**>(d + o_lp);
  S->d_nlev = reinterpret_cast<int32_t*>(d + o_nl);
  S->d_counter = reinterpret_cast<int*>(d + o_ct);
  S->d_bar = reinterpret_cast<int*>(d + o_bar);
  S->d_fault = reinterpret_cast<int*>(d + o_fault);
  std::memset(S->h_static, 0, bytes);
  std::memcpy(S->h_static, pv.data(), sizeof(PlanD) * n);
  std::memcpy(S->h_static + o_lp, lp.data(), sizeof(int32_t*) * n);
  std::memcpy(S->h_static + o_nl, nl.data(), sizeof(int32_t) * n);
  std::memcpy(S->h_static + o_coff, coff.data(), sizeof(int64_t) * (n + 1));
  S->ev_static = event_take();
  if (!S->ev_static || hipMemcpyAsync(d, S->h_static, bytes, hipMemcpyHostToDevice, st)) {
    *err = GCR_E_HIP;
    return nullptr;
  }
  if (coff[n] > 0)
    k_corner_ghosts<<<(unsigned)((coff[n] + 255) / 256), 256, 0, st>>>(
        S->d_plans, reinterpret_cast<const int64_t*>(d + o_coff), n, S->d_cgi);
  if (hipGetLastError() != hipSuccess || hipEventRecord(S->ev_static, st)) {
    *err = GCR_E_HIP;
    return nullptr;
  }
  g_bfs.emplace_back(b, std::move(S));
  return g_bfs.back().second.get();
}
}  // namespace

void gcr_batch_release_state(const gcr_batch* b) {
  std::lock_guard<std::mutex> lk(g_bfs_mu);
  for (size_t k = 0; k < g_bfs.size(); ++k)
    if (g_bfs[k].first == b) {
      g_bfs.erase(g_bfs.begin() + k);
      return;
    }
}

// With profiling on, every batched forward records HIP events around its two
// kernels; gcr_forward_times averages them.
namespace {
std::mutex g_fwd_ev_mu;
std::vector<std::array<hipEvent_t, 3>> g_fwd_ev;    // recorded, not yet read
std::vector<std::array<hipEvent_t, 3>> g_fwd_free;  // read, for reuse

// three timing events for one forward call (reused once read)
bool take_fwd_events(std::array<hipEvent_t, 3>* ev) {
  {
    std::lock_guard<std::mutex> lk(g_fwd_ev_mu);
    if (!g_fwd_free.empty()) {
      *ev = g_fwd_free.back();
      g_fwd_free.pop_back();
      return true;
    }
  }
  for (auto& e : *ev) e = nullptr;
  for (auto& e : *ev)
    if (hipEventCreate(&e) != hipSuccess) {
      (void)hipGetLastError();
      for (auto& x : *ev)
        if (x) (void)hipEventDestroy(x);
      return false;
    }
  return true;
}
}  // namespace

extern "C" gcr_status gcr_batch_shape(const gcr_batch* b, int32_t* threads, int32_t* grid) {
  if (!b || !threads || !grid) return GCR_E_ARG;
  *threads = 0;
  *grid = 0;
  std::lock_guard<std::mutex> lk(g_bfs_mu);
  for (auto& e : g_bfs)
    if (e.first == b) {
      *threads = e.second->threads;
      *grid = e.second->grid_mul;
    }
  return GCR_OK;
}

extern "C" gcr_status gcr_batch_tiled(const gcr_batch* b, int32_t* state) {
  if (!b || !state) return GCR_E_ARG;
  BatchFwdState* S = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_bfs_mu);
    for (auto& e : g_bfs)
      if (e.first == b) S = e.second.get();
  }
  *state = 0;
  if (!S || S->tiled == 0) return GCR_OK;
  if (S->tiled < 0) {
    *state = -1;
    return GCR_OK;
  }
  int32_t flag = 0;
  GCR_HIP(hipDeviceSynchronize());
  GCR_HIP(hipMemcpy(&flag, S->T.flag, sizeof(int32_t), hipMemcpyDeviceToHost));
  *state = flag == 0 ? 1 : 2;
  return GCR_OK;
}

extern "C" gcr_status gcr_forward_times(float* out) {
  if (!out) return GCR_E_ARG;
  std::lock_guard<std::mutex> lk(g_fwd_ev_mu);
  double a = 0.0, f = 0.0;
  int n = 0;
  for (auto& e : g_fwd_ev) {
    float ma = 0.f, mf = 0.f;
    if (hipEventSynchronize(e[2]) == hipSuccess &&
        hipEventElapsedTime(&ma, e[0], e[1]) == hipSuccess &&
        hipEventElapsedTime(&mf, e[1], e[2]) == hipSuccess) {
      a += ma;
      f += mf;
      ++n;
    }
    g_fwd_free.push_back(e);
  }
  g_fwd_ev.clear();
  (void)hipGetLastError();
  out[0] = n ? (float)(a / n) : -1.f;
  out[1] = n ? (float)(f / n) : -1.f;
  out[2] = (float)n;
  return GCR_OK;
}

namespace {
std::atomic<int> g_tiling{1};
std::atomic<int> g_force_shape{0};   // threads << 8 | (grid & 0xff); 0: tuned
}  // namespace

void gcr::set_batch_shape(int threads, int grid) {
  g_force_shape.store(threads ? (threads << 8) | (grid & 0xff) : 0);
}
void gcr::set_batch_tiling(int mode) { g_tiling.store(mode < 0 ? 0 : (mode > 2 ? 2 : mode)); }
int gcr::batch_tiling() { return g_tiling.load(); }

// Tile tables and closures of a batch, on the forward stream (first forward
// call).  false: the tiled fill is not used for this batch (switched off, a
// coupled unit, a graph deeper than kTileLev levels, or an instance whose
// position bitmap would not fit in LDS).
static bool tile_setup(BatchFwdState* S, gcr_batch* b, int dim, hipStream_t st,
                       gcr_status* err) {
  *err = GCR_OK;
  if (!batch_tiling()) return false;
  const int n = (int)b->plans.size();
  const int tb = dim == 3 ? kTileB3 : kTileB2;
  int64_t ng_total = 0, max_ng = 0;
  std::vector<int32_t> nt(4 * (size_t)n, 1);
  std::vector<int64_t> sb(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const gcr_plan* p = b->plans[i].get();
    if (p->info.nunits > 0 || p->nlev > kTileLev) return false;
    int64_t cnt = 1;
    for (int a = 0; a < 3; ++a) {
      nt[4 * i + a] = (p->inst.g.n[a] + tb - 1) / tb;
      cnt *= nt[4 * i + a];
    }
    sb[i + 1] = sb[i] + cnt;
    ng_total += p->ng;
    max_ng = std::max<int64_t>(max_ng, p->ng);
  }
  if (ng_total == 0) return false;
  const size_t lds_closure = 8 * (size_t)((max_ng + 31) / 32);
  if (lds_closure > 120 * 1024) return false;
  const int64_t slots = sb[n], tmax = std::min<int64_t>(slots, ng_total);
  const int64_t mcap = 4 * ng_total + 4096;
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  const size_t o_sb = al(sizeof(int32_t) * 4 * n);
  const size_t o_cnt = o_sb + al(sizeof(int64_t) * (n + 1));
  const size_t o_fill = o_cnt + al(sizeof(int32_t) * slots);
  const size_t o_off = o_fill + al(sizeof(int32_t) * slots);
  const size_t o_list = o_off + al(sizeof(int64_t) * (slots + 1));
  const size_t o_nlist = o_list + al(sizeof(int32_t) * slots);
  const size_t o_tsum = o_nlist + al(sizeof(int32_t) * 4);
  const size_t o_bucket = o_tsum + al(sizeof(int64_t) * ((slots + 8191) / 8192 + 2));
  const size_t o_mem = o_bucket + al(sizeof(int32_t) * ng_total);
  const size_t o_ref = o_mem + al(sizeof(int32_t) * mcap);
  const size_t o_mbase = o_ref + al(sizeof(int16_t) * 7 * mcap);
  const size_t o_tlev = o_mbase + al(sizeof(int32_t) * tmax);
  const size_t o_tinst = o_tlev + al(sizeof(int16_t) * (kTileLev + 1) * tmax);
  const size_t o_small = o_tinst + al(sizeof(int32_t) * tmax);   // mtotal, flag
  const size_t bytes = o_small + al(sizeof(int32_t) * 4);
  char* d = static_cast<char*>(pool_alloc(bytes));
  if (!d) {
    *err = GCR_E_NOMEM;
    return false;
  }
  S->owned.push_back(d);
  S->h_tile = static_cast<char*>(pinned_alloc(o_cnt));
  S->ev_tile = event_take();
  if (!S->h_tile || !S->ev_tile) {
    *err = GCR_E_NOMEM;
    return false;
  }
  std::memcpy(S->h_tile, nt.data(), sizeof(int32_t) * 4 * n);
  std::memcpy(S->h_tile + o_sb, sb.data(), sizeof(int64_t) * (n + 1));
  if (hipMemcpyAsync(d, S->h_tile, o_cnt, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipEventRecord(S->ev_tile, st) != hipSuccess) {
    *err = GCR_E_HIP;
    return false;
  }
  TileArgs& T = S->T;
  T.ninst = n;
  T.tb = tb;
  T.nt = reinterpret_cast<const int32_t*>(d);
  T.slot_base = reinterpret_cast<const int64_t*>(d + o_sb);
  T.goff = b->data->d_g_off;
  T.ng_total = ng_total;
  T.count = reinterpret_cast<int32_t*>(d + o_cnt);
  T.fillc = reinterpret_cast<int32_t*>(d + o_fill);
  int64_t* off = reinterpret_cast<int64_t*>(d + o_off);
  int32_t* list = reinterpret_cast<int32_t*>(d + o_list);
  int32_t* nlist = reinterpret_cast<int32_t*>(d + o_nlist);
  T.off = off;
  T.list = list;
  T.nlist = nlist;
  T.bucket = reinterpret_cast<int32_t*>(d + o_bucket);
  T.mem = reinterpret_cast<int32_t*>(d + o_mem);
  T.ref = reinterpret_cast<int16_t*>(d + o_ref);
  T.mbase = reinterpret_cast<int32_t*>(d + o_mbase);
  T.tlev = reinterpret_cast<int16_t*>(d + o_tlev);
  T.tinst = reinterpret_cast<int32_t*>(d + o_tinst);
  T.mtotal = reinterpret_cast<int32_t*>(d + o_small);
  T.flag = reinterpret_cast<int32_t*>(d + o_small) + 1;
  T.mcap = mcap;
  S->tmax = tmax;
  auto nb = [](int64_t v) { return (unsigned)((v + 255) / 256); };
  const int64_t nz = (int64_t)(o_off - o_cnt) / 4;   // count and fillc (with padding)
  k_tile_zero<<<nb(nz), 256, 0, st>>>(T.count, nz);
  k_tile_zero<<<1, 256, 0, st>>>(T.mtotal, 2);
  BStatic bs{S->d_plans, S->d_levp, S->d_nlev};
  k_tile_count<<<nb(ng_total), 256, 0, st>>>(bs, T, 0);
  launch_scan(T.count, slots, off, list, nlist, reinterpret_cast<int64_t*>(d + o_tsum), st);
  k_tile_count<<<nb(ng_total), 256, 0, st>>>(bs, T, 1);
  const void* kc = dim == 2 ? reinterpret_cast<const void*>(&k_tile_closure<2>)
                            : reinterpret_cast<const void*>(&k_tile_closure<3>);
  {
    // the attribute only grows (per dimension), so concurrent set-ups on
    // other host threads never leave it below a launch's size
    static std::mutex mu;
    static int64_t attr[2] = {48 * 1024, 48 * 1024};
    std::lock_guard<std::mutex> lk(mu);
    int64_t& a = attr[dim == 2 ? 0 : 1];
    if (lds_closure > a) {
      if (hipFuncSetAttribute(kc, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_closure) != hipSuccess) {
        (void)hipGetLastError();
        return false;
      }
      a = lds_closure;
    }
  }
  // set once for the process (a thread-safe static), before any tiled fill
  static const bool fill_attr = [] {
    const int mx = (int)(sizeof(double) * kTileCap * kMaxFields);
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tile_fill<2>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mx) != hipSuccess ||
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_tile_fill<3>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, mx) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    return true;
  }();
  if (!fill_attr) return false;
  if (dim == 2) k_tile_closure<2><<<(unsigned)tmax, 256, lds_closure, st>>>(bs, T);
  else k_tile_closure<3><<<(unsigned)tmax, 256, lds_closure, st>>>(bs, T);
  if (hipGetLastError() != hipSuccess) {
    *err = GCR_E_HIP;
    return false;
  }
  return true;
}

// Workgroups per instance of the split sweep: the grid stays within one
// workgroup per compute unit.
constexpr int kSplitMaxGrid = 256;

// Polls of a split sweep's wait before it gives up (process-wide; tests
// lower it to make the wait give up while every kernel still ends).
static std::atomic<int> g_split_spin{kSpinMax};

// Workgroups of k_batch_split<D> at `threads` that can be resident at once
// on the device (occupancy per compute unit times compute units), found once
// per shape.
static int split_capacity(int dim, int threads) {
  static std::mutex mu;
  static std::map<std::pair<int, int>, int> cap;
  std::lock_guard<std::mutex> lk(mu);
  const auto key = std::make_pair(dim, threads);
  auto it = cap.find(key);
  if (it != cap.end()) return it->second;
  int dev = 0, ncu = 0, per = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 0;
  const void* k = dim == 2 ? reinterpret_cast<const void*>(&k_batch_split<2>)
                           : reinterpret_cast<const void*>(&k_batch_split<3>);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, threads, 0) != hipSuccess) per = 0;
  (void)hipGetLastError();
  const int c = std::max(0, per * ncu);
  cap[key] = c;
  return c;
}

// Ghosts a workgroup's LDS can hold as sweep records (k_batch_forward), from
// the device's largest dynamic LDS, which the forward kernels are allowed
// once; 0 where that fails.
static int forward_rec_cap() {
  static std::mutex mu;
  static int cap = -1;
  std::lock_guard<std::mutex> lk(mu);
  if (cap >= 0) return cap;
  int dev = 0, a = 0, o = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&a, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) a = 0;
  if (hipDeviceGetAttribute(&o, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) o = 0;
  const int v = std::max(a, o) & ~255;
  bool ok = v > (int)(kRecUnitWS * sizeof(UnitWS));
  for (const void* k : {reinterpret_cast<const void*>(&k_batch_forward<2>),
                        reinterpret_cast<const void*>(&k_batch_forward<3>)})
    ok = ok && hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess;
  (void)hipGetLastError();
  cap = ok ? std::min<int>((v - (int)(kRecUnitWS * sizeof(UnitWS))) / (kRecWords * (int)sizeof(double)),
                           (int)kRecSkip - 1)
           : 0;
  return cap;
}

// gm > 0: per-item kernel over min(items, 256 gm) workgroups; gm < 0: split
// sweep with -gm workgroups per instance, launched cooperatively (refused
// with GCR_E_UNSUPPORTED where its workgroups cannot all be resident).
static gcr_status launch_batch(BatchFwdState* S, const BCall& C, int dim, int threads, int gm,
                               double* F, hipStream_t st) {
  BStatic bs{S->d_plans, S->d_levp, S->d_nlev};
  if (gm < 0) {
    const int G = -gm;
    if ((int64_t)G * C.ninst > kSplitMaxGrid || threads > 1024) return GCR_E_ARG;
    if ((int64_t)G * C.ninst > split_capacity(dim, threads)) return GCR_E_UNSUPPORTED;
  }
  if (C.tile_flag) {
    const size_t lds = sizeof(double) * kTileCap * C.nf;
    if (dim == 2) k_tile_fill<2><<<(unsigned)S->tmax, 256, lds, st>>>(bs, C, S->T);
    else k_tile_fill<3><<<(unsigned)S->tmax, 256, lds, st>>>(bs, C, S->T);
  }
  if (gm < 0) {
    int G = -gm;
    int par = S->bar_parity;
    S->bar_parity ^= 1;
    int spin = g_split_spin.load();
    BCall Cc = C;
    double* part = S->d_part;
    int* counter = S->d_counter;
    int* bar = S->d_bar;
    int* fault = S->d_fault;
    void* args[] = {&bs, &Cc, &G, &bar, &par, &part, &counter, &F, &fault, &spin};
    const void* k = dim == 2 ? reinterpret_cast<const void*>(&k_batch_split<2>)
                             : reinterpret_cast<const void*>(&k_batch_split<3>);
    GCR_HIP(hipLaunchCooperativeKernel(k, dim3((unsigned)(G * C.ninst)), dim3(threads), args, 0,
                                       st));
  } else {
    const int grid = std::min(C.nitems, 256 * gm);
    // LDS: the reduction rows, the unit workspaces, or (2D) the sweep records
    // of the largest item that takes them, whichever is largest
    const int rcap = forward_rec_cap();
    const int rec = dim == 2 && S->rec_ng <= rcap ? S->rec_ng : 0;
    const size_t lds =
        std::max({(size_t)threads * 3 * sizeof(double), 64 * sizeof(UnitWS),
                  rec ? (size_t)rec * kRecWords * sizeof(double) + kRecUnitWS * sizeof(UnitWS) : 0});
    if (rcap == 0 && lds > 64 * 1024) return GCR_E_UNSUPPORTED;
    if (dim == 2)
      k_batch_forward<2><<<grid, threads, lds, st>>>(bs, C, S->d_part, S->d_counter, F, rec);
    else
      k_batch_forward<3><<<grid, threads, lds, st>>>(bs, C, S->d_part, S->d_counter, F, rec);
  }
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

extern "C" gcr_status gcr_set_batch_spin(int32_t polls) {
  if (polls < 0) return GCR_E_ARG;
  g_split_spin.store(polls == 0 ? kSpinMax : polls - 1);
  return GCR_OK;
}

extern "C" gcr_status gcr_batch_status(const gcr_batch* batch) {
  if (!batch) return GCR_E_ARG;
  BatchFwdState* S = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_bfs_mu);
    for (auto& e : g_bfs)
      if (e.first == batch) S = e.second.get();
  }
  if (!S) return GCR_OK;   // never forwarded
  if (S->ev_done) GCR_HIP(hipEventSynchronize(S->ev_done));
  int fault = 0;
  GCR_HIP(hipMemcpy(&fault, S->d_fault, sizeof(int), hipMemcpyDeviceToHost));
  if (!fault) return GCR_OK;
  const int zero = 0;
  GCR_HIP(hipMemcpy(S->d_fault, &zero, sizeof(int), hipMemcpyHostToDevice));
  return GCR_E_TIMEOUT;
}

extern "C" gcr_status gcr_batch_forward(gcr_batch* batch, int32_t nf, double* const* fields,
                                        const int32_t* bc_kind, const uint8_t* const* bc_type,
                                        const double* const* bc_val, const int64_t* nq,
                                        const double* const* xq, const double* const* nrm,
                                        const double* const* wq, int32_t p_field,
                                        int32_t u_first, double mu, double* F,
                                        double* const* sval, double* const* sgrad,
                                        void* stream) {
  if (!batch || nf < 1 || nf > kMaxFields || !fields || !bc_kind || !bc_val) return GCR_E_ARG;
  const int n = (int)batch->plans.size();
  const int dim = batch->plans[0]->dim;
  for (int i = 0; i < n; ++i)
    if (batch->plans[i]->dim != dim) return GCR_E_UNSUPPORTED;
  for (int f = 0; f < nf; ++f)
    if (bc_kind[f] < 0 || bc_kind[f] > 2) return GCR_E_ARG;
  for (int w = 0; w < n * nf; ++w) {
    // (a plan without ghosts reads no boundary data)
    const bool reads_bc = batch->plans[w / nf]->ng > 0;
    if (!fields[w] || (reads_bc && !bc_val[w])) return GCR_E_ARG;
    if (reads_bc && bc_kind[w % nf] == GCR_MIXED && (!bc_type || !bc_type[w])) return GCR_E_ARG;
  }
  if ((sval || sgrad) && !nq) return GCR_E_ARG;
  if (nq) {
    if (!xq || !nrm || !wq || !F) return GCR_E_ARG;
    for (int i = 0; i < n; ++i)
      if (nq[i] < 0 || (nq[i] > 0 && (!xq[i] || !nrm[i] || !wq[i]))) return GCR_E_ARG;
  }
  hipStream_t st = (hipStream_t)stream;
  gcr_status err = GCR_OK;
  BatchFwdState* S = state_of(batch, st, &err);
  if (!S) return err;
  // every call rewrites the batch's call table, partial sums and counters:
  // a call on another stream than the last one waits for that one's launches
  if (S->ev_done) GCR_HIP(hipStreamWaitEvent(st, S->ev_done, 0));
  // a buffer that must grow is freed only once the launches that read it
  // have run (the pool hands it to other threads at once)
  auto retire = [&](void* p) -> bool {
    if (!p) return true;
    if (S->ev_done && hipEventSynchronize(S->ev_done) != hipSuccess) return false;
    pool_free(p);
    return true;
  };
  // tiles from the second forward call of a batch (mode 1: a batch used once
  // does not pay for the closures), or from the first (mode 2)
  ++S->calls;
  if (S->tiled == 0) {
    const int mode = batch_tiling();
    if (mode == 0) {
      S->tiled = -1;
    } else if (mode == 2 || S->calls >= 2) {
      S->tiled = tile_setup(S, batch, dim, st, &err) ? 1 : -1;
      if (err != GCR_OK) return err;
    }
  }
  // items, largest first: fill work ~ ghosts, latency ~ levels, surface ~ points
  const int nitems = n * nf;
  std::vector<double> cost(nitems);
  for (int w = 0; w < nitems; ++w) {
    const gcr_plan* p = batch->plans[w / nf].get();
    cost[w] = (double)p->ng / 256.0 + 4.0 * p->nlev + (nq ? (double)nq[w / nf] / 256.0 : 0.0);
  }
  std::vector<int32_t> order(nitems);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  // (the sort keeps an instance's nf items adjacent: their costs are equal)
  // Workgroups go to the eight XCDs in turn, each with its own L2: the items
  // of one instance, which read the same plan data, are placed 8 apart, so
  // that with a workgroup per item they share an XCD.  Instances are taken
  // in groups of eight by rank, which keeps the order largest first by group.
  if (nf > 1 && n >= 8) {
    std::vector<int32_t> x(nitems);
    const int full = n / 8 * 8;
    for (int r = 0; r < n; ++r)
      for (int f = 0; f < nf; ++f) {
        const int src = r * nf + f;
        x[r < full ? (r / 8) * 8 * nf + 8 * f + r % 8 : src] = order[src];
      }
    order.swap(x);
  }
  // call table: one upload
  const size_t np = (size_t)nitems;
  const size_t bytes = sizeof(void*) * (5 * np + 3 * n) + sizeof(int64_t) * (2 * n + 1) +
                       sizeof(int32_t) * np + 64;
  std::vector<char> host(bytes, 0);
  char* h = host.data();
  size_t o = 0;
  auto put = [&](const void* src, size_t sz) {
    std::memcpy(h + o, src, sz);
    size_t at = o;
    o += (sz + 7) & ~size_t(7);
    return at;
  };
  std::vector<const void*> bt(np, nullptr);
  if (bc_type)
    for (size_t w = 0; w < np; ++w) bt[w] = bc_type[w];
  const size_t o_fields = put(fields, sizeof(void*) * np);
  const size_t o_bcv = put(bc_val, sizeof(void*) * np);
  const size_t o_bct = put(bt.data(), sizeof(void*) * np);
  const size_t o_sval = sval ? put(sval, sizeof(void*) * np) : 0;
  const size_t o_sgrad = sgrad ? put(sgrad, sizeof(void*) * np) : 0;
  size_t o_nq = 0, o_xq = 0, o_nrm = 0, o_wq = 0, o_aoff = 0;
  std::vector<int64_t> aoff(n + 1, 0);
  if (nq) {
    for (int i = 0; i < n; ++i) aoff[i + 1] = aoff[i] + nq[i];
    o_nq = put(nq, sizeof(int64_t) * n);
    o_xq = put(xq, sizeof(void*) * n);
    o_nrm = put(nrm, sizeof(void*) * n);
    o_wq = put(wq, sizeof(void*) * n);
    o_aoff = put(aoff.data(), sizeof(int64_t) * (n + 1));
  }
  const int64_t npts = aoff[n];
  if (npts > 0 && S->anchor_cap < (size_t)npts) {
    if (!retire(S->d_anchor)) return GCR_E_HIP;
    S->d_anchor = static_cast<int32_t*>(pool_alloc(sizeof(int32_t) * npts));
    S->anchor_cap = S->d_anchor ? (size_t)npts : 0;
    if (!S->d_anchor) return GCR_E_NOMEM;
  }
  const size_t o_order = put(order.data(), sizeof(int32_t) * np);
  if (S->call_cap < o) {
    if (!retire(S->d_call)) return GCR_E_HIP;
    S->d_call = static_cast<char*>(pool_alloc(o));
    S->call_cap = S->d_call ? o : 0;
    if (!S->d_call) return GCR_E_NOMEM;
  }
  if (S->part_cap < np * 3) {
    if (!retire(S->d_part)) return GCR_E_HIP;
    S->d_part = static_cast<double*>(pool_alloc(sizeof(double) * np * 3));
    S->part_cap = S->d_part ? np * 3 : 0;
    if (!S->d_part) return GCR_E_NOMEM;
  }
  {
    const int k = S->call_slot;
    S->call_slot ^= 1;
    if (S->call_pending[k]) {
      GCR_HIP(hipEventSynchronize(S->ev_call[k]));
      S->call_pending[k] = false;
    }
    if (S->h_call_cap[k] < o) {
      pinned_free(S->h_call[k]);
      S->h_call[k] = static_cast<char*>(pinned_alloc(o));
      S->h_call_cap[k] = S->h_call[k] ? o : 0;
      if (!S->h_call[k]) return GCR_E_NOMEM;
    }
    if (!S->ev_call[k] && !(S->ev_call[k] = event_take())) return GCR_E_HIP;
    std::memcpy(S->h_call[k], h, o);
    GCR_HIP(hipMemcpyAsync(S->d_call, S->h_call[k], o, hipMemcpyHostToDevice, st));
    GCR_HIP(hipEventRecord(S->ev_call[k], st));
    S->call_pending[k] = true;
  }
  char* d = S->d_call;
  BCall C;
  std::memset(&C, 0, sizeof(C));
  C.nf = nf;
  C.ninst = n;
  C.p_field = nq ? p_field : -1;
  C.u_first = nq ? u_first : -1000;
  C.nitems = nitems;
  C.mu = mu;
  for (int f = 0; f < nf; ++f) C.kind[f] = bc_kind[f];
  C.fields = reinterpret_cast<double* const*>(d + o_fields);
  C.bcv = reinterpret_cast<const double* const*>(d + o_bcv);
  C.bct = bc_type ? reinterpret_cast<const uint8_t* const*>(d + o_bct) : nullptr;
  C.nq = nq ? reinterpret_cast<const int64_t*>(d + o_nq) : nullptr;
  C.xq = nq ? reinterpret_cast<const double* const*>(d + o_xq) : nullptr;
  C.nrm = nq ? reinterpret_cast<const double* const*>(d + o_nrm) : nullptr;
  C.wq = nq ? reinterpret_cast<const double* const*>(d + o_wq) : nullptr;
  C.order = reinterpret_cast<const int32_t*>(d + o_order);
  C.aoff = nq ? reinterpret_cast<const int64_t*>(d + o_aoff) : nullptr;
  C.anchor = S->d_anchor;
  C.tile_flag = S->tiled == 1 ? S->T.flag : nullptr;
  C.sval = sval ? reinterpret_cast<double* const*>(d + o_sval) : nullptr;
  C.sgrad = sgrad ? reinterpret_cast<double* const*>(d + o_sgrad) : nullptr;
  std::array<hipEvent_t, 3> ev{};
  bool timed = (profiling_mask() & 2) != 0 && take_fwd_events(&ev);
  if (timed) (void)hipEventRecord(ev[0], st);
  if (npts > 0) {
    BStatic bs{S->d_plans, S->d_levp, S->d_nlev};
    // a row of workgroups per instance, unless the rows' lengths are so
    // uneven that the grid would be more than twice the points' blocks
    const int64_t ppb = 256 / (dim == 2 ? anchor_lanes<2>() : anchor_lanes<3>());
    int64_t rowb = 0;
    for (int i = 0; i < n; ++i) rowb = std::max<int64_t>(rowb, (nq[i] + ppb - 1) / ppb);
    const int64_t flat = (npts + ppb - 1) / ppb;
    const dim3 grid = n > 1 && n <= 65535 && rowb * n <= 2 * flat
                          ? dim3((unsigned)rowb, (unsigned)n)
                          : dim3((unsigned)flat);
    if (dim == 2)
      k_batch_anchor<2><<<grid, 256, 0, st>>>(bs, C, npts, S->d_anchor);
    else
      k_batch_anchor<3><<<grid, 256, 0, st>>>(bs, C, npts, S->d_anchor);
    GCR_HIP(hipGetLastError());
  }
  double* Fo = F;
  double* Fdummy = nullptr;
  if (!nq) {
    Fdummy = static_cast<double*>(plan_scratch(batch->plans[0].get(), 5, sizeof(double) * 3 * n));
    if (!Fdummy) return GCR_E_NOMEM;
    Fo = Fdummy;
  }
  // the tuned launch shape of batches like this one (dimension, fields,
  // forces or not, and power-of-two buckets of items, ghosts and levels)
  int64_t max_ng = 0;
  int max_lev = 0;
  for (int i = 0; i < n; ++i) {
    max_ng = std::max<int64_t>(max_ng, batch->plans[i]->ng);
    max_lev = std::max(max_lev, batch->plans[i]->nlev);
  }
  auto bucket = [](int64_t v) {
    int b = 0;
    while ((int64_t(1) << b) < v) ++b;
    return b;
  };
  const auto key = std::make_tuple(dim, nf, (nq ? 1 : 0) | (S->tiled == 1 ? 2 : 0),
                                   bucket(nitems), bucket(max_ng), bucket(max_lev));
  if (S->threads == 0) {
    std::lock_guard<std::mutex> lk(g_shape_mu);
    auto it = g_shape.find(key);
    if (it != g_shape.end()) {
      S->threads = it->second.first;
      S->grid_mul = it->second.second;
    }
  }
  if (S->threads == 0) {
    // tuner: workgroup size x grid size, timed on the caller's data (the
    // forward is idempotent)
    hipEvent_t e0, e1;
    GCR_HIP(hipEventCreate(&e0));
    GCR_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    int bt_ = 256, bg = 1;
    const int cand_t[3] = {256, 512, 1024};
    // per-item grids of 256 and 1024 workgroups; split sweeps with 4 to 128
    // workgroups per instance (only where levels are swept)
    const int cand_g[8] = {1, 4, -4, -8, -16, -32, -64, -128};
    for (int tt : cand_t)
      for (int gm : cand_g) {
        if (gm > 1 && std::min(nitems, 256 * gm) == std::min(nitems, 256 * (gm / 4)))
          continue;   // same shape
        if (gm < 0 && (S->tiled == 1 || (int64_t)(-gm) * n > kSplitMaxGrid)) continue;
        gcr_status s = launch_batch(S, C, dim, tt, gm, Fo, st);
        if (s == GCR_E_UNSUPPORTED) continue;   // workgroups not co-resident
        if (s != GCR_OK) return s;
        GCR_HIP(hipEventRecord(e0, st));
        for (int r = 0; r < 3; ++r) launch_batch(S, C, dim, tt, gm, Fo, st);
        GCR_HIP(hipEventRecord(e1, st));
        GCR_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        GCR_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          bt_ = tt;
          bg = gm;
        }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    S->threads = bt_;
    S->grid_mul = bg;
    std::lock_guard<std::mutex> lk(g_shape_mu);
    g_shape[key] = {bt_, bg};
  }
  if (timed) (void)hipEventRecord(ev[1], st);
  int th = S->threads, gm = S->grid_mul;
  if (const int fs = g_force_shape.load()) {
    th = fs >> 8;
    gm = (int)(int8_t)(fs & 0xff);
  }
  const gcr_status rs = launch_batch(S, C, dim, th, gm, Fo, st);
  if (!S->ev_done && !(S->ev_done = event_take())) return GCR_E_HIP;
  GCR_HIP(hipEventRecord(S->ev_done, st));
  if (timed) {
    (void)hipEventRecord(ev[2], st);
    std::lock_guard<std::mutex> lk(g_fwd_ev_mu);
    g_fwd_ev.push_back(ev);
  }
  return rs;
}
