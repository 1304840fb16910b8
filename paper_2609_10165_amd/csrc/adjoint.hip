// adjoint.hip -- adjoints of the fill, the surface evaluation and the forces.
//
// The fill is affine: phi_G = ws b_G + sum_k w_k phi_{P_k}.  Its adjoint runs
// the levels in reverse.  Every value is produced by exactly one thread and
// every sum is taken in a fixed order, so results are bitwise reproducible.
// Both adjoints pull through the transposed stencil ("support"), built on
// the first adjoint call of a plan and kept with it: every cell that some
// ghost's stencil box touches gets a slot holding its readers (ghost,
// corner), sorted by (canonical ghost position, corner).  Then
//   * a ghost pulls w * lambda from the ghosts that read it (higher levels);
//   * a non-ghost cell sums all its readers once, in its own slot;
//   * a coupled unit solves its transposed system;
//   * the surface adjoint groups caller points by anchor ghost (sorted
//     buckets), forms per-corner seeds, and each slot sums the seeds of the
//     anchors whose box holds it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "gcr_apply.hpp"
#include "gcr_impl.hpp"

namespace gcr {

// Transposed stencil.  Entry = (reader << 4) | (corner << 1) | fill, with
// fill = 1 when the fill reads that corner (corner > 0, not skipped);
// corner 0 (the ghost's own cell) and skipped corners belong to the box the
// surface evaluation uses.
struct SupView {
  const int32_t* off;    // [bound + 1] slot -> first entry
  const int32_t* ent;    // [bound]
  const int32_t* cell;   // [bound] slot -> cell
  const int32_t* ghost;  // [bound] slot -> canonical ghost position or -1
  const int32_t* gslot;  // [ng] ghost -> slot of its own cell
  const int32_t* nslot;  // device count of slots
  int64_t bound;         // ng << dim
};

constexpr uint32_t kSupEmpty = 0xffffffffu;

__device__ __forceinline__ uint32_t sup_hash(uint32_t c) {
  uint32_t h = c * 2654435761u;
  return h ^ (h >> 15);
}

struct SupBuild {
  PlanD P;
  uint32_t* key;
  int32_t* val;
  uint32_t hmask;
  int32_t* nslot;
  int32_t* cnt;
  int32_t* off;
  int32_t* fillc;
  int32_t* ent;
  int32_t* cell;
  int32_t* ghost;
  int32_t* gslot;
  int64_t bound;
};

__device__ __forceinline__ int sup_find(const SupBuild& B, uint32_t q) {
  uint32_t h = sup_hash(q) & B.hmask;
  for (;;) {
    const uint32_t k = B.key[h];
    if (k == q) return B.val[h];
    if (k == kSupEmpty) return -1;
    h = (h + 1) & B.hmask;
  }
}

// corner m of ghost p, or -1 off the grid
template <int D>
__device__ __forceinline__ int sup_corner(const PlanD& P, int p, int m, uint32_t& code) {
  code = P.code[p];
  const int c = P.cell[p];
  int i, j, k;
  unlinear(P.g, c, i, j, k);
  if (!corner_in_grid(P.g, code, i, j, k, m)) return -1;
  return c + corner_offset(P.g, code, m);
}

__global__ void k_sup_clear(SupBuild B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t <= (int64_t)B.hmask) B.key[t] = kSupEmpty;
  if (t < B.bound) {
    B.cnt[t] = 0;
    B.fillc[t] = 0;
    B.ghost[t] = -1;
  }
  if (t == 0) B.nslot[0] = 0;
}

template <int D>
__global__ __launch_bounds__(256) void k_sup_insert(SupBuild B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B.bound) return;
  const int p = (int)(t >> D), m = (int)(t & ((1 << D) - 1));
  uint32_t code;
  const int q = sup_corner<D>(B.P, p, m, code);
  if (q < 0) return;
  // the table holds at most `bound` keys in >= 2 * bound entries: a free
  // entry is always reached
  uint32_t h = sup_hash((uint32_t)q) & B.hmask;
  for (;;) {
    const uint32_t prev = atomicCAS(&B.key[h], kSupEmpty, (uint32_t)q);
    if (prev == kSupEmpty) {
      B.val[h] = atomicAdd(B.nslot, 1);
      return;
    }
    if (prev == (uint32_t)q) return;
    h = (h + 1) & B.hmask;
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_sup_count(SupBuild B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B.bound) return;
  const int p = (int)(t >> D), m = (int)(t & ((1 << D) - 1));
  uint32_t code;
  const int q = sup_corner<D>(B.P, p, m, code);
  if (q < 0) return;
  const int s = sup_find(B, (uint32_t)q);
  if (s < 0) return;
  atomicAdd(&B.cnt[s], 1);
  B.cell[s] = q;
  if (m == 0) {
    B.ghost[s] = p;
    B.gslot[p] = s;
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_sup_fill(SupBuild B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B.bound) return;
  const int p = (int)(t >> D), m = (int)(t & ((1 << D) - 1));
  uint32_t code;
  const int q = sup_corner<D>(B.P, p, m, code);
  if (q < 0) return;
  const int s = sup_find(B, (uint32_t)q);
  if (s < 0) return;
  const int fill = (m != 0 && !(m & code_skip(code))) ? 1 : 0;
  B.ent[B.off[s] + atomicAdd(&B.fillc[s], 1)] = (p << 4) | (m << 1) | fill;
}

// each slot's readers in ascending (ghost, corner) order
__global__ __launch_bounds__(256) void k_sup_sort(SupBuild B) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B.bound || s >= B.nslot[0]) return;
  const int b = B.off[s], e = B.off[s + 1];
  for (int i = b + 1; i < e; ++i) {
    const int v = B.ent[i];
    int j = i - 1;
    while (j >= b && B.ent[j] > v) {
      B.ent[j + 1] = B.ent[j];
      --j;
    }
    B.ent[j + 1] = v;
  }
}

__global__ __launch_bounds__(1024) void k_sadj_scan(const int32_t* __restrict__ cnt, int n,
                                                    int32_t* __restrict__ off);

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

// Builds the transposed stencil of plan p on `st` (once; later calls reuse it).
static gcr_status plan_support(gcr_plan* p, hipStream_t st, SupView* out) {
  const int D = p->dim;
  const int64_t bound = p->ng << D;
  uint32_t H = 1;
  while ((int64_t)H < 2 * bound) H <<= 1;
  const size_t n32 = 2 * (size_t)H + 6 * (size_t)bound + 2 + (size_t)p->ng + 1;
  char* base = (char*)p->sup;
  if (!base) {
    base = (char*)pool_alloc(sizeof(int32_t) * n32);
    if (!base) return GCR_E_NOMEM;
    SupBuild B;
    std::memset(&B, 0, sizeof(B));
    B.P = plan_view(p);
    B.key = (uint32_t*)base;
    B.val = (int32_t*)(B.key + H);
    B.cnt = B.val + H;
    B.off = B.cnt + bound + 1;
    B.fillc = B.off + bound + 1;
    B.ent = B.fillc + bound;
    B.cell = B.ent + bound;
    B.ghost = B.cell + bound;
    B.gslot = B.ghost + bound;
    B.nslot = B.gslot + p->ng;
    B.hmask = H - 1;
    B.bound = bound;
    const int64_t nt = std::max<int64_t>((int64_t)H, bound);
    k_sup_clear<<<nblk(nt, 256), 256, 0, st>>>(B);
    if (D == 2) {
      k_sup_insert<2><<<nblk(bound, 256), 256, 0, st>>>(B);
      k_sup_count<2><<<nblk(bound, 256), 256, 0, st>>>(B);
    } else {
      k_sup_insert<3><<<nblk(bound, 256), 256, 0, st>>>(B);
      k_sup_count<3><<<nblk(bound, 256), 256, 0, st>>>(B);
    }
    k_sadj_scan<<<1, 1024, 0, st>>>(B.cnt, (int)bound, B.off);
    if (D == 2) k_sup_fill<2><<<nblk(bound, 256), 256, 0, st>>>(B);
    else k_sup_fill<3><<<nblk(bound, 256), 256, 0, st>>>(B);
    k_sup_sort<<<nblk(bound, 256), 256, 0, st>>>(B);
    GCR_HIP(hipGetLastError());
    p->sup = base;
    p->sup_bound = bound;
    p->sup_hmask = H - 1;
  }
  const uint32_t* key = (const uint32_t*)base;
  const int32_t* val = (const int32_t*)(key + (p->sup_hmask + 1));
  const int32_t* cnt = val + (p->sup_hmask + 1);
  out->off = cnt + bound + 1;
  const int32_t* fillc = out->off + bound + 1;
  out->ent = fillc + bound;
  out->cell = out->ent + bound;
  out->ghost = out->cell + bound;
  out->gslot = out->ghost + bound;
  out->nslot = out->gslot + p->ng;
  out->bound = bound;
  return GCR_OK;
}

struct AdjArgs {
  PlanD P;
  int nf;
  int kind[kMaxFields];
  const uint8_t* bt[kMaxFields];
  double* lam[kMaxFields];     // dense, in/out
  double* lam_bc[kMaxFields];  // [ng]
  double* Lam;                 // [nf][ng] adjoint of each filled ghost value
  const double* w[2];          // the plan's cached weights per kind, [2^D][ng]
  SupView S;
};

template <int D>
__device__ __forceinline__ void weights_of(const PlanD& P, int g, int bc, double w[8]) {
  double dl[3], nn[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dl[a] = a < D ? P.dl[a][g] : 0.0;
    nn[a] = a < D ? P.nn[a][g] : 0.0;
  }
  double X[3];
  stencil_span(P.g, P.code[g], P.cell[g], X);
  ghost_weights<D>(dl, nn, X, bc, w);
}

__device__ __forceinline__ int field_bc(const AdjArgs& A, int f, int g) {
  return A.kind[f] == 2 ? (int)A.bt[f][g] : A.kind[f];
}

// w[corner] * Lam of each fill reader of slot s, summed in entry order into
// acc[f]; readers inside unit `skip_unit` (>= 0) are left out.
template <int D>
__device__ __forceinline__ void pull_readers(const AdjArgs& A, int s, int skip_unit,
                                             double acc[kMaxFields]) {
  const PlanD& P = A.P;
  const int b = A.S.off[s], e = A.S.off[s + 1];
  for (int t = b; t < e; ++t) {
    const int en = A.S.ent[t];
    if (!(en & 1)) continue;
    const int r = en >> 4, m = (en >> 1) & 7;
    if (skip_unit >= 0 && P.blk[r] == skip_unit) continue;
    const double* const W0 = A.w[0];
    const double* const W1 = A.w[1];
#pragma unroll
    for (int f = 0; f < kMaxFields; ++f) {
      if (f >= A.nf) break;
      const double wm = (field_bc(A, f, r) == 0 ? W0 : W1)[(int64_t)m * P.ng + r];
      acc[f] += wm * A.Lam[(int64_t)f * P.ng + r];
    }
  }
}

// Adjoint of coupled unit u: (I - W_int)^T mu = lam + external pulls,
// solved in an LDS workspace (one unit per thread).
template <int D>
__device__ __forceinline__ void adj_unit(const AdjArgs& A, int u, UnitWS& ws) {
  const PlanD& P = A.P;
  const int k = P.unit_cnt[u];
  for (int i = 0; i < k; ++i) {
    ws.mem[i] = P.unit_mem[u * kMaxUnit + i];
    ws.cel[i] = P.cell[ws.mem[i]];
  }
  for (int f = 0; f < A.nf; ++f) {
    // transposed matrix directly: M[t][i] = delta - w(i reads t)
    for (int i = 0; i < k * k; ++i) ws.M[i] = 0.0;
    for (int i = 0; i < k; ++i) {
      ws.M[i * k + i] = 1.0;
      double acc[kMaxFields];
#pragma unroll
      for (int g = 0; g < kMaxFields; ++g) acc[g] = 0.0;
      pull_readers<D>(A, A.S.gslot[ws.mem[i]], u, acc);
      double a = A.lam[f][ws.cel[i]];
#pragma unroll
      for (int g = 0; g < kMaxFields; ++g)
        if (g == f) a += acc[g];
      ws.rhs[i] = a;
    }
    for (int i = 0; i < k; ++i) {
      double w[8];
      weights_of<D>(P, ws.mem[i], field_bc(A, f, ws.mem[i]), w);
      const uint32_t code = P.code[ws.mem[i]];
      for (int c = 1; c < (1 << D); ++c) {
        if (c & code_skip(code)) continue;
        const int q = ws.cel[i] + corner_offset(P.g, code, c);
        for (int t = 0; t < k; ++t)
          if (ws.cel[t] == q) ws.M[t * k + i] -= w[c];
      }
    }
    ws_solve(ws, k);
    for (int i = 0; i < k; ++i) A.Lam[(int64_t)f * P.ng + ws.mem[i]] = ws.rhs[i];
  }
}

template <int D>
__device__ __forceinline__ void adj_units_of_level(const AdjArgs& A, int level, UnitWS* ws,
                                                   int tid, int nthreads) {
  for (int s = tid; s < A.P.nunits; s += nthreads)
    if (A.P.unit_lev[s] == level) adj_unit<D>(A, s, ws[tid]);
}

template <int D>
__device__ __forceinline__ void adj_ghost(const AdjArgs& A, int p) {
  const PlanD& P = A.P;
  const int blk = P.blk[p];
  const int c = P.cell[p];
  const int s = A.S.gslot[p];
  if (blk >= 0) return;   // coupled units: adj_units_of_level
  double acc[kMaxFields];
#pragma unroll
  for (int f = 0; f < kMaxFields; ++f) acc[f] = f < A.nf ? A.lam[f][c] : 0.0;
  pull_readers<D>(A, s, -1, acc);
#pragma unroll
  for (int f = 0; f < kMaxFields; ++f)
    if (f < A.nf) A.Lam[(int64_t)f * P.ng + p] = acc[f];
}

template <int D>
__global__ __launch_bounds__(256) void k_adj_range(AdjArgs A, int lo, int hi) {
  const int p = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (p < hi) adj_ghost<D>(A, p);
}

template <int D>
__global__ __launch_bounds__(256) void k_adj_wg(AdjArgs A, const int32_t* __restrict__ lev_off,
                                                 int nlev) {
  __shared__ UnitWS ws[64];
  for (int l = nlev - 1; l >= 0; --l) {
    for (int p = lev_off[l] + (int)threadIdx.x; p < lev_off[l + 1]; p += blockDim.x)
      adj_ghost<D>(A, p);
    __syncthreads();
    if (A.P.nunits) {
      if (threadIdx.x < 64) adj_units_of_level<D>(A, l + 1, ws, threadIdx.x, 64);
      __syncthreads();
    }
  }
}

template <int D>
__global__ __launch_bounds__(64) void k_adj_units(AdjArgs A, int level) {
  __shared__ UnitWS ws[64];
  adj_units_of_level<D>(A, level, ws, threadIdx.x, 64);
}

// Per slot: a ghost's own cell gives its boundary-data sensitivity and is
// zeroed (the fill overwrites it); a non-ghost cell sums its readers once.
template <int D>
__global__ __launch_bounds__(256) void k_adj_support(AdjArgs A) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= A.S.bound || s >= A.S.nslot[0]) return;
  const PlanD& P = A.P;
  const int q = A.S.cell[s];
  const int p = A.S.ghost[s];
  if (p >= 0) {
    for (int f = 0; f < A.nf; ++f) {
      const double w0 = (field_bc(A, f, p) == 0 ? A.w[0] : A.w[1])[p];
      A.lam_bc[f][p] = w0 * A.Lam[(int64_t)f * P.ng + p];
      A.lam[f][q] = 0.0;
    }
    return;
  }
  bool any = false;
  for (int t = A.S.off[s]; t < A.S.off[s + 1]; ++t) any |= (A.S.ent[t] & 1) != 0;
  if (!any) return;
  double acc[kMaxFields];
#pragma unroll
  for (int f = 0; f < kMaxFields; ++f) acc[f] = 0.0;
  pull_readers<D>(A, (int)s, -1, acc);
#pragma unroll
  for (int f = 0; f < kMaxFields; ++f)
    if (f < A.nf) A.lam[f][q] += acc[f];
}

// --------------------------------------------------------------------------
// surface adjoint
// --------------------------------------------------------------------------

struct SurfAdjArgs {
  PlanD P;
  int nf;
  int64_t nq;
  const double* xq;
  const double* gval;    // [nf][nq] or null
  const double* ggrad;   // [nf][dim][nq] or null
  double* lam[kMaxFields];
  int32_t* anchor;       // [nq]
  int32_t* cnt;          // [ng+1]
  int32_t* off;          // [ng+1]
  int32_t* fillc;        // [ng]
  int32_t* bucket;       // [nq]
  double* seed;          // [nf][8][ng]
  SupView Sp;
};

__global__ void k_zero_i32(int32_t* __restrict__ a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0;
}

__global__ void k_zero_f64(double* __restrict__ a, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

template <int D>
__global__ __launch_bounds__(256) void k_sadj_anchor(SurfAdjArgs S) {
  constexpr int NL = anchor_lanes<D>();
  const int sub = (int)threadIdx.x % NL;
  const int64_t q = (int64_t)blockIdx.x * (256 / NL) + threadIdx.x / NL;
  const bool active = q < S.nq;
  double x[3] = {0.0, 0.0, 0.0};
  if (active)
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = S.xq[a * S.nq + q];
  const int g = find_anchor_group<D, NL>(S.P, x, sub, active);
  if (!active || sub != 0) return;
  S.anchor[q] = g;
  if (g >= 0) atomicAdd(&S.cnt[g], 1);
}

// exclusive scan of the per-ghost counts (one workgroup)
__global__ __launch_bounds__(1024) void k_sadj_scan(const int32_t* __restrict__ cnt, int n,
                                                    int32_t* __restrict__ off) {
  __shared__ int64_t sh[17];
  block_scan_i32(cnt, n, off, sh);
}

__global__ __launch_bounds__(256) void k_sadj_bucket(SurfAdjArgs S) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= S.nq) return;
  const int g = S.anchor[q];
  if (g >= 0) S.bucket[S.off[g] + atomicAdd(&S.fillc[g], 1)] = (int32_t)q;
}

// per anchor: sort its bucket (ascending point index), then the seeds
// seed[f][corner][g] = sum_q coef(corner, x_q) . (gval, ggrad)
template <int D>
__global__ __launch_bounds__(256) void k_sadj_seed(SurfAdjArgs S) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const PlanD& P = S.P;
  if (g >= P.ng) return;
  const int b = S.off[g], e = S.off[g + 1];
  if (b == e) return;
  for (int i = b + 1; i < e; ++i) {
    int v = S.bucket[i], j = i - 1;
    while (j >= b && S.bucket[j] > v) {
      S.bucket[j + 1] = S.bucket[j];
      --j;
    }
    S.bucket[j + 1] = v;
  }
  const uint32_t code = P.code[g];
  int i, j, k;
  unlinear(P.g, P.cell[g], i, j, k);
  const int ijk[3] = {i, j, k};
  double X[3];
  stencil_span(P.g, code, P.cell[g], X);
  // one field at a time keeps the 2^D corner sums in registers
  for (int f = 0; f < S.nf; ++f) {
    double acc[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) acc[m] = 0.0;
    for (int t = b; t < e; ++t) {
      const int64_t q = S.bucket[t];
      double rel[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int a = 0; a < D; ++a) rel[a] = S.xq[a * S.nq + q] - centre(P.g, a, ijk[a]);
      const double gv = S.gval ? S.gval[(int64_t)f * S.nq + q] : 0.0;
      double gg[3] = {0.0, 0.0, 0.0};
      if (S.ggrad)
#pragma unroll
        for (int a = 0; a < D; ++a) gg[a] = S.ggrad[((int64_t)f * D + a) * S.nq + q];
#pragma unroll
      for (int m = 0; m < (1 << D); ++m) {
        double cv, cg[3];
        box_coeffs<D>(rel, X, m, cv, cg);
        double s = cv * gv;
#pragma unroll
        for (int a = 0; a < D; ++a) s += cg[a] * gg[a];
        acc[m] += s;
      }
    }
#pragma unroll
    for (int m = 0; m < (1 << D); ++m) S.seed[((int64_t)f * 8 + m) * P.ng + g] = acc[m];
  }
}

// each slot: the seeds of every anchor whose box holds its cell, in entry
// order (ghosts that anchor no point have no seeds)
__global__ __launch_bounds__(256) void k_sadj_pull(SurfAdjArgs S) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= S.Sp.bound || s >= S.Sp.nslot[0]) return;
  const int ng = S.P.ng;
  double acc[kMaxFields];
#pragma unroll
  for (int f = 0; f < kMaxFields; ++f) acc[f] = 0.0;
  bool any = false;
  for (int t = S.Sp.off[s]; t < S.Sp.off[s + 1]; ++t) {
    const int en = S.Sp.ent[t];
    const int r = en >> 4, m = (en >> 1) & 7;
    if (S.off[r] == S.off[r + 1]) continue;
    any = true;
#pragma unroll
    for (int f = 0; f < kMaxFields; ++f)
      if (f < S.nf) acc[f] += S.seed[((int64_t)f * 8 + m) * ng + r];
  }
  if (!any) return;
  const int q = S.Sp.cell[s];
#pragma unroll
  for (int f = 0; f < kMaxFields; ++f)
    if (f < S.nf) S.lam[f][q] += acc[f];
}

// forces adjoint: J = gF . F gives, per point, d J / d p = -w (gF . n) and
// d J / d (d u_i / d x_j) = mu w (gF_i n_j + gF_j n_i)
__global__ void k_forces_seed(int64_t nq, int dim, const double* __restrict__ nrm,
                              const double* __restrict__ wq, double mu,
                              const double* __restrict__ gF, double* __restrict__ gval,
                              double* __restrict__ ggrad) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  double n[3] = {0.0, 0.0, 0.0}, g[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < dim; ++a) {
    n[a] = nrm[a * nq + q];
    g[a] = gF[a];
  }
  const double w = wq[q];
  double gn = 0.0;
  for (int a = 0; a < dim; ++a) gn += g[a] * n[a];
  gval[q] = -w * gn;
  for (int i = 0; i < dim; ++i) gval[(int64_t)(1 + i) * nq + q] = 0.0;
  for (int j = 0; j < dim; ++j) ggrad[(int64_t)j * nq + q] = 0.0;
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j)
      ggrad[((int64_t)(1 + i) * dim + j) * nq + q] = mu * w * (g[i] * n[j] + g[j] * n[i]);
}

static gcr_status surface_adjoint_impl(gcr_plan* p, int64_t nq, const double* xq, int nf,
                                       const double* gval, const double* ggrad,
                                       double* const* lam, hipStream_t st) {
  const int64_t ng = p->ng;
  if (nq == 0 || ng == 0) return GCR_OK;
  SurfAdjArgs S;
  std::memset(&S, 0, sizeof(S));
  S.P = plan_view(p);
  S.nf = nf;
  S.nq = nq;
  S.xq = xq;
  S.gval = gval;
  S.ggrad = ggrad;
  for (int f = 0; f < nf; ++f) S.lam[f] = lam[f];
  {
    const gcr_status ss = plan_support(p, st, &S.Sp);
    if (ss != GCR_OK) return ss;
  }
  char* ib = (char*)plan_scratch(p, 1, sizeof(int32_t) * (2 * nq + 3 * (ng + 1)));
  double* sb = (double*)plan_scratch(p, 2, sizeof(double) * (size_t)nf * 8 * ng);
  if (!ib || !sb) return GCR_E_NOMEM;
  S.anchor = (int32_t*)ib;
  S.bucket = S.anchor + nq;
  S.cnt = S.bucket + nq;
  S.off = S.cnt + (ng + 1);
  S.fillc = S.off + (ng + 1);
  S.seed = sb;
  k_zero_i32<<<nblk(ng + 1, 256), 256, 0, st>>>(S.cnt, ng + 1);
  k_zero_i32<<<nblk(ng + 1, 256), 256, 0, st>>>(S.fillc, ng + 1);
  const int D = p->dim;
  const unsigned nba = (unsigned)force_blocks(D, nq);
  if (D == 2) k_sadj_anchor<2><<<nba, 256, 0, st>>>(S);
  else k_sadj_anchor<3><<<nba, 256, 0, st>>>(S);
  k_sadj_scan<<<1, 1024, 0, st>>>(S.cnt, (int)ng, S.off);
  k_sadj_bucket<<<nblk(nq, 256), 256, 0, st>>>(S);
  if (D == 2) k_sadj_seed<2><<<nblk(ng, 256), 256, 0, st>>>(S);
  else k_sadj_seed<3><<<nblk(ng, 256), 256, 0, st>>>(S);
  k_sadj_pull<<<nblk(S.Sp.bound, 256), 256, 0, st>>>(S);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

static bool nonnull(int n, const void* const* a) {
  if (!a || n < 1 || n > kMaxFields) return false;
  for (int i = 0; i < n; ++i)
    if (!a[i]) return false;
  return true;
}

}  // namespace gcr

using namespace gcr;

extern "C" {

gcr_status gcr_surface_adjoint(const gcr_plan* plan, int64_t nq, const double* xq, int32_t nf,
                               const double* gval, const double* ggrad, double* const* lam,
                               void* stream) {
  if (!plan_ok(plan) || nq < 0 || (nq > 0 && !xq) || !nonnull(nf, (const void* const*)lam))
    return GCR_E_ARG;
  if (nq >= (int64_t(1) << 31)) return GCR_E_UNSUPPORTED;
  return surface_adjoint_impl(const_cast<gcr_plan*>(plan), nq, xq, nf, gval, ggrad, lam,
                              (hipStream_t)stream);
}

gcr_status gcr_forces_adjoint(const gcr_plan* plan, int64_t nq, const double* xq,
                              const double* nrm, const double* wq, double mu, const double* gF,
                              double* lam_p, double* const* lam_u, void* stream) {
  if (!plan_ok(plan) || nq < 0 || !gF || !lam_p || !lam_u) return GCR_E_ARG;
  if (nq > 0 && (!xq || !nrm || !wq)) return GCR_E_ARG;
  const int d = plan->dim;
  for (int a = 0; a < d; ++a)
    if (!lam_u[a]) return GCR_E_ARG;
  if (nq == 0) return GCR_OK;
  if (nq >= (int64_t(1) << 31)) return GCR_E_UNSUPPORTED;
  gcr_plan* p = const_cast<gcr_plan*>(plan);
  hipStream_t st = (hipStream_t)stream;
  double* buf = (double*)plan_scratch(p, 3, sizeof(double) * (size_t)nq * (1 + d) * (1 + d));
  if (!buf) return GCR_E_NOMEM;
  double* gval = buf;
  double* ggrad = buf + (size_t)(1 + d) * nq;
  k_forces_seed<<<nblk(nq, 256), 256, 0, st>>>(nq, d, nrm, wq, mu, gF, gval, ggrad);
  GCR_HIP(hipGetLastError());
  double* lam[4] = {lam_p, lam_u[0], lam_u[1], d == 3 ? lam_u[2] : nullptr};
  return surface_adjoint_impl(p, nq, xq, 1 + d, gval, ggrad, lam, st);
}

gcr_status gcr_fill_adjoint(const gcr_plan* plan, int32_t nf, double* const* lam,
                            const int32_t* bc_kind, const uint8_t* const* bc_type,
                            double* const* lam_bc, void* stream) {
  if (!plan_ok(plan) || !nonnull(nf, (const void* const*)lam) || !bc_kind ||
      !nonnull(nf, (const void* const*)lam_bc))
    return GCR_E_ARG;
  gcr_plan* p = const_cast<gcr_plan*>(plan);
  AdjArgs A;
  std::memset(&A, 0, sizeof(A));
  A.P = plan_view(p);
  A.nf = nf;
  for (int f = 0; f < nf; ++f) {
    if (bc_kind[f] < 0 || bc_kind[f] > 2) return GCR_E_ARG;
    if (bc_kind[f] == GCR_MIXED && (!bc_type || !bc_type[f])) return GCR_E_ARG;
    A.kind[f] = bc_kind[f];
    A.bt[f] = bc_kind[f] == GCR_MIXED ? bc_type[f] : nullptr;
    A.lam[f] = lam[f];
    A.lam_bc[f] = lam_bc[f];
  }
  const int64_t ng = p->ng;
  if (ng == 0) return GCR_OK;
  A.Lam = (double*)plan_scratch(p, 4, sizeof(double) * (size_t)nf * ng);
  if (!A.Lam) return GCR_E_NOMEM;
  hipStream_t st = (hipStream_t)stream;
  {
    const gcr_status ws = plan_weights(p, nf, A.kind, A.w, st);
    if (ws != GCR_OK) return ws;
  }
  {
    const gcr_status ss = plan_support(p, st, &A.S);
    if (ss != GCR_OK) return ss;
  }
  // the same schedule family as the fill: one workgroup, or one launch per level
  const bool wg = (p->schedule == kSchedWorkgroup) ||
                  (p->schedule == kSchedAuto && p->tuned == kSchedWorkgroup);
  if (wg) {
    if (p->dim == 2) k_adj_wg<2><<<1, 256, 0, st>>>(A, p->d_lev_off, p->nlev);
    else k_adj_wg<3><<<1, 256, 0, st>>>(A, p->d_lev_off, p->nlev);
  } else {
    for (int l = p->nlev - 1; l >= 0; --l) {
      const int lo = p->lev_off[l], hi = p->lev_off[l + 1];
      if (p->dim == 2) k_adj_range<2><<<nblk(hi - lo, 256), 256, 0, st>>>(A, lo, hi);
      else k_adj_range<3><<<nblk(hi - lo, 256), 256, 0, st>>>(A, lo, hi);
      for (int32_t ul : p->unit_lev_host)
        if (ul == l + 1) {
          if (p->dim == 2) k_adj_units<2><<<1, 64, 0, st>>>(A, l + 1);
          else k_adj_units<3><<<1, 64, 0, st>>>(A, l + 1);
          break;
        }
    }
  }
  if (p->dim == 2) k_adj_support<2><<<nblk(A.S.bound, 256), 256, 0, st>>>(A);
  else k_adj_support<3><<<nblk(A.S.bound, 256), 256, 0, st>>>(A);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

}  // extern "C"
