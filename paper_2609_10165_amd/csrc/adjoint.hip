// adjoint.hip -- adjoints of the fill, the surface evaluation and the forces.
//
// The fill is affine: phi_G = ws b_G + sum_k w_k phi_{P_k}.  Its adjoint runs
// the levels in reverse.  Every value is produced by exactly one thread and
// every sum is taken in a fixed order, so results are bitwise reproducible:
//   * a ghost pulls from the ghosts that read it (found by a fixed-order
//     search of the cells within the largest stencil multiplier, checking
//     each candidate's own stencil code) -- they sit in higher levels;
//   * a non-ghost cell read by several ghosts is updated by its first reader
//     in that search order (its "owner"), which sums all readers;
//   * a coupled unit solves its transposed system.
// The surface adjoint groups caller points by anchor ghost (sorted buckets)
// and pulls each box corner the same way.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "gcr_apply.hpp"
#include "gcr_impl.hpp"

namespace gcr {

struct AdjArgs {
  PlanD P;
  int nf;
  int kind[kMaxFields];
  const uint8_t* bt[kMaxFields];
  double* lam[kMaxFields];     // dense, in/out
  double* lam_bc[kMaxFields];  // [ng]
  double* Lam;                 // [nf][ng] adjoint of each filled ghost value
};

template <int D>
__device__ __forceinline__ void weights_of(const PlanD& P, int g, int bc, double w[8]) {
  double dl[3], nn[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dl[a] = a < D ? P.dl[a][g] : 0.0;
    nn[a] = a < D ? P.nn[a][g] : 0.0;
  }
  ghost_weights<D>(dl, nn, P.code[g], P.g.h, bc, w);
}

__device__ __forceinline__ int field_bc(const AdjArgs& A, int f, int g) {
  return A.kind[f] == 2 ? (int)A.bt[f][g] : A.kind[f];
}

// Ghosts whose (non-skipped) stencil contains cell c, in a fixed order;
// fn(g, corner) may return false to stop.
template <int D, class Fn>
__device__ __forceinline__ void for_each_reader(const PlanD& P, int c, Fn fn) {
  int i, j, k;
  unlinear(P.g, c, i, j, k);
  const int rx = P.rmax[0], ry = P.rmax[1], rz = D == 3 ? P.rmax[2] : 0;
  for (int oz = -rz; oz <= rz; ++oz) {
    const int qk = k - oz;
    if (D == 3 && (qk < 0 || qk >= P.g.n[2])) continue;
    for (int oy = -ry; oy <= ry; ++oy) {
      const int qj = j - oy;
      if (qj < 0 || qj >= P.g.n[1]) continue;
      for (int ox = -rx; ox <= rx; ++ox) {
        if (ox == 0 && oy == 0 && oz == 0) continue;
        const int qi = i - ox;
        if (qi < 0 || qi >= P.g.n[0]) continue;
        const int q = linear(P.g, qi, qj, qk);
        const int8_t t = P.tags[q];
        if (t != 2 && t != -2) continue;
        const int g = ghost_at(P, q);
        if (g < 0) continue;
        const uint32_t code = P.code[g];
        const int o[3] = {ox, oy, oz};
        int mask = 0;
        bool ok = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          if (o[a] == 0) continue;
          if (o[a] == code_e(code, a) * code_r(code, a)) mask |= 1 << a;
          else ok = false;
        }
        if (!ok || (mask & code_skip(code))) continue;
        if (!fn(g, mask)) return;
      }
    }
  }
}

// Adjoint of coupled unit u at level `level`: (I - W_int)^T mu = lam +
// external pulls, solved in an LDS workspace (one unit per thread).
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
      double acc = A.lam[f][ws.cel[i]];
      for_each_reader<D>(P, ws.cel[i], [&](int g, int mask) {
        if (P.blk[g] == u) return true;   // inside the unit: handled by the solve
        double w[8];
        weights_of<D>(P, g, field_bc(A, f, g), w);
        acc += w[mask] * A.Lam[(int64_t)f * P.ng + g];
        return true;
      });
      ws.rhs[i] = acc;
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
  if (P.blk[p] >= 0) return;   // coupled units: adj_units_of_level
  const int c = P.cell[p];
  // fully unrolled over the field slots so the accumulators stay in registers
  double acc[kMaxFields];
#pragma unroll
  for (int f = 0; f < kMaxFields; ++f) acc[f] = f < A.nf ? A.lam[f][c] : 0.0;
  for_each_reader<D>(P, c, [&](int g, int mask) {
    double wD[8], wN[8];
    bool hD = false, hN = false;
#pragma unroll
    for (int f = 0; f < kMaxFields; ++f) {
      if (f >= A.nf) break;
      const int bc = field_bc(A, f, g);
      if (bc == 0 && !hD) {
        weights_of<D>(P, g, 0, wD);
        hD = true;
      } else if (bc != 0 && !hN) {
        weights_of<D>(P, g, 1, wN);
        hN = true;
      }
      double wm = 0.0;
#pragma unroll
      for (int k = 1; k < (1 << D); ++k)
        if (k == mask) wm = bc == 0 ? wD[k] : wN[k];
      acc[f] += wm * A.Lam[(int64_t)f * P.ng + g];
    }
    return true;
  });
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
__global__ __launch_bounds__(1024) void k_adj_wg(AdjArgs A, const int32_t* __restrict__ lev_off,
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

// Boundary-data sensitivities, non-ghost cells (owner rule), ghost slots zeroed.
template <int D>
__global__ __launch_bounds__(256) void k_adj_support(AdjArgs A) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const PlanD& P = A.P;
  if (p >= P.ng) return;
  const int c = P.cell[p];
  const uint32_t code = P.code[p];
  for (int f = 0; f < A.nf; ++f) {
    double w[8];
    weights_of<D>(P, p, field_bc(A, f, p), w);
    A.lam_bc[f][p] = w[0] * A.Lam[(int64_t)f * P.ng + p];
  }
  for (int m = 1; m < (1 << D); ++m) {
    if (m & code_skip(code)) continue;
    const int q = c + corner_offset(P.g, code, m);
    const int8_t t = P.tags[q];
    if (t == 2 || t == -2) continue;   // ghosts pulled their readers already
    bool owner = true, first = true;
    double acc[kMaxFields];
    for (int f = 0; f < A.nf; ++f) acc[f] = 0.0;
    for_each_reader<D>(P, q, [&](int g, int mask) {
      if (first) {
        first = false;
        if (g != p) {
          owner = false;
          return false;
        }
      }
      for (int f = 0; f < A.nf; ++f) {
        double w[8];
        weights_of<D>(P, g, field_bc(A, f, g), w);
        acc[f] += w[mask] * A.Lam[(int64_t)f * P.ng + g];
      }
      return true;
    });
    if (owner)
      for (int f = 0; f < A.nf; ++f) A.lam[f][q] += acc[f];
  }
  for (int f = 0; f < A.nf; ++f) A.lam[f][c] = 0.0;
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
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= S.nq) return;
  double x[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = S.xq[a * S.nq + q];
  const int g = find_anchor<D>(S.P, x);
  S.anchor[q] = g;
  if (g >= 0) atomicAdd(&S.cnt[g], 1);
}

// exclusive scan of the per-ghost counts (one workgroup)
__global__ __launch_bounds__(1024) void k_sadj_scan(const int32_t* __restrict__ cnt, int n,
                                                    int32_t* __restrict__ off) {
  __shared__ int64_t sh[17];
  const int per = (n + 1023) / 1024;
  const int b = threadIdx.x * per, e = min(n, b + per);
  int64_t s = 0;
  for (int i = b; i < e; ++i) s += cnt[i];
  int64_t tot;
  int64_t run = block_excl_scan<1024>(s, &tot, sh);
  for (int i = b; i < e; ++i) {
    off[i] = (int32_t)run;
    run += cnt[i];
  }
  if (threadIdx.x == 0) off[n] = (int32_t)tot;
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
        box_coeffs<D>(rel, code, P.g.h, m, cv, cg);
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

// each box corner of each anchor: the first anchor (fixed search order) whose
// box holds the cell adds every anchor's seed for it
template <int D>
__global__ __launch_bounds__(256) void k_sadj_pull(SurfAdjArgs S) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const PlanD& P = S.P;
  if (g >= P.ng) return;
  if (S.off[g] == S.off[g + 1]) return;
  const uint32_t code = P.code[g];
  int gi, gj, gk;
  unlinear(P.g, P.cell[g], gi, gj, gk);
  for (int m = 0; m < (1 << D); ++m) {
    if (!corner_in_grid(P.g, code, gi, gj, gk, m)) continue;
    const int c = P.cell[g] + corner_offset(P.g, code, m);
    int i, j, k;
    unlinear(P.g, c, i, j, k);
    const int rx = P.rmax[0], ry = P.rmax[1], rz = D == 3 ? P.rmax[2] : 0;
    bool owner = true, first = true, stop = false;
    double acc[kMaxFields];
    for (int f = 0; f < S.nf; ++f) acc[f] = 0.0;
    for (int oz = -rz; oz <= rz && !stop; ++oz) {
      const int qk = k - oz;
      if (D == 3 && (qk < 0 || qk >= P.g.n[2])) continue;
      for (int oy = -ry; oy <= ry && !stop; ++oy) {
        const int qj = j - oy;
        if (qj < 0 || qj >= P.g.n[1]) continue;
        for (int ox = -rx; ox <= rx && !stop; ++ox) {
          const int qi = i - ox;
          if (qi < 0 || qi >= P.g.n[0]) continue;
          const int q = linear(P.g, qi, qj, qk);
          const int8_t t = P.tags[q];
          if (t != 2 && t != -2) continue;
          const int a2 = ghost_at(P, q);
          if (a2 < 0 || S.off[a2] == S.off[a2 + 1]) continue;
          const uint32_t c2 = P.code[a2];
          const int o[3] = {ox, oy, oz};
          int mask = 0;
          bool ok = true;
#pragma unroll
          for (int a = 0; a < D; ++a) {
            if (o[a] == 0) continue;
            if (o[a] == code_e(c2, a) * code_r(c2, a)) mask |= 1 << a;
            else ok = false;
          }
          if (!ok) continue;
          if (first) {
            first = false;
            if (a2 != g) {
              owner = false;
              stop = true;
              break;
            }
          }
          for (int f = 0; f < S.nf; ++f) acc[f] += S.seed[((int64_t)f * 8 + mask) * P.ng + a2];
        }
      }
    }
    if (owner && !first)
      for (int f = 0; f < S.nf; ++f) S.lam[f][c] += acc[f];
  }
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

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)std::max<int64_t>(1, (n + bs - 1) / bs); }

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
  if (D == 2) k_sadj_anchor<2><<<nblk(nq, 256), 256, 0, st>>>(S);
  else k_sadj_anchor<3><<<nblk(nq, 256), 256, 0, st>>>(S);
  k_sadj_scan<<<1, 1024, 0, st>>>(S.cnt, (int)ng, S.off);
  k_sadj_bucket<<<nblk(nq, 256), 256, 0, st>>>(S);
  if (D == 2) {
    k_sadj_seed<2><<<nblk(ng, 256), 256, 0, st>>>(S);
    k_sadj_pull<2><<<nblk(ng, 256), 256, 0, st>>>(S);
  } else {
    k_sadj_seed<3><<<nblk(ng, 256), 256, 0, st>>>(S);
    k_sadj_pull<3><<<nblk(ng, 256), 256, 0, st>>>(S);
  }
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
  if (!plan || nq < 0 || (nq > 0 && !xq) || !nonnull(nf, (const void* const*)lam))
    return GCR_E_ARG;
  if (nq >= (int64_t(1) << 31)) return GCR_E_UNSUPPORTED;
  return surface_adjoint_impl(const_cast<gcr_plan*>(plan), nq, xq, nf, gval, ggrad, lam,
                              (hipStream_t)stream);
}

gcr_status gcr_forces_adjoint(const gcr_plan* plan, int64_t nq, const double* xq,
                              const double* nrm, const double* wq, double mu, const double* gF,
                              double* lam_p, double* const* lam_u, void* stream) {
  if (!plan || nq < 0 || !gF || !lam_p || !lam_u) return GCR_E_ARG;
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
  if (!plan || !nonnull(nf, (const void* const*)lam) || !bc_kind ||
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
  // the same schedule family as the fill: one workgroup, or one launch per level
  const bool wg = (p->schedule == kSchedWorkgroup) ||
                  (p->schedule == kSchedAuto && p->tuned == kSchedWorkgroup);
  if (wg) {
    if (p->dim == 2) k_adj_wg<2><<<1, 1024, 0, st>>>(A, p->d_lev_off, p->nlev);
    else k_adj_wg<3><<<1, 1024, 0, st>>>(A, p->d_lev_off, p->nlev);
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
  if (p->dim == 2) k_adj_support<2><<<nblk(ng, 256), 256, 0, st>>>(A);
  else k_adj_support<3><<<nblk(ng, 256), 256, 0, st>>>(A);
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

}  // extern "C"
