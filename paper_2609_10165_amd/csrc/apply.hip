// apply.hip -- kernels that use a plan: the level-by-level ghost fill
// (Sec. 3.2 with the relations of Sec. 4.1 / 5.1), boundary values and
// gradients at foot points and caller points (Sec. 6), and forces.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "gcr_fill.hpp"

namespace gcr {

// --------------------------------------------------------------------------
// fill
// --------------------------------------------------------------------------

// Weights of every ghost for one boundary-condition kind (Sec. 4.1 / 5.1
// relations solved for the ghost value), w[k][p], k = 0 the datum.  They
// depend on the plan only, so a plan computes them once per kind.
template <int D>
__global__ __launch_bounds__(256) void k_weights(PlanD P, int bc, double* __restrict__ w,
                                                 uint8_t* __restrict__ kinds) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < 2) kinds[p] = (uint8_t)p;   // the {0, 1} table of uniform kinds
  if (p >= P.ng) return;
  double dl[3], nn[3], wk[8];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dl[a] = a < D ? P.dl[a][p] : 0.0;
    nn[a] = a < D ? P.nn[a][p] : 0.0;
  }
  double X[3];
  stencil_span(P.g, P.code[p], P.cell[p], X);
  ghost_weights<D>(dl, nn, X, bc, wk);
#pragma unroll
  for (int k = 0; k < (1 << D); ++k) w[(int64_t)k * P.ng + p] = wk[k];
}

void launch_weights(const PlanD& P, int bc, double* w, uint8_t* kinds, hipStream_t st) {
  const unsigned nb = (unsigned)std::max(1, (P.ng + 255) / 256);
  if (P.g.dim == 2) k_weights<2><<<nb, 256, 0, st>>>(P, bc, w, kinds);
  else k_weights<3><<<nb, 256, 0, st>>>(P, bc, w, kinds);
}

template <int D>
__global__ __launch_bounds__(256) void k_fill_range(FillArgs A, int lo, int hi) {
  const int p = lo + blockIdx.x * blockDim.x + threadIdx.x;
  if (p < hi) fill_ghost<D>(A, p);
}

// one workgroup sweeps every level; a barrier separates levels, and the
// coupled units of a level are solved (first 64 threads) before the next
template <int D>
__global__ __launch_bounds__(1024) void k_fill_wg(FillArgs A, const int32_t* __restrict__ lev_off,
                                                  int nlev) {
  __shared__ UnitWS ws[64];
  for (int l = 0; l < nlev; ++l) {
    const int lo = lev_off[l], hi = lev_off[l + 1];
    for (int p = lo + (int)threadIdx.x; p < hi; p += blockDim.x) fill_ghost<D>(A, p);
    __syncthreads();
    if (A.P.nunits) {
      if (threadIdx.x < 64) fill_units_of_level<D>(A, l + 1, ws, threadIdx.x, 64);
      __syncthreads();
    }
  }
}

// coupled units of one level
template <int D>
__global__ __launch_bounds__(64) void k_fill_units(FillArgs A, int level) {
  __shared__ UnitWS ws[64];
  fill_units_of_level<D>(A, level, ws, threadIdx.x, 64);
}

void launch_fill_range(const FillArgs& A, int lo, int hi, hipStream_t st) {
  if (hi <= lo) return;
  const unsigned nb = (unsigned)((hi - lo + 255) / 256);
  if (A.P.g.dim == 2) k_fill_range<2><<<nb, 256, 0, st>>>(A, lo, hi);
  else k_fill_range<3><<<nb, 256, 0, st>>>(A, lo, hi);
}

void launch_fill_units(const FillArgs& A, int level, hipStream_t st) {
  if (A.P.g.dim == 2) k_fill_units<2><<<1, 64, 0, st>>>(A, level);
  else k_fill_units<3><<<1, 64, 0, st>>>(A, level);
}

void launch_fill_wg(const FillArgs& A, const int32_t* d_lev_off, int nlev, int threads,
                    hipStream_t st) {
  if (nlev <= 0) return;
  if (A.P.g.dim == 2) k_fill_wg<2><<<1, threads, 0, st>>>(A, d_lev_off, nlev);
  else k_fill_wg<3><<<1, threads, 0, st>>>(A, d_lev_off, nlev);
}

// --------------------------------------------------------------------------
// boundary values and gradients
// --------------------------------------------------------------------------

template <int D>
__global__ __launch_bounds__(256) void k_surface_ghost(SurfArgs S) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const PlanD& P = S.P;
  if (p >= P.ng) return;
  const uint32_t code = P.code[p];
  double rel[3], X[3];
  stencil_span(P.g, code, P.cell[p], X);
#pragma unroll
  for (int a = 0; a < 3; ++a) rel[a] = a < D ? P.dl[a][p] : 0.0;
  for (int f = 0; f < S.nf; ++f) {
    double v[8], val, grad[3];
    corner_values<D>(P, p, S.f[f], v);
    box_eval<D>(rel, X, v, val, grad);
    if (S.val) S.val[(int64_t)f * P.ng + p] = val;
    if (S.grad)
#pragma unroll
      for (int a = 0; a < D; ++a) S.grad[((int64_t)f * D + a) * P.ng + p] = grad[a];
  }
}

// One group of anchor_lanes<D>() lanes per point: the group finds the
// anchor, then lane f evaluates field f.
template <int D>
__global__ __launch_bounds__(256) void k_surface_query(SurfArgs S, int64_t nq,
                                                       const double* __restrict__ xq) {
  constexpr int NL = anchor_lanes<D>();
  const int sub = (int)threadIdx.x % NL;
  const int64_t q = (int64_t)blockIdx.x * (256 / NL) + threadIdx.x / NL;
  const bool active = q < nq;
  const PlanD& P = S.P;
  double x[3] = {0.0, 0.0, 0.0};
  if (active)
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = xq[a * nq + q];
  const int g = find_anchor_group<D, NL>(P, x, sub, active);
  if (!active) return;
  if (sub == 0 && S.anchor) S.anchor[q] = g;
  if (sub >= S.nf) return;
  const int f = sub;
  const double nanv = __longlong_as_double(0x7ff8000000000000LL);
  double val = nanv, grad[3] = {nanv, nanv, nanv};
  if (g >= 0) {
    const uint32_t code = P.code[g];
    int i, j, k;
    unlinear(P.g, P.cell[g], i, j, k);
    const int ijk[3] = {i, j, k};
    double rel[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a) rel[a] = x[a] - centre(P.g, a, ijk[a]);
    double v[8], X[3];
    stencil_span(P.g, code, P.cell[g], X);
    corner_values<D>(P, g, S.f[f], v);
    box_eval<D>(rel, X, v, val, grad);
  }
  if (S.val) S.val[(int64_t)f * nq + q] = val;
  if (S.grad)
#pragma unroll
    for (int a = 0; a < D; ++a) S.grad[((int64_t)f * D + a) * nq + q] = grad[a];
}

void launch_surface_ghost(const SurfArgs& S, hipStream_t st) {
  if (S.P.ng <= 0) return;
  const unsigned nb = (unsigned)((S.P.ng + 255) / 256);
  if (S.P.g.dim == 2) k_surface_ghost<2><<<nb, 256, 0, st>>>(S);
  else k_surface_ghost<3><<<nb, 256, 0, st>>>(S);
}

void launch_surface_query(const SurfArgs& S, int64_t nq, const double* xq, hipStream_t st) {
  if (nq <= 0) return;
  const unsigned nb = (unsigned)force_blocks(S.P.g.dim, nq);
  if (S.P.g.dim == 2) k_surface_query<2><<<nb, 256, 0, st>>>(S, nq, xq);
  else k_surface_query<3><<<nb, 256, 0, st>>>(S, nq, xq);
}

// --------------------------------------------------------------------------
// forces: F = sum_q w_q (-p n + mu (grad u + grad u^T) n), reduced in a
// fixed tree order (per-block partials, then one block in block order)
// --------------------------------------------------------------------------

// One group per point: the group finds the anchor, lane 0 evaluates p and
// lane 1 + c the velocity component u_c; lane 0 gathers the gradients and
// forms the weighted traction.  Per-block partials are summed in point
// order by one thread, so the reduction order is fixed.
template <int D>
__global__ __launch_bounds__(256) void k_forces(PlanD P, ForceArgs F, double* __restrict__ part) {
  constexpr int NL = anchor_lanes<D>();
  constexpr int PPB = 256 / NL;
  __shared__ double sh[PPB][3];
  const int sub = (int)threadIdx.x % NL;
  const int grp = (int)threadIdx.x / NL;
  const int64_t q = (int64_t)blockIdx.x * PPB + grp;
  const bool active = q < F.nq;
  double x[3] = {0.0, 0.0, 0.0};
  if (active)
#pragma unroll
    for (int a = 0; a < D; ++a) x[a] = F.xq[a * F.nq + q];
  const int g = find_anchor_group<D, NL>(P, x, sub, active);
  // field of this lane: 0 = p, 1 + c = u_c
  double val = 0.0, grad[3] = {0.0, 0.0, 0.0};
  if (active && g >= 0 && sub <= D) {
    const uint32_t code = P.code[g];
    int i, j, k;
    unlinear(P.g, P.cell[g], i, j, k);
    const int ijk[3] = {i, j, k};
    double rel[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a) rel[a] = x[a] - centre(P.g, a, ijk[a]);
    double v[8], X[3];
    stencil_span(P.g, code, P.cell[g], X);
    corner_values<D>(P, g, sub == 0 ? F.p : F.u[sub - 1], v);
    box_eval<D>(rel, X, v, val, grad);
  }
  // gu[c][a] = d u_c / d x_a, from lane 1 + c of this group
  double gu[3][3];
  const int base = grp * NL;
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int a = 0; a < D; ++a) gu[c][a] = __shfl(grad[a], base + 1 + c, 64);
  if (sub == 0) {
    double t[3] = {0.0, 0.0, 0.0};
    if (active) {
      if (g < 0) {
        t[0] = t[1] = t[2] = __longlong_as_double(0x7ff8000000000000LL);
      } else {
        const double w = F.wq[q];
        double n[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < D; ++a) n[a] = F.nrm[a * F.nq + q];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double s = -val * n[a];
#pragma unroll
          for (int b = 0; b < D; ++b) s += F.mu * (gu[a][b] + gu[b][a]) * n[b];
          t[a] = w * s;
        }
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) sh[grp][a] = t[a];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < PPB; ++i)
#pragma unroll
      for (int a = 0; a < 3; ++a) s[a] += sh[i][a];
#pragma unroll
    for (int a = 0; a < 3; ++a) part[blockIdx.x * 3 + a] = s[a];
  }
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ part, int nb,
                                                      int dim, double* __restrict__ out) {
  __shared__ double sh[256][3];
  double s[3] = {0.0, 0.0, 0.0};
  // contiguous runs per thread, then a fixed tree: deterministic order
  const int per = (nb + 255) / 256;
  for (int b = threadIdx.x * per; b < min(nb, (int)(threadIdx.x + 1) * per); ++b)
    for (int a = 0; a < 3; ++a) s[a] += part[b * 3 + a];
  for (int a = 0; a < 3; ++a) sh[threadIdx.x][a] = s[a];
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k)
      for (int a = 0; a < 3; ++a) sh[threadIdx.x][a] += sh[threadIdx.x + k][a];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int a = 0; a < dim; ++a) out[a] = sh[0][a];
}

void launch_forces(const PlanD& P, const ForceArgs& F, double* part, double* out,
                   hipStream_t st) {
  const int nb = (int)force_blocks(P.g.dim, F.nq);
  if (P.g.dim == 2) k_forces<2><<<nb, 256, 0, st>>>(P, F, part);
  else k_forces<3><<<nb, 256, 0, st>>>(P, F, part);
  k_sum_partials<<<1, 256, 0, st>>>(part, nb, P.g.dim, out);
}

}  // namespace gcr
