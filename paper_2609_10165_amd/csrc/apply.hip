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
  double rel[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) rel[a] = a < D ? P.dl[a][p] : 0.0;
  for (int f = 0; f < S.nf; ++f) {
    double v[8], val, grad[3];
    corner_values<D>(P, p, S.f[f], v);
    box_eval<D>(rel, code, P.g.h, v, val, grad);
    if (S.val) S.val[(int64_t)f * P.ng + p] = val;
    if (S.grad)
#pragma unroll
      for (int a = 0; a < D; ++a) S.grad[((int64_t)f * D + a) * P.ng + p] = grad[a];
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_surface_query(SurfArgs S, int64_t nq,
                                                       const double* __restrict__ xq) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const PlanD& P = S.P;
  double x[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < D; ++a) x[a] = xq[a * nq + q];
  const int g = find_anchor<D>(P, x);
  if (S.anchor) S.anchor[q] = g;
  double rel[3] = {0.0, 0.0, 0.0};
  uint32_t code = 0;
  if (g >= 0) {
    code = P.code[g];
    int i, j, k;
    unlinear(P.g, P.cell[g], i, j, k);
    const int ijk[3] = {i, j, k};
#pragma unroll
    for (int a = 0; a < D; ++a) rel[a] = x[a] - centre(P.g, a, ijk[a]);
  }
  const double nanv = __longlong_as_double(0x7ff8000000000000LL);
  for (int f = 0; f < S.nf; ++f) {
    double val = nanv, grad[3] = {nanv, nanv, nanv};
    if (g >= 0) {
      double v[8];
      corner_values<D>(P, g, S.f[f], v);
      box_eval<D>(rel, code, P.g.h, v, val, grad);
    }
    if (S.val) S.val[(int64_t)f * nq + q] = val;
    if (S.grad)
#pragma unroll
      for (int a = 0; a < D; ++a) S.grad[((int64_t)f * D + a) * nq + q] = grad[a];
  }
}

void launch_surface_ghost(const SurfArgs& S, hipStream_t st) {
  if (S.P.ng <= 0) return;
  const unsigned nb = (unsigned)((S.P.ng + 255) / 256);
  if (S.P.g.dim == 2) k_surface_ghost<2><<<nb, 256, 0, st>>>(S);
  else k_surface_ghost<3><<<nb, 256, 0, st>>>(S);
}

void launch_surface_query(const SurfArgs& S, int64_t nq, const double* xq, hipStream_t st) {
  if (nq <= 0) return;
  const unsigned nb = (unsigned)((nq + 255) / 256);
  if (S.P.g.dim == 2) k_surface_query<2><<<nb, 256, 0, st>>>(S, nq, xq);
  else k_surface_query<3><<<nb, 256, 0, st>>>(S, nq, xq);
}

// --------------------------------------------------------------------------
// forces: F = sum_q w_q (-p n + mu (grad u + grad u^T) n), reduced in a
// fixed tree order (per-block partials, then one block in block order)
// --------------------------------------------------------------------------

template <int D>
__device__ __forceinline__ void traction(const PlanD& P, const ForceArgs& F, int64_t q,
                                         double t[3]) {
  t[0] = t[1] = t[2] = 0.0;
  double x[3] = {0.0, 0.0, 0.0}, n[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < D; ++a) {
    x[a] = F.xq[a * F.nq + q];
    n[a] = F.nrm[a * F.nq + q];
  }
  const int g = find_anchor<D>(P, x);
  if (g < 0) {
    t[0] = t[1] = t[2] = __longlong_as_double(0x7ff8000000000000LL);
    return;
  }
  const uint32_t code = P.code[g];
  int i, j, k;
  unlinear(P.g, P.cell[g], i, j, k);
  const int ijk[3] = {i, j, k};
  double rel[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int a = 0; a < D; ++a) rel[a] = x[a] - centre(P.g, a, ijk[a]);
  double v[8], pv, pg[3], gu[3][3];
  corner_values<D>(P, g, F.p, v);
  box_eval<D>(rel, code, P.g.h, v, pv, pg);
#pragma unroll
  for (int c = 0; c < D; ++c) {
    double uv;
    corner_values<D>(P, g, F.u[c], v);
    box_eval<D>(rel, code, P.g.h, v, uv, gu[c]);   // gu[c][a] = d u_c / d x_a
  }
  const double w = F.wq[q];
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double s = -pv * n[a];
#pragma unroll
    for (int b = 0; b < D; ++b) s += F.mu * (gu[a][b] + gu[b][a]) * n[b];
    t[a] = w * s;
  }
}

template <int D>
__global__ __launch_bounds__(256) void k_forces(PlanD P, ForceArgs F, double* __restrict__ part) {
  __shared__ double sh[256][3];
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double t[3] = {0.0, 0.0, 0.0};
  if (q < F.nq) traction<D>(P, F, q, t);
  for (int a = 0; a < 3; ++a) sh[threadIdx.x][a] = t[a];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int a = 0; a < 3; ++a) sh[threadIdx.x][a] += sh[threadIdx.x + s][a];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int a = 0; a < 3; ++a) part[blockIdx.x * 3 + a] = sh[0][a];
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
  const int nb = (int)std::max<int64_t>(1, (F.nq + 255) / 256);
  if (P.g.dim == 2) k_forces<2><<<nb, 256, 0, st>>>(P, F, part);
  else k_forces<3><<<nb, 256, 0, st>>>(P, F, part);
  k_sum_partials<<<1, 256, 0, st>>>(part, nb, P.g.dim, out);
}

}  // namespace gcr
