// gcr_apply.hpp -- argument blocks of the apply kernels and their launchers.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/gcr.h"
#include "gcr_device.hpp"

namespace gcr {

// Device view of one plan (canonical ghost order).
struct PlanD {
  GridD g;
  int ng;
  const int8_t* tags;
  const int32_t* cell;
  const double* dl[3];      // x_s - x_c
  const double* nn[3];      // unit normal into the fluid
  const uint32_t* code;
  const int32_t* blk;       // coupled-unit slot or -1
  const int32_t* unit_mem;  // [slot][kMaxUnit] canonical positions
  const int32_t* unit_cnt;
  const int32_t* sorted_cell;  // ghost cells in linear-index order
  const int32_t* sorted_pos;   // their canonical positions
  int rmax[3];                 // largest stencil multiplier per axis
  const unsigned long long* htab;  // open-addressing table cell -> canonical position
  unsigned hmask;
  int nunits;                  // coupled units
  const int32_t* unit_lev;     // their levels (1-based)
  // batched forward, 2D: [3][ng] the position of corner k + 1's ghost, -1 for
  // a fluid corner, -2 for a skipped one (null elsewhere)
  const int32_t* cgi;
};

constexpr unsigned long long kHashEmpty = ~0ull;

__device__ __forceinline__ unsigned cell_hash(int c) {
  unsigned h = (unsigned)c * 2654435761u;
  return h ^ (h >> 15);
}

// canonical position of the ghost in cell c, or -1 (linear probing; the
// table is at most half full, so every probe sequence reaches an empty slot)
__device__ __forceinline__ int ghost_at(const PlanD& P, int c) {
  unsigned h = cell_hash(c) & P.hmask;
  for (;;) {
    const unsigned long long e = P.htab[h];
    if (e == kHashEmpty) return -1;
    if ((int)(e >> 32) == c) return (int)(e & 0xffffffffu);
    h = (h + 1) & P.hmask;
  }
}

// LDS workspace of one coupled-unit solve
struct UnitWS {
  double M[kMaxUnit * kMaxUnit];
  double rhs[kMaxUnit];
  int cel[kMaxUnit];
  int mem[kMaxUnit];
};

// Gaussian elimination with partial pivoting on ws.M (k x k) ws.rhs, in place
__device__ __forceinline__ void ws_solve(UnitWS& ws, int k) {
  double* M = ws.M;
  double* rhs = ws.rhs;
  for (int c = 0; c < k; ++c) {
    int piv = c;
    for (int r = c + 1; r < k; ++r)
      if (fabs(M[r * k + c]) > fabs(M[piv * k + c])) piv = r;
    if (piv != c) {
      for (int t = 0; t < k; ++t) {
        double x = M[c * k + t];
        M[c * k + t] = M[piv * k + t];
        M[piv * k + t] = x;
      }
      double x = rhs[c];
      rhs[c] = rhs[piv];
      rhs[piv] = x;
    }
    for (int r = c + 1; r < k; ++r) {
      double fct = M[r * k + c] / M[c * k + c];
      for (int t = c; t < k; ++t) M[r * k + t] -= fct * M[c * k + t];
      rhs[r] -= fct * rhs[c];
    }
  }
  for (int c = k - 1; c >= 0; --c) {
    double v = rhs[c];
    for (int t = c + 1; t < k; ++t) v -= M[c * k + t] * rhs[t];
    rhs[c] = v / M[c * k + c];
  }
}

struct FillArgs {
  PlanD P;
  int nf;
  int kind[kMaxFields];            // 0 Dirichlet, 1 Neumann, 2 per-ghost
  double* f[kMaxFields];
  const double* b[kMaxFields];
  const uint8_t* bt[kMaxFields];   // kind of ghost p: bt[f][p * bts[f]] (per-ghost array,
  int bts[kMaxFields];             // stride 1, or the plan's {0, 1} table, stride 0)
  const double* w[2];              // cached weights per kind, [2^D][ng]
};

struct SurfArgs {
  PlanD P;
  int nf;
  const double* f[kMaxFields];
  double* val;
  double* grad;
  int32_t* anchor;
};

struct ForceArgs {
  int64_t nq;
  const double* xq;
  const double* nrm;
  const double* wq;
  const double* p;
  const double* u[3];
  double mu;
};

PlanD plan_view(const gcr_plan* p);

void launch_fill_range(const FillArgs& A, int lo, int hi, hipStream_t st);
void launch_weights(const PlanD& P, int bc, double* w, uint8_t* kinds, hipStream_t st);
void launch_fill_wg(const FillArgs& A, const int32_t* d_lev_off, int nlev, int threads,
                    hipStream_t st);
void launch_fill_units(const FillArgs& A, int level, hipStream_t st);
void launch_surface_ghost(const SurfArgs& S, hipStream_t st);
void launch_surface_query(const SurfArgs& S, int64_t nq, const double* xq, hipStream_t st);
void launch_forces(const PlanD& P, const ForceArgs& F, double* part, double* out,
                   hipStream_t st);

}  // namespace gcr

namespace gcr {

// Corner values of ghost p's stencil box; corners outside the grid read NaN.
template <int D>
__device__ __forceinline__ void corner_values(const PlanD& P, int p, const double* F, double v[8]) {
  const int c = P.cell[p];
  const uint32_t code = P.code[p];
  int i, j, k;
  unlinear(P.g, c, i, j, k);
#pragma unroll
  for (int m = 0; m < (1 << D); ++m)
    v[m] = corner_in_grid(P.g, code, i, j, k, m) ? F[c + corner_offset(P.g, code, m)]
                                                 : __longlong_as_double(0x7ff8000000000000LL);
}

// Anchor of a point: among ghosts within 2 cells per axis of the point's
// cell, the one whose foot point is nearest; ties go to the smaller linear
// index (cells are visited in ascending linear index, strict comparison).
template <int D>
__device__ __forceinline__ int find_anchor(const PlanD& P, const double x[3]) {
  int qi[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) qi[a] = cell_of(P.g, a, x[a]);
  int best = -1;
  double bd = 1e300;
  const int z0 = D == 3 ? qi[2] - 2 : 0, z1 = D == 3 ? qi[2] + 2 : 0;
  for (int kz = z0; kz <= z1; ++kz) {
    if (D == 3 && (kz < 0 || kz >= P.g.n[2])) continue;
    for (int jy = qi[1] - 2; jy <= qi[1] + 2; ++jy) {
      if (jy < 0 || jy >= P.g.n[1]) continue;
      for (int ix = qi[0] - 2; ix <= qi[0] + 2; ++ix) {
        if (ix < 0 || ix >= P.g.n[0]) continue;
        const int c = linear(P.g, ix, jy, kz);
        const int8_t t = P.tags[c];
        if (t != 2 && t != -2) continue;
        const int g = ghost_at(P, c);
        if (g < 0) continue;
        const int q[3] = {ix, jy, kz};
        double d2 = 0.0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double s = centre(P.g, a, q[a]) + P.dl[a][g];
          d2 += (x[a] - s) * (x[a] - s);
        }
        if (d2 < bd) {
          bd = d2;
          best = g;
        }
      }
    }
  }
  return best;
}

// The same anchor found by NL cooperating lanes (NL a power of two, the
// lanes sub = 0..NL-1 of one aligned group of a wave, all of them calling):
// each lane scans every NL-th cell of the 5^D neighbourhood, then the group
// reduces (d2, linear index) lexicographically, which picks the cell the
// serial scan picks.  `active` false makes a lane scan nothing (it still
// takes part in the reduction).
template <int D>
constexpr int anchor_lanes() { return D == 3 ? 64 : 32; }

template <int D, int NL>
__device__ __forceinline__ int find_anchor_group(const PlanD& P, const double x[3], int sub,
                                                 bool active) {
  constexpr int NC = D == 3 ? 125 : 25;
  int qi[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) qi[a] = cell_of(P.g, a, x[a]);
  double bd = 1e300;
  int bc = 0x7fffffff, bg = -1;
  if (active) {
    for (int t = sub; t < NC; t += NL) {
      const int ix = qi[0] - 2 + t % 5;
      const int jy = qi[1] - 2 + (t / 5) % 5;
      const int kz = D == 3 ? qi[2] - 2 + t / 25 : 0;
      if (ix < 0 || ix >= P.g.n[0] || jy < 0 || jy >= P.g.n[1]) continue;
      if (D == 3 && (kz < 0 || kz >= P.g.n[2])) continue;
      const int c = linear(P.g, ix, jy, kz);
      const int8_t tg = P.tags[c];
      if (tg != 2 && tg != -2) continue;
      const int g = ghost_at(P, c);
      if (g < 0) continue;
      const int q[3] = {ix, jy, kz};
      double d2 = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double s = centre(P.g, a, q[a]) + P.dl[a][g];
        d2 += (x[a] - s) * (x[a] - s);
      }
      if (d2 < bd || (d2 == bd && c < bc)) {
        bd = d2;
        bc = c;
        bg = g;
      }
    }
  }
#pragma unroll
  for (int o = NL / 2; o > 0; o >>= 1) {
    const double od = __shfl_xor(bd, o, NL);
    const int oc = __shfl_xor(bc, o, NL);
    const int og = __shfl_xor(bg, o, NL);
    if (od < bd || (od == bd && oc < bc)) {
      bd = od;
      bc = oc;
      bg = og;
    }
  }
  return bg;
}

// Blocks (and per-block force partials) of the force kernel for nq points.
inline int64_t force_blocks(int dim, int64_t nq) {
  const int ppb = 256 / (dim == 3 ? anchor_lanes<3>() : anchor_lanes<2>());
  return std::max<int64_t>(1, (nq + ppb - 1) / ppb);
}

}  // namespace gcr
