// gcr_fill.hpp -- per-ghost fill of the level-by-level reconstruction
// (relations of Sec. 4.1 / 5.1 in tensor-product form), shared by the
// single-plan and batched kernels.  Ghosts that belong to a coupled unit are
// skipped by the per-ghost path and solved together afterwards, one unit per
// thread, in an LDS workspace.
#pragma once

#include "gcr_apply.hpp"

namespace gcr {

// One field of coupled unit u: (I - W_int) phi = W_ext phi_ext + ws b.
template <int D>
__device__ __forceinline__ void fill_unit_field(const PlanD& P, int u, double* F,
                                                const double* b, const uint8_t* bt, int kind,
                                                UnitWS& ws) {
  const int k = P.unit_cnt[u];
  for (int i = 0; i < k; ++i) {
    ws.mem[i] = P.unit_mem[u * kMaxUnit + i];
    ws.cel[i] = P.cell[ws.mem[i]];
  }
  for (int i = 0; i < k; ++i) {
    const int p = ws.mem[i];
    const uint32_t code = P.code[p];
    const uint32_t skip = code_skip(code);
    double dl[3], nn[3], w[8];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      dl[a] = a < D ? P.dl[a][p] : 0.0;
      nn[a] = a < D ? P.nn[a][p] : 0.0;
    }
    const int bc = kind == 2 ? (int)bt[p] : kind;
    double X[3];
    stencil_span(P.g, code, ws.cel[i], X);
    ghost_weights<D>(dl, nn, X, bc, w);
    for (int t = 0; t < k; ++t) ws.M[i * k + t] = (t == i) ? 1.0 : 0.0;
    double r = w[0] * b[p];
#pragma unroll
    for (int c = 1; c < (1 << D); ++c) {
      if (c & skip) continue;
      const int q = ws.cel[i] + corner_offset(P.g, code, c);
      int t = -1;
      for (int s = 0; s < k; ++s)
        if (ws.cel[s] == q) t = s;
      if (t >= 0) ws.M[i * k + t] -= w[c];
      else r += w[c] * F[q];
    }
    ws.rhs[i] = r;
  }
  ws_solve(ws, k);
  for (int i = 0; i < k; ++i) F[ws.cel[i]] = ws.rhs[i];
}

// Loads are ordered so that each ghost costs two dependent round trips:
// first its metadata, boundary data and cached weights (none depends on
// another load), then its stencil corners; all stores come last.  A ghost of
// level k reads only fluid cells and ghosts of lower levels, never a slot
// that this launch writes, so this order is exact.  (The compiler cannot
// prove that on its own, since field and weight arrays could alias.)
// Ghosts of coupled units compute but do not store (their unit solve does).
constexpr int kFieldGroup = 4;

// Fields f0 .. f0 + kFieldGroup - 1 of ghost p (metadata already loaded).
template <int D>
__device__ __forceinline__ void fill_group(const FillArgs& A, int p, int f0, bool live, int c,
                                           uint32_t code) {
  const PlanD& P = A.P;
  const int ng = P.ng;
  const double* const W0 = A.w[0];
  const double* const W1 = A.w[1];
  int bc[kFieldGroup];
  double bv[kFieldGroup];
  // slots past nf load field nf - 1 again (never stored): no branches here
#pragma unroll
  for (int j = 0; j < kFieldGroup; ++j) {
    const int f = min(f0 + j, A.nf - 1);
    bc[j] = (int)A.bt[f][(int64_t)p * A.bts[f]];
    bv[j] = A.b[f][p];
  }
  // both kinds' arrays are always allocated (a kind no field uses holds
  // unused values), so the loads need not wait for the kinds
  double wD[8], wN[8];
#pragma unroll
  for (int k = 0; k < (1 << D); ++k) {
    wD[k] = W0[(int64_t)k * ng + p];
    wN[k] = W1[(int64_t)k * ng + p];
  }
  const uint32_t skip = code_skip(code);
  double val[kFieldGroup][8];
  // x-adjacent corners (multiplier 1 along x, x not skipped): one 16-byte
  // load per pair, as in fill_single
  const bool pair = !(skip & 1u) && code_r(code, 0) == 1;
  const int lo = code_e(code, 0) < 0 ? -1 : 0;
#pragma unroll
  for (int j = 0; j < kFieldGroup; ++j) {
    const double* F = A.f[min(f0 + j, A.nf - 1)];
    if (pair) {
#pragma unroll
      for (int k = 0; k < (1 << D); k += 2) {
        if (k & skip) {
          val[j][k] = val[j][k + 1] = 0.0;
          continue;
        }
        double two[2];
        __builtin_memcpy(two, F + c + corner_offset(P.g, code, k) + lo, 16);
        val[j][k] = lo ? two[1] : two[0];
        val[j][k + 1] = lo ? two[0] : two[1];
      }
    } else {
#pragma unroll
      for (int k = 1; k < (1 << D); ++k)
        val[j][k] = (k & skip) ? 0.0 : F[c + corner_offset(P.g, code, k)];
    }
  }
  double v[kFieldGroup];
#pragma unroll
  for (int j = 0; j < kFieldGroup; ++j) {
    const bool dir = bc[j] == 0;
    double sum = (dir ? wD[0] : wN[0]) * bv[j];
#pragma unroll
    for (int k = 1; k < (1 << D); ++k)
      if (!(k & skip)) sum += (dir ? wD[k] : wN[k]) * val[j][k];
    v[j] = sum;
  }
  if (live)
#pragma unroll
    for (int j = 0; j < kFieldGroup; ++j)
      if (f0 + j < A.nf) A.f[f0 + j][c] = v[j];
}

template <int D>
__device__ __forceinline__ void fill_ghost(const FillArgs& A, int p) {
  const PlanD& P = A.P;
  const bool live = P.blk[p] < 0;
  const int c = P.cell[p];
  const uint32_t code = P.code[p];
  // straight-line groups (kMaxFields = 2 * kFieldGroup), so the first
  // group's independent loads issue together with the metadata loads
  fill_group<D>(A, p, 0, live, c, code);
  if (A.nf > kFieldGroup) fill_group<D>(A, p, kFieldGroup, live, c, code);
}

// Units of level `level` (1-based), every field; threads tid < nthreads each
// take units round-robin, with ws[tid] as workspace.
template <int D>
__device__ __forceinline__ void fill_units_of_level(const FillArgs& A, int level, UnitWS* ws,
                                                    int tid, int nthreads) {
  const PlanD& P = A.P;
  for (int s = tid; s < P.nunits; s += nthreads) {
    if (P.unit_lev[s] != level) continue;
    for (int f = 0; f < A.nf; ++f) fill_unit_field<D>(P, s, A.f[f], A.b[f], A.bt[f], A.kind[f], ws[tid]);
  }
}

// One field of one ghost (the batched kernel's inner step).
template <int D>
__device__ __forceinline__ void fill_single(const PlanD& P, int p, double* F, const double* b,
                                            const uint8_t* bt, int kind) {
  const int blk = P.blk[p];
  const int c = P.cell[p];
  const uint32_t code = P.code[p];
  double dl[3], nn[3], w[8], val[8];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dl[a] = a < D ? P.dl[a][p] : 0.0;
    nn[a] = a < D ? P.nn[a][p] : 0.0;
  }
  const int bc = kind == 2 ? (int)bt[p] : kind;
  const double bv = b[p];
  if (blk >= 0) return;
  const uint32_t skip = code_skip(code);
  if (!(skip & 1u) && code_r(code, 0) == 1) {
    // corners k and k + 1 differ by one cell along x: one 16-byte load per
    // pair (corner 0's partner is the ghost's own slot, read and unused)
    const int lo = code_e(code, 0) < 0 ? -1 : 0;
#pragma unroll
    for (int k = 0; k < (1 << D); k += 2) {
      if (k & skip) {
        val[k] = val[k + 1] = 0.0;
        continue;
      }
      double two[2];
      __builtin_memcpy(two, F + c + corner_offset(P.g, code, k) + lo, 16);
      val[k] = lo ? two[1] : two[0];
      val[k + 1] = lo ? two[0] : two[1];
    }
  } else {
#pragma unroll
    for (int k = 1; k < (1 << D); ++k)
      val[k] = (k & skip) ? 0.0 : F[c + corner_offset(P.g, code, k)];
  }
  double X[3];
  stencil_span(P.g, code, c, X);
  ghost_weights<D>(dl, nn, X, bc, w);
  double v = w[0] * bv;
#pragma unroll
  for (int k = 1; k < (1 << D); ++k)
    if (!(k & skip)) v += w[k] * val[k];
  F[c] = v;
}

}  // namespace gcr
