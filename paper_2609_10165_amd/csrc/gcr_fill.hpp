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
    ghost_weights<D>(dl, nn, code, P.g.h, bc, w);
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

template <int D>
__device__ __forceinline__ void fill_ghost(const FillArgs& A, int p) {
  const PlanD& P = A.P;
  if (P.blk[p] >= 0) return;   // coupled unit: solved by fill_units_of_level
  const int c = P.cell[p];
  const uint32_t code = P.code[p];
  const uint32_t skip = code_skip(code);
  double dl[3], nn[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dl[a] = a < D ? P.dl[a][p] : 0.0;
    nn[a] = a < D ? P.nn[a][p] : 0.0;
  }
  int off[8];
#pragma unroll
  for (int k = 1; k < (1 << D); ++k) off[k] = c + corner_offset(P.g, code, k);
  double wD[8], wN[8];
  bool haveD = false, haveN = false;
  for (int f = 0; f < A.nf; ++f) {
    const int bc = A.kind[f] == 2 ? (int)A.bt[f][p] : A.kind[f];
    if (bc == 0 && !haveD) {
      ghost_weights<D>(dl, nn, code, P.g.h, 0, wD);
      haveD = true;
    } else if (bc != 0 && !haveN) {
      ghost_weights<D>(dl, nn, code, P.g.h, 1, wN);
      haveN = true;
    }
    double* F = A.f[f];
    double v = (bc == 0 ? wD[0] : wN[0]) * A.b[f][p];
#pragma unroll
    for (int k = 1; k < (1 << D); ++k)
      if (!(k & skip)) v += (bc == 0 ? wD[k] : wN[k]) * F[off[k]];
    F[c] = v;
  }
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
  if (P.blk[p] >= 0) return;
  const int c = P.cell[p];
  const uint32_t code = P.code[p];
  const uint32_t skip = code_skip(code);
  double dl[3], nn[3], w[8];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    dl[a] = a < D ? P.dl[a][p] : 0.0;
    nn[a] = a < D ? P.nn[a][p] : 0.0;
  }
  const int bc = kind == 2 ? (int)bt[p] : kind;
  ghost_weights<D>(dl, nn, code, P.g.h, bc, w);
  double v = w[0] * b[p];
#pragma unroll
  for (int k = 1; k < (1 << D); ++k)
    if (!(k & skip)) v += w[k] * F[c + corner_offset(P.g, code, k)];
  F[c] = v;
}

}  // namespace gcr
