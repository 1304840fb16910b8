// gcr_fill.hpp -- per-ghost fill of the level-by-level reconstruction
// (relations of Sec. 4.1 / 5.1 in tensor-product form, coupled units solved
// together), shared by the single-plan and batched kernels.
#pragma once

#include "gcr_apply.hpp"

namespace gcr {

template <int D>
__device__ __noinline__ void fill_unit(const FillArgs& A, int u) {
  const PlanD& P = A.P;
  const int k = P.unit_cnt[u];
  int mem[kMaxUnit], cel[kMaxUnit];
  for (int i = 0; i < k; ++i) {
    mem[i] = P.unit_mem[u * kMaxUnit + i];
    cel[i] = P.cell[mem[i]];
  }
  for (int f = 0; f < A.nf; ++f) {
    double M[kMaxUnit * kMaxUnit], rhs[kMaxUnit];
    double* F = A.f[f];
    for (int i = 0; i < k; ++i) {
      const int p = mem[i];
      const uint32_t code = P.code[p];
      const uint32_t skip = code_skip(code);
      double dl[3], nn[3], w[8];
      for (int a = 0; a < 3; ++a) {
        dl[a] = a < D ? P.dl[a][p] : 0.0;
        nn[a] = a < D ? P.nn[a][p] : 0.0;
      }
      const int bc = A.kind[f] == 2 ? (int)A.bt[f][p] : A.kind[f];
      ghost_weights<D>(dl, nn, code, P.g.h, bc, w);
      for (int t = 0; t < k; ++t) M[i * k + t] = (t == i) ? 1.0 : 0.0;
      rhs[i] = w[0] * A.b[f][p];
      for (int c = 1; c < (1 << D); ++c) {
        if (c & skip) continue;
        const int q = cel[i] + corner_offset(P.g, code, c);
        int t = -1;
        for (int s = 0; s < k; ++s)
          if (cel[s] == q) t = s;
        if (t >= 0) M[i * k + t] -= w[c];
        else rhs[i] += w[c] * F[q];
      }
    }
    // Gaussian elimination with partial pivoting
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
    for (int i = 0; i < k; ++i) F[cel[i]] = rhs[i];
  }
}

template <int D>
__device__ __forceinline__ void fill_ghost(const FillArgs& A, int p) {
  const PlanD& P = A.P;
  const int u = P.blk[p];
  if (u >= 0) {
    if (P.unit_mem[u * kMaxUnit] == p) fill_unit<D>(A, u);
    return;
  }
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
    const double* w;
    if (bc == 0) {
      if (!haveD) {
        ghost_weights<D>(dl, nn, code, P.g.h, 0, wD);
        haveD = true;
      }
      w = wD;
    } else {
      if (!haveN) {
        ghost_weights<D>(dl, nn, code, P.g.h, 1, wN);
        haveN = true;
      }
      w = wN;
    }
    double* F = A.f[f];
    double v = w[0] * A.b[f][p];
#pragma unroll
    for (int k = 1; k < (1 << D); ++k)
      if (!(k & skip)) v += w[k] * F[off[k]];
    F[c] = v;
  }
}


// One field of one ghost (the batched kernel's inner step).
template <int D>
__device__ __forceinline__ void fill_single(const PlanD& P, int p, double* F, const double* b,
                                            const uint8_t* bt, int kind) {
  const int u = P.blk[p];
  if (u >= 0) {
    if (P.unit_mem[u * kMaxUnit] == p) {
      FillArgs A;
      A.P = P;
      A.nf = 1;
      A.kind[0] = kind;
      A.f[0] = F;
      A.b[0] = b;
      A.bt[0] = bt;
      fill_unit<D>(A, u);
    }
    return;
  }
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
