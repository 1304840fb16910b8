// classify.hip -- classification of every cell of a batch (Sec. 3.1): the
// inside test at the cell centre (psi >= 0 solid) and the interface mark
// (a face neighbour of the other class).
//
// Three launches: a pre-pass settles whole 1024-cell spans from bounds on
// the body (a radial bound, or a Lipschitz bound on the star radius); the
// store pass writes every settled 16-cell row segment as constant stores and
// the cells of unsettled segments away from the body, and lists the segments
// that need an exact test of every cell; the band pass runs those, one wave
// per segment.
#include <hip/hip_runtime.h>

#include "gcr_impl.hpp"

namespace gcr {

// --------------------------------------------------------------------------
// 1. classification
// --------------------------------------------------------------------------

// Star and SH bodies: r over the directions a box subtends from the centre
// lies within r(w_c) +- lip * D, D the box's angular radius, so a box whose
// distances from the centre all exceed (or all stay below) that range is
// fluid (solid) throughout.  Returns 0 / 1, or -1 if the box may straddle.
__device__ __forceinline__ int star_box(const ShapeD& s, int dim, const double lo[3],
                                        const double hi[3]) {
  double xc[3] = {0.0, 0.0, 0.0}, rc2 = 0.0, hd2 = 0.0;
  for (int a = 0; a < dim; ++a) {
    xc[a] = 0.5 * (lo[a] + hi[a]) - s.c[a];
    const double e = 0.5 * (hi[a] - lo[a]);
    rc2 += xc[a] * xc[a];
    hd2 += e * e;
  }
  const double rc = sqrt(rc2), hd = sqrt(hd2);
  if (!(rc > 2.0 * hd)) return -1;
  const double D = asin(hd / rc) * (1.0 + 1e-12) + 1e-15;
  double r;
  if (s.kind == kStar2D) {
    double r1;
    star_r(s, xc[0] / rc, xc[1] / rc, r, r1);
  } else {
    const double u[3] = {xc[0] / rc, xc[1] / rc, xc[2] / rc};
    double gr[3];
    sh_r(s, u, r, gr);
  }
  const double spread = s.lip * D;
  if (rc - hd > (r + spread) * (1.0 + 1e-9) + 1e-300) return 0;
  if (rc + hd < (r - spread) * (1.0 - 1e-9)) return 1;
  return -1;
}

// Whether every point of the box [lo, hi] lies on one side of the boundary:
// 0 fluid, 1 solid, -1 undecided (radial bounds, then the Lipschitz test).
__device__ __forceinline__ int box_settled(const ShapeD& s, int dim, const double lo[3],
                                           const double hi[3]) {
  double dmin2 = 0.0, dmax2 = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double c = s.cull_c[a];
    const double dl = c < lo[a] ? lo[a] - c : (c > hi[a] ? c - hi[a] : 0.0);
    const double df = fmax(fabs(c - lo[a]), fabs(hi[a] - c));
    dmin2 += dl * dl;
    dmax2 += df * df;
  }
  if (sqrt(dmin2) > s.rmax * (1.0 + 1e-9) + 1e-300) return 0;
  if (sqrt(dmax2) < s.rmin * (1.0 - 1e-9)) return 1;
  if (s.kind == kStar2D || s.kind == kShStar) return star_box(s, dim, lo, hi);
  return -1;
}

// Solid test of cell (i, j, k); g and s come from registers and LDS (the
// caller copies them once per workgroup: read through the instance table,
// every field would be a dependent scalar load).
__device__ __forceinline__ bool cell_solid(const GridD& g, const ShapeD& s, int i, int j, int k) {
  double x[3] = {centre(g, 0, i), centre(g, 1, j), g.dim == 3 ? centre(g, 2, k) : 0.0};
  return inside(s, g.dim, x);
}

// One thread per span of 64 * kSeg cells (one classification wave): whether
// the box of the span's cells and their face neighbours, in index space,
// lies wholly on one side of the boundary (0 fluid, 1 solid, -1 undecided).
__global__ __launch_bounds__(256) void k_spans(const Inst* __restrict__ insts, int ninst,
                                               const int64_t* __restrict__ chunk_start,
                                               int64_t nspan, int8_t* __restrict__ span,
                                               int32_t* __restrict__ nband) {
  constexpr int kSpan = 64 * kSeg, kPer = kChunk / kSpan;
  const int64_t sp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (sp == 0) nband[0] = 0;   // the band list k_classify appends to starts empty
  if (sp >= nspan) return;
  const int64_t chunk = sp / kPer;
  const int ii = find_inst(chunk_start, ninst, chunk);
  const Inst& I = insts[ii];
  const GridD& g = I.g;
  const int64_t base = (chunk - I.chunk_off) * kChunk + (sp % kPer) * kSpan;
  int8_t r = -1;
  if (base < g.ncell) {
    int p0[3], p1[3], mn[3], mx[3];
    unlinear(g, (int)base, p0[0], p0[1], p0[2]);
    unlinear(g, (int)min(base + kSpan, g.ncell) - 1, p1[0], p1[1], p1[2]);
    for (int a = 0; a < 3; ++a) {
      mn[a] = p0[a];
      mx[a] = p1[a];
    }
    if (p0[2] != p1[2]) {
      mn[0] = mn[1] = 0;
      mx[0] = g.n[0] - 1;
      mx[1] = g.n[1] - 1;
    } else if (p0[1] != p1[1]) {
      mn[0] = 0;
      mx[0] = g.n[0] - 1;
    }
    double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < g.dim; ++a) {
      lo[a] = centre_below(g, a, mn[a]);
      hi[a] = centre_above(g, a, mx[a]);
    }
    r = (int8_t)box_settled(I.s, g.dim, lo, hi);
  }
  span[sp] = r;
}

__global__ __launch_bounds__(256) void k_classify(const Inst* __restrict__ insts, int ninst,
                                                  const int64_t* __restrict__ chunk_start,
                                                  const int8_t* __restrict__ span,
                                                  int8_t* __restrict__ tags,
                                                  int32_t* __restrict__ chunk_cnt,
                                                  int32_t* __restrict__ band,
                                                  int32_t* __restrict__ nband) {
  const int64_t chunk = blockIdx.x;
  const int ii = find_inst(chunk_start, ninst, chunk);
  const Inst& I = insts[ii];
  const GridD g = I.g;
  const int64_t chunk_off = I.chunk_off, cell_off = I.cell_off;
  __shared__ int s_cnt, s_band, s_base;
  __shared__ ShapeD sh_s;
  static_assert(sizeof(ShapeD) % 8 == 0, "ShapeD copied as doubles");
  constexpr int kSpans = kChunk / (64 * kSeg);
  // a workgroup whose spans are all whole and settled only stores: one round
  // of flag loads, no barrier (most workgroups of a large grid)
  bool need_shape = false;
  int8_t fl[kSpans];
  for (int q = 0; q < kSpans; ++q) {
    fl[q] = span[chunk * kSpans + q];
    need_shape |= (chunk - chunk_off) * kChunk + (int64_t)(q + 1) * 64 * kSeg > g.ncell ||
                  fl[q] < 0;
  }
  if (!need_shape) {
    const int8_t f = fl[threadIdx.x >> 6];
    const uint32_t v = f ? 0x01010101u : 0u;
    *reinterpret_cast<uint4*>(tags + cell_off + (chunk - chunk_off) * kChunk +
                              (int64_t)threadIdx.x * kSeg) = make_uint4(v, v, v, v);
    if (threadIdx.x == 0) chunk_cnt[chunk] = 0;
    return;
  }
  {
    const double* src = reinterpret_cast<const double*>(&I.s);
    double* dst = reinterpret_cast<double*>(&sh_s);
    for (int q = (int)threadIdx.x; q < (int)(sizeof(ShapeD) / 8); q += 256) dst[q] = src[q];
  }
  if (threadIdx.x == 0) {
    s_cnt = 0;
    s_band = 0;
  }
  __syncthreads();
  const ShapeD& S = sh_s;
  const int64_t base64 = (chunk - chunk_off) * kChunk + (int64_t)threadIdx.x * kSeg;
  int cnt = 0;
  // a wave whose span the pre-pass settled only stores (full spans only:
  // the last, partial span of an instance takes the per-segment path)
  const int64_t wbase = base64 - (int64_t)(threadIdx.x & 63) * kSeg;
  const int wset = wbase + 64 * kSeg <= g.ncell ? (int)span[chunk * (kChunk / (64 * kSeg)) +
                                                             (threadIdx.x >> 6)]
                                                : -1;
  int mode = 0;   // 0 no cells or stored here, 1 settled segment, 2 band, 3 cell by cell
  if (wset >= 0) {
    const uint32_t v = wset ? 0x01010101u : 0u;
    *reinterpret_cast<uint4*>(tags + cell_off + base64) = make_uint4(v, v, v, v);
  } else {
    // per lane: 1 row segment settled by its box, 2 row segment near the
    // boundary (tested by k_band), 3 segment crossing a row end or the grid
    // end (cell by cell)
    const bool valid = base64 < g.ncell;
    const int base = valid ? (int)base64 : 0;
    const int nvalid = valid ? (int)min((int64_t)kSeg, g.ncell - base64) : 0;
    int i0 = 0, j = 0, k = 0, settled = -1;
    if (valid) {
      unlinear(g, base, i0, j, k);
      if (nvalid == kSeg && i0 + kSeg - 1 < g.n[0]) {
        // radial culling on the segment's box (face neighbours included)
        double lo[3], hi[3];
        lo[0] = centre_below(g, 0, i0);
        hi[0] = centre_above(g, 0, i0 + kSeg - 1);
        lo[1] = centre_below(g, 1, j);
        hi[1] = centre_above(g, 1, j);
        lo[2] = hi[2] = 0.0;
        if (g.dim == 3) {
          lo[2] = centre_below(g, 2, k);
          hi[2] = centre_above(g, 2, k);
        }
        settled = box_settled(S, g.dim, lo, hi);
        mode = settled >= 0 ? 1 : 2;
      } else {
        // a segment crossing a row end (or cut by the grid end): the tail of
        // its first row and the head of its second, each boxed with its
        // face neighbours, usually settle it too (both sides must agree)
        int p1[3];
        unlinear(g, base + nvalid - 1, p1[0], p1[1], p1[2]);
        const bool one_row = p1[1] == j && p1[2] == k;
        double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
        int seg_a[3] = {i0, j, k}, seg_b[3] = {one_row ? p1[0] : g.n[0] - 1, j, k};
        // (axes unrolled: a runtime index into g would move it to scratch)
#pragma unroll
        for (int a = 0; a < 3; ++a)
          if (a < g.dim) {
            lo[a] = centre_below(g, a, seg_a[a]);
            hi[a] = centre_above(g, a, seg_b[a]);
          }
        // (with rows of 16 cells or more a segment meets at most two rows)
        int sa = g.n[0] >= kSeg ? box_settled(S, g.dim, lo, hi) : -1;
        if (!one_row && sa >= 0) {
          const int c0[3] = {0, p1[1], p1[2]};
#pragma unroll
          for (int a = 0; a < 3; ++a)
            if (a < g.dim) {
              lo[a] = centre_below(g, a, c0[a]);
              hi[a] = centre_above(g, a, p1[a]);
            }
          if (box_settled(S, g.dim, lo, hi) != sa) sa = -1;
        }
        settled = sa;
        mode = settled >= 0 ? 1 : 3;
      }
    }
    if (valid) {
      uint8_t t[kSeg];
      if (mode == 1) {
        for (int b = 0; b < nvalid; ++b) t[b] = (uint8_t)settled;
      } else if (mode == 2) {
        for (int b = 0; b < kSeg; ++b) t[b] = 0;   // written by k_band
      } else {
        for (int b = 0; b < nvalid; ++b) {
          int c = base + b, i, jj, kk;
          unlinear(g, c, i, jj, kk);
          bool sd = cell_solid(g, S, i, jj, kk);
          bool iface = false;
          int q[3] = {i, jj, kk};
#pragma unroll
          for (int a = 0; a < 3; ++a)
            for (int sg = -1; sg <= 1 && a < g.dim && !iface; sg += 2) {
              int qq[3] = {q[0], q[1], q[2]};
              qq[a] += sg;
              if (qq[a] < 0 || qq[a] >= g.n[a]) continue;
              if (cell_solid(g, S, qq[0], qq[1], qq[2]) != sd) {
                iface = true;
                break;
              }
            }
          t[b] = (uint8_t)((sd ? 1 : 0) | (iface ? 0x40 : 0));
          cnt += iface;
        }
      }
      int8_t* dst = tags + cell_off + base;
      if (mode == 2) {
        // k_band writes these 16 cells
      } else if (nvalid == kSeg) {
        uint4 w;
        w.x = t[0] | (t[1] << 8) | (t[2] << 16) | ((uint32_t)t[3] << 24);
        w.y = t[4] | (t[5] << 8) | (t[6] << 16) | ((uint32_t)t[7] << 24);
        w.z = t[8] | (t[9] << 8) | (t[10] << 16) | ((uint32_t)t[11] << 24);
        w.w = t[12] | (t[13] << 8) | (t[14] << 16) | ((uint32_t)t[15] << 24);
        *reinterpret_cast<uint4*>(dst) = w;
      } else {
        for (int b = 0; b < nvalid; ++b) dst[b] = (int8_t)t[b];
      }
    }
  }
  // near-boundary row segments go to the band list (k_band tests them with
  // a whole wave each): positions within the workgroup from an LDS counter,
  // one global atomic per workgroup; every thread reaches the barriers
  {
    const uint64_t bm = __ballot(mode == 2);
    const int lane = (int)(threadIdx.x & 63);
    int wofs = 0;
    if (bm && lane == 0) wofs = atomicAdd(&s_band, __popcll(bm));
    wofs = __shfl(wofs, 0);
    __syncthreads();
    if (threadIdx.x == 0 && s_band > 0) s_base = atomicAdd(nband, s_band);
    __syncthreads();
    if (mode == 2)
      band[s_base + wofs + __popcll(bm & ((1ull << lane) - 1))] =
          (int32_t)(chunk * (kChunk / kSeg) + threadIdx.x);
  }
  if (cnt) atomicAdd(&s_cnt, cnt);
  __syncthreads();
  if (threadIdx.x == 0) chunk_cnt[chunk] = s_cnt;
}

constexpr unsigned kBandWaves = 16384;   // workgroups of k_band (one wave each)

// Near-boundary row segments listed by k_classify, one wave each: the 82
// cells a segment needs (own row with both ends, rows j-1, j+1, k-1, k+1)
// spread over the lanes (t = 0..17 own row from i0 - 1, t = 18 + 16 r + o row
// r at i0 + o), two ballots, then lane 0 forms the segment's tags and
// interface marks.  Cells off the grid read as fluid in the own row; a whole
// neighbour row off the grid stands for the segment itself, since a face
// without a neighbour cannot make an interface.  Every wave leaves its loop
// once the list is exhausted.
__global__ __launch_bounds__(64) void k_band(const Inst* __restrict__ insts, int ninst,
                                             const int64_t* __restrict__ chunk_start,
                                             const int32_t* __restrict__ band,
                                             const int32_t* __restrict__ nband,
                                             int8_t* __restrict__ tags,
                                             int32_t* __restrict__ chunk_cnt) {
  __shared__ ShapeD sh_s;
  static_assert(sizeof(ShapeD) % 8 == 0, "ShapeD copied as doubles");
  const int lane = (int)threadIdx.x;
  const int nb = nband[0];
  int cached = -1;
  for (int b = (int)blockIdx.x; b < nb; b += (int)gridDim.x) {
    const int32_t seg = band[b];
    const int64_t chunk = seg / (kChunk / kSeg);
    const int ii = find_inst(chunk_start, ninst, chunk);
    const Inst& I = insts[ii];
    if (ii != cached) {   // uniform: one wave per workgroup
      __syncthreads();
      const double* src = reinterpret_cast<const double*>(&I.s);
      double* dst = reinterpret_cast<double*>(&sh_s);
      for (int q = lane; q < (int)(sizeof(ShapeD) / 8); q += 64) dst[q] = src[q];
      __syncthreads();
      cached = ii;
    }
    const ShapeD& S = sh_s;
    const GridD g = I.g;
    const int64_t cell_off = I.cell_off;
    const int base = (int)((chunk - I.chunk_off) * kChunk + (int64_t)(seg % (kChunk / kSeg)) * kSeg);
    int i0, j, k;
    unlinear(g, base, i0, j, k);
    bool r[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int t = lane + 64 * q;
      bool v = false;
      if (t < kSeg + 2 + 4 * kSeg) {
        int ci = i0, cj = j, ck = k, rr = -1;
        if (t < kSeg + 2) {
          ci = i0 - 1 + t;
        } else {
          rr = (t - (kSeg + 2)) / kSeg;
          ci = i0 + (t - (kSeg + 2)) % kSeg;
          if (rr == 0) cj = j - 1;
          else if (rr == 1) cj = j + 1;
          else if (rr == 2) ck = k - 1;
          else ck = k + 1;
        }
        const bool in = ci >= 0 && ci < g.n[0] && cj >= 0 && cj < g.n[1] &&
                        (g.dim == 3 ? (ck >= 0 && ck < g.n[2]) : rr < 2);
        if (in) v = cell_solid(g, S, ci, cj, ck);
      }
      r[q] = v;
    }
    const uint64_t m0 = __ballot(r[0]), m1 = __ballot(r[1]);
    if (lane == 0) {
      constexpr uint32_t M = (1u << kSeg) - 1;
      uint32_t row = (uint32_t)(m0 & ((1ull << (kSeg + 2)) - 1));   // i0-1 .. i0+16
      if (i0 == 0) row = (row & ~1u) | ((row >> 1) & 1u);
      if (i0 + kSeg >= g.n[0]) row = (row & ~(1u << (kSeg + 1))) | (((row >> kSeg) & 1u) << (kSeg + 1));
      const uint32_t self = (row >> 1) & M;
      uint32_t diff = (self ^ (row & M)) | (self ^ ((row >> 2) & M));
      uint32_t rjm = (uint32_t)(m0 >> 18) & M, rjp = (uint32_t)(m0 >> 34) & M;
      uint32_t rkm = (uint32_t)((m0 >> 50) | (m1 << 14)) & M, rkp = (uint32_t)(m1 >> 2) & M;
      if (j - 1 < 0) rjm = self;
      if (j + 1 >= g.n[1]) rjp = self;
      diff |= (self ^ rjm) | (self ^ rjp);
      if (g.dim == 3) {
        if (k - 1 < 0) rkm = self;
        if (k + 1 >= g.n[2]) rkp = self;
        diff |= (self ^ rkm) | (self ^ rkp);
      }
      uint32_t w[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        uint32_t v = 0;
#pragma unroll
        for (int bb = 0; bb < 4; ++bb) {
          const int c = 4 * q + bb;
          v |= (((self >> c) & 1u) | (((diff >> c) & 1u) << 6)) << (8 * bb);
        }
        w[q] = v;
      }
      *reinterpret_cast<uint4*>(tags + cell_off + base) = make_uint4(w[0], w[1], w[2], w[3]);
      if (diff) atomicAdd(&chunk_cnt[chunk], __popc(diff));
    }
  }
}


void launch_classify(const Inst* insts, int ninst, const int64_t* chunk_start, int64_t chunks,
                     int8_t* span, int8_t* tags, int32_t* chunk_cnt, int32_t* band,
                     int32_t* nband, hipEvent_t ev_prepass, hipEvent_t ev_store, hipStream_t st) {
  const int64_t nspan = chunks * (kChunk / (64 * kSeg));
  k_spans<<<(unsigned)((nspan + 255) / 256), 256, 0, st>>>(insts, ninst, chunk_start, nspan,
                                                           span, nband);
  if (ev_prepass) (void)hipEventRecord(ev_prepass, st);
  k_classify<<<(unsigned)chunks, 256, 0, st>>>(insts, ninst, chunk_start, span, tags, chunk_cnt,
                                                band, nband);
  if (ev_store) (void)hipEventRecord(ev_store, st);
  k_band<<<kBandWaves, 64, 0, st>>>(insts, ninst, chunk_start, band, nband, tags, chunk_cnt);
}

}  // namespace gcr
