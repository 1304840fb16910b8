// classify.hip -- classification of every cell of a batch (Sec. 3.1): the
// inside test at the cell centre (psi >= 0 solid) and the interface mark
// (a face neighbour of the other class).
//
// A span pass settles whole 1024-cell spans from bounds on the body (a
// radial bound, or a Lipschitz bound on the star radius) and stores them at
// once; the chunks of 4096 cells it leaves are listed, and the store pass
// writes their cells' solid bits, settling 16-cell row segments by the same
// bounds where it can and testing the cells of the others (the band)
// exactly; the interface pass marks the band cells that have a face
// neighbour of the other class.  The list keeps the heavy store pass (its
// FP64 tests hold many registers) off the chunks that only take a constant.
// A re-plan lists the chunks a move can change instead (section 2).
//
// (Band segments are counted for statistics in kBandStripes counters 64
// bytes apart, nband[16 s]; their sum is the count.)
#include <hip/hip_runtime.h>

#include <algorithm>

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
  // D bounds the angle the box subtends, asin(hd / rc): asin(x) / x grows
  // with x, so below x = 1/2 asin(x) <= x asin(1/2) / (1/2) = (pi / 3) x
  const double inv = 1.0 / rc;
  const double D = hd * inv * 1.0472 * (1.0 + 1e-12) + 1e-15;
  double r;
  if (s.kind == kStar2D) {
    double r1;
    star_r(s, xc[0] * inv, xc[1] * inv, r, r1);
  } else {
    const double u[3] = {xc[0] * inv, xc[1] * inv, xc[2] * inv};
    double gr[3];
    sh_r(s, u, r, gr);
  }
  const double spread = s.lip * D;
  if (rc - hd > (r + spread) * (1.0 + 1e-9) + 1e-300) return 0;
  if (rc + hd < (r - spread) * (1.0 - 1e-9)) return 1;
  return -1;
}

// Whether every point of the box [lo, hi] lies on one side of the boundary
// by the radial bounds alone: 0 fluid, 1 solid, -1 undecided.
__device__ __forceinline__ int box_radial(const ShapeD& s, int dim, const double lo[3],
                                          const double hi[3]) {
  double dmin2 = 0.0, dmax2 = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double c = s.cull_c[a];
    const double dl = c < lo[a] ? lo[a] - c : (c > hi[a] ? c - hi[a] : 0.0);
    const double df = fmax(fabs(c - lo[a]), fabs(hi[a] - c));
    dmin2 += dl * dl;
    dmax2 += df * df;
  }
  // on squares: the 1e-9 relative margins dwarf the rounding of either form
  const double rhi = s.rmax * (1.0 + 1e-9), rlo = s.rmin * (1.0 - 1e-9);
  if (dmin2 > rhi * rhi + 1e-300) return 0;
  if (rlo > 0.0 && dmax2 < rlo * rlo) return 1;
  return -1;
}

// The same, then the Lipschitz test for star and SH bodies.
__device__ __forceinline__ int box_settled(const ShapeD& s, int dim, const double lo[3],
                                           const double hi[3]) {
  const int r = box_radial(s, dim, lo, hi);
  if (r >= 0) return r;
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

// nvalid tags of value v (0 or 1) from cell `dst` on
__device__ __forceinline__ void store_const(int8_t* dst, int nvalid, int v) {
  if (nvalid == kSeg) {
    const uint32_t w = v ? 0x01010101u : 0u;
    *reinterpret_cast<uint4*>(dst) = make_uint4(w, w, w, w);
  } else {
    for (int b = 0; b < nvalid; ++b) dst[b] = (int8_t)v;
  }
}

// The span pass, kSpanChunks chunks (4 spans each) per workgroup: one lane
// per span of 64 * kSeg cells tests whether the box of the span's cells and
// their face neighbours, in index space, lies wholly on one side of the
// boundary (0 fluid, 1 solid, -1 undecided); then (tags set) every wave
// stores whole settled spans, 1 KB each, with 16-byte stores.  need[c] = 1
// for a chunk with a span left (undecided, or cut by the grid end), the
// chunks the store pass visits; every chunk's interface count and band mask
// start at zero.
constexpr int kSpanChunks = 8;
__global__ __launch_bounds__(256) void k_spans(const Inst* __restrict__ insts, int ninst,
                                               const int64_t* __restrict__ chunk_start,
                                               int64_t chunks, int8_t* __restrict__ span,
                                               int32_t* __restrict__ chunk_inst,
                                               int32_t* __restrict__ need,
                                               int32_t* __restrict__ chunk_cnt,
                                               uint64_t* __restrict__ bandmask,
                                               int8_t* __restrict__ tags,
                                               int32_t* __restrict__ nband) {
  constexpr int kSpan = 64 * kSeg, kPer = kChunk / kSpan, kSpans = kSpanChunks * kPer;
  static_assert(kSpans <= 64, "one wave tests the workgroup's spans");
  __shared__ int8_t s_flag[kSpans];
  __shared__ int64_t s_base[kSpans];   // tag offset of a whole settled span, else -1
  const int tid = (int)threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * kSpanChunks;
  if (blockIdx.x == 0 && tid < kBandStripes) nband[tid * 16] = 0;   // k_band_iface counts from zero
  if (tid < kSpans) {
    const int64_t chunk = c0 + tid / kPer;
    int8_t r = -1;
    int64_t whole = -1;
    if (chunk < chunks) {
      const int ii = find_inst(chunk_start, ninst, chunk);
      // the chunk's instance, for the passes after this one (one load instead
      // of a search at the start of each of their workgroups)
      if (tid % kPer == 0) {
        chunk_inst[chunk] = ii;
        chunk_cnt[chunk] = 0;
      }
      bandmask[chunk * 4 + tid % kPer] = 0ull;
      const Inst& I = insts[ii];
      const GridD& g = I.g;
      const int64_t base = (chunk - I.chunk_off) * kChunk + (tid % kPer) * kSpan;
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
        if (r >= 0 && base + kSpan <= g.ncell) whole = I.cell_off + base;
      }
      span[chunk * kPer + tid % kPer] = r;
    }
    s_flag[tid] = r;
    s_base[tid] = whole;
  }
  __syncthreads();
  if (tid < kSpanChunks && c0 + tid < chunks) {
    bool nd = false;
    for (int q = 0; q < kPer; ++q) nd = nd || s_base[tid * kPer + q] < 0;
    need[c0 + tid] = nd ? 1 : 0;
  }
  if (!tags) return;
  const int wv = tid >> 6, lane = tid & 63;
  for (int q = wv; q < kSpans; q += 4) {
    const int64_t b = s_base[q];
    if (b >= 0) store_const(tags + b + lane * kSeg, kSeg, s_flag[q]);
  }
}

// Whether the nvalid cells of the row segment starting at cell `base` and
// their face neighbours lie on one side of the boundary (0 fluid, 1 solid,
// -1 undecided); full: with the Lipschitz test, else radial bounds only.  A
// segment within one row is one box; one that crosses a row end (or is cut
// by the grid end) is the tail of its first row and the head of its second,
// each boxed with its face neighbours, both of which must agree.
__device__ __forceinline__ int seg_settled(const GridD& g, const ShapeD& S, int base, int nvalid,
                                           bool full) {
  int i0, j, k;
  unlinear(g, base, i0, j, k);
  if (nvalid == kSeg && i0 + kSeg - 1 < g.n[0]) {
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
    return full ? box_settled(S, g.dim, lo, hi) : box_radial(S, g.dim, lo, hi);
  }
  // (with rows of 16 cells or more a segment meets at most two rows)
  if (g.n[0] < kSeg) return -1;
  int p1[3];
  unlinear(g, base + nvalid - 1, p1[0], p1[1], p1[2]);
  const bool one_row = p1[1] == j && p1[2] == k;
  double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
  const int seg_a[3] = {i0, j, k}, seg_b[3] = {one_row ? p1[0] : g.n[0] - 1, j, k};
  // (axes unrolled: a runtime index into g would move it to scratch)
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a < g.dim) {
      lo[a] = centre_below(g, a, seg_a[a]);
      hi[a] = centre_above(g, a, seg_b[a]);
    }
  int sa = full ? box_settled(S, g.dim, lo, hi) : box_radial(S, g.dim, lo, hi);
  if (!one_row && sa >= 0) {
    const int c0[3] = {0, p1[1], p1[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
      if (a < g.dim) {
        lo[a] = centre_below(g, a, c0[a]);
        hi[a] = centre_above(g, a, p1[a]);
      }
    const int sb = full ? box_settled(S, g.dim, lo, hi) : box_radial(S, g.dim, lo, hi);
    if (sb != sa) sa = -1;
  }
  return sa;
}

// The store pass, one workgroup per chunk of kChunk cells, a 16-cell row
// segment per thread.  A wave whose span the span pass settled only stores
// it (nothing, when the span pass stored it already).  Otherwise the work
// is done densely in three rounds, so that no wave runs an expensive test
// for a few of its lanes: each lane's segment first meets
// the radial bounds (cheap); the segments they leave undecided are listed
// in LDS and, for star and SH bodies, their Lipschitz tests run one segment
// per thread; the segments still undecided form the chunk's band, whose
// cells are tested exactly one cell per thread.  Band cells get their solid
// bit here and their interface mark (a face neighbour of the other class)
// from k_band_iface; settled segments have none, since their boxes include
// the face neighbours.  The chunk's band is recorded as a 256-bit mask.
__device__ __forceinline__ void classify_chunk(int64_t chunk, int ii, const Inst* __restrict__ insts,
                                               const int8_t* __restrict__ span,
                                               int8_t* __restrict__ tags,
                                               int32_t* __restrict__ chunk_cnt,
                                               uint64_t* __restrict__ bandmask,
                                               bool spans_stored) {
  const Inst& I = insts[ii];
  const GridD g = I.g;
  const int64_t chunk_off = I.chunk_off, cell_off = I.cell_off;
  __shared__ ShapeD sh_s;
  __shared__ int s_na, s_nb;
  __shared__ uint8_t s_la[256], s_lb[256];
  __shared__ unsigned long long s_mask[4];
  static_assert(sizeof(ShapeD) % 8 == 0, "ShapeD copied as doubles");
  constexpr int kSpans = kChunk / (64 * kSeg);
  const int tid = (int)threadIdx.x;
  const int64_t cbase = (chunk - chunk_off) * kChunk;
  // a workgroup whose spans are all whole and settled only stores: one round
  // of flag loads, no barrier (most workgroups of a large grid)
  bool need_shape = false;
  int8_t fl[kSpans];
  for (int q = 0; q < kSpans; ++q) {
    fl[q] = span[chunk * kSpans + q];
    need_shape |= cbase + (int64_t)(q + 1) * 64 * kSeg > g.ncell || fl[q] < 0;
  }
  if (!need_shape) {
    store_const(tags + cell_off + cbase + (int64_t)tid * kSeg, kSeg, fl[tid >> 6]);
    if (tid < 4) bandmask[chunk * 4 + tid] = 0ull;
    if (tid == 0) chunk_cnt[chunk] = 0;
    return;
  }
  {
    const double* src = reinterpret_cast<const double*>(&I.s);
    double* dst = reinterpret_cast<double*>(&sh_s);
    for (int q = tid; q < (int)(sizeof(ShapeD) / 8); q += 256) dst[q] = src[q];
  }
  if (tid == 0) {
    s_na = 0;
    s_nb = 0;
  }
  if (tid < 4) s_mask[tid] = 0ull;
  __syncthreads();
  const ShapeD& S = sh_s;
  const bool lip = S.kind == kStar2D || S.kind == kShStar;
  const int64_t base64 = cbase + (int64_t)tid * kSeg;
  const int64_t wbase = base64 - (int64_t)(tid & 63) * kSeg;
  const int wset = wbase + 64 * kSeg <= g.ncell ? (int)fl[tid >> 6] : -1;
  const bool valid = base64 < g.ncell;
  const int nvalid = valid ? (int)min((int64_t)kSeg, g.ncell - base64) : 0;
  // round 1: the wave's span settled (stored here unless the span pass
  // stored it), else this lane's radial bounds
  if (wset >= 0) {
    if (!spans_stored) store_const(tags + cell_off + base64, kSeg, wset);
  } else if (valid) {
    const int r = seg_settled(g, S, (int)base64, nvalid, false);
    if (r >= 0) store_const(tags + cell_off + base64, nvalid, r);
    else if (lip) s_la[atomicAdd(&s_na, 1)] = (uint8_t)tid;
    else s_lb[atomicAdd(&s_nb, 1)] = (uint8_t)tid;
  }
  __syncthreads();
  // round 2: the Lipschitz tests of the undecided segments, one per thread
  for (int t = tid; t < s_na; t += 256) {
    const int l = s_la[t];
    const int64_t b = cbase + (int64_t)l * kSeg;
    const int nv = (int)min((int64_t)kSeg, g.ncell - b);
    const int r = seg_settled(g, S, (int)b, nv, true);
    if (r >= 0) store_const(tags + cell_off + b, nv, r);
    else s_lb[atomicAdd(&s_nb, 1)] = (uint8_t)l;
  }
  __syncthreads();
  // round 3: every cell of the band segments, one per thread (solid bit)
  const int nb = s_nb;
  for (int t = tid; t < nb * kSeg; t += 256) {
    const int l = s_lb[t / kSeg], o = t % kSeg;
    const int64_t c = cbase + (int64_t)l * kSeg + o;
    if (o == 0) atomicOr(&s_mask[l >> 6], 1ull << (l & 63));
    if (c >= g.ncell) continue;
    int i, j, k;
    unlinear(g, (int)c, i, j, k);
    tags[cell_off + c] = cell_solid(g, S, i, j, k) ? 1 : 0;
  }
  __syncthreads();
  if (tid < 4) bandmask[chunk * 4 + tid] = s_mask[tid];
  if (tid == 0) chunk_cnt[chunk] = 0;
}

// Mode 0: one workgroup per chunk.  Mode 1: one workgroup per entry of
// list[first, *nlist), up to the grid's size.  Mode 2: workgroups striding
// over the entries of list[first, *nlist) (first: the grid of a mode-1
// launch before it).  The loop of mode 2 costs registers, and so occupancy,
// that the one-chunk forms do without, so a list is taken by a mode-1 grid
// and a small mode-2 launch after it for whatever that grid left.
template <int Mode>
__global__ __launch_bounds__(256) void k_classify(const Inst* __restrict__ insts,
                                                  const int32_t* __restrict__ chunk_inst,
                                                  const int8_t* __restrict__ span,
                                                  int8_t* __restrict__ tags,
                                                  int32_t* __restrict__ chunk_cnt,
                                                  uint64_t* __restrict__ bandmask,
                                                  const int32_t* __restrict__ list,
                                                  const int32_t* __restrict__ nlist,
                                                  bool spans_stored, int first) {
  if (Mode == 0) {
    classify_chunk(blockIdx.x, chunk_inst[blockIdx.x], insts, span, tags, chunk_cnt, bandmask,
                   false);
    return;
  }
  const int nit = nlist[0];
  if (Mode == 1) {
    const int it = first + (int)blockIdx.x;
    if (it < nit) {
      const int64_t chunk = list[it];
      classify_chunk(chunk, chunk_inst[chunk], insts, span, tags, chunk_cnt, bandmask,
                     spans_stored);
    }
    return;
  }
  for (int it = first + (int)blockIdx.x; it < nit; it += gridDim.x) {
    const int64_t chunk = list[it];
    classify_chunk(chunk, chunk_inst[chunk], insts, span, tags, chunk_cnt, bandmask,
                   spans_stored);
    __syncthreads();   // the LDS lists are reused by the next chunk
  }
}

// Interface marks of the band cells, one workgroup per chunk (chunks
// without band segments leave at once): a band cell is marked when a face
// neighbour in the grid has the other solid bit; the chunk's count goes to
// chunk_cnt, and its band segments to one of the striped counters.
__device__ __forceinline__ void band_iface_chunk(int64_t chunk, const Inst* __restrict__ insts,
                                                 const int32_t* __restrict__ chunk_inst,
                                                 const uint64_t* __restrict__ bandmask,
                                                 int8_t* __restrict__ tags,
                                                 int32_t* __restrict__ chunk_cnt,
                                                 int32_t* __restrict__ nband) {
  const int ii = chunk_inst[chunk];   // loaded beside the masks
  unsigned long long m[4];
  int tot = 0;
  for (int w = 0; w < 4; ++w) {
    m[w] = bandmask[chunk * 4 + w];
    tot += __popcll(m[w]);
  }
  if (tot == 0) return;
  const int tid = (int)threadIdx.x;
  __shared__ uint8_t s_l[256];
  __shared__ int s_cnt;
  {
    // rank of this thread's segment among the chunk's band segments
    const int w = tid >> 6, b = tid & 63;
    if ((m[w] >> b) & 1ull) {
      int pos = __popcll(m[w] & ((1ull << b) - 1ull));
      for (int q = 0; q < w; ++q) pos += __popcll(m[q]);
      s_l[pos] = (uint8_t)tid;
    }
  }
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  const Inst& I = insts[ii];
  const GridD g = I.g;
  const int64_t cell_off = I.cell_off;
  const int64_t cbase = (chunk - I.chunk_off) * kChunk;
  const int8_t* T = tags + cell_off;   // written below too (own cell only)
  int cnt = 0;
  for (int t = tid; t < tot * kSeg; t += 256) {
    const int64_t c = cbase + (int64_t)s_l[t / kSeg] * kSeg + t % kSeg;
    if (c >= g.ncell) continue;
    int i, j, k;
    unlinear(g, (int)c, i, j, k);
    const int self = T[c] & 1;
    bool iface = false;
    if (i > 0) iface |= (T[c - 1] & 1) != self;
    if (i + 1 < g.n[0]) iface |= (T[c + 1] & 1) != self;
    const int64_t sy = g.n[0];
    if (j > 0) iface |= (T[c - sy] & 1) != self;
    if (j + 1 < g.n[1]) iface |= (T[c + sy] & 1) != self;
    if (g.dim == 3) {
      const int64_t sz = sy * g.n[1];
      if (k > 0) iface |= (T[c - sz] & 1) != self;
      if (k + 1 < g.n[2]) iface |= (T[c + sz] & 1) != self;
    }
    if (iface) {
      tags[cell_off + c] = (int8_t)(self | 0x40);
      ++cnt;
    }
  }
  if (cnt) atomicAdd(&s_cnt, cnt);
  __syncthreads();
  if (tid == 0) {
    chunk_cnt[chunk] += s_cnt;
    atomicAdd(&nband[(chunk % kBandStripes) * 16], tot);
  }
}

__global__ __launch_bounds__(256) void k_band_iface(const Inst* __restrict__ insts,
                                                    const int32_t* __restrict__ chunk_inst,
                                                    const uint64_t* __restrict__ bandmask,
                                                    int8_t* __restrict__ tags,
                                                    int32_t* __restrict__ chunk_cnt,
                                                    int32_t* __restrict__ nband,
                                                    const int32_t* __restrict__ list,
                                                    const int32_t* __restrict__ nlist) {
  if (!list) {
    band_iface_chunk(blockIdx.x, insts, chunk_inst, bandmask, tags, chunk_cnt, nband);
    return;
  }
  const int nit = nlist[0];
  for (int it = blockIdx.x; it < nit; it += gridDim.x) {
    band_iface_chunk(list[it], insts, chunk_inst, bandmask, tags, chunk_cnt, nband);
    __syncthreads();   // s_l and s_cnt are reused by the next chunk
  }
}

// --------------------------------------------------------------------------
// 2. incremental re-plan of a moved body
// --------------------------------------------------------------------------

// A chunk keeps its tags across a move when each of its spans was settled
// before and is settled to the same class after: then every cell of it and
// every face neighbour lies on that side of both boundaries, so the cell's
// class is unchanged and it is no interface cell either time.  Those tags
// are its settled value unless a ghost of the previous plan lies there (a
// second-layer ghost can sit in a settled solid span), which
// k_dirty_ghosts catches.  One thread per chunk: dirty[c] = 1 for a chunk
// to classify again.
__global__ __launch_bounds__(256) void k_dirty(const int8_t* __restrict__ span0,
                                               const int8_t* __restrict__ span1, int64_t chunks,
                                               int32_t* __restrict__ dirty) {
  constexpr int kPer = kChunk / (64 * kSeg);
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= chunks) return;
  bool d = false;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int8_t a = span0[c * kPer + q], b = span1[c * kPer + q];
    d = d || b < 0 || a != b;
  }
  dirty[c] = d ? 1 : 0;
}

// the chunks of the previous plan's ghosts (a single instance from chunk 0)
__global__ __launch_bounds__(256) void k_dirty_ghosts(const int32_t* __restrict__ cell,
                                                      int64_t ng, int32_t* __restrict__ dirty) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ng) dirty[cell[e] / kChunk] = 1;   // every writer stores 1
}


void launch_classify(const Inst* insts, int ninst, const int64_t* chunk_start, int64_t chunks,
                     int8_t* span, int32_t* chunk_inst, int8_t* tags, int32_t* chunk_cnt,
                     int32_t* band, int32_t* nband, hipEvent_t ev_prepass, hipEvent_t ev_store,
                     hipStream_t st, const ClassifyWork& W, const ClassifyUpdate* U) {
  uint64_t* mask = reinterpret_cast<uint64_t*>(band);   // [chunks][4]
  // Where chunks are rows of a 2D grid, about every other one meets the
  // body and the store pass takes them all (the settled ones with one
  // store each); elsewhere the span pass stores settled spans at once and
  // the store pass takes the chunks left.  A re-plan keeps the previous
  // plan's tags outside the chunks a move can change.
  const bool every = !U && W.every_chunk;
  k_spans<<<(unsigned)((chunks + kSpanChunks - 1) / kSpanChunks), 256, 0, st>>>(
      insts, ninst, chunk_start, chunks, span, chunk_inst, W.flag, chunk_cnt, mask,
      U || every ? nullptr : tags, nband);
  if (ev_prepass) (void)hipEventRecord(ev_prepass, st);
  if (every) {
    k_classify<0><<<(unsigned)chunks, 256, 0, st>>>(insts, chunk_inst, span, tags, chunk_cnt, mask,
                                                    nullptr, nullptr, false, 0);
    if (ev_store) (void)hipEventRecord(ev_store, st);
    k_band_iface<<<(unsigned)chunks, 256, 0, st>>>(insts, chunk_inst, mask, tags, chunk_cnt,
                                                   nband, nullptr, nullptr);
    return;
  }
  if (U) {
    // a re-plan: the chunks the move can change, instead of those left
    k_dirty<<<(unsigned)((chunks + 255) / 256), 256, 0, st>>>(U->span_prev, span, chunks,
                                                              W.flag);
    if (U->ng_prev > 0)
      k_dirty_ghosts<<<(unsigned)((U->ng_prev + 255) / 256), 256, 0, st>>>(
          U->ghost_prev, U->ng_prev, W.flag);
  }
  // the flagged chunks, listed in ascending order, are classified one
  // workgroup per entry, and entries beyond that grid (a list longer than
  // kListGrid) by a striding launch; the list's length stays on the device
  launch_scan(W.flag, chunks, W.scan_excl, W.list, W.nlist, W.scan_tmp, st);
  const unsigned G = (unsigned)std::min<int64_t>(chunks, kListGrid);
  // (a full build's span pass stored the whole settled spans already)
  k_classify<1><<<G, 256, 0, st>>>(insts, chunk_inst, span, tags, chunk_cnt, mask, W.list,
                                   W.nlist, U == nullptr, 0);
  if ((int64_t)G < chunks)   // entries beyond the first grid, if any
    k_classify<2><<<256, 256, 0, st>>>(insts, chunk_inst, span, tags, chunk_cnt, mask, W.list,
                                       W.nlist, U == nullptr, (int)G);
  if (ev_store) (void)hipEventRecord(ev_store, st);
  k_band_iface<<<G, 256, 0, st>>>(insts, chunk_inst, mask, tags, chunk_cnt, nband, W.list,
                                  W.nlist);
}

}  // namespace gcr
