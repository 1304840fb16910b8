// plan.hip -- building ghost-cell plans on the GPU.
//
// Pipeline (one launch per stage, all instances of a batch together):
//   classify      every cell: inside test at its centre (Sec. 3.1), and
//                 whether a face neighbour has the other class; far-field
//                 segments are settled by a radial bound and written as
//                 16-byte constant stores
//   scan/compact  interface cells in linear-index order
//   geometry      closest point, analytic normal, psi; ghost tags for CGC,
//                 CGC_ES and HGC (Eq. HGC_criterion with Eq. delta_n)
//   ghosts        order-preserving compaction of the ghost cells
//   deps          stencil code (e = sgn n, multipliers r), validation, and
//                 ghost-to-ghost dependencies (Sec. 3.2)
//   levels        Kahn layering per instance, emitting the canonical order
//                 (level, linear index) as it goes; a stall means a cycle:
//                 its strongly connected groups become coupled units
//   finalize      canonical structure-of-arrays for the apply kernels
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>

#include "gcr_impl.hpp"

namespace gcr {


// --------------------------------------------------------------------------
// closest point and normal
// --------------------------------------------------------------------------

// The contour point C(s) = (s^2, +-y_t(s^2)) (s >= 0 upper, s < 0 lower
// surface), its derivative D and second derivative E in s.
__device__ __forceinline__ void naca_point(double t, double s, double C[2], double D[2],
                                           double E[2]) {
  double s2 = s * s, sg = s < 0.0 ? -1.0 : 1.0;
  double poly = 0.1260 * s2 + 0.3516 * s2 * s2 - 0.2843 * s2 * s2 * s2 + 0.1036 * s2 * s2 * s2 * s2;
  double dpoly = s * (2.0 * 0.1260 + s2 * (4.0 * 0.3516 + s2 * (-6.0 * 0.2843 + s2 * 8.0 * 0.1036)));
  double d2poly = 2.0 * 0.1260 + s2 * (12.0 * 0.3516 + s2 * (-30.0 * 0.2843 + s2 * 56.0 * 0.1036));
  C[0] = s2;
  C[1] = 5.0 * t * (0.2969 * s - sg * poly);
  D[0] = 2.0 * s;
  D[1] = 5.0 * t * (0.2969 - sg * dpoly);
  E[0] = 2.0;
  E[1] = -5.0 * t * sg * d2poly;
}

__device__ bool project(const ShapeD& s, int dim, const double x[3], bool solid, double n[3],
                        double& psi) {
  double v[3] = {x[0] - s.c[0], x[1] - s.c[1], dim == 3 ? x[2] - s.c[2] : 0.0};
  n[2] = 0.0;
  if (s.kind == kSphere) {
    double rho2 = v[0] * v[0] + v[1] * v[1];
    if (dim == 3) rho2 += v[2] * v[2];
    double rho = sqrt(rho2);
    if (rho == 0.0) return false;
    for (int i = 0; i < dim; ++i) n[i] = v[i] / rho;
    psi = s.r0 - rho;
    return true;
  }
  double S[3] = {0.0, 0.0, 0.0};
  bool ok = false;
  if (s.kind == kStar2D) {
    // Gauss-Newton on a fixed chart of directions u(a) ~ w0 + a t0
    double rho = sqrt(v[0] * v[0] + v[1] * v[1]);
    if (rho == 0.0) return false;
    double w0[2] = {v[0] / rho, v[1] / rho}, t0[2] = {-w0[1], w0[0]};
    double a = 0.0, last = 1.0;
    int good = 0;
    for (int it = 0; it < 80 && good < 2; ++it) {
      double q0 = w0[0] + a * t0[0], q1 = w0[1] + a * t0[1];
      double nv = sqrt(q0 * q0 + q1 * q1);
      double u0 = q0 / nv, u1 = q1 / nv, r, r1;
      star_r(s, u0, u1, r, r1);
      double fac = (-u1 * t0[0] + u0 * t0[1]) / nv;
      double J0 = fac * (r1 * u0 - r * u1), J1 = fac * (r1 * u1 + r * u0);
      double R0 = s.c[0] + r * u0 - x[0], R1 = s.c[1] + r * u1 - x[1];
      double da = -(J0 * R0 + J1 * R1) / (J0 * J0 + J1 * J1);
      a += da;
      last = fabs(da);
      good = last < 1e-15 ? good + 1 : 0;
    }
    ok = good >= 2 || last < 1e-13;
    double q0 = w0[0] + a * t0[0], q1 = w0[1] + a * t0[1];
    double nv = sqrt(q0 * q0 + q1 * q1);
    double u0 = q0 / nv, u1 = q1 / nv, r, r1;
    if (!ok) {
      // Gauss-Newton leaves out the curvature term, so it crawls (or
      // wanders) where the point is nearly as deep as the boundary's radius
      // of curvature: a second-layer candidate inside a tight bend.  Newton
      // on the polar angle from where it stopped, with that term (f = |X -
      // x|^2 / 2, f' = R.X', f'' = X'.X' + R.X''), taking the Gauss-Newton
      // step wherever f'' is not positive.
      double th = atan2(u1, u0);
      good = 0;
      last = 1.0;
      for (int it = 0; it < 60 && good < 2; ++it) {
        double sn, cs, r2;
        sincos(th, &sn, &cs);
        star_r2(s, cs, sn, r, r1, r2);
        const double D1x = r1 * cs - r * sn, D1y = r1 * sn + r * cs;
        const double D2x = (r2 - r) * cs - 2.0 * r1 * sn, D2y = (r2 - r) * sn + 2.0 * r1 * cs;
        const double Rx = s.c[0] + r * cs - x[0], Ry = s.c[1] + r * sn - x[1];
        const double g1 = Rx * D1x + Ry * D1y;
        double g2 = D1x * D1x + D1y * D1y + Rx * D2x + Ry * D2y;
        if (!(g2 > 0.0)) g2 = D1x * D1x + D1y * D1y;
        const double dth = -g1 / g2;
        th += dth;
        last = fabs(dth);
        good = last < 1e-15 ? good + 1 : 0;
      }
      ok = good >= 2 || last < 1e-13;
      sincos(th, &u1, &u0);
    }
    star_r(s, u0, u1, r, r1);
    S[0] = s.c[0] + r * u0;
    S[1] = s.c[1] + r * u1;
    // tangent dX/dtheta = r' u + r u_perp; outward normal = tangent turned clockwise
    double T0 = r1 * u0 - r * u1, T1 = r1 * u1 + r * u0;
    double tn = sqrt(T0 * T0 + T1 * T1);
    n[0] = T1 / tn;
    n[1] = -T0 / tn;
  } else if (s.kind == kShStar) {
    double rho = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (rho == 0.0) return false;
    double w0[3] = {v[0] / rho, v[1] / rho, v[2] / rho};
    int ax = 0;
    if (fabs(w0[1]) < fabs(w0[ax])) ax = 1;
    if (fabs(w0[2]) < fabs(w0[ax])) ax = 2;
    double t1[3] = {0.0, 0.0, 0.0};
    t1[ax] = 1.0;
    double dd = w0[ax];
    for (int i = 0; i < 3; ++i) t1[i] -= dd * w0[i];
    double tl = sqrt(t1[0] * t1[0] + t1[1] * t1[1] + t1[2] * t1[2]);
    for (int i = 0; i < 3; ++i) t1[i] /= tl;
    double t2[3] = {w0[1] * t1[2] - w0[2] * t1[1], w0[2] * t1[0] - w0[0] * t1[2],
                    w0[0] * t1[1] - w0[1] * t1[0]};
    double p1 = 0.0, p2 = 0.0, last = 1.0;
    int good = 0;
    for (int it = 0; it < 80 && good < 2; ++it) {
      double q[3], u[3], r, g[3];
      for (int i = 0; i < 3; ++i) q[i] = w0[i] + p1 * t1[i] + p2 * t2[i];
      double nv = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
      for (int i = 0; i < 3; ++i) u[i] = q[i] / nv;
      sh_r(s, u, r, g);
      double ut1 = u[0] * t1[0] + u[1] * t1[1] + u[2] * t1[2];
      double ut2 = u[0] * t2[0] + u[1] * t2[1] + u[2] * t2[2];
      double J1[3], J2[3], R[3];
      double du1[3], du2[3];
      for (int i = 0; i < 3; ++i) {
        du1[i] = (t1[i] - ut1 * u[i]) / nv;
        du2[i] = (t2[i] - ut2 * u[i]) / nv;
      }
      double dr1 = g[0] * du1[0] + g[1] * du1[1] + g[2] * du1[2];
      double dr2 = g[0] * du2[0] + g[1] * du2[1] + g[2] * du2[2];
      for (int i = 0; i < 3; ++i) {
        J1[i] = dr1 * u[i] + r * du1[i];
        J2[i] = dr2 * u[i] + r * du2[i];
        R[i] = s.c[i] + r * u[i] - x[i];
      }
      double a11 = 0, a12 = 0, a22 = 0, b1 = 0, b2 = 0;
      for (int i = 0; i < 3; ++i) {
        a11 += J1[i] * J1[i];
        a12 += J1[i] * J2[i];
        a22 += J2[i] * J2[i];
        b1 -= J1[i] * R[i];
        b2 -= J2[i] * R[i];
      }
      double det = a11 * a22 - a12 * a12;
      double d1 = (b1 * a22 - b2 * a12) / det, d2 = (a11 * b2 - a12 * b1) / det;
      p1 += d1;
      p2 += d2;
      last = fabs(d1) + fabs(d2);
      good = last < 1e-15 ? good + 1 : 0;
    }
    ok = good >= 2 || last < 1e-13;
    double q[3], u[3], r, g[3];
    for (int i = 0; i < 3; ++i) q[i] = w0[i] + p1 * t1[i] + p2 * t2[i];
    double nv = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    for (int i = 0; i < 3; ++i) u[i] = q[i] / nv;
    sh_r(s, u, r, g);
    for (int i = 0; i < 3; ++i) {
      S[i] = s.c[i] + r * u[i];
      n[i] = u[i] - g[i] / r;   // gradient of |y - c| - r(direction)
    }
    double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int i = 0; i < 3; ++i) n[i] /= nl;
  } else if (s.kind == kAirfoil) {
    double dx = (x[0] - s.c[0]) / s.chord, dy = (x[1] - s.c[1]) / s.chord;
    double b0 = s.ca * dx - s.sa * dy, b1 = s.sa * dx + s.ca * dy;
    double xc = b0 < 0.0 ? 0.0 : (b0 > 1.0 ? 1.0 : b0);
    double sp = sqrt(xc);
    double best = 1e300, bs = 0.0;
    ok = true;
    for (int br = 0; br < 2; ++br) {
      double lo = br == 0 ? 0.0 : -1.0, hi = br == 0 ? 1.0 : 0.0;
      double sv = br == 0 ? sp : -sp;
      if (sv == 0.0) sv = br == 0 ? 1e-3 : -1e-3;
      double last = 1.0;
      // Newton on the squared distance along the contour parameter, clamped
      // to the branch; the Gauss-Newton step where the curvature term makes
      // the second derivative non-positive
      for (int it = 0; it < 200 && last > 1e-15; ++it) {
        double C[2], D[2], E[2];
        naca_point(s.thick, sv, C, D, E);
        const double r0 = C[0] - b0, r1 = C[1] - b1;
        const double dd = D[0] * D[0] + D[1] * D[1];
        double h = dd + r0 * E[0] + r1 * E[1];
        if (!(h > 0.0)) h = dd;
        double ns = sv - (r0 * D[0] + r1 * D[1]) / h;
        ns = ns < lo ? lo : (ns > hi ? hi : ns);
        last = fabs(ns - sv);
        sv = ns;
      }
      if (last > 1e-12) ok = false;
      double C[2], D[2], E[2];
      naca_point(s.thick, sv, C, D, E);
      double d2 = (C[0] - b0) * (C[0] - b0) + (C[1] - b1) * (C[1] - b1);
      if (d2 < best) {
        best = d2;
        bs = sv;
      }
    }
    double C[2], D[2], E[2], nb[2];
    naca_point(s.thick, bs, C, D, E);
    if (fabs(bs) >= 1.0) {
      // trailing-edge corner: the normal is the direction from the corner
      double e0 = b0 - C[0], e1 = b1 - C[1];
      double el = sqrt(e0 * e0 + e1 * e1);
      nb[0] = (solid ? -e0 : e0) / el;
      nb[1] = (solid ? -e1 : e1) / el;
    } else {
      // contour is clockwise in s: outward normal = tangent turned counter-clockwise
      double dl = sqrt(D[0] * D[0] + D[1] * D[1]);
      nb[0] = -D[1] / dl;
      nb[1] = D[0] / dl;
    }
    n[0] = s.ca * nb[0] + s.sa * nb[1];
    n[1] = -s.sa * nb[0] + s.ca * nb[1];
    S[0] = s.c[0] + s.chord * (s.ca * C[0] + s.sa * C[1]);
    S[1] = s.c[1] + s.chord * (-s.sa * C[0] + s.ca * C[1]);
  } else {
    return false;
  }
  double d2 = 0.0;
  for (int i = 0; i < dim; ++i) d2 += (x[i] - S[i]) * (x[i] - S[i]);
  psi = solid ? sqrt(d2) : -sqrt(d2);
  return ok;
}

// --------------------------------------------------------------------------
// 2. scans and compactions
// --------------------------------------------------------------------------

// excl[i] = sum cnt[0..i), excl[n] = total.  If list is given, the indices
// i with cnt[i] > 0 are written to it in ascending order and their number
// to nlist[0]: each count carries a flag in bits 40 and up, so one scan
// yields both (counts stay below 2^40).  Tiles of 8 values per thread of a
// 1024-thread workgroup.
constexpr int kScanT = 8, kScanTile = 1024 * kScanT;
constexpr int64_t kScanHi = int64_t(1) << 40;

__device__ __forceinline__ void scan_load(const int32_t* __restrict__ cnt, int64_t n, int64_t b,
                                          int v[kScanT]) {
  const bool vec = (reinterpret_cast<uintptr_t>(cnt) & 15) == 0;
  if (vec && b + kScanT <= n) {
    const int4 a = *reinterpret_cast<const int4*>(cnt + b);
    const int4 c = *reinterpret_cast<const int4*>(cnt + b + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
  } else {
#pragma unroll
    for (int q = 0; q < kScanT; ++q) v[q] = b + q < n ? cnt[b + q] : 0;
  }
}

// One tile from t0 with the packed prefix `carry`; returns the tile's
// packed total.  Every thread of the workgroup calls it.
__device__ __forceinline__ int64_t scan_tile(const int32_t* __restrict__ cnt, int64_t n,
                                             int64_t t0, int64_t carry,
                                             int64_t* __restrict__ excl,
                                             int32_t* __restrict__ list, int64_t* sh) {
  const int64_t b = t0 + (int64_t)threadIdx.x * kScanT;
  int v[kScanT];
  scan_load(cnt, n, b, v);
  int64_t sum = 0;
#pragma unroll
  for (int q = 0; q < kScanT; ++q) sum += v[q] + (v[q] > 0 ? kScanHi : 0);
  int64_t tot;
  int64_t run = carry + block_excl_scan<1024>(sum, &tot, sh);
#pragma unroll
  for (int q = 0; q < kScanT; ++q) {
    if (b + q < n) {
      excl[b + q] = run & (kScanHi - 1);
      if (list && v[q] > 0) list[run >> 40] = (int32_t)(b + q);
    }
    run += v[q] + (v[q] > 0 ? kScanHi : 0);
  }
  return tot;
}

// the whole scan by one workgroup (short inputs)
__global__ __launch_bounds__(1024) void k_scan(const int32_t* __restrict__ cnt, int64_t n,
                                               int64_t* __restrict__ excl,
                                               int32_t* __restrict__ list,
                                               int32_t* __restrict__ nlist) {
  __shared__ int64_t sh[17];
  int64_t carry = 0;
  for (int64_t t0 = 0; t0 < n; t0 += kScanTile) carry += scan_tile(cnt, n, t0, carry, excl, list, sh);
  if (threadIdx.x == 0) {
    excl[n] = carry & (kScanHi - 1);
    if (nlist) nlist[0] = (int32_t)(carry >> 40);
  }
}

// long inputs: packed total of each tile, one workgroup per tile ...
__global__ __launch_bounds__(1024) void k_scan_reduce(const int32_t* __restrict__ cnt, int64_t n,
                                                      int64_t* __restrict__ tsum) {
  __shared__ int64_t sh[17];
  int v[kScanT];
  scan_load(cnt, n, (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanT, v);
  int64_t sum = 0;
#pragma unroll
  for (int q = 0; q < kScanT; ++q) sum += v[q] + (v[q] > 0 ? kScanHi : 0);
  int64_t tot;
  (void)block_excl_scan<1024>(sum, &tot, sh);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

// ... their exclusive scan in place, the total and the list length ...
__global__ __launch_bounds__(1024) void k_scan_top(int64_t* __restrict__ tsum, int64_t ntiles,
                                                   int64_t* __restrict__ excl_n,
                                                   int32_t* __restrict__ nlist) {
  __shared__ int64_t sh[17];
  int64_t carry = 0;
  for (int64_t t0 = 0; t0 < ntiles; t0 += 1024) {
    const int64_t t = t0 + threadIdx.x;
    const int64_t v = t < ntiles ? tsum[t] : 0;
    int64_t tot;
    const int64_t pre = block_excl_scan<1024>(v, &tot, sh);
    if (t < ntiles) tsum[t] = carry + pre;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    excl_n[0] = carry & (kScanHi - 1);
    if (nlist) nlist[0] = (int32_t)(carry >> 40);
  }
}

// ... then every tile again from its offset
__global__ __launch_bounds__(1024) void k_scan_down(const int32_t* __restrict__ cnt, int64_t n,
                                                    const int64_t* __restrict__ toff,
                                                    int64_t* __restrict__ excl,
                                                    int32_t* __restrict__ list) {
  __shared__ int64_t sh[17];
  (void)scan_tile(cnt, n, (int64_t)blockIdx.x * kScanTile, toff[blockIdx.x], excl, list, sh);
}

// One workgroup up to two tiles, else the three-pass form (tsum: ntiles
// int64 of scratch).
void launch_scan(const int32_t* cnt, int64_t n, int64_t* excl, int32_t* list,
                 int32_t* nlist, int64_t* tsum, hipStream_t st) {
  const int64_t ntiles = (n + kScanTile - 1) / kScanTile;
  if (ntiles <= 2 || !tsum) {
    k_scan<<<1, 1024, 0, st>>>(cnt, n, excl, list, nlist);
    return;
  }
  k_scan_reduce<<<(unsigned)ntiles, 1024, 0, st>>>(cnt, n, tsum);
  k_scan_top<<<1, 1024, 0, st>>>(tsum, ntiles, excl + n, nlist);
  k_scan_down<<<(unsigned)ntiles, 1024, 0, st>>>(cnt, n, tsum, excl, list);
}

// Fresh cells of a moved body (Sec. 7.1: a moving boundary exposes fresh
// fluid cells): cells whose centre was solid before the move (tag 1 or 2)
// and is fluid after it (tag 0 or -2); uncovered ones were not ghosts before
// (tag 1), so no value was ever reconstructed there.  One workgroup per
// chunk of 4096 cells, 16 per thread (tag arrays are 256-byte aligned).  A
// chunk whose spans both plans settled to the same class holds no fresh
// cell (each of its cells lies on that side of both boundaries) and is
// skipped on its span flags alone.
__global__ void k_fresh_zero(int64_t* counts) {
  if (threadIdx.x < 2) counts[threadIdx.x] = 0;
}

__device__ __forceinline__ uint32_t fresh_bits(const int8_t* __restrict__ a,
                                               const int8_t* __restrict__ b, int64_t base,
                                               int64_t n, int& unc) {
  uint32_t m = 0;
  unc = 0;
  int8_t ta[kSeg], tb[kSeg];
  if (base + kSeg <= n) {
    *reinterpret_cast<uint4*>(ta) = *reinterpret_cast<const uint4*>(a + base);
    *reinterpret_cast<uint4*>(tb) = *reinterpret_cast<const uint4*>(b + base);
  } else {
    for (int q = 0; q < kSeg; ++q) {
      ta[q] = base + q < n ? a[base + q] : 0;
      tb[q] = base + q < n ? b[base + q] : 0;
    }
  }
#pragma unroll
  for (int q = 0; q < kSeg; ++q)
    if ((ta[q] == 1 || ta[q] == 2) && (tb[q] == 0 || tb[q] == -2)) {
      m |= 1u << q;
      unc += ta[q] == 1;
    }
  return m;
}

__device__ __forceinline__ bool spans_agree(const int8_t* __restrict__ sa,
                                            const int8_t* __restrict__ sb, int64_t chunk) {
  constexpr int kPer = kChunk / (64 * kSeg);
  bool same = true;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int8_t x = sa[chunk * kPer + q];
    same = same && x >= 0 && x == sb[chunk * kPer + q];
  }
  return same;
}

__global__ __launch_bounds__(256) void k_fresh_count(const int8_t* __restrict__ a,
                                                     const int8_t* __restrict__ b,
                                                     const int8_t* __restrict__ sa,
                                                     const int8_t* __restrict__ sb, int64_t n,
                                                     int32_t* __restrict__ chunk_cnt,
                                                     int64_t* __restrict__ counts) {
  __shared__ int s_cnt, s_unc;
  if (spans_agree(sa, sb, blockIdx.x)) {   // uniform over the workgroup
    if (threadIdx.x == 0) chunk_cnt[blockIdx.x] = 0;
    return;
  }
  if (threadIdx.x == 0) s_cnt = s_unc = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kSeg;
  int unc = 0;
  const uint32_t m = base < n ? fresh_bits(a, b, base, n, unc) : 0u;
  if (m) atomicAdd(&s_cnt, __popc(m));
  if (unc) atomicAdd(&s_unc, unc);
  __syncthreads();
  if (threadIdx.x == 0) {
    chunk_cnt[blockIdx.x] = s_cnt;
    if (s_cnt) atomicAdd(reinterpret_cast<unsigned long long*>(&counts[0]), (unsigned long long)s_cnt);
    if (s_unc) atomicAdd(reinterpret_cast<unsigned long long*>(&counts[1]), (unsigned long long)s_unc);
  }
}

__global__ __launch_bounds__(256) void k_fresh_scatter(const int8_t* __restrict__ a,
                                                       const int8_t* __restrict__ b,
                                                       const int8_t* __restrict__ sa,
                                                       const int8_t* __restrict__ sb, int64_t n,
                                                       const int64_t* __restrict__ excl,
                                                       int32_t* __restrict__ list, int64_t cap) {
  __shared__ int64_t sh[5];
  if (spans_agree(sa, sb, blockIdx.x)) return;   // no fresh cell here
  const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kSeg;
  int unc = 0;
  uint32_t m = base < n ? fresh_bits(a, b, base, n, unc) : 0u;
  int64_t tot;
  int64_t pos = excl[blockIdx.x] + block_excl_scan<256>(__popc(m), &tot, sh);
  while (m) {
    const int q = __ffs(m) - 1;
    m &= m - 1;
    if (pos < cap) list[pos] = (int32_t)(base + q);
    ++pos;
  }
}

extern "C" gcr_status gcr_plan_fresh_cells(const gcr_plan* a, const gcr_plan* b, int64_t* counts,
                                           int32_t* list, int64_t cap, void* stream) {
  if (!plan_ok(a) || !plan_ok(b) || !counts || cap < 0 || (cap > 0 && !list)) return GCR_E_ARG;
  if (a->dim != b->dim || a->ncell != b->ncell) return GCR_E_ARG;
  for (int ax = 0; ax < 3; ++ax)
    if (a->inst.g.n[ax] != b->inst.g.n[ax] || a->inst.g.lo[ax] != b->inst.g.lo[ax] ||
        a->inst.g.h[ax] != b->inst.g.h[ax])
      return GCR_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = a->ncell, nch = (n + kChunk - 1) / kChunk;
  const int64_t ntiles = (nch + kScanTile - 1) / kScanTile;
  auto al = [](size_t v) { return (v + 255) & ~size_t(255); };
  const size_t o_ex = al(sizeof(int32_t) * nch), o_ts = o_ex + al(sizeof(int64_t) * (nch + 1));
  char* scr = static_cast<char*>(
      plan_scratch(const_cast<gcr_plan*>(b), 6, o_ts + al(sizeof(int64_t) * (ntiles + 1))));
  if (!scr) return GCR_E_NOMEM;
  int32_t* ccnt = reinterpret_cast<int32_t*>(scr);
  int64_t* excl = reinterpret_cast<int64_t*>(scr + o_ex);
  int64_t* tsum = reinterpret_cast<int64_t*>(scr + o_ts);
  k_fresh_zero<<<1, 64, 0, st>>>(counts);
  k_fresh_count<<<(unsigned)nch, 256, 0, st>>>(a->tags, b->tags, a->span, b->span, n, ccnt,
                                               counts);
  if (list && cap > 0) {
    launch_scan(ccnt, nch, excl, nullptr, nullptr, tsum, st);
    k_fresh_scatter<<<(unsigned)nch, 256, 0, st>>>(a->tags, b->tags, a->span, b->span, n, excl,
                                                   list, cap);
  }
  GCR_HIP(hipGetLastError());
  return GCR_OK;
}

// Second ghost layer (Sec. 7.1): the solid cells within R_i cells along each
// axis i of a solid interface cell, R_i = floor((1.5 + sqrt(d)/2) w_max /
// w_min_i) + 1 (w_max the largest cell width, w_min_i the smallest along i;
// h_max / h_i on a uniform grid; set per instance on the host), get the
// candidate mark 0x20.  Every cell with psi <= 1.5 delta n is among them: a
// walk from it through its foot point reaches a fluid centre within that
// box (delta n <= w_max, psi 1-Lipschitz), and the last solid cell before it
// is a solid interface cell.  One workgroup per chunk
// of the interface chunk list (the grid covers every chunk; the rest exit):
// the chunk's solid interface cells go to an LDS list, then the workgroup
// walks the (cell, box offset) pairs, eight loads in flight per thread
// before any mark is set.
__global__ __launch_bounds__(256) void k_l2_mark(const Inst* __restrict__ insts, int ninst,
                                                 const int64_t* __restrict__ chunk_start,
                                                 const int32_t* __restrict__ chunk_list,
                                                 const int32_t* __restrict__ nlist,
                                                 int8_t* __restrict__ tags,
                                                 int32_t* __restrict__ dirty,
                                                 int32_t* __restrict__ dlist,
                                                 int32_t* __restrict__ ndirty) {
  __shared__ int s_cell[kChunk];
  __shared__ int s_n;
  if ((int)blockIdx.x >= nlist[0]) return;
  const int64_t chunk = chunk_list[blockIdx.x];
  const int ii = find_inst(chunk_start, ninst, chunk);
  const Inst& I = insts[ii];
  if (!I.layer2) return;
  const GridD g = I.g;
  const int8_t* T = tags + I.cell_off;
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  const int64_t base = (chunk - I.chunk_off) * kChunk;
  for (int t = threadIdx.x; t < kChunk; t += 256) {
    const int64_t c = base + t;
    if (c < g.ncell && (T[c] & 0x41) == 0x41) s_cell[atomicAdd(&s_n, 1)] = (int)c;
  }
  __syncthreads();
  const int R[3] = {I.l2r[0], I.l2r[1], I.l2r[2]};   // 0 beyond the grid's dimension
  const int W[3] = {2 * R[0] + 1, 2 * R[1] + 1, 2 * R[2] + 1};
  const int box = W[0] * W[1] * W[2];
  const int64_t items = (int64_t)s_n * box;
  constexpr int kFly = 8;
  for (int64_t i0 = threadIdx.x; i0 < items; i0 += 256 * kFly) {
    int64_t at[kFly];
    int8_t v[kFly];
#pragma unroll
    for (int u = 0; u < kFly; ++u) {
      const int64_t it = i0 + (int64_t)u * 256;
      at[u] = -1;
      v[u] = 0;
      if (it < items) {
        const int c = s_cell[it / box];
        int o = (int)(it % box);
        const int di = o % W[0] - R[0];
        o /= W[0];
        const int dj = o % W[1] - R[1];
        const int dk = o / W[1] - R[2];
        int i, j, k;
        unlinear(g, c, i, j, k);
        i += di;
        j += dj;
        k += dk;
        if (i >= 0 && i < g.n[0] && j >= 0 && j < g.n[1] && k >= 0 && k < g.n[2]) {
          at[u] = I.cell_off + linear(g, i, j, k);
          v[u] = tags[at[u]];
        }
      }
    }
    // plain solid, not yet marked: a byte store, as every writer of a cell
    // here stores the same value (1 -> 0x21) and no other kernel runs
#pragma unroll
    for (int u = 0; u < kFly; ++u)
      if (at[u] >= 0 && v[u] == 1) {
        tags[at[u]] = 0x21;
        if (dirty) {
          // a re-plan counts marks in the listed chunks only: list this one
          const int64_t ch = I.chunk_off + (at[u] - I.cell_off) / kChunk;
          if (dirty[ch] == 0 && atomicExch(&dirty[ch], 1) == 0)
            dlist[atomicAdd(ndirty, 1)] = (int32_t)ch;
        }
      }
  }
}

// per chunk: cells with an interface or candidate mark, for every chunk
// (list null) or the chunks of list[0, *nlist) (the classified ones and
// those a candidate mark reached; the others hold none)
__device__ __forceinline__ void count_marks_chunk(int64_t chunk, const Inst* __restrict__ insts,
                                                  int ninst,
                                                  const int64_t* __restrict__ chunk_start,
                                                  const int8_t* __restrict__ tags,
                                                  int32_t* __restrict__ chunk_cnt) {
  __shared__ int s;
  const int ii = find_inst(chunk_start, ninst, chunk);
  const Inst& I = insts[ii];
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  const int64_t base = (chunk - I.chunk_off) * kChunk + (int64_t)threadIdx.x * kSeg;
  int n = 0;
  if (base + kSeg <= I.g.ncell) {
    const uint4 w = *reinterpret_cast<const uint4*>(tags + I.cell_off + base);
    const uint32_t q[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const uint32_t m = q[b] & 0x60606060u;   // per byte: bit 0 set iff 0x20 or 0x40 is
      n += __popc(((m >> 5) | (m >> 6)) & 0x01010101u);
    }
  } else {
    for (int b = 0; b < kSeg; ++b)
      if (base + b < I.g.ncell && (tags[I.cell_off + base + b] & 0x60)) ++n;
  }
  if (n) atomicAdd(&s, n);
  __syncthreads();
  if (threadIdx.x == 0) chunk_cnt[chunk] = s;
}

__global__ __launch_bounds__(256) void k_count_marks(const Inst* __restrict__ insts, int ninst,
                                                     const int64_t* __restrict__ chunk_start,
                                                     const int8_t* __restrict__ tags,
                                                     int32_t* __restrict__ chunk_cnt,
                                                     const int32_t* __restrict__ list,
                                                     const int32_t* __restrict__ nlist) {
  if (!list) {   // every chunk, one workgroup each
    count_marks_chunk(blockIdx.x, insts, ninst, chunk_start, tags, chunk_cnt);
    return;
  }
  const int nit = nlist[0];
  for (int it = blockIdx.x; it < nit; it += gridDim.x) {
    count_marks_chunk(list[it], insts, ninst, chunk_start, tags, chunk_cnt);
    __syncthreads();   // s is reused by the next chunk
  }
}

// off[i] = excl[start[i]] for the instance boundaries
__global__ void k_gather_off(const int64_t* __restrict__ excl, const int64_t* __restrict__ start,
                             int n, int64_t* __restrict__ off) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n) off[i] = excl[start[i]];
}

__global__ __launch_bounds__(256) void k_compact_iface(const Inst* __restrict__ insts,
                                                       const int32_t* __restrict__ chunk_inst,
                                                       const int8_t* __restrict__ tags,
                                                       const int32_t* __restrict__ chunk_cnt,
                                                       const int64_t* __restrict__ chunk_excl,
                                                       const int32_t* __restrict__ chunk_list,
                                                       int32_t* __restrict__ if_cell,
                                                       unsigned long long* __restrict__ htab,
                                                       int64_t nhash) {
  // the cell -> ghost tables, emptied here for k_hash_build
  for (int64_t z = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; z < nhash;
       z += (int64_t)gridDim.x * blockDim.x)
    htab[z] = ~0ull;
  const int64_t chunk = chunk_list[blockIdx.x];   // chunks holding listed cells
  __shared__ int64_t sh[5];
  const int ii = chunk_inst[chunk];
  const Inst& I = insts[ii];
  const int64_t base64 = (chunk - I.chunk_off) * kChunk + (int64_t)threadIdx.x * kSeg;
  uint32_t mask = 0;
  int base = 0;
  if (base64 < I.g.ncell) {
    base = (int)base64;
    const int nvalid = (int)min((int64_t)kSeg, I.g.ncell - base64);
    const int8_t* src = tags + I.cell_off + base;
    if (nvalid == kSeg) {
      const uint4 w = *reinterpret_cast<const uint4*>(src);
      const uint32_t q[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int b = 0; b < kSeg; ++b)
        if ((q[b >> 2] >> (8 * (b & 3))) & 0x60u) mask |= 1u << b;
    } else {
      for (int b = 0; b < nvalid; ++b)
        if (src[b] & 0x60) mask |= 1u << b;
    }
  }
  int64_t tot;
  int64_t pos = chunk_excl[chunk] + block_excl_scan<256>(__popc(mask), &tot, sh);
  while (mask) {
    int b = __ffs(mask) - 1;
    mask &= mask - 1;
    if_cell[pos++] = base + b;
  }
}

// --------------------------------------------------------------------------
// 3. geometry and ghost tags
// --------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_geometry(const Inst* __restrict__ insts, int ninst,
                                                  const int64_t* __restrict__ if_off,
                                                  const int32_t* __restrict__ if_cell,
                                                  int8_t* __restrict__ tags,
                                                  double* __restrict__ if_psi,
                                                  double* __restrict__ if_n, int64_t cap,
                                                  uint8_t* __restrict__ if_flag,
                                                  InstInfo* __restrict__ info) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= if_off[ninst]) return;
  const int ii = find_inst(if_off, ninst, e);
  const Inst& I = insts[ii];
  const GridD& g = I.g;
  const int c = if_cell[e];
  int8_t* tp = tags + I.cell_off + c;
  const int8_t t0 = *tp;
  const bool solid = (t0 & 1) != 0;
  const bool iface = (t0 & 0x40) != 0;   // else a second-layer candidate
  int i, j, k;
  unlinear(g, c, i, j, k);
  double x[3] = {centre(g, 0, i), centre(g, 1, j), g.dim == 3 ? centre(g, 2, k) : 0.0};
  double n[3] = {0.0, 0.0, 0.0}, psi = 0.0;
  bool ok = project(I.s, g.dim, x, solid, n, psi);
  if (!ok) atomicOr(&info[ii].err, kErrGeometry);
  // Eq. delta_n with the cell's own widths
  const int ijk[3] = {i, j, k};
  double sum = 0.0;
  for (int a = 0; a < g.dim; ++a) {
    const double w = width(g, a, ijk[a]);
    sum += (n[a] / w) * (n[a] / w);
  }
  double dn = 1.0 / sqrt(sum);
  bool ghost = false;
  if (iface) {
    if (I.scheme == kHGC) ghost = solid ? (psi <= dn / 2.0) : (-psi < dn / 2.0);
    else ghost = solid;
  }
  // Sec. 7.1: a second layer adds the solid cells with psi <= 1.5 delta n,
  // reconstructed on the extended stencil
  const bool ext = I.layer2 && solid && !ghost && psi <= 1.5 * dn;
  ghost = ghost || ext;
  *tp = ghost ? (solid ? 2 : -2) : (solid ? 1 : 0);
  if_psi[e] = psi;
  for (int a = 0; a < 3; ++a) if_n[a * cap + e] = n[a];
  if_flag[e] = ghost ? (ext ? 3 : 1) : 0;   // bit 0 ghost, bit 1 extended stencil
}

// per 1024-entry block counts of flags
__global__ __launch_bounds__(256) void k_count_flags(const uint8_t* __restrict__ flag, int64_t n,
                                                     int32_t* __restrict__ cnt) {
  __shared__ int s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  int c = 0;
  for (int t = 0; t < 4; ++t) {
    int64_t e = (int64_t)blockIdx.x * 1024 + t * 256 + threadIdx.x;
    if (e < n) c += flag[e] & 1;
  }
  if (c) atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_scatter_ghosts(
    const uint8_t* __restrict__ flag, int64_t n, const int64_t* __restrict__ blk_excl,
    const int32_t* __restrict__ if_cell, const double* __restrict__ if_psi,
    const double* __restrict__ if_n, int64_t cap, int32_t* __restrict__ g_cell,
    double* __restrict__ g_psi, double* __restrict__ g_n, uint8_t* __restrict__ g_ext) {
  __shared__ int64_t sh[5];
  int64_t run = blk_excl[blockIdx.x];
  for (int t = 0; t < 4; ++t) {
    int64_t e = (int64_t)blockIdx.x * 1024 + t * 256 + threadIdx.x;
    const int fl = (e < n) ? flag[e] : 0;
    const int f = fl & 1;
    int64_t tot;
    int64_t pos = run + block_excl_scan<256>(f, &tot, sh);
    if (f) {
      g_ext[pos] = (uint8_t)(fl >> 1);
      g_cell[pos] = if_cell[e];
      g_psi[pos] = if_psi[e];
      for (int a = 0; a < 3; ++a) g_n[a * cap + pos] = if_n[a * cap + e];
    }
    run += tot;
  }
}

// ghost offsets of the instances: ghosts before interface entry if_off[i]
// one wave per offset i = 0..ninst: the ghosts before interface cell
// if_off[i] are those of the whole 1024-flag blocks before it plus the
// flags of its own block up to it
__global__ __launch_bounds__(64) void k_ghost_off(const uint8_t* __restrict__ flag,
                                                  const int64_t* __restrict__ blk_excl,
                                                  const int64_t* __restrict__ if_off, int ninst,
                                                  int64_t* __restrict__ g_off) {
  const int i = blockIdx.x;
  if (i > ninst) return;
  const int64_t e = if_off[i];
  const int64_t b = e / 1024;
  int c = 0;
  for (int64_t q = b * 1024 + threadIdx.x; q < e; q += 64) c += flag[q] & 1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
  if (threadIdx.x == 0) g_off[i] = blk_excl[b] + c;
}

// --------------------------------------------------------------------------
// 4. stencils and dependencies
// --------------------------------------------------------------------------

// value stored for cell c in one instance's table, or -1 (linear probing;
// the table is at most half full, so an empty slot ends every probe)
__device__ __forceinline__ int hash_find(const unsigned long long* t, uint32_t mask, int c) {
  uint32_t h = (uint32_t)c * 2654435761u;
  h = (h ^ (h >> 15)) & mask;
  for (;;) {
    const unsigned long long e = t[h];
    if (e == ~0ull) return -1;
    if ((int)(e >> 32) == c) return (int)(e & 0xffffffffu);
    h = (h + 1) & mask;
  }
}

__global__ __launch_bounds__(256) void k_deps(const Inst* __restrict__ insts, int ninst,
                                              const int64_t* __restrict__ g_off,
                                              const int32_t* __restrict__ g_cell,
                                              const double* __restrict__ g_psi,
                                              const double* __restrict__ g_n, int64_t cap,
                                              const uint8_t* __restrict__ g_ext,
                                              const int8_t* __restrict__ tags,
                                              const unsigned long long* __restrict__ htab,
                                              const int64_t* __restrict__ hoff,
                                              const uint32_t* __restrict__ hmask,
                                              uint32_t* __restrict__ g_code,
                                              int32_t* __restrict__ deps,
                                              int32_t* __restrict__ rcnt,
                                              uint8_t* __restrict__ dcnt,
                                              InstInfo* __restrict__ info) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g_off[ninst]) return;
  const int ii = find_inst(g_off, ninst, e);
  const Inst& I = insts[ii];
  const GridD& g = I.g;
  const int c = g_cell[e];
  const double psi = g_psi[e];
  double n[3];
  int r[3] = {1, 1, 1};
  for (int a = 0; a < 3; ++a) n[a] = g_n[a * cap + e];
  if (I.scheme == kCGC_ES || g_ext[e]) {
    // Eq. stencil_anisotropic: r_i = max(1, ceil(2 |x_1 - x_s|_i / dx_i)),
    // dx_i the ghost cell's own width
    int gi[3];
    unlinear(g, c, gi[0], gi[1], gi[2]);
    for (int a = 0; a < g.dim; ++a) {
      double d = psi * n[a];
      double q = 2.0 * fabs(d) / width(g, a, gi[a]);
      int ri = (int)ceil(q);
      r[a] = ri < 1 ? 1 : ri;
      if (r[a] > 15) {
        atomicOr(&info[ii].err, kErrUnsupported);
        r[a] = 15;
      }
    }
  }
  const uint32_t code = make_code(n, r, g.dim);
  g_code[e] = code;
  int i, j, k;
  unlinear(g, c, i, j, k);
  const int8_t* T = tags + I.cell_off;
  const int np = (1 << g.dim) - 1;
  const uint32_t skip = code_skip(code);
  int nd = 0;
  for (int m = 1; m <= np; ++m) {
    int32_t d = -1;
    if (!(m & skip)) {
      if (!corner_in_grid(g, code, i, j, k, m)) {
        atomicOr(&info[ii].err, kErrStencil);
      } else {
        int q = c + corner_offset(g, code, m);
        int8_t t = T[q];
        if (t == 1) atomicOr(&info[ii].err, kErrStencil);
        else if (t == 2 || t == -2) {
          const int v = hash_find(htab + hoff[ii], hmask[ii], q);
          if (v >= 0) d = (int32_t)(g_off[ii] + v);
        }
      }
    }
    deps[(int64_t)(m - 1) * cap + e] = d;
    if (d >= 0) {
      atomicAdd(&rcnt[d], 1);   // reverse edge d -> e
      ++nd;
    }
  }
  dcnt[e] = (uint8_t)nd;
}

// Reverse edges of the dependency graph as CSR over all ghosts (linear
// order): off[e] = first reader of ghost e, off[ng] = number of edges.
// One workgroup; the ghost count is read on the device.
__global__ __launch_bounds__(1024) void k_rscan(const int32_t* __restrict__ cnt,
                                                const int64_t* __restrict__ g_off, int ninst,
                                                int32_t* __restrict__ off) {
  __shared__ int64_t sh[17];
  block_scan_i32(cnt, g_off[ninst], off, sh);
}

// The same for long inputs, in three passes (tile totals; their scan,
// k_scan_top; tiles again from their offsets), tiles of kScanTile values.
// The counts past the ghost count are zero, so scanning the interface
// capacity gives the same offsets up to the ghost count.
__global__ __launch_bounds__(1024) void k_iscan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                       int64_t* __restrict__ tsum) {
  __shared__ int64_t sh[17];
  const int64_t b = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanT;
  int64_t sum = 0;
#pragma unroll
  for (int q = 0; q < kScanT; ++q) sum += b + q < n ? in[b + q] : 0;
  int64_t tot;
  (void)block_excl_scan<1024>(sum, &tot, sh);
  if (threadIdx.x == 0) tsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_iscan_down(const int32_t* __restrict__ in, int64_t n,
                                                     const int64_t* __restrict__ toff,
                                                     int32_t* __restrict__ out) {
  __shared__ int64_t sh[17];
  const int64_t b = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanT;
  int v[kScanT];
  int64_t sum = 0;
#pragma unroll
  for (int q = 0; q < kScanT; ++q) {
    v[q] = b + q < n ? in[b + q] : 0;
    sum += v[q];
  }
  int64_t tot;
  int64_t run = toff[blockIdx.x] + block_excl_scan<1024>(sum, &tot, sh);
#pragma unroll
  for (int q = 0; q < kScanT; ++q) {
    if (b + q < n) out[b + q] = (int32_t)run;
    run += v[q];
  }
  if (b < n && b + kScanT >= n) out[n] = (int32_t)run;   // the thread holding the last value
}

__global__ __launch_bounds__(256) void k_rfill(const Inst* __restrict__ insts,
                                               const int64_t* __restrict__ g_off, int ninst,
                                               int64_t cap, const int32_t* __restrict__ deps,
                                               const int32_t* __restrict__ off,
                                               int32_t* __restrict__ fillc,
                                               int32_t* __restrict__ radj) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g_off[ninst]) return;
  const int ii = find_inst(g_off, ninst, e);
  const int np = (1 << insts[ii].g.dim) - 1;
  for (int m = 0; m < np; ++m) {
    const int32_t d = deps[(int64_t)m * cap + e];
    if (d >= 0) radj[off[d] + atomicAdd(&fillc[d], 1)] = (int32_t)e;
  }
}

// --------------------------------------------------------------------------
// 6. canonical arrays
// --------------------------------------------------------------------------

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* a, double v) {
  if (v > 0.0) atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

// per-workgroup statistics of k_finalize, reduced per instance by
// k_units_canonical (inst -1: the workgroup held no ghosts, or ghosts of
// two instances, whose statistics it applied with atomics itself)
struct FinPart {
  double am[3];
  int32_t rm[3];
  int32_t fl;
  int32_t inst;
  int32_t pad;
};

__global__ __launch_bounds__(256) void k_finalize(
    const Inst* __restrict__ insts, int ninst, const int64_t* __restrict__ g_off, int64_t cap,
    const int32_t* __restrict__ g_cell, const double* __restrict__ g_psi,
    const double* __restrict__ g_n, const uint32_t* __restrict__ g_code,
    const int32_t* __restrict__ lev, const int32_t* __restrict__ blk_idx,
    const int32_t* __restrict__ perm, int32_t* __restrict__ cell, double* __restrict__ delta,
    double* __restrict__ nrm, double* __restrict__ psi, uint32_t* __restrict__ code,
    int32_t* __restrict__ level, int32_t* __restrict__ blk, InstInfo* __restrict__ info,
    FinPart* __restrict__ part) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ng_all = g_off[ninst];
  // per-thread statistics: max alpha and multiplier per axis, fluid-side count
  double am[3] = {0.0, 0.0, 0.0};
  int rm[3] = {0, 0, 0}, fl = 0, ii = -1;
  if (e < ng_all) {
    ii = find_inst(g_off, ninst, e);
    const GridD& g = insts[ii].g;
    const int pl = perm[e];
    if (pl >= 0 && pl < g_off[ii + 1] - g_off[ii]) {   // else the build failed earlier
      const int64_t p = g_off[ii] + pl;
      const double ps = g_psi[e];
      const uint32_t cd = g_code[e];
      cell[p] = g_cell[e];
      psi[p] = ps;
      code[p] = cd;
      level[p] = lev[e];
      blk[p] = blk_idx[e];
      for (int a = 0; a < 3; ++a) {
        double na = g_n[a * cap + e];
        double da = ps * na;
        nrm[a * cap + p] = na;
        delta[a * cap + p] = da;
        if (a < g.dim) {
          double Xs[3];
          stencil_span(g, cd, g_cell[e], Xs);
          am[a] = fmax(0.0, da / Xs[a]);
          rm[a] = code_r(cd, a);
        }
      }
      fl = ps < 0.0 ? 1 : 0;
    }
  }
  // one instance in the whole workgroup: reduce there, one atomic per value
  __shared__ int s_i0;
  __shared__ double s_am[3][256];
  __shared__ int s_rm[3][256], s_fl[256];
  if (threadIdx.x == 0) s_i0 = ii;
  __syncthreads();
  const bool uniform = __syncthreads_and(ii == s_i0 || ii < 0) && s_i0 >= 0;
  if (!uniform && threadIdx.x == 0) part[blockIdx.x].inst = -1;
  if (!uniform) {
    if (ii >= 0) {
      for (int a = 0; a < 3; ++a) {
        atomic_max_nonneg(&info[ii].max_alpha_bits[a], am[a]);
        if (rm[a]) atomicMax(&info[ii].rmax[a], rm[a]);
      }
      if (fl) atomicAdd(&info[ii].nfluid, 1);
    }
    return;
  }
  for (int a = 0; a < 3; ++a) {
    s_am[a][threadIdx.x] = am[a];
    s_rm[a][threadIdx.x] = rm[a];
  }
  s_fl[threadIdx.x] = fl;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int a = 0; a < 3; ++a) {
        s_am[a][threadIdx.x] = fmax(s_am[a][threadIdx.x], s_am[a][threadIdx.x + s]);
        s_rm[a][threadIdx.x] = max(s_rm[a][threadIdx.x], s_rm[a][threadIdx.x + s]);
      }
      s_fl[threadIdx.x] += s_fl[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // one record per workgroup (atomics from every workgroup of an instance
    // on its one record would serialise)
    FinPart r;
    for (int a = 0; a < 3; ++a) {
      r.am[a] = s_am[a][0];
      r.rm[a] = s_rm[a][0];
    }
    r.fl = s_fl[0];
    r.inst = s_i0;
    r.pad = 0;
    part[blockIdx.x] = r;
  }
}

// k_finalize's workgroup records of this instance folded into its info
// (max, max, sum: the order does not matter), then unit members:
// linear-order positions -> instance-local canonical positions
__global__ __launch_bounds__(256) void k_units_canonical(const int32_t* __restrict__ perm,
                                                         InstInfo* __restrict__ info,
                                                         int32_t* __restrict__ unit_mem_all,
                                                         const int32_t* __restrict__ unit_cnt_all,
                                                         const FinPart* __restrict__ part,
                                                         int64_t nparts) {
  const int ii = blockIdx.x;
  {
    double am[3] = {0.0, 0.0, 0.0};
    int rm[3] = {0, 0, 0}, fl = 0;
    for (int64_t b = threadIdx.x; b < nparts; b += blockDim.x) {
      const FinPart& r = part[b];
      if (r.inst != ii) continue;
      for (int a = 0; a < 3; ++a) {
        am[a] = fmax(am[a], r.am[a]);
        rm[a] = max(rm[a], r.rm[a]);
      }
      fl += r.fl;
    }
    __shared__ double s_am[3][256];
    __shared__ int s_rm[3][256], s_fl[256];
    for (int a = 0; a < 3; ++a) {
      s_am[a][threadIdx.x] = am[a];
      s_rm[a][threadIdx.x] = rm[a];
    }
    s_fl[threadIdx.x] = fl;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if ((int)threadIdx.x < st) {
        for (int a = 0; a < 3; ++a) {
          s_am[a][threadIdx.x] = fmax(s_am[a][threadIdx.x], s_am[a][threadIdx.x + st]);
          s_rm[a][threadIdx.x] = max(s_rm[a][threadIdx.x], s_rm[a][threadIdx.x + st]);
        }
        s_fl[threadIdx.x] += s_fl[threadIdx.x + st];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      InstInfo& I = info[ii];
      for (int a = 0; a < 3; ++a) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(s_am[0 + a][0]);
        if (bits > I.max_alpha_bits[a]) I.max_alpha_bits[a] = bits;   // non-negative: bit order
        I.rmax[a] = max(I.rmax[a], s_rm[a][0]);
      }
      I.nfluid += s_fl[0];
    }
  }
  const int nu = info[ii].nunits;
  int32_t* um = unit_mem_all + (int64_t)ii * kMaxUnits * kMaxUnit;
  const int32_t* uc = unit_cnt_all + (int64_t)ii * kMaxUnits;
  for (int t = threadIdx.x; t < nu * kMaxUnit; t += blockDim.x) {
    int u = t / kMaxUnit, q = t % kMaxUnit;
    if (q < uc[u]) um[t] = perm[um[t]];
  }
}

// --------------------------------------------------------------------------
// 7. cell -> ghost hash tables (open addressing, at most half full)
// --------------------------------------------------------------------------

__global__ void k_hash_clear(unsigned long long* __restrict__ t, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = ~0ull;
}

__global__ void k_hash_build(const int64_t* __restrict__ g_off, int ninst,
                             const int32_t* __restrict__ cell,
                             const int64_t* __restrict__ hoff,
                             const uint32_t* __restrict__ hmask,
                             unsigned long long* __restrict__ htab,
                             int32_t* __restrict__ zero, int64_t nzero) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // the dependency counters that the next launch fills, cleared here
  for (int64_t z = e; z < nzero; z += (int64_t)gridDim.x * blockDim.x) zero[z] = 0;
  if (e >= g_off[ninst]) return;
  const int ii = find_inst(g_off, ninst, e);
  const int c = cell[e];
  const unsigned long long entry =
      ((unsigned long long)(uint32_t)c << 32) | (uint32_t)(e - g_off[ii]);
  unsigned long long* t = htab + hoff[ii];
  const uint32_t mask = hmask[ii];
  uint32_t h = (uint32_t)c * 2654435761u;
  h = (h ^ (h >> 15)) & mask;
  while (atomicCAS(&t[h], ~0ull, entry) != ~0ull) h = (h + 1) & mask;
}

// linear-order ghost index -> canonical position, in place
__global__ void k_hash_remap(const int64_t* __restrict__ hoff, int ninst,
                             const int64_t* __restrict__ g_off, const int32_t* __restrict__ perm,
                             unsigned long long* __restrict__ htab) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= hoff[ninst]) return;
  const unsigned long long e = htab[s];
  if (e == ~0ull) return;
  const int ii = find_inst(hoff, ninst, s);
  const int32_t v = (int32_t)(e & 0xffffffffu);
  htab[s] = (e & 0xffffffff00000000ull) | (uint32_t)perm[g_off[ii] + v];
}

// --------------------------------------------------------------------------
// host orchestration
// --------------------------------------------------------------------------

static double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= (double)i;
  return f;
}

constexpr int kMaxL2Radius = 64;   // second-layer candidate box half-width, cells

static gcr_status make_shape(const gcr_shape& gs, int dim, ShapeD* out);

static gcr_status make_inst(const gcr_grid& gg, const gcr_shape& gs, int scheme, Inst* I) {
  std::memset(I, 0, sizeof(Inst));
  if (gg.dim != 2 && gg.dim != 3) return GCR_E_ARG;
  const int base = scheme & ~kLayer2;
  if (base < 0 || base > 2) return GCR_E_ARG;
  int64_t ncell = 1;
  for (int a = 0; a < gg.dim; ++a) {
    if (gg.n[a] < 1) return GCR_E_ARG;
    if (gg.faces[a]) {
      for (int64_t q = 0; q < gg.n[a]; ++q)
        if (!(gg.faces[a][q + 1] > gg.faces[a][q]) || !std::isfinite(gg.faces[a][q]) ||
            !std::isfinite(gg.faces[a][q + 1]))
          return GCR_E_ARG;
    } else if (!(gg.h[a] > 0.0) || !std::isfinite(gg.lo[a])) {
      return GCR_E_ARG;
    }
    ncell *= gg.n[a];
    if (ncell >= (int64_t(1) << 31)) return GCR_E_UNSUPPORTED;
  }
  I->g.dim = gg.dim;
  for (int a = 0; a < 3; ++a) {
    I->g.n[a] = a < gg.dim ? (int)gg.n[a] : 1;
    I->g.lo[a] = a < gg.dim ? gg.lo[a] : 0.0;
    I->g.h[a] = a < gg.dim ? gg.h[a] : 1.0;
    // a stretched axis: the caller's faces for now; build_batch puts a
    // device copy here before the instance table is uploaded
    I->g.face[a] = a < gg.dim ? gg.faces[a] : nullptr;
    if (I->g.face[a]) {
      I->g.lo[a] = gg.faces[a][0];
      I->g.h[a] = (gg.faces[a][gg.n[a]] - gg.faces[a][0]) / (double)gg.n[a];
    }
  }
  I->g.ncell = ncell;
  I->scheme = base;
  I->layer2 = (scheme & kLayer2) ? 1 : 0;
  if (I->layer2) {
    // second-layer candidate box: every solid cell with psi <= 1.5 delta n
    // has a fluid centre within (1.5 + sqrt(d)/2) w_max of its own (delta n
    // <= w_max, the largest cell width), which lies at most
    // floor(D / w_min_a) + 1 cells away along axis a (w_min_a the smallest
    // width along a)
    double wmax = 0.0, wmin[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < gg.dim; ++a) {
      wmin[a] = gg.faces[a] ? HUGE_VAL : gg.h[a];
      if (!gg.faces[a]) wmax = std::max(wmax, gg.h[a]);
      else
        for (int64_t q = 0; q < gg.n[a]; ++q) {
          const double w = gg.faces[a][q + 1] - gg.faces[a][q];
          wmax = std::max(wmax, w);
          wmin[a] = std::min(wmin[a], w);
        }
    }
    for (int a = 0; a < 3; ++a) {
      I->l2r[a] = 0;
      if (a >= gg.dim) continue;
      const double r = std::floor((1.5 + 0.5 * std::sqrt((double)gg.dim)) * wmax / wmin[a]) + 1.0;
      // box sizes stay far inside int range; wider boxes mean a grid
      // stretched beyond any use near the body
      if (!(r <= (double)kMaxL2Radius)) return GCR_E_UNSUPPORTED;
      I->l2r[a] = (int)r;
    }
  }
  return make_shape(gs, gg.dim, &I->s);
}

// The device description of body gs in dim dimensions (Sec. 7: the bodies
// of the test cases), with its culling bounds.
static gcr_status make_shape(const gcr_shape& gs, int dim, ShapeD* out) {
  ShapeD s;
  std::memset(&s, 0, sizeof(s));
  s.kind = gs.kind;
  for (int a = 0; a < 3; ++a) s.c[a] = a < dim ? gs.center[a] : 0.0;
  s.r0 = gs.r0;
  if (gs.kind == kSphere) {
    if (!(gs.r0 > 0.0)) return GCR_E_ARG;
    for (int a = 0; a < 3; ++a) s.cull_c[a] = s.c[a];
    s.rmin = s.rmax = gs.r0;
  } else if (gs.kind == kStar2D) {
    if (dim != 2 || !(gs.r0 > 0.0) || gs.ncoef < 0 || 2 * gs.ncoef > kMaxCoef) return GCR_E_ARG;
    if (gs.ncoef > 0 && !gs.coef) return GCR_E_ARG;
    s.ncoef = gs.ncoef;
    double sa = 0.0;
    for (int q = 0; q < 2 * gs.ncoef; ++q) {
      s.coef[q] = gs.coef[q];
      sa += std::fabs(gs.coef[q]);
    }
    for (int a = 0; a < 3; ++a) s.cull_c[a] = s.c[a];
    s.rmin = std::max(0.0, gs.r0 * (1.0 - sa));
    s.rmax = gs.r0 * (1.0 + sa);
    // |d/dt (A cos kt + B sin kt)| <= k sqrt(A^2 + B^2)
    double lip = 0.0;
    for (int k = 0; k < gs.ncoef; ++k)
      lip += (double)k * std::hypot(gs.coef[2 * k], gs.coef[2 * k + 1]);
    s.lip = gs.r0 * lip;
  } else if (gs.kind == kShStar) {
    int L = (int)std::lround(std::sqrt((double)gs.ncoef)) - 1;
    if (dim != 3 || !(gs.r0 > 0.0) || L < 0 || (L + 1) * (L + 1) != gs.ncoef || L > 8 ||
        !gs.coef)
      return GCR_E_ARG;
    s.ncoef = gs.ncoef;
    s.L = L;
    double sa = 0.0;
    for (int l = 0; l <= L; ++l)
      for (int m = -l; m <= l; ++m) {
        int am = m < 0 ? -m : m;
        double N = am == 0 ? 1.0 : std::sqrt(2.0 * factorial(l - am) / factorial(l + am));
        s.coef[l * l + l + m] = gs.coef[l * l + l + m] * N;
        sa += std::fabs(gs.coef[l * l + l + m]);   // |Y_lm| <= 1 (Schmidt)
      }
    for (int a = 0; a < 3; ++a) s.cull_c[a] = s.c[a];
    s.rmin = std::max(0.0, gs.r0 * (1.0 - sa));
    s.rmax = gs.r0 * (1.0 + sa);
    // on a great circle Y_lm is a trigonometric polynomial of degree <= l
    // with |Y_lm| <= 1, so (Bernstein) its derivative is at most l
    double lip = 0.0;
    for (int l = 1; l <= L; ++l)
      for (int m = -l; m <= l; ++m) lip += (double)l * std::fabs(gs.coef[l * l + l + m]);
    s.lip = gs.r0 * lip;
  } else if (gs.kind == kAirfoil) {
    if (dim != 2 || !(gs.chord > 0.0) || !(gs.thickness > 0.0) || gs.thickness > 0.5)
      return GCR_E_ARG;
    s.chord = gs.chord;
    s.thick = gs.thickness;
    s.ca = std::cos(gs.incidence);
    s.sa = std::sin(gs.incidence);
    // mid-chord in world coordinates; the section lies within 0.51 chords of it
    s.cull_c[0] = s.c[0] + gs.chord * (s.ca * 0.5);
    s.cull_c[1] = s.c[1] + gs.chord * (-s.sa * 0.5);
    s.rmin = 0.0;
    s.rmax = 0.51 * gs.chord;
  } else {
    return GCR_E_ARG;
  }
  *out = s;
  return GCR_OK;
}

BatchData::~BatchData() {
  for (void* p : owned) pool_free(p);
}

template <class T>
static T* own(BatchData& B, size_t n) {
  // bump allocation from pooled chunks of at least 4 MiB (a build makes a
  // few pool calls instead of one per array); 256-byte aligned
  constexpr size_t kArena = size_t(4) << 20;
  const size_t bytes = ((sizeof(T) * (n ? n : 1)) + 255) & ~size_t(255);
  if (bytes > B.arena_left) {
    const size_t chunk = std::max(bytes, kArena);
    char* c = static_cast<char*>(pool_alloc(chunk));
    if (!c) return nullptr;
    B.owned.push_back(c);
    if (bytes >= kArena) return reinterpret_cast<T*>(c);   // a chunk of its own
    B.arena_cur = c;
    B.arena_left = chunk;
  }
  T* p = reinterpret_cast<T*>(B.arena_cur);
  B.arena_cur += bytes;
  B.arena_left -= bytes;
  return p;
}

gcr_status status_from_err(uint32_t err) {
  if (err & kErrGeometry) return GCR_E_GEOMETRY;
  if (err & kErrCycle) return GCR_E_CYCLE;
  if (err & kErrStencil) return GCR_E_STENCIL;
  if (err & kErrDegenerate) return GCR_E_DEGENERATE;
  if (err & kErrUnsupported) return GCR_E_UNSUPPORTED;
  return GCR_OK;
}

static inline unsigned blocks(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// stage timing (process-wide switch, per-thread results)
static std::atomic<int> g_profiling{0};
static thread_local float g_stage_ms[kStages] = {};

struct StageEvents {
  hipEvent_t ev[12] = {};
  bool on = false;
  explicit StageEvents(bool enable) : on(enable) {
    if (on)
      for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) on = false;
  }
  void mark(int i, hipStream_t st) {
    if (on) (void)hipEventRecord(ev[i], st);
  }
  hipEvent_t event(int i) const { return on ? ev[i] : nullptr; }
  void collect(double call_ms) {
    if (!on) return;
    // stages 0..7 as documented; 8..10 split stage 0 into the span pass,
    // the store pass (k_classify) and the interface marks (k_band_iface);
    // 11 is the stream's wait for the host between the two halves (the
    // first synchronisation and the sizing); 12 the call's host time
    constexpr int kEv = kStages - 1;
    const int a[kEv] = {0, 1, 3, 4, 5, 6, 7, 8, 0, 10, 11, 2};
    const int b[kEv] = {1, 2, 4, 5, 6, 7, 8, 9, 10, 11, 1, 3};
    g_stage_ms[kEv] = (float)call_ms;
    for (int s = 0; s < kEv; ++s) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[a[s]], ev[b[s]]) != hipSuccess) ms = -1.f;
      g_stage_ms[s] = ms;
    }
  }
  ~StageEvents() {
    if (on)
      for (auto& e : ev) (void)hipEventDestroy(e);
  }
};

void set_profiling(int mask) { g_profiling.store(mask & 3); }
int profiling_mask() { return g_profiling.load(); }

static std::atomic<int64_t> g_wide_min{kWideMinInterface};
void set_wide_layering(int64_t v) { g_wide_min.store(v > 0 ? v : kWideMinInterface); }
int64_t wide_layering_min() { return g_wide_min.load(); }
static std::atomic<int> g_wave_res{kWaveResidual};
void set_wave_residual(int v) { g_wave_res.store(v < 0 ? 0 : (v > kWaveResidual ? kWaveResidual : v)); }
int wave_residual() { return g_wave_res.load(); }
static std::atomic<int> g_wide_buf{kWideBuf};
void set_wide_buffer(int v) { g_wide_buf.store(v <= 0 || v > kWideBuf ? kWideBuf : v); }
int wide_buffer() { return g_wide_buf.load(); }
bool wide_layering_forced() { return g_wide_min.load() != kWideMinInterface; }
void last_build_times(float* ms) {
  for (int s = 0; s < kStages; ++s) ms[s] = g_stage_ms[s];
}

template <class T>
static T* own_solo(BatchData& B, size_t n) {
  // a pool allocation of its own (so that a re-plan can take it over)
  T* p = static_cast<T*>(pool_alloc(sizeof(T) * (n ? n : 1)));
  if (p) B.owned.push_back(p);
  return p;
}

static gcr_status build_core(const std::shared_ptr<BatchData>& B, hipStream_t st,
                             BatchData* prev, std::shared_ptr<BatchData>* out);

gcr_status build_batch(int ninst, const gcr_grid* grids, const gcr_shape* shapes,
                       const int32_t* schemes, hipStream_t st, std::shared_ptr<BatchData>* out) {
  if (ninst < 1 || !grids || !shapes || !schemes || !out) return GCR_E_ARG;
  auto B = std::make_shared<BatchData>();
  B->ninst = ninst;
  B->inst.resize(ninst);
  for (int i = 0; i < ninst; ++i) {
    gcr_status s = make_inst(grids[i], shapes[i], schemes[i], &B->inst[i]);
    if (s != GCR_OK) return s;
  }
  // stretched axes: device copies of the faces (pageable sources, consumed
  // when each copy returns)
  for (int i = 0; i < ninst; ++i)
    for (int a = 0; a < 3; ++a) {
      const double* hf = B->inst[i].g.face[a];
      if (!hf) continue;
      const int64_t nf = (int64_t)B->inst[i].g.n[a] + 1;
      double* df = own<double>(*B, nf);
      if (!df) return GCR_E_NOMEM;
      GCR_HIP(hipMemcpyAsync(df, hf, sizeof(double) * nf, hipMemcpyHostToDevice, st));
      B->inst[i].g.face[a] = df;
    }
  return build_core(B, st, nullptr, out);
}

gcr_status build_update(BatchData& prev, const gcr_shape& shape, bool incremental,
                        hipStream_t st, std::shared_ptr<BatchData>* out) {
  if (prev.ninst != 1 || !out) return GCR_E_UNSUPPORTED;
  ShapeD sd;
  const gcr_status s = make_shape(shape, prev.inst[0].g.dim, &sd);
  if (s != GCR_OK) return s;
  return build_update(prev, sd, incremental, st, out);
}

gcr_status build_update(BatchData& prev, const ShapeD& shape, bool incremental, hipStream_t st,
                        std::shared_ptr<BatchData>* out) {
  if (prev.ninst != 1 || !out) return GCR_E_UNSUPPORTED;
  auto B = std::make_shared<BatchData>();
  B->ninst = 1;
  B->inst.resize(1);
  Inst I = prev.inst[0];
  I.s = shape;
  // the stretched faces: device copies of the previous plan's
  for (int a = 0; a < 3; ++a) {
    if (!I.g.face[a]) continue;
    const int64_t nf = (int64_t)I.g.n[a] + 1;
    double* df = own<double>(*B, nf);
    if (!df) return GCR_E_NOMEM;
    GCR_HIP(hipMemcpyAsync(df, I.g.face[a], sizeof(double) * nf, hipMemcpyDeviceToDevice, st));
    I.g.face[a] = df;
  }
  B->inst[0] = I;
  return build_core(B, st, incremental ? &prev : nullptr, out);
}

// The build proper: B holds its instances (device faces in place); with
// prev, a re-plan of prev's single instance that takes over its tags.
static gcr_status build_core(const std::shared_ptr<BatchData>& B, hipStream_t st,
                             BatchData* prev, std::shared_ptr<BatchData>* out) {
  const auto t_call = std::chrono::steady_clock::now();
  const int ninst = B->ninst;
  std::vector<int64_t> chunk_start(ninst + 1);
  int64_t cells = 0, chunks = 0;
  for (int i = 0; i < ninst; ++i) {
    Inst& I = B->inst[i];
    I.cell_off = cells;
    cells += (I.g.ncell + 255) / 256 * 256;
    I.chunk_off = chunks;
    I.nchunk = (I.g.ncell + kChunk - 1) / kChunk;
    chunk_start[i] = chunks;
    chunks += I.nchunk;
  }
  chunk_start[ninst] = chunks;
  B->ncells_total = cells;
  B->nchunks = chunks;
  BatchData& D = *B;
  // the small per-instance tables that cross between host and device live in
  // one device block with the layout of the pinned staging block, so each
  // transfer is one contiguous copy:
  //   R1 up:   instances | chunk starts | info (zeroed)
  //   R4 down:                            info | g_off | lev_off | unit_lev
  //   R2 down: if_off | chunk-list and band counts | interface offsets
  //   R3 up:   hash offsets | hash masks
  // each region 256-byte aligned
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  const size_t o_inst = 0, o_cs = o_inst + al(sizeof(Inst) * ninst);
  const size_t o_info = o_cs + al(8 * (ninst + 1));
  const size_t o_go = o_info + al(sizeof(InstInfo) * ninst);
  const size_t o_lo = o_go + al(8 * (ninst + 1));
  const size_t o_ul = o_lo + al(4 * (size_t)ninst * (kMaxLevels + 1));
  const size_t o_if = o_ul + al(4 * (size_t)ninst * kMaxUnits);
  const size_t o_nl = o_if + al(8 * (ninst + 1));   // chunk-list count, band stripes
  const size_t o_io = o_nl + al(64 + 64 * kBandStripes);
  const size_t o_ho = o_io + al(8 * (ninst + 1));
  const size_t o_hm = o_ho + al(8 * (ninst + 1));
  const size_t stage_bytes = o_hm + al(4 * ninst);
  char* tb = own<char>(D, stage_bytes);
  if (!tb) return GCR_E_NOMEM;
  D.d_inst = reinterpret_cast<Inst*>(tb + o_inst);
  D.d_chunk_start = reinterpret_cast<int64_t*>(tb + o_cs);
  D.d_info = reinterpret_cast<InstInfo*>(tb + o_info);
  D.d_g_off = reinterpret_cast<int64_t*>(tb + o_go);
  D.d_lev_off = reinterpret_cast<int32_t*>(tb + o_lo);
  D.d_unit_lev = reinterpret_cast<int32_t*>(tb + o_ul);
  D.d_if_off = reinterpret_cast<int64_t*>(tb + o_if);
  D.d_nchunk_list = reinterpret_cast<int32_t*>(tb + o_nl);
  D.d_nband = reinterpret_cast<int32_t*>(tb + o_nl + 64);
  D.d_iface_off = reinterpret_cast<int64_t*>(tb + o_io);
  D.d_hoff = reinterpret_cast<int64_t*>(tb + o_ho);
  D.d_hmask = reinterpret_cast<uint32_t*>(tb + o_hm);
  if (prev) {
    // the previous plan's tags, which the classification below updates
    if (prev->ninst != 1 || prev->nchunks != chunks || !prev->d_tags) return GCR_E_UNSUPPORTED;
    auto it = std::find(prev->owned.begin(), prev->owned.end(), (void*)prev->d_tags);
    if (it == prev->owned.end()) return GCR_E_UNSUPPORTED;
    prev->owned.erase(it);
    D.owned.push_back(prev->d_tags);
    D.d_tags = prev->d_tags;
    prev->d_tags = nullptr;
  } else {
    // a single instance's tags on their own, for a later re-plan to take over
    D.d_tags = ninst == 1 ? own_solo<int8_t>(D, cells) : own<int8_t>(D, cells);
  }
  D.d_chunk_cnt = own<int32_t>(D, chunks);
  D.d_dirty = own<int32_t>(D, chunks);
  D.d_dirty_list = own<int32_t>(D, chunks);
  D.d_ndirty = own<int32_t>(D, 1);
  if (!D.d_dirty || !D.d_dirty_list || !D.d_ndirty) return GCR_E_NOMEM;
  D.d_span = own<int8_t>(D, chunks * (kChunk / (64 * kSeg)));
  D.d_chunk_list = own<int32_t>(D, chunks);
  D.d_band = own<int32_t>(D, chunks * 8);   // band mask of each chunk (4 x 64 bits)
  D.d_chunk_inst = own<int32_t>(D, chunks);
  D.d_chunk_excl = own<int64_t>(D, chunks + 1);
  D.d_scan_tmp = own<int64_t>(D, (chunks + kScanTile - 1) / kScanTile + 1);
  D.d_unit_mem = own<int32_t>(D, (size_t)ninst * kMaxUnits * kMaxUnit);
  D.d_unit_cnt = own<int32_t>(D, (size_t)ninst * kMaxUnits);
  D.d_reach = own<uint32_t>(D, (size_t)ninst * kMaxResidual * (kMaxResidual / 32));
  if (!D.d_tags || !D.d_chunk_cnt || !D.d_chunk_excl || !D.d_scan_tmp || !D.d_span ||
      !D.d_chunk_list || !D.d_band || !D.d_chunk_inst || !D.d_unit_mem || !D.d_unit_cnt ||
      !D.d_reach)
    return GCR_E_NOMEM;
  bool any_layer2 = false, any_2d = false, any_3d = false;
  for (int i = 0; i < ninst; ++i) {
    any_layer2 = any_layer2 || D.inst[i].layer2;
    any_2d = any_2d || D.inst[i].g.dim == 2;
    any_3d = any_3d || D.inst[i].g.dim == 3;
  }
  PinnedStage PS;
  PS.st = st;
  PS.p = (char*)pinned_alloc(stage_bytes);
  if (!PS.p) return GCR_E_NOMEM;
  std::memcpy(PS.p + o_inst, D.inst.data(), sizeof(Inst) * ninst);
  std::memcpy(PS.p + o_cs, chunk_start.data(), 8 * (ninst + 1));
  std::memset(PS.p + o_info, 0, o_go - o_info);
  PS.pending = true;
  GCR_HIP(hipMemcpyAsync(tb, PS.p, o_go, hipMemcpyHostToDevice, st));   // R1

  StageEvents T((g_profiling.load() & 1) != 0);
  T.mark(0, st);
  ClassifyWork W{D.d_dirty, D.d_dirty_list, D.d_ndirty, D.d_chunk_excl, D.d_scan_tmp,
                 !any_3d};
  ClassifyUpdate U{};
  if (prev) {
    U.span_prev = prev->d_span;
    U.ghost_prev = prev->d_g_cell;
    U.ng_prev = prev->d_g_cell ? prev->g_off[1] : 0;
  }
  launch_classify(D.d_inst, ninst, D.d_chunk_start, chunks, D.d_span, D.d_chunk_inst, D.d_tags,
                  D.d_chunk_cnt, D.d_band, D.d_nband, T.event(10), T.event(11), st, W,
                  prev ? &U : nullptr);
  T.mark(1, st);
  launch_scan(D.d_chunk_cnt, chunks, D.d_chunk_excl, D.d_chunk_list, D.d_nchunk_list,
              D.d_scan_tmp, st);
  if (any_layer2) {
    // interface counts of the instances, then the second-layer candidates
    // join the list: mark, recount every chunk, scan again
    k_gather_off<<<blocks(ninst + 1, 64), 64, 0, st>>>(D.d_chunk_excl, D.d_chunk_start, ninst,
                                                       D.d_iface_off);
    // with a chunk list, marks outside it extend it, and the count covers
    // the list; else every chunk is counted
    const bool listed = prev || !W.every_chunk;
    k_l2_mark<<<(unsigned)chunks, 256, 0, st>>>(
        D.d_inst, ninst, D.d_chunk_start, D.d_chunk_list, D.d_nchunk_list, D.d_tags,
        listed ? D.d_dirty : nullptr, D.d_dirty_list, D.d_ndirty);
    k_count_marks<<<(unsigned)(listed ? std::min<int64_t>(chunks, kListGrid) : chunks), 256, 0,
                    st>>>(D.d_inst, ninst, D.d_chunk_start, D.d_tags, D.d_chunk_cnt,
                          listed ? D.d_dirty_list : nullptr, D.d_ndirty);
    launch_scan(D.d_chunk_cnt, chunks, D.d_chunk_excl, D.d_chunk_list, D.d_nchunk_list,
                D.d_scan_tmp, st);
  }
  k_gather_off<<<blocks(ninst + 1, 64), 64, 0, st>>>(D.d_chunk_excl, D.d_chunk_start, ninst,
                                                     D.d_if_off);
  T.mark(2, st);
  GCR_HIP(hipGetLastError());
  D.if_off.resize(ninst + 1);
  // R2 (the interface offsets only mean something with a second layer)
  GCR_HIP(hipMemcpyAsync(PS.p + o_if, tb + o_if, o_ho - o_if, hipMemcpyDeviceToHost, st));
  GCR_HIP(hipStreamSynchronize(st));
  std::memcpy(D.if_off.data(), PS.p + o_if, 8 * (ninst + 1));
  D.iface_off = D.if_off;   // interface cells alone (second-layer candidates excluded)
  if (any_layer2) std::memcpy(D.iface_off.data(), PS.p + o_io, 8 * (ninst + 1));
  int32_t nlist = 0, nband = 0;
  std::memcpy(&nlist, PS.p + o_nl, sizeof(int32_t));
  for (int q = 0; q < kBandStripes; ++q) {
    int32_t v = 0;
    std::memcpy(&v, PS.p + o_nl + 64 + 64 * q, sizeof(int32_t));
    nband += v;
  }
  D.nband = nband;
  const int64_t nif = D.if_off[ninst];
  const int64_t cap = std::max<int64_t>(nif, 1);
  D.nif = nif;
  D.cap = cap;
  // cell -> ghost tables: at most half full (ghosts <= interface cells);
  // keyed to linear-order ghost indices while the plan is built, remapped
  // to canonical positions once those are known
  D.hoff.assign(ninst + 1, 0);
  D.hmask.assign(ninst, 0);
  for (int i = 0; i < ninst; ++i) {
    int64_t size = 64;
    while (size < 2 * (D.if_off[i + 1] - D.if_off[i])) size <<= 1;
    D.hmask[i] = (uint32_t)(size - 1);
    D.hoff[i + 1] = D.hoff[i] + size;
  }
  D.d_htab = own<unsigned long long>(D, D.hoff[ninst]);
  if (!D.d_htab) return GCR_E_NOMEM;
  std::memcpy(PS.p + o_ho, D.hoff.data(), 8 * (ninst + 1));
  std::memcpy(PS.p + o_hm, D.hmask.data(), 4 * ninst);
  GCR_HIP(hipMemcpyAsync(tb + o_ho, PS.p + o_ho, stage_bytes - o_ho, hipMemcpyHostToDevice,
                         st));   // R3
  const int64_t nblk = (nif + 1023) / 1024;
  D.d_if_cell = own<int32_t>(D, cap);
  D.d_if_psi = own<double>(D, cap);
  D.d_if_n = own<double>(D, 3 * cap);
  D.d_if_flag = own<uint8_t>(D, cap);
  D.d_blkcnt = own<int32_t>(D, nblk + 1);
  D.d_blkexcl = own<int64_t>(D, nblk + 2);
  D.d_g_cell = own<int32_t>(D, cap);
  D.d_g_ext = own<uint8_t>(D, cap);
  D.d_g_psi = own<double>(D, cap);
  D.d_g_n = own<double>(D, 3 * cap);
  D.d_g_code = own<uint32_t>(D, cap);
  D.d_deps = own<int32_t>(D, 7 * cap);
  D.d_lev = own<int32_t>(D, cap);
  D.d_blk_idx = own<int32_t>(D, cap);
  D.d_perm = own<int32_t>(D, cap);
  D.d_cell = own<int32_t>(D, cap);
  D.d_delta = own<double>(D, 3 * cap);
  D.d_nrm = own<double>(D, 3 * cap);
  D.d_psi = own<double>(D, cap);
  D.d_code = own<uint32_t>(D, cap);
  D.d_level = own<int32_t>(D, cap);
  D.d_blk = own<int32_t>(D, cap);
  D.d_listA = own<int32_t>(D, cap);
  D.d_rcnt = own<int32_t>(D, 2 * cap);   // counts, then fill pointers
  D.d_roff = own<int32_t>(D, cap + 1);
  D.d_dcnt = own<uint8_t>(D, cap);
  D.d_radj = own<int32_t>(D, 7 * cap);
  D.d_cnt = own<uint32_t>(D, (cap >> 2) + ninst + 2);
  D.d_bits = own<uint32_t>(D, (cap >> 5) + ninst + 2);
  if (!D.d_listA || !D.d_rcnt || !D.d_roff || !D.d_radj || !D.d_cnt || !D.d_bits || !D.d_dcnt)
    return GCR_E_NOMEM;
  if (!D.d_if_cell || !D.d_if_psi || !D.d_if_n || !D.d_if_flag || !D.d_blkcnt || !D.d_blkexcl ||
      !D.d_g_cell || !D.d_g_ext || !D.d_g_psi || !D.d_g_n || !D.d_g_code || !D.d_deps || !D.d_lev ||
      !D.d_blk_idx || !D.d_perm || !D.d_cell || !D.d_delta || !D.d_nrm || !D.d_psi ||
      !D.d_code || !D.d_level || !D.d_blk)
    return GCR_E_NOMEM;
  // the third normal component of 2D ghosts stays zero
  if (any_2d) GCR_HIP(hipMemsetAsync(D.d_if_n + 2 * cap, 0, sizeof(double) * cap, st));

  T.mark(3, st);
  if (nif > 0) {
    k_compact_iface<<<(unsigned)nlist, 256, 0, st>>>(D.d_inst, D.d_chunk_inst, D.d_tags,
                                                     D.d_chunk_cnt, D.d_chunk_excl, D.d_chunk_list,
                                                     D.d_if_cell, D.d_htab, D.hoff[ninst]);
    T.mark(4, st);
    k_geometry<<<blocks(nif, 256), 256, 0, st>>>(D.d_inst, ninst, D.d_if_off, D.d_if_cell,
                                                  D.d_tags, D.d_if_psi, D.d_if_n, cap,
                                                  D.d_if_flag, D.d_info);
    T.mark(5, st);
    k_count_flags<<<(unsigned)nblk, 256, 0, st>>>(D.d_if_flag, nif, D.d_blkcnt);
    k_scan<<<1, 1024, 0, st>>>(D.d_blkcnt, nblk, D.d_blkexcl, nullptr, nullptr);
    k_scatter_ghosts<<<(unsigned)nblk, 256, 0, st>>>(D.d_if_flag, nif, D.d_blkexcl, D.d_if_cell,
                                                     D.d_if_psi, D.d_if_n, cap, D.d_g_cell,
                                                     D.d_g_psi, D.d_g_n, D.d_g_ext);
    k_ghost_off<<<(unsigned)(ninst + 1), 64, 0, st>>>(D.d_if_flag, D.d_blkexcl, D.d_if_off, ninst,
                                                      D.d_g_off);
    T.mark(6, st);
    // ghost count unknown on the host: launch over the interface capacity
    k_hash_build<<<blocks(nif, 256), 256, 0, st>>>(D.d_g_off, ninst, D.d_g_cell, D.d_hoff,
                                                    D.d_hmask, D.d_htab, D.d_rcnt,
                                                    2 * cap);   // + rcnt, rfill cleared
    k_deps<<<blocks(nif, 256), 256, 0, st>>>(D.d_inst, ninst, D.d_g_off, D.d_g_cell, D.d_g_psi,
                                              D.d_g_n, cap, D.d_g_ext, D.d_tags, D.d_htab, D.d_hoff,
                                              D.d_hmask, D.d_g_code, D.d_deps,
                                              D.d_rcnt, D.d_dcnt, D.d_info);
    {
      // reverse-edge offsets: one workgroup up to two tiles, else three passes
      // over the interface capacity
      const int64_t ntiles = (cap + kScanTile - 1) / kScanTile;
      if (ntiles <= 2) {
        k_rscan<<<1, 1024, 0, st>>>(D.d_rcnt, D.d_g_off, ninst, D.d_roff);
      } else {
        int64_t* tsum = own<int64_t>(D, ntiles + 1);
        if (!tsum) return GCR_E_NOMEM;
        k_iscan_reduce<<<(unsigned)ntiles, 1024, 0, st>>>(D.d_rcnt, cap, tsum);
        k_scan_top<<<1, 1024, 0, st>>>(tsum, ntiles, tsum + ntiles, nullptr);
        k_iscan_down<<<(unsigned)ntiles, 1024, 0, st>>>(D.d_rcnt, cap, tsum, D.d_roff);
      }
    }
    k_rfill<<<blocks(nif, 256), 256, 0, st>>>(D.d_inst, D.d_g_off, ninst, cap, D.d_deps,
                                               D.d_roff, D.d_rcnt + cap, D.d_radj);
    T.mark(7, st);
    {
      LevelsArgs L;
      L.insts = D.d_inst;
      L.g_off = D.d_g_off;
      L.deps = D.d_deps;
      L.cap = cap;
      L.lev = D.d_lev;
      L.blk_idx = D.d_blk_idx;
      L.perm = D.d_perm;
      L.lev_off = D.d_lev_off;
      L.unit_mem = D.d_unit_mem;
      L.unit_cnt = D.d_unit_cnt;
      L.unit_lev = D.d_unit_lev;
      L.reach = D.d_reach;
      L.listA = D.d_listA;
      L.dcnt = D.d_dcnt;
      L.roff = D.d_roff;
      L.radj = D.d_radj;
      L.cnt = D.d_cnt;
      L.bits = D.d_bits;
      L.info = D.d_info;
      int64_t max_if = 0;
      for (int i = 0; i < ninst; ++i) max_if = std::max(max_if, D.if_off[i + 1] - D.if_off[i]);
      L.listB = L.wide = L.hist = nullptr;
      L.cur_cap = 0;
      L.wave_res = wave_residual();
      L.wide_cap = wide_buffer();
      if (ninst == 1 && max_if >= wide_layering_min()) {
        // the reverse-edge counters are spent once the edges are filled
        L.listB = D.d_rcnt;
        L.wide = own<int32_t>(D, kWideState);
        L.hist = own<int32_t>(D, (size_t)kWideLevels * (cap / 256 + 1));
        if (!L.wide || !L.hist) return GCR_E_NOMEM;
      }
      const gcr_status ls = launch_levels(L, ninst, max_if, st);
      if (ls != GCR_OK) return ls;
    }
    T.mark(8, st);
    {
      const unsigned nfb = blocks(nif, 256);
      FinPart* fp = own<FinPart>(D, nfb);
      if (!fp) return GCR_E_NOMEM;
      k_finalize<<<nfb, 256, 0, st>>>(
          D.d_inst, ninst, D.d_g_off, cap, D.d_g_cell, D.d_g_psi, D.d_g_n, D.d_g_code, D.d_lev,
          D.d_blk_idx, D.d_perm, D.d_cell, D.d_delta, D.d_nrm, D.d_psi, D.d_code, D.d_level,
          D.d_blk, D.d_info, fp);
      k_units_canonical<<<ninst, 256, 0, st>>>(D.d_perm, D.d_info, D.d_unit_mem, D.d_unit_cnt,
                                               fp, (int64_t)nfb);
    }
    k_hash_remap<<<blocks(D.hoff[ninst], 256), 256, 0, st>>>(D.d_hoff, ninst, D.d_g_off, D.d_perm,
                                                              D.d_htab);
    T.mark(9, st);
  } else {
    k_hash_clear<<<blocks(D.hoff[ninst], 256), 256, 0, st>>>(D.d_htab, D.hoff[ninst]);
    for (int i = 4; i <= 9; ++i) T.mark(i, st);
    GCR_HIP(hipMemsetAsync(D.d_g_off, 0, sizeof(int64_t) * (ninst + 1), st));
    GCR_HIP(hipMemsetAsync(D.d_lev_off, 0, sizeof(int32_t) * ninst * (kMaxLevels + 1), st));
  }
  GCR_HIP(hipGetLastError());
  D.g_off.resize(ninst + 1);
  D.info.resize(ninst);
  D.lev_off.resize((size_t)ninst * (kMaxLevels + 1));
  D.unit_lev.resize((size_t)ninst * kMaxUnits);
  GCR_HIP(hipMemcpyAsync(PS.p + o_info, tb + o_info, o_if - o_info, hipMemcpyDeviceToHost,
                         st));   // R4
  GCR_HIP(hipStreamSynchronize(st));
  PS.pending = false;
  std::memcpy(D.g_off.data(), PS.p + o_go, 8 * (ninst + 1));
  std::memcpy(D.info.data(), PS.p + o_info, sizeof(InstInfo) * ninst);
  std::memcpy(D.lev_off.data(), PS.p + o_lo, 4 * (size_t)ninst * (kMaxLevels + 1));
  std::memcpy(D.unit_lev.data(), PS.p + o_ul, 4 * (size_t)ninst * kMaxUnits);
  T.collect(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call)
                .count());
  D.ng_total = D.g_off[ninst];
  for (int i = 0; i < ninst; ++i) {
    gcr_status s = status_from_err(D.info[i].err);
    if (s != GCR_OK) return s;
  }
  GCR_HIP(hipGetLastError());
  *out = B;
  return GCR_OK;
}

void make_plan_view(const std::shared_ptr<BatchData>& B, int i, gcr_plan* p) {
  const BatchData& D = *B;
  p->batch = B;
  p->index = i;
  p->inst = D.inst[i];
  p->dim = p->inst.g.dim;
  p->ncell = p->inst.g.ncell;
  p->goff = D.g_off[i];
  p->ng = D.g_off[i + 1] - D.g_off[i];
  p->nif = D.iface_off[i + 1] - D.iface_off[i];
  p->stride = D.cap;
  p->info = D.info[i];
  p->nlev = p->info.nlev;
  p->lev_off.assign(D.lev_off.begin() + (size_t)i * (kMaxLevels + 1),
                    D.lev_off.begin() + (size_t)i * (kMaxLevels + 1) + p->nlev + 1);
  p->tags = D.d_tags + p->inst.cell_off;
  p->span = D.d_span + p->inst.chunk_off * (kChunk / (64 * kSeg));
  const int64_t o = p->goff;
  if (D.d_cell) {
    p->cell = D.d_cell + o;
    for (int a = 0; a < 3; ++a) {
      p->delta[a] = D.d_delta + a * D.cap + o;
      p->nrm[a] = D.d_nrm + a * D.cap + o;
    }
    p->psi = D.d_psi + o;
    p->code = D.d_code + o;
    p->level = D.d_level + o;
    p->blk = D.d_blk + o;
    p->sorted_cell = D.d_g_cell + o;
    p->sorted_pos = D.d_perm + o;
  }
  p->unit_mem = D.d_unit_mem + (int64_t)i * kMaxUnits * kMaxUnit;
  p->unit_cnt = D.d_unit_cnt + (int64_t)i * kMaxUnits;
  p->d_lev_off = D.d_lev_off + (int64_t)i * (kMaxLevels + 1);
  p->unit_lev = D.d_unit_lev + (int64_t)i * kMaxUnits;
  p->unit_lev_host.assign(D.unit_lev.begin() + (size_t)i * kMaxUnits,
                          D.unit_lev.begin() + (size_t)i * kMaxUnits + p->info.nunits);
  p->htab = D.d_htab + D.hoff[i];
  p->hmask = D.hmask[i];
}

}  // namespace gcr
