// gcr_device.hpp -- device-side data structures and inline functions of the
// ghost-cell library: instance descriptors, body geometry (inside test,
// closest point, analytic normal), ghost stencil codes, and the ghost
// relations written in tensor-product Lagrange form on the stencil box.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gcr {

constexpr int kMaxCoef = 128;     // star: 2 * 64 harmonics; SH: (L+1)^2, L <= 8
constexpr int kMaxFields = 8;
constexpr int kMaxUnit = 8;       // largest coupled unit (strongly connected group)
constexpr int kMaxUnits = 1024;   // coupled units per instance
constexpr int kMaxLevels = 1024;  // levels per instance
constexpr int kChunk = 4096;      // cells per classification workgroup
constexpr int kSeg = 16;          // cells per classification thread
// the band-segment count (statistics) accumulates in this many counters, one
// per 64-byte line, so that chunks add to different addresses
constexpr int kBandStripes = 64;
constexpr int kMaxResidual = 1024;// ghosts left after plain Kahn layering

// error bits, reported per instance
enum : uint32_t {
  kErrStencil = 1u << 0,
  kErrGeometry = 1u << 1,
  kErrCycle = 1u << 2,
  kErrDegenerate = 1u << 3,
  kErrUnsupported = 1u << 4,
};

enum { kSphere = 0, kStar2D = 1, kShStar = 2, kAirfoil = 3 };
enum { kCGC = 0, kCGC_ES = 1, kHGC = 2 };
constexpr int kLayer2 = 4;   // scheme flag: a second ghost layer

struct GridD {
  int dim;
  int n[3];
  double lo[3];
  double h[3];
  int64_t ncell;
  const double* face[3];   // stretched axis: n + 1 cell faces (device), else null
};

struct ShapeD {
  int kind, ncoef, L, pad;
  double c[3];
  double r0;
  double cull_c[3];     // centre of the radial culling bounds
  double rmin, rmax;    // every boundary point lies at rmin <= |x - cull_c| <= rmax
  double lip;           // star / SH: |r(w) - r(w')| <= lip * angle(w, w')
  double chord, thick, ca, sa;   // airfoil: chord, thickness ratio, cos/sin incidence
  double coef[kMaxCoef];         // star: A_k, B_k pairs; SH: a_lm * N_lm at l*l+l+m
};

struct Inst {
  GridD g;
  ShapeD s;
  int scheme;          // kCGC, kCGC_ES, kHGC
  int layer2;          // 1: a second ghost layer (Sec. 7.1)
  int l2r[3];          // its candidate box half-widths in cells per axis
  int pad_;
  int64_t cell_off;    // offset of this instance in the concatenated tag array
  int64_t chunk_off;   // first classification chunk of this instance
  int64_t nchunk;
};

// Exclusive scan over a workgroup of BS threads (BS multiple of 64); every
// thread of the workgroup must call it.  sh: BS/64 + 1 shared slots.
template <int BS>
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* total, int64_t* sh) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < BS / 64; ++i) {
      int64_t t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[BS / 64] = run;
  }
  __syncthreads();
  int64_t res = sh[w] + x - v;
  *total = sh[BS / 64];
  __syncthreads();
  return res;
}

// Exclusive scan of in[0..n) into out[0..n], out[n] = total, by one
// workgroup of 1024 threads: tiles of 8 consecutive values per thread
// (two 16-byte loads when the tile is whole and aligned), a serial scan per
// thread, one workgroup scan per tile.  Every thread must call it.
__device__ __forceinline__ void block_scan_i32(const int32_t* __restrict__ in, int64_t n,
                                               int32_t* __restrict__ out, int64_t* sh) {
  constexpr int kT = 8, kTile = 1024 * kT;
  const bool vec = ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
  int64_t carry = 0;
  for (int64_t t0 = 0; t0 < n; t0 += kTile) {
    const int64_t b = t0 + (int64_t)threadIdx.x * kT;
    int v[kT];
    if (vec && b + kT <= n) {
      const int4 a = *reinterpret_cast<const int4*>(in + b);
      const int4 c = *reinterpret_cast<const int4*>(in + b + 4);
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
      v[4] = c.x; v[5] = c.y; v[6] = c.z; v[7] = c.w;
    } else {
#pragma unroll
      for (int q = 0; q < kT; ++q) v[q] = b + q < n ? in[b + q] : 0;
    }
    int64_t sum = 0;
#pragma unroll
    for (int q = 0; q < kT; ++q) sum += v[q];
    int64_t tot;
    int64_t run = carry + block_excl_scan<1024>(sum, &tot, sh);
    int o[kT];
#pragma unroll
    for (int q = 0; q < kT; ++q) {
      o[q] = (int32_t)run;
      run += v[q];
    }
    if (vec && b + kT <= n) {
      *reinterpret_cast<int4*>(out + b) = make_int4(o[0], o[1], o[2], o[3]);
      *reinterpret_cast<int4*>(out + b + 4) = make_int4(o[4], o[5], o[6], o[7]);
    } else {
#pragma unroll
      for (int q = 0; q < kT; ++q)
        if (b + q < n) out[b + q] = o[q];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) out[n] = (int32_t)carry;
}

// --------------------------------------------------------------------------
// grid helpers
// --------------------------------------------------------------------------

__device__ __forceinline__ double centre(const GridD& g, int ax, int i) {
  if (g.face[ax]) return 0.5 * (g.face[ax][i] + g.face[ax][i + 1]);
  return g.lo[ax] + ((double)i + 0.5) * g.h[ax];
}

// local spacing of cell i along axis ax: its width
__device__ __forceinline__ double width(const GridD& g, int ax, int i) {
  if (g.face[ax]) return g.face[ax][i + 1] - g.face[ax][i];
  return g.h[ax];
}

// centres of the face neighbours of cell i along ax (beyond the grid: one
// width further), bounding every point a box test must cover
__device__ __forceinline__ double centre_below(const GridD& g, int ax, int i) {
  if (!g.face[ax]) return centre(g, ax, i) - g.h[ax];
  return i > 0 ? centre(g, ax, i - 1) : centre(g, ax, i) - width(g, ax, i);
}
__device__ __forceinline__ double centre_above(const GridD& g, int ax, int i) {
  if (!g.face[ax]) return centre(g, ax, i) + g.h[ax];
  return i + 1 < g.n[ax] ? centre(g, ax, i + 1) : centre(g, ax, i) + width(g, ax, i);
}

// index of the cell holding coordinate x along ax (off the grid: < 0 or
// >= n, which callers test)
__device__ __forceinline__ int cell_of(const GridD& g, int ax, double x) {
  if (!g.face[ax]) return (int)floor((x - g.lo[ax]) / g.h[ax]);
  const double* f = g.face[ax];
  const int n = g.n[ax];
  if (x < f[0]) return -1;
  if (x >= f[n]) return n;
  int lo = 0, hi = n - 1;   // the last i with f[i] <= x
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (f[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ void unlinear(const GridD& g, int c, int& i, int& j, int& k) {
  i = c % g.n[0];
  int t = c / g.n[0];
  j = t % g.n[1];
  k = t / g.n[1];
}

__device__ __forceinline__ int linear(const GridD& g, int i, int j, int k) {
  return i + g.n[0] * (j + g.n[1] * k);
}

// --------------------------------------------------------------------------
// stencil code of a ghost: sign of each normal component (sgn 0 = +1),
// axes whose normal component is exactly zero (their displaced points carry
// zero weight and are never read), and the multipliers r_i (<= 15).
// --------------------------------------------------------------------------

__device__ __forceinline__ uint32_t make_code(const double n[3], const int r[3], int dim) {
  uint32_t code = 0;
  for (int i = 0; i < dim; ++i) {
    if (!(n[i] >= 0.0)) code |= 1u << i;          // e_i = -1
    if (n[i] == 0.0) code |= 1u << (3 + i);       // zero normal component
    code |= (uint32_t)(r[i] & 15) << (8 + 4 * i);
  }
  return code;
}
__device__ __forceinline__ int code_e(uint32_t code, int i) { return (code >> i) & 1u ? -1 : 1; }
__device__ __forceinline__ int code_r(uint32_t code, int i) { return (int)((code >> (8 + 4 * i)) & 15u); }

// x_2 - x_1 per axis of the stencil of the ghost in cell c: e_i r_i h_i, or
// on a stretched axis the difference of the two cell centres (a
// displacement off the grid, only along an axis the normal does not leave,
// takes the cell width)
__device__ __forceinline__ void stencil_span(const GridD& g, uint32_t code, int c,
                                             double X[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) X[a] = (double)(code_e(code, a) * code_r(code, a)) * g.h[a];
  if (!g.face[0] && !g.face[1] && !g.face[2]) return;   // uniform: no cell index needed
  int ijk[3];
  unlinear(g, c, ijk[0], ijk[1], ijk[2]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int er = code_e(code, a) * code_r(code, a);
    if (a >= g.dim || !g.face[a]) continue;
    const int q = ijk[a] + er;
    X[a] = (q >= 0 && q < g.n[a]) ? centre(g, a, q) - centre(g, a, ijk[a])
                                  : (double)er * width(g, a, ijk[a]);
  }
}
__device__ __forceinline__ uint32_t code_skip(uint32_t code) { return (code >> 3) & 7u; }

// Linear offset of stencil corner `k` (bit i set: displaced by e_i r_i along
// axis i) from the ghost's cell.
__device__ __forceinline__ int corner_offset(const GridD& g, uint32_t code, int k) {
  int off = 0;
  if (k & 1) off += code_e(code, 0) * code_r(code, 0);
  if (k & 2) off += code_e(code, 1) * code_r(code, 1) * g.n[0];
  if (k & 4) off += code_e(code, 2) * code_r(code, 2) * g.n[0] * g.n[1];
  return off;
}

// Whether corner k of a ghost at (i,j,k3) lies inside the grid.
__device__ __forceinline__ bool corner_in_grid(const GridD& g, uint32_t code, int i, int j, int k3,
                                               int k) {
  int q[3] = {i, j, k3};
  for (int a = 0; a < g.dim; ++a)
    if ((k >> a) & 1) {
      q[a] += code_e(code, a) * code_r(code, a);
      if (q[a] < 0 || q[a] >= g.n[a]) return false;
    }
  return true;
}

// --------------------------------------------------------------------------
// Ghost relations in tensor-product form.  With alpha_i = (x_s - x_1)_i /
// (x_2 - x_1)_i, the bilinear / trilinear polynomial through the stencil box
// is sum_k L_k phi_k, L_k = prod_i (bit_i(k) ? alpha_i : 1 - alpha_i).
// Dirichlet: sum_k L_k phi_k = phi_s; Neumann: sum_k (n . grad L_k) phi_k =
// dphi/dn, both at S.  Solving either for phi_G = phi_0 gives
// phi_G = ws * b + sum_{k>0} w_k phi_k.  These are the relations of the
// paper's Sec. 4.1 / 5.1 (same polynomial, same data), arranged for a GPU:
// one loop over corners, no per-dimension special cases.
// --------------------------------------------------------------------------

template <int D>
__device__ __forceinline__ void lagrange(const double a[3], int k, double& L) {
  L = 1.0;
#pragma unroll
  for (int i = 0; i < D; ++i) L *= ((k >> i) & 1) ? a[i] : 1.0 - a[i];
}

// d L_k / d x_i (X_i = e_i r_i h_i)
template <int D>
__device__ __forceinline__ double lagrange_grad(const double a[3], const double X[3], int k, int i) {
  double v = ((k >> i) & 1) ? 1.0 / X[i] : -1.0 / X[i];
#pragma unroll
  for (int j = 0; j < D; ++j)
    if (j != i) v *= ((k >> j) & 1) ? a[j] : 1.0 - a[j];
  return v;
}

// Weights of one ghost: w[0] = weight of the boundary datum, w[k] (k >= 1)
// weight of corner k.  Returns false on a zero denominator.
template <int D>
__device__ __forceinline__ bool ghost_weights(const double dl[3], const double nn[3],
                                              const double X[3], int bc, double w[8]) {
  double a[3];
#pragma unroll
  for (int i = 0; i < D; ++i) a[i] = dl[i] / X[i];
  double c[8];
  if (bc == 0) {
#pragma unroll
    for (int k = 0; k < (1 << D); ++k) lagrange<D>(a, k, c[k]);
  } else {
#pragma unroll
    for (int k = 0; k < (1 << D); ++k) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < D; ++i) s += nn[i] * lagrange_grad<D>(a, X, k, i);
      c[k] = s;
    }
  }
  if (c[0] == 0.0) return false;
  double inv = 1.0 / c[0];
  w[0] = inv;
#pragma unroll
  for (int k = 1; k < (1 << D); ++k) w[k] = -c[k] * inv;
  return true;
}

// Value and gradient of the box polynomial at a point whose offset from the
// ghost centre is rel[], from the 2^D corner values v[].
template <int D>
__device__ __forceinline__ void box_eval(const double rel[3], const double X[3],
                                         const double v[8], double& val, double grad[3]) {
  double a[3];
#pragma unroll
  for (int i = 0; i < D; ++i) a[i] = rel[i] / X[i];
  val = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) grad[i] = 0.0;
#pragma unroll
  for (int k = 0; k < (1 << D); ++k) {
    double L;
    lagrange<D>(a, k, L);
    val += L * v[k];
#pragma unroll
    for (int i = 0; i < D; ++i) grad[i] += lagrange_grad<D>(a, X, k, i) * v[k];
  }
}

// Coefficients of the value and gradient of the box polynomial at rel[] on
// corner k (for adjoints).
template <int D>
__device__ __forceinline__ void box_coeffs(const double rel[3], const double X[3], int k,
                                           double& cv, double cg[3]) {
  double a[3];
#pragma unroll
  for (int i = 0; i < D; ++i) a[i] = rel[i] / X[i];
  lagrange<D>(a, k, cv);
#pragma unroll
  for (int i = 0; i < D; ++i) cg[i] = lagrange_grad<D>(a, X, k, i);
}

// --------------------------------------------------------------------------
// body geometry
// --------------------------------------------------------------------------

__device__ __forceinline__ double naca_half_thickness(double t, double x) {
  double sx = sqrt(x);
  return 5.0 * t * (0.2969 * sx - 0.1260 * x - 0.3516 * x * x + 0.2843 * x * x * x -
                    0.1036 * x * x * x * x);
}

// star radius r(theta) and r'(theta) at the direction u (unit), using
// (cos k t, sin k t) = powers of (u_x + i u_y)
__device__ __forceinline__ void star_r(const ShapeD& s, double ux, double uy, double& r,
                                       double& r1) {
  double ck = 1.0, sk = 0.0, sum = 1.0, d = 0.0;
  for (int k = 0; k < s.ncoef; ++k) {
    double A = s.coef[2 * k], B = s.coef[2 * k + 1];
    sum += A * ck + B * sk;
    d += (double)k * (B * ck - A * sk);
    double nc = ck * ux - sk * uy;
    double ns = ck * uy + sk * ux;
    ck = nc;
    sk = ns;
  }
  r = s.r0 * sum;
  r1 = s.r0 * d;
}

// The same with r'' (d^2 r / d theta^2 = -r0 sum k^2 (A_k cos k theta +
// B_k sin k theta)).
__device__ __forceinline__ void star_r2(const ShapeD& s, double ux, double uy, double& r,
                                        double& r1, double& r2) {
  double ck = 1.0, sk = 0.0, sum = 1.0, d = 0.0, dd = 0.0;
  for (int k = 0; k < s.ncoef; ++k) {
    double A = s.coef[2 * k], B = s.coef[2 * k + 1];
    sum += A * ck + B * sk;
    d += (double)k * (B * ck - A * sk);
    dd -= (double)(k * k) * (A * ck + B * sk);
    double nc = ck * ux - sk * uy;
    double ns = ck * uy + sk * ux;
    ck = nc;
    sk = ns;
  }
  r = s.r0 * sum;
  r1 = s.r0 * d;
  r2 = s.r0 * dd;
}

// SH radius and its gradient on the unit sphere (tangential) at direction u.
// Y_lm = N_lm P~_l^|m|(u_z) {Re,Im}((u_x + i u_y)^|m|) with P~_l^m = d^m P_l/dt^m;
// coef[] holds a_lm N_lm.
__device__ __forceinline__ void sh_r(const ShapeD& s, const double u[3], double& r, double g[3]) {
  const int L = s.L;
  double t = u[2];
  double sum = 1.0, gx = 0.0, gy = 0.0, gz = 0.0;
  // zeta^m = (ux + i uy)^m and zeta^(m-1)
  double zr = 1.0, zi = 0.0;       // zeta^m
  double pr = 0.0, pi = 0.0;       // zeta^(m-1)
  for (int m = 0; m <= L; ++m) {
    // P~_l^m(t) for l = m..L and P~_l^{m+1}(t) (its t-derivative)
    double dfact = 1.0;
    for (int q = 1; q <= 2 * m - 1; q += 2) dfact *= (double)q;
    double dfact1 = dfact * (double)(2 * m + 1);   // (2(m+1)-1)!!
    double a0 = dfact, a1 = 0.0;   // P~_{l-1}, P~_l for order m
    double b0 = dfact1, b1 = 0.0;  // same for order m+1
    for (int l = m; l <= L; ++l) {
      double P, Pd;
      if (l == m) {
        P = dfact;
      } else if (l == m + 1) {
        P = (double)(2 * m + 1) * t * dfact;
      } else {
        P = ((double)(2 * l - 1) * t * a1 - (double)(l + m - 1) * a0) / (double)(l - m);
      }
      // derivative: P~_l^{m+1}
      if (l < m + 1) {
        Pd = 0.0;
      } else if (l == m + 1) {
        Pd = dfact1;
      } else if (l == m + 2) {
        Pd = (double)(2 * m + 3) * t * dfact1;
      } else {
        Pd = ((double)(2 * l - 1) * t * b1 - (double)(l + m) * b0) / (double)(l - m - 1);
      }
      if (l == m) {
        a1 = P;
      } else {
        a0 = a1;
        a1 = P;
      }
      if (l >= m + 1) {
        if (l == m + 1) {
          b1 = Pd;
        } else {
          b0 = b1;
          b1 = Pd;
        }
      }
      double cp = s.coef[l * l + l + m];                 // cos part (m >= 0)
      double cm = m > 0 ? s.coef[l * l + l - m] : 0.0;   // sin part
      double ang = cp * zr + cm * zi;                    // sum of harmonic parts
      sum += P * ang;
      // gradient of the polynomial extension at u
      gz += Pd * ang;
      if (m > 0) {
        // d/dx zeta^m = m zeta^(m-1), d/dy zeta^m = i m zeta^(m-1)
        double dxr = (double)m * pr, dxi = (double)m * pi;
        gx += P * (cp * dxr + cm * dxi);
        gy += P * (cp * (-dxi) + cm * dxr);
      }
    }
    pr = zr;
    pi = zi;
    double nzr = zr * u[0] - zi * u[1];
    double nzi = zr * u[1] + zi * u[0];
    zr = nzr;
    zi = nzi;
  }
  r = s.r0 * sum;
  double gu = gx * u[0] + gy * u[1] + gz * u[2];
  g[0] = s.r0 * (gx - gu * u[0]);
  g[1] = s.r0 * (gy - gu * u[1]);
  g[2] = s.r0 * (gz - gu * u[2]);
}

// Inside test: true for a solid centre (psi >= 0), boundary points solid.
__device__ __forceinline__ bool inside(const ShapeD& s, int dim, const double x[3]) {
  if (s.kind == kAirfoil) {
    double dx = (x[0] - s.c[0]) / s.chord, dy = (x[1] - s.c[1]) / s.chord;
    double b0 = s.ca * dx - s.sa * dy;
    double b1 = s.sa * dx + s.ca * dy;
    if (b0 < 0.0 || b0 > 1.0) return false;
    return fabs(b1) <= naca_half_thickness(s.thick, b0);
  }
  double dx = x[0] - s.c[0], dy = x[1] - s.c[1], dz = dim == 3 ? x[2] - s.c[2] : 0.0;
  double rho2 = dx * dx + dy * dy;
  if (dim == 3) rho2 += dz * dz;
  // rho^2 clearly below rmin^2 or above rmax^2 settles the test without a
  // square root; the 1e-10 relative margin dwarfs every rounding involved,
  // so the decision equals that of r - sqrt(rho^2) >= 0
  if (rho2 < s.rmin * s.rmin * (1.0 - 1e-10)) return true;
  if (rho2 > s.rmax * s.rmax * (1.0 + 1e-10)) return false;
  double rho = sqrt(rho2);
  double r;
  if (s.kind == kSphere) {
    r = s.r0;
  } else {
    if (rho == 0.0) return true;
    if (s.kind == kStar2D) {
      double r1;
      star_r(s, dx / rho, dy / rho, r, r1);
    } else {
      double u[3] = {dx / rho, dy / rho, dz / rho}, g[3];
      sh_r(s, u, r, g);
    }
  }
  return r - rho >= 0.0;
}

// Closest boundary point of x, analytic outward normal there, and the
// signed distance (+ for solid centres).  Returns false if the iteration
// does not converge.
__device__ bool project(const ShapeD& s, int dim, const double x[3], bool solid, double n[3],
                        double& psi);

}  // namespace gcr
